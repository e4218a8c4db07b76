"""Host-side checks of the C ABI (no GPU): the library loads and exports
every function include/vlg.h declares; the formula front end parses the same
language as the oracle, shares identical sub-expressions and reports errors
with positions."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2010_07284_amd as vlg
from paper_2010_07284_amd import _lib
from synth import formulas

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "vlg.h")).read()
    return sorted(set(re.findall(r"\b(vlg_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    L = ctypes.CDLL(_lib.LIB_PATH)
    names = declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(_lib.EXPORTS) == names


def info(src):
    return vlg.formula_info(vlg.compile_formula(None, src))


def test_hash_consing_shares_nodes():
    src = """
    let A = intensity(img) >. 0.5
    let B = intensity(img, 1) <. 0.25
    let x = A & B
    let y = B & A                 // commutative: same node as x
    let z = intensity(img) >. 0.5000000001   // same float32 threshold as A
    let f(p, q) = near(p) | q
    output "o1" f(x, y) & f(y, x)  // both calls expand to the same nodes
    output "o2" x & z
    """
    st = info(src)
    # nodes: A, B, A&B, near(A&B), near|, and-of-equal-operands, A&(A&B) -> 7
    assert st["nodes"] == 7
    assert st["parsed_nodes"] > st["nodes"]
    assert st["outputs"] == 2 and st["atoms"] == 2


def test_counts_of_workload_formulas():
    st = info(formulas.PLAIN_FORMULA)
    assert st["nodes"] == 12 and st["reach_nodes"] == 3 and st["outputs"] == 3
    st = info(formulas.ellipse_dag(2))
    assert 95 <= st["nodes"] <= 100 and st["reach_nodes"] == 10
    st = info(formulas.chain_dag(3))
    assert st["nodes"] == 10501 and st["reach_nodes"] == 500
    assert st["steps_fused"] < st["steps_perop"]


@pytest.mark.parametrize("src", [
    'output "x" foo',
    'let a = intensity(img) >. \noutput "x" a',
    'output "x" near(true',
    'let near = true',
    'output x true',
    'let f(a) = a & b\noutput "x" f(true)',
    'output "x" intensity(img, 1) >. percentile(img, 0)',
    'output "x" reach(true)',
    'output "x" true $',
])
def test_parse_errors_agree_with_oracle(src):
    with pytest.raises(vlg.VlgError) as e:
        vlg.compile_formula(None, src)
    assert e.value.code == -2 and "line" in str(e.value)
    with pytest.raises(oracle.OracleError):
        oracle.run(src, np.zeros((2, 2, 2), np.float32))


def test_macro_scoping_matches_oracle():
    # a macro sees the bindings made before its definition, like the oracle
    src = """
    let A = intensity(img) >. 0.5
    let f(x) = x & A
    let A = intensity(img) <. 0.2
    output "o" f(true)
    output "p" A
    """
    st = info(src)
    # nodes: first A, second A, true, true & first-A (no new atom for f's A)
    assert st["nodes"] == 4 and st["atoms"] == 2


def test_null_arguments_are_rejected():
    L = _lib.lib()
    assert L.vlg_compile_formula(None, None, None) == -1
    assert L.vlg_formula_info(None, None) == -1
    assert L.vlg_check(None, None, None, 0, None, 0, 1) == -1
    assert b"null" in L.vlg_last_error()


def test_stream_copy_rejects_bad_arguments():
    # rejected on the host before any device call
    L = _lib.lib()
    ms = ctypes.c_double()
    assert L.vlg_stream_copy(None, None, None, 16, 16, 1, ctypes.byref(ms)) == -1
    assert b"bad argument" in L.vlg_last_error()
