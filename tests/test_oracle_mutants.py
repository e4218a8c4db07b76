"""Mistakes planted in the oracle (on the CPU) must be caught by its pins.

Each mutant is a copy of oracle/oracle.c with one plausible slip (a dropped
term, a wrong operand, an off-by-one, a swapped precedence); it is compiled
to a temporary library and the pin suites are run against it in a
subprocess, which must fail.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

from oracle.build import SRC, build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "near_drops_bottom_row": ("for (int dy = -1; dy <= 1 && !v; dy++)",
                              "for (int dy = -1; dy <= 0 && !v; dy++)"),
    "reach_steps_onto_a": ("if (b[q] && !mark[q]) {", "if (a[q] && !mark[q]) {"),
    "reach_no_final_dilation": ("    oracle_near(mark, H, W, out);\n    free(mark);",
                                "    memcpy(out, mark, (size_t)n);\n    free(mark);"),
    "reach_endpoint_needs_b": ("        if (a[p]) {\n            mark[p] = 1;",
                               "        if (a[p] && b[p]) {\n            mark[p] = 1;"),
    "surrounded_or_for_and": ("oracle_and(na, nb, n, esc);", "oracle_or(na, nb, n, esc);"),
    "surrounded_wrong_sign": ("rc = oracle_reach(esc, nb, H, W, r);",
                              "rc = oracle_reach(esc, b, H, W, r);"),
    "grow_and_with_a": ("oracle_and(b, r, n, r);", "oracle_and(a, r, n, r);"),
    "threshold_gt_as_ge": ("case CMP_GT: r = v > t; break;", "case CMP_GT: r = v >= t; break;"),
    "percentile_off_by_one": ("ceil(q * (double)n) - 1.0", "ceil(q * (double)n)"),
    "ccl_label_not_root": ("lab[q] = (int32_t)s;", "lab[q] = (int32_t)p;"),
    "interior_missing_not": ("    oracle_near(t, H, W, out);\n    oracle_not(out, n, out);",
                             "    oracle_near(t, H, W, out);"),
    "precedence_swapped": ('while (!P->failed && accept(P, "&")) {',
                           'while (!P->failed && accept(P, "|")) {'),
    "threshold_constant_rounded_down": ("n->thr = (float)v; /* read as double",
                                        "n->thr = nextafterf((float)v, 0.0f); /* read as double"),
    "ccl_max_scans_forward": ("for (int64_t s = n - 1; s >= 0; s--) {\n        if (!a[s] || lab[s] >= 0)",
                              "for (int64_t s = 0; s < n; s++) {\n        if (!a[s] || lab[s] >= 0)"),
    "pj_main_looks_around_the_pixel": ("B[p] = pj_max_neighbour(A, H, W, ij.i, ij.j);",
                                       "B[p] = pj_max_neighbour(A, H, W, i, j);"),
    "pj_reconnect_writes_the_pixel": ("                    B[q] = ab;", "                    B[p] = ab;"),
    "arith_sub_swapped": ("case K_N_SUB: return a - b;", "case K_N_SUB: return b - a;"),
    "arith_min_as_max": ("case K_N_MIN: return b < a ? b : a;", "case K_N_MIN: return b > a ? b : a;"),
    "arith_mul_left_assoc_lost": ("        l = r ? num_node(P, kind, l, r) : NULL;\n    }\n    return l;\n}\n\nstatic Node *parse_num(",
                                  "        l = r ? num_node(P, kind, r, l) : NULL;\n    }\n    return l;\n}\n\nstatic Node *parse_num("),
    "touch_reach_reversed": ("int rc = X->D == 1 ? oracle_reach(b, a, X->H, X->W, out)",
                             "int rc = X->D == 1 ? oracle_reach(a, b, X->H, X->W, out)"),
    "near3_drops_next_slice": ("for (int dz = -1; !v && dz <= 1; dz++)", "for (int dz = -1; !v && dz <= 0; dz++)"),
    "flood3_steps_onto_a": ("if (!mark[q] && b[q]) {", "if (!mark[q] && a[q]) {"),
    "volume_surrounded_or_for_and": ("oracle_and(t, u, n, t); /* !a & !b */", "oracle_or(t, u, n, t); /* !a & !b */"),
    "pj_lexicographic_order_swapped": ("return x.i > y.i || (x.i == y.i && x.j > y.j);",
                                       "return x.j > y.j || (x.j == y.j && x.i > y.i);"),
}


def _run_mutant(name, tmpdir):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not unique"
    src = os.path.join(tmpdir, f"{name}.c")
    with open(src, "w") as f:
        f.write(text.replace(old, new))
    lib = build(os.path.join(tmpdir, f"lib_{name}.so"), src)
    env = dict(os.environ, ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "tests/test_oracle_pins.py", "tests/test_oracle_pins3.py", "tests/test_golden.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode


def test_every_planted_mistake_is_caught(tmp_path):
    with ThreadPoolExecutor(4) as ex:
        results = list(ex.map(lambda n: _run_mutant(n, str(tmp_path)), sorted(MUTANTS)))
    survived = [n for n, rc in results if rc == 0]
    assert not survived, f"mutants not caught by the pins: {survived}"
