"""Schedules checked on the CPU: every step of the per-operator and fused
plans (vlg_formula_plan), including fused segments at every halo cap, is
executed by the CPU emulator of tests/plan_emulator.py on the packed layout,
and every output must equal the oracle's mask.  This pins the schedule
builder, the slot allocator and the segment programs (register allocation,
operand complements, halo depth, stores) independently of the GPU."""
import numpy as np
import pytest

import oracle
import paper_2010_07284_amd as vlg
from synth import formulas, images
from tests import plan_emulator as E

OPS = """
let A = intensity(img, 0) >. {t0}
let B = intensity(img, 1) <=. {t1}
let C = intensity(img, 0) >=. {t2}
let D = intensity(img, 1) <. {t3}
output "not" !A
output "and" A & B
output "or" A | !B
output "near" near(A)
output "near_not" near(!B)
output "interior" interior(A | C)
output "reach" reach(A & !C, B | C)
output "reach_not" reach(!B, !A)
output "surrounded" surrounded(A | B, C)
output "grow" grow(A, !B)
output "const" true & near(false) | !true
output "chain" near(interior(reach(D, A) | grow(C, B))) & !surrounded(B, D)
output "deep" near(near(near(near(near(A) & B) | C) & !D) | interior(interior(B)))
"""


def cases():
    out = []
    for seed in range(5):
        rng = np.random.default_rng(100 + seed)
        h, w = int(rng.integers(1, 260)), int(rng.integers(1, 260))
        out.append((f"random{seed}", formulas.random_dag(seed, n_nodes=60, n_reach=6, channels=2),
                    rng.random((2, h, w)).astype(np.float32)))
    for h, w in [(1, 1), (3, 65), (64, 127), (97, 301)]:
        rng = np.random.default_rng(h * 7 + w)
        t = rng.uniform(0.25, 0.75, 4)
        out.append((f"ops{h}x{w}", OPS.format(t0=t[0], t1=t[1], t2=t[2], t3=t[3]),
                    rng.random((2, h, w)).astype(np.float32)))
    for h, w in [(5, 70), (61, 130)]:
        rng = np.random.default_rng(h + w)
        t = rng.uniform(0.25, 0.75, 4)
        src = formulas.ARITH_FORMULA.format(t0=t[0], t1=t[1], t2=t[2], t3=t[3])
        out.append((f"arith{h}x{w}", src, rng.random((2, h, w)).astype(np.float32)))
        out.append((f"arith_u16_{h}x{w}", src, rng.integers(0, 3, (2, h, w)).astype(np.uint16)))
    out.append(("plain", formulas.PLAIN_FORMULA, images.plain_image(1, 256)))
    out.append(("chain", formulas.chain_dag(3, n_chain=240, n_reach=12), images.random_mask_image(3, 190)))
    rng = np.random.default_rng(4)
    out.append(("segmentation", formulas.segmentation_dag(4), images.phantom_image(rng, 150, 203)))
    return out


CASES = cases()


@pytest.mark.parametrize("name,src,img", CASES, ids=[c[0] for c in CASES])
def test_plans_against_oracle(name, src, img):
    want = oracle.run(src, img)
    f = vlg.compile_formula(None, src)
    for mode, halo in [("perop", 1), ("fused", 1), ("fused", 2), ("fused", 4), ("fused", 8), ("fused", 16)]:
        plan = vlg.formula_plan(f, mode, halo)
        got = E.Emulator(plan, img).run()
        for k, (g, w) in enumerate(zip(got, want)):
            assert np.array_equal(g, w), f"{name} {mode} halo {halo}: output {k} differs in {int((g != w).sum())} px"


def test_segments_form_on_the_chain():
    f = vlg.compile_formula(None, formulas.chain_dag(3))
    plan = vlg.formula_plan(f, "fused", 8)
    assert len(plan["segments"]) >= 400
    assert all(s["halo"] <= 8 and s["nregs"] <= 16 for s in plan["segments"])
    assert len(plan["steps"]) <= 2500
    assert len(vlg.formula_plan(f, "fused", 1)["segments"]) == 0
