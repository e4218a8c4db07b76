"""Arithmetic atoms (the tool's built-in arithmetic, Sect. 3) and touch
(contact between regions, Sect. 2) on the GPU against the oracle, bit for
bit: float32, uint8 and uint16 pixels, every executor, ragged widths,
percentile leaves inside expressions, and the batched executor."""
import numpy as np
import pytest

import oracle
import paper_2010_07284_amd as vlg
from synth import formulas
from tests.gpu_util import assert_same, gpu_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["compiled", "interpreter"])
def ctx(request):
    """Every test runs with both kernels of arithmetic atoms: the programs
    compiled into a straight-line kernel, and the interpreter."""
    c = vlg.create()
    vlg.set_tunable(c, "arith_kernel",
                    vlg.ARITH_COMPILED if request.param == "compiled" else vlg.ARITH_INTERPRETER)
    return c


def arith_src(rng):
    t = rng.uniform(0.25, 0.75, 4)
    return formulas.ARITH_FORMULA.format(t0=t[0], t1=t[1], t2=t[2], t3=t[3])


@pytest.mark.parametrize("mode", ["perop", "fused", "graph"])
@pytest.mark.parametrize("h,w", [(1, 1), (7, 65), (130, 257), (513, 1000)])
def test_float_images(ctx, mode, h, w):
    rng = np.random.default_rng(h * 3 + w)
    img = rng.random((2, h, w)).astype(np.float32)
    src = arith_src(rng)
    assert_same(src, img, gpu_run(ctx, src, img, mode=mode), tag=f"{mode} {h}x{w}")


@pytest.mark.parametrize("dt", [np.uint8, np.uint16])
@pytest.mark.parametrize("mode", ["fused", "graph"])
def test_integer_images(ctx, dt, mode):
    rng = np.random.default_rng(7)
    img = rng.integers(0, 3, (2, 200, 301)).astype(dt)
    src = arith_src(rng)
    assert_same(src, img, gpu_run(ctx, src, img, mode=mode), tag=f"{dt.__name__} {mode}")
    big = rng.integers(0, np.iinfo(dt).max + 1, (2, 97, 130)).astype(dt)
    src2 = ('output "o" intensity(img, 0) * 2 - intensity(img, 1) >. percentile(img, 0, 0.5)\n'
            'output "p" abs(intensity(img, 0) - intensity(img, 1)) / 7 <=. 3\n')
    assert_same(src2, big, gpu_run(ctx, src2, big, mode=mode), tag=f"{dt.__name__} {mode} wide range")


def test_division_special_values(ctx):
    img = np.zeros((2, 3, 70), np.float32)
    img[0, 0, :] = 1.0
    img[0, 1, :] = -1.0
    img[1, 2, :] = 2.0
    src = ('output "a" intensity(img, 0) / intensity(img, 1) >. 0\n'
           'output "b" intensity(img, 0) / intensity(img, 1) <=. 0\n'
           'output "c" intensity(img, 0) / intensity(img, 1) >=. intensity(img, 0) / intensity(img, 1)\n')
    assert_same(src, img, gpu_run(ctx, src, img, mode="fused"), tag="division")


def test_batch_with_arithmetic(ctx):
    import torch
    rng = np.random.default_rng(9)
    src = arith_src(rng)
    f = vlg.compile_formula(ctx, src)
    vlg.set_mode(ctx, "graph")
    imgs = [rng.random((2, int(h), int(w))).astype(np.float32)
            for h, w in rng.integers(16, 400, (6, 2))]
    ims = [vlg.load_image(ctx, x) for x in imgs]
    outs = vlg.check_batch(ctx, f, ims)
    vlg.sync(ctx)
    for x, row in zip(imgs, outs):
        got = [vlg.unpack(o, x.shape[1], x.shape[2]) for o in row]
        assert_same(src, x, got, tag=f"batch {x.shape}")
    del torch


def full_group_src():
    """Eleven arithmetic atoms over eight channels: stacks eight deep, every
    operator, percentiles and constants; more programs and instructions than
    one launch takes, so the fused schedule splits them over launches."""
    I = [f"intensity(img, {c})" for c in range(8)]
    deep = f"{I[0]} + ({I[1]} * ({I[2]} - ({I[3]} / ({I[4]} + ({I[5]} - ({I[6]} * {I[7]}))))))"
    atoms = [
        f"{deep} >. 0.3",
        f"abs({I[0]} - {I[7]}) <=. min({I[3]}, 0.5)",
        f"max({I[1]}, {I[2]}) / ({I[4]} + 2) >=. percentile(img, 5, 0.3)",
        f"-{I[6]} * 3 <. {I[2]} - 1",
        f"{I[3]} * {I[3]} - {I[4]} >. {I[5]} / 3",
        f"min(max({I[0]}, {I[1]}), {I[2]}) <. max(min({I[3]}, {I[4]}), {I[5]})",
        f"({I[6]} - {I[7]}) / ({I[6]} + {I[7]}) >=. 0.1",
        f"abs(-{I[1]}) + abs({I[2]} - 0.25) <=. 1.5",
        f"{I[4]} - percentile(img, 4, 0.7) >. {I[0]} * 0.125",
        f"{deep} <=. {I[0]} * 2",
        f"-({I[5]} - {I[3]}) >. -0.2",
    ]
    return "".join(f'output "a{k}" {a}\n' for k, a in enumerate(atoms))


@pytest.mark.parametrize("mode", ["perop", "fused", "graph"])
def test_full_groups(ctx, mode):
    rng = np.random.default_rng(11)
    img = (rng.random((8, 67, 203)) * 2 - 0.5).astype(np.float32)
    src = full_group_src()
    assert_same(src, img, gpu_run(ctx, src, img, mode=mode), tag=f"full groups {mode}")
    if mode == "fused":
        plan = vlg.formula_plan(vlg.compile_formula(ctx, src), "fused", 1)
        groups = {st["group"] for st in plan["steps"] if st["kind"] == "arith"}
        assert len([g for g in groups if g >= 0]) >= 2

