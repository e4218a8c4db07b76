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


@pytest.fixture(scope="module")
def ctx():
    return vlg.create()


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
