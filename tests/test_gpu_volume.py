"""Volumes (the logic on 3-D images: N over 26 neighbours, 26-connected
paths) on the GPU against the oracle's volume evaluation, bit for bit:
operators and derived operators on random volumes of several shapes
(ragged widths, one-slice volumes, single rows), every executor, uint8 and
float32 voxels; the voxel labelling against the oracle's 26-connected
labels; the loop cap turning into VLG_ENOCONV."""
import numpy as np
import pytest

import oracle
import paper_2010_07284_amd as vlg
from synth import formulas

pytestmark = pytest.mark.gpu

VOL_FORMULA = """
let A = intensity(img, 0) >. {t0}
let B = intensity(img, 1) <=. {t1}
let C = intensity(img, 0) + intensity(img, 1) <. {t2}
output "near" near(A)
output "interior" interior(A | C)
output "reach" reach(A & !C, B | C)
output "surrounded" surrounded(A | B, C)
output "grow" grow(A, !B)
output "touch" touch(B, A)
output "chain" near(interior(reach(C, A) | grow(C, B))) & !surrounded(B, A)
output "pct" intensity(img, 1) >. percentile(img, 1, 0.8)
"""


@pytest.fixture(scope="module")
def ctx():
    return vlg.create()


def run_vol(ctx, src, vol, mode):
    vlg.set_mode(ctx, mode)
    im = vlg.load_volume(ctx, vol)
    f = vlg.compile_formula(ctx, src)
    C, D, H, W = vol.shape
    outs = vlg.check_all(ctx, f, im)
    vlg.sync(ctx)
    return [vlg.unpack(o, D * H, W).reshape(D, H, W) for o in outs]


def check(src, vol, got, tag):
    want = oracle.run3(src, vol)
    for k, (g, w) in enumerate(zip(got, want)):
        if not np.array_equal(g, w):
            raise AssertionError(f"{tag} output {k}: {int((g != w).sum())} voxels differ")


@pytest.mark.parametrize("mode", ["perop", "fused", "graph"])
@pytest.mark.parametrize("shape", [(2, 5, 70), (5, 33, 129), (16, 40, 64), (3, 1, 1), (1, 40, 50), (7, 1, 200)])
def test_volume_formula(ctx, mode, shape):
    rng = np.random.default_rng(sum(shape))
    vol = rng.random((2, *shape)).astype(np.float32)
    t = rng.uniform(0.3, 0.7, 3)
    src = VOL_FORMULA.format(t0=t[0], t1=t[1], t2=2 * t[2])
    check(src, vol, run_vol(ctx, src, vol, mode), f"{mode} {shape}")


def test_volume_uint8_and_arithmetic(ctx):
    rng = np.random.default_rng(5)
    vol = rng.integers(0, 256, (2, 9, 31, 77)).astype(np.uint8)
    src = VOL_FORMULA.format(t0=170, t1=90, t2=250) + 'output "ar" abs(intensity(img, 0) - intensity(img, 1)) >. 60\n'
    check(src, vol, run_vol(ctx, src, vol, "graph"), "uint8")


def test_volume_labels(ctx):
    import torch
    rng = np.random.default_rng(6)
    for shape in [(1, 1, 1), (3, 17, 65), (12, 30, 130), (40, 64, 64)]:
        for p in (0.15, 0.3, 0.5):
            m = (rng.random(shape) < p).astype(np.uint8)
            D, H, W = shape
            words = torch.from_numpy(vlg.pack(m.reshape(D * H, W))).cuda()
            lab = vlg.ccl_labels3(ctx, words, D, H, W)
            vlg.sync(ctx)
            assert np.array_equal(lab.cpu().numpy(), oracle.ccl3(m)), (shape, p)


def test_volume_corridor_across_slices(ctx):
    # a 1-voxel corridor that alternates direction row by row and slice by
    # slice: one component through every slice, reach from one end
    D, H, W = 6, 9, 70
    m = np.zeros((D, H, W), np.uint8)
    for z in range(D):
        m[z, 0::2, :] = 1
        for y in range(1, H, 2):
            m[z, y, W - 1 if (y // 2) % 2 == 0 else 0] = 1
    seed = np.zeros_like(m)
    seed[0, 0, 0] = 1
    vol = np.stack([m, seed]).astype(np.float32)
    src = 'output "r" reach(intensity(img, 1) >. 0.5, intensity(img, 0) >. 0.5)\noutput "g" grow(intensity(img, 1) >. 0.5, intensity(img, 0) >. 0.5)'
    check(src, vol, run_vol(ctx, src, vol, "graph"), "corridor")


def test_volume_loop_cap(ctx):
    rng = np.random.default_rng(8)
    vol = rng.random((2, 8, 40, 90)).astype(np.float32)
    src = 'output "r" reach(intensity(img, 0) >. 0.8, intensity(img, 1) >. 0.4)'
    vlg.set_loop_cap(ctx, 1)
    try:
        with pytest.raises(vlg.VlgError) as e:
            run_vol(ctx, src, vol, "fused")
        assert e.value.code == -6
    finally:
        vlg.set_loop_cap(ctx, 0)
    check(src, vol, run_vol(ctx, src, vol, "fused"), "after the cap")


def test_volumes_are_not_batched(ctx):
    vol = np.zeros((1, 2, 3, 4), np.float32)
    im = vlg.load_volume(ctx, vol)
    f = vlg.compile_formula(ctx, formulas.PLAIN_FORMULA)
    with pytest.raises(vlg.VlgError) as e:
        vlg.check_batch(ctx, f, [im])
    assert e.value.code == -1
