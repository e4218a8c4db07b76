"""The paper's own labelling (Sect. 3, Alg. CCL) on the GPU against the
oracle's step-by-step run of the same algorithm: identical labels (the
largest row-major index of each component) and the same number of main
iterations; reachability through it (VLG_TUNE_CCL_ALGO) against the oracle's
formula results; the round cap turning into VLG_ENOCONV."""
import numpy as np
import pytest

import oracle
import paper_2010_07284_amd as vlg
from synth import formulas, images
from tests.gpu_util import assert_same, gpu_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return vlg.create()


def pj_labels(ctx, mask, k):
    import torch
    H, W = mask.shape
    words = torch.from_numpy(vlg.pack(mask)).cuda()
    lab, st = vlg.ccl_labels_pj(ctx, words, H, W, k)
    vlg.sync(ctx)
    return lab.cpu().numpy(), st


@pytest.mark.parametrize("k", [1, 8, 16])
@pytest.mark.parametrize("h,w", [(1, 1), (1, 300), (300, 1), (2, 2), (33, 129), (65, 257), (200, 333)])
@pytest.mark.parametrize("p", [0.3, 0.5, 0.7])
def test_random_masks_labels_and_iterations(ctx, h, w, p, k):
    rng = np.random.default_rng(h * 31 + w + int(p * 10) + k)
    m = (rng.random((h, w)) < p).astype(np.uint8)
    want, iters = oracle.ccl_pj(m, k=k)
    got, st = pj_labels(ctx, m, k)
    assert np.array_equal(got, want)
    assert st["main_iterations"] == iters and st["rounds"] == iters // k
    assert st["launches"] == 1 + st["rounds"] * (k + 4) + 1


@pytest.mark.parametrize("k", [1, 8, 16])
def test_mazes_and_special_masks(ctx, k):
    cases = [images.serpentine_maze(41, 70), images.serpentine_maze(64, 129), np.zeros((50, 77), np.uint8),
             np.ones((50, 77), np.uint8), np.eye(97, dtype=np.uint8)[::-1].copy()]
    yy, xx = np.mgrid[:90, :130]
    cases += [((yy + xx) % 2 == 0), (xx % 3 == 0), ((yy // 2 + xx // 2) % 2 == 0)]
    for m in cases:
        m = np.ascontiguousarray(m, dtype=np.uint8)
        want, iters = oracle.ccl_pj(m, k=k)
        got, st = pj_labels(ctx, m, k)
        assert np.array_equal(got, want)
        assert st["main_iterations"] == iters


def test_2048_image_iterations_match_the_oracle(ctx):
    # a 2048 x 2048 labelling, the size of the paper's Fig. cc-movie (whose
    # test image is not available): thresholded smooth noise, reconnect
    # every 8 main iterations as in the figure
    img = images.plain_image(7, 2048)[0]
    m = (img > np.float32(0.5)).astype(np.uint8)
    want, iters = oracle.ccl_pj(m, k=8)
    got, st = pj_labels(ctx, m, 8)
    assert np.array_equal(got, want) and st["main_iterations"] == iters


def test_loop_cap_gives_enoconv(ctx):
    import torch
    m = images.serpentine_maze(41, 70).astype(np.uint8)
    _, iters = oracle.ccl_pj(m, k=1)
    assert iters > 1
    words = torch.from_numpy(vlg.pack(m)).cuda()
    vlg.set_loop_cap(ctx, 1)  # one round only
    try:
        with pytest.raises(vlg.VlgError) as e:
            vlg.ccl_labels_pj(ctx, words, *m.shape, 1)
        assert e.value.code == -6
    finally:
        vlg.set_loop_cap(ctx, 0)
    got, st = pj_labels(ctx, m, 1)
    assert np.array_equal(got, oracle.ccl_max(m)) and st["main_iterations"] == iters


@pytest.mark.parametrize("mode", ["perop", "fused", "graph"])
@pytest.mark.parametrize("k", [2, 16])
def test_reach_through_pointer_jumping(ctx, mode, k):
    vlg.set_tunable(ctx, "ccl_algo", vlg.CCL_POINTER_JUMPING)
    vlg.set_tunable(ctx, "pj_reconnect", k)
    vlg.ccl_counters(ctx)  # reading resets them
    try:
        img = images.plain_image(1, 256)
        src = formulas.PLAIN_FORMULA
        assert_same(src, img, gpu_run(ctx, src, img, mode=mode), tag=f"plain {mode} k={k}")
        rng = np.random.default_rng(5)
        img2 = rng.random((2, 131, 203)).astype(np.float32)
        from tests.test_gpu_parity import ops_src
        src2 = ops_src(rng)
        assert_same(src2, img2, gpu_run(ctx, src2, img2, mode=mode), tag=f"ops {mode} k={k}")
        c = vlg.ccl_counters(ctx)
        assert c["pj_labellings"] > 0 and c["pj_main_iterations"] % k == 0
    finally:
        vlg.set_tunable(ctx, "ccl_algo", 0)
        vlg.set_tunable(ctx, "pj_reconnect", 0)


def test_reach_through_pointer_jumping_maze(ctx):
    # the labelling reuse path (several seed sets on one labelling) and a
    # corridor that needs many reconnect rounds
    vlg.set_tunable(ctx, "ccl_algo", vlg.CCL_POINTER_JUMPING)
    try:
        img = images.ellipse_maze_image(2, 256)
        src = formulas.ellipse_dag(2)
        assert_same(src, img, gpu_run(ctx, src, img, mode="fused"), tag="ellipse maze 256")
    finally:
        vlg.set_tunable(ctx, "ccl_algo", 0)
