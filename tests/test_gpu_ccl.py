"""Connected-component labelling kernels against the oracle's labelling:
canonical labels (smallest row-major index per component) bit for bit, and
repeated runs give identical labels."""
import numpy as np
import pytest

import oracle
import paper_2010_07284_amd as vlg
from synth import images

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return vlg.create()


def gpu_labels(ctx, mask, tbh=0):
    import torch
    vlg.set_tunable(ctx, "ccl_tile_rows", tbh)
    H, W = mask.shape
    words = torch.from_numpy(vlg.pack(mask)).cuda()
    lab = vlg.ccl_labels(ctx, words, H, W)
    vlg.sync(ctx)
    return lab.cpu().numpy()


@pytest.mark.parametrize("h,w", [(1, 1), (1, 300), (300, 1), (2, 2), (33, 129), (64, 128), (65, 257),
                                 (200, 333), (513, 1029)])
@pytest.mark.parametrize("p", [0.3, 0.45, 0.6])
def test_random_masks(ctx, h, w, p):
    rng = np.random.default_rng(h * 7 + w + int(p * 10))
    m = (rng.random((h, w)) < p).astype(np.uint8)
    assert np.array_equal(gpu_labels(ctx, m), oracle.ccl(m))


@pytest.mark.parametrize("tbh", [8, 16, 32])
@pytest.mark.parametrize("shape", [(101, 77), (1024, 1024), (2048, 4096)])
def test_serpentine_maze(ctx, shape, tbh):
    m = images.serpentine_maze(*shape).astype(np.uint8)
    lab = gpu_labels(ctx, m, tbh)
    assert np.all(lab[m > 0] == 0) and np.all(lab[m == 0] == -1)


@pytest.mark.parametrize("tbh", [8, 32])
@pytest.mark.parametrize("h,w", [(17, 129), (65, 257), (333, 1029)])
def test_tile_heights(ctx, h, w, tbh):
    rng = np.random.default_rng(h + w + tbh)
    for p in (0.35, 0.55):
        m = (rng.random((h, w)) < p).astype(np.uint8)
        assert np.array_equal(gpu_labels(ctx, m, tbh), oracle.ccl(m))


def test_checkerboard_and_stripes(ctx):
    yy, xx = np.mgrid[:300, :517]
    for m in [((yy + xx) % 2).astype(np.uint8), (xx % 2).astype(np.uint8), (yy % 3 == 0).astype(np.uint8),
              ((yy // 2 + xx // 2) % 2).astype(np.uint8)]:
        assert np.array_equal(gpu_labels(ctx, m), oracle.ccl(m))


def test_repeatable(ctx):
    rng = np.random.default_rng(0)
    m = (rng.random((777, 1111)) < 0.5).astype(np.uint8)
    mz = images.serpentine_maze(640, 900).astype(np.uint8)
    for mask in (m, mz):
        first = gpu_labels(ctx, mask)
        for _ in range(20):
            assert np.array_equal(gpu_labels(ctx, mask), first)
