"""The allocation-free labelling entry point (vlg_ccl_labels_noalloc) against
vlg_ccl_labels through the C ABI: identical labels bit for bit on two calls in
a row (the second on a smaller image, so stale contents of the shared device
array from the first call must not leak into it), the canonical labels of the
oracle on the same masks, and a clear VLG_ESHAPE for an image whose labelling
arrays exceed the fixed array."""
import numpy as np
import pytest

import oracle
import paper_2010_07284_amd as vlg
from synth import images

pytestmark = pytest.mark.gpu


def _labels(ctx, mask, noalloc):
    import torch
    H, W = mask.shape
    words = torch.from_numpy(vlg.pack(mask)).cuda()
    out = torch.full((H, W), -7, dtype=torch.int32, device="cuda")
    if noalloc:
        vlg.ccl_labels_noalloc(ctx, words, H, W, out)
    else:
        vlg.ccl_labels(ctx, words, H, W, out)
    vlg.sync(ctx)
    return out.cpu().numpy()


def test_noalloc_matches_allocating_entry_point_twice():
    ctx = vlg.create()
    rng = np.random.default_rng(11)
    big = (rng.random((2048, 3000)) < 0.55).astype(np.uint8)
    small = images.serpentine_maze(333, 517).astype(np.uint8)
    small[::7, ::5] = 1  # extra contacts between the corridor rows
    for mask in (big, small):
        a = _labels(ctx, mask, noalloc=True)
        b = _labels(ctx, mask, noalloc=False)
        assert np.array_equal(a, b)
        assert np.array_equal(a, oracle.ccl(mask))


def test_noalloc_largest_and_too_large():
    import torch
    ctx = vlg.create()
    rng = np.random.default_rng(12)
    m = (rng.random((4096, 4096)) < 0.5).astype(np.uint8)
    a = _labels(ctx, m, noalloc=True)
    assert np.array_equal(a, _labels(ctx, m, noalloc=False))
    H, W = 4096, 4608  # 9 B per 2x2 block: beyond the 40 MiB array
    words = torch.zeros((H, (W + 63) // 64), dtype=torch.int64, device="cuda")
    out = torch.zeros((H, W), dtype=torch.int32, device="cuda")
    with pytest.raises(vlg.VlgError) as e:
        vlg.ccl_labels_noalloc(ctx, words, H, W, out)
    assert e.value.code == -3 and "fixed device array" in str(e.value)
    # the context is still usable after the rejection
    small = (rng.random((100, 130)) < 0.5).astype(np.uint8)
    assert np.array_equal(_labels(ctx, small, noalloc=True), oracle.ccl(small))
