"""The largest image the boundary accepts (H*W < 2^31): 46080 x 46080 pixels,
three float32 channels generated in device memory.  Sampled rows are checked
against the oracle on 3-row strips (N of row y depends on rows y-1..y+1
only); whole-image properties are checked on the device.  At this size every
atom and Boolean launch streams more than the last-level cache holds, so
these are the launches that read with the non-temporal hint (the connectives
both batched, in graph mode, and one per launch, in per-op mode)."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import assert_same

pytestmark = pytest.mark.gpu

SIDE = 46080

SRC = """
let A = intensity(img, 0) >. 0.5
let M = intensity(img, 1) >. 0.5
let S = intensity(img, 2) >. 0.5
output "atom" A
output "near" near(A)
output "reach" reach(S, M)
output "andnot" M & !A
output "or" A | S
"""
PIXELWISE = """
let A = intensity(img, 0) >. 0.5
let M = intensity(img, 1) >. 0.5
let S = intensity(img, 2) >. 0.5
output "atom" A
output "near" near(A)
output "andnot" M & !A
output "or" A | S
"""


def test_max_size_sampled_rows_and_properties():
    import torch
    import paper_2010_07284_amd as vlg
    assert SIDE * SIDE < 2**31
    dev = "cuda:0"
    g = torch.Generator(device=dev)
    g.manual_seed(12345)
    img = torch.empty((3, SIDE, SIDE), dtype=torch.float32, device=dev)
    img[0] = torch.rand((SIDE, SIDE), generator=g, device=dev)
    # serpentine maze: even rows open; odd row y open at x = W-1 if y % 4 == 1, at x = 0 if y % 4 == 3
    img[1].zero_()
    img[1, 0::2, :] = 1.0
    img[1, 1::4, SIDE - 1] = 1.0
    img[1, 3::4, 0] = 1.0
    img[2].zero_()
    img[2, 0, 0] = 1.0
    ctx = vlg.create()
    im = vlg.load_image(ctx, img)
    f = vlg.compile_formula(ctx, SRC)
    vlg.set_mode(ctx, "graph")
    atom, near, reach, andnot, orr = vlg.check_all(ctx, f, im)
    vlg.sync(ctx)
    torch.cuda.synchronize()
    # the pixel-wise outputs once more, one launch per operator
    vlg.set_mode(ctx, "perop")
    fp = vlg.compile_formula(ctx, PIXELWISE)
    per_op = vlg.check_all(ctx, fp, im)
    vlg.sync(ctx)
    torch.cuda.synchronize()

    # whole image: A is inside N(A); the maze is one component through the seed
    # and every pixel is in N(maze), so reach is all ones (W is a multiple of 64)
    assert bool(torch.all((atom & ~near) == 0))
    assert bool(torch.all(reach == -1))

    # sampled rows against the oracle
    rng = np.random.default_rng(7)
    rows = sorted({0, 1, SIDE // 2, SIDE - 2, SIDE - 1, *rng.integers(2, SIDE - 2, 8).tolist()})
    for r in rows:
        lo, hi = max(0, r - 1), min(SIDE, r + 2)
        strip = img[:, lo:hi].cpu().numpy()
        want = oracle.run(PIXELWISE, strip)
        k = r - lo
        want = [w[k:k + 1] for w in want]
        got = [vlg.unpack(o[r:r + 1], 1, SIDE) for o in (atom, near, andnot, orr)]
        assert_same("", None, got, want=want, tag=f"row {r}, graph")
        got = [vlg.unpack(o[r:r + 1], 1, SIDE) for o in per_op]
        assert_same("", None, got, want=want, tag=f"row {r}, per-op")
    del img, im, atom, near, reach, andnot, orr, per_op
    torch.cuda.empty_cache()
