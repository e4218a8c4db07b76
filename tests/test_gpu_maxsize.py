"""The largest image the boundary accepts (H*W < 2^31): 46080 x 46080 pixels,
three float32 channels generated in device memory.  Sampled rows are checked
against the oracle on 3-row strips (N of row y depends on rows y-1..y+1
only); whole-image properties are checked on the device."""
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
    atom, near, reach = vlg.check_all(ctx, f, im)
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
        strip = img[0:1, lo:hi].cpu().numpy()
        want = oracle.run('let A = intensity(img, 0) >. 0.5\noutput "atom" A\noutput "near" near(A)\n', strip)
        k = r - lo
        got_atom = vlg.unpack(atom[r:r + 1], 1, SIDE)
        got_near = vlg.unpack(near[r:r + 1], 1, SIDE)
        assert_same("", None, [got_atom, got_near], want=[want[0][k:k + 1], want[1][k:k + 1]], tag=f"row {r}")
    del img, im, atom, near, reach
    torch.cuda.empty_cache()
