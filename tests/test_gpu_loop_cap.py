"""Bounded device loops: every loop of the labelling kernels stops at a
host-set iteration cap.  With the cap forced to 1 on the serpentine maze (the
labelling's worst case: one 1-pixel corridor through every tile) the kernels
still exit normally and the next synchronising call reports VLG_ENOCONV; with
the default cap the same context gives the oracle's masks again."""
import numpy as np
import pytest

import oracle
import paper_2010_07284_amd as vlg
from synth import images

pytestmark = pytest.mark.gpu

SRC = """
let M = intensity(img, 1) >. 0.5
let S = intensity(img, 2) >. 0.5
output "reach" reach(S, M)
output "grow" grow(S, M)
output "surr" surrounded(!M, S)
"""


@pytest.fixture(scope="module")
def maze():
    return images.ellipse_maze_image(2, 1024)


def _expect_enoconv(fn):
    with pytest.raises(vlg.VlgError) as e:
        fn()
    assert e.value.code == -6, str(e.value)


@pytest.mark.parametrize("mode", ["perop", "fused", "graph"])
def test_cap_one_reports_enoconv_then_recovers(maze, mode):
    import torch
    ctx = vlg.create()
    vlg.set_mode(ctx, mode)
    im = vlg.load_image(ctx, torch.from_numpy(maze).cuda())
    f = vlg.compile_formula(ctx, SRC)
    want = oracle.run(SRC, maze)
    vlg.set_loop_cap(ctx, 1)
    vlg.check_all(ctx, f, im)
    _expect_enoconv(lambda: vlg.sync(ctx))
    # the condition is cleared by the report
    vlg.sync(ctx)
    # host outputs synchronise inside the call and report it there
    host = [torch.zeros((1024, 16), dtype=torch.int64) for _ in range(3)]
    _expect_enoconv(lambda: vlg.check_all(ctx, f, im, outs=host))
    vlg.set_loop_cap(ctx, 0)
    outs = vlg.check_all(ctx, f, im)
    vlg.sync(ctx)
    for k, (o, w) in enumerate(zip(outs, want)):
        assert np.array_equal(vlg.unpack(o, 1024, 1024), w), k


def test_cap_one_batched(maze):
    import torch
    ctx = vlg.create()
    ims = [vlg.load_image(ctx, torch.from_numpy(maze).cuda()),
           vlg.load_image(ctx, torch.from_numpy(np.ascontiguousarray(maze[:, :700, :513])).cuda())]
    f = vlg.compile_formula(ctx, SRC)
    vlg.set_loop_cap(ctx, 1)
    vlg.check_batch(ctx, f, ims)
    _expect_enoconv(lambda: vlg.sync(ctx))
    vlg.set_loop_cap(ctx, 0)
    outs = vlg.check_batch(ctx, f, ims)
    vlg.sync(ctx)
    for img, row in zip([maze, np.ascontiguousarray(maze[:, :700, :513])], outs):
        want = oracle.run(SRC, img)
        C, H, W = img.shape
        for k, (o, w) in enumerate(zip(row, want)):
            assert np.array_equal(vlg.unpack(o, H, W), w), k


def test_cap_validation():
    ctx = vlg.create()
    with pytest.raises(vlg.VlgError) as e:
        vlg.set_loop_cap(ctx, -1)
    assert e.value.code == -1
    vlg.set_loop_cap(ctx, 5)
    vlg.set_loop_cap(ctx, 0)
    # labellings run together: 1, 2, 4 or 8 lanes, nothing else
    for lanes in (1, 2, 4, 8):
        vlg.set_tunable(ctx, "ccl_lanes", lanes)
    for lanes in (3, 16, -1):
        with pytest.raises(vlg.VlgError) as e:
            vlg.set_tunable(ctx, "ccl_lanes", lanes)
        assert e.value.code == -1
    vlg.set_tunable(ctx, "ccl_lanes", 0)
