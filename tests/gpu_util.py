"""Helpers shared by the GPU tests: run formulas through the library (C ABI)
and compare with the oracle bit for bit."""
import numpy as np

import oracle
import paper_2010_07284_amd as vlg


def gpu_run(ctx, src, img, mode="graph", fmt="packed", host=False):
    """All outputs of `src` on `img` (numpy (C,H,W)) as numpy uint8 masks."""
    import torch
    vlg.set_mode(ctx, mode)
    im = vlg.load_image(ctx, img)
    f = vlg.compile_formula(ctx, src)
    C, H, W = im.shape
    n = vlg.formula_info(f)["outputs"]
    if host:
        if fmt == "packed":
            outs = [torch.zeros((H, (W + 63) // 64), dtype=torch.int64) for _ in range(n)]
        else:
            outs = [torch.zeros((H, W), dtype=torch.uint8) for _ in range(n)]
        vlg.check_all(ctx, f, im, outs=outs, fmt=fmt)
    else:
        outs = vlg.check_all(ctx, f, im, fmt=fmt)
        vlg.sync(ctx)
    if fmt == "packed":
        return [vlg.unpack(o, H, W) for o in outs]
    return [o.cpu().numpy() for o in outs]


def assert_same(src, img, got, want=None, tag=""):
    if want is None:
        want = oracle.run(src, img)
    assert len(got) == len(want)
    for k, (g, w) in enumerate(zip(got, want)):
        if not np.array_equal(g, w):
            diff = np.argwhere(g != w)
            raise AssertionError(f"{tag} output {k}: {len(diff)} pixels differ, first at {diff[:5].tolist()}")
