"""Labelling stress patterns against the oracle's canonical labels, at every
tile height: patterns that give every 2x2 block its own run (the most union
pairs a tile can have), components that cross every tile border, diagonal
8-connected chains and a spiral (one component folded through every tile)."""
import numpy as np
import pytest

import oracle
import paper_2010_07284_amd as vlg

pytestmark = pytest.mark.gpu

H, W = 1000, 2100  # ragged against the 128-pixel tile width and every tile height


@pytest.fixture(scope="module")
def ctx():
    return vlg.create()


def labels(ctx, mask, tbh):
    import torch
    vlg.set_tunable(ctx, "ccl_tile_rows", tbh)
    words = torch.from_numpy(vlg.pack(mask)).cuda()
    lab = vlg.ccl_labels(ctx, words, *mask.shape)
    vlg.sync(ctx)
    vlg.set_tunable(ctx, "ccl_tile_rows", 0)
    return lab.cpu().numpy()


def spiral(h, w):
    m = np.zeros((h, w), np.uint8)
    top, left, bottom, right = 0, 0, h - 1, w - 1
    while top <= bottom and left <= right:
        m[top, left:right + 1] = 1
        m[top:bottom + 1, right] = 1
        if top + 2 <= bottom:
            m[bottom, left:right + 1] = 1
        if left + 2 <= right:
            m[top + 2:bottom + 1, left] = 1
        top, left, bottom, right = top + 2, left + 2, bottom - 2, right - 2
        if top <= bottom and left - 2 >= 0:
            m[top, left - 2:left] = 1  # link to the next ring
    return m


def patterns():
    yy, xx = np.mgrid[:H, :W]
    rng = np.random.default_rng(11)
    return {
        "columns_pitch2": (xx % 2 == 0),                 # every block is a run; columns cross every tile
        "columns_pitch3": (xx % 3 == 0),
        "rows_pitch2": (yy % 2 == 0),                    # rows cross every tile boundary sideways
        "diagonals": ((xx + yy) % 5 == 0),               # 8-connected diagonal chains
        "anti_diagonals": ((xx - yy) % 7 == 0),
        "spiral": spiral(H, W).astype(bool),
        "grid_holes": ~((xx % 9 < 7) & (yy % 9 < 7)),   # one grid component with many holes
        "dense_noise": rng.random((H, W)) < 0.62,
    }


@pytest.mark.parametrize("tbh", [8, 16, 32])
def test_stress_patterns(ctx, tbh):
    for name, m in patterns().items():
        m = m.astype(np.uint8)
        got = labels(ctx, m, tbh)
        want = oracle.ccl(m)
        assert np.array_equal(got, want), f"{name} tbh={tbh}: {int((got != want).sum())} pixels differ"
