"""The volume labelling's decisions (tests/vol_block_model.py, a CPU model of
the block passes in vol.hip) give the 26-connected components that
scipy.ndimage.label finds, on random volumes whose widths leave ragged
chunks of 64 blocks and odd sizes along every axis."""
import numpy as np
import pytest
from scipy import ndimage

from tests import vol_block_model as M


def reference(vol):
    lab, _ = ndimage.label(vol, structure=np.ones((3, 3, 3), bool))
    D, S, W = vol.shape
    out = np.full(vol.shape, -1, np.int64)
    for k in range(1, lab.max() + 1):
        idx = np.flatnonzero(lab.ravel() == k)
        out.ravel()[idx] = idx.min()
    return out


def test_faces():
    assert M.face(0, 0, -1) == 0x55 and M.face(0, 0, 1) == 0xAA
    assert M.face(-1, -1, -1) == 0x01 and M.face(1, 1, 1) == 0x80 and M.face(0, 0, 0) == 0xFF


@pytest.mark.parametrize("shape,density,seed", [
    ((5, 7, 9), 0.3, 1), ((4, 6, 131), 0.25, 2), ((3, 5, 260), 0.2, 3), ((6, 4, 257), 0.35, 4),
    ((7, 3, 129), 0.15, 5), ((2, 2, 300), 0.3, 6), ((1, 9, 140), 0.4, 7)])
def test_model_matches_scipy(shape, density, seed):
    rng = np.random.default_rng(seed)
    vol = (rng.random(shape) < density).astype(np.uint8)
    assert np.array_equal(M.voxel_labels(vol), reference(vol))


def test_model_diagonal_chains_and_corridors():
    # a corner-to-corner diagonal (vertex contacts only) and a corridor that
    # crosses chunk borders in every row
    D, S, W = 6, 6, 260
    vol = np.zeros((D, S, W), np.uint8)
    for i in range(min(D, S)):
        vol[i, i, 3 * i] = 1
    vol[2, :, 127:131] = 1
    vol[4, 1::2, :] = 1
    assert np.array_equal(M.voxel_labels(vol), reference(vol))
