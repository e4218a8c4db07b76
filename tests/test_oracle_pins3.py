"""Pins of the oracle's volume evaluation (the logic on 3-D images: the
26-voxel Moore neighbourhood and 26-connected paths; the paper's tool is
restricted to 2-D, Sect. 1, Sect. 3, Sect. 5) against scipy's 3-D
morphology and labelling and a brute-force walk unrolling on tiny volumes.
No GPU."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from tests import brute

K27 = np.ones((3, 3, 3), bool)


def rand_vol(rng, d, h, w, p=0.5):
    return (rng.random((d, h, w)) < p).astype(np.uint8)


def dil3(a):
    return ndimage.binary_dilation(a, structure=K27, border_value=0).astype(np.uint8)


def z_closed_form3(a, b):
    lab, _ = ndimage.label(b, structure=K27)
    hit = np.unique(lab[(dil3(a) > 0) & (lab > 0)])
    return np.isin(lab, hit[hit > 0]).astype(np.uint8)


def test_near3_is_dilation_by_the_3x3x3_cube():
    rng = np.random.default_rng(41)
    for shape in [(1, 1, 1), (1, 5, 7), (3, 4, 5), (6, 9, 70)]:
        for p in (0.05, 0.3):
            a = rand_vol(rng, *shape, p)
            assert np.array_equal(oracle.near3(a), dil3(a))


def test_one_slice_volume_is_the_image():
    rng = np.random.default_rng(42)
    img = rng.random((2, 1, 23, 31)).astype(np.float32)
    src = ('let A = intensity(img, 0) >. 0.6\nlet B = intensity(img, 1) <. 0.5\n'
           'output "n" near(A)\noutput "r" reach(A, B)\noutput "s" surrounded(A | B, !B)\n'
           'output "g" grow(A, B)\noutput "i" interior(B)\noutput "t" touch(B, A)\n')
    for v3, v2 in zip(oracle.run3(src, img), oracle.run(src, img[:, 0])):
        assert np.array_equal(v3[0], v2)


def test_reach3_against_walk_unrolling():
    rng = np.random.default_rng(43)
    for shape in [(2, 2, 2), (2, 3, 3), (3, 3, 3), (1, 3, 4)]:
        for _ in range(25):
            a = rand_vol(rng, *shape, 0.15)
            b = rand_vol(rng, *shape, 0.5)
            assert np.array_equal(oracle.reach3(a, b), brute.reach_walks3(a, b))


def test_reach3_closed_form_through_components():
    rng = np.random.default_rng(44)
    for shape in [(4, 6, 7), (8, 10, 65)]:
        for p in (0.2, 0.3, 0.5):
            a = rand_vol(rng, *shape, 0.01)
            b = rand_vol(rng, *shape, p)
            assert np.array_equal(oracle.reach3(a, b), dil3(a | z_closed_form3(a, b)))


def test_ccl3_partition_and_smallest_index():
    rng = np.random.default_rng(45)
    for shape in [(1, 1, 1), (2, 5, 5), (5, 9, 13)]:
        for p in (0.2, 0.4):
            a = rand_vol(rng, *shape, p)
            lab = oracle.ccl3(a)
            ref, n = ndimage.label(a, structure=K27)
            assert len(set(lab[a > 0].tolist())) == n
            idx = np.arange(a.size).reshape(a.shape)
            for c in range(1, n + 1):
                comp = ref == c
                assert np.all(lab[comp] == idx[comp].min())
            assert np.all(lab[a == 0] == -1)


def test_volume_formulas_by_their_definitions():
    rng = np.random.default_rng(46)
    vol = rng.random((2, 6, 11, 70)).astype(np.float32)
    A = (vol[0] > np.float32(0.7)).astype(np.uint8)
    B = (vol[1] < np.float32(0.55)).astype(np.uint8)
    src = ('let A = intensity(img, 0) >. 0.7\nlet B = intensity(img, 1) <. 0.55\n'
           'output "i" interior(B)\noutput "g" grow(A, B)\noutput "s" surrounded(A, B)\n'
           'output "t" touch(B, A)\noutput "p" intensity(img, 0) >. percentile(img, 0, 0.9)\n')
    i, g, s, t, p = oracle.run3(src, vol)
    assert np.array_equal(i, ndimage.binary_erosion(B, structure=K27, border_value=1).astype(np.uint8))
    assert np.array_equal(g, A | z_closed_form3(A, B))
    nA, nB = 1 - A, 1 - B
    esc = dil3((nA & nB) | z_closed_form3(nA & nB, nB))
    assert np.array_equal(s, A & (1 - esc))
    lab, _ = ndimage.label(B, structure=K27)
    hit = np.unique(lab[(dil3(A) > 0) & (lab > 0)])
    assert np.array_equal(t, np.isin(lab, hit[hit > 0]).astype(np.uint8))
    v = np.sort(vol[0].reshape(-1))
    q = v[int(np.ceil(0.9 * v.size)) - 1]
    assert np.array_equal(p, (vol[0] > q).astype(np.uint8))


def test_volume_surrounded_cube_in_its_shell():
    # a cube whose outer layer is b: from the inner voxels every path to the
    # outside crosses b at an index after 0, so they are surrounded; the
    # shell voxels themselves touch the outside (a path of length 1) and are
    # not.  With one hole in the shell the inner voxels, all 26-connected
    # through non-b voxels, escape through it
    a = np.zeros((9, 9, 9), np.uint8)
    a[2:7, 2:7, 2:7] = 1
    b = a.copy()
    b[3:6, 3:6, 3:6] = 0
    inner = a - b
    vol = np.stack([a, b]).astype(np.float32)
    src = 'output "s" surrounded(intensity(img, 0) >. 0.5, intensity(img, 1) >. 0.5)'
    assert np.array_equal(oracle.run3(src, vol)[0], inner)
    b2 = b.copy()
    b2[2, 4, 4] = 0  # a hole in the top face
    vol2 = np.stack([a, b2]).astype(np.float32)
    assert oracle.run3(src, vol2)[0].sum() == 0
