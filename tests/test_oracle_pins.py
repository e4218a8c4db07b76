"""Pins of the CPU oracle against what the paper's definitions and plain
mathematics fix (no GPU).  Each test names the definition it follows:
Sect. 2 (atoms, Boolean operators, N, rho, derived operators), Sect. 3 (rho
computed through connected components; the CCL invariant).
"""
import itertools

import numpy as np
import pytest
from scipy import ndimage

import oracle
from tests import brute

K3 = np.ones((3, 3), bool)


def rand_mask(rng, h, w, p=0.5):
    return (rng.random((h, w)) < p).astype(np.uint8)


def all_masks(h, w):
    for bits in range(1 << (h * w)):
        yield np.array([(bits >> i) & 1 for i in range(h * w)], np.uint8).reshape(h, w)


def z_closed_form(a, b):
    """Union of the 8-components of b that meet N a (Sect. 3, rho via CCL)."""
    lab, n = ndimage.label(b, structure=K3)
    na = ndimage.binary_dilation(a, structure=K3, border_value=0)
    hit = np.unique(lab[(na > 0) & (b > 0)])
    return np.isin(lab, hit[hit > 0]).astype(np.uint8)


# ---------------------------------------------------------------- atoms

@pytest.mark.parametrize("op", [">", "<", ">=", "<="])
def test_threshold_f32_matches_numpy(op):
    rng = np.random.default_rng(1)
    img = rng.random((2, 17, 23)).astype(np.float32)
    t = 0.1  # not representable: rounded once to float32
    img[1, 3, 4] = np.float32(t)  # a pixel exactly at the rounded threshold
    ref = {">": np.greater, "<": np.less, ">=": np.greater_equal, "<=": np.less_equal}[op]
    for c in (0, 1):
        got = oracle.threshold(img, c, op, t)
        want = ref(img[c], np.float32(t)).astype(np.uint8)
        assert np.array_equal(got, want)


def test_threshold_rounds_constant_once_to_float32():
    # 0.1 as double lies between two float32 values; the pixel equal to
    # float32(0.1) is not > float32(0.1) but is >= it.
    img = np.full((1, 1, 3), np.float32(0.1), np.float32)
    img[0, 0, 1] = np.nextafter(np.float32(0.1), np.float32(1))
    img[0, 0, 2] = np.nextafter(np.float32(0.1), np.float32(0))
    assert oracle.threshold(img, 0, ">", 0.1).tolist() == [[0, 1, 0]]
    assert oracle.threshold(img, 0, ">=", 0.1).tolist() == [[1, 1, 0]]
    src = 'output "a" intensity(img) >. 0.1\noutput "b" intensity(img) >=. 0.1'
    a, b = oracle.run(src, img)
    assert a.tolist() == [[0, 1, 0]] and b.tolist() == [[1, 1, 0]]


def test_threshold_u8_exact():
    img = np.arange(256, dtype=np.uint8).reshape(1, 16, 16)
    got = oracle.threshold(img, 0, ">", 127.5)
    assert np.array_equal(got, (img[0] > 127).astype(np.uint8))
    got = oracle.threshold(img, 0, ">=", 128)
    assert np.array_equal(got, (img[0] >= 128).astype(np.uint8))


@pytest.mark.parametrize("q", [0.0, 1e-9, 0.01, 0.3, 0.5, 0.86, 0.95, 0.999, 1.0])
def test_percentile_nearest_rank(q):
    rng = np.random.default_rng(7)
    img = rng.random((2, 13, 31)).astype(np.float32)
    img[1, :3] = 0.25  # ties
    for c in (0, 1):
        v = np.sort(img[c].reshape(-1))
        n = v.size
        k = min(max(int(np.ceil(q * n)) - 1, 0), n - 1)
        assert oracle.percentile(img, c, q) == v[k]


def test_percentile_u8_and_threshold_use():
    rng = np.random.default_rng(8)
    img = rng.integers(0, 256, (1, 20, 20), dtype=np.uint8)
    t = np.sort(img.reshape(-1))[int(np.ceil(0.9 * 400)) - 1]
    assert oracle.percentile(img, 0, 0.9) == np.float32(t)
    (m,) = oracle.run('output "m" intensity(img) >. percentile(img, 0, 0.9)', img)
    assert np.array_equal(m, (img[0] > t).astype(np.uint8))


def test_threshold_u16_exact():
    # uint16 pixels (the paper's type) convert exactly to float32; the
    # specification's thresholds are uint16 values (Fig. specification)
    img = np.array([[0, 1, 56359, 56360, 56361, 62257, 62258, 62259, 65534, 65535]], np.uint16)[None]
    for op, t, ref in [(">", 62258, np.greater), (">", 56360, np.greater), (">=", 56360, np.greater_equal),
                       ("<", 1, np.less), ("<=", 65534.5, np.less_equal), (">", 62257.5, np.greater)]:
        got = oracle.threshold(img, 0, op, t)
        assert np.array_equal(got, ref(img[0].astype(np.float64), np.float32(t)).astype(np.uint8)), (op, t)


def test_percentile_u16_and_threshold_use():
    rng = np.random.default_rng(9)
    img = rng.integers(0, 65536, (2, 23, 37), dtype=np.uint16)
    img[1, :5] = 40000  # ties
    for c in (0, 1):
        for q in (0.0, 0.3, 0.86, 0.95, 1.0):
            v = np.sort(img[c].reshape(-1))
            k = min(max(int(np.ceil(q * v.size)) - 1, 0), v.size - 1)
            assert oracle.percentile(img, c, q) == np.float32(v[k])
    t = np.sort(img[0].reshape(-1))[int(np.ceil(0.95 * img[0].size)) - 1]
    (m,) = oracle.run('output "m" intensity(img) >. percentile(img, 0, 0.95)', img)
    assert np.array_equal(m, (img[0] > t).astype(np.uint8))


# ---------------------------------------------------------------- Boolean operators

def test_boolean_truth_tables():
    a = np.array([[0, 0, 1, 1]], np.uint8)
    b = np.array([[0, 1, 0, 1]], np.uint8)
    assert oracle.lnot(a).tolist() == [[1, 1, 0, 0]]
    assert oracle.land(a, b).tolist() == [[0, 0, 0, 1]]
    assert oracle.lor(a, b).tolist() == [[0, 1, 1, 1]]
    img = np.stack([a, b]).astype(np.float32)
    src = ('let A = intensity(img, 0) >. 0.5\nlet B = intensity(img, 1) >. 0.5\n'
           'output "not" !A\noutput "and" A & B\noutput "or" A | B\n'
           'output "t" true\noutput "f" false\noutput "prec" !A & B | A & !B')
    n, an, o, t, f, x = oracle.run(src, img)
    assert n.tolist() == [[1, 1, 0, 0]] and an.tolist() == [[0, 0, 0, 1]]
    assert o.tolist() == [[0, 1, 1, 1]] and t.tolist() == [[1] * 4] and f.tolist() == [[0] * 4]
    assert x.tolist() == [[0, 1, 1, 0]]  # '!' binds tighter than '&', '&' than '|'


# ---------------------------------------------------------------- near

def test_near_bruteforce_and_scipy():
    rng = np.random.default_rng(2)
    for h, w in [(1, 1), (1, 5), (5, 1), (2, 2), (3, 7), (6, 6)]:
        for _ in range(20):
            a = rand_mask(rng, h, w, rng.uniform(0.05, 0.6))
            assert np.array_equal(oracle.near(a), brute.near(a))
    for h, w in [(64, 64), (65, 127), (129, 63)]:
        a = rand_mask(rng, h, w, 0.1)
        want = ndimage.binary_dilation(a, structure=K3, border_value=0).astype(np.uint8)
        assert np.array_equal(oracle.near(a), want)


def test_near_invariants():
    rng = np.random.default_rng(3)
    for _ in range(30):
        a = rand_mask(rng, 9, 11, 0.2)
        b = a | rand_mask(rng, 9, 11, 0.2)
        na = oracle.near(a)
        assert np.all(na >= a)                       # extensive
        assert np.all(oracle.near(b) >= na)          # monotone
    one = np.zeros((5, 5), np.uint8)
    one[0, 0] = 1
    assert oracle.near(one).sum() == 4               # corner: no pixels outside
    one[0, 0], one[2, 2] = 0, 1
    assert oracle.near(one).sum() == 9


def test_interior_is_erosion_with_border_kept():
    rng = np.random.default_rng(4)
    for h, w in [(1, 1), (4, 9), (33, 17)]:
        for _ in range(10):
            a = rand_mask(rng, h, w, 0.8)
            want = ndimage.binary_erosion(a, structure=K3, border_value=1).astype(np.uint8)
            got = oracle.interior(a)
            assert np.array_equal(got, want)
            assert np.all(got <= a)
            assert np.array_equal(got, 1 - oracle.near(1 - a))
    full = np.ones((4, 6), np.uint8)
    assert np.array_equal(oracle.interior(full), full)


# ---------------------------------------------------------------- reach

def test_reach_exhaustive_small_against_path_enumeration():
    # every pair of masks on 2x3 and 3x2 images
    for h, w in [(2, 3), (3, 2)]:
        masks = list(all_masks(h, w))
        for a, b in itertools.product(masks, masks):
            assert np.array_equal(oracle.reach(a, b), brute.reach_paths(a, b)), (a, b)


def test_reach_random_against_paths_and_walks():
    rng = np.random.default_rng(5)
    for h, w in [(3, 3), (4, 4), (3, 5)]:
        for _ in range(120):
            a = rand_mask(rng, h, w, rng.uniform(0.0, 0.3))
            b = rand_mask(rng, h, w, rng.uniform(0.2, 0.7))
            got = oracle.reach(a, b)
            assert np.array_equal(got, brute.reach_paths(a, b))
            assert np.array_equal(got, brute.reach_walks(a, b))
    for h, w in [(5, 5), (6, 7), (8, 8)]:
        for _ in range(40):
            a = rand_mask(rng, h, w, rng.uniform(0.0, 0.15))
            b = rand_mask(rng, h, w, rng.uniform(0.3, 0.7))
            assert np.array_equal(oracle.reach(a, b), brute.reach_walks(a, b))


def test_reach_equals_ccl_closed_form():
    # rho a[b] = N(a | Z), Z = components of b meeting N a (Sect. 3)
    rng = np.random.default_rng(6)
    for h, w in [(1, 9), (9, 1), (16, 16), (31, 65), (64, 70)]:
        for _ in range(15):
            a = rand_mask(rng, h, w, 0.01)
            b = rand_mask(rng, h, w, rng.uniform(0.3, 0.6))
            want = ndimage.binary_dilation(a | z_closed_form(a, b), structure=K3,
                                           border_value=0).astype(np.uint8)
            assert np.array_equal(oracle.reach(a, b), want)


def test_reach_invariants_and_special_cases():
    rng = np.random.default_rng(9)
    for _ in range(40):
        a = rand_mask(rng, 12, 10, 0.03)
        b = rand_mask(rng, 12, 10, 0.5)
        r = oracle.reach(a, b)
        assert np.all(a <= oracle.near(a)) and np.all(oracle.near(a) <= r)
        a2 = a | rand_mask(rng, 12, 10, 0.02)
        b2 = b | rand_mask(rng, 12, 10, 0.1)
        assert np.all(oracle.reach(a2, b) >= r)       # monotone in a
        assert np.all(oracle.reach(a, b2) >= r)       # monotone in b
    z = np.zeros((7, 9), np.uint8)
    o = np.ones((7, 9), np.uint8)
    a = rand_mask(rng, 7, 9, 0.1)
    a[3, 3] = 1
    assert not oracle.reach(z, rand_mask(rng, 7, 9)).any()         # rho empty[b] = empty
    assert np.array_equal(oracle.reach(a, z), oracle.near(a))      # rho a[empty] = N a
    assert np.array_equal(oracle.reach(a, o), o)                   # rho a[all] = all


def test_reach_serpentine_maze():
    from synth.images import serpentine_maze
    m = serpentine_maze(41, 37).astype(np.uint8)
    seed = np.zeros_like(m)
    seed[0, 0] = 1
    assert np.array_equal(oracle.reach(seed, m), oracle.near(m | seed))
    assert np.array_equal(oracle.grow(seed, m), m)
    cut = m.copy()
    cut[21, 36] = 0   # close one opening: the corridor below row 21 is unreachable
    g = oracle.grow(seed, cut)
    assert g[:21].sum() == cut[:21].sum() and g[22:].sum() == 0


# ---------------------------------------------------------------- surrounded / grow

def test_surrounded_against_direct_definition():
    rng = np.random.default_rng(10)
    for h, w in [(2, 3), (3, 3)]:
        masks = list(all_masks(h, w))
        for a in masks:
            for _ in range(8):
                b = masks[int(rng.integers(0, len(masks)))]
                assert np.array_equal(oracle.surrounded(a, b), brute.surrounded_paths(a, b))
    for h, w in [(5, 5), (8, 9), (12, 12)]:
        for _ in range(60):
            a = rand_mask(rng, h, w, rng.uniform(0.3, 0.9))
            b = rand_mask(rng, h, w, rng.uniform(0.1, 0.5))
            got = oracle.surrounded(a, b)
            assert np.array_equal(got, brute.surrounded_paths(a, b))
            assert np.all(got <= a)
            b2 = b | rand_mask(rng, h, w, 0.2)
            assert np.all(oracle.surrounded(a, b2) >= got)   # monotone in b


def test_surrounded_disc_in_ring():
    n = 11
    yy, xx = np.mgrid[:n, :n]
    ring = ((np.maximum(abs(yy - 5), abs(xx - 5)) == 4)).astype(np.uint8)
    disc = (np.maximum(abs(yy - 5), abs(xx - 5)) <= 3).astype(np.uint8)
    assert np.array_equal(oracle.surrounded(disc, ring), disc)
    gap = ring.copy()
    gap[1, 5] = 0
    assert not oracle.surrounded(disc, gap).any()
    # surrounded(a, empty) is empty unless a is the whole image
    assert not oracle.surrounded(disc, np.zeros_like(disc)).any()
    full = np.ones_like(disc)
    assert np.array_equal(oracle.surrounded(full, np.zeros_like(disc)), full)


def test_grow_is_a_union_touching_components():
    rng = np.random.default_rng(11)
    for h, w in [(3, 3), (10, 13), (40, 40)]:
        for _ in range(20):
            a = rand_mask(rng, h, w, 0.02)
            b = rand_mask(rng, h, w, 0.5)
            assert np.array_equal(oracle.grow(a, b), a | z_closed_form(a, b))


# ---------------------------------------------------------------- CCL (Sect. 3)

def test_ccl_partition_and_canonical_labels():
    rng = np.random.default_rng(12)
    for h, w in [(1, 1), (1, 50), (50, 1), (7, 7), (64, 64), (33, 129)]:
        for p in (0.2, 0.45, 0.6):
            a = rand_mask(rng, h, w, p)
            lab = oracle.ccl(a)
            ref, n = ndimage.label(a, structure=K3)
            assert (lab >= 0).sum() == (ref > 0).sum()
            # same partition: bijection between labels
            pairs = set(zip(lab[a > 0].tolist(), ref[a > 0].tolist()))
            assert len(pairs) == n == len(set(lab[a > 0].tolist()))
            # canonical label = smallest row-major index of the component
            for comp in brute.components(a):
                m = min(y * w + x for y, x in comp)
                assert all(lab[y, x] == m for y, x in comp)
            # the paper's invariant: a pixel's label lies in its own component
            flat = lab.reshape(-1)
            for idx in np.flatnonzero(flat >= 0)[:200]:
                assert flat[flat[idx]] == flat[idx]


def test_ccl_concave_corner_is_one_component():
    # pixels (a,b), (a+1,b), (a,b+1) without (a+1,b+1): the case the paper's
    # pointer-jumping iteration can leave split (Sect. 3)
    a = np.zeros((4, 4), np.uint8)
    a[1, 1] = a[2, 1] = a[1, 2] = 1
    lab = oracle.ccl(a)
    assert set(lab[a > 0].tolist()) == {1 * 4 + 1}


# ------------------------------------- the paper's labelling (Sect. 3, Alg. CCL)

def scipy_max_labels(a):
    """Largest row-major index of each 8-component (scipy's partition)."""
    h, w = a.shape
    ref, n = ndimage.label(a, structure=K3)
    idx = np.arange(h * w).reshape(h, w)
    out = np.full((h, w), -1, np.int32)
    if n:
        mx = ndimage.maximum(idx, labels=ref, index=np.arange(1, n + 1))
        for c in range(1, n + 1):
            out[ref == c] = int(mx[c - 1])
    return out


def test_ccl_max_is_the_largest_index_of_the_component():
    rng = np.random.default_rng(21)
    for h, w in [(1, 1), (1, 40), (40, 1), (7, 9), (64, 64), (33, 129)]:
        for p in (0.2, 0.45, 0.6):
            a = rand_mask(rng, h, w, p)
            assert np.array_equal(oracle.ccl_max(a), scipy_max_labels(a))


@pytest.mark.parametrize("k", [1, 2, 3, 8, 16])
def test_ccl_pj_terminates_with_the_largest_label(k):
    # the paper: the algorithm exits only when every component is labelled
    # uniformly, and a label always lies in the pixel's own component, so
    # the final label of a component is its largest coordinate pair
    rng = np.random.default_rng(22 + k)
    cases = [rand_mask(rng, h, w, p) for h, w in [(1, 1), (5, 5), (17, 23), (48, 40)] for p in (0.3, 0.5, 0.7)]
    from synth import images
    cases.append(images.serpentine_maze(21, 14).astype(np.uint8))
    cases.append(np.ones((9, 11), np.uint8))
    for a in cases:
        lab, iters = oracle.ccl_pj(a, k=k)
        assert np.array_equal(lab, scipy_max_labels(a))
        assert iters % k == 0 and iters >= k


def test_ccl_pj_line_doubles_per_iteration():
    # on a straight line of n pixels, max-neighbour pointer jumping gives the
    # pixel at offset x the label min(x + 2^t - 1, n - 1) after t main
    # iterations, and reconnect never fires (the largest label around x is
    # never above the label stored at x's target); so the check first passes
    # at the end of the round in which t reaches ceil(log2 n)
    for n in range(1, 70):
        t = int(np.ceil(np.log2(n))) if n > 1 else 0
        for k in (1, 2, 3, 5, 8):
            want = k * max(1, -(-t // k))
            for a in (np.ones((1, n), np.uint8), np.ones((n, 1), np.uint8), np.eye(n, dtype=np.uint8)):
                lab, iters = oracle.ccl_pj(a, k=k)
                assert iters == want, (n, k, a.shape)
                assert np.all(lab[a > 0] == np.flatnonzero(a.reshape(-1))[-1])


def test_ccl_pj_hand_traced_turn():
    # rows 1111 / 0001 / 1111, one reconnect per main iteration (k = 1);
    # traced by hand: after iteration 1 the top row holds (0,1) (0,2) (1,3)
    # (1,3); after iteration 2 it holds (1,3) (2,3) (2,3) (2,3) and every
    # other pixel (2,3); reconnect changes nothing on the way and iteration 3
    # labels everything (2,3), so the check passes after 3 main iterations
    a = np.array([[1, 1, 1, 1], [0, 0, 0, 1], [1, 1, 1, 1]], np.uint8)
    lab, iters = oracle.ccl_pj(a, k=1)
    assert iters == 3
    assert np.all(lab[a > 0] == 2 * 4 + 3)


def test_ccl_pj_hand_traced_reconnect_target():
    # rows 111 / 101 / 001, k = 1, traced by hand.  Iteration 1 labels
    # (0,0)->(1,0), (0,1)->(1,2), (0,2)->(1,2), (1,0)->(1,0), (1,2)->(2,2),
    # (2,2)->(2,2).  Reconnect: pixel (0,0) points at (1,0) and sees (1,2)
    # around itself, larger than the (1,0) stored at (1,0), so (1,2) is
    # written at (1,0) -- the pointed-at pixel, not (0,0).  Iteration 2 then
    # leaves (0,0) at (1,2) and everything else at (2,2); iteration 3 ends it
    a = np.array([[1, 1, 1], [1, 0, 1], [0, 0, 1]], np.uint8)
    lab, iters = oracle.ccl_pj(a, k=1)
    assert iters == 3
    assert np.all(lab[a > 0] == 2 * 3 + 2)


def test_ccl_pj_needs_reconnect():
    # rows 1111 / 0001 / 1111 / 1000 / 1111: row 2 runs into row 4 at its
    # left end.  Pixels (1,3), (2,2), (2,3) and the top row point at (2,3),
    # whose neighbourhood never holds a larger label, so main iterations
    # alone settle with two labels; the first reconnect writes (4,3) at
    # (2,3) (from pixel (2,2), whose neighbour (2,1) already holds (4,3)),
    # which the check right after it still sees unpropagated; the second
    # round finishes
    a = np.array([[1, 1, 1, 1], [0, 0, 0, 1], [1, 1, 1, 1], [1, 0, 0, 0], [1, 1, 1, 1]], np.uint8)
    with pytest.raises(oracle.OracleError):
        oracle.ccl_pj(a, k=64, max_rounds=1)
    lab, iters = oracle.ccl_pj(a, k=64, max_rounds=2)
    assert iters == 128 and np.all(lab[a > 0] == 4 * 4 + 3)


# ------------------------------- arithmetic atoms and touch (Sect. 2, Sect. 3)

F32 = np.float32


def test_arithmetic_atoms_follow_float32_arithmetic():
    # each operation rounds once to float32, as numpy's float32 arithmetic does
    rng = np.random.default_rng(31)
    img = rng.uniform(-2, 2, (3, 17, 23)).astype(F32)
    a, b, c = img[0], img[1], img[2]
    cases = [
        ("intensity(img, 0) + intensity(img, 1) >. 0.25", (a + b) > F32(0.25)),
        ("intensity(img, 0) - intensity(img, 1) - intensity(img, 2) <. 0", ((a - b) - c) < F32(0)),
        ("intensity(img, 0) - intensity(img, 1) * intensity(img, 2) >=. 0.1", (a - b * c) >= F32(0.1)),
        ("(intensity(img, 0) - intensity(img, 1)) * intensity(img, 2) <=. -0.3", ((a - b) * c) <= F32(-0.3)),
        ("intensity(img, 0) / intensity(img, 1) >. 1.5", (a / b) > F32(1.5)),
        ("-intensity(img, 2) >. abs(intensity(img, 0))", (-c) > np.abs(a)),
        ("min(intensity(img, 0), intensity(img, 1)) >. max(intensity(img, 2), 0.5)",
         np.where(b < a, b, a) > np.where(F32(0.5) > c, F32(0.5), c)),
        ("2 * intensity(img, 1) + 0.1 <. intensity(img, 0) * 3", (F32(2) * b + F32(0.1)) < (a * F32(3))),
        ("intensity(img) >. intensity(img, 1)", a > b),
        ("0.5 <. intensity(img, 2)", F32(0.5) < c),
    ]
    for src, want in cases:
        got = oracle.run(f'output "o" {src}', img)[0]
        assert np.array_equal(got, want.astype(np.uint8)), src


def test_arithmetic_on_integer_pixels_and_percentiles():
    rng = np.random.default_rng(32)
    for dt in (np.uint8, np.uint16):
        img = rng.integers(0, np.iinfo(dt).max + 1, (2, 20, 30)).astype(dt)
        a, b = img[0].astype(F32), img[1].astype(F32)
        p = np.sort(img[1].reshape(-1))[int(np.ceil(0.7 * img[1].size)) - 1].astype(F32)
        src = 'output "o" intensity(img, 0) - percentile(img, 1, 0.7) >. intensity(img, 1) / 4'
        want = (a - p) > (b / F32(4))
        assert np.array_equal(oracle.run(src, img)[0], want.astype(np.uint8))


def test_division_by_zero_and_nan_compare_false():
    img = np.array([[[0.0, 1.0, -1.0, 0.0]], [[0.0, 0.0, 0.0, 2.0]]], F32)
    # 0/0 = nan (every comparison false), 1/0 = inf, -1/0 = -inf
    got = oracle.run('output "a" intensity(img, 0) / intensity(img, 1) >. 0\n'
                     'output "b" intensity(img, 0) / intensity(img, 1) <=. 0', img)
    assert got[0].tolist() == [[0, 1, 0, 0]] and got[1].tolist() == [[0, 0, 1, 1]]


def test_touch_keeps_the_regions_of_a_in_contact_with_b():
    # touch(a, b) = a & rho b[a]: a pixel of a whose 8-component in a meets
    # N b (by the path definition, the intermediate pixels lie in a)
    rng = np.random.default_rng(33)
    for h, w in [(1, 1), (6, 7), (30, 41)]:
        for _ in range(10):
            img = rng.random((2, h, w)).astype(F32)
            a = (img[0] > F32(0.45)).astype(np.uint8)
            b = (img[1] > F32(0.93)).astype(np.uint8)
            lab, n = ndimage.label(a, structure=K3)
            nb = ndimage.binary_dilation(b, structure=K3, border_value=0)
            keep = np.unique(lab[nb & (lab > 0)])
            want = np.isin(lab, keep[keep > 0]).astype(np.uint8)
            got = oracle.run('output "t" touch(intensity(img, 0) >. 0.45, intensity(img, 1) >. 0.93)', img)[0]
            assert np.array_equal(got, want)


def test_numeric_parse_errors():
    for src in ['output "x" intensity(img) + >. 1', 'output "x" intensity(img) * 2',
                'output "x" (intensity(img) >. 1', 'output "x" abs(intensity(img)) >. ',
                'let min = true']:
        with pytest.raises(oracle.OracleError):
            oracle.run(src, np.zeros((1, 2, 2), F32))


# ---------------------------------------------------------------- language

def test_macros_let_and_sharing():
    rng = np.random.default_rng(13)
    img = rng.random((2, 9, 12)).astype(np.float32)
    A = (img[0] > np.float32(0.5)).astype(np.uint8)
    B = (img[1] < np.float32(0.4)).astype(np.uint8)
    src = """
    // a parametric macro, expanded at each use
    let A = intensity(img, 0) >. 0.5
    let B = intensity(img, 1) <. 0.4
    let diff(x, y) = x & !y
    let twice(x) = near(near(x))
    output "d" diff(A, B)
    output "d2" diff(B, A)
    output "t" twice(diff(A, B))
    let A = !A   // rebinding shadows the earlier A from here on
    output "nA" A
    """
    d, d2, t, na = oracle.run(src, img)
    assert np.array_equal(d, A & (1 - B))
    assert np.array_equal(d2, B & (1 - A))
    assert np.array_equal(t, brute.near(brute.near(A & (1 - B))))
    assert np.array_equal(na, 1 - A)


@pytest.mark.parametrize("src,where", [
    ('output "x" foo', "undefined name"),
    ('let a = intensity(img) >. \noutput "x" a', "expected a numeric expression"),
    ('output "x" near(true', "expected ')'"),
    ('let near = true', "built-in"),
    ('output x true', "quoted"),
])
def test_parse_errors_have_positions(src, where):
    with pytest.raises(oracle.OracleError) as e:
        oracle.run(src, np.zeros((1, 2, 2), np.float32))
    assert where in str(e.value) and "line" in str(e.value)


def test_composed_formula_matches_independent_composition():
    rng = np.random.default_rng(14)
    for trial in range(20):
        img = rng.random((2, 14, 19)).astype(np.float32)
        t0, t1, t2 = (float(np.float32(v)) for v in rng.uniform(0.2, 0.8, 3))
        A = (img[0] > np.float32(t0)).astype(np.uint8)
        B = (img[1] <= np.float32(t1)).astype(np.uint8)
        C = (img[0] >= np.float32(t2)).astype(np.uint8)
        src = (f"let A = intensity(img) >. {t0!r}\nlet B = intensity(img, 1) <=. {t1!r}\n"
               f"let C = intensity(img, 0) >=. {t2!r}\n"
               'output "o1" reach(A & !C, B | C)\n'
               'output "o2" interior(near(A) | B) & !C\n'
               'output "o3" surrounded(A | B, C)\n'
               'output "o4" grow(A, !B)')
        o1, o2, o3, o4 = oracle.run(src, img)
        a1 = A & (1 - C)
        b1 = B | C
        w1 = ndimage.binary_dilation(a1 | z_closed_form(a1, b1), structure=K3,
                                     border_value=0).astype(np.uint8)
        assert np.array_equal(o1, w1)
        nb = ndimage.binary_dilation(A, structure=K3, border_value=0).astype(np.uint8) | B
        w2 = ndimage.binary_erosion(nb, structure=K3, border_value=1).astype(np.uint8) & (1 - C)
        assert np.array_equal(o2, w2)
        assert np.array_equal(o3, brute.surrounded_paths(A | B, C))
        assert np.array_equal(o4, A | z_closed_form(A, 1 - B))


def test_empty_image():
    img = np.zeros((1, 0, 5), np.float32)
    outs = oracle.run('output "r" reach(intensity(img) >. 0, true)', img)
    assert outs[0].shape == (0, 5)
