"""Percentiles on the GPU against the oracle (nearest rank over a channel,
the percentile thresholds of Sect. 3), for float32 channels large enough to
span many histogram workgroups: several quantiles of one channel per step
whose first-digit buckets differ or coincide, ties and signed zeros, and
channels where one bucket holds most or all of the pixels.  Single images and
batches (images of several histogram units).  Each quantile is checked
through both a >= and a > threshold, which differ exactly at the pixels equal
to the value: a wrong value moves at least one pixel."""
import zlib

import numpy as np
import pytest

import oracle
from tests.gpu_util import assert_same, gpu_run
from tests.test_gpu_batch import run_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2010_07284_amd as vlg
    return vlg.create()


def quantile_src(qs, c=0):
    lines = []
    for k, q in enumerate(qs):
        lines.append(f'output "ge{k}" intensity(img, {c}) >=. percentile(img, {c}, {q})')
        lines.append(f'output "gt{k}" intensity(img, {c}) >. percentile(img, {c}, {q})')
    return "\n".join(lines) + "\n"


# uniform values in [0, 1): the first 13 key bits are the sign, the exponent
# and four mantissa bits, so these four quantiles fall in four different
# first-digit buckets ...
SPREAD_QS = (0.95, 0.86, 0.5, 0.3)
# ... and these share one in pairs ([0.9375, 1) and [0.296875, 0.3125))
SHARED_QS = (0.95, 0.96, 0.3, 0.31)


def spread(rng, h, w):
    return rng.random((1, h, w)).astype(np.float32)


def clustered(rng, h, w):
    """60 % of the pixels exactly 0.5, the rest spread: the median's bucket
    holds most of every workgroup's range, and its value is tied."""
    x = spread(rng, h, w)
    x[0][rng.random((h, w)) < 0.6] = 0.5
    return x


def narrow(rng, h, w):
    """Every value in [1, 1.001): a single top-digit bucket for all."""
    return (1.0 + rng.random((1, h, w)) * 1e-3).astype(np.float32)


def signed(rng, h, w):
    x = (rng.standard_normal((1, h, w)) * 3).astype(np.float32)
    x[0, ::7, ::3] = -0.0
    x[0, 1::7, ::5] = 0.0
    return x


@pytest.mark.parametrize("qs", [SPREAD_QS, SHARED_QS, (0.5,), (0.0, 1.0)], ids=["spread", "shared", "one", "ends"])
@pytest.mark.parametrize("kind", [spread, clustered, narrow, signed], ids=lambda f: f.__name__)
def test_single_image(ctx, kind, qs):
    rng = np.random.default_rng(zlib.crc32(f"{kind.__name__} {qs}".encode()))
    img = kind(rng, 1100, 1301)
    src = quantile_src(qs)
    assert_same(src, img, gpu_run(ctx, src, img, "graph"), tag=f"{kind.__name__} {qs}")


def test_values_match_the_oracle_directly(ctx):
    # the >= / > pair pins the value; check the pair against the oracle's
    # own value for one case, so a systematic error in both would show too
    rng = np.random.default_rng(21)
    img = clustered(rng, 513, 700)
    for q in SPREAD_QS:
        v = oracle.percentile(img, 0, q)
        got = gpu_run(ctx, quantile_src((q,)), img, "fused")
        assert np.array_equal(got[0], (img[0] >= v).astype(np.uint8))
        assert np.array_equal(got[1], (img[0] > v).astype(np.uint8))


def test_crowded_and_sparse_buckets_in_one_step(ctx):
    # three buckets in one step: the median's holds the 0.5 cluster, the
    # others few pixels; and an image where the top bucket is the crowded one
    rng = np.random.default_rng(22)
    a = clustered(rng, 900, 1000)
    b = spread(rng, 900, 1000)
    b[0][rng.random((900, 1000)) < 0.5] = 0.99
    for img in (a, b):
        src = quantile_src((0.5, 0.995, 0.2))
        for mode in ("fused", "graph", "perop"):
            assert_same(src, img, gpu_run(ctx, src, img, mode), tag=mode)


def test_batch(ctx):
    rng = np.random.default_rng(23)
    # several histogram units per image for the large ones (262144 elements
    # a unit), crowded buckets in some images only
    imgs = [spread(rng, 700, 700), clustered(rng, 600, 900), spread(rng, 1, 1), narrow(rng, 33, 129),
            signed(rng, 520, 1030), clustered(rng, 5, 3), narrow(rng, 1100, 1300)]
    for qs in (SPREAD_QS, SHARED_QS):
        src = quantile_src(qs)
        for mode in ("graph", "fused"):
            got = run_batch(ctx, src, imgs, mode)
            for img, g in zip(imgs, got):
                assert_same(src, img, g, tag=f"batch {img.shape} {qs} {mode}")
