"""The tile-local labelling protocol under randomized lane schedules (CPU
model in tests/ccl_local_model.py): for the shipped resolution (each run start
by its own lane) and for the reverted variant (run starts spread over the
wave's lanes through the LDS queue), every interleaving tried gives each block
the smallest block id of its 8-connected component.  Patterns include union
queues that overflow into the direct-union path."""
import numpy as np
import pytest

from tests import ccl_local_model as M


def patterns(rng, tbh):
    yield (rng.random((2 * tbh, 128)) < 0.5).astype(np.uint8)
    yield (rng.random((2 * tbh, 128)) < 0.62).astype(np.uint8)
    stripes = np.zeros((2 * tbh, 128), np.uint8)
    stripes[:, ::2] = 1  # 64 runs per block row, one union per block: the queue overflows
    yield stripes
    diag = np.zeros((2 * tbh, 128), np.uint8)
    for y in range(2 * tbh):
        diag[y, (y * 3) % 128::7] = 1
    yield diag


@pytest.mark.parametrize("layout,variant", [("consecutive", "own"), ("interleaved", "own"),
                                            ("interleaved", "queue")])
@pytest.mark.parametrize("tbh,nwaves", [(8, 4), (16, 4), (32, 8)])
def test_protocol_under_random_schedules(layout, variant, tbh, nwaves):
    rng = np.random.default_rng(tbh * 10 + nwaves)
    for p, px in enumerate(patterns(rng, tbh)):
        bits = M.tile_blocks(px)
        ref = M.reference_roots(bits)
        for s in range(2 if tbh == 32 else 3):
            out = M.simulate(bits, nwaves, seed=1000 * p + s, variant=variant, layout=layout)
            assert np.array_equal(out, ref), (layout, variant, tbh, p, s)


def test_overflow_pattern_overflows():
    stripes = np.zeros((32, 128), np.uint8)
    stripes[:, ::2] = 1
    t = M.Tile(M.tile_blocks(stripes), 4, layout="interleaved")
    queue, early, overflow = t.wave_pairs(1)  # rows 1, 5, 9, 13: 4 x 64 unions
    assert len(queue) == 192 and sum(len(v) for v in overflow.values()) > 0
    # eight rows per wave: rows 9 .. 15 (7 x 64 unions) are listed before the
    # barrier, so the queue overflows there already
    tall = np.zeros((64, 128), np.uint8)
    tall[:, ::2] = 1
    t = M.Tile(M.tile_blocks(tall), 4)
    queue, early, overflow = t.wave_pairs(1)
    assert len(queue) == 192 and sum(len(v) for v in early.values()) > 0
    bits = M.tile_blocks(tall)
    for s in range(2):
        assert np.array_equal(M.simulate(bits, 4, seed=s), M.reference_roots(bits))
