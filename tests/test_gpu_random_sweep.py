"""Randomized parity sweep: random formulas (up to 120 nodes and 11
reach-type nodes) on random images (sides 1..1400; uniform noise, smoothed
noise or uint8), each with a random executor and labelling tile height,
every output bit-exact against the oracle.  The cases come from one fixed
seed, so a failure names a reproducible case."""
import numpy as np
import pytest

import oracle
from synth import formulas, images
from tests.gpu_util import gpu_run

pytestmark = pytest.mark.gpu

CASES = 80


def test_random_sweep():
    import paper_2010_07284_amd as vlg
    ctx = vlg.create()
    rng = np.random.default_rng(2026)
    try:
        for case in range(CASES):
            seed = int(rng.integers(0, 1 << 30))
            h, w = int(rng.integers(1, 1400)), int(rng.integers(1, 1400))
            kind = int(rng.integers(0, 3))
            if kind == 0:
                img = rng.random((2, h, w)).astype(np.float32)
            elif kind == 1:
                sub = np.random.default_rng(seed)
                sigma = float(rng.uniform(1, 6))
                img = np.stack([images.smoothed_noise(sub, h, w, sigma=sigma) for _ in range(2)]).astype(np.float32)
            else:
                img = (rng.random((2, h, w)) * 255).astype(np.uint8)
            src = formulas.random_dag(seed, n_nodes=int(rng.integers(20, 120)), n_reach=int(rng.integers(1, 12)),
                                      channels=2)
            tbh = int(rng.choice([8, 16, 32]))
            mode = str(rng.choice(["perop", "fused", "graph"]))
            vlg.set_tunable(ctx, "ccl_tile_rows", tbh)
            got = gpu_run(ctx, src, img, mode)
            want = oracle.run(src, img)
            for k, (g, wnt) in enumerate(zip(got, want)):
                n = int((g != wnt).sum())
                assert n == 0, f"case {case} (seed {seed}, {h}x{w}, kind {kind}, tbh {tbh}, {mode}) output {k}: {n} px"
    finally:
        vlg.set_tunable(ctx, "ccl_tile_rows", 0)
