"""Several independent labellings run together (VLG_TUNE_CCL_LANES = 2, 4,
8): the fused schedule groups ready labellings into one region with a
workspace each, and every union-find phase runs for all of them in one
launch on the context's stream.  Every output against the oracle, bit for
bit, in fused and graph mode: the headline-shaped formula (ten reach-type
nodes, labelling reuse across lanes), the segmentation formula, random
formulas and a long chain."""
import numpy as np
import pytest

import oracle
import paper_2010_07284_amd as vlg
from synth import formulas, images
from tests.gpu_util import assert_same, gpu_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return vlg.create()


def cases():
    out = [("ellipse512", formulas.ellipse_dag(2), images.ellipse_maze_image(2, 512)),
           ("segmentation", formulas.segmentation_dag(4), images.phantom_image(np.random.default_rng(4), 190, 257)),
           ("chain", formulas.chain_dag(3, n_chain=600, n_reach=30), images.random_mask_image(3, 300))]
    for seed in range(3):
        rng = np.random.default_rng(200 + seed)
        h, w = int(rng.integers(1, 300)), int(rng.integers(1, 300))
        out.append((f"random{seed}", formulas.random_dag(seed, n_nodes=80, n_reach=10, channels=2),
                    rng.random((2, h, w)).astype(np.float32)))
    return out


CASES = cases()


@pytest.mark.parametrize("lanes", [2, 4, 8])
@pytest.mark.parametrize("name,src,img", CASES, ids=[c[0] for c in CASES])
def test_labellings_together(ctx, lanes, name, src, img):
    want = oracle.run(src, img)
    vlg.set_tunable(ctx, "ccl_lanes", lanes)
    try:
        for mode in ("fused", "graph"):
            assert_same(src, img, gpu_run(ctx, src, img, mode), want, tag=f"{name} lanes={lanes} {mode}")
    finally:
        vlg.set_tunable(ctx, "ccl_lanes", 0)


def test_lanes_tunable_values(ctx):
    for bad in (3, 5, 16):
        with pytest.raises(vlg.VlgError):
            vlg.set_tunable(ctx, "ccl_lanes", bad)
    vlg.set_tunable(ctx, "ccl_lanes", 8)
    assert vlg.get_tunable(ctx, "ccl_lanes", 100, 100) == 8
    vlg.set_tunable(ctx, "ccl_lanes", 0)
