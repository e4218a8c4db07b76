"""Parity at the full sizes of the large-formula and serving workloads, where
the oracle takes minutes: every output is compared with the SHA-256 of the
oracle's mask in the packed layout, stored in tests/golden/digests.json by
tests/golden/make_digests.py (which calls only the oracle).

  - the 10,501-node chain with 500 reach nodes on the 1024x1024 uint8 random
    mask, in the per-operator, fused and graph executors;
  - the largest formula of the serving mix (2000 requested nodes, 50
    reach-type nodes, 50 outputs) on the 4096^2 and 8192^2 serving images,
    alone and inside a 4-slot server mix with the other formulas and sides.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import paper_2010_07284_amd as vlg
from synth import formulas, images

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
_DIGESTS = {}


def digests():
    if not _DIGESTS:
        with open(os.path.join(HERE, "golden", "digests.json")) as fh:
            _DIGESTS.update(json.load(fh)["cases"])
    return _DIGESTS


def digest(t):
    """SHA-256 of a packed device mask (int64 [H, ceil(W/64)])."""
    return hashlib.sha256(t.cpu().numpy().astype("<i8").tobytes()).hexdigest()


def assert_digests(key, outs, tag=""):
    want = digests()[key]["outputs"]
    assert len(outs) == len(want), key
    bad = [k for k, (o, w) in enumerate(zip(outs, want)) if digest(o) != w]
    assert not bad, f"{key} {tag}: outputs {bad} differ from the oracle"


@pytest.mark.parametrize("mode", ["perop", "fused", "graph"])
def test_chain_full_size(mode):
    import torch
    ctx = vlg.create()
    vlg.set_mode(ctx, mode)
    img = images.random_mask_image(3, 1024)
    im = vlg.load_image(ctx, torch.from_numpy(img).cuda())
    f = vlg.compile_formula(ctx, formulas.chain_dag(3))
    st = vlg.formula_info(f)
    assert st["nodes"] == 10501 and st["reach_nodes"] == 500
    outs = vlg.check_all(ctx, f, im)
    vlg.sync(ctx)
    assert_digests("chain_1024", outs, mode)
    # a replay of the same evaluation (graph mode: the captured graph)
    outs2 = vlg.check_all(ctx, f, im)
    vlg.sync(ctx)
    assert_digests("chain_1024", outs2, mode + " replay")


SERVE = formulas.serve_formulas()
LARGEST = len(SERVE) - 1  # 2000 requested nodes, 50 reach-type


@pytest.fixture(scope="module")
def serve_images():
    import torch
    ctx = vlg.create()
    ims = {}
    for i, s in enumerate(formulas.SERVE_SIDES):
        ims[s] = vlg.load_image(ctx, torch.from_numpy(images.serve_image(i, s)).cuda())
    return ctx, ims


@pytest.fixture(scope="module")
def serve_formulas_compiled(serve_images):
    ctx, _ = serve_images
    return [vlg.compile_formula(ctx, src) for src, _, _ in SERVE]


@pytest.mark.parametrize("side", [4096, 8192])
def test_largest_serve_formula_alone(serve_images, serve_formulas_compiled, side):
    ctx, ims = serve_images
    f = serve_formulas_compiled[LARGEST]
    st = vlg.formula_info(f)
    assert st["nodes"] >= 1900 and st["reach_nodes"] == 50
    for mode in ("graph", "perop"):
        vlg.set_mode(ctx, mode)
        outs = vlg.check_all(ctx, f, ims[side])
        vlg.sync(ctx)
        assert_digests(f"serve_f{LARGEST}_s{side}", outs, mode)


def test_serve_mix_full_size(serve_images, serve_formulas_compiled):
    import torch
    _, ims = serve_images
    fs = serve_formulas_compiled
    rng = np.random.default_rng(7)
    pairs = [(LARGEST, 4096), (LARGEST, 8192), (LARGEST, 8192), (0, 8192)]
    pairs += [(int(rng.integers(0, len(fs))), int(rng.choice(formulas.SERVE_SIDES))) for _ in range(28)]
    rng.shuffle(pairs)
    srv = vlg.Server(slots=4, budget_bytes=8 << 30)
    subs = []
    for k, s in pairs:
        C, H, W = ims[s].shape
        n = vlg.formula_info(fs[k])["outputs"]
        outs = [torch.full((H, (W + 63) // 64), -1, dtype=torch.int64, device="cuda") for _ in range(n)]
        subs.append((k, s, outs, srv.submit(fs[k], ims[s], outs)))
    for k, s, outs, rid in subs:
        srv.wait(rid)
        assert_digests(f"serve_f{k}_s{s}", outs, "in the mix")
    st = srv.stats()
    assert st["completed"] == len(pairs) and st["rejected"] == 0
    srv.close()
