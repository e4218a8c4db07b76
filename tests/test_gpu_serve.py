"""Serving loop: requests that overlap on the device give exactly the masks
they give alone (0 differing bits), admission respects the HBM budget, and
requests larger than the budget are rejected."""
import numpy as np
import pytest

import oracle
import paper_2010_07284_amd as vlg
from synth import formulas, images

pytestmark = pytest.mark.gpu


def make_requests(ctx, n_img=4, n_f=4, seed=0):
    import torch
    rng = np.random.default_rng(seed)
    imgs, fs, raw = [], [], []
    for i in range(n_img):
        side = int(rng.choice([130, 256, 517, 1024]))
        im = images.ellipse_maze_image(10 + i, side, n_ellipses=30)[:1]
        raw.append(im)
        imgs.append(vlg.load_image(ctx, torch.from_numpy(im).cuda()))
    srcs = [formulas.random_dag(20 + k, n_nodes=int(rng.integers(20, 120)), n_reach=int(rng.integers(1, 8)))
            for k in range(n_f)]
    fs = [vlg.compile_formula(ctx, s) for s in srcs]
    return imgs, fs, raw, srcs


def alloc(im, f):
    import torch
    C, H, W = im.shape
    n = vlg.formula_info(f)["outputs"]
    return [torch.full((H, (W + 63) // 64), -1, dtype=torch.int64, device="cuda") for _ in range(n)]


def test_results_alone_equal_results_in_the_mix():
    ctx = vlg.create()
    imgs, fs, raw, srcs = make_requests(ctx)
    pairs = [(i, k) for i in range(len(imgs)) for k in range(len(fs))] * 3
    rng = np.random.default_rng(1)
    rng.shuffle(pairs)
    # alone: one at a time on a plain context
    alone = {}
    for i, k in set(pairs):
        outs = vlg.check_all(ctx, fs[k], imgs[i])
        vlg.sync(ctx)
        alone[(i, k)] = [o.cpu().numpy() for o in outs]
    # in the mix: all submitted at once to a 4-slot server
    srv = vlg.Server(slots=4, budget_bytes=2 << 30)
    subs = []
    for i, k in pairs:
        outs = alloc(imgs[i], fs[k])
        subs.append((i, k, outs, srv.submit(fs[k], imgs[i], outs)))
    for i, k, outs, rid in subs:
        srv.wait(rid)
        for a, b in zip(alone[(i, k)], outs):
            assert np.array_equal(a, b.cpu().numpy()), (i, k)
    st = srv.stats()
    assert st["completed"] == len(pairs) and st["rejected"] == 0
    assert st["max_inflight"] >= 2  # several requests admitted at once (their kernels overlap on the device: see the serving kernel trace)
    srv.close()
    # and the standalone results are the oracle's
    for (i, k) in list(alone)[:4]:
        want = oracle.run(srcs[k], raw[i])
        C, H, W = raw[i].shape
        for a, w in zip(alone[(i, k)], want):
            assert np.array_equal(vlg.unpack(a, H, W), w)


def test_budget_admission_and_rejection():
    import torch
    ctx = vlg.create()
    im_small = vlg.load_image(ctx, torch.from_numpy(images.plain_image(1, 256)).cuda())
    im_big = vlg.load_image(ctx, torch.from_numpy(images.plain_image(2, 2048)).cuda())
    f = vlg.compile_formula(ctx, formulas.PLAIN_FORMULA)
    # budget for one small request at a time
    fp = vlg.evaluation_bytes(f, im_small)
    budget = fp * 3 // 2
    assert vlg.evaluation_bytes(f, im_big) > budget
    srv = vlg.Server(slots=4, budget_bytes=budget)
    rids = [(srv.submit(f, im_small, o), o) for o in [alloc(im_small, f) for _ in range(12)]]
    big_out = alloc(im_big, f)
    big = srv.submit(f, im_big, big_out)
    for rid, _ in rids:
        srv.wait(rid)
    with pytest.raises(vlg.VlgError) as e:
        srv.wait(big)
    assert e.value.code == -4
    st = srv.stats()
    assert st["rejected"] == 1 and st["completed"] == 13
    assert st["peak_reserved_bytes"] <= budget
    assert st["max_inflight"] == 1  # the budget admits one request at a time
    first = rids[0][1]
    for _, outs in rids[1:]:
        for a, b in zip(first, outs):
            assert torch.equal(a, b)
    srv.close()
