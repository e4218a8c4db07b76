"""Batched executor (vlg_check_batch): many images of uneven sizes, one
launch per schedule step, every mask bit-exact against the oracle and against
evaluating the images one at a time."""
import numpy as np
import pytest

import oracle
from synth import formulas, images
from tests.gpu_util import assert_same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2010_07284_amd as vlg
    return vlg.create()


def run_batch(ctx, src, imgs, mode="graph", fmt="packed", host=False, skip=()):
    """Every output of src on each image via one vlg_check_batch call, as
    numpy uint8 masks per image (None where the output was skipped)."""
    import torch
    import paper_2010_07284_amd as vlg
    vlg.set_mode(ctx, mode)
    f = vlg.compile_formula(ctx, src)
    n = vlg.formula_info(f)["outputs"]
    ims = [vlg.load_image(ctx, im) for im in imgs]
    dev = "cpu" if host else f"cuda:{ctx.device}"
    outs = []
    for k, im in enumerate(ims):
        _, H, W = im.shape
        row = []
        for o in range(n):
            if (k, o) in skip:
                row.append(None)
            elif fmt == "packed":
                row.append(torch.full((H, (W + 63) // 64), -1, dtype=torch.int64, device=dev))
            else:
                row.append(torch.full((H, W), 7, dtype=torch.uint8, device=dev))
        outs.append(row)
    vlg.check_batch(ctx, f, ims, outs=outs, fmt=fmt)
    vlg.sync(ctx)
    res = []
    for k, im in enumerate(ims):
        _, H, W = im.shape
        res.append([None if o is None else (vlg.unpack(o, H, W) if fmt == "packed" else o.cpu().numpy())
                    for o in outs[k]])
    return res


UNEVEN = [(1, 1), (1, 70), (70, 1), (33, 129), (64, 64), (65, 200), (131, 97), (2, 4097), (257, 300)]


@pytest.mark.parametrize("mode", ["fused", "graph", "perop"])
def test_batch_operators_uneven(ctx, mode):
    from tests.test_gpu_parity import ops_src
    rng = np.random.default_rng(5)
    src = ops_src(rng)
    imgs = [rng.random((2, h, w)).astype(np.float32) for h, w in UNEVEN]
    got = run_batch(ctx, src, imgs, mode)
    for (h, w), img, g in zip(UNEVEN, imgs, got):
        assert_same(src, img, g, tag=f"{h}x{w} {mode}")


def test_batch_segmentation_percentiles(ctx):
    # the shared segmentation formula: per-channel percentiles per image
    src = formulas.segmentation_dag(4)
    sizes = [(190, 257), (64, 1), (128, 130), (301, 77), (17, 17), (96, 513)]
    imgs = [images.phantom_image(np.random.default_rng([9, i]), h, w) for i, (h, w) in enumerate(sizes)]
    for mode in ("graph", "fused"):
        got = run_batch(ctx, src, imgs, mode)
        for (h, w), img, g in zip(sizes, imgs, got):
            assert_same(src, img, g, tag=f"{h}x{w} {mode}")


def test_batch_matches_single_image_runs(ctx):
    import paper_2010_07284_amd as vlg
    from tests.gpu_util import gpu_run
    src = formulas.random_dag(3, n_nodes=80, n_reach=8, channels=2)
    rng = np.random.default_rng(8)
    imgs = [rng.random((2, int(rng.integers(1, 400)), int(rng.integers(1, 400)))).astype(np.float32)
            for _ in range(12)]
    got = run_batch(ctx, src, imgs, "graph")
    for img, g in zip(imgs, got):
        assert_same(src, img, g, want=gpu_run(ctx, src, img, "fused"))
    vlg.set_mode(ctx, "graph")


def test_batch_mixed_dtypes_formats_and_skips(ctx):
    src = formulas.PLAIN_FORMULA
    rng = np.random.default_rng(12)
    imgs = [images.plain_image(3, 100), (rng.random((1, 40, 70)) * 255).astype(np.uint8),
            images.plain_image(4, 65), (rng.random((1, 3, 200)) * 255).astype(np.uint8)]
    src8 = src  # thresholds compare the stored values; both types are valid inputs
    want = [oracle.run(src8, im) for im in imgs]
    for fmt, host in (("packed", False), ("u8", False), ("u8", True), ("packed", True)):
        skip = {(1, 0), (2, 2)}
        got = run_batch(ctx, src8, imgs, "graph", fmt=fmt, host=host, skip=skip)
        for k, (g, w) in enumerate(zip(got, want)):
            for o, (go, wo) in enumerate(zip(g, w)):
                if (k, o) in skip:
                    assert go is None
                    continue
                assert np.array_equal(go, wo), f"image {k} output {o} {fmt} host={host}"


@pytest.mark.parametrize("tbh", [8, 16, 32])
def test_batch_tile_heights(ctx, tbh):
    import paper_2010_07284_amd as vlg
    from tests.test_gpu_parity import ops_src
    rng = np.random.default_rng(20 + tbh)
    src = ops_src(rng)
    sizes = [(389, 517), (70, 1), (129, 300), (33, 65)]
    imgs = [np.concatenate([images.smoothed_noise(rng, h, w, sigma=2.0)[None],
                            rng.random((1, h, w)).astype(np.float32)]) for h, w in sizes]
    vlg.set_tunable(ctx, "ccl_tile_rows", tbh)
    try:
        got = run_batch(ctx, src, imgs, "graph")
    finally:
        vlg.set_tunable(ctx, "ccl_tile_rows", 0)
    for (h, w), img, g in zip(sizes, imgs, got):
        assert_same(src, img, g, tag=f"{h}x{w} tbh={tbh}")


def test_batch_graph_replays(ctx):
    # the captured graph is replayed with eager work and host syncs in between;
    # every replay matches the eager (fused) result
    import torch
    import paper_2010_07284_amd as vlg
    src = formulas.segmentation_dag(4)
    sizes = [(150, 211), (77, 64), (200, 129)]
    imgs = [images.phantom_image(np.random.default_rng([31, i]), h, w) for i, (h, w) in enumerate(sizes)]
    f = vlg.compile_formula(ctx, src)
    ims = [vlg.load_image(ctx, im) for im in imgs]
    vlg.set_mode(ctx, "fused")
    ref = vlg.check_batch(ctx, f, ims)
    vlg.sync(ctx)
    ref = [[o.clone() for o in row] for row in ref]
    vlg.set_mode(ctx, "graph")
    outs = [[torch.empty_like(o) for o in row] for row in ref]
    for rep in range(4):
        for row in outs:
            for o in row:
                o.fill_(-1)
        vlg.check_batch(ctx, f, ims, outs=outs)
        vlg.check_all(ctx, f, ims[rep % len(ims)])  # other work on the same workspace
        vlg.sync(ctx)
        for k, (a, b) in enumerate(zip(outs, ref)):
            for o, (x, y) in enumerate(zip(a, b)):
                assert torch.equal(x, y), f"replay {rep} image {k} output {o}"


def test_batch_empty_and_zero_size(ctx):
    import paper_2010_07284_amd as vlg
    f = vlg.compile_formula(ctx, formulas.PLAIN_FORMULA)
    assert vlg.check_batch(ctx, f, [], outs=[]) == []
    imgs = [np.zeros((1, 0, 5), np.float32), images.plain_image(1, 64), np.zeros((1, 7, 0), np.float32)]
    got = run_batch(ctx, formulas.PLAIN_FORMULA, imgs, "graph")
    assert all(o.size == 0 for o in got[0] + got[2])
    assert_same(formulas.PLAIN_FORMULA, imgs[1], got[1])


def test_batch_uneven_full_config_sampled(ctx):
    """512 phantom images, sides uniform in [128, 2048], 4 float32 channels,
    the shared 60-node segmentation formula, one batched call: sampled images
    (smallest, largest, and two more) against the oracle."""
    import torch
    import paper_2010_07284_amd as vlg
    sizes = images.batch_sizes(4, 512, 128, 2048)
    src = formulas.segmentation_dag(4)
    f = vlg.compile_formula(ctx, src)
    n = vlg.formula_info(f)["outputs"]
    dev = f"cuda:{ctx.device}"
    ims, dimgs = [], {}
    order = sorted(range(len(sizes)), key=lambda i: sizes[i][0] * sizes[i][1])
    sample = {order[0], order[-1], order[len(order) // 2], 137}
    for i, (h, w) in enumerate(sizes):
        t = images.phantom_image_device(4, i, h, w, device=dev)
        ims.append(vlg.load_image(ctx, t))
        if i in sample:
            dimgs[i] = t.cpu().numpy()
        del t
    vlg.set_mode(ctx, "graph")
    outs = vlg.check_batch(ctx, f, ims)
    vlg.sync(ctx)
    for i in sorted(sample):
        h, w = sizes[i]
        got = [vlg.unpack(o, h, w) for o in outs[i]]
        assert len(got) == n
        assert_same(src, dimgs[i], got, tag=f"image {i} {h}x{w}")
    del outs
    torch.cuda.empty_cache()


def test_batch_autotune_picks_persists_and_keeps_results(ctx, tmp_path):
    import paper_2010_07284_amd as vlg
    src = formulas.segmentation_dag(4)
    sizes = [(190, 257), (300, 77), (128, 520), (64, 64)]
    imgs = [images.phantom_image(np.random.default_rng([41, i]), h, w) for i, (h, w) in enumerate(sizes)]
    f = vlg.compile_formula(ctx, src)
    ims = [vlg.load_image(ctx, im) for im in imgs]
    rep = vlg.autotune_batch(ctx, f, ims, iters=1)
    best, times = rep["ccl_tile_rows"]
    assert set(times) == {8, 16, 32} and best == min(times, key=times.get)
    gbest, gtimes = rep["batch_grid"]
    assert set(gtimes) == {1024, 2048, 4096, 8192} and gbest == min(gtimes, key=gtimes.get)
    path = str(tmp_path / "tune.jsonl")
    vlg.tune_save(ctx, path)
    assert '"ccl_tile_rows_batch"' in open(path).read()
    ctx2 = vlg.create()
    vlg.tune_load(ctx2, path)
    got = run_batch(ctx2, src, imgs, "graph")
    for (h, w), img, g in zip(sizes, imgs, got):
        assert_same(src, img, g, tag=f"{h}x{w} tuned")


@pytest.mark.parametrize("grid", [1024, 4096])
def test_batch_grid_sizes(ctx, grid):
    import paper_2010_07284_amd as vlg
    src = formulas.segmentation_dag(4)
    sizes = [(190, 257), (64, 1), (300, 301), (17, 17)]
    imgs = [images.phantom_image(np.random.default_rng([61, i]), h, w) for i, (h, w) in enumerate(sizes)]
    vlg.set_tunable(ctx, "batch_grid", grid)
    try:
        got = run_batch(ctx, src, imgs, "graph")
    finally:
        vlg.set_tunable(ctx, "batch_grid", 0)
    for (h, w), img, g in zip(sizes, imgs, got):
        assert_same(src, img, g, tag=f"{h}x{w} grid={grid}")


def test_batch_profile_counts_every_launch(ctx):
    # vlg_profile_batch: per kind, launches of the batched schedule and their
    # algorithmic bytes summed over the images; the batch still evaluates to
    # the oracle's masks afterwards
    import paper_2010_07284_amd as vlg
    src = formulas.segmentation_dag(4)
    sizes = [(190, 257), (64, 65), (301, 77)]
    imgs = [images.phantom_image(np.random.default_rng([11, i]), h, w) for i, (h, w) in enumerate(sizes)]
    vlg.set_mode(ctx, "fused")
    f = vlg.compile_formula(ctx, src)
    ims = [vlg.load_image(ctx, im) for im in imgs]
    prof = vlg.profile_batch(ctx, f, ims, iters=2)
    plan = vlg.formula_plan(f, "fused", 1)
    assert {"atoms", "ccl_local", "ccl_merge", "ccl_gather"} <= set(prof)
    for name, (n, ms, b) in prof.items():
        assert n > 0 and n % 2 == 0 and ms > 0 and b >= 0, name
    assert prof["ccl_local"][0] == 2 * sum(1 for st in plan["steps"] if st["kind"] == "ccl_local")
    got = run_batch(ctx, src, imgs, "graph")
    for (h, w), img, g in zip(sizes, imgs, got):
        assert_same(src, img, g, tag=f"after profile {h}x{w}")
