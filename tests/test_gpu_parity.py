"""GPU path (through the C ABI) against the CPU oracle, bit for bit.

Covers every operator, the three executor modes, ragged sizes around the
64-bit word and the 128x32-pixel labelling tile, the paper-shaped grow
specification, the maze worst case for labelling, and the full-size
4096x4096 ellipse/maze workload."""
import numpy as np
import pytest

import oracle
from synth import formulas, images
from tests import golden_io
from tests.gpu_util import assert_same, gpu_run

pytestmark = pytest.mark.gpu

MODES = ["perop", "fused", "graph"]

OPS_FORMULA = """
let A = intensity(img, 0) >. {t0}
let B = intensity(img, 1) <=. {t1}
let C = intensity(img, 0) >=. {t2}
let D = intensity(img, 1) <. {t3}
output "not" !A
output "and" A & B
output "or" A | !B
output "near" near(A)
output "near_not" near(!B)
output "interior" interior(A | C)
output "reach" reach(A & !C, B | C)
output "reach_not" reach(!B, !A)
output "surrounded" surrounded(A | B, C)
output "grow" grow(A, !B)
output "const" true & near(false) | !true
output "chain" near(interior(reach(D, A) | grow(C, B))) & !surrounded(B, D)
"""


@pytest.fixture(scope="module")
def ctx():
    import paper_2010_07284_amd as vlg
    return vlg.create()


def ops_src(rng):
    t = rng.uniform(0.25, 0.75, 4)
    return OPS_FORMULA.format(t0=t[0], t1=t[1], t2=t[2], t3=t[3])


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("h,w", [(1, 1), (1, 70), (70, 1), (2, 64), (3, 65), (33, 63), (64, 127),
                                 (65, 129), (31, 200), (97, 301)])
def test_operators_ragged(ctx, mode, h, w):
    rng = np.random.default_rng(h * 1000 + w)
    img = rng.random((2, h, w)).astype(np.float32)
    src = ops_src(rng)
    assert_same(src, img, gpu_run(ctx, src, img, mode), tag=f"{h}x{w} {mode}")


@pytest.mark.parametrize("mode", MODES)
def test_operators_tiles(ctx, mode):
    # several labelling tiles in both directions with ragged edges
    rng = np.random.default_rng(7)
    img = images.smoothed_noise(rng, 517, 389, sigma=2.0)[None]
    img = np.concatenate([img, rng.random((1, 517, 389)).astype(np.float32)])
    src = ops_src(rng)
    assert_same(src, img, gpu_run(ctx, src, img, mode), tag=mode)


@pytest.mark.parametrize("mode", MODES)
def test_plain_workload(ctx, mode):
    img = images.plain_image(1, 256)
    src = formulas.PLAIN_FORMULA
    assert_same(src, img, gpu_run(ctx, src, img, mode), tag=mode)


@pytest.mark.parametrize("fmt,host", [("u8", False), ("u8", True), ("packed", True)])
def test_output_formats(ctx, fmt, host):
    img = images.plain_image(5, 130)
    src = formulas.PLAIN_FORMULA
    assert_same(src, img, gpu_run(ctx, src, img, "graph", fmt=fmt, host=host))


@pytest.mark.parametrize("path", golden_io.all_fixtures(), ids=lambda p: p.split("/")[-1])
def test_golden_fixtures(ctx, path):
    fx = golden_io.load(path)
    B = fx["blocks"]
    if fx["op"] == "ccl":
        pytest.skip("labels are covered by test_ccl_labels")
    if fx["op"] == "formula":
        src, img = "\n".join(B["formula"]), golden_io.image(fx)
    else:
        a = golden_io.mask(B["a"]).astype(np.float32)
        b = golden_io.mask(B["b"]).astype(np.float32) if "b" in B else np.zeros_like(a)
        img = np.stack([a, b])
        arg = "A, B" if "b" in B else "A"
        src = ("let A = intensity(img, 0) >. 0.5\nlet B = intensity(img, 1) >. 0.5\n"
               f'output "r" {fx["op"]}({arg})')
    for mode in MODES:
        got = gpu_run(ctx, src, img, mode)
        assert np.array_equal(got[0], golden_io.mask(B["expect"])), mode


def test_grow_specification_shape(ctx):
    # the paper's specification (Fig. specification) on a synthetic
    # uint16-range image: thresholds 62258 and 56360, then grow
    rng = np.random.default_rng(3)
    base = images.smoothed_noise(rng, 384, 512, sigma=6.0) * 65535.0
    img = base.astype(np.float32)[None]
    src = formulas.GROW_SPEC.format(hi=62258, lo=56360)
    for mode in MODES:
        assert_same(src, img, gpu_run(ctx, src, img, mode), tag=mode)


def test_uint8_images(ctx):
    img = images.random_mask_image(3, 300)
    src = formulas.chain_dag(3, n_chain=300, n_reach=15)
    want = oracle.run(src, img)
    for mode in MODES:
        assert_same(src, img, gpu_run(ctx, src, img, mode), want, tag=mode)


@pytest.mark.parametrize("q", [0.0, 0.3, 0.5, 0.86, 0.95, 1.0])
def test_percentile_atoms(ctx, q):
    rng = np.random.default_rng(int(q * 100))
    img = rng.random((2, 77, 130)).astype(np.float32) - 0.25
    img[1, :10] = 0.5  # ties
    img[0, 5, :7] = -0.0
    src = (f'output "a" intensity(img, 0) >. percentile(img, 0, {q})\n'
           f'output "b" intensity(img, 1) <=. percentile(img, 1, {q})\n'
           f'output "c" intensity(img, 1) >=. percentile(img, 0, {q})')
    assert_same(src, img, gpu_run(ctx, src, img, "graph"))
    u8 = rng.integers(0, 256, (1, 50, 90), dtype=np.uint8)
    src8 = f'output "a" intensity(img) >. percentile(img, 0, {q})'
    assert_same(src8, u8, gpu_run(ctx, src8, u8, "fused"))


def test_segmentation_formula_small(ctx):
    rng = np.random.default_rng(4)
    img = images.phantom_image(rng, 190, 257)
    src = formulas.segmentation_dag(4)
    want = oracle.run(src, img)
    for mode in MODES:
        assert_same(src, img, gpu_run(ctx, src, img, mode), want, tag=mode)


@pytest.mark.parametrize("seed", range(6))
def test_random_formulas(ctx, seed):
    rng = np.random.default_rng(100 + seed)
    h, w = int(rng.integers(1, 300)), int(rng.integers(1, 300))
    img = rng.random((2, h, w)).astype(np.float32)
    src = formulas.random_dag(seed, n_nodes=60, n_reach=6, channels=2)
    want = oracle.run(src, img)
    for mode in MODES:
        assert_same(src, img, gpu_run(ctx, src, img, mode), want, tag=f"{h}x{w} {mode}")


def test_ellipse_maze_full_size(ctx):
    img = images.ellipse_maze_image(2, 4096)
    src = formulas.ellipse_dag(2)
    want = oracle.run(src, img)
    assert_same(src, img, gpu_run(ctx, src, img, "graph"), want, tag="graph")
    assert_same(src, img, gpu_run(ctx, src, img, "perop"), want, tag="perop")


@pytest.mark.parametrize("h,w", [(1, 70), (3, 130), (65, 200), (2, 4097)])
def test_many_atoms_one_channel(ctx, h, w):
    # 40 thresholds of all four comparisons on one channel: two atom launches
    # (32 + 8), every mask compared
    rng = np.random.default_rng(h + w)
    img = rng.random((1, h, w)).astype(np.float32)
    img[0, 0, : min(w, 8)] = np.float32(0.5)  # ties with one threshold
    ops = [">.", "<.", ">=.", "<=."]
    lines = [f'output "a{i}" intensity(img) {ops[i % 4]} {0.5 if i == 7 else rng.uniform(0.02, 0.98):.6f}'
             for i in range(40)]
    src = "\n".join(lines)
    want = oracle.run(src, img)
    for mode in ("perop", "fused"):
        assert_same(src, img, gpu_run(ctx, src, img, mode), want, tag=f"{h}x{w} {mode}")


def test_labelling_reuse(ctx):
    # ten reach-type nodes over the same passable masks B and !B: the fused
    # schedule labels B once per run of users (at most 7 seed sets each)
    rng = np.random.default_rng(11)
    img = rng.random((3, 301, 257)).astype(np.float32)
    lines = ["let B = intensity(img, 0) >. 0.45", "let C = intensity(img, 1) >. 0.5"]
    outs = []
    for i in range(10):
        t = 0.97 + 0.002 * i
        lines.append(f"let S{i} = intensity(img, 2) >. {t:.4f}")
        op = ["reach(S{i}, B)", "grow(S{i}, B)", "surrounded(S{i} | C, B)", "reach(S{i}, !B)"][i % 4]
        outs.append(op.format(i=i))
    src = "\n".join(lines) + "\n" + "\n".join(f'output "o{i}" {o}' for i, o in enumerate(outs))
    import paper_2010_07284_amd as vlg
    st = vlg.formula_info(vlg.compile_formula(None, src))
    assert st["labelling_reuse"] >= 3
    want = oracle.run(src, img)
    for mode in MODES:
        assert_same(src, img, gpu_run(ctx, src, img, mode), want, tag=mode)


@pytest.mark.parametrize("tbh", [8, 16, 32])
def test_tile_heights_all_operators(ctx, tbh):
    import paper_2010_07284_amd as vlg
    rng = np.random.default_rng(tbh)
    img = images.smoothed_noise(rng, 389, 517, sigma=2.0)[None]
    img = np.concatenate([img, rng.random((1, 389, 517)).astype(np.float32)])
    src = ops_src(rng)
    vlg.set_tunable(ctx, "ccl_tile_rows", tbh)
    try:
        assert_same(src, img, gpu_run(ctx, src, img, "graph"), tag=f"tbh={tbh}")
    finally:
        vlg.set_tunable(ctx, "ccl_tile_rows", 0)


def test_autotune_picks_and_persists(ctx, tmp_path):
    import paper_2010_07284_amd as vlg
    img = images.ellipse_maze_image(2, 512)
    src = formulas.ellipse_dag(2)
    im = vlg.load_image(ctx, img)
    f = vlg.compile_formula(ctx, src)
    rep = vlg.autotune(ctx, f, im, iters=2)
    best, times = rep["ccl_tile_rows"]
    assert set(times) == {8, 16, 32} and best == min(times, key=times.get)
    assert vlg.get_tunable(ctx, "ccl_tile_rows", 512, 512) == best
    path = str(tmp_path / "tune.jsonl")
    vlg.tune_save(ctx, path)
    ctx2 = vlg.create()
    vlg.tune_load(ctx2, path)
    assert vlg.get_tunable(ctx2, "ccl_tile_rows", 512, 512) == best
    # results do not depend on the choice
    assert_same(src, img, gpu_run(ctx, src, img, "graph"))


@pytest.mark.parametrize("h,w", [(1, 65), (37, 200), (128, 128)])
def test_epilogue_fusion_patterns(ctx, h, w):
    rng = np.random.default_rng(h * w)
    img = rng.random((2, h, w)).astype(np.float32)
    src = """
    let A = intensity(img, 0) >. 0.6
    let B = intensity(img, 1) <. 0.5
    output "o1" near(A) & B
    output "o2" B | interior(A)
    output "o3" near(A) & near(B)
    output "o4" near(!A) & true
    output "o5" near(B) | false
    output "o6" !(interior(!B) & !A)
    output "o7" near(A | B) & !near(B)
    output "o8" near(near(A) & B) | interior(B)
    """
    want = oracle.run(src, img)
    for mode in MODES:
        assert_same(src, img, gpu_run(ctx, src, img, mode), want, tag=f"{h}x{w} {mode}")


@pytest.mark.parametrize("rows", [4, 8, 16, 32])
def test_near_band_rows_all_operators(ctx, rows):
    import paper_2010_07284_amd as vlg
    rng = np.random.default_rng(50 + rows)
    img = rng.random((2, 301, 200)).astype(np.float32)
    src = ops_src(rng)
    vlg.set_tunable(ctx, "near_band_rows", rows)
    try:
        assert vlg.get_tunable(ctx, "near_band_rows", 301, 200) == rows
        for mode in MODES:
            assert_same(src, img, gpu_run(ctx, src, img, mode), tag=f"rows={rows} {mode}")
    finally:
        vlg.set_tunable(ctx, "near_band_rows", 0)


def test_autotune_reports_near_rows(ctx, tmp_path):
    import paper_2010_07284_amd as vlg
    img = images.plain_image(7, 512)
    src = formulas.PLAIN_FORMULA
    f = vlg.compile_formula(ctx, src)
    rep = vlg.autotune(ctx, f, vlg.load_image(ctx, img), iters=2)
    best, times = rep["near_band_rows"]
    assert set(times) == {4, 8, 16, 32} and best == min(times, key=times.get)
    assert vlg.get_tunable(ctx, "near_band_rows", 512, 512) == best
    path = str(tmp_path / "tune.jsonl")
    vlg.tune_save(ctx, path)
    ctx2 = vlg.create()
    vlg.tune_load(ctx2, path)
    assert vlg.get_tunable(ctx2, "near_band_rows", 512, 512) == best
    assert_same(src, img, gpu_run(ctx2, src, img, "graph"))


@pytest.mark.skip(reason="written for the multi-stream lanes executor, which ended twice in a host-side "
                         "segmentation fault (cause not found) and is deleted; grouped labellings on one stream "
                         "are tested in tests/test_gpu_lanes.py")
@pytest.mark.parametrize("lanes", [2, 4])
def test_ccl_lanes_opt_in(ctx, lanes):
    # concurrent labelling lanes (opt-in tunable): segmentation, labelling
    # reuse and random formulas, every executor mode against the oracle
    import paper_2010_07284_amd as vlg
    cases = [(formulas.segmentation_dag(4), images.phantom_image(np.random.default_rng(4), 190, 257))]
    for seed in range(3):
        rng = np.random.default_rng(100 + seed)
        h, w = int(rng.integers(1, 300)), int(rng.integers(1, 300))
        cases.append((formulas.random_dag(seed, n_nodes=60, n_reach=6, channels=2),
                      rng.random((2, h, w)).astype(np.float32)))
    vlg.set_tunable(ctx, "ccl_lanes", lanes)
    try:
        for src, img in cases:
            want = oracle.run(src, img)
            for mode in ("fused", "graph"):
                assert_same(src, img, gpu_run(ctx, src, img, mode), want, tag=f"lanes={lanes} {mode}")
    finally:
        vlg.set_tunable(ctx, "ccl_lanes", 0)


@pytest.mark.parametrize("halo", [1, 2, 4, 8, 16])
def test_fused_segments_every_halo_cap(ctx, halo):
    # fused segments (runs of Boolean and near steps in one tile kernel) at
    # every halo cap: deep near chains, complements, ragged sizes around the
    # word and the tile, and the small chain workload
    import paper_2010_07284_amd as vlg
    rng = np.random.default_rng(halo)
    deep = ops_src(rng) + 'output "deep" near(near(near(near(near(A) & B) | C) & !D) | interior(interior(B)))\n'
    cases = [(deep, rng.random((2, 97, 301)).astype(np.float32)),
             (deep, rng.random((2, 3, 65)).astype(np.float32)),
             (formulas.chain_dag(3, n_chain=300, n_reach=15), images.random_mask_image(3, 300)),
             (formulas.random_dag(7, n_nodes=120, n_reach=4, channels=2),
              rng.random((2, 517, 389)).astype(np.float32))]
    vlg.set_tunable(ctx, "fuse_halo", halo)
    try:
        for src, img in cases:
            want = oracle.run(src, img)
            for mode in ("fused", "graph"):
                assert_same(src, img, gpu_run(ctx, src, img, mode), want, tag=f"halo={halo} {mode} {img.shape}")
    finally:
        vlg.set_tunable(ctx, "fuse_halo", 0)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("h,w", [(1, 70), (37, 129), (300, 257)])
def test_uint16_images(ctx, mode, h, w):
    # the paper's pixel type: atoms of every comparison at uint16 thresholds
    # and between them, two-pass percentiles, the grow specification
    rng = np.random.default_rng(h + 3 * w)
    img = rng.integers(0, 65536, (2, h, w), dtype=np.uint16)
    img[0, 0, : min(w, 5)] = 62258  # ties with the threshold
    img[1, -1, :3] = 56360
    src = ("let hI = intensity(img) >. 62258\n"
           "let vI = intensity(img) >. 56360\n"
           'output "grow" grow(hI, vI)\n'
           'output "ge" intensity(img, 1) >=. 56360\n'
           'output "le" intensity(img, 1) <=. 1000.5\n'
           'output "pct" intensity(img, 0) >. percentile(img, 0, 0.95)\n'
           'output "pct1" intensity(img, 1) <. percentile(img, 1, 0.86)\n'
           'output "mix" near(intensity(img, 0) <. percentile(img, 1, 0.3)) & !vI\n')
    assert_same(src, img, gpu_run(ctx, src, img, mode), tag=f"u16 {h}x{w} {mode}")


def test_uint16_batch(ctx):
    import paper_2010_07284_amd as vlg
    rng = np.random.default_rng(16)
    imgs = [rng.integers(0, 65536, (1, h, w), dtype=np.uint16) for h, w in [(64, 64), (130, 77), (300, 513)]]
    src = formulas.GROW_SPEC.format(hi=62258, lo=56360) + 'output "p" intensity(img) >. percentile(img, 0, 0.86)\n'
    f = vlg.compile_formula(ctx, src)
    ims = [vlg.load_image(ctx, im) for im in imgs]
    for mode in ("fused", "graph"):
        vlg.set_mode(ctx, mode)
        outs = vlg.check_batch(ctx, f, ims)
        vlg.sync(ctx)
        for im, row in zip(imgs, outs):
            want = oracle.run(src, im)
            H, W = im.shape[1:]
            for k, (o, wm) in enumerate(zip(row, want)):
                assert np.array_equal(vlg.unpack(o, H, W), wm), (im.shape, k, mode)
