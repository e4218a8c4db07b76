#!/usr/bin/env python3
"""Benchmark of SLCS formula evaluation on one MI355X.

Workload (default): one 4096x4096 float32 image with three channels
(smoothed noise plus 200 ellipses of distinct intensities; a serpentine maze;
a seed pixel) and a 100-node formula with 10 reachability-type operators,
generated from seed 2.  A step evaluates every output of the formula on the
resident image (graph executor).  Metric: Gpixel-node evaluations per second
= H * W * (DAG nodes after hash-consing) / time per step.

Before timing, every output is compared bit for bit with the CPU oracle
(which is also timed, single-threaded, as the CPU baseline).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


KERNEL_OF_KIND = {"atoms": "k_atoms<{t}>", "logic": "k_logic", "near": "k_near", "ccl_local": "k_ccl_local<{tbh}>",
                  "ccl_merge": "k_ccl_merge<{tbh}>", "ccl_flag": "k_ccl_flag", "ccl_gather": "k_ccl_gather",
                  "ccl_reseed": "k_ccl_reseed"}


def measured_traffic(workload, kind, tbh, dtype="float"):
    """HBM bytes per dispatch of the kernel behind `kind`, from the committed
    rocprofv3 counter summary of `workload` (FETCH_SIZE and WRITE_SIZE scaled
    by a 1 GiB copy), or None when there is none or the kernel source has
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{workload}_hbm_traffic.json")
    if kind not in KERNEL_OF_KIND or not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    h = hashlib.sha256()
    for src in rec.get("sources", ["paper_2010_07284_amd/csrc/kernels.hip"]):
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec.get("kernels_source_sha256"):
        return None
    k = rec["per_dispatch"].get(KERNEL_OF_KIND[kind].format(tbh=tbh, t=dtype))
    return None if k is None else k["read_bytes"] + k["write_bytes"]


def time_mode(vlg, lib, ctx, f, im, arr, mode, steps, warmup):
    import torch
    vlg.set_mode(ctx, mode)
    for _ in range(warmup):
        rc = lib.vlg_check_all(ctx.handle, f.handle, im.handle, arr, 0, 1)
        if rc:
            raise RuntimeError(lib.vlg_last_error().decode())
    vlg.sync(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        lib.vlg_check_all(ctx.handle, f.handle, im.handle, arr, 0, 1)
    vlg.sync(ctx)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def load_digests():
    """Expected-mask digests of the full-size workloads, written by
    tests/golden/make_digests.py from the CPU oracle."""
    with open(os.path.join(ROOT, "tests", "golden", "digests.json")) as fh:
        return json.load(fh)["cases"]


def packed_digest(t):
    return hashlib.sha256(t.cpu().numpy().astype("<i8").tobytes()).hexdigest()


def check_digests(key, outs, digests, tag):
    want = digests[key]["outputs"]
    bad = [k for k, (o, w) in enumerate(zip(outs, want)) if packed_digest(o) != w]
    if len(outs) != len(want) or bad:
        raise SystemExit(f"[bench] PARITY FAILURE: {key} {tag}: outputs {bad} differ from the oracle")


def bench_chain(vlg, lib, steps, check_oracle):
    """Sequential large formula: 1024x1024 uint8 random mask (density 0.5),
    10,000 rotating near/and/not elements plus 500 reach elements; per-op
    launches against the fused schedule and its hipGraph.  Every output of
    every executor is first compared with the oracle's digests; compile time
    (parse, hash-consing, both schedules) and graph build time (capture and
    instantiation) are reported beside the evaluation time."""
    import torch
    from synth import formulas, images
    img = images.random_mask_image(3, 1024)
    src = formulas.chain_dag(3)
    ctx = vlg.create(0)
    im = vlg.load_image(ctx, torch.from_numpy(img).to("cuda:0"))
    t0 = time.perf_counter()
    f = vlg.compile_formula(ctx, src)
    info = vlg.formula_info(f)  # builds the per-op and fused schedules
    compile_ms = (time.perf_counter() - t0) * 1e3
    nout = info["outputs"]
    outs = [torch.empty((1024, 16), dtype=torch.int64, device="cuda:0") for _ in range(nout)]
    arr = (ctypes.c_void_p * nout)(*[o.data_ptr() for o in outs])
    digests = load_digests() if check_oracle else None
    tune = vlg.autotune(ctx, f, im, iters=2)
    for name, (best, times) in tune.items():
        log(f"[bench] chain_1024 autotune: {name} {best} "
            f"({', '.join(f'{k}: {v:.2f} ms' for k, v in sorted(times.items()))})")
    first_ms = {}
    for m in ("perop", "fused", "graph"):
        vlg.set_mode(ctx, m)
        vlg.sync(ctx)
        t0 = time.perf_counter()
        rc = lib.vlg_check_all(ctx.handle, f.handle, im.handle, arr, 0, 1)
        if rc:
            raise RuntimeError(lib.vlg_last_error().decode())
        vlg.sync(ctx)
        first_ms[m] = (time.perf_counter() - t0) * 1e3
        if check_oracle:
            check_digests("chain_1024", outs, digests, m)
    if check_oracle:
        log("[bench] chain_1024 parity: every output bit-exact (oracle digests) in perop, fused and graph")
    ms = {m: time_mode(vlg, lib, ctx, f, im, arr, m, steps, 1) for m in ("perop", "fused", "graph")}
    for m, t in ms.items():
        log(f"[bench] chain_1024 {m}: {t:.3f} ms/evaluation")
    halo = vlg.get_tunable(ctx, "fuse_halo", 1024, 1024)
    launches_tuned = len(vlg.formula_plan(f, "fused", halo)["steps"])
    # fused segments with halo cap 8, whether or not the tuner picked them
    vlg.set_tunable(ctx, "fuse_halo", 8)
    if check_oracle:
        vlg.set_mode(ctx, "graph")
        lib.vlg_check_all(ctx.handle, f.handle, im.handle, arr, 0, 1)
        vlg.sync(ctx)
        check_digests("chain_1024", outs, digests, "graph, segments")
    seg_ms = time_mode(vlg, lib, ctx, f, im, arr, "graph", steps, 1)
    seg_launches = len(vlg.formula_plan(f, "fused", 8)["steps"])
    vlg.set_tunable(ctx, "fuse_halo", 0)
    log(f"[bench] chain_1024 graph with segments (halo cap 8): {seg_ms:.3f} ms, {seg_launches} steps")
    return {"workload": f"chain_1024: 1024x1024 u8 random mask, {info['nodes']}-node chain "
                        f"({info['reach_nodes']} reach), {nout} outputs",
            "nodes": info["nodes"], "launches_perop": info["steps_perop"], "launches_fused": launches_tuned,
            "tuned": {k: v[0] for k, v in tune.items()},
            "graph_ms_with_segments": round(seg_ms, 3), "steps_with_segments": seg_launches,
            "parity": "oracle digests, every output, every executor" if check_oracle else None,
            "compile_ms": round(compile_ms, 2),
            "graph_build_ms": round(first_ms["graph"] - ms["graph"], 2),
            "perop_ms": round(ms["perop"], 3), "fused_ms": round(ms["fused"], 3), "graph_ms": round(ms["graph"], 3),
            "speedup_graph_vs_perop": round(ms["perop"] / ms["graph"], 3),
            "gpixel_node_per_s": round(1024 * 1024 * info["nodes"] / (ms["graph"] / 1e3) / 1e9, 3)}


def _oracle_run_one(src, img):
    import oracle
    oracle.run(src, img)
    return 0


def bench_batch(vlg, lib, steps, check_oracle, seed=4, n=512, square=False):
    """Uneven batch: `n` phantom images (sides uniform in [128, 2048], four
    float32 channels, generated in device memory) and the shared 60-node
    segmentation formula.  One vlg_check_batch call per step: per-image
    per-op launches (the baseline) against the batched fused schedule and its
    hipGraph.  Sampled images are checked against the oracle first."""
    import numpy as np
    import torch
    from synth import formulas, images
    sizes = images.batch_sizes(seed, n, 128, 2048, square=square)
    src = formulas.segmentation_dag(seed)
    ctx = vlg.create(0)
    f = vlg.compile_formula(ctx, src)
    info = vlg.formula_info(f)
    nodes, nout = info["nodes"], info["outputs"]
    log(f"[bench] batch: generating {n} phantom images on the device")
    order = sorted(range(n), key=lambda i: sizes[i][0] * sizes[i][1])
    sample = sorted({order[0], order[n // 2], order[-1]})
    # images timed with the oracle on the host cores: every 16th image
    cpu_sample = list(range(0, n, 16)) if check_oracle and not square else []
    ims, host = [], {}
    for i, (h, w) in enumerate(sizes):
        t = images.phantom_image_device(seed, i, h, w, device="cuda:0")
        ims.append(vlg.load_image(ctx, t))
        if i in sample or i in cpu_sample:
            host[i] = t.cpu().numpy()
        del t
    torch.cuda.empty_cache()
    outs = [[torch.empty((h, (w + 63) // 64), dtype=torch.int64, device="cuda:0") for _ in range(nout)]
            for h, w in sizes]
    flat = (ctypes.c_void_p * (n * nout))(*[o.data_ptr() for row in outs for o in row])
    harr = (ctypes.c_void_p * n)(*[im.handle.value for im in ims])
    # autotune the labelling tile on the batch itself
    tune = vlg.autotune_batch(ctx, f, ims, iters=1)
    for name, (best, times) in tune.items():
        log(f"[bench] batch: autotuned {name} {best} "
            f"({', '.join(f'{k}: {v:.2f} ms' for k, v in sorted(times.items()))})")

    def step():
        rc = lib.vlg_check_batch(ctx.handle, f.handle, harr, n, flat, 0, 1)
        if rc:
            raise RuntimeError(lib.vlg_last_error().decode())

    if check_oracle:
        import oracle
        for mode in ("perop", "graph"):
            vlg.set_mode(ctx, mode)
            step()
            vlg.sync(ctx)
            for i in sample:
                want = oracle.run(src, host[i])
                h, w = sizes[i]
                for k in range(nout):
                    if not np.array_equal(vlg.unpack(outs[i][k], h, w), want[k]):
                        raise SystemExit(f"[bench] PARITY FAILURE: batch {mode} image {i} output {k}")
        log(f"[bench] batch parity: images {sample} bit-exact (perop and graph)")
    cpu = None
    if cpu_sample:
        # the oracle on all host cores, one image per worker process
        import multiprocessing as mp
        cores = max(1, min(16, len(os.sched_getaffinity(0))))
        imgs = [host[i] for i in cpu_sample]
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(cores) as pool:
            pool.starmap(_oracle_run_one, [(src, x) for x in imgs])
        t_cpu = time.perf_counter() - t0
        px_s = sum(x.shape[1] * x.shape[2] for x in imgs)
        cpu = {"value": round(px_s * nodes / t_cpu / 1e9, 4), "unit": "Gpixel-node evals/s", "cores": cores,
               "kind": "oracle", "images_per_s": round(len(imgs) / t_cpu, 2),
               "sample": f"every 16th image of the batch ({len(imgs)} images, {px_s / 1e6:.1f} Mpx) on {cores} "
                         f"worker processes of {cpu_model()}, one image per process, {t_cpu:.1f} s"}
        log(f"[bench] batch oracle on {cores} host cores: {cpu}")
    ms = {}
    for mode in ("perop", "fused", "graph"):
        vlg.set_mode(ctx, mode)
        step()
        vlg.sync(ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        vlg.sync(ctx)
        torch.cuda.synchronize()
        ms[mode] = (time.perf_counter() - t0) * 1e3 / steps
        log(f"[bench] batch {mode}: {ms[mode]:.3f} ms per batch")
    # per-kind rates of the batched kernels: HIP events around every launch
    # of the batched schedule (fused, no graph)
    kb = {}
    for k, (nl, t, b) in vlg.profile_batch(ctx, f, ims, iters=2).items():
        kb[k] = {"launches_per_batch": nl // 2, "avg_launch_us": round(t / nl * 1e3, 2),
                 "ms_per_batch": round(t / 2, 3),
                 "achieved_gbs": round(b / (t / 1e3) / 1e9, 1) if t > 0 else None,
                 "frac": round(b / (t / 1e3) / 1e9 / HBM_PEAK_GBS, 4) if t > 0 else None}
    log(f"[bench] batch kernels: {kb}")
    px = sum(h * w for h, w in sizes)
    res = {"workload": f"uneven_batch_{n}{'_square' if square else ''}: {n} phantom images, "
                       f"{'square sides' if square else 'sides H, W'} U[128,2048], f32 x4 channels, "
                       f"{nodes}-node segmentation formula, {nout} outputs",
           "images": n, "gpixels": round(px / 1e9, 4), "nodes": nodes,
           "ccl_tile_rows": tune["ccl_tile_rows"][0], "batch_grid": tune["batch_grid"][0],
           "perop_ms": round(ms["perop"], 3), "fused_ms": round(ms["fused"], 3), "graph_ms": round(ms["graph"], 3),
           "speedup_graph_vs_perop": round(ms["perop"] / ms["graph"], 3),
           "gpixel_node_per_s": round(px * nodes / (ms["graph"] / 1e3) / 1e9, 3),
           "images_per_s": round(n / (ms["graph"] / 1e3), 1), "cpu_baseline_all_cores": cpu,
           "kernels_with_per_launch_events": kb}
    del outs, ims
    torch.cuda.empty_cache()
    return res


def bench_pixelwise(vlg, iters, side=46080):
    """Streaming roofline of the pixel-wise kernels on one side x side float32
    channel (side 46080: 2^31 - 24M pixels, the largest square image; 8.5 GB
    channel, 265 MB per mask, far above the 256 MB last-level cache): the
    threshold atom, N and a Boolean connective, timed per launch with HIP
    events, against algorithmic bytes (channel read once, masks read/written
    once)."""
    import torch
    src = ('let A = intensity(img) >. 0.5\n'
           'let D = near(A)\n'
           'output "atom" A\noutput "near" D\noutput "and" A & !D\n')
    ctx = vlg.create(0)
    t = torch.rand((1, side, side), device="cuda:0", dtype=torch.float32)
    im = vlg.load_image(ctx, t)
    del t
    torch.cuda.empty_cache()
    f = vlg.compile_formula(ctx, src)
    vlg.profile(ctx, f, im, iters=1)
    prof = vlg.profile(ctx, f, im, iters=iters)
    res = {"workload": f"pixelwise_{side}: {side}x{side} f32 channel, one atom, N, and-not",
           "peak_gbs": HBM_PEAK_GBS}
    for k, (n, ms, b) in prof.items():
        gbs = b / (ms / 1e3) / 1e9
        res[k] = {"avg_launch_us": round(ms / n * 1e3, 2), "bytes_per_launch": round(b / n),
                  "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
        log(f"[bench] pixelwise {k:8s} {ms / n * 1e3:9.1f} us/launch  {gbs:7.1f} GB/s  "
            f"({gbs / HBM_PEAK_GBS:.1%} of HBM peak)")
    # each kernel launched back to back (the step alone, repeated): without
    # the write-back of the previous kernel's output inside its time
    for k in ("atoms", "near", "logic"):
        try:
            bb_ms, bb = vlg.profile_step(ctx, f, im, k, reps=iters)
        except vlg.VlgError:
            continue
        gbs = bb / (bb_ms / 1e3) / 1e9
        res[k]["back_to_back"] = {"avg_launch_us": round(bb_ms * 1e3, 1), "achieved_gbs": round(gbs, 1),
                                  "frac": round(gbs / HBM_PEAK_GBS, 4)}
        log(f"[bench] pixelwise {k:8s} back to back {bb_ms * 1e3:9.1f} us/launch  {gbs:7.1f} GB/s  "
            f"({gbs / HBM_PEAK_GBS:.1%} of HBM peak)")
    # the whole pass (atom, N, connective): a launch that streams past the
    # last-level cache leaves the write-back of its output to the next one,
    # so the per-kernel rates shift cost between neighbours; the sum does not
    tb = sum(b for _, _, b in prof.values())
    tms = sum(ms for _, ms, _ in prof.values())
    gbs = tb / (tms / 1e3) / 1e9
    res["pass"] = {"us_per_pass": round(tms / iters * 1e3, 1), "bytes_per_pass": round(tb / iters),
                   "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    log(f"[bench] pixelwise pass     {tms / iters * 1e3:9.1f} us/pass    {gbs:7.1f} GB/s  "
        f"({gbs / HBM_PEAK_GBS:.1%} of HBM peak)")
    # references: the library's own non-temporal copy kernel (16- and 8-byte
    # accesses) and torch's device-to-device copy, each over 4 GiB: what
    # streaming reaches on this device
    a = torch.empty(1 << 30, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    nbytes = a.numel() * 4
    for width in (16, 8):
        ms = vlg.stream_copy(ctx, b, a, width=width, reps=iters)
        gbs = 2 * nbytes / (ms / 1e3) / 1e9
        res[f"stream_copy_{width}B_4GiB"] = {"avg_launch_us": round(ms * 1e3, 1), "achieved_gbs": round(gbs, 1),
                                            "frac": round(gbs / HBM_PEAK_GBS, 4)}
        log(f"[bench] pixelwise reference stream copy ({width} B accesses): {gbs:7.1f} GB/s "
            f"({gbs / HBM_PEAK_GBS:.1%} of HBM peak)")
    if not torch.equal(a, b):
        raise RuntimeError("stream copy: destination differs from source")
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(iters):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    gbs = 2 * nbytes / (ms / 1e3) / 1e9
    res["torch_copy_4GiB"] = {"avg_launch_us": round(ms * 1e3, 1), "achieved_gbs": round(gbs, 1),
                              "frac": round(gbs / HBM_PEAK_GBS, 4)}
    log(f"[bench] pixelwise reference torch copy: {gbs:7.1f} GB/s ({gbs / HBM_PEAK_GBS:.1%} of HBM peak)")
    del a, b, im, f, ctx
    torch.cuda.empty_cache()
    return res


def bench_paper_grow(vlg, lib, steps, check_oracle, side=7680):
    """The paper's specification workload (Sect. 4.2, Fig. specification): one
    7680x7680 uint16 image, hI = >.62258, vI = >.56360, grow(hI, vI).  The
    MRI slice is not available: a phantom (ellipses of intensities 0.2-1 with
    Rician-like noise) scaled to the uint16 range stands in for it.  Reports
    the device-resident evaluation, the evaluation with the byte mask copied
    to host memory, and, as in the paper's protocol (start of computation to
    result saved), upload of the uint16 slice from host memory + evaluation
    + readback."""
    import numpy as np
    import torch
    from synth import formulas, images
    host = images.paper_slice_u16(side)
    ctx = vlg.create(0)
    im = vlg.load_image(ctx, host)
    src = formulas.GROW_SPEC.format(hi=62258, lo=56360)
    f = vlg.compile_formula(ctx, src)
    dev = torch.empty((side, (side + 63) // 64), dtype=torch.int64, device="cuda:0")
    hst = torch.empty((side, side), dtype=torch.uint8).pin_memory()
    arr_d = (ctypes.c_void_p * 1)(dev.data_ptr())
    arr_h = (ctypes.c_void_p * 1)(hst.data_ptr())
    vlg.set_mode(ctx, "graph")
    if check_oracle:
        import oracle
        want = oracle.run(src, host)[0]
        lib.vlg_check_all(ctx.handle, f.handle, im.handle, arr_h, 1, 0)
        if not np.array_equal(hst.numpy(), want):
            raise SystemExit("[bench] PARITY FAILURE: paper grow workload")
        log("[bench] paper grow (uint16): bit-exact against the oracle")
    ms_dev = time_mode(vlg, lib, ctx, f, im, arr_d, "graph", steps, 2)
    for _ in range(2):
        lib.vlg_check_all(ctx.handle, f.handle, im.handle, arr_h, 1, 0)
    t0 = time.perf_counter()
    for _ in range(steps):
        lib.vlg_check_all(ctx.handle, f.handle, im.handle, arr_h, 1, 0)
    ms_host = (time.perf_counter() - t0) * 1e3 / steps
    # the paper's protocol: the slice starts in host memory (pinned here)
    pinned = torch.from_numpy(host.view(np.int16)).pin_memory()
    src_ptr = ctypes.c_void_p(pinned.data_ptr())
    h = ctypes.c_void_p()
    t0 = time.perf_counter()
    for _ in range(steps):
        rc = lib.vlg_load_image(ctx.handle, src_ptr, 2, 1, side, side, side, 0, ctypes.byref(h))
        if rc != 0:
            raise SystemExit(f"[bench] vlg_load_image failed: {rc}")
        lib.vlg_check_all(ctx.handle, f.handle, h, arr_h, 1, 0)
        lib.vlg_image_free(h)
    ms_e2e = (time.perf_counter() - t0) * 1e3 / steps
    log(f"[bench] paper grow {side}^2 uint16: {ms_dev:.3f} ms resident, {ms_host:.3f} ms with the byte mask "
        f"copied to host, {ms_e2e:.3f} ms host slice in to host mask out")
    return {"workload": f"paper_grow_{side}: {side}x{side} uint16 phantom, grow(>.62258, >.56360)",
            "device_ms": round(ms_dev, 3), "with_host_readback_ms": round(ms_host, 3),
            "host_to_host_ms": round(ms_e2e, 3),
            "mpixel_per_s": round(side * side / (ms_dev / 1e3) / 1e6, 1),
            "paper_context": "about 600 ms on a TITAN Xp and 3 s on an HD Graphics 630 for the same shape, "
                             "start of computation to file saved (OpenCL, uint16 MRI slice)"}


def bench_pj(vlg, lib, check_oracle, side=2048):
    """The paper's own labelling (Sect. 3, Alg. CCL) against the union-find
    labelling on the same masks: a 2048x2048 mask (the size of Fig.
    cc-movie, whose test image is not available: thresholded smooth noise)
    with reconnect every 8 main iterations as in the figure and every 16 as
    in the text, and the 4096^2 serpentine corridor of the headline.  Main
    iterations, rounds (each ends with the host waiting for the termination
    check, as in the paper's tool), launches and wall time per labelling."""
    import numpy as np
    import torch
    from synth import images
    ctx = vlg.create(0)
    out = {}
    masks = {f"noise_{side}": (images.plain_image(7, side)[0] > np.float32(0.5)).astype(np.uint8),
             "maze_4096": images.serpentine_maze(4096, 4096).astype(np.uint8)}
    for name, m in masks.items():
        H, W = m.shape
        words = torch.from_numpy(vlg.pack(m)).to("cuda:0")
        lab = torch.empty((H, W), dtype=torch.int32, device="cuda:0")
        row = {}
        for k in (8, 16):
            vlg.ccl_labels_pj(ctx, words, H, W, k, out=lab)  # warm-up
            vlg.sync(ctx)
            t0 = time.perf_counter()
            reps = 3
            for _ in range(reps):
                _, st = vlg.ccl_labels_pj(ctx, words, H, W, k, out=lab)
            vlg.sync(ctx)
            ms = (time.perf_counter() - t0) * 1e3 / reps
            row[f"reconnect_every_{k}"] = {"main_iterations": st["main_iterations"], "rounds": st["rounds"],
                                           "launches": st["launches"], "ms": round(ms, 3)}
            if check_oracle and name.startswith("noise"):
                import oracle
                want, iters = oracle.ccl_pj(m, k=k)
                if iters != st["main_iterations"] or not np.array_equal(lab.cpu().numpy(), want):
                    raise SystemExit(f"[bench] PARITY FAILURE: pointer-jumping labelling {name} k={k}")
                row[f"reconnect_every_{k}"]["parity"] = "labels and iteration count equal the oracle's run"
        uf = torch.empty((H, W), dtype=torch.int32, device="cuda:0")
        vlg.ccl_labels(ctx, words, H, W, out=uf)
        vlg.sync(ctx)
        t0 = time.perf_counter()
        for _ in range(20):
            vlg.ccl_labels(ctx, words, H, W, out=uf)
        vlg.sync(ctx)
        row["union_find_ms"] = round((time.perf_counter() - t0) * 1e3 / 20, 3)
        log(f"[bench] paper labelling {name}: {row}")
        out[name] = row
    out["paper_context"] = "Fig. cc-movie: 24 iterations (reconnect every 8) on the paper's 2048x2048 test image"
    return out


def bench_volume(vlg, lib, steps, check_oracle, side=256, check_side=96):
    """The logic on volumes: a two-channel ellipsoid phantom of side^3 voxels
    and an 18-node segmentation-shaped formula (percentile thresholds,
    arithmetic, N and interior over 26 neighbours, grow, surrounded, touch,
    reach through 26-connected components).  Parity against the oracle on a
    check_side^3 volume of the same recipe first (the oracle on side^3 takes
    minutes)."""
    import numpy as np
    from synth import formulas, images
    src = formulas.VOLUME_FORMULA
    ctx = vlg.create(0)
    f = vlg.compile_formula(ctx, src)
    info = vlg.formula_info(f)
    nout = info["outputs"]
    if check_oracle:
        import oracle
        v = images.volume_phantom_device(8, check_side, check_side, check_side).cpu().numpy()
        want = oracle.run3(src, v)
        im = vlg.load_volume(ctx, v)
        for mode in ("perop", "graph"):
            vlg.set_mode(ctx, mode)
            got = vlg.check_all(ctx, f, im)
            vlg.sync(ctx)
            for k in range(nout):
                g = vlg.unpack(got[k], check_side * check_side, check_side).reshape(v.shape[1:])
                if not np.array_equal(g, want[k]):
                    raise SystemExit(f"[bench] PARITY FAILURE: volume {check_side}^3 {mode} output {k}")
        log(f"[bench] volume {check_side}^3: bit-exact against the oracle (perop, graph)")
    vol = images.volume_phantom_device(8, side, side, side)
    im = vlg.load_volume(ctx, vol)
    del vol
    outs = [torch_empty_mask(side * side, side) for _ in range(nout)]
    arr = (ctypes.c_void_p * nout)(*[o.data_ptr() for o in outs])
    res = {"workload": f"volume_{side}: {side}^3 f32 x2 ellipsoid phantom, {info['nodes']}-node formula "
                       f"({info['reach_nodes']} reach-type), {nout} outputs",
           "nodes": info["nodes"]}
    for mode in ("perop", "graph"):
        res[f"{mode}_ms"] = round(time_mode(vlg, lib, ctx, f, im, arr, mode, steps, 2), 3)
    res["gvoxel_node_per_s"] = round(side ** 3 * info["nodes"] / (res["graph_ms"] / 1e3) / 1e9, 2)
    prof = vlg.profile(ctx, f, im, iters=3)
    res["kernels"] = {k: {"launches": n // 3, "avg_us": round(t / n * 1e3, 2),
                          "gbs": round(b / (t / 1e3) / 1e9, 1) if t else None} for k, (n, t, b) in prof.items()}
    log(f"[bench] volume {side}^3: {res}")
    return res


def torch_empty_mask(rows, width):
    import torch
    return torch.empty((rows, (width + 63) // 64), dtype=torch.int64, device="cuda:0")


def bench_arith(vlg, lib, steps, check_oracle, side=4096):
    """Arithmetic atoms and touch on a two-channel 4096^2 float32 image
    (smoothed noise and the ellipse channel of the headline workload)."""
    import numpy as np
    from synth import formulas, images
    img = images.ellipse_maze_image(2, side)[[0]]
    img = np.concatenate([img, images.plain_image(9, side)]).astype(np.float32)
    src = formulas.ARITH_FORMULA.format(t0=0.55, t1=-0.2, t2=0.35, t3=0.4)
    ctx = vlg.create(0)
    f = vlg.compile_formula(ctx, src)
    info = vlg.formula_info(f)
    nout = info["outputs"]
    im = vlg.load_image(ctx, img)
    outs = [torch_empty_mask(side, side) for _ in range(nout)]
    arr = (ctypes.c_void_p * nout)(*[o.data_ptr() for o in outs])
    if check_oracle:
        import oracle
        want = oracle.run(src, img)
        vlg.set_mode(ctx, "graph")
        lib.vlg_check_all(ctx.handle, f.handle, im.handle, arr, 0, 1)
        vlg.sync(ctx)
        for k in range(nout):
            if not np.array_equal(vlg.unpack(outs[k], side, side), want[k]):
                raise SystemExit(f"[bench] PARITY FAILURE: arithmetic workload output {k}")
        log("[bench] arithmetic workload: bit-exact against the oracle")
    res = {"workload": f"arith_{side}: {side}x{side} f32 x2, {info['nodes']}-node formula with arithmetic atoms "
                       f"and touch, {nout} outputs", "nodes": info["nodes"]}
    for mode in ("perop", "graph"):
        res[f"{mode}_ms"] = round(time_mode(vlg, lib, ctx, f, im, arr, mode, steps, 2), 4)
    res["gpixel_node_per_s"] = round(side * side * info["nodes"] / (res["graph_ms"] / 1e3) / 1e9, 1)
    prof = vlg.profile(ctx, f, im, iters=3)
    if "arith" in prof:
        n, t, b = prof["arith"]
        res["arith_kernel"] = {"launches": n // 3, "avg_us": round(t / n * 1e3, 2),
                               "gbs": round(b / (t / 1e3) / 1e9, 1)}
    log(f"[bench] arithmetic {side}^2: {res}")
    return res


def ccl_merge_counts(vlg, lib, src, img):
    """Cross-tile merge work per labelling: unions attempted and hook retries
    (compare-and-swap losses plus re-walks), from the library's device
    counters, for one fused evaluation of `src` on `img` and for the
    labelling of a serpentine maze of the same size (one component crossing
    every tile)."""
    import torch
    from synth import images
    os.environ["VLG_CCL_COUNTERS"] = "1"
    try:
        ctx = vlg.create(0)
    finally:
        del os.environ["VLG_CCL_COUNTERS"]
    C, H, W = img.shape
    im = vlg.load_image(ctx, torch.from_numpy(img).to("cuda:0"))
    f = vlg.compile_formula(ctx, src)
    info = vlg.formula_info(f)
    vlg.set_mode(ctx, "fused")
    vlg.ccl_counters(ctx)  # clears them
    vlg.check_all(ctx, f, im)
    vlg.sync(ctx)
    c = vlg.ccl_counters(ctx)
    nl = max(1, info["labellings"])
    res = {"labellings": info["labellings"], "merge_unions_per_labelling": round(c["merge_unions"] / nl),
           "merge_retries_per_labelling": round(c["merge_retries"] / nl),
           "launches_per_labelling": c["launches_per_ccl"]}
    maze = (images.serpentine_maze(H, W) > 0).astype("uint8")
    packed = torch.from_numpy(vlg.pack(maze)).to("cuda:0")
    vlg.ccl_counters(ctx)
    vlg.ccl_labels(ctx, packed, H, W)
    vlg.sync(ctx)
    c = vlg.ccl_counters(ctx)
    res["maze"] = {"merge_unions": c["merge_unions"], "merge_retries": c["merge_retries"]}
    log(f"[bench] labelling counters: {res}")
    del im, f, ctx
    return res


def _oracle_serve_one(src, side, index):
    import oracle
    from synth import images
    oracle.run(src, images.serve_image(index, side))
    return 0


def serve_cpu_baseline(formula_srcs, nodes, sides, max_side=2048):
    """The oracle on the host cores for the serving mix, on a bounded sample:
    every formula of the mix on every image of side <= max_side, one request
    per worker process.  Reports pixel-node evaluations per second, and the
    request rate that throughput gives for the mix (requests drawn uniformly
    over images and formulas, as the serving leg draws them)."""
    import multiprocessing as mp
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    jobs = [(src, sd, i) for i, sd in enumerate(sides) if sd <= max_side for src in formula_srcs]
    work = sum(sd * sd * n for i, sd in enumerate(sides) if sd <= max_side for n in nodes)
    # largest requests first, so that the pool does not end on one of them
    order = sorted(range(len(jobs)), key=lambda j: -jobs[j][1] * jobs[j][1] * nodes[j % len(nodes)])
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        pool.starmap(_oracle_serve_one, [jobs[j] for j in order])
    t_cpu = time.perf_counter() - t0
    rate = work / t_cpu
    mean_work = sum(sd * sd * n for sd in sides for n in nodes) / (len(sides) * len(nodes))
    return {"value": round(rate / 1e9, 4), "unit": "Gpixel-node evals/s", "cores": cores, "kind": "oracle",
            "req_per_s_for_mix": round(rate / mean_work, 3),
            "sample": f"{len(jobs)} requests: every formula on every image of side <= {max_side} "
                      f"({work / 1e9:.1f} G pixel-node evaluations), one request per worker process on {cores} "
                      f"processes of {cpu_model()}, {t_cpu:.1f} s; the mix rate divides by the mean request "
                      f"({mean_work / 1e9:.2f} G pixel-node evaluations)"}


def bench_serve(vlg, n_req, check_oracle, n_warm=200, seed=5, slots=4, budget=16 << 30, fracs=(0.5, 0.8, 0.95)):
    """Serving loop: Poisson arrivals over a pool of resident images (sides
    256 .. 8192, float32) and formulas (node counts log-uniform in [20, 2000]
    with up to 50 reach-type nodes, plus one 2000-node formula with 50);
    saturation throughput first, then p50/p99 latency (scheduled arrival to
    outputs written) and throughput at fractions of it, each level over n_req
    requests after n_warm warm-up requests.  One request per level writes to
    buffers of its own and is compared with the oracle's digests."""
    import numpy as np
    import torch
    from synth import formulas, images
    rng = np.random.default_rng(seed)
    ctx = vlg.create(0)
    sides = list(formulas.SERVE_SIDES)
    imgs = [vlg.load_image(ctx, torch.from_numpy(images.serve_image(i, sd)).to("cuda:0"))
            for i, sd in enumerate(sides)]
    fsrc = [src for src, _, _ in formulas.serve_formulas(seed)]
    fs = [vlg.compile_formula(ctx, src) for src in fsrc]
    nouts = [vlg.formula_info(f)["outputs"] for f in fs]
    nodes = [vlg.formula_info(f)["nodes"] for f in fs]
    digests = load_digests() if check_oracle else None
    ring = 8
    bufs = {}

    def fresh(i, k):
        C, H, W = imgs[i].shape
        return [torch.empty((H, (W + 63) // 64), dtype=torch.int64, device="cuda:0") for _ in range(nouts[k])]

    def outs_for(i, k, r):
        key = (i, k, r % ring)
        if key not in bufs:
            bufs[key] = fresh(i, k)
        return bufs[key]

    def work(i, k):  # pixel-node evaluations of one request
        _, H, W = imgs[i].shape
        return H * W * nodes[k]

    total = n_warm + n_req
    reqs = [(int(rng.integers(0, len(imgs))), int(rng.integers(0, len(fs)))) for _ in range(total)]
    for i, k in set(reqs):  # warm plans and buffers
        vlg.check_all(ctx, fs[k], imgs[i], outs=outs_for(i, k, 0))
    vlg.sync(ctx)
    srv = vlg.Server(slots=slots, budget_bytes=budget)
    t0 = time.perf_counter()
    ids = [srv.submit(fs[k], imgs[i], outs_for(i, k, r)) for r, (i, k) in enumerate(reqs)]
    for rid in ids:
        srv.wait(rid)
    sat = total / (time.perf_counter() - t0)
    log(f"[bench] serve: saturation {sat:.1f} req/s over {total} requests")
    out = {"workload": f"serve: {len(imgs)} resident images (sides {sides}), {len(fs)} formulas "
                       f"({nodes} nodes), {slots} slots, {budget >> 30} GiB pool, "
                       f"{n_req} requests per level after {n_warm} warm-up",
           "saturation_req_per_s": round(sat, 2), "levels": []}
    for frac in fracs:
        rate = frac * sat
        arrive = np.cumsum(rng.exponential(1.0 / rate, total))
        gate = n_warm + int(rng.integers(0, n_req))  # the request checked against the oracle
        gate_outs = fresh(*reqs[gate])
        t_start = time.perf_counter()
        ids, late = [], []
        for r, (i, k) in enumerate(reqs):
            d = t_start + arrive[r] - time.perf_counter()
            if d > 0:
                time.sleep(d)
            late.append(max(0.0, -d) * 1e3)  # submitted after its scheduled arrival
            ids.append(srv.submit(fs[k], imgs[i], gate_outs if r == gate else outs_for(i, k, r)))
        lat = []
        t_first = None
        for r, rid in enumerate(ids):
            q, rr = srv.wait(rid)
            if r == n_warm:
                t_first = t_start + arrive[r]
            lat.append(late[r] + q + rr)
        wall = time.perf_counter() - t_first
        i, k = reqs[gate]
        if check_oracle:
            check_digests(f"serve_f{k}_s{sides[i]}", gate_outs, digests, f"serve request {gate}")
        lat = np.array(lat[n_warm:])
        px = sum(work(i, k) for i, k in reqs[n_warm:])
        lvl = {"offered_req_per_s": round(float(rate), 2), "achieved_req_per_s": round(float(n_req / wall), 2),
               "gpixel_node_per_s": round(float(px / wall / 1e9), 2),
               "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
               "oracle_checked_request": {"formula": k, "side": sides[i], "nodes": nodes[k]} if check_oracle else None}
        log(f"[bench] serve at {frac:.0%}: {lvl}")
        out["levels"].append(lvl)
    st = srv.stats()
    out["max_inflight"] = st["max_inflight"]
    out["peak_reserved_gib"] = round(st["peak_reserved_bytes"] / 2**30, 3)
    srv.close()
    if check_oracle:
        out["cpu_baseline_all_cores"] = serve_cpu_baseline(fsrc, nodes, sides)
        log(f"[bench] serve oracle on the host cores: {out['cpu_baseline_all_cores']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--profile-iters", type=int, default=5)
    ap.add_argument("--skip-oracle", action="store_true", help="no parity gate, no CPU baseline")
    ap.add_argument("--no-chain", action="store_true", help="skip the 10,500-node chain measurement")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-loop measurement")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests per load level (after 200 warm-up)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-image uneven batch measurement")
    ap.add_argument("--batch-images", type=int, default=512)
    ap.add_argument("--no-pixelwise", action="store_true", help="skip the streaming roofline of the pixel-wise kernels")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper's 7680^2 grow specification workload")
    ap.add_argument("--no-pj", action="store_true", help="skip the paper's own labelling algorithm")
    ap.add_argument("--no-volume", action="store_true", help="skip the 256^3 volume workload")
    ap.add_argument("--no-arith", action="store_true", help="skip the arithmetic-atom workload")
    ap.add_argument("--lanes", type=int, default=0,
                    help="labellings run together (1, 2, 4, 8); default: what the autotuner picks")
    ap.add_argument("--hbm-calibration", action="store_true",
                    help="first copy 1 GiB device to device (torch three times, the library copy kernel four times): the scale for hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the formula path has no multi-GPU mode (images or "
              "requests shard across GPUs with no exchange); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2010_07284_amd as vlg
    from paper_2010_07284_amd import _lib
    from synth import formulas, images

    if args.hbm_calibration:
        src_t = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst_t = torch.empty_like(src_t)
        for _ in range(3):
            dst_t.copy_(src_t)
        cctx = vlg.create(0)
        for width in (16, 8):   # one warm-up and one timed dispatch each
            vlg.stream_copy(cctx, dst_t, src_t, width=width, reps=1)
        torch.cuda.synchronize()
        log("[bench] calibration: 3 torch copies and 4 library stream copies (16, 16, 8, 8 B accesses), "
            "1 GiB read + 1 GiB written each")
        del src_t, dst_t, cctx
        torch.cuda.empty_cache()

    S = args.size
    log(f"[bench] generating the {S}x{S} ellipse/maze image and the 100-node formula")
    img = images.ellipse_maze_image(2, S)
    src = formulas.ellipse_dag(2)
    ctx = vlg.create(0)
    lib = _lib.lib()
    im = vlg.load_image(ctx, torch.from_numpy(img).to("cuda:0"))
    f = vlg.compile_formula(ctx, src)
    info = vlg.formula_info(f)
    nodes, nout = info["nodes"], info["outputs"]
    outs = [torch.empty((S, (S + 63) // 64), dtype=torch.int64, device="cuda:0") for _ in range(nout)]
    arr = (ctypes.c_void_p * nout)(*[o.data_ptr() for o in outs])

    cpu = None
    if not args.skip_oracle:
        import oracle
        log("[bench] oracle (CPU, 1 thread) on the full workload: parity gate and CPU baseline")
        t0 = time.perf_counter()
        want = oracle.run(src, img)
        t_cpu = time.perf_counter() - t0
        cpu = {"value": round(S * S * nodes / t_cpu / 1e9, 4), "unit": "Gpixel-node evals/s", "cores": 1,
               "kind": "oracle",
               "sample": f"whole workload once: {S}x{S}, {nodes} nodes, {nout} outputs, {t_cpu:.2f} s, "
                         f"one thread of {cpu_model()}"}
        for mode in ("perop", "fused", "graph"):
            vlg.set_mode(ctx, mode)
            rc = lib.vlg_check_all(ctx.handle, f.handle, im.handle, arr, 0, 1)
            if rc:
                raise RuntimeError(lib.vlg_last_error().decode())
            vlg.sync(ctx)
            for k in range(nout):
                got = vlg.unpack(outs[k], S, S)
                if not np.array_equal(got, want[k]):
                    raise SystemExit(f"[bench] PARITY FAILURE: mode {mode} output {k}: "
                                     f"{int((got != want[k]).sum())} pixels differ")
        log("[bench] parity: all outputs bit-exact in perop, fused and graph modes")

    tune = vlg.autotune(ctx, f, im, iters=3)
    for name, (best, times) in tune.items():
        log(f"[bench] autotune: {name} {best} "
            f"({', '.join(f'{k}: {v:.3f} ms' for k, v in sorted(times.items()))})")
    tile_rows = tune["ccl_tile_rows"][0]
    near_rows = tune["near_band_rows"][0] if "near_band_rows" in tune else None
    ms = {}
    for mode in ("perop", "fused", "graph"):
        ms[mode] = time_mode(vlg, lib, ctx, f, im, arr, mode, args.steps, args.warmup)
        log(f"[bench] {mode}: {ms[mode]:.4f} ms/step")

    if args.lanes:
        vlg.set_tunable(ctx, "ccl_lanes", args.lanes)
    lanes_used = vlg.get_tunable(ctx, "ccl_lanes", S, S)
    # the same step with one labelling at a time, for comparison
    vlg.set_tunable(ctx, "ccl_lanes", 1)
    lanes1_ms = time_mode(vlg, lib, ctx, f, im, arr, "graph", args.steps, args.warmup)
    vlg.set_tunable(ctx, "ccl_lanes", args.lanes)
    log(f"[bench] graph with one labelling at a time: {lanes1_ms:.4f} ms/step "
        f"(headline: {lanes_used} labellings together)")

    prof = vlg.profile(ctx, f, im, iters=args.profile_iters)
    # every kernel kind's launch time without per-launch events: the first
    # step of the kind launched back to back between two HIP events on the
    # context's stream (merge and flag: with their labelling's earlier passes,
    # which are timed alone and subtracted); the dominant kernel is the kind
    # with the largest launches x that time per evaluation, one labelling at
    # a time.  The per-launch event averages of vlg_profile are kept beside.
    per_kind = {}
    for k, (n, t, b) in prof.items():
        try:
            bb_ms, bb_bytes = vlg.profile_step(ctx, f, im, k, reps=50)
        except vlg.VlgError:
            continue
        per_kind[k] = {"launches_per_evaluation": n // args.profile_iters, "avg_launch_us": round(bb_ms * 1e3, 2),
                       "avg_launch_us_with_per_launch_events": round(t / n * 1e3, 2),
                       "bytes_per_launch": round(bb_bytes),
                       "achieved_gbs": round(bb_bytes / (bb_ms / 1e3) / 1e9, 1) if bb_ms > 0 else None}
    dom_name = max(per_kind, key=lambda k: per_kind[k]["launches_per_evaluation"] * per_kind[k]["avg_launch_us"])
    dom_n, dom_ms, dom_bytes = prof[dom_name]
    dom_event_avg_ms = dom_ms / dom_n
    dom_avg_ms = per_kind[dom_name]["avg_launch_us"] / 1e3
    dom_step_bytes = per_kind[dom_name]["bytes_per_launch"]
    dom_gbs = dom_step_bytes / (dom_avg_ms / 1e3) / 1e9
    log(f"[bench] dominant kernel {dom_name}: {dom_avg_ms * 1e3:.2f} us per launch back to back "
        f"({dom_event_avg_ms * 1e3:.2f} us with per-launch events), {dom_step_bytes / 1e6:.2f} MB algorithmic")
    ccl_ms = sum(v[1] for k, v in prof.items() if k.startswith("ccl_")) / args.profile_iters
    n_ccl = info["reach_nodes"]
    for k, (n, t, b) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        log(f"[bench] profile {k:12s} launches/iter {n // args.profile_iters:4d}  "
            f"avg {t / n * 1e3:8.2f} us  {b / (t / 1e3) / 1e9 if t else 0:8.1f} GB/s")

    t = ms["graph"]
    value = S * S * nodes / (t / 1e3) / 1e9
    line = {
        "metric": "Gpixel-node evals/s",
        "value": round(value, 3),
        "unit": "Gpixel-node evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-in/bit-mask",
        "data": "synthetic",
        "config": {"workload": f"ellipse_maze_{S}: {S}x{S} f32 x3 channels, {nodes}-node formula "
                               f"({n_ccl} reach-type), {nout} outputs",
                   "image": [3, S, S], "nodes": nodes, "outputs": nout, "executor": "graph",
                   "ccl_tile_rows": tile_rows, "near_band_rows": near_rows, "ccl_lanes": lanes_used,
                   "labellings": info["labellings"],
                   "launches": info["launches_fused"],
                   "input_sha256": {"image": images.digest(img),
                                    "formula": hashlib.sha256(src.encode()).hexdigest()}},
        "perop_ms": round(ms["perop"], 4),
        "fused_ms": round(ms["fused"], 4),
        "speedup_graph_vs_perop": round(ms["perop"] / t, 3),
        "ccl_lanes": lanes_used,
        "graph_ms_one_labelling_at_a_time": round(lanes1_ms, 4),
        "ccl_gpixel_per_s": round(S * S / (ccl_ms / max(1, n_ccl) / 1e3) / 1e9, 3) if n_ccl else None,
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": round(dom_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(dom_gbs / HBM_PEAK_GBS, 4),
                     "avg_launch_us": round(dom_avg_ms * 1e3, 2),
                     "avg_launch_us_with_per_launch_events": round(dom_event_avg_ms * 1e3, 2),
                     "bytes_per_launch": round(dom_step_bytes),
                     "traffic": measured_traffic(f"ellipse_maze_{S}", dom_name, tile_rows)},
        "kernels_back_to_back": per_kind,
        "cpu_baseline": cpu,
    }
    line["ccl_counters"] = ccl_merge_counts(vlg, lib, src, img)
    if not args.no_chain:
        line["chain"] = bench_chain(vlg, lib, 3, not args.skip_oracle)
    if not args.no_paper:
        line["paper_grow"] = bench_paper_grow(vlg, lib, 10, not args.skip_oracle)
    if not args.no_pj:
        line["paper_labelling"] = bench_pj(vlg, lib, not args.skip_oracle)
    if not args.no_arith:
        line["arith"] = bench_arith(vlg, lib, 10, not args.skip_oracle)
    if not args.no_volume:
        line["volume"] = bench_volume(vlg, lib, 5, not args.skip_oracle)
    if not args.no_pixelwise:
        line["pixelwise"] = bench_pixelwise(vlg, 5)
    if not args.no_batch:
        line["batch"] = bench_batch(vlg, lib, 3, not args.skip_oracle, n=args.batch_images)
        line["batch_square"] = bench_batch(vlg, lib, 3, not args.skip_oracle, n=args.batch_images, square=True)
    if not args.no_serve:
        line["serve"] = bench_serve(vlg, args.serve_requests, not args.skip_oracle)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
