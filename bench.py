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
    with open(os.path.join(ROOT, "paper_2010_07284_amd", "csrc", "kernels.hip"), "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest() != rec.get("kernels_source_sha256"):
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
    return {"workload": f"chain_1024: 1024x1024 u8 random mask, {info['nodes']}-node chain "
                        f"({info['reach_nodes']} reach), {nout} outputs",
            "nodes": info["nodes"], "launches_perop": info["steps_perop"], "launches_fused": info["launches_fused"],
            "parity": "oracle digests, every output, every executor" if check_oracle else None,
            "compile_ms": round(compile_ms, 2),
            "graph_build_ms": round(first_ms["graph"] - ms["graph"], 2),
            "perop_ms": round(ms["perop"], 3), "fused_ms": round(ms["fused"], 3), "graph_ms": round(ms["graph"], 3),
            "speedup_graph_vs_perop": round(ms["perop"] / ms["graph"], 3),
            "gpixel_node_per_s": round(1024 * 1024 * info["nodes"] / (ms["graph"] / 1e3) / 1e9, 3)}


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
    ims, host = [], {}
    for i, (h, w) in enumerate(sizes):
        t = images.phantom_image_device(seed, i, h, w, device="cuda:0")
        ims.append(vlg.load_image(ctx, t))
        if i in sample:
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
    px = sum(h * w for h, w in sizes)
    res = {"workload": f"uneven_batch_{n}{'_square' if square else ''}: {n} phantom images, "
                       f"{'square sides' if square else 'sides H, W'} U[128,2048], f32 x4 channels, "
                       f"{nodes}-node segmentation formula, {nout} outputs",
           "images": n, "gpixels": round(px / 1e9, 4), "nodes": nodes,
           "ccl_tile_rows": tune["ccl_tile_rows"][0], "batch_grid": tune["batch_grid"][0],
           "perop_ms": round(ms["perop"], 3), "fused_ms": round(ms["fused"], 3), "graph_ms": round(ms["graph"], 3),
           "speedup_graph_vs_perop": round(ms["perop"] / ms["graph"], 3),
           "gpixel_node_per_s": round(px * nodes / (ms["graph"] / 1e3) / 1e9, 3),
           "images_per_s": round(n / (ms["graph"] / 1e3), 1)}
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
    # reference: a plain device-to-device copy of 4 GiB (what streaming
    # reaches on this device without any kernel of this library)
    a = torch.empty(1 << 30, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(iters):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    gbs = 2 * a.numel() * 4 / (ms / 1e3) / 1e9
    res["device_copy_4GiB"] = {"avg_launch_us": round(ms * 1e3, 1), "achieved_gbs": round(gbs, 1),
                               "frac": round(gbs / HBM_PEAK_GBS, 4)}
    log(f"[bench] pixelwise reference device copy: {gbs:7.1f} GB/s ({gbs / HBM_PEAK_GBS:.1%} of HBM peak)")
    del a, b, im, f, ctx
    torch.cuda.empty_cache()
    return res


def bench_paper_grow(vlg, lib, steps, check_oracle, side=7680):
    """The paper's specification workload (Fig. specification): one 7680x7680
    image in the uint16 range, hI = >.62258, vI = >.56360, grow(hI, vI).  The
    MRI slice is not available: a phantom (ellipses of intensities 0.2-1 with
    Rician-like noise) scaled to 65535 stands in for it.  Reports the
    device-resident evaluation and, as in the paper's protocol, the evaluation
    with the mask copied to host memory."""
    import numpy as np
    import torch
    from synth import formulas, images
    t = images.phantom_image_device(6, 0, side, side, channels=1, device="cuda:0") * 65535.0
    ctx = vlg.create(0)
    im = vlg.load_image(ctx, t)
    src = formulas.GROW_SPEC.format(hi=62258, lo=56360)
    f = vlg.compile_formula(ctx, src)
    host = t.cpu().numpy() if check_oracle else None
    del t
    torch.cuda.empty_cache()
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
        log("[bench] paper grow: bit-exact against the oracle")
    ms_dev = time_mode(vlg, lib, ctx, f, im, arr_d, "graph", steps, 2)
    for _ in range(2):
        lib.vlg_check_all(ctx.handle, f.handle, im.handle, arr_h, 1, 0)
    t0 = time.perf_counter()
    for _ in range(steps):
        lib.vlg_check_all(ctx.handle, f.handle, im.handle, arr_h, 1, 0)
    ms_host = (time.perf_counter() - t0) * 1e3 / steps
    log(f"[bench] paper grow {side}^2: {ms_dev:.3f} ms resident, {ms_host:.3f} ms with the byte mask copied to host")
    return {"workload": f"paper_grow_{side}: {side}x{side} f32 (uint16 range) phantom, grow(>.62258, >.56360)",
            "device_ms": round(ms_dev, 3), "with_host_readback_ms": round(ms_host, 3),
            "mpixel_per_s": round(side * side / (ms_dev / 1e3) / 1e6, 1),
            "paper_context": "about 600 ms on a TITAN Xp and 3 s on an HD Graphics 630 for the same shape, "
                             "start of computation to file saved (OpenCL, uint16 MRI slice)"}


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
    fs = [vlg.compile_formula(ctx, src) for src, _, _ in formulas.serve_formulas(seed)]
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
    ap.add_argument("--lanes", type=int, default=1,
                    help="concurrent labelling lanes: switched off, only 1 is accepted")
    ap.add_argument("--hbm-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy three times (scale for hardware byte counters)")
    args = ap.parse_args()
    if args.lanes != 1:
        print("--lanes: concurrent labelling lanes are switched off (a host-side crash seen with four lanes is "
              "not explained); only 1 is accepted", file=sys.stderr)
        sys.exit(2)
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
        torch.cuda.synchronize()
        log("[bench] calibration: 3 copies of 1 GiB (1 GiB read + 1 GiB written each)")
        del src_t, dst_t
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

    # concurrent labelling lanes (opt-in, experimental): parity, then graph timing
    lanes_ms = None
    if args.lanes > 1:
        vlg.set_tunable(ctx, "ccl_lanes", args.lanes)
        vlg.set_mode(ctx, "graph")
        lib.vlg_check_all(ctx.handle, f.handle, im.handle, arr, 0, 1)
        vlg.sync(ctx)
        if not args.skip_oracle:
            for k in range(nout):
                if not np.array_equal(vlg.unpack(outs[k], S, S), want[k]):
                    raise SystemExit(f"[bench] PARITY FAILURE: {args.lanes} labelling lanes, output {k}")
        lanes_ms = time_mode(vlg, lib, ctx, f, im, arr, "graph", args.steps, args.warmup)
        vlg.set_tunable(ctx, "ccl_lanes", 0)
        log(f"[bench] graph with {args.lanes} labelling lanes: {lanes_ms:.4f} ms/step")

    prof = vlg.profile(ctx, f, im, iters=args.profile_iters)
    dom_name, (dom_n, dom_ms, dom_bytes) = max(prof.items(), key=lambda kv: kv[1][1])
    dom_avg_ms = dom_ms / dom_n
    dom_gbs = dom_bytes / (dom_ms / 1e3) / 1e9
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
                   "ccl_tile_rows": tile_rows, "near_band_rows": near_rows, "labellings": info["labellings"],
                   "launches": info["launches_fused"],
                   "input_sha256": {"image": images.digest(img),
                                    "formula": hashlib.sha256(src.encode()).hexdigest()}},
        "perop_ms": round(ms["perop"], 4),
        "fused_ms": round(ms["fused"], 4),
        "speedup_graph_vs_perop": round(ms["perop"] / t, 3),
        "graph_ms_with_labelling_lanes": ({"lanes": args.lanes, "ms": round(lanes_ms, 4)} if lanes_ms else None),
        "ccl_gpixel_per_s": round(S * S / (ccl_ms / max(1, n_ccl) / 1e3) / 1e9, 3) if n_ccl else None,
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": round(dom_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(dom_gbs / HBM_PEAK_GBS, 4),
                     "avg_launch_us": round(dom_avg_ms * 1e3, 2),
                     "bytes_per_launch": round(dom_bytes / dom_n),
                     "traffic": measured_traffic(f"ellipse_maze_{S}", dom_name, tile_rows)},
        "cpu_baseline": cpu,
    }
    if not args.no_chain:
        line["chain"] = bench_chain(vlg, lib, 3, not args.skip_oracle)
    if not args.no_paper:
        line["paper_grow"] = bench_paper_grow(vlg, lib, 10, not args.skip_oracle)
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
