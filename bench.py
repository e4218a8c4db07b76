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
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--profile-iters", type=int, default=5)
    ap.add_argument("--skip-oracle", action="store_true", help="no parity gate, no CPU baseline")
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
               "sample": f"whole workload once: {S}x{S}, {nodes} nodes, {nout} outputs, {t_cpu:.2f} s"}
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
    tile_rows, tile_ms = tune["ccl_tile_rows"]
    log(f"[bench] autotune: labelling tile rows {tile_rows} "
        f"({', '.join(f'{k}: {v:.3f} ms' for k, v in sorted(tile_ms.items()))})")
    ms = {}
    for mode in ("perop", "fused", "graph"):
        ms[mode] = time_mode(vlg, lib, ctx, f, im, arr, mode, args.steps, args.warmup)
        log(f"[bench] {mode}: {ms[mode]:.4f} ms/step")

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
                   "ccl_tile_rows": tile_rows, "labellings": info["labellings"],
                   "launches": info["launches_fused"]},
        "perop_ms": round(ms["perop"], 4),
        "fused_ms": round(ms["fused"], 4),
        "speedup_graph_vs_perop": round(ms["perop"] / t, 3),
        "ccl_gpixel_per_s": round(S * S / (ccl_ms / max(1, n_ccl) / 1e3) / 1e9, 3) if n_ccl else None,
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": round(dom_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(dom_gbs / HBM_PEAK_GBS, 4),
                     "avg_launch_us": round(dom_avg_ms * 1e3, 2),
                     "bytes_per_launch": round(dom_bytes / dom_n), "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
