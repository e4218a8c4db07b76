"""Write the expected-mask digests of the full-size workloads that the oracle
takes minutes to evaluate (tests/golden/digests.json).

TEST INFRASTRUCTURE.  Every expected value here comes from the CPU oracle
(oracle/) on the seeded synthetic inputs of synth/; nothing calls the GPU
library.  A digest is the SHA-256 of a mask in the packed layout of the C ABI
(row-major little-endian uint64 words, ceil(W/64) per row, pixel (y, x) = bit
x % 64 of word x / 64, padding bits 0), computed here with numpy alone.

Workloads:
  chain_1024        the 10,501-node chain (500 reach nodes) of chain_dag(3)
                    on the 1024x1024 uint8 random mask random_mask_image(3)
  serve_f{k}_s{s}   serving-mix formula k of serve_formulas(5) on serving
                    image serve_image(i, s) for every side s of SERVE_SIDES

    python tests/golden/make_digests.py [--jobs 4]
"""
import argparse
import hashlib
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "digests.json")


def packed_digest(mask):
    import numpy as np
    h, w = mask.shape
    wpr = (w + 63) // 64
    padded = np.zeros((h, wpr * 64), np.uint8)
    padded[:, :w] = mask
    return hashlib.sha256(np.packbits(padded, axis=1, bitorder="little").tobytes()).hexdigest()


def cases():
    from synth import formulas
    out = [("chain_1024", "chain_dag(3) on random_mask_image(3, 1024)")]
    for k in range(len(formulas.serve_formulas())):
        for i, s in enumerate(formulas.SERVE_SIDES):
            out.append((f"serve_f{k}_s{s}", f"serve_formulas(5)[{k}] on serve_image({i}, {s})"))
    return out


def inputs(key):
    from synth import formulas, images
    if key == "chain_1024":
        return formulas.chain_dag(3), images.random_mask_image(3, 1024)
    k, s = key[len("serve_f"):].split("_s")
    k, s = int(k), int(s)
    return formulas.serve_formulas()[k][0], images.serve_image(formulas.SERVE_SIDES.index(s), s)


def run_case(key):
    sys.path.insert(0, ROOT)
    import oracle
    src, img = inputs(key)
    t0 = time.time()
    masks = oracle.run(src, img)
    return key, [packed_digest(m) for m in masks], list(img.shape), round(time.time() - t0, 1)


def main():
    sys.path.insert(0, ROOT)
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    args = ap.parse_args()
    todo = cases()
    res = {}
    # largest cases first so the pool stays busy
    order = sorted(todo, key=lambda kv: -int(kv[0].rsplit("_s", 1)[-1]) if kv[0].startswith("serve") else 0)
    with Pool(args.jobs, maxtasksperchild=1) as pool:
        for key, dig, shape, secs in pool.imap_unordered(run_case, [k for k, _ in order]):
            res[key] = {"inputs": dict(todo)[key], "image_shape": shape, "outputs": dig, "oracle_seconds": secs}
            print(f"{key}: {len(dig)} outputs, {secs} s", flush=True)
    with open(OUT, "w") as fh:
        json.dump({"generator": "tests/golden/make_digests.py (oracle only)",
                   "layout": "sha256 of packed64 masks",
                   "cases": dict(sorted(res.items()))}, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
