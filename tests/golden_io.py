"""Reader for the hand-derived fixtures in tests/golden/.

Format: '#' comment lines (citation and derivation), then 'op: NAME', then
blocks 'a:', 'b:', 'img:', 'formula:', 'expect:' of text rows.  In mask rows
'#' is 1 and '.' is 0; 'img:' rows map characters through 'map: C=value ...';
'expect:' rows of an 'ccl' fixture use one letter per component.
"""
import glob
import os

import numpy as np

DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(path):
    fx = {"name": os.path.basename(path), "blocks": {}}
    cur = None
    for raw in open(path):
        line = raw.rstrip("\n")
        if line.startswith("#") and cur is None:
            continue
        if line.startswith("op:"):
            fx["op"] = line.split(":", 1)[1].strip()
        elif line.startswith("map:"):
            fx["map"] = {kv.split("=")[0]: float(kv.split("=")[1]) for kv in line[4:].split()}
        elif line.rstrip().endswith(":") and line.strip()[:-1] in ("a", "b", "img", "formula", "expect"):
            cur = line.strip()[:-1]
            fx["blocks"][cur] = []
        elif cur is not None and line.strip():
            fx["blocks"][cur].append(line if cur == "formula" else line.strip())
    return fx


def mask(rows):
    return np.array([[1 if c == "#" else 0 for c in r] for r in rows], np.uint8)


def image(fx):
    m = fx["map"]
    return np.array([[m[c] for c in r] for r in fx["blocks"]["img"]], np.float32)[None]


def all_fixtures():
    return sorted(glob.glob(os.path.join(DIR, "*.txt")))
