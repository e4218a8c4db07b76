"""CPU model of the flatten pass of the volume labelling (k_vb_flatten in
vol.hip; it walks the same way over voxels in its first version and over
2 x 2 x 2 blocks now) under randomized thread schedules.

TEST INFRASTRUCTURE.  After the union pass every voxel's parent chain ends
at its component's root; the flatten pass gives every voxel its root.  Each
thread is a generator that yields before every memory access, and a seeded
scheduler picks which thread performs its next access (sequentially
consistent, one access at a time).  Two protocols:

  "compress"  walk to the root, pointing each walked entry at its
              grandparent on the way (path compression), then write the
              root into the own entry (the first version of the kernel);
  "read"      walk to the root reading only, then write the root into the
              own entry (the shipped kernel).
"""
import numpy as np


def walker(P, v, protocol):
    cur = P[v]
    yield
    if protocol == "compress":
        prev = v
        while True:
            nxt = P[cur]
            yield
            if not cur > nxt:
                break
            P[prev] = nxt
            yield
            prev, cur = cur, nxt
    else:
        while True:
            nxt = P[cur]
            yield
            if not cur > nxt:
                break
            cur = nxt
    P[v] = cur
    yield


def flatten(parent, protocol, seed):
    """Run one walker per non-root entry of `parent` (a forest whose parents
    are smaller than their children) under a random schedule."""
    P = list(parent)
    rng = np.random.default_rng(seed)
    live = [walker(P, v, protocol) for v in range(len(P)) if P[v] != v]
    while live:
        k = int(rng.integers(len(live)))
        try:
            next(live[k])
        except StopIteration:
            live.pop(k)
    return P


def roots(parent):
    out = []
    for v in range(len(parent)):
        r = v
        while parent[r] != r:
            r = parent[r]
        out.append(r)
    return out
