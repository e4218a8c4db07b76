"""Brute-force evaluations straight from the definitions, for pinning the
oracle on tiny inputs.  Independent of the oracle and of the GPU library:
plain Python loops and numpy, written from the paper's Sect. 2 definitions.

Masks are numpy arrays of 0/1, shape (H, W).  Pixels outside the image do not
exist; adjacency is the Moore (8-)neighbourhood.
"""
import numpy as np


def neighbours(y, x, h, w):
    """8-neighbours of (y, x) inside the image, excluding (y, x)."""
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if (dy or dx) and 0 <= y + dy < h and 0 <= x + dx < w:
                yield y + dy, x + dx


def near(a):
    """N a: pixels that are in a or share an edge or vertex with a pixel of a."""
    h, w = a.shape
    out = np.zeros_like(a, dtype=np.uint8)
    for y in range(h):
        for x in range(w):
            out[y, x] = 1 if a[y, x] or any(a[q] for q in neighbours(y, x, h, w)) else 0
    return out


def reach_paths(a, b):
    """rho a[b] by enumerating simple paths pi from each x: pi_0 = x, some
    pi_l in a (l >= 0), pi_1 .. pi_{l-1} in b.  Exponential; tiny inputs only."""
    h, w = a.shape
    out = np.zeros((h, w), np.uint8)

    def search(p, on_path):
        for q in neighbours(p[0], p[1], h, w):
            if q in on_path:
                continue
            if a[q]:
                return True           # q = pi_l
            if b[q]:                  # q is an intermediate pixel
                on_path.add(q)
                if search(q, on_path):
                    return True
                on_path.discard(q)
        return False

    for y in range(h):
        for x in range(w):
            out[y, x] = 1 if a[y, x] or search((y, x), {(y, x)}) else 0
    return out


def reach_walks(a, b):
    """rho a[b] by unrolling the existential over the path length l with an
    explicit adjacency matrix: T_1 = Adj a, T_l = Adj (b . T_{l-1});
    result = a or T_1 or ... or T_n (walks longer than n add nothing)."""
    h, w = a.shape
    n = h * w
    adj = np.zeros((n, n), np.int64)
    for y in range(h):
        for x in range(w):
            for q in neighbours(y, x, h, w):
                adj[y * w + x, q[0] * w + q[1]] = 1
    av = a.reshape(-1).astype(np.int64)
    bv = b.reshape(-1).astype(np.int64)
    res = av > 0
    t = (adj @ av) > 0
    for _ in range(n + 1):
        res = res | t
        t = (adj @ (bv * t)) > 0
    return res.reshape(h, w).astype(np.uint8)


def surrounded_paths(a, b):
    """a S b from the direct definition: x in a, and every path from x to a
    pixel outside a meets b at some index j in (0, l].  Searches for an
    escaping simple path that avoids b after index 0."""
    h, w = a.shape
    out = np.zeros((h, w), np.uint8)

    def escapes(p, seen):
        for q in neighbours(p[0], p[1], h, w):
            if q in seen or b[q]:
                continue              # meeting b satisfies the condition
            if not a[q]:
                return True           # left a without meeting b
            seen.add(q)
            if escapes(q, seen):
                return True
        return False

    for y in range(h):
        for x in range(w):
            out[y, x] = 1 if a[y, x] and not escapes((y, x), {(y, x)}) else 0
    return out


def components(a):
    """8-connected components as a list of pixel sets (plain DFS)."""
    h, w = a.shape
    seen = np.zeros((h, w), bool)
    comps = []
    for y in range(h):
        for x in range(w):
            if a[y, x] and not seen[y, x]:
                stack, comp = [(y, x)], set()
                seen[y, x] = True
                while stack:
                    p = stack.pop()
                    comp.add(p)
                    for q in neighbours(p[0], p[1], h, w):
                        if a[q] and not seen[q]:
                            seen[q] = True
                            stack.append(q)
                comps.append(comp)
    return comps


def neighbours3(z, y, x, d, h, w):
    """26-neighbours of voxel (z, y, x) inside a d x h x w volume, excluding it."""
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dz or dy or dx) and 0 <= z + dz < d and 0 <= y + dy < h and 0 <= x + dx < w:
                    yield z + dz, y + dy, x + dx


def reach_walks3(a, b):
    """rho a[b] on a volume by the same unrolled walk existential as
    reach_walks, over the 26-neighbour adjacency matrix."""
    d, h, w = a.shape
    n = d * h * w
    adj = np.zeros((n, n), np.int64)
    for z in range(d):
        for y in range(h):
            for x in range(w):
                for q in neighbours3(z, y, x, d, h, w):
                    adj[(z * h + y) * w + x, (q[0] * h + q[1]) * w + q[2]] = 1
    av = a.reshape(-1).astype(np.int64)
    bv = b.reshape(-1).astype(np.int64)
    res = av > 0
    t = (adj @ av) > 0
    for _ in range(n + 1):
        res = res | t
        t = (adj @ (bv * t)) > 0
    return res.reshape(d, h, w).astype(np.uint8)
