"""CPU emulation of a kernel schedule (vlg_formula_plan) on packed masks.

TEST INFRASTRUCTURE.  It executes the steps of a plan the way the kernels
define them, on the packed layout of the C ABI (uint64 words, padding bits
cleared), so that the schedule builder, the slot allocator and the fused
segment programs can be checked against the oracle on the CPU:

  atoms, percentile     float32 comparisons, nearest-rank order statistic
  arith                 the postfix program in numpy float32 (one rounding
                        per operation), then the comparison
  logic                 ((x ^ ix) OP (y ^ iy)) ^ io
  near                  (N(x ^ ix) ^ io) OP (z ^ iz) over the image's pixels
  ccl_local/gather/...  labelling of the passable mask with 8-connectivity
                        (scipy), seed flags per labelling user
  segment               the tile program of the segment kernels: tiles of TR
                        rows x TW words chosen as the launcher chooses them
                        (wide tiles of 62 words, or lane tiles of one word and
                        64 - 2 halo rows), extended by the halo rows and one
                        word on each side, registers per tile, the same
                        operand masking, stores of the tile centre only

Nothing here is shared with the library or the oracle.
"""
import math

import numpy as np
from scipy import ndimage

U64 = np.uint64
ONES = U64(0xFFFFFFFFFFFFFFFF)
SOP_LOAD, SOP_AND, SOP_OR, SOP_NEAR_AND, SOP_NEAR_OR, SOP_STORE = range(6)
NONE = 255


class Geo:
    def __init__(self, H, W):
        self.H, self.W = H, W
        self.wpr = (W + 63) // 64
        self.tail = U64((1 << (W % 64)) - 1) if W % 64 else ONES

    def keep(self):
        k = np.full(self.wpr, ONES, dtype=U64)
        if self.wpr:
            k[-1] = self.tail
        return k


def pack(mask, g):
    padded = np.zeros((g.H, g.wpr * 64), np.uint8)
    padded[:, :g.W] = mask
    return np.packbits(padded, axis=1, bitorder="little").view("<u8").reshape(g.H, g.wpr).astype(U64)


def unpack(words, g):
    if g.H == 0 or g.W == 0:
        return np.zeros((g.H, g.W), np.uint8)
    b = np.unpackbits(words.astype("<u8").view(np.uint8).reshape(g.H, -1), axis=1, bitorder="little")
    return b[:, :g.W].copy()


def hdilate(c, left, right):
    return c | (c << U64(1)) | (c >> U64(1)) | (left >> U64(63)) | (right << U64(63))


def near_words(x, g):
    """N of packed words x (padding bits already clear), rows/words outside
    the image count as background."""
    H, wpr = x.shape
    left = np.zeros_like(x)
    right = np.zeros_like(x)
    left[:, 1:] = x[:, :-1]
    right[:, :-1] = x[:, 1:]
    h = hdilate(x, left, right)
    out = h.copy()
    out[1:] |= h[:-1]
    out[:-1] |= h[1:]
    return out & g.keep()[None, :]


class Emulator:
    def __init__(self, plan, img):
        self.P = plan
        img = np.ascontiguousarray(img)
        if img.ndim == 2:
            img = img[None]
        self.img = img
        C, H, W = img.shape
        self.g = Geo(H, W)
        self.slots = {}
        self.pct = {}
        self.lab = None
        self.flags = {}

    # ---- operands
    def mask(self, slot):
        if slot == -1:
            return np.zeros((self.g.H, self.g.wpr), U64)
        return self.slots[slot]

    def ref(self, r):
        slot, inv = r
        v = self.mask(slot)
        return v ^ ONES if inv else v.copy()

    def put(self, slot, words):
        self.slots[slot] = words & self.g.keep()[None, :]

    # ---- steps
    def percentile(self, st):
        v = np.sort(self.img[st["chan"]].astype(np.float32).ravel())
        n = v.size
        for q, scalar in st["q"]:
            k = math.ceil(q * n) - 1
            k = 0 if (k < 0 or n == 0) else min(k, n - 1)
            self.pct[scalar] = np.float32(v[k]) if n else np.float32(0)

    def atoms(self, st):
        ch = self.img[st["chan"]].astype(np.float32)
        for cmp, use_pct, thr, scalar, out in st["atoms"]:
            t = self.pct[scalar] if use_pct else np.float32(thr)
            m = [ch > t, ch < t, ch >= t, ch <= t][cmp]
            self.put(out, pack(m.astype(np.uint8), self.g))

    def arith(self, st):
        F = np.float32
        prog, k = st["arith"], st["lhs_len"]

        def side(ins):
            stack = []
            for op, idx, c in ins:
                if op == 0:
                    stack.append(np.full((self.g.H, self.g.W), F(c), F))
                elif op == 1:
                    stack.append(self.img[idx].astype(F))
                elif op == 2:
                    stack.append(np.full((self.g.H, self.g.W), self.pct[idx], F))
                elif op == 3:
                    stack.append(-stack.pop())
                elif op == 4:
                    stack.append(np.abs(stack.pop()))
                else:
                    y, x = stack.pop(), stack.pop()
                    with np.errstate(all="ignore"):
                        stack.append([x + y, x - y, x * y, x / y, np.where(y < x, y, x),
                                      np.where(y > x, y, x)][op - 5])
            return stack[0]

        lhs, rhs = side(prog[:k]), side(prog[k:])
        m = [lhs > rhs, lhs < rhs, lhs >= rhs, lhs <= rhs][st["op"]]
        self.put(st["out"], pack(m.astype(np.uint8), self.g))

    def logic(self, st):
        x, y = self.ref(st["x"]), self.ref(st["y"])
        r = (x | y) if st["op"] else (x & y)
        if st["inv_out"]:
            r ^= ONES
        self.put(st["out"], r)

    def near(self, st):
        x = self.ref(st["x"]) & self.g.keep()[None, :]
        n = near_words(x, self.g)
        if st["inv_out"]:
            n ^= ONES
        z = self.ref(st["z"])
        self.put(st["out"], (n | z) if st["op"] else (n & z))

    def label(self, st):
        b = unpack(self.ref(st["x"]) & self.g.keep()[None, :], self.g)
        self.lab, _ = ndimage.label(b, structure=np.ones((3, 3), int))
        self.flags = {}

    def seeds_of(self, words, user):
        s = unpack(words & self.g.keep()[None, :], self.g).astype(bool)
        self.flags[user] = set(np.unique(self.lab[s & (self.lab > 0)]).tolist())

    def ccl_local(self, st):
        self.label(st)
        yz = self.ref(st["y"]) & self.ref(st["z"]) & self.g.keep()[None, :]
        sm = near_words(yz, self.g) & (self.ref(st["x"]))
        self.seeds_of(sm, 0)

    def ccl_reseed(self, st):
        self.seeds_of(self.ref(st["x"]), st["user"])

    def ccl_gather(self, st):
        yz = self.ref(st["y"]) & self.ref(st["z"])
        z = np.isin(self.lab, sorted(self.flags.get(st["user"], set()))) & (self.lab > 0)
        self.put(st["out"], yz | pack(z.astype(np.uint8), self.g))

    def segment(self, st):
        S = self.P["segments"][st["seg"]]
        g = self.g
        halo, nregs = S["halo"], S["nregs"]
        tr, tw = seg_tile(g, halo, nregs)
        RR, RW = tr + 2 * halo, tw + 2
        ptr = [self.mask(s) for s in S["inputs"]]
        outs = {k: np.zeros((g.H, g.wpr), U64) for k in range(len(S["outputs"]))}
        keep = g.keep()
        for ty in range((g.H + tr - 1) // tr):
            for tx in range((g.wpr + tw - 1) // tw):
                r0, w0 = ty * tr - halo, tx * tw - 1
                rows = np.arange(r0, r0 + RR)
                cols = np.arange(w0, w0 + RW)
                rin = (rows >= 0) & (rows < g.H)
                cin = (cols >= 0) & (cols < g.wpr)
                inside = rin[:, None] & cin[None, :]
                ckeep = np.where(cin, keep[np.clip(cols, 0, max(g.wpr - 1, 0))], U64(0)) if g.wpr else None
                regs = [None] * nregs
                for op, dst, a, b, inv in S["ins"]:
                    ia = ONES if inv & 1 else U64(0)
                    ib = ONES if inv & 2 else U64(0)
                    io = ONES if inv & 4 else U64(0)
                    if op == SOP_LOAD:
                        src = ptr[a]
                        v = np.zeros((RR, RW), U64)
                        rr, cc = np.nonzero(inside)
                        v[rr, cc] = src[rows[rr], cols[cc]]
                        regs[dst] = v
                        continue
                    A = regs[a] if a != NONE else np.zeros((RR, RW), U64)
                    B = regs[b] if b != NONE else np.zeros((RR, RW), U64)
                    if op == SOP_STORE:
                        v = (A ^ ia)[halo:halo + tr, 1:1 + tw]
                        orow, ocol = rows[halo:halo + tr], cols[1:1 + tw]
                        ok = (orow < g.H)[:, None] & (ocol < g.wpr)[None, :]
                        rr, cc = np.nonzero(ok)
                        outs[dst][orow[rr], ocol[cc]] = v[rr, cc] & keep[ocol[cc]]
                        continue
                    if op in (SOP_AND, SOP_OR):
                        x, y = A ^ ia, B ^ ib
                        regs[dst] = ((x | y) if op == SOP_OR else (x & y)) ^ io
                        continue
                    # near: operand words outside the image and padding bits are background
                    x = np.where(inside, (A ^ ia) & ckeep[None, :], U64(0))
                    left = np.zeros_like(x)
                    right = np.zeros_like(x)
                    left[:, 1:] = x[:, :-1]
                    right[:, :-1] = x[:, 1:]
                    h = hdilate(x, left, right)
                    n = h.copy()
                    n[1:] |= h[:-1]
                    n[:-1] |= h[1:]
                    n ^= io
                    z = B ^ ib
                    regs[dst] = (n | z) if op == SOP_NEAR_OR else (n & z)
        for k, slot in enumerate(S["outputs"]):
            self.slots[slot] = outs[k]

    def run(self):
        for st in self.P["steps"]:
            k = st["kind"]
            if k in ("ccl_merge", "ccl_flag"):
                continue
            getattr(self, {"percentile": "percentile", "atoms": "atoms", "logic": "logic", "near": "near",
                           "arith": "arith",
                           "ccl_local": "ccl_local", "ccl_gather": "ccl_gather", "ccl_reseed": "ccl_reseed",
                           "segment": "segment"}[k])(st)
        return [unpack(self.slots[-2 - k], self.g) for k in range(self.P["noutputs"])]


def seg_tile(g, halo, nregs, budget=48 * 1024, wide_budget=64 * 1024, min_tiles=1024):
    """The launcher's tile choice for a segment (same rule, restated): wide
    tiles of 62 words in 64-word LDS rows, or, where a narrow shape of 1-16
    words scores best, lane tiles of one word and 64 - 2 halo rows."""
    best, best_score = (4, 1), -1.0

    def consider(tr, tw, useful_w, rw):
        nonlocal best, best_score
        tiles = ((g.H + tr - 1) // tr) * ((g.wpr + tw - 1) // tw)
        eff = tr * useful_w / ((tr + 2 * halo) * rw)
        score = eff * min(1.0, tiles / min_tiles)
        if score > best_score:
            best_score, best = score, (tr, tw)

    for tr in (4, 8, 16, 32, 64):
        if nregs * (tr + 2 * halo) * 64 * 8 <= wide_budget:
            consider(tr, 62, min(62, g.wpr), 64)
    for tw in (1, 2, 4, 8, 16):
        if tw > 1 and tw // 2 >= g.wpr:
            break
        for tr in (4, 8, 16, 32):
            if nregs * (tr + 2 * halo) * (tw + 2) * 8 <= budget:
                consider(tr, tw, tw, tw + 2)
    return best if best[1] == 62 else (64 - 2 * halo, 1)
