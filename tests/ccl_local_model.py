"""CPU model of the tile-local labelling pass (ccl_local_tile in kernels.hip)
under randomized lane schedules.

TEST INFRASTRUCTURE.  It re-enacts the pass's shared-memory protocol, not its
arithmetic on pixels: the block forest L in LDS, the per-wave queue of union
pairs, the two-walk union with path halving and atomicMin hooking, and the
resolution of run starts with atomicMin path halving.  Every lane is a
generator that yields before each LDS access (load, plain store, atomic), and
a seeded scheduler picks which lane performs its next access, so the model
explores interleavings of the lanes of all waves between the workgroup
barriers (sequentially consistent per access, like one LDS per workgroup).

Two row layouts are modelled:
  "consecutive"  wave v owns block rows RPW*v .. RPW*v+RPW-1 (the shipped
                 kernel): rows after a wave's first list their union pairs
                 before the workgroup barrier (the row above is the wave's
                 own), and the pairs that do not fit the queue are united by
                 their lane at once, touching only the wave's own rows while
                 the other waves may still write theirs; the first row lists
                 its pairs after the barrier;
  "interleaved"  wave v owns rows v, v+NW, ... and lists every pair after
                 the barrier (the earlier layout).
and two resolution variants:
  "own"    each run start is resolved by the lane of its own column (the
           shipped kernel);
  "queue"  the run starts of a wave's rows are listed in the wave's LDS queue
           and spread over all its lanes (the variant that was reverted after
           wrong masks on the GPU).

The result is checked against the definition: every foreground block's root
(the entry its run start holds after resolution) is the smallest block id of
its 8-connected tile-local component.
"""
import numpy as np

# block bits: 1 top-left, 2 top-right, 4 bottom-left, 8 bottom-right


def tile_blocks(mask):
    """(2*TBH, 128) uint8 pixel tile -> (TBH, 64) 4-bit block codes."""
    m = mask.astype(np.uint8)
    return m[0::2, 0::2] | (m[0::2, 1::2] << 1) | (m[1::2, 0::2] << 2) | (m[1::2, 1::2] << 3)


def reference_roots(bits):
    """Smallest block id of each block's 8-connected component (pixel
    adjacency), by flood fill over pixels; -1 for background blocks."""
    TBH, TBW = bits.shape
    px = np.zeros((2 * TBH, 2 * TBW), np.uint8)
    px[0::2, 0::2] = bits & 1
    px[0::2, 1::2] = (bits >> 1) & 1
    px[1::2, 0::2] = (bits >> 2) & 1
    px[1::2, 1::2] = (bits >> 3) & 1
    H, W = px.shape
    comp = -np.ones((H, W), np.int64)
    ncomp = 0
    for y in range(H):
        for x in range(W):
            if px[y, x] and comp[y, x] < 0:
                stack = [(y, x)]
                comp[y, x] = ncomp
                while stack:
                    cy, cx = stack.pop()
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            ny, nx = cy + dy, cx + dx
                            if 0 <= ny < H and 0 <= nx < W and px[ny, nx] and comp[ny, nx] < 0:
                                comp[ny, nx] = ncomp
                                stack.append((ny, nx))
                ncomp += 1
    block_comp = -np.ones((TBH, TBW), np.int64)
    for by in range(TBH):
        for bx in range(TBW):
            c = comp[2 * by:2 * by + 2, 2 * bx:2 * bx + 2].max()
            block_comp[by, bx] = c
    out = -np.ones((TBH, TBW), np.int64)
    first = {}
    for by in range(TBH):
        for bx in range(TBW):
            c = block_comp[by, bx]
            if c >= 0:
                first.setdefault(c, by * TBW + bx)
                out[by, bx] = first[c]
    return out


class Tile:
    """Shared state of one workgroup and the per-lane programs."""

    def __init__(self, bits, nwaves, queue_cap=192, variant="own", layout="consecutive"):
        self.bits = bits
        self.TBH, self.TBW = bits.shape
        self.NW = nwaves
        self.RPW = self.TBH // nwaves
        self.cap = queue_cap
        self.variant = variant
        self.layout = layout
        n = self.TBH * self.TBW
        self.L = list(range(n))
        self.sbr = [0] * n
        self.rows()

    # ---- phase 1 (no shared writes that other lanes read before the barrier)
    def rows(self):
        TBW = self.TBW
        self.run = np.zeros(self.bits.shape, np.int64)
        self.conn = np.zeros(self.bits.shape, bool)
        for lby in range(self.TBH):
            run = -1
            for lane in range(TBW):
                b = int(self.bits[lby, lane])
                left = int(self.bits[lby, lane - 1]) if lane > 0 else 0
                conn = lane > 0 and (b & 5) != 0 and (left & 10) != 0
                if b and not conn:
                    run = lane
                r = run if (b and run >= 0) else lane
                self.run[lby, lane] = r
                self.conn[lby, lane] = conn
                i = lby * TBW + lane
                self.sbr[i] = b | (r << 4)
                self.L[i] = lby * TBW + r if b else i

    def row_of(self, wave, j):
        return self.RPW * wave + j if self.layout == "consecutive" else wave + self.NW * j

    def listing_order(self):
        """(j, before_barrier) in the order a wave lists its rows' pairs."""
        if self.layout == "consecutive":
            return [(j, True) for j in range(1, self.RPW)] + [(0, False)]
        return [(j, False) for j in range(self.RPW)]

    # ---- the wave-collective parts (ballot/mbcnt) are deterministic
    def wave_pairs(self, wave):
        """Union pairs of a wave in queue order, and the overflow pairs of each
        lane in program order (united at once by that lane): those listed
        before the barrier and those listed after it."""
        TBW = self.TBW
        queue = []
        early = {l: [] for l in range(TBW)}
        overflow = {l: [] for l in range(TBW)}
        npairs = 0
        for j, before in self.listing_order():
            lby = self.row_of(wave, j)
            cs_all = []
            for lane in range(TBW):
                b = int(self.bits[lby, lane])
                c0 = c1 = c2 = -1
                if lby > 0 and b:
                    up = (lby - 1) * TBW + lane
                    ul = self.sbr[up - 1] if lane > 0 else 0
                    uc = self.sbr[up]
                    ur = self.sbr[up + 1] if lane < TBW - 1 else 0
                    if (b & 1) and (ul & 8):
                        c0 = ul >> 4
                    if (b & 3) and (uc & 12):
                        c1 = uc >> 4
                    if (b & 2) and (ur & 4):
                        c2 = ur >> 4
                if c1 == c0:
                    c1 = -1
                if c2 == c0 or c2 == c1:
                    c2 = -1
                cs_all.append([c0, c1, c2])
            # the left neighbour's candidates as the lane shift delivers them
            # (before this removal)
            orig = [list(c) for c in cs_all]
            for lane in range(TBW):
                if self.conn[lby, lane]:
                    prev = orig[lane - 1]
                    for k in range(3):
                        if cs_all[lane][k] >= 0 and cs_all[lane][k] in prev:
                            cs_all[lane][k] = -1
            for k in range(3):
                for lane in range(TBW):
                    c = cs_all[lane][k]
                    if c < 0:
                        continue
                    me = lby * TBW + int(self.run[lby, lane])
                    pair = (me, (lby - 1) * TBW + c)
                    if npairs < self.cap:
                        queue.append(pair)
                    else:
                        (early if before else overflow)[lane].append(pair)
                    npairs += 1
        return queue, early, overflow

    # ---- lane programs: yield before each LDS access
    def unite(self, a, b):
        L = self.L
        while a != b:
            yield
            pa = L[a]
            yield
            pb = L[b]
            if pa == a and pb == b:
                hi, lo = max(a, b), min(a, b)
                yield
                old = L[hi]
                L[hi] = min(old, lo)  # atomicMin
                if old == hi:
                    return
                a, b = old, lo
                continue
            ga = gb = None
            if pa != a:
                yield
                ga = L[pa]
            else:
                ga = pa
            if pb != b:
                yield
                gb = L[pb]
            else:
                gb = pb
            if pa != a:
                if ga != pa:
                    yield
                    L[a] = ga  # plain halving store
                a = ga
            if pb != b:
                if gb != pb:
                    yield
                    L[b] = gb
                b = gb

    def root(self, x):
        L = self.L
        while True:
            yield
            p = L[x]
            if p == x:
                return x
            yield
            gp = L[p]
            if gp == p:
                return p
            yield
            L[x] = min(L[x], gp)  # atomicMin halving
            x = gp

    def resolve_store(self, i):
        r = yield from self.root(i)
        yield
        self.L[i] = r  # plain store of the root

    def union_program(self, pairs_direct, pairs_queue):
        for a, b in pairs_direct:
            yield from self.unite(a, b)
        yield "wave"
        for a, b in pairs_queue:
            yield from self.unite(a, b)

    def resolve_program(self, starts_own, starts_queue):
        for i in starts_own:
            yield from self.resolve_store(i)
        if starts_queue is not None:
            yield "wave"
            for i in starts_queue:
                yield from self.resolve_store(i)


def run_phase(progs, waves_of, rng):
    """Run lane generators to completion in a random interleaving; a lane
    that yields "wave" waits until every lane of its wave has reached it."""
    live = {k: g for k, g in enumerate(progs)}
    waiting = set()
    while live:
        runnable = [k for k in live if k not in waiting]
        if not runnable:
            waiting.clear()  # the whole wave (or group) arrived
            continue
        k = runnable[int(rng.integers(0, len(runnable)))]
        try:
            r = next(live[k])
        except StopIteration:
            del live[k]
            continue
        if r == "wave":
            waiting.add(k)
            wv = waves_of[k]
            if all((j in waiting) or (j not in live) for j in live if waves_of[j] == wv):
                for j in list(waiting):
                    if waves_of[j] == wv:
                        waiting.discard(j)


def simulate(bits, nwaves, seed, variant="own", queue_cap=192, layout="consecutive"):
    """Run the pass once under the schedule drawn from `seed`; returns the
    (TBH, 64) array of roots (-1 for background) it produces."""
    rng = np.random.default_rng(seed)
    t = Tile(bits, nwaves, queue_cap=queue_cap, variant=variant, layout=layout)
    TBW = t.TBW
    pairs = [t.wave_pairs(wave) for wave in range(nwaves)]
    # before the barrier: overflow pairs of the rows listed there, every wave
    # at once (each touches only its own rows of L)
    progs, waves_of = [], []
    for wave in range(nwaves):
        queue, early, overflow = pairs[wave]
        for lane in range(TBW):
            if early[lane]:
                progs.append(t.union_program(early[lane], []))
                waves_of.append(wave)
    run_phase(progs, waves_of, rng)
    # union phase after the barrier
    progs, waves_of = [], []
    for wave in range(nwaves):
        queue, early, overflow = pairs[wave]
        for lane in range(TBW):
            progs.append(t.union_program(overflow[lane], queue[lane::64]))
            waves_of.append(wave)
    run_phase(progs, waves_of, rng)
    # resolution phase
    progs, waves_of = [], []
    for wave in range(nwaves):
        starts = []
        for j in range(t.RPW):
            lby = t.row_of(wave, j)
            for lane in range(TBW):
                if t.bits[lby, lane] and t.run[lby, lane] == lane:
                    starts.append((lane, lby * TBW + lane))
        for lane in range(TBW):
            if variant == "own":
                own = [i for l, i in starts if l == lane]
                progs.append(t.resolve_program(own, None))
            else:
                progs.append(t.resolve_program([], [i for _, i in starts][lane::64]))
            waves_of.append(wave)
    run_phase(progs, waves_of, rng)
    out = -np.ones(bits.shape, np.int64)
    for lby in range(t.TBH):
        for lane in range(TBW):
            if bits[lby, lane]:
                out[lby, lane] = t.L[lby * TBW + int(t.run[lby, lane])]
    return out
