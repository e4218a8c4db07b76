// kernels.hip -- HIP kernels for gfx950 (CDNA4, wave64) on 1-bit-packed masks.
//
// Operators (paper "A spatial model checker in GPU", Sect. 2): threshold
// atoms, pixel-wise Boolean connectives, N (Moore-neighbourhood dilation) and
// reachability rho a[b].  rho follows the decomposition of Sect. 3: label the
// 8-connected components of b, keep the components that meet N a, and dilate
// their union with a.  The labelling is not the paper's iterative
// pointer-jumping scheme (Alg. CCL) but union-find over 2x2 pixel blocks
// (every foreground pixel of a 2x2 block lies in one 8-component), run as a
// tile-local pass in LDS followed by a global merge of tile borders with
// atomicMin hooking, so it needs a fixed number of launches and no host-side
// termination check.
//
// Every operator is written once as a per-unit device function; single-image
// kernels walk one image's units, batch kernels walk the units of many
// images of different sizes through per-image descriptors.
#include "kernels.h"

#include <algorithm>

namespace vlg {
namespace {

constexpr int kThreads = 256;
// channel elements per batched histogram unit: large enough that flushing a
// workgroup's LDS histograms (up to 8192 bins, global atomics that all units
// of an image aim at the same addresses) stays small next to the reads
constexpr int64_t kPctUnit = 262144;

__device__ __forceinline__ uint32_t fdiv(uint32_t n, uint32_t mul, uint32_t shift) {
    return (uint32_t)(((uint64_t)__umulhi(n, mul) + n) >> shift);
}

// Pointers read from descriptors in memory have no known address space and
// would be accessed with flat instructions, which also count against the LDS
// wait counter; every mask, label and image access therefore goes through a
// global-qualified pointer.
#define VLG_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ VLG_GLOBAL T *glb(T *p) {
    return (VLG_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ const VLG_GLOBAL T *glb(const T *p) {
    return (const VLG_GLOBAL T *)p;
}
// Constant address space: for tables that no kernel writes while it runs
// (the per-image descriptors of a batched launch).  A wave-uniform index into
// them becomes a scalar load whose result stays in scalar registers.
#define VLG_CONST __attribute__((address_space(4)))

__device__ __forceinline__ uint64_t ldm(const MRef &r, int64_t i) {
    return (r.p ? glb(r.p)[i] : 0ull) ^ r.inv;
}

__device__ __forceinline__ bool is_last_col(const Geo &g, int64_t i) {
    uint32_t row = fdiv((uint32_t)i, g.wpr_mul, g.wpr_shift);
    return (uint32_t)i - row * (uint32_t)g.wpr == (uint32_t)(g.wpr - 1);
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Workgroups are dispatched to the 8 XCDs in turn (workgroup i to XCD
// i mod 8), and each XCD has an L2 of its own.  The work item of workgroup b
// of n: each XCD takes a contiguous range of items, so that neighbouring
// tiles, which share the cache lines of their mask words, meet in one L2
// instead of each line being fetched by several.  A bijection of [0, n).
__device__ __forceinline__ int xcd_contiguous(int b, int n) {
    constexpr int X = 8;
    const int per = n / X, rem = n % X, x = b % X, k = b / X;
    return x * per + (x < rem ? x : rem) + k;
}

int grid_for(int64_t n, int per_block, int cap) {
    int64_t b = (n + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

// ------------------------------------------------------------------ batches
// image of global unit u: the largest i with prefix[i] <= u
__device__ __forceinline__ int find_img(const int64_t *prefix, int n, int64_t u) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= u) lo = mid;
        else hi = mid;
    }
    return lo;
}

// A workgroup of a persistent batch kernel takes a contiguous range of the
// launch's global units, finds the image of its first unit by binary search
// and then only steps forward (units of one image are consecutive).  Kernels
// copy the image's descriptor into registers per unit: read through a
// reference into memory, its fields would be reloaded after every LDS store
// or atomic (a generic pointer may alias LDS).
struct UnitRange {
    const int64_t *prefix;
    int64_t begin, end, next;
    int ii;
    __device__ UnitRange(const int64_t *p, int n) : prefix(p) {
        const int64_t total = p[n];
        begin = total * blockIdx.x / gridDim.x;
        end = total * (blockIdx.x + 1) / gridDim.x;
        ii = begin < end ? find_img(p, n, begin) : 0;
        next = begin < end ? p[ii + 1] : 0;
    }
    __device__ __forceinline__ int img(int64_t u) {
        while (u >= next) next = prefix[++ii + 1];
        return ii;
    }
};

__device__ __forceinline__ uint64_t *bptr(const BImg &d, int32_t slot) {
    if (slot == -1) return nullptr;
    if (slot <= -2) return glb(d.outs)[-2 - slot];
    return (uint64_t *)(d.ws + (uint64_t)slot * d.mask_bytes);
}

__device__ __forceinline__ MRef bref(const BImg &d, const BRef &r) {
    MRef m;
    m.p = bptr(d, r.slot);
    m.inv = r.inv ? ~0ull : 0ull;
    return m;
}

// ------------------------------------------------------------------ Boolean
// out = ((x ^ x.inv) OP (y ^ y.inv)) ^ inv_out, OP = and (op 0) / or (op 1).
// A null operand is a constant (its inv); the loops below are specialised on
// that once per launch so that every load is unconditional and a thread keeps
// kLogicUnroll words in flight.
constexpr int kLogicUnroll = 4;

// A launch whose operands add up to more than the last-level cache (256 MB
// Infinity Cache) cannot leave them cached for the next launch, so it reads
// them with the non-temporal hint (a connective over 265 MB masks went from
// 59% to over 80% of HBM peak with it); smaller launches read normally, since
// the next step of a schedule usually reads their operands again.
constexpr int64_t kStreamBytes = 256ll << 20;
template <bool NT, typename T>
__device__ __forceinline__ T ld_hint(const VLG_GLOBAL T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool HX, bool HY, bool NT>
__device__ __forceinline__ void logic_span(const Geo &g, const uint64_t *__restrict__ xg, uint64_t xinv,
                                           const uint64_t *__restrict__ yg, uint64_t yinv, int op, uint64_t inv_out,
                                           uint64_t *__restrict__ outg, int64_t i0, int64_t stride, int64_t iend) {
    const VLG_GLOBAL uint64_t *xp = glb(xg), *yp = glb(yg);
    VLG_GLOBAL uint64_t *out = glb(outg);
    for (int64_t i = i0; i < iend; i += kLogicUnroll * stride) {
        uint64_t a[kLogicUnroll], b[kLogicUnroll];
#pragma unroll
        for (int k = 0; k < kLogicUnroll; k++) {
            const int64_t j = min(i + k * stride, iend - 1);
            a[k] = HX ? ld_hint<NT>(&xp[j]) ^ xinv : xinv;
            b[k] = HY ? ld_hint<NT>(&yp[j]) ^ yinv : yinv;
        }
#pragma unroll
        for (int k = 0; k < kLogicUnroll; k++) {
            const int64_t j = i + k * stride;
            uint64_t r = (op ? (a[k] | b[k]) : (a[k] & b[k])) ^ inv_out;
            if (is_last_col(g, j)) r &= g.tail;
            if (j < iend) out[j] = r;
        }
    }
}

// words i0, i0 + stride, ... below iend
template <bool NT = false>
__device__ __forceinline__ void logic_words(const Geo &g, const MRef &x, const MRef &y, int op, uint64_t inv_out,
                                            uint64_t *out, int64_t i0, int64_t stride, int64_t iend) {
    if (x.p && y.p) logic_span<true, true, NT>(g, x.p, x.inv, y.p, y.inv, op, inv_out, out, i0, stride, iend);
    else if (x.p) logic_span<true, false, NT>(g, x.p, x.inv, y.p, y.inv, op, inv_out, out, i0, stride, iend);
    else if (y.p) logic_span<false, true, NT>(g, x.p, x.inv, y.p, y.inv, op, inv_out, out, i0, stride, iend);
    else logic_span<false, false, NT>(g, x.p, x.inv, y.p, y.inv, op, inv_out, out, i0, stride, iend);
}

// ------------------------------------------------------------------ near
// out = (N(x) ^ inv_out) OP z, OP = and (zop 0) / or (zop 1).  N over the
// in-image 3x3 block, as a vertical sliding window: a wave owns 64
// consecutive words of a band of rows and walks down it, loading every row
// word once (the two edge lanes also load the word beyond the wave's edge),
// taking the left and right neighbour words from the adjacent lanes, and
// keeping the horizontally dilated rows y-1, y, y+1 in registers.  Each input
// word is fetched once per band instead of three times (by the workgroups of
// rows y-1, y, y+1, which sit on different XCDs with separate L2s).
// Complemented inputs have their padding bits cleared first so nothing leaks
// in from beyond the right border.
// Loads are issued unconditionally from clamped addresses and masked
// afterwards, so a chunk of CH rows has all its loads in flight at once.
template <int CH, bool HZ>
__device__ __forceinline__ void near_band(const Geo &g, const uint64_t *__restrict__ xg, uint64_t xinv,
                                          uint64_t inv_out, const uint64_t *__restrict__ zg, uint64_t zinv, int zop,
                                          uint64_t *__restrict__ outg, int64_t task, int R) {
    const VLG_GLOBAL uint64_t *xp = glb(xg), *zp = glb(zg);
    VLG_GLOBAL uint64_t *out = glb(outg);
    const int lane = lane_id();
    const int nstrips = (g.wpr + 63) >> 6;
    const int64_t band = task / nstrips;
    const int w = (int)(task - band * nstrips) * 64 + lane;
    const bool valid = w < g.wpr, last = w == g.wpr - 1;
    const int wc = valid ? w : g.wpr - 1;
    const int nb = lane == 0 ? w - 1 : (lane == 63 ? w + 1 : -1);  // word beyond the wave's edge
    const bool nbv = nb >= 0 && nb < g.wpr;
    const int nbc = nbv ? nb : wc;
    const uint64_t keep = last ? g.tail : ~0ull;
    const int y0 = (int)band * R, y1 = min(y0 + R, g.H);
    // raw loads of row y (clamped into the image) and their masking; the empty
    // asm consumes every raw value of a chunk after all its loads are issued,
    // which keeps the compiler from sinking a load into a conditional block
    // (with a wait right behind it)
    auto addr = [&](int y) { return (int64_t)min(max(y, 0), g.H - 1) * g.wpr; };
    auto mask_c = [&](int y, int lim, uint64_t raw) {
        return (y >= 0 && y <= lim && valid) ? ((raw ^ xinv) & keep) : 0ull;
    };
    auto mask_e = [&](int y, int lim, uint64_t raw) { return (y >= 0 && y <= lim && nbv) ? (raw ^ xinv) : 0ull; };
    // horizontal dilation of one row: lanes beyond the row hold c = 0
    auto hrow = [&](uint64_t c, uint64_t e) {
        uint64_t l = __shfl_up(c, 1), r = __shfl_down(c, 1);
        if (lane == 0) l = e;
        if (lane == 63) r = e;
        return c | (c << 1) | (c >> 1) | (l >> 63) | (r << 63);
    };
    uint64_t hm, h0;
    {
        uint64_t rc0 = xp[addr(y0 - 1) + wc], re0 = xp[addr(y0 - 1) + nbc];
        uint64_t rc1 = xp[addr(y0) + wc], re1 = xp[addr(y0) + nbc];
        asm volatile("" : "+v"(rc0), "+v"(re0), "+v"(rc1), "+v"(re1));
        hm = hrow(mask_c(y0 - 1, g.H - 1, rc0), mask_e(y0 - 1, g.H - 1, re0));
        h0 = hrow(mask_c(y0, g.H - 1, rc1), mask_e(y0, g.H - 1, re1));
    }
    const int lim = min(y1, g.H - 1);
    for (int yb = y0; yb < y1; yb += CH) {
        uint64_t c[CH], e[CH], zz[CH];
#pragma unroll
        for (int k = 0; k < CH; k++) {
            const int64_t a = addr(yb + 1 + k);
            c[k] = xp[a + wc];
            e[k] = xp[a + nbc];
            zz[k] = HZ ? zp[addr(yb + k) + wc] : 0ull;
        }
#pragma unroll
        for (int k = 0; k < CH; k++) {
            if (HZ) asm volatile("" : "+v"(c[k]), "+v"(e[k]), "+v"(zz[k]));
            else asm volatile("" : "+v"(c[k]), "+v"(e[k]));
        }
#pragma unroll
        for (int k = 0; k < CH; k++) {
            const uint64_t hp = hrow(mask_c(yb + 1 + k, lim, c[k]), mask_e(yb + 1 + k, lim, e[k]));
            const uint64_t n = (hm | h0 | hp) ^ inv_out;
            const uint64_t zv = HZ ? (zz[k] ^ zinv) : zinv;
            const uint64_t res = (zop ? (n | zv) : (n & zv)) & keep;
            if (valid && yb + k < y1) out[(int64_t)(yb + k) * g.wpr + w] = res;
            hm = h0;
            h0 = hp;
        }
    }
}

// N of a constant mask (x.p == nullptr) is that constant over the image.
__device__ __forceinline__ void near_const_band(Geo g, uint64_t xinv, uint64_t inv_out, MRef z, int zop, uint64_t *out,
                                             int64_t task, int R) {
    const int nstrips = (g.wpr + 63) >> 6;
    const int64_t band = task / nstrips;
    const int w = (int)(task - band * nstrips) * 64 + lane_id();
    if (w >= g.wpr) return;
    const uint64_t keep = w == g.wpr - 1 ? g.tail : ~0ull;
    const int y0 = (int)band * R, y1 = min(y0 + R, g.H);
    for (int y = y0; y < y1; y++) {
        const int64_t i = (int64_t)y * g.wpr + w;
        const uint64_t n = xinv ^ inv_out, zz = ldm(z, i);
        out[i] = (zop ? (n | zz) : (n & zz)) & keep;
    }
}

// band `task` of height R (4, 8, 16 or 32 rows)
__device__ __forceinline__ void near_task(const Geo &g, const MRef &x, uint64_t inv_out, const MRef &z, int zop,
                                          uint64_t *out, int64_t task, int R) {
    if (!x.p) near_const_band(g, x.inv, inv_out, z, zop, out, task, R);
    else if (R == 4 && z.p) near_band<4, true>(g, x.p, x.inv, inv_out, z.p, z.inv, zop, out, task, R);
    else if (R == 4) near_band<4, false>(g, x.p, x.inv, inv_out, z.p, z.inv, zop, out, task, R);
    else if (z.p) near_band<8, true>(g, x.p, x.inv, inv_out, z.p, z.inv, zop, out, task, R);
    else near_band<8, false>(g, x.p, x.inv, inv_out, z.p, z.inv, zop, out, task, R);
}

// ------------------------------------------------------------------ atoms
// The image is stored with a row pitch of wpr*64 elements, so mask word i
// covers elements [64 i, 64 i + 64) of a channel.  A wave takes 64
// consecutive words: lane l loads element 64 k + l for k = 0..63 (coalesced,
// all loads issued before any compare), then for each atom the wave-wide
// compare of pixel row k is the packed word k and is written into lane k's
// register (v_writelane).  One coalesced 512-byte store per atom.  The
// channel is read once for up to kMaxAtomsPerLaunch atoms.
// Four pixel rows per asm block: four compares write four SGPR pairs
// (s[84:91], reserved by the clobber list), then eight v_writelane move them
// into lanes k..k+3.  Each SGPR is read at least three VALU instructions
// after it was written and VCC is not involved, so the block needs no
// wait states of its own.
#define VLG_ATOM4(OP)                                                                               \
    asm(OP " s[84:85], %[a], %[t]\n\t" OP " s[86:87], %[b], %[t]\n\t" OP " s[88:89], %[c], %[t]\n\t" OP \
           " s[90:91], %[d], %[t]\n\t"                                                                 \
           "v_writelane_b32 %[lo], s84, %[k0]\n\tv_writelane_b32 %[hi], s85, %[k0]\n\t"                \
           "v_writelane_b32 %[lo], s86, %[k1]\n\tv_writelane_b32 %[hi], s87, %[k1]\n\t"                \
           "v_writelane_b32 %[lo], s88, %[k2]\n\tv_writelane_b32 %[hi], s89, %[k2]\n\t"                \
           "v_writelane_b32 %[lo], s90, %[k3]\n\tv_writelane_b32 %[hi], s91, %[k3]"                    \
        : [lo] "+v"(lo), [hi] "+v"(hi)                                                                \
        : [a] "v"(v[k]), [b] "v"(v[k + 1]), [c] "v"(v[k + 2]), [d] "v"(v[k + 3]), [t] "v"(t),       \
          [k0] "i"(k), [k1] "i"(k + 1), [k2] "i"(k + 2), [k3] "i"(k + 3)                             \
        : "s84", "s85", "s86", "s87", "s88", "s89", "s90", "s91")

template <int CMP>
__device__ __forceinline__ uint64_t atom_words(const float (&v)[64], float t) {
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int k = 0; k < 64; k += 4) {
        if (CMP == 0) VLG_ATOM4("v_cmp_gt_f32_e64");
        else if (CMP == 1) VLG_ATOM4("v_cmp_lt_f32_e64");
        else if (CMP == 2) VLG_ATOM4("v_cmp_ge_f32_e64");
        else VLG_ATOM4("v_cmp_le_f32_e64");
    }
    return (uint64_t)lo | ((uint64_t)hi << 32);
}
#undef VLG_ATOM4

// One wave task: words [64 t, 64 t + 64) of image channel img, for atoms
// 0..n-1 with thresholds sthr (LDS) and comparisons cmp; outf(j) is atom j's
// output mask.
template <typename T, bool NT = false, typename OutF>
__device__ __forceinline__ void atoms_task(const Geo &g, const T *__restrict__ img, int n, const uint8_t *cmp,
                                           const float *sthr, OutF outf, int64_t t) {
    const int lane = lane_id();
    const int64_t w0 = t * 64;
    const int nw = (int)((g.nwords - w0) < 64 ? (g.nwords - w0) : 64);
    const VLG_GLOBAL T *src = glb(img) + w0 * 64 + lane;
    float v[64];
    if (nw == 64) {
#pragma unroll
        for (int k = 0; k < 64; k++) v[k] = (float)ld_hint<NT>(&src[k * 64]);
    } else {
#pragma unroll
        for (int k = 0; k < 64; k++) v[k] = k < nw ? (float)ld_hint<NT>(&src[k * 64]) : 0.f;
    }
    const int64_t wi = w0 + lane;
    const uint64_t keep = (lane < nw && is_last_col(g, wi)) ? g.tail : ~0ull;
    for (int j = 0; j < n; j++) {
        const float th = sthr[j];
        uint64_t w;
        switch (cmp[j]) {
        case 0: w = atom_words<0>(v, th); break;
        case 1: w = atom_words<1>(v, th); break;
        case 2: w = atom_words<2>(v, th); break;
        default: w = atom_words<3>(v, th); break;
        }
        if (lane < nw) glb(outf(j))[wi] = w & keep;
    }
}

// ------------------------------------------------------------------ CCL
// Blocks: block (by, bx) holds pixels rows 2by..2by+1, cols 2bx..2bx+1.  Its
// four bits: 1 = top-left, 2 = top-right, 4 = bottom-left, 8 = bottom-right.
// Any two foreground pixels of one block are 8-adjacent, so a block is a
// union-find node.  Block ids are row-major, id = by*BW + bx.  Inside a tile
// the root of a set is its smallest id; across tiles roots are linked by a
// pseudo-random priority of their ids (see g_unite).  Canonical pixel labels
// therefore take a minimum over each component.
//
// 8-adjacency between a block and its earlier neighbours:
//   left:       (tl|bl) of the block and (tr|br) of the left block
//   up:         (tl|tr) and (bl|br) of the upper block
//   up-left:    tl and br of the upper-left block
//   up-right:   tr and bl of the upper-right block

__device__ __forceinline__ int lds_ld(int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Value of v in the previous lane of the wave (DPP wave shift right by one;
// lane 0 receives 0).
__device__ __forceinline__ int lane_prev(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false);
}
// Value of v in the next lane of the wave (DPP wave shift left by one; lane
// 63 receives 0).
__device__ __forceinline__ int lane_next(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false);
}

// Union of a and b on the LDS forest L (L[x] <= x, a root is the smallest
// entry of its set).  Both walks advance together, one path-halving step per
// round, so their LDS latencies overlap; once both reach roots the larger
// root is hooked under the smaller with atomicMin, and if that root was
// hooked meanwhile the returned parent is united in its place.  Halving
// stores may race with other lanes' hooks; the hooking lane then unites the
// old parent as well, so no connection is lost.  At most `cap` rounds:
// returns false when the cap stops the walk (the union may be missing).
__device__ __forceinline__ bool lds_unite(int *L, int a, int b, int cap) {
    for (int it = 0; a != b; it++) {
        if (it >= cap) return false;
        const int pa = lds_ld(&L[a]), pb = lds_ld(&L[b]);
        if (pa == a && pb == b) {
            const int hi = a > b ? a : b, lo = a > b ? b : a;
            const int old = atomicMin(&L[hi], lo);
            if (old == hi) return true;
            a = old;
            b = lo;
            continue;
        }
        const int ga = pa != a ? lds_ld(&L[pa]) : pa, gb = pb != b ? lds_ld(&L[pb]) : pb;
        if (pa != a) {
            if (ga != pa) L[a] = ga;
            a = ga;
        }
        if (pb != b) {
            if (gb != pb) L[b] = gb;
            b = gb;
        }
    }
    return true;
}

// Root of x once all unions are done.  Path halving here goes through
// atomicMin: the root is the smallest entry of its set, so a stale halving
// store can never replace a root that its owner has already written.  At
// most `cap` rounds; when the cap stops the walk, ok is cleared and the
// ancestor reached so far (a block of the same tile) is returned.
__device__ __forceinline__ int lds_root(int *L, int x, int cap, bool &ok) {
    for (int it = 0; it < cap; it++) {
        const int p = lds_ld(&L[x]);
        if (p == x) return x;
        const int gp = lds_ld(&L[p]);
        if (gp == p) return p;
        __hip_atomic_fetch_min(&L[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        x = gp;
    }
    ok = false;
    return x;
}

// Raise the give-up flag of a launch (one vector atomic per wave).
// Called by every lane of the wave.
__device__ __forceinline__ void guard_report(const LoopGuard &gd, bool ok) {
    const uint64_t bad = __ballot(!ok);
    if (bad && lane_id() == __builtin_ctzll(bad) && gd.status)
        __hip_atomic_fetch_or(glb(gd.status), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Cross-lane handoff through LDS inside one wave: every lane's LDS writes
// before this point are complete (and visible to the other lanes) before any
// lane's LDS reads after it.  The workgroup-scope fences order the accesses
// for the compiler and wait for the outstanding LDS operations; the wave
// barrier keeps the lanes together.
__device__ __forceinline__ void wave_lds_handoff() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Global union-find for the cross-tile merge.  A root is hooked under the
// root of smaller priority uf_prio(id), a bijective mix of the id, so the
// priority strictly falls along every parent path.  Linking by id instead
// turns a row of tiles whose components join left to right (a corridor
// crossing the image) into a chain as long as the row, because every tile
// hooks under its left neighbour at the same time; pseudo-random priorities
// keep the expected depth logarithmic.  Plain loads and stores may see stale
// values (the L2 of one XCD is not coherent with another's within a kernel);
// that costs retries, never correctness: every value ever stored in L[x] is
// an ancestor of x, sets only grow, and a hook is a compare-and-swap that
// succeeds only on a current root and otherwise hands back the current
// parent, which is then united in turn.
//
// g_find2: the roots of a and b, walked in lockstep (path halving on both) so
// that the loads of the two paths overlap.  `budget` counts the rounds left
// to the caller's walk; returns false when it runs out.
__device__ __forceinline__ bool g_find2(VLG_GLOBAL int *L, int &a, int &b, int &budget) {
    while (true) {
        if (--budget < 0) return false;
        const int pa = L[a], pb = L[b];
        if (pa == a && pb == b) return true;
        const int ga = L[pa], gb = L[pb];
        if (pa != a) {
            if (ga == pa) {
                a = pa;
            } else {
                L[a] = ga;  // path halving
                a = ga;
            }
        }
        if (pb != b) {
            if (gb == pb) {
                b = pb;
            } else {
                L[b] = gb;
                b = gb;
            }
        }
    }
}

__device__ __forceinline__ uint32_t uf_prio(int x) {
    uint32_t h = (uint32_t)x * 0x9E3779B1u;  // odd multiplier: a bijection
    return h ^ (h >> 16);                     // invertible xor-shift
}

// Unite a and b; returns the number of hook attempts, and clears ok when the
// walk used up `cap` rounds (finds and hooks together) before it finished.
__device__ int g_unite(VLG_GLOBAL int *L, int a, int b, int cap, bool &ok) {
    int tries = 0, budget = cap;
    while (true) {
        tries++;
        if (!g_find2(L, a, b, budget)) {
            ok = false;
            return tries;
        }
        if (a == b) return tries;
        if (uf_prio(a) < uf_prio(b)) {
            const int t = a;
            a = b;
            b = t;
        }
        int old = a;  // hook a (larger priority) under b if a is still a root
        __hip_atomic_compare_exchange_strong(&L[a], &old, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        if (old == a) return tries;
        a = old;
    }
}

__device__ __forceinline__ uint32_t block_bits_g(const Geo &g, const MRef &b, int by, int bx) {
    const int w = bx >> 5, sh = (bx & 31) * 2, y0 = 2 * by;
    const uint64_t keep = w == g.wpr - 1 ? g.tail : ~0ull;
    const uint64_t t = ldm(b, (int64_t)y0 * g.wpr + w) & keep;
    const uint64_t u = y0 + 1 < g.H ? (ldm(b, (int64_t)(y0 + 1) * g.wpr + w) & keep) : 0ull;
    return (uint32_t)((t >> sh) & 3) | ((uint32_t)((u >> sh) & 3) << 2);
}

// Threads per workgroup of the tile-local pass: four block rows per wave at
// most (TBH = 32 takes eight waves), which bounds the per-row state each
// lane keeps in registers.
template <int TBH>
constexpr int ccl_local_threads() {
    return TBH > 16 ? 512 : 256;
}

// Tile-local labelling of b: TBH block rows x 64 block columns (2*TBH x 128
// pixels) per workgroup of NWAVES waves.  Wave v owns the RPW consecutive
// block rows RPW*v .. RPW*v+RPW-1, one lane per block column, and keeps each
// row's block state in a register from the first phase to the last.  Horizontally
// connected blocks form runs, found with a ballot and labelled by their first
// block without any atomics.  Runs of consecutive rows are then united once
// per touching pair (a block skips the upper runs its connected left
// neighbour already touches).  Also computes the seed test: a block meets the
// seeds when one of its b-pixels lies in N(y & z).
//
// Output: glab[id] = global id of the foreground block's tile-local root
// (background entries are left as they are); gflag[id] of a local root:
// bit0 = its component touches the tile border (only those can be joined to
// other tiles), bit1 = it meets the seeds (seed set of labelling user 0;
// bits 2..7 serve later users, see ccl_reseed).
template <int TBH>
__device__ void ccl_local_tile(const Geo &g, const MRef &b, const MRef &y, const MRef &z, int tx, int ty,
                               int32_t *__restrict__ glab_, uint8_t *__restrict__ gflag_, const LoopGuard &gd) {
    VLG_GLOBAL int32_t *glab = glb(glab_);
    VLG_GLOBAL uint8_t *gflag = glb(gflag_);
    constexpr int NT = ccl_local_threads<TBH>();
    constexpr int TWW = 2, TR = 2 * TBH, TBW = 64, NB = TBH * TBW, NWAVES = NT / 64;
    constexpr int RPW = TBH / NWAVES;
    static_assert(RPW * NWAVES == TBH, "tile rows must split evenly over the waves");
    constexpr int NSB = TR * TWW, NSA = (TR + 2) * (TWW + 2), NLD = NSB + NSA;
    constexpr int LIT = (NLD + NT - 1) / NT;
    __shared__ uint64_t sb[TR][TWW];
    __shared__ uint64_t sa[TR + 2][TWW + 2];
    __shared__ int L[NB];
    __shared__ uint16_t sbr[NB];              // block bits | run start column << 4
    __shared__ alignas(4) uint8_t sflag[NB];  // bit0 touches the tile border, bit1 seed
    __shared__ int sany;
    constexpr int kPairQueue = 192;              // union pairs per wave: me | other << 16
    __shared__ int spair[NWAVES][kPairQueue];
    // the thread index is made opaque per tile so that a persistent
    // workgroup recomputes its per-row addressing in each tile instead of
    // holding it in registers across the whole tile loop
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wave = tid >> 6;
    const int r0 = ty * TR, wc0 = tx * TWW;

    // b words of the tile and (y & z) words of the tile plus a one-pixel halo,
    // all loads in flight at once; sany: bit0 = some b pixel, bit1 = some seed
    if (tid == 0) sany = 0;
    __syncthreads();
    int any;
    {
        uint64_t v[LIT];
#pragma unroll
        for (int k = 0; k < LIT; k++) {
            const int i = tid + k * NT;
            v[k] = 0;
            if (i < NSB) {
                const int yy = r0 + i / TWW, ww = wc0 + i % TWW;
                if (yy < g.H && ww < g.wpr) v[k] = ldm(b, (int64_t)yy * g.wpr + ww) & (ww == g.wpr - 1 ? g.tail : ~0ull);
            } else if (i < NLD) {
                const int j = i - NSB, yy = r0 + j / (TWW + 2) - 1, ww = wc0 + j % (TWW + 2) - 1;
                if (yy >= 0 && yy < g.H && ww >= 0 && ww < g.wpr) {
                    const int64_t idx = (int64_t)yy * g.wpr + ww;
                    v[k] = ldm(y, idx) & ldm(z, idx) & (ww == g.wpr - 1 ? g.tail : ~0ull);
                }
            }
        }
        bool has_b = false, has_s = false;
#pragma unroll
        for (int k = 0; k < LIT; k++) {
            const int i = tid + k * NT;
            if (i < NSB) {
                sb[i / TWW][i % TWW] = v[k];
                has_b |= v[k] != 0;
            } else if (i < NLD) {
                const int j = i - NSB;
                sa[j / (TWW + 2)][j % (TWW + 2)] = v[k];
                has_s |= v[k] != 0;
            }
        }
        const int f = (__ballot(has_b) ? 1 : 0) | (__ballot(has_s) ? 2 : 0);
        if (lane == 0 && f) atomicOr(&sany, f);
        __syncthreads();
        any = sany;
    }
    // a tile without passable pixels only clears its flag bytes (the flag pass
    // reads every block's; no pass reads a background block's parent entry)
    if (!(any & 1)) {
        for (int i = tid; i < NB; i += NT) {
            const int by = ty * TBH + i / TBW, bx = tx * TBW + i % TBW;
            if (by < g.BH && bx < g.BW) gflag[(int64_t)by * g.BW + bx] = 0;
        }
        __syncthreads();  // sany is reset by the next tile of a persistent workgroup
        return;
    }

    // rows: block bits, runs, seeds.  st[j] (row RPW*wave + j) = bits | run << 4 |
    // seed << 10 | (connected to the left block) << 11
    const int w = lane >> 5, sh = (lane & 31) * 2;
    uint32_t st[RPW];
#pragma unroll
    for (int j = 0; j < RPW; j++) {
        const int lby = RPW * wave + j, i = lby * TBW + lane;
        const uint32_t bits = (uint32_t)((sb[2 * lby][w] >> sh) & 3) | ((uint32_t)((sb[2 * lby + 1][w] >> sh) & 3) << 2);
        uint32_t seed = 0;
        if (any & 2) {
            // seed pixels in the 4x4 window around the block: rows 2lby-1 ..
            // 2lby+2, cols 2lbx-1 .. 2lbx+2 (halo coordinates: +1 row, +64 cols)
            const int c = 64 * (w + 1) + sh - 1, q = c >> 6, s = c & 63;
            uint32_t win[4];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const uint64_t lo = sa[2 * lby + k][q] >> s;
                const uint64_t hi = s > 60 ? (sa[2 * lby + k][q + 1] << (64 - s)) : 0ull;
                win[k] = (uint32_t)((lo | hi) & 0xF);
            }
            const uint32_t top = win[0] | win[1] | win[2], bot = win[1] | win[2] | win[3];
            const uint32_t nmask = ((top & 0x7) ? 1u : 0u) | ((top & 0xE) ? 2u : 0u) |
                                   ((bot & 0x7) ? 4u : 0u) | ((bot & 0xE) ? 8u : 0u);
            seed = (bits & nmask) ? 1u : 0u;
        }
        const uint32_t left = (uint32_t)lane_prev((int)bits);
        const bool conn = lane > 0 && (bits & 5) && (left & 10);
        const uint64_t starts = __ballot(bits != 0 && !conn);
        const uint64_t upto = starts & (~0ull >> (63 - lane));
        const int run = upto ? 63 - __builtin_clzll(upto) : lane;
        st[j] = bits | ((uint32_t)run << 4) | (seed << 10) | (conn ? 1u << 11 : 0u);
        if (j == RPW - 1) sbr[i] = (uint16_t)(bits | ((uint32_t)run << 4));  // read by the next wave's row 0
        sflag[i] = (uint8_t)(seed << 1);
        L[i] = bits ? lby * TBW + run : i;
    }
    auto st_bits = [](uint32_t s) { return s & 15u; };
    auto st_run = [](uint32_t s) { return (int)((s >> 4) & 63u); };

    // unite the runs of each row with the runs they touch in the row above.
    // The wave first lists the pairs of all its rows (at most three per lane
    // and row) in its LDS queue, then every lane takes pairs from the queue:
    // a row's unions are usually held by a few lanes (the run starts), and
    // taking them row by row in those lanes would chain the rows' union walks
    // one after another.  Pairs beyond the queue's capacity are united by
    // their own lane at once (after the barrier, when every entry of L is
    // set).  The row above a wave's row j >= 1 is its row j-1, in registers
    // (its neighbours' entries through DPP lane shifts), so those rows list
    // their pairs before the barrier; only row 0 reads the row above, the
    // previous wave's last row, from LDS after it.
    int npairs = 0;  // wave-uniform
    bool ok = true;  // no walk of this lane hit the loop cap
    auto list_pairs = [&](int j, uint32_t ul, uint32_t uc, uint32_t ur) {
        const int lby = RPW * wave + j;
        const uint32_t bits = st_bits(st[j]);
        int c0 = -1, c1 = -1, c2 = -1;
        if (lby > 0 && bits) {
            if ((bits & 1) && (ul & 8)) c0 = (int)(ul >> 4);
            if ((bits & 3) && (uc & 12)) c1 = (int)(uc >> 4);
            if ((bits & 2) && (ur & 4)) c2 = (int)(ur >> 4);
        }
        if (c1 == c0) c1 = -1;
        if (c2 == c0 || c2 == c1) c2 = -1;
        const int l0 = lane_prev(c0), l1 = lane_prev(c1), l2 = lane_prev(c2);
        if (st[j] & (1u << 11)) {
            // the left block is in this run and already joins its upper runs
            if (c0 >= 0 && (c0 == l0 || c0 == l1 || c0 == l2)) c0 = -1;
            if (c1 >= 0 && (c1 == l0 || c1 == l1 || c1 == l2)) c1 = -1;
            if (c2 >= 0 && (c2 == l0 || c2 == l1 || c2 == l2)) c2 = -1;
        }
        const int me = lby * TBW + st_run(st[j]), ub = (lby - 1) * TBW;
        const int cs[3] = {c0, c1, c2};
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const uint64_t has = __ballot(cs[k] >= 0);
            if (cs[k] >= 0) {
                const int q = npairs + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(has >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)has, 0u));
                if (q < kPairQueue)
                    spair[wave][q] = me | ((ub + cs[k]) << 16);
                else
                    ok &= lds_unite(L, me, ub + cs[k], gd.cap);
            }
            npairs += __popcll(has);
        }
    };
    // (rows j >= 1 unite only blocks of this wave's rows, whose entries of L
    // this wave has written: a wave-level handoff makes them visible)
    wave_lds_handoff();
#pragma unroll
    for (int j = 1; j < RPW; j++) {
        // block state of the row above: bits | run << 4, for lanes l-1, l, l+1
        const uint32_t uc = st[j - 1] & 0x3FFu;
        list_pairs(j, (uint32_t)lane_prev((int)uc), uc, (uint32_t)lane_next((int)uc));
    }
    __syncthreads();
    {
        const int up = (RPW * wave - 1) * TBW + lane;  // the previous wave's last row
        const bool have = wave > 0;
        const uint32_t ul = have && lane > 0 ? sbr[up - 1] : 0u, uc = have ? sbr[up] : 0u,
                       ur = have && lane < 63 ? sbr[up + 1] : 0u;
        list_pairs(0, ul, uc, ur);
    }
    wave_lds_handoff();  // the queue entries of every lane, then the reads
    for (int q = lane; q < (npairs < kPairQueue ? npairs : kPairQueue); q += 64) {
        const int pr = spair[wave][q];
        ok &= lds_unite(L, pr & 0xFFFF, pr >> 16, gd.cap);
    }
    __syncthreads();

    // resolve each run start; the other blocks of a run reach their root
    // through their run start
#pragma unroll
    for (int j = 0; j < RPW; j++) {
        const int i = (RPW * wave + j) * TBW + lane;
        if (st_bits(st[j]) && st_run(st[j]) == lane) L[i] = lds_root(L, i, gd.cap, ok);
    }
    __syncthreads();

    // every block's root (through its run start); carry seed and
    // border-contact flags to the local roots (32-bit LDS atomics on the flag
    // bytes)
    int root[RPW];
#pragma unroll
    for (int j = 0; j < RPW; j++) root[j] = L[(RPW * wave + j) * TBW + st_run(st[j])];
#pragma unroll
    for (int j = 0; j < RPW; j++) {
        const int lby = RPW * wave + j;
        const uint32_t f = ((st[j] >> 9) & 2u) | ((lby == 0 || lby == TBH - 1 || lane == 0 || lane == TBW - 1) ? 1u : 0u);
        if (st_bits(st[j]) && f) {
            const int r = root[j];
            atomicOr((unsigned int *)(sflag + (r & ~3)), f << (8 * (r & 3)));
        }
    }
    __syncthreads();

#pragma unroll
    for (int j = 0; j < RPW; j++) {
        const int lby = RPW * wave + j, i = lby * TBW + lane;
        const int by = ty * TBH + lby, bx = tx * TBW + lane;
        if (by >= g.BH || bx >= g.BW) continue;
        const int64_t id = (int64_t)by * g.BW + bx;
        // background blocks point at themselves: no later pass reads their
        // parent entry (every lookup starts from a foreground block), but a
        // wave that writes every entry of its row writes whole cache lines;
        // leaving the background entries out made the memory side fetch the
        // lines it had to merge (counters: 34 MB read per launch at 4096^2,
        // against 6 MB of mask reads)
        if (st_bits(st[j])) {
            const int r = root[j];
            glab[id] = (ty * TBH + r / TBW) * g.BW + tx * TBW + r % TBW;
            gflag[id] = r == i ? sflag[i] : (uint8_t)0;
        } else {
            glab[id] = (int32_t)id;
            gflag[id] = 0;
        }
    }
    guard_report(gd, ok);
    __syncthreads();  // the next tile of a persistent workgroup reuses the LDS
}

// Cross-tile merge, two waves per tile (part 0 the top row, part 1 the side
// columns, so that the two chains of dependent global accesses run side by
// side): blocks on the tile's top row, left column and right column unite
// with their earlier neighbours in other tiles.
// A block skips a union that its connected predecessor along the same border
// (left neighbour on the top row, upper neighbour on a side column) already
// makes with the same tile-local component.
//
// The wave first stages the mask words around the tile's border in LDS: pixel
// rows 2*by0-4 .. 2*by0+2*TBH-1 and word columns 2*tx-1 .. 2*tx+2 (every block
// any border block or its neighbours and predecessors touch), all loads in
// flight at once.  Each lane then derives the block bits it needs from LDS and
// loads the labels of its candidates and predecessors together before uniting.
template <int TBH>
constexpr int merge_window_words() {
    return (2 * TBH + 4) * 4;
}

template <int TBH>
__device__ void ccl_merge_tile(const Geo &g, const MRef &b, int ntx, int tile, int part, int32_t *glab_,
                               uint64_t *win, int &unions, int &tries, const LoopGuard &gd) {
    constexpr int TBW = 64, WN = merge_window_words<TBH>(), NL = (WN + 63) / 64;
    VLG_GLOBAL int32_t *glab = glb(glab_);
    const int lane = lane_id();
    const int tx = tile % ntx, ty = tile / ntx;
    const int by0 = ty * TBH, bx0 = tx * TBW;
    const int r0 = 2 * by0 - 4, w0 = 2 * tx - 1;  // window origin: pixel row, word column
    {
        uint64_t v[NL];
        int64_t idx[NL];
#pragma unroll
        for (int k = 0; k < NL; k++) {
            const int i = lane + 64 * k, r = r0 + i / 4, w = w0 + (i & 3);
            const bool ok = i < WN && r >= 0 && r < g.H && w >= 0 && w < g.wpr;
            idx[k] = ok ? (int64_t)r * g.wpr + w : -1;
            v[k] = b.p ? glb(b.p)[ok ? idx[k] : 0] : 0ull;
        }
#pragma unroll
        for (int k = 0; k < NL; k++) {
            const int i = lane + 64 * k, w = w0 + (i & 3);
            if (i < WN) win[i] = idx[k] >= 0 ? ((v[k] ^ b.inv) & (w == g.wpr - 1 ? g.tail : ~0ull)) : 0ull;
        }
        wave_lds_handoff();  // every lane's window words, then the reads
    }
    // bits of block (by, bx), by in [by0-2, by0+TBH), bx in [bx0-2, bx0+64]
    auto bits = [&](int by, int bx) -> uint32_t {
        const int r = 2 * by - r0, p = 2 * bx - 64 * w0, q = p >> 6, sh = p & 63;
        return (uint32_t)((win[r * 4 + q] >> sh) & 3) | ((uint32_t)((win[(r + 1) * 4 + q] >> sh) & 3) << 2);
    };
    bool ok = true;  // no walk of this lane hit the loop cap
    auto link = [&](int id, int nid) {
        unions++;
        tries += g_unite(glab, id, nid, gd.cap, ok);
    };

    // top row: contacts with the row above (other tile): UL, U, UR
    if (part == 0 && by0 > 0 && by0 < g.BH) {
        const int by = by0, bx = bx0 + lane, id = by * g.BW + bx;
        const uint32_t bb = bx < g.BW ? bits(by, bx) : 0u;
        int c[3] = {-1, -1, -1}, p[3] = {-1, -1, -1};
        if (bb) {
            if (bx > 0 && (bb & 1) && (bits(by - 1, bx - 1) & 8)) c[0] = id - g.BW - 1;
            if ((bb & 3) && (bits(by - 1, bx) & 12)) c[1] = id - g.BW;
            if (bx + 1 < g.BW && (bb & 2) && (bits(by - 1, bx + 1) & 4)) c[2] = id - g.BW + 1;
            // predecessor on this border row: the left block, if connected
            if (lane > 0) {
                const uint32_t lb = bits(by, bx - 1);
                if ((bb & 5) && (lb & 10)) {
                    if (bx - 1 > 0 && (lb & 1) && (bits(by - 1, bx - 2) & 8)) p[0] = id - g.BW - 2;
                    if ((lb & 3) && (bits(by - 1, bx - 1) & 12)) p[1] = id - g.BW - 1;
                    if ((lb & 2) && (bits(by - 1, bx) & 4)) p[2] = id - g.BW;
                }
            }
        }
        int pl[3], lc[3];
#pragma unroll
        for (int j = 0; j < 3; j++) {
            pl[j] = p[j] >= 0 ? glab[p[j]] : -2;
            lc[j] = c[j] >= 0 ? glab[c[j]] : -4;
        }
        const int my = bb ? glab[id] : -1;  // loaded with the others: the unions start from the labels
        int done[2] = {-3, -3};
#pragma unroll
        for (int j = 0; j < 3; j++) {
            if (c[j] < 0) continue;
            if (lc[j] == pl[0] || lc[j] == pl[1] || lc[j] == pl[2] || lc[j] == done[0] || lc[j] == done[1]) continue;
            done[j < 2 ? j : 1] = lc[j];
            link(my, lc[j]);
        }
    }
    // side columns: lanes 0..TBH-1 the left column, lanes 32..32+TBH-1 the right
    const int lby = lane & 31, side = lane >> 5;
    const int by = by0 + lby;
    if (part == 1 && lby < TBH && by < g.BH) {
        if (side == 0 && bx0 > 0 && bx0 < g.BW) {
            // contacts in the column to the left (other tile): L, and UL below the top row
            const int bx = bx0, id = by * g.BW + bx;
            const uint32_t bb = bits(by, bx);
            int c[2] = {-1, -1}, p[2] = {-1, -1};
            if (bb) {
                if ((bb & 5) && (bits(by, bx - 1) & 10)) c[0] = id - 1;
                if (lby > 0 && (bb & 1) && (bits(by - 1, bx - 1) & 8)) c[1] = id - g.BW - 1;
                // predecessor on this border column: the upper block, if connected
                if (lby > 0) {
                    const uint32_t ub = bits(by - 1, bx);
                    if ((bb & 3) && (ub & 12)) {
                        if ((ub & 5) && (bits(by - 1, bx - 1) & 10)) p[0] = id - g.BW - 1;
                        if (lby > 1 && (ub & 1) && (bits(by - 2, bx - 1) & 8)) p[1] = id - 2 * g.BW - 1;
                    }
                }
            }
            const int pl0 = p[0] >= 0 ? glab[p[0]] : -2, pl1 = p[1] >= 0 ? glab[p[1]] : -2;
            const int lc0 = c[0] >= 0 ? glab[c[0]] : -4, lc1 = c[1] >= 0 ? glab[c[1]] : -4;
            const int my = bb ? glab[id] : -1;
            int first = -3;
            if (c[0] >= 0 && lc0 != pl0 && lc0 != pl1) {
                first = lc0;
                link(my, lc0);
            }
            if (c[1] >= 0 && lc1 != pl0 && lc1 != pl1 && lc1 != first) link(my, lc1);
        } else if (side == 1 && lby > 0 && bx0 + TBW < g.BW) {
            // contact UR (tile to the right); redundant when the upper block is
            // connected to this block and to that same block (its right neighbour)
            const int bx = bx0 + TBW - 1, id = by * g.BW + bx;
            const uint32_t bb = bits(by, bx);
            if ((bb & 2) && (bits(by - 1, bx + 1) & 4)) {
                const uint32_t ub = bits(by - 1, bx), ur = bits(by - 1, bx + 1);
                const bool covered = (bb & 3) && (ub & 12) && (ur & 5) && (ub & 10);
                if (!covered) link(id, id - g.BW + 1);
            }
        }
    }
    guard_report(gd, ok);
    wave_lds_handoff();  // the window is rewritten by the wave's next tile
}

// Point a border-touching tile-local root i (flag byte f) at its final root
// and carry its seed flag there.  Other local roots are final roots already.
// A walker writes only its own entry, so concurrent walkers never undo each
// other.  At most `cap` steps; a walk the cap stops writes nothing and clears
// ok.
__device__ __forceinline__ void ccl_flag_walk(VLG_GLOBAL int32_t *glab, VLG_GLOBAL uint8_t *gflag, int i, uint32_t f,
                                              int cap, bool &ok) {
    int x = i;
    for (int it = 0;; it++) {
        if (it >= cap) {
            ok = false;
            return;
        }
        const int p = glab[x];
        if (p == x) break;
        x = p;
    }
    if (x != i) {
        glab[i] = x;
        if (f & 2) gflag[x] = 3;  // final roots are border-touching local roots
    }
}

// Flag pass over blocks i0 .. i0+15 (i0 a multiple of 16): one 16-byte load
// of their flag bytes, then a walk for each border-touching local root among
// them (bit0 of its byte).  A byte that another walker rewrites after the
// load is either a final root (the walk ends at once) or unchanged.
template <int N>
__device__ __forceinline__ void ccl_flag_n(int32_t *glab_, uint8_t *gflag_, int64_t nb, int64_t i0, int cap,
                                           bool &ok) {
    static_assert(N == 4 || N == 16, "4 or 16 blocks per thread");
    VLG_GLOBAL int32_t *glab = glb(glab_);
    VLG_GLOBAL uint8_t *gflag = glb(gflag_);
    uint64_t lo = 0, hi = 0;
    if (N == 16 && i0 + 16 <= nb && ((uintptr_t)(gflag_ + i0) & 7) == 0) {
        const VLG_GLOBAL uint64_t *q = (const VLG_GLOBAL uint64_t *)(gflag + i0);
        lo = q[0];
        hi = q[1];
    } else if (N == 4 && i0 + 4 <= nb && ((uintptr_t)(gflag_ + i0) & 3) == 0) {
        lo = *(const VLG_GLOBAL uint32_t *)(gflag + i0);
    } else {
        for (int k = 0; k < N && i0 + k < nb; k++) {
            const uint64_t v = gflag[i0 + k];
            if (k < 8)
                lo |= v << (8 * k);
            else
                hi |= v << (8 * (k - 8));
        }
    }
    constexpr uint64_t kBit0 = 0x0101010101010101ull;
    uint64_t mlo = lo & kBit0, mhi = hi & kBit0;
    while (mlo | mhi) {
        int bit, k;
        uint32_t f;
        if (mlo) {
            bit = __builtin_ctzll(mlo);
            mlo &= mlo - 1;
            k = bit >> 3;
            f = (uint32_t)(lo >> bit) & 0xFF;
        } else {
            bit = __builtin_ctzll(mhi);
            mhi &= mhi - 1;
            k = 8 + (bit >> 3);
            f = (uint32_t)(hi >> bit) & 0xFF;
        }
        ccl_flag_walk(glab, gflag, (int)(i0 + k), f, cap, ok);
    }
}

// out = (y & z) | Z, Z = the b-pixels whose component meets the seeds.  Every
// foreground block points at a local root and every local root at its final
// root, so the root is two loads away; the flag byte of the local root is
// loaded beside its parent entry and is the final one when the local root is
// a final root.  A task is 256 blocks of one block row (512 pixels = 8 words
// of two rows); lane l owns blocks 4l .. 4l+3, i.e. byte l of those 8 words,
// assembled in LDS (zw: 8 words per task).  A wave takes NT consecutive tasks
// t0 .. t0+NT-1 (those below ntasks) and walks them together, so their
// dependent loads overlap.  Lanes 0..15 load the output words' operands up
// front.
template <int NT>
__device__ __forceinline__ void ccl_gather_tasks(const Geo &g, const MRef &b, const MRef &y, const MRef &z,
                                                 const int32_t *__restrict__ glab_, const uint8_t *__restrict__ gflag_,
                                                 int user, uint64_t *__restrict__ out_, int64_t t0, int64_t ntasks,
                                                 uint64_t *zw) {
    const VLG_GLOBAL int32_t *glab = glb(glab_);
    const VLG_GLOBAL uint8_t *gflag = glb(gflag_);
    VLG_GLOBAL uint64_t *out = glb(out_);
    const int lane = lane_id();
    const int nq = (g.wpr + 7) / 8;
    bool ovalid[NT];
    int64_t oi[NT];
    uint64_t oyz[NT], ob[NT];
    uint32_t any[NT];
    int by[NT], q[NT];
#pragma unroll
    for (int k = 0; k < NT; k++) {
        const int64_t t = t0 + k;
        const bool valid = t < ntasks;
        by[k] = valid ? (int)(t / nq) : 0;
        q[k] = valid ? (int)(t - (int64_t)by[k] * nq) : 0;
        const int y0 = 2 * by[k];
        // output word of lanes 0..15: row y0 + lane/8, word 8q + lane%8
        const int oy = y0 + (lane >> 3), ow = 8 * q[k] + (lane & 7);
        ovalid[k] = valid && lane < 16 && oy < g.H && ow < g.wpr;
        oi[k] = ovalid[k] ? (int64_t)oy * g.wpr + ow : 0;
        oyz[k] = 0;
        ob[k] = 0;
        if (ovalid[k]) {
            oyz[k] = ldm(y, oi[k]) & ldm(z, oi[k]);
            ob[k] = ldm(b, oi[k]);
        }
        const int w = 8 * q[k] + (lane >> 3), sh = (lane & 7) * 8;  // word and bit offset of my byte
        uint32_t top = 0, bot = 0;
        if (valid && w < g.wpr) {
            const uint64_t keep = w == g.wpr - 1 ? g.tail : ~0ull;
            top = (uint32_t)(((ldm(b, (int64_t)y0 * g.wpr + w) & keep) >> sh) & 0xFF);
            if (y0 + 1 < g.H) bot = (uint32_t)(((ldm(b, (int64_t)(y0 + 1) * g.wpr + w) & keep) >> sh) & 0xFF);
        }
        any[k] = top | bot;
    }
    int lr[NT][4];
#pragma unroll
    for (int k = 0; k < NT; k++) {
        const int64_t id0 = (int64_t)by[k] * g.BW + 256 * q[k] + 4 * lane;
#pragma unroll
        for (int j = 0; j < 4; j++) lr[k][j] = ((any[k] >> (2 * j)) & 3) ? glab[id0 + j] : -1;
    }
    int r[NT][4];
    uint32_t f[NT][4];
#pragma unroll
    for (int k = 0; k < NT; k++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
            r[k][j] = lr[k][j] >= 0 ? glab[lr[k][j]] : -1;
            f[k][j] = lr[k][j] >= 0 ? gflag[lr[k][j]] : 0u;
        }
#pragma unroll
    for (int k = 0; k < NT; k++)
#pragma unroll
        for (int j = 0; j < 4; j++)
            if (r[k][j] >= 0 && r[k][j] != lr[k][j]) f[k][j] = gflag[r[k][j]];
#pragma unroll
    for (int k = 0; k < NT; k++) {
        uint32_t zbyte = 0;
#pragma unroll
        for (int j = 0; j < 4; j++)
            if (r[k][j] >= 0 && ((f[k][j] >> (1 + user)) & 1)) zbyte |= 3u << (2 * j);
        ((uint8_t *)zw)[64 * k + lane] = (uint8_t)zbyte;
    }
    wave_lds_handoff();  // every lane's Z byte, then the word reads
#pragma unroll
    for (int k = 0; k < NT; k++)
        if (ovalid[k]) {
            const int ow = 8 * q[k] + (lane & 7);
            const uint64_t keep = ow == g.wpr - 1 ? g.tail : ~0ull;
            out[oi[k]] = (oyz[k] | (ob[k] & zw[8 * k + (lane & 7)])) & keep;
        }
    wave_lds_handoff();  // zw is rewritten by the wave's next tasks
}

constexpr int kGatherTasksPerWave = 2;

// Mark, for labelling user `user`, the components of the current labelling
// that meet the seed mask sm (= N(seeds) & b): bit 1+user of the root's flag
// byte.  Runs after the flag pass, so every block's root is two loads away.
// Called by every lane of a wave (block (by, bx), or valid = false).
__device__ __forceinline__ void ccl_reseed_lane(const Geo &g, const MRef &sm, const int32_t *__restrict__ glab_,
                                                uint8_t *gflag_, int user, bool valid, int by, int bx) {
    const VLG_GLOBAL int32_t *glab = glb(glab_);
    VLG_GLOBAL uint8_t *gflag = glb(gflag_);
    const int lane = lane_id();
    int r = -1;
    if (valid && block_bits_g(g, sm, by, bx)) r = glab[glab[(int64_t)by * g.BW + bx]];
    // neighbouring blocks mostly share a root: one atomic per distinct root
    // per wave (a giant component would otherwise serialise on one address)
    const uint32_t bit = 1u << (1 + user);
    uint64_t pending = __ballot(r >= 0);
    while (pending) {
        const int leader = __builtin_ctzll(pending);  // wave-uniform
        const int r0 = __builtin_amdgcn_readlane(r, leader);
        pending &= ~__ballot(r == r0);
        if (lane == leader && !(gflag[r0] & bit))
            __hip_atomic_fetch_or((VLG_GLOBAL unsigned int *)(gflag + (r0 & ~3)), bit << (8 * (r0 & 3)),
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ------------------------------------------------------------------ single-image kernels

template <bool NT>
__global__ __launch_bounds__(kThreads) void k_logic(Geo g, MRef x, MRef y, int op, uint64_t inv_out,
                                                    uint64_t *__restrict__ out) {
    logic_words<NT>(g, x, y, op, inv_out, out, (int64_t)blockIdx.x * kThreads + threadIdx.x,
                (int64_t)gridDim.x * kThreads, g.nwords);
}

__global__ __launch_bounds__(kThreads) void k_near(Geo g, MRef x, uint64_t inv_out, MRef z, int zop,
                                                   uint64_t *__restrict__ out, int R) {
    const int64_t ntasks = near_tasks(g, R), nwaves = (int64_t)gridDim.x * (kThreads / 64);
    for (int64_t t = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); t < ntasks; t += nwaves)
        near_task(g, x, inv_out, z, zop, out, t, R);
}

// Up to kBatchMax independent Boolean steps (or near steps) in one launch:
// blockIdx.y selects the step.
template <bool NT>
__global__ __launch_bounds__(kThreads) void k_logic_batch(Geo g, LogicBatch bt) {
    const LogicOp &o = bt.ops[blockIdx.y];
    logic_words<NT>(g, o.x, o.y, o.op, o.inv_out, o.out, (int64_t)blockIdx.x * kThreads + threadIdx.x,
                (int64_t)gridDim.x * kThreads, g.nwords);
}

__global__ __launch_bounds__(kThreads) void k_near_batch(Geo g, NearBatch bt, int R) {
    const NearOp &o = bt.ops[blockIdx.y];
    const int64_t ntasks = near_tasks(g, R), nwaves = (int64_t)gridDim.x * (kThreads / 64);
    for (int64_t t = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); t < ntasks; t += nwaves)
        near_task(g, o.x, o.inv_out, o.z, o.zop, o.out, t, R);
}

template <typename T, bool NT>
__global__ __launch_bounds__(kThreads) void k_atoms(Geo g, const T *__restrict__ img, AtomLaunch a) {
    __shared__ float sthr[kMaxAtomsPerLaunch];
    if ((int)threadIdx.x < a.n)
        sthr[threadIdx.x] = a.thr_dev[threadIdx.x] ? *a.thr_dev[threadIdx.x] : a.thr[threadIdx.x];
    __syncthreads();
    const int64_t nwaves = (int64_t)gridDim.x * (kThreads / 64);
    const int64_t ntasks = (g.nwords + 63) / 64;
    auto outf = [&](int j) { return a.out[j]; };
    for (int64_t t = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); t < ntasks; t += nwaves)
        atoms_task<T, NT>(g, img, a.n, a.cmp, sthr, outf, t);
}

template <int TBH>
__global__ __launch_bounds__(ccl_local_threads<TBH>()) void k_ccl_local(Geo g, MRef b, MRef y, MRef z, int ntx,
                                                        int32_t *__restrict__ glab,
                                                        uint8_t *__restrict__ gflag, LoopGuard gd) {
    const int tile = xcd_contiguous((int)blockIdx.x, (int)gridDim.x);
    ccl_local_tile<TBH>(g, b, y, z, tile % ntx, tile / ntx, glab, gflag, gd);
}

template <int TBH>
__global__ __launch_bounds__(kThreads) void k_ccl_merge(Geo g, MRef b, int ntx, int ntiles, int32_t *glab,
                                                        unsigned long long *counters, LoopGuard gd) {
    __shared__ uint64_t win[kThreads / 64][merge_window_words<TBH>()];
    const int wv = threadIdx.x >> 6;
    const int w = xcd_contiguous((int)blockIdx.x, (int)gridDim.x) * (kThreads / 64) + wv, tile = w >> 1;
    int unions = 0, tries = 0;
    if (tile < ntiles) ccl_merge_tile<TBH>(g, b, ntx, tile, w & 1, glab, win[wv], unions, tries, gd);
    if (counters && (unions | tries)) {
        atomicAdd(&counters[0], (unsigned long long)unions);
        atomicAdd(&counters[1], (unsigned long long)(tries - unions));
    }
}

// per: blocks per thread, 4 on small images (more threads walk at once) or 16
__global__ __launch_bounds__(kThreads) void k_ccl_flag(int64_t nblocks, int32_t *glab, uint8_t *gflag, LoopGuard gd,
                                                       int per) {
    const int64_t stride = (int64_t)gridDim.x * kThreads * per;
    bool ok = true;
    for (int64_t i0 = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * per; i0 < nblocks; i0 += stride) {
        if (per == 4)
            ccl_flag_n<4>(glab, gflag, nblocks, i0, gd.cap, ok);
        else
            ccl_flag_n<16>(glab, gflag, nblocks, i0, gd.cap, ok);
    }
    guard_report(gd, ok);
}

__global__ __launch_bounds__(kThreads) void k_ccl_gather(Geo g, MRef b, MRef y, MRef z,
                                                         const int32_t *__restrict__ glab,
                                                         const uint8_t *__restrict__ gflag, int user,
                                                         uint64_t *__restrict__ out) {
    constexpr int NT = kGatherTasksPerWave;
    __shared__ uint64_t zw[kThreads / 64][8 * NT];
    const int wv = threadIdx.x >> 6;
    const int64_t ntasks = (int64_t)g.BH * ((g.wpr + 7) / 8);
    const int64_t nwaves = (int64_t)gridDim.x * (kThreads / 64);
    for (int64_t t = ((int64_t)blockIdx.x * (kThreads / 64) + wv) * NT; t < ntasks; t += nwaves * NT)
        ccl_gather_tasks<NT>(g, b, y, z, glab, gflag, user, out, t, ntasks, zw[wv]);
}

__global__ __launch_bounds__(kThreads) void k_ccl_reseed(Geo g, MRef sm, const int32_t *__restrict__ glab,
                                                         uint8_t *gflag, int user) {
    const int bx = blockIdx.x * kThreads + threadIdx.x, by = blockIdx.y;
    ccl_reseed_lane(g, sm, glab, gflag, user, bx < g.BW, by, bx);
}

// ---- several labellings per launch (blockIdx.y selects the labelling)
template <int TBH>
__global__ __launch_bounds__(ccl_local_threads<TBH>()) void k_ccl_local_multi(Geo g, CclMulti m, int ntx,
                                                                              LoopGuard gd) {
    const int l = (int)blockIdx.y, tile = xcd_contiguous((int)blockIdx.x, (int)gridDim.x);
    ccl_local_tile<TBH>(g, m.b[l], m.y[l], m.z[l], tile % ntx, tile / ntx, m.glab[l], m.gflag[l], gd);
}

template <int TBH>
__global__ __launch_bounds__(kThreads) void k_ccl_merge_multi(Geo g, CclMulti m, int ntx, int ntiles,
                                                              unsigned long long *counters, LoopGuard gd) {
    __shared__ uint64_t win[kThreads / 64][merge_window_words<TBH>()];
    const int l = (int)blockIdx.y;
    const int wv = threadIdx.x >> 6;
    const int w = xcd_contiguous((int)blockIdx.x, (int)gridDim.x) * (kThreads / 64) + wv, tile = w >> 1;
    int unions = 0, tries = 0;
    if (tile < ntiles) ccl_merge_tile<TBH>(g, m.b[l], ntx, tile, w & 1, m.glab[l], win[wv], unions, tries, gd);
    if (counters && (unions | tries)) {
        atomicAdd(&counters[0], (unsigned long long)unions);
        atomicAdd(&counters[1], (unsigned long long)(tries - unions));
    }
}

__global__ __launch_bounds__(kThreads) void k_ccl_flag_multi(int64_t nblocks, CclMulti m, LoopGuard gd) {
    const int l = (int)blockIdx.y;
    const int64_t stride = (int64_t)gridDim.x * kThreads * 16;
    bool ok = true;
    for (int64_t i0 = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * 16; i0 < nblocks; i0 += stride)
        ccl_flag_n<16>(m.glab[l], m.gflag[l], nblocks, i0, gd.cap, ok);
    guard_report(gd, ok);
}

__global__ __launch_bounds__(kThreads) void k_ccl_gather_multi(Geo g, CclMulti m) {
    constexpr int NT = kGatherTasksPerWave;
    __shared__ uint64_t zw[kThreads / 64][8 * NT];
    const int l = (int)blockIdx.y;
    const int wv = threadIdx.x >> 6;
    const int64_t ntasks = (int64_t)g.BH * ((g.wpr + 7) / 8);
    const int64_t nwaves = (int64_t)gridDim.x * (kThreads / 64);
    for (int64_t t = ((int64_t)blockIdx.x * (kThreads / 64) + wv) * NT; t < ntasks; t += nwaves * NT)
        ccl_gather_tasks<NT>(g, m.b[l], m.y[l], m.z[l], m.glab[l], m.gflag[l], m.user[l], m.out[l], t, ntasks,
                             zw[wv]);
}

// Smallest row-major pixel index of each component, gathered at its root.
__global__ __launch_bounds__(kThreads) void k_ccl_canon(Geo g, MRef b, const int32_t *__restrict__ glab,
                                                        int32_t *canon) {
    const int bx = blockIdx.x * kThreads + threadIdx.x, by = blockIdx.y, lane = lane_id();
    int r = -1, p = 0x7fffffff;
    if (bx < g.BW) {
        const uint32_t bits = block_bits_g(g, b, by, bx);
        if (bits) {
            const int k = __builtin_ctz(bits);  // top-left, top-right, bottom-left, bottom-right
            p = (2 * by + (k >> 1)) * g.W + 2 * bx + (k & 1);
            r = glab[glab[(int64_t)by * g.BW + bx]];
        }
    }
    // one atomicMin per distinct root per wave, with the group's minimum
    uint64_t pending = __ballot(r >= 0);
    while (pending) {
        const int leader = __builtin_ctzll(pending);  // wave-uniform
        const int r0 = __builtin_amdgcn_readlane(r, leader);
        const bool mine = r == r0;
        pending &= ~__ballot(mine);
        int m = mine ? p : 0x7fffffff;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = min(m, __shfl_xor(m, off));
        // a giant component would serialise every wave on one address: skip
        // the atomic when the root already holds a smaller index
        if (lane == leader && m < __hip_atomic_load(&canon[r0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMin(&canon[r0], m);
    }
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Canonical labels: smallest row-major pixel index of each component.
__global__ __launch_bounds__(kThreads) void k_ccl_labels(Geo g, MRef b, const int32_t *__restrict__ glab,
                                                         const int32_t *__restrict__ canon,
                                                         int32_t *__restrict__ labels) {
    const int x = blockIdx.x * kThreads + threadIdx.x, yy = blockIdx.y;
    if (x >= g.W) return;
    const int w = x >> 6;
    uint64_t word = ldm(b, (int64_t)yy * g.wpr + w);
    if (w == g.wpr - 1) word &= g.tail;
    int32_t lab = -1;
    if ((word >> (x & 63)) & 1) {
        const int lr = glab[(int64_t)(yy >> 1) * g.BW + (x >> 1)];
        lab = canon[glab[lr]];
    }
    labels[(int64_t)yy * g.W + x] = lab;
}

__global__ __launch_bounds__(kThreads) void k_unpack(Geo g, const uint64_t *__restrict__ mask,
                                                     uint8_t *__restrict__ out) {
    const int x = blockIdx.x * kThreads + threadIdx.x, yy = blockIdx.y;
    if (x >= g.W) return;
    out[(int64_t)yy * g.W + x] = (uint8_t)((mask[(int64_t)yy * g.wpr + (x >> 6)] >> (x & 63)) & 1);
}

__global__ void k_fill_i64(unsigned long long *p, int n, unsigned long long v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ batch kernels
// Persistent: workgroup u-loop over the launch's global units.  Units per image:
//   BK_WORDS  256 mask words (atoms: four 64-word wave tasks)
//   BK_LOGIC  1024 mask words (Boolean steps)
//   BK_NEAR   four near bands (64 words wide, kBatchNearRows rows high)
//   BK_TILES  one labelling tile          BK_MERGE  four tiles (one per wave)
//   BK_BLOCKS 256 blocks                  BK_GATHER eight 256-block tasks (two per wave)
//   BK_FLAG   4096 blocks (16 per thread)
//   BK_PCTH   kPctUnit channel elements   BK_ONE    one per image

// The descriptor of image ii (wave-uniform) through scalar loads: the table
// is written before the launch and only read while it runs.
__device__ __forceinline__ BImg load_bimg(const BImg *imgs, int ii) {
    static_assert(sizeof(BImg) % 4 == 0, "descriptor copied as 32-bit words");
    const VLG_CONST uint32_t *p = (const VLG_CONST uint32_t *)(imgs + __builtin_amdgcn_readfirstlane(ii));
    BImg r;
    uint32_t *q = (uint32_t *)&r;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(BImg) / 4); k++) q[k] = p[k];
    return r;
}

// d: the descriptor of unit u_'s image, reloaded only when the image changes
#define VLG_BATCH_LOOP(A)                          \
    UnitRange ur_((A).prefix, (A).n);                  \
    int cur_ = -1;                                     \
    BImg dcur_;                                        \
    for (int64_t u_ = ur_.begin; u_ < ur_.end; u_++)
#define VLG_BATCH_IMG(A)                           \
    const int ii = ur_.img(u_);                        \
    if (ii != cur_) {                                  \
        dcur_ = load_bimg((A).imgs, ii);                \
        cur_ = ii;                                     \
    }                                                  \
    const BImg &d = dcur_;

__global__ __launch_bounds__(kThreads) void kb_logic(BatchArgs a, BLogic ops) {
    const BLogicOp &o = ops.ops[blockIdx.y];
    VLG_BATCH_LOOP(a) {
        VLG_BATCH_IMG(a)
        const int64_t i0 = (u_ - a.prefix[ii]) * (kThreads * kLogicUnroll);
        const int64_t iend = min(i0 + kThreads * kLogicUnroll, d.g.nwords);
        logic_words(d.g, bref(d, o.x), bref(d, o.y), o.op, o.inv_out ? ~0ull : 0ull, bptr(d, o.out),
                    i0 + threadIdx.x, kThreads, iend);
    }
}

__global__ __launch_bounds__(kThreads) void kb_near(BatchArgs a, BNear ops) {
    const BNearOp &o = ops.ops[blockIdx.y];
    VLG_BATCH_LOOP(a) {
        VLG_BATCH_IMG(a)
        const int64_t t = (u_ - a.prefix[ii]) * (kThreads / 64) + (threadIdx.x >> 6);
        if (t < near_tasks(d.g, kBatchNearRows))
            near_task(d.g, bref(d, o.x), o.inv_out ? ~0ull : 0ull, bref(d, o.z), o.zop, bptr(d, o.out), t,
                      kBatchNearRows);
    }
}

template <typename T, bool NT>
__global__ __launch_bounds__(kThreads) void kb_atoms(BatchArgs a, BAtoms op) {
    __shared__ float sthr[kMaxAtomsPerLaunch];
    VLG_BATCH_LOOP(a) {
        VLG_BATCH_IMG(a)
        __syncthreads();  // the previous unit is done with sthr
        if ((int)threadIdx.x < op.n) {
            const int p = op.pct[threadIdx.x];
            sthr[threadIdx.x] = p >= 0 ? glb((const float *)(d.ws + d.off_pct))[p] : op.thr[threadIdx.x];
        }
        __syncthreads();
        const T *img = (const T *)(d.img + (int64_t)op.chan * d.chan_bytes);
        const int64_t t = (u_ - a.prefix[ii]) * (kThreads / 64) + (threadIdx.x >> 6);
        auto outf = [&](int j) { return bptr(d, op.out[j]); };
        if (t * 64 < d.g.nwords) atoms_task<T, NT>(d.g, img, op.n, op.cmp, sthr, outf, t);
    }
}

// (at most 64 VGPRs, eight waves per SIMD: a few registers spill, and the
// 512-image batch's tile-local pass still takes 4% less time than at six)
template <int TBH>
__global__ __launch_bounds__(ccl_local_threads<TBH>()) __attribute__((amdgpu_waves_per_eu(8))) void kb_ccl_local(
    BatchArgs a, BRef b, BRef y, BRef z) {
    VLG_BATCH_LOOP(a) {
        VLG_BATCH_IMG(a)
        const int ntx = (d.g.BW + kTileBW - 1) / kTileBW;
        const int tile = (int)(u_ - a.prefix[ii]);
        ccl_local_tile<TBH>(d.g, bref(d, b), bref(d, y), bref(d, z), tile % ntx, tile / ntx,
                            (int32_t *)(d.ws + d.off_glab), (uint8_t *)(d.ws + d.off_gflag), a.guard);
    }
}

template <int TBH>
// (eight waves per SIMD: the descriptor's scalar registers otherwise hold
// it at seven; 1.76 -> 1.58 ms per 512-image batch)
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8))) void kb_ccl_merge(BatchArgs a, BRef b) {
    __shared__ uint64_t win[kThreads / 64][merge_window_words<TBH>()];
    const int wv = threadIdx.x >> 6;
    int unions = 0, tries = 0;
    VLG_BATCH_LOOP(a) {
        VLG_BATCH_IMG(a)
        const int ntx = (d.g.BW + kTileBW - 1) / kTileBW, nty = (d.g.BH + TBH - 1) / TBH;
        const int w = (int)(u_ - a.prefix[ii]) * (kThreads / 64) + wv, tile = w >> 1;
        if (tile < ntx * nty)
            ccl_merge_tile<TBH>(d.g, bref(d, b), ntx, tile, w & 1, (int32_t *)(d.ws + d.off_glab), win[wv], unions,
                                tries, a.guard);
    }
}

__global__ __launch_bounds__(kThreads) void kb_ccl_flag(BatchArgs a) {
    bool ok = true;
    VLG_BATCH_LOOP(a) {
        VLG_BATCH_IMG(a)
        const int64_t i0 = ((u_ - a.prefix[ii]) * kThreads + threadIdx.x) * 16, nb = (int64_t)d.g.BH * d.g.BW;
        if (i0 < nb) ccl_flag_n<16>((int32_t *)(d.ws + d.off_glab), (uint8_t *)(d.ws + d.off_gflag), nb, i0, a.guard.cap, ok);
    }
    guard_report(a.guard, ok);
}

// (eight waves per SIMD, as kb_ccl_merge: 3.97 -> 3.54 ms per 512-image batch)
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8))) void kb_ccl_gather(BatchArgs a, BRef b,
                                                                                                  BRef y, BRef z,
                                                                                                  int user,
                                                                                                  int32_t out) {
    constexpr int NT = kGatherTasksPerWave;
    __shared__ uint64_t zw[kThreads / 64][8 * NT];
    const int wv = threadIdx.x >> 6;
    VLG_BATCH_LOOP(a) {
        VLG_BATCH_IMG(a)
        const int64_t t = ((u_ - a.prefix[ii]) * (kThreads / 64) + wv) * NT;
        const int64_t ntasks = (int64_t)d.g.BH * ((d.g.wpr + 7) / 8);
        if (t < ntasks)
            ccl_gather_tasks<NT>(d.g, bref(d, b), bref(d, y), bref(d, z), (const int32_t *)(d.ws + d.off_glab),
                                 (const uint8_t *)(d.ws + d.off_gflag), user, bptr(d, out), t, ntasks, zw[wv]);
    }
}

__global__ __launch_bounds__(kThreads) void kb_ccl_reseed(BatchArgs a, BRef sm, int user) {
    VLG_BATCH_LOOP(a) {
        VLG_BATCH_IMG(a)
        const int64_t i = (u_ - a.prefix[ii]) * kThreads + threadIdx.x;
        const bool valid = i < (int64_t)d.g.BH * d.g.BW;
        const int by = valid ? (int)(i / d.g.BW) : 0, bx = valid ? (int)(i - (int64_t)by * d.g.BW) : 0;
        ccl_reseed_lane(d.g, bref(d, sm), (const int32_t *)(d.ws + d.off_glab), (uint8_t *)(d.ws + d.off_gflag),
                        user, valid, by, bx);
    }
}

#undef VLG_BATCH_LOOP
#undef VLG_BATCH_IMG

// ------------------------------------------------------------------ segments
// Lane tiles: one wave (a workgroup of its own) per tile of one word column
// and 64 rows, the halo above and below included; lane l takes row r0 + l of
// every register as three words, the column and its two neighbours.  The
// registers live in LDS, each lane reading and writing only its own entries,
// so no instruction needs a barrier; N takes the rows above and below from
// the adjacent lanes by DPP.  64 - 2 * halo rows are stored.  The neighbour
// words lose one bit per N at their far edge and the edge lanes one row, all
// within the halo.
//   LOAD    dst = ptr[a]
//   AND/OR  dst = ((a ^ ia) OP (b ^ ib)) ^ io
//   NEAR_*  dst = (N(a ^ ia) ^ io) OP (b ^ ib), N over the image's pixels only
//           (operand words outside the image and padding bits are background)
//   STORE   ptr[dst] = a ^ ia over the tile's centre (padding bits cleared)
__device__ __forceinline__ uint64_t lane_prev64(uint64_t v) {
    return (uint64_t)(uint32_t)lane_prev((int)(uint32_t)v) | ((uint64_t)(uint32_t)lane_prev((int)(v >> 32)) << 32);
}
__device__ __forceinline__ uint64_t lane_next64(uint64_t v) {
    return (uint64_t)(uint32_t)lane_next((int)(uint32_t)v) | ((uint64_t)(uint32_t)lane_next((int)(v >> 32)) << 32);
}

__global__ __launch_bounds__(64) void k_segment_lane(Geo g, SegProg p, int nty) {
    extern __shared__ uint64_t lreg[];  // [register][word l, c, r][lane]
    // each XCD takes a contiguous range of tiles, so the neighbour words and
    // halo rows that adjacent tiles load again come from that XCD's L2
    const int tile = xcd_contiguous((int)blockIdx.x, (int)gridDim.x);
    const int lane = (int)threadIdx.x, TR = 64 - 2 * p.halo;
    const int tx = tile % g.wpr, ty = tile / g.wpr;
    const int row = ty * TR - p.halo + lane;
    const bool rin = row >= 0 && row < g.H;
    // the image's pixels among the lane's three words (background elsewhere)
    const uint64_t ml = rin && tx >= 1 ? ~0ull : 0ull;
    const uint64_t mc = rin ? (tx == g.wpr - 1 ? g.tail : ~0ull) : 0ull;
    const uint64_t mr = rin && tx + 1 < g.wpr ? (tx + 1 == g.wpr - 1 ? g.tail : ~0ull) : 0ull;
    auto at = [&](int x, int w) -> uint64_t & { return lreg[(x * 3 + w) * 64 + lane]; };
    // the leading loads, all in flight together
    int nl = 0;
    while (nl < p.nins && p.ins[nl].op == SEG_LOAD) nl++;
    {
        const int64_t base = rin ? (int64_t)row * g.wpr + tx : 0;
        uint64_t v[kSegMaxRegs][3];
#pragma unroll
        for (int j = 0; j < kSegMaxRegs; j++)
            if (j < nl) {
                const VLG_GLOBAL uint64_t *src = glb(p.ptr[p.ins[j].a]);
                v[j][0] = ml ? src[base - 1] : 0ull;
                v[j][1] = rin ? src[base] : 0ull;
                v[j][2] = mr ? src[base + 1] : 0ull;
            }
#pragma unroll
        for (int j = 0; j < kSegMaxRegs; j++)
            if (j < nl)
                for (int w = 0; w < 3; w++) at(p.ins[j].dst, w) = v[j][w];
    }
    for (int k = nl; k < p.nins; k++) {
        const SegIns in = p.ins[k];
        const uint64_t ia = (in.inv & 1) ? ~0ull : 0ull, ib = (in.inv & 2) ? ~0ull : 0ull,
                       io = (in.inv & 4) ? ~0ull : 0ull;
        const bool ha = in.a != kSegNone, hb = in.b != kSegNone;  // (kSegNone: the all-zero mask)
        if (in.op == SEG_STORE) {
            if (lane >= p.halo && lane < p.halo + TR && rin) {
                const uint64_t v = (ha ? at(in.a, 1) : 0ull) ^ ia;
                glb(p.ptr[in.dst])[(int64_t)row * g.wpr + tx] = tx == g.wpr - 1 ? (v & g.tail) : v;
            }
            continue;
        }
        const uint64_t al = (ha ? at(in.a, 0) : 0ull) ^ ia, ac = (ha ? at(in.a, 1) : 0ull) ^ ia,
                       ar = (ha ? at(in.a, 2) : 0ull) ^ ia;
        const uint64_t bl = (hb ? at(in.b, 0) : 0ull) ^ ib, bc = (hb ? at(in.b, 1) : 0ull) ^ ib,
                       br = (hb ? at(in.b, 2) : 0ull) ^ ib;
        uint64_t dl, dc, dr;
        if (in.op == SEG_AND || in.op == SEG_OR) {
            const bool o = in.op == SEG_OR;
            dl = (o ? (al | bl) : (al & bl)) ^ io;
            dc = (o ? (ac | bc) : (ac & bc)) ^ io;
            dr = (o ? (ar | br) : (ar & br)) ^ io;
        } else {
            // N over the image's pixels only
            const uint64_t xl = al & ml, xc = ac & mc, xr = ar & mr;
            const uint64_t hl = xl | (xl << 1) | (xl >> 1) | (xc << 63);
            const uint64_t hc = xc | (xc << 1) | (xc >> 1) | (xl >> 63) | (xr << 63);
            const uint64_t hr = xr | (xr << 1) | (xr >> 1) | (xc >> 63);
            const uint64_t nl_ = (hl | lane_prev64(hl) | lane_next64(hl)) ^ io;
            const uint64_t nc = (hc | lane_prev64(hc) | lane_next64(hc)) ^ io;
            const uint64_t nr = (hr | lane_prev64(hr) | lane_next64(hr)) ^ io;
            const bool o = in.op == SEG_NEAR_OR;
            dl = o ? (nl_ | bl) : (nl_ & bl);
            dc = o ? (nc | bc) : (nc & bc);
            dr = o ? (nr | br) : (nr & br);
        }
        at(in.dst, 0) = dl;
        at(in.dst, 1) = dc;
        at(in.dst, 2) = dr;
    }
}

// Wide tiles: an LDS row is 64 words (62 interior words and one halo word on
// each side), so lane l of every wave owns column l of the rows it is given
// (rows wave, wave + 8, ...); left and right neighbour words come from the
// adjacent lanes, the rows above and below from LDS.  Row r of register x is
// sreg[x * NI + r * 64 + lane].  Same instruction semantics as k_segment_lane.
constexpr int kSegWideThreads = 512;
constexpr int kSegWideWaves = kSegWideThreads / 64;
constexpr int kSegWideTW = 62;
__global__ __launch_bounds__(kSegWideThreads) void k_segment_wide(Geo g, SegProg p, int TR, int ntx) {
    extern __shared__ uint64_t sreg[];
    const int RR = TR + 2 * p.halo, NI = RR * 64;
    const int tx = (int)(blockIdx.x % ntx), ty = (int)(blockIdx.x / ntx);
    const int r0 = ty * TR - p.halo, w0 = tx * kSegWideTW - 1;
    const int lane = lane_id(), wave = (int)(threadIdx.x >> 6);
    const int w = w0 + lane;
    const bool win = w >= 0 && w < g.wpr;
    const uint64_t keep = w == g.wpr - 1 ? g.tail : ~0ull;
    int nl = 0;
    while (nl < p.nins && p.ins[nl].op == SEG_LOAD) nl++;
    // the leading loads: for each input, all of this thread's rows in flight
    for (int j = 0; j < nl; j++) {
        const VLG_GLOBAL uint64_t *src = glb((const uint64_t *)p.ptr[p.ins[j].a]);
        uint64_t *dst = sreg + p.ins[j].dst * NI;
        for (int rb = wave; rb < RR; rb += kSegWideWaves * 8) {
            uint64_t v[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int rr = rb + kSegWideWaves * u, row = r0 + rr;
                const bool in = win && rr < RR && row >= 0 && row < g.H;
                v[u] = in ? src[(int64_t)row * g.wpr + w] : 0ull;
            }
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int rr = rb + kSegWideWaves * u;
                if (rr < RR) dst[rr * 64 + lane] = v[u];
            }
        }
    }
    __syncthreads();
    for (int k = nl; k < p.nins; k++) {
        const SegIns in = p.ins[k];
        const uint64_t ia = (in.inv & 1) ? ~0ull : 0ull, ib = (in.inv & 2) ? ~0ull : 0ull,
                       io = (in.inv & 4) ? ~0ull : 0ull;
        const uint64_t *A = in.a != kSegNone ? sreg + in.a * NI : nullptr;
        const uint64_t *B = in.b != kSegNone ? sreg + in.b * NI : nullptr;
        if (in.op == SEG_STORE) {
            // each thread stores the entries it owns (the same it writes in
            // every other instruction): no barrier needed before reuse
            VLG_GLOBAL uint64_t *out = glb(p.ptr[in.dst]);
            const bool col_ok = lane >= 1 && lane <= kSegWideTW && win;
            for (int rr = p.halo + wave; rr < p.halo + TR; rr += kSegWideWaves) {
                const int row = r0 + rr;
                if (!col_ok || row >= g.H) continue;
                out[(int64_t)row * g.wpr + w] = ((A ? A[rr * 64 + lane] : 0ull) ^ ia) & keep;
            }
            continue;
        }
        uint64_t *D = sreg + in.dst * NI;
        if (in.op == SEG_AND || in.op == SEG_OR) {
            for (int rr = wave; rr < RR; rr += kSegWideWaves) {
                const int i = rr * 64 + lane;
                const uint64_t x = (A ? A[i] : 0ull) ^ ia, y = (B ? B[i] : 0ull) ^ ib;
                D[i] = (in.op == SEG_OR ? (x | y) : (x & y)) ^ io;
            }
        } else {
            // N over the image's pixels only: rows and words outside the image
            // and padding bits count as background; rows outside the tile too
            // (they only reach the halo, which is inexact by design)
            auto hrow = [&](int r) -> uint64_t {
                const int row = r0 + r;
                const bool ok = win && r >= 0 && r < RR && row >= 0 && row < g.H;
                const uint64_t v = ok ? (((A ? A[r * 64 + lane] : 0ull) ^ ia) & keep) : 0ull;
                uint64_t l = __shfl_up(v, 1), h = __shfl_down(v, 1);
                if (lane == 0) l = 0ull;
                if (lane == 63) h = 0ull;
                return v | (v << 1) | (v >> 1) | (l >> 63) | (h << 63);
            };
            for (int rr = wave; rr < RR; rr += kSegWideWaves) {
                const uint64_t n = (hrow(rr - 1) | hrow(rr) | hrow(rr + 1)) ^ io;
                const int i = rr * 64 + lane;
                const uint64_t z = (B ? B[i] : 0ull) ^ ib;
                D[i] = in.op == SEG_NEAR_OR ? (n | z) : (n & z);
            }
        }
        __syncthreads();
    }
}

int ntiles_x(const Geo &g) { return (g.BW + kTileBW - 1) / kTileBW; }
int ntiles_y(const Geo &g, int tbh) { return (g.BH + tbh - 1) / tbh; }

}  // namespace

Geo make_geo(int H, int W) {
    Geo g;
    g.H = H;
    g.W = W;
    g.wpr = (W + 63) / 64;
    g.tail = (W % 64) ? ((1ull << (W % 64)) - 1) : ~0ull;
    g.nwords = (int64_t)H * g.wpr;
    g.BH = (H + 1) / 2;
    g.BW = (W + 1) / 2;
    // n / d = (umulhi(n, mul) + n) >> shift, valid for all 32-bit n
    uint32_t d = (uint32_t)(g.wpr > 0 ? g.wpr : 1), s = 0;
    while ((1ull << s) < d) s++;
    g.wpr_mul = (uint32_t)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
    g.wpr_shift = s;
    return g;
}

hipError_t launch_logic(hipStream_t s, const Geo &g, MRef x, MRef y, int op, int inv_out, uint64_t *out) {
    if (g.nwords == 0) return hipSuccess;
    const int grid = grid_for(g.nwords, kThreads, 4096);
    if (3 * g.nwords * 8 > kStreamBytes)
        k_logic<true><<<grid, kThreads, 0, s>>>(g, x, y, op, inv_out ? ~0ull : 0ull, out);
    else
        k_logic<false><<<grid, kThreads, 0, s>>>(g, x, y, op, inv_out ? ~0ull : 0ull, out);
    return hipGetLastError();
}

hipError_t launch_near(hipStream_t s, const Geo &g, MRef x, int inv_out, MRef z, int zop, uint64_t *out,
                       int rows) {
    if (g.nwords == 0) return hipSuccess;
    if (rows == 0) rows = near_band_rows(g);
    if (!valid_near_rows(rows)) return hipErrorInvalidValue;
    k_near<<<grid_for(near_tasks(g, rows), kThreads / 64, 8192), kThreads, 0, s>>>(g, x, inv_out ? ~0ull : 0ull, z,
                                                                                       zop, out, rows);
    return hipGetLastError();
}

template <typename T>
static hipError_t atoms_t(hipStream_t s, const Geo &g, const T *img, const AtomLaunch &a) {
    if (a.n < 1 || a.n > kMaxAtomsPerLaunch) return hipErrorInvalidValue;
    const int grid = grid_for((g.nwords + 63) / 64, kThreads / 64, 8192);
    if (g.nwords * 64 * (int64_t)sizeof(T) + a.n * g.nwords * 8 > kStreamBytes)
        k_atoms<T, true><<<grid, kThreads, 0, s>>>(g, img, a);
    else
        k_atoms<T, false><<<grid, kThreads, 0, s>>>(g, img, a);
    return hipGetLastError();
}

hipError_t launch_atoms(hipStream_t s, const Geo &g, const void *chan, int dtype, const AtomLaunch &a) {
    if (g.nwords == 0) return hipSuccess;
    if (dtype == 1) return atoms_t(s, g, (const uint8_t *)chan, a);
    if (dtype == 2) return atoms_t(s, g, (const uint16_t *)chan, a);
    return atoms_t(s, g, (const float *)chan, a);
}

hipError_t launch_ccl_local(hipStream_t s, const Geo &g, MRef b, MRef y, MRef z, const CclWork &w) {
    if (g.nwords == 0) return hipSuccess;
    if (!valid_tile_bh(w.tbh)) return hipErrorInvalidValue;
    const int ntx = ntiles_x(g), nty = ntiles_y(g, w.tbh);
    switch (w.tbh) {
    case 8: k_ccl_local<8><<<ntx * nty, ccl_local_threads<8>(), 0, s>>>(g, b, y, z, ntx, w.glab, w.gflag, w.guard); break;
    case 16: k_ccl_local<16><<<ntx * nty, ccl_local_threads<16>(), 0, s>>>(g, b, y, z, ntx, w.glab, w.gflag, w.guard); break;
    default: k_ccl_local<32><<<ntx * nty, ccl_local_threads<32>(), 0, s>>>(g, b, y, z, ntx, w.glab, w.gflag, w.guard); break;
    }
    return hipGetLastError();
}

hipError_t launch_ccl_merge(hipStream_t s, const Geo &g, MRef b, const CclWork &w) {
    if (g.nwords == 0) return hipSuccess;
    if (!valid_tile_bh(w.tbh)) return hipErrorInvalidValue;
    const int ntx = ntiles_x(g), nty = ntiles_y(g, w.tbh), ntiles = ntx * nty;
    const int grid = (2 * ntiles + kThreads / 64 - 1) / (kThreads / 64);  // two waves per tile
    switch (w.tbh) {
    case 8: k_ccl_merge<8><<<grid, kThreads, 0, s>>>(g, b, ntx, ntiles, w.glab, w.counters, w.guard); break;
    case 16: k_ccl_merge<16><<<grid, kThreads, 0, s>>>(g, b, ntx, ntiles, w.glab, w.counters, w.guard); break;
    default: k_ccl_merge<32><<<grid, kThreads, 0, s>>>(g, b, ntx, ntiles, w.glab, w.counters, w.guard); break;
    }
    return hipGetLastError();
}

hipError_t launch_ccl_flag(hipStream_t s, const Geo &g, const CclWork &w) {
    if (g.nwords == 0) return hipSuccess;
    const int64_t nb = (int64_t)g.BH * g.BW;
    // four blocks per thread unless sixteen still give 1024 workgroups
    const int per = nb >= (int64_t)16 * kThreads * 1024 ? 16 : 4;
    k_ccl_flag<<<grid_for((nb + per - 1) / per, kThreads, 65536), kThreads, 0, s>>>(nb, w.glab, w.gflag, w.guard,
                                                                                    per);
    return hipGetLastError();
}

hipError_t launch_ccl_gather(hipStream_t s, const Geo &g, MRef b, MRef y, MRef z, const CclWork &w,
                             int user, uint64_t *out) {
    if (g.nwords == 0) return hipSuccess;
    const int64_t tasks = (int64_t)g.BH * ((g.wpr + 7) / 8);
    const int grid = grid_for((tasks + kGatherTasksPerWave - 1) / kGatherTasksPerWave, kThreads / 64, 8192);
    k_ccl_gather<<<grid, kThreads, 0, s>>>(g, b, y, z, w.glab, w.gflag, user, out);
    return hipGetLastError();
}

hipError_t launch_ccl_reseed(hipStream_t s, const Geo &g, MRef sm, const CclWork &w, int user) {
    if (g.nwords == 0) return hipSuccess;
    dim3 grid((g.BW + kThreads - 1) / kThreads, g.BH);
    k_ccl_reseed<<<grid, kThreads, 0, s>>>(g, sm, w.glab, w.gflag, user);
    return hipGetLastError();
}

hipError_t launch_ccl_local_multi(hipStream_t s, const Geo &g, const CclMulti &m, const CclWork &w) {
    if (g.nwords == 0 || m.n == 0) return hipSuccess;
    if (m.n < 0 || m.n > kMaxMulti || !valid_tile_bh(w.tbh)) return hipErrorInvalidValue;
    const int ntx = ntiles_x(g), nty = ntiles_y(g, w.tbh);
    const dim3 grid((unsigned)(ntx * nty), (unsigned)m.n);
    switch (w.tbh) {
    case 8: k_ccl_local_multi<8><<<grid, ccl_local_threads<8>(), 0, s>>>(g, m, ntx, w.guard); break;
    case 16: k_ccl_local_multi<16><<<grid, ccl_local_threads<16>(), 0, s>>>(g, m, ntx, w.guard); break;
    default: k_ccl_local_multi<32><<<grid, ccl_local_threads<32>(), 0, s>>>(g, m, ntx, w.guard); break;
    }
    return hipGetLastError();
}

hipError_t launch_ccl_merge_multi(hipStream_t s, const Geo &g, const CclMulti &m, const CclWork &w) {
    if (g.nwords == 0 || m.n == 0) return hipSuccess;
    if (m.n < 0 || m.n > kMaxMulti || !valid_tile_bh(w.tbh)) return hipErrorInvalidValue;
    const int ntx = ntiles_x(g), nty = ntiles_y(g, w.tbh), ntiles = ntx * nty;
    const dim3 grid((unsigned)((2 * ntiles + kThreads / 64 - 1) / (kThreads / 64)), (unsigned)m.n);
    switch (w.tbh) {
    case 8: k_ccl_merge_multi<8><<<grid, kThreads, 0, s>>>(g, m, ntx, ntiles, w.counters, w.guard); break;
    case 16: k_ccl_merge_multi<16><<<grid, kThreads, 0, s>>>(g, m, ntx, ntiles, w.counters, w.guard); break;
    default: k_ccl_merge_multi<32><<<grid, kThreads, 0, s>>>(g, m, ntx, ntiles, w.counters, w.guard); break;
    }
    return hipGetLastError();
}

hipError_t launch_ccl_flag_multi(hipStream_t s, const Geo &g, const CclMulti &m, const CclWork &w) {
    if (g.nwords == 0 || m.n == 0) return hipSuccess;
    if (m.n < 0 || m.n > kMaxMulti) return hipErrorInvalidValue;
    const int64_t nb = (int64_t)g.BH * g.BW;
    const dim3 grid((unsigned)grid_for((nb + 15) / 16, kThreads, 65536), (unsigned)m.n);
    k_ccl_flag_multi<<<grid, kThreads, 0, s>>>(nb, m, w.guard);
    return hipGetLastError();
}

hipError_t launch_ccl_gather_multi(hipStream_t s, const Geo &g, const CclMulti &m) {
    if (g.nwords == 0 || m.n == 0) return hipSuccess;
    if (m.n < 0 || m.n > kMaxMulti) return hipErrorInvalidValue;
    const int64_t tasks = (int64_t)g.BH * ((g.wpr + 7) / 8);
    const dim3 grid((unsigned)grid_for((tasks + kGatherTasksPerWave - 1) / kGatherTasksPerWave, kThreads / 64, 8192),
                    (unsigned)m.n);
    k_ccl_gather_multi<<<grid, kThreads, 0, s>>>(g, m);
    return hipGetLastError();
}

hipError_t launch_logic_batch(hipStream_t s, const Geo &g, const LogicBatch &b) {
    if (g.nwords == 0 || b.n == 0) return hipSuccess;
    dim3 grid(grid_for(g.nwords, kThreads, 4096), b.n);
    if (3 * b.n * g.nwords * 8 > kStreamBytes) k_logic_batch<true><<<grid, kThreads, 0, s>>>(g, b);
    else k_logic_batch<false><<<grid, kThreads, 0, s>>>(g, b);
    return hipGetLastError();
}

hipError_t launch_near_batch(hipStream_t s, const Geo &g, const NearBatch &b, int rows) {
    if (g.nwords == 0 || b.n == 0) return hipSuccess;
    if (rows == 0) rows = near_band_rows(g);
    if (!valid_near_rows(rows)) return hipErrorInvalidValue;
    dim3 grid(grid_for(near_tasks(g, rows), kThreads / 64, 8192), b.n);
    k_near_batch<<<grid, kThreads, 0, s>>>(g, b, rows);
    return hipGetLastError();
}

hipError_t launch_ccl_labels(hipStream_t s, const Geo &g, MRef b, const CclWork &w, int32_t *canon,
                             int32_t *labels) {
    if (g.nwords == 0) return hipSuccess;
    const int64_t nb = (int64_t)g.BH * g.BW;
    k_fill_i32<<<grid_for(nb, kThreads, 8192), kThreads, 0, s>>>(canon, nb, 0x7fffffff);
    dim3 bgrid((g.BW + kThreads - 1) / kThreads, g.BH);
    k_ccl_canon<<<bgrid, kThreads, 0, s>>>(g, b, w.glab, canon);
    dim3 grid((g.W + kThreads - 1) / kThreads, g.H);
    k_ccl_labels<<<grid, kThreads, 0, s>>>(g, b, w.glab, canon, labels);
    return hipGetLastError();
}

hipError_t launch_unpack(hipStream_t s, const Geo &g, const uint64_t *mask, uint8_t *out) {
    if (g.nwords == 0) return hipSuccess;
    dim3 grid((g.W + kThreads - 1) / kThreads, g.H);
    k_unpack<<<grid, kThreads, 0, s>>>(g, mask, out);
    return hipGetLastError();
}

// Tile of a segment: the shape with the least halo overhead among those that
// fit the LDS budget and leave at least kMinSegTiles tiles (or the most tiles
// when no shape leaves that many).  Wide tiles (62 words, k_segment_wide)
// count only the words of the image they cover.  When a narrow shape (1-16
// words) wins, the segment runs on lane tiles instead (k_segment_lane: one
// word column, 64 - 2 * halo rows per wave), which replaced narrow LDS tiles.
constexpr size_t kSegLdsBudget = 48 * 1024;
constexpr size_t kSegWideLdsBudget = 64 * 1024;
constexpr int64_t kMinSegTiles = 1024;
// lane tiles store at least 16 of their 64 rows
constexpr int kLaneSegMaxHalo = 24;
SegTile seg_tile(const Geo &g, int halo, int nregs) {
    SegTile best{4, 1, 0};
    double best_score = -1.0;
    auto consider = [&](int tr, int tw, size_t lds, double useful_w, int rw) {
        const int64_t tiles = (int64_t)((g.H + tr - 1) / tr) * ((g.wpr + tw - 1) / tw);
        const double eff = (double)tr * useful_w / ((double)(tr + 2 * halo) * rw);
        const double score = eff * std::min(1.0, (double)tiles / kMinSegTiles);
        if (score > best_score) {
            best_score = score;
            best = SegTile{tr, tw, lds};
        }
    };
    for (int tr : {4, 8, 16, 32, 64}) {
        const size_t lds = (size_t)nregs * (tr + 2 * halo) * 64 * 8;
        if (lds <= kSegWideLdsBudget) consider(tr, kSegWideTW, lds, std::min(kSegWideTW, g.wpr), 64);
    }
    for (int tw : {1, 2, 4, 8, 16}) {
        if (tw > 1 && tw / 2 >= g.wpr) break;
        for (int tr : {4, 8, 16, 32}) {
            const size_t lds = (size_t)nregs * (tr + 2 * halo) * (tw + 2) * 8;
            if (lds <= kSegLdsBudget) consider(tr, tw, lds, tw, tw + 2);
        }
    }
    if (best.lds_bytes == 0) best.lds_bytes = (size_t)nregs * (best.tr + 2 * halo) * (best.tw + 2) * 8;
    return best;
}

hipError_t launch_segment(hipStream_t s, const Geo &g, const SegProg &p) {
    if (g.nwords == 0) return hipSuccess;
    if (p.nins < 1 || p.nins > kSegMaxIns || p.nregs < 1 || p.nregs > kSegMaxRegs || p.halo < 0 || p.halo > 32)
        return hipErrorInvalidValue;
    const SegTile t = seg_tile(g, p.halo, p.nregs);
    const int ntx = (g.wpr + t.tw - 1) / t.tw, nty = (g.H + t.tr - 1) / t.tr;
    if (t.tw != kSegWideTW) {
        // lane tiles: one wave per word column and 64 - 2 * halo rows
        if (p.halo > kLaneSegMaxHalo) return hipErrorInvalidValue;
        const int lnty = (g.H + (64 - 2 * p.halo) - 1) / (64 - 2 * p.halo);
        const size_t lds = (size_t)p.nregs * 3 * 64 * 8;
        k_segment_lane<<<(int)((int64_t)g.wpr * lnty), 64, lds, s>>>(g, p, lnty);
    } else {
        if (t.lds_bytes > kSegWideLdsBudget) return hipErrorInvalidValue;
        k_segment_wide<<<ntx * nty, kSegWideThreads, t.lds_bytes, s>>>(g, p, t.tr, ntx);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ measurement
// Device-to-device copy for the HBM reference: each lane moves W-byte units
// (8 or 16) in a grid-stride loop with non-temporal loads and stores, so
// the copy streams past the caches like the large pixel-wise launches.
namespace {
template <typename T>
__global__ __launch_bounds__(kThreads) void k_stream_copy(const T *__restrict__ src, T *__restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(glb(src) + i), glb(dst) + i);
}
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
}  // namespace

hipError_t launch_stream_copy(hipStream_t s, void *dst, const void *src, int64_t bytes, int width) {
    if (bytes <= 0) return hipSuccess;
    if ((width != 8 && width != 16) || bytes % width) return hipErrorInvalidValue;
    const int64_t n = bytes / width;
    const int grid = grid_for(n, kThreads, 256 * 64);
    if (width == 16)
        k_stream_copy<u32x4><<<grid, kThreads, 0, s>>>((const u32x4 *)src, (u32x4 *)dst, n);
    else
        k_stream_copy<uint64_t><<<grid, kThreads, 0, s>>>((const uint64_t *)src, (uint64_t *)dst, n);
    return hipGetLastError();
}

hipError_t launch_fill_i64(hipStream_t s, unsigned long long *p, int n, unsigned long long v) {
    k_fill_i64<<<(n + 255) / 256, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

// ------------------------------------------------------------------ batch launchers

int64_t batch_units(const Geo &g, int kind, int tbh) {
    if (g.nwords == 0) return 0;
    const int64_t nb = (int64_t)g.BH * g.BW;
    const int64_t ntiles = (int64_t)ntiles_x(g) * ntiles_y(g, tbh);
    switch (kind) {
    case BK_WORDS: return (g.nwords + kThreads - 1) / kThreads;
    case BK_LOGIC: return (g.nwords + kThreads * kLogicUnroll - 1) / (kThreads * kLogicUnroll);
    case BK_NEAR: return (near_tasks(g, kBatchNearRows) + kThreads / 64 - 1) / (kThreads / 64);
    case BK_TILES: return ntiles;
    case BK_MERGE: return (2 * ntiles + kThreads / 64 - 1) / (kThreads / 64);  // two waves per tile
    case BK_BLOCKS: return (nb + kThreads - 1) / kThreads;
    case BK_FLAG: return (nb + 16 * kThreads - 1) / (16 * kThreads);
    case BK_GATHER: {
        const int64_t per = (int64_t)kGatherTasksPerWave * (kThreads / 64);  // tasks per unit
        return ((int64_t)g.BH * ((g.wpr + 7) / 8) + per - 1) / per;
    }
    case BK_PCTH: return ((int64_t)g.H * g.wpr * 64 + kPctUnit - 1) / kPctUnit;
    case BK_ONE: return 1;
    }
    return 0;
}

static int persistent_grid(const BatchArgs &a, int64_t total) {
    return grid_for(total, 1, valid_batch_grid(a.grid_cap) ? a.grid_cap : kBatchGridDefault);
}

hipError_t launch_b_atoms(hipStream_t s, const BatchArgs &a, int64_t total, const BAtoms &op) {
    if (total == 0) return hipSuccess;
    if (op.n < 1 || op.n > kMaxAtomsPerLaunch) return hipErrorInvalidValue;
    // a unit is 256 words: 16384 channel elements in, 256 words out per atom
    const int64_t bytes = total * (16384 * (a.dtype == 1 ? 1 : a.dtype == 2 ? 2 : 4) + op.n * 256 * 8);
    const int grid = persistent_grid(a, total);
    if (a.dtype == 1) {
        if (bytes > kStreamBytes) kb_atoms<uint8_t, true><<<grid, kThreads, 0, s>>>(a, op);
        else kb_atoms<uint8_t, false><<<grid, kThreads, 0, s>>>(a, op);
    } else if (a.dtype == 2) {
        if (bytes > kStreamBytes) kb_atoms<uint16_t, true><<<grid, kThreads, 0, s>>>(a, op);
        else kb_atoms<uint16_t, false><<<grid, kThreads, 0, s>>>(a, op);
    } else {
        if (bytes > kStreamBytes) kb_atoms<float, true><<<grid, kThreads, 0, s>>>(a, op);
        else kb_atoms<float, false><<<grid, kThreads, 0, s>>>(a, op);
    }
    return hipGetLastError();
}

hipError_t launch_b_logic(hipStream_t s, const BatchArgs &a, int64_t total, const BLogic &op) {
    if (total == 0 || op.n == 0) return hipSuccess;
    dim3 grid(persistent_grid(a, total), op.n);
    kb_logic<<<grid, kThreads, 0, s>>>(a, op);
    return hipGetLastError();
}

hipError_t launch_b_near(hipStream_t s, const BatchArgs &a, int64_t total, const BNear &op) {
    if (total == 0 || op.n == 0) return hipSuccess;
    dim3 grid(persistent_grid(a, total), op.n);
    kb_near<<<grid, kThreads, 0, s>>>(a, op);
    return hipGetLastError();
}

hipError_t launch_b_ccl_local(hipStream_t s, const BatchArgs &a, int64_t total, int tbh, BRef b, BRef y, BRef z) {
    if (total == 0) return hipSuccess;
    const int grid = persistent_grid(a, total);
    switch (tbh) {
    case 8: kb_ccl_local<8><<<grid, ccl_local_threads<8>(), 0, s>>>(a, b, y, z); break;
    case 16: kb_ccl_local<16><<<grid, ccl_local_threads<16>(), 0, s>>>(a, b, y, z); break;
    case 32: kb_ccl_local<32><<<grid, ccl_local_threads<32>(), 0, s>>>(a, b, y, z); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_b_ccl_merge(hipStream_t s, const BatchArgs &a, int64_t total, int tbh, BRef b) {
    if (total == 0) return hipSuccess;
    const int grid = persistent_grid(a, total);
    switch (tbh) {
    case 8: kb_ccl_merge<8><<<grid, kThreads, 0, s>>>(a, b); break;
    case 16: kb_ccl_merge<16><<<grid, kThreads, 0, s>>>(a, b); break;
    case 32: kb_ccl_merge<32><<<grid, kThreads, 0, s>>>(a, b); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_b_ccl_flag(hipStream_t s, const BatchArgs &a, int64_t total) {
    if (total == 0) return hipSuccess;
    kb_ccl_flag<<<persistent_grid(a, total), kThreads, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_b_ccl_gather(hipStream_t s, const BatchArgs &a, int64_t total, BRef b, BRef y, BRef z, int user,
                               int32_t out) {
    if (total == 0) return hipSuccess;
    kb_ccl_gather<<<persistent_grid(a, total), kThreads, 0, s>>>(a, b, y, z, user, out);
    return hipGetLastError();
}

hipError_t launch_b_ccl_reseed(hipStream_t s, const BatchArgs &a, int64_t total, BRef sm, int user) {
    if (total == 0) return hipSuccess;
    kb_ccl_reseed<<<persistent_grid(a, total), kThreads, 0, s>>>(a, sm, user);
    return hipGetLastError();
}

}  // namespace vlg

// ------------------------------------------------------------------ percentile
// Radix select: keys are the float32 bit patterns made order-preserving
// (negatives complemented, positives with the sign bit set) or the uint8
// values.  Each pass histograms one digit of the keys that agree with the
// digits chosen so far, then a single workgroup finds the bucket holding rank
// k.  float32 uses digits of 13, 10 and 9 bits in batches (the first pass
// has a single group, so its histogram takes the LDS of all four) and 11, 11
// and 10 bits on single images (whose workgroups read fewer elements, so a
// wider histogram to clear and add costs more than its fewer LDS conflicts
// save); uint8 one digit of 8 bits, uint16 two.
namespace vlg {
namespace {

// Selections of a pass whose digits chosen so far agree share one
// histogram: that of the first of them in the step, whose slot is `src`.
// Passes 0 and 2 count into `a`, pass 1 into `b`, so the selection of pass 1
// can clear `a` while others still read `b`.
struct PctState {
    uint32_t prefix, mask, k, src;
    uint32_t a[8192];
    uint32_t b[2048];
};
static_assert(sizeof(PctState) <= kPctStateBytes, "percentile state");

__device__ __forceinline__ uint32_t f32_key(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_f32(uint32_t k) {
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}

__device__ void pct_init_wg(PctState *st_, uint32_t k, int slot) {
    VLG_GLOBAL PctState *st = glb(st_);
    for (int i = threadIdx.x; i < 8192; i += blockDim.x) st->a[i] = 0;
    for (int i = threadIdx.x; i < 2048; i += blockDim.x) st->b[i] = 0;
    if (threadIdx.x == 0) {
        st->prefix = 0;
        st->mask = 0;
        st->k = k;
        st->src = (uint32_t)slot;
    }
}


template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Vec4<uint8_t> { typedef uint8_t type __attribute__((ext_vector_type(4))); };
template <> struct Vec4<uint16_t> { typedef uint16_t type __attribute__((ext_vector_type(4))); };

// Histogram the channel elements of the chunks [c, c + 1024) for c = i0,
// i0 + stride, ... below i1 (a channel is stored with pitch wpr*64; i0,
// stride and i1 are multiples of 1024 or of the pitch, so four consecutive
// elements share a row), for the n selections st[0..n): selections whose
// digits chosen so far agree share one LDS histogram (in the first pass all
// of them do), which is then added into the state of the group's first
// selection.
// The streaming part of a histogram pass over elements [i0, i1): MG is the
// number of groups the group test has to try (one in every first pass).
template <typename T, int MG, bool NT>
__device__ __forceinline__ void pct_hist_stream(const Geo &g, const T *__restrict__ img, int m, const uint32_t *pre,
                                                const uint32_t *msk, int shift, int bins, int64_t i0, int64_t i1,
                                                int64_t stride, uint32_t (*h)[2048]) {
    const int64_t pitch = (int64_t)g.wpr * 64;
    const uint32_t dmask = (uint32_t)(bins - 1);
    using V = typename Vec4<T>::type;
    constexpr int U = 8;  // chunks per iteration: U vector loads in flight per thread
    for (int64_t c = i0; c < i1; c += U * stride) {
        V v[U];
        int64_t idx[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            idx[u] = c + u * stride + threadIdx.x * 4;
            v[u] = ld_hint<NT>((const VLG_GLOBAL V *)(glb(img) + (idx[u] < i1 ? idx[u] : i0)));
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i = idx[u];
            const bool in = i < i1;
            const uint32_t row = fdiv((uint32_t)(i >> 6), g.wpr_mul, g.wpr_shift);
            const int64_t col = i - (int64_t)row * pitch;
            const float f[4] = {(float)v[u].x, (float)v[u].y, (float)v[u].z, (float)v[u].w};
            uint32_t key[4];
#pragma unroll
            for (int e = 0; e < 4; e++) key[e] = sizeof(T) < 4 ? (uint32_t)f[e] : f32_key(f[e]);
            // the groups of a pass share the digit mask and differ in prefix,
            // so an element belongs to at most one of them
            uint32_t bin[4];
            bool act[4];
#pragma unroll
            for (int e = 0; e < 4; e++) {
                int grp = -1;
#pragma unroll
                for (int q = MG - 1; q >= 0; q--)
                    if (q < m && (key[e] & msk[q]) == pre[q]) grp = q;
                act[e] = in && col + e < g.W && grp >= 0;
                bin[e] = (uint32_t)max(grp, 0) * 2048u + ((key[e] >> shift) & dmask);
            }
            // four neighbouring elements in one bin (channel values cluster)
            // take one atomic; otherwise each active element adds its own
            uint32_t *hh = &h[0][0];
            if (act[0] && act[1] && act[2] && act[3] && bin[0] == bin[1] && bin[1] == bin[2] && bin[2] == bin[3]) {
                atomicAdd(&hh[bin[0]], 4u);
            } else {
#pragma unroll
                for (int e = 0; e < 4; e++)
                    if (act[e]) atomicAdd(&hh[bin[e]], 1u);
            }
        }
    }
}

template <typename T, bool NT>
__device__ void pct_hist_range(const Geo &g, const T *__restrict__ img, PctState *const *st, const int32_t *slot,
                               int n, int pass, int shift, int bins, int64_t i0, int64_t i1, int64_t stride,
                               uint32_t (*h)[2048]) {
    __shared__ uint32_t gpre[kMaxPctSel], gmask[kMaxPctSel];
    __shared__ int rep[kMaxPctSel], first[kMaxPctSel], ngroups;
    if (threadIdx.x == 0) {
        int m = 0;
        for (int j = 0; j < n; j++) {
            const uint32_t p = glb(st[j])->prefix, mk = glb(st[j])->mask;
            int r = -1;
            for (int q = 0; q < m; q++)
                if (gpre[q] == p && gmask[q] == mk) r = q;
            if (r < 0) {
                gpre[m] = p;
                gmask[m] = mk;
                first[m] = j;
                r = m++;
            }
            rep[j] = r;
        }
        ngroups = m;
        // (every workgroup writes the same values)
        for (int j = 0; j < n; j++) glb(st[j])->src = (uint32_t)slot[first[rep[j]]];
    }
    __syncthreads();
    // the group table in registers: the histogram atomics below write LDS, so
    // values left in LDS would be reloaded after every one of them
    const int m = ngroups;
    uint32_t pre[kMaxPctSel], msk[kMaxPctSel];
#pragma unroll
    for (int q = 0; q < kMaxPctSel; q++) {
        pre[q] = q < m ? gpre[q] : 0u;
        msk[q] = q < m ? gmask[q] : 0u;
    }
    // group q's bins at q * 2048 (a single group may take all 8192)
    uint32_t *hh = &h[0][0];
    for (int i = threadIdx.x; i < (m - 1) * 2048 + bins; i += kThreads) hh[i] = 0;
    __syncthreads();
    if (m == 1)
        pct_hist_stream<T, 1, NT>(g, img, m, pre, msk, shift, bins, i0, i1, stride, h);
    else
        pct_hist_stream<T, kMaxPctSel, NT>(g, img, m, pre, msk, shift, bins, i0, i1, stride, h);
    __syncthreads();
    // each group's histogram into its first selection's state
    for (int q = 0; q < m; q++) {
        VLG_GLOBAL uint32_t *gh = pass == 1 ? glb(st[first[q]])->b : glb(st[first[q]])->a;
        for (int i = threadIdx.x; i < bins; i += kThreads) {
            const uint32_t cnt = hh[q * 2048 + i];
            if (cnt) __hip_atomic_fetch_add(&gh[i], cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
}

// one workgroup of 256 threads: find the bucket holding rank k
// (src: the state whose histogram the selection shares in this pass)
__device__ void pct_select_wg(PctState *st_, const PctState *src, int pass, int shift, int bins, int last,
                              int is_int, float *result_, uint32_t *part) {
    VLG_GLOBAL PctState *st = glb(st_);
    VLG_GLOBAL float *result = glb(result_);
    const VLG_GLOBAL uint32_t *hist = pass == 1 ? glb(src)->b : glb(src)->a;
    const int per = bins / kThreads;
    uint32_t local = 0;
    for (int j = 0; j < per; j++) local += hist[threadIdx.x * per + j];
    part[threadIdx.x] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0, k = st->k;
        int t = 0;
        while (t < kThreads - 1 && acc + part[t] <= k) acc += part[t++];
        int b = t * per;
        while (b < t * per + per - 1 && acc + hist[b] <= k) acc += hist[b++];
        st->k = k - acc;
        st->prefix |= (uint32_t)b << shift;
        st->mask |= (uint32_t)(bins - 1) << shift;
        if (last) *result = is_int ? (float)st->prefix : key_f32(st->prefix);
    }
    // `a` is read only by the selections of passes 0 and 2: after pass 1 it
    // is cleared for pass 2
    if (pass == 1)
        for (int i = threadIdx.x; i < 8192; i += kThreads) st->a[i] = 0;
    __syncthreads();
}

__device__ __forceinline__ PctState *sstate(void *states, int slot) {
    return (PctState *)((char *)states + (size_t)slot * kPctStateBytes);
}

__global__ void k_pct_init(PctSel sel, void *states) {
    pct_init_wg(sstate(states, sel.slot[blockIdx.x]), sel.k[blockIdx.x], sel.slot[blockIdx.x]);
}

template <typename T, bool NT>
__global__ __launch_bounds__(kThreads) void k_pct_hist(Geo g, const T *__restrict__ img, PctSel sel, void *states,
                                                       int pass, int shift, int bins) {
    __shared__ uint32_t h[kMaxPctSel][2048];
    PctState *st[kMaxPctSel];
    for (int j = 0; j < sel.n; j++) st[j] = sstate(states, sel.slot[j]);
    // one contiguous range of whole chunks per workgroup: neighbouring
    // pixels share bins, so the histogram a workgroup adds into the state has
    // fewer nonzero bins than that of a strided range
    const int64_t n = (int64_t)g.H * g.wpr * 64, chunks = (n + kThreads * 4 - 1) / (kThreads * 4);
    const int64_t per = (chunks + gridDim.x - 1) / gridDim.x * (kThreads * 4);
    const int64_t i0 = (int64_t)blockIdx.x * per, i1 = i0 + per < n ? i0 + per : n;
    pct_hist_range<T, NT>(g, img, st, sel.slot, sel.n, pass, shift, bins, i0, i1, kThreads * 4, h);
}

__global__ __launch_bounds__(kThreads) void k_pct_select(PctSel sel, void *states, int pass, int shift, int bins,
                                                         int last, int is_int, float *results) {
    __shared__ uint32_t part[kThreads];
    const int slot = sel.slot[blockIdx.x];
    PctState *st = sstate(states, slot);
    pct_select_wg(st, sstate(states, (int)glb(st)->src), pass, shift, bins, last, is_int, results + slot, part);
}

// batch variants: state and result of percentile slot p live in each image's workspace
__device__ __forceinline__ PctState *bstate(const BImg &d, int p) {
    return (PctState *)(d.ws + d.off_pctst + (uint64_t)p * kPctStateBytes);
}

__global__ void kb_pct_init(BatchArgs a, PctSel sel) {
    UnitRange ur(a.prefix, a.n);
    for (int64_t u = ur.begin; u < ur.end; u++) {
        const int ii = ur.img(u);
        for (int j = 0; j < sel.n; j++) {
            pct_init_wg(bstate(a.imgs[ii], sel.slot[j]), a.imgs[ii].ranks[sel.slot[j]], sel.slot[j]);
            __syncthreads();
        }
    }
}

template <typename T, bool NT>
__global__ __launch_bounds__(kThreads) void kb_pct_hist(BatchArgs a, int chan, PctSel sel, int pass, int shift,
                                                        int bins) {
    __shared__ uint32_t h[kMaxPctSel][2048];
    UnitRange ur(a.prefix, a.n);
    for (int64_t u = ur.begin; u < ur.end; u++) {
        const int ii = ur.img(u);
        const BImg d = a.imgs[ii];  // by value (see UnitRange)
        PctState *st[kMaxPctSel];
        for (int j = 0; j < sel.n; j++) st[j] = bstate(d, sel.slot[j]);
        const int64_t i0 = (u - a.prefix[ii]) * kPctUnit;
        const int64_t n = (int64_t)d.g.H * d.g.wpr * 64;
        const int64_t i1 = i0 + kPctUnit < n ? i0 + kPctUnit : n;
        pct_hist_range<T, NT>(d.g, (const T *)(d.img + (int64_t)chan * d.chan_bytes), st, sel.slot, sel.n, pass, shift,
                              bins, i0, i1,
                       kThreads * 4, h);
    }
}

__global__ __launch_bounds__(kThreads) void kb_pct_select(BatchArgs a, PctSel sel, int pass, int shift, int bins,
                                                          int last, int is_int) {
    __shared__ uint32_t part[kThreads];
    const int slot = sel.slot[blockIdx.y];
    UnitRange ur(a.prefix, a.n);
    for (int64_t u = ur.begin; u < ur.end; u++) {
        const int ii = ur.img(u);
        const BImg d = a.imgs[ii];  // by value (see UnitRange)
        PctState *st = bstate(d, slot);
        pct_select_wg(st, bstate(d, (int)glb(st)->src), pass, shift, bins, last, is_int,
                      (float *)(d.ws + d.off_pct) + slot, part);
    }
}

}  // namespace

hipError_t launch_percentile(hipStream_t s, const Geo &g, const void *chan, int dtype, const PctSel &sel,
                             void *states, float *results) {
    if (sel.n < 1 || sel.n > kMaxPctSel) return hipErrorInvalidValue;
    k_pct_init<<<sel.n, kThreads, 0, s>>>(sel, states);
    const int64_t n = (int64_t)g.H * g.wpr * 64;
    if (n == 0) return hipGetLastError();
    // at least 32 chunks of 1024 elements per workgroup, so that clearing and
    // adding its histogram (up to 8192 bins) stays small next to its reads
    const int grid = grid_for(n, kThreads * 4 * 32, 2048);
    if (dtype == 1) {
        if (n > kStreamBytes) k_pct_hist<uint8_t, true><<<grid, kThreads, 0, s>>>(g, (const uint8_t *)chan, sel, states, 0, 0, 256);
        else k_pct_hist<uint8_t, false><<<grid, kThreads, 0, s>>>(g, (const uint8_t *)chan, sel, states, 0, 0, 256);
        k_pct_select<<<sel.n, kThreads, 0, s>>>(sel, states, 0, 0, 256, 1, 1, results);
        return hipGetLastError();
    }
    if (dtype == 2) {  // uint16: two 8-bit digits
        for (int p = 0; p < 2; p++) {
            if (2 * n > kStreamBytes)
                k_pct_hist<uint16_t, true><<<grid, kThreads, 0, s>>>(g, (const uint16_t *)chan, sel, states, p, 8 - 8 * p, 256);
            else
                k_pct_hist<uint16_t, false><<<grid, kThreads, 0, s>>>(g, (const uint16_t *)chan, sel, states, p, 8 - 8 * p, 256);
            k_pct_select<<<sel.n, kThreads, 0, s>>>(sel, states, p, 8 - 8 * p, 256, p == 1, 1, results);
        }
        return hipGetLastError();
    }
    const int shifts[3] = {21, 10, 0}, bins[3] = {2048, 2048, 1024};
    for (int p = 0; p < 3; p++) {
        if (4 * n > kStreamBytes)
            k_pct_hist<float, true><<<grid, kThreads, 0, s>>>(g, (const float *)chan, sel, states, p, shifts[p], bins[p]);
        else
            k_pct_hist<float, false><<<grid, kThreads, 0, s>>>(g, (const float *)chan, sel, states, p, shifts[p], bins[p]);
        k_pct_select<<<sel.n, kThreads, 0, s>>>(sel, states, p, shifts[p], bins[p], p == 2, 0, results);
    }
    return hipGetLastError();
}

hipError_t launch_b_percentile(hipStream_t s, const BatchArgs &one, int64_t total_one, const BatchArgs &hist,
                               int64_t total_hist, int chan, const PctSel &sel) {
    if (total_one == 0) return hipSuccess;
    if (sel.n < 1 || sel.n > kMaxPctSel) return hipErrorInvalidValue;
    const int g1 = persistent_grid(one, total_one), gh = persistent_grid(hist, total_hist);
    kb_pct_init<<<g1, kThreads, 0, s>>>(one, sel);
    dim3 gs(g1, sel.n);
    // a histogram unit is kPctUnit channel elements
    const bool nt = total_hist * kPctUnit * (hist.dtype == 1 ? 1 : hist.dtype == 2 ? 2 : 4) > kStreamBytes;
    if (hist.dtype == 1) {
        if (nt) kb_pct_hist<uint8_t, true><<<gh, kThreads, 0, s>>>(hist, chan, sel, 0, 0, 256);
        else kb_pct_hist<uint8_t, false><<<gh, kThreads, 0, s>>>(hist, chan, sel, 0, 0, 256);
        kb_pct_select<<<gs, kThreads, 0, s>>>(one, sel, 0, 0, 256, 1, 1);
        return hipGetLastError();
    }
    if (hist.dtype == 2) {  // uint16: two 8-bit digits
        for (int p = 0; p < 2; p++) {
            if (nt) kb_pct_hist<uint16_t, true><<<gh, kThreads, 0, s>>>(hist, chan, sel, p, 8 - 8 * p, 256);
            else kb_pct_hist<uint16_t, false><<<gh, kThreads, 0, s>>>(hist, chan, sel, p, 8 - 8 * p, 256);
            kb_pct_select<<<gs, kThreads, 0, s>>>(one, sel, p, 8 - 8 * p, 256, p == 1, 1);
        }
        return hipGetLastError();
    }
    const int shifts[3] = {19, 9, 0}, bins[3] = {8192, 1024, 512};
    for (int p = 0; p < 3; p++) {
        if (nt) kb_pct_hist<float, true><<<gh, kThreads, 0, s>>>(hist, chan, sel, p, shifts[p], bins[p]);
        else kb_pct_hist<float, false><<<gh, kThreads, 0, s>>>(hist, chan, sel, p, shifts[p], bins[p]);
        kb_pct_select<<<gs, kThreads, 0, s>>>(one, sel, p, shifts[p], bins[p], p == 2, 0);
    }
    return hipGetLastError();
}

}  // namespace vlg
