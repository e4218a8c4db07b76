// vol.hip -- the logic on volumes (3-D images of D slices of H x W): N over
// the 26 voxels sharing a face, an edge or a vertex (the voxel included),
// and the labelling of 26-connected components behind reachability.
//
// A volume mask is D*H rows of packed words, slice after slice, exactly like
// a 2-D mask of D*H rows; only the spatial operators know the slices.  The
// labelling's union-find nodes are blocks of 2 x 2 x 2 voxels: any two
// voxels of such a block share a face, an edge or a vertex, so the
// foreground voxels of a block lie in one 26-component (the 3-D form of the
// 2 x 2 blocks of the images).  parent[k] for every block k (-1 for a block
// without foreground), compare-and-swap hooks of the larger root under the
// smaller, so a component's root is its smallest block; flag bytes indexed
// by a root block carry the seed bits (bit 1+u for labelling user u), as in
// the 2-D labellings.
#include "kernels.h"

namespace vlg {
namespace {

#define VL_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ VL_GLOBAL T *gv(T *p) {
    return (VL_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ const VL_GLOBAL T *gv(const T *p) {
    return (const VL_GLOBAL T *)p;
}

constexpr int kVlThreads = 256;
constexpr int kVlWaves = kVlThreads / 64;

struct VlBlocks {  // the block grid of a volume (see vb_of_voxel)
    int BX, BY, BZ;
};
VlBlocks vl_blocks(const Geo &g, int S, int D) { return VlBlocks{g.BW, (S + 1) / 2, (D + 1) / 2}; }

__device__ __forceinline__ uint32_t vl_div(uint32_t n, uint32_t mul, uint32_t shift) {
    return (uint32_t)(((uint64_t)__umulhi(n, mul) + n) >> shift);
}

// The word of operand r at (slice z, row y, word w), complement applied,
// padding bits 0; 0 outside the volume.
__device__ __forceinline__ uint64_t vl_word(const Geo &g, int S, int D, const MRef &r, int z, int y, int w) {
    if (z < 0 || z >= D || y < 0 || y >= S || w < 0 || w >= g.wpr) return 0ull;
    const int64_t i = ((int64_t)z * S + y) * g.wpr + w;
    const uint64_t v = (r.p ? gv(r.p)[i] : 0ull) ^ r.inv;
    return w == g.wpr - 1 ? (v & g.tail) : v;
}

// N of operand x at word (z, y, w): the OR over the 3 x 3 rows (z+dz, y+dy)
// of each row dilated by one bit to each side.
__device__ __forceinline__ uint64_t vl_near_word(const Geo &g, int S, int D, const MRef &x, int z, int y, int w) {
    uint64_t n = 0;
#pragma unroll
    for (int dz = -1; dz <= 1; dz++) {
#pragma unroll
        for (int dy = -1; dy <= 1; dy++) {
            const uint64_t c = vl_word(g, S, D, x, z + dz, y + dy, w);
            const uint64_t l = vl_word(g, S, D, x, z + dz, y + dy, w - 1);
            const uint64_t h = vl_word(g, S, D, x, z + dz, y + dy, w + 1);
            n |= c | (c << 1) | (c >> 1) | (l >> 63) | (h << 63);
        }
    }
    return n;
}

// out = (N(x) ^ inv_out) OP z, one thread per word
__global__ __launch_bounds__(kVlThreads) void k_near3(Geo g, int S, int D, MRef x, uint64_t inv_out, MRef z, int zop,
                                                    uint64_t *out) {
    const int64_t wi = (int64_t)blockIdx.x * kVlThreads + threadIdx.x;
    if (wi >= g.nwords) return;
    const uint32_t row = vl_div((uint32_t)wi, g.wpr_mul, g.wpr_shift);
    const int w = (int)((uint32_t)wi - row * (uint32_t)g.wpr), zz = (int)row / S, y = (int)row - zz * S;
    const uint64_t n = vl_near_word(g, S, D, x, zz, y, w) ^ inv_out;
    const uint64_t zw = vl_word(g, S, D, z, zz, y, w);
    const uint64_t keep = w == g.wpr - 1 ? g.tail : ~0ull;
    gv(out)[wi] = (zop ? (n | zw) : (n & zw)) & keep;
}

// One wave per mask word, lane l owning voxel 64*w + l of its row.
struct VlPos {
    int64_t wi, v;
    int z, y, w, x, lane;
    uint64_t bw;
    bool mine;
};
__device__ __forceinline__ bool vl_pos(const Geo &g, int S, int D, const MRef &b, VlPos &q) {
    q.wi = (int64_t)blockIdx.x * kVlWaves + (threadIdx.x >> 6);
    if (q.wi >= g.nwords) return false;
    const uint32_t row = vl_div((uint32_t)q.wi, g.wpr_mul, g.wpr_shift);
    q.w = (int)((uint32_t)q.wi - row * (uint32_t)g.wpr);
    q.z = (int)row / S;
    q.y = (int)row - q.z * S;
    q.lane = (int)(threadIdx.x & 63);
    q.x = q.w * 64 + q.lane;
    q.v = (int64_t)row * g.W + q.x;
    q.bw = vl_word(g, S, D, b, q.z, q.y, q.w);
    q.mine = (q.bw >> q.lane) & 1ull;
    return true;
}

// Root of x: walks up (a parent is never larger than its child) and points
// the walked entries at their grandparents.  `budget` counts the steps left.
__device__ __forceinline__ int vl_find(int *P_, int x, int &budget) {
    VL_GLOBAL int *P = gv(P_);
    int cur = P[x];
    if (cur != x) {
        int prev = x, next;
        while (budget > 0 && cur > (next = P[cur])) {
            budget--;
            P[prev] = next;
            prev = cur;
            cur = next;
        }
    }
    return cur;
}

// Unite the sets of a and b: the larger root is hooked under the smaller by
// compare-and-swap; a failed swap (the root was hooked meanwhile) retries
// from the new parent.  Returns false when the budget ran out.
__device__ __forceinline__ bool vl_unite(int *P, int a, int b, int cap) {
    int budget = cap;
    while (budget > 0) {
        a = vl_find(P, a, budget);
        b = vl_find(P, b, budget);
        if (a == b) return true;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = atomicCAS(P + a, a, b);
        if (old == a) return true;
        a = old;
        budget--;
    }
    return false;
}

__device__ __forceinline__ void vl_report(const LoopGuard &gd, bool ok) {
    const uint64_t bad = __ballot(!ok);
    if (bad && (threadIdx.x & 63) == (unsigned)__builtin_ctzll(bad) && gd.status)
        __hip_atomic_fetch_or(gv(gd.status), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Blocks: block (bz, by, bx) holds slices 2bz, 2bz+1, rows 2by, 2by+1 and
// columns 2bx, 2bx+1; id = (bz*BY + by)*BX + bx; its bits: bit dz*4 + dy*2 + dx
// for voxel (2bz+dz, 2by+dy, 2bx+dx).
__device__ __forceinline__ int64_t vb_of_voxel(const VlBlocks &B, int z, int y, int x) {
    return ((int64_t)(z >> 1) * B.BY + (y >> 1)) * B.BX + (x >> 1);
}

// The voxels of a block that can touch a neighbouring block at offset o
// (-1, 0, 1) along one axis: coordinate 0 (o = -1), any (o = 0), 1 (o = 1);
// the neighbour's side is the mirror image.  Two blocks at offset (oz, oy, ox)
// are 26-connected exactly when the first has a voxel of
// vb_face(oz, oy, ox) and the second one of vb_face(-oz, -oy, -ox): every
// such pair differs by at most one along each axis.
__host__ __device__ constexpr uint32_t vb_face(int oz, int oy, int ox) {
    uint32_t m = 0;
    for (int dz = 0; dz < 2; dz++)
        for (int dy = 0; dy < 2; dy++)
            for (int dx = 0; dx < 2; dx++) {
                const bool in = (oz == 0 || (oz < 0) == (dz == 0)) && (oy == 0 || (oy < 0) == (dy == 0)) &&
                                (ox == 0 || (ox < 0) == (dx == 0));
                if (in) m |= 1u << (dz * 4 + dy * 2 + dx);
            }
    return m;
}
static_assert(vb_face(0, 0, -1) == 0x55 && vb_face(0, 0, 1) == 0xAA && vb_face(-1, -1, -1) == 0x01 &&
                  vb_face(1, 1, 1) == 0x80 && vb_face(0, 0, 0) == 0xFF,
              "block faces");

// The block rows of the labelling passes: one wave per 64 consecutive blocks
// of a block row (bz, by), chunk cx, lane l owning block bx = 64*cx + l.
struct VbRow {
    int bz, by, cx, lane, bx;
    int64_t id;
    bool valid;
};
__device__ __forceinline__ bool vb_row(const VlBlocks &B, int CX, VbRow &r) {
    const int64_t wv = (int64_t)blockIdx.x * kVlWaves + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (wv >= (int64_t)B.BZ * B.BY * CX) return false;
    r.cx = (int)(wv % CX);
    const int64_t zy = wv / CX;
    r.by = (int)(zy % B.BY);
    r.bz = (int)(zy / B.BY);
    r.lane = (int)(threadIdx.x & 63);
    r.bx = 64 * r.cx + r.lane;
    r.valid = r.bx < B.BX;
    r.id = zy * B.BX + r.bx;
    return true;
}

// Bits of the blocks bx-1, bx and bx+1 of block row (bz, by) for lane l of
// chunk cx (bx = 64*cx + l): 0 outside the volume.  Each of the block row's
// four voxel rows contributes the six voxels x = 2bx-2 .. 2bx+3, taken from
// the four mask words 2cx-1 .. 2cx+2 that the chunk and its neighbours span.
__device__ __forceinline__ void vb_row_bits(const Geo &g, int S, int D, const MRef &b, int bz, int by, int cx,
                                            int lane, uint32_t (&o)[3]) {
    o[0] = o[1] = o[2] = 0;
    if (bz < 0 || by < 0 || 2 * bz >= D || 2 * by >= S) return;
    const int off = 62 + 2 * lane, k = off >> 6, sh = off & 63;  // bit of voxel 2bx-2 in the four words
#pragma unroll
    for (int dz = 0; dz < 2; dz++)
#pragma unroll
        for (int dy = 0; dy < 2; dy++) {
            uint64_t w[4];
#pragma unroll
            for (int j = 0; j < 4; j++) w[j] = vl_word(g, S, D, b, 2 * bz + dz, 2 * by + dy, 2 * cx - 1 + j);
            const uint64_t lo = k == 0 ? w[0] : k == 1 ? w[1] : w[2];
            const uint64_t hi = k == 0 ? w[1] : k == 1 ? w[2] : w[3];
            const uint32_t win = (uint32_t)(((lo >> sh) | (sh > 58 ? hi << (64 - sh) : 0ull)) & 63u);
            const int r = dz * 2 + dy;
#pragma unroll
            for (int j = 0; j < 3; j++) o[j] |= ((win >> (2 * j)) & 3u) << (2 * r);
        }
}

__device__ __forceinline__ int vb_lane_prev(int v) {  // lane l-1's v; lane 0 gets 0
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int vb_lane_next(int v) {  // lane l+1's v; lane 63 gets 0
    return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false);
}

// Lane of the first block of each lane's run in a chunk: blocks joined to
// their left neighbour through the x faces form runs; a chunk's first block
// starts a run.
__device__ __forceinline__ int vb_run(uint32_t bits, uint32_t left_bits, int lane, bool &conn) {
    conn = lane > 0 && (bits & vb_face(0, 0, -1)) && (left_bits & vb_face(0, 0, 1));
    const uint64_t starts = __ballot(bits != 0 && !conn);
    const uint64_t upto = starts & (~0ull >> (63 - lane));
    return upto ? 63 - __builtin_clzll(upto) : lane;
}

// Initial parents: every block of b points at the first block of its run in
// its chunk; the run starts are roots.
__global__ __launch_bounds__(kVlThreads) void k_vb_init(Geo g, int S, int D, VlBlocks B, int CX, MRef b, int *P) {
    VbRow r;
    if (!vb_row(B, CX, r)) return;
    uint32_t cur[3];
    vb_row_bits(g, S, D, b, r.bz, r.by, r.cx, r.lane, cur);
    const uint32_t bits = r.valid ? cur[1] : 0u;
    bool conn;
    const int run = vb_run(bits, cur[0], r.lane, conn);
    if (r.valid) gv(P)[r.id] = bits ? (int)(r.id - (r.lane - run)) : -1;
}

// Unions of every block of b with its earlier neighbours: the left block
// across a chunk border (inside a chunk the runs join them), and the blocks
// bx-1, bx, bx+1 of the four earlier block rows (bz, by-1), (bz-1, by-1),
// (bz-1, by), (bz-1, by+1) that it touches.  The runs of each earlier row are
// found the same way; a block unites its run with each touched run of that
// row once, and not at all with a run that its left neighbour, in its own
// run, already touches.
__global__ __launch_bounds__(kVlThreads) void k_vb_union(Geo g, int S, int D, VlBlocks B, int CX, MRef b, int *P,
                                                       LoopGuard gd) {
    VbRow r;
    if (!vb_row(B, CX, r)) return;
    uint32_t cur[3];
    vb_row_bits(g, S, D, b, r.bz, r.by, r.cx, r.lane, cur);
    const uint32_t bits = r.valid ? cur[1] : 0u;
    bool conn;
    const int run = vb_run(bits, cur[0], r.lane, conn);
    const int me = (int)(r.id - (r.lane - run));  // this block's run start
    bool ok = true;
    if (r.lane == 0 && bits && (bits & vb_face(0, 0, -1)) && (cur[0] & vb_face(0, 0, 1)))
        ok &= vl_unite(P, (int)r.id, (int)r.id - 1, gd.cap);
    const int rz[4] = {0, -1, -1, -1}, ry[4] = {-1, -1, 0, 1};
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int oz = rz[q], oy = ry[q], bz = r.bz + oz, by = r.by + oy;
        uint32_t nb[3];
        vb_row_bits(g, S, D, b, bz, by, r.cx, r.lane, nb);
        if (bz < 0 || by < 0 || by >= B.BY) continue;  // wave-uniform
        const uint32_t rb = r.valid ? nb[1] : 0u;
        bool rconn;
        const int rrun = vb_run(rb, nb[0], r.lane, rconn);
        const int rprev = vb_lane_prev(rrun), rnext = vb_lane_next(rrun);
        // run tags of the touched blocks bx-1, bx, bx+1 (the run start's lane;
        // 64 and 65: blocks of the neighbouring chunks), -1 untouched
        int t[3];
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const int ox = j - 1;
            const bool touch = (bits & vb_face(oz, oy, ox)) && (nb[j] & vb_face(-oz, -oy, -ox));
            t[j] = !touch ? -1 : ox < 0 ? (r.lane == 0 ? 64 : rprev) : ox > 0 ? (r.lane == 63 ? 65 : rnext) : rrun;
        }
        if (t[1] == t[0]) t[1] = -1;
        if (t[2] == t[0] || t[2] == t[1]) t[2] = -1;
        const int l0 = vb_lane_prev(t[0]), l1 = vb_lane_prev(t[1]), l2 = vb_lane_prev(t[2]);
        const int64_t row0 = ((int64_t)bz * B.BY + by) * B.BX + 64 * r.cx;  // block of lane 0 in that row
#pragma unroll
        for (int j = 0; j < 3; j++) {
            if (t[j] < 0) continue;
            if (conn && (t[j] == l0 || t[j] == l1 || t[j] == l2)) continue;
            const int64_t other = t[j] == 64 ? row0 - 1 : t[j] == 65 ? row0 + 64 : row0 + t[j];
            ok &= vl_unite(P, me, (int)other, gd.cap);
        }
    }
    vl_report(gd, ok);
}

// Every block of b points at its root.  The walk only reads: a walker writes
// its own entry alone, and only with the root.  (Compressing the entries it
// walks through could overwrite, with a stale non-root ancestor, the root
// that the entry's own walker has already written.)
__global__ __launch_bounds__(kVlThreads) void k_vb_flatten(int64_t nb, int *P_, LoopGuard gd) {
    VL_GLOBAL int *P = gv(P_);
    bool ok = true;
    for (int64_t k = (int64_t)blockIdx.x * kVlThreads + threadIdx.x; k < nb; k += (int64_t)gridDim.x * kVlThreads) {
        int cur = P[k], next;
        if (cur < 0) continue;
        int budget = gd.cap;
        while (budget > 0 && cur > (next = P[cur])) {
            budget--;
            cur = next;
        }
        if (P[cur] == cur)
            P[k] = cur;
        else
            ok = false;  // the walk stopped at its cap
    }
    vl_report(gd, ok);
}

// Seeds of a reachability: flag the roots of the voxels of N(y & z) & b.
// The word of N(y & z) is the OR of 27 pieces, one per lane: lane k < 27
// loads the (y & z) word at slice offset k/9 - 1, row offset (k/3)%3 - 1 and
// word offset k%3 - 1 and keeps what it contributes to this word (the word
// dilated by one bit to each side, or the edge bit of a neighbour word); a
// wave-wide OR then gives every lane the whole word.
__global__ __launch_bounds__(kVlThreads) void k_vl_seed(Geo g, int S, int D, VlBlocks B, MRef b, MRef y, MRef z,
                                                      const int *__restrict__ P, uint8_t *flag, uint32_t bit) {
    VlPos q;
    if (!vl_pos(g, S, D, b, q) || q.bw == 0) return;
    uint64_t n = 0;
    if (q.lane < 27) {
        const int dz = q.lane / 9 - 1, dy = (q.lane / 3) % 3 - 1, dw = q.lane % 3 - 1;
        const uint64_t c = vl_word(g, S, D, y, q.z + dz, q.y + dy, q.w + dw) &
                           vl_word(g, S, D, z, q.z + dz, q.y + dy, q.w + dw);
        n = dw == 0 ? (c | (c << 1) | (c >> 1)) : dw < 0 ? (c >> 63) : (c << 63);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) n |= __shfl_xor(n, off);
    if (!q.mine || !((n >> q.lane) & 1ull)) return;
    VL_GLOBAL uint8_t *f = gv(flag) + gv(P)[vb_of_voxel(B, q.z, q.y, q.x)];
    if (!(*f & bit)) *f = (uint8_t)(*f | bit);
}

// Another seed set on the same labelling: the roots of the voxels of s.
__global__ __launch_bounds__(kVlThreads) void k_vl_reseed(Geo g, int S, int D, VlBlocks B, MRef s,
                                                        const int *__restrict__ P, uint8_t *flag, uint32_t bit) {
    VlPos q;
    if (!vl_pos(g, S, D, s, q) || q.bw == 0 || !q.mine) return;
    const int r = gv(P)[vb_of_voxel(B, q.z, q.y, q.x)];
    if (r < 0) return;
    VL_GLOBAL uint8_t *f = gv(flag) + r;
    if (!(*f & bit)) *f = (uint8_t)(*f | bit);
}

// out = (y & z) | (voxels of b whose root carries `bit`)
__global__ __launch_bounds__(kVlThreads) void k_vl_gather(Geo g, int S, int D, VlBlocks B, MRef b, MRef y, MRef z,
                                                        const int *__restrict__ P, const uint8_t *__restrict__ flag,
                                                        uint32_t bit, uint64_t *out) {
    VlPos q;
    if (!vl_pos(g, S, D, b, q)) return;
    bool in = false;
    if (q.mine) in = (gv(flag)[gv(P)[vb_of_voxel(B, q.z, q.y, q.x)]] & bit) != 0;
    const uint64_t zw = __ballot(in);
    if (q.lane == 0)
        gv(out)[q.wi] = (vl_word(g, S, D, y, q.z, q.y, q.w) & vl_word(g, S, D, z, q.z, q.y, q.w)) | (q.bw & zw);
}

// Canonical labels: canon[root] = the smallest voxel of the root's component
// (canon filled with INT_MAX first), then labels[v] = canon[root of v], -1
// for background.
__global__ __launch_bounds__(kVlThreads) void k_vb_canon(Geo g, int S, int D, VlBlocks B, MRef b,
                                                       const int *__restrict__ P, int *canon) {
    VlPos q;
    if (!vl_pos(g, S, D, b, q) || !q.mine) return;
    __hip_atomic_fetch_min(canon + gv(P)[vb_of_voxel(B, q.z, q.y, q.x)], (int)q.v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
__global__ __launch_bounds__(kVlThreads) void k_vb_labels(Geo g, int S, int D, VlBlocks B, MRef b,
                                                        const int *__restrict__ P, const int *__restrict__ canon,
                                                        int *labels) {
    VlPos q;
    if (!vl_pos(g, S, D, b, q) || q.x >= g.W) return;
    gv(labels)[q.v] = q.mine ? gv(canon)[gv(P)[vb_of_voxel(B, q.z, q.y, q.x)]] : -1;
}

__global__ __launch_bounds__(kVlThreads) void k_vl_fill(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * kVlThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVlThreads)
        gv(p)[i] = v;
}

unsigned vl_waves_grid(const Geo &g) { return (unsigned)((g.nwords + kVlWaves - 1) / kVlWaves); }

}  // namespace

hipError_t launch_near3(hipStream_t s, const Geo &g, int S, int D, MRef x, int inv_out, MRef z, int zop,
                        uint64_t *out) {
    if (g.nwords == 0) return hipSuccess;
    if (S < 1 || D < 1 || (int64_t)S * D != g.H) return hipErrorInvalidValue;
    k_near3<<<(unsigned)((g.nwords + kVlThreads - 1) / kVlThreads), kVlThreads, 0, s>>>(
        g, S, D, x, inv_out ? ~0ull : 0ull, z, zop, out);
    return hipGetLastError();
}

int64_t vl_nblocks(const Geo &g, int S, int D) {
    const VlBlocks B = vl_blocks(g, S, D);
    return (int64_t)B.BX * B.BY * B.BZ;
}

hipError_t launch_vl_label(hipStream_t s, const Geo &g, int S, int D, MRef b, int *P, const LoopGuard &gd) {
    if (g.nwords == 0) return hipSuccess;
    if (S < 1 || D < 1 || (int64_t)S * D != g.H) return hipErrorInvalidValue;
    const VlBlocks B = vl_blocks(g, S, D);
    const int CX = (B.BX + 63) / 64;
    const int64_t waves = (int64_t)B.BZ * B.BY * CX, nb = (int64_t)B.BX * B.BY * B.BZ;
    const unsigned grid = (unsigned)((waves + kVlWaves - 1) / kVlWaves);
    k_vb_init<<<grid, kVlThreads, 0, s>>>(g, S, D, B, CX, b, P);
    k_vb_union<<<grid, kVlThreads, 0, s>>>(g, S, D, B, CX, b, P, gd);
    int64_t fb = (nb + kVlThreads - 1) / kVlThreads;
    if (fb > 8192) fb = 8192;
    k_vb_flatten<<<(unsigned)fb, kVlThreads, 0, s>>>(nb, P, gd);
    return hipGetLastError();
}

hipError_t launch_vl_labels(hipStream_t s, const Geo &g, int S, int D, MRef b, const int *P, int *canon,
                            int *labels) {
    if (g.nwords == 0) return hipSuccess;
    if (S < 1 || D < 1 || (int64_t)S * D != g.H) return hipErrorInvalidValue;
    const VlBlocks B = vl_blocks(g, S, D);
    const int64_t nb = (int64_t)B.BX * B.BY * B.BZ;
    int64_t fb = (nb + kVlThreads - 1) / kVlThreads;
    if (fb > 8192) fb = 8192;
    k_vl_fill<<<(unsigned)fb, kVlThreads, 0, s>>>((uint32_t *)canon, nb, 0x7FFFFFFFu);
    k_vb_canon<<<vl_waves_grid(g), kVlThreads, 0, s>>>(g, S, D, B, b, P, canon);
    k_vb_labels<<<vl_waves_grid(g), kVlThreads, 0, s>>>(g, S, D, B, b, P, canon, labels);
    return hipGetLastError();
}

hipError_t launch_vl_clear_flags(hipStream_t s, const Geo &g, int S, int D, uint8_t *flag) {
    if (g.nwords == 0) return hipSuccess;
    const int64_t n = (vl_nblocks(g, S, D) + 3) / 4;
    if (n == 0) return hipSuccess;
    int64_t blocks = (n + kVlThreads - 1) / kVlThreads;
    if (blocks > 8192) blocks = 8192;
    k_vl_fill<<<(unsigned)blocks, kVlThreads, 0, s>>>((uint32_t *)flag, n, 0u);
    return hipGetLastError();
}

hipError_t launch_vl_seed(hipStream_t s, const Geo &g, int S, int D, MRef b, MRef y, MRef z, const int *P,
                          uint8_t *flag, int user) {
    if (g.nwords == 0) return hipSuccess;
    k_vl_seed<<<vl_waves_grid(g), kVlThreads, 0, s>>>(g, S, D, vl_blocks(g, S, D), b, y, z, P, flag, 2u << user);
    return hipGetLastError();
}

hipError_t launch_vl_reseed(hipStream_t s, const Geo &g, int S, int D, MRef sm, const int *P, uint8_t *flag,
                            int user) {
    if (g.nwords == 0) return hipSuccess;
    k_vl_reseed<<<vl_waves_grid(g), kVlThreads, 0, s>>>(g, S, D, vl_blocks(g, S, D), sm, P, flag, 2u << user);
    return hipGetLastError();
}

hipError_t launch_vl_gather(hipStream_t s, const Geo &g, int S, int D, MRef b, MRef y, MRef z, const int *P,
                            const uint8_t *flag, int user, uint64_t *out) {
    if (g.nwords == 0) return hipSuccess;
    k_vl_gather<<<vl_waves_grid(g), kVlThreads, 0, s>>>(g, S, D, vl_blocks(g, S, D), b, y, z, P, flag, 2u << user,
                                                        out);
    return hipGetLastError();
}

}  // namespace vlg
