// vol.hip -- the logic on volumes (3-D images of D slices of H x W): N over
// the 26 voxels sharing a face, an edge or a vertex (the voxel included),
// and the labelling of 26-connected components behind reachability.
//
// A volume mask is D*H rows of packed words, slice after slice, exactly like
// a 2-D mask of D*H rows; only the spatial operators know the slices.  The
// labelling works on voxels: parent[v] for every voxel v = (z*H + y)*W + x
// (-1 for background), union-find with compare-and-swap hooks of the larger
// root under the smaller, so a component's root is its smallest voxel;
// flag bytes indexed by a root's voxel carry the seed bits (bit 1+u for
// labelling user u), as in the 2-D labellings.
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

__device__ __forceinline__ bool vl_bit(const Geo &g, int S, int D, const MRef &b, int z, int y, int x) {
    if (x < 0 || x >= g.W) return false;
    return (vl_word(g, S, D, b, z, y, x >> 6) >> (x & 63)) & 1ull;
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

// Initial parents: each voxel of b points at the first voxel of its run
// (consecutive voxels of b in its row) within its mask word; the run start
// is a root.  Runs that continue across a word boundary are joined by the
// union pass.
__global__ __launch_bounds__(kVlThreads) void k_vl_init(Geo g, int S, int D, MRef b, int *P) {
    VlPos q;
    if (!vl_pos(g, S, D, b, q) || q.x >= g.W) return;
    int r = -1;
    if (q.mine) {
        const uint64_t gaps = ~q.bw & ((1ull << q.lane) - 1ull);  // background voxels before this one
        const int start = gaps ? 64 - __builtin_clzll(gaps) : 0;
        r = (int)(q.v - (q.lane - start));
    }
    gv(P)[q.v] = r;
}

// Unions with the voxels before each voxel of b in linear order: the
// neighbours in the row above and in the three rows of the slice before
// (rows R), and the left neighbour across a word boundary (inside a word
// the run's parents already join it).  Connections that are already made
// are skipped: a voxel whose left neighbour is in b leaves the neighbours
// at x-1 and x of each row R to that neighbour and unites only with x+1,
// and only when x is not in b (otherwise x+1 is in the run of x); a run's
// first voxel unites with x if it is in b, else with x-1 and x+1.
__global__ __launch_bounds__(kVlThreads) void k_vl_union(Geo g, int S, int D, MRef b, int *P, LoopGuard gd) {
    VlPos q;
    if (!vl_pos(g, S, D, b, q)) return;
    bool ok = true;
    if (q.mine) {
        const bool left = vl_bit(g, S, D, b, q.z, q.y, q.x - 1);
        if (left && q.lane == 0) ok &= vl_unite(P, (int)q.v, (int)q.v - 1, gd.cap);
        const int rz[4] = {q.z - 1, q.z - 1, q.z - 1, q.z}, ry[4] = {q.y - 1, q.y, q.y + 1, q.y - 1};
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int z = rz[k], y = ry[k];
            if (z < 0 || y < 0 || y >= S) continue;
            const int64_t base = ((int64_t)z * S + y) * g.W;
            const bool c = vl_bit(g, S, D, b, z, y, q.x), r = vl_bit(g, S, D, b, z, y, q.x + 1);
            if (left) {
                if (!c && r) ok &= vl_unite(P, (int)q.v, (int)(base + q.x + 1), gd.cap);
            } else if (c) {
                ok &= vl_unite(P, (int)q.v, (int)(base + q.x), gd.cap);
            } else {
                if (vl_bit(g, S, D, b, z, y, q.x - 1)) ok &= vl_unite(P, (int)q.v, (int)(base + q.x - 1), gd.cap);
                if (r) ok &= vl_unite(P, (int)q.v, (int)(base + q.x + 1), gd.cap);
            }
        }
    }
    vl_report(gd, ok);
}

// Every voxel points at its root.  The walk only reads: a walker writes its
// own entry alone, and only with the root.  (Compressing the entries it
// walks through could overwrite, with a stale non-root ancestor, the root
// that the entry's own walker has already written.)
__global__ __launch_bounds__(kVlThreads) void k_vl_flatten(Geo g, int S, int D, MRef b, int *P_, LoopGuard gd) {
    VlPos q;
    if (!vl_pos(g, S, D, b, q)) return;
    VL_GLOBAL int *P = gv(P_);
    bool ok = true;
    if (q.mine) {
        int cur = P[q.v], next;
        int budget = gd.cap;
        while (budget > 0 && cur > (next = P[cur])) {
            budget--;
            cur = next;
        }
        if (P[cur] == cur)
            P[q.v] = cur;
        else
            ok = false;  // the walk stopped at its cap
    }
    vl_report(gd, ok);
}

// Seeds of a reachability: flag the roots of the voxels of N(y & z) & b.
__global__ __launch_bounds__(kVlThreads) void k_vl_seed(Geo g, int S, int D, MRef b, MRef y, MRef z,
                                                      const int *__restrict__ P, uint8_t *flag, uint32_t bit) {
    VlPos q;
    if (!vl_pos(g, S, D, b, q) || q.bw == 0) return;
    uint64_t n = 0;
#pragma unroll
    for (int dz = -1; dz <= 1; dz++) {
#pragma unroll
        for (int dy = -1; dy <= 1; dy++) {
            auto yz = [&](int w) {
                return vl_word(g, S, D, y, q.z + dz, q.y + dy, w) & vl_word(g, S, D, z, q.z + dz, q.y + dy, w);
            };
            const uint64_t c = yz(q.w), l = yz(q.w - 1), h = yz(q.w + 1);
            n |= c | (c << 1) | (c >> 1) | (l >> 63) | (h << 63);
        }
    }
    if (!q.mine || !((n >> q.lane) & 1ull)) return;
    VL_GLOBAL uint8_t *f = gv(flag) + gv(P)[q.v];
    if (!(*f & bit)) *f = (uint8_t)(*f | bit);
}

// Another seed set on the same labelling: the roots of the voxels of s.
__global__ __launch_bounds__(kVlThreads) void k_vl_reseed(Geo g, int S, int D, MRef s, const int *__restrict__ P,
                                                        uint8_t *flag, uint32_t bit) {
    VlPos q;
    if (!vl_pos(g, S, D, s, q) || q.bw == 0 || !q.mine) return;
    const int r = gv(P)[q.v];
    if (r < 0) return;
    VL_GLOBAL uint8_t *f = gv(flag) + r;
    if (!(*f & bit)) *f = (uint8_t)(*f | bit);
}

// out = (y & z) | (voxels of b whose root carries `bit`)
__global__ __launch_bounds__(kVlThreads) void k_vl_gather(Geo g, int S, int D, MRef b, MRef y, MRef z,
                                                        const int *__restrict__ P, const uint8_t *__restrict__ flag,
                                                        uint32_t bit, uint64_t *out) {
    VlPos q;
    if (!vl_pos(g, S, D, b, q)) return;
    bool in = false;
    if (q.mine) in = (gv(flag)[gv(P)[q.v]] & bit) != 0;
    const uint64_t zw = __ballot(in);
    if (q.lane == 0)
        gv(out)[q.wi] = (vl_word(g, S, D, y, q.z, q.y, q.w) & vl_word(g, S, D, z, q.z, q.y, q.w)) | (q.bw & zw);
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

hipError_t launch_vl_label(hipStream_t s, const Geo &g, int S, int D, MRef b, int *P, const LoopGuard &gd) {
    if (g.nwords == 0) return hipSuccess;
    if (S < 1 || D < 1 || (int64_t)S * D != g.H) return hipErrorInvalidValue;
    k_vl_init<<<vl_waves_grid(g), kVlThreads, 0, s>>>(g, S, D, b, P);
    k_vl_union<<<vl_waves_grid(g), kVlThreads, 0, s>>>(g, S, D, b, P, gd);
    k_vl_flatten<<<vl_waves_grid(g), kVlThreads, 0, s>>>(g, S, D, b, P, gd);
    return hipGetLastError();
}

hipError_t launch_vl_clear_flags(hipStream_t s, const Geo &g, uint8_t *flag) {
    const int64_t n = ((int64_t)g.H * g.W + 3) / 4;
    if (n == 0) return hipSuccess;
    int64_t blocks = (n + kVlThreads - 1) / kVlThreads;
    if (blocks > 8192) blocks = 8192;
    k_vl_fill<<<(unsigned)blocks, kVlThreads, 0, s>>>((uint32_t *)flag, n, 0u);
    return hipGetLastError();
}

hipError_t launch_vl_seed(hipStream_t s, const Geo &g, int S, int D, MRef b, MRef y, MRef z, const int *P,
                          uint8_t *flag, int user) {
    if (g.nwords == 0) return hipSuccess;
    k_vl_seed<<<vl_waves_grid(g), kVlThreads, 0, s>>>(g, S, D, b, y, z, P, flag, 2u << user);
    return hipGetLastError();
}

hipError_t launch_vl_reseed(hipStream_t s, const Geo &g, int S, int D, MRef sm, const int *P, uint8_t *flag,
                            int user) {
    if (g.nwords == 0) return hipSuccess;
    k_vl_reseed<<<vl_waves_grid(g), kVlThreads, 0, s>>>(g, S, D, sm, P, flag, 2u << user);
    return hipGetLastError();
}

hipError_t launch_vl_gather(hipStream_t s, const Geo &g, int S, int D, MRef b, MRef y, MRef z, const int *P,
                            const uint8_t *flag, int user, uint64_t *out) {
    if (g.nwords == 0) return hipSuccess;
    k_vl_gather<<<vl_waves_grid(g), kVlThreads, 0, s>>>(g, S, D, b, y, z, P, flag, 2u << user, out);
    return hipGetLastError();
}

}  // namespace vlg
