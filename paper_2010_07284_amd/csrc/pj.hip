// pj.hip -- the paper's own connected-component labelling (Sect. 3, Alg. CCL):
// coordinate labels, max-neighbour pointer jumping (mainIteration), a
// periodic reconnect with an atomic write, and a termination check the host
// waits on; plus the reachability steps (seed flags, gather) on its labels.
//
// Labels are 32-bit keys ((row << 16) | column) + 1, so the key order is the
// lexicographic order of (row, column) pairs, and 0 is null (below every
// pair).  Rows and columns must stay below 65535.  Label arrays are
// row-major [H][W]; background pixels hold 0 in both ping-pong buffers from
// initialization on and are never written again.
//
// Every kernel gives one wave to one mask word: lane l owns pixel 64*w + l of
// the row, reads the word once (the same address in every lane) and returns
// at once when the word has no pixel of the labelled set.
#include "kernels.h"

namespace vlg {
namespace {

#define PJ_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ PJ_GLOBAL T *gp(T *p) {
    return (PJ_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ const PJ_GLOBAL T *gp(const T *p) {
    return (const PJ_GLOBAL T *)p;
}

constexpr int kPjThreads = 256;
constexpr int kPjWaves = kPjThreads / 64;

// The word of operand r at (row, w), complement applied, padding bits 0;
// 0 outside the image.
__device__ __forceinline__ uint64_t pj_word(const Geo &g, const MRef &r, int row, int w) {
    if (row < 0 || row >= g.H || w < 0 || w >= g.wpr) return 0ull;
    const uint64_t v = (r.p ? gp(r.p)[(int64_t)row * g.wpr + w] : 0ull) ^ r.inv;
    return w == g.wpr - 1 ? (v & g.tail) : v;
}

__device__ __forceinline__ uint32_t pj_key(int row, int col) { return (((uint32_t)row << 16) | (uint32_t)col) + 1u; }
__device__ __forceinline__ int64_t pj_index(const Geo &g, uint32_t key) {
    const uint32_t k = key - 1u;
    return (int64_t)(k >> 16) * g.W + (k & 0xFFFFu);
}

// Largest key in the 3x3 neighbourhood of (row, col), that pixel included.
__device__ __forceinline__ uint32_t pj_max_around(const Geo &g, const uint32_t *__restrict__ lab_, int row, int col) {
    const PJ_GLOBAL uint32_t *lab = gp(lab_);
    uint32_t m = 0;
#pragma unroll
    for (int dr = -1; dr <= 1; dr++) {
        const int r = row + dr;
        if (r < 0 || r >= g.H) continue;
        const int64_t base = (int64_t)r * g.W;
#pragma unroll
        for (int dc = -1; dc <= 1; dc++) {
            const int c = col + dc;
            if (c < 0 || c >= g.W) continue;
            const uint32_t v = lab[base + c];
            m = v > m ? v : m;
        }
    }
    return m;
}

// Common prologue: this wave's row, word, pixel column and the word of the
// labelled set b.  Returns false for waves past the row's last word.
struct PjPos {
    int row, w, col;
    int64_t p;
    uint64_t bw;
    bool mine;  // this lane's pixel is in b
};
__device__ __forceinline__ bool pj_pos(const Geo &g, const MRef &b, PjPos &q) {
    q.row = (int)blockIdx.y;
    q.w = (int)blockIdx.x * kPjWaves + (int)(threadIdx.x >> 6);
    if (q.w >= g.wpr) return false;
    const int lane = (int)(threadIdx.x & 63);
    q.col = q.w * 64 + lane;
    q.p = (int64_t)q.row * g.W + q.col;
    q.bw = pj_word(g, b, q.row, q.w);
    q.mine = (q.bw >> lane) & 1ull;
    return true;
}

__global__ __launch_bounds__(kPjThreads) void k_pj_init(Geo g, MRef b, uint32_t *a_, uint32_t *b_) {
    PjPos q;
    if (!pj_pos(g, b, q) || q.col >= g.W) return;
    const uint32_t key = q.mine ? pj_key(q.row, q.col) : 0u;
    gp(a_)[q.p] = key;
    gp(b_)[q.p] = key;
}

// mainIteration: a pixel holding (i', j') takes the largest label around (i', j').
__global__ __launch_bounds__(kPjThreads) void k_pj_main(Geo g, MRef b, const uint32_t *__restrict__ in,
                                                      uint32_t *__restrict__ out) {
    PjPos q;
    if (!pj_pos(g, b, q) || q.bw == 0 || !q.mine) return;
    const uint32_t t = gp(in)[q.p] - 1u;
    gp(out)[q.p] = pj_max_around(g, in, (int)(t >> 16), (int)(t & 0xFFFFu));
}

// reconnect, first half: the output starts as a copy of the input labels.
__global__ __launch_bounds__(kPjThreads) void k_pj_copy(Geo g, MRef b, const uint32_t *__restrict__ in,
                                                      uint32_t *__restrict__ out) {
    PjPos q;
    if (!pj_pos(g, b, q) || q.bw == 0 || !q.mine) return;
    gp(out)[q.p] = gp(in)[q.p];
}

// reconnect, second half: the largest label around the pixel, when above the
// label stored at the pixel it points to, is written there by atomic
// maximum (several pixels may point to the same one).  Reads only `in`.
__global__ __launch_bounds__(kPjThreads) void k_pj_reconnect(Geo g, MRef b, const uint32_t *__restrict__ in,
                                                           uint32_t *out) {
    PjPos q;
    if (!pj_pos(g, b, q) || q.bw == 0 || !q.mine) return;
    const uint32_t t = gp(in)[q.p];
    const int64_t ti = pj_index(g, t);
    const uint32_t ab = pj_max_around(g, in, q.row, q.col), cd = gp(in)[ti];
    if (ab > cd) __hip_atomic_fetch_max(gp(out) + ti, ab, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Termination check: does any pixel of b have a neighbour of b with another
// label?  Each pair of neighbours is compared once (right, and the three
// below); a background neighbour holds 0 and is not compared.
__global__ __launch_bounds__(kPjThreads) void k_pj_check(Geo g, MRef b, const uint32_t *__restrict__ lab_,
                                                       uint32_t *term) {
    PjPos q;
    if (!pj_pos(g, b, q) || q.bw == 0) return;
    const PJ_GLOBAL uint32_t *lab = gp(lab_);
    bool bad = false;
    if (q.mine) {
        const uint32_t v = lab[q.p];
        auto differs = [&](int r, int c) {
            if (r >= g.H || c < 0 || c >= g.W) return false;
            const uint32_t u = lab[(int64_t)r * g.W + c];
            return u != 0u && u != v;
        };
        bad = differs(q.row, q.col + 1) || differs(q.row + 1, q.col - 1) || differs(q.row + 1, q.col) ||
              differs(q.row + 1, q.col + 1);
    }
    const uint64_t any = __ballot(bad);
    if (any && (threadIdx.x & 63) == (unsigned)__builtin_ctzll(any)) gp(term)[0] = 1u;
}

// Seeds of a reachability: flag the labels of the pixels of N(y & z) & b.
__global__ __launch_bounds__(kPjThreads) void k_pj_seed(Geo g, MRef b, MRef y, MRef z,
                                                      const uint32_t *__restrict__ lab, uint8_t *flag,
                                                      uint32_t bit) {
    PjPos q;
    if (!pj_pos(g, b, q) || q.bw == 0) return;
    uint64_t n = 0;
#pragma unroll
    for (int dr = -1; dr <= 1; dr++) {
        const int r = q.row + dr;
        const uint64_t c = pj_word(g, y, r, q.w) & pj_word(g, z, r, q.w);
        const uint64_t l = pj_word(g, y, r, q.w - 1) & pj_word(g, z, r, q.w - 1);
        const uint64_t h = pj_word(g, y, r, q.w + 1) & pj_word(g, z, r, q.w + 1);
        n |= c | (c << 1) | (c >> 1) | (l >> 63) | (h << 63);
    }
    if (!q.mine || !((n >> (threadIdx.x & 63)) & 1ull)) return;
    PJ_GLOBAL uint8_t *f = gp(flag) + pj_index(g, gp(lab)[q.p]);
    if (!(*f & bit)) *f = (uint8_t)(*f | bit);
}

// Another seed set on the same labelling: flag the labels of the pixels of
// the mask s (a subset of the labelled set, N(seeds) & b).
__global__ __launch_bounds__(kPjThreads) void k_pj_reseed(Geo g, MRef s, const uint32_t *__restrict__ lab,
                                                        uint8_t *flag, uint32_t bit) {
    PjPos q;
    if (!pj_pos(g, s, q) || q.bw == 0 || !q.mine) return;
    const uint32_t key = gp(lab)[q.p];
    if (key == 0u) return;
    PJ_GLOBAL uint8_t *f = gp(flag) + pj_index(g, key);
    if (!(*f & bit)) *f = (uint8_t)(*f | bit);
}

// out = (y & z) | (pixels of b whose label carries `bit`)
__global__ __launch_bounds__(kPjThreads) void k_pj_gather(Geo g, MRef b, MRef y, MRef z,
                                                        const uint32_t *__restrict__ lab,
                                                        const uint8_t *__restrict__ flag, uint32_t bit,
                                                        uint64_t *out) {
    PjPos q;
    if (!pj_pos(g, b, q)) return;
    bool in = false;
    if (q.mine) in = (gp(flag)[pj_index(g, gp(lab)[q.p])] & bit) != 0;
    const uint64_t zw = __ballot(in);
    if ((threadIdx.x & 63) == 0) {
        const uint64_t v = (pj_word(g, y, q.row, q.w) & pj_word(g, z, q.row, q.w)) | (q.bw & zw);
        gp(out)[(int64_t)q.row * g.wpr + q.w] = v;
    }
}

// Keys to row-major indices (y*W + x of the label's pixel), -1 for null.
__global__ __launch_bounds__(kPjThreads) void k_pj_labels(Geo g, const uint32_t *__restrict__ lab,
                                                        int32_t *__restrict__ labels) {
    const int64_t i = (int64_t)blockIdx.x * kPjThreads + threadIdx.x, n = (int64_t)g.H * g.W;
    if (i >= n) return;
    const uint32_t key = gp(lab)[i];
    gp(labels)[i] = key == 0u ? -1 : (int32_t)pj_index(g, key);
}

__global__ __launch_bounds__(kPjThreads) void k_pj_fill(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * kPjThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kPjThreads)
        gp(p)[i] = v;
}

int pj_blocks(int64_t n, int cap) {
    int64_t b = (n + kPjThreads - 1) / kPjThreads;
    return (int)(b < 1 ? 1 : b > cap ? cap : b);
}

dim3 pj_grid(const Geo &g) { return dim3((unsigned)((g.wpr + kPjWaves - 1) / kPjWaves), (unsigned)g.H); }

}  // namespace

bool pj_shape_ok(int H, int W) { return H < 65535 && W < 65535; }

hipError_t launch_pj_init(hipStream_t s, const Geo &g, MRef b, const PjWork &w) {
    if (g.nwords == 0) return hipSuccess;
    k_pj_init<<<pj_grid(g), kPjThreads, 0, s>>>(g, b, w.lab[0], w.lab[1]);
    return hipGetLastError();
}

hipError_t launch_pj_main(hipStream_t s, const Geo &g, MRef b, const PjWork &w, int from) {
    if (g.nwords == 0) return hipSuccess;
    k_pj_main<<<pj_grid(g), kPjThreads, 0, s>>>(g, b, w.lab[from], w.lab[1 - from]);
    return hipGetLastError();
}

hipError_t launch_pj_reconnect(hipStream_t s, const Geo &g, MRef b, const PjWork &w, int from) {
    if (g.nwords == 0) return hipSuccess;
    k_pj_copy<<<pj_grid(g), kPjThreads, 0, s>>>(g, b, w.lab[from], w.lab[1 - from]);
    k_pj_reconnect<<<pj_grid(g), kPjThreads, 0, s>>>(g, b, w.lab[from], w.lab[1 - from]);
    return hipGetLastError();
}

hipError_t launch_pj_check(hipStream_t s, const Geo &g, MRef b, const PjWork &w, int at) {
    if (g.nwords == 0) return hipSuccess;
    k_pj_fill<<<1, kPjThreads, 0, s>>>(w.term, 1, 0u);
    k_pj_check<<<pj_grid(g), kPjThreads, 0, s>>>(g, b, w.lab[at], w.term);
    return hipGetLastError();
}

hipError_t launch_pj_clear_flags(hipStream_t s, const Geo &g, const PjWork &w) {
    const int64_t n = ((int64_t)g.H * g.W + 3) / 4;
    if (n == 0) return hipSuccess;
    k_pj_fill<<<(unsigned)pj_blocks(n, 8192), kPjThreads, 0, s>>>((uint32_t *)w.flag, n, 0u);
    return hipGetLastError();
}

hipError_t launch_pj_seed(hipStream_t s, const Geo &g, MRef b, MRef y, MRef z, const PjWork &w, int at, int user) {
    if (g.nwords == 0) return hipSuccess;
    k_pj_seed<<<pj_grid(g), kPjThreads, 0, s>>>(g, b, y, z, w.lab[at], w.flag, 2u << user);
    return hipGetLastError();
}

hipError_t launch_pj_reseed(hipStream_t s, const Geo &g, MRef sm, const PjWork &w, int at, int user) {
    if (g.nwords == 0) return hipSuccess;
    k_pj_reseed<<<pj_grid(g), kPjThreads, 0, s>>>(g, sm, w.lab[at], w.flag, 2u << user);
    return hipGetLastError();
}

hipError_t launch_pj_gather(hipStream_t s, const Geo &g, MRef b, MRef y, MRef z, const PjWork &w, int at, int user,
                            uint64_t *out) {
    if (g.nwords == 0) return hipSuccess;
    k_pj_gather<<<pj_grid(g), kPjThreads, 0, s>>>(g, b, y, z, w.lab[at], w.flag, 2u << user, out);
    return hipGetLastError();
}

hipError_t launch_pj_labels(hipStream_t s, const Geo &g, const PjWork &w, int at, int32_t *labels) {
    const int64_t n = (int64_t)g.H * g.W;
    if (n == 0) return hipSuccess;
    k_pj_labels<<<(unsigned)((n + kPjThreads - 1) / kPjThreads), kPjThreads, 0, s>>>(g, w.lab[at], labels);
    return hipGetLastError();
}

}  // namespace vlg
