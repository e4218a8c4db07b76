// arith.hip -- arithmetic atoms (the tool's built-in arithmetic, Sect. 3): a
// pixel-wise comparison of two numeric expressions over the image's channel
// values, constants and percentile scalars, evaluated in float32.
//
// A wave evaluates four consecutive mask words: lane l takes pixel 64*w + l
// of each word w, so every channel load of a wave reads 64 consecutive
// elements.  The channels of a launch are loaded for all four pixels before
// any arithmetic, once for every program of the launch.  Programs are kernel
// arguments, the same for every lane: an instruction is fetched with scalar
// loads and decoded with uniform branches once for the lane's four pixels.
// The evaluation stack is registers addressed by the depth the host recorded
// for each instruction (a uniform switch), so nothing is shifted and no
// private memory is indexed.  No contraction into fused multiply-adds: each
// operation rounds once.
#include "kernels.h"

#include <cmath>

namespace vlg {
namespace {

#define AR_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ AR_GLOBAL T *ag(T *p) {
    return (AR_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ const AR_GLOBAL T *ag(const T *p) {
    return (const AR_GLOBAL T *)p;
}

constexpr int kArThreads = 256;
constexpr int kArWords = 4;  // mask words per wave

// op codes: ArOp of compiler.h
enum : uint8_t { KA_CONST = 0, KA_CHAN, KA_PCT, KA_NEG, KA_ABS, KA_ADD, KA_SUB, KA_MUL, KA_DIV, KA_MIN, KA_MAX };

// one value per pixel of the lane (a vector value, never memory)
typedef float Px __attribute__((ext_vector_type(kArWords)));
static_assert(kArWords == 4, "the pixel components are written out");

// a OP b (a the left operand), one rounding
template <int OP>
__device__ __forceinline__ float ar_op(float a, float b) {
#pragma clang fp contract(off)
    if constexpr (OP == KA_ADD) return a + b;
    else if constexpr (OP == KA_SUB) return a - b;
    else if constexpr (OP == KA_MUL) return a * b;
    else if constexpr (OP == KA_DIV) return a / b;
    else if constexpr (OP == KA_MIN) return b < a ? b : a;
    else return b > a ? b : a;  // KA_MAX
}

template <int OP>
__device__ __forceinline__ Px px_bin(const Px &x, const Px &y) {
    Px r;
    r.x = ar_op<OP>(x.x, y.x);
    r.y = ar_op<OP>(x.y, y.y);
    r.z = ar_op<OP>(x.z, y.z);
    r.w = ar_op<OP>(x.w, y.w);
    return r;
}

__device__ __forceinline__ Px px_un(const Px &x, bool neg) {
    Px r;
    r.x = neg ? -x.x : fabsf(x.x);
    r.y = neg ? -x.y : fabsf(x.y);
    r.z = neg ? -x.z : fabsf(x.z);
    r.w = neg ? -x.w : fabsf(x.w);
    return r;
}

// The evaluation stack and the channel values: named members holding whole
// vectors, never an array, so that no access can become an indexed
// (private-memory) one
struct Stk {
    Px e0, e1, e2, e3, e4, e5, e6, e7;
};
struct Chn {
    Px c0, c1, c2, c3, c4, c5, c6, c7;
};
static_assert(kArithDepth == 8 && kArithChans == 8, "the stack and channel members are written out");

// entry d of the stack = t
__device__ __forceinline__ void ar_push(Stk &s, int d, const Px &t) {
    switch (d) {
    case 0: s.e0 = t; break;
    case 1: s.e1 = t; break;
    case 2: s.e2 = t; break;
    case 3: s.e3 = t; break;
    case 4: s.e4 = t; break;
    case 5: s.e5 = t; break;
    case 6: s.e6 = t; break;
    default: s.e7 = t; break;
    }
}

// the binary operation on the top two entries of a stack of height d
template <int OP>
__device__ __forceinline__ void ar_bin(Stk &s, int d) {
    switch (d) {
    case 2: s.e0 = px_bin<OP>(s.e0, s.e1); break;
    case 3: s.e1 = px_bin<OP>(s.e1, s.e2); break;
    case 4: s.e2 = px_bin<OP>(s.e2, s.e3); break;
    case 5: s.e3 = px_bin<OP>(s.e3, s.e4); break;
    case 6: s.e4 = px_bin<OP>(s.e4, s.e5); break;
    case 7: s.e5 = px_bin<OP>(s.e5, s.e6); break;
    default: s.e6 = px_bin<OP>(s.e6, s.e7); break;
    }
}

// negation or absolute value of the top entry of a stack of height d
__device__ __forceinline__ void ar_un(Stk &s, int d, bool neg) {
    switch (d) {
    case 1: s.e0 = px_un(s.e0, neg); break;
    case 2: s.e1 = px_un(s.e1, neg); break;
    case 3: s.e2 = px_un(s.e2, neg); break;
    case 4: s.e3 = px_un(s.e3, neg); break;
    case 5: s.e4 = px_un(s.e4, neg); break;
    case 6: s.e5 = px_un(s.e5, neg); break;
    case 7: s.e6 = px_un(s.e6, neg); break;
    default: s.e7 = px_un(s.e7, neg); break;
    }
}

__device__ __forceinline__ Px ar_chan(const Chn &v, int c) {
    switch (c) {
    case 0: return v.c0;
    case 1: return v.c1;
    case 2: return v.c2;
    case 3: return v.c3;
    case 4: return v.c4;
    case 5: return v.c5;
    case 6: return v.c6;
    default: return v.c7;
    }
}

// One side of a program, ins[k0, k1), for the lane's four pixels.
__device__ __forceinline__ Px ar_side(const ArithGroup &a, int k0, int k1, const Chn &v,
                                      const float *__restrict__ pct) {
    const Px zero = {0.f, 0.f, 0.f, 0.f};
    Stk s{zero, zero, zero, zero, zero, zero, zero, zero};
    for (int k = k0; k < k1; k++) {
        const ArithIns in = a.ins[k];
        const int d = in.depth;
        switch (in.op) {
        case KA_CONST: {
            const Px t = {in.c, in.c, in.c, in.c};
            ar_push(s, d, t);
            break;
        }
        case KA_CHAN: ar_push(s, d, ar_chan(v, in.idx)); break;
        case KA_PCT: {
            const float x = ag(pct)[in.idx];
            const Px t = {x, x, x, x};
            ar_push(s, d, t);
            break;
        }
        case KA_NEG: ar_un(s, d, true); break;
        case KA_ABS: ar_un(s, d, false); break;
        case KA_ADD: ar_bin<KA_ADD>(s, d); break;
        case KA_SUB: ar_bin<KA_SUB>(s, d); break;
        case KA_MUL: ar_bin<KA_MUL>(s, d); break;
        case KA_DIV: ar_bin<KA_DIV>(s, d); break;
        case KA_MIN: ar_bin<KA_MIN>(s, d); break;
        default: ar_bin<KA_MAX>(s, d); break;
        }
    }
    return s.e0;
}

// the lane's four pixels of channel position c (0 beyond nch)
template <typename T>
__device__ __forceinline__ Px ar_load(const T *__restrict__ img, const ArithGroup &a, int c, int64_t chan_elems,
                                      const int64_t (&e)[kArWords]) {
    Px x = {0.f, 0.f, 0.f, 0.f};
    if (c < a.nch) {
        const AR_GLOBAL T *p = ag(img) + (int64_t)a.ch[c] * chan_elems;
        x.x = (float)p[e[0]];
        x.y = (float)p[e[1]];
        x.z = (float)p[e[2]];
        x.w = (float)p[e[3]];
    }
    return x;
}

__device__ __forceinline__ uint32_t ar_fdiv(uint32_t n, uint32_t mul, uint32_t shift) {
    return (uint32_t)(((uint64_t)__umulhi(n, mul) + n) >> shift);
}

template <typename T>
__global__ __launch_bounds__(kArThreads) void k_arith(Geo g, const T *__restrict__ img, int64_t chan_elems,
                                                      ArithGroup a, const float *__restrict__ pct) {
    const int64_t w0 = ((int64_t)blockIdx.x * (kArThreads / 64) + (threadIdx.x >> 6)) * kArWords;
    if (w0 >= g.nwords) return;
    const int lane = (int)(threadIdx.x & 63);
    // channel element of pixel 64*w + lane of word w: rows are 64*wpr elements
    // apart (the pitch), so the element index is 64*w + lane; a word past the
    // end reads word w0 again and is not stored
    int64_t e[kArWords];
#pragma unroll
    for (int j = 0; j < kArWords; j++) e[j] = (w0 + j < g.nwords ? w0 + j : w0) * 64 + lane;
    const Chn v{ar_load(img, a, 0, chan_elems, e), ar_load(img, a, 1, chan_elems, e),
                ar_load(img, a, 2, chan_elems, e), ar_load(img, a, 3, chan_elems, e),
                ar_load(img, a, 4, chan_elems, e), ar_load(img, a, 5, chan_elems, e),
                ar_load(img, a, 6, chan_elems, e), ar_load(img, a, 7, chan_elems, e)};
    // lane j stores word w0 + j of every program
    const int64_t wi = w0 + (lane < kArWords ? lane : 0);
    const bool store = lane < kArWords && wi < g.nwords;
    uint64_t keep = ~0ull;
    if (store) {
        const uint32_t row = ar_fdiv((uint32_t)wi, g.wpr_mul, g.wpr_shift);
        if ((uint32_t)wi - row * (uint32_t)g.wpr == (uint32_t)g.wpr - 1) keep = g.tail;
    }
    for (int p = 0; p < a.n; p++) {
        const Px l = ar_side(a, a.lhs[p], a.rhs[p], v, pct), r = ar_side(a, a.rhs[p], a.end[p], v, pct);
        const int cmp = a.cmp[p];
        uint64_t mine = 0;
#pragma unroll
        for (int j = 0; j < kArWords; j++) {
            const float x = j == 0 ? l.x : j == 1 ? l.y : j == 2 ? l.z : l.w;
            const float y = j == 0 ? r.x : j == 1 ? r.y : j == 2 ? r.z : r.w;
            const bool b = cmp == 0 ? x > y : cmp == 1 ? x < y : cmp == 2 ? x >= y : x <= y;
            const uint64_t word = __ballot(b);
            if (lane == j) mine = word;
        }
        if (store) ag(a.out[p])[wi] = mine & keep;
    }
}

// The programs of a launch keep to the limits of ArithGroup, and each side's
// recorded depths are those its instructions reach.
bool arith_group_ok(const ArithGroup &a, const float *pct) {
    if (a.n < 1 || a.n > kArithGroupProgs || a.nch < 0 || a.nch > kArithChans) return false;
    for (int p = 0; p < a.n; p++) {
        if (!(0 <= a.lhs[p] && a.lhs[p] < a.rhs[p] && a.rhs[p] < a.end[p] && a.end[p] <= kArithGroupIns)) return false;
        if (a.end[p] - a.lhs[p] > kArithMax || a.cmp[p] < 0 || a.cmp[p] > 3 || !a.out[p]) return false;
        for (int side = 0; side < 2; side++) {
            const int k0 = side ? a.rhs[p] : a.lhs[p], k1 = side ? a.end[p] : a.rhs[p];
            int h = 0;
            for (int k = k0; k < k1; k++) {
                const ArithIns &in = a.ins[k];
                if (in.depth != h) return false;
                if (in.op <= KA_PCT) {
                    if (h >= kArithDepth) return false;
                    if (in.op == KA_CHAN && (in.idx < 0 || in.idx >= a.nch)) return false;
                    if (in.op == KA_PCT && (in.idx < 0 || !pct)) return false;
                    h++;
                } else if (in.op <= KA_ABS) {
                    if (h < 1) return false;
                } else if (in.op <= KA_MAX) {
                    if (h < 2) return false;
                    h--;
                } else {
                    return false;
                }
            }
            if (h != 1) return false;
        }
    }
    return true;
}

}  // namespace

hipError_t launch_arith(hipStream_t s, const Geo &g, const void *img, int64_t chan_elems, int dtype,
                        const ArithGroup &a, const float *pct) {
    if (g.nwords == 0) return hipSuccess;
    if (!arith_group_ok(a, pct)) return hipErrorInvalidValue;
    const int64_t per_block = (int64_t)(kArThreads / 64) * kArWords;
    const int64_t blocks = (g.nwords + per_block - 1) / per_block;
    if (dtype == 1)
        k_arith<uint8_t><<<(unsigned)blocks, kArThreads, 0, s>>>(g, (const uint8_t *)img, chan_elems, a, pct);
    else if (dtype == 2)
        k_arith<uint16_t><<<(unsigned)blocks, kArThreads, 0, s>>>(g, (const uint16_t *)img, chan_elems, a, pct);
    else
        k_arith<float><<<(unsigned)blocks, kArThreads, 0, s>>>(g, (const float *)img, chan_elems, a, pct);
    return hipGetLastError();
}

}  // namespace vlg
