// kernels.h -- host-side launchers of the HIP kernels (gfx950, wave64).
//
// All masks are 1-bit-packed: row-major uint64 words, wpr = ceil(W/64) per
// row, pixel (y, x) = bit x%64 of word y*wpr + x/64, bits x >= W kept zero.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace vlg {

// Operand: a packed mask, optionally complemented.  p == nullptr stands for
// the all-zero mask (all-one when complemented).
struct MRef {
    const uint64_t *p;
    uint64_t inv;  // 0 or ~0
};

struct Geo {
    int32_t H, W, wpr;
    uint64_t tail;     // valid-bit mask of the last word of a row
    int64_t nwords;    // H * wpr
    int32_t BH, BW;    // 2x2 block grid: ceil(H/2) x ceil(W/2)
    uint32_t wpr_mul;  // fast division by wpr (see fastdiv in kernels.hip)
    uint32_t wpr_shift;
};

Geo make_geo(int H, int W);

// near works on bands of rows 64 words wide.  For one image the band height
// grows with the image (4 .. 32 rows) while at least 2048 bands remain to
// fill the chip; a batch always has bands enough and uses kBatchNearRows.
__host__ __device__ inline int near_band_rows(const Geo &g) {
    const int64_t rows = (int64_t)g.H * ((g.wpr + 63) / 64);
    int R = 4;
    while (R < 32 && rows / (2 * R) >= 2048) R *= 2;
    return R;
}
constexpr int kBatchNearRows = 8;
inline bool valid_near_rows(int r) { return r == 4 || r == 8 || r == 16 || r == 32; }
constexpr int kBatchGridDefault = 8192;
inline bool valid_batch_grid(int n) { return n == 1024 || n == 2048 || n == 4096 || n == 8192; }
__host__ __device__ inline int64_t near_tasks(const Geo &g, int R) {
    return (int64_t)((g.H + R - 1) / R) * ((g.wpr + 63) / 64);
}
__host__ __device__ inline int64_t near_tasks(const Geo &g) { return near_tasks(g, near_band_rows(g)); }

// Tile geometry of the reachability labelling: TBH x 64 blocks per tile
// (2*TBH pixel rows x 128 pixel columns); TBH is tunable (8, 16 or 32).
constexpr int kTileBW = 64;
constexpr int kTileBHDefault = 16;
inline bool valid_tile_bh(int t) { return t == 8 || t == 16 || t == 32; }
inline int64_t tile_count(int H, int W, int tbh) {
    const int64_t bh = (H + 1) / 2, bw = (W + 1) / 2;
    return ((bh + tbh - 1) / tbh) * ((bw + kTileBW - 1) / kTileBW);
}
// Untuned tile height for a labelling of `tiles(t)` tiles at height t: the
// tallest that still leaves kMinTiles tiles (about four per compute unit;
// taller tiles leave fewer borders to merge), else the shortest.
constexpr int64_t kMinTiles = 1024;
template <typename Tiles>
inline int default_tile_bh(Tiles tiles) {
    for (int t : {32, 16})
        if (tiles(t) >= kMinTiles) return t;
    return 8;
}

// Every loop of the labelling kernels (union-find walks, hooks, retries) runs
// at most `cap` iterations per walk.  A walk that reaches the cap stops, leaves
// the arrays in a state every later pass can still read (all stored values are
// valid block ids), and sets *status to a non-zero value; the host turns that
// into VLG_ENOCONV.  A correct labelling never comes near the default cap.
constexpr int kLoopCapDefault = 1 << 20;
struct LoopGuard {
    unsigned int *status;  // device word, set to 1 when a loop gives up
    int cap;               // iterations per walk (>= 1)
};

struct CclWork {
    int32_t *glab;       // [BH*BW] parent pointers (block ids, row-major)
    uint8_t *gflag;      // [BH*BW] local roots: bit0 touches the tile border,
                         // bit 1+u meets the seeds of labelling user u
    unsigned long long *counters; // [2] merge unions, merge retries (may be null)
    int tbh = kTileBHDefault;     // block rows per labelling tile
    LoopGuard guard{nullptr, kLoopCapDefault};
};

constexpr int kMaxAtomsPerLaunch = 32;

struct AtomLaunch {
    int n;
    uint8_t cmp[kMaxAtomsPerLaunch];
    float thr[kMaxAtomsPerLaunch];
    const float *thr_dev[kMaxAtomsPerLaunch];  // device scalar (percentile) or null
    uint64_t *out[kMaxAtomsPerLaunch];
};

hipError_t launch_logic(hipStream_t s, const Geo &g, MRef x, MRef y, int op, int inv_out, uint64_t *out);
// out = (N(x) ^ inv_out) OP z with OP = and (zop 0) or or (zop 1)
// rows: band height (4, 8, 16 or 32; 0 = near_band_rows(g))
hipError_t launch_near(hipStream_t s, const Geo &g, MRef x, int inv_out, MRef z, int zop, uint64_t *out,
                       int rows = 0);
hipError_t launch_atoms(hipStream_t s, const Geo &g, const void *chan, int dtype, const AtomLaunch &a);
hipError_t launch_ccl_local(hipStream_t s, const Geo &g, MRef b, MRef y, MRef z, const CclWork &w);
hipError_t launch_ccl_merge(hipStream_t s, const Geo &g, MRef b, const CclWork &w);
hipError_t launch_ccl_flag(hipStream_t s, const Geo &g, const CclWork &w);
hipError_t launch_ccl_gather(hipStream_t s, const Geo &g, MRef b, MRef y, MRef z, const CclWork &w,
                             int user, uint64_t *out);
hipError_t launch_ccl_reseed(hipStream_t s, const Geo &g, MRef sm, const CclWork &w, int user);

// Several independent labellings of one image in each launch (blockIdx.y =
// labelling): each with its own passable mask b, seeds y & z, workspace
// (glab, gflag) and, for the gather, its user bit and output.
constexpr int kMaxMulti = 8;
struct CclMulti {
    int n;
    MRef b[kMaxMulti], y[kMaxMulti], z[kMaxMulti];
    int32_t *glab[kMaxMulti];
    uint8_t *gflag[kMaxMulti];
    int user[kMaxMulti];
    uint64_t *out[kMaxMulti];
};
// w supplies the tile height, loop guard and counters (its arrays are unused)
hipError_t launch_ccl_local_multi(hipStream_t s, const Geo &g, const CclMulti &m, const CclWork &w);
hipError_t launch_ccl_merge_multi(hipStream_t s, const Geo &g, const CclMulti &m, const CclWork &w);
hipError_t launch_ccl_flag_multi(hipStream_t s, const Geo &g, const CclMulti &m, const CclWork &w);
hipError_t launch_ccl_gather_multi(hipStream_t s, const Geo &g, const CclMulti &m);

constexpr int kBatchMax = 16;
struct LogicOp {
    MRef x, y;
    uint64_t inv_out;
    uint64_t *out;
    int op;
};
struct LogicBatch {
    int n;
    LogicOp ops[kBatchMax];
};
struct NearOp {
    MRef x, z;
    uint64_t inv_out;
    uint64_t *out;
    int zop;
};
struct NearBatch {
    int n;
    NearOp ops[kBatchMax];
};
hipError_t launch_logic_batch(hipStream_t s, const Geo &g, const LogicBatch &b);
hipError_t launch_near_batch(hipStream_t s, const Geo &g, const NearBatch &b, int rows = 0);
// canon: [BH*BW] int32 scratch
hipError_t launch_ccl_labels(hipStream_t s, const Geo &g, MRef b, const CclWork &w, int32_t *canon,
                             int32_t *labels);
hipError_t launch_unpack(hipStream_t s, const Geo &g, const uint64_t *mask, uint8_t *out);

// Arithmetic atoms (arith.hip): postfix programs over channel values,
// constants and percentile scalars, evaluated per pixel in float32 (one
// rounding per operation).  Program p of a launch is ins[lhs[p], rhs[p]) (the
// left side) and ins[rhs[p], end[p]) (the right side); out[p] = lhs CMP rhs
// (cmp[p]: 0 >, 1 <, 2 >=, 3 <=).  Op codes as ArOp in compiler.h.  depth is
// the height of the side's evaluation stack before the instruction (at most
// 8 after it).  Every program of a launch reads its channels from one set of
// at most kArithChans distinct channels, loaded once per pixel for all of
// them; outputs are written in program order.
constexpr int kArithMax = 32;        // instructions per program (both sides)
constexpr int kArithGroupIns = 96;   // instructions of all programs of a launch
constexpr int kArithGroupProgs = 8;  // programs per launch
constexpr int kArithDepth = 8;       // evaluation stack per side
struct ArithIns {
    uint8_t op;
    uint8_t depth;
    uint8_t pad[2];
    int32_t idx;  // position in ArithGroup::ch (AR_CHAN) or percentile scalar (AR_PCT)
    float c;      // AR_CONST
};
constexpr int kArithChans = 8;  // distinct channels the programs of a launch may read
struct ArithGroup {
    int32_t n, nch;
    int32_t ch[kArithChans];  // the distinct channels read (AR_CHAN idx = position here)
    int32_t lhs[kArithGroupProgs], rhs[kArithGroupProgs], end[kArithGroupProgs], cmp[kArithGroupProgs];
    uint64_t *out[kArithGroupProgs];
    ArithIns ins[kArithGroupIns];
};
// img: channel 0 of the image; chan_elems: elements per channel (H * pitch).
// Rejects (hipErrorInvalidValue) a group whose programs break the limits above.
hipError_t launch_arith(hipStream_t s, const Geo &g, const void *img, int64_t chan_elems, int dtype,
                        const ArithGroup &a, const float *pct);

// Volumes (vol.hip): D slices of S rows; the Geo is that of the D*S-row mask.
// N over the 26-neighbourhood: out = (N(x) ^ inv_out) OP z (zop 0 and, 1 or).
hipError_t launch_near3(hipStream_t s, const Geo &g, int S, int D, MRef x, int inv_out, MRef z, int zop,
                        uint64_t *out);
// 26-connected labelling of b over blocks of 2 x 2 x 2 voxels: P[k] = the
// root block (the smallest block id) of block k's component, -1 for a block
// without voxels of b; P has vl_nblocks entries, at most g.BH * g.BW (the
// block count of the D*S-row mask).
int64_t vl_nblocks(const Geo &g, int S, int D);
hipError_t launch_vl_label(hipStream_t s, const Geo &g, int S, int D, MRef b, int *P, const LoopGuard &gd);
// labels[v] (voxel index (z*S + y)*W + x) = the smallest voxel of v's
// component, -1 for background, from a labelling P; canon: vl_nblocks ints.
hipError_t launch_vl_labels(hipStream_t s, const Geo &g, int S, int D, MRef b, const int *P, int *canon,
                            int *labels);
// flag: one byte per block
hipError_t launch_vl_clear_flags(hipStream_t s, const Geo &g, int S, int D, uint8_t *flag);
hipError_t launch_vl_seed(hipStream_t s, const Geo &g, int S, int D, MRef b, MRef y, MRef z, const int *P,
                          uint8_t *flag, int user);
hipError_t launch_vl_reseed(hipStream_t s, const Geo &g, int S, int D, MRef sm, const int *P, uint8_t *flag,
                            int user);
hipError_t launch_vl_gather(hipStream_t s, const Geo &g, int S, int D, MRef b, MRef y, MRef z, const int *P,
                            const uint8_t *flag, int user, uint64_t *out);

// The paper's labelling (Sect. 3, Alg. CCL), pj.hip.  lab[0], lab[1]: the
// ping-pong label arrays [H][W] (keys ((row << 16) | column) + 1, 0 = null);
// flag: [H][W] seed bytes indexed by a label's pixel (bit 1+u: the seeds of
// labelling user u); term: the termination check's word (non-zero: some
// pixel has a neighbour with another label).  `from` / `at` select the
// label array a step reads.
struct PjWork {
    uint32_t *lab[2];
    uint8_t *flag;
    uint32_t *term;
};
bool pj_shape_ok(int H, int W);  // rows and columns below 65535
inline size_t pj_bytes(const Geo &g) {
    const size_t n = (size_t)g.H * g.W;
    return 2 * ((n * 4 + 255) & ~(size_t)255) + ((n + 255) & ~(size_t)255) + 256;
}
inline PjWork pj_work(void *base, const Geo &g) {
    const size_t n = (size_t)g.H * g.W, l = (n * 4 + 255) & ~(size_t)255;
    PjWork w;
    w.lab[0] = (uint32_t *)base;
    w.lab[1] = (uint32_t *)((char *)base + l);
    w.flag = (uint8_t *)((char *)base + 2 * l);
    w.term = (uint32_t *)((char *)base + 2 * l + ((n + 255) & ~(size_t)255));
    return w;
}
hipError_t launch_pj_init(hipStream_t s, const Geo &g, MRef b, const PjWork &w);
hipError_t launch_pj_main(hipStream_t s, const Geo &g, MRef b, const PjWork &w, int from);
hipError_t launch_pj_reconnect(hipStream_t s, const Geo &g, MRef b, const PjWork &w, int from);
hipError_t launch_pj_check(hipStream_t s, const Geo &g, MRef b, const PjWork &w, int at);
hipError_t launch_pj_clear_flags(hipStream_t s, const Geo &g, const PjWork &w);
hipError_t launch_pj_seed(hipStream_t s, const Geo &g, MRef b, MRef y, MRef z, const PjWork &w, int at, int user);
hipError_t launch_pj_reseed(hipStream_t s, const Geo &g, MRef sm, const PjWork &w, int at, int user);
hipError_t launch_pj_gather(hipStream_t s, const Geo &g, MRef b, MRef y, MRef z, const PjWork &w, int at, int user,
                            uint64_t *out);
hipError_t launch_pj_labels(hipStream_t s, const Geo &g, const PjWork &w, int at, int32_t *labels);

// ------------------------------------------------------------------ segments
// A segment: consecutive Boolean and near steps of the fused schedule run by
// one kernel.  A workgroup takes a tile of TR rows x TW words of the image,
// extended by `halo` rows above and below and one word left and right, and
// keeps every mask of the segment for that extended tile in LDS registers:
// operands from outside the segment are loaded once, results that are read
// later are stored once, and everything else never leaves LDS.  After d near
// steps along a path a register is exact except in its d outermost rows (and
// the outermost d bits of the two halo words), so with halo >= the deepest
// near chain the tile itself is exact.
constexpr int kSegMaxIns = 64;
constexpr int kSegMaxRegs = 16;
constexpr int kSegMaxPtrs = 32;
constexpr uint8_t kSegNone = 255;  // operand "no register": the all-zero mask
enum SegOpcode : uint8_t { SEG_LOAD = 0, SEG_AND, SEG_OR, SEG_NEAR_AND, SEG_NEAR_OR, SEG_STORE };
struct SegIns {
    uint8_t op;
    uint8_t dst;  // register; SEG_STORE: pointer index
    uint8_t a;    // register (kSegNone: zero mask); SEG_LOAD: pointer index
    uint8_t b;    // register or kSegNone
    uint8_t inv;  // bit0 complements a, bit1 complements b, bit2 complements the
                  // Boolean result (logic) or N(a) (near, before its epilogue)
};
// LOAD    dst = ptr[a]
// AND/OR  dst = ((a ^ ia) OP (b ^ ib)) ^ io
// NEAR_*  dst = (N(a ^ ia) ^ io) OP (b ^ ib)     (OP = and / or)
// STORE   ptr[dst] = a ^ ia over the tile (padding bits cleared)
// The leading LOADs of a program are issued together.
struct SegProg {
    int32_t nins, nregs, halo;
    SegIns ins[kSegMaxIns];
    uint64_t *ptr[kSegMaxPtrs];
};
// Tile shape of a segment on an image: TR rows x TW words.
struct SegTile {
    int tr, tw;
    size_t lds_bytes;
};
SegTile seg_tile(const Geo &g, int halo, int nregs);
hipError_t launch_segment(hipStream_t s, const Geo &g, const SegProg &p);
hipError_t launch_fill_i64(hipStream_t s, unsigned long long *p, int n, unsigned long long v);
// bytes (a multiple of width) copied in width-byte units (8 or 16)
hipError_t launch_stream_copy(hipStream_t s, void *dst, const void *src, int64_t bytes, int width);


// ------------------------------------------------------------------ batches
// One launch per schedule step for a whole batch of images of different
// sizes.  Every image has a descriptor in device memory; a kernel walks a
// global unit space (the concatenation of every image's units, by a prefix
// array per unit kind) with a persistent grid.
struct BImg {
    Geo g;
    const char *img;        // channel 0
    int64_t chan_bytes;     // bytes per channel
    char *ws;               // this image's workspace: mask slots, labelling, percentiles
    uint64_t mask_bytes;    // slot stride
    uint64_t off_glab, off_gflag, off_pct, off_pctst;
    uint64_t *const *outs;  // packed output buffer per external slot
    const uint32_t *ranks;  // percentile rank per percentile slot
};

// A mask operand of a batched step: slot id (>= 0 workspace slot, <= -2
// external output, -1 none) and complement flag, resolved per image.
struct BRef {
    int32_t slot;
    uint32_t inv;
};

enum BatchKind { BK_WORDS = 0, BK_LOGIC, BK_NEAR, BK_TILES, BK_MERGE, BK_BLOCKS, BK_FLAG, BK_GATHER, BK_PCTH, BK_ONE, BK_COUNT };

struct BatchArgs {
    int n;
    int dtype;                // image pixel type (all images of a batch share it)
    int grid_cap;             // most workgroups of a persistent launch (host side)
    const BImg *imgs;
    const int64_t *prefix;    // [n+1] units of the launch's kind, prefix sums
    LoopGuard guard;          // loop cap and give-up flag of the labelling kernels
};

struct BAtoms {
    int chan, n;
    uint8_t cmp[kMaxAtomsPerLaunch];
    float thr[kMaxAtomsPerLaunch];
    int32_t pct[kMaxAtomsPerLaunch];  // percentile slot or -1
    int32_t out[kMaxAtomsPerLaunch];
};
struct BLogicOp {
    BRef x, y;
    int32_t op, inv_out, out;
};
struct BLogic {
    int n;
    BLogicOp ops[kBatchMax];
};
struct BNearOp {
    BRef x, z;
    int32_t inv_out, zop, out;
};
struct BNear {
    int n;
    BNearOp ops[kBatchMax];
};

// units of each kind for one image (host side)
int64_t batch_units(const Geo &g, int kind, int tbh);

hipError_t launch_b_atoms(hipStream_t s, const BatchArgs &a, int64_t total, const BAtoms &op);
hipError_t launch_b_logic(hipStream_t s, const BatchArgs &a, int64_t total, const BLogic &op);
hipError_t launch_b_near(hipStream_t s, const BatchArgs &a, int64_t total, const BNear &op);
hipError_t launch_b_ccl_local(hipStream_t s, const BatchArgs &a, int64_t total, int tbh, BRef b, BRef y, BRef z);
hipError_t launch_b_ccl_merge(hipStream_t s, const BatchArgs &a, int64_t total, int tbh, BRef b);
hipError_t launch_b_ccl_flag(hipStream_t s, const BatchArgs &a, int64_t total);
hipError_t launch_b_ccl_gather(hipStream_t s, const BatchArgs &a, int64_t total, BRef b, BRef y, BRef z, int user,
                               int32_t out);
hipError_t launch_b_ccl_reseed(hipStream_t s, const BatchArgs &a, int64_t total, BRef sm, int user);
// up to kMaxPctSel quantiles of one channel: rank k[j] (single image; a batch
// takes each image's ranks from its descriptor) into percentile slot slot[j]
constexpr int kMaxPctSel = 4;
struct PctSel {
    int n;
    int32_t slot[kMaxPctSel];
    uint32_t k[kMaxPctSel];
};
hipError_t launch_b_percentile(hipStream_t s, const BatchArgs &one, int64_t total_one, const BatchArgs &hist,
                               int64_t total_hist, int chan, const PctSel &sel);
}  // namespace vlg

namespace vlg {
// Percentiles (k-th smallest value of a channel, nearest rank) by radix
// select over order-preserving uint32 keys, several ranks of one channel per
// pass over it.  Slot p has kPctStateBytes of device state at
// states + p * kPctStateBytes; its value is written to results[p].
constexpr size_t kPctStateBytes = 41216;
hipError_t launch_percentile(hipStream_t s, const Geo &g, const void *chan, int dtype, const PctSel &sel,
                             void *states, float *results);
}  // namespace vlg
