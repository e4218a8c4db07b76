// capi.cpp -- the C ABI (include/vlg.h): contexts, resident images, formula
// compilation, and the executor that runs a schedule on a HIP stream, either
// launch by launch or as a captured hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "compiler.h"
#include "arith_jit.h"
#include "kernels.h"
#include "vlg.h"

using namespace vlg;

static_assert(kMaxPctSel == kMaxPctPerStep, "percentile selections per step");
static_assert(kMaxCclLanes <= kMaxMulti, "a region's labellings fit one multi-launch");

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return fail(VLG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// The fixed device array behind vlg_ccl_labels_noalloc: labelling scratch for
// callers that cannot allocate.  Each GPU holds its own copy from the moment
// the library's code object is loaded on it until the process ends.  In host
// code `scratch` names a host-side stand-in, never the device memory: kernels
// and copies get the device address that hipGetSymbolAddress returns for the
// current device (noalloc_scratch).
constexpr size_t kNoallocScratchBytes = 40ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_dev;  // device -> address of its `scratch`

// Device address of `scratch` on `device`, which must be current.  Looked up
// once per device (vlg_create does it at set-up) and cached.
int noalloc_scratch(int device, void **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_dev.find(device);
    if (it != g_scratch_dev.end()) {
        *out = it->second;
        return VLG_OK;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(VLG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_dev[device] = p;
    *out = p;
    return VLG_OK;
}

}  // namespace

std::atomic<uint64_t> g_serial{1};

struct vlg_formula {
    uint64_t serial = g_serial.fetch_add(1);
    Dag dag;
    int32_t max_chan = -1;
    std::mutex mu;
    std::map<std::pair<std::vector<int>, int>, std::unique_ptr<Plan>> plans;

    // lanes: concurrent labelling lanes of the fused schedule (1: sequential);
    // fuse: segment halo cap of the fused schedule (1: no segments)
    const Plan &plan(const std::vector<int> &which, Mode m, int lanes = 1, int fuse = 1) {
        std::lock_guard<std::mutex> lk(mu);
        auto key = std::make_pair(which, ((int)m * 16 + lanes) * 64 + fuse);
        auto it = plans.find(key);
        if (it != plans.end()) return *it->second;
        auto p = std::make_unique<Plan>(build_plan(dag, which, m, lanes, m == Mode::Fused ? fuse : 1));
        const Plan &ref = *p;
        plans.emplace(key, std::move(p));
        return ref;
    }
};

struct vlg_image {
    int device;
    int dtype, C, H, W;   // H: rows of all slices together
    int D = 1, S = 0;     // a volume: D slices of S rows (S = H / D); an image: D = 1
    int64_t pitch;  // elements per row (wpr * 64)
    void *dev;      // from the device's stream-ordered pool (hipMallocAsync)
    size_t bytes;
    size_t esize() const { return dtype == VLG_U8 ? 1 : dtype == VLG_U16 ? 2 : 4; }
    const char *chan(int c) const { return (const char *)dev + (size_t)c * H * pitch * esize(); }
    // the last enqueued use of the image on each stream that read it: its
    // release waits for these events instead of for the whole device
    mutable std::mutex mu;
    mutable std::vector<std::pair<hipStream_t, hipEvent_t>> uses;
    int note_use(hipStream_t s) const {
        std::lock_guard<std::mutex> lk(mu);
        hipEvent_t ev = nullptr;
        for (auto &u : uses)
            if (u.first == s) ev = u.second;
        if (!ev) {
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return VLG_EHIP;
            uses.emplace_back(s, ev);
        }
        return hipEventRecord(ev, s) == hipSuccess ? VLG_OK : VLG_EHIP;
    }
};

namespace {
// One stream per device (created on first use, kept until the process ends)
// on which images are released once every stream that read them is done.
std::mutex g_release_mu;
std::map<int, hipStream_t> g_release_stream;
hipStream_t release_stream(int device) {
    std::lock_guard<std::mutex> lk(g_release_mu);
    auto it = g_release_stream.find(device);
    if (it != g_release_stream.end()) return it->second;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    g_release_stream[device] = s;
    return s;
}
}  // namespace

struct GraphKey {
    std::vector<uintptr_t> v;
    bool operator<(const GraphKey &o) const { return v < o.v; }
};

// Tunables (VLG_TUNE_*): a value of 0 means "not set" (default rule).
constexpr int kNumTunables = 8;
const char *const kTunableNames[kNumTunables] = {"ccl_tile_rows", "near_band_rows", "batch_grid",   "ccl_lanes",
                                                 "fuse_halo",     "ccl_algo",       "pj_reconnect", "arith_kernel"};
constexpr int kPjReconnectDefault = 16;

bool tunable_valid(int which, int v) {
    switch (which) {
    case VLG_TUNE_CCL_TILE_ROWS: return valid_tile_bh(v);
    case VLG_TUNE_NEAR_ROWS: return valid_near_rows(v);
    case VLG_TUNE_BATCH_GRID: return valid_batch_grid(v);
    case VLG_TUNE_CCL_LANES: return v == 1 || v == 2 || v == 4 || v == 8;
    case VLG_TUNE_FUSE_HALO: return valid_fuse_halo(v);
    case VLG_TUNE_CCL_ALGO: return v == VLG_CCL_UNION_FIND || v == VLG_CCL_POINTER_JUMPING;
    case VLG_TUNE_PJ_RECONNECT: return v >= 1 && v <= 64;
    case VLG_TUNE_ARITH: return v == VLG_ARITH_INTERPRETER || v == VLG_ARITH_COMPILED;
    }
    return false;
}

struct Tuning {
    int v[kNumTunables] = {};
};

struct vlg_ctx {
    int device = 0;
    std::string arch;
    Tuning forced;                                  // 0 entries: not forced
    std::map<std::pair<int, int>, Tuning> tuned;    // shape class -> tuning
    std::map<std::pair<int, int>, Tuning> tuned_batch;  // (batch class, mean image class) -> tuning
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int mode = VLG_MODE_GRAPH;
    int loop_cap = kLoopCapDefault;  // iterations per labelling walk (vlg_set_loop_cap)
    void *ws = nullptr;
    size_t ws_size = 0;
    bool ws_external = false;       // workspace lent by a server slot
    // device [4]: merge unions, merge retries, then the 32-bit give-up flag of
    // the labelling loops (status) and padding
    unsigned long long *counters = nullptr;
    unsigned int *status_host = nullptr;     // pinned staging of the flag
    unsigned int *status() const { return (unsigned int *)(counters + 2); }
    LoopGuard guard() const { return LoopGuard{status(), loop_cap}; }
    bool count_ccl = false;         // collect merge counters (VLG_CCL_COUNTERS=1)
    // pointer-jumping labellings since the counters were last read: main
    // iterations, rounds (reconnect + termination check), kernel launches
    int64_t pj_iters = 0, pj_rounds = 0, pj_launches = 0, pj_labellings = 0;
    std::map<GraphKey, hipGraphExec_t> graphs;
    // pinned host staging of batch descriptors; `desc_done` marks the end of
    // the last upload from it
    void *desc_host = nullptr;
    size_t desc_host_size = 0;
    hipEvent_t desc_done = nullptr;

    // an executable graph may still be running from an earlier launch: wait
    // for the stream (its parallel branches join into it) before destroying
    void drop_graphs() {
        if (graphs.empty()) return;
        (void)hipStreamSynchronize(stream);
        for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }
};

namespace {

// Read and clear the give-up flag of the labelling loops; waits for the
// context's stream.  VLG_ENOCONV when a loop stopped at its iteration cap in
// work enqueued since the last check.
int check_status(vlg_ctx *c) {
    HIP_TRY(hipMemcpyAsync(c->status_host, c->status(), sizeof(unsigned int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (*c->status_host) {
        *c->status_host = 0;
        HIP_TRY(launch_fill_i64(c->stream, c->counters + 2, 1, 0));
        HIP_TRY(hipStreamSynchronize(c->stream));
        return fail(VLG_ENOCONV, "a labelling loop stopped at its iteration cap (" + std::to_string(c->loop_cap) +
                                     "): the results of the work since the last synchronisation are not valid");
    }
    return VLG_OK;
}


// Workspace layout of one evaluation.
struct Layout {
    size_t mask_bytes = 0;
    size_t off_slots = 0, off_stage = 0, off_u8 = 0, off_glab = 0, off_gflag = 0, off_pct = 0,
           off_pctst = 0, total = 0;
    size_t lane_bytes = 0;  // labelling workspace of lane l at off_glab / off_gflag + l * lane_bytes
    bool pj = false;        // pointer-jumping labelling: its arrays (pj_work) start at off_glab
    bool vol = false;       // volume labelling: voxel parents (4 B) then flag bytes at off_glab
};

// the block parents of a volume labelling (vl_nblocks <= g.BH * g.BW)
size_t vol_label_bytes(const Geo &g) { return align256((size_t)g.BH * g.BW * 4); }

Layout layout_for(const Plan &P, const Geo &g, bool stage_packed, bool stage_u8, bool pj = false,
                  bool vol = false) {
    Layout L;
    L.mask_bytes = align256((size_t)g.nwords * 8);
    size_t off = 0;
    L.off_slots = off;
    off += (size_t)P.nslots * L.mask_bytes;
    L.off_stage = off;
    if (stage_packed) off += (size_t)P.noutputs * L.mask_bytes;
    L.off_u8 = off;
    if (stage_u8) off += (size_t)P.noutputs * align256((size_t)g.H * g.W);
    L.off_glab = off;
    const size_t nb = (size_t)g.BH * g.BW;
    L.pj = pj && !vol;
    L.vol = vol;
    L.lane_bytes = P.ccl_count == 0 ? 0
                   : vol          ? vol_label_bytes(g) + align256((size_t)g.BH * g.BW)
                   : L.pj         ? align256(pj_bytes(g))
                                  : align256(nb * 4) + align256(nb);
    L.off_gflag = off + (P.ccl_count > 0 ? align256(nb * 4) : 0);
    off += (size_t)std::max(P.ccl_lanes, 1) * L.lane_bytes;
    L.off_pct = off;
    off += align256((size_t)P.npct * 4);
    L.off_pctst = off;
    off += (size_t)P.npct * kPctStateBytes;
    L.total = off + 256;
    return L;
}

int ensure_ws(vlg_ctx *c, size_t need) {
    if (c->ws_size >= need) return VLG_OK;
    if (c->ws_external) return fail(VLG_ENOMEM, "admitted workspace smaller than the evaluation needs");
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->drop_graphs();
    const size_t sz = std::max(need, c->ws_size + c->ws_size / 4);
    if (c->ws) HIP_TRY(hipFree(c->ws));
    c->ws = nullptr;
    c->ws_size = 0;
    if (hipMalloc(&c->ws, sz) != hipSuccess) {
        (void)hipGetLastError();
        c->ws = nullptr;
        return fail(VLG_ENOMEM, "workspace allocation of " + std::to_string(sz) + " bytes failed");
    }
    c->ws_size = sz;
    return VLG_OK;
}

int log2_class(int n) {
    int c = 0;
    while ((1ll << c) < (long long)n) c++;
    return c;
}

// The value of a tunable for an image of H x W: forced, else the shape
// class's tuned value, else the default (0 for the near band height: chosen
// from the image size by the launcher).
int tuned_value(const vlg_ctx *c, int which, int H, int W) {
    if (c->forced.v[which]) return c->forced.v[which];
    auto it = c->tuned.find({log2_class(H), log2_class(W)});
    if (it != c->tuned.end() && it->second.v[which]) return it->second.v[which];
    switch (which) {
    case VLG_TUNE_CCL_TILE_ROWS: return default_tile_bh([&](int t) { return tile_count(H, W, t); });
    case VLG_TUNE_BATCH_GRID: return kBatchGridDefault;
    case VLG_TUNE_CCL_LANES: return 1;
    case VLG_TUNE_FUSE_HALO: return kFuseHaloDefault;
    case VLG_TUNE_ARITH: return VLG_ARITH_COMPILED;
    }
    return 0;
}

struct TuningShim {
    int ccl_tbh;
};
TuningShim tuning_for(const vlg_ctx *c, int H, int W) { return {tuned_value(c, VLG_TUNE_CCL_TILE_ROWS, H, W)}; }

// (ceil(log2 n), ceil(log2 mean pixels per image)) of a batch
std::pair<int, int> batch_class(int n, int64_t pixels) {
    return {log2_class(n), log2_class((int)std::min<int64_t>(pixels / std::max(n, 1), 1 << 30))};
}

// The value of a tunable for a batch: forced, else the batch class's tuned
// value, else `fallback`.
int batch_value(const vlg_ctx *c, int which, int n, int64_t pixels, int fallback) {
    if (c->forced.v[which]) return c->forced.v[which];
    auto it = c->tuned_batch.find(batch_class(n, pixels));
    if (it != c->tuned_batch.end() && it->second.v[which]) return it->second.v[which];
    return fallback;
}

uint32_t pct_rank(double q, int64_t n) {
    // k = clamp(ceil(q * n) - 1, 0, n - 1)
    double kk = std::ceil(q * (double)n) - 1.0;
    if (kk < 0.0 || n == 0) return 0;
    if (kk > (double)(n - 1)) return (uint32_t)(n - 1);
    return (uint32_t)kk;
}

const char *kind_name(SK k) {
    switch (k) {
    case SK::Pct: return "percentile";
    case SK::Atoms: return "atoms";
    case SK::Logic: return "logic";
    case SK::Near: return "near";
    case SK::CclLocal: return "ccl_local";
    case SK::CclMerge: return "ccl_merge";
    case SK::CclFlag: return "ccl_flag";
    case SK::CclGather: return "ccl_gather";
    case SK::CclReseed: return "ccl_reseed";
    case SK::Segment: return "segment";
    case SK::Arith: return "arith";
    }
    return "?";
}

// Bytes a step must move at the least: its image channel or input masks
// read once, its outputs written once (and the labelling arrays it owns).
double algorithmic_bytes(const Plan &P, const Step &s, const Geo &g, int dtype, int tbh) {
    const double mb = (double)g.nwords * 8.0, npix = (double)g.H * g.W;
    const double nb = (double)g.BH * g.BW;
    auto ins = [&](std::initializer_list<Ref> rs) {
        double n = 0;
        for (const Ref &r : rs) n += r.slot != kNone ? mb : 0.0;
        return n;
    };
    switch (s.kind) {
    case SK::Pct: return npix * (dtype == VLG_U8 ? 1.0 : dtype == VLG_U16 ? 2.0 * 2.0 : 3.0 * 4.0);  // per pass
    case SK::Atoms: return npix * (dtype == VLG_U8 ? 1.0 : dtype == VLG_U16 ? 2.0 : 4.0) + s.natoms * mb;
    case SK::Logic: return ins({s.x, s.y}) + mb;
    case SK::Near: return ins({s.x, s.z}) + mb;
    case SK::CclLocal: return ins({s.x, s.y, s.z}) + nb * 5.0;      // labels + flags written
    case SK::CclMerge: {
        const double ntiles = std::ceil(g.BH / (double)tbh) * std::ceil(g.BW / (double)kTileBW);
        return ntiles * (kTileBW + 2 * tbh) * 16.0;                   // border words read
    }
    case SK::CclFlag: return nb;                                      // flags read
    case SK::CclGather: return ins({s.x, s.y, s.z}) + nb * 4.0 + mb;  // labels read
    case SK::CclReseed: return ins({s.x});                            // seed mask read
    case SK::Arith: {
        // every channel the program reads, once, and the mask; in a group
        // (one launch) only the channels no earlier member reads
        std::vector<int32_t> seen, ch;
        const size_t si = (size_t)(&s - P.steps.data());
        for (size_t k = si; s.group >= 0 && si < P.steps.size() && k-- > 0 && P.steps[k].group == s.group;)
            for (const ArInstr &in : P.ariths[(size_t)P.steps[k].arith].ins)
                if (in.op == AR_CHAN) seen.push_back(in.chan);
        for (const ArInstr &in : P.ariths[(size_t)s.arith].ins)
            if (in.op == AR_CHAN && std::find(ch.begin(), ch.end(), in.chan) == ch.end() &&
                std::find(seen.begin(), seen.end(), in.chan) == seen.end())
                ch.push_back(in.chan);
        return npix * (dtype == VLG_U8 ? 1.0 : dtype == VLG_U16 ? 2.0 : 4.0) * (double)ch.size() + mb;
    }
    case SK::Segment: {                                               // loads + stores
        const Segment &S = P.segments[(size_t)s.seg];
        return (double)(S.inputs.size() + S.outputs.size()) * mb;
    }
    }
    return 0.0;
}

// The labelling schedule of reach-type nodes for an image of H x W
// (VLG_TUNE_CCL_ALGO; default union-find).
int ccl_algo(const vlg_ctx *c, int H, int W) {
    const int v = tuned_value(c, VLG_TUNE_CCL_ALGO, H, W);
    return v == VLG_CCL_POINTER_JUMPING ? v : VLG_CCL_UNION_FIND;
}

int pj_reconnect_every(const vlg_ctx *c, int H, int W) {
    const int v = tuned_value(c, VLG_TUNE_PJ_RECONNECT, H, W);
    return v >= 1 ? v : kPjReconnectDefault;
}

// The paper's labelling of b (Sect. 3, Alg. CCL): initialization, then
// rounds of k main iterations, one reconnect and the termination check, the
// host waiting for the check's word after every round as the paper's tool
// does.  On return the labels are in w.lab[at].  VLG_ENOCONV when the check
// still fails after the context's loop cap of rounds.
int pj_label(vlg_ctx *c, hipStream_t s, const Geo &g, MRef b, const PjWork &w, int k, int &at) {
    HIP_TRY(launch_pj_init(s, g, b, w));
    at = 0;
    int64_t launches = 1;
    for (int64_t round = 0;; round++) {
        if (round >= c->loop_cap)
            return fail(VLG_ENOCONV, "pointer-jumping labelling: the termination check still fails after " +
                                         std::to_string(round) + " rounds (the loop cap)");
        for (int it = 0; it < k; it++) {
            HIP_TRY(launch_pj_main(s, g, b, w, at));
            at ^= 1;
        }
        HIP_TRY(launch_pj_reconnect(s, g, b, w, at));
        at ^= 1;
        HIP_TRY(launch_pj_check(s, g, b, w, at));
        launches += k + 4;
        c->pj_iters += k;
        c->pj_rounds++;
        HIP_TRY(hipMemcpyAsync(c->status_host + 1, w.term, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (c->status_host[1] == 0) break;
    }
    c->pj_launches += launches;
    c->pj_labellings++;
    return VLG_OK;
}

// The kernel form of the Arith steps si..sj (one group, or one step): their
// programs, with the stack height before each instruction, and the distinct
// channels they read.  out[] is left to the caller.  Programs beyond the
// kernel's limits leave the group empty (n = 0), which the launcher rejects.
static_assert(kArGroupProgs == kArithGroupProgs && kArGroupInstrs == kArithGroupIns && kArGroupChans == kArithChans &&
                  kArMaxInstrs == kArithMax && kArMaxDepth == kArithDepth,
              "the scheduler's arithmetic groups fit the kernel's");
ArithGroup arith_group(const Plan &P, size_t si, size_t sj) {
    ArithGroup a;
    std::memset(&a, 0, sizeof a);
    bool bad = sj - si + 1 > (size_t)kArithGroupProgs;
    int k = 0;
    for (size_t t = si; t <= sj && !bad; t++) {
        const Step &s = P.steps[t];
        const ArProgram &pr = P.ariths[(size_t)s.arith];
        const int p = (int)(t - si);
        if (k + (int)pr.ins.size() > kArithGroupIns) {
            bad = true;
            break;
        }
        a.lhs[p] = k;
        a.rhs[p] = k + pr.lhs_len;
        a.end[p] = k + (int)pr.ins.size();
        a.cmp[p] = s.op;
        int h = 0;  // stack height of the side being written
        for (size_t i = 0; i < pr.ins.size() && !bad; i++, k++) {
            if ((int)i == pr.lhs_len) h = 0;
            ArithIns &in = a.ins[k];
            in.op = pr.ins[i].op;
            in.c = pr.ins[i].c;
            in.depth = (uint8_t)std::min(h, 255);
            if (in.op == AR_PCT) {
                in.idx = pr.ins[i].pct;
            } else if (in.op == AR_CHAN) {
                // position of the channel among the distinct channels read
                int c = 0;
                while (c < a.nch && a.ch[c] != pr.ins[i].chan) c++;
                if (c == a.nch) {
                    if (a.nch == kArithChans) bad = true;
                    else a.ch[a.nch++] = pr.ins[i].chan;
                }
                in.idx = c;
            }
            h += in.op <= AR_PCT ? 1 : in.op <= AR_ABS ? 0 : -1;
        }
        a.n = p + 1;
    }
    if (bad) a.n = 0;
    return a;
}

// Launch the Arith group `a` with the kernel VLG_TUNE_ARITH selects for an
// image of H x W: its compiled kernel (compiled on first use; see
// prepare_arith), or the interpreter when that is selected or the group
// does not compile.
hipError_t arith_launch(const vlg_ctx *c, hipStream_t s, const Geo &g, int H, int W, const void *img,
                        int64_t chan_elems, int dtype, const ArithGroup &a, const float *pct) {
    if (a.n >= 1 && tuned_value(c, VLG_TUNE_ARITH, H, W) != VLG_ARITH_INTERPRETER) {
        if (hipFunction_t fn = arith_jit_function(c->device, a, dtype, nullptr))
            return launch_arith_jit(fn, s, g, img, chan_elems, a, pct);
    }
    return launch_arith(s, g, img, chan_elems, dtype, a, pct);
}

// Compile the Arith groups of P before anything is captured (compiling loads
// a module, which stream capture must not see).
void prepare_arith(const vlg_ctx *c, const Plan &P, int H, int W, int dtype) {
    if (tuned_value(c, VLG_TUNE_ARITH, H, W) == VLG_ARITH_INTERPRETER) return;
    for (size_t si = 0; si < P.steps.size(); si++) {
        if (P.steps[si].kind != SK::Arith) continue;
        size_t sj = si;
        while (P.steps[si].group >= 0 && sj + 1 < P.steps.size() && P.steps[sj + 1].group == P.steps[si].group) sj++;
        const ArithGroup a = arith_group(P, si, sj);
        if (a.n >= 1) (void)arith_jit_function(c->device, a, dtype, nullptr);
        si = sj;
    }
}

using StepHook = void (*)(void *, size_t, bool);

// Enqueue every step of P on the stream.  ext[k] is the packed device buffer
// of external slot k.  hook (optional) runs before and after each step.
// base_ (optional) is the workspace to use instead of the context's.
// [first, last) (optional) restricts the steps enqueued.
int enqueue_plan(vlg_ctx *c, const Plan &P, const vlg_image *img, const Layout &L,
                 const std::vector<uint64_t *> &ext, StepHook hook = nullptr, void *hook_ctx = nullptr,
                 char *base_ = nullptr, size_t first = 0, size_t last = SIZE_MAX) {
    const Geo g = make_geo(img->H, img->W);
    char *base = base_ ? base_ : (char *)c->ws;
    auto slot_ptr = [&](int32_t s) -> uint64_t * {
        if (s == kNone) return nullptr;
        if (is_ext(s)) return ext[(size_t)ext_index(s)];
        return (uint64_t *)(base + L.off_slots + (size_t)s * L.mask_bytes);
    };
    auto mref = [&](const Ref &r) {
        MRef m;
        m.p = slot_ptr(r.slot);
        m.inv = r.inv ? ~0ull : 0ull;
        return m;
    };
    float *pct = (float *)(base + L.off_pct);
    CclWork w0;
    w0.counters = c->count_ccl ? c->counters : nullptr;
    w0.guard = c->guard();
    w0.tbh = tuning_for(c, img->H, img->W).ccl_tbh;
    const int near_rows = tuned_value(c, VLG_TUNE_NEAR_ROWS, img->H, img->W);
    const int64_t npix = (int64_t)img->H * img->W;
    // pointer-jumping labellings (L.pj): the label array the current
    // labelling's steps read
    const int pj_k = pj_reconnect_every(c, img->H, img->W);
    int pj_at = 0;
    // volumes: N over 26 neighbours, voxel labelling (L.vol)
    const bool vol = img->D > 1;
    const int vS = img->S, vD = img->D;
    // The labellings of a concurrent region (steps of one span with lanes,
    // each lane with its own labelling workspace) run on the context's
    // stream: the union-find phases of all lanes go into one launch each
    // (blockIdx.y = lane), the other steps launch one by one, every lane's
    // steps in their order.  Pointer-jumping and volume labellings run the
    // region's steps in plan order.
    auto lane_work = [&](int lane) {
        CclWork w = w0;
        w.glab = (int32_t *)(base + L.off_glab + (size_t)lane * L.lane_bytes);
        w.gflag = (uint8_t *)(base + L.off_gflag + (size_t)lane * L.lane_bytes);
        return w;
    };
    auto run_region = [&](size_t r0, size_t r1) -> int {
        std::vector<std::vector<size_t>> q((size_t)kMaxCclLanes);
        for (size_t k = r0; k < r1; k++) q[(size_t)P.steps[k].lane].push_back(k);
        std::vector<size_t> head(q.size(), 0);
        // one level per iteration: each lane's next step as it stood at the
        // iteration's start, so the lanes' phases line up
        for (;;) {
            bool any = false;
            const std::vector<size_t> at = head;
            for (SK kind : {SK::CclLocal, SK::CclMerge, SK::CclFlag, SK::CclGather}) {
                CclMulti m;
                std::memset(&m, 0, sizeof m);
                for (size_t l = 0; l < q.size(); l++) {
                    if (at[l] >= q[l].size() || head[l] != at[l] || P.steps[q[l][at[l]]].kind != kind) continue;
                    const Step &t = P.steps[q[l][head[l]++]];
                    const CclWork lw = lane_work((int)l);
                    m.b[m.n] = mref(t.x);
                    m.y[m.n] = mref(t.y);
                    m.z[m.n] = mref(t.z);
                    m.glab[m.n] = lw.glab;
                    m.gflag[m.n] = lw.gflag;
                    m.user[m.n] = t.user;
                    m.out[m.n] = slot_ptr(t.out);
                    m.n++;
                }
                if (m.n == 0) continue;
                any = true;
                hipError_t e = kind == SK::CclLocal   ? launch_ccl_local_multi(c->stream, g, m, w0)
                               : kind == SK::CclMerge ? launch_ccl_merge_multi(c->stream, g, m, w0)
                               : kind == SK::CclFlag  ? launch_ccl_flag_multi(c->stream, g, m, w0)
                                                      : launch_ccl_gather_multi(c->stream, g, m);
                if (e != hipSuccess) return fail(VLG_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
            }
            for (size_t l = 0; l < q.size(); l++) {
                if (at[l] >= q[l].size() || head[l] != at[l]) continue;
                const Step &t = P.steps[q[l][head[l]]];
                hipError_t e = hipSuccess;
                if (t.kind == SK::Logic)
                    e = launch_logic(c->stream, g, mref(t.x), mref(t.y), t.op, t.inv_out, slot_ptr(t.out));
                else if (t.kind == SK::Near)
                    e = launch_near(c->stream, g, mref(t.x), t.inv_out, mref(t.z), t.op, slot_ptr(t.out), near_rows);
                else if (t.kind == SK::CclReseed)
                    e = launch_ccl_reseed(c->stream, g, mref(t.x), lane_work((int)l), t.user);
                else
                    continue;  // a labelling phase: next round
                head[l]++;
                any = true;
                if (e != hipSuccess) return fail(VLG_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
            }
            if (!any) break;
        }
        for (size_t l = 0; l < q.size(); l++)
            if (head[l] < q[l].size()) return fail(VLG_EINVAL, "internal: a region step of an unexpected kind");
        return VLG_OK;
    };
    for (size_t si = first; si < P.steps.size() && si < last; si++) {
        const Step &s = P.steps[si];
        if (s.lane >= 0 && !L.pj && !vol && !hook) {
            size_t sj = si;
            while (sj < P.steps.size() && sj < last && P.steps[sj].span == s.span && P.steps[sj].lane >= 0) sj++;
            const int rc = run_region(si, sj);
            if (rc != VLG_OK) return rc;
            si = sj - 1;
            continue;
        }
        const int lane = s.lane > 0 ? s.lane : 0;
        hipStream_t stream = c->stream;
        CclWork w = lane_work(lane);
        const PjWork pw = pj_work(base + L.off_glab + (size_t)lane * L.lane_bytes, g);
        int *vP = (int *)(base + L.off_glab + (size_t)lane * L.lane_bytes);
        uint8_t *vflag = (uint8_t *)vP + vol_label_bytes(g);
        if (hook) hook(hook_ctx, si, true);
        hipError_t e = hipSuccess;
        if (s.group >= 0) {
            // a batched group: consecutive Logic (or Near) steps, one launch
            size_t sj = si;
            while (sj + 1 < P.steps.size() && sj + 1 < last && P.steps[sj + 1].group == s.group) sj++;
            if (s.kind == SK::Arith) {
                ArithGroup a = arith_group(P, si, sj);
                for (size_t k = si; k <= sj && k - si < (size_t)kArithGroupProgs; k++)
                    a.out[k - si] = slot_ptr(P.steps[k].out);
                e = arith_launch(c, stream, g, img->H, img->W, img->dev, (int64_t)img->H * img->pitch, img->dtype, a,
                                 pct);
            } else if (s.kind == SK::Logic) {
                LogicBatch b;
                b.n = (int)(sj - si + 1);
                for (size_t k = si; k <= sj; k++) {
                    const Step &t = P.steps[k];
                    b.ops[k - si] = LogicOp{mref(t.x), mref(t.y), t.inv_out ? ~0ull : 0ull, slot_ptr(t.out), t.op};
                }
                e = launch_logic_batch(stream, g, b);
            } else if (vol) {
                for (size_t k = si; k <= sj && e == hipSuccess; k++) {
                    const Step &t = P.steps[k];
                    e = launch_near3(stream, g, vS, vD, mref(t.x), t.inv_out, mref(t.z), t.op, slot_ptr(t.out));
                }
            } else {
                NearBatch b;
                b.n = (int)(sj - si + 1);
                for (size_t k = si; k <= sj; k++) {
                    const Step &t = P.steps[k];
                    b.ops[k - si] = NearOp{mref(t.x), mref(t.z), t.inv_out ? ~0ull : 0ull, slot_ptr(t.out), t.op};
                }
                e = launch_near_batch(stream, g, b, near_rows);
            }
            if (e != hipSuccess) return fail(VLG_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
            for (size_t k = si; k < sj; k++) {
                // the group is timed as a whole: attribute it to its last step
                if (hook) hook(hook_ctx, k, false);
                if (hook) hook(hook_ctx, k + 1, true);
            }
            if (hook) hook(hook_ctx, sj, false);
            si = sj;
            continue;
        }
        switch (s.kind) {
        case SK::Pct:
        {
            PctSel sel;
            std::memset(&sel, 0, sizeof sel);
            sel.n = s.npq;
            for (int j = 0; j < s.npq; j++) {
                sel.slot[j] = s.pct_out[j];
                sel.k[j] = pct_rank(s.q[j], npix);
            }
            e = launch_percentile(stream, g, img->chan(s.chan), img->dtype, sel, base + L.off_pctst, pct);
        }
            break;
        case SK::Atoms: {
            AtomLaunch a;
            std::memset(&a, 0, sizeof a);
            a.n = s.natoms;
            for (int j = 0; j < s.natoms; j++) {
                a.cmp[j] = s.atoms[j].cmp;
                a.thr[j] = s.atoms[j].thr;
                a.thr_dev[j] = s.atoms[j].use_pct ? pct + s.atoms[j].pct : nullptr;
                a.out[j] = slot_ptr(s.atoms[j].out);
            }
            e = launch_atoms(stream, g, img->chan(s.chan), img->dtype, a);
            break;
        }
        case SK::Logic:
            e = launch_logic(stream, g, mref(s.x), mref(s.y), s.op, s.inv_out, slot_ptr(s.out));
            break;
        case SK::Arith: {
            ArithGroup a = arith_group(P, si, si);
            a.out[0] = slot_ptr(s.out);
            e = arith_launch(c, stream, g, img->H, img->W, img->dev, (int64_t)img->H * img->pitch, img->dtype, a, pct);
            break;
        }
        case SK::Near:
            if (vol)
                e = launch_near3(stream, g, vS, vD, mref(s.x), s.inv_out, mref(s.z), s.op, slot_ptr(s.out));
            else
                e = launch_near(stream, g, mref(s.x), s.inv_out, mref(s.z), s.op, slot_ptr(s.out), near_rows);
            break;
        case SK::CclLocal:
            if (L.vol) {
                // the whole voxel labelling, then the seeds
                e = launch_vl_label(stream, g, vS, vD, mref(s.x), vP, w.guard);
                if (e == hipSuccess) e = launch_vl_clear_flags(stream, g, vS, vD, vflag);
                if (e == hipSuccess) e = launch_vl_seed(stream, g, vS, vD, mref(s.x), mref(s.y), mref(s.z), vP, vflag, 0);
            } else if (L.pj) {
                // the whole labelling (host-waited rounds), then the seeds
                const int rc = pj_label(c, stream, g, mref(s.x), pw, pj_k, pj_at);
                if (rc != VLG_OK) return rc;
                e = launch_pj_clear_flags(stream, g, pw);
                if (e == hipSuccess) e = launch_pj_seed(stream, g, mref(s.x), mref(s.y), mref(s.z), pw, pj_at, 0);
            } else {
                e = launch_ccl_local(stream, g, mref(s.x), mref(s.y), mref(s.z), w);
            }
            break;
        case SK::CclMerge:  // the pointer-jumping and voxel labellings have no merge or flag pass
            if (!L.pj && !L.vol) e = launch_ccl_merge(stream, g, mref(s.x), w);
            break;
        case SK::CclFlag:
            if (!L.pj && !L.vol) e = launch_ccl_flag(stream, g, w);
            break;
        case SK::CclGather:
            if (L.vol)
                e = launch_vl_gather(stream, g, vS, vD, mref(s.x), mref(s.y), mref(s.z), vP, vflag, s.user,
                                     slot_ptr(s.out));
            else if (L.pj)
                e = launch_pj_gather(stream, g, mref(s.x), mref(s.y), mref(s.z), pw, pj_at, s.user, slot_ptr(s.out));
            else
                e = launch_ccl_gather(stream, g, mref(s.x), mref(s.y), mref(s.z), w, s.user, slot_ptr(s.out));
            break;
        case SK::CclReseed:
            if (L.vol)
                e = launch_vl_reseed(stream, g, vS, vD, mref(s.x), vP, vflag, s.user);
            else if (L.pj)
                e = launch_pj_reseed(stream, g, mref(s.x), pw, pj_at, s.user);
            else
                e = launch_ccl_reseed(stream, g, mref(s.x), w, s.user);
            break;
        case SK::Segment: {
            if (vol) return fail(VLG_EINVAL, "internal: no fused segments on volumes");
            const Segment &S = P.segments[(size_t)s.seg];
            SegProg sp;
            std::memset(&sp, 0, sizeof sp);
            const size_t ni = S.inputs.size();
            if (S.ins.size() > (size_t)kSegMaxIns || ni + S.outputs.size() > (size_t)kSegMaxPtrs ||
                S.nregs > kSegMaxRegs)
                return fail(VLG_EINVAL, "internal: segment exceeds the kernel's program limits");
            sp.nins = (int32_t)S.ins.size();
            sp.nregs = S.nregs;
            sp.halo = S.halo;
            for (size_t k = 0; k < S.ins.size(); k++) {
                const SegInstr &q = S.ins[k];
                sp.ins[k] = SegIns{q.op, q.dst, q.a, q.b, q.inv};
                if (q.op == SOP_STORE) sp.ins[k].dst = (uint8_t)(ni + q.dst);
            }
            for (size_t k = 0; k < ni; k++) sp.ptr[k] = slot_ptr(S.inputs[k]);
            for (size_t k = 0; k < S.outputs.size(); k++) sp.ptr[ni + k] = slot_ptr(S.outputs[k]);
            e = launch_segment(stream, g, sp);
            break;
        }
        }
        if (e != hipSuccess) return fail(VLG_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
        if (hook) hook(hook_ctx, si, false);
    }
    return VLG_OK;
}

// Evaluate the outputs `which` of f on img.  outs[k] receives output which[k].
int run(vlg_ctx *c, vlg_formula *f, const vlg_image *img, const std::vector<int> &which,
        const std::vector<void *> &outs, int fmt, int where) {
    if (fmt != VLG_PACKED64 && fmt != VLG_U8MASK) return fail(VLG_EINVAL, "bad mask format");
    if (where != VLG_HOST && where != VLG_DEVICE) return fail(VLG_EINVAL, "bad memory kind");
    if (f->max_chan >= img->C)
        return fail(VLG_ESHAPE, "formula uses channel " + std::to_string(f->max_chan) + " but the image has " +
                                    std::to_string(img->C));
    if (img->device != c->device) return fail(VLG_EINVAL, "image lives on another device");
    DeviceGuard dg(c->device);
    const Mode m = c->mode == VLG_MODE_PEROP ? Mode::PerOp : Mode::Fused;
    const bool vol = img->D > 1;  // volumes: no fused segments, voxel labelling
    const Plan &P = f->plan(which, m, m == Mode::Fused ? tuned_value(c, VLG_TUNE_CCL_LANES, img->H, img->W) : 1,
                            vol ? 1 : tuned_value(c, VLG_TUNE_FUSE_HALO, img->H, img->W));
    const Geo g = make_geo(img->H, img->W);
    if (g.nwords == 0 || which.empty()) return VLG_OK;
    const bool direct = fmt == VLG_PACKED64 && where == VLG_DEVICE;
    const bool stage_u8 = fmt == VLG_U8MASK && where == VLG_HOST;
    // the pointer-jumping labelling waits on the host between its rounds, so
    // a formula that labels with it is never captured as a graph
    const bool pj = !vol && P.ccl_count > 0 && ccl_algo(c, img->H, img->W) == VLG_CCL_POINTER_JUMPING;
    if (pj && !pj_shape_ok(img->H, img->W))
        return fail(VLG_ESHAPE, "pointer-jumping labelling: rows and columns must stay below 65535");
    Layout L = layout_for(P, g, !direct, stage_u8, pj, vol);
    int rc = ensure_ws(c, L.total);
    if (rc != VLG_OK) return rc;
    char *base = (char *)c->ws;
    std::vector<uint64_t *> ext(which.size());
    for (size_t k = 0; k < which.size(); k++)
        ext[k] = direct && outs[k] ? (uint64_t *)outs[k]
                                   : (uint64_t *)(base + L.off_stage + k * L.mask_bytes);
    const size_t u8_bytes = align256((size_t)g.H * g.W);

    auto enqueue_all = [&]() -> int {
        int r = enqueue_plan(c, P, img, L, ext);
        if (r != VLG_OK) return r;
        if (fmt == VLG_U8MASK) {
            for (size_t k = 0; k < which.size(); k++) {
                if (!outs[k]) continue;
                uint8_t *dst = where == VLG_DEVICE ? (uint8_t *)outs[k] : (uint8_t *)(base + L.off_u8 + k * u8_bytes);
                hipError_t e = launch_unpack(c->stream, g, ext[k], dst);
                if (e != hipSuccess) return fail(VLG_EHIP, hipGetErrorString(e));
            }
        }
        return VLG_OK;
    };

    prepare_arith(c, P, img->H, img->W, img->dtype);
    if (c->mode == VLG_MODE_GRAPH && !pj) {
        GraphKey key;
        key.v = {(uintptr_t)f->serial, (uintptr_t)&P, (uintptr_t)img->dev, (uintptr_t)img->H, (uintptr_t)img->W,
                 (uintptr_t)img->dtype, (uintptr_t)fmt, (uintptr_t)where, (uintptr_t)c->ws,
                 (uintptr_t)tuning_for(c, img->H, img->W).ccl_tbh,
                 (uintptr_t)tuned_value(c, VLG_TUNE_NEAR_ROWS, img->H, img->W), (uintptr_t)c->loop_cap,
                 (uintptr_t)img->D, (uintptr_t)tuned_value(c, VLG_TUNE_ARITH, img->H, img->W)};
        for (size_t k = 0; k < which.size(); k++) key.v.push_back((uintptr_t)outs[k]);
        auto it = c->graphs.find(key);
        if (it == c->graphs.end()) {
            HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            int r = enqueue_all();
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(c->stream, &graph);
            if (r != VLG_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return r;
            }
            if (e != hipSuccess) return fail(VLG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
            hipGraphExec_t exec = nullptr;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return fail(VLG_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
            if (c->graphs.size() >= 64) c->drop_graphs();
            it = c->graphs.emplace(key, exec).first;
        }
        HIP_TRY(hipGraphLaunch(it->second, c->stream));
    } else {
        rc = enqueue_all();
        if (rc != VLG_OK) return rc;
    }
    if (img->note_use(c->stream) != VLG_OK) return fail(VLG_EHIP, "event record failed");

    if (where == VLG_HOST) {
        for (size_t k = 0; k < which.size(); k++) {
            if (!outs[k]) continue;
            if (fmt == VLG_PACKED64)
                HIP_TRY(hipMemcpyAsync(outs[k], ext[k], (size_t)g.nwords * 8, hipMemcpyDeviceToHost, c->stream));
            else
                HIP_TRY(hipMemcpyAsync(outs[k], base + L.off_u8 + k * u8_bytes, (size_t)g.H * g.W,
                                       hipMemcpyDeviceToHost, c->stream));
        }
        return check_status(c);
    }
    return VLG_OK;
}

// ------------------------------------------------------------------ batches
// Evaluate every output of f on n images of one pixel type with one launch
// per schedule step: each image gets its own workspace region (mask slots,
// labelling arrays, percentile state) and a descriptor; the batch kernels
// walk the concatenated units of all images.  Descriptors, output tables,
// percentile ranks and unit prefix sums are uploaded before the steps run.
// hook (optional): called around every launch of a step or group (before:
// its first step, after: its last), for per-step timing; no graph is
// captured then.  bytes (optional): receives each step's algorithmic bytes
// summed over the images.
int run_batch(vlg_ctx *c, vlg_formula *f, const vlg_image *const *imgs, const std::vector<int> &idx,
              void *const *outs, int fmt, int where, StepHook hook = nullptr, void *hook_ctx = nullptr,
              std::vector<double> *bytes = nullptr) {
    const size_t nout = f->dag.outputs.size();
    std::vector<int> all(nout);
    for (size_t i = 0; i < nout; i++) all[i] = (int)i;
    const Plan &P = f->plan(all, Mode::Fused);
    const int n = (int)idx.size();
    if (n == 0 || nout == 0) return VLG_OK;
    const int dtype = imgs[idx[0]]->dtype;
    const bool direct = fmt == VLG_PACKED64 && where == VLG_DEVICE;
    const bool stage_u8 = fmt == VLG_U8MASK && where == VLG_HOST;

    // one labelling tile height for the batch: forced, else the batch class's
    // tuned value, else the tallest tile that leaves enough tiles over the
    // whole batch
    int64_t pixels = 0;
    for (int i : idx) pixels += (int64_t)imgs[i]->H * imgs[i]->W;
    const int tbh_untuned = default_tile_bh([&](int t) {
        int64_t sum = 0;
        for (int i : idx) sum += tile_count(imgs[i]->H, imgs[i]->W, t);
        return sum;
    });
    const int tbh = batch_value(c, VLG_TUNE_CCL_TILE_ROWS, n, pixels, tbh_untuned);
    const int grid_cap = batch_value(c, VLG_TUNE_BATCH_GRID, n, pixels, kBatchGridDefault);

    // workspace: per-image layouts, then the descriptor block
    std::vector<Geo> geo(n);
    std::vector<Layout> lay(n);
    std::vector<size_t> off(n);
    size_t total = 0;
    for (int k = 0; k < n; k++) {
        geo[k] = make_geo(imgs[idx[k]]->H, imgs[idx[k]]->W);
        lay[k] = layout_for(P, geo[k], true, stage_u8);
        off[k] = total;
        total += align256(lay[k].total);
    }
    const size_t npct = (size_t)P.npct;
    const size_t d_imgs = total;
    const size_t d_outs = d_imgs + align256((size_t)n * sizeof(BImg));
    const size_t d_ranks = d_outs + align256((size_t)n * nout * sizeof(uint64_t *));
    const size_t d_prefix = d_ranks + align256((size_t)n * std::max<size_t>(npct, 1) * 4);
    const size_t d_end = d_prefix + align256((size_t)BK_COUNT * (n + 1) * 8);
    int rc = ensure_ws(c, d_end);
    if (rc != VLG_OK) return rc;
    char *base = (char *)c->ws;

    // descriptors in pinned host memory, reused once the previous upload is done
    const size_t dbytes = d_end - d_imgs;
    if (c->desc_done) HIP_TRY(hipEventSynchronize(c->desc_done));
    if (c->desc_host_size < dbytes) {
        if (c->desc_host) HIP_TRY(hipHostFree(c->desc_host));
        c->desc_host = nullptr;
        c->desc_host_size = 0;
        HIP_TRY(hipHostMalloc(&c->desc_host, dbytes, hipHostMallocDefault));
        c->desc_host_size = dbytes;
    }
    if (!c->desc_done) HIP_TRY(hipEventCreateWithFlags(&c->desc_done, hipEventDisableTiming));
    char *h = (char *)c->desc_host;
    std::memset(h, 0, dbytes);
    BImg *hi = (BImg *)h;
    uint64_t **ho = (uint64_t **)(h + (d_outs - d_imgs));
    uint32_t *hr = (uint32_t *)(h + (d_ranks - d_imgs));
    int64_t *hp = (int64_t *)(h + (d_prefix - d_imgs));
    std::vector<double> pct_q(npct, 0.0);
    for (const Step &s : P.steps)
        if (s.kind == SK::Pct)
            for (int j = 0; j < s.npq; j++) pct_q[(size_t)s.pct_out[j]] = s.q[j];
    std::vector<uint64_t *> ext((size_t)n * nout);
    for (int k = 0; k < n; k++) {
        const vlg_image *im = imgs[idx[k]];
        const Layout &L = lay[k];
        char *wb = base + off[k];
        BImg &d = hi[k];
        d.g = geo[k];
        d.img = (const char *)im->dev;
        d.chan_bytes = (int64_t)im->H * im->pitch * (int64_t)im->esize();
        d.ws = wb + L.off_slots;
        d.mask_bytes = L.mask_bytes;
        d.off_glab = L.off_glab - L.off_slots;
        d.off_gflag = L.off_gflag - L.off_slots;
        d.off_pct = L.off_pct - L.off_slots;
        d.off_pctst = L.off_pctst - L.off_slots;
        d.outs = (uint64_t *const *)(base + d_outs) + (size_t)k * nout;
        d.ranks = (const uint32_t *)(base + d_ranks) + (size_t)k * std::max<size_t>(npct, 1);
        const int64_t npix = (int64_t)im->H * im->W;
        for (size_t p = 0; p < npct; p++)
            hr[(size_t)k * std::max<size_t>(npct, 1) + p] = pct_rank(pct_q[p], npix);
        for (size_t o = 0; o < nout; o++) {
            void *user = outs[(size_t)idx[k] * nout + o];
            uint64_t *e = direct && user ? (uint64_t *)user : (uint64_t *)(wb + L.off_stage + o * L.mask_bytes);
            ext[(size_t)k * nout + o] = e;
            ho[(size_t)k * nout + o] = e;
        }
        for (int kind = 0; kind < BK_COUNT; kind++)
            hp[(size_t)kind * (n + 1) + k + 1] = hp[(size_t)kind * (n + 1) + k] + batch_units(geo[k], kind, tbh);
    }
    HIP_TRY(hipMemcpyAsync(base + d_imgs, h, dbytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipEventRecord(c->desc_done, c->stream));

    auto args = [&](int kind) {
        BatchArgs a;
        a.n = n;
        a.dtype = dtype;
        a.grid_cap = grid_cap;
        a.imgs = (const BImg *)(base + d_imgs);
        a.prefix = (const int64_t *)(base + d_prefix) + (size_t)kind * (n + 1);
        a.guard = c->guard();
        return a;
    };
    auto units = [&](int kind) { return hp[(size_t)kind * (n + 1) + n]; };
    auto bref = [](const Ref &r) { return BRef{r.slot, (uint32_t)(r.inv ? 1 : 0)}; };

    // Arith steps si..sj: one launch per image (the arithmetic kernel has no
    // batched form)
    auto arith_images = [&](size_t si, size_t sj) -> hipError_t {
        ArithGroup a = arith_group(P, si, sj);
        hipError_t e = hipSuccess;
        for (int k = 0; k < n && e == hipSuccess; k++) {
            const vlg_image *im = imgs[idx[k]];
            char *wb = base + off[k];
            for (size_t t = si; t <= sj && t - si < (size_t)kArithGroupProgs; t++) {
                const int32_t o = P.steps[t].out;
                a.out[t - si] = is_ext(o) ? ext[(size_t)k * nout + (size_t)ext_index(o)]
                                          : (uint64_t *)(wb + lay[k].off_slots + (size_t)o * lay[k].mask_bytes);
            }
            e = arith_launch(c, c->stream, geo[k], im->H, im->W, im->dev, (int64_t)im->H * im->pitch, im->dtype, a,
                             (const float *)(wb + lay[k].off_pct));
        }
        return e;
    };

    if (bytes) {
        bytes->assign(P.steps.size(), 0.0);
        for (size_t si = 0; si < P.steps.size(); si++)
            for (int k = 0; k < n; k++) (*bytes)[si] += algorithmic_bytes(P, P.steps[si], geo[k], dtype, tbh);
    }
    auto enqueue_steps = [&]() -> int {
        for (size_t si = 0; si < P.steps.size(); si++) {
            const Step &s = P.steps[si];
            hipError_t e = hipSuccess;
            if (hook) hook(hook_ctx, si, true);
            if (s.group >= 0) {
                size_t sj = si;
                while (sj + 1 < P.steps.size() && P.steps[sj + 1].group == s.group) sj++;
                if (hook && sj > si) {
                    // the group is timed as a whole: attribute it to its last step
                    hook(hook_ctx, si, false);
                    for (size_t k = si + 1; k < sj; k++) {
                        hook(hook_ctx, k, true);
                        hook(hook_ctx, k, false);
                    }
                    hook(hook_ctx, sj, true);
                }
                if (s.kind == SK::Arith) {
                    e = arith_images(si, sj);
                } else if (s.kind == SK::Logic) {
                    BLogic b;
                    std::memset(&b, 0, sizeof b);
                    b.n = (int)(sj - si + 1);
                    for (size_t k = si; k <= sj; k++) {
                        const Step &t = P.steps[k];
                        b.ops[k - si] = BLogicOp{bref(t.x), bref(t.y), t.op, t.inv_out, t.out};
                    }
                    e = launch_b_logic(c->stream, args(BK_LOGIC), units(BK_LOGIC), b);
                } else {
                    BNear b;
                    std::memset(&b, 0, sizeof b);
                    b.n = (int)(sj - si + 1);
                    for (size_t k = si; k <= sj; k++) {
                        const Step &t = P.steps[k];
                        b.ops[k - si] = BNearOp{bref(t.x), bref(t.z), t.inv_out, t.op, t.out};
                    }
                    e = launch_b_near(c->stream, args(BK_NEAR), units(BK_NEAR), b);
                }
                if (e != hipSuccess) return fail(VLG_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
                if (hook) hook(hook_ctx, sj, false);
                si = sj;
                continue;
            }
            switch (s.kind) {
            case SK::Pct:
            {
                PctSel sel;
                std::memset(&sel, 0, sizeof sel);
                sel.n = s.npq;
                for (int j = 0; j < s.npq; j++) sel.slot[j] = s.pct_out[j];
                e = launch_b_percentile(c->stream, args(BK_ONE), units(BK_ONE), args(BK_PCTH), units(BK_PCTH), s.chan,
                                        sel);
            }
                break;
            case SK::Atoms: {
                BAtoms a;
                std::memset(&a, 0, sizeof a);
                a.chan = s.chan;
                a.n = s.natoms;
                for (int j = 0; j < s.natoms; j++) {
                    a.cmp[j] = s.atoms[j].cmp;
                    a.thr[j] = s.atoms[j].thr;
                    a.pct[j] = s.atoms[j].use_pct ? s.atoms[j].pct : -1;
                    a.out[j] = s.atoms[j].out;
                }
                e = launch_b_atoms(c->stream, args(BK_WORDS), units(BK_WORDS), a);
                break;
            }
            case SK::Logic: {
                BLogic b;
                std::memset(&b, 0, sizeof b);
                b.n = 1;
                b.ops[0] = BLogicOp{bref(s.x), bref(s.y), s.op, s.inv_out, s.out};
                e = launch_b_logic(c->stream, args(BK_LOGIC), units(BK_LOGIC), b);
                break;
            }
            case SK::Near: {
                BNear b;
                std::memset(&b, 0, sizeof b);
                b.n = 1;
                b.ops[0] = BNearOp{bref(s.x), bref(s.z), s.inv_out, s.op, s.out};
                e = launch_b_near(c->stream, args(BK_NEAR), units(BK_NEAR), b);
                break;
            }
            case SK::CclLocal:
                e = launch_b_ccl_local(c->stream, args(BK_TILES), units(BK_TILES), tbh, bref(s.x), bref(s.y),
                                       bref(s.z));
                break;
            case SK::CclMerge:
                e = launch_b_ccl_merge(c->stream, args(BK_MERGE), units(BK_MERGE), tbh, bref(s.x));
                break;
            case SK::CclFlag:
                e = launch_b_ccl_flag(c->stream, args(BK_FLAG), units(BK_FLAG));
                break;
            case SK::CclGather:
                e = launch_b_ccl_gather(c->stream, args(BK_GATHER), units(BK_GATHER), bref(s.x), bref(s.y),
                                        bref(s.z), s.user, s.out);
                break;
            case SK::CclReseed:
                e = launch_b_ccl_reseed(c->stream, args(BK_BLOCKS), units(BK_BLOCKS), bref(s.x), s.user);
                break;
            case SK::Segment:
                return fail(VLG_EINVAL, "internal: the batched schedule has no segments");
            case SK::Arith:
                e = arith_images(si, si);
                break;
            }
            if (e != hipSuccess) return fail(VLG_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
            if (hook) hook(hook_ctx, si, false);
        }
        if (fmt == VLG_U8MASK) {
            for (int k = 0; k < n; k++)
                for (size_t o = 0; o < nout; o++) {
                    void *user = outs[(size_t)idx[k] * nout + o];
                    if (!user) continue;
                    uint8_t *dst = where == VLG_DEVICE
                                       ? (uint8_t *)user
                                       : (uint8_t *)(base + off[k] + lay[k].off_u8 +
                                                     o * align256((size_t)geo[k].H * geo[k].W));
                    hipError_t e = launch_unpack(c->stream, geo[k], ext[(size_t)k * nout + o], dst);
                    if (e != hipSuccess) return fail(VLG_EHIP, hipGetErrorString(e));
                }
        }
        return VLG_OK;
    };

    for (int k = 0; k < n; k++) {
        const vlg_image *im = imgs[idx[k]];
        if (k == 0 || im->H != imgs[idx[k - 1]]->H || im->W != imgs[idx[k - 1]]->W ||
            im->dtype != imgs[idx[k - 1]]->dtype)
            prepare_arith(c, P, im->H, im->W, im->dtype);
    }
    if (c->mode == VLG_MODE_GRAPH && !hook) {
        GraphKey key;
        key.v = {(uintptr_t)0xBA7C, (uintptr_t)f->serial, (uintptr_t)&P, (uintptr_t)c->ws, (uintptr_t)tbh,
                 (uintptr_t)grid_cap, (uintptr_t)fmt, (uintptr_t)where, (uintptr_t)n, (uintptr_t)c->loop_cap};
        for (int k = 0; k < n; k++) {
            const vlg_image *im = imgs[idx[k]];
            key.v.insert(key.v.end(), {(uintptr_t)im->dev, (uintptr_t)im->H, (uintptr_t)im->W,
                                       (uintptr_t)im->dtype, (uintptr_t)im->pitch,
                                       (uintptr_t)tuned_value(c, VLG_TUNE_ARITH, im->H, im->W)});
            for (size_t o = 0; o < nout; o++) key.v.push_back((uintptr_t)outs[(size_t)idx[k] * nout + o]);
        }
        auto it = c->graphs.find(key);
        if (it == c->graphs.end()) {
            HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            int r = enqueue_steps();
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(c->stream, &graph);
            if (r != VLG_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return r;
            }
            if (e != hipSuccess) return fail(VLG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
            hipGraphExec_t exec = nullptr;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return fail(VLG_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
            if (c->graphs.size() >= 64) c->drop_graphs();
            it = c->graphs.emplace(key, exec).first;
        }
        HIP_TRY(hipGraphLaunch(it->second, c->stream));
    } else {
        rc = enqueue_steps();
        if (rc != VLG_OK) return rc;
    }
    for (int k = 0; k < n; k++)
        if (imgs[idx[k]]->note_use(c->stream) != VLG_OK) return fail(VLG_EHIP, "event record failed");

    if (where == VLG_HOST) {
        for (int k = 0; k < n; k++)
            for (size_t o = 0; o < nout; o++) {
                void *user = outs[(size_t)idx[k] * nout + o];
                if (!user) continue;
                if (fmt == VLG_PACKED64)
                    HIP_TRY(hipMemcpyAsync(user, ext[(size_t)k * nout + o], (size_t)geo[k].nwords * 8,
                                           hipMemcpyDeviceToHost, c->stream));
                else
                    HIP_TRY(hipMemcpyAsync(user,
                                           base + off[k] + lay[k].off_u8 + o * align256((size_t)geo[k].H * geo[k].W),
                                           (size_t)geo[k].H * geo[k].W, hipMemcpyDeviceToHost, c->stream));
            }
        return check_status(c);
    }
    return VLG_OK;
}

}  // namespace

namespace vlg {
// Used by the serving loop (server.cpp).
size_t evaluation_footprint(vlg_formula *f, const vlg_image *img) {
    std::vector<int> all(f->dag.outputs.size());
    for (size_t i = 0; i < all.size(); i++) all[i] = (int)i;
    // server slots run one labelling lane and the default segment halo cap
    const bool vol = img->D > 1;
    const Plan &P = f->plan(all, Mode::Fused, 1, vol ? 1 : kFuseHaloDefault);
    return layout_for(P, make_geo(img->H, img->W), false, false, false, vol).total;
}
int evaluate_all_on(vlg_ctx *c, vlg_formula *f, const vlg_image *img, void *const *outs, void *ws, size_t ws_size) {
    c->ws = ws;
    c->ws_size = ws_size;
    c->ws_external = true;
    std::vector<int> which;
    std::vector<void *> o;
    for (size_t i = 0; i < f->dag.outputs.size(); i++) {
        if (!outs[i]) continue;
        which.push_back((int)i);
        o.push_back(outs[i]);
    }
    int rc = run(c, f, img, which, o, VLG_PACKED64, VLG_DEVICE);
    if (rc == VLG_OK) rc = check_status(c);
    return rc;
}
const char *last_error_text() { return g_err.c_str(); }
int set_last_error(int code, const std::string &msg) { return fail(code, msg); }
size_t formula_outputs(const vlg_formula *f) { return f->dag.outputs.size(); }
}  // namespace vlg

namespace {

// Time `run` (which enqueues one evaluation) for every candidate of each
// tunable in turn, each forced in turn; the fastest value of a tunable is
// kept (via `keep`) before the next tunable is tried.
template <typename Run, typename Keep>
int tune_loop(vlg_ctx *c, const std::vector<std::pair<int, std::vector<int>>> &space, int iters, Run run,
              Keep keep, vlg_tune_report *out, int max_out, int *n_out) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = VLG_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(VLG_EHIP, "event create");
    const Tuning saved = c->forced;
    *n_out = 0;
    for (size_t t = 0; t < space.size() && rc == VLG_OK; t++) {
        const int which = space[t].first;
        vlg_tune_report rep;
        std::memset(&rep, 0, sizeof rep);
        rep.which = which;
        double best_ms = 1e30;
        for (int cand : space[t].second) {
            c->forced.v[which] = cand;
            // the warm-up is timed too: a candidate more than 8x slower than
            // the best so far is not timed again
            float ms = 0.f;
            if (hipEventRecord(e0, c->stream) != hipSuccess) rc = fail(VLG_EHIP, "event record");
            if (rc == VLG_OK) rc = run();  // warm-up
            if (rc == VLG_OK && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = fail(VLG_EHIP, "event timing");
            int timed = 1;
            if (rc == VLG_OK && ms < 8.0 * best_ms) {
                if (hipEventRecord(e0, c->stream) != hipSuccess) rc = fail(VLG_EHIP, "event record");
                for (int it = 0; it < iters && rc == VLG_OK; it++) rc = run();
                if (rc == VLG_OK && (hipEventRecord(e1, c->stream) != hipSuccess ||
                                     hipEventSynchronize(e1) != hipSuccess ||
                                     hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    rc = fail(VLG_EHIP, "event timing");
                timed = iters;
            }
            if (rc == VLG_ENOCONV && which == VLG_TUNE_CCL_ALGO) {
                rc = VLG_OK;  // a labelling that did not terminate within the cap is not a candidate
                (void)hipStreamSynchronize(c->stream);
                continue;
            }
            if (rc != VLG_OK) break;
            rep.candidates[rep.n] = cand;
            rep.ms[rep.n] = ms / timed;
            if (rep.ms[rep.n] < best_ms) {
                best_ms = rep.ms[rep.n];
                rep.best = cand;
            }
            rep.n++;
        }
        c->forced.v[which] = saved.v[which];
        if (rc != VLG_OK) break;
        keep(which, rep.best);
        if (out && *n_out < max_out) out[*n_out] = rep;
        (*n_out)++;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}

}  // namespace

namespace {

// Labelling scratch of vlg_ccl_labels: parent pointers (4 B per 2x2 block),
// flag bytes (1 B per block) and the canonical-label table (4 B per block).
size_t ccl_labels_scratch_bytes(const Geo &g) {
    const size_t nb = (size_t)g.BH * g.BW;
    return 2 * align256(nb * 4) + align256(nb) + 256;
}

// Labels of the mask into labels_dev, with the labelling arrays in `scratch`
// (at least ccl_labels_scratch_bytes(g) bytes of device memory).  Every array
// the kernels read is written first in the same call (the local pass writes
// every block's parent and flag byte, the table is filled before use), so the
// scratch needs no clearing between calls.
int ccl_labels_on(vlg_ctx *c, const Geo &g, const uint64_t *mask_dev, int32_t *labels_dev, void *scratch) {
    const size_t nb = (size_t)g.BH * g.BW;
    CclWork w;
    w.glab = (int32_t *)scratch;
    w.gflag = (uint8_t *)scratch + align256(nb * 4);
    int32_t *canon = (int32_t *)((char *)scratch + align256(nb * 4) + align256(nb));
    w.counters = c->counters;
    w.tbh = tuning_for(c, g.H, g.W).ccl_tbh;
    w.guard = c->guard();
    MRef b{mask_dev, 0ull}, none{nullptr, 0ull};
    HIP_TRY(launch_fill_i64(c->stream, c->counters, 2, 0));
    HIP_TRY(launch_ccl_local(c->stream, g, b, none, none, w));
    HIP_TRY(launch_ccl_merge(c->stream, g, b, w));
    HIP_TRY(launch_ccl_flag(c->stream, g, w));
    HIP_TRY(launch_ccl_labels(c->stream, g, b, w, canon, labels_dev));
    return VLG_OK;
}

}  // namespace

extern "C" {

const char *vlg_last_error(void) { return g_err.c_str(); }

int vlg_create(vlg_ctx **out, int device, void *hip_stream) {
    if (!out) return fail(VLG_EINVAL, "null output handle");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return fail(VLG_EINVAL, "no HIP device " + std::to_string(device));
    }
    DeviceGuard dg(device);
    auto c = std::make_unique<vlg_ctx>();
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        c->arch = prop.gcnArchName;
        const size_t colon = c->arch.find(':');
        if (colon != std::string::npos) c->arch.resize(colon);
    }
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    const char *cc = std::getenv("VLG_CCL_COUNTERS");
    c->count_ccl = cc && cc[0] == '1';
    HIP_TRY(hipMalloc(&c->counters, 4 * sizeof(unsigned long long)));
    HIP_TRY(hipHostMalloc((void **)&c->status_host, 256, hipHostMallocDefault));
    *c->status_host = 0;
    HIP_TRY(launch_fill_i64(c->stream, c->counters, 4, 0));
    HIP_TRY(hipStreamSynchronize(c->stream));
    void *scratch_dev = nullptr;  // set-up of vlg_ccl_labels_noalloc on this device
    const int rc = noalloc_scratch(device, &scratch_dev);
    if (rc != VLG_OK) return rc;
    *out = c.release();
    return VLG_OK;
}

void vlg_destroy(vlg_ctx *c) {
    if (!c) return;
    DeviceGuard dg(c->device);
    (void)hipStreamSynchronize(c->stream);
    c->drop_graphs();
    if (c->ws && !c->ws_external) (void)hipFree(c->ws);
    if (c->counters) (void)hipFree(c->counters);
    if (c->status_host) (void)hipHostFree(c->status_host);
    if (c->desc_host) (void)hipHostFree(c->desc_host);
    if (c->desc_done) (void)hipEventDestroy(c->desc_done);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

int vlg_sync(vlg_ctx *c) {
    if (!c) return fail(VLG_EINVAL, "null context");
    DeviceGuard dg(c->device);
    return check_status(c);
}

int vlg_set_loop_cap(vlg_ctx *c, int cap) {
    if (!c || cap < 0) return fail(VLG_EINVAL, "bad loop cap");
    c->loop_cap = cap == 0 ? kLoopCapDefault : cap;
    return VLG_OK;
}

int vlg_set_mode(vlg_ctx *c, int mode) {
    if (!c || mode < VLG_MODE_PEROP || mode > VLG_MODE_GRAPH) return fail(VLG_EINVAL, "bad mode");
    c->mode = mode;
    return VLG_OK;
}

int vlg_load_image(vlg_ctx *c, const void *data, int dtype, int channels, int height, int width,
                   int64_t pitch_elems, int where, vlg_image **out) {
    if (!c || !out) return fail(VLG_EINVAL, "null handle");
    *out = nullptr;
    if (dtype != VLG_F32 && dtype != VLG_U8 && dtype != VLG_U16)
        return fail(VLG_EINVAL, "dtype must be VLG_F32, VLG_U8 or VLG_U16");
    if (where != VLG_HOST && where != VLG_DEVICE) return fail(VLG_EINVAL, "bad memory kind");
    if (channels < 1 || height < 0 || width < 0) return fail(VLG_ESHAPE, "bad image shape");
    if ((int64_t)height * width >= (1ll << 31)) return fail(VLG_ESHAPE, "image too large (H*W >= 2^31)");
    if (pitch_elems == 0) pitch_elems = width;
    if (pitch_elems < width) return fail(VLG_ESHAPE, "pitch smaller than width");
    if (!data && (int64_t)height * width > 0) return fail(VLG_EINVAL, "null image data");
    DeviceGuard dg(c->device);
    auto im = std::make_unique<vlg_image>();
    im->device = c->device;
    im->dtype = dtype;
    im->C = channels;
    im->H = height;
    im->W = width;
    im->pitch = (int64_t)((width + 63) / 64) * 64;
    const size_t es = im->esize();
    im->bytes = std::max<size_t>(256, (size_t)channels * height * im->pitch * es);
    if (hipMallocAsync(&im->dev, im->bytes, c->stream) != hipSuccess) {
        (void)hipGetLastError();
        return fail(VLG_ENOMEM, "image allocation failed");
    }
    HIP_TRY(hipMemsetAsync(im->dev, 0, im->bytes, c->stream));
    if ((int64_t)height * width > 0) {
        const hipMemcpyKind kind = where == VLG_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        for (int ch = 0; ch < channels; ch++) {
            const char *src = (const char *)data + (size_t)ch * height * pitch_elems * es;
            HIP_TRY(hipMemcpy2DAsync((char *)im->dev + (size_t)ch * height * im->pitch * es, im->pitch * es, src,
                                     (size_t)pitch_elems * es, (size_t)width * es, (size_t)height, kind,
                                     c->stream));
        }
    }
    if (where == VLG_HOST) HIP_TRY(hipStreamSynchronize(c->stream));
    const int ru = im->note_use(c->stream);  // the upload is the first use
    if (ru != VLG_OK) return fail(ru, "event record failed");
    *out = im.release();
    return VLG_OK;
}

int vlg_image_free(vlg_image *img) {
    if (!img) return VLG_OK;
    DeviceGuard dg(img->device);
    hipStream_t rel = release_stream(img->device);
    hipError_t e = rel ? hipSuccess : hipErrorOutOfMemory;
    {
        std::lock_guard<std::mutex> lk(img->mu);
        for (auto &u : img->uses) {
            if (e == hipSuccess) e = hipStreamWaitEvent(rel, u.second, 0);
            (void)hipEventDestroy(u.second);
        }
        img->uses.clear();
    }
    // stream-ordered release: after every enqueued use, without waiting for
    // the rest of the device (other contexts and server slots keep running)
    if (e == hipSuccess) e = hipFreeAsync(img->dev, rel);
    delete img;
    if (e != hipSuccess) return fail(VLG_EHIP, std::string("image release: ") + hipGetErrorString(e));
    return VLG_OK;
}

int vlg_image_shape(const vlg_image *img, int *channels, int *height, int *width) {
    if (!img) return fail(VLG_EINVAL, "null image");
    if (channels) *channels = img->C;
    if (height) *height = img->H;
    if (width) *width = img->W;
    return VLG_OK;
}

int vlg_load_volume(vlg_ctx *c, const void *data, int dtype, int channels, int depth, int height, int width,
                    int where, vlg_image **out) {
    if (out) *out = nullptr;
    if (depth < 1 || height < 0 || width < 0) return fail(VLG_ESHAPE, "bad volume shape");
    if ((int64_t)depth * height * width >= (1ll << 31) || (int64_t)depth * height >= (1ll << 31))
        return fail(VLG_ESHAPE, "volume too large (D*H*W >= 2^31)");
    // [C][D][H][W] with rows of W elements is [C][D*H][W]: loaded as D*H rows
    const int rc = vlg_load_image(c, data, dtype, channels, depth * height, width, width, where, out);
    if (rc != VLG_OK) return rc;
    (*out)->D = depth;
    (*out)->S = height;
    return VLG_OK;
}

int vlg_image_shape3(const vlg_image *img, int *channels, int *depth, int *height, int *width) {
    if (!img) return fail(VLG_EINVAL, "null image");
    if (channels) *channels = img->C;
    if (depth) *depth = img->D;
    if (height) *height = img->D > 1 ? img->S : img->H;
    if (width) *width = img->W;
    return VLG_OK;
}

int vlg_ccl_labels3(vlg_ctx *c, const uint64_t *mask_dev, int depth, int height, int width, int32_t *labels_dev) {
    const int64_t n = (int64_t)depth * height * width;
    if (!c || (!mask_dev && n > 0) || (!labels_dev && n > 0)) return fail(VLG_EINVAL, "null argument");
    if (depth < 1 || height < 0 || width < 0 || n >= (1ll << 31)) return fail(VLG_ESHAPE, "bad volume shape");
    DeviceGuard dg(c->device);
    const Geo g = make_geo(depth * height, width);
    if (g.nwords == 0) return VLG_OK;
    // block parents and each component's smallest voxel in the workspace
    const size_t pb = align256((size_t)vl_nblocks(g, height, depth) * 4);
    int rc = ensure_ws(c, 2 * pb);
    if (rc != VLG_OK) return rc;
    int *P = (int *)c->ws, *canon = (int *)((char *)c->ws + pb);
    const MRef b{mask_dev, 0ull};
    HIP_TRY(launch_vl_label(c->stream, g, height, depth, b, P, c->guard()));
    HIP_TRY(launch_vl_labels(c->stream, g, height, depth, b, P, canon, labels_dev));
    return VLG_OK;
}

int vlg_compile_formula(vlg_ctx *c, const char *src, vlg_formula **out) {
    (void)c;
    if (!src || !out) return fail(VLG_EINVAL, "null argument");
    *out = nullptr;
    auto f = std::make_unique<vlg_formula>();
    std::string err;
    try {
        if (!parse_formula(src, f->dag, err)) return fail(VLG_EPARSE, err);
    } catch (const std::bad_alloc &) {
        return fail(VLG_ENOMEM, "out of host memory while compiling");
    }
    for (const Node &n : f->dag.nodes) {
        if (n.op == Op::Atom) {
            f->max_chan = std::max(f->max_chan, n.chan);
            if (n.pct) f->max_chan = std::max(f->max_chan, n.pchan);
        }
    }
    for (const ArProgram &pr : f->dag.ariths)
        for (const ArInstr &in : pr.ins)
            if (in.op == AR_CHAN || in.op == AR_PCT) f->max_chan = std::max(f->max_chan, in.chan);
    *out = f.release();
    return VLG_OK;
}

int vlg_formula_plan(const vlg_formula *cf, int mode, int fuse_halo, char *buf, int64_t len, int64_t *needed) {
    if (!cf || (!buf && len > 0) || len < 0) return fail(VLG_EINVAL, "null argument");
    if (mode != VLG_MODE_PEROP && mode != VLG_MODE_FUSED) return fail(VLG_EINVAL, "mode must be per-op or fused");
    if (mode == VLG_MODE_FUSED && !valid_fuse_halo(fuse_halo)) return fail(VLG_EINVAL, "bad segment halo cap");
    vlg_formula *f = const_cast<vlg_formula *>(cf);
    std::vector<int> all(f->dag.outputs.size());
    for (size_t i = 0; i < all.size(); i++) all[i] = (int)i;
    std::string t;
    try {
        const Plan &P = f->plan(all, mode == VLG_MODE_PEROP ? Mode::PerOp : Mode::Fused, 1, fuse_halo);
        char tmp[256];
        auto ref = [&](const Ref &r) {
            std::snprintf(tmp, sizeof tmp, "[%d, %d]", r.slot, (int)r.inv);
            return std::string(tmp);
        };
        std::snprintf(tmp, sizeof tmp, "{\"nslots\": %d, \"npct\": %d, \"noutputs\": %d, \"steps\": [", P.nslots,
                      P.npct, P.noutputs);
        t += tmp;
        for (size_t si = 0; si < P.steps.size(); si++) {
            const Step &st = P.steps[si];
            std::snprintf(tmp, sizeof tmp, "%s{\"kind\": \"%s\", \"out\": %d, \"op\": %d, \"inv_out\": %d, "
                                           "\"chan\": %d, \"user\": %d, \"group\": %d, \"seg\": %d, ",
                          si ? ", " : "", kind_name(st.kind), st.out, (int)st.op, (int)st.inv_out, st.chan, st.user,
                          st.group, st.seg);
            t += tmp;
            t += "\"x\": " + ref(st.x) + ", \"y\": " + ref(st.y) + ", \"z\": " + ref(st.z) + ", \"q\": [";
            for (int j = 0; j < st.npq; j++) {
                std::snprintf(tmp, sizeof tmp, "%s[%.17g, %d]", j ? ", " : "", st.q[j], st.pct_out[j]);
                t += tmp;
            }
            t += "], \"atoms\": [";
            for (int j = 0; j < st.natoms; j++) {
                const AtomEntry &e = st.atoms[j];
                std::snprintf(tmp, sizeof tmp, "%s[%d, %d, %.9g, %d, %d]", j ? ", " : "", (int)e.cmp, (int)e.use_pct,
                              (double)e.thr, e.pct, e.out);
                t += tmp;
            }
            t += "]";
            if (st.kind == SK::Arith) {
                // [op, channel or percentile scalar, constant]; the left side first
                const ArProgram &pr = P.ariths[(size_t)st.arith];
                std::snprintf(tmp, sizeof tmp, ", \"lhs_len\": %d, \"arith\": [", pr.lhs_len);
                t += tmp;
                for (size_t q = 0; q < pr.ins.size(); q++) {
                    const ArInstr &in = pr.ins[q];
                    std::snprintf(tmp, sizeof tmp, "%s[%d, %d, %.9g]", q ? ", " : "", (int)in.op,
                                  in.op == AR_PCT ? in.pct : in.chan, (double)in.c);
                    t += tmp;
                }
                t += "]";
            }
            t += "}";
        }
        t += "], \"segments\": [";
        for (size_t k = 0; k < P.segments.size(); k++) {
            const Segment &S = P.segments[k];
            std::snprintf(tmp, sizeof tmp, "%s{\"halo\": %d, \"nregs\": %d, \"inputs\": [", k ? ", " : "", S.halo,
                          S.nregs);
            t += tmp;
            for (size_t q = 0; q < S.inputs.size(); q++) t += (q ? ", " : "") + std::to_string(S.inputs[q]);
            t += "], \"outputs\": [";
            for (size_t q = 0; q < S.outputs.size(); q++) t += (q ? ", " : "") + std::to_string(S.outputs[q]);
            t += "], \"ins\": [";
            for (size_t q = 0; q < S.ins.size(); q++) {
                const SegInstr &in = S.ins[q];
                std::snprintf(tmp, sizeof tmp, "%s[%d, %d, %d, %d, %d]", q ? ", " : "", in.op, in.dst, in.a, in.b,
                              in.inv);
                t += tmp;
            }
            t += "]}";
        }
        t += "]}";
    } catch (const std::bad_alloc &) {
        return fail(VLG_ENOMEM, "out of host memory");
    }
    if (needed) *needed = (int64_t)t.size() + 1;
    if (len < (int64_t)t.size() + 1) return len == 0 ? VLG_OK : fail(VLG_EINVAL, "buffer too small");
    std::memcpy(buf, t.c_str(), t.size() + 1);
    return VLG_OK;
}

int vlg_formula_info(const vlg_formula *cf, vlg_formula_stats *st) {
    if (!cf || !st) return fail(VLG_EINVAL, "null argument");
    vlg_formula *f = const_cast<vlg_formula *>(cf);
    std::vector<int> all(f->dag.outputs.size());
    for (size_t i = 0; i < all.size(); i++) all[i] = (int)i;
    const Plan &pp = f->plan(all, Mode::PerOp);
    const Plan &pf = f->plan(all, Mode::Fused, 1, kFuseHaloDefault);
    st->parsed_nodes = f->dag.parsed_nodes;
    st->nodes = (int64_t)f->dag.nodes.size();
    st->reach_nodes = count_op(f->dag, true);
    st->atoms = count_op(f->dag, false);
    st->outputs = (int64_t)f->dag.outputs.size();
    st->steps_perop = (int64_t)pp.steps.size();
    st->steps_fused = (int64_t)pf.steps.size();
    st->peak_masks = pf.nslots;
    int64_t launches = 0;
    for (size_t i = 0; i < pf.steps.size(); i++) {
        if (pf.steps[i].group >= 0 && i > 0 && pf.steps[i - 1].group == pf.steps[i].group) continue;
        launches += pf.steps[i].kind == SK::Pct ? 7 : 1;
    }
    st->launches_fused = launches;
    st->labellings = pf.ccl_count;
    st->labelling_reuse = pf.ccl_reuse;
    st->segments = (int64_t)pf.segments.size();
    return VLG_OK;
}

const char *vlg_formula_output_name(const vlg_formula *f, int index) {
    if (!f || index < 0 || index >= (int)f->dag.output_names.size()) return nullptr;
    return f->dag.output_names[(size_t)index].c_str();
}

int vlg_formula_free(vlg_formula *f) {
    delete f;
    return VLG_OK;
}

int vlg_check(vlg_ctx *c, const vlg_formula *cf, const vlg_image *img, int output_index, void *out_mask,
              int fmt, int where) {
    if (!c || !cf || !img || !out_mask) return fail(VLG_EINVAL, "null argument");
    vlg_formula *f = const_cast<vlg_formula *>(cf);
    if (output_index < 0 || output_index >= (int)f->dag.outputs.size())
        return fail(VLG_EINVAL, "output index out of range");
    try {
        return run(c, f, img, {output_index}, {out_mask}, fmt, where);
    } catch (const std::bad_alloc &) {
        return fail(VLG_ENOMEM, "out of host memory");
    }
}

int vlg_check_all(vlg_ctx *c, const vlg_formula *cf, const vlg_image *img, void *const *outs, int fmt,
                  int where) {
    if (!c || !cf || !img || !outs) return fail(VLG_EINVAL, "null argument");
    vlg_formula *f = const_cast<vlg_formula *>(cf);
    std::vector<int> which;
    std::vector<void *> o;
    for (size_t i = 0; i < f->dag.outputs.size(); i++) {
        if (!outs[i]) continue;
        which.push_back((int)i);
        o.push_back(outs[i]);
    }
    try {
        return run(c, f, img, which, o, fmt, where);
    } catch (const std::bad_alloc &) {
        return fail(VLG_ENOMEM, "out of host memory");
    }
}

int vlg_check_batch(vlg_ctx *c, const vlg_formula *cf, const vlg_image *const *imgs, int n, void *const *outs,
                    int fmt, int where) {
    if (!c || !cf || (!imgs && n > 0) || (!outs && n > 0) || n < 0) return fail(VLG_EINVAL, "null argument");
    if (fmt != VLG_PACKED64 && fmt != VLG_U8MASK) return fail(VLG_EINVAL, "bad mask format");
    if (where != VLG_HOST && where != VLG_DEVICE) return fail(VLG_EINVAL, "bad memory kind");
    vlg_formula *f = const_cast<vlg_formula *>(cf);
    const size_t nout = f->dag.outputs.size();
    for (int i = 0; i < n; i++) {
        if (!imgs[i]) return fail(VLG_EINVAL, "null image in batch");
        if (imgs[i]->D > 1)
            return fail(VLG_EINVAL, "image " + std::to_string(i) + " is a volume: volumes are evaluated one at a time");
        if (f->max_chan >= imgs[i]->C)
            return fail(VLG_ESHAPE, "image " + std::to_string(i) + " lacks channel " + std::to_string(f->max_chan));
        if (imgs[i]->device != c->device) return fail(VLG_EINVAL, "image lives on another device");
    }
    try {
        if (c->mode == VLG_MODE_PEROP) {
            // the per-operator baseline: one image after the other
            for (int i = 0; i < n; i++) {
                int rc = vlg_check_all(c, cf, imgs[i], outs + (size_t)i * nout, fmt, where);
                if (rc != VLG_OK) return rc;
            }
            return VLG_OK;
        }
        DeviceGuard dg(c->device);
        // one batched pass per pixel type; empty images have no units
        for (int dt : {VLG_F32, VLG_U8, VLG_U16}) {
            std::vector<int> idx;
            for (int i = 0; i < n; i++)
                if (imgs[i]->dtype == dt) idx.push_back(i);
            int rc = run_batch(c, f, imgs, idx, outs, fmt, where);
            if (rc != VLG_OK) return rc;
        }
        return VLG_OK;
    } catch (const std::bad_alloc &) {
        return fail(VLG_ENOMEM, "out of host memory");
    }
}

int vlg_ccl_labels(vlg_ctx *c, const uint64_t *mask_dev, int height, int width, int32_t *labels_dev) {
    if (!c || (!mask_dev && (int64_t)height * width > 0) || (!labels_dev && (int64_t)height * width > 0))
        return fail(VLG_EINVAL, "null argument");
    if (height < 0 || width < 0 || (int64_t)height * width >= (1ll << 31)) return fail(VLG_ESHAPE, "bad shape");
    DeviceGuard dg(c->device);
    const Geo g = make_geo(height, width);
    if (g.nwords == 0) return VLG_OK;
    int rc = ensure_ws(c, ccl_labels_scratch_bytes(g));
    if (rc != VLG_OK) return rc;
    return ccl_labels_on(c, g, mask_dev, labels_dev, c->ws);
}

int vlg_ccl_labels_noalloc(vlg_ctx *c, const uint64_t *mask_dev, int height, int width, int32_t *labels_dev) {
    if (!c || (!mask_dev && (int64_t)height * width > 0) || (!labels_dev && (int64_t)height * width > 0))
        return fail(VLG_EINVAL, "null argument");
    if (height < 0 || width < 0 || (int64_t)height * width >= (1ll << 31)) return fail(VLG_ESHAPE, "bad shape");
    const Geo g = make_geo(height, width);
    if (g.nwords == 0) return VLG_OK;
    const size_t need = ccl_labels_scratch_bytes(g);
    if (need > kNoallocScratchBytes)
        return fail(VLG_ESHAPE, "vlg_ccl_labels_noalloc: a " + std::to_string(height) + " x " + std::to_string(width) +
                                    " image needs " + std::to_string(need) + " bytes of labelling scratch, more than the " +
                                    std::to_string(kNoallocScratchBytes) + " of the fixed device array");
    DeviceGuard dg(c->device);
    void *scratch_dev = nullptr;
    int rc = noalloc_scratch(c->device, &scratch_dev);
    if (rc != VLG_OK) return rc;
    return ccl_labels_on(c, g, mask_dev, labels_dev, scratch_dev);
}

int vlg_profile(vlg_ctx *c, const vlg_formula *cf, const vlg_image *img, int iters, vlg_kernel_time *out,
                int max_out, int *n_out) {
    if (!c || !cf || !img || !out || !n_out || iters < 1) return fail(VLG_EINVAL, "bad argument");
    vlg_formula *f = const_cast<vlg_formula *>(cf);
    if (f->max_chan >= img->C) return fail(VLG_ESHAPE, "formula uses a channel the image lacks");
    DeviceGuard dg(c->device);
    std::vector<int> which(f->dag.outputs.size());
    for (size_t i = 0; i < which.size(); i++) which[i] = (int)i;
    const Plan &P = f->plan(which, Mode::Fused, 1, img->D > 1 ? 1 : tuned_value(c, VLG_TUNE_FUSE_HALO, img->H, img->W));
    const Geo g = make_geo(img->H, img->W);
    *n_out = 0;
    if (g.nwords == 0 || which.empty()) return VLG_OK;
    const bool vol = img->D > 1;
    const bool pj = !vol && P.ccl_count > 0 && ccl_algo(c, img->H, img->W) == VLG_CCL_POINTER_JUMPING;
    if (pj && !pj_shape_ok(img->H, img->W))
        return fail(VLG_ESHAPE, "pointer-jumping labelling: rows and columns must stay below 65535");
    Layout L = layout_for(P, g, true, false, pj, vol);
    int rc = ensure_ws(c, L.total);
    if (rc != VLG_OK) return rc;
    std::vector<uint64_t *> ext(which.size());
    for (size_t k = 0; k < which.size(); k++) ext[k] = (uint64_t *)((char *)c->ws + L.off_stage + k * L.mask_bytes);
    struct Ev {
        std::vector<hipEvent_t> ev;
    } E;
    E.ev.resize(2 * P.steps.size());
    for (auto &e : E.ev) HIP_TRY(hipEventCreate(&e));
    std::vector<double> ms(P.steps.size(), 0.0);
    struct Tr {
        Ev *e;
        hipStream_t s;
    } tr{&E, c->stream};
    auto hook2 = [](void *p, size_t si, bool before) {
        Tr *t = (Tr *)p;
        (void)hipEventRecord(t->e->ev[2 * si + (before ? 0 : 1)], t->s);
    };
    for (int it = 0; it < iters && rc == VLG_OK; it++) {
        rc = enqueue_plan(c, P, img, L, ext, hook2, &tr);
        if (rc != VLG_OK) break;
        if (hipStreamSynchronize(c->stream) != hipSuccess) {
            rc = fail(VLG_EHIP, "synchronize failed");
            break;
        }
        for (size_t si = 0; si < P.steps.size(); si++) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, E.ev[2 * si], E.ev[2 * si + 1]) == hipSuccess) ms[si] += t;
        }
    }
    for (auto &e : E.ev) (void)hipEventDestroy(e);
    if (rc != VLG_OK) return rc;
    std::vector<vlg_kernel_time> kinds;
    for (size_t si = 0; si < P.steps.size(); si++) {
        const SK kind = P.steps[si].kind;
        if ((pj || vol) && (kind == SK::CclMerge || kind == SK::CclFlag)) continue;  // not run
        const char *nm = vol && kind == SK::CclLocal    ? "vol_label"
                         : vol && kind == SK::CclGather ? "vol_gather"
                         : vol && kind == SK::CclReseed ? "vol_reseed"
                         : vol && kind == SK::Near      ? "near3"
                         : pj && kind == SK::CclLocal    ? "pj_label"
                         : pj && kind == SK::CclGather ? "pj_gather"
                         : pj && kind == SK::CclReseed ? "pj_reseed"
                                                       : kind_name(kind);
        auto it = std::find_if(kinds.begin(), kinds.end(),
                               [&](const vlg_kernel_time &k) { return std::strcmp(k.name, nm) == 0; });
        if (it == kinds.end()) {
            vlg_kernel_time k;
            std::memset(&k, 0, sizeof k);
            std::snprintf(k.name, sizeof k.name, "%s", nm);
            kinds.push_back(k);
            it = kinds.end() - 1;
        }
        // a batched group is one launch, timed as a whole on its last step
        const bool grouped_not_last = P.steps[si].group >= 0 && si + 1 < P.steps.size() &&
                                      P.steps[si + 1].group == P.steps[si].group;
        if (!grouped_not_last) it->launches += iters;
        it->ms += ms[si];
        if ((pj || vol) && kind == SK::CclLocal)  // labels written once, mask read once
            it->bytes += iters * ((double)g.H * g.W * 4.0 + (double)g.nwords * 8.0);
        else if ((pj || vol) && (kind == SK::CclGather || kind == SK::CclReseed))  // labels read once
            it->bytes += iters * ((double)g.H * g.W * 4.0 + (double)g.nwords * 8.0 * 2.0);
        else
            it->bytes += iters * algorithmic_bytes(P, P.steps[si], g, img->dtype, tuning_for(c, img->H, img->W).ccl_tbh);
    }
    for (size_t i = 0; i < kinds.size() && (int)i < max_out; i++) out[i] = kinds[i];
    *n_out = (int)kinds.size();
    return VLG_OK;
}

int vlg_profile_batch(vlg_ctx *c, const vlg_formula *cf, const vlg_image *const *imgs, int n, int iters,
                      vlg_kernel_time *out, int max_out, int *n_out) {
    if (!c || !cf || !imgs || n < 1 || !out || !n_out || iters < 1) return fail(VLG_EINVAL, "bad argument");
    vlg_formula *f = const_cast<vlg_formula *>(cf);
    const int dtype = imgs[0] ? imgs[0]->dtype : 0;
    for (int i = 0; i < n; i++) {
        if (!imgs[i]) return fail(VLG_EINVAL, "null image in batch");
        if (imgs[i]->D > 1) return fail(VLG_EINVAL, "volumes are not batched");
        if (f->max_chan >= imgs[i]->C) return fail(VLG_ESHAPE, "formula uses a channel an image lacks");
        if (imgs[i]->dtype != dtype) return fail(VLG_EINVAL, "batch profiling needs one pixel type");
        if (imgs[i]->device != c->device) return fail(VLG_EINVAL, "image lives on another device");
    }
    DeviceGuard dg(c->device);
    *n_out = 0;
    const size_t nout = f->dag.outputs.size();
    std::vector<int> all(nout), idx((size_t)n);
    for (size_t i = 0; i < nout; i++) all[i] = (int)i;
    for (int i = 0; i < n; i++) idx[(size_t)i] = i;
    const Plan &P = f->plan(all, Mode::Fused);
    if (P.steps.empty()) return VLG_OK;
    std::vector<void *> outs((size_t)n * nout, nullptr);
    std::vector<hipEvent_t> ev(2 * P.steps.size(), nullptr);
    int rc = VLG_OK;
    for (auto &e : ev)
        if (rc == VLG_OK && hipEventCreate(&e) != hipSuccess) rc = fail(VLG_EHIP, "event create");
    struct Tr {
        std::vector<hipEvent_t> *ev;
        hipStream_t s;
    } tr{&ev, c->stream};
    auto hook = [](void *p, size_t si, bool before) {
        Tr *t = (Tr *)p;
        (void)hipEventRecord((*t->ev)[2 * si + (before ? 0 : 1)], t->s);
    };
    std::vector<double> ms(P.steps.size(), 0.0), bytes;
    for (int it = 0; it < iters && rc == VLG_OK; it++) {
        rc = run_batch(c, f, imgs, idx, outs.data(), VLG_PACKED64, VLG_DEVICE, hook, &tr, &bytes);
        if (rc != VLG_OK) break;
        if (hipStreamSynchronize(c->stream) != hipSuccess) {
            rc = fail(VLG_EHIP, "synchronize failed");
            break;
        }
        for (size_t si = 0; si < P.steps.size(); si++) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, ev[2 * si], ev[2 * si + 1]) == hipSuccess) ms[si] += t;
        }
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc != VLG_OK) return rc;
    std::vector<vlg_kernel_time> kinds;
    for (size_t si = 0; si < P.steps.size(); si++) {
        const char *nm = kind_name(P.steps[si].kind);
        auto it = std::find_if(kinds.begin(), kinds.end(),
                               [&](const vlg_kernel_time &k) { return std::strcmp(k.name, nm) == 0; });
        if (it == kinds.end()) {
            vlg_kernel_time k;
            std::memset(&k, 0, sizeof k);
            std::snprintf(k.name, sizeof k.name, "%s", nm);
            kinds.push_back(k);
            it = kinds.end() - 1;
        }
        // a batched group is one launch, timed as a whole on its last step
        const bool grouped_not_last = P.steps[si].group >= 0 && si + 1 < P.steps.size() &&
                                      P.steps[si + 1].group == P.steps[si].group;
        if (!grouped_not_last) it->launches += iters;
        it->ms += ms[si];
        it->bytes += iters * (si < bytes.size() ? bytes[si] : 0.0);
    }
    std::sort(kinds.begin(), kinds.end(), [](const vlg_kernel_time &a, const vlg_kernel_time &b) { return a.ms > b.ms; });
    for (size_t k = 0; k < kinds.size() && (int)k < max_out; k++) out[k] = kinds[k];
    *n_out = (int)std::min(kinds.size(), (size_t)max_out);
    return check_status(c);
}

int vlg_profile_step(vlg_ctx *c, const vlg_formula *cf, const vlg_image *img, const char *kind, int reps,
                     double *avg_ms, double *bytes) {
    if (!c || !cf || !img || !kind || reps < 1 || !avg_ms || !bytes) return fail(VLG_EINVAL, "bad argument");
    vlg_formula *f = const_cast<vlg_formula *>(cf);
    if (f->max_chan >= img->C) return fail(VLG_ESHAPE, "formula uses a channel the image lacks");
    const std::string k(kind);
    SK sk;
    if (k == "atoms") sk = SK::Atoms;
    else if (k == "logic") sk = SK::Logic;
    else if (k == "near") sk = SK::Near;
    else if (k == "ccl_local") sk = SK::CclLocal;
    else if (k == "ccl_gather") sk = SK::CclGather;
    else if (k == "segment") sk = SK::Segment;
    else if (k == "arith") sk = SK::Arith;
    else if (k == "ccl_merge") sk = SK::CclMerge;
    else if (k == "ccl_flag") sk = SK::CclFlag;
    else return fail(VLG_EINVAL, "kind must be atoms, logic, near, ccl_local, ccl_merge, ccl_flag, ccl_gather, "
                                 "segment or arith");
    DeviceGuard dg(c->device);
    std::vector<int> which(f->dag.outputs.size());
    for (size_t i = 0; i < which.size(); i++) which[i] = (int)i;
    const bool vol = img->D > 1;
    const Plan &P = f->plan(which, Mode::Fused, 1, vol ? 1 : tuned_value(c, VLG_TUNE_FUSE_HALO, img->H, img->W));
    const Geo g = make_geo(img->H, img->W);
    *avg_ms = 0.0;
    *bytes = 0.0;
    if (g.nwords == 0) return VLG_OK;
    size_t at = SIZE_MAX;
    for (size_t si = 0; si < P.steps.size() && at == SIZE_MAX; si++)
        if (P.steps[si].kind == sk && P.steps[si].group < 0) at = si;
    if (at == SIZE_MAX) return fail(VLG_EINVAL, "the fused schedule has no single (ungrouped) step of kind " + k);
    const bool pj = !vol && P.ccl_count > 0 && ccl_algo(c, img->H, img->W) == VLG_CCL_POINTER_JUMPING;
    if (pj) return fail(VLG_EINVAL, "not with the pointer-jumping labelling (its rounds wait on the host)");
    const Layout L = layout_for(P, g, true, false, false, vol);
    int rc = ensure_ws(c, L.total);
    if (rc != VLG_OK) return rc;
    std::vector<uint64_t *> ext(which.size());
    for (size_t q = 0; q < which.size(); q++) ext[q] = (uint64_t *)((char *)c->ws + L.off_stage + q * L.mask_bytes);
    // A merge or flag step repeated alone would find its work done by the
    // launch before: its unit starts at its labelling's tile-local pass, and
    // the time of the unit without the step is subtracted.
    size_t from = at;
    if (sk == SK::CclMerge || sk == SK::CclFlag) {
        while (from > 0 && P.steps[from].kind != SK::CclLocal) from--;
        for (size_t q = from + 1; q < at; q++)
            if (P.steps[q].kind != SK::CclMerge && P.steps[q].kind != SK::CclFlag) from = SIZE_MAX;
        if (from == SIZE_MAX || P.steps[from].kind != SK::CclLocal)
            return fail(VLG_EINVAL, "the labelling of that step is not one run of local, merge, flag");
    }
    // the steps before it make its inputs; then the unit, back to back
    rc = enqueue_plan(c, P, img, L, ext, nullptr, nullptr, nullptr, 0, at + 1);
    if (rc != VLG_OK) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(VLG_EHIP, "event create");
    }
    auto timed = [&](size_t first, size_t last, float &ms) {
        ms = 0.f;
        int r0 = hipEventRecord(e0, c->stream) == hipSuccess ? VLG_OK : fail(VLG_EHIP, "event record");
        for (int r = 0; r < reps && r0 == VLG_OK; r++)
            r0 = enqueue_plan(c, P, img, L, ext, nullptr, nullptr, nullptr, first, last);
        if (r0 == VLG_OK && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            r0 = fail(VLG_EHIP, "event timing");
        return r0;
    };
    float ms = 0.f, ms_prefix = 0.f;
    rc = timed(from, at + 1, ms);
    if (rc == VLG_OK && from < at) rc = timed(from, at, ms_prefix);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != VLG_OK) return rc;
    *avg_ms = (ms - ms_prefix) / reps;
    *bytes = algorithmic_bytes(P, P.steps[at], g, img->dtype, tuning_for(c, img->H, img->W).ccl_tbh);
    return check_status(c);
}

int vlg_stream_copy(vlg_ctx *c, void *dst_dev, const void *src_dev, int64_t bytes, int width, int reps,
                    double *avg_ms) {
    if (!c || !dst_dev || !src_dev || bytes <= 0 || reps < 1 || !avg_ms) return fail(VLG_EINVAL, "bad argument");
    if ((width != 8 && width != 16) || bytes % width) return fail(VLG_EINVAL, "width must be 8 or 16 and divide bytes");
    DeviceGuard dg(c->device);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(VLG_EHIP, "event create");
    }
    int rc = VLG_OK;
    if (launch_stream_copy(c->stream, dst_dev, src_dev, bytes, width) != hipSuccess)  // warm-up
        rc = fail(VLG_EHIP, "copy launch");
    if (rc == VLG_OK && hipEventRecord(e0, c->stream) != hipSuccess) rc = fail(VLG_EHIP, "event record");
    for (int r = 0; r < reps && rc == VLG_OK; r++)
        if (launch_stream_copy(c->stream, dst_dev, src_dev, bytes, width) != hipSuccess) rc = fail(VLG_EHIP, "copy launch");
    float ms = 0.f;
    if (rc == VLG_OK && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = fail(VLG_EHIP, "event timing");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == VLG_OK) *avg_ms = ms / reps;
    return rc;
}

int vlg_set_tunable(vlg_ctx *c, int which, int value) {
    if (!c) return fail(VLG_EINVAL, "null context");
    if (which < 0 || which >= kNumTunables) return fail(VLG_EINVAL, "unknown tunable");
    if (value != 0 && !tunable_valid(which, value))
        return fail(VLG_EINVAL, std::string("bad value for ") + kTunableNames[which]);
    c->forced.v[which] = value;
    return VLG_OK;
}

int vlg_get_tunable(vlg_ctx *c, int which, int height, int width, int *value) {
    if (!c || !value) return fail(VLG_EINVAL, "null argument");
    if (which < 0 || which >= kNumTunables) return fail(VLG_EINVAL, "unknown tunable");
    *value = tuned_value(c, which, height, width);
    if (which == VLG_TUNE_NEAR_ROWS && *value == 0) *value = near_band_rows(make_geo(height, width));
    return VLG_OK;
}

int vlg_autotune(vlg_ctx *c, const vlg_formula *cf, const vlg_image *img, int iters, vlg_tune_report *out,
                 int max_out, int *n_out) {
    if (!c || !cf || !img || iters < 1 || !n_out) return fail(VLG_EINVAL, "bad argument");
    vlg_formula *f = const_cast<vlg_formula *>(cf);
    if (f->max_chan >= img->C) return fail(VLG_ESHAPE, "formula uses a channel the image lacks");
    DeviceGuard dg(c->device);
    *n_out = 0;
    std::vector<int> which(f->dag.outputs.size());
    for (size_t i = 0; i < which.size(); i++) which[i] = (int)i;
    const Geo g = make_geo(img->H, img->W);
    // volumes run the 3-D kernels, which have none of these tunables
    if (g.nwords == 0 || img->D > 1) return VLG_OK;
    // the step kinds of the schedule without segments, and a workspace that
    // fits the plan of every candidate the tuner may try
    const std::vector<int> fuse_cands = {1, 4, 8, 16}, lane_cands = {1, 2, 4, 8};
    const Plan &P1 = f->plan(which, Mode::Fused, 1, 1);
    bool has_near = false, has_arith = false;
    int local_steps = 0;
    for (const Step &st : P1.steps) {
        has_near |= st.kind == SK::Near;
        has_arith |= st.kind == SK::Arith;
        local_steps += st.kind == SK::Near || st.kind == SK::Logic;
    }
    const bool try_pj = P1.ccl_count > 0 && pj_shape_ok(img->H, img->W);
    const bool try_lanes = P1.ccl_count > 1;
    size_t need = 0;
    for (int fz : fuse_cands)
        for (int pj = 0; pj <= (int)try_pj; pj++)
            for (int ln : lane_cands)
                if (ln == 1 || try_lanes)
                    need = std::max(need, layout_for(f->plan(which, Mode::Fused, ln, fz), g, true, false, pj).total);
    std::vector<std::pair<int, std::vector<int>>> space;
    // the labelling schedule first (union-find, then the paper's pointer
    // jumping), then its tile height, then how many labellings run together
    if (try_pj) space.push_back({VLG_TUNE_CCL_ALGO, {VLG_CCL_UNION_FIND, VLG_CCL_POINTER_JUMPING}});
    if (P1.ccl_count > 0) space.push_back({VLG_TUNE_CCL_TILE_ROWS, {8, 16, 32}});
    if (try_lanes) space.push_back({VLG_TUNE_CCL_LANES, lane_cands});
    if (local_steps >= 2) space.push_back({VLG_TUNE_FUSE_HALO, fuse_cands});
    if (has_near) space.push_back({VLG_TUNE_NEAR_ROWS, {4, 8, 16, 32}});
    if (has_arith) space.push_back({VLG_TUNE_ARITH, {VLG_ARITH_COMPILED, VLG_ARITH_INTERPRETER}});
    int rc = ensure_ws(c, need);
    if (rc != VLG_OK) return rc;
    const std::pair<int, int> cls{log2_class(img->H), log2_class(img->W)};
    auto run_once = [&]() {
        const Plan &P = f->plan(which, Mode::Fused, tuned_value(c, VLG_TUNE_CCL_LANES, img->H, img->W),
                                tuned_value(c, VLG_TUNE_FUSE_HALO, img->H, img->W));
        const bool pj = P.ccl_count > 0 && ccl_algo(c, img->H, img->W) == VLG_CCL_POINTER_JUMPING;
        const Layout L = layout_for(P, g, true, false, pj);
        std::vector<uint64_t *> ext(which.size());
        for (size_t k = 0; k < which.size(); k++) ext[k] = (uint64_t *)((char *)c->ws + L.off_stage + k * L.mask_bytes);
        return enqueue_plan(c, P, img, L, ext);
    };
    return tune_loop(
        c, space, iters, run_once, [&](int w, int best) { c->tuned[cls].v[w] = best; }, out, max_out, n_out);
}

int vlg_autotune_batch(vlg_ctx *c, const vlg_formula *cf, const vlg_image *const *imgs, int n, int iters,
                       vlg_tune_report *out, int max_out, int *n_out) {
    if (!c || !cf || !imgs || n < 1 || iters < 1 || !n_out) return fail(VLG_EINVAL, "bad argument");
    vlg_formula *f = const_cast<vlg_formula *>(cf);
    const int dtype = imgs[0]->dtype;
    int64_t pixels = 0;
    for (int i = 0; i < n; i++) {
        if (!imgs[i]) return fail(VLG_EINVAL, "null image in batch");
        if (imgs[i]->D > 1) return fail(VLG_EINVAL, "volumes are not batched");
        if (f->max_chan >= imgs[i]->C) return fail(VLG_ESHAPE, "formula uses a channel an image lacks");
        if (imgs[i]->dtype != dtype) return fail(VLG_EINVAL, "batch autotuning needs one pixel type");
        if (imgs[i]->device != c->device) return fail(VLG_EINVAL, "image lives on another device");
        pixels += (int64_t)imgs[i]->H * imgs[i]->W;
    }
    DeviceGuard dg(c->device);
    *n_out = 0;
    const size_t nout = f->dag.outputs.size();
    std::vector<int> all(nout);
    for (size_t i = 0; i < nout; i++) all[i] = (int)i;
    const Plan &P = f->plan(all, Mode::Fused);
    std::vector<void *> outs((size_t)n * nout, nullptr);
    std::vector<int> idx((size_t)n);
    for (int i = 0; i < n; i++) idx[(size_t)i] = i;
    std::vector<std::pair<int, std::vector<int>>> space;
    if (P.ccl_count > 0) space.push_back({VLG_TUNE_CCL_TILE_ROWS, {8, 16, 32}});
    space.push_back({VLG_TUNE_BATCH_GRID, {1024, 2048, 4096, 8192}});
    const int saved_mode = c->mode;
    c->mode = VLG_MODE_FUSED;
    const std::pair<int, int> cls = batch_class(n, pixels);
    const int rc = tune_loop(
        c, space, iters, [&] { return run_batch(c, f, imgs, idx, outs.data(), VLG_PACKED64, VLG_DEVICE); },
        [&](int w, int best) { c->tuned_batch[cls].v[w] = best; }, out, max_out, n_out);
    c->mode = saved_mode;
    return rc;
}

int vlg_tune_save(vlg_ctx *c, const char *path) {
    if (!c || !path) return fail(VLG_EINVAL, "null argument");
    FILE *fp = std::fopen(path, "w");
    if (!fp) return fail(VLG_EINVAL, std::string("cannot write ") + path);
    for (int batch = 0; batch < 2; batch++)
        for (const auto &kv : batch ? c->tuned_batch : c->tuned)
            for (int w = 0; w < kNumTunables; w++)
                if (kv.second.v[w])
                    std::fprintf(fp,
                                 "{\"arch\": \"%s\", \"tunable\": \"%s%s\", \"h_class\": %d, \"w_class\": %d, "
                                 "\"value\": %d}\n",
                                 c->arch.c_str(), kTunableNames[w], batch ? "_batch" : "", kv.first.first,
                                 kv.first.second, kv.second.v[w]);
    std::fclose(fp);
    return VLG_OK;
}

int vlg_tune_load(vlg_ctx *c, const char *path) {
    if (!c || !path) return fail(VLG_EINVAL, "null argument");
    FILE *fp = std::fopen(path, "r");
    if (!fp) return fail(VLG_EINVAL, std::string("cannot read ") + path);
    char line[512];
    while (std::fgets(line, sizeof line, fp)) {
        char arch[64] = {0}, tun[64] = {0};
        int hc = 0, wc = 0, v = 0;
        if (std::sscanf(line, " {\"arch\": \"%63[^\"]\", \"tunable\": \"%63[^\"]\", \"h_class\": %d, \"w_class\": %d, "
                              "\"value\": %d}",
                        arch, tun, &hc, &wc, &v) != 5)
            continue;
        if (c->arch != arch) continue;
        const std::string name(tun);
        for (int w = 0; w < kNumTunables; w++) {
            if (!tunable_valid(w, v)) continue;
            if (name == kTunableNames[w]) c->tuned[{hc, wc}].v[w] = v;
            if (name == std::string(kTunableNames[w]) + "_batch") c->tuned_batch[{hc, wc}].v[w] = v;
        }
    }
    std::fclose(fp);
    return VLG_OK;
}

int vlg_ccl_read_counters(vlg_ctx *c, vlg_ccl_counters *out) {
    if (!c || !out) return fail(VLG_EINVAL, "null argument");
    DeviceGuard dg(c->device);
    unsigned long long h[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(h, c->counters, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    out->merge_unions = h[0];
    out->merge_retries = h[1];
    HIP_TRY(launch_fill_i64(c->stream, c->counters, 2, 0));
    out->launches_per_ccl = 4;
    out->pj_labellings = c->pj_labellings;
    out->pj_main_iterations = c->pj_iters;
    out->pj_rounds = c->pj_rounds;
    out->pj_launches = c->pj_launches;
    c->pj_labellings = c->pj_iters = c->pj_rounds = c->pj_launches = 0;
    return VLG_OK;
}

int vlg_ccl_labels_pj(vlg_ctx *c, const uint64_t *mask_dev, int height, int width, int reconnect_every,
                      int32_t *labels_dev, vlg_pj_stats *stats) {
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (!c || (!mask_dev && (int64_t)height * width > 0) || (!labels_dev && (int64_t)height * width > 0))
        return fail(VLG_EINVAL, "null argument");
    if (reconnect_every < 0 || reconnect_every > 64) return fail(VLG_EINVAL, "reconnect period must be 0..64");
    if (height < 0 || width < 0 || !pj_shape_ok(height, width))
        return fail(VLG_ESHAPE, "pointer-jumping labelling: rows and columns must stay below 65535");
    DeviceGuard dg(c->device);
    const Geo g = make_geo(height, width);
    if (g.nwords == 0) return VLG_OK;
    int rc = ensure_ws(c, pj_bytes(g));
    if (rc != VLG_OK) return rc;
    const PjWork w = pj_work(c->ws, g);
    const int k = reconnect_every ? reconnect_every : pj_reconnect_every(c, height, width);
    const int64_t it0 = c->pj_iters, r0 = c->pj_rounds, l0 = c->pj_launches;
    int at = 0;
    rc = pj_label(c, c->stream, g, MRef{mask_dev, 0ull}, w, k, at);
    if (stats) {
        stats->main_iterations = c->pj_iters - it0;
        stats->rounds = c->pj_rounds - r0;
        stats->launches = rc == VLG_OK ? c->pj_launches - l0 + 1 : 0;
    }
    if (rc != VLG_OK) return rc;
    HIP_TRY(launch_pj_labels(c->stream, g, w, at, labels_dev));
    return VLG_OK;
}

}  // extern "C"
