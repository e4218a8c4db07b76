// compiler.h -- formula front end and schedule builder (host side).
//
// Text (ImgQL subset, paper Sect. 3 Syntax) -> hash-consed DAG of SLCS
// operators (Sect. 2, Eq. def:syntax plus the derived interior, surrounded
// and grow) -> a linear schedule of kernel steps over 1-bit-packed masks.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace vlg {

enum class Op : uint8_t { True, False, Atom, Not, And, Or, Near, Interior, Reach, Surr, Grow, Arith };

enum Cmp : uint8_t { CMP_GT = 0, CMP_LT = 1, CMP_GE = 2, CMP_LE = 3 };

// Arithmetic atoms (the tool's built-in arithmetic, Sect. 3): a comparison
// of two numeric expressions evaluated pixel by pixel in float32, kept as one
// postfix program (the left side, then the right side).
enum ArOp : uint8_t { AR_CONST = 0, AR_CHAN, AR_PCT, AR_NEG, AR_ABS, AR_ADD, AR_SUB, AR_MUL, AR_DIV, AR_MIN, AR_MAX };
struct ArInstr {
    uint8_t op = AR_CONST;
    int32_t chan = 0;    // AR_CHAN: channel; AR_PCT: percentile channel
    float c = 0.f;       // AR_CONST
    double q = 0.0;      // AR_PCT: quantile
    int32_t pct = -1;    // AR_PCT in a plan: its percentile scalar
};
struct ArProgram {
    std::vector<ArInstr> ins;
    int32_t lhs_len = 0;
};
constexpr int kArMaxInstrs = 32;  // per program (both sides)
constexpr int kArMaxDepth = 8;    // evaluation stack per side
// arithmetic atoms evaluated by one launch (fused schedules): at most this
// many programs, instructions in all, and distinct channels read
constexpr int kArGroupProgs = 8, kArGroupInstrs = 96, kArGroupChans = 8;

struct Node {
    Op op;
    int32_t a = -1, b = -1;  // operand node ids
    // Atom: float32(img[chan]) CMP t; t = thr, or the percentile (pchan, q)
    int32_t chan = 0;
    uint8_t cmp = CMP_GT;
    uint8_t pct = 0;
    float thr = 0.f;
    int32_t pchan = 0;
    double q = 0.0;
    int32_t arith = -1;  // Arith: program index in Dag::ariths (cmp holds the comparison)
};

struct Dag {
    std::vector<Node> nodes;             // topologically ordered: operands first
    std::vector<int32_t> outputs;        // node id per `output` statement
    std::vector<std::string> output_names;
    std::vector<ArProgram> ariths;       // programs of Arith nodes (shared by equal ones)
    int64_t parsed_nodes = 0;            // operator applications before hash-consing
};

// Parse `src`; on failure returns false and sets err to "line L col C: msg".
bool parse_formula(const char *src, Dag &dag, std::string &err);

// ---------------------------------------------------------------- schedule

// An operand: a mask slot with an optional complement.  slot == kNone means
// the all-zero mask (all-one when inv is set).
constexpr int32_t kNone = -1;
inline constexpr int32_t ext_slot(int k) { return -2 - k; }  // caller output k
inline constexpr bool is_ext(int32_t s) { return s <= -2; }
inline constexpr int ext_index(int32_t s) { return -2 - s; }

struct Ref {
    int32_t slot = kNone;
    uint8_t inv = 0;
};

enum class SK : uint8_t {
    Pct,        // percentiles of channel `chan` at q[0..npq) -> pct scalars pct_out[]
    Atoms,      // up to kMaxAtoms thresholds of channel `chan` -> masks (one read)
    Logic,      // out = ((x ^ x.inv) OP (y ^ y.inv)) ^ inv_out ; OP = and/or
    Near,       // out = (N(x ^ x.inv) ^ inv_out) & (z ^ z.inv)
    CclLocal,   // tile-local union-find of b = x; seeds = N(y & z) & b
    CclMerge,   // cross-tile merge of the labelling of b = x
    CclFlag,    // propagate seed flags to the final roots
    CclGather,  // out = (y & z) | (pixels of b = x whose component has a seed)
    CclReseed,  // mark the components of the current labelling that meet the
                // seed mask x (= N(seeds) & b) for labelling user `user`
    Segment,    // consecutive Logic/Near steps run by one tile kernel with a
                // halo: Plan::segments[seg]
    Arith,      // out = lhs(pixel) CMP rhs(pixel): Plan::ariths[arith], CMP = op
};

// A fused segment (see SegProg in kernels.h; same opcodes and operand rules):
// inputs are loaded into registers first, members run in schedule order,
// each result read after the segment (or requested as an output) is stored
// right after it is computed.  Before slot allocation inputs/outputs hold SSA
// values, afterwards mask slots.
enum SegOpc : uint8_t { SOP_LOAD = 0, SOP_AND, SOP_OR, SOP_NEAR_AND, SOP_NEAR_OR, SOP_STORE };
constexpr uint8_t kSegNoReg = 255;
constexpr int kSegRegs = 16, kSegInstrs = 64, kSegPtrs = 32;
struct SegInstr {
    uint8_t op, dst, a, b, inv;  // LOAD: a = input index; STORE: dst = output index
};
struct Segment {
    std::vector<int32_t> inputs, outputs;
    std::vector<SegInstr> ins;
    int32_t nregs = 0, halo = 0;
};

constexpr int kMaxAtoms = 32;

// A percentile step selects up to this many quantiles of one channel in
// shared passes over it.
constexpr int kMaxPctPerStep = 4;

struct AtomEntry {
    uint8_t cmp = CMP_GT;
    uint8_t use_pct = 0;
    float thr = 0.f;
    int32_t pct = -1;    // pct scalar index if use_pct
    int32_t out = kNone; // output slot
};

struct Step {
    SK kind;
    int32_t out = kNone;
    Ref x, y, z;
    uint8_t op = 0;       // Logic: 0 = and, 1 = or
    uint8_t inv_out = 0;
    int32_t chan = 0;
    int npq = 0;                     // Pct: ranks of channel `chan` selected together
    double q[kMaxPctPerStep] = {};   //      quantiles
    int32_t pct_out[kMaxPctPerStep] = {-1, -1, -1, -1};  // their percentile scalars
    int natoms = 0;
    AtomEntry atoms[kMaxAtoms];
    int32_t user = 0;     // CclGather / CclReseed: which seed set of the labelling
    int32_t group = -1;   // consecutive Logic (or Near) steps of one group run
                          // as one batched launch; they never read each other
    int32_t lane = -1;    // labelling lane (>= 0): the steps of one concurrent
                          // region (same span) run on their lane's stream,
                          // lanes concurrently; -1: the main stream
    int32_t span = -1;    // consecutive steps with one span id are allocated
                          // mask slots as one step (batched group, region)
    int32_t seg = -1;     // Segment: index into Plan::segments
    int32_t arith = -1;   // Arith: index into Plan::ariths
};

// A labelling serves at most this many reach-type nodes with the same
// passable mask (one seed bit each in the per-block flag byte).
constexpr int kMaxCclUsers = 7;
constexpr int kMaxBatch = 16;

enum class Mode : uint8_t { PerOp = 0, Fused = 1 };

struct Plan {
    std::vector<Step> steps;
    int32_t nslots = 0;        // internal mask slots
    int32_t npct = 0;          // percentile scalars
    int32_t noutputs = 0;      // requested outputs (external slots 0..noutputs-1)
    int64_t ccl_count = 0;     // reachability labellings per evaluation
    int64_t ccl_reuse = 0;     // reach-type nodes served by an earlier labelling
    int32_t ccl_lanes = 1;     // labelling workspaces (concurrent labelling lanes)
    std::vector<int32_t> output_ids;  // formula output index per external slot
    std::vector<Segment> segments;
    std::vector<ArProgram> ariths;    // percentile leaves resolved to scalars
};

// Build the schedule evaluating formula outputs `which` (indices into
// dag.outputs); external slot k receives output which[k].  With lanes > 1
// (fused mode) up to `lanes` independent labellings of one scheduling round
// form a concurrent region, each on its own lane with its own labelling
// workspace.
// With fuse_halo >= 2 (fused mode) runs of consecutive Logic/Near steps
// become segments whose deepest chain of near steps is at most fuse_halo;
// fuse_halo <= 1 forms no segments.
constexpr int kMaxCclLanes = 8;
constexpr int kFuseHaloDefault = 1;  // no segments unless tuned or forced
inline bool valid_fuse_halo(int v) { return v == 1 || v == 2 || v == 4 || v == 8 || v == 16; }
Plan build_plan(const Dag &dag, const std::vector<int> &which, Mode mode, int lanes = 1, int fuse_halo = 1);

// Number of reach/surrounded/grow nodes and of atoms.
int64_t count_op(const Dag &dag, bool reach_like);

}  // namespace vlg
