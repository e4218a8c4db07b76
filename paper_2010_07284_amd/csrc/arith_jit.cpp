// arith_jit.cpp -- arithmetic atoms compiled into straight-line kernels.
//
// The interpreter kernel of arith.hip decodes every instruction of every
// program once per four pixels of a lane; on the 4096^2 arithmetic workload
// that decoding, not HBM, bounds it.  Here the programs of one launch become
// the source of a kernel of their own (every channel read once per pixel,
// then each program's operations as plain float expressions in postfix
// order, one temporary per stack entry), compiled with hipRTC for the
// device's architecture the first time a launch needs it and cached for the
// life of the process.  The arithmetic is the interpreter's: the same
// operations on the same operands in the same order, each rounded once
// (contraction off, IEEE division), so the results are bit-identical.
#include "arith_jit.h"

#include <hip/hiprtc.h>

#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

namespace vlg {
namespace {

constexpr int kJitThreads = 256;
constexpr int kJitWords = 4;  // mask words per wave, as in the interpreter

// op codes: ArOp of compiler.h
enum : uint8_t { JA_CONST = 0, JA_CHAN, JA_PCT, JA_NEG, JA_ABS, JA_ADD, JA_SUB, JA_MUL, JA_DIV, JA_MIN, JA_MAX };

const char *type_name(int dtype) { return dtype == 1 ? "unsigned char" : dtype == 2 ? "unsigned short" : "float"; }

std::string hexf(float x) {
    char b[64];
    std::snprintf(b, sizeof b, "%a", (double)x);
    std::string s = b;
    // %a of a finite float is exact; infinities and NaN need names
    if (s.find("inf") != std::string::npos) return x < 0 ? "(-__builtin_huge_valf())" : "__builtin_huge_valf()";
    if (s.find("nan") != std::string::npos) return "__builtin_nanf(\"\")";
    return "((float)" + s + ")";
}

// One side of a program, ins[k0, k1), as statements for pixel j: every
// operation gets a temporary of its own (named after `pre` and its
// instruction), and the host keeps the evaluation stack of the names.
// Returns the expression of the side's value, or "" when the side is not a
// well-formed postfix program.
std::string emit_side(const ArithGroup &a, int k0, int k1, const std::string &pre, std::string &out) {
    std::vector<std::string> st;
    for (int k = k0; k < k1; k++) {
        const ArithIns &in = a.ins[k];
        const std::string t = pre + std::to_string(k);
        switch (in.op) {
        case JA_CONST: st.push_back(hexf(in.c)); break;
        case JA_CHAN:
            if (in.idx < 0 || in.idx >= a.nch) return {};
            st.push_back("c" + std::to_string(in.idx) + "[j]");
            break;
        case JA_PCT:
            if (in.idx < 0) return {};
            st.push_back("pct[" + std::to_string(in.idx) + "]");
            break;
        case JA_NEG:
        case JA_ABS: {
            if (st.empty()) return {};
            const std::string x = st.back();
            st.pop_back();
            out += "            const float " + t + " = " + (in.op == JA_NEG ? "-(" + x + ")" : "__builtin_fabsf(" + x + ")") +
                   ";\n";
            st.push_back(t);
            break;
        }
        default: {
            if (st.size() < 2 || in.op > JA_MAX) return {};
            const std::string y = st.back();
            st.pop_back();
            const std::string x = st.back();
            st.pop_back();
            std::string e;
            switch (in.op) {
            case JA_ADD: e = x + " + " + y; break;
            case JA_SUB: e = x + " - " + y; break;
            case JA_MUL: e = x + " * " + y; break;
            case JA_DIV: e = x + " / " + y; break;
            case JA_MIN: e = y + " < " + x + " ? " + y + " : " + x; break;
            default: e = y + " > " + x + " ? " + y + " : " + x; break;
            }
            out += "            const float " + t + " = " + e + ";\n";
            st.push_back(t);
            break;
        }
        }
    }
    if (st.size() != 1) return {};
    // the side's value as a temporary (a constant or channel read included)
    const std::string r = pre + "v";
    out += "            const float " + r + " = " + st.back() + ";\n";
    return r;
}

}  // namespace

std::string arith_jit_source(const ArithGroup &a, int dtype) {
    if (a.n < 1 || a.n > kArithGroupProgs || a.nch < 0 || a.nch > kArithChans) return {};
    const std::string T = type_name(dtype);
    std::string s;
    s += "extern \"C\" __global__ void __launch_bounds__(" + std::to_string(kJitThreads) + ")\n";
    s += "vlg_arith(const " + T + " *__restrict__ img, long long chan_elems, long long nwords, int wpr,\n";
    s += "          unsigned int wpr_mul, unsigned int wpr_shift, unsigned long long tail,\n";
    s += "          const float *__restrict__ pct";
    for (int p = 0; p < a.n; p++) s += ", unsigned long long *__restrict__ o" + std::to_string(p);
    s += ") {\n";
    s += "#pragma clang fp contract(off)\n";
    s += "    const long long w0 = ((long long)blockIdx.x * " + std::to_string(kJitThreads / 64) +
         " + (threadIdx.x >> 6)) * " + std::to_string(kJitWords) + ";\n";
    s += "    if (w0 >= nwords) return;\n";
    s += "    const int lane = (int)(threadIdx.x & 63);\n";
    s += "    long long e[" + std::to_string(kJitWords) + "];\n";
    s += "    for (int j = 0; j < " + std::to_string(kJitWords) + "; j++) e[j] = (w0 + j < nwords ? w0 + j : w0) * 64 + lane;\n";
    for (int c = 0; c < a.nch; c++) {
        const std::string cs = std::to_string(c);
        s += "    float c" + cs + "[" + std::to_string(kJitWords) + "];\n";
        s += "    for (int j = 0; j < " + std::to_string(kJitWords) + "; j++) c" + cs + "[j] = (float)img[" +
             std::to_string((long long)a.ch[c]) + "LL * chan_elems + e[j]];\n";
    }
    s += "    const long long wi = w0 + (lane < " + std::to_string(kJitWords) + " ? lane : 0);\n";
    s += "    const bool store = lane < " + std::to_string(kJitWords) + " && wi < nwords;\n";
    s += "    unsigned long long keep = ~0ull;\n";
    s += "    if (store) {\n";
    s += "        const unsigned int row = (unsigned int)((((unsigned long long)__umulhi((unsigned int)wi, wpr_mul)) + "
         "(unsigned int)wi) >> wpr_shift);\n";
    s += "        if ((unsigned int)wi - row * (unsigned int)wpr == (unsigned int)wpr - 1) keep = tail;\n";
    s += "    }\n";
    for (int p = 0; p < a.n; p++) {
        if (!(0 <= a.lhs[p] && a.lhs[p] < a.rhs[p] && a.rhs[p] < a.end[p] && a.end[p] <= kArithGroupIns)) return {};
        const std::string ps = std::to_string(p);
        s += "    {  // program " + ps + "\n";
        s += "        unsigned long long mine = 0;\n";
        s += "#pragma unroll\n";
        s += "        for (int j = 0; j < " + std::to_string(kJitWords) + "; j++) {\n";
        std::string body;
        const std::string l = emit_side(a, a.lhs[p], a.rhs[p], "l" + ps + "_", body);
        const std::string r = emit_side(a, a.rhs[p], a.end[p], "r" + ps + "_", body);
        if (l.empty() || r.empty()) return {};
        s += body;
        const char *cmp = a.cmp[p] == 0 ? ">" : a.cmp[p] == 1 ? "<" : a.cmp[p] == 2 ? ">=" : "<=";
        s += "            const unsigned long long word = __ballot(" + l + " " + cmp + " " + r + ");\n";
        s += "            if (lane == j) mine = word;\n";
        s += "        }\n";
        s += "        if (store) o" + ps + "[wi] = mine & keep;\n";
        s += "    }\n";
    }
    s += "}\n";
    return s;
}

namespace {

struct JitEntry {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;  // nullptr: the source did not compile
    std::string err;
};

std::mutex g_jit_mu;
std::map<std::tuple<int, int, std::string>, JitEntry> g_jit;  // (device, dtype, source); kept for the process

}  // namespace

hipFunction_t arith_jit_function(int device, const ArithGroup &a, int dtype, std::string *err) {
    const std::string src = arith_jit_source(a, dtype);
    if (src.empty()) {
        if (err) *err = "program outside the compiled kernel's limits";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_jit_mu);
    const auto key = std::make_tuple(device, dtype, src);
    auto it = g_jit.find(key);
    if (it != g_jit.end()) {
        if (!it->second.fn && err) *err = it->second.err;
        return it->second.fn;
    }
    auto failed = [&](const std::string &why) -> hipFunction_t {
        JitEntry e;
        e.err = why;
        g_jit[key] = e;
        if (err) *err = why;
        return nullptr;
    };
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return failed("device properties");
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "vlg_arith.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
        return failed("hiprtcCreateProgram");
    const std::string archopt = "--offload-arch=" + arch;
    // the library's own flags: no contraction, IEEE division, no packed fp32
    // instructions (see the build script)
    const char *opts[] = {archopt.c_str(), "-O3", "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    if (rc != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        return failed("hiprtc: " + log);
    }
    size_t n = 0;
    hiprtcGetCodeSize(prog, &n);
    std::vector<char> code(n);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    JitEntry e;
    if (hipModuleLoadData(&e.mod, code.data()) != hipSuccess) return failed("module load");
    if (hipModuleGetFunction(&e.fn, e.mod, "vlg_arith") != hipSuccess) {
        e.fn = nullptr;
        return failed("module function");
    }
    g_jit[key] = e;
    return e.fn;
}

hipError_t launch_arith_jit(hipFunction_t fn, hipStream_t s, const Geo &g, const void *img, int64_t chan_elems,
                            const ArithGroup &a, const float *pct) {
    if (g.nwords == 0) return hipSuccess;
    const int64_t per_block = (int64_t)(kJitThreads / 64) * kJitWords;
    const int64_t blocks = (g.nwords + per_block - 1) / per_block;
    long long ce = chan_elems, nw = g.nwords;
    int wpr = g.wpr;
    unsigned int mul = g.wpr_mul, shift = g.wpr_shift;
    unsigned long long tail = g.tail;
    const void *im = img;
    const float *pc = pct;
    void *args[8 + kArithGroupProgs] = {(void *)&im, &ce, &nw, &wpr, &mul, &shift, &tail, (void *)&pc};
    uint64_t *outs[kArithGroupProgs];
    for (int p = 0; p < a.n; p++) {
        outs[p] = a.out[p];
        args[8 + p] = &outs[p];
    }
    return hipModuleLaunchKernel(fn, (unsigned)blocks, 1, 1, kJitThreads, 1, 1, 0, s, args, nullptr);
}

}  // namespace vlg
