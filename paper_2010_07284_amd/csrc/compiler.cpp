// compiler.cpp -- parser, hash-consing DAG builder and schedule builder.
//
// The front end follows the paper's tool (Sect. 3, Implementation details):
// parametric macros are expanded and identical sub-expressions are shared, so
// the result is a DAG of operator tasks.  Here the sharing is hash-consing on
// (operator, operands, parameters), with & and | commutative.
#include "compiler.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <unordered_map>

namespace vlg {
namespace {

// ---------------------------------------------------------------- lexer

enum TokKind { T_END, T_IDENT, T_NUM, T_STR, T_PUNCT };

struct Tok {
    TokKind k;
    std::string s;
    double num = 0.0;
    int line = 1, col = 1;
};

std::string at(int line, int col, const std::string &msg) {
    char buf[64];
    std::snprintf(buf, sizeof buf, "line %d col %d: ", line, col);
    return buf + msg;
}

bool lex(const char *src, std::vector<Tok> &out, std::string &err) {
    static const char *puncts[] = {">=.", "<=.", ">.", "<.", "(", ")", ",", "=", "!", "&", "|", "-", "+", "*", "/"};
    int line = 1, col = 1;
    size_t i = 0;
    auto step = [&](size_t n) {
        for (size_t k = 0; k < n; k++) {
            if (src[i] == '\n') {
                line++;
                col = 1;
            } else {
                col++;
            }
            i++;
        }
    };
    while (true) {
        char c = src[i];
        if (c == ' ' || c == '\t' || c == '\r' || c == '\n' || c == ';') {
            step(1);
            continue;
        }
        if (c == '/' && src[i + 1] == '/') {
            while (src[i] && src[i] != '\n') step(1);
            continue;
        }
        Tok t;
        t.line = line;
        t.col = col;
        if (c == 0) {
            t.k = T_END;
            out.push_back(t);
            return true;
        }
        if (std::isalpha((unsigned char)c) || c == '_') {
            size_t n = 0;
            while (std::isalnum((unsigned char)src[i + n]) || src[i + n] == '_') n++;
            t.k = T_IDENT;
            t.s.assign(src + i, n);
            step(n);
        } else if (std::isdigit((unsigned char)c) || (c == '.' && std::isdigit((unsigned char)src[i + 1]))) {
            char *end = nullptr;
            t.k = T_NUM;
            t.num = std::strtod(src + i, &end);
            t.s.assign(src + i, (size_t)(end - (src + i)));
            step((size_t)(end - (src + i)));
        } else if (c == '"') {
            size_t n = 1;
            while (src[i + n] && src[i + n] != '"' && src[i + n] != '\n') n++;
            if (src[i + n] != '"') {
                err = at(line, col, "unterminated string");
                return false;
            }
            t.k = T_STR;
            t.s.assign(src + i + 1, n - 1);
            step(n + 1);
        } else {
            bool ok = false;
            for (const char *p : puncts) {
                size_t n = std::strlen(p);
                if (std::strncmp(src + i, p, n) == 0) {
                    t.k = T_PUNCT;
                    t.s = p;
                    step(n);
                    ok = true;
                    break;
                }
            }
            if (!ok) {
                err = at(line, col, std::string("unexpected character '") + c + "'");
                return false;
            }
        }
        out.push_back(std::move(t));
    }
}

// ---------------------------------------------------------------- hash-consing

struct Key {
    uint8_t op, cmp, pct;
    int32_t a, b, chan, pchan;
    uint32_t thr_bits;
    uint64_t q_bits;
    bool operator==(const Key &o) const {
        return op == o.op && cmp == o.cmp && pct == o.pct && a == o.a && b == o.b &&
               chan == o.chan && pchan == o.pchan && thr_bits == o.thr_bits && q_bits == o.q_bits;
    }
};

struct KeyHash {
    size_t operator()(const Key &k) const {
        uint64_t h = 1469598103934665603ull;
        auto mix = [&](uint64_t v) {
            h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
        };
        mix(k.op | (uint64_t)k.cmp << 8 | (uint64_t)k.pct << 16);
        mix((uint32_t)k.a | (uint64_t)(uint32_t)k.b << 32);
        mix((uint32_t)k.chan | (uint64_t)(uint32_t)k.pchan << 32);
        mix(k.thr_bits);
        mix(k.q_bits);
        return (size_t)h;
    }
};

struct Builder {
    Dag &dag;
    std::unordered_map<Key, int32_t, KeyHash> memo;
    explicit Builder(Dag &d) : dag(d) {}

    int32_t make(Node n) {
        dag.parsed_nodes++;
        if ((n.op == Op::And || n.op == Op::Or) && n.a > n.b) std::swap(n.a, n.b);
        Key k;
        std::memset(&k, 0, sizeof k);
        k.op = (uint8_t)n.op;
        k.a = n.a;
        k.b = n.b;
        if (n.op == Op::Arith) {
            k.cmp = n.cmp;
            k.chan = n.arith;  // interned: equal programs share one index
        }
        if (n.op == Op::Atom) {
            k.cmp = n.cmp;
            k.pct = n.pct;
            k.chan = n.chan;
            if (n.pct) {
                k.pchan = n.pchan;
                std::memcpy(&k.q_bits, &n.q, sizeof n.q);
            } else {
                std::memcpy(&k.thr_bits, &n.thr, sizeof n.thr);
            }
        }
        auto it = memo.find(k);
        if (it != memo.end()) return it->second;
        int32_t id = (int32_t)dag.nodes.size();
        dag.nodes.push_back(n);
        memo.emplace(k, id);
        return id;
    }

    // index of an arithmetic program, equal programs sharing one
    std::map<std::string, int32_t> arith_ids;
    int32_t intern(const ArProgram &pr) {
        std::string key((const char *)&pr.lhs_len, sizeof pr.lhs_len);
        for (const ArInstr &in : pr.ins) {
            key.append((const char *)&in.op, sizeof in.op);
            key.append((const char *)&in.chan, sizeof in.chan);
            key.append((const char *)&in.c, sizeof in.c);
            key.append((const char *)&in.q, sizeof in.q);
        }
        auto it = arith_ids.find(key);
        if (it != arith_ids.end()) return it->second;
        const int32_t id = (int32_t)dag.ariths.size();
        dag.ariths.push_back(pr);
        arith_ids.emplace(key, id);
        return id;
    }
};

// ---------------------------------------------------------------- parser

bool is_builtin(const std::string &s) {
    static const char *names[] = {"let",  "output",     "true", "false", "intensity", "percentile", "img",
                                  "near", "N",          "interior", "reach", "surrounded", "grow", "touch",
                                  "abs",  "min",        "max"};
    for (const char *n : names)
        if (s == n) return true;
    return false;
}

struct Macro {
    std::vector<std::string> params;
    size_t body_begin = 0, body_end = 0;
    int def_pos = 0;
};

struct Binding {
    int pos;
    int32_t node;   // constant binding
    int macro;      // >= 0 for a macro binding
};

struct Parser {
    const std::vector<Tok> &t;
    Builder &B;
    size_t p = 0;
    bool failed = false;
    std::string err;
    bool dry = false;  // syntax check of a macro body: build no nodes
    std::unordered_map<std::string, std::vector<Binding>> binds;
    std::vector<Macro> macros;
    const std::vector<std::string> *env_names = nullptr;
    const std::vector<int32_t> *env_nodes = nullptr;
    int limit = INT_MAX;  // only bindings with pos < limit are visible

    Parser(const std::vector<Tok> &toks, Builder &b) : t(toks), B(b) {}

    const Tok &cur() const { return t[p]; }
    void fail(const std::string &msg) {
        if (failed) return;
        failed = true;
        err = at(cur().line, cur().col, msg);
    }
    bool is_punct(const char *s) const { return cur().k == T_PUNCT && cur().s == s; }
    bool accept(const char *s) {
        if (is_punct(s)) {
            p++;
            return true;
        }
        return false;
    }
    void expect(const char *s) {
        if (!accept(s)) fail(std::string("expected '") + s + "'");
    }
    int32_t make(const Node &n) { return dry ? 0 : B.make(n); }

    const Binding *lookup(const std::string &name) const {
        auto it = binds.find(name);
        if (it == binds.end()) return nullptr;
        for (auto r = it->second.rbegin(); r != it->second.rend(); ++r)
            if (r->pos < limit) return &*r;
        return nullptr;
    }

    int read_channel() {
        if (cur().k != T_NUM || cur().s.find_first_not_of("0123456789") != std::string::npos) {
            fail("expected channel index");
            return 0;
        }
        int c = (int)cur().num;
        p++;
        return c;
    }

    void img_channel(int32_t &chan, bool allow_default) {
        if (cur().k != T_IDENT || cur().s != "img") {
            fail("expected 'img'");
            return;
        }
        p++;
        chan = 0;
        if (accept(",")) {
            chan = read_channel();
        } else if (!allow_default) {
            fail("expected ','");
        }
    }

    // ---- arithmetic atoms: a numeric expression (postfix into `out`)
    // followed by a comparison and another numeric expression.  The parse is
    // speculative: false (the caller backs up) when the tokens here are not
    // a numeric expression.
    bool num_factor(std::vector<ArInstr> &out) {
        if (failed) return false;
        if (accept("-")) {
            if (!num_factor(out)) return false;
            ArInstr in;
            in.op = AR_NEG;
            out.push_back(in);
            return true;
        }
        if (accept("(")) return num_expr(out) && accept(")");
        if (cur().k == T_NUM) {
            ArInstr in;
            in.op = AR_CONST;
            in.c = (float)cur().num;  // read as double, rounded once to float32
            p++;
            out.push_back(in);
            return true;
        }
        if (cur().k != T_IDENT) return false;
        const std::string id = cur().s;
        ArInstr in;
        if (id == "intensity") {
            p++;
            if (!accept("(")) return false;
            in.op = AR_CHAN;
            img_channel(in.chan, true);
            if (failed || !accept(")")) return false;
            out.push_back(in);
            return true;
        }
        if (id == "percentile") {
            p++;
            if (!accept("(")) return false;
            in.op = AR_PCT;
            img_channel(in.chan, false);
            if (failed || !accept(",") || cur().k != T_NUM) return false;
            in.q = cur().num;
            p++;
            if (!accept(")")) return false;
            out.push_back(in);
            return true;
        }
        if (id == "abs" || id == "min" || id == "max") {
            p++;
            if (!accept("(") || !num_expr(out)) return false;
            if (id != "abs" && !(accept(",") && num_expr(out))) return false;
            if (!accept(")")) return false;
            in.op = id == "abs" ? AR_ABS : id == "min" ? AR_MIN : AR_MAX;
            out.push_back(in);
            return true;
        }
        return false;
    }
    bool num_term(std::vector<ArInstr> &out) {
        if (!num_factor(out)) return false;
        for (;;) {
            uint8_t op;
            if (accept("*")) op = AR_MUL;
            else if (accept("/")) op = AR_DIV;
            else return true;
            if (!num_factor(out)) return false;
            ArInstr in;
            in.op = op;
            out.push_back(in);
        }
    }
    bool num_expr(std::vector<ArInstr> &out) {
        if (!num_term(out)) return false;
        for (;;) {
            uint8_t op;
            if (accept("+")) op = AR_ADD;
            else if (accept("-")) op = AR_SUB;
            else return true;
            if (!num_term(out)) return false;
            ArInstr in;
            in.op = op;
            out.push_back(in);
        }
    }
    static int stack_depth(const std::vector<ArInstr> &v) {
        int d = 0, m = 0;
        for (const ArInstr &in : v) {
            if (in.op == AR_CONST || in.op == AR_CHAN || in.op == AR_PCT) d++;
            else if (in.op != AR_NEG && in.op != AR_ABS) d--;
            m = std::max(m, d);
        }
        return m;
    }
    bool at_cmp() const {
        return cur().k == T_PUNCT && (cur().s == ">." || cur().s == "<." || cur().s == ">=." || cur().s == "<=.");
    }
    // An atom at the current position (matched = true), or nothing consumed.
    // The paper's plain atom, intensity(img[, c]) CMP constant-or-percentile,
    // stays an Atom node; any other comparison becomes an Arith node.
    int32_t arith_atom(bool &matched) {
        matched = false;
        const size_t save = p;
        std::vector<ArInstr> lhs;
        if (!num_expr(lhs) || !at_cmp()) {
            if (!failed) p = save;
            return -1;
        }
        matched = true;
        const std::string c = cur().s;
        p++;
        const uint8_t cmp = c == ">=." ? CMP_GE : c == "<=." ? CMP_LE : c == ">." ? CMP_GT : CMP_LT;
        std::vector<ArInstr> rhs;
        if (!num_expr(rhs)) {
            fail("expected a numeric expression after the comparison");
            return -1;
        }
        Node n;
        n.cmp = cmp;
        if (lhs.size() == 1 && lhs[0].op == AR_CHAN) {
            const bool konst = rhs.size() == 1 && rhs[0].op == AR_CONST;
            const bool neg = rhs.size() == 2 && rhs[0].op == AR_CONST && rhs[1].op == AR_NEG;
            if (konst || neg || (rhs.size() == 1 && rhs[0].op == AR_PCT)) {
                n.op = Op::Atom;
                n.chan = lhs[0].chan;
                if (rhs[0].op == AR_PCT) {
                    n.pct = 1;
                    n.pchan = rhs[0].chan;
                    n.q = rhs[0].q;
                } else {
                    n.thr = neg ? -rhs[0].c : rhs[0].c;
                }
                return make(n);
            }
        }
        if (lhs.size() + rhs.size() > (size_t)kArMaxInstrs || stack_depth(lhs) > kArMaxDepth ||
            stack_depth(rhs) > kArMaxDepth) {
            fail("arithmetic expression too large (at most 32 terms and operators, nesting depth 8 per side)");
            return -1;
        }
        {
            std::vector<int32_t> chans;
            for (const std::vector<ArInstr> *side : {&lhs, &rhs})
                for (const ArInstr &in : *side)
                    if (in.op == AR_CHAN && std::find(chans.begin(), chans.end(), in.chan) == chans.end())
                        chans.push_back(in.chan);
            if (chans.size() > 8) {
                fail("an arithmetic atom reads at most 8 distinct channels");
                return -1;
            }
        }
        ArProgram pr;
        pr.ins = lhs;
        pr.ins.insert(pr.ins.end(), rhs.begin(), rhs.end());
        pr.lhs_len = (int32_t)lhs.size();
        n.op = Op::Arith;
        n.arith = dry ? 0 : B.intern(pr);
        return make(n);
    }

    int32_t call(Op op, int nargs) {
        expect("(");
        int32_t a = expr(), b = -1;
        if (nargs == 2) {
            expect(",");
            b = expr();
        }
        expect(")");
        if (failed) return -1;
        Node n;
        n.op = op;
        n.a = a;
        n.b = b;
        return make(n);
    }

    int32_t expand(const Macro &m, const std::vector<int32_t> &args) {
        size_t save_p = p;
        auto save_names = env_names;
        auto save_nodes = env_nodes;
        int save_limit = limit;
        p = m.body_begin;
        env_names = &m.params;
        env_nodes = &args;
        limit = m.def_pos;
        int32_t r = expr();
        if (!failed && p != m.body_end) fail("internal: macro body length mismatch");
        p = save_p;
        env_names = save_names;
        env_nodes = save_nodes;
        limit = save_limit;
        return r;
    }

    int32_t primary() {
        if (failed) return -1;
        bool matched = false;
        const int32_t at = arith_atom(matched);
        if (matched || failed) return at;
        if (accept("(")) {
            int32_t e = expr();
            expect(")");
            return e;
        }
        if (cur().k != T_IDENT) {
            fail("expected an expression");
            return -1;
        }
        std::string id = cur().s;
        p++;
        Node n;
        if (id == "true") {
            n.op = Op::True;
            return make(n);
        }
        if (id == "false") {
            n.op = Op::False;
            return make(n);
        }
        if (id == "intensity" || id == "percentile" || id == "abs" || id == "min" || id == "max") {
            p--;
            fail("expected a comparison '>.', '<.', '>=.' or '<=.' after a numeric expression");
            return -1;
        }
        if (id == "touch") {
            // touch(a, b) = a & reach(b, a): the regions of a in contact with b
            expect("(");
            const int32_t a = expr();
            expect(",");
            const int32_t b = expr();
            expect(")");
            if (failed) return -1;
            Node r;
            r.op = Op::Reach;
            r.a = b;  // seeds
            r.b = a;  // passable
            Node n;
            n.op = Op::And;
            n.a = a;
            n.b = make(r);
            return make(n);
        }
        if (id == "near" || id == "N") return call(Op::Near, 1);
        if (id == "interior") return call(Op::Interior, 1);
        if (id == "reach") return call(Op::Reach, 2);
        if (id == "surrounded") return call(Op::Surr, 2);
        if (id == "grow") return call(Op::Grow, 2);
        if (is_builtin(id)) {
            p--;
            fail("unexpected keyword");
            return -1;
        }
        if (env_names) {
            for (size_t i = 0; i < env_names->size(); i++)
                if ((*env_names)[i] == id) return (*env_nodes)[i];
        }
        const Binding *bd = lookup(id);
        if (!bd) {
            p--;
            fail("undefined name '" + id + "'");
            return -1;
        }
        if (bd->macro < 0) return bd->node;
        const Macro &m = macros[(size_t)bd->macro];
        std::vector<int32_t> args;
        expect("(");
        for (size_t i = 0; i < m.params.size() && !failed; i++) {
            if (i > 0) expect(",");
            args.push_back(expr());
        }
        expect(")");
        if (failed) return -1;
        if (dry) return 0;
        return expand(m, args);
    }

    int32_t unary() {
        if (failed) return -1;
        if (accept("!")) {
            int32_t a = unary();
            if (failed) return -1;
            Node n;
            n.op = Op::Not;
            n.a = a;
            return make(n);
        }
        return primary();
    }

    int32_t binary_chain(bool is_or) {
        int32_t l = is_or ? binary_chain(false) : unary();
        while (!failed && accept(is_or ? "|" : "&")) {
            int32_t r = is_or ? binary_chain(false) : unary();
            if (failed) return -1;
            Node n;
            n.op = is_or ? Op::Or : Op::And;
            n.a = l;
            n.b = r;
            l = make(n);
        }
        return l;
    }

    int32_t expr() { return binary_chain(true); }

    void program() {
        int pos = 0;
        while (!failed && cur().k != T_END) {
            if (cur().k != T_IDENT || (cur().s != "let" && cur().s != "output")) {
                fail("expected 'let' or 'output'");
                return;
            }
            if (cur().s == "let") {
                p++;
                if (cur().k != T_IDENT) {
                    fail("expected a name after 'let'");
                    return;
                }
                std::string name = cur().s;
                if (is_builtin(name)) {
                    fail("cannot redefine a built-in name");
                    return;
                }
                p++;
                Macro m;
                if (accept("(")) {
                    do {
                        if (m.params.size() >= 16) {
                            fail("too many parameters");
                            return;
                        }
                        if (cur().k != T_IDENT) {
                            fail("expected a parameter name");
                            return;
                        }
                        m.params.push_back(cur().s);
                        p++;
                    } while (accept(","));
                    expect(")");
                }
                expect("=");
                if (failed) return;
                if (!m.params.empty()) {
                    // check the body now (names resolve to earlier bindings);
                    // it is expanded at each call
                    m.body_begin = p;
                    m.def_pos = pos;
                    std::vector<int32_t> dummy(m.params.size(), 0);
                    env_names = &m.params;
                    env_nodes = &dummy;
                    dry = true;
                    expr();
                    dry = false;
                    env_names = nullptr;
                    env_nodes = nullptr;
                    if (failed) return;
                    m.body_end = p;
                    macros.push_back(m);
                    binds[name].push_back(Binding{pos, -1, (int)macros.size() - 1});
                } else {
                    int32_t node = expr();
                    if (failed) return;
                    binds[name].push_back(Binding{pos, node, -1});
                }
                pos++;
            } else {
                p++;
                if (cur().k != T_STR) {
                    fail("expected a quoted output name");
                    return;
                }
                std::string oname = cur().s;
                p++;
                int32_t node = expr();
                if (failed) return;
                B.dag.outputs.push_back(node);
                B.dag.output_names.push_back(oname);
            }
        }
    }
};

}  // namespace

bool parse_formula(const char *src, Dag &dag, std::string &err) {
    std::vector<Tok> toks;
    if (!lex(src, toks, err)) return false;
    Builder B(dag);
    Parser P(toks, B);
    P.program();
    if (P.failed) {
        err = P.err;
        return false;
    }
    return true;
}

int64_t count_op(const Dag &dag, bool reach_like) {
    int64_t n = 0;
    for (const Node &x : dag.nodes) {
        if (reach_like && (x.op == Op::Reach || x.op == Op::Surr || x.op == Op::Grow)) n++;
        if (!reach_like && (x.op == Op::Atom || x.op == Op::Arith)) n++;
    }
    return n;
}

// ---------------------------------------------------------------- schedule

namespace {

struct Lower {
    const Dag &dag;
    Mode mode;
    std::vector<Step> steps;   // operand/out fields hold SSA value ids
    int32_t nssa = 0;
    std::vector<Ref> val;      // per node
    std::vector<char> have;
    std::map<std::pair<int32_t, uint64_t>, int32_t> pct_memo;
    int32_t npct = 0;
    // epilogue fusion: a near/interior node whose only consumer is & or | is
    // not emitted on its own; the consumer runs it with itself as epilogue
    std::vector<int32_t> uses, consumer;
    std::vector<char> deferred;
    std::vector<Ref> dx;
    std::vector<uint8_t> dinv;
    std::vector<ArProgram> ariths;  // programs of the Arith steps, percentile leaves resolved

    Lower(const Dag &d, Mode m)
        : dag(d), mode(m), val(d.nodes.size()), have(d.nodes.size(), 0), uses(d.nodes.size(), 0),
          consumer(d.nodes.size(), -1), deferred(d.nodes.size(), 0), dx(d.nodes.size()), dinv(d.nodes.size(), 0) {}

    bool can_defer(int32_t id) const {
        const int32_t c = consumer[(size_t)id];
        return mode == Mode::Fused && uses[(size_t)id] == 1 && c >= 0 &&
               (dag.nodes[(size_t)c].op == Op::And || dag.nodes[(size_t)c].op == Op::Or);
    }
    Ref materialize(int32_t id) {
        if (deferred[(size_t)id]) {
            val[(size_t)id] = near(dx[(size_t)id], dinv[(size_t)id], Const(1));
            deferred[(size_t)id] = 0;
        }
        return val[(size_t)id];
    }

    int32_t fresh() { return nssa++; }

    static Ref R(int32_t s, int inv = 0) {
        Ref r;
        r.slot = s;
        r.inv = (uint8_t)(inv & 1);
        return r;
    }
    static Ref Const(int v) { return R(kNone, v); }
    static Ref Neg(Ref r) {
        r.inv ^= 1;
        return r;
    }

    Step &emit(SK k) {
        steps.emplace_back();
        steps.back().kind = k;
        return steps.back();
    }

    int32_t pct_of(int32_t chan, double q) {
        uint64_t qb;
        std::memcpy(&qb, &q, sizeof q);
        auto key = std::make_pair(chan, qb);
        auto it = pct_memo.find(key);
        if (it != pct_memo.end()) return it->second;
        int32_t idx = npct++;
        Step &s = emit(SK::Pct);
        s.chan = chan;
        s.npq = 1;
        s.q[0] = q;
        s.pct_out[0] = idx;
        pct_memo.emplace(key, idx);
        return idx;
    }

    // an arithmetic atom: its percentile leaves first, then one Arith step
    Ref arith(int32_t id) {
        const Node &n = dag.nodes[(size_t)id];
        ArProgram pr = dag.ariths[(size_t)n.arith];
        for (ArInstr &in : pr.ins)
            if (in.op == AR_PCT) in.pct = pct_of(in.chan, in.q);
        Step &s = emit(SK::Arith);
        s.op = n.cmp;
        s.arith = (int32_t)ariths.size();
        ariths.push_back(std::move(pr));
        s.out = fresh();
        return R(s.out);
    }

    // materialise (x OP y) ^ inv_out
    Ref logic(Ref x, Ref y, int op, int inv_out = 0) {
        Step &s = emit(SK::Logic);
        s.x = x;
        s.y = y;
        s.op = (uint8_t)op;
        s.inv_out = (uint8_t)inv_out;
        s.out = fresh();
        return R(s.out);
    }
    Ref near(Ref x, int inv_out, Ref z, int zop = 0) {
        Step &s = emit(SK::Near);
        s.x = x;
        s.inv_out = (uint8_t)inv_out;
        s.z = z;
        s.op = (uint8_t)zop;
        s.out = fresh();
        return R(s.out);
    }
    // G = seeds | (pixels of b whose component meets N(seeds)), seeds = y & z
    Ref reach_core(Ref b, Ref y, Ref z) {
        Step &l = emit(SK::CclLocal);
        l.x = b;
        l.y = y;
        l.z = z;
        Step &m = emit(SK::CclMerge);
        m.x = b;
        emit(SK::CclFlag);
        Step &g = emit(SK::CclGather);
        g.x = b;
        g.y = y;
        g.z = z;
        g.out = fresh();
        return R(g.out);
    }

    // per-operator schedule: every node materialised by its own kernels
    Ref perop(int32_t id) {
        const Node &n = dag.nodes[(size_t)id];
        const Ref one = Const(1);
        switch (n.op) {
        case Op::True:
        case Op::False:
            return logic(Const(n.op == Op::True), one, 0);
        case Op::Atom: {
            int32_t pi = n.pct ? pct_of(n.pchan, n.q) : -1;
            Step &s = emit(SK::Atoms);
            s.chan = n.chan;
            s.natoms = 1;
            s.atoms[0].cmp = n.cmp;
            s.atoms[0].use_pct = n.pct;
            s.atoms[0].thr = n.thr;
            s.atoms[0].pct = pi;
            s.atoms[0].out = fresh();
            return R(s.atoms[0].out);
        }
        case Op::Arith:
            return arith(id);
        case Op::Not:
            return logic(Neg(val[(size_t)n.a]), one, 0);
        case Op::And:
        case Op::Or:
            return logic(val[(size_t)n.a], val[(size_t)n.b], n.op == Op::Or);
        case Op::Near:
            return near(val[(size_t)n.a], 0, one);
        case Op::Interior: {
            Ref t = logic(Neg(val[(size_t)n.a]), one, 0);
            Ref u = near(t, 0, one);
            return logic(Neg(u), one, 0);
        }
        case Op::Reach: {
            Ref g = reach_core(val[(size_t)n.b], val[(size_t)n.a], one);
            return near(g, 0, one);
        }
        case Op::Grow: {
            Ref a = val[(size_t)n.a], b = val[(size_t)n.b];
            Ref g = reach_core(b, a, one);
            Ref r = near(g, 0, one);
            Ref t = logic(b, r, 0);
            return logic(a, t, 1);
        }
        case Op::Surr: {
            Ref a = val[(size_t)n.a], b = val[(size_t)n.b];
            Ref na = logic(Neg(a), one, 0);
            Ref nb = logic(Neg(b), one, 0);
            Ref e = logic(na, nb, 0);
            Ref g = reach_core(nb, e, one);
            Ref r = near(g, 0, one);
            Ref nr = logic(Neg(r), one, 0);
            return logic(a, nr, 0);
        }
        }
        return Const(0);
    }

    // fused schedule: negations folded into consumers, derived operators run
    // on complemented operands without materialising them
    Ref fused(int32_t id) {
        const Node &n = dag.nodes[(size_t)id];
        const Ref one = Const(1);
        auto is_const = [](Ref r) { return r.slot == kNone; };
        switch (n.op) {
        case Op::True:
            return Const(1);
        case Op::False:
            return Const(0);
        case Op::Atom:
            return val[(size_t)id];  // made by the atom groups
        case Op::Arith:
            return arith(id);
        case Op::Not:
            return Neg(val[(size_t)n.a]);
        case Op::And:
        case Op::Or: {
            const bool isor = n.op == Op::Or;
            if (deferred[(size_t)n.a] || deferred[(size_t)n.b]) {
                const int32_t d = deferred[(size_t)n.a] ? n.a : n.b, o = d == n.a ? n.b : n.a;
                const Ref other = materialize(o);
                if (!is_const(other)) {
                    deferred[(size_t)d] = 0;
                    return near(dx[(size_t)d], dinv[(size_t)d], other, isor);
                }
                materialize(d);
            }
            Ref a = val[(size_t)n.a], b = val[(size_t)n.b];
            // x & 0 = 0, x & 1 = x, x | 1 = 1, x | 0 = x
            if (is_const(a)) std::swap(a, b);
            if (is_const(b)) return (b.inv == (isor ? 1 : 0)) ? b : a;
            return logic(a, b, isor);
        }
        case Op::Near: {
            Ref a = val[(size_t)n.a];
            if (is_const(a)) return a;  // N 0 = 0, N 1 = 1
            if (can_defer(id)) {
                deferred[(size_t)id] = 1;
                dx[(size_t)id] = a;
                dinv[(size_t)id] = 0;
                return Ref();
            }
            return near(a, 0, one);
        }
        case Op::Interior: {
            Ref a = val[(size_t)n.a];
            if (is_const(a)) return a;
            if (can_defer(id)) {
                deferred[(size_t)id] = 1;
                dx[(size_t)id] = Neg(a);
                dinv[(size_t)id] = 1;
                return Ref();
            }
            return near(Neg(a), 1, one);  // !N!a
        }
        case Op::Reach: {
            Ref a = val[(size_t)n.a], b = val[(size_t)n.b];
            if (is_const(a)) return a;                   // rho 0[b] = 0, rho 1[b] = 1
            if (is_const(b) && b.inv == 0) return near(a, 0, one);  // rho a[0] = N a
            Ref g = reach_core(b, a, one);
            return near(g, 0, one);
        }
        case Op::Grow: {
            Ref a = val[(size_t)n.a], b = val[(size_t)n.b];
            if (is_const(a)) return a;
            if (is_const(b) && b.inv == 0) return a;     // grow(a, 0) = a
            return reach_core(b, a, one);                // a | Z
        }
        case Op::Surr: {
            // a & !rho(!a & !b)[!b]
            Ref a = val[(size_t)n.a], b = val[(size_t)n.b];
            if (is_const(a) && a.inv == 0) return a;     // surrounded(0, b) = 0
            Ref g = reach_core(Neg(b), Neg(a), Neg(b));
            return near(g, 1, a);
        }
        }
        return Const(0);
    }

    void atom_groups(const std::vector<char> &need) {
        // one pass per channel reads the channel once for all its atoms
        std::map<int32_t, std::vector<int32_t>> by_chan;
        for (size_t i = 0; i < dag.nodes.size(); i++)
            if (need[i] && dag.nodes[i].op == Op::Atom) by_chan[dag.nodes[i].chan].push_back((int32_t)i);
        for (auto &kv : by_chan)
            for (int32_t id : kv.second)
                if (dag.nodes[(size_t)id].pct) pct_of(dag.nodes[(size_t)id].pchan, dag.nodes[(size_t)id].q);
        for (auto &kv : by_chan) {
            const auto &ids = kv.second;
            for (size_t i = 0; i < ids.size(); i += kMaxAtoms) {
                Step &s = emit(SK::Atoms);
                s.chan = kv.first;
                for (size_t j = i; j < ids.size() && j < i + kMaxAtoms; j++) {
                    const Node &n = dag.nodes[(size_t)ids[j]];
                    AtomEntry &e = s.atoms[s.natoms++];
                    e.cmp = n.cmp;
                    e.use_pct = n.pct;
                    e.thr = n.thr;
                    e.pct = n.pct ? pct_of(n.pchan, n.q) : -1;
                    e.out = fresh();
                    val[(size_t)ids[j]] = R(e.out);
                    have[(size_t)ids[j]] = 1;
                }
            }
        }
    }
};



// Reorder the fused schedule level by level: every ready Logic (resp. Near)
// step joins one batched launch, and a reach labelling whose passable mask is
// the one of the labelling emitted last is reused (reseed + gather) instead of
// being recomputed.  Works on SSA ids, before slot allocation.
constexpr int64_t kPctBase = int64_t(1) << 40;

void schedule_fused(Lower &L, int lanes) {
    struct Unit {
        int first = 0, count = 1;
        bool ccl = false;
        std::vector<int64_t> reads, writes;
    };
    auto refs_of = [&L](const Step &st, std::vector<int64_t> &rd, std::vector<int64_t> &wr) {
        for (const Ref *r : {&st.x, &st.y, &st.z})
            if (r->slot != kNone) rd.push_back(r->slot);
        if (st.kind == SK::Atoms) {
            for (int j = 0; j < st.natoms; j++) {
                wr.push_back(st.atoms[j].out);
                if (st.atoms[j].use_pct) rd.push_back(kPctBase + st.atoms[j].pct);
            }
        } else if (st.kind == SK::Pct) {
            for (int j = 0; j < st.npq; j++) wr.push_back(kPctBase + st.pct_out[j]);
        } else if (st.kind == SK::Arith) {
            wr.push_back(st.out);
            for (const ArInstr &in : L.ariths[(size_t)st.arith].ins)
                if (in.op == AR_PCT) rd.push_back(kPctBase + in.pct);
        } else if (st.out != kNone) {
            wr.push_back(st.out);
        }
    };
    std::vector<Unit> units;
    for (size_t i = 0; i < L.steps.size();) {
        Unit u;
        u.first = (int)i;
        if (L.steps[i].kind == SK::CclLocal) {
            u.count = 4;
            u.ccl = true;
        }
        for (int k = 0; k < u.count; k++) refs_of(L.steps[i + (size_t)k], u.reads, u.writes);
        i += (size_t)u.count;
        units.push_back(std::move(u));
    }
    const int n = (int)units.size();
    std::unordered_map<int64_t, int> producer;
    for (int u = 0; u < n; u++)
        for (int64_t w : units[(size_t)u].writes) producer[w] = u;
    std::vector<std::vector<int>> users((size_t)n);
    std::vector<int> indeg((size_t)n, 0);
    for (int u = 0; u < n; u++) {
        std::vector<int> deps;
        for (int64_t r : units[(size_t)u].reads) {
            auto it = producer.find(r);
            if (it != producer.end() && it->second != u) deps.push_back(it->second);
        }
        std::sort(deps.begin(), deps.end());
        deps.erase(std::unique(deps.begin(), deps.end()), deps.end());
        for (int d : deps) users[(size_t)d].push_back(u);
        indeg[(size_t)u] = (int)deps.size();
    }
    std::vector<char> done((size_t)n, 0);
    std::vector<Step> out;
    int emitted = 0, group = 0, span = 0;
    bool have_last = false;
    Ref last_b;
    int last_users = 0;
    // labelling lanes (lanes > 1): the passable mask each lane's workspace
    // holds a labelling of, and how many seed sets it serves
    struct LaneState {
        bool have = false;
        Ref b;
        int users = 0;
    };
    std::vector<LaneState> lane_st((size_t)std::max(lanes, 1));
    auto finish = [&](int u) {
        done[(size_t)u] = 1;
        emitted++;
        for (int v : users[(size_t)u]) indeg[(size_t)v]--;
    };
    auto ready = [&](auto pred) {
        std::vector<int> r;
        for (int u = 0; u < n; u++)
            if (!done[(size_t)u] && indeg[(size_t)u] == 0 && pred(units[(size_t)u])) r.push_back(u);
        return r;
    };
    auto kind_of = [&](const Unit &u) { return L.steps[(size_t)u.first].kind; };
    auto same = [](const Ref &a, const Ref &b) { return a.slot == b.slot && a.inv == b.inv; };
    while (emitted < n) {
        int before = emitted;
        const std::ptrdiff_t pct_round_start = (std::ptrdiff_t)out.size();
        for (int u : ready([&](const Unit &x) {
                 return !x.ccl && (kind_of(x) == SK::Pct || kind_of(x) == SK::Atoms || kind_of(x) == SK::Arith);
             })) {
            const Step &st = L.steps[(size_t)units[(size_t)u].first];
            // ready percentiles of one channel share their passes over it
            Step *merged = nullptr;
            if (st.kind == SK::Pct)
                for (Step &o : out)
                    if (&o - out.data() >= pct_round_start && o.kind == SK::Pct && o.chan == st.chan &&
                        o.npq + st.npq <= kMaxPctPerStep)
                        merged = &o;
            if (merged) {
                for (int j = 0; j < st.npq; j++) {
                    merged->q[merged->npq] = st.q[j];
                    merged->pct_out[merged->npq++] = st.pct_out[j];
                }
            } else {
                out.push_back(st);
            }
            finish(u);
        }
        {
            // this scheduling round's arithmetic atoms after its other steps (all of them
            // were ready together, so none reads another), in groups that one
            // launch evaluates: the channels are then read once per group
            std::stable_partition(out.begin() + pct_round_start, out.end(),
                                  [](const Step &x) { return x.kind != SK::Arith; });
            std::ptrdiff_t i = pct_round_start;
            while (i < (std::ptrdiff_t)out.size() && out[(size_t)i].kind != SK::Arith) i++;
            while (i < (std::ptrdiff_t)out.size()) {
                std::ptrdiff_t j = i;
                int ins = 0;
                std::vector<int32_t> chans;
                for (; j < (std::ptrdiff_t)out.size() && j - i < kArGroupProgs; j++) {
                    const ArProgram &pr = L.ariths[(size_t)out[(size_t)j].arith];
                    std::vector<int32_t> ch = chans;
                    for (const ArInstr &in : pr.ins)
                        if (in.op == AR_CHAN && std::find(ch.begin(), ch.end(), in.chan) == ch.end())
                            ch.push_back(in.chan);
                    if (ins + (int)pr.ins.size() > kArGroupInstrs || (int)ch.size() > kArGroupChans) break;
                    ins += (int)pr.ins.size();
                    chans = std::move(ch);
                }
                if (j - i > 1) {
                    group++;
                    for (std::ptrdiff_t k = i; k < j; k++) {
                        out[(size_t)k].group = group;
                        out[(size_t)k].span = 1000000 + group;
                    }
                }
                i = j;
            }
        }
        for (SK k : {SK::Logic, SK::Near}) {
            std::vector<int> r = ready([&](const Unit &x) { return !x.ccl && kind_of(x) == k; });
            for (size_t i = 0; i < r.size(); i++) {
                if (i % kMaxBatch == 0) group++;
                Step st = L.steps[(size_t)units[(size_t)r[i]].first];
                st.group = r.size() > 1 ? group : -1;
                st.span = r.size() > 1 ? 1000000 + group : -1;
                out.push_back(st);
            }
            for (int u : r) finish(u);
        }
        std::vector<int> rc = ready([&](const Unit &x) { return x.ccl; });
        // reuse of an existing labelling of b: seed mask N(y & z) & b, mark, gather
        auto emit_reuse = [&](int u, int users, int lane, int sp) {
            const Step loc = L.steps[(size_t)units[(size_t)u].first];
            Step gat = L.steps[(size_t)units[(size_t)u].first + 3];
            const Ref y = loc.y, z = loc.z;
            const bool yone = y.slot == kNone && y.inv, zone = z.slot == kNone && z.inv;
            Ref t = y;
            if (!zone) {
                if (yone) {
                    t = z;
                } else {
                    Step lg;
                    lg.kind = SK::Logic;
                    lg.x = y;
                    lg.y = z;
                    lg.op = 0;
                    lg.out = L.fresh();
                    lg.lane = lane;
                    lg.span = sp;
                    out.push_back(lg);
                    t = Lower::R(lg.out);
                }
            }
            Step nr;
            nr.kind = SK::Near;
            nr.x = t;
            nr.z = loc.x;
            nr.out = L.fresh();
            nr.lane = lane;
            nr.span = sp;
            out.push_back(nr);
            Step rs;
            rs.kind = SK::CclReseed;
            rs.x = Lower::R(nr.out);
            rs.user = users;
            rs.lane = lane;
            rs.span = sp;
            out.push_back(rs);
            gat.user = users;
            gat.lane = lane;
            gat.span = sp;
            out.push_back(gat);
        };
        auto emit_fresh = [&](int u, int lane, int sp) {
            for (int k = 0; k < 4; k++) {
                Step st = L.steps[(size_t)units[(size_t)u].first + (size_t)k];
                st.user = 0;
                st.lane = lane;
                st.span = sp;
                out.push_back(st);
            }
        };
        if (!rc.empty() && lanes <= 1) {
            int pick = rc[0];
            if (have_last && last_users < kMaxCclUsers)
                for (int u : rc)
                    if (same(L.steps[(size_t)units[(size_t)u].first].x, last_b)) {
                        pick = u;
                        break;
                    }
            const Step loc = L.steps[(size_t)units[(size_t)pick].first];
            if (have_last && last_users < kMaxCclUsers && same(loc.x, last_b)) {
                emit_reuse(pick, last_users, -1, -1);
                last_users++;
            } else {
                emit_fresh(pick, -1, -1);
                have_last = true;
                last_b = loc.x;
                last_users = 1;
            }
            finish(pick);
        } else if (!rc.empty()) {
            // one concurrent region: a labelling that can reuse the labelling a
            // lane holds (or starts in this region) follows it on that lane
            // (a lane's steps run in order); any other takes a free lane
            const int sp = span++;
            std::vector<char> busy((size_t)lanes, 0);
            for (int u : rc) {
                const Ref b = L.steps[(size_t)units[(size_t)u].first].x;
                int l = 0;
                while (l < lanes && !(lane_st[(size_t)l].have && lane_st[(size_t)l].users < kMaxCclUsers &&
                                      same(lane_st[(size_t)l].b, b)))
                    l++;
                if (l < lanes) {
                    emit_reuse(u, lane_st[(size_t)l].users++, l, sp);
                    busy[(size_t)l] = 1;
                    finish(u);
                    continue;
                }
                l = 0;
                while (l < lanes && busy[(size_t)l]) l++;
                if (l == lanes) continue;  // next round
                emit_fresh(u, l, sp);
                lane_st[(size_t)l] = LaneState{true, b, 1};
                busy[(size_t)l] = 1;
                finish(u);
            }
        }
        if (emitted == before) break;  // cannot happen for a DAG
    }
    L.steps = std::move(out);
}

// Turn runs of consecutive Logic/Near steps of the (SSA) schedule into
// segments: a run grows while its deepest chain of near steps stays within
// `cap` and its program fits the kernel (registers, instructions, pointers);
// a run of one step stays a plain step.  ext_of marks the SSA values that are
// requested outputs (they are always stored).
struct SegBuild {
    Segment seg;
    bool ok = false;
};

SegBuild build_segment(const std::vector<Step> &steps, size_t i, size_t j, const std::vector<int64_t> &last_read,
                       const std::vector<int32_t> &ext_of, int cap) {
    SegBuild r;
    Segment &S = r.seg;
    std::unordered_map<int32_t, int> depth, last_in;  // SSA -> near depth; -> last member reading it
    std::unordered_map<int32_t, int> input_idx;
    auto operands = [](const Step &st) {
        std::vector<Ref> v;
        if (st.kind == SK::Logic) v = {st.x, st.y};
        else v = {st.x, st.z};
        return v;
    };
    for (size_t k = i; k < j; k++) {
        const Step &st = steps[k];
        int d = 0;
        for (const Ref &o : operands(st)) {
            if (o.slot == kNone) continue;
            auto it = depth.find(o.slot);
            if (it == depth.end() && !input_idx.count(o.slot)) {
                input_idx[o.slot] = (int)S.inputs.size();
                S.inputs.push_back(o.slot);
            }
            last_in[o.slot] = (int)(k - i);
        }
        if (st.kind == SK::Near) {
            const int dx = st.x.slot != kNone && depth.count(st.x.slot) ? depth[st.x.slot] : 0;
            const int dz = st.z.slot != kNone && depth.count(st.z.slot) ? depth[st.z.slot] : 0;
            d = std::max(dx + 1, dz);
        } else {
            for (const Ref &o : operands(st))
                if (o.slot != kNone && depth.count(o.slot)) d = std::max(d, depth[o.slot]);
        }
        if (d > cap) return r;
        depth[st.out] = d;
        S.halo = std::max(S.halo, d);
    }
    // registers: inputs first, then members in order; a register is freed
    // after the last member that reads it (results are stored right away)
    std::vector<int> free_regs;
    int nregs = 0;
    auto alloc = [&]() {
        if (!free_regs.empty()) {
            const int x = free_regs.back();
            free_regs.pop_back();
            return x;
        }
        return nregs++;
    };
    std::unordered_map<int32_t, int> reg;
    for (size_t q = 0; q < S.inputs.size(); q++) {
        const int x = alloc();
        reg[S.inputs[q]] = x;
        S.ins.push_back(SegInstr{SOP_LOAD, (uint8_t)x, (uint8_t)q, kSegNoReg, 0});
    }
    auto reg_of = [&](const Ref &o) -> uint8_t { return o.slot == kNone ? kSegNoReg : (uint8_t)reg[o.slot]; };
    for (size_t k = i; k < j; k++) {
        const Step &st = steps[k];
        const std::vector<Ref> ops = operands(st);
        const int x = alloc();
        SegInstr in;
        if (st.kind == SK::Logic) in.op = st.op ? SOP_OR : SOP_AND;
        else in.op = st.op ? SOP_NEAR_OR : SOP_NEAR_AND;
        in.dst = (uint8_t)x;
        in.a = reg_of(ops[0]);
        in.b = reg_of(ops[1]);
        in.inv = (uint8_t)((ops[0].inv ? 1 : 0) | (ops[1].inv ? 2 : 0) | (st.inv_out ? 4 : 0));
        S.ins.push_back(in);
        reg[st.out] = x;
        const bool stored = last_read[(size_t)st.out] >= (int64_t)j || ext_of[(size_t)st.out] != kNone;
        if (stored) {
            S.ins.push_back(SegInstr{SOP_STORE, (uint8_t)S.outputs.size(), (uint8_t)x, kSegNoReg, 0});
            S.outputs.push_back(st.out);
        }
        for (const Ref &o : ops) {
            if (o.slot == kNone) continue;
            auto it = last_in.find(o.slot);
            if (it != last_in.end() && it->second == (int)(k - i) && reg.count(o.slot)) {
                free_regs.push_back(reg[o.slot]);
                last_in.erase(it);
            }
        }
        if (!last_in.count(st.out)) free_regs.push_back(x);  // never read inside the segment
    }
    S.nregs = nregs;
    r.ok = nregs <= kSegRegs && (int)S.ins.size() <= kSegInstrs &&
           (int)(S.inputs.size() + S.outputs.size()) <= kSegPtrs;
    return r;
}

void form_segments(Lower &L, const std::vector<int32_t> &ext_of, int cap, std::vector<Segment> &segs) {
    const std::vector<Step> &steps = L.steps;
    const size_t n = steps.size();
    std::vector<int64_t> last_read((size_t)L.nssa, -1);
    for (size_t si = 0; si < n; si++)
        for (const Ref *r : {&steps[si].x, &steps[si].y, &steps[si].z})
            if (r->slot != kNone) last_read[(size_t)r->slot] = (int64_t)si;
    auto local = [](const Step &st) { return (st.kind == SK::Logic || st.kind == SK::Near) && st.lane < 0; };
    std::vector<Step> out;
    for (size_t i = 0; i < n;) {
        if (!local(steps[i])) {
            out.push_back(steps[i++]);
            continue;
        }
        // the longest run from i that builds
        size_t j = i + 1;
        SegBuild best;
        while (j < n && local(steps[j])) {
            SegBuild b = build_segment(steps, i, j + 1, last_read, ext_of, cap);
            if (!b.ok) break;
            best = std::move(b);
            j++;
        }
        if (!best.ok) {
            out.push_back(steps[i++]);
            continue;
        }
        Step sg;
        sg.kind = SK::Segment;
        sg.seg = (int32_t)segs.size();
        segs.push_back(std::move(best.seg));
        out.push_back(sg);
        i = j;
    }
    L.steps = std::move(out);
}

}  // namespace

Plan build_plan(const Dag &dag, const std::vector<int> &which, Mode mode, int lanes, int fuse_halo) {
    Lower L(dag, mode);
    const size_t N = dag.nodes.size();
    std::vector<char> need(N, 0);
    for (int k : which) need[(size_t)dag.outputs[(size_t)k]] = 1;
    for (size_t i = N; i-- > 0;) {
        if (!need[i]) continue;
        const Node &n = dag.nodes[i];
        if (n.a >= 0) need[(size_t)n.a] = 1;
        if (n.b >= 0) need[(size_t)n.b] = 1;
    }
    for (size_t i = 0; i < N; i++) {
        if (!need[i]) continue;
        for (int32_t o : {dag.nodes[i].a, dag.nodes[i].b}) {
            if (o < 0) continue;
            L.uses[(size_t)o]++;
            L.consumer[(size_t)o] = (int32_t)i;
        }
    }
    for (int k : which) {
        L.uses[(size_t)dag.outputs[(size_t)k]]++;
        L.consumer[(size_t)dag.outputs[(size_t)k]] = -1;
    }
    if (mode == Mode::Fused) L.atom_groups(need);
    for (size_t i = 0; i < N; i++) {
        if (!need[i] || L.have[i]) continue;
        L.val[i] = mode == Mode::Fused ? L.fused((int32_t)i) : L.perop((int32_t)i);
        L.have[i] = 1;
    }

    // route each requested output to its external slot: the first output of
    // an SSA value takes it over directly, any other use gets a copy step
    const Ref one = Lower::Const(1);
    std::vector<int32_t> ext_of(L.nssa, kNone);
    for (size_t k = 0; k < which.size(); k++) {
        Ref r = L.val[(size_t)dag.outputs[(size_t)which[k]]];
        if (r.slot != kNone && r.inv == 0 && ext_of[(size_t)r.slot] == kNone) {
            ext_of[(size_t)r.slot] = ext_slot((int)k);
        } else {
            Step &s = L.emit(SK::Logic);
            s.x = r;
            s.y = one;
            s.op = 0;
            s.out = L.fresh();
            ext_of.push_back(ext_slot((int)k));
        }
    }

    std::vector<Segment> segs;
    if (mode == Mode::Fused) {
        schedule_fused(L, std::min(std::max(lanes, 1), kMaxCclLanes));
        ext_of.resize((size_t)L.nssa, kNone);
        if (fuse_halo >= 2) form_segments(L, ext_of, fuse_halo, segs);
    }
    // SSA values a step reads and writes (pointers, rewritten to slots below)
    auto reads_of = [&](Step &s) {
        std::vector<int32_t *> v;
        if (s.kind == SK::Segment) {
            for (int32_t &x : segs[(size_t)s.seg].inputs) v.push_back(&x);
        } else {
            for (Ref *r : {&s.x, &s.y, &s.z})
                if (r->slot != kNone) v.push_back(&r->slot);
        }
        return v;
    };
    auto writes_of = [&](Step &s) {
        std::vector<int32_t *> v;
        if (s.kind == SK::Segment) {
            for (int32_t &x : segs[(size_t)s.seg].outputs) v.push_back(&x);
        } else if (s.kind == SK::Atoms) {
            for (int j = 0; j < s.natoms; j++) v.push_back(&s.atoms[j].out);
        } else if (s.out != kNone) {
            v.push_back(&s.out);
        }
        return v;
    };

    // liveness over SSA values, then greedy slot reuse; a span (a batched
    // group, or a concurrent region of labelling lanes) is allocated as one
    // step so that no member writes a slot another reads
    const int32_t nv = L.nssa;
    std::vector<int64_t> last(nv, -1);
    for (size_t si = 0; si < L.steps.size(); si++)
        for (int32_t *r : reads_of(L.steps[si])) last[(size_t)*r] = (int64_t)si;
    std::vector<int32_t> slot_of(nv, kNone);
    std::vector<int32_t> free_slots;
    int32_t nslots = 0;
    auto alloc = [&](int32_t v) {
        if (ext_of[(size_t)v] != kNone) {
            slot_of[(size_t)v] = ext_of[(size_t)v];
            return;
        }
        if (!free_slots.empty()) {
            slot_of[(size_t)v] = free_slots.back();
            free_slots.pop_back();
        } else {
            slot_of[(size_t)v] = nslots++;
        }
    };
    auto release = [&](int32_t v) {
        int32_t s = slot_of[(size_t)v];
        if (s >= 0) free_slots.push_back(s);
    };
    for (size_t s0 = 0; s0 < L.steps.size();) {
        size_t s1 = s0 + 1;
        if (L.steps[s0].span >= 0)
            while (s1 < L.steps.size() && L.steps[s1].span == L.steps[s0].span) s1++;
        std::vector<int32_t> outs;
        for (size_t si = s0; si < s1; si++)
            for (int32_t *w : writes_of(L.steps[si])) outs.push_back(*w);
        for (int32_t v : outs) alloc(v);
        std::vector<int32_t> dying;
        for (size_t si = s0; si < s1; si++) {
            Step &s = L.steps[si];
            for (int32_t *r : reads_of(s)) {
                int32_t v = *r;
                if (last[(size_t)v] >= (int64_t)s0 && last[(size_t)v] < (int64_t)s1 &&
                    std::find(dying.begin(), dying.end(), v) == dying.end())
                    dying.push_back(v);
                *r = slot_of[(size_t)v];
            }
            for (int32_t *w : writes_of(s)) *w = slot_of[(size_t)*w];
        }
        for (int32_t v : dying) release(v);
        for (int32_t v : outs)
            if (last[(size_t)v] < 0 && !is_ext(slot_of[(size_t)v])) release(v);
        s0 = s1;
    }

    Plan P;
    P.steps = std::move(L.steps);
    P.nslots = nslots;
    P.npct = L.npct;
    P.noutputs = (int32_t)which.size();
    P.ccl_count = 0;
    P.ccl_reuse = 0;
    for (const Step &st : P.steps) {
        if (st.kind == SK::CclLocal) P.ccl_count++;
        if (st.kind == SK::CclReseed) P.ccl_reuse++;
        P.ccl_lanes = std::max(P.ccl_lanes, st.lane + 1);
    }
    P.output_ids.assign(which.begin(), which.end());
    P.segments = std::move(segs);
    P.ariths = std::move(L.ariths);
    return P;
}

}  // namespace vlg
