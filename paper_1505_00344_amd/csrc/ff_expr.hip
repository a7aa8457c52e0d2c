// ff_expr.hip — right-hand sides given at run time as expressions.
//
// A system defined by the user carries one expression per state variable
// (Appendix A, State Variables); the step kernel is the general RK4 template
// with that right-hand side filled in, compiled for the GPU when the system is
// first used (Appendix A.1).  Here the template is the library's own fused
// kernel skeleton (ff_kernel.h, the same text the built-in systems are
// instantiated from), the right-hand side becomes a system struct with the
// D/NP/NQ/derive/f interface, and hipRTC compiles it for the device's
// architecture; the code object is loaded per device and precision and kept
// with the system handle.
//
// Expression language (names x0..x{dim-1}, p0..p{n_params-1}):
//   sum     := product (('+' | '-') product)*        left-associative
//   product := prefix (('*' | '/') prefix)*          left-associative
//   prefix  := '-' prefix | '+' prefix | atom        a sign binds tightest
//   atom    := number | name | func '(' sum (',' sum)* ')' | '(' sum ')'
// number: a decimal or hexadecimal literal as strtod reads it, starting with
// a digit or '.', then rounded to the working precision; name: x<k> or p<k>
// with k a decimal index without leading zeros; functions exp expm1 log log1p
// sqrt sin cos tan tanh sinh cosh atan fabs (one argument), pow fmin fmax
// (two), fma (three, fused).  Every operation rounds to the working precision
// (the code is compiled without contraction and without fast math), so the
// tree fixes the result up to the accuracy of the device math library.
//
// With FF_EXPR_FAST_F32, single precision evaluates exp(x) as the hardware
// 2^(x log2 e) and a / b as a * rcp(b) (about 1 ulp each, the built-in
// systems' single-precision policy); everything else is unchanged.
//
// Two rewrites that leave every value unchanged: identical subtrees are
// evaluated once, and subtrees that depend on parameters and literals only
// are evaluated once per particle (the system's derived constants q) instead
// of four times per step.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "ff_embedded_src.h"
#include "ff_internal.h"
#include "ff_adjoint.h"
#include "ff_rk4.h"

namespace ff {
namespace {

constexpr int kMaxNodes = 4096;
constexpr size_t kMaxExprChars = 65536;
constexpr int kMaxDepth = 256;  // nesting of signs, parentheses and calls

struct FnInfo {
    const char* name;
    int arity;
    const char* f64;
    const char* f32;
};
const FnInfo kFn[] = {
    {"exp", 1, "exp", "expf"},       {"expm1", 1, "expm1", "expm1f"}, {"log", 1, "log", "logf"},
    {"log1p", 1, "log1p", "log1pf"}, {"sqrt", 1, "sqrt", "sqrtf"},    {"sin", 1, "sin", "sinf"},
    {"cos", 1, "cos", "cosf"},       {"tan", 1, "tan", "tanf"},       {"tanh", 1, "tanh", "tanhf"},
    {"sinh", 1, "sinh", "sinhf"},    {"cosh", 1, "cosh", "coshf"},    {"atan", 1, "atan", "atanf"},
    {"fabs", 1, "fabs", "fabsf"},    {"pow", 2, "pow", "powf"},       {"fmin", 2, "fmin", "fminf"},
    {"fmax", 2, "fmax", "fmaxf"},    {"fma", 3, "__builtin_fma", "__builtin_fmaf"},
};
constexpr int kNumFn = sizeof(kFn) / sizeof(kFn[0]);

enum Op : int { kNum, kX, kP, kNeg, kAdd, kSub, kMul, kDiv, kCall };

struct Node {
    int op;
    int fn;           // kCall: index into kFn
    int arg[3];       // operands (node indices), -1 if unused
    uint64_t bits;    // kNum: the double's bit pattern
    int idx;          // kX / kP: the index
    bool varying;     // depends on the state
};

// Hash-consed expression DAG shared by the dim right-hand sides.
struct Dag {
    std::vector<Node> nodes;
    std::map<std::tuple<int, int, int, int, int, uint64_t, int>, int> seen;

    int add(Node n) {
        const auto key = std::make_tuple(n.op, n.fn, n.arg[0], n.arg[1], n.arg[2], n.bits, n.idx);
        auto it = seen.find(key);
        if (it != seen.end()) return it->second;
        n.varying = n.op == kX;
        for (int a : n.arg)
            if (a >= 0 && nodes[a].varying) n.varying = true;
        nodes.push_back(n);
        const int id = (int)nodes.size() - 1;
        seen.emplace(key, id);
        return id;
    }
    int leaf(int op, uint64_t bits, int idx) { return add(Node{op, -1, {-1, -1, -1}, bits, idx, false}); }
    int op(int o, int a, int b = -1, int c = -1, int fn = -1) { return add(Node{o, fn, {a, b, c}, 0, 0, false}); }
};

class Parser {
   public:
    Parser(const char* text, int dim, int np, Dag& dag) : s_(text), dim_(dim), np_(np), dag_(dag) {}

    // Parses the whole text; returns the root node or -1 (see error()).
    int parse_all() {
        const int r = sum();
        if (r < 0) return -1;
        skip();
        if (s_[pos_]) return bad("unexpected '" + std::string(1, s_[pos_]) + "'");
        return r;
    }
    const std::string& error() const { return err_; }
    size_t where() const { return err_pos_; }

   private:
    const char* s_;
    size_t pos_ = 0;
    int dim_, np_;
    Dag& dag_;
    std::string err_;
    size_t err_pos_ = 0;
    int depth_ = 0;

    int bad(const std::string& m) {
        if (err_.empty()) {
            err_ = m;
            err_pos_ = pos_;
        }
        return -1;
    }
    void skip() {
        while (s_[pos_] && std::isspace((unsigned char)s_[pos_])) ++pos_;
    }
    char peek() {
        skip();
        return s_[pos_];
    }
    bool guard() {
        if ((int)dag_.nodes.size() >= kMaxNodes) {
            bad("expressions too large (more than " + std::to_string(kMaxNodes) + " distinct operations)");
            return false;
        }
        return true;
    }

    // binary levels: 1 for + -, 2 for * /
    int sum() { return climb(1); }
    int climb(int min_level) {
        int lhs = prefix();
        while (lhs >= 0) {
            const char c = peek();
            const int level = (c == '+' || c == '-') ? 1 : (c == '*' || c == '/') ? 2 : 0;
            if (level == 0 || level < min_level) break;
            ++pos_;
            const int rhs = climb(level + 1);
            if (rhs < 0 || !guard()) return -1;
            const int op = c == '+' ? kAdd : c == '-' ? kSub : c == '*' ? kMul : kDiv;
            lhs = dag_.op(op, lhs, rhs);
        }
        return lhs;
    }
    int prefix() {
        struct Depth {
            int& d;
            explicit Depth(int& v) : d(v) { ++d; }
            ~Depth() { --d; }
        } depth(depth_);
        if (depth_ > kMaxDepth) return bad("expression nested deeper than " + std::to_string(kMaxDepth) + " levels");
        const char c = peek();
        if (c == '-') {
            ++pos_;
            const int a = prefix();
            if (a < 0 || !guard()) return -1;
            return dag_.op(kNeg, a);
        }
        if (c == '+') {
            ++pos_;
            return prefix();
        }
        return atom();
    }
    int atom() {
        const char c = peek();
        if (c == '(') {
            ++pos_;
            const int a = sum();
            if (a < 0) return -1;
            if (peek() != ')') return bad("expected ')'");
            ++pos_;
            return a;
        }
        if (std::isdigit((unsigned char)c) || c == '.') {
            const char* start = s_ + pos_;
            char* end = nullptr;
            const double v = std::strtod(start, &end);
            if (end == start) return bad("malformed number");
            pos_ += (size_t)(end - start);
            uint64_t bits;
            std::memcpy(&bits, &v, sizeof bits);
            if (!guard()) return -1;
            return dag_.leaf(kNum, bits, 0);
        }
        if (std::isalpha((unsigned char)c)) {
            const size_t start = pos_;
            while (std::isalnum((unsigned char)s_[pos_]) || s_[pos_] == '_') ++pos_;
            const std::string name(s_ + start, pos_ - start);
            if ((name[0] == 'x' || name[0] == 'p') && name.size() > 1 &&
                std::isdigit((unsigned char)name[1])) {
                const std::string digits = name.substr(1);
                if (digits.find_first_not_of("0123456789") != std::string::npos) {
                    pos_ = start;
                    return bad("unknown name '" + name + "'");
                }
                if (digits.size() > 1 && digits[0] == '0') {
                    pos_ = start;
                    return bad("index with a leading zero in '" + name + "'");
                }
                const int k = digits.size() > 3 ? 1000 : std::atoi(digits.c_str());
                const bool is_x = name[0] == 'x';
                if (k >= (is_x ? dim_ : np_)) {
                    pos_ = start;
                    return bad(std::string(is_x ? "state variable" : "parameter") + " index out of range in '" +
                               name + "'");
                }
                if (!guard()) return -1;
                return dag_.leaf(is_x ? kX : kP, 0, k);
            }
            int fn = -1;
            for (int k = 0; k < kNumFn; ++k)
                if (name == kFn[k].name) fn = k;
            if (fn < 0) {
                pos_ = start;
                return bad("unknown name '" + name + "'");
            }
            if (peek() != '(') return bad("expected '(' after " + name);
            ++pos_;
            int args[3] = {-1, -1, -1};
            for (int k = 0; k < kFn[fn].arity; ++k) {
                if (k > 0) {
                    if (peek() != ',') return bad(name + " takes " + std::to_string(kFn[fn].arity) + " arguments");
                    ++pos_;
                }
                args[k] = sum();
                if (args[k] < 0) return -1;
            }
            if (peek() != ')') return bad("expected ')' to close " + name);
            ++pos_;
            if (!guard()) return -1;
            return dag_.op(kCall, args[0], args[1], args[2], fn);
        }
        if (!c) return bad("unexpected end of expression");
        return bad("unexpected '" + std::string(1, c) + "'");
    }
};

std::string literal(uint64_t bits, bool f32) {
    double v;
    std::memcpy(&v, &bits, sizeof v);
    char buf[64];
    if (std::isinf(v))
        std::snprintf(buf, sizeof buf, "%s__builtin_huge_val()", v < 0 ? "-" : "");
    else
        std::snprintf(buf, sizeof buf, "%a", v);
    return f32 ? "((float)(" + std::string(buf) + "))" : "(" + std::string(buf) + ")";
}

}  // namespace

struct ExprProgram {
    int dim = 0, np = 0;
    uint32_t flags = 0;
    std::vector<std::string> text;  // the expressions as given
    Dag dag;
    std::vector<int> roots;
    std::mutex mu;
    struct Module {
        hipModule_t mod = nullptr;
        hipFunction_t fn[kExprKernels] = {};
    };
    std::map<std::tuple<int, int, int>, Module> modules;  // (device, prec, kind)

    // Unloading a code object while its kernels are queued or running is
    // undefined, so each device is drained first (destroying a system is rare).
    ~ExprProgram() {
        if (modules.empty()) return;
        int cur = 0;
        const bool have = hipGetDevice(&cur) == hipSuccess;
        for (auto& kv : modules) {
            if (!kv.second.mod) continue;
            if (hipSetDevice(std::get<0>(kv.first)) == hipSuccess) {
                (void)hipDeviceSynchronize();
                (void)hipModuleUnload(kv.second.mod);
            }
        }
        if (have) (void)hipSetDevice(cur);
    }
};

// The system struct of one precision: derive (state-free subtrees, once per
// particle), f (the right-hand side) and vjp (its vector-Jacobian product by
// reverse-mode differentiation of the DAG: node values forward, then node
// adjoints in reverse order, each operation passing its local partials to
// its operands).
std::string expr_struct(const ExprProgram& P, int prec) {
    const bool f32 = prec != FF_FP64;
    const bool fast = f32 && (P.flags & FF_EXPR_FAST_F32);
    const char* R = f32 ? "float" : "double";
    const std::vector<Node>& N = P.dag.nodes;
    auto internal = [&](int id) { return N[id].op != kNum && N[id].op != kX && N[id].op != kP; };
    // which state-free internal nodes does the per-step code (or a root) use?
    std::vector<char> need_q(N.size(), 0);
    for (size_t i = 0; i < N.size(); ++i) {
        if (!N[i].varying) continue;
        for (int a : N[i].arg)
            if (a >= 0 && !N[a].varying && internal(a)) need_q[a] = 1;
    }
    for (int r : P.roots)
        if (!N[r].varying && internal(r)) need_q[r] = 1;
    std::vector<int> qslot(N.size(), -1);
    int nq = 0;
    for (size_t i = 0; i < N.size(); ++i)
        if (need_q[i]) qslot[i] = nq++;
    // operand text: in derive() state-free temps are c<i>; in f() the varying
    // ones are t<i> and the state-free ones q[...]; in vjp() every internal
    // node is a local v<i>
    enum { kDerive, kF, kVjp };
    auto ref = [&](int id, int where) -> std::string {
        const Node& n = N[id];
        if (n.op == kNum) return literal(n.bits, f32);
        if (n.op == kX) return "x[" + std::to_string(n.idx) + "]";
        if (n.op == kP) return "p[" + std::to_string(n.idx) + "]";
        if (where == kF && !n.varying) return "q[" + std::to_string(qslot[id]) + "]";
        return (where == kF ? "t" : where == kDerive ? "c" : "v") + std::to_string(id);
    };
    auto fname = [&](const char* name) -> std::string {
        for (const FnInfo& f : kFn)
            if (std::strcmp(f.name, name) == 0) return f32 ? f.f32 : f.f64;
        return name;
    };
    auto div = [&](const std::string& a, const std::string& b) {
        return fast ? "(" + a + ") * __builtin_amdgcn_rcpf(" + b + ")" : "(" + a + ") / (" + b + ")";
    };
    auto expr_of = [&](int id, int where) -> std::string {
        const Node& n = N[id];
        const std::string a = n.arg[0] >= 0 ? ref(n.arg[0], where) : "";
        const std::string b = n.arg[1] >= 0 ? ref(n.arg[1], where) : "";
        switch (n.op) {
            case kNeg: return "-" + a;
            case kAdd: return a + " + " + b;
            case kSub: return a + " - " + b;
            case kMul: return a + " * " + b;
            case kDiv: return fast ? a + " * __builtin_amdgcn_rcpf(" + b + ")" : a + " / " + b;
            case kCall: {
                if (fast && std::string(kFn[n.fn].name) == "exp")
                    return "__builtin_amdgcn_exp2f(" + a + " * 0x1.715476p+0f)";
                std::string s = std::string(f32 ? kFn[n.fn].f32 : kFn[n.fn].f64) + "(" + a;
                for (int k = 1; k < kFn[n.fn].arity; ++k) s += ", " + ref(n.arg[k], where);
                return s + ")";
            }
        }
        return "";
    };

    std::string src = "namespace ffx {\n\nstruct Sys {\n";
    src += std::string("    using R = ") + R + ";\n";
    src += "    static constexpr int D = " + std::to_string(P.dim) + ", NP = " + std::to_string(P.np > 0 ? P.np : 1) +
           ", NQ = " + std::to_string(nq > 0 ? nq : 1) + ", UNROLL = " + (P.dim <= 4 ? "2" : "1") + ", FUSED_INC = 0;\n";
    src += "    static __device__ __forceinline__ void derive(const R (&p)[NP], R (&q)[NQ]) {\n        (void)p;\n";
    if (nq == 0) src += "        q[0] = R(0);\n";
    for (size_t i = 0; i < N.size(); ++i) {
        if (N[i].varying || !internal((int)i)) continue;
        src += "        const R c" + std::to_string(i) + " = " + expr_of((int)i, kDerive) + ";\n";
        if (need_q[i]) src += "        q[" + std::to_string(qslot[i]) + "] = c" + std::to_string(i) + ";\n";
    }
    src += "    }\n";
    src += "    static __device__ __forceinline__ void f(const R (&p)[NP], const R (&q)[NQ], const R (&x)[D], "
           "R (&o)[D]) {\n        (void)p; (void)q; (void)x;\n";
    for (size_t i = 0; i < N.size(); ++i) {
        if (!N[i].varying || !internal((int)i)) continue;
        src += "        const R t" + std::to_string(i) + " = " + expr_of((int)i, kF) + ";\n";
    }
    for (int d = 0; d < P.dim; ++d) src += "        o[" + std::to_string(d) + "] = " + ref(P.roots[d], kF) + ";\n";
    src += "    }\n";

    // vjp: gx += J^T a, gp += (df/dp)^T a.  A node is active if it depends on
    // a state variable or a parameter; only active operands receive adjoints.
    std::vector<char> act(N.size(), 0);
    for (size_t i = 0; i < N.size(); ++i) {
        act[i] = N[i].op == kX || N[i].op == kP;
        for (int a : N[i].arg)
            if (a >= 0 && act[a]) act[i] = 1;
    }
    src += "    static __device__ __forceinline__ void vjp(const R (&p)[NP], const R (&q)[NQ], const R (&x)[D], "
           "const R (&a)[D], R (&gx)[D], R (&gp)[NP]) {\n        (void)p; (void)q; (void)x; (void)a; (void)gx; "
           "(void)gp;\n";
    for (size_t i = 0; i < N.size(); ++i)
        if (internal((int)i)) src += "        const R v" + std::to_string(i) + " = " + expr_of((int)i, kVjp) + ";\n";
    for (size_t i = 0; i < N.size(); ++i)
        if (internal((int)i) && act[i]) src += "        R b" + std::to_string(i) + " = R(0);\n";
    // contribution c to the adjoint of operand `id`
    auto add = [&](int id, const std::string& c) -> std::string {
        if (id < 0 || !act[id]) return "";
        const Node& n = N[id];
        if (n.op == kX) return "        gx[" + std::to_string(n.idx) + "] += " + c + ";\n";
        if (n.op == kP) return "        gp[" + std::to_string(n.idx) + "] += " + c + ";\n";
        return "        b" + std::to_string(id) + " += " + c + ";\n";
    };
    for (int d = 0; d < P.dim; ++d) src += add(P.roots[d], "a[" + std::to_string(d) + "]");
    for (int i = (int)N.size() - 1; i >= 0; --i) {
        if (!internal(i) || !act[i]) continue;
        const Node& n = N[i];
        const std::string B = "b" + std::to_string(i), t = ref(i, kVjp);
        const int ia = n.arg[0], ib = n.arg[1], ic = n.arg[2];
        const std::string va = ia >= 0 ? ref(ia, kVjp) : "", vb = ib >= 0 ? ref(ib, kVjp) : "";
        switch (n.op) {
            case kNeg: src += add(ia, "-" + B); break;
            case kAdd: src += add(ia, B) + add(ib, B); break;
            case kSub: src += add(ia, B) + add(ib, "-" + B); break;
            case kMul: src += add(ia, B + " * " + vb) + add(ib, B + " * " + va); break;
            case kDiv: src += add(ia, div(B, vb)) + add(ib, "-" + div(B + " * " + t, vb)); break;
            case kCall: {
                const std::string f = kFn[n.fn].name;
                if (f == "exp") src += add(ia, B + " * " + t);
                else if (f == "expm1") src += add(ia, B + " * (" + t + " + R(1))");
                else if (f == "log") src += add(ia, div(B, va));
                else if (f == "log1p") src += add(ia, div(B, "R(1) + " + va));
                else if (f == "sqrt") src += add(ia, div(B, "R(2) * " + t));
                else if (f == "sin") src += add(ia, B + " * " + fname("cos") + "(" + va + ")");
                else if (f == "cos") src += add(ia, "-" + B + " * " + fname("sin") + "(" + va + ")");
                else if (f == "tan") src += add(ia, B + " * (R(1) + " + t + " * " + t + ")");
                else if (f == "tanh") src += add(ia, B + " * (R(1) - " + t + " * " + t + ")");
                else if (f == "sinh") src += add(ia, B + " * " + fname("cosh") + "(" + va + ")");
                else if (f == "cosh") src += add(ia, B + " * " + fname("sinh") + "(" + va + ")");
                else if (f == "atan") src += add(ia, div(B, "R(1) + " + va + " * " + va));
                else if (f == "fabs") src += add(ia, "(" + va + " >= R(0) ? " + B + " : -" + B + ")");  // slope +1 at 0
                else if (f == "pow")
                    src += add(ia, B + " * " + vb + " * " + fname("pow") + "(" + va + ", " + vb + " - R(1))") +
                           add(ib, B + " * " + t + " * " + fname("log") + "(" + va + ")");
                else if (f == "fmin" || f == "fmax")  // the returned operand (the first on a tie)
                    src += add(ia, "(" + t + " == " + va + " ? " + B + " : R(0))") +
                           add(ib, "(" + t + " == " + va + " ? R(0) : " + B + ")");
                else if (f == "fma")
                    src += add(ia, B + " * " + vb) + add(ib, B + " * " + va) + add(ic, B);
                break;
            }
        }
    }
    src += "    }\n};\n\n}  // namespace ffx\n";
    return src;
}

// The program of one precision and kind: the kernel skeleton, the system
// struct, layout checks of the argument structs the host packs, and the
// kernel instances requested by name.
std::string expr_program(const ExprProgram& P, int prec, int kind, std::vector<std::string>* names) {
    const char* R = prec == FF_FP64 ? "double" : "float";
    const std::string K = prec == FF_FP32_KAHAN ? "true" : "false";
    std::string src = "// generated: fused RK4 kernels for a user right-hand side\n";
    src += kind == kExprAdjoint ? "#include \"ff_adjoint_kernel.h\"\n\n" : "#include \"ff_kernel.h\"\n\n";
    src += expr_struct(P, prec) + "\n";
    names->clear();
    if (kind == kExprAdjoint) {
        src += "static_assert(sizeof(ff::AdjArgs) == " + std::to_string(sizeof(AdjArgs)) + ", \"AdjArgs layout\");\n";
        const bool small = P.dim <= 4;
        names->push_back(std::string("&ff::k_adj<ffx::Sys, ") + R + ", " + K + (small ? ", 8, false>" : ", 1, true>"));
        return src;
    }
    src += "static_assert(sizeof(ff::RK4Args) == " + std::to_string(sizeof(RK4Args)) + ", \"RK4Args layout\");\n";
    src += "static_assert(sizeof(ff::ResetArgs) == " + std::to_string(sizeof(ResetArgs)) + ", \"ResetArgs layout\");\n";
    src += "static_assert(sizeof(ff::RecordArgs) == " + std::to_string(sizeof(RecordArgs)) + ", \"RecordArgs layout\");\n";
    const std::string T = std::string("ffx::Sys, ") + R + ", " + K;
    for (int ppt : {1, 2}) {
        const std::string P2 = std::to_string(ppt);
        names->push_back("&ff::k_rk4<" + T + ", " + P2 + ">");
        names->push_back("&ff::k_rk4_reset<" + T + ", " + P2 + ">");
        names->push_back("&ff::k_rk4_record<" + T + ", " + P2 + ", false>");
        names->push_back("&ff::k_rk4_record<" + T + ", " + P2 + ", true>");
    }
    return src;
}

namespace {

const char* const kHeaderNames[] = {"ff_kernel.h", "ff_math.h", "ff_rng.h", "ff_adjoint_kernel.h"};
const char* const kHeaders[] = {kEmbedded_ff_kernel_h, kEmbedded_ff_math_h, kEmbedded_ff_rng_h,
                                kEmbedded_ff_adjoint_kernel_h};
constexpr int kNumHeaders = 4;

// Compiles the program of `prec` and `kind` for `arch`; code receives the
// code object and lowered holds the mangled names of the kernels, in the
// order of the name expressions.
ff_status compile(const ExprProgram& P, int prec, int kind, const std::string& arch, std::vector<char>* code,
                  std::vector<std::string>* lowered) {
    std::vector<std::string> names;
    const std::string src = expr_program(P, prec, kind, &names);
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "ff_user_rhs.hip", kNumHeaders, kHeaders, kHeaderNames) !=
        HIPRTC_SUCCESS)
        return fail(FF_E_DEVICE, "hiprtcCreateProgram failed");
    for (const std::string& n : names) {
        if (hiprtcAddNameExpression(prog, n.c_str()) != HIPRTC_SUCCESS) {
            hiprtcDestroyProgram(&prog);
            return fail(FF_E_DEVICE, "hiprtcAddNameExpression failed for " + n);
        }
    }
    const std::string arch_opt = "--offload-arch=" + arch;
    const char* opts[] = {arch_opt.c_str(), "-O3", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        return fail(FF_E_INVALID, std::string("compiling the right-hand side failed (") + hiprtcGetErrorString(r) +
                                      "):\n" + log);
    }
    size_t n = 0;
    hiprtcGetCodeSize(prog, &n);
    code->assign(n, 0);
    hiprtcGetCode(prog, code->data());
    lowered->clear();
    for (const std::string& nm : names) {
        const char* low = nullptr;
        if (hiprtcGetLoweredName(prog, nm.c_str(), &low) != HIPRTC_SUCCESS || !low) {
            hiprtcDestroyProgram(&prog);
            return fail(FF_E_DEVICE, "hiprtcGetLoweredName failed for " + nm);
        }
        lowered->push_back(low);
    }
    hiprtcDestroyProgram(&prog);
    return FF_OK;
}

}  // namespace

ff_status expr_prepare(const ff_system_s* sys, int prec, int kind) {
    ExprProgram& P = *sys->expr;
    int dev = 0;
    if (hipError_t e = hipGetDevice(&dev)) return device_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(P.mu);
    if (P.modules.count({dev, prec, kind})) return FF_OK;
    hipDeviceProp_t prop;
    if (hipError_t e = hipGetDeviceProperties(&prop, dev)) return device_fail(e, "hipGetDeviceProperties");
    std::vector<char> code;
    std::vector<std::string> lowered;
    // the processor name without its feature suffix (":sramecc+:xnack-"): a
    // code object built for "any" setting of a feature loads on every one
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    if (ff_status s = compile(P, prec, kind, arch, &code, &lowered)) return s;
    ExprProgram::Module m;
    if (hipError_t e = hipModuleLoadData(&m.mod, code.data())) return device_fail(e, "hipModuleLoadData");
    for (size_t k = 0; k < lowered.size(); ++k) {
        if (hipError_t e = hipModuleGetFunction(&m.fn[k], m.mod, lowered[k].c_str())) {
            (void)hipModuleUnload(m.mod);
            return device_fail(e, "hipModuleGetFunction");
        }
    }
    P.modules[{dev, prec, kind}] = m;
    return FF_OK;
}

hipError_t launch_rk4_expr(const ff_system_s* sys, const RK4Launch& L) {
    ExprProgram& P = *sys->expr;
    int dev = 0;
    if (hipError_t e = hipGetDevice(&dev)) return e;
    hipFunction_t fn[kExprKernels];
    {
        std::lock_guard<std::mutex> lk(P.mu);
        auto it = P.modules.find({dev, L.prec, kExprForward});
        if (it == P.modules.end()) return hipErrorNotInitialized;  // expr_prepare was not called
        std::memcpy(fn, it->second.fn, sizeof fn);
    }
    const int ppt = L.ppt >= 2 ? 2 : 1;
    const int64_t per_block = (int64_t)L.block * ppt;
    const int64_t grid = (L.n + per_block - 1) / per_block;
    if (grid <= 0) return hipSuccess;
    RK4Args a = make_args(L);
    ResetArgs none;
    std::memset(&none, 0, sizeof none);
    ResetArgs r = L.reset ? *L.reset : none;
    RecordArgs rc;
    std::memset(&rc, 0, sizeof rc);
    if (L.record) rc = *L.record;
    void* params[3] = {&a, &r, &rc};
    // kernel order per ppt: step, reset, record, record with reset
    const int which = L.record ? (L.reset ? 3 : 2) : (L.reset ? 1 : 0);
    return hipModuleLaunchKernel(fn[(ppt - 1) * 4 + which], (unsigned)grid, 1, 1, (unsigned)L.block, 1, 1, 0, L.stream,
                                 params, nullptr);
}

hipError_t launch_adj_expr(const ff_system_s* sys, const AdjLaunch& A) {
    ExprProgram& P = *sys->expr;
    int dev = 0;
    if (hipError_t e = hipGetDevice(&dev)) return e;
    hipFunction_t fn;
    {
        std::lock_guard<std::mutex> lk(P.mu);
        auto it = P.modules.find({dev, A.f.prec, kExprAdjoint});
        if (it == P.modules.end()) return hipErrorNotInitialized;  // expr_prepare was not called
        fn = it->second.fn[0];
    }
    const int64_t grid = (A.f.n + kAdjBlock - 1) / kAdjBlock;
    if (grid <= 0) return hipSuccess;
    AdjArgs a = make_adj_args(A);
    void* params[1] = {&a};
    return hipModuleLaunchKernel(fn, (unsigned)grid, 1, 1, kAdjBlock, 1, 1, 0, A.f.stream, params, nullptr);
}

void expr_destroy(ExprProgram* P) { delete P; }

}  // namespace ff

using namespace ff;

extern "C" {

ff_status ff_system_create_expr(int32_t dim, const char* const* exprs, int32_t n_params, const double* params,
                                uint32_t flags, ff_system_t* out) {
    set_error("");
    if (!out) return fail(FF_E_INVALID, "out is NULL");
    *out = nullptr;
    if (flags & ~(uint32_t)FF_EXPR_FAST_F32) return fail(FF_E_INVALID, "unknown flags");
    if (dim < 1 || dim > kMaxDim) return fail(FF_E_INVALID, "dim must be in [1, 15]");
    if (n_params < 0 || n_params > kMaxParams) return fail(FF_E_INVALID, "n_params must be in [0, 16]");
    if (n_params > 0 && !params) return fail(FF_E_INVALID, "params is NULL");
    if (!exprs) return fail(FF_E_INVALID, "exprs is NULL");
    ExprProgram* P = new (std::nothrow) ExprProgram;
    if (!P) return fail(FF_E_NOMEM, "out of host memory");
    P->dim = dim;
    P->np = n_params;
    P->flags = flags;
    for (int d = 0; d < dim; ++d) {
        if (!exprs[d] || std::strlen(exprs[d]) > kMaxExprChars) {
            delete P;
            return fail(FF_E_INVALID, "expression " + std::to_string(d) + " is NULL or longer than 65536 characters");
        }
        P->text.push_back(exprs[d]);
        Parser ps(exprs[d], dim, n_params, P->dag);
        const int root = ps.parse_all();
        if (root < 0) {
            const std::string msg = "expression for x" + std::to_string(d) + ", column " +
                                    std::to_string(ps.where() + 1) + ": " + ps.error();
            delete P;
            return fail(FF_E_INVALID, msg);
        }
        P->roots.push_back(root);
    }
    ff_system_s* s = new (std::nothrow) ff_system_s;
    if (!s) {
        delete P;
        return fail(FF_E_NOMEM, "out of host memory");
    }
    s->rhs = FF_RHS_EXPR;
    s->dim = dim;
    s->n_params = n_params;
    for (int q = 0; q < kMaxParams; ++q) s->params[q] = q < n_params ? params[q] : 0.0;
    s->expr = P;
    *out = s;
    return FF_OK;
}

ff_status ff_system_compile(ff_system_t sys, int32_t prec, const char* arch) {
    set_error("");
    if (ff_status s = check_system(sys)) return s;
    if (!sys->expr) return fail(FF_E_INVALID, "not an expression system (built-in systems need no compilation)");
    if (prec != FF_FP64 && prec != FF_FP32 && prec != FF_FP32_KAHAN) return fail(FF_E_INVALID, "unknown precision");
    for (int kind : {kExprForward, kExprAdjoint}) {
        if (!arch) {
            if (ff_status s = expr_prepare(sys, prec, kind)) return s;
        } else {
            std::vector<char> code;
            std::vector<std::string> lowered;
            if (ff_status s = compile(*sys->expr, prec, kind, arch, &code, &lowered)) return s;
        }
    }
    return FF_OK;
}

ff_status ff_system_source(ff_system_t sys, int32_t prec, char* buf, size_t cap, size_t* len) {
    set_error("");
    if (ff_status s = check_system(sys)) return s;
    if (!sys->expr) return fail(FF_E_INVALID, "not an expression system");
    if (prec != FF_FP64 && prec != FF_FP32 && prec != FF_FP32_KAHAN) return fail(FF_E_INVALID, "unknown precision");
    const std::string src = expr_struct(*sys->expr, prec);
    if (len) *len = src.size() + 1;
    if (buf && cap > 0) {
        const size_t n = src.size() < cap - 1 ? src.size() : cap - 1;
        std::memcpy(buf, src.data(), n);
        buf[n] = '\0';
        if (src.size() + 1 > cap) return fail(FF_E_NOMEM, "buffer too small for the source");
    }
    return FF_OK;
}

}  // extern "C"
