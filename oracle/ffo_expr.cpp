// ffo_expr.cpp — the oracle's expression right-hand sides (TEST
// INFRASTRUCTURE ONLY, see ffo.h).  A user system is given as one expression
// per state variable (the paper's State Variables, Appendix A), over the names
// x0 .. x{dim-1} and p0 .. p{n_params-1}.  This file parses each expression
// into a tree and evaluates it directly, in double precision, one operation
// at a time, left to right with the usual precedence; it is the plain
// definition that the compiled kernels are checked against.
//
// Grammar:  expr := term (('+' | '-') term)*
//           term := unary (('*' | '/') unary)*
//           unary := '-' unary | '+' unary | primary
//           primary := number | x<d> | p<k> | func '(' expr (',' expr)* ')' | '(' expr ')'
// Functions: exp expm1 log log1p sqrt sin cos tan tanh sinh cosh atan fabs
// (one argument), pow fmin fmax (two), fma (three, rounded once).  Numbers
// start with a digit or '.' and are read by strtod; x<k> and p<k> take an
// index without leading zeros.
#include <cctype>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "ffo.h"

namespace {

struct Node {
    enum Kind { NUM, VAR, PAR, NEG, ADD, SUB, MUL, DIV, FUN } kind;
    double val = 0.0;
    int index = 0;
    int fn = 0;  // index into kFuncs
    std::vector<std::unique_ptr<Node>> kids;
};

const char* const kFuncs[] = {"exp",  "expm1", "log",  "log1p", "sqrt", "sin",
                              "cos",  "tan",   "tanh", "sinh",  "cosh", "atan",
                              "fabs", "pow",   "fmin", "fmax",  "fma"};
constexpr int kNumFuncs = 17, kFirstBinary = 13, kTernary = 16;

struct Parser {
    const char* s;
    int dim, np;
    std::string err;

    void ws() {
        while (*s && std::isspace((unsigned char)*s)) ++s;
    }
    bool eat(char c) {
        ws();
        if (*s == c) {
            ++s;
            return true;
        }
        return false;
    }
    std::unique_ptr<Node> fail(const std::string& m) {
        if (err.empty()) err = m;
        return nullptr;
    }
    std::unique_ptr<Node> expr() {
        auto a = term();
        while (a) {
            ws();
            if (*s != '+' && *s != '-') break;
            const char op = *s++;
            auto b = term();
            if (!b) return nullptr;
            auto n = std::make_unique<Node>();
            n->kind = op == '+' ? Node::ADD : Node::SUB;
            n->kids.push_back(std::move(a));
            n->kids.push_back(std::move(b));
            a = std::move(n);
        }
        return a;
    }
    std::unique_ptr<Node> term() {
        auto a = unary();
        while (a) {
            ws();
            if (*s != '*' && *s != '/') break;
            const char op = *s++;
            auto b = unary();
            if (!b) return nullptr;
            auto n = std::make_unique<Node>();
            n->kind = op == '*' ? Node::MUL : Node::DIV;
            n->kids.push_back(std::move(a));
            n->kids.push_back(std::move(b));
            a = std::move(n);
        }
        return a;
    }
    std::unique_ptr<Node> unary() {
        if (eat('-')) {
            auto a = unary();
            if (!a) return nullptr;
            auto n = std::make_unique<Node>();
            n->kind = Node::NEG;
            n->kids.push_back(std::move(a));
            return n;
        }
        if (eat('+')) return unary();
        return primary();
    }
    std::unique_ptr<Node> primary() {
        ws();
        if (eat('(')) {
            auto a = expr();
            if (!a) return nullptr;
            if (!eat(')')) return fail("missing )");
            return a;
        }
        if (std::isdigit((unsigned char)*s) || *s == '.') {
            char* end = nullptr;
            const double v = std::strtod(s, &end);
            if (end == s) return fail("bad number");
            s = end;
            auto n = std::make_unique<Node>();
            n->kind = Node::NUM;
            n->val = v;
            return n;
        }
        if (std::isalpha((unsigned char)*s)) {
            std::string id;
            while (std::isalnum((unsigned char)*s) || *s == '_') id += *s++;
            if ((id[0] == 'x' || id[0] == 'p') && id.size() > 1 &&
                id.find_first_not_of("0123456789", 1) == std::string::npos) {
                if (id.size() > 2 && id[1] == '0') return fail("leading zero in " + id);
                const int k = id.size() > 4 ? 1000 : std::atoi(id.c_str() + 1);
                auto n = std::make_unique<Node>();
                n->kind = id[0] == 'x' ? Node::VAR : Node::PAR;
                n->index = k;
                if (id[0] == 'x' && k >= dim) return fail("state index out of range");
                if (id[0] == 'p' && k >= np) return fail("parameter index out of range");
                return n;
            }
            int fn = -1;
            for (int k = 0; k < kNumFuncs; ++k)
                if (id == kFuncs[k]) fn = k;
            if (fn < 0) return fail("unknown name " + id);
            const int arity = fn == kTernary ? 3 : fn >= kFirstBinary ? 2 : 1;
            if (!eat('(')) return fail("missing ( after " + id);
            auto n = std::make_unique<Node>();
            n->kind = Node::FUN;
            n->fn = fn;
            for (int k = 0; k < arity; ++k) {
                if (k && !eat(',')) return fail("missing , in " + id);
                auto a = expr();
                if (!a) return nullptr;
                n->kids.push_back(std::move(a));
            }
            if (!eat(')')) return fail("missing ) after " + id);
            return n;
        }
        return fail(std::string("unexpected character ") + (*s ? std::string(1, *s) : "end"));
    }
};

// Evaluates one tree in precision T: a literal is the double that strtod
// reads, rounded to T; every operation rounds to T.
template <class T> T eval(const Node* n, const T* x, const T* p) {
    switch (n->kind) {
        case Node::NUM: return static_cast<T>(n->val);
        case Node::VAR: return x[n->index];
        case Node::PAR: return p[n->index];
        case Node::NEG: return -eval(n->kids[0].get(), x, p);
        case Node::ADD: return eval(n->kids[0].get(), x, p) + eval(n->kids[1].get(), x, p);
        case Node::SUB: return eval(n->kids[0].get(), x, p) - eval(n->kids[1].get(), x, p);
        case Node::MUL: return eval(n->kids[0].get(), x, p) * eval(n->kids[1].get(), x, p);
        case Node::DIV: return eval(n->kids[0].get(), x, p) / eval(n->kids[1].get(), x, p);
        case Node::FUN: {
            const T a = eval(n->kids[0].get(), x, p);
            switch (n->fn) {
                case 0: return std::exp(a);
                case 1: return std::expm1(a);
                case 2: return std::log(a);
                case 3: return std::log1p(a);
                case 4: return std::sqrt(a);
                case 5: return std::sin(a);
                case 6: return std::cos(a);
                case 7: return std::tan(a);
                case 8: return std::tanh(a);
                case 9: return std::sinh(a);
                case 10: return std::cosh(a);
                case 11: return std::atan(a);
                case 12: return std::fabs(a);
            }
            const T b = eval(n->kids[1].get(), x, p);
            if (n->fn == kTernary) return std::fma(a, b, eval(n->kids[2].get(), x, p));
            if (n->fn == 13) return std::pow(a, b);
            if (n->fn == 14) return std::fmin(a, b);
            return std::fmax(a, b);
        }
    }
    return T(0);
}

// Forward-mode derivative: a value and its derivative along one direction.
// The value part follows exactly the operations of eval<double>; the
// derivative part applies the chain rule to each operation.
struct Dual {
    double v, d;
};

Dual eval_dual(const Node* n, const Dual* x, const Dual* p) {
    switch (n->kind) {
        case Node::NUM: return {n->val, 0.0};
        case Node::VAR: return x[n->index];
        case Node::PAR: return p[n->index];
        case Node::NEG: {
            const Dual a = eval_dual(n->kids[0].get(), x, p);
            return {-a.v, -a.d};
        }
        case Node::ADD:
        case Node::SUB:
        case Node::MUL:
        case Node::DIV: {
            const Dual a = eval_dual(n->kids[0].get(), x, p);
            const Dual b = eval_dual(n->kids[1].get(), x, p);
            if (n->kind == Node::ADD) return {a.v + b.v, a.d + b.d};
            if (n->kind == Node::SUB) return {a.v - b.v, a.d - b.d};
            if (n->kind == Node::MUL) return {a.v * b.v, a.d * b.v + a.v * b.d};
            const double q = a.v / b.v;  // (a/b)' = (a' - q b') / b
            return {q, (a.d - q * b.d) / b.v};
        }
        case Node::FUN: {
            const Dual a = eval_dual(n->kids[0].get(), x, p);
            switch (n->fn) {
                case 0: { const double e = std::exp(a.v); return {e, e * a.d}; }
                case 1: return {std::expm1(a.v), std::exp(a.v) * a.d};
                case 2: return {std::log(a.v), a.d / a.v};
                case 3: return {std::log1p(a.v), a.d / (1.0 + a.v)};
                case 4: { const double r = std::sqrt(a.v); return {r, a.d / (2.0 * r)}; }
                case 5: return {std::sin(a.v), std::cos(a.v) * a.d};
                case 6: return {std::cos(a.v), -std::sin(a.v) * a.d};
                case 7: { const double t = std::tan(a.v); return {t, (1.0 + t * t) * a.d}; }
                case 8: { const double t = std::tanh(a.v); return {t, (1.0 - t * t) * a.d}; }
                case 9: return {std::sinh(a.v), std::cosh(a.v) * a.d};
                case 10: return {std::cosh(a.v), std::sinh(a.v) * a.d};
                case 11: return {std::atan(a.v), a.d / (1.0 + a.v * a.v)};
                case 12: return {std::fabs(a.v), a.v >= 0.0 ? a.d : -a.d};  // slope +1 at 0
            }
            const Dual b = eval_dual(n->kids[1].get(), x, p);
            if (n->fn == kTernary) {
                const Dual c = eval_dual(n->kids[2].get(), x, p);
                return {std::fma(a.v, b.v, c.v), a.d * b.v + a.v * b.d + c.d};
            }
            if (n->fn == 13) {
                // d(a^b) = b a^(b-1) a' + a^b log(a) b'; a term whose direction is
                // zero is left out (a constant exponent needs no log of a)
                const double t = std::pow(a.v, b.v);
                double d = 0.0;
                if (a.d != 0.0) d += b.v * std::pow(a.v, b.v - 1.0) * a.d;
                if (b.d != 0.0) d += t * std::log(a.v) * b.d;
                return {t, d};
            }
            // fmin / fmax follow the argument they return (the first on a tie)
            const double t = n->fn == 14 ? std::fmin(a.v, b.v) : std::fmax(a.v, b.v);
            return {t, t == a.v ? a.d : b.d};
        }
    }
    return {0.0, 0.0};
}

constexpr int kExprMaxDim = 16;
constexpr int kExprMaxParams = 32;

struct ExprSystem {
    int dim, np;
    std::vector<std::unique_ptr<Node>> f;
};

bool build(int dim, int np, const char* const* exprs, ExprSystem* out, std::string* err) {
    out->dim = dim;
    out->np = np;
    for (int d = 0; d < dim; ++d) {
        Parser ps{exprs[d], dim, np, ""};
        auto n = ps.expr();
        ps.ws();
        if (n && *ps.s) {
            ps.err = "trailing characters";
            n.reset();
        }
        if (!n) {
            *err = "x" + std::to_string(d) + "': " + ps.err;
            return false;
        }
        out->f.push_back(std::move(n));
    }
    return true;
}

thread_local std::string g_expr_err;

// Classical RK4 with the stage combination in the fixed order
// s = k2 + k3; s = fma(2, s, k1); s = s + k4; x = fma(h/6, s, x), stage
// points y = fma(h/2, k, x) and fma(h, k3, x); with comp != null the
// increment (h/6) s is added by Kahan's compensated summation.
template <class T>
int expr_rk4(int dim, const char* const* exprs, const double* params, int n_params,
             const int32_t* pp_slot, int n_pp, const T* pparams, T* state, T* comp, int64_t n,
             int64_t ld, T h, int64_t nsteps) {
    if (dim < 1 || dim > kExprMaxDim || n_params < 0 || n_params > kExprMaxParams || n < 0 ||
        ld < n || nsteps < 0 || n_pp < 0 || n_pp > 4 || (n_pp > 0 && !pp_slot) ||
        (n_params > 0 && !params))
        return -1;
    for (int k = 0; k < n_pp; ++k)
        if (pp_slot[k] < 0 || pp_slot[k] >= n_params) return -1;
    ExprSystem sys;
    if (!build(dim, n_params, exprs, &sys, &g_expr_err)) return -2;
    const T h2 = h * T(0.5), h6 = h / T(6);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        T p[kExprMaxParams], x[kExprMaxDim], c[kExprMaxDim];
        T k1[kExprMaxDim], k2[kExprMaxDim], k3[kExprMaxDim], k4[kExprMaxDim], y[kExprMaxDim];
        for (int q = 0; q < n_params; ++q) p[q] = static_cast<T>(params[q]);
        for (int q = 0; q < n_pp; ++q) p[pp_slot[q]] = pparams[q * ld + i];
        for (int d = 0; d < dim; ++d) {
            x[d] = state[d * ld + i];
            c[d] = comp ? comp[d * ld + i] : T(0);
        }
        auto f = [&](const T* at, T* out) {
            for (int d = 0; d < dim; ++d) out[d] = eval(sys.f[d].get(), at, p);
        };
        for (int64_t s = 0; s < nsteps; ++s) {
            f(x, k1);
            for (int d = 0; d < dim; ++d) y[d] = std::fma(h2, k1[d], x[d]);
            f(y, k2);
            for (int d = 0; d < dim; ++d) y[d] = std::fma(h2, k2[d], x[d]);
            f(y, k3);
            for (int d = 0; d < dim; ++d) y[d] = std::fma(h, k3[d], x[d]);
            f(y, k4);
            for (int d = 0; d < dim; ++d) {
                T sum = k2[d] + k3[d];
                sum = std::fma(T(2), sum, k1[d]);
                sum = sum + k4[d];
                if (comp) {
                    const T inc = h6 * sum;
                    const T yk = inc - c[d];
                    const T t = x[d] + yk;
                    c[d] = (t - x[d]) - yk;
                    x[d] = t;
                } else {
                    x[d] = std::fma(h6, sum, x[d]);
                }
            }
        }
        for (int d = 0; d < dim; ++d) {
            state[d * ld + i] = x[d];
            if (comp) comp[d * ld + i] = c[d];
        }
    }
    return 0;
}
// The FP64 map of expr_rk4 carried with its derivative along the directions
// dx0 (state), dparams (global parameters) and dpp (per-particle parameters).
int expr_rk4_dual(int dim, const char* const* exprs, const double* params, int n_params,
                  const int32_t* pp_slot, int n_pp, const double* pparams, const double* x0,
                  const double* dx0, const double* dparams, const double* dpp, double* xT, double* dxT,
                  int64_t n, int64_t ld, double h, int64_t nsteps) {
    if (dim < 1 || dim > kExprMaxDim || n_params < 0 || n_params > kExprMaxParams || n < 0 ||
        ld < n || nsteps < 0 || n_pp < 0 || n_pp > 4 || (n_pp > 0 && !pp_slot) ||
        (n_params > 0 && !params))
        return -1;
    for (int k = 0; k < n_pp; ++k)
        if (pp_slot[k] < 0 || pp_slot[k] >= n_params) return -1;
    ExprSystem sys;
    if (!build(dim, n_params, exprs, &sys, &g_expr_err)) return -2;
    const double h2 = h * 0.5, h6 = h / 6.0;
    // y = fma(w, k, x) on duals: value fma(w, k.v, x.v), derivative w k.d + x.d
    auto stage = [](double w, Dual k, Dual x) { return Dual{std::fma(w, k.v, x.v), w * k.d + x.d}; };
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        Dual p[kExprMaxParams], x[kExprMaxDim];
        Dual k1[kExprMaxDim], k2[kExprMaxDim], k3[kExprMaxDim], k4[kExprMaxDim], y[kExprMaxDim];
        for (int q = 0; q < n_params; ++q) p[q] = {params[q], dparams ? dparams[q] : 0.0};
        for (int q = 0; q < n_pp; ++q)
            p[pp_slot[q]] = {pparams[q * ld + i], dpp ? dpp[q * ld + i] : 0.0};
        for (int d = 0; d < dim; ++d) x[d] = {x0[d * ld + i], dx0 ? dx0[d * ld + i] : 0.0};
        auto f = [&](const Dual* at, Dual* out) {
            for (int d = 0; d < dim; ++d) out[d] = eval_dual(sys.f[d].get(), at, p);
        };
        for (int64_t s = 0; s < nsteps; ++s) {
            f(x, k1);
            for (int d = 0; d < dim; ++d) y[d] = stage(h2, k1[d], x[d]);
            f(y, k2);
            for (int d = 0; d < dim; ++d) y[d] = stage(h2, k2[d], x[d]);
            f(y, k3);
            for (int d = 0; d < dim; ++d) y[d] = stage(h, k3[d], x[d]);
            f(y, k4);
            for (int d = 0; d < dim; ++d) {
                Dual sum{k2[d].v + k3[d].v, k2[d].d + k3[d].d};
                sum = {std::fma(2.0, sum.v, k1[d].v), 2.0 * sum.d + k1[d].d};
                sum = {sum.v + k4[d].v, sum.d + k4[d].d};
                x[d] = stage(h6, sum, x[d]);
            }
        }
        for (int d = 0; d < dim; ++d) {
            xT[d * ld + i] = x[d].v;
            dxT[d * ld + i] = x[d].d;
        }
    }
    return 0;
}

}  // namespace

extern "C" {

const char* ffo_expr_error(void) { return g_expr_err.c_str(); }

int ffo_expr_rk4(int dim, const char* const* exprs, const double* params, int n_params,
                 const int32_t* pp_slot, int n_pp, const double* pparams, double* state,
                 int64_t n, int64_t ld, double h, int64_t nsteps) {
    return expr_rk4<double>(dim, exprs, params, n_params, pp_slot, n_pp, pparams, state, nullptr,
                            n, ld, h, nsteps);
}

int ffo_expr_rk4_f32(int dim, const char* const* exprs, const double* params, int n_params,
                     const int32_t* pp_slot, int n_pp, const float* pparams, float* state,
                     float* comp, int64_t n, int64_t ld, float h, int64_t nsteps) {
    return expr_rk4<float>(dim, exprs, params, n_params, pp_slot, n_pp, pparams, state, comp, n,
                           ld, h, nsteps);
}

int ffo_expr_rk4_dual(int dim, const char* const* exprs, const double* params, int n_params,
                      const int32_t* pp_slot, int n_pp, const double* pparams, const double* x0,
                      const double* dx0, const double* dparams, const double* dpp, double* xT,
                      double* dxT, int64_t n, int64_t ld, double h, int64_t nsteps) {
    return expr_rk4_dual(dim, exprs, params, n_params, pp_slot, n_pp, pparams, x0, dx0, dparams,
                         dpp, xT, dxT, n, ld, h, nsteps);
}

}  // extern "C"
