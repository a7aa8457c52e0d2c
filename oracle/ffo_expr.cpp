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

}  // extern "C"
