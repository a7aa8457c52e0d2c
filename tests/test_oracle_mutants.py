"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake (a wrong weight, sign, index or operand, a
dropped term) in a copy of oracle/ffo.cpp (or oracle/ffo_expr.cpp for the
expression evaluator), builds it on the CPU, points the
oracle wrapper at it (FFO_LIB) and runs the pin tests in a subprocess: at
least one pin must fail.  The unmodified source must pass the same run.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ffo.cpp")
SRC_EXPR = os.path.join(ROOT, "oracle", "ffo_expr.cpp")
PINS = ["tests/test_oracle_expr.py", "tests/test_oracle_tableau.py", "tests/test_oracle_linear.py", "tests/test_oracle_lorenz.py",
        "tests/test_oracle_wilson_cowan.py", "tests/test_oracle_hh.py", "tests/test_oracle_adjoint.py",
        "tests/test_oracle_histogram.py", "tests/test_oracle_reset.py"]

MUTANTS = {
    "rk4_weight": ("s = fma_(T(2), s, k1[d]);", "s = fma_(T(3), s, k1[d]);"),
    "rk4_stage4_coef": ("y[d] = fma_(h, k3[d], x[d]);\n    rhs(sys, dim, p, y, k4);\n    for (int d = 0; d < dim; ++d) {\n        T s",
                        "y[d] = fma_(h2, k3[d], x[d]);\n    rhs(sys, dim, p, y, k4);\n    for (int d = 0; d < dim; ++d) {\n        T s"),
    "rk4_stage3_slope": ("for (int d = 0; d < dim; ++d) y[d] = fma_(h2, k2[d], x[d]);\n    rhs(sys, dim, p, y, k3);\n    for (int d = 0; d < dim; ++d) y[d] = fma_(h, k3[d], x[d]);\n    rhs(sys, dim, p, y, k4);\n    for (int d = 0; d < dim; ++d) {\n        T s",
                         "for (int d = 0; d < dim; ++d) y[d] = fma_(h2, k1[d], x[d]);\n    rhs(sys, dim, p, y, k3);\n    for (int d = 0; d < dim; ++d) y[d] = fma_(h, k3[d], x[d]);\n    rhs(sys, dim, p, y, k4);\n    for (int d = 0; d < dim; ++d) {\n        T s"),
    "lorenz_sign": ("f[1] = fma_(x[0], r - x[2], -x[1]);", "f[1] = fma_(x[0], r - x[2], x[1]);"),
    "lorenz_transposed": ("f[0] = sigma * (x[1] - x[0]);", "f[0] = sigma * (x[0] - x[1]);"),
    "lorenz_dropped_term": ("f[2] = fma_(x[0], x[1], -(beta * x[2]));", "f[2] = x[0] * x[1];"),
    "wc_index": ("fma_(-p[1], I, p[8])", "fma_(-p[3], I, p[8])"),
    "wc_sigmoid_shift": ("exp_(-(p[4] * (uE - p[5])))", "exp_(-(p[4] * uE - p[5]))"),
    "hh_ring_index": ("x[5 * ((j + N - 1) % N) + 4]", "x[5 * ((j + 1) % N) + 4]"),
    "hh_rate_constant": ("r.bm = T(4.0) * exp_(v65 * km18);", "r.bm = T(4.0) * exp_(v65 * km20);"),
    "hh_gate_power": ("const T IK = (gK * (n2 * n2)) * (EK - V);", "const T IK = (gK * (n2 * n)) * (EK - V);"),
    "hh_sign": ("f[5 * j + 3] = fma_(r.an, T(1) - n, -(r.bn * n));", "f[5 * j + 3] = fma_(r.an, T(1) - n, (r.bn * n));"),
    "adjoint_stage_weight": ("const double wprev[4] = {h2, h2, h, 0.0};", "const double wprev[4] = {h2, h, h2, 0.0};"),
    "jacobian_entry": ("const double Jl[9] = {-sigma, sigma, 0.0, r - Z, -1.0, -X, Y, X, -beta};",
                       "const double Jl[9] = {-sigma, sigma, 0.0, r + Z, -1.0, -X, Y, X, -beta};"),
    "hist_edge": ("if (vx >= 0.0 && vx < nx && vy >= 0.0 && vy < ny) {", "if (vx >= 0.0 && vx <= nx && vy >= 0.0 && vy < ny) {"),
    "kahan_sign": ("c[d] = (t - x[d]) - yk;", "c[d] = (t - x[d]) + yk;"),
    "philox_multiplier": ("const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];",
                          "const uint64_t p1 = (uint64_t)0xCD9E8D55u * c[2];"),
    "philox_key_bump": ("k1 += 0xBB67AE85u;", "k1 += 0xBB67AE84u;"),
    "philox_rounds": ("for (int round = 0; round < 10; ++round) {", "for (int round = 0; round < 9; ++round) {"),
    "reset_uniform_shift": ("((double)(a >> 5) * 67108864.0 + (double)(b >> 6))",
                            "((double)(a >> 6) * 67108864.0 + (double)(b >> 6))"),
    "reset_age_rule": ("if (escaped(dim, x, bound_lo, bound_hi) || (max_age >= 0 && a > max_age)) {\n                redraw(dim, box_lo, box_hi, seed, id_offset + (uint64_t)i, r, x);\n                a = 0;",
                       "if (escaped(dim, x, bound_lo, bound_hi) || (max_age >= 0 && a >= max_age)) {\n                redraw(dim, box_lo, box_hi, seed, id_offset + (uint64_t)i, r, x);\n                a = 0;"),
}

# mistakes in the expression evaluator (oracle/ffo_expr.cpp)
MUTANTS_EXPR = {
    "expr_sub_operands": ("case Node::SUB: return eval(n->kids[0].get(), x, p) - eval(n->kids[1].get(), x, p);",
                          "case Node::SUB: return eval(n->kids[1].get(), x, p) - eval(n->kids[0].get(), x, p);"),
    "expr_sum_binds_product": ("            const char op = *s++;\n            auto b = term();",
                               "            const char op = *s++;\n            auto b = unary();"),
    "expr_right_assoc": ("            const char op = *s++;\n            auto b = term();",
                         "            const char op = *s++;\n            auto b = expr();"),
    "expr_function_table": ("case 5: return std::sin(a);", "case 5: return std::cos(a);"),
    "expr_negation": ("case Node::NEG: return -eval(n->kids[0].get(), x, p);",
                      "case Node::NEG: return eval(n->kids[0].get(), x, p);"),
    "expr_stage4": ("for (int d = 0; d < dim; ++d) y[d] = std::fma(h, k3[d], x[d]);",
                    "for (int d = 0; d < dim; ++d) y[d] = std::fma(h2, k3[d], x[d]);"),
    "expr_pp_slot": ("for (int q = 0; q < n_pp; ++q) p[pp_slot[q]] = pparams[q * ld + i];",
                     "for (int q = 0; q < n_pp; ++q) p[q] = pparams[q * ld + i];"),
    "expr_kahan_sign": ("c[d] = (t - x[d]) - yk;", "c[d] = (t - x[d]) + yk;"),
    "dual_cos_sign": ("case 6: return {std::cos(a.v), -std::sin(a.v) * a.d};",
                      "case 6: return {std::cos(a.v), std::sin(a.v) * a.d};"),
    "dual_quotient_rule": ("return {q, (a.d - q * b.d) / b.v};", "return {q, (a.d + q * b.d) / b.v};"),
    "dual_fma_addend": ("return {std::fma(a.v, b.v, c.v), a.d * b.v + a.v * b.d + c.d};",
                        "return {std::fma(a.v, b.v, c.v), a.d * b.v + a.v * b.d};"),
    "dual_pow_exponent": ("if (b.d != 0.0) d += t * std::log(a.v) * b.d;", "if (b.d != 0.0) d += t * b.d;"),
    "dual_stage_weight": ("return Dual{std::fma(w, k.v, x.v), w * k.d + x.d};",
                          "return Dual{std::fma(w, k.v, x.v), k.d + x.d};"),
    "dual_fmin_route": ("return {t, t == a.v ? a.d : b.d};", "return {t, t == a.v ? b.d : a.d};"),
}


def build_variant(tmp_path, name, text, text_expr=None):
    src = tmp_path / f"{name}.cpp"
    src.write_text(text)
    src_expr = tmp_path / f"{name}_expr.cpp"
    src_expr.write_text(text_expr if text_expr is not None else open(SRC_EXPR).read())
    lib = tmp_path / f"{name}.so"
    subprocess.run(["g++", "-std=c++17", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", "-I", os.path.join(ROOT, "oracle"), str(src), str(src_expr), "-o", str(lib)],
                   check=True)
    return lib


def run_pins(lib):
    env = dict(os.environ, FFO_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def test_unmodified_copy_passes(tmp_path):
    lib = build_variant(tmp_path, "original", open(SRC).read())
    rc, out = run_pins(lib)
    assert rc == 0, out


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, name):
    before, after = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(before) == 1, f"mutation site of {name} not found exactly once"
    lib = build_variant(tmp_path, name, text.replace(before, after))
    rc, out = run_pins(lib)
    assert rc != 0, f"no pin failed for mutant {name}:\n{out}"


@pytest.mark.parametrize("name", sorted(MUTANTS_EXPR))
def test_pins_catch_expression_mutant(tmp_path, name):
    before, after = MUTANTS_EXPR[name]
    text = open(SRC_EXPR).read()
    assert text.count(before) == 1, f"mutation site of {name} not found exactly once"
    lib = build_variant(tmp_path, name, open(SRC).read(), text.replace(before, after))
    rc, out = run_pins(lib)
    assert rc != 0, f"no pin failed for mutant {name}:\n{out}"
