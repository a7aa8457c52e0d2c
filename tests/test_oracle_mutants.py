"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake (a wrong weight, sign, index or operand, a
dropped term) in a copy of oracle/ffo.cpp, builds it on the CPU, points the
oracle wrapper at it (FFO_LIB) and runs the pin tests in a subprocess: at
least one pin must fail.  The unmodified source must pass the same run.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ffo.cpp")
PINS = ["tests/test_oracle_tableau.py", "tests/test_oracle_linear.py", "tests/test_oracle_lorenz.py",
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


def build_variant(tmp_path, name, text):
    src = tmp_path / f"{name}.cpp"
    src.write_text(text)
    lib = tmp_path / f"{name}.so"
    subprocess.run(["g++", "-std=c++17", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", "-I", os.path.join(ROOT, "oracle"), str(src), "-o", str(lib)], check=True)
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
