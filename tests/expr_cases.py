"""Expression texts shared by the expression-system tests (test data only:
strings, and the hand-evaluated values of constant expressions)."""

# the built-in Lorenz and Wilson-Cowan right-hand sides, written with the same
# operations in the same order as the compiled-in ones
LORENZ_EXPR = ["p0*(x1-x0)", "fma(x0, p1-x2, -x1)", "fma(x0, x1, -(p2*x2))"]
WC_EXPR = ["1/(1+exp(-(p4*(fma(p0, x0, fma(-p1, x1, p8)) - p5)))) - x0",
           "1/(1+exp(-(p6*(fma(p2, x0, fma(-p3, x1, p9)) - p7)))) - x1"]

# constant right-hand sides and their values (exact in float and double)
CONSTANTS = [("1-2-3", -4), ("2*3+4*5", 26), ("2*3-4/2", 4), ("-2*3", -6), ("8/4/2", 1), ("2-(3-4)", 3),
             ("2*-3", -6), ("--2", 2), ("+2", 2), ("- 2 - -3", 1), ("1e1+.5", 10.5), ("0x10", 16),
             ("fma(2,3,4)", 10), ("pow(2,10)", 1024), ("fmin(3,-1)", -1), ("fmax(3,-1)", 3),
             ("fabs(-2.5)", 2.5), ("sqrt(16)", 4), ("exp(0)", 1), ("log(1)", 0), ("expm1(0)", 0),
             ("(((7)))", 7), ("3 * (1 + 1) / 4", 1.5)]

# texts that are not expressions of a 3-variable system without parameters
BAD = ["x0 +", "x3", "p0*x0", "foo(x0)", "exp x0", "x01", "2*(x0", "x0 x1", "_a", "pow(x0)", "fma(1,2)",
       "", "x", "1e", "(", ")", "x0)", "2..5", "x0 ^ 2", "sin(x0,)", "x0 ** 2", "1 +* 2"]

# integrands of time x0 (the quadrature system is ["1"] + QUAD_EXPRS, dim 15)
QUAD_EXPRS = ["exp(x0)", "expm1(x0)", "log(1+x0)", "log1p(x0)", "sin(x0)", "cos(x0)", "tan(x0)", "tanh(x0)",
              "sinh(x0)", "cosh(x0)", "atan(x0)", "pow(x0, 3)", "1/(1+x0*x0)", "sqrt(1+x0)"]
