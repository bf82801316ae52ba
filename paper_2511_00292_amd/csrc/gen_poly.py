"""Derive the polynomial coefficients of the device arctangent.

atan(z) = z * P(z^2) on |z| <= tan(pi/8) = sqrt(2) - 1 (after the reduction
atan(q) = pi/4 + atan((q - 1)/(q + 1)) for q in (tan(pi/8), 1]).
P is fitted to f(u) = atan(sqrt(u))/sqrt(u) on u in [0, (sqrt(2)-1)^2] by
weighted least squares on Chebyshev nodes (relative error), in 60-digit
mpmath arithmetic, then checked on a dense grid.  Prints C++ constants.

Usage: python gen_poly.py  (the output is pasted into eig3_math.hpp)
"""
import mpmath

mpmath.mp.dps = 60


def fit(degree: int, nodes: int = 400):
    lo, hi = mpmath.mpf(0), (mpmath.sqrt(2) - 1) ** 2
    us = [lo + (hi - lo) * (1 - mpmath.cos(mpmath.pi * (k + mpmath.mpf(0.5)) / nodes)) / 2 for k in range(nodes)]

    def f(u):
        if u == 0:
            return mpmath.mpf(1)
        s = mpmath.sqrt(u)
        return mpmath.atan(s) / s

    rows = [[u ** j for j in range(degree + 1)] for u in us]
    rhs = [f(u) for u in us]
    # relative weighting: f >= 0.88 on the interval, so plain least squares
    # is within a few percent of the relative fit
    a = mpmath.matrix(rows)
    b = mpmath.matrix(rhs)
    coef = mpmath.lu_solve(a.T * a, a.T * b)
    grid = [lo + (hi - lo) * k / 20000 for k in range(20001)]
    err = max(abs(sum(coef[j] * u ** j for j in range(degree + 1)) / f(u) - 1) for u in grid)
    return [coef[j] for j in range(degree + 1)], err


if __name__ == "__main__":
    for name, deg in (("f64", 10), ("f32", 4)):
        c, e = fit(deg)
        print(f"// atan {name}: degree {deg} in z^2, max relative error {mpmath.nstr(e, 3)}")
        for j, x in enumerate(c):
            print(f"    {mpmath.nstr(x, 25)},  // z^{2 * j + 1}")
