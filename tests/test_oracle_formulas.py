"""The plain oracle's generated formulas (oracle/gen_formulas.py ->
oracle/eig3_plain_formulas.h): the committed header is the generator's
output, and what the generator derives is pinned to independent
definitions."""
import numpy as np

from oracle import exact
from oracle import gen_formulas as g


def test_header_is_the_generator_output():
    with open(g.HEADER) as f:
        assert f.read() == g.header_text()


def test_factor_classes_of_the_cauchy_binet_expansion():
    """64 nonzero minors in 14 classes of sizes 9, 6 x 3, 8 x 3, 2 x 6, 1; the
    weighted sum of products equals 4 J2^3 - 27 J3^2 as polynomials (and,
    numerically, the exact Delta on random rational matrices)."""
    cls = g.factor_classes()
    assert sorted(w for w, _, _ in cls) == sorted([9, 6, 6, 6, 8, 8, 8, 2, 2, 2, 2, 2, 2, 1])
    g.check_factors(cls)
    rng = np.random.default_rng(3)
    for _ in range(20):
        a = rng.integers(-20, 21, 9).astype(np.float64) / 8.0
        at = [a[k] for k in g.TRANSPOSE]

        def ev(p, x):
            from fractions import Fraction
            return sum(c * np.prod([Fraction(x[k]) ** m[k] for k in range(9)]) for m, c in p.items())
        val = sum(w * ev(u, a) * ev(u, at) for w, u, _ in cls)
        assert val == exact.invariants(a)[3]


def test_factors_vanish_at_a_double_eigenvalue():
    """Every factor vanishes when A has a repeated eigenvalue with a
    two-dimensional eigenspace (the Cayley-Hamilton argument of the
    discriminant section): A = V diag(2, 2, 5) V^-1 with an integer
    unimodular V."""
    from fractions import Fraction
    v = np.array([[1, 1, 0], [0, 1, 1], [1, 1, 1]])
    assert round(abs(np.linalg.det(v))) == 1
    vi = np.round(np.linalg.inv(v)).astype(int)
    a = (v @ np.diag([2, 2, 5]) @ vi).ravel().astype(np.float64)
    for _, u, _ in g.factor_classes():
        val = sum(c * np.prod([Fraction(a[k]) ** m[k] for k in range(9)]) for m, c in u.items())
        assert val == 0


def test_naive_expansions_equal_the_definitions():
    from fractions import Fraction
    j2, j3 = g.naive_polys()
    rng = np.random.default_rng(4)
    for _ in range(20):
        a = rng.integers(-30, 31, 9).astype(np.float64) / 4.0
        ev = lambda p: sum(c * np.prod([Fraction(a[k]) ** m[k] for k in range(9)]) for m, c in p.items())
        ex = exact.invariants(a)
        assert ev(j2) == 3 * ex[1] and ev(j3) == 27 * ex[2]


def test_a_wrong_sign_fails_the_identity():
    """Planted in the generator's output on the CPU: flipping one term of one
    factor breaks the checked identity (the check is not vacuous)."""
    import pytest
    cls = g.factor_classes()
    w, u, terms = cls[7]
    m = next(iter(u))
    bad = dict(u)
    bad[m] = -bad[m]
    with pytest.raises(AssertionError):
        g.check_factors(cls[:7] + [(w, bad, terms)] + cls[8:])
