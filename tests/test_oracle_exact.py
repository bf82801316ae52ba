"""Pins of the exact oracle (oracle/exact.py) to closed forms, independent
definitions and library routines -- never to itself."""
import itertools
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle import exact


def _rand_int_matrix(rng, lo=-6, hi=7):
    return [float(x) for x in rng.integers(lo, hi, 9)]


def _unimodular(rng):
    """Integer matrix with det +-1 (product of elementary integer shears), so
    its inverse is an integer matrix too."""
    p = np.eye(3, dtype=object)
    for _ in range(4):
        i, j = rng.choice(3, 2, replace=False)
        e = np.eye(3, dtype=object)
        e[i, j] = int(rng.integers(-2, 3))
        p = p.dot(e)
    return p


def _inv_int(p):
    m = [[Fraction(int(p[i, j])) for j in range(3)] for i in range(3)]
    d = exact.det3(m)
    c = exact.cof(m)
    return np.array([[c[j][i] / d for j in range(3)] for i in range(3)], dtype=object)


def _spectrum_closed_forms(lam):
    lam = [Fraction(x) for x in lam]
    mean = sum(lam) / 3
    mu = [x - mean for x in lam]
    j2 = (mu[0] ** 2 + mu[1] ** 2 + mu[2] ** 2) / 2
    j3 = mu[0] * mu[1] * mu[2]
    disc = ((lam[0] - lam[1]) * (lam[0] - lam[2]) * (lam[1] - lam[2])) ** 2
    return sum(lam), j2, j3, disc


def test_diagonal_closed_forms():
    """diag(l): J2 = sum(mu^2)/2, J3 = prod(mu), Delta = prod_{i<j}(l_i - l_j)^2."""
    rng = np.random.default_rng(10)
    for _ in range(50):
        lam = rng.integers(-20, 21, 3) / 8.0
        a = [lam[0], 0, 0, 0, lam[1], 0, 0, 0, lam[2]]
        assert exact.invariants(a) == _spectrum_closed_forms(lam)


def test_similar_integer_matrices_closed_forms():
    """A = P D P^-1 with unimodular integer P: nonsymmetric integer matrices of
    exactly known spectrum -> invariants from the spectrum, exactly."""
    rng = np.random.default_rng(11)
    for _ in range(40):
        p = _unimodular(rng)
        lam = [int(x) for x in rng.integers(-5, 6, 3)]
        d = np.diag(np.array(lam, dtype=object))
        a = p.dot(d).dot(_inv_int(p))
        a9 = [float(x) for x in a.ravel()]
        assert all(Fraction(x) == y for x, y in zip(a9, a.ravel()))  # representable
        assert exact.invariants(a9) == _spectrum_closed_forms(lam)
        roots = exact.eigvals(a9)
        assert all(abs(r - x) < mpmath.mpf(10) ** -60 for r, x in zip(roots, sorted(lam)))


def test_parlett_determinant_equals_definition():
    """Two independent definitions of Delta agree exactly (Eq. disc-determinant)."""
    rng = np.random.default_rng(12)
    for _ in range(30):
        a = list(rng.standard_normal(9))
        assert exact.invariants(a)[3] == exact.discriminant_parlett(a)
    for _ in range(30):
        a = _rand_int_matrix(rng)
        assert exact.invariants(a)[3] == exact.discriminant_parlett(a)


def _naive_j2(a):
    """Alg. alg:J2-naive, the paper's monomial sum (exact arithmetic)."""
    A = exact.to_fraction_matrix(a)
    return (A[0][0] ** 2 - A[0][0] * A[1][1] - A[0][0] * A[2][2] + 3 * A[0][1] * A[1][0]
            + 3 * A[0][2] * A[2][0] + A[1][1] ** 2 - A[1][1] * A[2][2] + 3 * A[1][2] * A[2][1]
            + A[2][2] ** 2) / 3


def _naive_j3(a):
    """Alg. alg:J3-naive, the paper's 21-monomial sum (exact arithmetic)."""
    A = exact.to_fraction_matrix(a)
    a00, a01, a02 = A[0]
    a10, a11, a12 = A[1]
    a20, a21, a22 = A[2]
    return (2 * a00 ** 3 - 3 * a00 ** 2 * a11 - 3 * a00 ** 2 * a22 + 9 * a00 * a01 * a10
            + 9 * a00 * a02 * a20 - 3 * a00 * a11 ** 2 + 12 * a00 * a11 * a22 - 18 * a00 * a12 * a21
            - 3 * a00 * a22 ** 2 + 9 * a01 * a10 * a11 - 18 * a01 * a10 * a22 + 27 * a01 * a12 * a20
            + 27 * a02 * a10 * a21 - 18 * a02 * a11 * a20 + 9 * a02 * a20 * a22 + 2 * a11 ** 3
            - 3 * a11 ** 2 * a22 + 9 * a11 * a12 * a21 - 3 * a11 * a22 ** 2 + 9 * a12 * a21 * a22
            + 2 * a22 ** 3) / 27


def test_naive_monomial_sums_equal_definitions():
    """The paper's monomial expansions (Alg. alg:J2-naive, alg:J3-naive) are an
    independent statement of the same polynomials."""
    rng = np.random.default_rng(13)
    for _ in range(40):
        a = list(rng.standard_normal(9) * 10.0 ** rng.integers(-3, 4))
        _, j2, j3, _ = exact.invariants(a)
        assert j2 == _naive_j2(a)
        assert j3 == _naive_j3(a)


def test_eigvals_vieta_and_numpy():
    """Roots satisfy Vieta's relations with the exact characteristic polynomial
    and agree with LAPACK (numpy.linalg.eigvals) on well-separated spectra."""
    rng = np.random.default_rng(14)
    for _ in range(40):
        a = list(rng.standard_normal(9))
        r = exact.eigvals(a, dps=60)
        i1, i2, i3 = exact.char_poly(a)
        with mpmath.workdps(60):
            tol = mpmath.mpf(10) ** -50
            assert abs(r[0] + r[1] + r[2] - exact._mpf(i1)) < tol
            assert abs(r[0] * r[1] + r[0] * r[2] + r[1] * r[2] - exact._mpf(i2)) < tol
            assert abs(r[0] * r[1] * r[2] - exact._mpf(i3)) < tol
        ref = np.linalg.eigvals(np.array(a).reshape(3, 3))
        ref = sorted(ref, key=lambda z: (z.real, z.imag))
        got = [complex(x) for x in r]
        assert np.allclose(got, ref, atol=1e-10)


def test_eigvals_special_cases():
    assert exact.eigvals([2, 0, 0, 0, 2, 0, 0, 0, 2]) == [2, 2, 2]
    assert [float(x) for x in exact.eigvals([1, 0, 0, 0, 1, 0, 0, 0, 2])] == [1, 1, 2]
    assert [float(x) for x in exact.eigvals([-3, 0, 0, 0, 1, 0, 0, 0, 1.5])] == [-3, 1, 1.5]
    # rotation by 90 degrees about the z axis: eigenvalues -i, i, 1
    r = exact.eigvals_float([0, -1, 0, 1, 0, 0, 0, 0, 1])
    assert np.allclose(r, [-1j, 1j, 1], atol=1e-60)
    # upper triangular: the diagonal
    assert [float(x) for x in exact.eigvals([3, 7, -2, 0, -1, 5, 0, 0, 0.5])] == [-1, 0.5, 3]


def test_eigvals_constructed_near_double():
    """fl(U D U^-1) for U_symm and D2 = diag(-1, 1, 1+d): spectrum within the
    rounding of the construction of the prescribed one."""
    import workloads as w
    for d in (1e-2, 1e-8, 1e-14):
        c = w.paper_path("D2", "symm", [d])
        r = exact.eigvals_float(c["a"][0])
        assert np.allclose(np.real(r), c["lam"][0], atol=1e-15, rtol=0)


def test_gradient_identities():
    """g = 1 -> I; g = lambda -> A^T; g = lambda^2 -> (A^2)^T (sums of the
    eigenprojectors against powers of the eigenvalues)."""
    rng = np.random.default_rng(15)
    import workloads as w
    c = w.differentiation_batch(6, seed=77)
    for a in c["a"]:
        lam = [float(x) for x in exact.eigvals(a)]
        am = np.array(a).reshape(3, 3)
        np.testing.assert_allclose(exact.eigvals_vjp(a, [1, 1, 1]), np.eye(3).ravel(), atol=1e-12)
        np.testing.assert_allclose(exact.eigvals_vjp(a, lam), am.T.ravel(), atol=1e-12)
        np.testing.assert_allclose(exact.eigvals_vjp(a, [x * x for x in lam]), (am @ am).T.ravel(), atol=1e-11)
    del rng


def test_gradient_eigenvector_formula_and_fd():
    """d(lambda_i) = y_i^T dA x_i / (y_i^T x_i) with x_i = V[:, i], y_i^T = V^-1[i, :]
    from the generator; and central differences of the exact eigenvalues."""
    import workloads as w
    c = w.differentiation_batch(5, seed=78, with_basis=True)
    rng = np.random.default_rng(16)
    for m in range(5):
        a = c["a"][m]
        g = rng.standard_normal(3)
        v = c["v"][m].reshape(3, 3)
        vi = c["vinv"][m].reshape(3, 3)
        ref = sum(g[i] * np.outer(vi[i, :], v[:, i]) for i in range(3))
        got = np.array(exact.eigvals_vjp(a, g)).reshape(3, 3)
        np.testing.assert_allclose(got, ref, atol=1e-9 * np.abs(ref).max())
        # central differences (h = 1e-7 on the entry, 40-digit eigenvalues)
        h = 1e-7
        for e in (0, 1, 5, 7):
            ap = np.array(a, dtype=np.float64); ap[e] += h
            am = np.array(a, dtype=np.float64); am[e] -= h
            lp = [float(x) for x in exact.eigvals(ap, 40)]
            lm = [float(x) for x in exact.eigvals(am, 40)]
            fd = sum(g[k] * (lp[k] - lm[k]) for k in range(3)) / (ap[e] - am[e])
            assert abs(fd - got.ravel()[e]) < 1e-5 * max(1.0, np.abs(got).max())


def _fd_grad(f, a, h):
    out = []
    for e in range(9):
        ap = list(a); ap[e] = Fraction(ap[e]) + h
        am = list(a); am[e] = Fraction(am[e]) - h
        out.append((f(ap) - f(am)) / (2 * h))
    return out


def _inv_exact_frac(a9):
    """invariants of a matrix given as 9 Fractions (finite differences)."""
    a = [[Fraction(a9[3 * i + j]) for j in range(3)] for i in range(3)]
    s = exact.dev(a)
    j2 = exact.trace(exact.matmul(s, s)) / 2
    j3 = exact.det3(s)
    return j2, j3, 4 * j2 ** 3 - 27 * j3 ** 2


def test_bound_scales_are_jacobian_norms():
    """The bound scales use the Jacobians of Lemmas lem:J2-condition,
    lem:J3-jacobian and lem:disc-jacobian; check each against central
    differences of the exact invariant (exact arithmetic, h = 2^-30)."""
    rng = np.random.default_rng(17)
    h = Fraction(1, 2 ** 30)
    for _ in range(6):
        a = list(rng.standard_normal(9))
        s = exact.bound_scales(a)
        af = exact.to_fraction_matrix(a)
        ns = float(exact.frob_sq(exact.dev(af))) ** 0.5
        for idx, key in ((0, "J2"), (1, "J3"), (2, "Delta")):
            g = _fd_grad(lambda x: _inv_exact_frac(x)[idx], [Fraction(x) for x in a], h)
            gn = float(sum(x * x for x in g)) ** 0.5
            assert abs(gn * ns - s[key]) <= 1e-6 * s[key]
        assert s["I1"] == pytest.approx(float(np.linalg.norm(a)), rel=1e-15)


def test_scaled_identity_and_j3_example():
    """Scaled identity: J2 = J3 = Delta = 0 (definitions); diag(1,2,3): J3 = 0
    (Sec. "Invariant J3" example, tests/golden/paper_j3_example.txt)."""
    assert exact.invariants([0.7, 0, 0, 0, 0.7, 0, 0, 0, 0.7])[1:] == (0, 0, 0)
    assert exact.invariants([1, 0, 0, 0, 2, 0, 0, 0, 3])[2] == 0


def test_exhaustive_small_integer_triangular():
    """Triangular matrices: invariants depend only on the diagonal."""
    for d in itertools.product((-1, 0, 2), repeat=3):
        up = [d[0], 3, -1, 0, d[1], 2, 0, 0, d[2]]
        lo = [d[0], 0, 0, 5, d[1], 0, -4, 1, d[2]]
        dg = [d[0], 0, 0, 0, d[1], 0, 0, 0, d[2]]
        assert exact.invariants(up) == exact.invariants(dg) == exact.invariants(lo)


def test_mohr_coulomb_closed_form_and_fd():
    """For |K| < 1 the pair (1, 3) attains the maximum, so
    f = (m s_3 - s_1)/S_yc - 1 and df/dsigma = (m E_3 - E_1)/S_yc; checked
    against that closed form and central differences of the exact f."""
    rng = np.random.default_rng(18)
    for _ in range(12):
        s = rng.standard_normal(6) * 50
        a = [s[0], s[3], s[4], s[3], s[1], s[5], s[4], s[5], s[2]]
        m, syc = float(rng.uniform(1.5, 12)), float(rng.uniform(20, 200))
        f, g = exact.mohr_coulomb(a, syc, m)
        lam = [float(x) for x in exact.eigvals(a)]
        assert f == pytest.approx((m * lam[2] - lam[0]) / syc - 1, rel=1e-14, abs=1e-14)
        ref = exact.eigvals_vjp(a, [-1 / syc, 0.0, m / syc])
        np.testing.assert_allclose(g, ref, rtol=1e-12, atol=1e-15)
        h = 1e-6
        for e in (0, 1, 4, 8):
            ap = list(a); ap[e] += h
            am = list(a); am[e] -= h
            fd = (exact.mohr_coulomb(ap, syc, m, 40)[0] - exact.mohr_coulomb(am, syc, m, 40)[0]) / (2 * h)
            assert abs(fd - g[e]) < 1e-6


def test_eigenprojector_identities():
    """sum E_k = I, sum lambda_k E_k = A, E_k E_j = delta_kj E_k, and
    E_k = x_k y_k^T with x_k = V[:, k], y_k^T = V^-1[k, :] of the generator."""
    import workloads as w
    c = w.differentiation_batch(6, seed=79, with_basis=True)
    for m in range(6):
        a = c["a"][m]
        e = np.array(exact.eigenprojectors(a)).reshape(3, 3, 3)
        lam = [float(x) for x in exact.eigvals(a)]
        am = np.array(a).reshape(3, 3)
        np.testing.assert_allclose(e.sum(0), np.eye(3), atol=1e-10)
        np.testing.assert_allclose(sum(lam[k] * e[k] for k in range(3)), am, atol=1e-10)
        for k in range(3):
            for j in range(3):
                np.testing.assert_allclose(e[k] @ e[j], e[k] if k == j else 0 * e[k], atol=1e-8)
        v = c["v"][m].reshape(3, 3)
        vi = c["vinv"][m].reshape(3, 3)
        for k in range(3):
            np.testing.assert_allclose(e[k], np.outer(v[:, k], vi[k, :]), atol=1e-9 * np.abs(e[k]).max())


def _spd(rng, lo=0.3, hi=3.0):
    """Symmetric positive definite: Q diag(l) Q^T with Haar Q, l ~ U[lo, hi]."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    lam = np.sort(rng.uniform(lo, hi, 3))
    return (q @ np.diag(lam) @ q.T).ravel()


def test_matrix_functions_against_scipy():
    """exp against scipy.linalg.expm (Pade scaling and squaring) on general
    matrices; log and sqrt against scipy.linalg.logm / sqrtm (Schur based) on
    symmetric positive definite ones: independent algorithms."""
    import scipy.linalg as sl
    import workloads as w
    c = w.differentiation_batch(6, seed=11)
    for m in range(6):
        a = c["a"][m]
        e = np.array(exact.matrix_function(a, "exp")).reshape(3, 3)
        ref = sl.expm(a.reshape(3, 3))
        assert np.abs(e - ref).max() <= 1e-12 * np.abs(ref).max()
    rng = np.random.default_rng(12)
    for _ in range(6):
        a = _spd(rng)
        for fn, ref in (("log", sl.logm(a.reshape(3, 3))), ("sqrt", sl.sqrtm(a.reshape(3, 3)))):
            got = np.array(exact.matrix_function(a, fn)).reshape(3, 3)
            assert np.abs(got - np.real(ref)).max() <= 1e-12 * np.abs(ref).max(), fn


def test_matrix_functions_closed_forms_and_identities():
    """f(diag(d)) = diag(f(d)); f of a similarity transform is the similarity
    transform of f on the diagonal (exactly invertible integer basis);
    sqrt(A)^2 = A and exp(log A) = A."""
    d = [0.5, 2.0, 7.0]
    a = np.diag(d).ravel()
    for fn, f in (("exp", np.exp), ("log", np.log), ("sqrt", np.sqrt)):
        assert np.allclose(np.array(exact.matrix_function(a, fn)).reshape(3, 3), np.diag(f(d)), rtol=1e-15, atol=0)
    p = np.array([[1, 1, 0], [0, 1, 1], [0, 0, 1]], dtype=float)   # unimodular
    pinv = np.array([[1, -1, 1], [0, 1, -1], [0, 0, 1]], dtype=float)
    b = (p @ np.diag(d) @ pinv).ravel()
    got = np.array(exact.matrix_function(b, "exp")).reshape(3, 3)
    ref = p @ np.diag(np.exp(d)) @ pinv
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
    rng = np.random.default_rng(13)
    a = _spd(rng)
    s = np.array(exact.matrix_function(a, "sqrt")).reshape(3, 3)
    assert np.abs(s @ s - a.reshape(3, 3)).max() <= 1e-14 * np.abs(a).max()
    lg = np.array(exact.matrix_function(a, "log"))
    assert np.abs(np.array(exact.matrix_function(lg, "exp")) - a).max() <= 1e-13 * np.abs(a).max()
    with pytest.raises(ValueError):
        exact.matrix_function(np.diag([-1.0, 1.0, 2.0]).ravel(), "log")


def test_matrix_function_vjp_against_torch_and_differences():
    """The Daleckii-Krein vector-Jacobian product against torch's autograd of
    torch.linalg.matrix_exp (an independent algorithm, binary64 on the CPU)
    for exp, and against central differences of the exact f(A) (80 digits,
    h = 1e-20) for exp, log and sqrt."""
    import torch
    import workloads as w
    c = w.differentiation_batch(4, seed=14)
    rng = np.random.default_rng(15)
    for m in range(4):
        a = c["a"][m]
        g = rng.standard_normal(9)
        got = np.array(exact.matrix_function_vjp(a, "exp", g))
        at = torch.tensor(a.reshape(3, 3), dtype=torch.float64, requires_grad=True)
        (torch.linalg.matrix_exp(at) * torch.tensor(g.reshape(3, 3))).sum().backward()
        ref = at.grad.numpy().ravel()
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max(), m
    a = _spd(rng)
    for fn in ("exp", "log", "sqrt"):
        g = rng.standard_normal(9)
        got = exact.matrix_function_vjp(a, fn, g)
        with mpmath.workdps(80):
            h = mpmath.mpf("1e-20")
            for e in range(9):
                ap = [mpmath.mpf(float(x)) for x in a]
                am = list(ap)
                ap[e] += h
                am[e] -= h
                # exact f at the perturbed matrices through the eigenprojector sum
                fp = _matrix_function_mp(ap, fn)
                fm = _matrix_function_mp(am, fn)
                fd = sum(mpmath.mpf(float(g[i])) * (fp[i] - fm[i]) / (2 * h) for i in range(9))
                assert abs(float(fd) - got[e]) <= 1e-13 * max(abs(x) for x in got), (fn, e)


def _matrix_function_mp(a_mp, fn):
    """f(A) for an mpmath 9-vector A (characteristic-polynomial roots by
    mpmath.polyroots and the Frobenius covariants), for the differences."""
    a = [[a_mp[3 * i + j] for j in range(3)] for i in range(3)]
    tr_a = a[0][0] + a[1][1] + a[2][2]
    i2 = (a[0][0] * a[1][1] - a[0][1] * a[1][0]) + (a[0][0] * a[2][2] - a[0][2] * a[2][0]) + \
         (a[1][1] * a[2][2] - a[1][2] * a[2][1])
    det = (a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0])
           + a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]))
    lam = sorted(mpmath.re(r) for r in mpmath.polyroots([1, -tr_a, i2, -det], maxsteps=200, extraprec=200))
    f = exact.MATRIX_FUNCTIONS[fn]
    out = [mpmath.mpf(0)] * 9
    for k in range(3):
        i, j = [m for m in range(3) if m != k]
        den = (lam[k] - lam[i]) * (lam[k] - lam[j])
        for r in range(3):
            for c in range(3):
                e = sum((a[r][t] - (lam[i] if r == t else 0)) * (a[t][c] - (lam[j] if t == c else 0)) for t in range(3))
                out[3 * r + c] += f(lam[k]) * e / den
    return out
