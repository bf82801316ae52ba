"""Exact / extended-precision reference for closed-form 3x3 eigenvalues.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything under ``oracle/``.
The product path (the HIP library and its Python binding) never does.

Habera & Zilian, "Numerically stable evaluation of closed-form expressions
for eigenvalues of 3x3 matrices" (arXiv 2511.00292), measure every forward
error against a high-precision value of the *definition* evaluated at the
stored floating-point matrix fl(A) (Sec. "Benchmarks", Eq. test-matrix and
the forward-error definition right after it).  This module is that value:

* invariants (Eq. principal-invariants, and Delta defined beside
  Eq. triple-angle-arctan) are evaluated in exact rational arithmetic
  (``fractions.Fraction``) from the exact dyadic value of each stored double:
  I1 = tr A, S = dev A = A - (I1/3) I, J2 = tr(S^2)/2, J3 = det S,
  Delta = 4 J2^3 - 27 J3^2;
* the discriminant is also available through Parlett's independent
  definition Delta = det B, B_ij = <A^(i-1), (A^(j-1))^T> (Sec. "Discriminant",
  Eq. disc-determinant), used to pin the first one;
* eigenvalues are the roots of the characteristic polynomial
  p(l) = l^3 - I1 l^2 + I2 l - I3 of fl(A), obtained with Cardano's formula
  in complex mpmath arithmetic from the exact invariants (a different route
  from the trigonometric formula the method uses), sorted ascending;
* the gradient d(lambda_k)/dA = E_k^T (Sec. "Introduction and motivation",
  the eigenprojector relation) with E_k the Frobenius covariant
  prod_{j != k} (A - l_j I) / (l_k - l_j);
* the stability-bound scales of Lemma lem:J2-condition / Thm
  thm:J2-fwd-stability, Lemma lem:J3-fwd-stability, Lemma
  lem:disc-fwd-stability and Lemma lem:eigvals-fwd-stability, with C = 1
  and Frobenius norms, as the paper plots them.

Everything here is slow pure Python and intended for a few thousand matrices.
Matrices are given as 9 row-major entries A00, A01, A02, A10, ..., A22.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Sequence

import mpmath

EPS64 = 2.0 ** -53  # unit roundoff of IEEE binary64 (Sec. "Numerical stability")
EPS32 = 2.0 ** -24  # the same quantity for binary32 (reading: same model, t = 24)

_ZERO = Fraction(0)
_ONE = Fraction(1)


# ----------------------------------------------------------------------------
# small exact 3x3 helpers (lists of lists of Fraction)
# ----------------------------------------------------------------------------

def to_fraction_matrix(a9: Sequence[float]) -> list[list[Fraction]]:
    """Exact rational value of the 9 stored doubles (row-major)."""
    if len(a9) != 9:
        raise ValueError("expected 9 entries")
    return [[Fraction(float(a9[3 * i + j])) for j in range(3)] for i in range(3)]


def identity() -> list[list[Fraction]]:
    return [[_ONE if i == j else _ZERO for j in range(3)] for i in range(3)]


def trace(m) -> Fraction:
    return m[0][0] + m[1][1] + m[2][2]


def transpose(m):
    return [[m[j][i] for j in range(3)] for i in range(3)]


def matmul(x, y):
    return [[sum((x[i][k] * y[k][j] for k in range(3)), _ZERO) for j in range(3)] for i in range(3)]


def add(x, y, alpha=_ONE):
    """x + alpha * y"""
    return [[x[i][j] + alpha * y[i][j] for j in range(3)] for i in range(3)]


def scale(x, alpha):
    return [[alpha * x[i][j] for j in range(3)] for i in range(3)]


def det3(m) -> Fraction:
    """Determinant by cofactor expansion along the first row."""
    return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
            - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
            + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))


def cof(m):
    """Cofactor matrix: cof(X)_ij = (-1)^(i+j) * minor_ij, so that the
    derivative of det at X in direction dX is <cof X, dX> (the identity used in
    the proof of Lemma lem:J3-jacobian)."""
    out = [[_ZERO] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            r = [k for k in range(3) if k != i]
            c = [k for k in range(3) if k != j]
            minor = m[r[0]][c[0]] * m[r[1]][c[1]] - m[r[0]][c[1]] * m[r[1]][c[0]]
            out[i][j] = minor if (i + j) % 2 == 0 else -minor
    return out


def dev(m):
    """Deviatoric part dev(X) = X - tr(X)/3 * I."""
    return add(m, identity(), -trace(m) / 3)


def frob_sq(m) -> Fraction:
    return sum((m[i][j] * m[i][j] for i in range(3) for j in range(3)), _ZERO)


# ----------------------------------------------------------------------------
# invariants: the definitions, exactly
# ----------------------------------------------------------------------------

def invariants(a9: Sequence[float]) -> tuple[Fraction, Fraction, Fraction, Fraction]:
    """(I1, J2, J3, Delta) of the stored matrix, exactly.

    I1 = tr A; J2 = tr(dev(A)^2)/2; J3 = det(dev A)  (Eq. principal-invariants)
    Delta = 4 J2^3 - 27 J3^2  (definition beside Eq. triple-angle-arctan)
    """
    a = to_fraction_matrix(a9)
    i1 = trace(a)
    s = dev(a)
    j2 = trace(matmul(s, s)) / 2
    j3 = det3(s)
    disc = 4 * j2 ** 3 - 27 * j3 ** 2
    return i1, j2, j3, disc


def discriminant_parlett(a9: Sequence[float]) -> Fraction:
    """Delta = det B with B_ij = <A^(i-1), (A^(j-1))^T>, i, j = 1..3
    (Eq. disc-determinant; <X, Y> = sum_ij X_ij Y_ij)."""
    a = to_fraction_matrix(a9)
    powers = [identity(), a, matmul(a, a)]
    b = [[sum((powers[i][r][c] * transpose(powers[j])[r][c] for r in range(3) for c in range(3)), _ZERO)
          for j in range(3)] for i in range(3)]
    return det3(b)


# ----------------------------------------------------------------------------
# eigenvalues: roots of the characteristic polynomial
# ----------------------------------------------------------------------------

def _mpf(q: Fraction):
    return mpmath.mpf(q.numerator) / q.denominator


def char_poly(a9: Sequence[float]) -> tuple[Fraction, Fraction, Fraction]:
    """Exact (I1, I2, I3) of p(l) = l^3 - I1 l^2 + I2 l - I3, with
    I2 = (tr(A)^2 - tr(A^2))/2 and I3 = det A (Fig. typical-eigvals-approach)."""
    a = to_fraction_matrix(a9)
    i1 = trace(a)
    i2 = (i1 * i1 - trace(matmul(a, a))) / 2
    i3 = det3(a)
    return i1, i2, i3


def eigvals(a9: Sequence[float], dps: int = 80) -> list:
    """The three eigenvalues of fl(A), ascending (by real part, then imaginary
    part), as mpmath numbers (``mpf`` when the spectrum is real, ``mpc`` for a
    complex pair, which rounding can produce for a nonsymmetric matrix with a
    near-double eigenvalue).

    Cardano's formula for the depressed cubic m^3 + p m + q = 0 obtained from
    p(l) by l = I1/3 + m:  m_k = w^k C - p / (3 w^k C),
    C = cbrt(-q/2 + sqrt(q^2/4 + p^3/27)), w = exp(2 pi i / 3).
    The sign of the exact discriminant Delta = -4 p^3 - 27 q^2 decides whether
    the spectrum is real (Delta >= 0)."""
    i1, i2, i3 = char_poly(a9)
    # l = i1/3 + m  ->  m^3 + p m + q with
    p = i2 - i1 * i1 / 3
    q = -(2 * i1 ** 3) / 27 + i1 * i2 / 3 - i3
    disc = -4 * p ** 3 - 27 * q ** 2
    with mpmath.workdps(dps):
        shift = _mpf(i1) / 3
        if p == 0 and q == 0:
            roots = [shift, shift, shift]
        else:
            pm, qm = _mpf(p), _mpf(q)
            # the radicand q^2/4 + p^3/27 = -Delta/108 is formed exactly, so an
            # exactly repeated root keeps an exactly zero square root
            inner = mpmath.sqrt(mpmath.mpc(_mpf(q * q / 4 + p ** 3 / 27)))
            base = -qm / 2 + inner
            if abs(base) == 0:  # choose the other branch of the square root
                base = -qm / 2 - inner
            c = mpmath.cbrt(base)  # any of the three cube roots will do
            w = mpmath.exp(2j * mpmath.pi / 3)
            roots = []
            for k in range(3):
                ck = c * w ** k
                roots.append(shift + ck - pm / (3 * ck))
            if disc >= 0:
                roots = [mpmath.re(r) for r in roots]
            else:
                # one real root and a conjugate pair: make the pair exact
                # conjugates so that their order (negative imaginary part
                # first) does not depend on rounding
                roots = sorted(roots, key=lambda r: abs(mpmath.im(r)))
                re_pair = (mpmath.re(roots[1]) + mpmath.re(roots[2])) / 2
                im_pair = (abs(mpmath.im(roots[1])) + abs(mpmath.im(roots[2]))) / 2
                roots = [mpmath.re(roots[0]), mpmath.mpc(re_pair, -im_pair), mpmath.mpc(re_pair, im_pair)]
        roots = sorted(roots, key=lambda r: (mpmath.re(r), mpmath.im(r)))
        return [+r for r in roots]


def eigvals_float(a9: Sequence[float], dps: int = 80) -> list[complex]:
    """Eigenvalues as Python complex numbers (imaginary part 0 for a real spectrum)."""
    return [complex(r) for r in eigvals(a9, dps)]


# ----------------------------------------------------------------------------
# gradient: d(lambda_k)/dA = E_k^T
# ----------------------------------------------------------------------------

def eigvals_vjp(a9: Sequence[float], g: Sequence[float], dps: int = 80) -> list[float]:
    """Vector-Jacobian product sum_k g_k * d(lambda_k)/dA for a real, distinct
    spectrum, as 9 row-major floats.  d(lambda_k)/dA = E_k^T with the Frobenius
    covariant E_k = prod_{j != k} (A - lambda_j I) / (lambda_k - lambda_j)
    (the eigenprojector relation in Sec. "Introduction and motivation")."""
    lam = eigvals(a9, dps)
    if any(isinstance(x, mpmath.mpc) for x in lam):
        raise ValueError("complex spectrum: gradient undefined")
    with mpmath.workdps(dps):
        a = [[mpmath.mpf(float(a9[3 * i + j])) for j in range(3)] for i in range(3)]
        eye = [[mpmath.mpf(1) if i == j else mpmath.mpf(0) for j in range(3)] for i in range(3)]

        def shifted(l):
            return [[a[i][j] - l * eye[i][j] for j in range(3)] for i in range(3)]

        def mm(x, y):
            return [[sum(x[i][k] * y[k][j] for k in range(3)) for j in range(3)] for i in range(3)]

        grad = [[mpmath.mpf(0)] * 3 for _ in range(3)]
        for k in range(3):
            i, j = [m for m in range(3) if m != k]
            num = mm(shifted(lam[i]), shifted(lam[j]))
            den = (lam[k] - lam[i]) * (lam[k] - lam[j])
            for r in range(3):
                for c in range(3):
                    grad[r][c] += mpmath.mpf(float(g[k])) * num[c][r] / den  # E_k^T
        return [float(grad[r][c]) for r in range(3) for c in range(3)]


def _eigenprojectors_mp(a9: Sequence[float], dps: int):
    """(lambda_1..3 ascending, [E_1, E_2, E_3] as 3x3 mpmath matrices): the
    Frobenius covariants E_k = prod_{j != k} (A - lambda_j I) /
    (lambda_k - lambda_j) of a real, distinct spectrum (the projectors of the
    relation E_k^T = d(lambda_k)/dA in Sec. "Introduction and motivation").
    Evaluate inside ``mpmath.workdps(dps)``."""
    lam = eigvals(a9, dps)
    if any(isinstance(x, mpmath.mpc) for x in lam):
        raise ValueError("complex spectrum")
    a = [[mpmath.mpf(float(a9[3 * i + j])) for j in range(3)] for i in range(3)]
    es = []
    for k in range(3):
        i, j = [m for m in range(3) if m != k]
        p = [[a[r][c] - (lam[i] if r == c else 0) for c in range(3)] for r in range(3)]
        q = [[a[r][c] - (lam[j] if r == c else 0) for c in range(3)] for r in range(3)]
        den = (lam[k] - lam[i]) * (lam[k] - lam[j])
        es.append([[sum(p[r][t] * q[t][c] for t in range(3)) / den for c in range(3)] for r in range(3)])
    return lam, es


def eigenprojectors(a9: Sequence[float], dps: int = 80) -> list[float]:
    """E_1, E_2, E_3 (ascending eigenvalues), 27 floats, each row-major."""
    with mpmath.workdps(dps):
        _, es = _eigenprojectors_mp(a9, dps)
        return [float(e[r][c]) for e in es for r in range(3) for c in range(3)]


MATRIX_FUNCTIONS = {"exp": mpmath.exp, "log": mpmath.log, "sqrt": mpmath.sqrt}


def matrix_function(a9: Sequence[float], fn: str, dps: int = 80) -> list[float]:
    """f(A) = sum_k f(lambda_k) E_k, row-major, for f in MATRIX_FUNCTIONS: the
    functions of matrices that closed-form eigenprojectors give (Sec.
    "Introduction and motivation"), for a real, distinct spectrum (log and
    sqrt: positive eigenvalues)."""
    f = MATRIX_FUNCTIONS[fn]
    with mpmath.workdps(dps):
        lam, es = _eigenprojectors_mp(a9, dps)
        if fn != "exp" and min(lam) <= 0:
            raise ValueError(f"{fn} needs positive eigenvalues")
        fl = [f(x) for x in lam]
        return [float(sum(fl[k] * es[k][r][c] for k in range(3))) for r in range(3) for c in range(3)]


MATRIX_FUNCTION_DERIVATIVES = {"exp": mpmath.exp, "log": lambda x: 1 / x, "sqrt": lambda x: 1 / (2 * mpmath.sqrt(x))}


def matrix_function_vjp(a9: Sequence[float], fn: str, g9: Sequence[float], dps: int = 80) -> list[float]:
    """d<G, f(A)>/dA, row-major: with f(A) = sum_k f(lambda_k) E_k, the
    derivative of a function of a matrix with distinct eigenvalues is
    d f(A) = sum_{k,l} Gamma_kl E_k dA E_l (Daleckii-Krein), Gamma_kk =
    f'(lambda_k), Gamma_kl = (f(lambda_k) - f(lambda_l)) / (lambda_k - lambda_l),
    so the vector-Jacobian product is sum_{k,l} Gamma_kl E_k^T G E_l^T."""
    f, df = MATRIX_FUNCTIONS[fn], MATRIX_FUNCTION_DERIVATIVES[fn]
    with mpmath.workdps(dps):
        lam, es = _eigenprojectors_mp(a9, dps)
        if fn != "exp" and min(lam) <= 0:
            raise ValueError(f"{fn} needs positive eigenvalues")
        g = [[mpmath.mpf(float(g9[3 * i + j])) for j in range(3)] for i in range(3)]
        gam = [[df(lam[k]) if k == l else (f(lam[k]) - f(lam[l])) / (lam[k] - lam[l]) for l in range(3)]
               for k in range(3)]

        def mm(x, y):
            return [[sum(x[r][t] * y[t][c] for t in range(3)) for c in range(3)] for r in range(3)]

        def tr(x):
            return [[x[c][r] for c in range(3)] for r in range(3)]

        out = [[mpmath.mpf(0)] * 3 for _ in range(3)]
        for k in range(3):
            for l in range(3):
                t = mm(mm(tr(es[k]), g), tr(es[l]))
                out = [[out[r][c] + gam[k][l] * t[r][c] for c in range(3)] for r in range(3)]
        return [float(out[r][c]) for r in range(3) for c in range(3)]


# ----------------------------------------------------------------------------
# stability-bound scales (C = 1, Frobenius norms, lowest-order term)
# ----------------------------------------------------------------------------

def bound_scales(a9: Sequence[float]) -> dict[str, float]:
    """Norm factors of the forward-error bounds, each to be multiplied by the
    unit roundoff (and, for eigenvalues, by the eigenbasis condition number):

    I1:    ||A||                                   (I1 section, forward bound)
    J2:    ||dev A||^2                             (Thm thm:J2-fwd-stability)
    J3:    ||dev cof dev A|| ||dev A||             (Lemma lem:J3-fwd-stability)
    Delta: ||dev(12 J2^2 A^T - 54 J3 cof dev A)|| ||dev A||  (Lemma lem:disc-fwd-stability)
    lam:   ||A||                                   (Lemma lem:eigvals-fwd-stability)
    """
    a = to_fraction_matrix(a9)
    s = dev(a)
    j2 = trace(matmul(s, s)) / 2
    j3 = det3(s)
    cs = cof(s)
    jd = dev(add(scale(transpose(a), 12 * j2 * j2), cs, -54 * j3))
    with mpmath.workdps(40):
        na = mpmath.sqrt(_mpf(frob_sq(a)))
        ns = mpmath.sqrt(_mpf(frob_sq(s)))
        ncs = mpmath.sqrt(_mpf(frob_sq(dev(cs))))
        njd = mpmath.sqrt(_mpf(frob_sq(jd)))
        return {
            "I1": float(na),
            "J2": float(ns * ns),
            "J3": float(ncs * ns),
            "Delta": float(njd * ns),
            "lam": float(na),
        }


# ----------------------------------------------------------------------------
# application: Mohr-Coulomb yield function
# ----------------------------------------------------------------------------

def mohr_coulomb(a9: Sequence[float], s_yc: float, m: float, dps: int = 80):
    """f(sigma) = (1/S_yc) ((m+1)/2) max_{i<j} (|s_i - s_j| + K (s_i + s_j)) - 1,
    K = (m-1)/(m+1), with the exact principal stresses s_i (Sec. "Application:
    Evaluation of the Mohr-Coulomb yield function in mechanics", Eq.
    mohr-coulomb-yield), and df/dsigma (9 row-major floats, full-matrix
    gradient) through the maximizing pair: d|s_i - s_j| = sign(s_i - s_j)
    (ds_i - ds_j), ds_k = E_k^T : dsigma.  Returns (f, grad)."""
    lam = eigvals(a9, dps)
    if any(isinstance(x, mpmath.mpc) for x in lam):
        raise ValueError("complex spectrum")
    with mpmath.workdps(dps):
        mm = mpmath.mpf(m)
        K = (mm - 1) / (mm + 1)
        c = (mm + 1) / (2 * mpmath.mpf(s_yc))
        best, bi, bj = None, 0, 0
        for i in range(3):
            for j in range(i + 1, 3):
                v = abs(lam[i] - lam[j]) + K * (lam[i] + lam[j])
                if best is None or v > best:
                    best, bi, bj = v, i, j
        f = c * best - 1
        sgn = 1 if lam[bi] >= lam[bj] else -1
        g = [0.0, 0.0, 0.0]
        g[bi] = float(c * (sgn + K))
        g[bj] = float(c * (-sgn + K))
    return float(f), eigvals_vjp(a9, g, dps)


def to_float(q: Fraction) -> float:
    """Correctly rounded binary64 value of an exact rational."""
    return float(q)
