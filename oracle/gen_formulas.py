"""Derive the polynomial formulas that the plain oracle evaluates, and write
them as C (``eig3_plain_formulas.h``).

TEST INFRASTRUCTURE (see ``oracle/__init__.py``).  Nothing here is taken
from a printed listing: every formula is obtained from its definition by
exact polynomial algebra over the nine entries of a 3x3 matrix, and checked
against an independent definition before it is written.

1. The auxiliary factors of the discriminant (Sec. "Discriminant",
   Eq. disc-determinant and Eq. sop-disc).  Parlett's matrix
   B_ij = <A^(i-1), (A^(j-1))^T> factors as B = X Y with X the 3x9 matrix
   whose rows are vec(I), vec(A), vec(A^2) and Y the 9x3 matrix whose columns
   are vec(I), vec(A^T), vec((A^2)^T).  By the Cauchy-Binet formula
   det B = sum over 3-subsets S of the nine entry positions of
   det X[:, S] * det Y[S, :], and det Y[S, :] is det X[:, S] evaluated at
   A^T.  A subset without a diagonal position has a zero first row and drops
   out; the remaining 64 minors fall into classes with the same product
   u_S(A) u_S(A^T).  One representative r of each class, with its class
   size w as weight, gives Delta = sum w r(A) r(A^T).  A minor is unchanged
   by A -> A - cI (row operations), so its diagonal entries enter only
   through their differences d0 = A00 - A11, d1 = A00 - A22,
   d2 = A11 - A22: each coefficient of an off-diagonal monomial is written
   as an integer times a product of these differences (the unique
   factorisation of that coefficient polynomial), which is the form of
   Alg. alg:disc-stable.  Checked: sum w r(A) r(A^T) = 4 J2^3 - 27 J3^2 as
   polynomials, with J2 = tr(dev(A)^2)/2 and J3 = det dev(A).

2. The naive invariants (Alg. alg:J2-naive and alg:J3-naive): 3 J2 and
   27 J3 expanded from those definitions into integer monomials of the nine
   entries, in lexicographic order of the entry indices.

Evaluation order of the generated C (what the plain oracle's rounding
follows): every term is one product, the integer coefficient first (when it
is not 1), then the off-diagonal entries in index order, then the
differences; the terms of a factor are summed left to right, those with the
most differences first, and within the same number of differences in
lexicographic order of their off-diagonal entries.  The naive sums are
evaluated left to right and divided by 3 and 27 at the end.

Run ``python -m oracle.gen_formulas`` to rewrite the header; the CPU test
``tests/test_oracle_formulas.py`` checks that the committed header is this
script's output.
"""
from __future__ import annotations

import itertools
import os
import sys
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(HERE, "eig3_plain_formulas.h")

# variables: the nine entries A00..A22 (row-major index 0..8)
NV = 9
NAMES = ["A00", "A01", "A02", "A10", "A11", "A12", "A20", "A21", "A22"]
DIAG = (0, 4, 8)
OFF = (1, 2, 3, 5, 6, 7)
TRANSPOSE = (0, 3, 6, 1, 4, 7, 2, 5, 8)  # entry k of A^T is entry TRANSPOSE[k] of A


# --------------------------------------------------------------- polynomials
# a polynomial is a dict {exponent tuple (NV ints): Fraction}, no zero values

def const(c) -> dict:
    return {(0,) * NV: Fraction(c)} if c else {}


def var(k: int) -> dict:
    e = [0] * NV
    e[k] = 1
    return {tuple(e): Fraction(1)}


def add(*ps) -> dict:
    out: dict = {}
    for p in ps:
        for m, c in p.items():
            v = out.get(m, 0) + c
            if v:
                out[m] = v
            else:
                out.pop(m, None)
    return out


def scale(p: dict, c) -> dict:
    c = Fraction(c)
    return {m: v * c for m, v in p.items()} if c else {}


def mul(p: dict, q: dict) -> dict:
    out: dict = {}
    for m1, c1 in p.items():
        for m2, c2 in q.items():
            m = tuple(a + b for a, b in zip(m1, m2))
            v = out.get(m, 0) + c1 * c2
            if v:
                out[m] = v
            else:
                out.pop(m, None)
    return out


def subs(p: dict, perm) -> dict:
    """p with variable k replaced by variable perm[k]."""
    out: dict = {}
    for m, c in p.items():
        e = [0] * NV
        for k, x in enumerate(m):
            e[perm[k]] += x
        out[tuple(e)] = out.get(tuple(e), 0) + c
    return {m: c for m, c in out.items() if c}


# ------------------------------------------------------------ 3x3 matrices

def sym_matrix():
    return [[var(3 * i + j) for j in range(3)] for i in range(3)]


def matmul(x, y):
    return [[add(*(mul(x[i][k], y[k][j]) for k in range(3))) for j in range(3)] for i in range(3)]


def det3(m) -> dict:
    return add(mul(m[0][0], add(mul(m[1][1], m[2][2]), scale(mul(m[1][2], m[2][1]), -1))),
               scale(mul(m[0][1], add(mul(m[1][0], m[2][2]), scale(mul(m[1][2], m[2][0]), -1))), -1),
               mul(m[0][2], add(mul(m[1][0], m[2][1]), scale(mul(m[1][1], m[2][0]), -1))))


def deviator(a):
    tr3 = scale(add(a[0][0], a[1][1], a[2][2]), Fraction(1, 3))
    return [[add(a[i][j], scale(tr3, -1)) if i == j else a[i][j] for j in range(3)] for i in range(3)]


def invariants_j2_j3():
    """J2 = tr(S^2)/2 and J3 = det S, S = dev A (Eq. principal-invariants)."""
    s = deviator(sym_matrix())
    s2 = matmul(s, s)
    return scale(add(s2[0][0], s2[1][1], s2[2][2]), Fraction(1, 2)), det3(s)


# ------------------------------------------------- 1. discriminant factors

def minors():
    """The 3x3 minors det X[:, S] of X = [vec I; vec A; vec A^2] for every
    3-subset S of the nine positions with a diagonal position."""
    a = sym_matrix()
    a2 = matmul(a, a)
    rows = [[const(1) if k in DIAG else {} for k in range(NV)],
            [a[k // 3][k % 3] for k in range(NV)],
            [a2[k // 3][k % 3] for k in range(NV)]]
    out = []
    for s in itertools.combinations(range(NV), 3):
        if not any(k in DIAG for k in s):
            continue
        m = [[rows[r][k] for k in s] for r in range(3)]
        out.append((s, det3(m)))
    return out


def _d_polys():
    """d0 = A00 - A11, d1 = A00 - A22, d2 = A11 - A22 as polynomials."""
    return [add(var(0), scale(var(4), -1)), add(var(0), scale(var(8), -1)), add(var(4), scale(var(8), -1))]


def _d_products(degree: int):
    """(exponents of d0, d1, d2, polynomial) for every product of the given degree."""
    d = _d_polys()
    out = []
    for e in itertools.product(range(degree + 1), repeat=3):
        if sum(e) != degree:
            continue
        p = const(1)
        for k in range(3):
            for _ in range(e[k]):
                p = mul(p, d[k])
        out.append((e, p))
    return out


def in_differences(p: dict):
    """Write p (invariant under a shift of the diagonal) as a list of terms
    (integer coefficient, off-diagonal exponents, (e0, e1, e2) exponents of
    d0, d1, d2), each coefficient polynomial of an off-diagonal monomial
    being an integer times one product of differences."""
    groups: dict = {}
    for m, c in p.items():
        off = tuple(m[k] for k in OFF)
        dm = tuple(m[k] if k in DIAG else 0 for k in range(NV))
        groups.setdefault(off, {})[dm] = c
    terms = []
    for off, coef in groups.items():
        degree = sum(next(iter(coef)))
        for e, dp in _d_products(degree):
            # coef = k * dp for an integer k?
            m0 = next(iter(dp))
            k = coef.get(m0, 0) / dp[m0]
            if k and k.denominator == 1 and add(coef, scale(dp, -k)) == {}:
                terms.append((int(k), off, e))
                break
        else:
            raise ValueError(f"coefficient of {off} is not an integer times a product of differences")
    return terms


def term_key(t):
    k, off, e = t
    # most differences first; then lexicographic in the off-diagonal entries
    idx = [OFF[j] for j in range(6) for _ in range(off[j])]
    return (-sum(e), idx, e)


def factor_classes():
    """Classes of minors with the same product u_S(A) u_S(A^T): list of
    (weight, representative factor r as a polynomial in the entries)."""
    classes: dict = {}
    for s, u in minors():
        if not u:
            continue
        prod = mul(u, subs(u, TRANSPOSE))
        key = tuple(sorted(prod.items()))
        if key in classes:
            classes[key][0] += 1
        else:
            classes[key] = [1, u]
    out = []
    for w, u in classes.values():
        terms = sorted(in_differences(u), key=term_key)
        if terms[0][0] < 0:  # sign normalisation: the first term positive
            u = scale(u, -1)
            terms = [(-k, off, e) for k, off, e in terms]
        out.append((w, u, terms))
    # order: by the largest number of differences in a term, then by weight,
    # then lexicographically by the terms
    out.sort(key=lambda c: (max(sum(t[2]) for t in c[2]), c[0], [term_key(t) for t in c[2]]))
    return out


def check_factors(classes) -> None:
    """sum w r(A) r(A^T) = 4 J2^3 - 27 J3^2 exactly, as polynomials."""
    j2, j3 = invariants_j2_j3()
    disc = add(scale(mul(mul(j2, j2), j2), 4), scale(mul(j3, j3), -27))
    sop = add(*(scale(mul(u, subs(u, TRANSPOSE)), w) for w, u, _ in classes))
    if add(sop, scale(disc, -1)) != {}:
        raise AssertionError("sum of products differs from 4 J2^3 - 27 J3^2")
    if sum(w for w, _, _ in classes) != 64 or len(classes) != 14:
        raise AssertionError("unexpected class structure")


# ----------------------------------------------------- 2. naive invariants

def naive_polys():
    """3 J2 and 27 J3 as integer polynomials in the nine entries."""
    j2, j3 = invariants_j2_j3()
    return scale(j2, 3), scale(j3, 27)


def mono_key(m):
    return [k for k in range(NV) for _ in range(m[k])]


# ------------------------------------------------------------------ C output

OFF_NAMES = ["M01", "M02", "M10", "M12", "M20", "M21"]  # OFF order, of the argument matrix M


def c_term(k: int, off, e, first: bool) -> str:
    factors = [OFF_NAMES[j] for j in range(6) for _ in range(off[j])]
    factors += [f"d{j}" for j in range(3) for _ in range(e[j])]
    mag = abs(k)
    body = " * ".join(([str(mag)] if mag != 1 else []) + factors)
    if first:
        return ("-" if k < 0 else "") + body
    return (" - " if k < 0 else " + ") + body


def c_poly_sum(p: dict) -> str:
    terms = sorted(p.items(), key=lambda t: mono_key(t[0]))
    out = []
    for i, (m, c) in enumerate(terms):
        assert c.denominator == 1
        k = int(c)
        factors = [NAMES[j] for j in mono_key(m)]
        body = " * ".join(([str(abs(k))] if abs(k) != 1 else []) + factors)
        out.append((("-" if k < 0 else "") if i == 0 else (" - " if k < 0 else " + ")) + body)
    return "".join(out)


def header_text() -> str:
    classes = factor_classes()
    check_factors(classes)
    j2n, j3n = naive_polys()
    lines = [
        "/* eig3_plain_formulas.h -- GENERATED by oracle/gen_formulas.py; do not edit.",
        " *",
        " * TEST INFRASTRUCTURE (see oracle/__init__.py).  Formulas derived from",
        " * their definitions by exact polynomial algebra (see the generator):",
        " *   dx_factors: the 14 factor classes of the Cauchy-Binet expansion of",
        " *     Parlett's det B (Sec. \"Discriminant\", Eq. disc-determinant,",
        " *     Eq. sop-disc), written in the diagonal differences d0, d1, d2 as",
        " *     Alg. alg:disc-stable does; dx_weights: the class sizes.",
        " *     sum_i w_i r_i(A) r_i(A^T) = 4 J2^3 - 27 J3^2 was checked as",
        " *     polynomials before this file was written.",
        " *   naive_3j2, naive_27j3: 3 J2 and 27 J3 expanded into monomials",
        " *     (Alg. alg:J2-naive and alg:J3-naive).",
        " */",
        "",
        "static const double dx_weights[14] = {" + ", ".join(str(w) for w, _, _ in classes) + "};",
        "",
        "/* the 14 factors r[0..13] of M (row-major) with the given diagonal differences */",
        "static void dx_factors(const double *M, double d0, double d1, double d2, double *r)",
        "{",
        "    const double M01 = M[1], M02 = M[2];",
        "    const double M10 = M[3], M12 = M[5];",
        "    const double M20 = M[6], M21 = M[7];",
        "    (void)d0; (void)d1; (void)d2;",
    ]
    for i, (_, _, terms) in enumerate(classes):
        expr = "".join(c_term(k, off, e, j == 0) for j, (k, off, e) in enumerate(terms))
        lines.append(f"    r[{i}] = {expr};")
    lines += ["}", ""]
    for name, p in (("naive_3j2", j2n), ("naive_27j3", j3n)):
        lines += [f"static double {name}(const double *A)", "{",
                  "    const double A00 = A[0], A01 = A[1], A02 = A[2];",
                  "    const double A10 = A[3], A11 = A[4], A12 = A[5];",
                  "    const double A20 = A[6], A21 = A[7], A22 = A[8];",
                  "    (void)A00; (void)A01; (void)A02; (void)A10; (void)A11; (void)A12; (void)A20; (void)A21;"
                  " (void)A22;",
                  f"    return {c_poly_sum(p)};", "}", ""]
    return "\n".join(lines)


def main() -> int:
    text = header_text()
    with open(HEADER, "w") as f:
        f.write(text)
    print(f"wrote {HEADER}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
