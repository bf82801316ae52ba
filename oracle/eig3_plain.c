/*
 * eig3_plain.c -- the paper's algorithms in plain binary64 C, one matrix at a
 * time.
 *
 * TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code,
 * header or constant with the HIP library.
 *
 * Habera & Zilian, "Numerically stable evaluation of closed-form expressions
 * for eigenvalues of 3x3 matrices" (arXiv 2511.00292):
 *   I1     -- Alg. alg:I1-stable     (Sec. "Invariant I1")
 *   J2     -- Alg. alg:J2-stable     (Sec. "Invariant J2")
 *   J3     -- Alg. alg:J3-stable     (Sec. "Invariant J3")
 *   Delta  -- Alg. alg:disc-stable   (Sec. "Discriminant"), sum of products
 *             of the auxiliary vectors u = dx(A), v = dx(A^T) with weights w
 *   lambda -- Alg. alg:eigvals-stable (Sec. "Eigenvalues") with the
 *             trigonometric formula Eq. eigvals-trig.
 *
 * Readings where the printed text is silent or inconsistent:
 *   - the factors of dx are derived from the Cauchy-Binet expansion (see
 *     oracle/gen_formulas.py), not typed in; the derived factor that
 *     contains M01 d1 d2 and M01 M02 M20 has + M02 M21 d2, where the printed
 *     r10 has - M02 M21 d2 (with the printed sign the sum of products is not
 *     4 J2^3 - 27 J3^2).
 *   - the triple angle is atan2(sqrt(27 Delta), 27 J3) in [0, pi], the branch
 *     that equals arccos((3 sqrt3 / 2) J3 / J2^(3/2)) of Eq. eigvals-trig's
 *     definition of phi; a plain arctan of the quotient is wrong for J3 < 0.
 *   - Delta < 0 and J2 < 0 (possible after rounding for nonsymmetric input)
 *     are clamped to 0 before the square roots.
 *   - the three values are sorted ascending at the end (ties may swap by an
 *     ulp otherwise).
 *   - the fractions 1/3, 1/6, 1/27 are divisions, sums run left to right
 *     (for the generated formulas in the order the generator states), and
 *     the file is built with -ffp-contract=off (no FMA).
 *
 * Backward (vector-Jacobian product) follows the eigenprojector relation
 * d(lambda_k)/dA = E_k^T of Sec. "Introduction and motivation", with the
 * Frobenius covariant E_k = (A - l_i I)(A - l_j I) / ((l_k - l_i)(l_k - l_j)),
 * a route that does not go through the invariants.
 *
 * Matrices are stored row-major, 9 doubles per matrix (A00 A01 A02 A10 ...).
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- Alg. 1 */
static double alg_I1(const double *A)
{
    return A[0] + A[4] + A[8];
}

/* ---------------------------------------------------------------- Alg. 2 */
static double alg_J2(const double *A)
{
    const double A00 = A[0], A01 = A[1], A02 = A[2];
    const double A10 = A[3], A11 = A[4], A12 = A[5];
    const double A20 = A[6], A21 = A[7], A22 = A[8];
    double d0 = A00 - A11, d1 = A00 - A22, d2 = A11 - A22;
    double offdiag = A01 * A10 + A02 * A20 + A12 * A21;
    double diag = (d0 * d0 + d1 * d1 + d2 * d2) / 6.0;
    return diag + offdiag;
}

/* ---------------------------------------------------------------- Alg. 5 */
static double alg_J3(const double *A)
{
    const double A00 = A[0], A01 = A[1], A02 = A[2];
    const double A10 = A[3], A11 = A[4], A12 = A[5];
    const double A20 = A[6], A21 = A[7], A22 = A[8];
    double d0 = A00 - A11, d1 = A00 - A22, d2 = A11 - A22;
    double t1 = d1 + d2;
    double t2 = d0 - d2;
    double t3 = -d0 - d1;
    double offdiag = A01 * A12 * A20 + A02 * A10 * A21;
    double mixed = (A01 * A10 * t1 + A02 * A20 * t2 + A12 * A21 * t3) / 3.0;
    double diag = t1 * t2 * t3 / 27.0;
    return offdiag + mixed - diag;
}

/* ---------------------------------------------------------------- Alg. 8 */
/* The factors r_i of the auxiliary vectors and their weights w_i are not
   typed in: oracle/gen_formulas.py derives them from the Cauchy-Binet
   expansion of Parlett's determinant (Sec. "Discriminant") and writes them
   to eig3_plain_formulas.h, together with the naive monomial sums below.
   Delta = sum_i w_i u_i v_i, u = dx(A), v = dx(A^T), with the same diagonal
   differences for both, summed left to right. */
#include "eig3_plain_formulas.h"

static double alg_disc(const double *A)
{
    double At[9] = {A[0], A[3], A[6], A[1], A[4], A[7], A[2], A[5], A[8]};
    double d0 = A[0] - A[4], d1 = A[0] - A[8], d2 = A[4] - A[8];
    double u[14], v[14];
    dx_factors(A, d0, d1, d2, u);
    dx_factors(At, d0, d1, d2, v);
    double disc = 0.0;
    for (int i = 0; i < 14; ++i)
        disc = disc + dx_weights[i] * u[i] * v[i];
    return disc;
}

/* ------------------------------------------------- comparators (naive) */
/* Alg. alg:J2-naive and alg:J3-naive: the monomial expansions of 3 J2 and
   27 J3 (generated, lexicographic order), summed left to right, then divided. */
static double alg_J2_naive(const double *A)
{
    return naive_3j2(A) / 3.0;
}

static double alg_J3_naive(const double *A)
{
    return naive_27j3(A) / 27.0;
}

/* Alg. alg:J2-tensor / alg:J3-tensor: S = A - tr(A)/3 I, then tr(S S)/2 and
   det S, the determinant by LU with partial pivoting (row operations with
   the reciprocal of the pivot, as the LAPACK factorisation used by NumPy's
   determinant does). */
static void tensor_dev(const double *A, double *S)
{
    double mean = (A[0] + A[4] + A[8]) / 3.0;
    for (int e = 0; e < 9; ++e)
        S[e] = A[e];
    S[0] -= mean;
    S[4] -= mean;
    S[8] -= mean;
}

static double alg_J2_tensor(const double *A)
{
    double S[9];
    tensor_dev(A, S);
    double tr = 0.0;
    for (int i = 0; i < 3; ++i) {
        double sii = 0.0;
        for (int k = 0; k < 3; ++k)
            sii = sii + S[3 * i + k] * S[3 * k + i];
        tr = tr + sii;
    }
    return tr / 2.0;
}

static double det_lu(double *M)
{
    double sign = 1.0;
    for (int c = 0; c < 2; ++c) {
        int p = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(M[3 * r + c]) > fabs(M[3 * p + c]))
                p = r;
        if (p != c) {
            for (int k = 0; k < 3; ++k) {
                double t = M[3 * c + k];
                M[3 * c + k] = M[3 * p + k];
                M[3 * p + k] = t;
            }
            sign = -sign;
        }
        if (M[3 * c + c] != 0.0) {
            double inv = 1.0 / M[3 * c + c];
            for (int r = c + 1; r < 3; ++r) {
                double l = M[3 * r + c] * inv;
                for (int k = c + 1; k < 3; ++k)
                    M[3 * r + k] = M[3 * r + k] - l * M[3 * c + k];
            }
        }
    }
    return sign * (M[0] * M[4] * M[8]);
}

static double alg_J3_tensor(const double *A)
{
    double S[9];
    tensor_dev(A, S);
    return det_lu(S);
}

/* ---------------------------------------------------------------- Alg. 9 */
static void alg_eigvals(double I1, double J2, double J3, double disc, double *lam)
{
    const double pi = 3.14159265358979323846;
    double phi = atan2(sqrt(27.0 * fmax(disc, 0.0)), 27.0 * J3);
    double r = 2.0 * sqrt(3.0 * fmax(J2, 0.0));
    for (int k = 1; k <= 3; ++k)
        lam[k - 1] = (I1 + r * cos((phi + 2.0 * pi * k) / 3.0)) / 3.0;
    /* ascending order */
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2 - i; ++j)
            if (lam[j] > lam[j + 1]) {
                double t = lam[j];
                lam[j] = lam[j + 1];
                lam[j + 1] = t;
            }
}

static void one_eigvals(const double *A, double *lam)
{
    alg_eigvals(alg_I1(A), alg_J2(A), alg_J3(A), alg_disc(A), lam);
}

/* naive comparators: variant 1 = Alg. alg:J2-naive / alg:J3-naive,
   variant 2 = Alg. alg:J2-tensor / alg:J3-tensor; Delta = 4 J2^3 - 27 J3^2 */
static void one_invariants_naive(const double *A, int variant, double *out)
{
    double j2 = variant == 1 ? alg_J2_naive(A) : alg_J2_tensor(A);
    double j3 = variant == 1 ? alg_J3_naive(A) : alg_J3_tensor(A);
    out[0] = alg_I1(A);
    out[1] = j2;
    out[2] = j3;
    out[3] = 4.0 * j2 * j2 * j2 - 27.0 * j3 * j3;
}

/* -------------------------------------------------- backward, E_k route */
static void one_backward(const double *A, const double *g, double *grad)
{
    double lam[3];
    one_eigvals(A, lam);
    for (int e = 0; e < 9; ++e)
        grad[e] = 0.0;
    for (int k = 0; k < 3; ++k) {
        int i = (k + 1) % 3, j = (k + 2) % 3;
        double P[9], Q[9], E[9];
        for (int e = 0; e < 9; ++e) {
            P[e] = A[e];
            Q[e] = A[e];
        }
        P[0] -= lam[i]; P[4] -= lam[i]; P[8] -= lam[i];
        Q[0] -= lam[j]; Q[4] -= lam[j]; Q[8] -= lam[j];
        double den = (lam[k] - lam[i]) * (lam[k] - lam[j]);
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                E[3 * r + c] = (P[3 * r + 0] * Q[0 + c] + P[3 * r + 1] * Q[3 + c] + P[3 * r + 2] * Q[6 + c]) / den;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                grad[3 * r + c] += g[k] * E[3 * c + r]; /* E_k^T */
    }
}

/* ------------------------------------------------------------ exports */
#define EXPORT __attribute__((visibility("default")))

static void set_threads(int threads)
{
#ifdef _OPENMP
    if (threads > 0)
        omp_set_num_threads(threads);
#else
    (void)threads;
#endif
}

EXPORT int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* I1, J2, J3, Delta of n row-major matrices a[n*9]; each output has n doubles */
EXPORT void oracle_invariants(int64_t n, const double *a, double *i1, double *j2, double *j3,
                              double *disc, int threads)
{
    set_threads(threads);
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < n; ++m) {
        const double *A = a + 9 * m;
        i1[m] = alg_I1(A);
        j2[m] = alg_J2(A);
        j3[m] = alg_J3(A);
        disc[m] = alg_disc(A);
    }
}

/* the auxiliary vectors u = dx(A), v = dx(A^T) of one matrix (14 each) */
EXPORT void oracle_aux_vectors(const double *A, double *u, double *v)
{
    double At[9] = {A[0], A[3], A[6], A[1], A[4], A[7], A[2], A[5], A[8]};
    double d0 = A[0] - A[4], d1 = A[0] - A[8], d2 = A[4] - A[8];
    dx_factors(A, d0, d1, d2, u);
    dx_factors(At, d0, d1, d2, v);
}

/* naive comparators (variant 1: monomial sums, 2: tensor) -- invariants
   out[n*4] = (I1, J2, J3, Delta) and eigenvalues lam[n*3] */
EXPORT void oracle_naive(int64_t n, const double *a, int variant, double *inv, double *lam)
{
    for (int64_t m = 0; m < n; ++m) {
        double *o = inv + 4 * m;
        one_invariants_naive(a + 9 * m, variant, o);
        alg_eigvals(o[0], o[1], o[2], o[3], lam + 3 * m);
    }
}

/* eigenvalues, ascending: lam[n*3] */
EXPORT void oracle_eigvals(int64_t n, const double *a, double *lam, int threads)
{
    set_threads(threads);
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < n; ++m)
        one_eigvals(a + 9 * m, lam + 3 * m);
}

/* eigenvalues from given invariants (Alg. 9 alone): lam[n*3] */
EXPORT void oracle_eigvals_from_invariants(int64_t n, const double *i1, const double *j2,
                                           const double *j3, const double *disc, double *lam)
{
    for (int64_t m = 0; m < n; ++m)
        alg_eigvals(i1[m], j2[m], j3[m], disc[m], lam + 3 * m);
}

/* vector-Jacobian product: grad[n*9] = sum_k g[n*3]_k d(lambda_k)/dA */
EXPORT void oracle_eigvals_backward(int64_t n, const double *a, const double *g, double *grad,
                                    int threads)
{
    set_threads(threads);
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < n; ++m)
        one_backward(a + 9 * m, g + 3 * m, grad + 9 * m);
}
