/*
 * eig3.h -- C ABI of libeig3: batched closed-form eigenvalues of real,
 * diagonalizable 3x3 matrices on AMD Instinct MI355X (gfx950).
 *
 * Method: Habera & Zilian, "Numerically stable evaluation of closed-form
 * expressions for eigenvalues of 3x3 matrices" (arXiv 2511.00292).  The
 * eigenvalues of a real, diagonalizable 3x3 matrix A with real spectrum are
 * obtained from four invariants (Sec. "Introduction and motivation",
 * Eq. principal-invariants and Eq. triple-angle-arctan):
 *   I1 = tr A                       (Alg. alg:I1-stable)
 *   J2 = tr(dev(A)^2) / 2           (Alg. alg:J2-stable, diagonal differences)
 *   J3 = det(dev A)                 (Alg. alg:J3-stable)
 *   Delta = 4 J2^3 - 27 J3^2        (Alg. alg:disc-stable, sum of products)
 * and the trigonometric formula (Eq. eigvals-trig, Alg. alg:eigvals-stable)
 *   lambda_k = (I1 + 2 sqrt(3 J2) cos((phi + 2 pi k) / 3)) / 3,
 *   phi = atan2(sqrt(27 Delta), 27 J3) in [0, pi].
 *
 * Conventions shared by every call:
 *  - All data pointers are DEVICE pointers owned by the caller, on the
 *    calling thread's current HIP device, which is where the kernels run
 *    (`stream` must belong to that device).  The library never allocates,
 *    frees or synchronizes and keeps no state between calls, so it may be
 *    called from several threads at once; each call only enqueues kernels on
 *    `stream` (a hipStream_t; NULL = the default stream) and returns.
 *  - Inputs are read-only.  Outputs must not alias inputs or each other.
 *  - n == 0 is a no-op returning EIG3_OK.  Invalid arguments (NULL pointers,
 *    pointers not aligned to the element size, n < 0 or n > 2^56, unknown
 *    enum values, outputs aliasing inputs or each other) return EIG3_EINVAL
 *    and launch nothing.  A failed launch returns EIG3_ELAUNCH.
 *  - Precondition (not checked): real, diagonalizable input with real
 *    spectrum.  Outside it the results stay finite for finite input: J2 < 0
 *    and Delta < 0 (possible after rounding for nonsymmetric input) are
 *    clamped to 0 before the square roots, so a complex pair a +- ib comes
 *    back as a double real value near a.  NaN input propagates to NaN output.
 *  - Range: binary64 batches are evaluated on A scaled by the power of two
 *    that brings its largest entry into [1/2, 1) (exact; the results scale
 *    back exactly), so eigenvalues, their adjoint, the eigenprojectors and
 *    the Mohr-Coulomb function hold over the whole binary64 range;
 *    eig3_invariants returns the invariants themselves, which overflow
 *    (Delta ~ |A|^6) beyond about 2^170 and underflow below about 2^-170;
 *    the functions of matrices take their eigenvalues from the scaled
 *    invariants and work with A's own entries otherwise, so they hold while
 *    products of two entries and f's own values stay in range (log and
 *    sqrt: about 2^+-450; their adjoints, whose divided differences reach
 *    the fifth order, about 2^+-200).  The naive comparators are evaluated
 *    as printed, without scaling.
 *  - Eigenvalues are returned in ascending order lambda_1 <= lambda_2 <=
 *    lambda_3 (Sec. "Introduction and motivation", ordering property).
 *  - Accuracy: with unit roundoff eps (2^-53 binary64, 2^-24 binary32),
 *    kappa_2 the condition number of the eigenbasis, and Frobenius norms,
 *    the paper's forward-error bounds (C = 1, lowest order) are
 *      |I1 err| <= ||A|| eps, |J2 err| <= ||dev A||^2 eps  (Thm thm:J2-fwd-stability)
 *      |J3 err| <= ||dev cof dev A|| ||dev A|| eps          (Lemma lem:J3-fwd-stability)
 *      |Delta err| <= ||dev(12 J2^2 A^T - 54 J3 cof dev A)|| ||dev A|| eps
 *                                                            (Lemma lem:disc-fwd-stability)
 *      |lambda err| <= kappa_2 ||A|| eps                     (Lemma lem:eigvals-fwd-stability)
 *    EIG3_DOUBLE_WORD and EIG3_COMPENSATED stay within a small multiple of
 *    these bounds also for ill-conditioned eigenbases (measured on the
 *    synthetic workloads up to kappa_2 = 100, and on the paper's own paths
 *    with kappa_2 ~ 9e3: worst 3.8x for every invariant and eigenvalue),
 *    where the plain algorithms (EIG3_FMA, and the paper's algorithms in
 *    plain binary64) exceed them by up to three orders of magnitude.
 */
#ifndef EIG3_H
#define EIG3_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum eig3_status {
    EIG3_OK = 0,
    EIG3_EINVAL = -1,       /* invalid argument; nothing was launched */
    EIG3_EUNSUPPORTED = -2, /* valid combination that the library does not provide */
    EIG3_ELAUNCH = -3       /* the HIP runtime reported a launch error */
} eig3_status;

typedef enum eig3_dtype {
    EIG3_F64 = 0, /* binary64 storage and arithmetic */
    EIG3_F32 = 1  /* binary32 storage and results.  Delta is always formed and
                     kept in binary64 (it underflows binary32 near isotropic
                     states) and the triple-angle argument is formed in
                     binary64; arctangent, sine, cosine and the final
                     eigenvalues are binary32.  The invariants are computed
                     per eig3_accuracy, see there. */
} eig3_dtype;

typedef enum eig3_structure {
    EIG3_GENERAL = 0,  /* 9 entries: A00 A01 A02 A10 A11 A12 A20 A21 A22 */
    EIG3_SYMMETRIC = 1 /* 6 entries: A00 A11 A22 A01 A02 A12 (A10 = A01, ...) */
} eig3_structure;

typedef enum eig3_layout {
    EIG3_SOA = 0, /* structure of arrays: one array of n values per entry */
    EIG3_AOS = 1  /* array of structures: one array, matrix m at m*9 (or m*6),
                     entries in the order above (row-major (n,3,3) for GENERAL) */
} eig3_layout;

typedef enum eig3_accuracy {
    /* binary64: the paper's algorithms with fused multiply-adds.
       binary32: entries widened exactly to binary64 and the binary64 FMA
       invariants (the paper's algorithms on the widened entries). */
    EIG3_FMA = 0,
    /* binary64: error-free products (FMA TwoProduct) and sums (TwoSum) in J2,
       J3, every r_i of dx and sum w u v: the accuracy of twice the working
       precision before the final rounding of each invariant.  The diagonal
       differences are d0 = A00 - A11 and d2 = A11 - A22 rounded and
       d1 = d0 + d2 carried exactly, so that they are the differences of one
       (perturbed) diagonal.
       binary32: K2 = 6 J2 and K3 = 27 J3 by Alg. alg:J2-stable and
       alg:J3-stable with binary32 error-free products and sums (the
       evaluation of EIG3_DOUBLE_WORD in binary32 pairs, on the deviatoric
       data, scaled by a power of two where their largest magnitude lies
       outside [2^-10, 2^36)), binary64 only for the Delta
       accumulation (K2^3 - 2 K3^2)/54 from the widened pairs and for the
       triple-angle argument. */
    EIG3_COMPENSATED = 1,
    /* Comparators (binary64 eig3_invariants / eig3_eigvals only; other calls
       return EIG3_EUNSUPPORTED): the paper's naive evaluations in plain
       binary64, Delta = 4 J2^3 - 27 J3^2 from them.
       NAIVE: monomial sums, Alg. alg:J2-naive and alg:J3-naive.
       NAIVE_TENSOR: S = A - tr(A)/3 I, J2 = tr(S S)/2, J3 = det S by LU with
       partial pivoting, Alg. alg:J2-tensor and alg:J3-tensor. */
    EIG3_NAIVE = 2,
    EIG3_NAIVE_TENSOR = 3,
    /* binary64: J2 and J3 by Alg. alg:J2-stable and alg:J3-stable (as
       K2 = 6 J2 and K3 = 27 J3) in double-word arithmetic: error-free
       products and sums from the consistent diagonal differences described
       under EIG3_COMPENSATED, each kept unrounded as hi + lo (exact to
       O(eps^2) times the size of its terms); Delta from its definition
       4 J2^3 - 27 J3^2 = (K2^3 - 2 K3^2) / 54 (beside Eq.
       triple-angle-arctan) in double-word arithmetic from those unrounded
       values, so the cancellation between its two terms costs only
       O(eps^2 |dev A|^6).  Delta is the definition, not the sum of products
       of Alg. alg:disc-stable.  About the cost of EIG3_FMA, with the
       accuracy of EIG3_COMPENSATED.
       binary32: the double word of the binary32 data held in one binary64
       number: entries widened exactly, each product of two of them exact
       in binary64 (their error-free product), K2, K3 and Delta formed in
       binary64 (rounding at 2^-53, below a binary32 pair's 2^-48); the
       cheapest accurate binary32 evaluation on gfx950, where a binary64
       FMA issues at the rate of a non-packed binary32 one. */
    EIG3_DOUBLE_WORD = 4
} eig3_accuracy;

/* A batch of n matrices resident in device memory. */
typedef struct eig3_matrices {
    int64_t n;         /* number of matrices, 0 <= n <= 2^56 */
    int32_t dtype;     /* eig3_dtype */
    int32_t structure; /* eig3_structure */
    int32_t layout;    /* eig3_layout */
    int32_t accuracy;  /* eig3_accuracy */
    /* SOA: a[k] points to n values of entry k (k < 9 GENERAL, k < 6 SYMMETRIC).
       AOS: a[0] points to n*9 (GENERAL) or n*6 (SYMMETRIC) values; a[1..] unused.
       Every pointer must be aligned to its element size. */
    const void *a[9];
} eig3_matrices;

/*
 * The four invariants of each matrix (Alg. alg:I1-stable, alg:J2-stable,
 * alg:J3-stable, alg:disc-stable).  i1, j2, j3, disc: n values each, in the
 * element type of A.  Delta is not clamped here.
 */
int eig3_invariants(const eig3_matrices *A, void *i1, void *j2, void *j3, void *disc,
                    hipStream_t stream);

/*
 * Ascending eigenvalues of each matrix (Alg. alg:eigvals-stable applied to
 * the invariants, with phi read as atan2 in [0, pi]).
 * out_layout EIG3_SOA: lam[k] -> n values of lambda_(k+1), k = 0, 1, 2.
 * out_layout EIG3_AOS: lam[0] -> n*3 values, (lambda_1, lambda_2, lambda_3)
 *                      per matrix; lam[1], lam[2] unused.
 * Element type = that of A.
 */
int eig3_eigvals(const eig3_matrices *A, int32_t out_layout, void *const lam[3],
                 hipStream_t stream);

/*
 * Vector-Jacobian product of the eigenvalues: grad_a = sum_k g_k d(lambda_k)/dA,
 * through the invariants: d(lambda_k)/dA = I/3 + (mu_k dev(A)^T + dev(cof dev A))
 * / ((lambda_k - lambda_i)(lambda_k - lambda_j)), mu_k = lambda_k - I1/3, from
 * the Jacobians of Lemma lem:J2-condition and Lemma lem:J3-jacobian and the
 * implicit derivative of the depressed cubic mu^3 - J2 mu - J3 = 0.
 * g: upstream gradient, 3 values per matrix, layout g_layout as for
 *    eig3_eigvals' output.
 * grad_a: same structure, layout and entry order as A.  For SYMMETRIC input
 *    the result is the gradient with respect to the 6 stored entries (the
 *    off-diagonal value counts both of its positions).
 * Undefined at repeated eigenvalues (zero gap): the result is then +-Inf or
 * NaN.  Computed in binary64 for both storage types: binary32 entries and g
 * are widened exactly and each gradient entry is rounded once to binary32.
 */
int eig3_eigvals_backward(const eig3_matrices *A, int32_t g_layout, const void *const g[3],
                          void *const grad_a[9], hipStream_t stream);

/*
 * Mohr-Coulomb yield function of stress tensors (Sec. "Application:
 * Evaluation of the Mohr-Coulomb yield function in mechanics"):
 *   f(sigma) = (1/S_yc) ((m + 1)/2) max_{i<j} (|s_i - s_j| + K (s_i + s_j)) - 1,
 *   K = (m - 1)/(m + 1), m = S_yc / S_yt, s_i the principal stresses
 * (eigenvalues of sigma from the same path as eig3_eigvals, per
 * sigma->accuracy, including the comparator modes).
 * f: n values, element type of sigma.
 * dfds: NULL, or df/dsigma in the structure, layout and entry order of sigma.
 *   GENERAL: the 9 entries of the full-matrix gradient.  SYMMETRIC: the 6
 *   components of the (symmetric) tensor derivative; the derivative with
 *   respect to a stored off-diagonal entry is twice its component.
 *   +-Inf/NaN at the corners of the yield surface (s_1 = s_2 or s_2 = s_3).
 * 0 < s_yc <= 1e300 and 0 < m <= 1e300, else EIG3_EINVAL.  Arithmetic in
 * binary64.
 */
int eig3_mohr_coulomb(const eig3_matrices *sigma, double s_yc, double m, void *f, void *const dfds[9],
                      hipStream_t stream);

/*
 * Eigenprojectors E_k = prod_{j != k} (A - lambda_j I) / (lambda_k - lambda_j),
 * k = 1, 2, 3 for the ascending eigenvalues: the projectors behind the
 * relation E_k^T = d(lambda_k)/dA that the paper uses for closed-form
 * functions of matrices (Sec. "Introduction and motivation"), evaluated
 * through the invariants as E_k = I/3 + (mu_k S + dev(cof S)^T) / G_k,
 * S = dev A, G_k = (lambda_k - lambda_i)(lambda_k - lambda_j).
 * GENERAL: 9 row-major entries per projector; SYMMETRIC: the 6 components
 * (A00 A11 A22 A01 A02 A12 order) of each symmetric projector.
 * out_layout EIG3_SOA: E[K*k + e] -> n values of entry e of E_(k+1)
 *   (K = 9 or 6; 27 or 18 pointers).  EIG3_AOS: E[0] -> n*3*K values,
 *   per matrix E_1, E_2, E_3 one after the other.
 * Undefined at repeated eigenvalues (+-Inf/NaN).  Arithmetic in binary64,
 * results in the element type of A.
 */
int eig3_eigenprojectors(const eig3_matrices *A, int32_t out_layout, void *const E[27], hipStream_t stream);

typedef enum eig3_function {
    EIG3_EXP = 0,  /* matrix exponential */
    EIG3_LOG = 1,  /* principal logarithm: needs positive eigenvalues */
    EIG3_SQRT = 2  /* principal square root: needs positive eigenvalues (a zero
                      eigenvalue computed a rounding error below zero, or a
                      repeated one, gives NaN) */
} eig3_function;

/*
 * A function of each matrix, f(A) = sum_k f(lambda_k) E_k with the closed-form
 * eigenvalues and eigenprojectors above (the use of closed-form
 * eigenprojectors that Sec. "Introduction and motivation" names, e.g. the
 * matrix exponential).  The sum is the polynomial that interpolates f at the
 * three eigenvalues, evaluated at A; it is formed in Newton form,
 *   f(A) = f(lambda1) I + f[lambda1, lambda2] P1 + f[lambda1, lambda2, lambda3] P1 P2,
 *   P_k = A - lambda_k I,
 * with the first divided differences taken from the eigenvalue gaps without
 * cancellation, so the result stays accurate as eigenvalues coalesce and
 * exactly repeated eigenvalues are covered (f(p I) = f(p) I), where the
 * eigenprojectors themselves are not.
 * out: the structure and layout of A (GENERAL: 9 entries; SYMMETRIC: the 6
 * components of the symmetric result), element type of A; arithmetic in
 * binary64.  fn: an eig3_function.  Eigenvalues outside the domain of f
 * (log, sqrt) give NaN.  Where computed eigenvalues coincide exactly the
 * divided differences take their confluent limits (f', f''/2), so the result
 * is the Hermite interpolant, f(A) also for a defective A (e.g. p I + N, N
 * strictly triangular); a defective A whose repeated eigenvalue comes out
 * split gets it only to the accuracy of the computed eigenvalues.
 * accuracy: FMA or COMPENSATED (the comparators return EIG3_EUNSUPPORTED).
 */
int eig3_matrix_function(const eig3_matrices *A, int32_t fn, void *const out[9], hipStream_t stream);

/*
 * Vector-Jacobian product of eig3_matrix_function: grad_a = d<G, f(A)>/dA.
 * The derivative of a function of a matrix follows from the same closed
 * forms (Sec. "Introduction and motivation": closed forms for functions of
 * matrices and their derivatives); for distinct eigenvalues it is the
 * Daleckii-Krein sum
 *   d f(A) = sum_{k,l} Gamma_kl E_k dA E_l,  grad_a = sum_{k,l} Gamma_kl E_k^T G E_l^T,
 * Gamma_kk = f'(lambda_k), Gamma_kl = (f(lambda_k) - f(lambda_l)) / (lambda_k - lambda_l).
 * It is evaluated as the equal bivariate interpolant in tensor Newton form,
 *   grad_a = sum_{p,q <= 2} f[z0..zp, z0..zq] N_p G N_q,
 *   N_0 = I, N_1 = A^T - z0 I, N_2 = (A^T - z0 I)(A^T - z1 I),
 * with the nodes z0 = lambda_min, z1 = lambda_max, z2 = lambda_mid and the
 * divided differences (up to fifth order, each eigenvalue at most twice)
 * from cancellation-free first differences (exp: e^y expm1(d)/d, log:
 * log1p(d/y)/d, sqrt: 1/(sqrt x + sqrt y)) by a recursion that divides by the
 * spread wherever it can; gaps below 2^-26 of the spread take the confluent
 * values f^(k)/k!.  So the result stays accurate as eigenvalues coalesce,
 * with repeated eigenvalues (grad_a = f'(p) G at A = p I) and defective A
 * included.
 * g: the upstream gradient in the structure and layout of the forward's
 * output (GENERAL: 9 entries; SYMMETRIC: dL/d of the 6 stored components).
 * grad_a: the structure and layout of A (SYMMETRIC: the derivative with
 * respect to each stored entry).  Arithmetic in binary64.  Outside the domain
 * of f the result is NaN.
 */
int eig3_matrix_function_backward(const eig3_matrices *A, int32_t fn, const void *const g[9], void *const grad_a[9],
                                  hipStream_t stream);

/* Placement of a structure-of-arrays batch: the recommended distance, in
 * elements of the given dtype, between consecutive arrays of a batch of n
 * matrices stored in one allocation (array k at element k * stride): n
 * elements rounded up to a multiple of 64 KiB, plus 42 KiB.  The same index
 * of every array is read and written at the same time; arrays that start
 * at the same offset within large power-of-two blocks (separate large
 * allocations, for instance) can then meet on the same HBM channels, and on
 * MI355X that cost the symmetric binary64 forward kernel up to 10 points of
 * HBM bandwidth (68% against 78% of 8 TB/s on 2^26 matrices).  A stagger
 * that is a single power of two can itself cancel against one address bit
 * of the array size (8 KiB measured 62% on 2^25 general binary64
 * matrices); 42 KiB = 32 + 8 + 2 KiB measured 71-80% on every size from
 * 2^22 to 2^28 matrices.  Every array start keeps the alignment of the
 * buffer up to 2 KiB.  A pure function: no device access.  Returns -1 for
 * n < 0, n > 2^56 or an unknown dtype. */
int64_t eig3_soa_stride(int64_t n, int32_t dtype);

/* Static, human-readable name of a status code. */
const char *eig3_status_string(int status);

/* Library version, "major.minor.patch". */
const char *eig3_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EIG3_H */
