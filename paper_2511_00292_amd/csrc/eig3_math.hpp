// eig3_math.hpp -- per-lane arithmetic of closed-form 3x3 eigenvalues for
// gfx950.  One matrix per lane; everything lives in registers.
//
// Habera & Zilian, "Numerically stable evaluation of closed-form expressions
// for eigenvalues of 3x3 matrices" (arXiv 2511.00292):
//   I1     Alg. alg:I1-stable
//   J2     Alg. alg:J2-stable (diagonal differences d0, d1, d2 + off-diagonal products)
//   J3     Alg. alg:J3-stable (t1, t2, t3 from the differences; offdiag, mixed, diag parts)
//   Delta  Alg. alg:disc-stable: sum_i w_i u_i v_i with u = dx(A), v = dx(A^T),
//          w = (9, 6, 6, 6, 8, 8, 8, 2, 2, 2, 2, 2, 2, 1); r10 of dx is taken
//          with + M02 M21 d2 (the printed minus sign does not reproduce
//          4 J2^3 - 27 J3^2).
//   lambda Alg. alg:eigvals-stable / Eq. eigvals-trig.
//
// Three evaluations of the invariants share the trigonometric tail: FMA (the
// algorithms above with explicit fused multiply-adds), COMPENSATED (the same
// algorithms with error-free products and sums throughout) and DOUBLE WORD
// (J2 and J3 kept unrounded as K2 = 6 J2 and K3 = 27 J3 in double-word
// arithmetic, Delta from its definition (K2^3 - 2 K3^2) / 54 in double-word
// arithmetic); the binary32 section at the end adapts them to binary32 data.
//
// This file is compiled with -ffp-contract=off: every fused multiply-add is
// written out, and the error-free transformations below rely on the absence
// of any other contraction.
#pragma once

#include <hip/hip_runtime.h>

namespace eig3 {

struct Inv {
    double i1, j2, j3, disc;
};

// ------------------------------------------------------------------ basics
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// exact product a*b = p + e (FMA error-free transformation)
template <class T> __device__ __forceinline__ void two_prod(T a, T b, T &p, T &e)
{
    p = a * b;
    e = fma_(a, b, -p);
}

// exact sum a+b = s + e (Knuth's branch-free TwoSum)
template <class T> __device__ __forceinline__ void two_sum(T a, T b, T &s, T &e)
{
    s = a + b;
    T bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// A pair product kept exactly as hi + lo.
template <class T> struct PairT {
    T hi, lo;
};
template <class T> __device__ __forceinline__ PairT<T> pair(T a, T b)
{
    PairT<T> p;
    two_prod(a, b, p.hi, p.lo);
    return p;
}
// k*x*y for a small integer constant k, kept exactly as hi + lo: the pair
// product x*y is exact, k*hi is split exactly by TwoProduct, and k*lo adds a
// rounding of order eps^2 |k x y| (rounding k*x first would cost eps |k x y|)
template <class T> __device__ __forceinline__ PairT<T> pair_scaled(T k, T x, T y)
{
    const PairT<T> p = pair(x, y);
    PairT<T> r;
    two_prod(k, p.hi, r.hi, r.lo);
    r.lo = fma_(k, p.lo, r.lo);
    return r;
}
template <class T> __device__ __forceinline__ PairT<T> neg(PairT<T> p) { return PairT<T>{-p.hi, -p.lo}; }
using Pair = PairT<double>;

// Compensated accumulator of triple products (x*y)*z with x*y given exactly
// as a pair: the running value is s + c, where s collects the rounded leading
// parts through TwoSum and c collects every rounding error to first order
// (Ogita, Rump & Oishi's compensated dot product, applied to the factored
// products).  The result is as accurate as if computed in twice the working
// precision and then rounded.
template <class T> struct AccT {
    T s, c;
    __device__ __forceinline__ void first(PairT<T> xy, T z)
    {
        two_prod(xy.hi, z, s, c);
        c = fma_(xy.lo, z, c);
    }
    __device__ __forceinline__ void add(PairT<T> xy, T z)
    {
        T q, qe, t, te;
        two_prod(xy.hi, z, q, qe);
        two_sum(s, q, t, te);
        s = t;
        c = c + (te + fma_(xy.lo, z, qe));
    }
    __device__ __forceinline__ T value() const { return s + c; }
    // the value rounded once (hi) and its remainder (lo, exact when |s| >= |c|)
    __device__ __forceinline__ void split(T &hi, T &lo) const
    {
        hi = s + c;
        lo = c - (hi - s);
    }
};
using Acc = AccT<double>;

// ------------------------------------------------------------ diagonal part
struct Diag {
    double d0, d1, d2; // A00 - A11, A00 - A22, A11 - A22
    double i1;
};
__device__ __forceinline__ Diag diag_part(double a00, double a11, double a22)
{
    Diag g;
    g.d0 = a00 - a11;
    g.d1 = a00 - a22;
    g.d2 = a11 - a22;
    g.i1 = (a00 + a11) + a22; // Alg. alg:I1-stable
    return g;
}

// For the compensated evaluations: d0 and d2 as rounded differences and
// d1 = d0 + d2 exactly, as d1 + d1l.  The three rounded differences
// A00 - A11, A00 - A22, A11 - A22 need not satisfy d1 = d0 + d2, and then they
// are the diagonal differences of no matrix: near a triple root the factors
// of Delta, evaluated exactly from such a triple, miss Delta by far more than
// the stability bound allows.  A consistent triple is the exact difference
// data of a diagonal perturbed by one rounding, a backward error.
template <class T> struct DiagC {
    T d0, d1, d2, d1l;
};
template <class T> __device__ __forceinline__ DiagC<T> diag_consistent(T a00, T a11, T a22)
{
    DiagC<T> g;
    g.d0 = a00 - a11;
    g.d2 = a11 - a22;
    two_sum(g.d0, g.d2, g.d1, g.d1l);
    return g;
}

constexpr double kSixth = 1.0 / 6.0;
constexpr double kThird = 1.0 / 3.0;
constexpr double kTwentySeventh = 1.0 / 27.0;

// binary64 constants with full mantissas live in the constant address space:
// the kernels read them with scalar loads into SGPRs, which a VALU operation
// takes as its scalar operand, instead of rebuilding each one per wave with
// two vector moves.
struct ConstTable {
    double atan[11]; // arctangent polynomial, z^1 .. z^21 (see below)
    double sinc[7];  // Taylor coefficients of sin, t^3 .. t^15
    double cosc[7];  // Taylor coefficients of cos, t^2 .. t^14
};
__constant__ ConstTable kC = {
    {0.9999999999999999665383002, -0.3333333333332857960189553, 0.1999999999888207705532328,
     -0.1428571418297856464657463, 0.1111110625599581821334887, -0.09090774712795826084526493,
     0.07689975128569665072030238, -0.06640410811535267761156447, 0.05689223501766054343064029,
     -0.04350445257430010837229732, 0.02116321748124264808858265},
    {-1.0 / 6.0, 1.0 / 120.0, -1.0 / 5040.0, 1.0 / 362880.0, -1.0 / 39916800.0, 1.0 / 6227020800.0,
     -1.0 / 1307674368000.0},
    {-0.5, 1.0 / 24.0, -1.0 / 720.0, 1.0 / 40320.0, -1.0 / 3628800.0, 1.0 / 479001600.0, -1.0 / 87178291200.0},
};

// ====================================================================== FMA
// The paper's algorithms as printed, with products and sums fused where a
// fused multiply-add applies.

// --------------------------------------------------------------- general
struct Gen {
    double a00, a01, a02, a10, a11, a12, a20, a21, a22;
};

// Off-diagonal entries of M (M = A or A^T) and the diagonal differences of A.
struct Off {
    double M01, M02, M10, M12, M20, M21;
};

// r_(I+1) of dx(M; d0, d1, d2) with fused multiply-adds.
template <int I> __device__ __forceinline__ double dx_fma_r(const Off &m, double d0, double d1, double d2)
{
    const double M01 = m.M01, M02 = m.M02, M10 = m.M10, M12 = m.M12, M20 = m.M20, M21 = m.M21;
    if constexpr (I == 0)
        return fma_(M01 * M12, M20, -(M02 * M10 * M21));
    else if constexpr (I == 1)
        return fma_(-(M01 * M02), d2, fma_(M01 * M01, M12, -(M02 * M02 * M21)));
    else if constexpr (I == 2)
        return fma_(M01 * M21, d1, fma_(-(M01 * M01), M20, M02 * M21 * M21));
    else if constexpr (I == 3)
        return fma_(M02 * M12, d0, fma_(M01 * M12, M12, -(M02 * M02 * M10)));
    else if constexpr (I == 4)
        return fma_(M01 * M12, d1, fma_(-(M01 * M02), M10, M02 * M12 * M21));
    else if constexpr (I == 5)
        return fma_(M02 * M21, d0, fma_(-(M01 * M02), M20, M01 * M12 * M21));
    else if constexpr (I == 6)
        return fma_(-(M02 * M10), d2, fma_(M01 * M10, M12, -(M02 * M12 * M20)));
    else if constexpr (I == 7)
        return fma_(M12, d0 * d1, fma_(-(M02 * M10), d1, fma_(M01 * M10, M12, -(M12 * M12 * M21))));
    else if constexpr (I == 8)
        return fma_(M12, d0 * d1, fma_(-(M02 * M10), d0, fma_(M02 * M12, M20, -(M12 * M12 * M21))));
    else if constexpr (I == 9)
        return fma_(M01, d1 * d2, fma_(M02 * M21, d2, fma_(M01 * M02, M20, -(M01 * M01 * M10))));
    else if constexpr (I == 10)
        return fma_(M01, d1 * d2, fma_(M02 * M21, d1, fma_(M01 * M12, M21, -(M01 * M01 * M10))));
    else if constexpr (I == 11)
        return fma_(-M02, d0 * d2, fma_(M01 * M12, d0, fma_(M02 * M12, M21, -(M02 * M02 * M20))));
    else if constexpr (I == 12)
        return fma_(M02, d0 * d2, fma_(M01 * M12, d2, fma_(-(M01 * M02), M10, M02 * M02 * M20)));
    else
        return fma_(d0 * d1, d2, fma_(-(M01 * M10), d0, fma_(M02 * M20, d1, -(M12 * M21 * d2))));
}

constexpr double kW[14] = {9, 6, 6, 6, 8, 8, 8, 2, 2, 2, 2, 2, 2, 1};

// Delta = sum_i w_i u_i v_i, u = dx(A), v = dx(A^T), each pair formed and
// accumulated in turn (small weights first) so that few values stay live.
template <int I> __device__ __forceinline__ double disc_fma_acc(const Off &a, const Off &at, double d0, double d1,
                                                                double d2, double s)
{
    const double u = dx_fma_r<I>(a, d0, d1, d2);
    const double v = dx_fma_r<I>(at, d0, d1, d2);
    s = (I == 13) ? u * v : fma_(kW[I] * u, v, s);
    if constexpr (I > 0)
        return disc_fma_acc<I - 1>(a, at, d0, d1, d2, s);
    else
        return s;
}

__device__ __forceinline__ Inv invariants_general_fma(const Gen &A)
{
    Inv r;
    const Diag g = diag_part(A.a00, A.a11, A.a22);
    r.i1 = g.i1;
    // J2 (Alg. alg:J2-stable)
    const double off2 = fma_(A.a01, A.a10, fma_(A.a02, A.a20, A.a12 * A.a21));
    r.j2 = fma_(fma_(g.d0, g.d0, fma_(g.d1, g.d1, g.d2 * g.d2)), kSixth, off2);
    // J3 (Alg. alg:J3-stable)
    const double t1 = g.d1 + g.d2, t2 = g.d0 - g.d2, t3 = -g.d0 - g.d1;
    const double off3 = fma_(A.a01 * A.a12, A.a20, A.a02 * A.a10 * A.a21);
    const double mixed = fma_(A.a01 * A.a10, t1, fma_(A.a02 * A.a20, t2, A.a12 * A.a21 * t3));
    r.j3 = fma_(-(t1 * t2) * t3, kTwentySeventh, fma_(mixed, kThird, off3));
    // Delta (Alg. alg:disc-stable); M = A for u, M = A^T for v
    const Off a{A.a01, A.a02, A.a10, A.a12, A.a20, A.a21};
    const Off at{A.a10, A.a20, A.a01, A.a21, A.a02, A.a12};
    r.disc = disc_fma_acc<13>(a, at, g.d0, g.d1, g.d2, 0.0);
    return r;
}

// --------------------------------------------------------------- symmetric
struct Sym {
    double s00, s11, s22, s01, s02, s12;
};

// For a symmetric matrix u = v, r1 = 0, r2 = r7, r3 = r5, r4 = r6, so
// Delta = 14 (u2^2 + u3^2 + u4^2) + 2 (u8^2 + ... + u13^2) + u14^2: a sum of
// squares with positive weights (no cancellation in the final sum).
__device__ __forceinline__ Inv invariants_symmetric_fma(const Sym &S)
{
    Inv r;
    const Diag g = diag_part(S.s00, S.s11, S.s22);
    r.i1 = g.i1;
    const double q01 = S.s01 * S.s01, q02 = S.s02 * S.s02, q12 = S.s12 * S.s12;
    r.j2 = fma_(fma_(g.d0, g.d0, fma_(g.d1, g.d1, g.d2 * g.d2)), kSixth, q01 + (q02 + q12));
    const double t1 = g.d1 + g.d2, t2 = g.d0 - g.d2, t3 = -g.d0 - g.d1;
    const double off3 = 2.0 * (S.s01 * S.s12 * S.s02);
    const double mixed = fma_(q01, t1, fma_(q02, t2, q12 * t3));
    r.j3 = fma_(-(t1 * t2) * t3, kTwentySeventh, fma_(mixed, kThird, off3));
    const double d0 = g.d0, d1 = g.d1, d2 = g.d2;
    const double a = S.s01, b = S.s02, c = S.s12;
    const double ab = a * b, ac = a * c, bc = b * c;
    // the three differences of squares, each also used negated
    const double q01m02 = q01 - q02, q01m12 = q01 - q12, q02m12 = q02 - q12;
    const double u2 = fma_(-ab, d2, q01m02 * c);
    const double u3 = fma_(ac, d1, fma_(-q01, b, q12 * b));
    const double u4 = fma_(bc, d0, fma_(-q02, a, q12 * a));
    const double d0d1 = d0 * d1, d1d2 = d1 * d2, d0d2 = d0 * d2;
    const double u8 = fma_(c, d0d1, fma_(-ab, d1, q01m12 * c));
    const double u9 = fma_(c, d0d1, fma_(-ab, d0, q02m12 * c));
    const double u10 = fma_(a, d1d2, fma_(bc, d2, -q01m02 * a));
    const double u11 = fma_(a, d1d2, fma_(bc, d1, -q01m12 * a));
    const double u12 = fma_(-b, d0d2, fma_(ac, d0, -q02m12 * b));
    const double u13 = fma_(b, d0d2, fma_(ac, d2, -q01m02 * b));
    const double u14 = fma_(d0d1, d2, fma_(-q01, d0, fma_(q02, d1, -q12 * d2)));
    // the squares grouped by weight; every partial sum is nonnegative
    double s2 = u13 * u13;
    s2 = fma_(u12, u12, s2);
    s2 = fma_(u11, u11, s2);
    s2 = fma_(u10, u10, s2);
    s2 = fma_(u9, u9, s2);
    s2 = fma_(u8, u8, s2);
    double s14 = u4 * u4;
    s14 = fma_(u3, u3, s14);
    s14 = fma_(u2, u2, s14);
    r.disc = fma_(14.0, s14, fma_(2.0, s2, u14 * u14));
    return r;
}

// ============================================================ COMPENSATED
// Same algorithms; every sum of (triple) products is accumulated with exact
// pair products and TwoSum, so that each r_i, J2 and J3 carries the accuracy
// of twice the working precision before its final rounding.

// The operands of dx(M; d0, d1, d2) with every pair product formed once,
// exactly, as hi + lo.
template <class T> struct DxPairs {
    T M01, M02, M10, M12, M20, M21, d0, d1, d2;
    T d1l; // d1 = d0 + d2 exactly as d1 + d1l (see diag_consistent)
    PairT<T> d0d1, d1d2, d0d2;
    PairT<T> m01m12, m02m10, m01m02, m01m01, m02m02, m01m21, m02m21, m02m12, m01m10, m12m12, m02m20, m12m21;
};

template <class T>
__device__ __forceinline__ DxPairs<T> dx_pairs(T M01, T M02, T M10, T M12, T M20, T M21, T d0, T d1, T d2,
                                               const PairT<T> &d0d1, const PairT<T> &d1d2, const PairT<T> &d0d2,
                                               T d1l = T(0))
{
    DxPairs<T> p{M01, M02, M10, M12, M20, M21, d0, d1, d2, d1l, d0d1, d1d2, d0d2, {}, {}, {}, {}, {}, {}, {}, {}, {},
                 {}, {}, {}};
    // d0 d1 and d1 d2 with d1's low part (its product is of order eps^2)
    p.d0d1.lo = fma_(d0, d1l, p.d0d1.lo);
    p.d1d2.lo = fma_(d1l, d2, p.d1d2.lo);
    p.m01m12 = pair(M01, M12);
    p.m02m10 = pair(M02, M10);
    p.m01m02 = pair(M01, M02);
    p.m01m01 = pair(M01, M01);
    p.m02m02 = pair(M02, M02);
    p.m01m21 = pair(M01, M21);
    p.m02m21 = pair(M02, M21);
    p.m02m12 = pair(M02, M12);
    p.m01m10 = pair(M01, M10);
    p.m12m12 = pair(M12, M12);
    p.m02m20 = pair(M02, M20);
    p.m12m21 = pair(M12, M21);
    return p;
}

// r_(I+1) of dx, compensated, returned as hi + lo.
template <int I, class T> __device__ __forceinline__ void dx_comp_r(const DxPairs<T> &p, T &hi, T &lo)
{
    AccT<T> a;
    if constexpr (I == 0) {
        a.first(p.m01m12, p.M20);
        a.add(neg(p.m02m10), p.M21);
    } else if constexpr (I == 1) {
        a.first(neg(p.m01m02), p.d2);
        a.add(p.m01m01, p.M12);
        a.add(neg(p.m02m02), p.M21);
    } else if constexpr (I == 2) {
        a.first(p.m01m21, p.d1);
        a.c = fma_(p.m01m21.hi, p.d1l, a.c);
        a.add(neg(p.m01m01), p.M20);
        a.add(p.m02m21, p.M21);
    } else if constexpr (I == 3) {
        a.first(p.m02m12, p.d0);
        a.add(p.m01m12, p.M12);
        a.add(neg(p.m02m02), p.M10);
    } else if constexpr (I == 4) {
        a.first(p.m01m12, p.d1);
        a.c = fma_(p.m01m12.hi, p.d1l, a.c);
        a.add(neg(p.m01m02), p.M10);
        a.add(p.m02m12, p.M21);
    } else if constexpr (I == 5) {
        a.first(p.m02m21, p.d0);
        a.add(neg(p.m01m02), p.M20);
        a.add(p.m01m12, p.M21);
    } else if constexpr (I == 6) {
        a.first(neg(p.m02m10), p.d2);
        a.add(p.m01m10, p.M12);
        a.add(neg(p.m02m12), p.M20);
    } else if constexpr (I == 7) {
        a.first(p.d0d1, p.M12);
        a.add(neg(p.m02m10), p.d1);
        a.c = fma_(-p.m02m10.hi, p.d1l, a.c);
        a.add(p.m01m10, p.M12);
        a.add(neg(p.m12m12), p.M21);
    } else if constexpr (I == 8) {
        a.first(p.d0d1, p.M12);
        a.add(neg(p.m02m10), p.d0);
        a.add(p.m02m12, p.M20);
        a.add(neg(p.m12m12), p.M21);
    } else if constexpr (I == 9) {
        a.first(p.d1d2, p.M01);
        a.add(p.m02m21, p.d2);
        a.add(p.m01m02, p.M20);
        a.add(neg(p.m01m01), p.M10);
    } else if constexpr (I == 10) {
        a.first(p.d1d2, p.M01);
        a.add(p.m02m21, p.d1);
        a.c = fma_(p.m02m21.hi, p.d1l, a.c);
        a.add(p.m01m12, p.M21);
        a.add(neg(p.m01m01), p.M10);
    } else if constexpr (I == 11) {
        a.first(neg(p.d0d2), p.M02);
        a.add(p.m01m12, p.d0);
        a.add(p.m02m12, p.M21);
        a.add(neg(p.m02m02), p.M20);
    } else if constexpr (I == 12) {
        a.first(p.d0d2, p.M02);
        a.add(p.m01m12, p.d2);
        a.add(neg(p.m01m02), p.M10);
        a.add(p.m02m02, p.M20);
    } else {
        a.first(p.d0d1, p.d2);
        a.add(neg(p.m01m10), p.d0);
        a.add(p.m02m20, p.d1);
        a.c = fma_(p.m02m20.hi, p.d1l, a.c);
        a.add(neg(p.m12m21), p.d2);
    }
    a.split(hi, lo);
}

// r_(I+1) and r_(I+2) for I = 7, 9, 11, which share two of their four terms:
// r8, r9 share M12 d0 d1 - M12^2 M21; r10, r11 share M01 d1 d2 - M01^2 M10;
// r13 = -(r12's -M02 d0 d2 - M02^2 M20) + two terms.  The shared part is
// accumulated once.
template <int I, class T>
__device__ __forceinline__ void dx_comp_r2(const DxPairs<T> &p, T &hi0, T &lo0, T &hi1, T &lo1)
{
    static_assert(I == 7 || I == 9 || I == 11, "paired factors");
    AccT<T> a, b;
    if constexpr (I == 7) {
        a.first(p.d0d1, p.M12);
        a.add(neg(p.m12m12), p.M21);
        b = a;
        a.add(neg(p.m02m10), p.d1);
        a.c = fma_(-p.m02m10.hi, p.d1l, a.c);
        a.add(p.m01m10, p.M12);
        b.add(neg(p.m02m10), p.d0);
        b.add(p.m02m12, p.M20);
    } else if constexpr (I == 9) {
        a.first(p.d1d2, p.M01);
        a.add(neg(p.m01m01), p.M10);
        b = a;
        a.add(p.m02m21, p.d2);
        a.add(p.m01m02, p.M20);
        b.add(p.m02m21, p.d1);
        b.c = fma_(p.m02m21.hi, p.d1l, b.c);
        b.add(p.m01m12, p.M21);
    } else {
        a.first(neg(p.d0d2), p.M02);
        a.add(neg(p.m02m02), p.M20);
        b.s = -a.s;
        b.c = -a.c;
        a.add(p.m01m12, p.d0);
        a.add(p.m02m12, p.M21);
        b.add(p.m01m12, p.d2);
        b.add(neg(p.m01m02), p.M10);
    }
    a.split(hi0, lo0);
    b.split(hi1, lo1);
}

template <int I, class T> __device__ __forceinline__ void dx_comp_all(const DxPairs<T> &p, T rh[14], T rl[14])
{
    if constexpr (I == 7 || I == 9 || I == 11) {
        dx_comp_r2<I>(p, rh[I], rl[I], rh[I + 1], rl[I + 1]);
        dx_comp_all<I + 2>(p, rh, rl);
    } else {
        dx_comp_r<I>(p, rh[I], rl[I]);
        if constexpr (I < 13)
            dx_comp_all<I + 1>(p, rh, rl);
    }
}

// all fourteen r_i of dx, compensated
template <class T>
__device__ __forceinline__ void dx_comp(T M01, T M02, T M10, T M12, T M20, T M21, T d0, T d1, T d2,
                                        const PairT<T> &d0d1, const PairT<T> &d1d2, const PairT<T> &d0d2,
                                        T rh[14], T rl[14], T d1l = T(0))
{
    dx_comp_all<0>(dx_pairs(M01, M02, M10, M12, M20, M21, d0, d1, d2, d0d1, d1d2, d0d2, d1l), rh, rl);
}

// sum_i w_i u_i v_i, u = dx(A) and v = dx(A^T) as hi + lo, compensated;
// weights scale exactly except 6 and 9, which are applied as exact pair
// products.  u_i and v_i are formed index by index and consumed at once
// rather than all fourteen of each first (fewer values live).
template <int I> __device__ __forceinline__ void wuv_acc(double uh, double ul, double vh, double vl, double &s, double &c)
{
    constexpr double w = kW[I];
    double p, pe;
    two_prod(uh, vh, p, pe);
    const double corr = fma_(uh, vl, fma_(ul, vh, pe));
    if constexpr (I == 0) {
        s = w * p;
        // w * p is exact up to one rounding; keep its error
        c = w * corr + fma_(w, p, -s);
    } else if constexpr (w == 8.0 || w == 2.0 || w == 1.0) {
        // a power of two scales exactly
        double t, te;
        two_sum(s, w * p, t, te);
        c = c + fma_(w, corr, te);
        s = t;
    } else {
        double wp, wpe, t, te;
        two_prod(w, p, wp, wpe);
        two_sum(s, wp, t, te);
        c = c + (te + fma_(w, corr, wpe));
        s = t;
    }
}

template <int I>
__device__ __forceinline__ void sum_wuv_comp_step(const DxPairs<double> &pu, const DxPairs<double> &pv, double &s,
                                                  double &c)
{
    if constexpr (I == 7 || I == 9 || I == 11) {
        double uh0, ul0, uh1, ul1, vh0, vl0, vh1, vl1;
        dx_comp_r2<I>(pu, uh0, ul0, uh1, ul1);
        dx_comp_r2<I>(pv, vh0, vl0, vh1, vl1);
        wuv_acc<I>(uh0, ul0, vh0, vl0, s, c);
        wuv_acc<I + 1>(uh1, ul1, vh1, vl1, s, c);
        sum_wuv_comp_step<I + 2>(pu, pv, s, c);
    } else if constexpr (I == 0 || I == 13) {
        // r1 changes sign and r14 is unchanged under A -> A^T (the same
        // products, commuted), so v1 = -u1 and v14 = u14
        double uh, ul;
        dx_comp_r<I>(pu, uh, ul);
        const double sg = I == 0 ? -1.0 : 1.0;
        wuv_acc<I>(uh, ul, sg * uh, sg * ul, s, c);
        if constexpr (I < 13)
            sum_wuv_comp_step<I + 1>(pu, pv, s, c);
    } else {
        double uh, ul, vh, vl;
        dx_comp_r<I>(pu, uh, ul);
        dx_comp_r<I>(pv, vh, vl);
        wuv_acc<I>(uh, ul, vh, vl, s, c);
        sum_wuv_comp_step<I + 1>(pu, pv, s, c);
    }
}

__device__ __forceinline__ double sum_wuv_comp(const DxPairs<double> &pu, const DxPairs<double> &pv)
{
    double s = 0.0, c = 0.0;
    sum_wuv_comp_step<0>(pu, pv, s, c);
    return s + c;
}

__device__ __forceinline__ Inv invariants_general_comp(const Gen &A)
{
    Inv r;
    r.i1 = diag_part(A.a00, A.a11, A.a22).i1;
    const DiagC<double> g = diag_consistent(A.a00, A.a11, A.a22);
    // J2: the sum of squares needs no compensation; the off-diagonal products do
    {
        const Pair p01 = pair(A.a01, A.a10), p02 = pair(A.a02, A.a20), p12 = pair(A.a12, A.a21);
        const double sq = fma_(g.d0, g.d0, fma_(g.d1, g.d1, g.d2 * g.d2)) * kSixth;
        double s, e1, t, e2;
        two_sum(p01.hi, p02.hi, s, e1);
        two_sum(s, p12.hi, t, e2);
        double u, e3;
        two_sum(t, sq, u, e3);
        r.j2 = u + (((e1 + e2) + e3) + fma_(g.d1 * kThird, g.d1l, (p01.lo + p02.lo) + p12.lo));
    }
    // J3: 27 J3 = 27 offdiag + 9 mixed - t1 t2 t3, accumulated compensated
    // (the t's are rounded sums of two differences; their rounding is the
    // backward error the paper's analysis allows)
    {
        const double t1 = g.d1 + g.d2, t2 = g.d0 - g.d2, t3 = -g.d0 - g.d1;
        Acc a;
        a.first(pair_scaled(27.0, A.a01, A.a12), A.a20);
        a.add(pair_scaled(27.0, A.a02, A.a10), A.a21);
        a.add(pair_scaled(9.0, A.a01, A.a10), t1);
        a.add(pair_scaled(9.0, A.a02, A.a20), t2);
        a.add(pair_scaled(9.0, A.a12, A.a21), t3);
        a.add(pair(-t1, t2), t3);
        r.j3 = a.value() * kTwentySeventh;
    }
    // Delta
    {
        const Pair d0d1 = pair(g.d0, g.d1), d1d2 = pair(g.d1, g.d2), d0d2 = pair(g.d0, g.d2);
        r.disc = sum_wuv_comp(
            dx_pairs(A.a01, A.a02, A.a10, A.a12, A.a20, A.a21, g.d0, g.d1, g.d2, d0d1, d1d2, d0d2, g.d1l),
            dx_pairs(A.a10, A.a20, A.a01, A.a21, A.a02, A.a12, g.d0, g.d1, g.d2, d0d1, d1d2, d0d2, g.d1l));
    }
    return r;
}

__device__ __forceinline__ Inv invariants_symmetric_comp(const Sym &S)
{
    // the symmetric path is exactly the general one with A^T = A; u = v
    // keeps the final sum a sum of nonnegative terms
    Gen A{S.s00, S.s01, S.s02, S.s01, S.s11, S.s12, S.s02, S.s12, S.s22};
    Inv r;
    r.i1 = diag_part(S.s00, S.s11, S.s22).i1;
    const DiagC<double> g = diag_consistent(S.s00, S.s11, S.s22);
    const double q01 = S.s01 * S.s01, q02 = S.s02 * S.s02, q12 = S.s12 * S.s12;
    r.j2 = fma_(fma_(g.d0, g.d0, fma_(g.d1, g.d1, g.d2 * g.d2)), kSixth, q01 + (q02 + q12));
    {
        const double t1 = g.d1 + g.d2, t2 = g.d0 - g.d2, t3 = -g.d0 - g.d1;
        Acc a;
        a.first(pair_scaled(54.0, S.s01, S.s12), S.s02);
        a.add(pair_scaled(9.0, S.s01, S.s01), t1);
        a.add(pair_scaled(9.0, S.s02, S.s02), t2);
        a.add(pair_scaled(9.0, S.s12, S.s12), t3);
        a.add(pair(-t1, t2), t3);
        r.j3 = a.value() * kTwentySeventh;
    }
    {
        const Pair d0d1 = pair(g.d0, g.d1), d1d2 = pair(g.d1, g.d2), d0d2 = pair(g.d0, g.d2);
        double uh[14], ul[14];
        dx_comp(A.a01, A.a02, A.a10, A.a12, A.a20, A.a21, g.d0, g.d1, g.d2, d0d1, d1d2, d0d2, uh, ul, g.d1l);
        // Delta = 14 (u2^2 + u3^2 + u4^2) + 2 (u8^2 + ... + u13^2) + u14^2
        // (u1 = M01 M12 M20 - M02 M10 M21 vanishes identically for A^T = A)
        double s = 0.0, c = 0.0;
        const double w[14] = {0, 14, 14, 14, 0, 0, 0, 2, 2, 2, 2, 2, 2, 1};
#pragma unroll
        for (int i = 0; i < 14; ++i) {
            if (w[i] == 0.0)
                continue;
            double p, pe, wp, wpe, t, te;
            two_prod(uh[i], uh[i], p, pe);
            two_prod(w[i], p, wp, wpe);
            two_sum(s, wp, t, te);
            s = t;
            c = c + (te + fma_(w[i], fma_(2.0 * uh[i], ul[i], pe), wpe));
        }
        r.disc = s + c;
    }
    return r;
}

// ============================================================ DOUBLE WORD
// J2 and J3 by Alg. alg:J2-stable and alg:J3-stable, scaled to
//   K2 = 6 J2  = d0^2 + d1^2 + d2^2 + 6 (A01 A10 + A02 A20 + A12 A21),
//   K3 = 27 J3 = 27 (A01 A12 A20 + A02 A10 A21) + 9 (A01 A10 t1 + A02 A20 t2 + A12 A21 t3) - t1 t2 t3,
// and evaluated in double-word arithmetic: every product is split exactly
// (TwoProduct), every sum of leading parts exactly (TwoSum), the low parts
// are summed plainly, and K2, K3 are kept unrounded as hi + lo, exact to
// O(eps^2 sum |terms|).  The inputs are the consistent diagonal differences
// (d0, d2 rounded, d1 = d0 + d2 and t1, t2, t3 exact as pairs), so K2 and K3
// are the invariants of one matrix, the stored one with its diagonal moved
// by one rounding of its differences.  Delta is then its definition beside
// Eq. triple-angle-arctan, 4 J2^3 - 27 J3^2 = (K2^3 - 2 K3^2) / 54, formed
// from the unrounded K2, K3 in double-word arithmetic: the cancellation
// between the two terms, which ruins that formula in working precision and
// which the sum of products of Alg. alg:disc-stable avoids, costs here only
// O(eps^2 |dev A|^6) (second order in the unit roundoff), and Delta = 0 comes
// out exactly where K2, K3 describe an exactly repeated eigenvalue.

// s + c with the leading parts summed exactly
template <class T> struct DWSum {
    T s, c;
    __device__ __forceinline__ void add(T x)
    {
        T t, e;
        two_sum(s, x, t, e);
        s = t;
        c = c + e;
    }
    __device__ __forceinline__ void add(PairT<T> x)
    {
        add(x.hi);
        c = c + x.lo;
    }
    // the value rounded once and its remainder
    __device__ __forceinline__ PairT<T> pair() const
    {
        PairT<T> r;
        r.hi = s + c;
        r.lo = c - (r.hi - s);
        return r;
    }
};

// k * x for a small integer constant k and x = hi + lo, as hi + lo
template <class T> __device__ __forceinline__ PairT<T> scaled(T k, PairT<T> x)
{
    PairT<T> r;
    two_prod(k, x.hi, r.hi, r.lo);
    r.lo = fma_(k, x.lo, r.lo);
    return r;
}

template <class T> struct KPair {
    PairT<T> k2, k3; // 6 J2 and 27 J3, unrounded
};

// K2 and K3 from the consistent differences g, the three diagonal-pair
// products p = A01 A10, q = A02 A20, r = A12 A21 (exact pairs) and the
// off-diagonal triple part 27 (A01 A12 A20 + A02 A10 A21), already
// accumulated in a.
template <class T>
__device__ __forceinline__ KPair<T> k23_dw(const DiagC<T> &g, PairT<T> p, PairT<T> q, PairT<T> r, AccT<T> a)
{
    KPair<T> k;
    {
        // d0^2 + d1^2 + d2^2 with d1 = d0 + d2 exactly (d1 + d1l)
        DWSum<T> sq;
        two_prod(g.d0, g.d0, sq.s, sq.c);
        PairT<T> d1s = pair(g.d1, g.d1);
        d1s.lo = fma_(T(2) * g.d1, g.d1l, d1s.lo);
        sq.add(d1s);
        sq.add(pair(g.d2, g.d2));
        DWSum<T> off{p.hi, p.lo};
        off.add(q);
        off.add(r);
        sq.add(scaled(T(6), PairT<T>{off.s, off.c}));
        k.k2 = sq.pair();
    }
    {
        // t1 = d1 + d2, t2 = d0 - d2, t3 = -d0 - d1, exact as pairs
        T t1, t1l, t2, t2l, t3, t3l;
        two_sum(g.d1, g.d2, t1, t1l);
        t1l = t1l + g.d1l;
        two_sum(g.d0, -g.d2, t2, t2l);
        two_sum(-g.d0, -g.d1, t3, t3l);
        t3l = t3l - g.d1l;
        a.add(scaled(T(9), p), t1);
        a.add(scaled(T(9), q), t2);
        a.add(scaled(T(9), r), t3);
        const PairT<T> t12 = pair(-t1, t2);
        a.add(t12, t3);
        // the low parts of the t's, to first order
        const T lo9 = fma_(p.hi, t1l, fma_(q.hi, t2l, r.hi * t3l));
        const T lot = fma_(t12.hi, t3l, -(fma_(t1l, t2, t1 * t2l) * t3));
        a.c = fma_(T(9), lo9, a.c + lot);
        PairT<T> k3;
        a.split(k3.hi, k3.lo);
        k.k3 = k3;
    }
    return k;
}

template <class T> __device__ __forceinline__ KPair<T> k23_general_dw(const T (&m)[9], const DiagC<T> &g)
{
    // m: A00 A01 A02 A10 A11 A12 A20 A21 A22 (or the deviatoric data in the
    // same positions)
    AccT<T> a;
    a.first(pair_scaled(T(27), m[1], m[5]), m[6]);
    a.add(pair_scaled(T(27), m[2], m[3]), m[7]);
    return k23_dw(g, pair(m[1], m[3]), pair(m[2], m[6]), pair(m[5], m[7]), a);
}

template <class T> __device__ __forceinline__ KPair<T> k23_symmetric_dw(T s01, T s02, T s12, const DiagC<T> &g)
{
    AccT<T> a;
    a.first(pair_scaled(T(54), s01, s12), s02);
    return k23_dw(g, pair(s01, s01), pair(s02, s02), pair(s12, s12), a);
}

// 54 Delta = K2^3 - 2 K3^2 in double-word arithmetic (binary64)
__device__ __forceinline__ double disc54_dw(PairT<double> k2, PairT<double> k3)
{
    double s2, e2;
    two_prod(k2.hi, k2.hi, s2, e2);
    e2 = fma_(2.0 * k2.hi, k2.lo, e2);
    double c3, c3e;
    two_prod(s2, k2.hi, c3, c3e);
    c3e = c3e + fma_(e2, k2.hi, s2 * k2.lo);
    double q2, q2e;
    two_prod(k3.hi, k3.hi, q2, q2e);
    q2e = fma_(2.0 * k3.hi, k3.lo, q2e);
    double d, de;
    two_sum(c3, -2.0 * q2, d, de);
    return d + (de + fma_(-2.0, q2e, c3e));
}

constexpr double kFiftyFourth = 1.0 / 54.0;

__device__ __forceinline__ Inv invariants_of_k(double i1, const KPair<double> &k)
{
    Inv r;
    r.i1 = i1;
    r.j2 = (k.k2.hi + k.k2.lo) * kSixth;
    r.j3 = (k.k3.hi + k.k3.lo) * kTwentySeventh;
    r.disc = disc54_dw(k.k2, k.k3) * kFiftyFourth;
    return r;
}

__device__ __forceinline__ Inv invariants_general_dw(const Gen &A)
{
    const double m[9] = {A.a00, A.a01, A.a02, A.a10, A.a11, A.a12, A.a20, A.a21, A.a22};
    return invariants_of_k(diag_part(A.a00, A.a11, A.a22).i1,
                           k23_general_dw(m, diag_consistent(A.a00, A.a11, A.a22)));
}

__device__ __forceinline__ Inv invariants_symmetric_dw(const Sym &S)
{
    return invariants_of_k(diag_part(S.s00, S.s11, S.s22).i1,
                           k23_symmetric_dw(S.s01, S.s02, S.s12, diag_consistent(S.s00, S.s11, S.s22)));
}

// ======================================================= transcendentals
// The triple angle needs atan2 of two nonnegative numbers and the sine and
// cosine of a third of it, t in [0, pi/6]; neither needs a general range
// reduction.
//
// atan: q = min/max in [0, 1]; for q > tan(pi/8) the identity
// atan(q) = pi/4 + atan((q - 1)/(q + 1)) maps it into [-tan(pi/8), 0], folded
// into the same single division.  atan(z) = z P(z^2) on |z| <= tan(pi/8), P
// a least-squares polynomial on Chebyshev nodes (csrc/gen_poly.py): relative
// error 3.4e-17 (binary64, degree 10) and 1.8e-8 (binary32, degree 4).
// sin, cos: Taylor polynomials on [0, pi/6]; the first omitted term is below
// 2e-18 (binary64: to t^15 and t^14) and 4e-10 (binary32: to t^9 and t^8).
constexpr double kPi2 = 1.5707963267948966192;
constexpr double kPi4 = 0.78539816339744830962;
constexpr double kTanPi8 = 0.41421356237309504880;

// The coefficient tables exist twice: in constant memory (read into SGPRs by
// scalar loads; used where the kernel has SGPRs to spare) and as immediates
// (rebuilt in VGPRs; used where the kernel's pointer arguments already fill
// the SGPR file, i.e. the adjoint with its 21 pointers).
constexpr double kAtanImm[11] = {0.9999999999999999665383002, -0.3333333333332857960189553,
                                 0.1999999999888207705532328, -0.1428571418297856464657463,
                                 0.1111110625599581821334887, -0.09090774712795826084526493,
                                 0.07689975128569665072030238, -0.06640410811535267761156447,
                                 0.05689223501766054343064029, -0.04350445257430010837229732,
                                 0.02116321748124264808858265};
constexpr double kSinImm[7] = {-1.0 / 6.0, 1.0 / 120.0, -1.0 / 5040.0, 1.0 / 362880.0, -1.0 / 39916800.0,
                               1.0 / 6227020800.0, -1.0 / 1307674368000.0};
constexpr double kCosImm[7] = {-0.5, 1.0 / 24.0, -1.0 / 720.0, 1.0 / 40320.0, -1.0 / 3628800.0,
                               1.0 / 479001600.0, -1.0 / 87178291200.0};

template <bool Table> __device__ __forceinline__ double atan_coef(int j) { return Table ? kC.atan[j] : kAtanImm[j]; }
template <bool Table> __device__ __forceinline__ double sin_coef(int j) { return Table ? kC.sinc[j] : kSinImm[j]; }
template <bool Table> __device__ __forceinline__ double cos_coef(int j) { return Table ? kC.cosc[j] : kCosImm[j]; }

template <bool Table> __device__ __forceinline__ double atan_poly(double u)
{
    double p = atan_coef<Table>(10);
#pragma unroll
    for (int j = 9; j >= 0; --j)
        p = fma_(p, u, atan_coef<Table>(j));
    return p;
}

template <bool Table> __device__ __forceinline__ float atan_poly(float u)
{
    float p = 0.07984962911065899521160472f;
    p = fma_(p, u, -0.1385147842677151367970504f);
    p = fma_(p, u, 0.1997440478587335297876003f);
    p = fma_(p, u, -0.3333279693519533346875533f);
    p = fma_(p, u, 0.9999999818725111375741227f);
    return p;
}

// atan2(y, x) for y, x >= 0, in [0, pi/2]; atan2(0, 0) = 0; NaN in, NaN out.
template <class T> struct AngleConsts;
template <> struct AngleConsts<double> {
    __device__ static double tanpi8() { return kTanPi8; }
    __device__ static double pi4() { return kPi4; }
    __device__ static double pi2() { return kPi2; }
};
template <> struct AngleConsts<float> {
    __device__ static float tanpi8() { return float(kTanPi8); }
    __device__ static float pi4() { return float(kPi4); }
    __device__ static float pi2() { return float(kPi2); }
};

// Quotient inside the arctangent, where den >= M, the larger operand.
// binary64: correctly rounded division (any operand range).  binary32: the
// caller scales the pair by a power of two so that M lies in [1/2, 1), hence
// den in [1/2, 2): the hardware reciprocal (1 ulp) plus one residual
// correction, with no range handling needed.
__device__ __forceinline__ double quot_reduced(double num, double den) { return num / den; }
__device__ __forceinline__ float quot_reduced(float num, float den)
{
    const float r = __builtin_amdgcn_rcpf(den);
    const float q = num * r;
    return fma_(fma_(-den, q, num), r, q);
}

template <bool Table = true, class T> __device__ __forceinline__ T atan2_nonneg(T y, T x)
{
    const T m = y < x ? y : x;
    const T M = y < x ? x : y;
    const bool far = m > AngleConsts<T>::tanpi8() * M;
    const T num = far ? m - M : m;
    const T den = far ? m + M : M;
    // 0/0 -> 0; a NaN operand fails the comparison and propagates
    const T z = M == T(0) ? T(0) : quot_reduced(num, den);
    T r = z * atan_poly<Table>(z * z);
    r = far ? r + AngleConsts<T>::pi4() : r;
    return y > x ? AngleConsts<T>::pi2() - r : r;
}

template <bool Table> __device__ __forceinline__ void sincos_sixth(double t, double &s, double &c)
{
    const double u = t * t;
    double ps = sin_coef<Table>(6);
#pragma unroll
    for (int j = 5; j >= 0; --j)
        ps = fma_(ps, u, sin_coef<Table>(j));
    s = fma_(t * u, ps, t);
    double pc = cos_coef<Table>(6);
#pragma unroll
    for (int j = 5; j >= 0; --j)
        pc = fma_(pc, u, cos_coef<Table>(j));
    c = fma_(u, pc, 1.0);
}

template <bool Table> __device__ __forceinline__ void sincos_sixth(float t, float &s, float &c)
{
    const float u = t * t;
    float ps = 1.0f / 362880.0f;
    ps = fma_(ps, u, -1.0f / 5040.0f);
    ps = fma_(ps, u, 1.0f / 120.0f);
    ps = fma_(ps, u, -1.0f / 6.0f);
    s = fma_(t * u, ps, t);
    float pc = 1.0f / 40320.0f;
    pc = fma_(pc, u, -1.0f / 720.0f);
    pc = fma_(pc, u, 1.0f / 24.0f);
    pc = fma_(pc, u, -0.5f);
    c = fma_(u, pc, 1.0f);
}

// ============================================================ eigenvalues
// lambda_k = I1/3 + mu_k with the deviatoric eigenvalues mu_k = 2 sqrt(J2/3)
// cos((phi + 2 pi k)/3), phi = atan2(sqrt(27 Delta), 27 J3) in [0, pi]
// (Eq. eigvals-trig with the atan2 reading of Eq. triple-angle-arctan).
// Evaluated through psi = atan2(sqrt(27 Delta), 27 |J3|) in [0, pi/2]: the
// roots for -J3 are the negated roots for J3, so for J3 < 0 the values are
// negated and reversed.  t = psi/3 stays in [0, pi/6], both coalescence
// limits (phi -> 0 and phi -> pi) become small angles, the three gaps
//   mu3 - mu1 = r (3c + sqrt3 s), mu3 - mu2 = r (3c - sqrt3 s),
//   mu2 - mu1 = 2 sqrt3 r s          (r = sqrt(J2/3), c = cos t, s = sin t)
// have no cancellation, and mu1 <= mu2 <= mu3 holds after rounding.
struct Trig {
    double mean; // I1 / 3
    double r;    // sqrt(J2 / 3)
    double c, s; // cos t, sin t
    bool neg;    // J3 < 0
};

constexpr double kSqrt3 = 1.7320508075688772935;

// max(x, 0) that keeps NaN (fmax would drop it)
__device__ __forceinline__ double clamp0(double x) { return x < 0.0 ? 0.0 : x; }

// Square root of x >= 0 (NaN propagates): the hardware reciprocal square
// root (relative error about 2^-23, denormals supported) refined by one
// Goldschmidt step and two Newton corrections of the root, within an ulp.
// The library's own sequence also rescales tiny and huge operands and fixes
// up 0 and Inf; here only 0 needs it (rsq(0) = Inf), the operands being the
// scaled matrix's J2 / 3 and 27 Delta.
__device__ __forceinline__ double sqrt_nonneg(double x)
{
    const double r = __builtin_amdgcn_rsq(x);
    double g = x * r, h = 0.5 * r;
    const double e = fma_(-h, g, 0.5);
    g = fma_(g, e, g);
    h = fma_(h, e, h);
    g = fma_(fma_(-g, g, x), h, g);
    g = fma_(fma_(-g, g, x), h, g);
    return x == 0.0 ? x : g;
}

// From I1, J2 / 3, 27 Delta and 27 J3 (each up to rounding; J2 < 0 and
// Delta < 0 are clamped to 0).
template <bool Table> __device__ __forceinline__ Trig trig_core(double i1, double j2_3, double disc27, double j3_27)
{
    Trig t;
    double psi = atan2_nonneg<Table>(sqrt_nonneg(clamp0(disc27)), fabs(j3_27));
    psi = j3_27 == j3_27 ? psi : j3_27; // NaN in J3 reaches the eigenvalues
    sincos_sixth<Table>(psi * kThird, t.s, t.c);
    t.r = sqrt_nonneg(clamp0(j2_3));
    t.mean = i1 * kThird;
    t.neg = j3_27 < 0.0;
    return t;
}

template <bool Table = true> __device__ __forceinline__ Trig trig_from_invariants(const Inv &v)
{
    return trig_core<Table>(v.i1, v.j2 * kThird, 27.0 * v.disc, 27.0 * v.j3);
}

// The double-word evaluation's K2 = 6 J2, K3 = 27 J3 and 54 Delta give
// J2 / 3 = K2 / 18, 27 Delta = 54 Delta / 2 and 27 J3 = K3 directly.
template <bool Table = true> __device__ __forceinline__ Trig trig_from_k(double i1, const KPair<double> &k)
{
    constexpr double kEighteenth = 1.0 / 18.0;
    return trig_core<Table>(i1, (k.k2.hi + k.k2.lo) * kEighteenth, 0.5 * disc54_dw(k.k2, k.k3), k.k3.hi + k.k3.lo);
}

__device__ __forceinline__ void mu_from_trig(const Trig &t, double &m1, double &m2, double &m3)
{
    const double a1 = -t.r * fma_(kSqrt3, t.s, t.c);
    const double a2 = t.r * fma_(kSqrt3, t.s, -t.c);
    const double a3 = 2.0 * t.r * t.c;
    m1 = t.neg ? -a3 : a1;
    m2 = t.neg ? -a2 : a2;
    m3 = t.neg ? -a1 : a3;
}

// The eigenvalue gaps mu2 - mu1, mu3 - mu1, mu3 - mu2 (all >= 0) from the
// trigonometric form, free of cancellation (for the |J3| configuration, with
// the roles of the two outer gaps swapped when J3 < 0).
struct Gaps {
    double e12, e13, e23;
};
__device__ __forceinline__ Gaps gaps_from_trig(const Trig &t)
{
    const double e13 = t.r * fma_(3.0, t.c, kSqrt3 * t.s);
    const double e23p = t.r * fma_(3.0, t.c, -kSqrt3 * t.s);
    const double e12p = 2.0 * kSqrt3 * t.r * t.s;
    return Gaps{t.neg ? e23p : e12p, e13, t.neg ? e12p : e23p};
}

__device__ __forceinline__ void eigvals_from_trig(const Trig &t, double &l1, double &l2, double &l3)
{
    double m1, m2, m3;
    mu_from_trig(t, m1, m2, m3);
    l1 = t.mean + m1;
    l2 = t.mean + m2;
    l3 = t.mean + m3;
}

__device__ __forceinline__ void eigvals_from_invariants(const Inv &v, double &l1, double &l2, double &l3)
{
    eigvals_from_trig(trig_from_invariants(v), l1, l2, l3);
}

// ============================================================ comparators
// The paper's naive evaluations, kept as GPU comparators that show why the
// stable algorithms are needed.  Plain products and sums, no FMA, in the
// printed (left-to-right) order, so that they reproduce a plain binary64
// evaluation operation for operation.
//   naive:  Alg. alg:J2-naive and alg:J3-naive (monomial sums)
//   tensor: Alg. alg:J2-tensor and alg:J3-tensor (S = A - tr(A)/3 I,
//           tr(S S)/2, det S by LU with partial pivoting and reciprocal
//           pivots, the LAPACK factorisation behind NumPy's determinant)
//   both:   Delta = 4 J2^3 - 27 J3^2.

__device__ __forceinline__ Inv invariants_general_naive(const Gen &A)
{
    const double A00 = A.a00, A01 = A.a01, A02 = A.a02, A10 = A.a10, A11 = A.a11, A12 = A.a12, A20 = A.a20,
                 A21 = A.a21, A22 = A.a22;
    Inv r;
    r.i1 = (A00 + A11) + A22;
    r.j2 = (A00 * A00 - A00 * A11 - A00 * A22 + 3 * A01 * A10 + 3 * A02 * A20 + A11 * A11 - A11 * A22 +
            3 * A12 * A21 + A22 * A22) / 3.0;
    r.j3 = (2 * A00 * A00 * A00 - 3 * A00 * A00 * A11 - 3 * A00 * A00 * A22 + 9 * A00 * A01 * A10 +
            9 * A00 * A02 * A20 - 3 * A00 * A11 * A11 + 12 * A00 * A11 * A22 - 18 * A00 * A12 * A21 -
            3 * A00 * A22 * A22 + 9 * A01 * A10 * A11 - 18 * A01 * A10 * A22 + 27 * A01 * A12 * A20 +
            27 * A02 * A10 * A21 - 18 * A02 * A11 * A20 + 9 * A02 * A20 * A22 + 2 * A11 * A11 * A11 -
            3 * A11 * A11 * A22 + 9 * A11 * A12 * A21 - 3 * A11 * A22 * A22 + 9 * A12 * A21 * A22 +
            2 * A22 * A22 * A22) / 27.0;
    r.disc = 4.0 * r.j2 * r.j2 * r.j2 - 27.0 * r.j3 * r.j3;
    return r;
}

// one elimination step of LU with partial pivoting on column c of the 3x3
// row-major m (rows c..2), as selects: the first row with the largest
// magnitude is the pivot, rows are swapped (sign flipped), and rows below are
// updated with l = m[r][c] * (1 / pivot) unless the pivot is zero.
template <int C> __device__ __forceinline__ void lu_step(double m[9], double &sign)
{
    int p = C;
#pragma unroll
    for (int r = C + 1; r < 3; ++r)
        p = fabs(m[3 * r + C]) > fabs(m[3 * p + C]) ? r : p;
#pragma unroll
    for (int r = C + 1; r < 3; ++r) {
        const bool sw = p == r;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double a = m[3 * C + k], b = m[3 * r + k];
            m[3 * C + k] = sw ? b : a;
            m[3 * r + k] = sw ? a : b;
        }
        sign = sw ? -sign : sign;
    }
    const double piv = m[3 * C + C];
    const bool live = piv != 0.0;
    const double inv = 1.0 / piv;
#pragma unroll
    for (int r = C + 1; r < 3; ++r) {
        const double l = m[3 * r + C] * inv;
#pragma unroll
        for (int k = C + 1; k < 3; ++k) {
            const double upd = m[3 * r + k] - l * m[3 * C + k];
            m[3 * r + k] = live ? upd : m[3 * r + k];
        }
    }
}

__device__ __forceinline__ Inv invariants_general_tensor(const Gen &A)
{
    Inv r;
    r.i1 = (A.a00 + A.a11) + A.a22;
    const double mean = r.i1 / 3.0;
    double S[9] = {A.a00 - mean, A.a01, A.a02, A.a10, A.a11 - mean, A.a12, A.a20, A.a21, A.a22 - mean};
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double sii = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            sii = sii + S[3 * i + k] * S[3 * k + i];
        tr = tr + sii;
    }
    r.j2 = tr / 2.0;
    double sign = 1.0;
    lu_step<0>(S, sign);
    lu_step<1>(S, sign);
    r.j3 = sign * (S[0] * S[4] * S[8]);
    r.disc = 4.0 * r.j2 * r.j2 * r.j2 - 27.0 * r.j3 * r.j3;
    return r;
}

// ================================================================ binary32
// Three evaluations of binary32 batches; each forms the triple-angle argument
// in binary64 (sqrt(27 Delta) and 27 |J3|, rescaled by an exact power of two
// into binary32 range) and finishes with binary32 arctangent, sine and cosine.
// The double-word and compensated evaluations hand K2, K3 and 54 Delta to
// that tail directly (J2 / 3 = K2 / 18, 27 Delta = 54 Delta / 2, 27 J3 = K3).
//
// Widened (EIG3_FMA): entries are converted to binary64 and the invariants
// come from the binary64 FMA path above (the paper's algorithms).
//
// Double word (EIG3_DOUBLE_WORD): K2 = 6 J2 and K3 = 27 J3 by Alg.
// alg:J2-stable and alg:J3-stable and Delta = (K2^3 - 2 K3^2) / 54 (the
// double-word evaluation of the binary64 path) with the double word of the
// binary32 data held in one binary64 number: the entries are widened
// exactly, the product of two binary32 numbers is exact in binary64 (it is
// their error-free product hi + lo), and the remaining products and sums
// round at 2^-53, below a binary32 pair's 2^-48.  On gfx950 a binary64 FMA
// issues at the rate of a non-packed binary32 one, so this is the cheapest
// accurate evaluation.
//
// Compensated (EIG3_COMPENSATED): binary32 arithmetic for the invariants:
// K2 and K3 by the same algorithms with binary32 error-free products
// (FMA TwoProduct) and sums (TwoSum) on prescaled deviatoric data, kept as
// unrounded binary32 pairs; binary64 only for the Delta accumulation
// (K2^3 - 2 K3^2 from the widened pairs) and the angle argument.

struct InvW {
    double i1, j2, j3, disc; // binary64 values of the invariants
};

// J2, J3 and Delta depend on the matrix only through the diagonal
// differences d0, d1, d2 and the off-diagonal entries (its deviatoric data).
// The binary32 products below reach the third degree in those (J3 and the
// factors of Delta), so taken as they are they overflow beyond about 2^42 and
// lose accuracy to underflow below about 2^-42.  The data are therefore
// scaled by one exact power of two that brings their largest magnitude into
// [2^31, 2^32): every product then stays below 2^105, products of data down
// to 2^-74 times the largest stay normal, and the invariants scale back
// exactly in binary64 (J2 by 2^2s, J3 by 2^3s, Delta by 2^6s).  Powers of two
// commute with every rounding in between.
// Where the largest magnitude of every matrix of the wave already lies in
// [2^-10, 2^36) the scaling is skipped (s = 0): the products then stay below
// 2^117, and an operation that underflows errs by at most 2^-150, a part in
// 2^120 of the cube of the largest magnitude (2^110 of its square), on
// which the double-word K's are accurate to about 2^-48: they keep their
// accuracy.
struct DevF32 {
    float d0, d1, d2, d1l; // d1 = d0 + d2 exactly as d1 + d1l
    float o[6]; // general: A01 A02 A10 A12 A20 A21; symmetric: S01 S02 S12
    int sc;     // the data are the matrix's times 2^-sc
};

template <int KO> __device__ __forceinline__ DevF32 dev_data_f32(float a00, float a11, float a22, const float *off)
{
    DevF32 v;
    const DiagC<float> g = diag_consistent(a00, a11, a22);
    const float d[3] = {g.d0, g.d1, g.d2};
    float m = fmaxf(fmaxf(fabsf(d[0]), fabsf(d[1])), fabsf(d[2]));
#pragma unroll
    for (int k = 0; k < KO; ++k)
        m = fmaxf(m, fabsf(off[k]));
    const int e = __builtin_amdgcn_frexp_expf(m); // frexp exponent 0 for 0, Inf, NaN
    v.d0 = d[0];
    v.d1 = d[1];
    v.d2 = d[2];
    v.d1l = g.d1l;
#pragma unroll
    for (int k = 0; k < KO; ++k)
        v.o[k] = off[k];
    v.sc = 0;
    if (!__all(e >= -9 && e <= 36)) {
        v.sc = e - 32;
        v.d0 = ldexpf(v.d0, -v.sc);
        v.d1 = ldexpf(v.d1, -v.sc);
        v.d2 = ldexpf(v.d2, -v.sc);
        v.d1l = ldexpf(v.d1l, -v.sc);
#pragma unroll
        for (int k = 0; k < KO; ++k)
            v.o[k] = ldexpf(v.o[k], -v.sc);
    }
    return v;
}

// I1 and K2 = 6 J2, K3 = 27 J3, 54 Delta of the deviatoric data scaled by
// 2^-sc (binary64)
struct KW {
    double i1, k2, k3, d54;
    int sc;
};

__device__ __forceinline__ InvW invariants_of_kw(const KW &k)
{
    InvW r;
    r.i1 = k.i1;
    r.j2 = ldexp(k.k2 * kSixth, 2 * k.sc);
    r.j3 = ldexp(k.k3 * kTwentySeventh, 3 * k.sc);
    r.disc = ldexp(k.d54 * kFiftyFourth, 6 * k.sc);
    return r;
}

// Binary32 pairs (EIG3_COMPENSATED): K2, K3 from the error-free binary32
// evaluation of the binary64 double-word path on the (possibly scaled)
// deviatoric data; the unrounded pairs are widened to binary64 (exactly up
// to 2^-53 relative) and 54 Delta = K2^3 - 2 K3^2 is accumulated in binary64,
// whose rounding (~2^-53 K2^3) stays far below the pairs' own accuracy
// (~2^-48 |terms|).  The scale stays attached (binary32 data keep every
// scaled-back value a normal binary64 number).
__device__ __forceinline__ KW kw_of_f32_pairs(double i1, const KPair<float> &k, int sc)
{
    const double k2 = double(k.k2.hi) + double(k.k2.lo);
    const double k3 = double(k.k3.hi) + double(k.k3.lo);
    KW r;
    r.i1 = i1;
    r.k2 = k2;
    r.k3 = k3;
    r.d54 = fma_(k2 * k2, k2, -2.0 * (k3 * k3));
    r.sc = sc;
    return r;
}

__device__ __forceinline__ KW kw_f32_comp_general(const float a[9])
{
    const float off[6] = {a[1], a[2], a[3], a[5], a[6], a[7]};
    const DevF32 v = dev_data_f32<6>(a[0], a[4], a[8], off);
    const float m[9] = {0.0f, v.o[0], v.o[1], v.o[2], 0.0f, v.o[3], v.o[4], v.o[5], 0.0f};
    const DiagC<float> g{v.d0, v.d1, v.d2, v.d1l};
    return kw_of_f32_pairs(double((a[0] + a[4]) + a[8]), k23_general_dw<float>(m, g), v.sc);
}

__device__ __forceinline__ KW kw_f32_comp_symmetric(const float a[6])
{
    const DevF32 v = dev_data_f32<3>(a[0], a[1], a[2], a + 3);
    const DiagC<float> g{v.d0, v.d1, v.d2, v.d1l};
    return kw_of_f32_pairs(double((a[0] + a[1]) + a[2]), k23_symmetric_dw<float>(v.o[0], v.o[1], v.o[2], g),
                           v.sc);
}

// Binary64 double word of binary32 data (EIG3_DOUBLE_WORD): the widened
// differences d0, d2 are exact for binary32 operands of nearby exponents
// (else rounded once at 2^-53, a backward error) and d1 = d0 + d2 is formed
// from them, as are the t's; the diagonal-pair products p, q, r of two
// binary32 numbers are exact; the triple products and the sums round once
// each at 2^-53.  off3 = A01 A12 A20 + A02 A10 A21.
__device__ __forceinline__ KW kw_k64(double x00, double x11, double x22, double p, double q, double r, double off3)
{
    const double d0 = x00 - x11, d2 = x11 - x22, d1 = d0 + d2;
    const double k2 = fma_(d0, d0, fma_(d1, d1, fma_(d2, d2, 6.0 * ((p + q) + r))));
    const double t1 = d1 + d2, t2 = d0 - d2, t3 = -d0 - d1;
    const double k3 = fma_(27.0, off3, fma_(9.0, fma_(p, t1, fma_(q, t2, r * t3)), -(t1 * t2) * t3));
    KW v;
    v.i1 = (x00 + x11) + x22;
    v.k2 = k2;
    v.k3 = k3;
    v.d54 = fma_(k2 * k2, k2, -2.0 * (k3 * k3));
    v.sc = 0;
    return v;
}

__device__ __forceinline__ KW kw_f32_dw_general(const float a[9])
{
    double x[9];
#pragma unroll
    for (int k = 0; k < 9; ++k)
        x[k] = a[k];
    return kw_k64(x[0], x[4], x[8], x[1] * x[3], x[2] * x[6], x[5] * x[7], fma_(x[1] * x[5], x[6], x[2] * x[3] * x[7]));
}

__device__ __forceinline__ KW kw_f32_dw_symmetric(const float a[6])
{
    double x[6];
#pragma unroll
    for (int k = 0; k < 6; ++k)
        x[k] = a[k];
    return kw_k64(x[0], x[1], x[2], x[3] * x[3], x[4] * x[4], x[5] * x[5], 2.0 * (x[3] * x[4] * x[5]));
}

// The binary64 arguments of the binary32 eigenvalue tail: I1, J2 / 3,
// 27 Delta and 27 J3 (the operands of Eq. triple-angle-arctan and of the
// radius in Eq. eigvals-trig), the last three those of the deviatoric data
// scaled by 2^-sc: the angle depends only on the ratio of sqrt(27 Delta) and
// 27 |J3|, which scale alike (by 2^3sc), so only the radius is scaled back.
struct TrigArgW {
    double i1, j2_3, disc27, j3_27;
    int sc;
};

__device__ __forceinline__ TrigArgW trig_args_of_invariants(const InvW &v)
{
    return TrigArgW{v.i1, v.j2 * kThird, 27.0 * v.disc, 27.0 * v.j3, 0};
}

// from K2, K3 and 54 Delta: J2 / 3 = K2 / 18 in one rounding, 27 Delta =
// 54 Delta / 2 and 27 J3 = K3 exactly
__device__ __forceinline__ TrigArgW trig_args_of_kw(const KW &k)
{
    constexpr double kEighteenth = 1.0 / 18.0;
    return TrigArgW{k.i1, k.k2 * kEighteenth, 0.5 * k.d54, k.k3, k.sc};
}

// Eigenvalues in binary32 from the binary64 arguments.
__device__ __forceinline__ void eigvals_f32_from_args(const TrigArgW &v, float &l1, float &l2, float &l3)
{
    // The square roots sqrt(27 Delta) and r = sqrt(J2 / 3) are taken by the
    // hardware binary64 square root, an approximation with relative error
    // below 2^-25 over the whole binary64 range (measured on gfx950; a binary32
    // result needs 2^-24), so no range reduction is needed.  The angle pair
    // (sqrt(27 Delta), 27 |J3|) is then scaled by one exact power of two that
    // puts its larger member in [1/2, 1) before it is rounded to binary32 (a
    // smaller member that underflows there only means an angle below 2^-126).
    // (NaN in J2 or Delta comes only from NaN or Inf entries, which make J3
    // NaN too; the J3 test below carries it to the output, so plain max
    // clamps suffice here)
    const double y = __builtin_amdgcn_sqrt(fmax(v.disc27, 0.0));
    const double x = fabs(v.j3_27);
    const int e = __builtin_amdgcn_frexp_exp(fmax(x, y));
    const float yf = float(ldexp(y, -e));
    const float xf = float(ldexp(x, -e));
    float psi = atan2_nonneg<false>(yf, xf);
    psi = v.j3_27 == v.j3_27 ? psi : float(v.j3_27); // NaN in J3 reaches the eigenvalues
    float s, c;
    sincos_sixth<false>(psi * (1.0f / 3.0f), s, c);
    const float r = float(ldexp(__builtin_amdgcn_sqrt(fmax(v.j2_3, 0.0)), v.sc));
    const float mean = float(v.i1 * kThird);
    const float a1 = -r * fma_(float(kSqrt3), s, c);
    const float a2 = r * fma_(float(kSqrt3), s, -c);
    const float a3 = 2.0f * r * c;
    const bool neg = v.j3_27 < 0.0;
    l1 = mean + (neg ? -a3 : a1);
    l2 = mean + (neg ? -a2 : a2);
    l3 = mean + (neg ? -a1 : a3);
}

// ============================================================== backward
// d(lambda_k)/dA = I/3 + (mu_k S^T + dev(cof S)) / ((lambda_k - lambda_i)(lambda_k - lambda_j)),
// S = dev A.  Implicit differentiation of mu_k^3 - J2 mu_k - J3 = 0 gives
// d mu_k = (mu_k dJ2 + dJ3) / (3 mu_k^2 - J2), 3 mu_k^2 - J2 = prod_{j != k}(mu_k - mu_j),
// with dJ2 = <S^T, dA> (Lemma lem:J2-condition) and dJ3 = <dev cof S, dA>
// (Lemma lem:J3-jacobian).  The vector-Jacobian product is
//   grad = (g1 + g2 + g3)/3 I + a S^T + b dev(cof S),
//   a = sum_k g_k mu_k / G_k, b = sum_k g_k / G_k, G_k the gap products.
struct Coef {
    double gsum3; // (g1 + g2 + g3) / 3
    double a, b;
};

__device__ __forceinline__ Coef backward_coefficients(const Trig &t, double g1, double g2, double g3)
{
    double m1, m2, m3;
    mu_from_trig(t, m1, m2, m3);
    const Gaps gp = gaps_from_trig(t);
    const double e12 = gp.e12, e13 = gp.e13, e23 = gp.e23;
    const double G1 = e12 * e13;   // (mu1 - mu2)(mu1 - mu3)
    const double G2 = -e12 * e23;  // (mu2 - mu1)(mu2 - mu3)
    const double G3 = e13 * e23;   // (mu3 - mu1)(mu3 - mu2)
    // a zero weight contributes nothing, also where its gap product vanishes
    const double q1 = g1 == 0.0 ? 0.0 : g1 / G1;
    const double q2 = g2 == 0.0 ? 0.0 : g2 / G2;
    const double q3 = g3 == 0.0 ? 0.0 : g3 / G3;
    Coef c;
    c.gsum3 = (g1 + g2 + g3) * kThird;
    c.b = q1 + q2 + q3;
    c.a = fma_(q1, m1, fma_(q2, m2, q3 * m3));
    return c;
}

__device__ __forceinline__ Coef backward_coefficients(const Inv &v, double g1, double g2, double g3)
{
    return backward_coefficients(trig_from_invariants<false>(v), g1, g2, g3);
}

// grad (row-major 9) for a general matrix
__device__ __forceinline__ void backward_general(const Gen &A, const Coef &k, double grad[9])
{
    const Diag g = diag_part(A.a00, A.a11, A.a22);
    // S = dev A from the differences (no rounding of I1/3 enters)
    const double s00 = (g.d0 + g.d1) * kThird, s11 = (g.d2 - g.d0) * kThird, s22 = -(g.d1 + g.d2) * kThird;
    const double s01 = A.a01, s02 = A.a02, s10 = A.a10, s12 = A.a12, s20 = A.a20, s21 = A.a21;
    // cofactor matrix of S
    double c00 = fma_(s11, s22, -s12 * s21);
    double c01 = fma_(s12, s20, -s10 * s22);
    double c02 = fma_(s10, s21, -s11 * s20);
    double c10 = fma_(s02, s21, -s01 * s22);
    double c11 = fma_(s00, s22, -s02 * s20);
    double c12 = fma_(s01, s20, -s00 * s21);
    double c20 = fma_(s01, s12, -s02 * s11);
    double c21 = fma_(s02, s10, -s00 * s12);
    double c22 = fma_(s00, s11, -s01 * s10);
    const double tr3 = ((c00 + c11) + c22) * kThird;
    c00 -= tr3;
    c11 -= tr3;
    c22 -= tr3;
    grad[0] = fma_(k.a, s00, fma_(k.b, c00, k.gsum3));
    grad[1] = fma_(k.a, s10, k.b * c01);
    grad[2] = fma_(k.a, s20, k.b * c02);
    grad[3] = fma_(k.a, s01, k.b * c10);
    grad[4] = fma_(k.a, s11, fma_(k.b, c11, k.gsum3));
    grad[5] = fma_(k.a, s21, k.b * c12);
    grad[6] = fma_(k.a, s02, k.b * c20);
    grad[7] = fma_(k.a, s12, k.b * c21);
    grad[8] = fma_(k.a, s22, fma_(k.b, c22, k.gsum3));
}

// ============================================================ Mohr-Coulomb
// Yield function of the paper's application section:
//   f(sigma) = (1/S_yc) ((m + 1)/2) max_{i<j} (|s_i - s_j| + K (s_i + s_j)) - 1,
//   K = (m - 1)/(m + 1), s_1 <= s_2 <= s_3 the principal stresses.
// With ascending s, |s_i - s_j| = s_j - s_i for i < j, and for |K| < 1 the
// pair (1, 3) attains the maximum, so df/dsigma = cf ((1 + K) E_3 - (1 - K) E_1)
// with cf = (m + 1)/(2 S_yc) and E_k = d(s_k)/dsigma: the adjoint with
// g = (cf (K - 1), 0, cf (1 + K)).  At s_1 = s_2 or s_2 = s_3 (the corners of
// the yield surface) f is not differentiable and the gradient is +-Inf/NaN.
struct MohrCoulomb {
    double f;
    double g1, g3; // weights of d(s_1)/dsigma and d(s_3)/dsigma
    Trig t;        // the triple-angle quantities, reused by the gradient
};

// (v may be the invariants of sigma 2^-e: the stresses scale back by 2^e)
template <bool Table = true>
__device__ __forceinline__ MohrCoulomb mohr_coulomb(const Inv &v, double cf, double K, int e = 0)
{
    const Trig t = trig_from_invariants<Table>(v);
    double m1, m2, m3;
    mu_from_trig(t, m1, m2, m3);
    const double s1 = t.mean + m1, s2 = t.mean + m2, s3 = t.mean + m3;
    const double p12 = (s2 - s1) + K * (s1 + s2);
    const double p13 = (s3 - s1) + K * (s1 + s3);
    const double p23 = (s3 - s2) + K * (s2 + s3);
    const double pm = ldexp(fmax(fmax(p12, p13), p23), e);
    MohrCoulomb r;
    r.f = fma_(cf, pm, -1.0);
    r.g1 = cf * (K - 1.0);
    r.g3 = cf * (1.0 + K);
    r.t = t;
    return r;
}

// ============================================================ eigenprojectors
// E_k = prod_{j != k} (A - lambda_j I) / (lambda_k - lambda_j), the projector
// onto the k-th eigenspace; the paper relates it to the eigenvalue
// derivative, E_k^T = d(lambda_k)/dA (Sec. "Introduction and motivation").
// Through the invariants (as for the adjoint), with S = dev A:
//   E_k^T = I/3 + (mu_k S^T + dev(cof S)) / G_k,  G_k = prod_{j != k}(mu_k - mu_j),
// so E_k = I/3 + (mu_k S + dev(cof S)^T) / G_k.  Row-major 9 entries per k.
__device__ __forceinline__ void eigenprojectors_general(const Gen &A, const Trig &t, double E[27])
{
    double m1, m2, m3;
    mu_from_trig(t, m1, m2, m3);
    const Gaps gp = gaps_from_trig(t);
    const double e12 = gp.e12, e13 = gp.e13, e23 = gp.e23;
    const double inv[3] = {1.0 / (e12 * e13), -1.0 / (e12 * e23), 1.0 / (e13 * e23)};
    const double mu[3] = {m1, m2, m3};
    const Diag g = diag_part(A.a00, A.a11, A.a22);
    const double S[9] = {(g.d0 + g.d1) * kThird, A.a01, A.a02, A.a10, (g.d2 - g.d0) * kThird, A.a12,
                         A.a20, A.a21, -(g.d1 + g.d2) * kThird};
    // cofactor matrix of S, made deviatoric
    double C[9] = {fma_(S[4], S[8], -S[5] * S[7]), fma_(S[5], S[6], -S[3] * S[8]), fma_(S[3], S[7], -S[4] * S[6]),
                   fma_(S[2], S[7], -S[1] * S[8]), fma_(S[0], S[8], -S[2] * S[6]), fma_(S[1], S[6], -S[0] * S[7]),
                   fma_(S[1], S[5], -S[2] * S[4]), fma_(S[2], S[3], -S[0] * S[5]), fma_(S[0], S[4], -S[1] * S[3])};
    const double tr3 = ((C[0] + C[4]) + C[8]) * kThird;
    C[0] -= tr3;
    C[4] -= tr3;
    C[8] -= tr3;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double a = mu[k] * inv[k], b = inv[k];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                E[9 * k + 3 * r + c] = fma_(a, S[3 * r + c], fma_(b, C[3 * c + r], r == c ? kThird : 0.0));
    }
}

// ============================================================ functions of A
// f(A) = sum_k f(lambda_k) E_k, E_k = I/3 + (mu_k S + dev(cof S)^T) / G_k:
// the transpose of the adjoint above with g_k = f(lambda_k).
template <int Fn> __device__ __forceinline__ double scalar_function(double x)
{
    if constexpr (Fn == EIG3_EXP)
        return exp(x);
    else if constexpr (Fn == EIG3_LOG)
        return log(x);
    else
        return sqrt(x);
}

// Divided difference f[x, y] = (f(x) - f(y)) / (x - y) from y, f(y) and the
// gap d = x - y >= 0 (computed without cancellation), f'(y) at d = 0.
template <int Fn> __device__ __forceinline__ double divided_difference(double y, double fx, double fy, double d)
{
    if constexpr (Fn == EIG3_EXP)
        return d == 0.0 ? fy : fy * (expm1(d) / d);
    else if constexpr (Fn == EIG3_LOG)
        return d == 0.0 ? 1.0 / y : log1p(d / y) / d;
    else
        return 1.0 / (fx + fy);
}

// f at three ascending nodes y0 <= y1 <= y2, given with their gaps g01 = y1 - y0
// and g12 = y2 - y1 (>= 0, free of cancellation), and the three first divided
// differences.  For exp and log the later values follow from the first and
// the increments the divided differences need anyway: e^y1 = e^y0 (1 +
// expm1(g01)), log y1 = log y0 + log1p(g01 / y0), and over the whole spread
// expm1(g01 + g12) = a + b + a b, log1p = a + b (sums of nonnegative terms),
// so one exp or log and two expm1 or log1p serve all six values.
struct Chain {
    double f0, f1, f2;    // f(y0), f(y1), f(y2)
    double d01, d12, d02; // f[y0, y1], f[y1, y2], f[y0, y2]
};
template <int Fn> __device__ __forceinline__ Chain node_chain(double y0, double y1, double y2, double g01, double g12)
{
    Chain c;
    const double g02 = g01 + g12;
    if constexpr (Fn == EIG3_EXP) {
        const double a = expm1(g01), b = expm1(g12);
        c.f0 = exp(y0);
        c.f1 = fma_(c.f0, a, c.f0);
        c.f2 = fma_(c.f1, b, c.f1);
        c.d01 = g01 == 0.0 ? c.f0 : c.f0 * (a / g01);
        c.d12 = g12 == 0.0 ? c.f1 : c.f1 * (b / g12);
        c.d02 = g02 == 0.0 ? c.f0 : c.f0 * (fma_(a, b, a + b) / g02);
    } else if constexpr (Fn == EIG3_LOG) {
        const double a = log1p(g01 / y0), b = log1p(g12 / y1);
        c.f0 = log(y0);
        c.f1 = c.f0 + a;
        c.f2 = c.f1 + b;
        c.d01 = g01 == 0.0 ? 1.0 / y0 : a / g01;
        c.d12 = g12 == 0.0 ? 1.0 / y1 : b / g12;
        c.d02 = g02 == 0.0 ? 1.0 / y0 : (a + b) / g02;
    } else {
        c.f0 = sqrt(y0);
        c.f1 = sqrt(y1);
        c.f2 = sqrt(y2);
        c.d01 = 1.0 / (c.f0 + c.f1);
        c.d12 = 1.0 / (c.f1 + c.f2);
        c.d02 = 1.0 / (c.f0 + c.f2);
    }
    return c;
}

// f''(y) / 2 from y and fy = f(y)
template <int Fn> __device__ __forceinline__ double half_second_derivative(double y, double fy)
{
    if constexpr (Fn == EIG3_EXP)
        return 0.5 * fy;
    else if constexpr (Fn == EIG3_LOG)
        return -0.5 / (y * y);
    else
        return -0.125 / (y * fy);
}

// f(A) = sum_k f(lambda_k) E_k is the polynomial interpolating f at the three
// eigenvalues, evaluated at A; in Newton form
//   f(A) = f(lambda1) I + f[lambda1, lambda2] P1 + f[lambda1, lambda2, lambda3] P1 P2,
//   P_k = A - lambda_k I = S - mu_k I,
// it stays accurate as eigenvalues coalesce (the E_k themselves diverge like
// 1/gap): the first divided differences come from the gaps without
// cancellation, and the rounding error of the second, which grows like
// 1/(lambda3 - lambda1), multiplies P1 P2, which shrinks like the square of
// the spread.  With exactly repeated eigenvalues the divided differences take
// their confluent limits (f', f''/2): the Hermite interpolant, which is f(A)
// also for a defective A.
template <int Fn> __device__ __forceinline__ void matrix_function_general(const Gen &A, const Trig &t, double F[9])
{
    double m1, m2, m3;
    mu_from_trig(t, m1, m2, m3);
    const double l1 = t.mean + m1, l2 = t.mean + m2;
    const Gaps gp = gaps_from_trig(t);
    const Chain ch = node_chain<Fn>(l1, l2, t.mean + m3, gp.e12, gp.e23);
    const double f1 = ch.f0, d12 = ch.d01, d23 = ch.d12;
    // all three equal: the confluent limit f''(lambda) / 2 (P1 P2 is the square
    // of the nilpotent part, zero unless A is a single Jordan block)
    const double d123 = gp.e13 == 0.0 ? half_second_derivative<Fn>(l1, f1) : (d23 - d12) / gp.e13;
    const Diag g = diag_part(A.a00, A.a11, A.a22);
    // P1 = S - mu1 I, P2 = S - mu2 I with S = dev A from the differences
    const double s00 = (g.d0 + g.d1) * kThird, s11 = (g.d2 - g.d0) * kThird, s22 = -(g.d1 + g.d2) * kThird;
    const double P1[9] = {s00 - m1, A.a01, A.a02, A.a10, s11 - m1, A.a12, A.a20, A.a21, s22 - m1};
    const double P2[9] = {s00 - m2, A.a01, A.a02, A.a10, s11 - m2, A.a12, A.a20, A.a21, s22 - m2};
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double pp = fma_(P1[3 * r], P2[c], fma_(P1[3 * r + 1], P2[3 + c], P1[3 * r + 2] * P2[6 + c]));
            F[3 * r + c] = fma_(d123, pp, fma_(d12, P1[3 * r + c], r == c ? f1 : 0.0));
        }
}


// C = A B for 3x3 row-major matrices
__device__ __forceinline__ void matmul3(const double A[9], const double B[9], double C[9])
{
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            C[3 * r + c] = fma_(A[3 * r], B[c], fma_(A[3 * r + 1], B[3 + c], A[3 * r + 2] * B[6 + c]));
}

// f^(k)(x) / k! for k = 1..5, given fx = f(x)
template <int Fn> __device__ __forceinline__ double taylor_coefficient(int k, double x, double fx)
{
    if constexpr (Fn == EIG3_EXP) {
        constexpr double inv_fact[6] = {1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0};
        return fx * inv_fact[k];
    } else if constexpr (Fn == EIG3_LOG) {
        // (-1)^(k+1) / (k x^k)
        const double r = 1.0 / x;
        double p = r;
        for (int j = 1; j < k; ++j)
            p *= -r;
        return p / double(k);
    } else {
        // binomial(1/2, k) x^(1/2 - k)
        constexpr double binom[6] = {1.0, 0.5, -0.125, 0.0625, -0.0390625, 0.02734375};
        const double r = 1.0 / x;
        double p = fx;
        for (int j = 0; j < k; ++j)
            p *= r;
        return binom[k] * p;
    }
}

// The vector-Jacobian product of f(A), grad = d<G, f(A)>/dA = L_f(A^T)[G],
// the Frechet derivative of f at A^T applied to G (for f with real Taylor
// coefficients).  With X = A^T and the eigenvalues as nodes in the order
// z0 = lambda_min, z1 = lambda_max, z2 = lambda_mid, the Daleckii-Krein sum
// sum_{k,l} f[lambda_k, lambda_l] E_k G E_l is the bivariate interpolant of
// f[x, y] in tensor Newton form,
//   grad = sum_{p,q <= 2} f[z0..zp, z0..zq] N_p G N_q,
//   N_0 = I, N_1 = X - z0 I, N_2 = (X - z0 I)(X - z1 I),
// whose coefficients are divided differences of f over the merged node lists
// (each eigenvalue at most twice).  They are formed by the recursion that
// divides by the largest gap z1 - z0 wherever both ends are present; the
// divisions by the smaller gaps (z2 - z0, z1 - z2) enter only coefficients
// of N_2, which shrinks with those gaps, so the result stays accurate as
// eigenvalues coalesce.  A gap below 2^-26 of the spread is treated as zero
// (the confluent value f^(k)/k! at the end node: an error of second order in
// the gap after the factor N_2), as is a zero spread.  N_1 and N_2 come from
// the deviatoric part of X (diagonal differences), so the isotropic part
// cancels exactly.  G and grad are 3x3 row-major.
template <int Fn>
__device__ __forceinline__ void matrix_function_backward_general(const Gen &A, const Trig &t, const double G[9],
                                                                 double grad[9])
{
    double m1, m2, m3;
    mu_from_trig(t, m1, m2, m3);
    const Gaps gp = gaps_from_trig(t);
    const double z0 = t.mean + m1, z1 = t.mean + m3, z2 = t.mean + m2;
    const Chain ch = node_chain<Fn>(z0, z2, z1, gp.e12, gp.e23); // ascending: z0, z2, z1
    const double f0 = ch.f0, f1 = ch.f2, f2 = ch.f1;
    const double spread = gp.e13;
    const bool iso = spread == 0.0;
    constexpr double kTau = 0x1p-26;
    const bool low = gp.e12 <= kTau * spread;  // z2 merges with z0
    const bool high = gp.e23 <= kTau * spread; // z2 merges with z1
    // first order (cancellation-free formulas, exact zero gaps included)
    const double d01 = ch.d02; // f[z0, z1]
    const double d02 = ch.d01; // f[z0, z2]
    const double d12 = ch.d12; // f[z2, z1]
    const double c00 = taylor_coefficient<Fn>(1, z0, f0);              // f[z0, z0]
    const double c11 = taylor_coefficient<Fn>(1, z1, f1);              // f[z1, z1]
    const double c22 = taylor_coefficient<Fn>(1, z2, f2);              // f[z2, z2]
    // D(m0, m1, m2): divided difference with z0, z1, z2 taken m0, m1, m2 times
    auto ruleA = [&](double without_z0, double without_z1, int order) {
        return iso ? taylor_coefficient<Fn>(order, z0, f0) : (without_z0 - without_z1) / spread;
    };
    auto ruleB = [&](double without_z0, double without_z2, int order) {
        return low ? taylor_coefficient<Fn>(order, z0, f0) : (without_z0 - without_z2) / gp.e12;
    };
    auto ruleC = [&](double without_z1, double without_z2, int order) {
        return high ? taylor_coefficient<Fn>(order, z1, f1) : (without_z1 - without_z2) / (-gp.e23);
    };
    const double D210 = ruleA(d01, c00, 2);
    const double D120 = ruleA(c11, d01, 2);
    const double D220 = ruleA(D120, D210, 3);
    const double D111 = ruleA(d12, d02, 2);
    const double D201 = ruleB(d02, c00, 2);
    const double D211 = ruleA(D111, D201, 3);
    const double D021 = ruleC(d12, c11, 2);
    const double D121 = ruleA(D021, D111, 3);
    const double D221 = ruleA(D121, D211, 4);
    const double D012 = ruleC(c22, d12, 2);
    const double D102 = ruleB(c22, d02, 2);
    const double D022 = ruleC(D012, D021, 3);
    const double D112 = ruleA(D012, D102, 3);
    const double D202 = ruleB(D102, D201, 3);
    const double D122 = ruleA(D022, D112, 4);
    const double D212 = ruleA(D112, D202, 4);
    const double D222 = ruleA(D122, D212, 5);
    const double F00 = c00, F10 = D210, F11 = D220, F20 = D211, F21 = D221, F22 = D222;
    // N1 = X - z0 I and X - z1 I from the deviatoric part of X = A^T
    const Diag g = diag_part(A.a00, A.a11, A.a22);
    const double s00 = (g.d0 + g.d1) * kThird, s11 = (g.d2 - g.d0) * kThird, s22 = -(g.d1 + g.d2) * kThird;
    const double N1[9] = {s00 - m1, A.a10, A.a20, A.a01, s11 - m1, A.a21, A.a02, A.a12, s22 - m1};
    const double M3[9] = {s00 - m3, A.a10, A.a20, A.a01, s11 - m3, A.a21, A.a02, A.a12, s22 - m3};
    // N1 and M3 are polynomials in X and commute, so N2 = N1 M3 = M3 N1 is
    // never formed: N2 G = M3 (N1 G) and W1 N1 + W2 N2 = (W1 + W2 M3) N1
    double U1[9], U2[9];
    matmul3(N1, G, U1);
    matmul3(M3, U1, U2);
    double V[9], W1[9], W2[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        V[e] = fma_(F00, G[e], fma_(F10, U1[e], F20 * U2[e]));
        W1[e] = fma_(F10, G[e], fma_(F11, U1[e], F21 * U2[e]));
        W2[e] = fma_(F20, G[e], fma_(F21, U1[e], F22 * U2[e]));
    }
    // T = W1 + W2 M3, grad = V + T N1
    double T[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double acc = W1[3 * r + c];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                acc = fma_(W2[3 * r + k], M3[3 * k + c], acc);
            T[3 * r + c] = acc;
        }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double acc = V[3 * r + c];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                acc = fma_(T[3 * r + k], N1[3 * k + c], acc);
            grad[3 * r + c] = acc;
        }
}

} // namespace eig3
