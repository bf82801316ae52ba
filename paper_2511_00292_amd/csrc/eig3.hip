// eig3.hip -- kernels and C ABI of libeig3 (see include/eig3.h).
//
// Execution model: one 3x3 matrix per lane, wave64, 256-lane workgroups; the
// grid strides over spans of 256 consecutive matrices (one launch normally
// covers the batch with one span per workgroup).  Structure-of-arrays inputs
// are read with one coalesced buffer load per entry and lane (a scalar buffer
// resource per array over the span, 32-bit lane offsets); array-of-structures
// inputs are staged through LDS by the workgroup with 16-byte loads and then
// read back one matrix per lane.  Nothing here is a dense contraction, so
// there is no MFMA: the kernels are HBM-bandwidth bound with a binary64 VALU
// budget (MI355X runs binary64 FMA at the binary32 non-packed rate).
#include "eig3.h"
#include "eig3_math.hpp"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

namespace {

using namespace eig3;

constexpr int kBlock = 256;
constexpr int64_t kMaxBlocks = int64_t(1) << 20;

#define EIG3_KERNEL __global__ __launch_bounds__(kBlock)

// Streaming accesses: every input is read once and every output written once,
// so loads and stores carry the nontemporal hint (measured 5-10% faster than
// without on the binary64 patterns).
template <class T> __device__ __forceinline__ T ld(const T *p)
{
    return __builtin_nontemporal_load(p);
}

template <class T> __device__ __forceinline__ void st(T v, T *p)
{
    __builtin_nontemporal_store(v, p);
}

// The workgroup's span of matrices [first, first + cnt) and this lane's place
// in it.  Per-array accesses go through a buffer resource whose base is the
// span's first row (wave-uniform, held in scalar registers) and whose size is
// the span: a lane adds only a 32-bit offset, and the hardware range check
// keeps every access inside the span (reads beyond it return 0 and writes
// beyond it are dropped; the drivers below do not issue them anyway).
struct Span {
    int64_t first;
    int cnt; // 1 .. kBlock
    int lane;
    __device__ bool live() const { return lane < cnt; }
};

__device__ __forceinline__ Span span_at(int64_t first, int64_t n)
{
    const int64_t rem = n - first;
    return Span{first, rem < kBlock ? int(rem) : kBlock, int(threadIdx.x)};
}

// raw buffer, 32-bit data format: the gfx9-family descriptor word 3
constexpr int kBufferWord3 = 0x00020000;
// cache-policy operand: the nontemporal bit of gfx940-family memory operations
constexpr int kBufferAux = 2;

// rows of `per` values: the span's rows of array p
template <class T> __device__ __forceinline__ __amdgpu_buffer_rsrc_t span_rsrc(const T *p, const Span &s, int per)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(p) + int64_t(per) * s.first, 0,
                                             s.cnt * per * int(sizeof(T)), kBufferWord3);
}

using u32x2 = unsigned __attribute__((ext_vector_type(2)));

// value c of the lane's row of `per` values
template <class T> __device__ __forceinline__ T span_ld(const T *p, const Span &s, int per = 1, int c = 0)
{
    const __amdgpu_buffer_rsrc_t r = span_rsrc(p, s, per);
    const int off = (s.lane * per + c) * int(sizeof(T));
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kBufferAux));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kBufferAux));
}

template <class T> __device__ __forceinline__ void span_st(T v, T *p, const Span &s, int per = 1, int c = 0)
{
    const __amdgpu_buffer_rsrc_t r = span_rsrc(p, s, per);
    const int off = (s.lane * per + c) * int(sizeof(T));
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, kBufferAux);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, kBufferAux);
}

template <class T> struct In9 {
    const T *p[9];
};
// KO output slots per matrix: one array per slot (structure of arrays,
// p[e] + i) or one array of KO values per matrix (array of structures, p[0])
template <class T, int KO> struct OutK {
    T *p[KO];
};
template <class T> struct G3 {
    const T *p[3];
};

// ------------------------------------------------------------------ loads
// AoS staging: the workgroup copies its contiguous span of kBlock matrices
// (kBlock*K elements) into LDS with 16-byte loads, then each lane reads its K
// entries.  K = 9 (general) or 6 (symmetric).  binary64 rows of even length
// are padded by one value so that the per-lane 8-byte reads spread over the
// banks; binary32 rows stay unpadded, which lets the staging loop store its
// 16-byte vectors whole.
template <class T, int K> constexpr int aos_stride() { return (sizeof(T) == 8 && K % 2 == 0) ? K + 1 : K; }

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <class T> struct Vec16;
template <> struct Vec16<double> {
    using type = f64x2;
    static constexpr int N = 2;
};
template <> struct Vec16<float> {
    using type = f32x4;
    static constexpr int N = 4;
};

template <class T, int K>
__device__ __forceinline__ void aos_stage(const T *__restrict__ base, int64_t first, int64_t n, T *tile)
{
    // elements [first*K, min(n, first+kBlock)*K) of base; the span starts at
    // a multiple of kBlock*K elements, so its 16-byte alignment is that of
    // base and the branch below is uniform over the grid
    const int64_t m_end = (first + kBlock < n) ? first + kBlock : n;
    const int count = int((m_end - first) * K);
    const T *src = base + first * K;
    constexpr int kS = aos_stride<T, K>();
    int done = 0;
    if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {
        using V = typename Vec16<T>::type;
        constexpr int NV = Vec16<T>::N;
        // a full span is kBlock*K/NV vectors: at most kPer per lane, all
        // loads issued before the first LDS write (one memory round trip)
        constexpr int kPer = (kBlock * K / NV + kBlock - 1) / kBlock;
        const int nvec = count / NV;
        const V *vsrc = reinterpret_cast<const V *>(src);
        if (nvec > 0) {
            // branch-free loads: a lane past the end reloads the last vector
            V x[kPer];
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                const int v = int(threadIdx.x) + r * kBlock;
                x[r] = ld(vsrc + (v < nvec ? v : nvec - 1));
            }
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                const int v = int(threadIdx.x) + r * kBlock;
                if (v < nvec) {
                    if constexpr (kS == K) {
                        // unpadded rows: the tile is the span itself
                        reinterpret_cast<V *>(tile)[v] = x[r];
                    } else {
#pragma unroll
                        for (int j = 0; j < NV; ++j) {
                            const int e = v * NV + j, m = e / K, k = e - m * K;
                            tile[m * kS + k] = x[r][j];
                        }
                    }
                }
            }
        }
        done = nvec * NV;
    }
    for (int e = done + threadIdx.x; e < count; e += kBlock) {
        const int m = e / K, k = e - m * K;
        tile[m * kS + k] = ld(src + e);
    }
}

// The reverse for outputs: the workgroup's staged rows (KO values per matrix,
// contiguous in LDS) are written to the contiguous output span with 16-byte
// stores where the span is 16-byte aligned.
template <class T, int KO>
__device__ __forceinline__ void aos_flush(T *__restrict__ base, int64_t first, int64_t n, const T *tile)
{
    const int64_t m_end = (first + kBlock < n) ? first + kBlock : n;
    const int count = int((m_end - first) * KO);
    T *dst = base + first * KO;
    int done = 0;
    if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
        using V = typename Vec16<T>::type;
        constexpr int NV = Vec16<T>::N;
        const int nvec = count / NV;
        V *vdst = reinterpret_cast<V *>(dst);
        const V *vtile = reinterpret_cast<const V *>(tile);
        constexpr int kPer = (kBlock * KO / NV + kBlock - 1) / kBlock;
        if (nvec > 0) {
            V x[kPer];
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                const int v = int(threadIdx.x) + r * kBlock;
                x[r] = vtile[v < nvec ? v : nvec - 1];
            }
#pragma unroll
            for (int r = 0; r < kPer; ++r) {
                const int v = int(threadIdx.x) + r * kBlock;
                if (v < nvec)
                    st(x[r], vdst + v);
            }
        }
        done = nvec * NV;
    }
    for (int e = done + threadIdx.x; e < count; e += kBlock)
        st(tile[e], dst + e);
}

template <class T, int S> struct Mat;
template <class T> struct Mat<T, EIG3_GENERAL> {
    static constexpr int K = 9;
    T a[9];
};
template <class T> struct Mat<T, EIG3_SYMMETRIC> {
    static constexpr int K = 6;
    T a[6];
};

template <class T, int S>
__device__ __forceinline__ void load_soa(const In9<T> &in, const Span &sp, Mat<T, S> &m)
{
#pragma unroll
    for (int k = 0; k < Mat<T, S>::K; ++k)
        m.a[k] = span_ld(in.p[k], sp);
}

__device__ __forceinline__ Gen to_gen(const Mat<double, EIG3_GENERAL> &m)
{
    return Gen{m.a[0], m.a[1], m.a[2], m.a[3], m.a[4], m.a[5], m.a[6], m.a[7], m.a[8]};
}
__device__ __forceinline__ Sym to_sym(const Mat<double, EIG3_SYMMETRIC> &m)
{
    return Sym{m.a[0], m.a[1], m.a[2], m.a[3], m.a[4], m.a[5]};
}

template <int S, int Acc> __device__ __forceinline__ Inv invariants_of(const Mat<double, S> &m)
{
    if constexpr (Acc == EIG3_NAIVE || Acc == EIG3_NAIVE_TENSOR) {
        Gen g;
        if constexpr (S == EIG3_GENERAL) {
            g = to_gen(m);
        } else {
            const Sym y = to_sym(m);
            g = Gen{y.s00, y.s01, y.s02, y.s01, y.s11, y.s12, y.s02, y.s12, y.s22};
        }
        if constexpr (Acc == EIG3_NAIVE)
            return invariants_general_naive(g);
        else
            return invariants_general_tensor(g);
    } else if constexpr (S == EIG3_GENERAL) {
        if constexpr (Acc == EIG3_COMPENSATED)
            return invariants_general_comp(to_gen(m));
        else if constexpr (Acc == EIG3_DOUBLE_WORD)
            return invariants_general_dw(to_gen(m));
        else
            return invariants_general_fma(to_gen(m));
    } else {
        if constexpr (Acc == EIG3_COMPENSATED)
            return invariants_symmetric_comp(to_sym(m));
        else if constexpr (Acc == EIG3_DOUBLE_WORD)
            return invariants_symmetric_dw(to_sym(m));
        else
            return invariants_symmetric_fma(to_sym(m));
    }
}

// The triple-angle quantities of m: through K2, K3 and 54 Delta directly in
// the double-word evaluation, else through the invariants.
template <int S, int Acc, bool Table>
__device__ __forceinline__ Trig trig_of_matrix(const Mat<double, S> &m)
{
    if constexpr (Acc == EIG3_DOUBLE_WORD) {
        if constexpr (S == EIG3_GENERAL) {
            const Gen A = to_gen(m);
            const double e[9] = {A.a00, A.a01, A.a02, A.a10, A.a11, A.a12, A.a20, A.a21, A.a22};
            return trig_from_k<Table>(diag_part(A.a00, A.a11, A.a22).i1,
                                      k23_general_dw(e, diag_consistent(A.a00, A.a11, A.a22)));
        } else {
            const Sym y = to_sym(m);
            return trig_from_k<Table>(diag_part(y.s00, y.s11, y.s22).i1,
                                      k23_symmetric_dw(y.s01, y.s02, y.s12, diag_consistent(y.s00, y.s11, y.s22)));
        }
    } else {
        return trig_from_invariants<Table>(invariants_of<S, Acc>(m));
    }
}

template <class T, int KO>
__device__ __forceinline__ void store_rows(const OutK<T, KO> &out, int layout, const Span &sp, const double (&o)[KO])
{
    if (layout == EIG3_SOA) {
#pragma unroll
        for (int e = 0; e < KO; ++e)
            span_st(T(o[e]), out.p[e], sp);
    } else {
#pragma unroll
        for (int e = 0; e < KO; ++e)
            span_st(T(o[e]), out.p[0], sp, KO, e);
    }
}

// Per-matrix driver shared by every kernel: the grid strides over spans of
// kBlock matrices; each lane loads its matrix (from the structure-of-arrays
// arrays, or from the LDS tile for array-of-structures input), calls
// body(span, matrix, o), which fills the KO output values o[], and stores them
// in output layout OL.  For AoS input and AoS output the rows go back through
// LDS and leave with 16-byte stores.
template <class T, int S, int L, int KO, int OL, class Body>
__device__ __forceinline__ void for_each_matrix(int64_t n, const In9<T> &in, const OutK<T, KO> &out, Body body)
{
    constexpr int K = Mat<T, S>::K;
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    if constexpr (L == EIG3_SOA) {
        for (int64_t first = int64_t(blockIdx.x) * kBlock; first < n; first += stride) {
            const Span sp = span_at(first, n);
            if (!sp.live())
                continue;
            Mat<T, S> m;
            load_soa<T, S>(in, sp, m);
            double o[KO];
            body(sp, m, o);
            store_rows(out, OL, sp, o);
        }
    } else {
        constexpr int kS = aos_stride<T, K>();
        constexpr int kIn = kBlock * kS;
        constexpr int kOut = OL == EIG3_AOS ? kBlock * KO : 0;
        __shared__ __attribute__((aligned(16))) T tile[kIn > kOut ? kIn : kOut];
        for (int64_t first = int64_t(blockIdx.x) * kBlock; first < n; first += stride) {
            __syncthreads(); // the previous iteration is done with the tile
            aos_stage<T, K>(in.p[0], first, n, tile);
            __syncthreads();
            const Span sp = span_at(first, n);
            double o[KO];
            if (sp.live()) {
                Mat<T, S> m;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    m.a[k] = tile[threadIdx.x * kS + k];
                body(sp, m, o);
            }
            if constexpr (OL == EIG3_AOS) {
                __syncthreads(); // every lane has read its input row
                if (sp.live()) {
#pragma unroll
                    for (int e = 0; e < KO; ++e)
                        tile[threadIdx.x * KO + e] = T(o[e]);
                }
                __syncthreads();
                aos_flush<T, KO>(out.p[0], first, n, tile);
            } else {
                if (sp.live())
                    store_rows(out, EIG3_SOA, sp, o);
            }
        }
    }
}

// binary32 data: K2, K3 and 54 Delta of the double-word and compensated
// evaluations
template <int S, int Acc> __device__ __forceinline__ KW kw_of(const Mat<float, S> &m)
{
    static_assert(Acc == EIG3_COMPENSATED || Acc == EIG3_DOUBLE_WORD, "K route");
    if constexpr (Acc == EIG3_COMPENSATED) {
        if constexpr (S == EIG3_GENERAL)
            return kw_f32_comp_general(m.a);
        else
            return kw_f32_comp_symmetric(m.a);
    } else {
        if constexpr (S == EIG3_GENERAL)
            return kw_f32_dw_general(m.a);
        else
            return kw_f32_dw_symmetric(m.a);
    }
}

template <int S, int Acc> __device__ __forceinline__ InvW invariants_of(const Mat<float, S> &m)
{
    if constexpr (Acc == EIG3_COMPENSATED || Acc == EIG3_DOUBLE_WORD) {
        return invariants_of_kw(kw_of<S, Acc>(m));
    } else {
        Inv v;
        if constexpr (S == EIG3_GENERAL)
            v = invariants_general_fma(Gen{double(m.a[0]), double(m.a[1]), double(m.a[2]), double(m.a[3]),
                                           double(m.a[4]), double(m.a[5]), double(m.a[6]), double(m.a[7]),
                                           double(m.a[8])});
        else
            v = invariants_symmetric_fma(
                Sym{double(m.a[0]), double(m.a[1]), double(m.a[2]), double(m.a[3]), double(m.a[4]), double(m.a[5])});
        return InvW{v.i1, v.j2, v.j3, v.disc};
    }
}

// the arguments of the binary32 eigenvalue tail
template <int S, int Acc> __device__ __forceinline__ TrigArgW f32_args_of(const Mat<float, S> &m)
{
    if constexpr (Acc == EIG3_COMPENSATED || Acc == EIG3_DOUBLE_WORD)
        return trig_args_of_kw(kw_of<S, Acc>(m));
    else
        return trig_args_of_invariants(invariants_of<S, Acc>(m));
}

// Binary64 batches are evaluated on A 2^-e, 2^e the binade of A's largest
// entry (max |A_ij| in [1/2, 1) after scaling).  I1, J2, J3 and Delta are
// homogeneous of degree 1, 2, 3, 6 in the entries, so the scaled evaluation
// is the unscaled one times exact powers of two (bitwise the same results
// where nothing under- or overflows), while Delta ~ |A|^6 stays inside the
// binary64 range for every finite input (unscaled it over- or underflows
// beyond about 2^+-160).  Eigenvalues and the Mohr-Coulomb stresses scale
// back by 2^e; the eigenvalue gradient and the eigenprojectors do not change
// with the scale.  (Binary32 entries widened to binary64 stay in range
// without it; the paper's naive comparators are left as printed.)
// Where the largest entry of every matrix of the wave lies in [2^-64, 2^64)
// the scaling is skipped: nothing then over- or underflows that the scaled
// evaluation would keep, and the results are bitwise those of the scaled
// evaluation (every operation commutes with an exact power of two).
// (The window test compares the entries' high words with the sign cleared:
// they order the entries by magnitude up to the low word, so their maximum
// carries the binade of the largest entry; a zero, infinite or NaN entry
// fails it and its wave takes the exact exponent below, which scales such
// matrices by 2^0 as before.)
template <int S> __device__ __forceinline__ int prescale(Mat<double, S> &m)
{
    uint32_t h = 0;
#pragma unroll
    for (int k = 0; k < Mat<double, S>::K; ++k) {
        const uint32_t hk = uint32_t(__builtin_bit_cast(uint64_t, m.a[k]) >> 32) & 0x7fffffffu;
        h = hk > h ? hk : h;
    }
    // biased exponent of the largest entry in [959, 1086]: frexp exponent in [-63, 64]
    if (__all(h - (959u << 20) < (128u << 20)))
        return 0;
    double mx = 0.0;
#pragma unroll
    for (int k = 0; k < Mat<double, S>::K; ++k)
        mx = fmax(mx, fabs(m.a[k]));
    const int e = __builtin_amdgcn_frexp_exp(mx); // 0 for 0, Inf and NaN: no scaling
#pragma unroll
    for (int k = 0; k < Mat<double, S>::K; ++k)
        m.a[k] = ldexp(m.a[k], -e);
    return e;
}

template <class T, int Acc> constexpr bool scaled_path()
{
    return sizeof(T) == 8 && (Acc == EIG3_FMA || Acc == EIG3_COMPENSATED || Acc == EIG3_DOUBLE_WORD);
}

// The triple-angle quantities of a binary64 matrix from its invariants
// evaluated on the prescaled copy (so that Delta ~ |A|^6 neither over- nor
// underflows), with the mean and the radius scaled back by 2^e: the
// eigenvalues of A itself, for kernels that keep working with A's entries.
template <int S, int Acc> __device__ __forceinline__ Trig trig_of(Mat<double, S> m)
{
    int e = 0;
    if constexpr (scaled_path<double, Acc>())
        e = prescale(m);
    Trig t = trig_of_matrix<S, Acc, false>(m);
    t.mean = ldexp(t.mean, e);
    t.r = ldexp(t.r, e);
    return t;
}

// ------------------------------------------------------------------ kernels
template <class T, int S, int L, int Acc>
EIG3_KERNEL void k_invariants(int64_t n, In9<T> in, OutK<T, 4> out)
{
    for_each_matrix<T, S, L, 4, EIG3_SOA>(n, in, out, [&](const Span &, const Mat<T, S> &m, double (&o)[4]) {
        const auto v = invariants_of<S, Acc>(m);
        o[0] = v.i1;
        o[1] = v.j2;
        o[2] = v.j3;
        o[3] = v.disc;
    });
}

template <class T, int S, int L, int OL, int Acc>
EIG3_KERNEL void k_eigvals(int64_t n, In9<T> in, OutK<T, 3> out)
{
    for_each_matrix<T, S, L, 3, OL>(n, in, out, [&](const Span &, const Mat<T, S> &mt, double (&o)[3]) {
        if constexpr (scaled_path<T, Acc>()) {
            Mat<double, S> m = mt;
            const int e = prescale(m);
            eigvals_from_trig(trig_of_matrix<S, Acc, true>(m), o[0], o[1], o[2]);
#pragma unroll
            for (int k = 0; k < 3; ++k)
                o[k] = ldexp(o[k], e);
        } else if constexpr (sizeof(T) == 8) {
            eigvals_from_invariants(invariants_of<S, Acc>(mt), o[0], o[1], o[2]);
        } else {
            float l1, l2, l3;
            eigvals_f32_from_args(f32_args_of<S, Acc>(mt), l1, l2, l3);
            o[0] = l1;
            o[1] = l2;
            o[2] = l3;
        }
    });
}

// Binary32 structure-of-arrays in and out, two adjacent matrices per lane:
// a workgroup covers a span of 2 kBlock matrices, lane i owns matrices 2i and
// 2i + 1 of it and moves both with one 8-byte access per array, so each wave
// keeps twice the bytes in flight of the one-matrix-per-lane launch.  A
// ragged last span is done one matrix per lane, as two spans of kBlock.
// (Only launched when every array is 8-byte aligned.)
template <int S, int Acc> __device__ __forceinline__ void eigvals_f32(const Mat<float, S> &m, float (&l)[3])
{
    eigvals_f32_from_args(f32_args_of<S, Acc>(m), l[0], l[1], l[2]);
}

template <int S, int Acc> EIG3_KERNEL void k_eigvals_f32x2(int64_t n, In9<float> in, OutK<float, 3> out)
{
    constexpr int K = Mat<float, S>::K;
    constexpr int kSpan = 2 * kBlock;
    const int64_t stride = int64_t(gridDim.x) * kSpan;
    for (int64_t first = int64_t(blockIdx.x) * kSpan; first < n; first += stride) {
        if (n - first >= kSpan) {
            const int off = int(threadIdx.x) * 8;
            Mat<float, S> m0, m1;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<float *>(in.p[k]) + first, 0, kSpan * int(sizeof(float)), kBufferWord3);
                // (split as a 64-bit integer: a bit cast of the loaded pair to
                // a two-lane vector lets the compiler narrow the load to 4 bytes)
                const uint64_t v = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kBufferAux));
                m0.a[k] = __builtin_bit_cast(float, uint32_t(v));
                m1.a[k] = __builtin_bit_cast(float, uint32_t(v >> 32));
            }
            float l0[3], l1[3];
            eigvals_f32<S, Acc>(m0, l0);
            eigvals_f32<S, Acc>(m1, l1);
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
                    out.p[e] + first, 0, kSpan * int(sizeof(float)), kBufferWord3);
                const u32x2 v = {__builtin_bit_cast(unsigned, l0[e]), __builtin_bit_cast(unsigned, l1[e])};
                __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, kBufferAux);
            }
        } else {
#pragma unroll 1
            for (int64_t f = first; f < n && f < first + kSpan; f += kBlock) {
                const Span sp = span_at(f, n);
                if (!sp.live())
                    continue;
                Mat<float, S> m;
                load_soa<float, S>(in, sp, m);
                float l[3];
                eigvals_f32<S, Acc>(m, l);
                const double o[3] = {l[0], l[1], l[2]};
                store_rows(out, EIG3_SOA, sp, o);
            }
        }
    }
}

template <class T, int S> __device__ __forceinline__ Mat<double, S> widen(const Mat<T, S> &mt)
{
    Mat<double, S> m;
#pragma unroll
    for (int k = 0; k < Mat<T, S>::K; ++k)
        m.a[k] = double(mt.a[k]);
    return m;
}

template <int S> __device__ __forceinline__ Gen general_of(const Mat<double, S> &m)
{
    if constexpr (S == EIG3_GENERAL) {
        return to_gen(m);
    } else {
        const Sym y = to_sym(m);
        return Gen{y.s00, y.s01, y.s02, y.s01, y.s11, y.s12, y.s02, y.s12, y.s22};
    }
}

// full-matrix gradient -> the K outputs of the storage: general 9 entries;
// symmetric: the derivative with respect to each stored entry (Stored) or
// the components of the symmetric tensor derivative (Tensor)
enum { kStored = 0, kTensor = 1 };
template <int S, int Kind, int KO>
__device__ __forceinline__ void gradient_rows(const double (&gr)[9], double (&o)[KO])
{
    if constexpr (S == EIG3_GENERAL) {
#pragma unroll
        for (int k = 0; k < 9; ++k)
            o[k] = gr[k];
    } else {
        const double h = Kind == kStored ? 1.0 : 0.5;
        o[0] = gr[0];
        o[1] = gr[4];
        o[2] = gr[8];
        o[3] = h * (gr[1] + gr[3]);
        o[4] = h * (gr[2] + gr[6]);
        o[5] = h * (gr[5] + gr[7]);
    }
}

// The adjoint runs in binary64 for either storage type (binary32 entries and
// upstream gradients are widened exactly; the result is rounded once).
template <class T, int S, int L, int GL, int Acc>
EIG3_KERNEL void k_backward(int64_t n, In9<T> in, G3<T> g, OutK<T, Mat<T, S>::K> out)
{
    constexpr int KO = Mat<T, S>::K;
    for_each_matrix<T, S, L, KO, L>(n, in, out, [&](const Span &sp, const Mat<T, S> &mt, double (&o)[KO]) {
        double g1, g2, g3;
        if constexpr (GL == EIG3_SOA) {
            g1 = double(span_ld(g.p[0], sp));
            g2 = double(span_ld(g.p[1], sp));
            g3 = double(span_ld(g.p[2], sp));
        } else {
            g1 = double(span_ld(g.p[0], sp, 3, 0));
            g2 = double(span_ld(g.p[0], sp, 3, 1));
            g3 = double(span_ld(g.p[0], sp, 3, 2));
        }
        Mat<double, S> m = widen(mt);
        if constexpr (scaled_path<T, Acc>())
            prescale(m); // the gradient does not change with the scale
        const Coef c = backward_coefficients(trig_of_matrix<S, Acc, false>(m), g1, g2, g3);
        double gr[9];
        backward_general(general_of(m), c, gr);
        gradient_rows<S, kStored>(gr, o);
    });
}

// Mohr-Coulomb yield function f and, if Grad, df/dsigma (binary64
// arithmetic for either storage type).  For symmetric storage df/dsigma is
// the tensor derivative: its 6 components.  Without the gradient f is the
// single output slot; with it, f goes straight to its own array and the
// slots carry the gradient in the layout of sigma.
template <class T, int S, int L, int Acc, bool Grad>
EIG3_KERNEL void k_mohr_coulomb(int64_t n, In9<T> in, double cf, double K, T *__restrict__ f,
                                OutK<T, Grad ? Mat<T, S>::K : 1> out)
{
    constexpr int KO = Grad ? Mat<T, S>::K : 1;
    constexpr int OL = Grad ? L : EIG3_SOA;
    for_each_matrix<T, S, L, KO, OL>(n, in, out, [&](const Span &sp, const Mat<T, S> &mt, double (&o)[KO]) {
        Mat<double, S> m = widen(mt);
        int e = 0;
        if constexpr (scaled_path<T, Acc>())
            e = prescale(m);
        const Inv v = invariants_of<S, Acc>(m);
        // the gradient kernel carries many pointers: its coefficients are
        // immediates rather than SGPR-resident constants
        const MohrCoulomb mc = mohr_coulomb<!Grad>(v, cf, K, e);
        if constexpr (Grad) {
            span_st(T(mc.f), f, sp);
            const Coef c = backward_coefficients(mc.t, mc.g1, 0.0, mc.g3);
            double gr[9];
            backward_general(general_of(m), c, gr);
            gradient_rows<S, kTensor>(gr, o);
        } else {
            o[0] = mc.f;
        }
    });
}

// Eigenprojectors E_1, E_2, E_3 (ascending eigenvalues); binary64 arithmetic
// for either storage type.  GENERAL: 9 entries per projector; SYMMETRIC: the
// 6 components of each (symmetric) projector.  Slot 9k+e (general) or 6k+e
// (symmetric).
template <class T, int S, int L, int OL, int Acc>
EIG3_KERNEL void k_eigenprojectors(int64_t n, In9<T> in, OutK<T, 3 * Mat<T, S>::K> out)
{
    constexpr int KS = Mat<T, S>::K;
    constexpr int KO = 3 * KS;
    for_each_matrix<T, S, L, KO, OL>(n, in, out, [&](const Span &, const Mat<T, S> &mt, double (&o)[KO]) {
        Mat<double, S> m = widen(mt);
        if constexpr (scaled_path<T, Acc>())
            prescale(m); // the projectors do not change with the scale
        const Trig t = trig_of_matrix<S, Acc, false>(m);
        double E[27];
        eigenprojectors_general(general_of(m), t, E);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if constexpr (S == EIG3_GENERAL) {
#pragma unroll
                for (int e = 0; e < 9; ++e)
                    o[9 * k + e] = E[9 * k + e];
            } else {
                o[6 * k + 0] = E[9 * k + 0];
                o[6 * k + 1] = E[9 * k + 4];
                o[6 * k + 2] = E[9 * k + 8];
                o[6 * k + 3] = 0.5 * (E[9 * k + 1] + E[9 * k + 3]);
                o[6 * k + 4] = 0.5 * (E[9 * k + 2] + E[9 * k + 6]);
                o[6 * k + 5] = 0.5 * (E[9 * k + 5] + E[9 * k + 7]);
            }
        }
    });
}

// A function of each matrix (exp, log, sqrt) through the eigenprojectors;
// binary64 arithmetic for either storage type; the result in the structure
// and layout of A (symmetric: the 6 components).
template <class T, int S, int L, int Acc, int Fn>
__device__ __forceinline__ void matrix_function_spans(int64_t n, const In9<T> &in, const OutK<T, Mat<T, S>::K> &out)
{
    constexpr int KO = Mat<T, S>::K;
    for_each_matrix<T, S, L, KO, L>(n, in, out, [&](const Span &, const Mat<T, S> &mt, double (&o)[KO]) {
        const Mat<double, S> m = widen(mt);
        double F[9];
        matrix_function_general<Fn>(general_of(m), trig_of<S, Acc>(m), F);
        gradient_rows<S, kTensor>(F, o);
    });
}

template <class T, int S, int L, int Acc, int Fn>
EIG3_KERNEL void k_matrix_function(int64_t n, In9<T> in, OutK<T, Mat<T, S>::K> out)
{
    matrix_function_spans<T, S, L, Acc, Fn>(n, in, out);
}

// The fma and double-word evaluations with at most 168 VGPRs: 3 resident
// waves per SIMD instead of the 2 that the compiler's default allocation
// (172 for exp) leaves (measured 18% faster for exp); the compensated
// evaluation spills at that limit and keeps the default.
template <class T, int S, int L, int Acc, int Fn>
EIG3_KERNEL __attribute__((amdgpu_waves_per_eu(3))) void k_matrix_function_w3(int64_t n, In9<T> in,
                                                                               OutK<T, Mat<T, S>::K> out)
{
    matrix_function_spans<T, S, L, Acc, Fn>(n, in, out);
}

// Vector-Jacobian product of the matrix function: g in the layout of A
// (the forward's output), the gradient in the structure and layout of A.
template <class T, int S, int L, int Acc, int Fn>
__device__ __forceinline__ void matrix_function_backward_spans(int64_t n, const In9<T> &in, const In9<T> &gin,
                                                              const OutK<T, Mat<T, S>::K> &out)
{
    constexpr int KO = Mat<T, S>::K;
    for_each_matrix<T, S, L, KO, L>(n, in, out, [&](const Span &sp, const Mat<T, S> &mt, double (&o)[KO]) {
        const Mat<double, S> m = widen(mt);
        const Trig t = trig_of<S, Acc>(m);
        double gk[KO];
#pragma unroll
        for (int k = 0; k < KO; ++k)
            gk[k] = double(L == EIG3_SOA ? span_ld(gin.p[k], sp) : span_ld(gin.p[0], sp, KO, k));
        double G[9];
        if constexpr (S == EIG3_GENERAL) {
#pragma unroll
            for (int k = 0; k < 9; ++k)
                G[k] = gk[k];
        } else {
            // dL/dF for the symmetric F from dL/d(its 6 stored components)
            G[0] = gk[0];
            G[4] = gk[1];
            G[8] = gk[2];
            G[1] = G[3] = 0.5 * gk[3];
            G[2] = G[6] = 0.5 * gk[4];
            G[5] = G[7] = 0.5 * gk[5];
        }
        double gr[9];
        matrix_function_backward_general<Fn>(general_of(m), t, G, gr);
        gradient_rows<S, kStored>(gr, o);
    });
}

template <class T, int S, int L, int Acc, int Fn>
EIG3_KERNEL void k_matrix_function_backward(int64_t n, In9<T> in, In9<T> gin, OutK<T, Mat<T, S>::K> out)
{
    matrix_function_backward_spans<T, S, L, Acc, Fn>(n, in, gin, out);
}

// The fma and double-word evaluations with at most 168 VGPRs, so that 3 waves
// per SIMD are resident instead of 2 (measured 5-7% faster for exp; the
// compensated evaluation spills at that limit and keeps the default).
template <class T, int S, int L, int Acc, int Fn>
EIG3_KERNEL __attribute__((amdgpu_waves_per_eu(3))) void k_matrix_function_backward_w3(int64_t n, In9<T> in,
                                                                                        In9<T> gin,
                                                                                        OutK<T, Mat<T, S>::K> out)
{
    matrix_function_backward_spans<T, S, L, Acc, Fn>(n, in, gin, out);
}

// ------------------------------------------------------------------- host
// one workgroup per span of kBlock matrices, up to kMaxBlocks (the grid
// strides beyond that)
int64_t grid_for(int64_t n, int64_t span = kBlock)
{
    const int64_t b = (n + span - 1) / span;
    return b < kMaxBlocks ? b : kMaxBlocks;
}

// largest batch: keeps every operand's byte size far inside size_t
constexpr int64_t kMaxMatrices = int64_t(1) << 56;

bool valid_enum(int v, int hi) { return v >= 0 && v <= hi; }

size_t elem_size(int dtype) { return dtype == EIG3_F64 ? 8 : 4; }

struct Range {
    uintptr_t lo, hi;
};

// byte ranges of the input matrices
int input_ranges(const eig3_matrices *A, Range *r)
{
    const size_t es = elem_size(A->dtype);
    const int K = A->structure == EIG3_GENERAL ? 9 : 6;
    if (A->layout == EIG3_AOS) {
        r[0] = {uintptr_t(A->a[0]), uintptr_t(A->a[0]) + size_t(A->n) * K * es};
        return 1;
    }
    for (int k = 0; k < K; ++k)
        r[k] = {uintptr_t(A->a[k]), uintptr_t(A->a[k]) + size_t(A->n) * es};
    return K;
}

bool overlaps(const Range &a, const Range &b) { return a.lo < b.hi && b.lo < a.hi; }

bool aligned(const void *p, size_t a) { return (uintptr_t(p) % a) == 0; }

// every input array of a structure-of-arrays batch and every output array
// aligned to a bytes
bool all_aligned(const eig3_matrices *A, void *const *outs, size_t a)
{
    const int K = A->structure == EIG3_GENERAL ? 9 : 6;
    for (int k = 0; k < K; ++k)
        if (!aligned(A->a[k], a))
            return false;
    for (int e = 0; e < 3; ++e)
        if (!aligned(outs[e], a))
            return false;
    return true;
}

// common validation of the matrix batch; K = number of stored entries
int check_matrices(const eig3_matrices *A)
{
    if (A == nullptr || A->n < 0 || A->n > kMaxMatrices)
        return EIG3_EINVAL;
    if (!valid_enum(A->dtype, 1) || !valid_enum(A->structure, 1) || !valid_enum(A->layout, 1) ||
        !valid_enum(A->accuracy, 4))
        return EIG3_EINVAL;
    if (A->n == 0)
        return EIG3_OK;
    const int K = A->structure == EIG3_GENERAL ? 9 : 6;
    const int np = A->layout == EIG3_AOS ? 1 : K;
    for (int k = 0; k < np; ++k)
        if (A->a[k] == nullptr || !aligned(A->a[k], elem_size(A->dtype)))
            return EIG3_EINVAL;
    return EIG3_OK;
}

constexpr int kMaxOutputs = 27; // eig3_eigenprojectors, general SoA

int check_outputs(const eig3_matrices *A, void *const *outs, int nout, size_t count_each)
{
    Range in[9];
    const int nin = input_ranges(A, in);
    const size_t es = elem_size(A->dtype);
    Range o[kMaxOutputs];
    if (nout < 0 || nout > kMaxOutputs)
        return EIG3_EINVAL;
    for (int j = 0; j < nout; ++j) {
        if (outs[j] == nullptr || !aligned(outs[j], es))
            return EIG3_EINVAL;
        o[j] = {uintptr_t(outs[j]), uintptr_t(outs[j]) + count_each * es};
        for (int k = 0; k < nin; ++k)
            if (overlaps(o[j], in[k]))
                return EIG3_EINVAL;
        for (int k = 0; k < j; ++k)
            if (overlaps(o[j], o[k]))
                return EIG3_EINVAL;
    }
    return EIG3_OK;
}

int launched()
{
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? EIG3_OK : EIG3_ELAUNCH;
}

template <class T> In9<T> inputs_of(const eig3_matrices *A)
{
    In9<T> in;
    for (int k = 0; k < 9; ++k)
        in.p[k] = static_cast<const T *>(A->a[k]);
    return in;
}

// dispatch helpers: turn runtime enums into template arguments
template <class F> void dispatch_sla(int s, int l, int acc, F f)
{
    auto a = [&](auto S, auto L) {
        if (acc == EIG3_COMPENSATED)
            f(S, L, std::integral_constant<int, EIG3_COMPENSATED>{});
        else if (acc == EIG3_DOUBLE_WORD)
            f(S, L, std::integral_constant<int, EIG3_DOUBLE_WORD>{});
        else
            f(S, L, std::integral_constant<int, EIG3_FMA>{});
    };
    auto b = [&](auto S) {
        if (l == EIG3_AOS)
            a(S, std::integral_constant<int, EIG3_AOS>{});
        else
            a(S, std::integral_constant<int, EIG3_SOA>{});
    };
    if (s == EIG3_SYMMETRIC)
        b(std::integral_constant<int, EIG3_SYMMETRIC>{});
    else
        b(std::integral_constant<int, EIG3_GENERAL>{});
}

// the same with the two comparator modes (binary64 forward kernels only)
template <class F> void dispatch_sla4(int s, int l, int acc, F f)
{
    if (acc == EIG3_NAIVE || acc == EIG3_NAIVE_TENSOR) {
        auto a = [&](auto S, auto L) {
            if (acc == EIG3_NAIVE)
                f(S, L, std::integral_constant<int, EIG3_NAIVE>{});
            else
                f(S, L, std::integral_constant<int, EIG3_NAIVE_TENSOR>{});
        };
        auto b = [&](auto S) {
            if (l == EIG3_AOS)
                a(S, std::integral_constant<int, EIG3_AOS>{});
            else
                a(S, std::integral_constant<int, EIG3_SOA>{});
        };
        if (s == EIG3_SYMMETRIC)
            b(std::integral_constant<int, EIG3_SYMMETRIC>{});
        else
            b(std::integral_constant<int, EIG3_GENERAL>{});
        return;
    }
    dispatch_sla(s, l, acc, f);
}

bool comparator(int acc) { return acc == EIG3_NAIVE || acc == EIG3_NAIVE_TENSOR; }

template <class T, int KO> OutK<T, KO> out_slots(void *const *outs, int nout)
{
    OutK<T, KO> o;
    for (int k = 0; k < KO; ++k)
        o.p[k] = k < nout ? static_cast<T *>(outs[k]) : nullptr;
    return o;
}


} // namespace

// ===================================================================== C ABI
extern "C" {

const char *eig3_status_string(int status)
{
    switch (status) {
    case EIG3_OK:
        return "EIG3_OK";
    case EIG3_EINVAL:
        return "EIG3_EINVAL: invalid argument";
    case EIG3_EUNSUPPORTED:
        return "EIG3_EUNSUPPORTED: combination not provided by the library";
    case EIG3_ELAUNCH:
        return "EIG3_ELAUNCH: kernel launch failed";
    default:
        return "unknown eig3 status";
    }
}

int eig3_matrix_function(const eig3_matrices *A, int32_t fn, void *const out[9], hipStream_t stream)
{
    int st = check_matrices(A);
    if (st != EIG3_OK)
        return st;
    if (out == nullptr || !valid_enum(fn, 2))
        return EIG3_EINVAL;
    if (A->n == 0)
        return EIG3_OK;
    if (comparator(A->accuracy))
        return EIG3_EUNSUPPORTED;
    const int K = A->structure == EIG3_GENERAL ? 9 : 6;
    const int nout = A->layout == EIG3_SOA ? K : 1;
    void *outs[9];
    for (int k = 0; k < nout; ++k)
        outs[k] = out[k];
    if ((st = check_outputs(A, outs, nout, size_t(A->n) * (nout == 1 ? K : 1))) != EIG3_OK)
        return st;
    const dim3 grid(unsigned(grid_for(A->n))), block(kBlock);
    auto launch = [&](auto tag) {
        using T = decltype(tag);
        const In9<T> in = inputs_of<T>(A);
        dispatch_sla(A->structure, A->layout, A->accuracy, [&](auto S, auto L, auto Acc) {
            constexpr int KO = S.value == EIG3_GENERAL ? 9 : 6;
            const OutK<T, KO> o = out_slots<T, KO>(outs, nout);
            auto go = [&](auto fnv) {
                constexpr int F = decltype(fnv)::value;
                if constexpr (Acc.value == EIG3_COMPENSATED)
                    hipLaunchKernelGGL((k_matrix_function<T, S.value, L.value, Acc.value, F>), grid, block, 0, stream,
                                       A->n, in, o);
                else
                    hipLaunchKernelGGL((k_matrix_function_w3<T, S.value, L.value, Acc.value, F>), grid, block, 0,
                                       stream, A->n, in, o);
            };
            if (fn == EIG3_EXP)
                go(std::integral_constant<int, EIG3_EXP>{});
            else if (fn == EIG3_LOG)
                go(std::integral_constant<int, EIG3_LOG>{});
            else
                go(std::integral_constant<int, EIG3_SQRT>{});
        });
    };
    if (A->dtype == EIG3_F32)
        launch(float{});
    else
        launch(double{});
    return launched();
}

int eig3_matrix_function_backward(const eig3_matrices *A, int32_t fn, const void *const g[9], void *const grad_a[9],
                                  hipStream_t stream)
{
    int st = check_matrices(A);
    if (st != EIG3_OK)
        return st;
    if (g == nullptr || grad_a == nullptr || !valid_enum(fn, 2))
        return EIG3_EINVAL;
    if (A->n == 0)
        return EIG3_OK;
    if (comparator(A->accuracy))
        return EIG3_EUNSUPPORTED;
    const int K = A->structure == EIG3_GENERAL ? 9 : 6;
    const size_t es = elem_size(A->dtype);
    const int np = A->layout == EIG3_SOA ? K : 1;
    const size_t each = size_t(A->n) * (np == 1 ? K : 1);
    for (int k = 0; k < np; ++k)
        if (g[k] == nullptr || !aligned(g[k], es))
            return EIG3_EINVAL;
    void *outs[9];
    for (int k = 0; k < np; ++k)
        outs[k] = grad_a[k];
    if ((st = check_outputs(A, outs, np, each)) != EIG3_OK)
        return st;
    for (int j = 0; j < np; ++j) {
        const Range o{uintptr_t(outs[j]), uintptr_t(outs[j]) + each * es};
        for (int k = 0; k < np; ++k)
            if (overlaps(o, Range{uintptr_t(g[k]), uintptr_t(g[k]) + each * es}))
                return EIG3_EINVAL;
    }
    const dim3 grid(unsigned(grid_for(A->n))), block(kBlock);
    auto launch = [&](auto tag) {
        using T = decltype(tag);
        const In9<T> in = inputs_of<T>(A);
        In9<T> gin;
        for (int k = 0; k < 9; ++k)
            gin.p[k] = k < np ? static_cast<const T *>(g[k]) : nullptr;
        dispatch_sla(A->structure, A->layout, A->accuracy, [&](auto S, auto L, auto Acc) {
            constexpr int KO = S.value == EIG3_GENERAL ? 9 : 6;
            const OutK<T, KO> o = out_slots<T, KO>(outs, np);
            auto go = [&](auto fnv) {
                constexpr int F = decltype(fnv)::value;
                if constexpr (Acc.value != EIG3_COMPENSATED)
                    hipLaunchKernelGGL((k_matrix_function_backward_w3<T, S.value, L.value, Acc.value, F>), grid,
                                       block, 0, stream, A->n, in, gin, o);
                else
                    hipLaunchKernelGGL((k_matrix_function_backward<T, S.value, L.value, Acc.value, F>), grid,
                                       block, 0, stream, A->n, in, gin, o);
            };
            if (fn == EIG3_EXP)
                go(std::integral_constant<int, EIG3_EXP>{});
            else if (fn == EIG3_LOG)
                go(std::integral_constant<int, EIG3_LOG>{});
            else
                go(std::integral_constant<int, EIG3_SQRT>{});
        });
    };
    if (A->dtype == EIG3_F32)
        launch(float{});
    else
        launch(double{});
    return launched();
}

const char *eig3_version(void) { return "0.1.0"; }

int64_t eig3_soa_stride(int64_t n, int32_t dtype)
{
    if (n < 0 || n > kMaxMatrices || !valid_enum(dtype, 1))
        return -1;
    // 42 KiB = 32 + 8 + 2 KiB: three address bits, so that no single high
    // address bit of an array size can cancel the stagger in the interleave
    constexpr int64_t kRound = int64_t(64) << 10, kStagger = int64_t(42) << 10;
    const int64_t size = dtype == EIG3_F64 ? 8 : 4;
    return ((n * size + kRound - 1) / kRound * kRound + kStagger) / size;
}

int eig3_invariants(const eig3_matrices *A, void *i1, void *j2, void *j3, void *disc, hipStream_t stream)
{
    int st = check_matrices(A);
    if (st != EIG3_OK || A->n == 0)
        return st;
    void *outs[4] = {i1, j2, j3, disc};
    if ((st = check_outputs(A, outs, 4, size_t(A->n))) != EIG3_OK)
        return st;
    if (A->dtype == EIG3_F32 && comparator(A->accuracy))
        return EIG3_EUNSUPPORTED;
    const dim3 grid(unsigned(grid_for(A->n))), block(kBlock);
    auto launch = [&](auto tag, auto dispatch) {
        using T = decltype(tag);
        const In9<T> in = inputs_of<T>(A);
        const OutK<T, 4> out = out_slots<T, 4>(outs, 4);
        dispatch(A->structure, A->layout, A->accuracy, [&](auto S, auto L, auto Acc) {
            hipLaunchKernelGGL((k_invariants<T, S.value, L.value, Acc.value>), grid, block, 0, stream, A->n, in,
                               out);
        });
    };
    if (A->dtype == EIG3_F32)
        launch(float{}, [](int s, int l, int acc, auto f) { dispatch_sla(s, l, acc, f); });
    else
        launch(double{}, [](int s, int l, int acc, auto f) { dispatch_sla4(s, l, acc, f); });
    return launched();
}

int eig3_eigvals(const eig3_matrices *A, int32_t out_layout, void *const lam[3], hipStream_t stream)
{
    int st = check_matrices(A);
    if (st != EIG3_OK)
        return st;
    if (lam == nullptr || !valid_enum(out_layout, 1))
        return EIG3_EINVAL;
    if (A->n == 0)
        return EIG3_OK;
    void *outs[3] = {lam[0], out_layout == EIG3_SOA ? lam[1] : nullptr, out_layout == EIG3_SOA ? lam[2] : nullptr};
    const int nout = out_layout == EIG3_SOA ? 3 : 1;
    if ((st = check_outputs(A, outs, nout, size_t(A->n) * (nout == 1 ? 3 : 1))) != EIG3_OK)
        return st;
    if (A->dtype == EIG3_F32 && comparator(A->accuracy))
        return EIG3_EUNSUPPORTED;
    const dim3 grid(unsigned(grid_for(A->n))), block(kBlock);
    auto launch = [&](auto tag, auto dispatch) {
        using T = decltype(tag);
        const In9<T> in = inputs_of<T>(A);
        const OutK<T, 3> out = out_slots<T, 3>(outs, nout);
        dispatch(A->structure, A->layout, A->accuracy, [&](auto S, auto L, auto Acc) {
            if (out_layout == EIG3_AOS)
                hipLaunchKernelGGL((k_eigvals<T, S.value, L.value, EIG3_AOS, Acc.value>), grid, block, 0, stream,
                                   A->n, in, out);
            else
                hipLaunchKernelGGL((k_eigvals<T, S.value, L.value, EIG3_SOA, Acc.value>), grid, block, 0, stream,
                                   A->n, in, out);
        });
    };
    if (A->dtype == EIG3_F32 && A->layout == EIG3_SOA && out_layout == EIG3_SOA &&
        all_aligned(A, outs, 8)) {
        const In9<float> in = inputs_of<float>(A);
        const OutK<float, 3> out = out_slots<float, 3>(outs, nout);
        const dim3 g2(unsigned(grid_for(A->n, 2 * kBlock)));
        dispatch_sla(A->structure, A->layout, A->accuracy, [&](auto S, auto, auto Acc) {
            hipLaunchKernelGGL((k_eigvals_f32x2<S.value, Acc.value>), g2, block, 0, stream, A->n, in, out);
        });
    } else if (A->dtype == EIG3_F32) {
        launch(float{}, [](int s, int l, int acc, auto f) { dispatch_sla(s, l, acc, f); });
    } else {
        launch(double{}, [](int s, int l, int acc, auto f) { dispatch_sla4(s, l, acc, f); });
    }
    return launched();
}

int eig3_eigvals_backward(const eig3_matrices *A, int32_t g_layout, const void *const g[3], void *const grad_a[9],
                          hipStream_t stream)
{
    int st = check_matrices(A);
    if (st != EIG3_OK)
        return st;
    if (g == nullptr || grad_a == nullptr || !valid_enum(g_layout, 1))
        return EIG3_EINVAL;
    if (A->n == 0)
        return EIG3_OK;
    if (comparator(A->accuracy))
        return EIG3_EUNSUPPORTED;
    const int K = A->structure == EIG3_GENERAL ? 9 : 6;
    const size_t es = elem_size(A->dtype);
    // g: inputs, must be valid and not alias the outputs
    const int ng = g_layout == EIG3_SOA ? 3 : 1;
    for (int k = 0; k < ng; ++k)
        if (g[k] == nullptr || !aligned(g[k], es))
            return EIG3_EINVAL;
    const int nout = A->layout == EIG3_SOA ? K : 1;
    void *outs[9];
    for (int k = 0; k < nout; ++k)
        outs[k] = grad_a[k];
    if ((st = check_outputs(A, outs, nout, size_t(A->n) * (nout == 1 ? K : 1))) != EIG3_OK)
        return st;
    for (int j = 0; j < nout; ++j) {
        const Range o{uintptr_t(outs[j]), uintptr_t(outs[j]) + size_t(A->n) * (nout == 1 ? K : 1) * es};
        for (int k = 0; k < ng; ++k) {
            const Range gr{uintptr_t(g[k]), uintptr_t(g[k]) + size_t(A->n) * (ng == 1 ? 3 : 1) * es};
            if (overlaps(o, gr))
                return EIG3_EINVAL;
        }
    }
    const dim3 grid(unsigned(grid_for(A->n))), block(kBlock);
    auto launch = [&](auto tag) {
        using T = decltype(tag);
        const In9<T> in = inputs_of<T>(A);
        G3<T> gg{{static_cast<const T *>(g[0]), static_cast<const T *>(ng == 3 ? g[1] : nullptr),
                  static_cast<const T *>(ng == 3 ? g[2] : nullptr)}};
        dispatch_sla(A->structure, A->layout, A->accuracy, [&](auto S, auto L, auto Acc) {
            constexpr int KO = S.value == EIG3_GENERAL ? 9 : 6;
            const OutK<T, KO> out = out_slots<T, KO>(outs, nout);
            if (g_layout == EIG3_AOS)
                hipLaunchKernelGGL((k_backward<T, S.value, L.value, EIG3_AOS, Acc.value>), grid, block, 0, stream,
                                   A->n, in, gg, out);
            else
                hipLaunchKernelGGL((k_backward<T, S.value, L.value, EIG3_SOA, Acc.value>), grid, block, 0, stream,
                                   A->n, in, gg, out);
        });
    };
    if (A->dtype == EIG3_F32)
        launch(float{});
    else
        launch(double{});
    return launched();
}

int eig3_mohr_coulomb(const eig3_matrices *sigma, double s_yc, double m, void *f, void *const dfds[9],
                      hipStream_t stream)
{
    int st = check_matrices(sigma);
    if (st != EIG3_OK)
        return st;
    if (!(s_yc > 0.0) || !(m > 0.0) || s_yc > 1e300 || m > 1e300)
        return EIG3_EINVAL;
    if (sigma->n == 0)
        return EIG3_OK;
    if (f == nullptr)
        return EIG3_EINVAL;
    const int K = sigma->structure == EIG3_GENERAL ? 9 : 6;
    const bool grad = dfds != nullptr;
    const int nout = grad ? (sigma->layout == EIG3_SOA ? K : 1) : 0;
    void *outs[10];
    outs[0] = f;
    for (int k = 0; k < nout; ++k)
        outs[1 + k] = dfds[k];
    // f holds n values; every gradient array n (SoA) or n*K (AoS) values
    if ((st = check_outputs(sigma, outs, 1, size_t(sigma->n))) != EIG3_OK)
        return st;
    if (grad) {
        if ((st = check_outputs(sigma, outs + 1, nout, size_t(sigma->n) * (nout == 1 ? K : 1))) != EIG3_OK)
            return st;
        const size_t es = elem_size(sigma->dtype);
        const Range fr{uintptr_t(f), uintptr_t(f) + size_t(sigma->n) * es};
        for (int k = 0; k < nout; ++k) {
            const Range o{uintptr_t(outs[1 + k]), uintptr_t(outs[1 + k]) + size_t(sigma->n) * (nout == 1 ? K : 1) * es};
            if (overlaps(o, fr))
                return EIG3_EINVAL;
        }
    }
    const double cf = (m + 1.0) / (2.0 * s_yc);
    const double Kc = (m - 1.0) / (m + 1.0);
    const dim3 grid(unsigned(grid_for(sigma->n))), block(kBlock);
    auto launch = [&](auto tag) {
        using T = decltype(tag);
        const In9<T> in = inputs_of<T>(sigma);
        T *fo = static_cast<T *>(f);
        dispatch_sla4(sigma->structure, sigma->layout, sigma->accuracy, [&](auto S, auto L, auto Acc) {
            constexpr int KS = S.value == EIG3_GENERAL ? 9 : 6;
            if (grad) {
                const OutK<T, KS> out = out_slots<T, KS>(outs + 1, nout);
                hipLaunchKernelGGL((k_mohr_coulomb<T, S.value, L.value, Acc.value, true>), grid, block, 0, stream,
                                   sigma->n, in, cf, Kc, fo, out);
            } else {
                const OutK<T, 1> out = out_slots<T, 1>(outs, 1); // f is the only slot
                hipLaunchKernelGGL((k_mohr_coulomb<T, S.value, L.value, Acc.value, false>), grid, block, 0,
                                   stream, sigma->n, in, cf, Kc, fo, out);
            }
        });
    };
    if (sigma->dtype == EIG3_F32)
        launch(float{});
    else
        launch(double{});
    return launched();
}

int eig3_eigenprojectors(const eig3_matrices *A, int32_t out_layout, void *const E[27], hipStream_t stream)
{
    int st = check_matrices(A);
    if (st != EIG3_OK)
        return st;
    if (E == nullptr || !valid_enum(out_layout, 1))
        return EIG3_EINVAL;
    if (A->n == 0)
        return EIG3_OK;
    const int K = A->structure == EIG3_GENERAL ? 9 : 6;
    const int nout = out_layout == EIG3_SOA ? 3 * K : 1;
    void *outs[27];
    for (int k = 0; k < nout; ++k)
        outs[k] = E[k];
    if ((st = check_outputs(A, outs, nout, size_t(A->n) * (nout == 1 ? 3 * K : 1))) != EIG3_OK)
        return st;
    const dim3 grid(unsigned(grid_for(A->n))), block(kBlock);
    auto launch = [&](auto tag) {
        using T = decltype(tag);
        const In9<T> in = inputs_of<T>(A);
        dispatch_sla4(A->structure, A->layout, A->accuracy, [&](auto S, auto L, auto Acc) {
            constexpr int KO = S.value == EIG3_GENERAL ? 27 : 18;
            const OutK<T, KO> out = out_slots<T, KO>(outs, nout);
            if (out_layout == EIG3_AOS)
                hipLaunchKernelGGL((k_eigenprojectors<T, S.value, L.value, EIG3_AOS, Acc.value>), grid, block, 0,
                                   stream, A->n, in, out);
            else
                hipLaunchKernelGGL((k_eigenprojectors<T, S.value, L.value, EIG3_SOA, Acc.value>), grid, block, 0,
                                   stream, A->n, in, out);
        });
    };
    if (A->dtype == EIG3_F32)
        launch(float{});
    else
        launch(double{});
    return launched();
}

} // extern "C"
