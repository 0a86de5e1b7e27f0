// engine.hpp -- device building blocks shared by the gfx950 kernels.
//
// The Pauli coefficients of a 2^n x 2^n matrix A are, for every X-pattern x
// and Z-pattern z (qubit q = bit q; letter (x_q, z_q) = (0,0) I, (1,0) X,
// (1,1) Y, (0,1) Z),
//
//     c[x][z] = 2^-n * i^popcount(x & z) * sum_k (-1)^popcount(z & k) * A[k][k ^ x].
//
// This is the definition c_P = 2^-n Tr(P A) (paper, Sec. II-A) with P's single
// nonzero per row (Sec. II-A, first optimization of the trace) written in
// closed form: P[r][r ^ x] = (-i)^popcount(x & z) * (-1)^popcount(z & r), and
// the Y phase P = (-i)^{n_Y} P~ of Sec. II-B collected into one power of i.
// For each x the inner sum is a length-2^n Walsh-Hadamard transform (WHT)
// of the generalised diagonal d_x[k] = A[k][k ^ x].
//
// Kernels here hold a small set of vectors in LDS and run the WHT as rounds:
// each round applies the radix-2 butterflies of up to 5 consecutive index
// bits in registers (a radix-16 or radix-32 step per work item), reading its operands
// from a source functor and writing results to a destination functor (global
// gather, LDS, or global store with the fused phase and scale).
//
// Floating point: butterflies are plain adds and subtracts, one radix-2 stage
// per index bit, so the network is invariant under XOR-permuting its input
// (fl(b + a) = fl(a + b), fl(b - a) = -fl(a - b)).  For a Hermitian A this
// makes the imaginary part of every phased coefficient exactly zero.  The
// phase is a swap/negation and the scale an exact power of two.
#pragma once

#include "internal.hpp"
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptd {

template <class V>
struct alignas(2 * sizeof(V)) cplx {
    V re, im;
};

// In-place radix-2^NB WHT of (re[m], im[m]), m < 2^NB, natural order.
template <class V, int NB>
__device__ __forceinline__ void wht_reg(V* re, V* im)
{
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int m = 0; m < (1 << NB); ++m) {
            if (!(m & (1 << b))) {
                const int p = m | (1 << b);
                const V ur = re[m], ui = im[m], vr = re[p], vi = im[p];
                re[m] = ur + vr;
                im[m] = ui + vi;
                re[p] = ur - vr;
                im[p] = ui - vi;
            }
        }
    }
}

// v with NB zero bits inserted at bit position B0.
__device__ __forceinline__ int insert_zero_bits(int v, int b0, int nb)
{
    const int low = v & ((1 << b0) - 1);
    return low | ((v >> b0) << (b0 + nb));
}

// (re, im) *= i^p for p in 0..3 (swaps and negations only: exact).
template <class V>
__device__ __forceinline__ void mul_ipow(int p, V& re, V& im)
{
    const V r = re, i = im;
    const V nr = (p & 1) ? i : r;
    const V ni = (p & 1) ? r : i;
    re = (p == 1 || p == 2) ? -nr : nr;
    im = (p >= 2) ? -ni : ni;
}

// One WHT round over index bits [B0, B0 + NB) of 2^LOG_NV vectors of length
// 2^LOG_L.  Work items enumerate (vector, position with the round bits
// cleared); VEC_FAST puts the vector index in the fastest-varying lanes (so
// lanes of one wave read one matrix row in a gather), otherwise the free
// position bits vary fastest (contiguous positions per wave).
template <class V, int LOG_NV, int LOG_L, int B0, int NB, int NTHR, bool VEC_FAST, class Src, class Dst>
__device__ __forceinline__ void wht_round(const Src& src, const Dst& dst)
{
    static_assert(NB >= 1 && NB <= 5, "radix 2..32 per round");
    static_assert(B0 + NB <= LOG_L, "round bits inside the vector");
    constexpr int R = 1 << NB;
    constexpr int NITEMS = 1 << (LOG_NV + LOG_L - NB);
    for (int it = threadIdx.x; it < NITEMS; it += NTHR) {
        int vec, base;
        if constexpr (VEC_FAST) {
            vec = it & ((1 << LOG_NV) - 1);
            base = insert_zero_bits(it >> LOG_NV, B0, NB);
        } else {
            constexpr int PB = LOG_L - NB;
            base = insert_zero_bits(it & ((1 << PB) - 1), B0, NB);
            vec = it >> PB;
        }
        V re[R], im[R];
#pragma unroll
        for (int m = 0; m < R; ++m) src(vec, base + (m << B0), re[m], im[m]);
        wht_reg<V, NB>(re, im);
#pragma unroll
        for (int m = 0; m < R; ++m) dst(vec, base + (m << B0), re[m], im[m]);
    }
}

// LDS vector storage: element (vec, pos) at p[vec * (2^LOG_L + 1) + pos].  The
// one-element pad keeps lanes that differ in vec on different banks.
template <class V, int LOG_L>
struct LdsVecs {
    static constexpr int PITCH = (1 << LOG_L) + 1;
    cplx<V>* p;
    __device__ __forceinline__ void operator()(int vec, int pos, V& re, V& im) const
    {
        const cplx<V> v = p[vec * PITCH + pos];
        re = v.re;
        im = v.im;
    }
};

template <class V, int LOG_L>
struct LdsVecsW {
    static constexpr int PITCH = (1 << LOG_L) + 1;
    cplx<V>* p;
    __device__ __forceinline__ void operator()(int vec, int pos, V re, V im) const
    {
        cplx<V> v;
        v.re = re;
        v.im = im;
        p[vec * PITCH + pos] = v;
    }
};

// d_x[k] = A[k][k ^ x] from the source kind SRC (internal.hpp).
template <class V, int SRC>
__device__ __forceinline__ cplx<V> source_entry(const cplx<V>* __restrict__ A, int64_t lda, int logn, int k, int col)
{
    if constexpr (SRC == SRC_TOEPLITZ) {
        return A[col - k + ((1 << logn) - 1)];
    } else if constexpr (SRC == SRC_PURE) {
        const cplx<V> a = A[k], b = A[col];
        cplx<V> v;  // a * conj(b), two products and one sum per part
        v.re = a.re * b.re + a.im * b.im;
        v.im = a.im * b.re - a.re * b.im;
        return v;
    } else if constexpr (SRC == SRC_LOWRANK) {
        // sum over the factor's columns j of U[k][j] conj(U[col][j]), in
        // ascending j; the mirror entry (col, k) takes the same products in
        // the same order, so the matrix is Hermitian bit for bit
        const int rank = (int)(lda & 63);
        const int64_t ld = lda >> 6;
        const cplx<V>* a = A + (int64_t)k * ld;
        const cplx<V>* b = A + (int64_t)col * ld;
        cplx<V> v;
        v.re = (V)0;
        v.im = (V)0;
#pragma unroll 4
        for (int j = 0; j < rank; ++j) {
            const cplx<V> u = a[j], w = b[j];
            v.re += u.re * w.re + u.im * w.im;
            v.im += u.im * w.re - u.re * w.im;
        }
        return v;
    } else if constexpr (SRC == SRC_LOWRANK_T) {
        // the same products in the same order as SRC_LOWRANK, from the
        // transposed factor: lanes over k read consecutive values
        const int rank = (int)(lda & 63);
        const int64_t N = (int64_t)1 << logn;
        cplx<V> v;
        v.re = (V)0;
        v.im = (V)0;
#pragma unroll 4
        for (int j = 0; j < rank; ++j) {
            const cplx<V> u = A[j * N + k], w = A[j * N + col];
            v.re += u.re * w.re + u.im * w.im;
            v.im += u.im * w.re - u.re * w.im;
        }
        return v;
    } else {
        return A[(int64_t)k * lda + col];
    }
}

template <class V>
__device__ __forceinline__ V exp2_neg(int n)
{
    // 2^-n exactly (n <= 30 keeps it a normal number in both precisions)
    return (V)1 / (V)(1u << n);
}

}  // namespace ptd

// ---------------------------------------------------------------------------
// Compensated butterflies (complex64 accuracy mode).  Every value carries a
// (hi, lo) pair; each radix-2 step computes hi with the error-free TwoSum
// transformation (Knuth) and adds the rounding error to the low parts, so a
// run of stages loses no more than the final rounding of hi + lo.  TwoSum is
// commutative and odd, which keeps the XOR-permutation symmetry of the plain
// network (exactly real coefficients for Hermitian input).

namespace ptd {

template <class V>
__device__ __forceinline__ void two_sum(V a, V b, V& s, V& e)
{
    s = a + b;
    const V bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// In-place radix-2^NB WHT of compensated pairs.
template <class V, int NB>
__device__ __forceinline__ void wht_reg_comp(V* rh, V* rl, V* ih, V* il)
{
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int m = 0; m < (1 << NB); ++m) {
            if (!(m & (1 << b))) {
                const int p = m | (1 << b);
                V s, e, d, f;
                two_sum(rh[m], rh[p], s, e);
                two_sum(rh[m], -rh[p], d, f);
                const V sl = rl[m] + rl[p] + e, dl = rl[m] - rl[p] + f;
                rh[m] = s;
                rl[m] = sl;
                rh[p] = d;
                rl[p] = dl;
                two_sum(ih[m], ih[p], s, e);
                two_sum(ih[m], -ih[p], d, f);
                const V tl = il[m] + il[p] + e, ul = il[m] - il[p] + f;
                ih[m] = s;
                il[m] = tl;
                ih[p] = d;
                il[p] = ul;
            }
        }
    }
    // renormalise: hi takes the rounded sum, lo the remainder
#pragma unroll
    for (int m = 0; m < (1 << NB); ++m) {
        V s, e;
        two_sum(rh[m], rl[m], s, e);
        rh[m] = s;
        rl[m] = e;
        two_sum(ih[m], il[m], s, e);
        ih[m] = s;
        il[m] = e;
    }
}

// Compensated round: like wht_round, with src(vec, pos, rh, rl, ih, il) and
// dst(vec, pos, rh, rl, ih, il).
template <class V, int LOG_NV, int LOG_L, int B0, int NB, int NTHR, bool VEC_FAST, class Src, class Dst>
__device__ __forceinline__ void wht_round_comp(const Src& src, const Dst& dst)
{
    static_assert(NB >= 1 && NB <= 4, "radix 2..16 per round");
    constexpr int R = 1 << NB;
    constexpr int NITEMS = 1 << (LOG_NV + LOG_L - NB);
    for (int it = threadIdx.x; it < NITEMS; it += NTHR) {
        int vec, base;
        if constexpr (VEC_FAST) {
            vec = it & ((1 << LOG_NV) - 1);
            base = insert_zero_bits(it >> LOG_NV, B0, NB);
        } else {
            constexpr int PB = LOG_L - NB;
            base = insert_zero_bits(it & ((1 << PB) - 1), B0, NB);
            vec = it >> PB;
        }
        V rh[R], rl[R], ih[R], il[R];
#pragma unroll
        for (int m = 0; m < R; ++m) src(vec, base + (m << B0), rh[m], rl[m], ih[m], il[m]);
        wht_reg_comp<V, NB>(rh, rl, ih, il);
#pragma unroll
        for (int m = 0; m < R; ++m) dst(vec, base + (m << B0), rh[m], rl[m], ih[m], il[m]);
    }
}

// LDS storage of compensated pairs: hi and lo in two arrays of the LdsVecs
// layout.
template <class V, int LOG_L>
struct LdsVecsComp {
    static constexpr int PITCH = (1 << LOG_L) + 1;
    cplx<V>* hi;
    cplx<V>* lo;
    __device__ __forceinline__ void operator()(int vec, int pos, V& rh, V& rl, V& ih, V& il) const
    {
        const cplx<V> a = hi[vec * PITCH + pos], b = lo[vec * PITCH + pos];
        rh = a.re;
        ih = a.im;
        rl = b.re;
        il = b.im;
    }
};

template <class V, int LOG_L>
struct LdsVecsCompW {
    static constexpr int PITCH = (1 << LOG_L) + 1;
    cplx<V>* hi;
    cplx<V>* lo;
    __device__ __forceinline__ void operator()(int vec, int pos, V rh, V rl, V ih, V il) const
    {
        cplx<V> a, b;
        a.re = rh;
        a.im = ih;
        b.re = rl;
        b.im = il;
        hi[vec * PITCH + pos] = a;
        lo[vec * PITCH + pos] = b;
    }
};

}  // namespace ptd
