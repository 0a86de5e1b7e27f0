// group.hpp -- single-pass decomposition of one X-pattern group (n <= 10).
//
// One workgroup owns the T = 2^LOGT consecutive X-patterns x = g*T + x_lo of
// a 2^LOGN x 2^LOGN matrix.  For row k those patterns read the T contiguous
// columns ((k >> LOGT) ^ g) * T + [0, T), one 128-byte segment per row for
// T = 16 complex64 / 8 complex128.  The whole band (2^LOGN rows x T) sits in
// LDS, the length-2^LOGN Walsh-Hadamard transforms run as radix-16 rounds
// (engine.hpp), and T full output rows are written once with the phase
// i^popcount(x&z) and the 2^-n scale applied.  Reconstruction runs the same
// rounds in the other order after the inverse phase (-i)^popcount(x&z) and
// scatters d_x back to A[k][k ^ x].
#pragma once

#include "engine.hpp"

namespace ptd {

constexpr int GROUP_THREADS = 512;

template <class V>
constexpr int group_logt(int logn)
{
    // 128-byte row segments: 16 complex64 or 8 complex128
    return logn < (sizeof(V) == 4 ? 4 : 3) ? logn : (sizeof(V) == 4 ? 4 : 3);
}


// LDS elements the group routines need for a 2^logn matrix.
template <class V>
constexpr int group_lds_elems(int logn)
{
    return (1 << group_logt<V>(logn)) * ((1 << logn) + 1);
}

// First radix-16 round (index bits 0..3) for Hermitian input, group base
// xg with xh = xg >> 4 != 0.  Position blocks B and B ^ xh of 16 rows hold
// mirror entries, d_x[k ^ x] = conj(d_x[k]), so for c = x & 15 the round
// outputs obey W0[B ^ xh][u] = (-1)^popcount(u & c) conj(W0[B][u]) exactly
// (each radix-2 stage only swaps and negates under an XOR-permuted input).
// Only the blocks whose bit hb (the top bit of xh) is clear are gathered;
// each writes its own outputs and its mirror block's.
template <class V, int LOGN, int LOGT, class G, class W>
__device__ __forceinline__ void first_round_hermitian(const G& gather, const W& lw, uint32_t xg)
{
    constexpr int NT = GROUP_THREADS;
    constexpr int NITEMS = (1 << LOGT) << (LOGN - 5);  // half of the (vector, block) pairs
    const int xh = (int)(xg >> 4);
    const int hb = 31 - __clz(xh);
    for (int it = threadIdx.x; it < NITEMS; it += NT) {
        const int vec = it & ((1 << LOGT) - 1);
        const int base = insert_zero_bits(it >> LOGT, hb, 1) << 4;
        const int c = (int)((xg | (uint32_t)vec) & 15u);
        const int basep = base ^ (xh << 4);
        V re[16], im[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) gather(vec, base + m, re[m], im[m]);
        wht_reg<V, 4>(re, im);
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            lw(vec, base + u, re[u], im[u]);
            const bool s = __popc(u & c) & 1;
            lw(vec, basep + u, s ? -re[u] : re[u], s ? im[u] : -im[u]);
        }
    }
}

template <class V, int LOGN, int LOGT, bool REAL_OUT>
__device__ __forceinline__ void group_fwd(const cplx<V>* __restrict__ A, int64_t lda, void* __restrict__ out,
                                          int64_t ldo, int g, cplx<V>* lds)
{
    constexpr int NT = GROUP_THREADS;
    const uint32_t xg = (uint32_t)g << LOGT;
    const V scale = exp2_neg<V>(LOGN);
    auto gather = [&](int vec, int pos, V& re, V& im) {
        const cplx<V> v = A[(int64_t)pos * lda + (pos ^ (int)(xg | vec))];
        re = v.re;
        im = v.im;
    };
    auto store = [&](int vec, int pos, V re, V im) {
        const uint32_t x = xg | (uint32_t)vec;
        mul_ipow(__popc(x & (uint32_t)pos) & 3, re, im);
        re *= scale;
        im *= scale;
        if constexpr (REAL_OUT) {
            ((V*)out)[(int64_t)x * ldo + pos] = re;
        } else {
            cplx<V> c;
            c.re = re;
            c.im = im;
            ((cplx<V>*)out)[(int64_t)x * ldo + pos] = c;
        }
    };
    LdsVecs<V, LOGN> lr{lds};
    LdsVecsW<V, LOGN> lw{lds};
    if constexpr (LOGN <= 4) {
        wht_round<V, LOGT, LOGN, 0, LOGN, NT, true>(gather, store);
    } else {
        if constexpr (REAL_OUT) {
            if ((xg >> 4) != 0)
                first_round_hermitian<V, LOGN, LOGT>(gather, lw, xg);
            else
                wht_round<V, LOGT, LOGN, 0, 4, NT, true>(gather, lw);
        } else {
            wht_round<V, LOGT, LOGN, 0, 4, NT, true>(gather, lw);
        }
        __syncthreads();
        if constexpr (LOGN <= 8) {
            wht_round<V, LOGT, LOGN, 4, LOGN - 4, NT, false>(lr, store);
        } else {
            wht_round<V, LOGT, LOGN, 4, 4, NT, false>(lr, lw);
            __syncthreads();
            wht_round<V, LOGT, LOGN, 8, LOGN - 8, NT, false>(lr, store);
        }
    }
}

template <class V, int LOGN, int LOGT, bool REAL_IN>
__device__ __forceinline__ void group_rec(const void* __restrict__ coeff, cplx<V>* __restrict__ A, int64_t lda,
                                          V scale, int g, cplx<V>* lds)
{
    constexpr int NT = GROUP_THREADS;
    const uint32_t xg = (uint32_t)g << LOGT;
    auto load = [&](int vec, int pos, V& re, V& im) {
        const uint32_t x = xg | (uint32_t)vec;
        const int64_t o = (int64_t)x * (1 << LOGN) + pos;
        if constexpr (REAL_IN) {
            re = ((const V*)coeff)[o];
            im = (V)0;
        } else {
            const cplx<V> c = ((const cplx<V>*)coeff)[o];
            re = c.re;
            im = c.im;
        }
        // (-i)^p = i^{-p}
        mul_ipow((4 - (__popc(x & (uint32_t)pos) & 3)) & 3, re, im);
    };
    auto scatter = [&](int vec, int pos, V re, V im) {
        cplx<V> c;
        c.re = re * scale;
        c.im = im * scale;
        A[(int64_t)pos * lda + (pos ^ (int)(xg | vec))] = c;
    };
    LdsVecs<V, LOGN> lr{lds};
    LdsVecsW<V, LOGN> lw{lds};
    if constexpr (LOGN <= 4) {
        wht_round<V, LOGT, LOGN, 0, LOGN, NT, true>(load, scatter);
    } else if constexpr (LOGN <= 8) {
        wht_round<V, LOGT, LOGN, LOGN - 4, 4, NT, false>(load, lw);
        __syncthreads();
        wht_round<V, LOGT, LOGN, 0, LOGN - 4, NT, true>(lr, scatter);
    } else {
        wht_round<V, LOGT, LOGN, LOGN - 4, 4, NT, false>(load, lw);
        __syncthreads();
        wht_round<V, LOGT, LOGN, LOGN - 8, 4, NT, false>(lr, lw);
        __syncthreads();
        wht_round<V, LOGT, LOGN, 0, LOGN - 8, NT, true>(lr, scatter);
    }
}

}  // namespace ptd
