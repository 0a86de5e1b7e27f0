// group.hpp -- single-pass decomposition of one X-pattern group (n <= 10).
//
// One workgroup owns the T = 2^LOGT consecutive X-patterns x = g*T + x_lo of
// a 2^LOGN x 2^LOGN matrix.  For row k those patterns read the T contiguous
// columns ((k >> LOGT) ^ g) * T + [0, T), one 128-byte segment per row for
// T = 16 complex64 / 8 complex128.  The whole band (2^LOGN rows x T) sits in
// LDS, the length-2^LOGN Walsh-Hadamard transforms run as rounds of up to
// RMAX index bits (radix 16 or 32, engine.hpp), and T full output rows are
// written once with the phase i^popcount(x&z) and the 2^-n scale applied.
// Reconstruction runs rounds of 4 bits in the other order after the inverse
// phase (-i)^popcount(x&z) and scatters d_x back to A[k][k ^ x].
//
// A plan (group_plan_nt / group_plan_rmax) picks the workgroup size (512 or
// 1024 threads) and the widest round (4 or 5 bits; 5 for complex64 only:
// 32 complex doubles per work item would not fit the register budget).
#pragma once

#include "engine.hpp"

namespace ptd {

constexpr int GROUP_THREADS = 512;  // default workgroup size

// plan bits: 1 = 1024 threads per workgroup, 2 = rounds of up to 5 bits
constexpr int group_plan_nt(int plan) { return (plan & 1) ? 1024 : 512; }
constexpr int group_plan_rmax(int plan) { return (plan & 2) ? 5 : 4; }

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

// First round (index bits 0..NB0-1) for Hermitian input, group base xg with
// xh = xg >> NB0 != 0 (NB0 >= LOGT, so xh is the same for every x of the
// group).  Position blocks B and B ^ xh of 2^NB0 rows hold mirror entries,
// d_x[k ^ x] = conj(d_x[k]), so for c = x & (2^NB0 - 1) the round outputs
// obey W0[B ^ xh][u] = (-1)^popcount(u & c) conj(W0[B][u]) exactly (each
// radix-2 stage only swaps and negates under an XOR-permuted input).  Only
// the blocks whose bit hb (the top bit of xh) is clear are gathered; each
// writes its own outputs and its mirror block's.
template <class V, int LOGN, int LOGT, int NB0, int NT, class G, class W>
__device__ __forceinline__ void first_round_hermitian(const G& gather, const W& lw, uint32_t xg)
{
    static_assert(NB0 >= LOGT && NB0 < LOGN, "mirror blocks of whole segments");
    constexpr int R = 1 << NB0;
    constexpr int NITEMS = (1 << LOGT) << (LOGN - NB0 - 1);  // half of the (vector, block) pairs
    const int xh = (int)(xg >> NB0);
    const int hb = 31 - __clz(xh);
    for (int it = threadIdx.x; it < NITEMS; it += NT) {
        const int vec = it & ((1 << LOGT) - 1);
        const int base = insert_zero_bits(it >> LOGT, hb, 1) << NB0;
        const int c = (int)((xg | (uint32_t)vec) & (uint32_t)(R - 1));
        const int basep = base ^ (xh << NB0);
        V re[R], im[R];
#pragma unroll
        for (int m = 0; m < R; ++m) gather(vec, base + m, re[m], im[m]);
        wht_reg<V, NB0>(re, im);
#pragma unroll
        for (int u = 0; u < R; ++u) {
            lw(vec, base + u, re[u], im[u]);
            const bool s = __popc(u & c) & 1;
            lw(vec, basep + u, s ? -re[u] : re[u], s ? im[u] : -im[u]);
        }
    }
}

// Rounds over bits [B0, LOGN) of the group's vectors, RMAX bits at most
// each: the first gathers (lanes over vectors), the last stores (lanes over
// positions), LDS in between.
template <class V, int LOGN, int LOGT, bool REAL_OUT, int NT, int RMAX, int B0, class G, class St>
__device__ __forceinline__ void group_rounds(const G& gather, const St& store, cplx<V>* lds, uint32_t xg)
{
    constexpr int NB = (LOGN - B0) < RMAX ? (LOGN - B0) : RMAX;
    constexpr bool FIRST = B0 == 0, LAST = B0 + NB == LOGN;
    LdsVecs<V, LOGN> lr{lds};
    LdsVecsW<V, LOGN> lw{lds};
    if constexpr (FIRST && LAST) {
        wht_round<V, LOGT, LOGN, B0, NB, NT, true>(gather, store);
    } else if constexpr (FIRST) {
        if constexpr (REAL_OUT && NB >= LOGT) {
            if ((xg >> NB) != 0)
                first_round_hermitian<V, LOGN, LOGT, NB, NT>(gather, lw, xg);
            else
                wht_round<V, LOGT, LOGN, B0, NB, NT, true>(gather, lw);
        } else {
            wht_round<V, LOGT, LOGN, B0, NB, NT, true>(gather, lw);
        }
        __syncthreads();
        group_rounds<V, LOGN, LOGT, REAL_OUT, NT, RMAX, B0 + NB>(gather, store, lds, xg);
    } else if constexpr (LAST) {
        wht_round<V, LOGT, LOGN, B0, NB, NT, false>(lr, store);
    } else {
        wht_round<V, LOGT, LOGN, B0, NB, NT, false>(lr, lw);
        __syncthreads();
        group_rounds<V, LOGN, LOGT, REAL_OUT, NT, RMAX, B0 + NB>(gather, store, lds, xg);
    }
}

// SRC: where the matrix entries come from (engine.hpp, source_entry); for the
// matrix-free kinds A holds their defining vector and lda is unused.
template <class V, int LOGN, int LOGT, bool REAL_OUT, int NT = GROUP_THREADS, int RMAX = 4, int SRC = SRC_MATRIX>
__device__ __forceinline__ void group_fwd(const cplx<V>* __restrict__ A, int64_t lda, void* __restrict__ out,
                                          int64_t ldo, int g, cplx<V>* lds, V scale)
{
    // scale: 2^-n, or 1 for the unscaled traces Tr(P A) (an exact power of two)
    static_assert(RMAX == 4 || (RMAX == 5 && sizeof(V) == 4), "radix 32 for complex64 only");
    const uint32_t xg = (uint32_t)g << LOGT;
    auto gather = [&](int vec, int pos, V& re, V& im) {
        const cplx<V> v = source_entry<V, SRC>(A, lda, LOGN, pos, pos ^ (int)(xg | vec));
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
    group_rounds<V, LOGN, LOGT, REAL_OUT, NT, RMAX, 0>(gather, store, lds, xg);
}

template <class V, int LOGN, int LOGT, bool REAL_IN, int NT = GROUP_THREADS>
__device__ __forceinline__ void group_rec(const void* __restrict__ coeff, cplx<V>* __restrict__ A, int64_t lda,
                                          V scale, int g, cplx<V>* lds)
{
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
