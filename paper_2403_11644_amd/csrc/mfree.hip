// mfree.hip -- dense decomposition of a matrix-free input (a Toeplitz matrix
// given by its defining entries, or a density matrix given by a state vector
// or a low-rank factor)
// for n >= 11: one workgroup per X-pattern.
//
// A matrix-free source costs no HBM read: its defining vector (at most
// 2^(n+1) complex values) or low-rank factor stays in L2.  So the whole length-2^n transform of
// one X-pattern runs in one workgroup, out of LDS, and the output row is
// written once with coalesced stores; the only HBM traffic is the output.
// (The single-launch schedule for stored matrices exchanges partial
// transforms through the memory side, because a group's band of a stored
// matrix must be read in whole 128-byte segments and does not fit one CU.)
//
// LDS holds 2^m values of the row: m = n while 2^n values fit in 128 KiB
// (n <= 13 complex128, n <= 14 complex64).  One size beyond (n = 14
// complex128, n = 15 complex64) the workgroup transforms the two halves
// k < 2^(n-1) and k >= 2^(n-1) one after the other, runs each half's last
// round into registers, and finishes there with the butterfly over the top
// bit.
//
// For a Toeplitz source every path applies the radix-2 stages in ascending
// bit order with the same additions as the kernels for stored matrices, so a
// matrix-free call gives the bits of a dense call on the materialised
// matrix.  The density-matrix sources take one real transform per row (real
// rows below): the same coefficients within rounding, half the transform
// work and half the LDS per row.
//
// The kernels are bound by LDS traffic as much as by the output writes, so
// the two-halves kernel keeps each half's last round in registers (the
// halves join there without another LDS pass).  Measured on MI355X at
// n = 14: 0.97 ms complex128 (4.4 TB/s of output writes), 0.54 ms
// complex64; n = 15 complex64 2.11 ms.  Gathering with 8 or 16 loads in
// flight per thread, 256 or 1024 threads, or radix 8 rounds changed it by
// -5% to +35%; the single-launch schedule of stored matrices took 1.64 ms.
#include "engine.hpp"
#include "internal.hpp"

namespace ptd {

namespace {

// Widest round: radix 32 for complex64, radix 16 for complex128 (radix 32
// measured no faster for the complex128 row at n = 13, and does not fit
// beside the register-held half of the two-halves kernel).
template <class V>
constexpr int mf_rmax()
{
    return sizeof(V) == 4 ? 5 : 4;
}

// workgroup size of the whole-row kernel: one radix-16 item per thread
constexpr int mf_threads(int logn)
{
    return (1 << logn) / 16 < 64 ? 64 : ((1 << logn) / 16 > 1024 ? 1024 : (1 << logn) / 16);
}

constexpr int MF_HALF_THREADS = 512;

// LDS slot of row position p: one pad element after every 2^RMAX, the
// positions one thread owns in the first round, so that its lanes read
// conflict-free (32 complex64 lanes or 16 complex128 lanes fill the 64
// banks once).  A pad after every 32 complex128 values measured two bank
// conflict cycles per LDS instruction.
template <class V>
__device__ __forceinline__ int mf_slot(int p)
{
    return p + (p >> mf_rmax<V>());
}
template <class V>
constexpr int mf_lds_elems(int logm)
{
    return (1 << logm) + (1 << (logm - mf_rmax<V>()));
}

template <class V>
struct MfRead {
    cplx<V>* p;
    __device__ __forceinline__ void operator()(int, int pos, V& re, V& im) const
    {
        const cplx<V> v = p[mf_slot<V>(pos)];
        re = v.re;
        im = v.im;
    }
};

template <class V>
struct MfWrite {
    cplx<V>* p;
    __device__ __forceinline__ void operator()(int, int pos, V re, V im) const
    {
        cplx<V> v;
        v.re = re;
        v.im = im;
        p[mf_slot<V>(pos)] = v;
    }
};

// d_x[kb + p] for the 2^LM positions p, into LDS; consecutive lanes take
// consecutive positions, so the source reads of a wave stay within a few
// cache lines
template <class V, int LM, int NT, int SRC>
__device__ __forceinline__ void mf_gather(const cplx<V>* __restrict__ src, int64_t ld, int logn, uint32_t x, int kb,
                                          cplx<V>* lds)
{
#pragma unroll 4
    for (int p = threadIdx.x; p < (1 << LM); p += NT) {
        const int k = kb + p;
        lds[mf_slot<V>(p)] = source_entry<V, SRC>(src, ld, logn, k, k ^ (int)x);
    }
}

// Rounds over bits [B0, LM) of the LDS row, RMAX bits at most each, in
// ascending bit order; the last round hands its values to `last`.
template <class V, int LM, int NT, int RMAX, int B0, class Last>
__device__ __forceinline__ void mf_rounds(cplx<V>* lds, const Last& last)
{
    constexpr int NB = (LM - B0) < RMAX ? (LM - B0) : RMAX;
    MfRead<V> rd{lds};
    if constexpr (B0 + NB == LM) {
        wht_round<V, 0, LM, B0, NB, NT, false>(rd, last);
    } else {
        wht_round<V, 0, LM, B0, NB, NT, false>(rd, MfWrite<V>{lds});
        __syncthreads();
        mf_rounds<V, LM, NT, RMAX, B0 + NB>(lds, last);
    }
}

// Rounds over bits [B0, END) of the LDS row in place, then a barrier each.
template <class V, int LM, int NT, int RMAX, int B0, int END>
__device__ __forceinline__ void mf_rounds_to(cplx<V>* lds)
{
    if constexpr (B0 < END) {
        constexpr int NB = (END - B0) < RMAX ? (END - B0) : RMAX;
        wht_round<V, 0, LM, B0, NB, NT, false>(MfRead<V>{lds}, MfWrite<V>{lds});
        __syncthreads();
        mf_rounds_to<V, LM, NT, RMAX, B0 + NB, END>(lds);
    }
}

// The last round, over bits [B0, LM), kept in registers: thread t holds
// positions t + NT i + (m << B0) for i < ITER and m < R.
template <class V, int LM, int NT, int B0>
struct MfLast {
    static constexpr int NB = LM - B0, R = 1 << NB, ITER = (1 << B0) / NT;
    static_assert(ITER >= 1 && ITER * NT == (1 << B0), "whole items per thread");
    V re[ITER][R], im[ITER][R];
    __device__ __forceinline__ void run(const cplx<V>* lds)
    {
#pragma unroll
        for (int i = 0; i < ITER; ++i) {
            const int base = (int)threadIdx.x + NT * i;
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const cplx<V> v = lds[mf_slot<V>(base + (m << B0))];
                re[i][m] = v.re;
                im[i][m] = v.im;
            }
            wht_reg<V, NB>(re[i], im[i]);
        }
    }
};

template <class V, bool REAL_OUT>
__device__ __forceinline__ void mf_store(void* __restrict__ out, int logn, uint32_t x, uint32_t z, V re, V im,
                                         V scale)
{
    mul_ipow(__popc(x & z) & 3, re, im);
    re *= scale;
    im *= scale;
    const int64_t o = ((int64_t)x << logn) + z;
    if constexpr (REAL_OUT) {
        __builtin_nontemporal_store(re, (V*)out + o);
    } else {
        typedef V v2 __attribute__((ext_vector_type(2)));
        v2 v;
        v.x = re;
        v.y = im;
        __builtin_nontemporal_store(v, (v2*)out + o);
    }
}

template <class V, int LOGN, bool REAL_OUT, int SRC>
__global__ __launch_bounds__(mf_threads(LOGN)) void k_mfree_row(const cplx<V>* __restrict__ src, int64_t ld,
                                                                void* __restrict__ out)
{
    constexpr int NT = mf_threads(LOGN);
    __shared__ cplx<V> lds[mf_lds_elems<V>(LOGN)];
    const uint32_t x = blockIdx.x;
    const V scale = exp2_neg<V>(LOGN);
    mf_gather<V, LOGN, NT, SRC>(src, ld, LOGN, x, 0, lds);
    __syncthreads();
    auto store = [&](int, int pos, V re, V im) { mf_store<V, REAL_OUT>(out, LOGN, x, (uint32_t)pos, re, im, scale); };
    mf_rounds<V, LOGN, NT, mf_rmax<V>(), 0>(lds, store);
}

template <class V, int LOGN, bool REAL_OUT, int SRC>
__global__ __launch_bounds__(MF_HALF_THREADS) void k_mfree_halves(const cplx<V>* __restrict__ src, int64_t ld,
                                                                  void* __restrict__ out)
{
    constexpr int LH = LOGN - 1;
    constexpr int NT = MF_HALF_THREADS;
    constexpr int RM = mf_rmax<V>();
    constexpr int LB0 = ((LH - 1) / RM) * RM;  // first bit of the last round
    __shared__ cplx<V> lds[mf_lds_elems<V>(LH)];
    const uint32_t x = blockIdx.x;
    const int t = threadIdx.x;

    // the transform over bits 0 .. LH-1 of half h: the rounds below LB0 in
    // LDS, the last one into registers
    auto half = [&](int h, MfLast<V, LH, NT, LB0>& r) {
        mf_gather<V, LH, NT, SRC>(src, ld, LOGN, x, h << LH, lds);
        __syncthreads();
        mf_rounds_to<V, LH, NT, RM, 0, LB0>(lds);
        r.run(lds);
        __syncthreads();  // every thread has its values before LDS is reused
    };
    MfLast<V, LH, NT, LB0> w0, w1;
    half(0, w0);
    half(1, w1);

    // the top bit: z and z + 2^LH from the two halves' values at z
    const V scale = exp2_neg<V>(LOGN);
#pragma unroll
    for (int i = 0; i < w0.ITER; ++i) {
#pragma unroll
        for (int m = 0; m < w0.R; ++m) {
            const uint32_t z = (uint32_t)(t + NT * i + (m << LB0));
            mf_store<V, REAL_OUT>(out, LOGN, x, z, w0.re[i][m] + w1.re[i][m], w0.im[i][m] + w1.im[i][m], scale);
            mf_store<V, REAL_OUT>(out, LOGN, x, z | (1u << LH), w0.re[i][m] - w1.re[i][m],
                                  w0.im[i][m] - w1.im[i][m], scale);
        }
    }
}

// ---------------------------------------------------------------------------
// Real rows.  Density-matrix sources (a state vector or a low-rank factor)
// are Hermitian by construction, which halves their transform: the row
// transform W = WHT(d_x) of Hermitian input is real where popcount(x & z) is
// even and imaginary where it is odd (pairing k with k ^ x), so the real
// transform of e_x = Re d_x + Im d_x equals the nonzero part of W at every
// z, and the coefficient is s(p) WHT(e_x)[z] 2^-n with p = popcount(x & z)
// mod 4 and s = +1, -1, -1, +1 for p = 0..3.  One workgroup per X-pattern
// holds the real row (or half-row) in LDS, at most 64 KiB, so two
// workgroups share a CU.  The rounds are the complex ones with a reader
// that returns 0 for the imaginary part (folded away) and a writer that
// drops it; the stages keep their ascending order.
template <class V>
__device__ __forceinline__ int mf_slot_r(int p)
{
    return p + (p >> 4);
}
template <class V>
constexpr int mf_lds_r(int logm)
{
    return (1 << logm) + (1 << (logm - 4));
}

template <class V>
struct MfReadR {
    const V* p;
    __device__ __forceinline__ void operator()(int, int pos, V& re, V& im) const
    {
        re = p[mf_slot_r<V>(pos)];
        im = (V)0;
    }
};

template <class V>
struct MfWriteR {
    V* p;
    __device__ __forceinline__ void operator()(int, int pos, V re, V) const { p[mf_slot_r<V>(pos)] = re; }
};

template <class V, int LM, int NT, int RMAX, int B0, int END>
__device__ __forceinline__ void mf_rounds_to_r(V* lds)
{
    if constexpr (B0 < END) {
        constexpr int NB = (END - B0) < RMAX ? (END - B0) : RMAX;
        wht_round<V, 0, LM, B0, NB, NT, false>(MfReadR<V>{lds}, MfWriteR<V>{lds});
        __syncthreads();
        mf_rounds_to_r<V, LM, NT, RMAX, B0 + NB, END>(lds);
    }
}

template <class V, int LM, int NT, int RMAX, int B0, class Last>
__device__ __forceinline__ void mf_rounds_r(V* lds, const Last& last)
{
    constexpr int NB = (LM - B0) < RMAX ? (LM - B0) : RMAX;
    if constexpr (B0 + NB == LM) {
        wht_round<V, 0, LM, B0, NB, NT, false>(MfReadR<V>{lds}, last);
    } else {
        wht_round<V, 0, LM, B0, NB, NT, false>(MfReadR<V>{lds}, MfWriteR<V>{lds});
        __syncthreads();
        mf_rounds_r<V, LM, NT, RMAX, B0 + NB>(lds, last);
    }
}

// e_x[kb + p] = Re d + Im d for the 2^LM positions p
template <class V, int LM, int NT, int SRC>
__device__ __forceinline__ void mf_gather_r(const cplx<V>* __restrict__ src, int64_t ld, int logn, uint32_t x,
                                            int kb, V* lds)
{
#pragma unroll 4
    for (int p = threadIdx.x; p < (1 << LM); p += NT) {
        const int k = kb + p;
        const cplx<V> d = source_entry<V, SRC>(src, ld, logn, k, k ^ (int)x);
        lds[mf_slot_r<V>(p)] = d.re + d.im;
    }
}

// coefficient s(p) v 2^-n of row x at z (imaginary part 0 in complex output)
template <class V, bool REAL_OUT>
__device__ __forceinline__ void mf_store_r(void* __restrict__ out, int logn, uint32_t x, uint32_t z, V v, V scale)
{
    v *= scale;
    if ((__popc(x & z) + 1) & 2) v = -v;
    const int64_t o = ((int64_t)x << logn) + z;
    if constexpr (REAL_OUT) {
        __builtin_nontemporal_store(v, (V*)out + o);
    } else {
        typedef V v2 __attribute__((ext_vector_type(2)));
        v2 a;
        a.x = v;
        a.y = (V)0;
        __builtin_nontemporal_store(a, (v2*)out + o);
    }
}

constexpr int MFR_THREADS = 512;

template <class V, int LOGN, bool REAL_OUT, int SRC>
__global__ __launch_bounds__(MFR_THREADS, 4) void k_mfree_row_r(const cplx<V>* __restrict__ src, int64_t ld,
                                                                void* __restrict__ out)
{
    constexpr int NT = MFR_THREADS;
    __shared__ V lds[mf_lds_r<V>(LOGN)];
    const uint32_t x = blockIdx.x;
    const V scale = exp2_neg<V>(LOGN);
    mf_gather_r<V, LOGN, NT, SRC>(src, ld, LOGN, x, 0, lds);
    __syncthreads();
    auto store = [&](int, int pos, V re, V) { mf_store_r<V, REAL_OUT>(out, LOGN, x, (uint32_t)pos, re, scale); };
    mf_rounds_r<V, LOGN, NT, 4, 0>(lds, store);
}

template <class V, int LM, int NT, int B0>
struct MfLastR {
    static constexpr int NB = LM - B0, R = 1 << NB, ITER = (1 << B0) / NT;
    static_assert(ITER >= 1 && ITER * NT == (1 << B0), "whole items per thread");
    V re[ITER][R];
    __device__ __forceinline__ void run(const V* lds)
    {
#pragma unroll
        for (int i = 0; i < ITER; ++i) {
            const int base = (int)threadIdx.x + NT * i;
            V im[R];
#pragma unroll
            for (int m = 0; m < R; ++m) {
                re[i][m] = lds[mf_slot_r<V>(base + (m << B0))];
                im[m] = (V)0;
            }
            wht_reg<V, NB>(re[i], im);
        }
    }
};

template <class V, int LOGN, bool REAL_OUT, int SRC>
__global__ __launch_bounds__(MFR_THREADS, 4) void k_mfree_halves_r(const cplx<V>* __restrict__ src, int64_t ld,
                                                                   void* __restrict__ out)
{
    constexpr int LH = LOGN - 1;
    constexpr int NT = MFR_THREADS;
    constexpr int LB0 = ((LH - 1) / 4) * 4;  // first bit of the last round
    __shared__ V lds[mf_lds_r<V>(LH)];
    const uint32_t x = blockIdx.x;
    const int t = threadIdx.x;
    auto half = [&](int h, MfLastR<V, LH, NT, LB0>& r) {
        mf_gather_r<V, LH, NT, SRC>(src, ld, LOGN, x, h << LH, lds);
        __syncthreads();
        mf_rounds_to_r<V, LH, NT, 4, 0, LB0>(lds);
        r.run(lds);
        __syncthreads();
    };
    MfLastR<V, LH, NT, LB0> w0, w1;
    half(0, w0);
    half(1, w1);
    const V scale = exp2_neg<V>(LOGN);
#pragma unroll
    for (int i = 0; i < w0.ITER; ++i) {
#pragma unroll
        for (int m = 0; m < w0.R; ++m) {
            const uint32_t z = (uint32_t)(t + NT * i + (m << LB0));
            mf_store_r<V, REAL_OUT>(out, LOGN, x, z, w0.re[i][m] + w1.re[i][m], scale);
            mf_store_r<V, REAL_OUT>(out, LOGN, x, z | (1u << LH), w0.re[i][m] - w1.re[i][m], scale);
        }
    }
}

template <int SRC>
constexpr bool mf_real_rows()
{
    return SRC == SRC_PURE || SRC == SRC_LOWRANK || SRC == SRC_LOWRANK_T;
}

template <class V, bool REAL_OUT, int SRC>
hipError_t mfree_real_t(int n, const void* src, int64_t ld, void* out, hipStream_t st)
{
    const dim3 grid(1u << n);
    const cplx<V>* s = (const cplx<V>*)src;
    constexpr int FULL_MAX = sizeof(V) == 8 ? 13 : 14;  // 2^n values in 64 KiB
    switch (n) {
#define PTD_ROWR(NN)                                                                                          \
    case NN:                                                                                                  \
        if constexpr (NN <= FULL_MAX)                                                                         \
            hipLaunchKernelGGL((k_mfree_row_r<V, NN, REAL_OUT, SRC>), grid, dim3(MFR_THREADS), 0, st, s, ld, out); \
        else                                                                                                  \
            hipLaunchKernelGGL((k_mfree_halves_r<V, NN, REAL_OUT, SRC>), grid, dim3(MFR_THREADS), 0, st, s, ld,  \
                               out);                                                                          \
        break;
        PTD_ROWR(11) PTD_ROWR(12) PTD_ROWR(13) PTD_ROWR(14)
#undef PTD_ROWR
        case 15:
            if constexpr (sizeof(V) == 4) {
                hipLaunchKernelGGL((k_mfree_halves_r<V, 15, REAL_OUT, SRC>), grid, dim3(MFR_THREADS), 0, st, s, ld,
                                   out);
                break;
            }
            return hipErrorInvalidValue;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class V, bool REAL_OUT, int SRC>
hipError_t mfree_t(int n, const void* src, int64_t ld, void* out, hipStream_t st)
{
    if constexpr (mf_real_rows<SRC>()) return mfree_real_t<V, REAL_OUT, SRC>(n, src, ld, out, st);
    const dim3 grid(1u << n);
    const cplx<V>* s = (const cplx<V>*)src;
    switch (n) {
#define PTD_ROW(NN)                                                                                         \
    case NN:                                                                                                \
        hipLaunchKernelGGL((k_mfree_row<V, NN, REAL_OUT, SRC>), grid, dim3(mf_threads(NN)), 0, st, s, ld, out); \
        break;
        PTD_ROW(11) PTD_ROW(12) PTD_ROW(13)
#undef PTD_ROW
        case 14:
            if constexpr (sizeof(V) == 4)
                hipLaunchKernelGGL((k_mfree_row<V, 14, REAL_OUT, SRC>), grid, dim3(mf_threads(14)), 0, st, s, ld,
                                   out);
            else
                hipLaunchKernelGGL((k_mfree_halves<V, 14, REAL_OUT, SRC>), grid, dim3(MF_HALF_THREADS), 0, st, s,
                                   ld, out);
            break;
        case 15:
            if constexpr (sizeof(V) == 4) {
                hipLaunchKernelGGL((k_mfree_halves<V, 15, REAL_OUT, SRC>), grid, dim3(MF_HALF_THREADS), 0, st, s,
                                   ld, out);
                break;
            }
            return hipErrorInvalidValue;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class V, bool REAL_OUT>
hipError_t mfree_src(int n, int src, const void* t, int64_t ld, void* out, hipStream_t st)
{
    if (src == SRC_TOEPLITZ) return mfree_t<V, REAL_OUT, SRC_TOEPLITZ>(n, t, ld, out, st);
    if (src == SRC_PURE) return mfree_t<V, REAL_OUT, SRC_PURE>(n, t, ld, out, st);
    if (src == SRC_LOWRANK) return mfree_t<V, REAL_OUT, SRC_LOWRANK>(n, t, ld, out, st);
    if (src == SRC_LOWRANK_T) return mfree_t<V, REAL_OUT, SRC_LOWRANK_T>(n, t, ld, out, st);
    return hipErrorInvalidValue;
}

template <class V>
__global__ void k_lowrank_transpose(const cplx<V>* __restrict__ U, int64_t ld, int rank, int logn,
                                    cplx<V>* __restrict__ UT)
{
    const int64_t N = (int64_t)1 << logn;
    const int64_t total = N * rank;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = i >> logn, r = i & (N - 1);  // consecutive threads write consecutive r
        UT[i] = U[r * ld + j];
    }
}

}  // namespace

hipError_t launch_lowrank_transpose(int n, ptd_dtype dt, const void* U, int64_t ld, int rank, void* UT,
                                    hipStream_t st)
{
    const int64_t total = ((int64_t)1 << n) * rank;
    const int blocks = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
    if (dt == PTD_C128)
        hipLaunchKernelGGL(k_lowrank_transpose<double>, dim3(blocks), dim3(256), 0, st, (const cplx<double>*)U, ld,
                           rank, n, (cplx<double>*)UT);
    else
        hipLaunchKernelGGL(k_lowrank_transpose<float>, dim3(blocks), dim3(256), 0, st, (const cplx<float>*)U, ld,
                           rank, n, (cplx<float>*)UT);
    return hipGetLastError();
}

hipError_t launch_mfree(int n, ptd_dtype dt, bool herm, int src, const void* t, int64_t ld, void* out,
                        hipStream_t st)
{
    if (dt == PTD_C128)
        return herm ? mfree_src<double, true>(n, src, t, ld, out, st)
                    : mfree_src<double, false>(n, src, t, ld, out, st);
    return herm ? mfree_src<float, true>(n, src, t, ld, out, st) : mfree_src<float, false>(n, src, t, ld, out, st);
}

}  // namespace ptd
