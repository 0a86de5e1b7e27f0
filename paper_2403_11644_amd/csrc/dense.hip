// dense.hip -- dense Pauli decomposition and reconstruction kernels (gfx950).
//
// Forward map, per X-pattern x (see engine.hpp):
//   c[x][z] = 2^-n i^popcount(x&z) WHT_z( d_x ),  d_x[k] = A[k][k ^ x].
//
// Two schedules:
//
//  * single pass, n <= 10 ("group" kernel): one workgroup owns T = 2^t
//    consecutive X-patterns x = g*T + x_lo.  For row k those patterns read the
//    T contiguous columns ((k >> t) ^ g) * T + [0, T): one 128-byte segment
//    per row (T = 16 complex64 / 8 complex128).  The whole band (2^n rows x T)
//    sits in LDS (<= 128 KiB), the length-2^n WHTs run as radix-16 rounds,
//    and T full output rows are written once.
//
//  * two passes, n >= 11: a 64 x 64 tile (R, C) of A holds d_x[R*64 + k_lo]
//    for the 64 patterns x = (R ^ C)*64 + x_lo.  Pass 1 ("tile") applies the
//    six low WHT bits to every tile and writes the partial transform to
//    coeff[x][R*64 + z_lo] (in place in the output buffer, no workspace).
//    Pass 2 ("high") applies the remaining n-6 bits along each output row
//    (stride 64), then the phase i^popcount(x&z) and the 2^-n scale.
//
// Hermitian input, real output: the partial transform W1 of the two tiles
// (R, C) and (C, R) is related by W1[x][C][z_lo] =
// (-1)^popcount(z_lo & x_lo) * conj(W1[x][R][z_lo]), so pass 1 stores only
// one real number per slot (the real part in the lower block of the pair,
// the imaginary part in the upper one; the single nonzero part when R == C)
// and pass 2 rebuilds both complex values from the pair of slots.
//
// Reconstruction runs the inverse: the phase (-i)^popcount(x&z) first, the
// same WHTs, and a scatter of d_x back to A[k][k ^ x].  For n >= 11 pass 1
// transforms 64 x 64 coefficient tiles over z_lo and places them in A's
// tiles (z_hi, z_hi ^ x_hi); pass 2 runs the WHT over the block index in
// place on A (the WHT over z_hi and the one over z_lo act on different bits
// and commute).
#include "engine.hpp"
#include "group.hpp"
#include "internal.hpp"

namespace ptd {

namespace {

constexpr int TILE_THREADS = 256;
constexpr int HIGH_THREADS = 256;

template <class V>
constexpr int high_logw()
{
    return sizeof(V) == 4 ? 4 : 3;
}

// Row pass shape: 2^LOGW columns (128 bytes) per block.  Compensated mode
// keeps hi and lo in LDS and halves the columns from LOGM = 9 on, so that two
// 512-thread blocks fit on a CU: its butterflies are bound by vector adds,
// and the second block hides their latency (n = 15: 9.14 -> 8.64 ms for the
// whole compensated call, bit-identical output).
template <class V, int LOGM, bool COMP>
constexpr int row_logw()
{
    return (COMP && LOGM >= 9) ? high_logw<V>() - 1 : high_logw<V>();
}

template <int LOGM, bool COMP>
constexpr int row_threads()
{
    return (COMP && LOGM == 9) ? 512 : HIGH_THREADS;
}

// ------------------------------------------------------------------------
// single pass, n <= 10

template <class V, int LOGN, bool REAL_OUT, int NT, int RMAX, int SRC = SRC_MATRIX>
__global__ __launch_bounds__(NT) void k_group_fwd(const cplx<V>* __restrict__ A, int64_t lda,
                                                  void* __restrict__ out, int64_t ldo, V scale)
{
    constexpr int LOGT = group_logt<V>(LOGN);
    __shared__ cplx<V> lds[(1 << LOGT) * ((1 << LOGN) + 1)];
    group_fwd<V, LOGN, LOGT, REAL_OUT, NT, RMAX, SRC>(A, lda, out, ldo, blockIdx.x, lds, scale);
}

template <class V, int LOGN, bool REAL_IN>
__global__ __launch_bounds__(GROUP_THREADS) void k_group_rec(const void* __restrict__ coeff,
                                                             cplx<V>* __restrict__ A, int64_t lda, V scale)
{
    constexpr int LOGT = group_logt<V>(LOGN);
    __shared__ cplx<V> lds[(1 << LOGT) * ((1 << LOGN) + 1)];
    group_rec<V, LOGN, LOGT, REAL_IN>(coeff, A, lda, scale, blockIdx.x, lds);
}

// ------------------------------------------------------------------------
// two passes, pass 1: 64 x 64 tiles, low six WHT bits

// grid (nb, nb): tile (R, C) = (blockIdx.y, blockIdx.x).  With xh_count > 0
// the grid is (nb, xh_count) instead and covers the tiles of the X-pattern
// groups x_hi = xh0 + blockIdx.y only (R = blockIdx.x, C = R ^ x_hi).
template <class V, bool HERM, bool COMP>
__global__ __launch_bounds__(TILE_THREADS) void k_tile_fwd(const cplx<V>* __restrict__ A, int64_t lda,
                                                           void* __restrict__ out, int64_t ldo, int xh0,
                                                           int xh_count)
{
    __shared__ cplx<V> lds[(COMP ? 2 : 1) * 64 * 65];
    const int R = xh_count ? (int)blockIdx.x : (int)blockIdx.y;
    const int C = xh_count ? (R ^ (xh0 + (int)blockIdx.y)) : (int)blockIdx.x;
    const int xh = R ^ C;
    const cplx<V>* tile = A + (int64_t)R * 64 * lda + (int64_t)C * 64;
    auto gather = [&](int vec, int pos, V& re, V& im) {
        const cplx<V> v = tile[(int64_t)pos * lda + (pos ^ vec)];
        re = v.re;
        im = v.im;
    };
    auto store = [&](int vec, int pos, V re, V im) {
        const int64_t o = (int64_t)((xh << 6) | vec) * ldo + ((int64_t)R << 6) + pos;
        if constexpr (HERM) {
            const bool sneg = __popc((uint32_t)(pos & vec)) & 1;
            V val;
            if (R < C)
                val = re;
            else if (R > C)
                val = sneg ? im : -im;
            else
                val = sneg ? im : re;
            ((V*)out)[o] = val;
        } else {
            cplx<V> c;
            c.re = re;
            c.im = im;
            ((cplx<V>*)out)[o] = c;
        }
    };
    if constexpr (COMP) {
        // compensated pairs; the pass boundary keeps hi (= fl(hi + lo))
        auto gather_c = [&](int vec, int pos, V& rh, V& rl, V& ih, V& il) {
            gather(vec, pos, rh, ih);
            rl = (V)0;
            il = (V)0;
        };
        auto store_c = [&](int vec, int pos, V rh, V, V ih, V) { store(vec, pos, rh, ih); };
        LdsVecsComp<V, 6> cr{lds, lds + 64 * 65};
        LdsVecsCompW<V, 6> cw{lds, lds + 64 * 65};
        wht_round_comp<V, 6, 6, 0, 4, TILE_THREADS, true>(gather_c, cw);
        __syncthreads();
        wht_round_comp<V, 6, 6, 4, 2, TILE_THREADS, false>(cr, store_c);
    } else {
        LdsVecs<V, 6> lr{lds};
        LdsVecsW<V, 6> lw{lds};
        wht_round<V, 6, 6, 0, 4, TILE_THREADS, true>(gather, lw);
        __syncthreads();
        wht_round<V, 6, 6, 4, 2, TILE_THREADS, false>(lr, store);
    }
}

// pass 2: WHT over the block index (stride 64) of each output row chunk,
// then the phase and the scale.
template <class V, int LOGM, bool HERM, bool COMP>
__global__ __launch_bounds__((row_threads<LOGM, COMP>())) void k_high_fwd(void* __restrict__ out, int64_t ldo, int x0,
                                                                                               V scale)
{
    constexpr int LOGW = row_logw<V, LOGM, COMP>();
    constexpr int CH = 6 - LOGW;
    constexpr int NT = row_threads<LOGM, COMP>();
    constexpr int PLANE = (1 << LOGW) * ((1 << LOGM) + 1);
    __shared__ cplx<V> lds[(COMP ? 2 : 1) * PLANE];
    const int x = x0 + (int)(blockIdx.x >> CH);
    const int z0 = (blockIdx.x & ((1 << CH) - 1)) << LOGW;
    const int xh = x >> 6, xl = x & 63;
    V* rowr = (V*)out + (int64_t)x * ldo;
    cplx<V>* rowc = (cplx<V>*)out + (int64_t)x * ldo;
    auto load = [&](int vec, int pos, V& re, V& im) {
        const int zl = z0 + vec;
        if constexpr (HERM) {
            const int pp = pos ^ xh;
            const V a = rowr[(pos << 6) + zl];
            const bool sneg = __popc((uint32_t)(zl & xl)) & 1;
            if (pos < pp) {
                re = a;
                im = rowr[(pp << 6) + zl];
            } else if (pos > pp) {
                const V b = rowr[(pp << 6) + zl];
                re = sneg ? -b : b;
                im = sneg ? a : -a;
            } else {
                re = sneg ? (V)0 : a;
                im = sneg ? a : (V)0;
            }
        } else {
            const cplx<V> v = rowc[(pos << 6) + zl];
            re = v.re;
            im = v.im;
        }
    };
    auto store = [&](int vec, int pos, V re, V im) {
        const int z = (pos << 6) + z0 + vec;
        mul_ipow(__popc((uint32_t)(x & z)) & 3, re, im);
        if constexpr (HERM) {
            rowr[z] = re * scale;
        } else {
            cplx<V> c;
            c.re = re * scale;
            c.im = im * scale;
            rowc[z] = c;
        }
    };
    if constexpr (COMP) {
        auto load_c = [&](int vec, int pos, V& rh, V& rl, V& ih, V& il) {
            load(vec, pos, rh, ih);
            rl = (V)0;
            il = (V)0;
        };
        // the phase and the power-of-two scale are exact on hi and lo alike;
        // hi = fl(hi + lo) after the last renormalisation
        auto store_c = [&](int vec, int pos, V rh, V, V ih, V) { store(vec, pos, rh, ih); };
        LdsVecsComp<V, LOGM> cr{lds, lds + PLANE};
        LdsVecsCompW<V, LOGM> cw{lds, lds + PLANE};
        if constexpr (LOGM <= 4) {
            wht_round_comp<V, LOGW, LOGM, 0, LOGM, NT, true>(load_c, store_c);
        } else if constexpr (LOGM <= 8) {
            wht_round_comp<V, LOGW, LOGM, 0, 4, NT, true>(load_c, cw);
            __syncthreads();
            wht_round_comp<V, LOGW, LOGM, 4, LOGM - 4, NT, true>(cr, store_c);
        } else {
            wht_round_comp<V, LOGW, LOGM, 0, 4, NT, true>(load_c, cw);
            __syncthreads();
            wht_round_comp<V, LOGW, LOGM, 4, 4, NT, true>(cr, cw);
            __syncthreads();
            wht_round_comp<V, LOGW, LOGM, 8, LOGM - 8, NT, true>(cr, store_c);
        }
    } else {
        LdsVecs<V, LOGM> lr{lds};
        LdsVecsW<V, LOGM> lw{lds};
        if constexpr (LOGM <= 4) {
            wht_round<V, LOGW, LOGM, 0, LOGM, NT, true>(load, store);
        } else if constexpr (LOGM <= 8) {
            wht_round<V, LOGW, LOGM, 0, 4, NT, true>(load, lw);
            __syncthreads();
            wht_round<V, LOGW, LOGM, 4, LOGM - 4, NT, true>(lr, store);
        } else {
            wht_round<V, LOGW, LOGM, 0, 4, NT, true>(load, lw);
            __syncthreads();
            wht_round<V, LOGW, LOGM, 4, 4, NT, true>(lr, lw);
            __syncthreads();
            wht_round<V, LOGW, LOGM, 8, LOGM - 8, NT, true>(lr, store);
        }
    }
}

// reconstruction pass 1: coefficient tile (x_hi, zb) -> A tile (zb, zb ^ x_hi)
template <class V, bool REAL_IN>
__global__ __launch_bounds__(TILE_THREADS) void k_tile_rec(const void* __restrict__ coeff, int64_t ldc,
                                                           cplx<V>* __restrict__ A, int64_t lda)
{
    __shared__ cplx<V> lds[64 * 65];
    const int xh = blockIdx.y, zb = blockIdx.x;
    auto load = [&](int vec, int pos, V& re, V& im) {
        const uint32_t x = (uint32_t)((xh << 6) | vec);
        const uint32_t z = (uint32_t)((zb << 6) | pos);
        const int64_t o = (int64_t)x * ldc + z;
        if constexpr (REAL_IN) {
            re = ((const V*)coeff)[o];
            im = (V)0;
        } else {
            const cplx<V> c = ((const cplx<V>*)coeff)[o];
            re = c.re;
            im = c.im;
        }
        mul_ipow((4 - (__popc(x & z) & 3)) & 3, re, im);
    };
    cplx<V>* tile = A + (int64_t)zb * 64 * lda + (int64_t)(zb ^ xh) * 64;
    auto scatter = [&](int vec, int pos, V re, V im) {
        cplx<V> c;
        c.re = re;
        c.im = im;
        tile[(int64_t)pos * lda + (pos ^ vec)] = c;
    };
    LdsVecs<V, 6> lr{lds};
    LdsVecsW<V, 6> lw{lds};
    wht_round<V, 6, 6, 0, 4, TILE_THREADS, false>(load, lw);
    __syncthreads();
    wht_round<V, 6, 6, 4, 2, TILE_THREADS, true>(lr, scatter);
}

// reconstruction pass 2: WHT over the block index along the x_hi band of A,
// in place.  Workgroup = (x_hi, k_lo, chunk of x_lo).
template <class V, int LOGM>
__global__ __launch_bounds__(HIGH_THREADS) void k_high_rec(cplx<V>* __restrict__ A, int64_t lda, V scale)
{
    constexpr int LOGW = high_logw<V>();
    constexpr int CH = 6 - LOGW;
    constexpr int NT = HIGH_THREADS;
    __shared__ cplx<V> lds[(1 << LOGW) * ((1 << LOGM) + 1)];
    const int id = blockIdx.x;
    const int x0 = (id & ((1 << CH) - 1)) << LOGW;
    const int klo = (id >> CH) & 63;
    const int xh = id >> (CH + 6);
    auto addr = [&](int vec, int pos) -> int64_t {
        return ((int64_t)pos * 64 + klo) * lda + (int64_t)(pos ^ xh) * 64 + (klo ^ (x0 + vec));
    };
    auto load = [&](int vec, int pos, V& re, V& im) {
        const cplx<V> v = A[addr(vec, pos)];
        re = v.re;
        im = v.im;
    };
    auto store = [&](int vec, int pos, V re, V im) {
        cplx<V> c;
        c.re = re * scale;
        c.im = im * scale;
        A[addr(vec, pos)] = c;
    };
    LdsVecs<V, LOGM> lr{lds};
    LdsVecsW<V, LOGM> lw{lds};
    if constexpr (LOGM <= 4) {
        wht_round<V, LOGW, LOGM, 0, LOGM, NT, true>(load, store);
    } else if constexpr (LOGM <= 8) {
        wht_round<V, LOGW, LOGM, 0, 4, NT, true>(load, lw);
        __syncthreads();
        wht_round<V, LOGW, LOGM, 4, LOGM - 4, NT, true>(lr, store);
    } else {
        wht_round<V, LOGW, LOGM, 0, 4, NT, true>(load, lw);
        __syncthreads();
        wht_round<V, LOGW, LOGM, 4, 4, NT, true>(lr, lw);
        __syncthreads();
        wht_round<V, LOGW, LOGM, 8, LOGM - 8, NT, true>(lr, store);
    }
}

// ------------------------------------------------------------------------
// compensated single pass for n <= 6: every X-pattern of the matrix in one
// workgroup (2^n vectors of 2^n positions, hi and lo planes in LDS)

template <class V, int LOGN, bool HERM>
__global__ __launch_bounds__(TILE_THREADS) void k_small_comp(const cplx<V>* __restrict__ A, int64_t lda,
                                                             void* __restrict__ out)
{
    constexpr int N = 1 << LOGN;
    constexpr int PLANE = N * (N + 1);
    __shared__ cplx<V> lds[2 * PLANE];
    const V scale = exp2_neg<V>(LOGN);
    auto gather = [&](int vec, int pos, V& rh, V& rl, V& ih, V& il) {
        const cplx<V> v = A[(int64_t)pos * lda + (pos ^ vec)];
        rh = v.re;
        ih = v.im;
        rl = (V)0;
        il = (V)0;
    };
    auto store = [&](int vec, int pos, V re, V, V im, V) {
        mul_ipow(__popc((uint32_t)(vec & pos)) & 3, re, im);
        if constexpr (HERM) {
            ((V*)out)[(int64_t)vec * N + pos] = re * scale;
        } else {
            cplx<V> c;
            c.re = re * scale;
            c.im = im * scale;
            ((cplx<V>*)out)[(int64_t)vec * N + pos] = c;
        }
    };
    LdsVecsComp<V, LOGN> cr{lds, lds + PLANE};
    LdsVecsCompW<V, LOGN> cw{lds, lds + PLANE};
    if constexpr (LOGN <= 4) {
        wht_round_comp<V, LOGN, LOGN, 0, LOGN, TILE_THREADS, true>(gather, store);
    } else {
        wht_round_comp<V, LOGN, LOGN, 0, 4, TILE_THREADS, true>(gather, cw);
        __syncthreads();
        wht_round_comp<V, LOGN, LOGN, 4, LOGN - 4, TILE_THREADS, false>(cr, store);
    }
}

// ------------------------------------------------------------------------
// dispatch over n (compile-time sizes)

template <class V, bool HERM, int NT, int RMAX>
hipError_t fwd_group_plan(int n, const cplx<V>* a, int64_t lda, void* out, int64_t ldo, V scale, hipStream_t st)
{
    const int logt = group_logt<V>(n);
    const dim3 grid(1u << (n - logt)), block(NT);
    switch (n) {
#define PTD_CASE(NN) \
    case NN: hipLaunchKernelGGL((k_group_fwd<V, NN, HERM, NT, RMAX>), grid, block, 0, st, a, lda, out, ldo, scale); break;
        PTD_CASE(1) PTD_CASE(2) PTD_CASE(3) PTD_CASE(4) PTD_CASE(5)
        PTD_CASE(6) PTD_CASE(7) PTD_CASE(8) PTD_CASE(9) PTD_CASE(10)
#undef PTD_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// plan: see group.hpp (workgroup size, widest round); radix 32 is complex64 only
template <class V, bool HERM>
hipError_t fwd_group(int n, const void* A, int64_t lda, void* out, int plan, hipStream_t st, bool unscaled = false)
{
    const cplx<V>* a = (const cplx<V>*)A;
    const int64_t ldo = (int64_t)1 << n;
    const bool big = group_plan_nt(plan) == 1024;
    const V scale = unscaled ? (V)1 : (V)1 / (V)(1u << n);
    if constexpr (sizeof(V) == 4) {
        if (group_effective_rmax(n, PTD_C64, plan) == 5)
            return big ? fwd_group_plan<V, HERM, 1024, 5>(n, a, lda, out, ldo, scale, st)
                       : fwd_group_plan<V, HERM, 512, 5>(n, a, lda, out, ldo, scale, st);
    }
    return big ? fwd_group_plan<V, HERM, 1024, 4>(n, a, lda, out, ldo, scale, st)
               : fwd_group_plan<V, HERM, 512, 4>(n, a, lda, out, ldo, scale, st);
}

// stage: 3 = both passes, 1 = tile pass only, 2 = row pass only (timing)
template <class V, bool HERM, bool COMP = false>
hipError_t fwd_two_pass(int n, const void* A, int64_t lda, void* out, hipStream_t st, int stage = 3,
                        bool unscaled = false)
{
    const V scale = unscaled ? (V)1 : (V)1 / (V)(1u << n);
    const cplx<V>* a = (const cplx<V>*)A;
    const int64_t ldo = (int64_t)1 << n;
    const int nb = 1 << (n - 6);
    // chunk > 0: alternate the passes over chunks of `chunk` X-pattern groups
    const int chunk = stage >> 2;
    const int nchunks = chunk ? (nb + chunk - 1) / chunk : 1;
    for (int c = 0; c < nchunks; ++c) {
        const int xh0 = chunk ? c * chunk : 0;
        const int cnt = chunk ? (nb - xh0 < chunk ? nb - xh0 : chunk) : nb;
        if (stage & 1) {
            if (chunk)
                hipLaunchKernelGGL((k_tile_fwd<V, HERM, COMP>), dim3(nb, cnt), dim3(TILE_THREADS), 0, st, a, lda, out, ldo,
                                   xh0, cnt);
            else
                hipLaunchKernelGGL((k_tile_fwd<V, HERM, COMP>), dim3(nb, nb), dim3(TILE_THREADS), 0, st, a, lda, out, ldo,
                                   0, 0);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        if (!(stage & 2)) continue;
        const int x0 = xh0 * 64;
        switch (n - 6) {
#define PTD_CASE(MM)                                                                                              \
    case MM:                                                                                                      \
        hipLaunchKernelGGL((k_high_fwd<V, MM, HERM, COMP>),                                                       \
                           dim3((unsigned)(((int64_t)cnt * 64) << (6 - row_logw<V, MM, COMP>()))),                \
                           dim3(row_threads<MM, COMP>()), 0, st, out, ldo, x0, scale);                            \
        break;
            PTD_CASE(1) PTD_CASE(2) PTD_CASE(3) PTD_CASE(4) PTD_CASE(5)
            PTD_CASE(6) PTD_CASE(7) PTD_CASE(8) PTD_CASE(9) PTD_CASE(10)
#undef PTD_CASE
            default: return hipErrorInvalidValue;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <class V, bool HERM>
hipError_t rec_group(int n, const void* coeff, void* A, int64_t lda, V scale, hipStream_t st)
{
    cplx<V>* a = (cplx<V>*)A;
    const int logt = group_logt<V>(n);
    const dim3 grid(1u << (n - logt)), block(GROUP_THREADS);
    switch (n) {
#define PTD_CASE(NN) \
    case NN: hipLaunchKernelGGL((k_group_rec<V, NN, HERM>), grid, block, 0, st, coeff, a, lda, scale); break;
        PTD_CASE(1) PTD_CASE(2) PTD_CASE(3) PTD_CASE(4) PTD_CASE(5)
        PTD_CASE(6) PTD_CASE(7) PTD_CASE(8) PTD_CASE(9) PTD_CASE(10)
#undef PTD_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class V, bool HERM>
hipError_t rec_two_pass(int n, const void* coeff, void* A, int64_t lda, V scale, hipStream_t st)
{
    cplx<V>* a = (cplx<V>*)A;
    const int64_t ldc = (int64_t)1 << n;
    const int nb = 1 << (n - 6);
    hipLaunchKernelGGL((k_tile_rec<V, HERM>), dim3(nb, nb), dim3(TILE_THREADS), 0, st, coeff, ldc, a, lda);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 g2((unsigned)(((int64_t)1 << n) << (6 - high_logw<V>())));
    switch (n - 6) {
#define PTD_CASE(MM) \
    case MM: hipLaunchKernelGGL((k_high_rec<V, MM>), g2, dim3(HIGH_THREADS), 0, st, a, lda, scale); break;
        PTD_CASE(1) PTD_CASE(2) PTD_CASE(3) PTD_CASE(4) PTD_CASE(5)
        PTD_CASE(6) PTD_CASE(7) PTD_CASE(8) PTD_CASE(9) PTD_CASE(10)
#undef PTD_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dense_fwd(int n, ptd_dtype dt, bool herm, const void* A, int64_t lda, void* out, int path,
                            hipStream_t st, bool unscaled)
{
    const bool two = path == 2 ? true : path == 1 ? false : n > 10;
    if (two && n < 7) return hipErrorInvalidValue;
    if (!two && n > 10) return hipErrorInvalidValue;
    const int plan = two ? 0 : group_plan(n, dt, herm);
    const bool u = unscaled;
    if (dt == PTD_C128) {
        if (two)
            return herm ? fwd_two_pass<double, true>(n, A, lda, out, st, 3, u)
                        : fwd_two_pass<double, false>(n, A, lda, out, st, 3, u);
        return herm ? fwd_group<double, true>(n, A, lda, out, plan, st, u)
                    : fwd_group<double, false>(n, A, lda, out, plan, st, u);
    }
    if (two)
        return herm ? fwd_two_pass<float, true>(n, A, lda, out, st, 3, u)
                    : fwd_two_pass<float, false>(n, A, lda, out, st, 3, u);
    return herm ? fwd_group<float, true>(n, A, lda, out, plan, st, u) : fwd_group<float, false>(n, A, lda, out, plan, st, u);
}

hipError_t launch_dense_fwd_stage(int n, ptd_dtype dt, bool herm, const void* A, int64_t lda, void* out, int stage,
                                  hipStream_t st)
{
    if (n < 7 || stage < 1 || (stage & 3) == 0) return hipErrorInvalidValue;
    if (dt == PTD_C128)
        return herm ? fwd_two_pass<double, true>(n, A, lda, out, st, stage)
                    : fwd_two_pass<double, false>(n, A, lda, out, st, stage);
    return herm ? fwd_two_pass<float, true>(n, A, lda, out, st, stage)
                : fwd_two_pass<float, false>(n, A, lda, out, st, stage);
}

hipError_t launch_dense_fwd_comp(int n, bool herm, const void* A, int64_t lda, void* out, hipStream_t st)
{
    const cplx<float>* a = (const cplx<float>*)A;
    if (n >= 7) return herm ? fwd_two_pass<float, true, true>(n, A, lda, out, st) : fwd_two_pass<float, false, true>(n, A, lda, out, st);
    switch (n) {
#define PTD_CASE(NN)                                                                                               \
    case NN:                                                                                                       \
        if (herm)                                                                                                  \
            hipLaunchKernelGGL((k_small_comp<float, NN, true>), dim3(1), dim3(TILE_THREADS), 0, st, a, lda, out);  \
        else                                                                                                       \
            hipLaunchKernelGGL((k_small_comp<float, NN, false>), dim3(1), dim3(TILE_THREADS), 0, st, a, lda, out); \
        break;
        PTD_CASE(1) PTD_CASE(2) PTD_CASE(3) PTD_CASE(4) PTD_CASE(5) PTD_CASE(6)
#undef PTD_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dense_rec(int n, ptd_dtype dt, bool herm, bool adjoint, const void* coeff, void* A, int64_t lda,
                            int path, hipStream_t st)
{
    const bool two = path == 2 ? true : path == 1 ? false : n > 10;
    if (two && n < 7) return hipErrorInvalidValue;
    if (!two && n > 10) return hipErrorInvalidValue;
    if (dt == PTD_C128) {
        const double sc = adjoint ? 1.0 / (double)(1u << n) : 1.0;
        if (two) return herm ? rec_two_pass<double, true>(n, coeff, A, lda, sc, st) : rec_two_pass<double, false>(n, coeff, A, lda, sc, st);
        return herm ? rec_group<double, true>(n, coeff, A, lda, sc, st) : rec_group<double, false>(n, coeff, A, lda, sc, st);
    }
    const float sc = adjoint ? 1.0f / (float)(1u << n) : 1.0f;
    if (two) return herm ? rec_two_pass<float, true>(n, coeff, A, lda, sc, st) : rec_two_pass<float, false>(n, coeff, A, lda, sc, st);
    return herm ? rec_group<float, true>(n, coeff, A, lda, sc, st) : rec_group<float, false>(n, coeff, A, lda, sc, st);
}

// Matrix-free input for n <= 10 (src: SRC_TOEPLITZ or SRC_PURE): the
// single-pass group kernel with 512-thread workgroups and radix-16 rounds
// (the results do not depend on the plan).
template <class V, int SRC>
hipError_t group_src_t(int n, bool herm, const void* src, int64_t ld, void* out, hipStream_t st)
{
    const int N = 1 << n;
    const dim3 grid(N >> group_logt<V>(n));
    switch (n) {
#define PTD_T(NN)                                                                                             \
    case NN:                                                                                                  \
        if (herm)                                                                                             \
            hipLaunchKernelGGL((k_group_fwd<V, NN, true, 512, 4, SRC>), grid, dim3(512), 0, st,               \
                               (const cplx<V>*)src, ld, out, (int64_t)N, (V)1 / (V)(1u << NN));                    \
        else                                                                                                  \
            hipLaunchKernelGGL((k_group_fwd<V, NN, false, 512, 4, SRC>), grid, dim3(512), 0, st,              \
                               (const cplx<V>*)src, ld, out, (int64_t)N, (V)1 / (V)(1u << NN));                    \
        break;
        PTD_T(1) PTD_T(2) PTD_T(3) PTD_T(4) PTD_T(5) PTD_T(6) PTD_T(7) PTD_T(8) PTD_T(9) PTD_T(10)
#undef PTD_T
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_group_src(int n, ptd_dtype dt, bool herm, int src, const void* ptr, int64_t ld, void* out,
                            hipStream_t st)
{
    if (n < 1 || n > 10) return hipErrorInvalidValue;
    if (src == SRC_TOEPLITZ)
        return dt == PTD_C128 ? group_src_t<double, SRC_TOEPLITZ>(n, herm, ptr, ld, out, st)
                              : group_src_t<float, SRC_TOEPLITZ>(n, herm, ptr, ld, out, st);
    if (src == SRC_PURE)
        return dt == PTD_C128 ? group_src_t<double, SRC_PURE>(n, herm, ptr, ld, out, st)
                              : group_src_t<float, SRC_PURE>(n, herm, ptr, ld, out, st);
    if (src == SRC_LOWRANK)
        return dt == PTD_C128 ? group_src_t<double, SRC_LOWRANK>(n, herm, ptr, ld, out, st)
                              : group_src_t<float, SRC_LOWRANK>(n, herm, ptr, ld, out, st);
    return hipErrorInvalidValue;
}

}  // namespace ptd
