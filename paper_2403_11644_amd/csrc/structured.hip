// structured.hip -- diagonal, banded and anti-diagonal inputs: only
// nonempty X-patterns.
//
// For a band matrix with half-bandwidth s (a[r][c] = 0 when |r - c| > s;
// s = 0 diagonal, s = 1 tridiagonal; paper Sec. IV-A) the strings with
// X-pattern x read only the entries (k, k ^ x), so x can carry nonzero
// coefficients only if some entry (k, k ^ x) lies in the band:
// x = 0, or x = 2^h + y with 0 <= y < 2^h and 2^h - y <= s (the smallest
// |(k ^ x) - k| over k is 2^h - y).  There are 1 + sum_{h<n} min(s, 2^h)
// such x, the paper's (s n - c(s)) per 2^n terms, listed in ascending order
// as: 0, then for h = 0, 1, ... the interval [2^(h+1) - min(s, 2^h), 2^(h+1)).
//
// Each listed x gets d_x[k] = A[k][k ^ x] for in-band entries and 0 outside
// the band, read either from the dense matrix (touching only in-band
// entries) or from the row-indexed bands band[d + s][k] = A[k][k + d], then
// one length-2^n WHT and the fused phase/scale.  An anti-diagonal matrix
// (a[r][c] = 0 unless r + c = 2^n - 1) reads only the entries (k, k ^ x)
// with x = 2^n - 1, so that is its one X-pattern: every string has X or Y on
// every qubit (the remark after the diagonal case in Sec. IV-A); it is coded
// as s < 0 below, with the compressed input ad[k] = A[k][2^n - 1 - k].  n <= 10: one pass, several
// X-patterns per workgroup in LDS.  n >= 11: a 1024-position pass and a
// strided pass over the remaining bits, in place in the output rows.
#include "engine.hpp"
#include "internal.hpp"

namespace ptd {

namespace {

constexpr int SM_THREADS = 256;
constexpr int SM_VECS = 4;  // X-patterns per workgroup for n <= 10
constexpr int SP_KAP = 10;  // positions per first-pass item for n >= 11

// i-th nonempty X-pattern (ascending); s = 0 means diagonal, s < 0
// anti-diagonal (the single X-pattern 2^n - 1: X or Y on every qubit).
__device__ __forceinline__ uint32_t listed_x(int i, int n, int s, const uint32_t* __restrict__ xs)
{
    if (xs) return xs[i];  // sparse input: the caller's list
    if (s < 0) return (1u << n) - 1u;
    if (i == 0) return 0u;
    int r = i - 1;
    for (int h = 0; h < n; ++h) {
        const int cnt = s < (1 << h) ? s : (1 << h);
        if (r < cnt) return (uint32_t)((2 << h) - cnt + r);
        r -= cnt;
    }
    return 0u;  // unreachable for i < count
}

__device__ __forceinline__ bool is_listed(uint32_t x, int n, int s)
{
    if (s < 0) return x == (1u << n) - 1u;
    if (x == 0u) return true;
    const int h = 31 - __clz(x);
    const int y = (int)x - (1 << h);
    return (1 << h) - y <= s;
}

// d_x[k] from the dense matrix or from the row-indexed bands; 0 off band.
// Anti-diagonal (s < 0): A[k][k ^ x] with x = 2^n - 1, or entry k of the
// compressed vector ad[k] = A[k][2^n - 1 - k].
template <class V, bool BANDS>
__device__ __forceinline__ void band_entry(const cplx<V>* __restrict__ A, int64_t lda, int s, int k, uint32_t x,
                                           V& re, V& im)
{
    const int c = k ^ (int)x;
    if (s < 0) {
        const cplx<V> v = BANDS ? A[k] : A[(int64_t)k * lda + c];
        re = v.re;
        im = v.im;
        return;
    }
    const int d = c - k;
    if (d > s || d < -s) {
        re = (V)0;
        im = (V)0;
        return;
    }
    const cplx<V> v = BANDS ? A[(int64_t)(d + s) * lda + k] : A[(int64_t)k * lda + c];
    re = v.re;
    im = v.im;
}

// Input modes of the structured kernels.
constexpr int SRC_DENSE = 0;  // the dense matrix A[k][k ^ x]
constexpr int SRC_BANDS = 1;  // row-indexed bands (or the anti-diagonal vector)
constexpr int SRC_ROWS = 2;   // d_x already scattered into the output row of x (sparse input), in place

// d_x[k] for the listed X-pattern x whose output row is `row`.
template <class V, int SRC>
__device__ __forceinline__ void src_entry(const cplx<V>* __restrict__ A, int64_t lda, int s, const void* out,
                                          int64_t row, int n, int k, uint32_t x, V& re, V& im)
{
    if constexpr (SRC == SRC_ROWS) {
        const cplx<V> v = ((const cplx<V>*)out)[(row << n) + k];
        re = v.re;
        im = v.im;
    } else {
        band_entry<V, SRC == SRC_BANDS>(A, lda, s, k, x, re, im);
    }
}

template <class V, bool HERM>
__device__ __forceinline__ void put_final(void* __restrict__ out, int64_t o, V re, V im)
{
    if constexpr (HERM) {
        ((V*)out)[o] = re;
    } else {
        cplx<V> c;
        c.re = re;
        c.im = im;
        ((cplx<V>*)out)[o] = c;
    }
}

// ---------------------------------------------------------------- n <= 10

template <class V, int LOGN, int SRC, bool HERM>
__global__ __launch_bounds__(SM_THREADS) void k_struct_small(const cplx<V>* __restrict__ A, int64_t lda, int s,
                                                             int count, int compact, void* __restrict__ out,
                                                             const uint32_t* __restrict__ xs)
{
    constexpr int N = 1 << LOGN;
    constexpr int LV = 2;  // log2(SM_VECS)
    __shared__ cplx<V> lds[SM_VECS * (N + 1)];
    const int i0 = blockIdx.x * SM_VECS;
    const V scale = exp2_neg<V>(LOGN);
    auto gather = [&](int vec, int pos, V& re, V& im) {
        const int i = i0 + vec;
        if (i >= count) {
            re = (V)0;
            im = (V)0;
            return;
        }
        const uint32_t x = listed_x(i, LOGN, s, xs);
        src_entry<V, SRC>(A, lda, s, out, compact ? i : (int64_t)x, LOGN, pos, x, re, im);
    };
    auto store = [&](int vec, int pos, V re, V im) {
        const int i = i0 + vec;
        if (i >= count) return;
        const uint32_t x = listed_x(i, LOGN, s, xs);
        mul_ipow(__popc(x & (uint32_t)pos) & 3, re, im);
        const int64_t row = compact ? i : (int64_t)x;
        put_final<V, HERM>(out, row * N + pos, re * scale, im * scale);
    };
    LdsVecs<V, LOGN> lr{lds};
    LdsVecsW<V, LOGN> lw{lds};
    if constexpr (LOGN <= 4) {
        wht_round<V, LV, LOGN, 0, LOGN, SM_THREADS, true>(gather, store);
    } else if constexpr (LOGN <= 8) {
        wht_round<V, LV, LOGN, 0, 4, SM_THREADS, false>(gather, lw);
        __syncthreads();
        wht_round<V, LV, LOGN, 4, LOGN - 4, SM_THREADS, false>(lr, store);
    } else {
        wht_round<V, LV, LOGN, 0, 4, SM_THREADS, false>(gather, lw);
        __syncthreads();
        wht_round<V, LV, LOGN, 4, 4, SM_THREADS, false>(lr, lw);
        __syncthreads();
        wht_round<V, LV, LOGN, 8, LOGN - 8, SM_THREADS, false>(lr, store);
    }
}

// ---------------------------------------------------------------- n >= 11
// pass 1, item (i, b): positions [b*1024, (b+1)*1024) of d_x, low ten bits.
// Hermitian real output stores one real per slot: blocks b and b ^ (x >> 10)
// of one row are conjugate-symmetric partners (see dense.hip).
template <class V, int SRC, bool HERM>
__global__ __launch_bounds__(SM_THREADS) void k_struct_p1(const cplx<V>* __restrict__ A, int64_t lda, int s, int n,
                                                          int compact, void* __restrict__ out,
                                                          const uint32_t* __restrict__ xs)
{
    __shared__ cplx<V> lds[(1 << SP_KAP) + 1];
    const int i = blockIdx.x;
    const int b = blockIdx.y;
    const uint32_t x = listed_x(i, n, s, xs);
    const int k0 = b << SP_KAP;
    const int64_t N = (int64_t)1 << n;
    const int64_t row = compact ? i : (int64_t)x;
    const int bp = b ^ (int)(x >> SP_KAP);
    // in place for SRC_ROWS: this item reads its 1024 positions of the row in
    // the first round and writes the same positions in the last
    auto gather = [&](int, int pos, V& re, V& im) { src_entry<V, SRC>(A, lda, s, out, row, n, k0 + pos, x, re, im); };
    auto store = [&](int, int pos, V re, V im) {
        const int64_t o = row * N + k0 + pos;
        if constexpr (HERM) {
            const bool sneg = __popc((uint32_t)pos & (x & ((1u << SP_KAP) - 1))) & 1;
            V val;
            if (b < bp)
                val = re;
            else if (b > bp)
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
    LdsVecs<V, SP_KAP> lr{lds};
    LdsVecsW<V, SP_KAP> lw{lds};
    wht_round<V, 0, SP_KAP, 0, 4, SM_THREADS, false>(gather, lw);
    __syncthreads();
    wht_round<V, 0, SP_KAP, 4, 4, SM_THREADS, false>(lr, lw);
    __syncthreads();
    wht_round<V, 0, SP_KAP, 8, 2, SM_THREADS, false>(lr, store);
}

// pass 2, item (i, chunk of 16 positions z_lo): WHT over the 2^(n-10)
// positions z_lo + 1024 j, then phase and scale.
template <class V, int LOGM, bool HERM>
__global__ __launch_bounds__(SM_THREADS) void k_struct_p2(int s, int n, int compact, void* __restrict__ out,
                                                          const uint32_t* __restrict__ xs)
{
    constexpr int LOGW = 4;
    constexpr int NT = SM_THREADS;
    __shared__ cplx<V> lds[(1 << LOGW) * ((1 << LOGM) + 1)];
    const int i = blockIdx.x;
    const int z0 = blockIdx.y << LOGW;
    const uint32_t x = listed_x(i, n, s, xs);
    const int64_t N = (int64_t)1 << n;
    const int64_t row = compact ? i : (int64_t)x;
    const int xh = (int)(x >> SP_KAP);
    const uint32_t xl = x & ((1u << SP_KAP) - 1);
    V* rowr = (V*)out + row * N;
    cplx<V>* rowc = (cplx<V>*)out + row * N;
    const V scale = exp2_neg<V>(n);
    auto load = [&](int vec, int pos, V& re, V& im) {
        const int zl = z0 + vec;
        if constexpr (HERM) {
            const int pp = pos ^ xh;
            const V a = rowr[((int64_t)pos << SP_KAP) + zl];
            const bool sneg = __popc((uint32_t)zl & xl) & 1;
            if (pos < pp) {
                re = a;
                im = rowr[((int64_t)pp << SP_KAP) + zl];
            } else if (pos > pp) {
                const V bq = rowr[((int64_t)pp << SP_KAP) + zl];
                re = sneg ? -bq : bq;
                im = sneg ? a : -a;
            } else {
                re = sneg ? (V)0 : a;
                im = sneg ? a : (V)0;
            }
        } else {
            const cplx<V> v = rowc[((int64_t)pos << SP_KAP) + zl];
            re = v.re;
            im = v.im;
        }
    };
    auto store = [&](int vec, int pos, V re, V im) {
        const uint32_t z = ((uint32_t)pos << SP_KAP) | (uint32_t)(z0 + vec);
        mul_ipow(__popc(x & z) & 3, re, im);
        put_final<V, HERM>(out, row * N + z, re * scale, im * scale);
    };
    LdsVecs<V, LOGM> lr{lds};
    LdsVecsW<V, LOGM> lw{lds};
    if constexpr (LOGM <= 4) {
        wht_round<V, LOGW, LOGM, 0, LOGM, NT, true>(load, store);
    } else {
        static_assert(LOGM <= 6, "n <= 16");
        wht_round<V, LOGW, LOGM, 0, 4, NT, true>(load, lw);
        __syncthreads();
        wht_round<V, LOGW, LOGM, 4, LOGM - 4, NT, true>(lr, store);
    }
}

// zero rows of the dense output whose X-pattern is not listed
template <class V, bool HERM>
__global__ void k_zero_unlisted(void* __restrict__ out, int n, int s)
{
    const int64_t N = (int64_t)1 << n;
    const int64_t total = N * N;
    constexpr int EB = HERM ? (int)sizeof(V) : 2 * (int)sizeof(V);  // output element bytes
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (N * EB >= 16 && ((uintptr_t)out & 15) == 0) {
        // whole 16-byte words of each unlisted row (rows are whole words)
        const int lw = n + (EB == 4 ? 2 : EB == 8 ? 3 : 4) - 4;  // log2 of words per row
        const int64_t words = total * EB / 16;
        uint4* w = (uint4*)out;
        const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
            if (!is_listed((uint32_t)(i >> lw), n, s)) w[i] = zero;
        return;
    }
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const uint32_t x = (uint32_t)(e >> n);
        if (!is_listed(x, n, s)) put_final<V, HERM>(out, e, (V)0, (V)0);
    }
}

template <class V, int SRC, bool HERM>
hipError_t struct_launch(int n, int s, int count, bool compact, const void* A, int64_t lda, void* out,
                         const uint32_t* xs, hipStream_t st)
{
    const cplx<V>* a = (const cplx<V>*)A;
    if (!compact && SRC != SRC_ROWS) {
        // plain 16-byte stores, one 256-thread workgroup per CU: the shape of
        // the fastest write-only sweep
        hipLaunchKernelGGL((k_zero_unlisted<V, HERM>), dim3(device_cu_count()), dim3(256), 0, st, out, n, s);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int cp = compact ? 1 : 0;
    if (n <= 10) {
        const dim3 grid((count + SM_VECS - 1) / SM_VECS);
        switch (n) {
#define PTD_CASE(NN)                                                                                      \
    case NN:                                                                                              \
        hipLaunchKernelGGL((k_struct_small<V, NN, SRC, HERM>), grid, dim3(SM_THREADS), 0, st, a, lda, s, \
                           count, cp, out, xs);                                                           \
        break;
            PTD_CASE(1) PTD_CASE(2) PTD_CASE(3) PTD_CASE(4) PTD_CASE(5)
            PTD_CASE(6) PTD_CASE(7) PTD_CASE(8) PTD_CASE(9) PTD_CASE(10)
#undef PTD_CASE
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_struct_p1<V, SRC, HERM>), dim3(count, 1u << (n - SP_KAP)), dim3(SM_THREADS), 0, st, a,
                       lda, s, n, cp, out, xs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 g2(count, 1u << (SP_KAP - 4));
    switch (n - SP_KAP) {
#define PTD_CASE(MM) \
    case MM: hipLaunchKernelGGL((k_struct_p2<V, MM, HERM>), g2, dim3(SM_THREADS), 0, st, s, n, cp, out, xs); break;
        PTD_CASE(1) PTD_CASE(2) PTD_CASE(3) PTD_CASE(4) PTD_CASE(5) PTD_CASE(6)
#undef PTD_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- sparse
// A sparse matrix given by nnz coordinate entries (r, c, v), or in
// compressed-row form: its strings with X-pattern x read only entries
// (k, k ^ x), so the X-patterns that can carry a nonzero coefficient are the
// distinct r ^ c, the same argument as for the diagonal and band cases
// above.  Entries with r or c outside [0, 2^n) are ignored.

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t count, uint32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// zero `words` 16-byte words (the output before the scatter)
__global__ void k_zero_words16(uint4* __restrict__ p, int64_t words)
{
    const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = zero;
}

__global__ void k_mark_x(const int32_t* __restrict__ rows, const int32_t* __restrict__ cols, int64_t nnz, int n,
                         uint32_t* __restrict__ flags)
{
    const int32_t N = 1 << n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = rows[e], c = cols[e];
        if (r >= 0 && r < N && c >= 0 && c < N) flags[r ^ c] = 1u;
    }
}

// One workgroup lists the flagged X-patterns in ascending order: each thread
// counts a contiguous slice, a scan of the counts gives its first slot.
constexpr int LIST_THREADS = 1024;
__global__ __launch_bounds__(LIST_THREADS) void k_list_x(const uint32_t* __restrict__ flags, int n,
                                                          uint32_t* __restrict__ xs, uint32_t* __restrict__ count)
{
    __shared__ uint32_t part[LIST_THREADS];
    const int N = 1 << n;
    const int per = (N + LIST_THREADS - 1) / LIST_THREADS;
    const int lo = (int)threadIdx.x * per;
    const int hi = lo + per < N ? lo + per : N;
    uint32_t c = 0;
    for (int x = lo; x < hi; ++x) c += flags[x] ? 1u : 0u;
    part[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < LIST_THREADS; off <<= 1) {  // inclusive scan
        const uint32_t v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t pos = part[threadIdx.x] - c;
    for (int x = lo; x < hi; ++x)
        if (flags[x]) xs[pos++] = (uint32_t)x;
    if (threadIdx.x == LIST_THREADS - 1) count[0] = part[LIST_THREADS - 1];
}

// bad[0] = 1 unless xs[0..count) is strictly ascending inside [0, 2^n)
__global__ void k_check_xs(const uint32_t* __restrict__ xs, int count, int n, uint32_t* __restrict__ bad)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const uint32_t x = xs[i];
        if (x >= (1u << n) || (i > 0 && xs[i - 1] >= x)) bad[0] = 1u;
    }
}

// xpos[xs[i]] = i (xpos preset to -1)
__global__ void k_xpos(const uint32_t* __restrict__ xs, int count, int32_t* __restrict__ xpos)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) xpos[xs[i]] = i;
}

// d_x[r] += v for every entry (r, r ^ x, v) with x listed: added atomically
// into the zeroed output row of x, so repeated coordinates are summed
template <class V>
__global__ void k_scatter(const int32_t* __restrict__ rows, const int32_t* __restrict__ cols,
                          const cplx<V>* __restrict__ vals, int64_t nnz, int n, const int32_t* __restrict__ xpos,
                          int compact, cplx<V>* __restrict__ out)
{
    const int32_t N = 1 << n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = rows[e], c = cols[e];
        if (r < 0 || r >= N || c < 0 || c >= N) continue;
        const int32_t x = r ^ c;
        const int32_t i = xpos[x];
        if (i < 0) continue;
        const cplx<V> v = vals[e];
        V* p = (V*)(out + (((int64_t)(compact ? i : x)) << n) + r);
        __hip_atomic_fetch_add(p, v.re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(p + 1, v.im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Compressed-row input: row r holds the entries row_ptr[r] .. row_ptr[r+1]-1
// of cols / vals, the range clipped to [0, nnz) (its end raised to its start
// where below it), so every access stays inside the caller's arrays whatever
// the pointers hold.  One wave per row, its lanes over the row's entries
// (consecutive, so the column and value loads of a wave are coalesced).
constexpr int CSR_THREADS = 256;
constexpr int CSR_WAVES = CSR_THREADS / 64;

__device__ __forceinline__ void csr_range(const int64_t* __restrict__ row_ptr, int r, int64_t nnz, int64_t& lo,
                                          int64_t& hi)
{
    const int64_t a = row_ptr[r], b = row_ptr[r + 1];
    lo = a < 0 ? 0 : (a > nnz ? nnz : a);
    hi = b < lo ? lo : (b > nnz ? nnz : b);
}

__global__ __launch_bounds__(CSR_THREADS) void k_mark_x_csr(const int64_t* __restrict__ row_ptr,
                                                             const int32_t* __restrict__ cols, int64_t nnz, int n,
                                                             uint32_t* __restrict__ flags)
{
    const int32_t N = 1 << n;
    const int lane = threadIdx.x & 63;
    for (int r = blockIdx.x * CSR_WAVES + (int)(threadIdx.x >> 6); r < N; r += gridDim.x * CSR_WAVES) {
        int64_t lo, hi;
        csr_range(row_ptr, r, nnz, lo, hi);
        for (int64_t e = lo + lane; e < hi; e += 64) {
            const int32_t c = cols[e];
            if (c >= 0 && c < N) flags[r ^ c] = 1u;
        }
    }
}

// d_x[r] += v for the entries (r, c, v) of row r with x = r ^ c listed,
// atomically as for coordinate input (a row may repeat a column)
template <class V>
__global__ __launch_bounds__(CSR_THREADS) void k_scatter_csr(const int64_t* __restrict__ row_ptr,
                                                              const int32_t* __restrict__ cols,
                                                              const cplx<V>* __restrict__ vals, int64_t nnz, int n,
                                                              const int32_t* __restrict__ xpos, int compact,
                                                              cplx<V>* __restrict__ out)
{
    const int32_t N = 1 << n;
    const int lane = threadIdx.x & 63;
    for (int r = blockIdx.x * CSR_WAVES + (int)(threadIdx.x >> 6); r < N; r += gridDim.x * CSR_WAVES) {
        int64_t lo, hi;
        csr_range(row_ptr, r, nnz, lo, hi);
        for (int64_t e = lo + lane; e < hi; e += 64) {
            const int32_t c = cols[e];
            if (c < 0 || c >= N) continue;
            const int32_t x = r ^ c;
            const int32_t i = xpos[x];
            if (i < 0) continue;
            const cplx<V> v = vals[e];
            V* p = (V*)(out + (((int64_t)(compact ? i : x)) << n) + r);
            __hip_atomic_fetch_add(p, v.re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(p + 1, v.im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

int csr_grid(int n)
{
    const int rows_blocks = ((1 << n) + CSR_WAVES - 1) / CSR_WAVES;
    return rows_blocks < 8192 ? rows_blocks : 8192;
}

// rows == nullptr: the entries are in compressed-row form (row_ptr)
template <class V>
hipError_t sparse_t(int n, bool compact, int64_t nnz, const int32_t* rows, const int64_t* row_ptr,
                    const int32_t* cols, const void* vals, const uint32_t* xs, int count, void* out, void* ws,
                    bool* bad_xs, hipStream_t st)
{
    const int64_t N = (int64_t)1 << n;
    int32_t* xpos = (int32_t*)ws;
    uint32_t* bad = (uint32_t*)((unsigned char*)ws + sparse_workspace_bytes(n) - 256);
    const int grid = 1024;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, bad, (int64_t)1, 0u);
    hipLaunchKernelGGL(k_check_xs, dim3(grid), dim3(256), 0, st, xs, count, n, bad);
    uint32_t h = 1;
    hipError_t e = hipMemcpyAsync(&h, bad, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    *bad_xs = h != 0;
    if (*bad_xs) return hipSuccess;
    // zero the output (compact rows, or the whole dense array), scatter, then
    // the transform in place over the listed rows
    const int64_t out_bytes = (compact ? (int64_t)count * N : N * N) * (int64_t)sizeof(cplx<V>);
    if (((uintptr_t)out & 15) == 0 && (out_bytes & 15) == 0)  // plain 16-byte stores, one workgroup per CU
        hipLaunchKernelGGL(k_zero_words16, dim3(device_cu_count()), dim3(256), 0, st, (uint4*)out, out_bytes / 16);
    else
        hipLaunchKernelGGL(k_fill_u32, dim3(4096), dim3(256), 0, st, (uint32_t*)out, out_bytes / 4, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, st, (uint32_t*)xpos, N, 0xffffffffu);
    hipLaunchKernelGGL(k_xpos, dim3(grid), dim3(256), 0, st, xs, count, xpos);
    if (nnz > 0 && rows)
        hipLaunchKernelGGL(k_scatter<V>, dim3(4096), dim3(256), 0, st, rows, cols, (const cplx<V>*)vals, nnz, n,
                           xpos, compact ? 1 : 0, (cplx<V>*)out);
    else if (nnz > 0)
        hipLaunchKernelGGL(k_scatter_csr<V>, dim3(csr_grid(n)), dim3(CSR_THREADS), 0, st, row_ptr, cols,
                           (const cplx<V>*)vals, nnz, n, xpos, compact ? 1 : 0, (cplx<V>*)out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (count == 0) return hipSuccess;
    return struct_launch<V, SRC_ROWS, false>(n, 0, count, compact, nullptr, 0, out, xs, st);
}

}  // namespace

hipError_t launch_structured(int n, ptd_dtype dt, bool herm, bool bands, bool compact, int s, int count,
                             const void* A, int64_t lda, void* out, hipStream_t st)
{
    if (dt == PTD_C128) {
        if (bands)
            return herm ? struct_launch<double, SRC_BANDS, true>(n, s, count, compact, A, lda, out, nullptr, st)
                        : struct_launch<double, SRC_BANDS, false>(n, s, count, compact, A, lda, out, nullptr, st);
        return herm ? struct_launch<double, SRC_DENSE, true>(n, s, count, compact, A, lda, out, nullptr, st)
                    : struct_launch<double, SRC_DENSE, false>(n, s, count, compact, A, lda, out, nullptr, st);
    }
    if (bands)
        return herm ? struct_launch<float, SRC_BANDS, true>(n, s, count, compact, A, lda, out, nullptr, st)
                    : struct_launch<float, SRC_BANDS, false>(n, s, count, compact, A, lda, out, nullptr, st);
    return herm ? struct_launch<float, SRC_DENSE, true>(n, s, count, compact, A, lda, out, nullptr, st)
                : struct_launch<float, SRC_DENSE, false>(n, s, count, compact, A, lda, out, nullptr, st);
}

size_t sparse_workspace_bytes(int n) { return ((size_t)4 << n) + 256; }

hipError_t launch_sparse_nonempty_x(int n, int64_t nnz, const int32_t* rows, const int64_t* row_ptr,
                                    const int32_t* cols, uint32_t* xs, int* count_host, void* ws, hipStream_t st)
{
    uint32_t* flags = (uint32_t*)ws;
    uint32_t* cnt = (uint32_t*)((unsigned char*)ws + sparse_workspace_bytes(n) - 256);
    hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, st, flags, (int64_t)1 << n, 0u);
    if (nnz > 0 && rows) hipLaunchKernelGGL(k_mark_x, dim3(4096), dim3(256), 0, st, rows, cols, nnz, n, flags);
    else if (nnz > 0)
        hipLaunchKernelGGL(k_mark_x_csr, dim3(csr_grid(n)), dim3(CSR_THREADS), 0, st, row_ptr, cols, nnz, n, flags);
    hipLaunchKernelGGL(k_list_x, dim3(1), dim3(LIST_THREADS), 0, st, flags, n, xs, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t h = 0;
    e = hipMemcpyAsync(&h, cnt, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    *count_host = (int)h;
    return hipSuccess;
}

hipError_t launch_sparse(int n, ptd_dtype dt, bool compact, int64_t nnz, const int32_t* rows, const int64_t* row_ptr,
                         const int32_t* cols, const void* vals, const uint32_t* xs, int count, void* out, void* ws,
                         bool* bad_xs, hipStream_t st)
{
    return dt == PTD_C128
               ? sparse_t<double>(n, compact, nnz, rows, row_ptr, cols, vals, xs, count, out, ws, bad_xs, st)
               : sparse_t<float>(n, compact, nnz, rows, row_ptr, cols, vals, xs, count, out, ws, bad_xs, st);
}

}  // namespace ptd
