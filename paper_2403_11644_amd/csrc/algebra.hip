// algebra.hip -- coefficient arrays of matrices assembled from matrices whose
// coefficients are known (Sec. IV-B): block-diagonal assembly and its m = 1
// case the direct sum, Hermitian augmentation, linear combination.  Each is
// one pass over HBM (read the inputs once, write the output once), so the
// kernels are streams with coalesced row accesses, each workgroup over one
// contiguous range; the block-diagonal one applies a length-2^m transform
// over the block index in registers.
#include "engine.hpp"
#include "internal.hpp"

namespace ptd {

namespace {

constexpr int ALG_THREADS = 256;

int alg_grid() { return device_cu_count() * 8; }

// The one-pass combinations run in the shape of the fastest copy measured on
// MI355X: one 1024-thread workgroup per CU, each owning one contiguous range
// of positions, non-temporal loads and stores.
constexpr int ALG_BLK_THREADS = 1024;

int alg_blk_grid() { return device_cu_count(); }

__device__ __forceinline__ void block_range(int64_t count, int64_t& lo, int64_t& hi)
{
    const int64_t per = (count + gridDim.x - 1) / gridDim.x;
    lo = (int64_t)blockIdx.x * per;
    hi = lo + per < count ? lo + per : count;
}

template <class V>
__device__ __forceinline__ cplx<V> ld_nt(const cplx<V>* p)
{
    typedef V v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load((const v2*)p);
    cplx<V> c;
    c.re = v.x;
    c.im = v.y;
    return c;
}

template <class V>
__device__ __forceinline__ void st_nt(cplx<V>* p, V re, V im)
{
    typedef V v2 __attribute__((ext_vector_type(2)));
    v2 v;
    v.x = re;
    v.y = im;
    __builtin_nontemporal_store(v, (v2*)p);
}

// Output element (x, (t << k) | z) of diag(A_0, ..., A_{2^M - 1}) for every
// input position idx = x * 2^k + z < count = 4^k: the sum over blocks i of
// (-1)^popcount(t & i) c_i[idx], times 2^-M.  The pairwise direct sums of the
// paper, (A_0 (+) A_1) (+) (A_2 (+) A_3) and so on, each combine two halves
// with (a + b) / 2 and (a - b) / 2 on a new top qubit; unrolled, that is this
// transform, and wht_reg applies its radix-2 stages in the same order (lowest
// block bit first), with the halvings gathered into one exact 2^-M.
// (One position per thread and grid step: unrolling four to eight positions
// per thread to put more loads in flight measured 5-10% slower.)
template <class V, int M>
__global__ __launch_bounds__(ALG_BLK_THREADS) void k_block_diag(BlockPtrs blocks, cplx<V>* __restrict__ out, int k,
                                                                int64_t count)
{
    constexpr int NB = 1 << M;
    const V scale = exp2_neg<V>(M);
    const int64_t zmask = ((int64_t)1 << k) - 1;
    const int64_t pitch = (int64_t)1 << (k + M);
    int64_t lo, hi;
    block_range(count, lo, hi);
    for (int64_t idx = lo + threadIdx.x; idx < hi; idx += ALG_BLK_THREADS) {
        V re[NB], im[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const cplx<V> c = ld_nt<V>((const cplx<V>*)blocks.p[i] + idx);
            re[i] = c.re;
            im[i] = c.im;
        }
        wht_reg<V, M>(re, im);
        cplx<V>* row = out + (idx >> k) * pitch + (idx & zmask);
#pragma unroll
        for (int t = 0; t < NB; ++t) st_nt<V>(row + ((int64_t)t << k), re[t] * scale, im[t] * scale);
    }
}

// X on the new top qubit carries Re c, Y carries Im c: row 2^n + x (row x when
// compact) of the 2^(n+1)-wide real output gets Re c[x][z] at z and Im c[x][z]
// at 2^n + z.
template <class V>
__global__ __launch_bounds__(ALG_BLK_THREADS) void k_herm_augment(const cplx<V>* __restrict__ in,
                                                                  V* __restrict__ out, int n, int compact,
                                                                  int64_t count)
{
    const int64_t zmask = ((int64_t)1 << n) - 1;
    const int64_t half = (int64_t)1 << n;
    int64_t lo, hi;
    block_range(count, lo, hi);
    for (int64_t idx = lo + threadIdx.x; idx < hi; idx += ALG_BLK_THREADS) {
        const cplx<V> c = ld_nt<V>(in + idx);
        const int64_t x = idx >> n, z = idx & zmask;
        V* row = out + ((compact ? 0 : half) + x) * (half << 1);
        __builtin_nontemporal_store(c.re, row + z);
        __builtin_nontemporal_store(c.im, row + half + z);
    }
}

// out = mu * a + b, each part rounded in this order (no fused multiply-add).
template <class V>
__global__ __launch_bounds__(ALG_BLK_THREADS) void k_lincomb(const cplx<V>* a, const cplx<V>* b, cplx<V>* out, V mr,
                                                             V mi, int64_t count)
{
    int64_t lo, hi;
    block_range(count, lo, hi);
    for (int64_t idx = lo + threadIdx.x; idx < hi; idx += ALG_BLK_THREADS) {
        const cplx<V> u = ld_nt<V>(a + idx), v = ld_nt<V>(b + idx);
        st_nt<V>(out + idx, (mr * u.re - mi * u.im) + v.re, (mr * u.im + mi * u.re) + v.im);
    }
}

__global__ __launch_bounds__(ALG_THREADS) void k_zero16(uint4* __restrict__ p, int64_t count)
{
    const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = zero;
}

// dst (2^n x 2^n, contiguous) = src (rows x cols at pitch ld) in the
// top-left corner, zero elsewhere.
template <class V>
__global__ __launch_bounds__(ALG_THREADS) void k_zero_pad(const cplx<V>* __restrict__ src, int64_t ld, int64_t rows,
                                                         int64_t cols, int n, cplx<V>* __restrict__ dst)
{
    const int64_t N = (int64_t)1 << n;
    const int64_t total = N * N;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i >> n, c = i & (N - 1);
        cplx<V> v;
        v.re = (V)0;
        v.im = (V)0;
        if (r < rows && c < cols) v = src[r * ld + c];
        dst[i] = v;
    }
}

// Zero `bytes` (a multiple of 16) at p.
hipError_t zero_bytes(void* p, int64_t bytes, hipStream_t st)
{
    if (bytes <= 0) return hipSuccess;
    // one 256-thread workgroup per CU: the shape of the fastest write-only sweep
    hipLaunchKernelGGL(k_zero16, dim3(device_cu_count()), dim3(ALG_THREADS), 0, st, (uint4*)p, bytes / 16);
    return hipGetLastError();
}

template <class V>
hipError_t block_diag_t(int k, int m, bool compact, const BlockPtrs& blocks, void* out, hipStream_t st)
{
    const int64_t count = (int64_t)1 << (2 * k);
    switch (m) {
#define PTD_M(MM)                                                                                         \
    case MM:                                                                                              \
        hipLaunchKernelGGL((k_block_diag<V, MM>), dim3(alg_blk_grid()), dim3(ALG_BLK_THREADS), 0, st, blocks,     \
                           (cplx<V>*)out, k, count);                                                      \
        break;
        PTD_M(1) PTD_M(2) PTD_M(3) PTD_M(4) PTD_M(5)
#undef PTD_M
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || compact) return e;
    // rows 2^k .. 2^(k+m) - 1 of the dense output: every string with X or Y
    // on a new qubit has coefficient zero
    const int64_t pitch = (int64_t)1 << (k + m);
    const int64_t first = ((int64_t)1 << k) * pitch;
    return zero_bytes((cplx<V>*)out + first, (pitch * pitch - first) * (int64_t)sizeof(cplx<V>), st);
}

template <class V>
hipError_t herm_augment_t(int n, bool compact, const void* in, void* out, hipStream_t st)
{
    const int64_t count = (int64_t)1 << (2 * n);
    hipLaunchKernelGGL(k_herm_augment<V>, dim3(alg_blk_grid()), dim3(ALG_BLK_THREADS), 0, st, (const cplx<V>*)in,
                       (V*)out, n,
                       compact ? 1 : 0, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || compact) return e;
    // rows 0 .. 2^n - 1: strings with I or Z on the new qubit are absent
    return zero_bytes(out, ((int64_t)1 << n) * ((int64_t)2 << n) * (int64_t)sizeof(V), st);
}

}  // namespace

hipError_t launch_block_diagonal(int k, int m, ptd_dtype dt, bool compact, const BlockPtrs& blocks, void* out,
                                 hipStream_t st)
{
    return dt == PTD_C128 ? block_diag_t<double>(k, m, compact, blocks, out, st)
                          : block_diag_t<float>(k, m, compact, blocks, out, st);
}

hipError_t launch_hermitian_augment(int n, ptd_dtype dt, bool compact, const void* in, void* out, hipStream_t st)
{
    return dt == PTD_C128 ? herm_augment_t<double>(n, compact, in, out, st)
                          : herm_augment_t<float>(n, compact, in, out, st);
}

hipError_t launch_zero_pad(ptd_dtype dt, const void* src, int64_t ld, int64_t rows, int64_t cols, int n, void* dst,
                           hipStream_t st)
{
    if (dt == PTD_C128)
        hipLaunchKernelGGL(k_zero_pad<double>, dim3(alg_grid()), dim3(ALG_THREADS), 0, st, (const cplx<double>*)src, ld,
                           rows, cols, n, (cplx<double>*)dst);
    else
        hipLaunchKernelGGL(k_zero_pad<float>, dim3(alg_grid()), dim3(ALG_THREADS), 0, st, (const cplx<float>*)src, ld,
                           rows, cols, n, (cplx<float>*)dst);
    return hipGetLastError();
}

hipError_t launch_linear_combination(int n, ptd_dtype dt, double mu_re, double mu_im, const void* a, const void* b,
                                     void* out, hipStream_t st)
{
    const int64_t count = (int64_t)1 << (2 * n);
    if (dt == PTD_C128)
        hipLaunchKernelGGL(k_lincomb<double>, dim3(alg_blk_grid()), dim3(ALG_BLK_THREADS), 0, st, (const cplx<double>*)a,
                           (const cplx<double>*)b, (cplx<double>*)out, mu_re, mu_im, count);
    else
        hipLaunchKernelGGL(k_lincomb<float>, dim3(alg_blk_grid()), dim3(ALG_BLK_THREADS), 0, st, (const cplx<float>*)a,
                           (const cplx<float>*)b, (cplx<float>*)out, (float)mu_re, (float)mu_im, count);
    return hipGetLastError();
}

}  // namespace ptd
