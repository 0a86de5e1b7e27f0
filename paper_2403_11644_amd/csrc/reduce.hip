// reduce.hip -- float64 norm reductions: the Parseval residual and the
// 1-norm behind the LCU state preparation.
//
// Theorem 1 of the paper makes the Pauli strings orthogonal with
// Tr(P^* P) = 2^n, hence ||A||_F^2 = 2^n sum_P |c_P|^2.  Both sides are summed
// here in float64 (also for complex64 data) with a fixed two-level tree, so
// the result is deterministic for a given input.
#include "engine.hpp"
#include "internal.hpp"

namespace ptd {

namespace {

constexpr int RED_BLOCKS = 2048;
constexpr int RED_THREADS = 256;

__device__ __forceinline__ double block_sum(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

// The Parseval sums read A and c once each: PAR_BLOCKS workgroups of
// PAR_THREADS threads, each block owning one contiguous range, PAR_U
// non-temporal 16-byte (complex128) loads in flight per thread: the shape
// of the fastest read-only sweep on MI355X (7.2 TB/s, one workgroup per CU).
// The block count is fixed, so the summation tree, and the float64 result,
// is the same on every device.
constexpr int PAR_BLOCKS = 256;
constexpr int PAR_THREADS = 512;
constexpr int PAR_U = 4;
static_assert(PAR_BLOCKS <= RED_BLOCKS, "partial sums fit the workspace");

__device__ __forceinline__ double block_sum_par(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = PAR_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

template <class V>
__device__ __forceinline__ void ld_pair_nt(const V* p, double& a, double& b)
{
    typedef V v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load((const v2*)p);
    a = (double)v.x;
    b = (double)v.y;
}

// sum of |A[r][c]|^2 over the 2^n x 2^n matrix with row pitch lda, in row-
// major order of the flattened index
template <class V>
__global__ __launch_bounds__(PAR_THREADS) void k_sumsq_matrix(const cplx<V>* __restrict__ A, int64_t lda, int n,
                                                              double* __restrict__ partial)
{
    __shared__ double sh[PAR_THREADS];
    const int64_t N = (int64_t)1 << n;
    const int64_t total = N * N;
    const int64_t per = (total + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < total ? lo + per : total;
    double acc = 0.0;
    int64_t i = lo + threadIdx.x;
    for (; i + (PAR_U - 1) * PAR_THREADS < hi; i += PAR_U * PAR_THREADS) {
        double a[PAR_U], b[PAR_U];
#pragma unroll
        for (int u = 0; u < PAR_U; ++u) {
            const int64_t k = i + u * PAR_THREADS;
            ld_pair_nt<V>((const V*)(A + (k >> n) * lda + (k & (N - 1))), a[u], b[u]);
        }
#pragma unroll
        for (int u = 0; u < PAR_U; ++u) {
            acc += a[u] * a[u];
            acc += b[u] * b[u];
        }
    }
    for (; i < hi; i += PAR_THREADS) {
        double a, b;
        ld_pair_nt<V>((const V*)(A + (i >> n) * lda + (i & (N - 1))), a, b);
        acc += a * a;
        acc += b * b;
    }
    const double s = block_sum_par(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// sum of squares of `count` real values: blocked 16-byte non-temporal loads
// over the body when the pointer is 16-byte aligned, the rest (or all of it
// when not aligned) with scalar loads
template <class V>
__global__ __launch_bounds__(PAR_THREADS) void k_sumsq_vec(const V* __restrict__ v, int64_t count,
                                                           double* __restrict__ partial)
{
    __shared__ double sh[PAR_THREADS];
    constexpr int PER = 16 / sizeof(V);
    typedef V vec_t __attribute__((ext_vector_type(PER)));
    double acc = 0.0;
    int64_t body = 0;
    if (((uintptr_t)v & 15) == 0) {
        const vec_t* w = (const vec_t*)v;
        const int64_t nw = count / PER;
        body = nw * PER;
        const int64_t per = (nw + gridDim.x - 1) / gridDim.x;
        const int64_t lo = (int64_t)blockIdx.x * per;
        const int64_t hi = lo + per < nw ? lo + per : nw;
        int64_t i = lo + threadIdx.x;
        for (; i + (PAR_U - 1) * PAR_THREADS < hi; i += PAR_U * PAR_THREADS) {
            vec_t x[PAR_U];
#pragma unroll
            for (int u = 0; u < PAR_U; ++u) x[u] = __builtin_nontemporal_load(w + i + u * PAR_THREADS);
#pragma unroll
            for (int u = 0; u < PAR_U; ++u) {
#pragma unroll
                for (int e = 0; e < PER; ++e) {
                    const double a = (double)x[u][e];
                    acc += a * a;
                }
            }
        }
        for (; i < hi; i += PAR_THREADS) {
            const vec_t x = __builtin_nontemporal_load(w + i);
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const double a = (double)x[e];
                acc += a * a;
            }
        }
    }
    const int64_t stride = (int64_t)gridDim.x * PAR_THREADS;
    for (int64_t i = body + (int64_t)blockIdx.x * PAR_THREADS + threadIdx.x; i < count; i += stride) {
        const double a = (double)v[i];
        acc += a * a;
    }
    const double s = block_sum_par(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(RED_THREADS) void k_finish(const double* __restrict__ pa, const double* __restrict__ pc,
                                                        int nblk, double* __restrict__ out2)
{
    __shared__ double sh[RED_THREADS];
    double a = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < nblk; i += RED_THREADS) {
        a += pa[i];
        c += pc[i];
    }
    const double sa = block_sum(a, sh);
    __syncthreads();
    const double sc = block_sum(c, sh);
    if (threadIdx.x == 0) {
        out2[0] = sa;
        out2[1] = sc;
    }
}

// |c_i| in float64: sqrt(re^2 + im^2) for complex c, the absolute value for
// real c (non-temporal loads)
template <class V, bool REAL>
__device__ __forceinline__ double abs_at(const void* __restrict__ c, int64_t i)
{
    if constexpr (REAL) {
        const double a = (double)__builtin_nontemporal_load((const V*)c + i);
        return a < 0 ? -a : a;
    } else {
        double a, b;
        ld_pair_nt<V>((const V*)((const cplx<V>*)c + i), a, b);
        return sqrt(a * a + b * b);
    }
}

// 1-norm sum_P |c_P| in float64 over `count` values of the array's element
// type, in the blocked shape of the Parseval sums (fixed tree)
template <class V, bool REAL>
__global__ __launch_bounds__(PAR_THREADS) void k_abssum(const void* __restrict__ c, int64_t count,
                                                        double* __restrict__ partial)
{
    __shared__ double sh[PAR_THREADS];
    const int64_t per = (count + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < count ? lo + per : count;
    double acc = 0.0;
    int64_t i = lo + threadIdx.x;
    for (; i + (PAR_U - 1) * PAR_THREADS < hi; i += PAR_U * PAR_THREADS) {
        double a[PAR_U];
#pragma unroll
        for (int u = 0; u < PAR_U; ++u) a[u] = abs_at<V, REAL>(c, i + u * PAR_THREADS);
#pragma unroll
        for (int u = 0; u < PAR_U; ++u) acc += a[u];
    }
    for (; i < hi; i += PAR_THREADS) acc += abs_at<V, REAL>(c, i);
    const double s = block_sum_par(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(RED_THREADS) void k_finish1(const double* __restrict__ p, int nblk,
                                                         double* __restrict__ out)
{
    __shared__ double sh[RED_THREADS];
    double a = 0.0;
    for (int i = threadIdx.x; i < nblk; i += RED_THREADS) a += p[i];
    const double s = block_sum(a, sh);
    if (threadIdx.x == 0) out[0] = s;
}

// amp[i] = sqrt(|c_i| / lambda), lambda = *norm1 (0 for an all-zero array),
// evaluated in float64 and rounded once to V; blocked, non-temporal
template <class V, bool REAL>
__global__ __launch_bounds__(PAR_THREADS) void k_lcu_amp(const void* __restrict__ c, V* __restrict__ amp,
                                                         int64_t count, const double* __restrict__ norm1)
{
    const double lam = *norm1;
    const double inv = lam > 0.0 ? 1.0 / lam : 0.0;
    const int64_t per = (count + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < count ? lo + per : count;
    int64_t i = lo + threadIdx.x;
    for (; i + (PAR_U - 1) * PAR_THREADS < hi; i += PAR_U * PAR_THREADS) {
        double a[PAR_U];
#pragma unroll
        for (int u = 0; u < PAR_U; ++u) a[u] = abs_at<V, REAL>(c, i + u * PAR_THREADS);
#pragma unroll
        for (int u = 0; u < PAR_U; ++u) __builtin_nontemporal_store((V)sqrt(a[u] * inv), amp + i + u * PAR_THREADS);
    }
    for (; i < hi; i += PAR_THREADS) __builtin_nontemporal_store((V)sqrt(abs_at<V, REAL>(c, i) * inv), amp + i);
}

template <class V, bool REAL>
hipError_t lcu_t(int64_t count, const void* c, void* amp, double* partial, double* fin, hipStream_t st)
{
    hipLaunchKernelGGL((k_abssum<V, REAL>), dim3(PAR_BLOCKS), dim3(PAR_THREADS), 0, st, c, count, partial);
    hipLaunchKernelGGL(k_finish1, dim3(1), dim3(RED_THREADS), 0, st, partial, PAR_BLOCKS, fin);
    hipLaunchKernelGGL((k_lcu_amp<V, REAL>), dim3(PAR_BLOCKS), dim3(PAR_THREADS), 0, st, c, (V*)amp, count,
                       (const double*)fin);
    return hipGetLastError();
}

}  // namespace

size_t reduce_workspace_bytes() { return (size_t)(2 * RED_BLOCKS + 2) * sizeof(double); }

hipError_t launch_parseval(int n, ptd_dtype dt, bool real_coeff, const void* A, int64_t lda, const void* coeff,
                           void* ws, double* out_host, hipStream_t st)
{
    double* pa = (double*)ws;
    double* pc = pa + RED_BLOCKS;
    double* fin = pc + RED_BLOCKS;
    const int64_t count = ((int64_t)1 << (2 * n)) * (real_coeff ? 1 : 2);
    if (dt == PTD_C128) {
        hipLaunchKernelGGL(k_sumsq_matrix<double>, dim3(PAR_BLOCKS), dim3(PAR_THREADS), 0, st,
                           (const cplx<double>*)A, lda, n, pa);
        hipLaunchKernelGGL(k_sumsq_vec<double>, dim3(PAR_BLOCKS), dim3(PAR_THREADS), 0, st, (const double*)coeff,
                           count, pc);
    } else {
        hipLaunchKernelGGL(k_sumsq_matrix<float>, dim3(PAR_BLOCKS), dim3(PAR_THREADS), 0, st,
                           (const cplx<float>*)A, lda, n, pa);
        hipLaunchKernelGGL(k_sumsq_vec<float>, dim3(PAR_BLOCKS), dim3(PAR_THREADS), 0, st, (const float*)coeff,
                           count, pc);
    }
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(RED_THREADS), 0, st, pa, pc, PAR_BLOCKS, fin);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double h[2];
    e = hipMemcpyAsync(h, fin, sizeof h, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    out_host[0] = h[0];
    out_host[1] = h[1] * (double)((int64_t)1 << n);
    const double d = out_host[0] - out_host[1];
    out_host[2] = (d < 0 ? -d : d) / (out_host[0] > 0 ? out_host[0] : 1.0);
    return hipSuccess;
}

hipError_t launch_lcu_amplitudes(int n, ptd_dtype dt, bool real_coeff, const void* coeff, void* amp, void* ws,
                                 double* lambda_host, hipStream_t st)
{
    double* partial = (double*)ws;
    double* fin = partial + RED_BLOCKS;
    const int64_t count = (int64_t)1 << (2 * n);
    hipError_t e;
    if (dt == PTD_C128)
        e = real_coeff ? lcu_t<double, true>(count, coeff, amp, partial, fin, st)
                       : lcu_t<double, false>(count, coeff, amp, partial, fin, st);
    else
        e = real_coeff ? lcu_t<float, true>(count, coeff, amp, partial, fin, st)
                       : lcu_t<float, false>(count, coeff, amp, partial, fin, st);
    if (e != hipSuccess) return e;
    double h = 0.0;
    e = hipMemcpyAsync(&h, fin, sizeof h, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    *lambda_host = h;
    return hipSuccess;
}

}  // namespace ptd
