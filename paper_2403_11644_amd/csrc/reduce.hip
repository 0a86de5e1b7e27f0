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
constexpr int RED_UNROLL = 4;  // independent loads in flight per thread

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

// sum of |A[r][c]|^2 over the 2^n x 2^n matrix with row pitch lda; every
// thread walks a fixed index sequence, RED_UNROLL loads at a time
template <class V>
__global__ __launch_bounds__(RED_THREADS) void k_sumsq_matrix(const cplx<V>* __restrict__ A, int64_t lda, int n,
                                                               double* __restrict__ partial)
{
    __shared__ double sh[RED_THREADS];
    const int64_t N = (int64_t)1 << n;
    const int64_t total = N * N;
    const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
    double acc = 0.0;
    for (int64_t i0 = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i0 < total; i0 += stride * RED_UNROLL) {
        cplx<V> v[RED_UNROLL];
#pragma unroll
        for (int u = 0; u < RED_UNROLL; ++u) {
            const int64_t i = i0 + u * stride;
            if (i < total) {
                v[u] = A[(i >> n) * lda + (i & (N - 1))];
            } else {
                v[u].re = (V)0;
                v[u].im = (V)0;
            }
        }
#pragma unroll
        for (int u = 0; u < RED_UNROLL; ++u) {
            const double a = (double)v[u].re, b = (double)v[u].im;
            acc += a * a;
            acc += b * b;
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// sum of squares of `count` real values: 16-byte loads over the body when
// the pointer is 16-byte aligned, scalar loads otherwise
template <class V>
__global__ __launch_bounds__(RED_THREADS) void k_sumsq_vec(const V* __restrict__ v, int64_t count,
                                                            double* __restrict__ partial)
{
    __shared__ double sh[RED_THREADS];
    constexpr int PER = 16 / sizeof(V);
    typedef V vec_t __attribute__((ext_vector_type(PER)));
    const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
    const int64_t tid = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x;
    double acc = 0.0;
    int64_t body = 0;
    if (((uintptr_t)v & 15) == 0) {
        const vec_t* w = (const vec_t*)v;
        const int64_t nw = count / PER;
        body = nw * PER;
        for (int64_t i0 = tid; i0 < nw; i0 += stride * RED_UNROLL) {
            vec_t x[RED_UNROLL];
#pragma unroll
            for (int u = 0; u < RED_UNROLL; ++u) {
                const int64_t i = i0 + u * stride;
                if (i < nw) {
                    x[u] = w[i];
                } else {
#pragma unroll
                    for (int e = 0; e < PER; ++e) x[u][e] = (V)0;
                }
            }
#pragma unroll
            for (int u = 0; u < RED_UNROLL; ++u) {
#pragma unroll
                for (int e = 0; e < PER; ++e) {
                    const double a = (double)x[u][e];
                    acc += a * a;
                }
            }
        }
    }
    for (int64_t i = body + tid; i < count; i += stride) {
        const double a = (double)v[i];
        acc += a * a;
    }
    const double s = block_sum(acc, sh);
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

// 1-norm sum_P |c_P| in float64: |c| = sqrt(re^2 + im^2) for complex c, the
// absolute value for real c (count values of the array's element type)
template <class V, bool REAL>
__global__ __launch_bounds__(RED_THREADS) void k_abssum(const void* __restrict__ c, int64_t count,
                                                         double* __restrict__ partial)
{
    __shared__ double sh[RED_THREADS];
    const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < count; i += stride) {
        if constexpr (REAL) {
            const double a = (double)((const V*)c)[i];
            acc += a < 0 ? -a : a;
        } else {
            const cplx<V> v = ((const cplx<V>*)c)[i];
            const double a = (double)v.re, b = (double)v.im;
            acc += sqrt(a * a + b * b);
        }
    }
    const double s = block_sum(acc, sh);
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
// evaluated in float64 and rounded once to V
template <class V, bool REAL>
__global__ __launch_bounds__(RED_THREADS) void k_lcu_amp(const void* __restrict__ c, V* __restrict__ amp,
                                                          int64_t count, const double* __restrict__ norm1)
{
    const double lam = *norm1;
    const double inv = lam > 0.0 ? 1.0 / lam : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * RED_THREADS) {
        double a;
        if constexpr (REAL) {
            a = (double)((const V*)c)[i];
            a = a < 0 ? -a : a;
        } else {
            const cplx<V> v = ((const cplx<V>*)c)[i];
            const double x = (double)v.re, y = (double)v.im;
            a = sqrt(x * x + y * y);
        }
        amp[i] = (V)sqrt(a * inv);
    }
}

template <class V, bool REAL>
hipError_t lcu_t(int64_t count, const void* c, void* amp, double* partial, double* fin, hipStream_t st)
{
    hipLaunchKernelGGL((k_abssum<V, REAL>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, c, count, partial);
    hipLaunchKernelGGL(k_finish1, dim3(1), dim3(RED_THREADS), 0, st, partial, RED_BLOCKS, fin);
    hipLaunchKernelGGL((k_lcu_amp<V, REAL>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, c, (V*)amp, count,
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
        hipLaunchKernelGGL(k_sumsq_matrix<double>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st,
                           (const cplx<double>*)A, lda, n, pa);
        hipLaunchKernelGGL(k_sumsq_vec<double>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, (const double*)coeff,
                           count, pc);
    } else {
        hipLaunchKernelGGL(k_sumsq_matrix<float>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st,
                           (const cplx<float>*)A, lda, n, pa);
        hipLaunchKernelGGL(k_sumsq_vec<float>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st, (const float*)coeff,
                           count, pc);
    }
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(RED_THREADS), 0, st, pa, pc, RED_BLOCKS, fin);
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
