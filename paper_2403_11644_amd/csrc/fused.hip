// fused.hip -- host side of the single-launch dense schedule (fused.hpp):
// device queries, workspace size, default setting and dtype dispatch.
#include "internal.hpp"

namespace ptd {

namespace {

struct DevInfo {
    int cus = 0;
    int xcds = 1;
};

DevInfo device_info()
{
    static thread_local int cached_dev = -1;
    static thread_local DevInfo cached;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DevInfo{256, 8};
    if (dev != cached_dev) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cached.cus = cus;
        // 32 compute units per XCD on MI355X; partitioned modes expose fewer
        int x = cus / 32;
        cached.xcds = x < 1 ? 1 : (x > 8 ? 8 : x);
        cached_dev = dev;
    }
    return cached;
}

__global__ void k_zero_words(uint32_t* __restrict__ p, int count)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0u;
}

__global__ void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

int device_cu_count() { return device_info().cus; }
int device_xcd_count() { return device_info().xcds; }

hipError_t launch_zero_words(uint32_t* p, int count, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_words, dim3((count + 255) / 256), dim3(256), 0, st, p, count);
    return hipGetLastError();
}

FusedTuning fused_default(int n, ptd_dtype dt, bool herm)
{
    // The fastest settings measured on MI355X.  Shape: 512-thread workgroups
    // with 512-row phase-1 items up to n = 14, 1024-thread ones at n = 15.
    // Cache policy: non-temporal gathers, final stores and phase-2 loads,
    // except complex128 at n = 14, where phase-2 loads stay cached.
    // Lookahead: deep enough that phase-2 items rarely wait for their group
    // (the 64 workgroups of an XCD hold more groups' items at small n).
    FusedTuning t{0, 4};
    const int shape = n <= 14 ? 2 : 1;
    t.cfg = (dt == PTD_C128 && n == 14) ? (shape | 4 | 8) : (shape | 4 | 8 | 16);
    switch (n) {
        case 11: t.la = 16; break;
        case 12: t.la = 12; break;
        case 13: t.la = 8; break;
        case 14: t.la = (dt == PTD_C128 && !herm) ? 4 : 6; break;
        default: t.la = 4; break;
    }
    return t;
}

size_t fused_workspace_bytes(int n, ptd_dtype dt)
{
    // 32 words of queue heads and flags, then enough group counters for the
    // smallest groups any shape uses
    const int logt = dt == PTD_C64 ? 3 : 2;
    return (size_t)(32 + (1 << (n - logt))) * sizeof(uint32_t);
}

hipError_t launch_fused_fwd(int n, ptd_dtype dt, bool herm, const void* A, int64_t lda, void* out, void* ws, int la,
                            int cfg, hipStream_t st)
{
    if (n < 11 || n > 15 || la < 1) return hipErrorInvalidValue;
    if (dt == PTD_C128)
        return herm ? fused_launch_c128_herm(n, A, lda, out, ws, la, cfg, st)
                    : fused_launch_c128(n, A, lda, out, ws, la, cfg, st);
    return herm ? fused_launch_c64_herm(n, A, lda, out, ws, la, cfg, st)
                : fused_launch_c64(n, A, lda, out, ws, la, cfg, st);
}

hipError_t launch_fused_rec(int n, ptd_dtype dt, bool herm, bool adjoint, const void* coeff, void* A, int64_t lda,
                            void* ws, int la, hipStream_t st)
{
    if (n < 11 || n > 14 || la < 1) return hipErrorInvalidValue;
    if (dt == PTD_C128)
        return herm ? fused_rec_c128_herm(n, coeff, A, lda, ws, la, adjoint, st)
                    : fused_rec_c128(n, coeff, A, lda, ws, la, adjoint, st);
    return herm ? fused_rec_c64_herm(n, coeff, A, lda, ws, la, adjoint, st)
                : fused_rec_c64(n, coeff, A, lda, ws, la, adjoint, st);
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t st)
{
    const int64_t count = (int64_t)(bytes / 16);
    hipLaunchKernelGGL(k_copy16, dim3(device_cu_count() * 4), dim3(256), 0, st, (const uint4*)src, (uint4*)dst,
                       count);
    return hipGetLastError();
}

}  // namespace ptd
