// fused.hip -- host side of the single-launch dense schedule (fused.hpp):
// device queries, workspace size, default setting and dtype dispatch.
#include <atomic>

#include "fused.hpp"
#include "internal.hpp"

namespace ptd {

namespace {
std::atomic<bool> g_wait_test{false};
}  // namespace

WaitLimits wait_limits()
{
    // about 0.2 s of polling; the test hook gives up after 16 polls with a
    // target no producer count reaches
    if (g_wait_test.load(std::memory_order_relaxed)) return WaitLimits{16u, 1u};
    return WaitLimits{1u << 22, 0u};
}

void set_wait_test_mode(bool on) { g_wait_test.store(on, std::memory_order_relaxed); }

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
        // XCDs (accelerator complex dies) the runtime reports for this device
        // (8 on MI355X; partitioned modes expose fewer).  Workgroups read
        // their die from HW_REG_XCC_ID, which runs over 0 .. xcds-1 (checked
        // by a probe kernel in the test suite).
        int x = 0;
        if (hipDeviceGetAttribute(&x, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || x < 1) x = 1;
        cached.xcds = x > 16 ? 16 : x;
        cached_dev = dev;
    }
    return cached;
}

__global__ void k_zero_words(uint32_t* __restrict__ p, int count)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0u;
}

__device__ unsigned g_xcc_seen;

// Every workgroup records the die it runs on.
__global__ void k_xcc_probe()
{
    if (threadIdx.x == 0) atomicOr(&g_xcc_seen, 1u << fused::xcc_id());
}

__global__ void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

int device_cu_count() { return device_info().cus; }

hipError_t probe_xcc_ids(unsigned* mask, int* count)
{
    const unsigned zero = 0;
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(g_xcc_seen), &zero, sizeof(zero));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_xcc_probe, dim3(device_cu_count() * 8), dim3(64), 0, 0);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpyFromSymbol(mask, HIP_SYMBOL(g_xcc_seen), sizeof(unsigned));
    *count = device_xcd_count();
    return e;
}
int device_xcd_count() { return device_info().xcds; }

hipError_t launch_zero_words(uint32_t* p, int count, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_words, dim3((count + 255) / 256), dim3(256), 0, st, p, count);
    return hipGetLastError();
}

FusedTuning fused_default(int n, ptd_dtype dt, bool herm)
{
    // The fastest settings the autotuner found on MI355X (cfg: shape | POL
    // bits, see fused_dispatch; la: queue lookahead in groups).  1024-thread
    // workgroups with 1024-row phase-1 items (shape 1) win at n <= 12 and for
    // Hermitian input, 512-thread ones (shape 2) for dense n = 13, 14;
    // non-temporal gathers and final stores almost everywhere.  The
    // lookahead is deep enough that phase-2 items rarely wait for their
    // group (an XCD's workgroups hold more groups' items at small n).
    const bool c128 = dt == PTD_C128;
    switch (n) {
        case 11:
            return c128 && !herm ? FusedTuning{29, 16} : FusedTuning{1, 16};
        case 12:
            if (c128) return herm ? FusedTuning{29, 12} : FusedTuning{29, 16};
            return herm ? FusedTuning{1, 12} : FusedTuning{1, 8};
        case 13:
            if (herm) return c128 ? FusedTuning{13, 8} : FusedTuning{29, 4};
            return FusedTuning{30, 8};
        case 14:
            // complex64 Hermitian: half-width groups (shape 3) win
            if (herm) return c128 ? FusedTuning{30, 6} : FusedTuning{31, 8};
            return c128 ? FusedTuning{14, 4} : FusedTuning{30, 6};
        default:
            return FusedTuning{29, 4};
    }
}

size_t fused_workspace_bytes(int n, ptd_dtype dt)
{
    // 32 words of queue heads and flags, then enough group counters for the
    // smallest groups any shape uses
    const int logt = dt == PTD_C64 ? 3 : 2;
    return (size_t)(32 + (1 << (n - logt))) * sizeof(uint32_t);
}

hipError_t launch_fused_fwd(int n, ptd_dtype dt, bool herm, const void* A, int64_t lda, void* out, void* ws, int la,
                            int cfg, hipStream_t st, bool unscaled)
{
    if (n < 11 || n > 15 || la < 1) return hipErrorInvalidValue;
    if (dt == PTD_C128)
        return herm ? fused_launch_c128_herm(n, A, lda, out, ws, la, cfg, unscaled, st)
                    : fused_launch_c128(n, A, lda, out, ws, la, cfg, unscaled, st);
    return herm ? fused_launch_c64_herm(n, A, lda, out, ws, la, cfg, unscaled, st)
                : fused_launch_c64(n, A, lda, out, ws, la, cfg, unscaled, st);
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

bool describe_fused(int n, ptd_dtype dt, bool herm, int cfg, int* threads, int* phase1_bits, int* group_patterns)
{
    int logt = 0;
    if (!fused::fused_describe(n, dt == PTD_C64, herm, cfg, threads, phase1_bits, &logt)) return false;
    *group_patterns = 1 << logt;
    return true;
}

}  // namespace ptd
