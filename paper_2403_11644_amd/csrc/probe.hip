// probe.hip -- bandwidth references for the measurement of the kernels: a
// small sweep of copy, read-only and write-only kernels over the same bytes
// a decomposition moves, to state the practical ceiling of this device next
// to the 8 TB/s HBM3E peak.  Not used by any decomposition.
//
// Variant bits (ptd_debug_bandwidth):
//   bits 0-1  mode: 0 copy, 1 read only, 2 write only, 3 write-back probe
//             (below; no other bits)
//   bits 2-3  log2 of the 16-byte accesses per thread and iteration (1..8)
//   bit  4    non-temporal loads;  bit 5  non-temporal stores
//   bit  6    blocked: each workgroup owns one contiguous chunk (otherwise
//             the whole grid strides over the buffer)
//   bits 8-9  log2 of the workgroup size / 256 (256, 512, 1024)
//   bits 10-11 log2 of the workgroups per CU (1, 2, 4, 8)
#include "internal.hpp"

namespace ptd {

namespace {

typedef unsigned int u4v __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ u4v ld16(const u4v* p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NT>
__device__ __forceinline__ void st16(u4v* p, u4v v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <int MODE, int U, bool NTL, bool NTS, bool BLK>
__global__ void k_bw(const u4v* __restrict__ src, u4v* __restrict__ dst, int64_t count, unsigned* __restrict__ sink)
{
    int64_t i, end, stride;
    if constexpr (BLK) {
        const int64_t per = (count + gridDim.x - 1) / gridDim.x;
        i = (int64_t)blockIdx.x * per + threadIdx.x;
        end = (int64_t)blockIdx.x * per + per < count ? (int64_t)blockIdx.x * per + per : count;
        stride = blockDim.x;
    } else {
        i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        end = count;
        stride = (int64_t)gridDim.x * blockDim.x;
    }
    u4v acc = {0u, 0u, 0u, 0u};
    for (; i + (U - 1) * stride < end; i += U * stride) {
        u4v v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (MODE == 2)
                v[u] = u4v{(unsigned)i, (unsigned)u, 1u, 2u};
            else
                v[u] = ld16<NTL>(src + i + u * stride);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (MODE == 1)
                acc ^= v[u];
            else
                st16<NTS>(dst + i + u * stride, v[u]);
        }
    }
    for (; i < end; i += stride) {
        if constexpr (MODE == 1)
            acc ^= ld16<NTL>(src + i);
        else if constexpr (MODE == 0)
            st16<NTS>(dst + i, ld16<NTL>(src + i));
        else
            st16<NTS>(dst + i, u4v{1u, 2u, 3u, 4u});
    }
    // keeps the read-only loads alive; never true for the data the bench uses
    if (MODE == 1 && (acc.x ^ acc.y ^ acc.z ^ acc.w) == 0x9E3779B9u) sink[threadIdx.x & 63] = acc.x;
}

typedef void (*BwKernel)(const u4v*, u4v*, int64_t, unsigned*);

template <int MODE, int U, bool NTL, bool NTS>
BwKernel pick_blk(bool blk)
{
    return blk ? k_bw<MODE, U, NTL, NTS, true> : k_bw<MODE, U, NTL, NTS, false>;
}

template <int MODE, int U>
BwKernel pick_nt(bool ntl, bool nts, bool blk)
{
    if (ntl) return nts ? pick_blk<MODE, U, true, true>(blk) : pick_blk<MODE, U, true, false>(blk);
    return nts ? pick_blk<MODE, U, false, true>(blk) : pick_blk<MODE, U, false, false>(blk);
}

template <int MODE>
BwKernel pick_u(int lu, bool ntl, bool nts, bool blk)
{
    switch (lu) {
        case 0: return pick_nt<MODE, 1>(ntl, nts, blk);
        case 1: return pick_nt<MODE, 2>(ntl, nts, blk);
        case 2: return pick_nt<MODE, 4>(ntl, nts, blk);
        default: return pick_nt<MODE, 8>(ntl, nts, blk);
    }
}

// Write-back probe: every 1024-thread workgroup writes its own 64 KiB,
// reads it back (each lane another lane's 16 bytes, so the L1 holds none of
// them) and overwrites it.  Its FETCH_SIZE / WRITE_SIZE counters tell
// whether the L2 keeps written lines for a later read and merges the two
// writes of one line (then the launch would fetch nothing and write the
// region once) or passes every store on.
__global__ __launch_bounds__(1024) void k_l2_rewrite(u4v* __restrict__ buf, unsigned* __restrict__ sink)
{
    u4v* base = buf + (size_t)blockIdx.x * 4096;
    const int t = threadIdx.x;
#pragma unroll
    for (int u = 0; u < 4; ++u) base[t + 1024 * u] = u4v{(unsigned)blockIdx.x, (unsigned)u, 1u, 2u};
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    u4v acc = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int u = 0; u < 4; ++u) acc ^= base[((t + 64) & 1023) + 1024 * u];
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) base[t + 1024 * u] = acc + u4v{3u, 4u, 5u, (unsigned)u};
    if ((acc.x ^ acc.y) == 0x9E3779B9u) sink[t & 63] = acc.z;
}

__device__ unsigned g_bw_sink[64];

}  // namespace

hipError_t launch_bandwidth(int variant, const void* src, void* dst, size_t bytes, hipStream_t st)
{
    const int mode = variant & 3;
    if (variant & ~0xF7F) return hipErrorInvalidValue;
    if (mode == 3) {
        if (variant != 3 || (bytes & 65535) || bytes == 0) return hipErrorInvalidValue;
        unsigned* sink3 = nullptr;
        hipError_t e3 = hipGetSymbolAddress((void**)&sink3, HIP_SYMBOL(g_bw_sink));
        if (e3 != hipSuccess) return e3;
        hipLaunchKernelGGL(k_l2_rewrite, dim3((unsigned)(bytes >> 16)), dim3(1024), 0, st, (u4v*)dst, sink3);
        return hipGetLastError();
    }
    const int lu = (variant >> 2) & 3;
    const bool ntl = variant & 16, nts = variant & 32, blk = variant & 64;
    const int threads = 256 << ((variant >> 8) & 3);
    const int per_cu = 1 << ((variant >> 10) & 3);
    if (threads > 1024 || threads * per_cu > 2048) return hipErrorInvalidValue;
    BwKernel k = mode == 0 ? pick_u<0>(lu, ntl, nts, blk) : mode == 1 ? pick_u<1>(lu, ntl, nts, blk)
                                                                      : pick_u<2>(lu, ntl, nts, blk);
    unsigned* sink = nullptr;
    hipError_t e = hipGetSymbolAddress((void**)&sink, HIP_SYMBOL(g_bw_sink));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(device_cu_count() * per_cu), dim3(threads), 0, st, (const u4v*)src, (u4v*)dst,
                       (int64_t)(bytes / 16), sink);
    return hipGetLastError();
}

}  // namespace ptd
