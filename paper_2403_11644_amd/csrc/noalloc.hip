// noalloc.hip -- pauli_decompose_noalloc: pauli_decompose with its workspace
// in a fixed device array of the library instead of caller memory, for
// callers that cannot allocate device memory.
//
// The only workspace any decomposition path needs is the one-launch
// schedule's queue heads, group counters and error word (dense n = 11..15,
// at most 16.5 KiB).  `scratch` holds it: a file-scope device array, one
// copy per GPU, resident until the process ends.  In host code the name
// `scratch` stands for a host-side shadow, not the device address, so the
// address is looked up once per device with hipGetSymbolAddress (with that
// device current) and kept; kernels receive that address as their
// workspace argument, exactly as they receive a caller's workspace.
//
// Every call on one GPU shares its array.  Each call clears the counters it
// uses (a zero-fill kernel on the call's stream, before the decomposition
// kernel), so consecutive calls need nothing from the caller; calls that
// overlap in time on one GPU (two streams, or two host threads) race on the
// array and are not supported.
#include <mutex>

#include "internal.hpp"

namespace {

constexpr size_t kScratchBytes = PTD_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint32_t scratch[kScratchBytes / sizeof(uint32_t)];

std::mutex g_mu;
void* g_addr[kMaxDevices];  // device address of `scratch` per GPU, null until looked up

// Device address of this GPU's `scratch` (the current device's).
ptd_status scratch_address(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return ptd::status_from_hip(e);
    if (dev < 0 || dev >= kMaxDevices) return PTD_EUNSUP;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return ptd::status_from_hip(e);
        if (!p) return ptd::status_from_hip(hipErrorInvalidSymbol);
        g_addr[dev] = p;
    }
    *out = g_addr[dev];
    return PTD_OK;
}

}  // namespace

extern "C" ptd_status pauli_decompose_noalloc(int n, ptd_dtype dtype, unsigned flags, int s, const void* A,
                                              int64_t lda, void* coeff, ptd_stream stream)
{
    const ptd_status chk = ptd::decompose_check(n, dtype, flags, s, A, lda, coeff);
    if (chk != PTD_OK) return chk;
    const size_t need = ptd_workspace_bytes(n, dtype, flags, s);
    if (need > kScratchBytes) return PTD_ENOSPC;
    void* ws = nullptr;
    if (need) {
        const ptd_status st = scratch_address(&ws);
        if (st != PTD_OK) return st;
    }
    return pauli_decompose(n, dtype, flags, s, A, lda, coeff, ws, need, stream);
}
