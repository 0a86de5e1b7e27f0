// batched.hip -- many matrices of uneven size (n <= 10) in one persistent launch.
//
// Work items are (matrix, X-pattern group) pairs; each is the single-pass
// group routine of group.hpp for that matrix's n, chosen by a switch inside
// the kernel.  Items are listed largest matrices first (longest-processing-
// time order) and taken from one atomic counter, so workgroups that finish
// small items early keep pulling work and the tail is short.  The forward
// map and the reconstruction (with optional 2^-n adjoint scale) share the
// kernel.
//
// Workspace / plan buffer layout (bytes):
//   [0, 256)          queue counter (zeroed by a kernel before each launch)
//   [256, ...)        BatchMat[count] then BatchItem[items]
#include <vector>

#include "engine.hpp"
#include "group.hpp"
#include "internal.hpp"

namespace ptd {

namespace {

struct BatchMat {
    int64_t in_off;   // elements of the input type
    int64_t out_off;  // elements of the output type
    int32_t n;
    int32_t pad;
};

struct BatchItem {
    uint32_t mat;
    uint32_t group;
};

constexpr size_t HEAD_BYTES = 256;

template <class V>
__host__ __device__ constexpr int batch_logt(int n)
{
    return group_logt<V>(n);
}

template <class V, bool HERM, bool REC>
__global__ __launch_bounds__(GROUP_THREADS) void k_batched(const void* __restrict__ in_base, void* __restrict__ out_base,
                                                          const BatchMat* __restrict__ mats,
                                                          const BatchItem* __restrict__ items, int nitems,
                                                          uint32_t* __restrict__ counter, int adjoint)
{
    __shared__ cplx<V> lds[group_lds_elems<V>(10)];
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0)
            s_item = (int)__hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int i = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (i >= nitems) break;
        const BatchItem it = items[i];
        const BatchMat m = mats[it.mat];
        const int g = (int)it.group;
        const int64_t N = (int64_t)1 << m.n;
        if constexpr (!REC) {
            const cplx<V>* A = (const cplx<V>*)in_base + m.in_off;
            void* out = HERM ? (void*)((V*)out_base + m.out_off) : (void*)((cplx<V>*)out_base + m.out_off);
            switch (m.n) {
#define PTD_CASE(NN)                                                                   \
    case NN: group_fwd<V, NN, group_logt<V>(NN), HERM>(A, N, out, N, g, lds); break;
                PTD_CASE(1) PTD_CASE(2) PTD_CASE(3) PTD_CASE(4) PTD_CASE(5)
                PTD_CASE(6) PTD_CASE(7) PTD_CASE(8) PTD_CASE(9) PTD_CASE(10)
#undef PTD_CASE
                default: break;
            }
        } else {
            const void* C = HERM ? (const void*)((const V*)in_base + m.in_off)
                                 : (const void*)((const cplx<V>*)in_base + m.in_off);
            cplx<V>* A = (cplx<V>*)out_base + m.out_off;
            const V scale = adjoint ? exp2_neg<V>(m.n) : (V)1;
            switch (m.n) {
#define PTD_CASE(NN)                                                                      \
    case NN: group_rec<V, NN, group_logt<V>(NN), HERM>(C, A, N, scale, g, lds); break;
                PTD_CASE(1) PTD_CASE(2) PTD_CASE(3) PTD_CASE(4) PTD_CASE(5)
                PTD_CASE(6) PTD_CASE(7) PTD_CASE(8) PTD_CASE(9) PTD_CASE(10)
#undef PTD_CASE
                default: break;
            }
        }
        __syncthreads();  // LDS and s_item reuse
    }
}

__global__ void k_zero_counter(uint32_t* __restrict__ p)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0u;
}

int logt_of(ptd_dtype dt, int n)
{
    return dt == PTD_C64 ? batch_logt<float>(n) : batch_logt<double>(n);
}

}  // namespace

int64_t batched_item_count(int count, ptd_dtype dt, const int32_t* n_host)
{
    int64_t items = 0;
    for (int i = 0; i < count; ++i) items += (int64_t)1 << (n_host[i] - logt_of(dt, n_host[i]));
    return items;
}

size_t batched_buffer_bytes(int count, ptd_dtype dt, const int32_t* n_host)
{
    return HEAD_BYTES + (size_t)count * sizeof(BatchMat) +
           (size_t)batched_item_count(count, dt, n_host) * sizeof(BatchItem);
}

// Fill the host image of the descriptor buffer (after the head).
void batched_fill(int count, ptd_dtype dt, const int32_t* n_host, const int64_t* in_off, const int64_t* out_off,
                  std::vector<unsigned char>& img, int* nitems_out)
{
    const int64_t items = batched_item_count(count, dt, n_host);
    img.assign((size_t)count * sizeof(BatchMat) + (size_t)items * sizeof(BatchItem), 0);
    BatchMat* mats = (BatchMat*)img.data();
    BatchItem* its = (BatchItem*)(img.data() + (size_t)count * sizeof(BatchMat));
    for (int i = 0; i < count; ++i) {
        mats[i].in_off = in_off[i];
        mats[i].out_off = out_off[i];
        mats[i].n = n_host[i];
        mats[i].pad = 0;
    }
    // largest matrices first; ties keep the caller's order
    std::vector<int> byn[17];
    for (int i = 0; i < count; ++i) byn[n_host[i]].push_back(i);
    int64_t k = 0;
    for (int n = 16; n >= 1; --n)
        for (int mi : byn[n]) {
            const int groups = 1 << (n - logt_of(dt, n));
            for (int g = 0; g < groups; ++g) {
                its[k].mat = (uint32_t)mi;
                its[k].group = (uint32_t)g;
                ++k;
            }
        }
    *nitems_out = (int)items;
}

hipError_t batched_launch(ptd_dtype dt, bool herm, bool rec, bool adjoint, const void* in_base, void* out_base,
                          void* buf, int count, int nitems, int cus, hipStream_t st)
{
    uint32_t* counter = (uint32_t*)buf;
    const BatchMat* mats = (const BatchMat*)((unsigned char*)buf + HEAD_BYTES);
    const BatchItem* its = (const BatchItem*)((unsigned char*)buf + HEAD_BYTES + (size_t)count * sizeof(BatchMat));
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, st, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid(cus), block(GROUP_THREADS);
    const int adj = adjoint ? 1 : 0;
#define PTD_LAUNCH(VV, HH, RR) \
    hipLaunchKernelGGL((k_batched<VV, HH, RR>), grid, block, 0, st, in_base, out_base, mats, its, nitems, counter, adj)
    if (dt == PTD_C128) {
        if (rec) {
            if (herm) PTD_LAUNCH(double, true, true); else PTD_LAUNCH(double, false, true);
        } else {
            if (herm) PTD_LAUNCH(double, true, false); else PTD_LAUNCH(double, false, false);
        }
    } else {
        if (rec) {
            if (herm) PTD_LAUNCH(float, true, true); else PTD_LAUNCH(float, false, true);
        } else {
            if (herm) PTD_LAUNCH(float, true, false); else PTD_LAUNCH(float, false, false);
        }
    }
#undef PTD_LAUNCH
    return hipGetLastError();
}

}  // namespace ptd
