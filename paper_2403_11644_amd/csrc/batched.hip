// batched.hip -- many matrices of uneven size (n <= 10) in persistent launches.
//
// Work items are (matrix, X-pattern group) pairs; each is the single-pass
// group routine of group.hpp.  Items are listed largest matrices first
// (longest-processing-time order).  Every size from 8 to 10 present gets one
// persistent launch over its own contiguous range of items, taken two at a
// time from its own atomic counter, so workgroups that finish items early
// keep pulling work and the tail is short.  One launch per size gives each kernel the register
// budget and LDS of its own size, hence its own occupancy (one 131 KiB
// workgroup per CU at n = 10, two below), and lets the tuned plan of each
// size (workgroup size, radix) apply.  Sizes 1..7 share one launch of small
// workgroups that stride over their items (k_batched_small).  The forward map and the reconstruction (with optional
// 2^-n adjoint scale) share the kernel.  A batch plan captures all launches
// in one graph.
//
// Workspace / plan buffer layout (bytes):
//   [0, BATCH_HEAD_BYTES)   queue counters, index n for size n, 64 bytes
//                           apart (only sizes 8..10 take them)
//                           (zeroed by a kernel before each launch)
//   [BATCH_HEAD_BYTES, ...) BatchMat[count] then BatchItem[items]
#include <mutex>
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

constexpr int COUNTER_STRIDE = 16;  // uint32 words: one 64-byte line per counter
static_assert(11 * COUNTER_STRIDE * 4 <= (int)BATCH_HEAD_BYTES, "counters fit the head");

template <class V>
__host__ __device__ constexpr int batch_logt(int n)
{
    return group_logt<V>(n);
}

// 512-thread workgroups per CU that the LDS of size NN allows, at most 2
template <class V, int NN>
constexpr int wgs_per_cu()
{
    return (160 * 1024) / (group_lds_elems<V>(NN) * (int)sizeof(cplx<V>)) >= 2 ? 2 : 1;
}

// Sizes 1..SMALL_MAX share one launch (a switch per item) of one-wave
// workgroups, SMALL_WGS of them per CU, each striding over the items.  An
// item of these sizes moves at most 16 KiB: a launch per size would cost more
// than its work, and a shared queue counter, one atomic round trip to the
// memory side per item, more than the item itself (measured: 4096 Hermitian
// complex64 matrices, the sizes <= 7 took 137 us through per-size queues and
// 30 us this way).  Larger items keep the queues, whose balance pays there.
constexpr int SMALL_MAX = BATCH_SMALL_MAX;
constexpr int SMALL_NT = 64;
constexpr int SMALL_WGS = 8;

template <class V, int NN, bool HERM, bool REC>
__device__ __forceinline__ void batched_item(const void* __restrict__ in_base, void* __restrict__ out_base,
                                             const BatchMat& m, int g, int adjoint, cplx<V>* lds)
{
    constexpr int LOGT = group_logt<V>(NN);
    constexpr int64_t N = (int64_t)1 << NN;
    (void)adjoint;
    if constexpr (!REC) {
        const cplx<V>* A = (const cplx<V>*)in_base + m.in_off;
        void* out = HERM ? (void*)((V*)out_base + m.out_off) : (void*)((cplx<V>*)out_base + m.out_off);
        group_fwd<V, NN, LOGT, HERM, SMALL_NT, 4>(A, N, out, N, g, lds, exp2_neg<V>(NN));
    } else {
        const void* C = HERM ? (const void*)((const V*)in_base + m.in_off)
                             : (const void*)((const cplx<V>*)in_base + m.in_off);
        cplx<V>* A = (cplx<V>*)out_base + m.out_off;
        const V scale = adjoint ? exp2_neg<V>(NN) : (V)1;
        group_rec<V, NN, LOGT, HERM, SMALL_NT>(C, A, N, scale, g, lds);
    }
}

template <class V, bool HERM, bool REC>
__global__ __launch_bounds__(SMALL_NT) void k_batched_small(const void* __restrict__ in_base, void* __restrict__ out_base,
                                                       const BatchMat* __restrict__ mats,
                                                       const BatchItem* __restrict__ items, int begin, int end,
                                                       int adjoint)
{
    // static round-robin; the list is sorted by size, so striding hands every
    // workgroup a like mix
    __shared__ cplx<V> lds[group_lds_elems<V>(SMALL_MAX)];
    for (int i = begin + (int)blockIdx.x; i < end; i += (int)gridDim.x) {
        const BatchItem it = items[i];
        const BatchMat m = mats[it.mat];
        switch (m.n) {
            case 1: batched_item<V, 1, HERM, REC>(in_base, out_base, m, (int)it.group, adjoint, lds); break;
            case 2: batched_item<V, 2, HERM, REC>(in_base, out_base, m, (int)it.group, adjoint, lds); break;
            case 3: batched_item<V, 3, HERM, REC>(in_base, out_base, m, (int)it.group, adjoint, lds); break;
            case 4: batched_item<V, 4, HERM, REC>(in_base, out_base, m, (int)it.group, adjoint, lds); break;
            case 5: batched_item<V, 5, HERM, REC>(in_base, out_base, m, (int)it.group, adjoint, lds); break;
            case 6: batched_item<V, 6, HERM, REC>(in_base, out_base, m, (int)it.group, adjoint, lds); break;
            case 7: batched_item<V, 7, HERM, REC>(in_base, out_base, m, (int)it.group, adjoint, lds); break;
            default: break;
        }
        __syncthreads();  // LDS reuse
    }
}

// Items [begin, end) of size-NN matrices.
template <class V, int NN, bool HERM, bool REC, int NT, int RMAX>
__global__ __launch_bounds__(NT, (NT / 256) * (NT == 512 ? wgs_per_cu<V, NN>() : 1)) void k_batched(
    const void* __restrict__ in_base, void* __restrict__ out_base, const BatchMat* __restrict__ mats,
    const BatchItem* __restrict__ items, int begin, int end, uint32_t* __restrict__ counter, int adjoint)
{
    constexpr int LOGT = group_logt<V>(NN);
    constexpr int64_t N = (int64_t)1 << NN;
    __shared__ cplx<V> lds[group_lds_elems<V>(NN)];
    __shared__ int s_ticket;
    // A ticket from the queue counter covers CLAIM consecutive items, and the
    // next ticket is taken while the current items run: the counter's atomic
    // is performed at the memory side, and an n = 10 item takes only ~7 us
    // with one workgroup per CU (measured on the 4096-matrix batch: 1.222 ms
    // with one item per ticket taken after each item, 1.163 ms this way; 4
    // items per ticket lengthen the tail).  Items do not wait on each other,
    // so holding the next ticket early cannot stall anyone.
    constexpr int CLAIM = 2;
    if (threadIdx.x == 0)
        s_ticket = (int)__hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    int ticket = __builtin_amdgcn_readfirstlane(s_ticket);
    for (;;) {
        const int first = begin + ticket * CLAIM;
        if (first >= end) break;
        int next = 0;
        if (threadIdx.x == 0)
            next = (int)__hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int i = first; i < first + CLAIM && i < end; ++i) {
            const BatchItem it = items[i];
            const BatchMat m = mats[it.mat];
            const int g = (int)it.group;
            if constexpr (!REC) {
                const cplx<V>* A = (const cplx<V>*)in_base + m.in_off;
                void* out = HERM ? (void*)((V*)out_base + m.out_off) : (void*)((cplx<V>*)out_base + m.out_off);
                group_fwd<V, NN, LOGT, HERM, NT, RMAX>(A, N, out, N, g, lds, exp2_neg<V>(NN));
            } else {
                const void* C = HERM ? (const void*)((const V*)in_base + m.in_off)
                                     : (const void*)((const cplx<V>*)in_base + m.in_off);
                cplx<V>* A = (cplx<V>*)out_base + m.out_off;
                const V scale = adjoint ? exp2_neg<V>(NN) : (V)1;
                group_rec<V, NN, LOGT, HERM, NT>(C, A, N, scale, g, lds);
            }
            __syncthreads();  // LDS reuse; every thread has read s_ticket
        }
        if (threadIdx.x == 0) s_ticket = next;
        __syncthreads();
        ticket = __builtin_amdgcn_readfirstlane(s_ticket);
        __syncthreads();  // s_ticket reuse
    }
}

__global__ void k_zero_counters(uint32_t* __restrict__ p)
{
    if (blockIdx.x == 0 && threadIdx.x <= 10) p[threadIdx.x * COUNTER_STRIDE] = 0u;
}

int logt_of(ptd_dtype dt, int n)
{
    return dt == PTD_C64 ? batch_logt<float>(n) : batch_logt<double>(n);
}

template <class V, int NN, bool HERM, bool REC, int NT, int RMAX>
void launch_size(const void* in_base, void* out_base, const BatchMat* mats, const BatchItem* its, int begin, int end,
                 uint32_t* counter, int adj, int cus, hipStream_t st)
{
    const int per_cu = NT == 512 ? wgs_per_cu<V, NN>() : 1;
    // persistent: every resident workgroup slot, but no more than there are items
    const int grid = cus * per_cu < end - begin ? cus * per_cu : end - begin;
    hipLaunchKernelGGL((k_batched<V, NN, HERM, REC, NT, RMAX>), dim3(grid), dim3(NT), 0, st, in_base, out_base,
                       mats, its, begin, end, counter, adj);
}

// The plan of size NN: 1024-thread workgroups only at n = 10 (where one
// workgroup fills a CU), radix-32 rounds only for complex64 and n >= 6.
template <class V, int NN, bool HERM, bool REC>
void launch_size_plan(int plan, const void* in_base, void* out_base, const BatchMat* mats, const BatchItem* its,
                      int begin, int end, uint32_t* counter, int adj, int cus, hipStream_t st)
{
    constexpr bool CAN_BIG = NN == 10 && !REC;
    constexpr bool CAN_R5 = !REC && sizeof(V) == 4 && NN >= 6;
    const bool big = CAN_BIG && group_plan_nt(plan) == 1024;
    const bool r5 = CAN_R5 && group_effective_rmax(NN, PTD_C64, plan) == 5;
    if constexpr (CAN_BIG) {
        if (big) {
            if constexpr (CAN_R5) {
                if (r5) {
                    launch_size<V, NN, HERM, REC, 1024, 5>(in_base, out_base, mats, its, begin, end, counter, adj, cus,
                                                          st);
                    return;
                }
            }
            launch_size<V, NN, HERM, REC, 1024, 4>(in_base, out_base, mats, its, begin, end, counter, adj, cus, st);
            return;
        }
    }
    if constexpr (CAN_R5) {
        if (r5) {
            launch_size<V, NN, HERM, REC, 512, 5>(in_base, out_base, mats, its, begin, end, counter, adj, cus, st);
            return;
        }
    }
    launch_size<V, NN, HERM, REC, 512, 4>(in_base, out_base, mats, its, begin, end, counter, adj, cus, st);
}

// The launches of a batch: one per size 10..SMALL_MAX+1 present, largest
// first, then the shared launch of the small sizes; launch i goes to
// lanes[i] (all the same stream, or one stream each).
int batch_launch_count(const BatchLaunch& bl)
{
    int k = bl.begin[0] > bl.begin[SMALL_MAX] ? 1 : 0;
    for (int n = 10; n > SMALL_MAX; --n) k += bl.begin[n - 1] > bl.begin[n] ? 1 : 0;
    return k;
}

template <class V, bool HERM, bool REC>
void launch_all(const BatchLaunch& bl, const void* in_base, void* out_base, const BatchMat* mats,
                const BatchItem* its, uint32_t* counters, int adj, int cus, const hipStream_t* lanes)
{
    int li = 0;
    for (int n = 10; n > SMALL_MAX; --n) {
        const int b = bl.begin[n], e = bl.begin[n - 1];
        if (e <= b) continue;
        uint32_t* c = counters + n * COUNTER_STRIDE;
        const int plan = bl.plan[n];
        const hipStream_t st = lanes[li++];
        switch (n) {
#define PTD_CASE(NN)                                                                                    \
    case NN:                                                                                            \
        launch_size_plan<V, NN, HERM, REC>(plan, in_base, out_base, mats, its, b, e, c, adj, cus, st); \
        break;
            PTD_CASE(8) PTD_CASE(9) PTD_CASE(10)
#undef PTD_CASE
            default: break;
        }
    }
    {
        // sizes 1..SMALL_MAX are contiguous at the end of the list
        const int b = bl.begin[SMALL_MAX], e = bl.begin[0];
        if (e > b) {
            const int cap = SMALL_WGS * cus;
            hipLaunchKernelGGL((k_batched_small<V, HERM, REC>), dim3(e - b < cap ? e - b : cap), dim3(SMALL_NT), 0,
                               lanes[li++], in_base, out_base, mats, its, b, e, adj);
        }
    }
}

// Side streams of this device for concurrent batch launches (created once,
// kept until the process ends), and the events that fork and join them.
constexpr int MAX_LANES = 4;
struct SideLanes {
    bool ready = false;
    hipStream_t s[MAX_LANES - 1] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[MAX_LANES - 1] = {};
};
std::mutex g_lanes_mu;
SideLanes g_lanes[64];

hipError_t side_lanes(SideLanes** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    SideLanes& L = g_lanes[dev];
    if (!L.ready) {
        for (int i = 0; i < MAX_LANES - 1 && e == hipSuccess; ++i) {
            if (!L.s[i]) e = hipStreamCreateWithFlags(&L.s[i], hipStreamNonBlocking);
            if (e == hipSuccess && !L.join[i]) e = hipEventCreateWithFlags(&L.join[i], hipEventDisableTiming);
        }
        if (e == hipSuccess && !L.fork) e = hipEventCreateWithFlags(&L.fork, hipEventDisableTiming);
        if (e != hipSuccess) return e;
        L.ready = true;
    }
    *out = &L;
    return hipSuccess;
}

}  // namespace

hipError_t prepare_batch_lanes()
{
    std::lock_guard<std::mutex> lk(g_lanes_mu);
    SideLanes* L = nullptr;
    return side_lanes(&L);
}

int64_t batched_item_count(int count, ptd_dtype dt, const int32_t* n_host)
{
    int64_t items = 0;
    for (int i = 0; i < count; ++i) items += (int64_t)1 << (n_host[i] - logt_of(dt, n_host[i]));
    return items;
}

size_t batched_buffer_bytes(int count, ptd_dtype dt, const int32_t* n_host)
{
    return BATCH_HEAD_BYTES + (size_t)count * sizeof(BatchMat) +
           (size_t)batched_item_count(count, dt, n_host) * sizeof(BatchItem);
}

// Fill the host image of the descriptor buffer (after the head), the item
// range of every size and the plan of every size.
void batched_fill(int count, ptd_dtype dt, bool herm, bool rec, const int32_t* n_host, const int64_t* in_off,
                  const int64_t* out_off, std::vector<unsigned char>& img, BatchLaunch* bl, int force_plan)
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
    // largest matrices first; ties keep the caller's order.  Items of size n
    // occupy [begin[n], begin[n - 1]).
    std::vector<int> byn[11];
    for (int i = 0; i < count; ++i) byn[n_host[i]].push_back(i);
    int64_t k = 0;
    for (int n = 10; n >= 1; --n) {
        bl->begin[n] = (int)k;
        for (int mi : byn[n]) {
            const int groups = 1 << (n - logt_of(dt, n));
            for (int g = 0; g < groups; ++g) {
                its[k].mat = (uint32_t)mi;
                its[k].group = (uint32_t)g;
                ++k;
            }
        }
    }
    bl->begin[0] = (int)k;
    bl->nitems = (int)items;
    for (int n = 1; n <= 10; ++n)
        bl->plan[n] = rec ? 0 : (force_plan >= 0 ? force_plan : group_plan(n, dt, herm));
}

hipError_t batched_launch(ptd_dtype dt, bool herm, bool rec, bool adjoint, const void* in_base, void* out_base,
                          void* buf, int count, const BatchLaunch& bl, int cus, hipStream_t st, bool concurrent)
{
    uint32_t* counters = (uint32_t*)buf;
    const BatchMat* mats = (const BatchMat*)((unsigned char*)buf + BATCH_HEAD_BYTES);
    const BatchItem* its =
        (const BatchItem*)((unsigned char*)buf + BATCH_HEAD_BYTES + (size_t)count * sizeof(BatchMat));
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(256), 0, st, counters);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int adj = adjoint ? 1 : 0;
    hipStream_t lanes[MAX_LANES] = {st, st, st, st};
    const int nl = batch_launch_count(bl);
    SideLanes* L = nullptr;
    std::unique_lock<std::mutex> lk(g_lanes_mu, std::defer_lock);
    if (concurrent && nl > 1) {
        // fork: every launch after the first waits for the counters' reset
        // on a side stream of its own; the caller's stream joins them all
        lk.lock();
        if ((e = side_lanes(&L)) != hipSuccess) return e;
        if ((e = hipEventRecord(L->fork, st)) != hipSuccess) return e;
        for (int i = 1; i < nl; ++i) {
            lanes[i] = L->s[i - 1];
            if ((e = hipStreamWaitEvent(lanes[i], L->fork, 0)) != hipSuccess) return e;
        }
    }
#define PTD_ALL(VV, HH, RR) launch_all<VV, HH, RR>(bl, in_base, out_base, mats, its, counters, adj, cus, lanes)
    if (dt == PTD_C128) {
        if (rec) {
            if (herm) PTD_ALL(double, true, true); else PTD_ALL(double, false, true);
        } else {
            if (herm) PTD_ALL(double, true, false); else PTD_ALL(double, false, false);
        }
    } else {
        if (rec) {
            if (herm) PTD_ALL(float, true, true); else PTD_ALL(float, false, true);
        } else {
            if (herm) PTD_ALL(float, true, false); else PTD_ALL(float, false, false);
        }
    }
#undef PTD_ALL
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (L) {
        for (int i = 1; i < nl; ++i) {
            if ((e = hipEventRecord(L->join[i - 1], lanes[i])) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(st, L->join[i - 1], 0)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

}  // namespace ptd
