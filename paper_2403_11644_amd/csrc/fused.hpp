// fused.hpp -- single-launch dense decomposition for n = 11..15 (gfx950).
//
// The X-patterns are split into groups of T = 2^t consecutive patterns
// (T = 16 complex64 / 8 complex128: each row of A contributes one 128-byte
// segment to a group, see dense.hip).  For group g the length-2^n WHT over k
// runs in two phases with K = 2^KAP rows per phase-1 item:
//
//   phase 1, item (g, b):  rows k in [b K, (b+1) K) of the group's band are
//       gathered (d_x[k] = A[k][k ^ x]), the low KAP WHT bits are applied in
//       registers and LDS, and the partial result is stored in the output
//       rows of the group at the same positions (in place, no workspace);
//   phase 2, item (g, r, c):  a block of positions z_lo < K of output row
//       x = g T + r: every position owns the 2^(n-KAP) values z_lo + K j,
//       the remaining WHT bits run in registers (the top bit across the two
//       32-lane halves of a wave when there are 32 values), then the phase
//       i^popcount(x&z) and the 2^-n scale are applied and the final
//       coefficients stored.
//
// Hermitian input (Theorem 2).  With xh = x >> KAP (the same for the whole
// group), the partial results of row blocks b and b ^ xh are related by
// W1[x][b ^ xh][z] = (-1)^popcount(z & x & (K-1)) conj(W1[x][b][z]): the
// rows of block b ^ xh read the mirror entries A[k ^ x][k] = conj(A[k][k ^ x]).
// The real output row has room for one real per partial value, so the item
// of the lower block index stores Re W1 in its own slot and Im W1 in the
// partner's, and the partner item reads nothing (the matrix is read in the
// upper block triangle only).  Phase 2 rebuilds each complex partial value
// from the two slots.
//
// Schedule.  A phase-2 item needs every phase-1 item of its group.  Both
// phases run in one persistent launch: each workgroup reads the id of the XCD
// (accelerator complex die) it runs on and takes items from that XCD's queue
// only.  Queue q owns the groups g = q (mod Q) and lists, for m = 0, 1, ...,
// the phase-1 items of its m-th group followed by the phase-2 items of its
// (m - LA)-th group.  Producer and consumer of every partial result share
// one L2: a producer makes its stores complete (s_waitcnt) in every thread,
// meets the workgroup barrier, and then bumps the group's counter with an
// atomic; a consumer polls that counter with an atomic and then reads lines
// that no CU of this launch has read before.  So no L2 write-back or
// invalidation is needed.
//
// Latency hiding comes from two resident workgroups per CU (512 threads,
// 64 KiB of LDS each).  Cache policies are options (POL bits): non-temporal
// gathers of A, non-temporal final stores, non-temporal phase-2 loads of the
// partial results (each is read once, then overwritten).
//
// Measured on MI355X: every store crosses the L2 boundary (a region
// written, read back and overwritten by one workgroup moves twice its size
// out of L2 and its size back in), and reads from the memory-side cache
// come no faster than from HBM.  So the partial band costs one extra write
// and one extra read of the output size at the L2 boundary whatever the
// schedule, and the launch runs near that boundary's throughput.
//
// Progress: a phase-2 item only waits for phase-1 items that precede it in
// the same queue; those were taken by running workgroups, which never wait
// before publishing their own completions, so every wait ends.  The poll is
// bounded anyway: a wait that gives up sets the workspace error word
// (reported by ptd_workspace_status) and its item stores NaN in place of
// every value it would have written, so an incomplete exchange can never
// yield finite coefficients.  If the hardware put no
// workgroup on some XCD, the last workgroup to finish runs that XCD's
// untouched queue by itself.
#pragma once

#include "engine.hpp"
#include "internal.hpp"

namespace ptd {
namespace fused {

// workspace layout (uint32 words)
constexpr int WS_HEAD = 0;    // [16] queue heads
constexpr int WS_DONE = 16;   // finished workgroups
constexpr int WS_ERR = FUSED_WS_ERR_WORD;  // nonzero: a bounded wait ran out
constexpr int WS_GROUP = 32;  // [num groups] phase-1 completions per group

// Bounded poll of a group counter by one thread: true once ws[word] >= need.
// Gives up (false) after wl.spins polls, or at once when another wait of the
// launch has already given up; a give-up sets the error word WS_ERR, which
// ptd_workspace_status reports.  wl.extra raises the target above what the
// producers can reach: a test hook that makes every wait give up.
__device__ __forceinline__ bool bounded_wait(uint32_t* __restrict__ ws, int word, uint32_t need, WaitLimits wl)
{
    const uint32_t target = need + wl.extra;
    uint32_t spins = 0;
    while (__hip_atomic_fetch_add(ws + word, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > wl.spins ||
            ((spins & 255) == 0 && __hip_atomic_load(ws + WS_ERR, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)) {
            __hip_atomic_store(ws + WS_ERR, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    return true;
}

// 2^-n on the host (exact power of two).
template <class V>
inline V exp2_neg_host(int n)
{
    return (V)1 / (V)(1u << n);
}

// cache-policy bits
constexpr int POL_NT_GATHER = 1;
constexpr int POL_NT_STORE = 2;
constexpr int POL_NT_P2LOAD = 4;

template <class V>
constexpr int fused_logt()
{
    return sizeof(V) == 4 ? 4 : 3;
}

__device__ __forceinline__ int xcc_id()
{
    // hwreg(HW_REG_XCC_ID, 0, 4): id 20, offset 0, width 4
    return (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 0xF);
}

struct Item {
    int phase;  // 1 or 2, 0 = none
    int group;
    int sub;
};

// i-th item of queue q; NP1 / NP2 items per group, LA groups of lookahead.
__device__ __forceinline__ Item decode_item(int i, int q, int Q, int groups_q, int NP1, int NP2, int LA)
{
    Item it{0, 0, 0};
    // block m holds P1(m) (if m < groups_q) then P2(m - la) (if m >= la):
    // blocks 0..la-1 hold NP1 items, blocks la..groups_q-1 hold NP1+NP2,
    // blocks groups_q..groups_q+la-1 hold NP2.
    const int la = LA < groups_q ? LA : groups_q;
    const int pre = la * NP1;
    if (i < pre) {
        it.phase = 1;
        it.group = i / NP1;
        it.sub = i % NP1;
    } else {
        const int i2 = i - pre;
        const int mid = (groups_q - la) * (NP1 + NP2);
        if (i2 < mid) {
            const int m = la + i2 / (NP1 + NP2);
            const int r = i2 % (NP1 + NP2);
            if (r < NP1) {
                it.phase = 1;
                it.group = m;
                it.sub = r;
            } else {
                it.phase = 2;
                it.group = m - la;
                it.sub = r - NP1;
            }
        } else {
            const int i3 = i2 - mid;
            if (i3 < la * NP2) {
                it.phase = 2;
                it.group = groups_q - la + i3 / NP2;
                it.sub = i3 % NP2;
            }
        }
    }
    it.group = it.group * Q + q;
    return it;
}

template <class V>
struct VecOf;
template <>
struct VecOf<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct VecOf<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};

template <class V, bool NT>
__device__ __forceinline__ void load_c(const cplx<V>* p, V& re, V& im)
{
    if constexpr (NT) {
        const typename VecOf<V>::type v = __builtin_nontemporal_load((const typename VecOf<V>::type*)p);
        re = v.x;
        im = v.y;
    } else {
        const cplx<V> v = *p;
        re = v.re;
        im = v.im;
    }
}

template <class V, bool NT>
__device__ __forceinline__ void store_c(cplx<V>* p, V re, V im)
{
    if constexpr (NT) {
        typename VecOf<V>::type v;
        v.x = re;
        v.y = im;
        __builtin_nontemporal_store(v, (typename VecOf<V>::type*)p);
    } else {
        cplx<V> v;
        v.re = re;
        v.im = im;
        *p = v;
    }
}

template <class V, bool NT>
__device__ __forceinline__ V load_r(const V* p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <class V, bool NT>
__device__ __forceinline__ void store_r(V* p, V v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Compile-time shape of one configuration: 2^LOGT X-patterns per group,
// 2^KAP rows per phase-1 item, NT threads per workgroup.
template <class V, int LOGN_, int KAP_, int NT_, int LOGT_>
struct Shape {
    static constexpr int LOGN = LOGN_;
    static constexpr int KAP = KAP_;
    static constexpr int NT = NT_;
    static constexpr int LOGT = LOGT_;
    static constexpr int NB2 = LOGN - KAP;  // phase-2 WHT bits
    // top WHT bit across the two halves of a wave (keeps phase 2 within 128
    // registers): above 16 complex64 or 8 complex128 values per thread
    static constexpr bool SWAP = NT == 512 && (sizeof(V) == 8 ? NB2 >= 4 : NB2 >= 5);
    static constexpr bool STASH = (NB2 == 5 && NT == 1024);  // 16 values wait in LDS
    static constexpr int ZB = SWAP ? NT / 2 : NT;            // positions per phase-2 item
    static constexpr int IPR = (1 << KAP) / ZB;              // phase-2 items per row
    static constexpr int NP1 = 1 << (LOGN - KAP);
    static constexpr int NP2 = (1 << LOGT) * IPR;
    static constexpr int NG = 1 << (LOGN - LOGT);
    static_assert(ZB <= (1 << KAP), "phase-2 block within a row");
    static_assert(NB2 >= 1 && NB2 <= 5, "phase-2 radix 2..32");
};

// Phase-1 rounds over bits [B0, KAP): radix-16 steps, the first gathering
// from A (vector index fastest across lanes), the last storing (positions
// fastest across lanes for contiguous output rows, or with VEC_LAST the
// vector index fastest, for stores into the band's row segments).
template <class V, class S, int B0, bool VEC_LAST = false, class G, class St>
__device__ __forceinline__ void p1_rounds(const G& gather, const St& store, cplx<V>* lds)
{
    constexpr int KAP = S::KAP, LOGT = S::LOGT, NT = S::NT;
    constexpr int NB = (KAP - B0) < 4 ? (KAP - B0) : 4;
    constexpr bool FIRST = B0 == 0, LAST = B0 + NB == KAP;
    LdsVecs<V, KAP> lr{lds};
    LdsVecsW<V, KAP> lw{lds};
    if constexpr (FIRST && LAST) {
        wht_round<V, LOGT, KAP, B0, NB, NT, true>(gather, store);
    } else if constexpr (FIRST) {
        wht_round<V, LOGT, KAP, B0, NB, NT, true>(gather, lw);
        __syncthreads();
        p1_rounds<V, S, B0 + NB, VEC_LAST>(gather, store, lds);
    } else if constexpr (LAST) {
        wht_round<V, LOGT, KAP, B0, NB, NT, VEC_LAST>(lr, store);
    } else {
        wht_round<V, LOGT, KAP, B0, NB, NT, false>(lr, lw);
        __syncthreads();
        p1_rounds<V, S, B0 + NB, VEC_LAST>(gather, store, lds);
    }
}

template <class V, class S, bool HERM, int POL>
__device__ __forceinline__ void phase1(const cplx<V>* __restrict__ A, int64_t lda, void* __restrict__ out, int g,
                                       int b, cplx<V>* lds)
{
    constexpr int KAP = S::KAP, LOGT = S::LOGT;
    constexpr int N = 1 << S::LOGN;
    const uint32_t xg = (uint32_t)g << LOGT;
    const int k0 = b << KAP;
    // partner block of b under the conjugate symmetry of Hermitian input
    const int bp = b ^ (int)(xg >> KAP);
    if constexpr (HERM) {
        if (b > bp) return;  // the partner item stores this block's slots
    }
    auto gather = [&](int vec, int pos, V& re, V& im) {
        const int k = k0 + pos;
        load_c<V, (POL & POL_NT_GATHER) != 0>(A + (int64_t)k * lda + (k ^ (int)(xg | vec)), re, im);
    };
    auto store = [&](int vec, int pos, V re, V im) {
        const uint32_t x = xg | (uint32_t)vec;
        const int64_t row = (int64_t)x * N;
        if constexpr (HERM) {
            if (b < bp) {
                ((V*)out)[row + k0 + pos] = re;
                ((V*)out)[row + (bp << KAP) + pos] = im;
            } else {
                // self-partnered block: W1 is real or imaginary by the sign
                const bool sneg = __popc((uint32_t)pos & (x & ((1u << KAP) - 1))) & 1;
                ((V*)out)[row + k0 + pos] = sneg ? im : re;
            }
        } else {
            cplx<V> c;
            c.re = re;
            c.im = im;
            ((cplx<V>*)out)[row + k0 + pos] = c;
        }
    };
    p1_rounds<V, S, 0>(gather, store, lds);
}

// Phase-2 epilogue of one value: phase i^popcount(x&z), scale, store.
template <class V, bool HERM, bool NT>
__device__ __forceinline__ void store_final(void* __restrict__ out, int64_t o, uint32_t x, uint32_t z, V re, V im,
                                            V scale)
{
    mul_ipow(__popc(x & z) & 3, re, im);
    if constexpr (HERM)
        store_r<V, NT>((V*)out + o, re * scale);
    else
        store_c<V, NT>((cplx<V>*)out + o, re * scale, im * scale);
}

// a[j] <- a[j ^ m] for a runtime mask m < 2^NB (conditional swaps per bit).
template <class V, int NB>
__device__ __forceinline__ void xor_permute(V* a, int m)
{
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const bool flip = (m >> b) & 1;
#pragma unroll
        for (int j = 0; j < (1 << NB); ++j) {
            if (!(j & (1 << b))) {
                const V u = a[j], v = a[j | (1 << b)];
                a[j] = flip ? v : u;
                a[j | (1 << b)] = flip ? u : v;
            }
        }
    }
}

template <class V>
__device__ __forceinline__ V swap_halves(V v)
{
    return __shfl_xor(v, 32, 64);
}

template <class V, class S, bool HERM, int POL>
__device__ __forceinline__ void phase2(void* __restrict__ out, int g, int sub, cplx<V>* lds, bool poison, V unit)
{
    constexpr int KAP = S::KAP, NB2 = S::NB2;
    constexpr int N = 1 << S::LOGN;
    constexpr bool NTS = (POL & POL_NT_STORE) != 0, NTL = (POL & POL_NT_P2LOAD) != 0;
    const int r = sub / S::IPR;
    const int zl0 = (sub % S::IPR) * S::ZB;
    const uint32_t x = ((uint32_t)g << S::LOGT) | (uint32_t)r;
    // a group whose partial results never all arrived: every value of the
    // item becomes NaN (the scale is multiplied into every stored value)
    const V scale = poison ? __builtin_nan("") : unit;
    const int64_t rowo = (int64_t)x * N;
    if constexpr (S::STASH) {
        // 32 values per position: the first 16 take a 16-point transform and
        // wait in this thread's own LDS slots while the second 16 take theirs;
        // the last radix-2 stage pairs j with j + 16.
        static_assert(!HERM, "32-point phase 2 with LDS stash is complex only");
        const int zl = zl0 + (int)threadIdx.x;
        const cplx<V>* row = (const cplx<V>*)out + rowo;
        V re[16], im[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) load_c<V, NTL>(row + (j << KAP) + zl, re[j], im[j]);
        wht_reg<V, 4>(re, im);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            cplx<V> c;
            c.re = re[j];
            c.im = im[j];
            lds[(j << KAP) + threadIdx.x] = c;
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) load_c<V, NTL>(row + ((j + 16) << KAP) + zl, re[j], im[j]);
        wht_reg<V, 4>(re, im);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const cplx<V> u = lds[(j << KAP) + threadIdx.x];
            const uint32_t z0 = ((uint32_t)j << KAP) | (uint32_t)zl;
            const uint32_t z1 = ((uint32_t)(j + 16) << KAP) | (uint32_t)zl;
            store_final<V, HERM, NTS>(out, rowo + z0, x, z0, u.re + re[j], u.im + im[j], scale);
            store_final<V, HERM, NTS>(out, rowo + z1, x, z1, u.re - re[j], u.im - im[j], scale);
        }
    } else {
        // NL values per thread; with SWAP the thread's global index is
        // jg = (jh << NBL) | jl, jh = lane bit 5.
        constexpr int NBL = S::SWAP ? NB2 - 1 : NB2;
        constexpr int NL = 1 << NBL;
        const int lane = (int)(threadIdx.x & 63);
        const int jh = S::SWAP ? (lane >> 5) : 0;
        const int zl = S::SWAP ? zl0 + (int)((threadIdx.x >> 6) << 5) + (lane & 31) : zl0 + (int)threadIdx.x;
        V re[NL], im[NL];
        if constexpr (HERM) {
            // slots j and j ^ xh hold (Re, Im) of one partial value; rebuild
            const V* row = (const V*)out + rowo;
#pragma unroll
            for (int j = 0; j < NL; ++j) re[j] = load_r<V, NTL>(row + ((((jh << NBL) | j) << KAP) + zl));
            const int xh = (int)(x >> KAP);
#pragma unroll
            for (int j = 0; j < NL; ++j) im[j] = re[j];
            xor_permute<V, NBL>(im, xh & (NL - 1));
            if constexpr (S::SWAP) {
                if ((xh >> NBL) & 1) {
#pragma unroll
                    for (int j = 0; j < NL; ++j) im[j] = swap_halves(im[j]);
                }
            }
            const bool sneg = __popc((uint32_t)zl & (x & ((1u << KAP) - 1))) & 1;
            const int hb = xh ? 31 - __clz(xh) : -1;
#pragma unroll
            for (int j = 0; j < NL; ++j) {
                const int jg = (jh << NBL) | j;
                const V own = re[j], par = im[j];
                if (hb < 0) {
                    re[j] = sneg ? (V)0 : own;
                    im[j] = sneg ? own : (V)0;
                } else if (!((jg >> hb) & 1)) {  // jg < jg ^ xh
                    re[j] = own;
                    im[j] = par;
                } else {
                    re[j] = sneg ? -par : par;
                    im[j] = sneg ? own : -own;
                }
            }
        } else {
            const cplx<V>* row = (const cplx<V>*)out + rowo;
#pragma unroll
            for (int j = 0; j < NL; ++j) load_c<V, NTL>(row + ((((jh << NBL) | j) << KAP) + zl), re[j], im[j]);
        }
        wht_reg<V, NBL>(re, im);
        if constexpr (S::SWAP) {
            // radix-2 over jh between lane l and lane l ^ 32
#pragma unroll
            for (int j = 0; j < NL; ++j) {
                const V pr = swap_halves(re[j]), pi = swap_halves(im[j]);
                re[j] = jh ? pr - re[j] : re[j] + pr;
                im[j] = jh ? pi - im[j] : im[j] + pi;
            }
        }
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            const uint32_t z = ((uint32_t)((jh << NBL) | j) << KAP) | (uint32_t)zl;
            store_final<V, HERM, NTS>(out, rowo + z, x, z, re[j], im[j], scale);
        }
    }
}

template <class V, class S, bool HERM, int POL>
// at least 4 waves per SIMD: two 512-thread workgroups fit on one CU
__global__ __launch_bounds__(S::NT, 4) void k_fused_fwd(const cplx<V>* __restrict__ A, int64_t lda,
                                                     void* __restrict__ out, uint32_t* __restrict__ ws, int Q,
                                                     int LA, WaitLimits wl, V unit)
{
    // Hermitian phase-2 rows are half the bytes of complex ones: several per
    // item (one ticket and one counter wait for all of them).  Measured at
    // n = 13: complex64 0.2045 / 0.190 / 0.187 ms with 1 / 2 / 4 rows per
    // item, complex128 unchanged with 2; complex rows stay one per item
    // (2 per item: n = 15 complex64 4.94 -> 6.64 ms).  Listing only the
    // Hermitian phase-1 blocks that do work (half the items where a block's
    // mirror is another block) measured 0.187 -> 0.185 ms complex64 but
    // 0.342 -> 0.368 ms complex128: phase-2 items reach their group sooner
    // and wait, so the empty items stay
    constexpr int P2M = HERM ? (sizeof(V) == 4 ? 4 : 2) : 1;
    constexpr int NP1 = S::NP1, NP2 = S::NP2 / P2M, NG = S::NG;
    static_assert(S::NP2 % P2M == 0, "whole phase-2 pairs");
    __shared__ cplx<V> lds[(1 << S::LOGT) * ((1 << S::KAP) + 1)];
    __shared__ int s_next;
    __shared__ int s_last;

    // completion of a phase-1 item: every thread's stores are complete in
    // L2 (s_waitcnt), the barrier covers every other thread, then one bump
    auto publish = [&](int grp) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(ws + WS_GROUP + grp, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    __shared__ int s_fail;
    auto wait_group = [&](int grp) -> bool {
        if (threadIdx.x == 0) s_fail = bounded_wait(ws, WS_GROUP + grp, (uint32_t)NP1, wl) ? 0 : 1;
        __syncthreads();
        return s_fail != 0;
    };
    auto groups_of = [&](int q) { return (NG - q + Q - 1) / Q; };
    auto drain = [&](int q) {
        const int gq = groups_of(q);
        const int total = gq * (NP1 + NP2);
        if (threadIdx.x == 0)
            s_next = (int)__hip_atomic_fetch_add(ws + WS_HEAD + q, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        int cur = __builtin_amdgcn_readfirstlane(s_next);
        while (cur < total) {
            const Item it = decode_item(cur, q, Q, gq, NP1, NP2, LA);
            if (it.phase == 1) {
                phase1<V, S, HERM, POL>(A, lda, out, it.group, it.sub, lds);
                publish(it.group);
            } else {
                const bool failed = wait_group(it.group);
#pragma unroll
                for (int u = 0; u < P2M; ++u) phase2<V, S, HERM, POL>(out, it.group, it.sub * P2M + u, lds, failed, unit);
            }
            __syncthreads();  // LDS reuse, s_next reuse
            if (threadIdx.x == 0)
                s_next = (int)__hip_atomic_fetch_add(ws + WS_HEAD + q, 1u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            cur = __builtin_amdgcn_readfirstlane(s_next);
        }
    };

    drain(xcc_id() % Q);
    // last workgroup: run any queue no workgroup was placed on
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0)
        s_last = __hip_atomic_fetch_add(ws + WS_DONE, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                 gridDim.x - 1;
    __syncthreads();
    if (!s_last) return;
    for (int qq = 0; qq < Q; ++qq) drain(qq);
}

// ------------------------------------------------------------------------
// Reconstruction, the same schedule run backwards.  For X-pattern x,
// d_x = WHT( (-i)^popcount(x&z) c[x][z] ) over z, and A[k][k ^ x] = d_x[k]
// (times 2^-n for the adjoint).  The group's band of A (one 128-byte
// segment per row) holds the intermediate: slot x_lo of row k's segment.
//
//   phase R1, item (g, s):  coefficient columns z_lo in [s Z, (s+1) Z) of
//       the group's T rows: inverse phase, the WHT over the high bits (the
//       row-block index j of k = j K + z_lo) in registers, then a transpose
//       through LDS so that lanes over x_lo store whole segments
//       A[j K + z_lo][seg + x_lo];
//   phase R2, item (g, b):  rows k in [b K, (b+1) K) of the band: the low
//       KAP WHT bits in registers and LDS, and d_x[k] stored to A[k][k ^ x]
//       (the same segment, slots permuted), in place.
//
// R2 items of a group wait for all its R1 items (counter per group), as in
// the forward launch.

template <class V, class S>
struct RecShape {
    static constexpr bool SW = S::SWAP;
    static constexpr int NBL = SW ? S::NB2 - 1 : S::NB2;
    static constexpr int NL = 1 << NBL;                     // values per thread
    static constexpr int PAIRS = SW ? S::NT / 2 : S::NT;  // (x_lo, z_lo) pairs per item
    static constexpr int T = 1 << S::LOGT;
    static constexpr int ZR = PAIRS / T;                  // z_lo columns per R1 item
    static constexpr int NR1 = (1 << S::KAP) / ZR;        // R1 items per group
    static constexpr int NR2 = 1 << (S::LOGN - S::KAP);   // R2 items per group
    static constexpr int H = SW ? 2 : 1;
    // values per thread moved through LDS per transpose round
    static constexpr int RB_FIT = ((1 << S::KAP) + 1) / (H * (ZR + 1));
    static constexpr int RB = RB_FIT >= 16 ? 16 : RB_FIT >= 8 ? 8 : RB_FIT >= 4 ? 4 : RB_FIT >= 2 ? 2 : 1;
    static constexpr int RBU = RB < NL ? RB : NL;
    static_assert(ZR >= 1 && (1 << S::KAP) % ZR == 0, "R1 items tile the row block");
    static_assert(H * RBU * T * (ZR + 1) <= T * ((1 << S::KAP) + 1), "transpose fits the LDS of phase 1");
};

template <class V, class S, bool REAL_IN>
__device__ __forceinline__ void rec_phase1(const void* __restrict__ coeff, cplx<V>* __restrict__ A, int64_t lda,
                                           int g, int sub, cplx<V>* lds)
{
    typedef RecShape<V, S> R;
    constexpr int KAP = S::KAP, LOGT = S::LOGT, T = R::T, ZR = R::ZR, NBL = R::NBL, NL = R::NL;
    constexpr int N = 1 << S::LOGN;
    const int lane = (int)(threadIdx.x & 63);
    const int jh = R::SW ? (lane >> 5) : 0;
    const int p = R::SW ? (((int)threadIdx.x >> 6) << 5) | (lane & 31) : (int)threadIdx.x;
    const uint32_t xg = (uint32_t)g << LOGT;
    const int z0 = sub * ZR;
    // load side: z_lo fastest across lanes (contiguous coefficient runs)
    const int xl = p / ZR, zl = p % ZR;
    const uint32_t x = xg | (uint32_t)xl;
    V re[NL], im[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) {
        const uint32_t z = (uint32_t)(z0 + zl) | ((uint32_t)((jh << NBL) | j) << KAP);
        const int64_t o = (int64_t)x * N + z;
        if constexpr (REAL_IN) {
            re[j] = __builtin_nontemporal_load((const V*)coeff + o);
            im[j] = (V)0;
        } else {
            load_c<V, true>((const cplx<V>*)coeff + o, re[j], im[j]);
        }
        mul_ipow((4 - (__popc(x & z) & 3)) & 3, re[j], im[j]);
    }
    wht_reg<V, NBL>(re, im);
    if constexpr (R::SW) {
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            const V pr = swap_halves(re[j]), pi = swap_halves(im[j]);
            re[j] = jh ? pr - re[j] : re[j] + pr;
            im[j] = jh ? pi - im[j] : im[j] + pi;
        }
    }
    // store side: x_lo fastest across lanes (whole 128-byte segments)
    const int xs = p % T, zs = p / T;
    constexpr int PITCH = ZR + 1;
#pragma unroll
    for (int r0 = 0; r0 < NL; r0 += R::RBU) {
        __syncthreads();  // previous round's reads are done
#pragma unroll
        for (int jr = 0; jr < R::RBU; ++jr) {
            cplx<V> c;
            c.re = re[r0 + jr];
            c.im = im[r0 + jr];
            lds[((jh * R::RBU + jr) * T + xl) * PITCH + zl] = c;
        }
        __syncthreads();
#pragma unroll
        for (int jr = 0; jr < R::RBU; ++jr) {
            const cplx<V> c = lds[((jh * R::RBU + jr) * T + xs) * PITCH + zs];
            const int k = (((jh << NBL) | (r0 + jr)) << KAP) | (z0 + zs);
            const int64_t col = (int64_t)(((uint32_t)k ^ xg) & ~(uint32_t)(T - 1)) + xs;
            A[(int64_t)k * lda + col] = c;
        }
    }
}

template <class V, class S>
__device__ __forceinline__ void rec_phase2(cplx<V>* __restrict__ A, int64_t lda, int g, int b, cplx<V>* lds,
                                           V scale, bool poison)
{
    if (poison) scale = __builtin_nan("");  // the group's intermediate is incomplete
    constexpr int KAP = S::KAP, LOGT = S::LOGT, T = 1 << LOGT;
    const uint32_t xg = (uint32_t)g << LOGT;
    const int k0 = b << KAP;
    auto gather = [&](int vec, int pos, V& re, V& im) {
        const int k = k0 + pos;
        const int64_t col = (int64_t)(((uint32_t)k ^ xg) & ~(uint32_t)(T - 1)) + vec;
        load_c<V, false>(A + (int64_t)k * lda + col, re, im);
    };
    auto store = [&](int vec, int pos, V re, V im) {
        const int k = k0 + pos;
        store_c<V, true>(A + (int64_t)k * lda + ((uint32_t)k ^ (xg | (uint32_t)vec)), re * scale, im * scale);
    };
    // lanes over the vector index in the last round: whole segments per store
    p1_rounds<V, S, 0, true>(gather, store, lds);
}

template <class V, class S, bool REAL_IN>
__global__ __launch_bounds__(S::NT, 4) void k_fused_rec(const void* __restrict__ coeff, cplx<V>* __restrict__ A,
                                                     int64_t lda, uint32_t* __restrict__ ws, int Q, int LA,
                                                     WaitLimits wl, V scale)
{
    typedef RecShape<V, S> R;
    constexpr int NP1 = R::NR1, NP2 = R::NR2, NG = S::NG;
    __shared__ cplx<V> lds[(1 << S::LOGT) * ((1 << S::KAP) + 1)];
    __shared__ int s_next;
    __shared__ int s_last;

    auto publish = [&](int grp) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(ws + WS_GROUP + grp, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    __shared__ int s_fail;
    auto wait_group = [&](int grp) -> bool {
        if (threadIdx.x == 0) s_fail = bounded_wait(ws, WS_GROUP + grp, (uint32_t)NP1, wl) ? 0 : 1;
        __syncthreads();
        return s_fail != 0;
    };
    auto groups_of = [&](int q) { return (NG - q + Q - 1) / Q; };
    auto drain = [&](int q) {
        const int gq = groups_of(q);
        const int total = gq * (NP1 + NP2);
        if (threadIdx.x == 0)
            s_next = (int)__hip_atomic_fetch_add(ws + WS_HEAD + q, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        int cur = __builtin_amdgcn_readfirstlane(s_next);
        while (cur < total) {
            const Item it = decode_item(cur, q, Q, gq, NP1, NP2, LA);
            if (it.phase == 1) {
                rec_phase1<V, S, REAL_IN>(coeff, A, lda, it.group, it.sub, lds);
                publish(it.group);
            } else {
                const bool failed = wait_group(it.group);
                rec_phase2<V, S>(A, lda, it.group, it.sub, lds, scale, failed);
            }
            __syncthreads();  // LDS reuse, s_next reuse
            if (threadIdx.x == 0)
                s_next = (int)__hip_atomic_fetch_add(ws + WS_HEAD + q, 1u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            cur = __builtin_amdgcn_readfirstlane(s_next);
        }
    };

    drain(xcc_id() % Q);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0)
        s_last = __hip_atomic_fetch_add(ws + WS_DONE, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                 gridDim.x - 1;
    __syncthreads();
    if (!s_last) return;
    for (int qq = 0; qq < Q; ++qq) drain(qq);
}

template <class V, int LOGN, bool REAL_IN>
hipError_t launch_rec_n(const void* coeff, void* A, int64_t lda, void* ws, int la, bool adjoint, hipStream_t st)
{
    // 512-thread workgroups, 512-row R2 items, 128-byte segments
    typedef Shape<V, LOGN, 9, 512, fused_logt<V>()> S;
    const int words = WS_GROUP + S::NG;
    hipError_t e = launch_zero_words((uint32_t*)ws, words, st);
    if (e != hipSuccess) return e;
    const V scale = adjoint ? (V)1 / (V)(1u << LOGN) : (V)1;  // exact power of two
    hipLaunchKernelGGL((k_fused_rec<V, S, REAL_IN>), dim3(device_cu_count() * 2), dim3(512), 0, st, coeff,
                       (cplx<V>*)A, lda, (uint32_t*)ws, device_xcd_count(), la, wait_limits(), scale);
    return hipGetLastError();
}

template <class V, bool REAL_IN>
hipError_t fused_rec_dispatch(int n, const void* coeff, void* A, int64_t lda, void* ws, int la, bool adjoint,
                              hipStream_t st)
{
    switch (n) {
        case 11: return launch_rec_n<V, 11, REAL_IN>(coeff, A, lda, ws, la, adjoint, st);
        case 12: return launch_rec_n<V, 12, REAL_IN>(coeff, A, lda, ws, la, adjoint, st);
        case 13: return launch_rec_n<V, 13, REAL_IN>(coeff, A, lda, ws, la, adjoint, st);
        case 14: return launch_rec_n<V, 14, REAL_IN>(coeff, A, lda, ws, la, adjoint, st);
        default: return hipErrorInvalidValue;
    }
}

template <class V, int LOGN, int KAP, int NT, int LOGT, bool HERM, int POL>
hipError_t launch_cfg(const void* A, int64_t lda, void* out, void* ws, int la, bool unscaled, hipStream_t st)
{
    typedef Shape<V, LOGN, KAP, NT, LOGT> S;
    const int words = WS_GROUP + S::NG;
    hipError_t e = launch_zero_words((uint32_t*)ws, words, st);
    if (e != hipSuccess) return e;
    // persistent grid: as many workgroups as fit at once (LDS-limited)
    const int per_cu = NT == 512 ? 2 : 1;
    hipLaunchKernelGGL((k_fused_fwd<V, S, HERM, POL>), dim3(device_cu_count() * per_cu), dim3(NT), 0, st,
                       (const cplx<V>*)A, lda, out, (uint32_t*)ws, device_xcd_count(), la, wait_limits(),
                       unscaled ? (V)1 : exp2_neg_host<V>(LOGN));
    return hipGetLastError();
}

template <class V, int LOGN, int KAP, int NT, int LOGT, bool HERM>
hipError_t launch_pol(int pol, const void* A, int64_t lda, void* out, void* ws, int la, bool unscaled, hipStream_t st)
{
    switch (pol & 7) {
#define PTD_POL(P) \
    case P: return launch_cfg<V, LOGN, KAP, NT, LOGT, HERM, P>(A, lda, out, ws, la, unscaled, st);
        PTD_POL(0) PTD_POL(1) PTD_POL(2) PTD_POL(3) PTD_POL(4) PTD_POL(5) PTD_POL(6) PTD_POL(7)
#undef PTD_POL
    }
    return hipErrorInvalidValue;
}

// cfg & 3 selects the shape: 1 = 1024 threads, 1024-row items, 128-byte
// row segments (16 complex64 / 8 complex128 X-patterns per group);
// 2 = 512 threads, 512-row items, 128-byte segments; 3 = 512 threads,
// 1024-row items, 64-byte segments (half the X-patterns per group, so half
// the partial band in flight); 0 = default.  +4: non-temporal gather loads;
// +8: non-temporal final stores; +16: non-temporal phase-2 loads.
template <class V, bool HERM>
hipError_t fused_dispatch(int n, const void* A, int64_t lda, void* out, void* ws, int la, int cfg, bool unscaled,
                          hipStream_t st)
{
    constexpr int LT = fused_logt<V>();
    if (cfg == 0) cfg = fused_default(n, sizeof(V) == 8 ? PTD_C128 : PTD_C64, HERM).cfg;
    const int shape = cfg & 3;
    const int pol = (cfg >> 2) & 7;
    if (shape == 0) return hipErrorInvalidValue;
    if (shape >= 2 && n > 14) return hipErrorInvalidValue;
#define PTD_CFG(NN, KK, TT, LL) return launch_pol<V, NN, KK, TT, LL, HERM>(pol, A, lda, out, ws, la, unscaled, st);
    if (shape == 2) {
        switch (n) {
            case 11: PTD_CFG(11, 9, 512, LT)
            case 12: PTD_CFG(12, 9, 512, LT)
            case 13: PTD_CFG(13, 9, 512, LT)
            case 14: PTD_CFG(14, 9, 512, LT)
            default: return hipErrorInvalidValue;
        }
    }
    if (shape == 3) {
        switch (n) {
            case 11: PTD_CFG(11, 10, 512, LT - 1)
            case 12: PTD_CFG(12, 10, 512, LT - 1)
            case 13: PTD_CFG(13, 10, 512, LT - 1)
            case 14: PTD_CFG(14, 10, 512, LT - 1)
            default: return hipErrorInvalidValue;
        }
    }
    switch (n) {
        case 11: PTD_CFG(11, 10, 1024, LT)
        case 12: PTD_CFG(12, 10, 1024, LT)
        case 13: PTD_CFG(13, 10, 1024, LT)
        case 14: PTD_CFG(14, 10, 1024, LT)
        case 15:
            if constexpr (!HERM && sizeof(V) == 4) {
                PTD_CFG(15, 10, 1024, LT)
            }
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
#undef PTD_CFG
}

// What fused_dispatch builds for a setting, in the schedule's own terms:
// workgroup threads, the low WHT stages each phase-1 item applies (the
// remaining n - kap run in phase 2: the stage split) and log2 of the
// X-patterns per group (the tile width T).  False where fused_dispatch
// would refuse the setting.
inline bool fused_describe(int n, bool c64, bool herm, int cfg, int* threads, int* kap, int* logt)
{
    const int LT = c64 ? 4 : 3;
    if (n < 11 || n > 15 || (n == 15 && (!c64 || herm))) return false;
    if (cfg == 0) cfg = fused_default(n, c64 ? PTD_C64 : PTD_C128, herm).cfg;
    const int shape = cfg & 3;
    if (shape == 0 || (shape >= 2 && n > 14) || (cfg >> 5) != 0) return false;
    *threads = shape == 1 ? 1024 : 512;
    *kap = shape == 2 ? 9 : 10;
    *logt = shape == 3 ? LT - 1 : LT;
    return true;
}


}  // namespace fused
}  // namespace ptd
