// internal.hpp -- launchers shared between the host API and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/ptd.h"

namespace ptd {

// Where a decomposition reads the entries d_x[k] = A[k][k ^ x].  SRC_MATRIX:
// the dense matrix (row pitch lda).  Matrix-free inputs, whose few defining
// values stay in cache: SRC_TOEPLITZ, A[r][c] = t[c - r + 2^n - 1] with t at
// A; SRC_PURE, the density matrix of a pure state, A[r][c] = psi[r]
// conj(psi[c]) with psi at A; SRC_LOWRANK, a mixed state U U^* given by its
// 2^n x R factor U at A, A[r][c] = sum_j U[r][j] conj(U[c][j]), whose row
// pitch and rank travel packed in the lda argument (lowrank_ld).
constexpr int SRC_MATRIX = 0;
constexpr int SRC_TOEPLITZ = 1;
constexpr int SRC_PURE = 2;
constexpr int SRC_LOWRANK = 3;
// SRC_LOWRANK_T: the same mixed state from the factor's transpose
// UT[j][r] = U[r][j] (column j of U contiguous, 2^n values), staged in the
// workspace so that consecutive lanes (consecutive r) read consecutive
// values; lowrank_ld carries the rank (pitch 2^n).
constexpr int SRC_LOWRANK_T = 4;
constexpr int LOWRANK_MAX = 32;
inline int64_t lowrank_ld(int64_t pitch, int rank) { return (pitch << 6) | (int64_t)rank; }

// Dense decompose: coeff[x][z] (complex, or real when herm) for n in 1..16.
// path: 0 = automatic, 1 = force the single-pass group kernel (n <= 10),
// 2 = force the two-pass tile + high kernels (n >= 7).
// unscaled: Tr(P A) instead of 2^-n Tr(P A) (the adjoint of reconstruction).
hipError_t launch_dense_fwd(int n, ptd_dtype dt, bool herm, const void* A, int64_t lda, void* out,
                            int path, hipStream_t st, bool unscaled = false);

// One pass of the two-pass dense schedule (1 = tile, 2 = row, 3 = both); timing hook.
hipError_t launch_dense_fwd_stage(int n, ptd_dtype dt, bool herm, const void* A, int64_t lda, void* out, int stage,
                                  hipStream_t st);

// Dense complex64 decompose with compensated (TwoSum) butterflies: one
// workgroup for n <= 6, the two-pass schedule otherwise.
hipError_t launch_dense_fwd_comp(int n, bool herm, const void* A, int64_t lda, void* out, hipStream_t st);

// Dense reconstruct: A = scale_log2 ... A = 2^-adj_n * sum_P c_P P.
hipError_t launch_dense_rec(int n, ptd_dtype dt, bool herm, bool adjoint, const void* coeff, void* A,
                            int64_t lda, int path, hipStream_t st);

// Diagonal (s = 0) and banded decompose over the `count` nonempty X-patterns.
hipError_t launch_structured(int n, ptd_dtype dt, bool herm, bool bands, bool compact, int s, int count,
                             const void* A, int64_t lda, void* out, hipStream_t st);

// Sparse input given as nnz coordinate entries (rows, cols: int32 device
// arrays; vals: complex of dt), or, when rows is null, in compressed-row form
// (row_ptr: 2^n + 1 int64 device values, each row's range clipped to
// [0, nnz)).  ws holds sparse_workspace_bytes(n).
size_t sparse_workspace_bytes(int n);
// The distinct r ^ c over the entries, ascending, into xs; synchronises st.
hipError_t launch_sparse_nonempty_x(int n, int64_t nnz, const int32_t* rows, const int64_t* row_ptr,
                                    const int32_t* cols, uint32_t* xs, int* count_host, void* ws, hipStream_t st);
// Coefficients of the listed X-patterns xs[0..count); *bad_xs is set (and
// nothing launched after the check) unless xs is strictly ascending inside
// [0, 2^n).  Synchronises st once, after the check.
hipError_t launch_sparse(int n, ptd_dtype dt, bool compact, int64_t nnz, const int32_t* rows, const int64_t* row_ptr,
                         const int32_t* cols, const void* vals, const uint32_t* xs, int count, void* out, void* ws,
                         bool* bad_xs, hipStream_t st);

// Bandwidth reference kernels (probe.hip): copy / read / write of `bytes`
// (a multiple of 16) in the shape `variant` encodes.
hipError_t launch_bandwidth(int variant, const void* src, void* dst, size_t bytes, hipStream_t st);

// Test hook: the set of HW_REG_XCC_ID values that workgroups of a wide
// launch observe (bit i for die i), and the XCD count the library uses.
hipError_t probe_xcc_ids(unsigned* mask, int* count);

// Every argument check of pauli_decompose except those of the workspace
// (api.hip): PTD_OK, PTD_EINVAL or PTD_EUNSUP, before any HIP call.
ptd_status decompose_check(int n, ptd_dtype dtype, unsigned flags, int s, const void* A, int64_t lda,
                           const void* coeff);
// PTD_OK, or PTD_EHIP with e recorded for ptd_last_hip_error (api.hip).
ptd_status status_from_hip(hipError_t e);

// Limits of the bounded waits in the single-launch kernels (fused.hpp): a
// phase-2 item polls its group's counter at most `spins` times; `extra` is
// added to the counter target (0, except in the test hook below, where no
// target can be reached and every wait gives up).
struct WaitLimits {
    uint32_t spins;
    uint32_t extra;
};
WaitLimits wait_limits();
// Test hook: while on, every bounded wait gives up after a few polls, so a
// test can observe the failure path (NaN outputs, the workspace error word)
// with every kernel still ending normally.
void set_wait_test_mode(bool on);
// Workspace word that a bounded wait sets when it gives up.
constexpr int FUSED_WS_ERR_WORD = 17;

// Single-launch dense decompose for n = 11..15 (fused.hpp); ws holds
// fused_workspace_bytes() bytes of queue and group counters; la = lookahead.
size_t fused_workspace_bytes(int n, ptd_dtype dt);
// cfg 0 = default shape; see fused.hpp for the others.
// The single-launch schedule's reading of a setting (0 = the default):
// workgroup threads, low WHT stages per phase-1 item, X-patterns per group.
bool describe_fused(int n, ptd_dtype dt, bool herm, int cfg, int* threads, int* phase1_bits, int* group_patterns);
hipError_t launch_fused_fwd(int n, ptd_dtype dt, bool herm, const void* A, int64_t lda, void* out, void* ws, int la,
                            int cfg, hipStream_t st, bool unscaled = false);
// Per-dtype instantiations of the single-launch schedule (fused_*.hip).
hipError_t fused_launch_c64(int n, const void* A, int64_t lda, void* out, void* ws, int la, int cfg, bool unscaled,
                            hipStream_t st);
hipError_t fused_launch_c128(int n, const void* A, int64_t lda, void* out, void* ws, int la, int cfg, bool unscaled,
                            hipStream_t st);
hipError_t fused_launch_c64_herm(int n, const void* A, int64_t lda, void* out, void* ws, int la, int cfg, bool unscaled,
                            hipStream_t st);
hipError_t fused_launch_c128_herm(int n, const void* A, int64_t lda, void* out, void* ws, int la, int cfg, bool unscaled,
                            hipStream_t st);
// Single-launch dense reconstruction for n = 11..14 (fused.hpp); ws holds
// fused_workspace_bytes() bytes; real coefficients for the Hermitian forms.
hipError_t fused_rec_c64(int n, const void* coeff, void* A, int64_t lda, void* ws, int la, bool adjoint,
                         hipStream_t st);
hipError_t fused_rec_c128(int n, const void* coeff, void* A, int64_t lda, void* ws, int la, bool adjoint,
                          hipStream_t st);
hipError_t fused_rec_c64_herm(int n, const void* coeff, void* A, int64_t lda, void* ws, int la, bool adjoint,
                              hipStream_t st);
hipError_t fused_rec_c128_herm(int n, const void* coeff, void* A, int64_t lda, void* ws, int la, bool adjoint,
                               hipStream_t st);
hipError_t launch_fused_rec(int n, ptd_dtype dt, bool herm, bool adjoint, const void* coeff, void* A, int64_t lda,
                            void* ws, int la, hipStream_t st);
// Matrix-free input (src: SRC_TOEPLITZ, SRC_PURE or SRC_LOWRANK) given by
// its defining vector or factor (ld: 0, or lowrank_ld for SRC_LOWRANK): the
// single-pass group kernel (n <= 10).
hipError_t launch_group_src(int n, ptd_dtype dt, bool herm, int src, const void* t, int64_t ld, void* out,
                            hipStream_t st);
// Matrix-free input for n = 11..14 (15 for complex64): one workgroup per
// X-pattern, the row's transform in LDS (mfree.hip).
hipError_t launch_mfree(int n, ptd_dtype dt, bool herm, int src, const void* t, int64_t ld, void* out,
                        hipStream_t st);
// UT[j][r] = U[r][j] for r < 2^n, j < rank (U row-major with pitch ld).
hipError_t launch_lowrank_transpose(int n, ptd_dtype dt, const void* U, int64_t ld, int rank, void* UT,
                                    hipStream_t st);
// Zero `count` uint32 words with a small kernel (capturable, unlike a memset node).
hipError_t launch_zero_words(uint32_t* p, int count, hipStream_t st);
// Plain 16-byte-per-lane device copy (bandwidth reference).
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t st);

// Tuned settings of the single-launch schedule (autotune.hip).
struct FusedTuning {
    int cfg;  // shape and options, see fused.hpp (0 = default)
    int la;   // queue lookahead in groups
};
// Default setting at (n, dtype, Hermitian) (fused.hip); cfg = 0 in a call
// stands for its cfg.
FusedTuning fused_default(int n, ptd_dtype dt, bool herm);
bool get_fused_tuning(int n, ptd_dtype dt, bool herm, FusedTuning* t);
void set_fused_tuning(int n, ptd_dtype dt, bool herm, const FusedTuning& t);
void clear_fused_tuning();
hipError_t autotune_fused(int n, ptd_dtype dt, bool herm, int reps, hipStream_t st, FusedTuning* best, float* best_ms,
                          int* tried, int* admitted);

// Plan of the single-pass group kernel at (n, dtype, Hermitian), n <= 10
// (group.hpp plan bits; tuned value if one was set, else the default).
int group_plan(int n, ptd_dtype dt, bool herm);
// Widest WHT round a plan gives size n: radix 32 only for complex64 and
// n >= 6 (single calls and batched launches must agree, since the round
// structure decides the rounding order).
inline int group_effective_rmax(int n, ptd_dtype dt, int plan)
{
    return (dt == PTD_C64 && n >= 6 && (plan & 2)) ? 5 : 4;
}
int group_default_plan(int n, ptd_dtype dt, bool herm);
bool get_group_tuning(int n, ptd_dtype dt, bool herm, int* plan);
void set_group_tuning(int n, ptd_dtype dt, bool herm, int plan);
// Medians and spread of the last autotune of a point (autotune.hip).
bool get_tune_report(int n, ptd_dtype dt, bool herm, float* default_ms, float* best_ms, float* spread_ms, int* kept);
hipError_t autotune_group(int n, ptd_dtype dt, bool herm, int reps, hipStream_t st, int* best, float* best_ms,
                          int* tried, int* admitted);

// Compute units of the current device (256 on MI355X) and its XCD count
// (32 compute units per XCD; partitioned modes expose fewer).
int device_cu_count();
int device_xcd_count();

// Batched single-pass launches over (matrix, group) items, n <= 10 each.
constexpr size_t BATCH_HEAD_BYTES = 1024;  // queue counters, one 64-byte line per size
constexpr int BATCH_SMALL_MAX = 7;  // sizes 1..7 share one batched launch that ignores the group plan
struct BatchLaunch {
    int nitems = 0;      // all items, largest sizes first
    int begin[11] = {};  // items of size n: [begin[n], begin[n - 1]); begin[0] = nitems
    int plan[11] = {};   // group plan per size (group.hpp)
};
int64_t batched_item_count(int count, ptd_dtype dt, const int32_t* n_host);
size_t batched_buffer_bytes(int count, ptd_dtype dt, const int32_t* n_host);
// force_plan >= 0 applies that group plan to every size (autotuning); -1
// takes each size's tuned or default plan (forward only).
void batched_fill(int count, ptd_dtype dt, bool herm, bool rec, const int32_t* n_host, const int64_t* in_off,
                  const int64_t* out_off, std::vector<unsigned char>& img, BatchLaunch* bl, int force_plan = -1);
// concurrent: the per-size launches go to side streams forked from st after
// the counter reset and joined back into st, so each can take the CUs the
// previous one leaves as it drains (within a graph capture: parallel branches)
hipError_t batched_launch(ptd_dtype dt, bool herm, bool rec, bool adjoint, const void* in_base, void* out_base,
                          void* buf, int count, const BatchLaunch& bl, int cus, hipStream_t st,
                          bool concurrent = false);
// Creates this device's side streams and events for concurrent launches
// (once); called before a graph capture so that none is created inside it.
hipError_t prepare_batch_lanes();

// Combinations of decompositions (algebra.hip).  Block i of a block-diagonal
// assembly is read from blocks.p[i] (4^k elements each, 2^m blocks, m <= 5).
struct BlockPtrs {
    const void* p[32];
};
hipError_t launch_block_diagonal(int k, int m, ptd_dtype dt, bool compact, const BlockPtrs& blocks, void* out,
                                 hipStream_t st);
hipError_t launch_hermitian_augment(int n, ptd_dtype dt, bool compact, const void* in, void* out, hipStream_t st);
// dst (2^n x 2^n) = src (rows x cols, pitch ld) top-left, zeros elsewhere.
hipError_t launch_zero_pad(ptd_dtype dt, const void* src, int64_t ld, int64_t rows, int64_t cols, int n, void* dst,
                           hipStream_t st);
hipError_t launch_linear_combination(int n, ptd_dtype dt, double mu_re, double mu_im, const void* a, const void* b,
                                     void* out, hipStream_t st);

// LCU preparation amplitudes amp = sqrt(|c| / sum|c|) (ws: reduce_workspace_bytes()).
hipError_t launch_lcu_amplitudes(int n, ptd_dtype dt, bool real_coeff, const void* coeff, void* amp, void* ws,
                                 double* lambda_host, hipStream_t st);

// Parseval residual: out_host[0] = ||A||_F^2, [1] = 2^n sum|c|^2, [2] = relative gap.
size_t reduce_workspace_bytes();
hipError_t launch_parseval(int n, ptd_dtype dt, bool real_coeff, const void* A, int64_t lda, const void* coeff,
                           void* ws, double* out_host, hipStream_t st);

}  // namespace ptd
