// api.hip -- the C ABI (include/ptd.h): argument validation first, then
// dispatch to the kernel launchers.  Nothing here touches the GPU before the
// arguments have been checked, so every argument error is testable on a
// machine without one.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "internal.hpp"

namespace {

thread_local int g_last_hip_error = 0;

constexpr unsigned kAllFlags = PTD_HERMITIAN | PTD_DIAGONAL | PTD_BANDED | PTD_BANDS_IN | PTD_COMPACT |
                               PTD_COMPENSATED | PTD_ADJOINT | PTD_ANTIDIAGONAL | PTD_TOEPLITZ | PTD_PURE_STATE |
                               PTD_LOW_RANK;
constexpr unsigned kMatrixFree = PTD_TOEPLITZ | PTD_PURE_STATE | PTD_LOW_RANK;
constexpr unsigned kStructure = PTD_DIAGONAL | PTD_BANDED | PTD_ANTIDIAGONAL;

ptd_status hip_status(hipError_t e)
{
    if (e == hipSuccess) return PTD_OK;
    g_last_hip_error = (int)e;
    return PTD_EHIP;
}

bool valid_dtype(ptd_dtype dt) { return dt == PTD_C128 || dt == PTD_C64; }

// Do the byte ranges [a, a + na) and [b, b + nb) meet?
bool overlap(const void* a, size_t na, const void* b, size_t nb)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

size_t elem_bytes(ptd_dtype dt) { return dt == PTD_C128 ? 16 : 8; }

// Bytes of a row-major array of `rows` rows of `cols` elements at pitch ld.
size_t span_bytes(int64_t rows, int64_t cols, int64_t ld, size_t eb)
{
    return rows < 1 ? 0 : (size_t)((rows - 1) * ld + cols) * eb;
}

// Bytes pauli_decompose reads from A for these arguments (flags checked).
size_t decompose_in_bytes(int n, ptd_dtype dt, unsigned flags, int s, int64_t lda)
{
    const int64_t N = (int64_t)1 << n;
    const size_t eb = elem_bytes(dt);
    if (flags & PTD_TOEPLITZ) return (size_t)(2 * N - 1) * eb;
    if (flags & PTD_PURE_STATE) return (size_t)N * eb;
    if (flags & PTD_LOW_RANK) return span_bytes(N, s, lda, eb);
    if (flags & PTD_BANDS_IN) {
        const int64_t rows = (flags & PTD_BANDED) ? 2 * (int64_t)s + 1 : 1;
        return span_bytes(rows, N, lda, eb);
    }
    return span_bytes(N, N, lda, eb);
}

// Structured-flag checks shared by the decompose entry points.
ptd_status check_structure(int n, unsigned flags, int s)
{
    const bool diag = flags & PTD_DIAGONAL, band = flags & PTD_BANDED, anti = flags & PTD_ANTIDIAGONAL;
    if ((int)diag + (int)band + (int)anti > 1) return PTD_EINVAL;
    if ((flags & (PTD_BANDS_IN | PTD_COMPACT)) && !(diag || band || anti)) return PTD_EINVAL;
    if (band && (s < 1 || s >= (1 << n))) return PTD_EINVAL;
    return PTD_OK;
}

// Dense decompositions of n = 11..15 run as one persistent launch (fused.hip)
// except at n = 15 for complex128 or Hermitian input (the 32-point row
// transform is built for complex64 values only); those and n = 16 use the
// two-pass schedule.
// Dense reconstruction for n = 11..14 runs in one launch (fused.hpp).
bool use_fused_rec(int n) { return n >= 11 && n <= 14; }

bool use_fused(int n, ptd_dtype dt, unsigned flags)
{
    if (flags & (kStructure | PTD_COMPENSATED)) return false;
    if (n < 11 || n > 15) return false;
    if (n == 15 && (dt == PTD_C128 || (flags & PTD_HERMITIAN))) return false;
    return true;
}


}  // namespace

extern "C" {

const char* ptd_status_str(ptd_status st)
{
    switch (st) {
        case PTD_OK: return "PTD_OK";
        case PTD_EINVAL: return "PTD_EINVAL: invalid argument";
        case PTD_ENOSPC: return "PTD_ENOSPC: workspace too small";
        case PTD_EUNSUP: return "PTD_EUNSUP: unsupported request";
        case PTD_EHIP: return "PTD_EHIP: HIP runtime error";
        case PTD_ENOMEM: return "PTD_ENOMEM: allocation failed";
        default: return "PTD_E?: unknown status";
    }
}

int ptd_last_hip_error(void) { return g_last_hip_error; }

const char* ptd_build_arch(void) { return "gfx950"; }

size_t ptd_workspace_bytes(int n, ptd_dtype dtype, unsigned flags, int s)
{
    (void)s;
    if (n < 1 || n > 16 || !valid_dtype(dtype)) return 0;
    // a low-rank factor is staged transposed for the one-row-per-workgroup
    // kernels (n >= 11): rank columns of 2^n values
    if ((flags & PTD_LOW_RANK) && n >= 11 && s >= 1 && s <= ptd::LOWRANK_MAX)
        return (size_t)s * ((size_t)1 << n) * elem_bytes(dtype);
    if (flags & (kStructure | kMatrixFree)) return 0;
    if (use_fused(n, dtype, flags)) return ptd::fused_workspace_bytes(n, dtype);
    return 0;
}

int ptd_num_nonempty_x(int n, unsigned flags, int s)
{
    if (n < 1 || n > 16 || (flags & ~kAllFlags)) return -1;
    if (flags & PTD_ANTIDIAGONAL) return (flags & (PTD_DIAGONAL | PTD_BANDED)) ? -1 : 1;
    if (flags & PTD_DIAGONAL) return (flags & PTD_BANDED) ? -1 : 1;
    if (flags & PTD_BANDED) {
        if (s < 1 || s >= (1 << n)) return -1;
        int count = 1;
        for (int h = 0; h < n; ++h) count += (s < (1 << h)) ? s : (1 << h);
        return count;
    }
    return 1 << n;
}

ptd_status ptd_nonempty_x(int n, unsigned flags, int s, uint32_t* xs_host)
{
    const int cnt = ptd_num_nonempty_x(n, flags, s);
    if (cnt < 0 || !xs_host) return PTD_EINVAL;
    if (flags & PTD_ANTIDIAGONAL) {
        xs_host[0] = (uint32_t)((1u << n) - 1u);
        return PTD_OK;
    }
    if (!(flags & (PTD_DIAGONAL | PTD_BANDED))) {
        for (int i = 0; i < cnt; ++i) xs_host[i] = (uint32_t)i;
        return PTD_OK;
    }
    int i = 0;
    xs_host[i++] = 0;
    if (flags & PTD_BANDED) {
        // x = 2^h + y, 0 <= y < 2^h, with min_k |(k ^ x) - k| = 2^h - y <= s
        for (int h = 0; h < n; ++h) {
            const int top = 2 << h;
            const int lo = (top - s > (1 << h)) ? top - s : (1 << h);
            for (int x = lo; x < top; ++x) xs_host[i++] = (uint32_t)x;
        }
    }
    return PTD_OK;
}

}  // extern "C"

namespace ptd {

// Every argument check of pauli_decompose except those of the workspace:
// PTD_OK, PTD_EINVAL or PTD_EUNSUP, with no HIP call.
ptd_status decompose_check(int n, ptd_dtype dtype, unsigned flags, int s, const void* A, int64_t lda,
                           const void* coeff)
{
    if (n < 1 || n > 16 || !valid_dtype(dtype) || !A || !coeff) return PTD_EINVAL;
    if (flags & ~kAllFlags) return PTD_EINVAL;
    // unscaled traces (the adjoint of reconstruction): dense input only
    if ((flags & PTD_ADJOINT) && (flags & (kStructure | kMatrixFree | PTD_COMPENSATED))) return PTD_EINVAL;
    const ptd_status sst = check_structure(n, flags, s);
    if (sst != PTD_OK) return sst;
    // matrix-free input: a defining vector or factor instead of the matrix
    const unsigned mf = flags & kMatrixFree;
    if (mf & (mf - 1)) return PTD_EINVAL;  // at most one kind
    const bool mfree = mf != 0;
    if (!mfree && lda < ((int64_t)1 << n)) return PTD_EINVAL;
    if ((flags & PTD_LOW_RANK) && (s < 1 || s > ptd::LOWRANK_MAX || lda < s || lda > ((int64_t)1 << 40)))
        return PTD_EINVAL;
    if ((flags & PTD_COMPENSATED) && dtype != PTD_C64) return PTD_EUNSUP;
    // A and coeff must be disjoint (the one-launch schedule keeps partial
    // results in coeff while it still reads A)
    const int rows = (flags & PTD_COMPACT) ? ptd_num_nonempty_x(n, flags, s) : (1 << n);
    if (rows < 1) return PTD_EINVAL;
    const size_t out_eb = (flags & PTD_HERMITIAN) ? elem_bytes(dtype) / 2 : elem_bytes(dtype);
    if (overlap(A, decompose_in_bytes(n, dtype, flags, s, lda), coeff, ((size_t)rows << n) * out_eb))
        return PTD_EINVAL;
    if (mfree) {
        if (flags & (kStructure | PTD_COMPENSATED)) return PTD_EUNSUP;
        if (n > 15 || (n == 15 && dtype == PTD_C128)) return PTD_EUNSUP;
    }
    if ((flags & kStructure) && (flags & PTD_COMPENSATED)) return PTD_EUNSUP;
    return PTD_OK;
}

ptd_status status_from_hip(hipError_t e) { return hip_status(e); }

}  // namespace ptd

namespace {

// Bytes pauli_decompose writes to coeff (arguments already checked).
size_t decompose_out_bytes(int n, ptd_dtype dtype, unsigned flags, int s)
{
    const int rows = (flags & PTD_COMPACT) ? ptd_num_nonempty_x(n, flags, s) : (1 << n);
    const size_t out_eb = (flags & PTD_HERMITIAN) ? elem_bytes(dtype) / 2 : elem_bytes(dtype);
    return ((size_t)rows << n) * out_eb;
}

}  // namespace

extern "C" {

ptd_status pauli_decompose(int n, ptd_dtype dtype, unsigned flags, int s, const void* A, int64_t lda, void* coeff,
                           void* ws, size_t ws_bytes, ptd_stream stream)
{
    const ptd_status chk = ptd::decompose_check(n, dtype, flags, s, A, lda, coeff);
    if (chk != PTD_OK) return chk;
    const size_t need = ptd_workspace_bytes(n, dtype, flags, s);
    if (ws_bytes < need || (need && !ws)) return PTD_ENOSPC;
    if (ws && ws_bytes &&
        (overlap(ws, ws_bytes, A, decompose_in_bytes(n, dtype, flags, s, lda)) ||
         overlap(ws, ws_bytes, coeff, decompose_out_bytes(n, dtype, flags, s))))
        return PTD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const bool herm = flags & PTD_HERMITIAN;
    if (flags & kMatrixFree) {
        const int src = (flags & PTD_TOEPLITZ) ? ptd::SRC_TOEPLITZ
                        : (flags & PTD_PURE_STATE) ? ptd::SRC_PURE
                                                   : ptd::SRC_LOWRANK;
        const int64_t ld = src == ptd::SRC_LOWRANK ? ptd::lowrank_ld(lda, s) : 0;
        if (n <= 10) return hip_status(ptd::launch_group_src(n, dtype, herm, src, A, ld, coeff, st));
        if (src == ptd::SRC_LOWRANK) {
            // factor columns contiguous in the workspace, then the rows
            hipError_t e = ptd::launch_lowrank_transpose(n, dtype, A, lda, s, ws, st);
            if (e != hipSuccess) return hip_status(e);
            return hip_status(ptd::launch_mfree(n, dtype, herm, ptd::SRC_LOWRANK_T, ws, ptd::lowrank_ld(0, s), coeff,
                                                st));
        }
        return hip_status(ptd::launch_mfree(n, dtype, herm, src, A, ld, coeff, st));
    }
    if (flags & kStructure) {
        // s < 0 codes the anti-diagonal for the structured kernels
        const int se = (flags & PTD_ANTIDIAGONAL) ? -1 : (flags & PTD_DIAGONAL) ? 0 : s;
        const int count = ptd_num_nonempty_x(n, flags, s);
        return hip_status(ptd::launch_structured(n, dtype, herm, flags & PTD_BANDS_IN, flags & PTD_COMPACT, se, count,
                                                 A, lda, coeff, st));
    }
    if (flags & PTD_COMPENSATED) return hip_status(ptd::launch_dense_fwd_comp(n, herm, A, lda, coeff, st));
    if (use_fused(n, dtype, flags)) {
        if (!ws) return PTD_ENOSPC;
        ptd::FusedTuning t = ptd::fused_default(n, dtype, herm);
        (void)ptd::get_fused_tuning(n, dtype, herm, &t);
        return hip_status(ptd::launch_fused_fwd(n, dtype, herm, A, lda, coeff, ws, t.la, t.cfg, st,
                                                (flags & PTD_ADJOINT) != 0));
    }
    return hip_status(ptd::launch_dense_fwd(n, dtype, herm, A, lda, coeff, 0, st, (flags & PTD_ADJOINT) != 0));
}

size_t ptd_reconstruct_workspace_bytes(int n, ptd_dtype dtype, unsigned flags)
{
    if (n < 1 || n > 16 || !valid_dtype(dtype) || (flags & ~(PTD_HERMITIAN | PTD_ADJOINT))) return 0;
    return use_fused_rec(n) ? ptd::fused_workspace_bytes(n, dtype) : 0;
}

ptd_status pauli_reconstruct(int n, ptd_dtype dtype, unsigned flags, const void* coeff, void* A, int64_t lda,
                             void* ws, size_t ws_bytes, ptd_stream stream)
{
    if (n < 1 || n > 16 || !valid_dtype(dtype) || !A || !coeff) return PTD_EINVAL;
    if (flags & ~(PTD_HERMITIAN | PTD_ADJOINT)) return PTD_EINVAL;
    if (lda < ((int64_t)1 << n)) return PTD_EINVAL;
    {
        const int64_t N = (int64_t)1 << n;
        const size_t a_bytes = span_bytes(N, N, lda, elem_bytes(dtype));
        const size_t c_bytes = ((size_t)N << n) * ((flags & PTD_HERMITIAN) ? elem_bytes(dtype) / 2 : elem_bytes(dtype));
        if (overlap(A, a_bytes, coeff, c_bytes)) return PTD_EINVAL;
        if (ws && ws_bytes && (overlap(ws, ws_bytes, A, a_bytes) || overlap(ws, ws_bytes, coeff, c_bytes)))
            return PTD_EINVAL;
    }
    const bool herm = flags & PTD_HERMITIAN, adj = flags & PTD_ADJOINT;
    if (use_fused_rec(n)) {
        if (!ws || ws_bytes < ptd_reconstruct_workspace_bytes(n, dtype, flags)) return PTD_ENOSPC;
        // lookahead as measured on MI355X: the forward's at n <= 13, 4 at 14
        const int la = n == 14 ? 4 : ptd::fused_default(n, dtype, herm).la;
        return hip_status(ptd::launch_fused_rec(n, dtype, herm, adj, coeff, A, lda, ws, la, (hipStream_t)stream));
    }
    return hip_status(ptd::launch_dense_rec(n, dtype, herm, adj, coeff, A, lda, 0, (hipStream_t)stream));
}

ptd_status ptd_workspace_status(const void* ws, size_t ws_bytes, ptd_stream stream)
{
    if (ws_bytes == 0) return PTD_OK;
    if (!ws || ws_bytes < 32 * sizeof(uint32_t)) return PTD_EINVAL;
    uint32_t word = 0;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(&word, (const uint32_t*)ws + ptd::FUSED_WS_ERR_WORD, sizeof(word),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_status(e);
    return word ? hip_status(hipErrorLaunchTimeOut) : PTD_OK;
}

size_t ptd_reduce_workspace_bytes(void) { return ptd::reduce_workspace_bytes(); }

ptd_status ptd_parseval_residual(int n, ptd_dtype dtype, unsigned flags, const void* A, int64_t lda, const void* coeff,
                                 double* out_host, void* ws, size_t ws_bytes, ptd_stream stream)
{
    if (n < 1 || n > 16 || !valid_dtype(dtype) || !A || !coeff || !out_host) return PTD_EINVAL;
    if (flags & ~PTD_HERMITIAN) return PTD_EINVAL;
    if (lda < ((int64_t)1 << n)) return PTD_EINVAL;
    if (!ws || ws_bytes < ptd::reduce_workspace_bytes()) return PTD_ENOSPC;
    return hip_status(ptd::launch_parseval(n, dtype, flags & PTD_HERMITIAN, A, lda, coeff, ws, out_host,
                                           (hipStream_t)stream));
}

}  // extern "C"

namespace {


// Outputs whose zero rows are written with 16-byte stores.
bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace

extern "C" {

ptd_status ptd_block_diagonal(int k, int m, ptd_dtype dtype, unsigned flags, const void* blocks, void* coeff_out,
                              ptd_stream stream)
{
    if (k < 1 || m < 1 || m > 5 || k + m > 16 || !valid_dtype(dtype) || !blocks || !coeff_out) return PTD_EINVAL;
    if (flags & ~PTD_COMPACT) return PTD_EINVAL;
    if (!aligned16(coeff_out)) return PTD_EINVAL;
    const bool compact = flags & PTD_COMPACT;
    const size_t blk = elem_bytes(dtype) << (2 * k);
    const size_t out_rows = compact ? ((size_t)1 << k) : ((size_t)1 << (k + m));
    const size_t out_bytes = out_rows * (elem_bytes(dtype) << (k + m));
    if (overlap(blocks, blk << m, coeff_out, out_bytes)) return PTD_EINVAL;
    ptd::BlockPtrs p{};
    for (int i = 0; i < (1 << m); ++i) p.p[i] = (const unsigned char*)blocks + (size_t)i * blk;
    return hip_status(ptd::launch_block_diagonal(k, m, dtype, compact, p, coeff_out, (hipStream_t)stream));
}

ptd_status ptd_direct_sum(int n, ptd_dtype dtype, unsigned flags, const void* ca, const void* cb, void* coeff_out,
                          ptd_stream stream)
{
    if (n < 1 || n + 1 > 16 || !valid_dtype(dtype) || !ca || !cb || !coeff_out) return PTD_EINVAL;
    if (flags & ~PTD_COMPACT) return PTD_EINVAL;
    if (!aligned16(coeff_out)) return PTD_EINVAL;
    const bool compact = flags & PTD_COMPACT;
    const size_t blk = elem_bytes(dtype) << (2 * n);
    const size_t out_bytes = (compact ? ((size_t)1 << n) : ((size_t)2 << n)) * (elem_bytes(dtype) << (n + 1));
    if (overlap(ca, blk, coeff_out, out_bytes) || overlap(cb, blk, coeff_out, out_bytes)) return PTD_EINVAL;
    ptd::BlockPtrs p{};
    p.p[0] = ca;
    p.p[1] = cb;
    return hip_status(ptd::launch_block_diagonal(n, 1, dtype, compact, p, coeff_out, (hipStream_t)stream));
}

ptd_status ptd_hermitian_augment(int n, ptd_dtype dtype, unsigned flags, const void* coeff, void* coeff_out,
                                 ptd_stream stream)
{
    if (n < 1 || n + 1 > 16 || !valid_dtype(dtype) || !coeff || !coeff_out) return PTD_EINVAL;
    if (flags & ~PTD_COMPACT) return PTD_EINVAL;
    if (!aligned16(coeff_out)) return PTD_EINVAL;
    const bool compact = flags & PTD_COMPACT;
    const size_t in_bytes = elem_bytes(dtype) << (2 * n);
    const size_t out_bytes = (compact ? ((size_t)1 << n) : ((size_t)2 << n)) * ((elem_bytes(dtype) / 2) << (n + 1));
    if (overlap(coeff, in_bytes, coeff_out, out_bytes)) return PTD_EINVAL;
    return hip_status(ptd::launch_hermitian_augment(n, dtype, compact, coeff, coeff_out, (hipStream_t)stream));
}

ptd_status ptd_linear_combination(int n, ptd_dtype dtype, double mu_re, double mu_im, const void* ca, const void* cb,
                                  void* c_out, ptd_stream stream)
{
    if (n < 1 || n > 16 || !valid_dtype(dtype) || !ca || !cb || !c_out) return PTD_EINVAL;
    const size_t bytes = elem_bytes(dtype) << (2 * n);
    // elementwise: c_out may be c_a or c_b, but not a shifted view of either
    if ((c_out != ca && overlap(ca, bytes, c_out, bytes)) || (c_out != cb && overlap(cb, bytes, c_out, bytes)))
        return PTD_EINVAL;
    return hip_status(ptd::launch_linear_combination(n, dtype, mu_re, mu_im, ca, cb, c_out, (hipStream_t)stream));
}

ptd_status ptd_zero_pad(ptd_dtype dtype, const void* src, int64_t ld, int64_t rows, int64_t cols, void* dst,
                        int n, ptd_stream stream)
{
    if (!valid_dtype(dtype) || !src || !dst || n < 1 || n > 16) return PTD_EINVAL;
    if (rows < 1 || cols < 1 || rows > ((int64_t)1 << n) || cols > ((int64_t)1 << n) || ld < cols) return PTD_EINVAL;
    const size_t eb = elem_bytes(dtype);
    if (overlap(src, span_bytes(rows, cols, ld, eb), dst, ((size_t)1 << (2 * n)) * eb)) return PTD_EINVAL;
    return hip_status(ptd::launch_zero_pad(dtype, src, ld, rows, cols, n, dst, (hipStream_t)stream));
}

size_t ptd_sparse_workspace_bytes(int n)
{
    if (n < 1 || n > 16) return 0;
    return ptd::sparse_workspace_bytes(n);
}

ptd_status ptd_sparse_nonempty_x(int n, int64_t nnz, const int32_t* rows, const int32_t* cols, uint32_t* xs_out,
                                 int* count_host, void* ws, size_t ws_bytes, ptd_stream stream)
{
    if (n < 1 || n > 16 || nnz < 0 || !xs_out || !count_host) return PTD_EINVAL;
    if (nnz > 0 && (!rows || !cols)) return PTD_EINVAL;
    if (!ws || ws_bytes < ptd::sparse_workspace_bytes(n)) return PTD_ENOSPC;
    return hip_status(
        ptd::launch_sparse_nonempty_x(n, nnz, rows, nullptr, cols, xs_out, count_host, ws, (hipStream_t)stream));
}

ptd_status pauli_decompose_sparse(int n, ptd_dtype dtype, unsigned flags, int64_t nnz, const int32_t* rows,
                                  const int32_t* cols, const void* vals, const uint32_t* xs, int count, void* coeff,
                                  void* ws, size_t ws_bytes, ptd_stream stream)
{
    if (n < 1 || n > 16 || !valid_dtype(dtype) || nnz < 0 || !coeff) return PTD_EINVAL;
    if (flags & ~PTD_COMPACT) return PTD_EINVAL;
    if (nnz > 0 && (!rows || !cols || !vals)) return PTD_EINVAL;
    if (count < 0 || count > (1 << n) || (count > 0 && !xs)) return PTD_EINVAL;
    if (coeff == vals) return PTD_EINVAL;
    if (!ws || ws_bytes < ptd::sparse_workspace_bytes(n)) return PTD_ENOSPC;
    bool bad = false;
    const ptd_status st = hip_status(ptd::launch_sparse(n, dtype, flags & PTD_COMPACT, nnz, rows, nullptr, cols, vals,
                                                        xs, count, coeff, ws, &bad, (hipStream_t)stream));
    if (st != PTD_OK) return st;
    return bad ? PTD_EINVAL : PTD_OK;
}

ptd_status ptd_csr_nonempty_x(int n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx, uint32_t* xs_out,
                              int* count_host, void* ws, size_t ws_bytes, ptd_stream stream)
{
    if (n < 1 || n > 16 || nnz < 0 || !xs_out || !count_host) return PTD_EINVAL;
    if (nnz > 0 && (!row_ptr || !col_idx)) return PTD_EINVAL;
    if (!ws || ws_bytes < ptd::sparse_workspace_bytes(n)) return PTD_ENOSPC;
    const size_t N = (size_t)1 << n;
    const size_t wsb = ptd::sparse_workspace_bytes(n);
    if (nnz > 0 && (overlap(ws, wsb, xs_out, std::min((size_t)nnz, N) * 4) || overlap(ws, wsb, row_ptr, (N + 1) * 8) || overlap(ws, wsb, col_idx, (size_t)nnz * 4) ||
                    overlap(xs_out, std::min((size_t)nnz, N) * 4, row_ptr, (N + 1) * 8) ||
                    overlap(xs_out, std::min((size_t)nnz, N) * 4, col_idx, (size_t)nnz * 4)))
        return PTD_EINVAL;
    return hip_status(
        ptd::launch_sparse_nonempty_x(n, nnz, nullptr, row_ptr, col_idx, xs_out, count_host, ws, (hipStream_t)stream));
}

ptd_status pauli_decompose_csr(int n, ptd_dtype dtype, unsigned flags, int64_t nnz, const int64_t* row_ptr,
                               const int32_t* col_idx, const void* vals, const uint32_t* xs, int count, void* coeff,
                               void* ws, size_t ws_bytes, ptd_stream stream)
{
    if (n < 1 || n > 16 || !valid_dtype(dtype) || nnz < 0 || !coeff) return PTD_EINVAL;
    if (flags & ~PTD_COMPACT) return PTD_EINVAL;
    if (nnz > 0 && (!row_ptr || !col_idx || !vals)) return PTD_EINVAL;
    if (count < 0 || count > (1 << n) || (count > 0 && !xs)) return PTD_EINVAL;
    if (!ws || ws_bytes < ptd::sparse_workspace_bytes(n)) return PTD_ENOSPC;
    const size_t N = (size_t)1 << n;
    const size_t eb = elem_bytes(dtype);
    const size_t out_bytes = ((flags & PTD_COMPACT) ? (size_t)count : N) * N * eb;
    const size_t wsb = ptd::sparse_workspace_bytes(n);
    // the output and the workspace are written: neither may overlap an input or each other
    const void* ins[4] = {row_ptr, col_idx, vals, xs};
    const size_t in_bytes[4] = {nnz > 0 ? (N + 1) * 8 : 0, (size_t)nnz * 4, (size_t)nnz * eb, (size_t)count * 4};
    for (int i = 0; i < 4; ++i)
        if (in_bytes[i] && (overlap(coeff, out_bytes, ins[i], in_bytes[i]) || overlap(ws, wsb, ins[i], in_bytes[i])))
            return PTD_EINVAL;
    if (overlap(coeff, out_bytes, ws, wsb)) return PTD_EINVAL;
    bool bad = false;
    const ptd_status st = hip_status(ptd::launch_sparse(n, dtype, flags & PTD_COMPACT, nnz, nullptr, row_ptr, col_idx,
                                                        vals, xs, count, coeff, ws, &bad, (hipStream_t)stream));
    if (st != PTD_OK) return st;
    return bad ? PTD_EINVAL : PTD_OK;
}

ptd_status ptd_lcu_amplitudes(int n, ptd_dtype dtype, unsigned flags, const void* coeff, void* amp_out,
                              double* lambda_host, void* ws, size_t ws_bytes, ptd_stream stream)
{
    if (n < 1 || n > 16 || !valid_dtype(dtype) || !coeff || !amp_out || !lambda_host) return PTD_EINVAL;
    if (flags & ~PTD_HERMITIAN) return PTD_EINVAL;
    if (coeff == amp_out) return PTD_EINVAL;
    if (!ws || ws_bytes < ptd::reduce_workspace_bytes()) return PTD_ENOSPC;
    return hip_status(ptd::launch_lcu_amplitudes(n, dtype, flags & PTD_HERMITIAN, coeff, amp_out, ws, lambda_host,
                                                 (hipStream_t)stream));
}

// Testing hook: force the single-pass (path 1) or two-pass (path 2) schedule.
ptd_status ptd_debug_decompose_path(int n, ptd_dtype dtype, unsigned flags, const void* A, int64_t lda,
                                    void* coeff, int path, ptd_stream stream)
{
    if (n < 1 || n > 16 || !valid_dtype(dtype) || !A || !coeff || lda < ((int64_t)1 << n)) return PTD_EINVAL;
    if (flags & ~PTD_HERMITIAN) return PTD_EINVAL;
    if (path == 1 && n > 10) return PTD_EINVAL;
    if (path == 2 && n < 7) return PTD_EINVAL;
    if (path < 0 || path > 2) return PTD_EINVAL;
    return hip_status(ptd::launch_dense_fwd(n, dtype, flags & PTD_HERMITIAN, A, lda, coeff, path,
                                            (hipStream_t)stream));
}

ptd_status ptd_debug_reconstruct_path(int n, ptd_dtype dtype, unsigned flags, const void* coeff, void* A,
                                      int64_t lda, int path, ptd_stream stream)
{
    if (n < 1 || n > 16 || !valid_dtype(dtype) || !A || !coeff || lda < ((int64_t)1 << n)) return PTD_EINVAL;
    if (flags & ~(PTD_HERMITIAN | PTD_ADJOINT)) return PTD_EINVAL;
    if (path == 1 && n > 10) return PTD_EINVAL;
    if (path == 2 && n < 7) return PTD_EINVAL;
    if (path < 0 || path > 2) return PTD_EINVAL;
    return hip_status(ptd::launch_dense_rec(n, dtype, flags & PTD_HERMITIAN, flags & PTD_ADJOINT, coeff, A, lda,
                                            path, (hipStream_t)stream));
}

// ------------------------------------------------------------------ batched

namespace {

ptd_status check_batch(int count, ptd_dtype dtype, const int32_t* n_host, const int64_t* in_off,
                       const int64_t* out_off, const void* in_base, const void* out_base)
{
    if (count < 1 || !valid_dtype(dtype) || !n_host || !in_off || !out_off || !in_base || !out_base)
        return PTD_EINVAL;
    for (int i = 0; i < count; ++i) {
        if (n_host[i] < 1 || n_host[i] > 10) return PTD_EINVAL;
        if (in_off[i] < 0 || out_off[i] < 0) return PTD_EINVAL;
    }
    if (ptd::batched_item_count(count, dtype, n_host) > (int64_t)0x7fffffff) return PTD_EINVAL;
    return PTD_OK;
}

ptd_status batched_common(bool rec, int count, ptd_dtype dtype, unsigned flags, const int32_t* n_host,
                          const int64_t* in_off, const int64_t* out_off, const void* in_base, void* out_base,
                          void* ws, size_t ws_bytes, ptd_stream stream)
{
    const ptd_status c = check_batch(count, dtype, n_host, in_off, out_off, in_base, out_base);
    if (c != PTD_OK) return c;
    const unsigned allowed = rec ? (PTD_HERMITIAN | PTD_ADJOINT) : PTD_HERMITIAN;
    if (flags & ~allowed) return PTD_EINVAL;
    if (!ws || ws_bytes < ptd::batched_buffer_bytes(count, dtype, n_host)) return PTD_ENOSPC;
    std::vector<unsigned char> img;
    ptd::BatchLaunch bl;
    ptd::batched_fill(count, dtype, flags & PTD_HERMITIAN, rec, n_host, in_off, out_off, img, &bl);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync((unsigned char*)ws + ptd::BATCH_HEAD_BYTES, img.data(), img.size(),
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // img is released on return
    if (e != hipSuccess) return hip_status(e);
    return hip_status(ptd::batched_launch(dtype, flags & PTD_HERMITIAN, rec, flags & PTD_ADJOINT, in_base, out_base,
                                          ws, count, bl, ptd::device_cu_count(), st));
}

}  // namespace

struct ptd_plan {
    void* buf = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

size_t ptd_batched_workspace_bytes(int count, ptd_dtype dtype, const int32_t* n_host)
{
    if (count < 1 || !valid_dtype(dtype) || !n_host) return 0;
    for (int i = 0; i < count; ++i)
        if (n_host[i] < 1 || n_host[i] > 10) return 0;
    return ptd::batched_buffer_bytes(count, dtype, n_host);
}

ptd_status pauli_decompose_batched(int count, ptd_dtype dtype, unsigned flags, const int32_t* n_host,
                                   const int64_t* in_off_host, const int64_t* out_off_host, const void* in_base,
                                   void* out_base, void* ws, size_t ws_bytes, ptd_stream stream)
{
    return batched_common(false, count, dtype, flags, n_host, in_off_host, out_off_host, in_base, out_base, ws,
                          ws_bytes, stream);
}

ptd_status pauli_reconstruct_batched(int count, ptd_dtype dtype, unsigned flags, const int32_t* n_host,
                                     const int64_t* in_off_host, const int64_t* out_off_host, const void* in_base,
                                     void* out_base, void* ws, size_t ws_bytes, ptd_stream stream)
{
    return batched_common(true, count, dtype, flags, n_host, in_off_host, out_off_host, in_base, out_base, ws,
                          ws_bytes, stream);
}

ptd_status ptd_batch_plan_create(int count, ptd_dtype dtype, unsigned flags, const int32_t* n_host,
                                 const int64_t* in_off_host, const int64_t* out_off_host, const void* in_base,
                                 void* out_base, ptd_plan** plan_out)
{
    if (!plan_out) return PTD_EINVAL;
    *plan_out = nullptr;
    const ptd_status c = check_batch(count, dtype, n_host, in_off_host, out_off_host, in_base, out_base);
    if (c != PTD_OK) return c;
    if (flags & ~(PTD_HERMITIAN | PTD_ADJOINT | PTD_PLAN_RECONSTRUCT)) return PTD_EINVAL;
    const bool rec = flags & PTD_PLAN_RECONSTRUCT;
    if ((flags & PTD_ADJOINT) && !rec) return PTD_EINVAL;
    std::vector<unsigned char> img;
    ptd::BatchLaunch bl;
    ptd::batched_fill(count, dtype, flags & PTD_HERMITIAN, rec, n_host, in_off_host, out_off_host, img, &bl);
    ptd_plan* p = new (std::nothrow) ptd_plan;
    if (!p) return PTD_ENOMEM;
    const size_t bytes = ptd::BATCH_HEAD_BYTES + img.size();
    if (hipMalloc(&p->buf, bytes) != hipSuccess) {
        delete p;
        return PTD_ENOMEM;
    }
    hipError_t e = hipMemcpy((unsigned char*)p->buf + ptd::BATCH_HEAD_BYTES, img.data(), img.size(), hipMemcpyHostToDevice);
    hipStream_t cs = nullptr;
    if (e == hipSuccess) e = ptd::prepare_batch_lanes();
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        // the queue counter is reset by a kernel node (no memset node in the graph)
        hipError_t le = ptd::batched_launch(dtype, flags & PTD_HERMITIAN, rec, flags & PTD_ADJOINT, in_base, out_base,
                                            p->buf, count, bl, ptd::device_cu_count(), cs, true);
        e = hipStreamEndCapture(cs, &p->graph);
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        ptd_batch_plan_destroy(p);
        return hip_status(e);
    }
    *plan_out = p;
    return PTD_OK;
}

ptd_status ptd_batch_plan_launch(ptd_plan* plan, ptd_stream stream)
{
    if (!plan || !plan->exec) return PTD_EINVAL;
    return hip_status(hipGraphLaunch(plan->exec, (hipStream_t)stream));
}

void ptd_batch_plan_destroy(ptd_plan* plan)
{
    if (!plan) return;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->buf) (void)hipFree(plan->buf);
    delete plan;
}

// ------------------------------------------------------------------ tuning

// Sizes n <= 10 tune the single-pass group plan: cfg = plan (bit 0: 1024
// threads, bit 1: radix-32 rounds, complex64 only), lookahead unused.
static bool group_tunable(int n) { return n >= 1 && n <= 10; }

ptd_status ptd_set_tuning(int n, ptd_dtype dtype, unsigned flags, int cfg, int lookahead)
{
    if (!valid_dtype(dtype) || (flags & ~PTD_HERMITIAN)) return PTD_EINVAL;
    if (group_tunable(n)) {
        if (cfg < 0 || cfg > (dtype == PTD_C64 ? 3 : 1) || lookahead < 0) return PTD_EINVAL;
        ptd::set_group_tuning(n, dtype, flags & PTD_HERMITIAN, cfg);
        return PTD_OK;
    }
    if (!use_fused(n, dtype, flags)) return PTD_EINVAL;
    if (cfg < 0 || cfg > 31 || lookahead < 1 || lookahead > 64) return PTD_EINVAL;
    // cfg 0 is the default; otherwise a shape (bits 0-1) must be named, and
    // n = 15 is built with shape 1 only
    if (cfg != 0 && ((cfg & 3) == 0 || (n == 15 && (cfg & 3) != 1))) return PTD_EINVAL;
    ptd::set_fused_tuning(n, dtype, flags & PTD_HERMITIAN, ptd::FusedTuning{cfg, lookahead});
    return PTD_OK;
}

ptd_status ptd_describe_tuning(int n, ptd_dtype dtype, unsigned flags, int cfg, int* threads, int* phase1_bits,
                               int* group_patterns)
{
    if (!valid_dtype(dtype) || (flags & ~PTD_HERMITIAN) || !threads || !phase1_bits || !group_patterns)
        return PTD_EINVAL;
    if (!ptd::describe_fused(n, dtype, flags & PTD_HERMITIAN, cfg, threads, phase1_bits, group_patterns))
        return PTD_EINVAL;
    return PTD_OK;
}

int ptd_get_tuning(int n, ptd_dtype dtype, unsigned flags, int* cfg, int* lookahead)
{
    if (!valid_dtype(dtype) || (flags & ~PTD_HERMITIAN) || !cfg || !lookahead) return PTD_EINVAL;
    if (group_tunable(n)) {
        int plan = ptd::group_default_plan(n, dtype, flags & PTD_HERMITIAN);
        const bool tuned = ptd::get_group_tuning(n, dtype, flags & PTD_HERMITIAN, &plan);
        *cfg = plan;
        *lookahead = 0;
        return tuned ? 1 : 0;
    }
    ptd::FusedTuning t = use_fused(n, dtype, flags) ? ptd::fused_default(n, dtype, flags & PTD_HERMITIAN)
                                                    : ptd::FusedTuning{0, 0};
    const bool tuned = ptd::get_fused_tuning(n, dtype, flags & PTD_HERMITIAN, &t);
    *cfg = t.cfg;
    *lookahead = t.la;
    return tuned ? 1 : 0;
}

void ptd_clear_tuning(void) { ptd::clear_fused_tuning(); }

int ptd_autotune_report(int n, ptd_dtype dtype, unsigned flags, float* default_ms, float* best_ms, float* spread_ms,
                        int* kept)
{
    if (!valid_dtype(dtype) || (flags & ~PTD_HERMITIAN) || !default_ms || !best_ms || !spread_ms || !kept)
        return PTD_EINVAL;
    return ptd::get_tune_report(n, dtype, flags & PTD_HERMITIAN, default_ms, best_ms, spread_ms, kept) ? 1 : 0;
}

ptd_status ptd_autotune(int n, ptd_dtype dtype, unsigned flags, int reps, ptd_stream stream, int* cfg, int* lookahead,
                        float* ms, int* tried, int* admitted)
{
    if (!valid_dtype(dtype) || (flags & ~PTD_HERMITIAN) || reps < 1 || !cfg || !lookahead || !ms || !tried ||
        !admitted)
        return PTD_EINVAL;
    if (n < 1 || n > 16) return PTD_EINVAL;
    if (group_tunable(n)) {
        int plan = 0;
        hipError_t e = ptd::autotune_group(n, dtype, flags & PTD_HERMITIAN, reps, (hipStream_t)stream, &plan, ms, tried,
                                           admitted);
        if (e != hipSuccess) return hip_status(e);
        *cfg = plan;
        *lookahead = 0;
        return PTD_OK;
    }
    if (!use_fused(n, dtype, flags)) return PTD_EUNSUP;
    ptd::FusedTuning best = ptd::fused_default(n, dtype, flags & PTD_HERMITIAN);
    hipError_t e = ptd::autotune_fused(n, dtype, flags & PTD_HERMITIAN, reps, (hipStream_t)stream, &best, ms, tried,
                                       admitted);
    if (e != hipSuccess) return hip_status(e);
    *cfg = best.cfg;
    *lookahead = best.la;
    return PTD_OK;
}

// Testing hook: the single-launch schedule with an explicit lookahead.
ptd_status ptd_debug_decompose_fused(int n, ptd_dtype dtype, unsigned flags, const void* A, int64_t lda, void* coeff,
                                     void* ws, size_t ws_bytes, int lookahead, int cfg, ptd_stream stream)
{
    if (n < 11 || n > 15 || !valid_dtype(dtype) || !A || !coeff || lda < ((int64_t)1 << n)) return PTD_EINVAL;
    if ((flags & ~PTD_HERMITIAN) || lookahead < 1) return PTD_EINVAL;
    if (!use_fused(n, dtype, flags)) return PTD_EUNSUP;
    if (!ws || ws_bytes < ptd::fused_workspace_bytes(n, dtype)) return PTD_ENOSPC;
    if (cfg < 0 || cfg > 31) return PTD_EINVAL;
    return hip_status(ptd::launch_fused_fwd(n, dtype, flags & PTD_HERMITIAN, A, lda, coeff, ws, lookahead, cfg,
                                            (hipStream_t)stream));
}

// Test hook: the dies workgroups run on (bit i: HW_REG_XCC_ID == i was seen)
// and the XCD count the one-launch schedules use.  Synchronises the device.
ptd_status ptd_debug_xcc_ids(unsigned* mask_host, int* count_host)
{
    if (!mask_host || !count_host) return PTD_EINVAL;
    return hip_status(ptd::probe_xcc_ids(mask_host, count_host));
}

// Test hook: while on, every bounded wait of the one-launch schedules gives
// up after a few polls (the failure path of ptd_workspace_status).
void ptd_debug_wait_test_mode(int on) { ptd::set_wait_test_mode(on != 0); }

// Bandwidth reference: a plain 16-byte-per-lane device copy of `bytes` bytes.
ptd_status ptd_debug_copy(const void* src, void* dst, size_t bytes, ptd_stream stream)
{
    if (!src || !dst || (bytes & 15)) return PTD_EINVAL;
    return hip_status(ptd::launch_copy(src, dst, bytes, (hipStream_t)stream));
}

// Bandwidth reference of one shape (probe.hip: mode, accesses per thread,
// cache hints, partition, workgroup size and count); the read-only mode
// ignores dst, the write-only mode src.
ptd_status ptd_debug_bandwidth(int variant, const void* src, void* dst, size_t bytes, ptd_stream stream)
{
    const int mode = variant & 3;
    if ((bytes & 15) || bytes == 0) return PTD_EINVAL;
    if (mode == 3) {
        // write-back probe over dst: 64 KiB per workgroup, at most 1 GiB
        if (variant != 3 || !dst || (bytes & 65535) || bytes > ((size_t)1 << 30)) return PTD_EINVAL;
        return hip_status(ptd::launch_bandwidth(variant, src, dst, bytes, (hipStream_t)stream));
    }
    if ((mode != 2 && !src) || (mode != 1 && !dst)) return PTD_EINVAL;
    if ((variant & ~0xF7F) || ((variant >> 8) & 3) == 3 || (256 << ((variant >> 8) & 3)) * (1 << ((variant >> 10) & 3)) > 2048)
        return PTD_EINVAL;
    return hip_status(ptd::launch_bandwidth(variant, src, dst, bytes, (hipStream_t)stream));
}

// Timing hook: launch one pass of the two-pass dense schedule (n >= 7).
ptd_status ptd_debug_decompose_stage(int n, ptd_dtype dtype, unsigned flags, const void* A, int64_t lda,
                                     void* coeff, int stage, ptd_stream stream)
{
    if (n < 7 || n > 16 || !valid_dtype(dtype) || !A || !coeff || lda < ((int64_t)1 << n)) return PTD_EINVAL;
    // stage bits 0..1: passes; bits 2..: chunk size in X-pattern groups (0 = whole)
    if ((flags & ~PTD_HERMITIAN) || (stage & 3) == 0 || (stage >> 2) > (1 << (n - 6))) return PTD_EINVAL;
    return hip_status(ptd::launch_dense_fwd_stage(n, dtype, flags & PTD_HERMITIAN, A, lda, coeff, stage,
                                                  (hipStream_t)stream));
}

}  // extern "C"
