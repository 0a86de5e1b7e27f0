/*
 * ptd.h -- C ABI of the MI355X (gfx950) Pauli decomposition library.
 *
 * The library computes the coefficients of a 2^n x 2^n complex matrix A in
 * the Pauli operator basis P_n = { s_{n-1} (x) ... (x) s_0 : s_q in {I,X,Y,Z} }
 * (paper, Sec. II-A, Theorem 1 and the decomposition formula):
 *
 *     c_P = 2^-n * Tr(P A),        A = sum_P c_P P.
 *
 * Conventions (the paper leaves them open):
 *   - qubit q is bit q of the row and column index, so s_{n-1} is the most
 *     significant (leftmost) Kronecker factor, as in P = s_{n-1} (x) ... (x) s_0
 *     of Sec. II-B; a label's leftmost character is qubit n-1;
 *   - a string is indexed by its X-pattern x and Z-pattern z, with
 *     (x_q, z_q) = (0,0) I, (1,0) X, (1,1) Y, (0,1) Z on qubit q; the dense
 *     coefficient array stores c[x * 2^n + z].
 *
 * Memory: A, coeff and ws are DEVICE pointers owned by the caller; the
 * library neither allocates nor frees them.  Complex data is interleaved
 * (re, im): PTD_C128 = two doubles (16 B), PTD_C64 = two floats (8 B).  A
 * dense matrix has element (r, c) at A + r*lda + c (lda in elements).
 *
 * Execution: every compute entry point validates its arguments on the host
 * BEFORE any HIP call (argument errors are returned synchronously and need
 * no GPU), then enqueues kernels on `stream` and returns without waiting.
 * Device-side failures surface as PTD_EHIP; ptd_last_hip_error() gives the
 * HIP error code.  Functions never print and never throw.  Concurrent calls
 * on different streams are safe; the batch plans below are not thread-safe
 * objects.
 */
#ifndef PTD_H
#define PTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int ptd_status;
#define PTD_OK 0
#define PTD_EINVAL (-1) /* bad argument: n out of [1,16], null pointer, lda < 2^n, bad flag mix, s < 0 ... */
#define PTD_ENOSPC (-2) /* workspace smaller than ptd_workspace_bytes() */
#define PTD_EUNSUP (-3) /* valid request this build does not support (e.g. compensated FP64) */
#define PTD_EHIP (-4)   /* HIP runtime or launch error, see ptd_last_hip_error() */
#define PTD_ENOMEM (-5) /* a batch plan could not allocate its own descriptors */

typedef enum { PTD_C128 = 0, PTD_C64 = 1 } ptd_dtype;

/* A hipStream_t; NULL means the null stream. */
typedef void *ptd_stream;

/* Flags (bitwise OR). */
/* A is Hermitian (Theorem 2: real coefficients).  The output is REAL: doubles
 * for PTD_C128, floats for PTD_C64, one per string.  The caller guarantees
 * A == A^* exactly: the dense kernels may read only one element of a
 * mirrored pair (r, c), (c, r) and take the other as its conjugate (for
 * n = 5..14 about half the matrix is read), so for a non-Hermitian A the
 * result is unspecified.  The imaginary part dropped is exactly zero in the
 * butterfly network. */
#define PTD_HERMITIAN (1u << 0)
/* A is diagonal (Sec. IV-A, diagonal matrices): only x = 0 can be nonzero. */
#define PTD_DIAGONAL (1u << 1)
/* A is banded with half-bandwidth s >= 1: a[r][c] = 0 when |r - c| > s
 * (Sec. IV-A, band-diagonal matrices; s = 1 is tridiagonal).  Only the
 * X-patterns with an in-band entry are computed (ptd_nonempty_x). */
#define PTD_BANDED (1u << 2)
/* With PTD_DIAGONAL or PTD_BANDED: A is given as row-indexed bands,
 * band[d + s][k] = A[k][k + d] for d in [-s, s] (s = 0 for diagonal), the
 * band rows lda elements apart; slots whose column falls outside [0, 2^n)
 * are ignored. */
#define PTD_BANDS_IN (1u << 3)
/* With PTD_DIAGONAL or PTD_BANDED: write only the nonempty X-patterns, as
 * rows [i][z] in ascending x order (row i belongs to the i-th entry of
 * ptd_nonempty_x).  Without it the output is the dense [x][z] array with
 * the empty rows written as zeros. */
#define PTD_COMPACT (1u << 4)
/* PTD_C64 dense only: Walsh-Hadamard butterflies with compensated (TwoSum)
 * float32 arithmetic; results are rounded to float32 at every pass
 * boundary (the two-pass schedule is used for n >= 7, so the call moves
 * twice the bytes of the default path).  PTD_EUNSUP with structure flags;
 * PTD_EUNSUP for PTD_C128. */
#define PTD_COMPENSATED (1u << 5)
/* Adjoint pairs.  pauli_reconstruct: multiply the result by 2^-n, which
 * makes the call the adjoint (vector-Jacobian product) of pauli_decompose.
 * pauli_decompose (dense input only; not with a structure, a matrix-free
 * kind or PTD_COMPENSATED): leave out the 2^-n, i.e. coeff = Tr(P A), the
 * adjoint of pauli_reconstruct.  The scale is an exact power of two either
 * way. */
#define PTD_ADJOINT (1u << 6)
/* ptd_batch_plan_create only: the plan reconstructs (coefficients -> matrices). */
#define PTD_PLAN_RECONSTRUCT (1u << 7)
/* A is anti-diagonal: a[r][c] = 0 unless r + c = 2^n - 1 (the remark after
 * the diagonal case of Sec. IV-A: I and Z give way to X and Y).  Only
 * x = 2^n - 1 can be nonzero, every string having X or Y on every qubit.
 * With PTD_BANDS_IN, A is the vector ad[k] = A[k][2^n - 1 - k]; PTD_COMPACT
 * writes the one row.  Not combined with PTD_DIAGONAL or PTD_BANDED; s is
 * ignored. */
#define PTD_ANTIDIAGONAL (1u << 8)
/* Matrix-free Toeplitz input (the paper's note that A may be evaluated from
 * a function instead of stored, Sec. V-B): A is the vector t of 2^(n+1) - 1
 * elements with A[r][c] = t[c - r + 2^n - 1] (t[0] is the bottom-left entry,
 * t[2^n - 1] the diagonal, t[2^(n+1) - 2] the top-right); lda is ignored.
 * The kernels read t (a few MiB at most, cache-resident) instead of 4^n
 * entries.  Dense decompositions only: n <= 14, or n = 15 for complex64;
 * PTD_EUNSUP beyond, and with structure flags or PTD_COMPENSATED.  With
 * PTD_HERMITIAN, t[2^n - 1 - d] = conj(t[2^n - 1 + d]). */
#define PTD_TOEPLITZ (1u << 9)
/* Matrix-free pure-state input: A is the density matrix |psi><psi| of the
 * state vector psi (2^n elements of dtype at A), A[r][c] = psi[r]
 * conj(psi[c]), formed on the fly (per entry: re = a.re b.re + a.im b.im,
 * im = a.im b.re - a.re b.im for a = psi[r], b = psi[c], no fused
 * multiply-add); lda is ignored.  The coefficients are the Pauli expectation
 * values <psi|P|psi> / 2^n, real (exactly zero imaginary parts in the complex
 * output; PTD_HERMITIAN gives the real array).  Same sizes and exclusions as
 * PTD_TOEPLITZ, with which it does not combine. */
#define PTD_PURE_STATE (1u << 10)
/* Matrix-free mixed-state input: A = U U^* for the 2^n x s factor U at A
 * (dtype elements, row-major, row pitch lda >= s elements, lda <= 2^40),
 * A[r][c] = sum_j U[r][j] conj(U[c][j]) formed on the fly with the products
 * of PTD_PURE_STATE summed over ascending j (1 <= s <= 32, PTD_EINVAL
 * otherwise).  A density matrix of rank <= s, the weights absorbed into the
 * columns: the coefficients are the Pauli expectation values
 * sum_j <u_j|P|u_j> / 2^n of the mixed state, real (PTD_HERMITIAN gives
 * the real array).  Same sizes and exclusions as PTD_TOEPLITZ; one
 * matrix-free flag per call. */
#define PTD_LOW_RANK (1u << 11)

/* Workspace (device bytes) a pauli_decompose call with these arguments
 * needs: a few KiB of queue counters for dense decompositions with
 * n = 11..15 (one persistent launch); for PTD_LOW_RANK with n >= 11 the
 * factor's transpose, s * 2^n elements of dtype (the kernels read its
 * columns contiguously); 0 otherwise.  Host-only, pure. */
size_t ptd_workspace_bytes(int n, ptd_dtype dtype, unsigned flags, int s);

/* Workspace (device bytes) a pauli_reconstruct call with these arguments
 * needs: a few KiB of queue counters for n = 11..14 (one persistent launch),
 * 0 otherwise; 0 for bad arguments.  Host-only, pure. */
size_t ptd_reconstruct_workspace_bytes(int n, ptd_dtype dtype, unsigned flags);

/* Number of X-patterns x that can carry a nonzero coefficient: 2^n for a
 * dense matrix, 1 for PTD_DIAGONAL, and for PTD_BANDED
 * 1 + sum_{h<n} min(s, 2^h) = s n - c(s), c(s) = s(floor(log2 s)+1) - 2^{floor(log2 s)+1}
 * (Sec. IV-A band-diagonal theorem: (s n - c(s)) 2^n terms at most).  x is
 * nonempty when some entry (k, k ^ x) lies in the band, i.e. x = 0 or
 * x = 2^h + y with 0 <= y < 2^h and 2^h - y <= s.  Host-only, pure; returns
 * -1 on bad arguments. */
int ptd_num_nonempty_x(int n, unsigned flags, int s);

/* Writes those X-patterns in ascending order to xs_host (host memory,
 * ptd_num_nonempty_x entries). */
ptd_status ptd_nonempty_x(int n, unsigned flags, int s, uint32_t *xs_host);

/*
 * pauli_decompose: coeff = { c_P } for the 2^n x 2^n matrix A.
 *
 *   n        number of qubits, 1..16
 *   dtype    element type of A (and of coeff unless PTD_HERMITIAN)
 *   flags    PTD_HERMITIAN | PTD_DIAGONAL | PTD_BANDED | PTD_ANTIDIAGONAL |
 *            PTD_BANDS_IN | PTD_COMPACT | PTD_COMPENSATED | PTD_ADJOINT
 *            (unscaled Tr(P A), dense input only), or one of the
 *            matrix-free kinds PTD_TOEPLITZ | PTD_PURE_STATE | PTD_LOW_RANK
 *            (with PTD_HERMITIAN at most)
 *   s        half-bandwidth for PTD_BANDED (>= 1), the factor's rank for
 *            PTD_LOW_RANK (1..32), else ignored
 *   A, lda   input matrix (or bands with PTD_BANDS_IN), lda >= 2^n elements;
 *            for a matrix-free kind its defining vector (lda ignored) or
 *            low-rank factor (lda = its row pitch)
 *   coeff    output, 4^n values (complex, or real with PTD_HERMITIAN; with
 *            PTD_COMPACT ptd_num_nonempty_x * 2^n values); must not overlap A
 *   ws       workspace of ws_bytes >= ptd_workspace_bytes(...) (may be NULL
 *            when that is 0)
 *
 * Diagonal and banded calls read only the entries inside the band.
 */
ptd_status pauli_decompose(int n, ptd_dtype dtype, unsigned flags, int s, const void *A, int64_t lda,
                           void *coeff, void *ws, size_t ws_bytes, ptd_stream stream);

/*
 * pauli_reconstruct: A = sum_P c_P P (the expansion of Sec. II-A), the
 * inverse of pauli_decompose; with PTD_ADJOINT, A = 2^-n sum_P c_P P.
 *
 *   coeff    dense [x][z] coefficients (complex of dtype; real with
 *            PTD_HERMITIAN, giving a Hermitian A)
 *   A, lda   output matrix, lda >= 2^n; all 4^n entries are written (for
 *            n = 11..14 A also holds the intermediate transform, so coeff
 *            must not overlap it)
 *   flags    PTD_HERMITIAN | PTD_ADJOINT
 *   ws       ptd_reconstruct_workspace_bytes() device bytes (NULL when 0);
 *            PTD_ENOSPC if smaller
 */
ptd_status pauli_reconstruct(int n, ptd_dtype dtype, unsigned flags, const void *coeff, void *A,
                             int64_t lda, void *ws, size_t ws_bytes, ptd_stream stream);

/*
 * ptd_workspace_status: did the last pauli_decompose / pauli_reconstruct
 * that used this workspace complete its exchange?  The one-launch schedules
 * (dense n = 11..15 decomposition, n = 11..14 reconstruction) pass partial
 * transforms between workgroups and wait for them with bounded polls.  A
 * wait that gives up (about 0.2 s, which needs another process or a device
 * fault to starve the launch) sets an error word in the workspace, and the
 * affected coefficients (or entries of A) are written as NaN, never as
 * finite wrong values.  This call copies that word to the host on `stream`
 * and synchronises the stream: PTD_OK if clear, PTD_EHIP (with
 * ptd_last_hip_error() = hipErrorLaunchTimeOut) if a wait gave up.  The
 * word is cleared by the next call that uses the workspace.  ws may be NULL
 * when ws_bytes is 0 (such calls never wait): PTD_OK.  PTD_EINVAL when
 * ws_bytes is nonzero but smaller than one workspace header (128 bytes).
 */
ptd_status ptd_workspace_status(const void *ws, size_t ws_bytes, ptd_stream stream);

/*
 * pauli_decompose_noalloc: pauli_decompose for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments and results as
 * pauli_decompose, bit for bit, without the workspace: the one-launch
 * schedule's counters live in a fixed device array of the library
 * (PTD_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends).  The
 * call allocates nothing and needs no set-up; its first call on a device
 * looks up that device's array.  Each call clears the counters it uses, but
 * all calls on one GPU share the array: calls that overlap in time on the
 * same GPU (other streams, other host threads) race and are not supported.
 * PTD_ENOSPC if the request needs more than PTD_NOALLOC_SCRATCH_BYTES:
 * the dense and structured paths never do; a PTD_LOW_RANK factor with
 * n >= 11 does when rank * 2^n elements exceed it.  A bounded wait that
 * gives up leaves NaN in the affected coefficients, as in pauli_decompose.
 */
#define PTD_NOALLOC_SCRATCH_BYTES 65536
ptd_status pauli_decompose_noalloc(int n, ptd_dtype dtype, unsigned flags, int s, const void *A, int64_t lda,
                                   void *coeff, ptd_stream stream);

/*
 * Batched decomposition: `count` matrices of uneven size in one persistent
 * launch whose workgroups take (matrix, X-pattern group) items from an
 * atomic queue, largest matrices first.  Every n_i must lie in 1..10 (one
 * group of 2^n_i rows fits a workgroup's LDS).  Matrix i is dense with
 * lda = 2^n_i at in_base + in_off_host[i] elements of dtype; its 4^n_i
 * coefficients go to out_base + out_off_host[i] elements of the output type
 * (complex of dtype, or real with PTD_HERMITIAN).  flags: PTD_HERMITIAN.
 * The descriptors are uploaded into ws with a copy that synchronises
 * `stream`; a batch plan (below) uploads them once instead.
 */
size_t ptd_batched_workspace_bytes(int count, ptd_dtype dtype, const int32_t *n_host);
ptd_status pauli_decompose_batched(int count, ptd_dtype dtype, unsigned flags, const int32_t *n_host,
                                   const int64_t *in_off_host, const int64_t *out_off_host, const void *in_base,
                                   void *out_base, void *ws, size_t ws_bytes, ptd_stream stream);
/* The batched reconstruction: coefficients at in_base + in_off_host[i]
 * (complex, or real with PTD_HERMITIAN), matrices written to out_base +
 * out_off_host[i].  flags: PTD_HERMITIAN | PTD_ADJOINT. */
ptd_status pauli_reconstruct_batched(int count, ptd_dtype dtype, unsigned flags, const int32_t *n_host,
                                     const int64_t *in_off_host, const int64_t *out_off_host, const void *in_base,
                                     void *out_base, void *ws, size_t ws_bytes, ptd_stream stream);

/*
 * Batch plan: the descriptors of one batched call uploaded once into
 * plan-owned device memory, and the launch (queue reset + persistent kernel)
 * captured in a HIP graph.  ptd_batch_plan_launch replays the graph on
 * `stream` (asynchronous).  Buffers and offsets are fixed at creation; the
 * plan allocates device memory only in create and frees it in destroy.
 * flags: PTD_HERMITIAN, PTD_ADJOINT, PTD_PLAN_RECONSTRUCT.  A plan must not
 * be launched concurrently with itself.
 */
typedef struct ptd_plan ptd_plan;
ptd_status ptd_batch_plan_create(int count, ptd_dtype dtype, unsigned flags, const int32_t *n_host,
                                 const int64_t *in_off_host, const int64_t *out_off_host, const void *in_base,
                                 void *out_base, ptd_plan **plan_out);
ptd_status ptd_batch_plan_launch(ptd_plan *plan, ptd_stream stream);
void ptd_batch_plan_destroy(ptd_plan *plan);

/*
 * Sparse input.  The argument of Sec. IV-A for diagonal and band matrices
 * holds for any sparsity pattern: the strings with X-pattern x read only the
 * entries (k, k ^ x), so only the x = r ^ c of nonzero entries (r, c) can
 * carry a coefficient.  The matrix is given as nnz coordinate entries in
 * device memory: rows[i], cols[i] (int32) and vals[i] (complex of dtype);
 * repeated coordinates are summed, entries outside [0, 2^n) ignored.
 *
 * ptd_sparse_nonempty_x writes those X-patterns, ascending, to the device
 * array xs_out (room for min(nnz, 2^n) entries) and their number to
 * *count_host; it synchronises `stream`.
 *
 * pauli_decompose_sparse computes the coefficients of the listed X-patterns
 * xs[0..count) (device array, strictly ascending in [0, 2^n), as
 * ptd_sparse_nonempty_x gives them; else PTD_EINVAL after a device-side check
 * that synchronises `stream` once): the entries are added into their zeroed
 * output rows, then transformed in place.  Output: the dense 2^n x 2^n
 * coefficient array (rows not listed are zero), or with PTD_COMPACT the
 * count x 2^n rows of the listed X-patterns.  Entries whose X-pattern is
 * not listed are ignored.  flags: 0 or PTD_COMPACT.  ws holds
 * ptd_sparse_workspace_bytes(n) bytes (both calls).
 */
size_t ptd_sparse_workspace_bytes(int n);
ptd_status ptd_sparse_nonempty_x(int n, int64_t nnz, const int32_t *rows, const int32_t *cols, uint32_t *xs_out,
                                 int *count_host, void *ws, size_t ws_bytes, ptd_stream stream);
ptd_status pauli_decompose_sparse(int n, ptd_dtype dtype, unsigned flags, int64_t nnz, const int32_t *rows,
                                  const int32_t *cols, const void *vals, const uint32_t *xs, int count, void *coeff,
                                  void *ws, size_t ws_bytes, ptd_stream stream);

/*
 * Sparse input in compressed-row (CSR) form: the same argument (Sec. IV-A
 * for any pattern) and the same two calls as for coordinate entries, with
 * row_ptr in place of rows.  Device arrays: row_ptr holds 2^n + 1 int64
 * values, col_idx nnz int32 columns, vals nnz complex values of dtype.  Row
 * r holds the entries row_ptr[r] .. row_ptr[r + 1] - 1, each range clipped
 * to [0, nnz) (its end raised to its start where it lies below it), so no
 * read leaves the arrays whatever row_ptr holds; a column repeated within a
 * row is summed, columns outside [0, 2^n) are ignored.  row_ptr, col_idx
 * and vals may be null only when nnz == 0.
 *
 * ptd_csr_nonempty_x: the X-patterns of the entries, ascending, into xs_out
 * (room for min(nnz, 2^n)), their number into *count_host; synchronises
 * `stream`.  pauli_decompose_csr: the coefficients of the listed X-patterns,
 * with the list check, flags and output of pauli_decompose_sparse.  ws holds
 * ptd_sparse_workspace_bytes(n) bytes.  PTD_EINVAL also when the output or
 * the workspace overlaps an input array or each other.
 */
ptd_status ptd_csr_nonempty_x(int n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx, uint32_t *xs_out,
                              int *count_host, void *ws, size_t ws_bytes, ptd_stream stream);
ptd_status pauli_decompose_csr(int n, ptd_dtype dtype, unsigned flags, int64_t nnz, const int64_t *row_ptr,
                               const int32_t *col_idx, const void *vals, const uint32_t *xs, int count, void *coeff,
                               void *ws, size_t ws_bytes, ptd_stream stream);

/*
 * Combinations of decompositions (Sec. IV-B, "Combinations of matrices"):
 * the coefficients of a matrix assembled from matrices whose coefficients
 * are known, computed from those coefficients alone, with no matrix formed
 * and nothing decomposed again.  Coefficient arrays are dense, c[x * 2^n +
 * z] as pauli_decompose writes them, in caller-owned device memory; each
 * call is one pass over its inputs and outputs on `stream`.  Outputs must
 * not overlap inputs (PTD_EINVAL), except as stated for the linear
 * combination.  Arrays are aligned to their element size, and the outputs
 * of the first three calls to 16 bytes (PTD_EINVAL otherwise: their zero
 * rows are written 16 bytes per lane).  flags: 0, or PTD_COMPACT where
 * stated.
 *
 * ptd_block_diagonal: diag(A_0, ..., A_{2^m - 1}) on k + m qubits from the
 * coefficients of its 2^m diagonal blocks A_i on k qubits (Sec. IV-B
 * "Block-diagonal matrices"; the direct sum is m = 1).  Block i's array is at
 * blocks + i * 4^k elements of dtype.  The new top m qubits carry I or Z
 * only:
 *     c'[x][(t << k) | z] = 2^-m sum_i (-1)^popcount(t & i) c_i[x][z]
 * for x, z < 2^k and t < 2^m (the paper's pairwise direct sums, unrolled; the
 * pairs of the lowest block bit are combined first); rows x' >= 2^k are zero.
 * The output is 2^(k+m) x 2^(k+m) complex of dtype with those rows written as
 * zeros, or with PTD_COMPACT only its first 2^k rows (2^k x 2^(k+m)).
 * k >= 1, 1 <= m <= 5, k + m <= 16.
 */
ptd_status ptd_block_diagonal(int k, int m, ptd_dtype dtype, unsigned flags, const void *blocks, void *coeff_out,
                              ptd_stream stream);
/*
 * Direct sum A (+) B on n + 1 qubits (Sec. IV-B "Direct sum"): the m = 1 case
 * of ptd_block_diagonal with the two arrays at separate addresses: the top
 * qubit's I carries (c_A + c_B) / 2 and its Z carries (c_A - c_B) / 2.
 * flags: PTD_COMPACT as above.  n >= 1, n + 1 <= 16.
 */
ptd_status ptd_direct_sum(int n, ptd_dtype dtype, unsigned flags, const void *ca, const void *cb, void *coeff_out,
                          ptd_stream stream);
/*
 * Hermitian augmentation [[0, A^H], [A, 0]] on n + 1 qubits (Sec. IV-B
 * "Hermitian matrix augmentation"): X on the new top qubit carries Re c and
 * Y carries Im c, so the coefficients are real (float64 for PTD_C128, float32
 * for PTD_C64):
 *     c'[2^n + x][z] = Re c[x][z],   c'[2^n + x][2^n + z] = Im c[x][z];
 * rows x' < 2^n are zero.  The output is 2^(n+1) x 2^(n+1) reals with those
 * rows written as zeros, or with PTD_COMPACT the 2^n x 2^(n+1) rows x' >= 2^n
 * only (output row x holds row 2^n + x).  n >= 1, n + 1 <= 16.
 */
ptd_status ptd_hermitian_augment(int n, ptd_dtype dtype, unsigned flags, const void *coeff, void *coeff_out,
                                 ptd_stream stream);
/*
 * Linear combination mu A + B (Sec. IV-B "Linear combination"): c_out =
 * mu c_A + c_B elementwise over the 4^n coefficients, mu = mu_re + i mu_im
 * (rounded to float32 for PTD_C64).  Per element, without fused
 * multiply-adds: re = (mu_re a_re - mu_im a_im) + b_re, im = (mu_re a_im +
 * mu_im a_re) + b_im.  c_out may be c_a or c_b itself (not a shifted view).
 * 1 <= n <= 16.
 */
ptd_status ptd_linear_combination(int n, ptd_dtype dtype, double mu_re, double mu_im, const void *ca, const void *cb,
                                  void *c_out, ptd_stream stream);

/*
 * State preparation for a block-encoding by a linear combination of the
 * Pauli strings (Sec. VI-C, "Block-encoding using Pauli decomposition"): the
 * ancilla state sum_i sqrt(|alpha_i|) |i> / sqrt(sum_j |alpha_j|), one real
 * amplitude per coefficient of the dense array coeff (zero coefficients get
 * amplitude zero; the phase of alpha_i is carried by the controlled string,
 * as the paper absorbs signs into V_i).  amp_out[P] = sqrt(|c_P| / lambda)
 * with lambda = sum_P |c_P| (|c| = sqrt(re^2 + im^2)), all in float64 and
 * rounded once to the output type (float64 for PTD_C128, float32 for
 * PTD_C64); lambda, the block-encoding's normalisation, is written to
 * *lambda_host.  flags: PTD_HERMITIAN means coeff is real.  ws holds
 * ptd_reduce_workspace_bytes() bytes; the call synchronises `stream`.
 */
ptd_status ptd_lcu_amplitudes(int n, ptd_dtype dtype, unsigned flags, const void *coeff, void *amp_out,
                              double *lambda_host, void *ws, size_t ws_bytes, ptd_stream stream);

/*
 * Parseval check (Theorem 1: the strings are orthogonal with Tr(P^* P) = 2^n,
 * so ||A||_F^2 = 2^n sum_P |c_P|^2).  Reduces both sides in float64 on the
 * device (also for PTD_C64 data) and copies them to out_host[0] =
 * ||A||_F^2, out_host[1] = 2^n sum |c|^2, out_host[2] = |out[0] - out[1]| /
 * out[0].  flags: PTD_HERMITIAN means coeff is real.  Synchronises `stream`.
 * ws must hold ptd_reduce_workspace_bytes() bytes.
 */
size_t ptd_reduce_workspace_bytes(void);
ptd_status ptd_parseval_residual(int n, ptd_dtype dtype, unsigned flags, const void *A, int64_t lda,
                                 const void *coeff, double *out_host, void *ws, size_t ws_bytes,
                                 ptd_stream stream);

/*
 * Autotuning of the dense schedules (flags 0 or PTD_HERMITIAN).
 *
 * n = 1..10, the single-pass group kernel (single calls and batched
 * launches): cfg is the plan, bit 0 = 1024 threads per workgroup (else 512),
 * bit 1 = radix-32 WHT rounds (complex64 only; else radix 16); lookahead is
 * unused (0).  ptd_autotune times the plans on a batch of equal-size
 * matrices through the batched kernel.  In a batch, matrices of n <= 7
 * share one launch that runs a fixed plan, so for those sizes the plan
 * reaches single calls only (and the tuner times plan 0 alone).  Every plan
 * gives the same bits.
 *
 * n = 11..15, the single-launch schedule (complex128 for n <= 14): cfg & 3
 * is the shape, which fixes the tile and the stage split: 1 = 1024-thread
 * workgroups, 10 low WHT stages per phase-1 item (n - 10 in phase 2), a
 * group of X-patterns filling a 128-byte row segment (T = 16 complex64 or 8
 * complex128); 2 = 512 threads, 9 low stages, the same T; 3 = 512 threads,
 * 10 low stages, half that T (64-byte segments, half the partial band in
 * flight); shapes 2 and 3 exist for n <= 14.  cfg bits 2..4 are the cache
 * policies (non-temporal gathers of A, final stores, phase-2 loads of the
 * partial results); lookahead is the queue lookahead (1..64).
 * ptd_describe_tuning decodes a setting into these terms.
 *
 * ptd_autotune times the candidate settings at this (n, dtype, Hermitian)
 * point on device buffers it allocates itself, admits a candidate only if
 * its output on a Gaussian-integer matrix equals the default setting's bit
 * for bit, records the fastest in a process-wide registry that
 * pauli_decompose uses from then on, and returns it with its mean time over
 * `reps` launches.  Synchronises `stream`.  ptd_set_tuning records a setting
 * directly (e.g. one loaded from a cache file); ptd_get_tuning returns 1 and
 * the tuned setting, or 0 and the default; ptd_clear_tuning forgets all.
 */
ptd_status ptd_autotune(int n, ptd_dtype dtype, unsigned flags, int reps, ptd_stream stream, int *cfg,
                        int *lookahead, float *ms, int *tried, int *admitted);

/* The last ptd_autotune of (n, dtype, flags & PTD_HERMITIAN) on this
 * process: the default setting's median time per call, the chosen
 * setting's, and the run-to-run spread that decided (every candidate and the
 * default are timed in 5 rounds; a setting other than the default is kept
 * only if its median beats the default's by more than the larger spread of
 * the two; *kept = 1 then).  Returns 1 if such a tuning exists, 0 if not,
 * PTD_EINVAL on a bad argument.  Host-only. */
int ptd_autotune_report(int n, ptd_dtype dtype, unsigned flags, float *default_ms, float *best_ms, float *spread_ms,
                        int *kept);
/* The single-launch schedule's reading of setting cfg (0 = the default) at
 * (n, dtype, flags & PTD_HERMITIAN), n = 11..15: workgroup threads, the low
 * WHT stages a phase-1 item applies (the other n - phase1_bits run in phase
 * 2) and the X-patterns per group (T).  PTD_EINVAL for a setting the
 * schedule does not build there.  Host-only. */
ptd_status ptd_describe_tuning(int n, ptd_dtype dtype, unsigned flags, int cfg, int *threads, int *phase1_bits,
                               int *group_patterns);
ptd_status ptd_set_tuning(int n, ptd_dtype dtype, unsigned flags, int cfg, int lookahead);
int ptd_get_tuning(int n, ptd_dtype dtype, unsigned flags, int *cfg, int *lookahead);
void ptd_clear_tuning(void);

/*
 * The paper's own method on the host's cores, as a baseline beside the
 * device path (no HIP call; no other entry point uses it): the Pauli tree
 * walk of Sec. III-A (Algorithms 1-4: arrays k, m updated child by child in
 * the order I, X, Y, Z, one trace per leaf) and the forest of Sec. V-B that
 * cuts every branch at depth `split` into independent trees run by
 * `threads` host threads (0 = one per hardware thread).  With PTD_DIAGONAL
 * only I and Z children are visited and only m is kept (Sec. IV-A); flags
 * otherwise 0.
 *
 * A: host complex128 matrix (interleaved re, im), row-major, row pitch lda
 * >= 2^n elements; n = 1..16.  coeff_out: host complex128 array of 2^n x
 * 2^n, c[x][z] as for pauli_decompose; only the strings of trees
 * [tree_begin, tree_end) are written (the x = 0 row's strings with
 * PTD_DIAGONAL), everything else is left as it was.  The forest has 4^split
 * trees (2^split with PTD_DIAGONAL), 0 <= split <= n, numbered in the order
 * the single walk reaches their roots.  Every coefficient is summed in the
 * same order whatever the split, the range and the thread count, so results
 * agree bit for bit.  *ops_out (if not null) receives the elementary
 * operations of the updates, counted as Sec. III-B and IV-A count them:
 * 9/7 + 5/7 8^n for split 0, 4/3 + 2/3 4^n with PTD_DIAGONAL; each tree of
 * a forest adds the replay of its path.  Blocks the calling thread.
 * PTD_EINVAL on a bad argument, PTD_ENOMEM if a worker cannot allocate its
 * arrays (its trees may then be missing).
 */
ptd_status ptd_host_tree_decompose(int n, unsigned flags, const void *A, int64_t lda, void *coeff_out, int split,
                                   int64_t tree_begin, int64_t tree_end, int threads, uint64_t *ops_out);

/*
 * ptd_zero_pad: the zero padding of a matrix whose size is not a power of
 * two (the decomposition formula of Sec. II-A needs 2^n x 2^n; the paper
 * pads with zeros without fixing where the matrix goes).  dst (2^n x 2^n,
 * contiguous, dtype elements) receives src (rows x cols, row pitch ld >=
 * cols) in its top-left corner and zeros elsewhere; 1 <= rows, cols <= 2^n.
 * Both device memory, disjoint (PTD_EINVAL otherwise).  Asynchronous on
 * `stream`.
 */
ptd_status ptd_zero_pad(ptd_dtype dtype, const void *src, int64_t ld, int64_t rows, int64_t cols, void *dst, int n,
                        ptd_stream stream);

/* Human-readable name of a status code (static string). */
const char *ptd_status_str(ptd_status st);
/* HIP error code of the most recent PTD_EHIP on this thread (0 if none). */
int ptd_last_hip_error(void);
/* gfx architecture the library was built for, e.g. "gfx950". */
const char *ptd_build_arch(void);

#ifdef __cplusplus
}
#endif

#endif /* PTD_H */
