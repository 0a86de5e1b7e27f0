/*
 * oracle.c -- slow, plain CPU oracle for the Pauli decomposition.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it (through oracle/oracle.py).  It
 * shares no code, header or table with the GPU path.
 *
 * What it computes (paper, Sec. II-A, "Decomposition in the Pauli operator
 * basis"): for every Pauli operator P = s_{n-1} (x) ... (x) s_0 the
 * coefficient
 *
 *        c_P = 2^-n * Tr(P . A)
 *
 * of a 2^n x 2^n complex matrix A.  The trace is evaluated with the paper's
 * "first optimization of the trace computation" (Sec. II-A): P has exactly
 * one nonzero per row, so Tr(P.A) = sum_j P[j][k[j]] * A[k[j]][j], which is
 * the sum in Algorithm 2 (compute_coeff) read as A[k[j]][j] (row k[j],
 * column j).  The sparse form (k, m) of P is built from the 2x2 letter
 * matrices of Sec. I with the PauliComposer iteration of Sec. II-B:
 *
 *   k[0]     = binary number d(s_{n-1}) ... d(s_0)
 *   m[0]     = product over qubits of s_q[0][d(s_q)]   (the Y factors carry -i)
 *   k[j+2^l] = k[j] + (-1)^{d(s_l)} 2^l               for j < 2^l
 *   m[j+2^l] = zeta_l * m[j],  zeta_l = +1 for I, X and -1 for Y, Z
 *
 * m holds the complete entry of P (the -i of every Y is in m[0]), so no
 * separate (-i)^{n_Y} factor is applied afterwards.  A second builder,
 * oracle_pauli_sparse_kron, takes every entry straight from the Kronecker
 * product definition; the tests check that the two builders agree.
 *
 * Conventions (readings of the paper that it leaves open):
 *   - qubit q is bit q of the row / column index, so s_{n-1} is the most
 *     significant factor (Sec. II-B writes P = s_{n-1} (x) ... (x) s_0 and
 *     k[0] as the binary number d(s_{n-1})...d(s_0));
 *   - the output is a dense array indexed by (x, z): coefficient of the
 *     string with letter (x_q, z_q) = (0,0) I, (1,0) X, (1,1) Y, (0,1) Z on
 *     qubit q is stored at out[x * 2^n + z].
 *
 * Matrices are row-major N x N with interleaved (re, im) pairs; element
 * (r, c) is at index 2*(r*N + c).  Accumulation is in double precision; the
 * integer entry points accumulate Gaussian integers exactly in int64 and
 * return 2^n * c_P.
 *
 * Threads split the work over the X-pattern (the d-bits of the string),
 * like the forest split of the paper's multi-threaded code (Sec. V-B).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

enum { L_I = 0, L_X = 1, L_Y = 2, L_Z = 3 };

/* The four 2x2 Pauli matrices of Sec. I as (re, im) integer entries:
 * PAULI[letter][row][col][0 = re, 1 = im]. */
static const int PAULI[4][2][2][2] = {
    /* I */ {{{1, 0}, {0, 0}}, {{0, 0}, {1, 0}}},
    /* X */ {{{0, 0}, {1, 0}}, {{1, 0}, {0, 0}}},
    /* Y */ {{{0, 0}, {0, -1}}, {{0, 1}, {0, 0}}},
    /* Z */ {{{1, 0}, {0, 0}}, {{0, 0}, {-1, 0}}},
};

/* Diagonality function d of Sec. II-B: 0 for I, Z and 1 for X, Y. */
static int diag_d(int letter) { return (letter == L_X || letter == L_Y) ? 1 : 0; }

/* Letter of qubit q for the string stored at index (x, z). */
static int letter_of(uint64_t x, uint64_t z, int q)
{
    int xb = (int)((x >> q) & 1u), zb = (int)((z >> q) & 1u);
    if (!xb && !zb) return L_I;
    if (xb && !zb) return L_X;
    if (xb && zb) return L_Y;
    return L_Z;
}

/* Complex product of two small Gaussian integers. */
static void cmul_i(int ar, int ai, int br, int bi, int *cr, int *ci)
{
    *cr = ar * br - ai * bi;
    *ci = ar * bi + ai * br;
}

/*
 * Sparse form of P = s_{n-1} (x) ... (x) s_0 by the PauliComposer iteration
 * (Sec. II-B).  letters[q] is s_q.  col has 2^n entries; mre/mim hold m[j]
 * (entries of P are 1, -1, i or -i).
 */
void oracle_pauli_sparse(int n, const uint8_t *letters, uint64_t *col, int8_t *mre, int8_t *mim)
{
    uint64_t k0 = 0;
    int vr = 1, vi = 0;
    for (int q = n - 1; q >= 0; --q) {
        int d = diag_d(letters[q]);
        k0 = (k0 << 1) | (uint64_t)d;
        /* s_q[0][d(s_q)] is the nonzero of row 0 of that letter */
        int er = PAULI[letters[q]][0][d][0], ei = PAULI[letters[q]][0][d][1];
        cmul_i(vr, vi, er, ei, &vr, &vi);
    }
    col[0] = k0;
    mre[0] = (int8_t)vr;
    mim[0] = (int8_t)vi;
    for (int l = 0; l < n; ++l) {
        uint64_t h = (uint64_t)1 << l;
        int d = diag_d(letters[l]);
        int zeta = (letters[l] == L_I || letters[l] == L_X) ? 1 : -1;
        for (uint64_t j = 0; j < h; ++j) {
            col[j + h] = d ? col[j] - h : col[j] + h;
            mre[j + h] = (int8_t)(zeta * mre[j]);
            mim[j + h] = (int8_t)(zeta * mim[j]);
        }
    }
}

/*
 * The same sparse form taken entry by entry from the Kronecker product
 * definition: (s_{n-1} (x) ... (x) s_0)[j][c] = prod_q s_q[j_q][c_q].  Row j's
 * single nonzero sits where every factor's row j_q has its nonzero.
 */
void oracle_pauli_sparse_kron(int n, const uint8_t *letters, uint64_t *col, int8_t *mre, int8_t *mim)
{
    uint64_t N = (uint64_t)1 << n;
    for (uint64_t j = 0; j < N; ++j) {
        uint64_t c = 0;
        int vr = 1, vi = 0;
        for (int q = 0; q < n; ++q) {
            int jq = (int)((j >> q) & 1u);
            int cq = -1;
            for (int t = 0; t < 2; ++t)
                if (PAULI[letters[q]][jq][t][0] != 0 || PAULI[letters[q]][jq][t][1] != 0) cq = t;
            c |= (uint64_t)cq << q;
            cmul_i(vr, vi, PAULI[letters[q]][jq][cq][0], PAULI[letters[q]][jq][cq][1], &vr, &vi);
        }
        col[j] = c;
        mre[j] = (int8_t)vr;
        mim[j] = (int8_t)vi;
    }
}

/* ------------------------------------------------------------------------ */
/* Work split over X-patterns.                                               */

typedef struct {
    int n;
    int mode;            /* 0: double, 1: int64 */
    const double *Ad;    /* interleaved complex, N x N */
    const int64_t *Ai;
    double *outd;        /* interleaved complex, [x][z] */
    int64_t *outi;
    /* sampled mode: list of (x, z) */
    int64_t count;
    const uint32_t *xs, *zs;
    const uint64_t *keys; /* (x << 40) | sample index, sorted */
    const uint32_t *rows; /* row mode: the X-patterns to evaluate */
    int nthreads, tid;
} job_t;

/* Tr(P.A) = sum_j m[j] * A[k[j]][j] (Algorithm 2), accumulated in double.
 * The column walk A[k[j]][j] of one X-pattern is copied into a contiguous
 * buffer first: it depends only on the d-bits of the string, because k[j]
 * does. */
static void trace_d_hoisted(int n, const double *walk, const int8_t *mre, const int8_t *mim,
                            double *re, double *im)
{
    uint64_t N = (uint64_t)1 << n;
    double sr = 0.0, si = 0.0;
    for (uint64_t j = 0; j < N; ++j) {
        double ar = walk[2 * j], ai = walk[2 * j + 1];
        sr += mre[j] * ar - mim[j] * ai;
        si += mre[j] * ai + mim[j] * ar;
    }
    *re = sr;
    *im = si;
}

static void trace_i_hoisted(int n, const int64_t *walk, const int8_t *mre, const int8_t *mim,
                            int64_t *re, int64_t *im)
{
    uint64_t N = (uint64_t)1 << n;
    int64_t sr = 0, si = 0;
    for (uint64_t j = 0; j < N; ++j) {
        int64_t ar = walk[2 * j], ai = walk[2 * j + 1];
        sr += mre[j] * ar - mim[j] * ai;
        si += mre[j] * ai + mim[j] * ar;
    }
    *re = sr;
    *im = si;
}

static void letters_of(int n, uint64_t x, uint64_t z, uint8_t *letters)
{
    for (int q = 0; q < n; ++q) letters[q] = (uint8_t)letter_of(x, z, q);
}

static void *full_worker(void *arg)
{
    job_t *jb = (job_t *)arg;
    int n = jb->n;
    uint64_t N = (uint64_t)1 << n;
    uint64_t *col = malloc(N * sizeof(uint64_t));
    int8_t *mre = malloc(N), *mim = malloc(N);
    void *walk = malloc(N * 2 * sizeof(double));
    uint8_t letters[64];
    double scale = 1.0;
    for (int q = 0; q < n; ++q) scale *= 0.5;
    for (uint64_t x = (uint64_t)jb->tid; x < N; x += (uint64_t)jb->nthreads) {
        /* every string with this X-pattern reads the same column walk */
        letters_of(n, x, 0, letters);
        oracle_pauli_sparse(n, letters, col, mre, mim);
        if (jb->mode == 0) {
            double *w = (double *)walk;
            for (uint64_t j = 0; j < N; ++j) {
                w[2 * j] = jb->Ad[2 * (col[j] * N + j)];
                w[2 * j + 1] = jb->Ad[2 * (col[j] * N + j) + 1];
            }
        } else {
            int64_t *w = (int64_t *)walk;
            for (uint64_t j = 0; j < N; ++j) {
                w[2 * j] = jb->Ai[2 * (col[j] * N + j)];
                w[2 * j + 1] = jb->Ai[2 * (col[j] * N + j) + 1];
            }
        }
        for (uint64_t z = 0; z < N; ++z) {
            letters_of(n, x, z, letters);
            oracle_pauli_sparse(n, letters, col, mre, mim);
            if (jb->mode == 0) {
                double re, im;
                trace_d_hoisted(n, (const double *)walk, mre, mim, &re, &im);
                jb->outd[2 * (x * N + z)] = re * scale;
                jb->outd[2 * (x * N + z) + 1] = im * scale;
            } else {
                int64_t re, im;
                trace_i_hoisted(n, (const int64_t *)walk, mre, mim, &re, &im);
                jb->outi[2 * (x * N + z)] = re;
                jb->outi[2 * (x * N + z) + 1] = im;
            }
        }
    }
    free(col);
    free(mre);
    free(mim);
    free(walk);
    return NULL;
}

/* Sampled strings, grouped by X-pattern: every thread takes whole runs of
 * equal x from the sorted key list, builds the column walk of that x once and
 * evaluates each of its strings from it. */
static void *sample_worker(void *arg)
{
    job_t *jb = (job_t *)arg;
    int n = jb->n;
    uint64_t N = (uint64_t)1 << n;
    uint64_t *col = malloc(N * sizeof(uint64_t));
    int8_t *mre = malloc(N), *mim = malloc(N);
    double *walk = malloc(N * 2 * sizeof(double));
    uint8_t letters[64];
    double scale = 1.0;
    for (int q = 0; q < n; ++q) scale *= 0.5;
    const uint64_t *keys = jb->keys;
    int64_t run = 0;
    for (int64_t i = 0; i < jb->count;) {
        uint64_t x = keys[i] >> 40;
        int64_t e = i;
        while (e < jb->count && (keys[e] >> 40) == x) ++e;
        if (run % jb->nthreads == jb->tid) {
            letters_of(n, x, 0, letters);
            oracle_pauli_sparse(n, letters, col, mre, mim);
            for (uint64_t j = 0; j < N; ++j) {
                walk[2 * j] = jb->Ad[2 * (col[j] * N + j)];
                walk[2 * j + 1] = jb->Ad[2 * (col[j] * N + j) + 1];
            }
            for (int64_t s = i; s < e; ++s) {
                int64_t idx = (int64_t)(keys[s] & (((uint64_t)1 << 40) - 1));
                letters_of(n, jb->xs[idx], jb->zs[idx], letters);
                oracle_pauli_sparse(n, letters, col, mre, mim);
                double re, im;
                trace_d_hoisted(n, walk, mre, mim, &re, &im);
                jb->outd[2 * idx] = re * scale;
                jb->outd[2 * idx + 1] = im * scale;
            }
        }
        ++run;
        i = e;
    }
    free(col);
    free(mre);
    free(mim);
    free(walk);
    return NULL;
}

/* Whole rows: every string of each listed X-pattern, out[i][z]. */
static void *rows_worker(void *arg)
{
    job_t *jb = (job_t *)arg;
    int n = jb->n;
    uint64_t N = (uint64_t)1 << n;
    uint64_t *col = malloc(N * sizeof(uint64_t));
    int8_t *mre = malloc(N), *mim = malloc(N);
    double *walk = malloc(N * 2 * sizeof(double));
    uint8_t letters[64];
    double scale = 1.0;
    for (int q = 0; q < n; ++q) scale *= 0.5;
    for (int64_t i = jb->tid; i < jb->count; i += jb->nthreads) {
        uint64_t x = jb->rows[i];
        letters_of(n, x, 0, letters);
        oracle_pauli_sparse(n, letters, col, mre, mim);
        for (uint64_t j = 0; j < N; ++j) {
            walk[2 * j] = jb->Ad[2 * (col[j] * N + j)];
            walk[2 * j + 1] = jb->Ad[2 * (col[j] * N + j) + 1];
        }
        for (uint64_t z = 0; z < N; ++z) {
            letters_of(n, x, z, letters);
            oracle_pauli_sparse(n, letters, col, mre, mim);
            double re, im;
            trace_d_hoisted(n, walk, mre, mim, &re, &im);
            jb->outd[2 * ((uint64_t)i * N + z)] = re * scale;
            jb->outd[2 * ((uint64_t)i * N + z) + 1] = im * scale;
        }
    }
    free(col);
    free(mre);
    free(mim);
    free(walk);
    return NULL;
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

static int run_threads(job_t *tmpl, int nthreads, void *(*fn)(void *))
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    job_t jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *tmpl;
        jobs[t].nthreads = nthreads;
        jobs[t].tid = t;
        if (pthread_create(&th[t], NULL, fn, &jobs[t]) != 0) return -1;
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    return 0;
}

/* All 4^n coefficients, double accumulation.  out has 2 * 4^n doubles. */
int oracle_decompose_f64(int n, const double *A, double *out, int nthreads)
{
    if (n < 1 || n > 20 || !A || !out) return -1;
    job_t jb;
    memset(&jb, 0, sizeof jb);
    jb.n = n;
    jb.mode = 0;
    jb.Ad = A;
    jb.outd = out;
    return run_threads(&jb, nthreads, full_worker);
}

/* All 4^n values 2^n * c_P exactly, for Gaussian-integer A (int64 pairs). */
int oracle_decompose_i64(int n, const int64_t *A, int64_t *out, int nthreads)
{
    if (n < 1 || n > 20 || !A || !out) return -1;
    job_t jb;
    memset(&jb, 0, sizeof jb);
    jb.n = n;
    jb.mode = 1;
    jb.Ai = A;
    jb.outi = out;
    return run_threads(&jb, nthreads, full_worker);
}

/* Selected coefficients: out[2i], out[2i+1] = c of the string (xs[i], zs[i]). */
int oracle_coeffs_f64(int n, const double *A, int64_t count, const uint32_t *xs,
                      const uint32_t *zs, double *out, int nthreads)
{
    if (n < 1 || n > 20 || !A || !out || count < 0 || (count > 0 && (!xs || !zs))) return -1;
    job_t jb;
    memset(&jb, 0, sizeof jb);
    jb.n = n;
    jb.Ad = A;
    jb.outd = out;
    jb.count = count;
    jb.xs = xs;
    jb.zs = zs;
    if (count == 0) return 0;
    if (count >= ((int64_t)1 << 40)) return -1;
    uint64_t N = (uint64_t)1 << n;
    uint64_t *keys = malloc((size_t)count * sizeof(uint64_t));
    if (!keys) return -1;
    for (int64_t i = 0; i < count; ++i) {
        if (xs[i] >= N || zs[i] >= N) {
            free(keys);
            return -1;
        }
        keys[i] = ((uint64_t)xs[i] << 40) | (uint64_t)i;
    }
    qsort(keys, (size_t)count, sizeof(uint64_t), cmp_u64);
    jb.keys = keys;
    int rc = run_threads(&jb, nthreads, sample_worker);
    free(keys);
    return rc;
}

/*
 * Reconstruction A = sum_P c_P P (the expansion of Sec. II-A) from the dense
 * [x][z] coefficient array: every string adds c_P * m[j] at (j, k[j]).
 * Single-threaded; meant for small n.
 */
int oracle_reconstruct_f64(int n, const double *coeff, double *A)
{
    if (n < 1 || n > 14 || !coeff || !A) return -1;
    uint64_t N = (uint64_t)1 << n;
    uint64_t *col = malloc(N * sizeof(uint64_t));
    int8_t *mre = malloc(N), *mim = malloc(N);
    uint8_t letters[64];
    memset(A, 0, (size_t)(N * N * 2) * sizeof(double));
    for (uint64_t x = 0; x < N; ++x)
        for (uint64_t z = 0; z < N; ++z) {
            double cr = coeff[2 * (x * N + z)], ci = coeff[2 * (x * N + z) + 1];
            letters_of(n, x, z, letters);
            oracle_pauli_sparse(n, letters, col, mre, mim);
            for (uint64_t j = 0; j < N; ++j) {
                double *a = A + 2 * (j * N + col[j]);
                a[0] += cr * mre[j] - ci * mim[j];
                a[1] += cr * mim[j] + ci * mre[j];
            }
        }
    free(col);
    free(mre);
    free(mim);
    return 0;
}

/* Every coefficient of the listed X-patterns: out[i * 2^n + z] (complex,
 * interleaved) for x = xs[i]. */
int oracle_rows_f64(int n, const double *A, int64_t count, const uint32_t *xs, double *out, int nthreads)
{
    if (n < 1 || n > 20 || !A || !out || count < 0 || (count > 0 && !xs)) return -1;
    for (int64_t i = 0; i < count; ++i)
        if (xs[i] >= ((uint64_t)1 << n)) return -1;
    job_t jb;
    memset(&jb, 0, sizeof jb);
    jb.n = n;
    jb.Ad = A;
    jb.outd = out;
    jb.count = count;
    jb.rows = xs;
    return run_threads(&jb, nthreads, rows_worker);
}
