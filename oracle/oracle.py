"""Plain CPU oracle for the Pauli decomposition -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark (its CPU baseline,
and the errors it states against the oracle on sampled strings) may import
this module.  The product library never does, and this
module imports nothing from the product package: the two share no code.

Two independent evaluations of the definition (paper, Sec. II-A)

    c_P = 2^-n Tr(P A),   P = s_{n-1} (x) ... (x) s_0,  s_q in {I, X, Y, Z}

are provided:

* ``decompose_textbook`` (numpy, tiny n): builds every P with ``np.kron`` from
  the 2x2 matrices printed in Sec. I and takes ``np.trace(P @ A) / 2^n`` --
  the "straightforward decomposition method" of Sec. II-A, cost O(2^{4n}).
* ``decompose`` / ``decompose_int`` / ``coeffs`` (C, ``oracle.c``): the
  sparse form (k, m) of each P from the PauliComposer iteration (Sec. II-B)
  and the trace sum of Algorithm 2, read as sum_j m[j] A[k[j]][j], in
  double precision (exact int64 for Gaussian-integer inputs).

Output layout (a convention the paper leaves open, see oracle.c): a complex
array ``c`` of shape (2^n, 2^n) with ``c[x, z]`` the coefficient of the string
whose qubit q carries (x_q, z_q) = (0,0) I, (1,0) X, (1,1) Y, (0,1) Z; qubit q
is bit q of the matrix index, so the leftmost letter of a label is qubit n-1.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

# Sec. I: the four Pauli matrices.
PAULI_MATRICES = {
    "I": np.array([[1, 0], [0, 1]], dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}
_LETTER_CODE = {"I": 0, "X": 1, "Y": 2, "Z": 3}
_XZ_TO_LETTER = {(0, 0): "I", (1, 0): "X", (1, 1): "Y", (0, 1): "Z"}


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain C11 + pthreads)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build()
            lib = ctypes.CDLL(_LIB_PATH)
            P = ctypes.c_void_p
            lib.oracle_pauli_sparse.argtypes = [ctypes.c_int, P, P, P, P]
            lib.oracle_pauli_sparse.restype = None
            lib.oracle_pauli_sparse_kron.argtypes = [ctypes.c_int, P, P, P, P]
            lib.oracle_pauli_sparse_kron.restype = None
            lib.oracle_decompose_f64.argtypes = [ctypes.c_int, P, P, ctypes.c_int]
            lib.oracle_decompose_f64.restype = ctypes.c_int
            lib.oracle_decompose_i64.argtypes = [ctypes.c_int, P, P, ctypes.c_int]
            lib.oracle_decompose_i64.restype = ctypes.c_int
            lib.oracle_coeffs_f64.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P, P, ctypes.c_int]
            lib.oracle_coeffs_f64.restype = ctypes.c_int
            lib.oracle_rows_f64.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P, ctypes.c_int]
            lib.oracle_rows_f64.restype = ctypes.c_int
            lib.oracle_reconstruct_f64.argtypes = [ctypes.c_int, P, P]
            lib.oracle_reconstruct_f64.restype = ctypes.c_int
            _lib = lib
    return _lib


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count() or 1)


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _nqubits(A: np.ndarray) -> int:
    N = A.shape[0]
    if A.ndim != 2 or A.shape[1] != N or N < 2 or (N & (N - 1)):
        raise ValueError("expected a square 2^n x 2^n matrix, got shape %r" % (A.shape,))
    return N.bit_length() - 1


# --------------------------------------------------------------------------
# labels and letters (conventions only, no arithmetic of the method)

def letters(x: int, z: int, n: int) -> list[str]:
    """Letters [s_0, ..., s_{n-1}] of the string stored at (x, z)."""
    return [_XZ_TO_LETTER[((x >> q) & 1, (z >> q) & 1)] for q in range(n)]


def label(x: int, z: int, n: int) -> str:
    """Label s_{n-1} ... s_0 (leftmost character is qubit n-1)."""
    return "".join(reversed(letters(x, z, n)))


def pauli_matrix(lab: str) -> np.ndarray:
    """Dense P for a label s_{n-1}...s_0 by Kronecker products (Sec. II-A)."""
    M = np.array([[1.0 + 0j]])
    for ch in lab:
        M = np.kron(M, PAULI_MATRICES[ch])
    return M


# --------------------------------------------------------------------------
# the sparse form of P (Sec. II-B)

def pauli_sparse(lab: str, method: str = "composer"):
    """(k, m) of P for a label: k[j] = column of row j's nonzero, m[j] its value."""
    n = len(lab)
    lets = np.array([_LETTER_CODE[ch] for ch in reversed(lab)], dtype=np.uint8)  # lets[q] = s_q
    N = 1 << n
    col = np.zeros(N, dtype=np.uint64)
    mre = np.zeros(N, dtype=np.int8)
    mim = np.zeros(N, dtype=np.int8)
    fn = _load().oracle_pauli_sparse if method == "composer" else _load().oracle_pauli_sparse_kron
    fn(n, _ptr(lets), _ptr(col), _ptr(mre), _ptr(mim))
    return col.astype(np.int64), mre.astype(np.float64) + 1j * mim.astype(np.float64)


# --------------------------------------------------------------------------
# decompositions

def decompose_textbook(A: np.ndarray) -> np.ndarray:
    """c[x, z] = trace(P @ A) / 2^n with P from np.kron (Sec. II-A).  Tiny n only."""
    A = np.asarray(A, dtype=np.complex128)
    n = _nqubits(A)
    if n > 6:
        raise ValueError("textbook oracle is O(2^{4n}); n <= 6 only")
    N = 1 << n
    c = np.empty((N, N), dtype=np.complex128)
    for x in range(N):
        for z in range(N):
            P = pauli_matrix(label(x, z, n))
            c[x, z] = np.trace(P @ A) / N
    return c


def reconstruct_textbook(c: np.ndarray) -> np.ndarray:
    """A = sum_P c_P P with P from np.kron (the expansion of Sec. II-A)."""
    c = np.asarray(c, dtype=np.complex128)
    n = _nqubits(c)
    N = 1 << n
    A = np.zeros((N, N), dtype=np.complex128)
    for x in range(N):
        for z in range(N):
            A += c[x, z] * pauli_matrix(label(x, z, n))
    return A


def decompose(A: np.ndarray, nthreads: int | None = None) -> np.ndarray:
    """All 4^n coefficients, c[x, z], accumulated in float64 (C oracle)."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    n = _nqubits(A)
    N = 1 << n
    out = np.empty((N, N), dtype=np.complex128)
    rc = _load().oracle_decompose_f64(n, _ptr(A), _ptr(out), nthreads or default_threads())
    if rc != 0:
        raise RuntimeError("oracle_decompose_f64 failed (%d)" % rc)
    return out


def decompose_int(A_re: np.ndarray, A_im: np.ndarray, nthreads: int | None = None):
    """Exact 2^n c[x, z] for a Gaussian-integer A, as two int64 arrays (re, im)."""
    A_re = np.asarray(A_re, dtype=np.int64)
    A_im = np.asarray(A_im, dtype=np.int64)
    n = _nqubits(A_re)
    N = 1 << n
    inter = np.empty((N, N, 2), dtype=np.int64)
    inter[..., 0] = A_re
    inter[..., 1] = A_im
    out = np.empty((N, N, 2), dtype=np.int64)
    rc = _load().oracle_decompose_i64(n, _ptr(inter), _ptr(out), nthreads or default_threads())
    if rc != 0:
        raise RuntimeError("oracle_decompose_i64 failed (%d)" % rc)
    return out[..., 0].copy(), out[..., 1].copy()


def coeffs(A: np.ndarray, xs, zs, nthreads: int | None = None) -> np.ndarray:
    """Coefficients of the strings (xs[i], zs[i]) only (float64)."""
    A = np.ascontiguousarray(A)
    if A.dtype != np.complex128:
        A = A.astype(np.complex128)
    n = _nqubits(A)
    xs = np.ascontiguousarray(xs, dtype=np.uint32)
    zs = np.ascontiguousarray(zs, dtype=np.uint32)
    if xs.shape != zs.shape or xs.ndim != 1:
        raise ValueError("xs and zs must be 1-D arrays of equal length")
    out = np.empty(xs.shape[0], dtype=np.complex128)
    rc = _load().oracle_coeffs_f64(n, _ptr(A), xs.shape[0], _ptr(xs), _ptr(zs), _ptr(out),
                                   nthreads or default_threads())
    if rc != 0:
        raise RuntimeError("oracle_coeffs_f64 failed (%d)" % rc)
    return out


def rows(A: np.ndarray, xs, nthreads: int | None = None) -> np.ndarray:
    """Every coefficient of the X-patterns xs: out[i, z] = c[xs[i], z] (float64)."""
    A = np.ascontiguousarray(A)
    if A.dtype != np.complex128:
        A = A.astype(np.complex128)
    n = _nqubits(A)
    xs = np.ascontiguousarray(xs, dtype=np.uint32)
    out = np.empty((xs.shape[0], 1 << n), dtype=np.complex128)
    rc = _load().oracle_rows_f64(n, _ptr(A), xs.shape[0], _ptr(xs), _ptr(out), nthreads or default_threads())
    if rc != 0:
        raise RuntimeError("oracle_rows_f64 failed (%d)" % rc)
    return out


def reconstruct(c: np.ndarray) -> np.ndarray:
    """A = sum_P c_P P from a dense c[x, z] (C oracle, single thread)."""
    c = np.ascontiguousarray(c, dtype=np.complex128)
    n = _nqubits(c)
    N = 1 << n
    A = np.empty((N, N), dtype=np.complex128)
    rc = _load().oracle_reconstruct_f64(n, _ptr(c), _ptr(A))
    if rc != 0:
        raise RuntimeError("oracle_reconstruct_f64 failed (%d)" % rc)
    return A


# --------------------------------------------------------------------------
# norms for the Parseval check (Theorem 1: the strings are orthogonal with
# <P, P> = Tr(P^* P) = 2^n, so ||A||_F^2 = 2^n sum_P |c_P|^2)

def frobenius_sq(A: np.ndarray) -> float:
    A = np.asarray(A)
    return float(np.sum(A.real.astype(np.float64) ** 2) + np.sum(A.imag.astype(np.float64) ** 2))


def coeff_energy(c: np.ndarray, n: int) -> float:
    c = np.asarray(c)
    return float(2.0 ** n * (np.sum(c.real.astype(np.float64) ** 2) + np.sum(c.imag.astype(np.float64) ** 2)))


# --------------------------------------------------------------------------
# structured supports (Sec. IV-A), by brute force over the matrix entries

def nonempty_x_bruteforce(n: int, s: int) -> list[int]:
    """X-patterns x with at least one in-band entry (k, k^x), |(k^x) - k| <= s.

    Only those x can carry a nonzero coefficient of a band matrix with
    half-bandwidth s, because the strings with d-bits x read exactly the
    entries A[k, k^x].  s = 0 is the diagonal case, s = 1 tridiagonal.
    """
    N = 1 << n
    k = np.arange(N, dtype=np.int64)
    out = []
    for x in range(N):
        if np.any(np.abs((k ^ x) - k) <= s):
            out.append(x)
    return out


def band_term_bound(n: int, s: int) -> int:
    """The paper's bound (s n - c(s)) 2^n on the number of nonzero terms of a
    band matrix of width 2s+1, c(s) = s(floor(log2 s) + 1) - 2^{floor(log2 s)+1}
    (Sec. IV-A, band-diagonal theorem)."""
    L = int(np.floor(np.log2(s)))
    c = s * (L + 1) - 2 ** (L + 1)
    return (s * n - c) * (1 << n)


# --------------------------------------------------------------------------
# combinations of decompositions (Sec. IV-B), from the coefficients alone

def direct_sum(ca: np.ndarray, cb: np.ndarray) -> np.ndarray:
    """Coefficients of A (+) B = [[A, 0], [0, B]] on n + 1 qubits (Sec. IV-B,
    "Direct sum"): C = I (x) (A + B)/2 + Z (x) (A - B)/2, the new factor on the
    left, i.e. the most significant qubit.  In the (x, z) layout its I is
    (x_n, z_n) = (0, 0) and its Z is (0, 1); X and Y do not occur."""
    ca = np.asarray(ca)
    cb = np.asarray(cb)
    N = ca.shape[0]
    out = np.zeros((2 * N, 2 * N), dtype=np.result_type(ca, cb))
    out[:N, :N] = (ca + cb) / 2
    out[:N, N:] = (ca - cb) / 2
    return out


def block_diagonal(blocks) -> np.ndarray:
    """Coefficients of diag(A_1, ..., A_N), N = 2^m blocks of one size, by the
    recursion of Sec. IV-B ("Block-diagonal matrices"): neighbouring blocks are
    joined two by two with direct_sum, then the results two by two again,
    ((A_1 (+) A_2) (+) (A_3 (+) A_4)) (+) ..., until one matrix remains."""
    level = [np.asarray(b) for b in blocks]
    if len(level) < 2 or len(level) & (len(level) - 1):
        raise ValueError("need a power-of-two number (>= 2) of blocks")
    while len(level) > 1:
        level = [direct_sum(level[i], level[i + 1]) for i in range(0, len(level), 2)]
    return level[0]


def hermitian_augment(c: np.ndarray) -> np.ndarray:
    """Real coefficients of [[0, A^H], [A, 0]] on n + 1 qubits (Sec. IV-B,
    "Hermitian matrix augmentation"): X (x) sum a_j P_j + Y (x) sum b_j P_j with
    a_j, b_j the real and imaginary parts of A's coefficients.  The new factor
    is the most significant qubit: X is (x_n, z_n) = (1, 0), Y is (1, 1)."""
    c = np.asarray(c)
    N = c.shape[0]
    out = np.zeros((2 * N, 2 * N), dtype=c.real.dtype)
    out[N:, :N] = c.real
    out[N:, N:] = c.imag
    return out


def linear_combination(mu: complex, ca: np.ndarray, cb: np.ndarray) -> np.ndarray:
    """Coefficients of mu A + B (Sec. IV-B, "Linear combination"): mu c_A + c_B,
    elementwise, in the precision of the arrays (mu rounded to it), each part
    rounded as re = (mu_re a_re - mu_im a_im) + b_re, im = (mu_re a_im +
    mu_im a_re) + b_im."""
    ca = np.asarray(ca)
    cb = np.asarray(cb)
    rt = ca.real.dtype
    mr, mi = rt.type(complex(mu).real), rt.type(complex(mu).imag)
    out = np.empty_like(ca)
    out.real = (mr * ca.real - mi * ca.imag) + cb.real
    out.imag = (mr * ca.imag + mi * ca.real) + cb.imag
    return out


# --------------------------------------------------------------------------
# block-encoding by a linear combination of the strings (Sec. VI-C)

def lcu_amplitudes(c: np.ndarray):
    """Amplitudes of the ancilla state sum_i sqrt(|alpha_i|) |i> /
    sqrt(sum_j |alpha_j|) over the strings, in float64, and the 1-norm
    lambda = sum_j |alpha_j|; the phase of each alpha goes with its string."""
    a = np.abs(np.asarray(c).astype(np.complex128))
    lam = float(a.sum())
    return (np.sqrt(a / lam) if lam > 0 else np.zeros_like(a)), lam


# --------------------------------------------------------------------------
# matrix-free input: a Toeplitz matrix from its 2^(n+1) - 1 defining entries

def toeplitz_matrix(t: np.ndarray) -> np.ndarray:
    """Dense A with A[r][c] = t[c - r + N - 1] (t[0] the bottom-left entry,
    t[N - 1] the diagonal, t[2N - 2] the top-right), for the oracle to
    decompose by the definition."""
    t = np.asarray(t)
    N = (t.shape[0] + 1) // 2
    r = np.arange(N)[:, None]
    c = np.arange(N)[None, :]
    return t[c - r + N - 1]


# --------------------------------------------------------------------------
# sparse input (the structured-case argument of Sec. IV-A, for any pattern)

def sparse_to_dense(n: int, rows, cols, vals) -> np.ndarray:
    """The 2^n x 2^n matrix with the coordinate entries added up; entries
    outside [0, 2^n) are dropped."""
    N = 1 << n
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals)
    ok = (rows >= 0) & (rows < N) & (cols >= 0) & (cols < N)
    A = np.zeros((N, N), dtype=np.complex128)
    np.add.at(A, (rows[ok], cols[ok]), vals[ok].astype(np.complex128))
    return A


def sparse_nonempty_x(n: int, rows, cols) -> list[int]:
    """The X-patterns r ^ c of the entries in range, ascending: the strings
    with X-pattern x read only the entries (k, k ^ x)."""
    N = 1 << n
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    ok = (rows >= 0) & (rows < N) & (cols >= 0) & (cols < N)
    return sorted({int(x) for x in (rows[ok] ^ cols[ok])})


def sparse_coeffs(n: int, rows, cols, vals, xs, zs) -> np.ndarray:
    """Coefficients (xs[i], zs[i]) of the matrix with these coordinate
    entries (repeats summed, entries outside [0, 2^n) dropped), from the
    entries alone, for sizes whose dense matrix does not fit in memory.
    Algorithm 2's sum over k reads A[k][k ^ x], which is nonzero only at
    stored entries, so c[x][z] = 2^-n i^popcount(x & z) times the sum, over
    the entries (r, c, v) with r ^ c = x, of (-1)^popcount(z & r) v.
    A loop over the requested strings (float64)."""
    N = 1 << n
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals).astype(np.complex128)
    ok = (rows >= 0) & (rows < N) & (cols >= 0) & (cols < N)
    rows, cols, vals = rows[ok], cols[ok], vals[ok]
    xe = rows ^ cols
    order = np.argsort(xe, kind="stable")
    xe, re_, ve = xe[order], rows[order], vals[order]
    out = np.empty(len(xs), dtype=np.complex128)
    for i, (x, z) in enumerate(zip(xs, zs)):
        x, z = int(x), int(z)
        lo, hi = np.searchsorted(xe, x, "left"), np.searchsorted(xe, x, "right")
        r = re_[lo:hi]
        par = np.zeros(len(r), dtype=np.int64)
        zr = r & z
        for b in range(n):  # parity of popcount(z & r), bit by bit
            par ^= (zr >> b) & 1
        total = np.sum(np.where(par == 1, -ve[lo:hi], ve[lo:hi]))
        out[i] = (1j ** (bin(x & z).count("1") % 4)) * total / N
    return out


def csr_to_coo(n: int, row_ptr, col_idx, vals):
    """The coordinate entries (rows, cols, vals) of a matrix in compressed
    row form: row r holds the entries row_ptr[r] .. row_ptr[r + 1] - 1 of
    col_idx and vals, the range's ends clipped to [0, nnz) (nnz = len(col_idx))
    and the end raised to the start where it lies below it.  Plain loops."""
    N = 1 << n
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    vals = np.asarray(vals)
    nnz = len(col_idx)
    rows, cols, vs = [], [], []
    for r in range(N):
        lo = min(max(int(row_ptr[r]), 0), nnz)
        hi = min(max(int(row_ptr[r + 1]), lo), nnz)
        for e in range(lo, hi):
            rows.append(r)
            cols.append(int(col_idx[e]))
            vs.append(vals[e])
    return (np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64),
            np.array(vs, dtype=vals.dtype if len(vs) else np.complex128))


def csr_to_dense(n: int, row_ptr, col_idx, vals) -> np.ndarray:
    """The 2^n x 2^n matrix of compressed-row entries (csr_to_coo), repeated
    coordinates added up and columns outside [0, 2^n) dropped."""
    return sparse_to_dense(n, *csr_to_coo(n, row_ptr, col_idx, vals))


def csr_nonempty_x(n: int, row_ptr, col_idx) -> list[int]:
    """The X-patterns r ^ c of the compressed-row entries, ascending."""
    rows, cols, _ = csr_to_coo(n, row_ptr, col_idx, np.zeros(len(col_idx), dtype=np.complex128))
    return sparse_nonempty_x(n, rows, cols)


def mixed_density(U: np.ndarray) -> np.ndarray:
    """The matrix U U^* = sum_r u_r u_r^* over the columns u_r of the
    2^n x R factor U: a mixed state (a density matrix of rank <= R, the
    weights absorbed into the columns) given by its factor.  Its
    coefficients are sum_r <u_r|P|u_r> / 2^n."""
    U = np.asarray(U).astype(np.complex128)
    rho = np.zeros((U.shape[0], U.shape[0]), dtype=np.complex128)
    for r in range(U.shape[1]):
        rho += np.outer(U[:, r], np.conj(U[:, r]))
    return rho


def pure_density(psi: np.ndarray) -> np.ndarray:
    """The density matrix |psi><psi| of a state vector, A[r][c] = psi[r]
    conj(psi[c]); its coefficients are the Pauli expectation values
    <psi|P|psi> / 2^n (c_P = 2^-n Tr(P |psi><psi|))."""
    psi = np.asarray(psi).astype(np.complex128)
    return np.outer(psi, np.conj(psi))
