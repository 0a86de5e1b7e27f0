"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module holds only random-number generation and array assembly; none of
the decomposition's arithmetic lives here.  Every generator uses numpy's
``default_rng(seed)`` (PCG64).  A complex N(0, 1) array draws the real part
first and then the imaginary part, each as one C-order ``standard_normal``
call, so the oracle and the GPU path read identical bits.

The paper measures on generic dense matrices "with no specific structure"
and on diagonal, tridiagonal and band matrices (Sec. IV-A, Sec. V); it uses
no public dataset, so these generators are the whole input recipe.
"""
from __future__ import annotations

import numpy as np


def complex_normal(shape, seed: int, dtype=np.complex128) -> np.ndarray:
    """Entries with real and imaginary parts iid N(0, 1)."""
    rng = np.random.default_rng(seed)
    fdt = np.float32 if np.dtype(dtype) == np.complex64 else np.float64
    re = rng.standard_normal(shape, dtype=fdt)
    im = rng.standard_normal(shape, dtype=fdt)
    out = np.empty(shape, dtype=dtype)
    out.real = re
    out.imag = im
    return out


def dense(n: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Generic 2^n x 2^n complex matrix, re and im iid N(0, 1)."""
    N = 1 << n
    return complex_normal((N, N), seed, dtype)


def hermitian(n: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """A = (B + B^H) / 2 with B complex N(0, 1); exactly Hermitian in floating
    point because fl(a + conj(b)) = conj(fl(b + conj(a)))."""
    B = dense(n, seed, dtype)
    A = B + B.conj().T
    A *= 0.5
    return A


def gaussian_int(n: int, seed: int, lo: int = -8, hi: int = 8):
    """(re, im) int64 arrays, entries uniform integers in [lo, hi]."""
    N = 1 << n
    rng = np.random.default_rng(seed)
    re = rng.integers(lo, hi + 1, size=(N, N), dtype=np.int64)
    im = rng.integers(lo, hi + 1, size=(N, N), dtype=np.int64)
    return re, im


def gaussian_int_hermitian(n: int, seed: int, lo: int = -8, hi: int = 8):
    """Hermitian Gaussian-integer matrix built directly (not (B + B^H)/2, which
    would give half-integers): the upper triangle's re, im and the real
    diagonal are uniform integers in [lo, hi]; the lower triangle mirrors the
    upper one conjugated."""
    re, im = gaussian_int(n, seed, lo, hi)
    iu = np.triu_indices(1 << n, 1)
    re_h = np.triu(re)
    re_h[(iu[1], iu[0])] = re[iu]
    im_h = np.triu(im, 1)
    im_h[(iu[1], iu[0])] = -im[iu]
    return re_h, im_h


def int_to_complex(re: np.ndarray, im: np.ndarray, dtype=np.complex128) -> np.ndarray:
    out = np.empty(re.shape, dtype=dtype)
    out.real = re
    out.imag = im
    return out


def diagonal_real(n: int, seed: int) -> np.ndarray:
    """Diagonal entries iid N(0, 1), real."""
    return np.random.default_rng(seed).standard_normal(1 << n)


def tridiag_real_sym(n: int, seed: int):
    """Real symmetric tridiagonal: main diagonal a (length N), off-diagonal b
    (length N-1), all iid N(0, 1); a is drawn before b."""
    N = 1 << n
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(N)
    b = rng.standard_normal(N - 1)
    return a, b


def banded_complex(n: int, s: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Row-indexed compressed bands of a complex band matrix with half-bandwidth
    s: band[d + s][k] = A[k][k + d] for d in [-s, s]; slots whose column falls
    outside [0, N) are zero.  In-band entries are complex N(0, 1)."""
    N = 1 << n
    band = complex_normal((2 * s + 1, N), seed, dtype)
    k = np.arange(N)
    for d in range(-s, s + 1):
        bad = (k + d < 0) | (k + d >= N)
        band[d + s][bad] = 0
    return band


def bands_from_diag(diag: np.ndarray, dtype=np.complex128) -> np.ndarray:
    return np.asarray(diag, dtype=dtype)[None, :].copy()


def bands_from_tridiag(a: np.ndarray, b: np.ndarray, dtype=np.complex128) -> np.ndarray:
    """Rows d = -1, 0, +1 of the row-indexed band layout for a symmetric
    tridiagonal matrix with diagonal a and off-diagonal b."""
    N = a.shape[0]
    band = np.zeros((3, N), dtype=dtype)
    band[0, 1:] = b        # A[k][k-1] = b[k-1]
    band[1, :] = a
    band[2, :-1] = b       # A[k][k+1] = b[k]
    return band


def dense_from_bands(band: np.ndarray, dtype=None) -> np.ndarray:
    """Dense matrix from the row-indexed band layout band[d + s][k] = A[k][k + d]."""
    band = np.asarray(band)
    s = (band.shape[0] - 1) // 2
    N = band.shape[1]
    A = np.zeros((N, N), dtype=dtype or band.dtype)
    k = np.arange(N)
    for d in range(-s, s + 1):
        ok = (k + d >= 0) & (k + d < N)
        A[k[ok], k[ok] + d] = band[d + s][ok]
    return A


def antidiagonal_complex(n: int, seed: int, dtype=np.complex128, hermitian: bool = False) -> np.ndarray:
    """Anti-diagonal entries ad[k] = A[k][N - 1 - k], complex N(0, 1); with
    hermitian=True the second half mirrors the first, ad[N - 1 - k] =
    conj(ad[k]) (A[N-1-k][k] = conj(A[k][N-1-k]))."""
    N = 1 << n
    ad = complex_normal(N, seed, dtype)
    if hermitian:
        ad[N // 2:] = np.conj(ad[:N // 2][::-1])
    return ad


def dense_from_antidiagonal(ad: np.ndarray) -> np.ndarray:
    """Dense matrix with A[k][N - 1 - k] = ad[k], zero elsewhere."""
    ad = np.asarray(ad)
    N = ad.shape[0]
    A = np.zeros((N, N), dtype=ad.dtype)
    k = np.arange(N)
    A[k, N - 1 - k] = ad
    return A


def batched_ns(count: int = 4096, seed: int = 0, lo: int = 2, hi: int = 10) -> np.ndarray:
    """Qubit counts of a batch, uniform on [lo, hi]."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=count)


def batched_hermitian(ns, seed: int = 1, dtype=np.complex64):
    """One Hermitian matrix (B + B^H)/2 per entry of ns, B complex N(0, 1)
    drawn from a single generator in index order (re then im per matrix).
    Returns (packed 1-D buffer, element offsets)."""
    rng = np.random.default_rng(seed)
    fdt = np.float32 if np.dtype(dtype) == np.complex64 else np.float64
    sizes = np.array([1 << (2 * int(n)) for n in ns], dtype=np.int64)
    offs = np.zeros(len(ns), dtype=np.int64)
    offs[1:] = np.cumsum(sizes)[:-1]
    buf = np.empty(int(sizes.sum()), dtype=dtype)
    for i, n in enumerate(ns):
        N = 1 << int(n)
        re = rng.standard_normal((N, N), dtype=fdt)
        im = rng.standard_normal((N, N), dtype=fdt)
        B = np.empty((N, N), dtype=dtype)
        B.real = re
        B.imag = im
        A = B + B.conj().T
        A *= 0.5
        buf[offs[i]:offs[i] + sizes[i]] = A.ravel()
    return buf, offs


def sample_strings(n: int, count: int, seed: int):
    """count distinct string indices drawn without replacement from 4^n, as
    (xs, zs) with index = x * 2^n + z."""
    total = 1 << (2 * n)
    count = min(count, total)
    idx = np.random.default_rng(seed).choice(total, count, replace=False)
    idx = np.sort(idx.astype(np.int64))
    return (idx >> n).astype(np.uint32), (idx & ((1 << n) - 1)).astype(np.uint32)


def sample_every_row(n: int, per_x: int, seed: int, low_bits: int = 9):
    """per_x strings for EVERY X-pattern x: the j-th one has a Z-pattern whose
    low `low_bits` bits fall in the j-th of per_x equal blocks of
    [0, 2^low_bits) (the rest of z uniform), so that every row, and every
    run of low Z-positions a kernel may give to one work item, is sampled.
    Returns (xs, zs) as uint32 arrays of length per_x * 2^n."""
    N = 1 << n
    low_bits = min(low_bits, n)
    L = 1 << low_bits
    if per_x < 1 or L % per_x:
        raise ValueError("per_x must divide 2^low_bits")
    blk = L // per_x
    rng = np.random.default_rng(seed)
    xs = np.repeat(np.arange(N, dtype=np.int64), per_x)
    j = np.tile(np.arange(per_x, dtype=np.int64), N)
    high = rng.integers(0, N, size=N * per_x, dtype=np.int64) & ~np.int64(L - 1)
    low = j * blk + rng.integers(0, blk, size=N * per_x, dtype=np.int64)
    return xs.astype(np.uint32), (high | low).astype(np.uint32)
