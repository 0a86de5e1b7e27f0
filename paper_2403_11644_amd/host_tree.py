"""Binding of ptd_host_tree_decompose: the paper's tree walk (Sec. III-A,
Algorithms 1-4) and its multi-threaded forest (Sec. V-B) on the host's
cores, a baseline of the paper's own method beside the device path.

Takes and returns numpy arrays (host memory); the work runs in the
library's C++ code, never on the GPU and never in Python.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native

DIAGONAL = 1 << 1


def num_trees(split: int, diagonal: bool = False) -> int:
    """Trees in the forest cut at depth `split` (4^split, 2^split diagonal)."""
    return 1 << (split if diagonal else 2 * split)


def host_tree_decompose(A, *, diagonal: bool = False, split: int = 0, trees: tuple[int, int] | None = None,
                        threads: int = 0, out: np.ndarray | None = None):
    """Coefficients c[x][z] of the 2^n x 2^n complex128 matrix A by the tree
    walk; returns (coeff, ops) with ops the elementary update operations
    counted as Sec. III-B counts them.

    split: depth at which the forest cuts the tree; trees: the range
    [begin, end) of forest trees to run (all by default); threads: host
    threads (0 = one per hardware thread).  Only the strings of the trees
    run are written: a fresh output starts as zeros, and `out` (complex128,
    2^n x 2^n, C-contiguous) keeps what the call does not write.
    With diagonal=True only the I/Z strings (row x = 0) are visited and only
    A's diagonal is read (Sec. IV-A)."""
    A = np.asarray(A)
    if A.dtype != np.complex128 or A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be a square complex128 matrix")
    N = A.shape[0]
    if N < 2 or N & (N - 1):
        raise ValueError("matrix size must be a power of two >= 2, got %d" % N)
    if A.strides[1] != 16:
        raise ValueError("A must have contiguous rows")
    if A.strides[0] % 16:
        raise ValueError("A's row pitch must be a whole number of elements")
    n = N.bit_length() - 1
    if out is None:
        out = np.zeros((N, N), dtype=np.complex128)
    elif out.dtype != np.complex128 or out.shape != (N, N) or not out.flags.c_contiguous:
        raise ValueError("out must be a C-contiguous complex128 array of shape %s" % ((N, N),))
    begin, end = (0, num_trees(split, diagonal)) if trees is None else trees
    ops = ctypes.c_uint64(0)
    st = _native.lib().ptd_host_tree_decompose(
        n, DIAGONAL if diagonal else 0, ctypes.c_void_p(A.ctypes.data), A.strides[0] // 16,
        ctypes.c_void_p(out.ctypes.data), split, begin, end, threads, ctypes.byref(ops))
    _native.check(st, "ptd_host_tree_decompose")
    return out, int(ops.value)
