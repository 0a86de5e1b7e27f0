"""Pauli-string labels <-> (x, z) indices.

A string is stored at coeff[x][z] (x = X-pattern, z = Z-pattern) with
(x_q, z_q) = (0,0) I, (1,0) X, (1,1) Y, (0,1) Z on qubit q; qubit q is bit q
of the matrix index, so the leftmost label character is qubit n-1
(P = s_{n-1} (x) ... (x) s_0, paper Sec. II-B).
"""
from __future__ import annotations

_TO_LETTER = {(0, 0): "I", (1, 0): "X", (1, 1): "Y", (0, 1): "Z"}
_FROM_LETTER = {v: k for k, v in _TO_LETTER.items()}


def label(x: int, z: int, n: int) -> str:
    if not (0 <= x < (1 << n) and 0 <= z < (1 << n)):
        raise ValueError("x and z must lie in [0, 2^n)")
    return "".join(_TO_LETTER[((x >> q) & 1, (z >> q) & 1)] for q in range(n - 1, -1, -1))


def index(lab: str) -> tuple[int, int]:
    """(x, z) of a label such as 'XIZY'."""
    x = z = 0
    n = len(lab)
    for j, ch in enumerate(lab.upper()):
        try:
            xb, zb = _FROM_LETTER[ch]
        except KeyError:
            raise ValueError("bad Pauli letter %r" % ch) from None
        q = n - 1 - j
        x |= xb << q
        z |= zb << q
    return x, z


def flat_index(lab: str) -> int:
    x, z = index(lab)
    return (x << len(lab)) | z


def to_dict(coeff, tol: float = 0.0, xs=None) -> dict:
    """The decomposition as {label: coefficient} over the strings whose
    coefficient exceeds tol in magnitude (the paper keeps its output as such a
    list of strings and values, Algorithm 2).  coeff is a dense (2^n, 2^n)
    array (numpy, or a torch tensor on any device, copied to the host), or a
    compact one of len(xs) rows whose X-patterns are xs.  Host-side
    formatting of a result, not part of the computation."""
    import numpy as np

    if hasattr(coeff, "detach"):
        coeff = coeff.detach().cpu().numpy()
    c = np.asarray(coeff)
    if c.ndim != 2:
        raise ValueError("coeff must be 2-D")
    N = c.shape[1]
    if N < 2 or N & (N - 1):
        raise ValueError("rows must have 2^n entries")
    n = N.bit_length() - 1
    rows = np.arange(c.shape[0]) if xs is None else np.asarray(xs, dtype=np.int64)
    if xs is None and c.shape[0] != N:
        raise ValueError("a compact array needs its X-patterns xs")
    if len(rows) != c.shape[0]:
        raise ValueError("xs must list one X-pattern per row")
    r, z = np.nonzero(np.abs(c) > tol)
    out = {}
    for i, zz in zip(r.tolist(), z.tolist()):
        v = c[i, zz]
        out[label(int(rows[i]), int(zz), n)] = complex(v) if np.iscomplexobj(c) else float(v)
    return out
