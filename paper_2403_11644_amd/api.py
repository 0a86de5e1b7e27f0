"""PyTorch-facing wrappers around the C ABI (argument marshalling only).

Tensors must live on a ROCm device; PyTorch supplies device memory (outputs
are allocated with ``torch.empty``) and the current stream.  Every step of
the computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import functools

import torch

from . import _native

C128 = 0
C64 = 1

HERMITIAN = 1 << 0
DIAGONAL = 1 << 1
BANDED = 1 << 2
BANDS_IN = 1 << 3
COMPACT = 1 << 4
ANTIDIAGONAL = 1 << 8
TOEPLITZ = 1 << 9
PURE_STATE = 1 << 10
LOW_RANK = 1 << 11
COMPENSATED = 1 << 5
ADJOINT = 1 << 6


def _dtype_code(t: torch.dtype) -> int:
    if t == torch.complex128:
        return C128
    if t == torch.complex64:
        return C64
    raise TypeError("expected complex128 or complex64, got %s" % t)


def _real_dtype(code: int) -> torch.dtype:
    return torch.float64 if code == C128 else torch.float32


def _complex_dtype(code: int) -> torch.dtype:
    return torch.complex128 if code == C128 else torch.complex64


def _nqubits(N: int) -> int:
    if N < 2 or N & (N - 1):
        raise ValueError("matrix size must be a power of two >= 2 (use pad=True), got %d" % N)
    return N.bit_length() - 1


def _stream_handle(device: torch.device, stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def _on_stream(fn):
    """Run a wrapper with ``stream=`` as torch's current stream.

    The workspace and the outputs a wrapper allocates then belong to the
    stream the kernels run on: when the workspace is freed on return, the
    caching allocator hands its block only to later work on that same stream,
    which runs after these kernels.
    """

    @functools.wraps(fn)
    def wrapper(*args, stream=None, **kwargs):
        if stream is None:
            return fn(*args, stream=None, **kwargs)
        with torch.cuda.stream(stream):
            return fn(*args, stream=stream, **kwargs)

    return wrapper


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _require_device(t: torch.Tensor, name: str) -> None:
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor (the library has no CPU path)" % name)


def _rows(t: torch.Tensor, name: str) -> int:
    """Row pitch in elements of a 2-D tensor whose rows are contiguous."""
    if t.dim() != 2 or (t.stride(1) != 1 and t.shape[1] > 1):
        raise ValueError("%s must be 2-D with contiguous rows" % name)
    # a single row may carry any stride (numpy and torch give new axes 0)
    return t.stride(0) if t.shape[0] > 1 else t.shape[1]


def pad_to_power_of_two(A: torch.Tensor, stream=None) -> torch.Tensor:
    """Embed A top-left in the smallest 2^n x 2^n zero matrix (n >= 1).

    The paper allows zero padding to reach a power-of-two size (Sec. II-A)
    without fixing where A goes; this library puts it in the top-left block.
    The padded copy is written by the library's ptd_zero_pad kernel."""
    r, c = A.shape
    N = 2
    while N < max(r, c):
        N *= 2
    if (r, c) == (N, N):
        return A
    _require_device(A, "A")
    code = _dtype_code(A.dtype)
    n = N.bit_length() - 1
    if stream is not None:
        with torch.cuda.stream(stream):
            out = torch.empty((N, N), dtype=A.dtype, device=A.device)
    else:
        out = torch.empty((N, N), dtype=A.dtype, device=A.device)
    st = _native.lib().ptd_zero_pad(code, _ptr(A), _rows(A, "A"), r, c, _ptr(out), n,
                                    _stream_handle(A.device, stream))
    _native.check(st, "ptd_zero_pad")
    return out


def num_nonempty_x(n: int, structure: str | None = None, s: int = 0) -> int:
    flags = {None: 0, "diagonal": DIAGONAL, "banded": BANDED, "antidiagonal": ANTIDIAGONAL}[structure]
    v = _native.lib().ptd_num_nonempty_x(n, flags, s)
    if v < 0:
        raise ValueError("bad (n, structure, s) = (%d, %r, %d)" % (n, structure, s))
    return v


def nonempty_x(n: int, structure: str | None = None, s: int = 0) -> list[int]:
    """X-patterns that can carry a nonzero coefficient, ascending (Sec. IV-A)."""
    import numpy as np

    flags = {None: 0, "diagonal": DIAGONAL, "banded": BANDED, "antidiagonal": ANTIDIAGONAL}[structure]
    cnt = num_nonempty_x(n, structure, s)
    buf = np.empty(cnt, dtype=np.uint32)
    _native.check(_native.lib().ptd_nonempty_x(n, flags, s, ctypes.c_void_p(buf.ctypes.data)), "ptd_nonempty_x")
    return buf.tolist()


@_on_stream
def decompose(A: torch.Tensor, *, hermitian: bool = False, structure: str | None = None, s: int | None = None,
              bands: bool = False, compact: bool = False, compensated: bool = False, pad: bool = False,
              toeplitz: bool = False, pure_state: bool = False, low_rank: bool = False,
              adjoint: bool = False, out: torch.Tensor | None = None, check: bool = False,
              stream=None) -> torch.Tensor:
    """Pauli coefficients of A, as a (2^n, 2^n) tensor c[x, z].

    hermitian   A == A^*: return the (real) coefficients as float64/float32.
    structure   None, 'diagonal', 'banded' (with half-bandwidth s) or
                'antidiagonal'.
    bands       A is the row-indexed band array band[d + s][k] = A[k][k + d]
                (anti-diagonal: the one row ad[k] = A[k][2^n - 1 - k]).
    compact     structured only: return rows of the nonempty X-patterns only.
    compensated complex64 only: TwoSum butterflies.
    pad         zero-pad a non-power-of-two A (top-left embedding).
    toeplitz    A is the 1-D vector t of 2^(n+1) - 1 entries of a Toeplitz
                matrix, A[r][c] = t[c - r + 2^n - 1] (matrix-free input).
    pure_state  A is a state vector psi of 2^n entries and the matrix is
                |psi><psi| (matrix-free): the coefficients are the Pauli
                expectation values <psi|P|psi> / 2^n.
    low_rank    A is a 2^n x r factor U (r <= 32, rows contiguous) and the
                matrix is the mixed state U U^* (matrix-free): the
                coefficients are sum_j <u_j|P|u_j> / 2^n over its columns.
    adjoint     dense input only: Tr(P A) without the 2^-n, the adjoint of
                reconstruct (used by autograd).
    check       wait for the call and raise if the one-launch schedule's
                exchange did not complete (its coefficients are then NaN;
                see ptd_workspace_status).  Off by default: the call stays
                asynchronous.
    """
    _require_device(A, "A")
    code = _dtype_code(A.dtype)
    if toeplitz or pure_state or low_rank:
        if int(toeplitz) + int(pure_state) + int(low_rank) > 1:
            raise ValueError("toeplitz, pure_state and low_rank exclude each other")
        if structure is not None or bands or pad or compact or compensated or adjoint:
            raise ValueError("matrix-free input takes a dense decomposition only")
        if low_rank:
            if A.dim() != 2 or not 1 <= A.shape[1] <= 32:
                raise ValueError("a low-rank factor is 2-D with 1..32 columns")
            N = A.shape[0]
            n = _nqubits(N)
            flags = LOW_RANK | (HERMITIAN if hermitian else 0)
            odt = _real_dtype(code) if hermitian else _complex_dtype(code)
            out = _check_out(out, (N, N), odt, A.device)
            L = _native.lib()
            rank = int(A.shape[1])
            wsb = L.ptd_workspace_bytes(n, code, flags, rank)
            ws = torch.empty(wsb, dtype=torch.uint8, device=A.device) if wsb else None
            st = L.pauli_decompose(n, code, flags, rank, _ptr(A), _rows(A, "U"), _ptr(out),
                                   _ptr(ws) if ws is not None else None, wsb, _stream_handle(A.device, stream))
            _native.check(st, "pauli_decompose")
            return out
        if A.dim() != 1 or not A.is_contiguous():
            raise ValueError("matrix-free input is a contiguous vector")
        if toeplitz:
            if (A.shape[0] + 1) & A.shape[0] or A.shape[0] < 3:
                raise ValueError("a Toeplitz input has 2^(n+1) - 1 entries")
            N = (A.shape[0] + 1) // 2
        else:
            N = A.shape[0]
        n = _nqubits(N)
        flags = (TOEPLITZ if toeplitz else PURE_STATE) | (HERMITIAN if hermitian else 0)
        odt = _real_dtype(code) if hermitian else _complex_dtype(code)
        out = _check_out(out, (N, N), odt, A.device)
        L = _native.lib()
        wsb = L.ptd_workspace_bytes(n, code, flags, 0)
        ws = torch.empty(wsb, dtype=torch.uint8, device=A.device) if wsb else None
        st = L.pauli_decompose(n, code, flags, 0, _ptr(A), 0, _ptr(out), _ptr(ws) if ws is not None else None, wsb,
                               _stream_handle(A.device, stream))
        _native.check(st, "pauli_decompose")
        return out
    flags = 0
    sv = 0
    if structure == "diagonal":
        flags |= DIAGONAL
    elif structure == "banded":
        if s is None or s < 1:
            raise ValueError("banded structure needs s >= 1")
        flags |= BANDED
        sv = int(s)
    elif structure == "antidiagonal":
        flags |= ANTIDIAGONAL
    elif structure is not None:
        raise ValueError("structure must be None, 'diagonal', 'banded' or 'antidiagonal'")
    if bands:
        if structure is None:
            raise ValueError("bands=True needs a structure")
        flags |= BANDS_IN
        N = A.shape[1]
        if A.shape[0] != 2 * sv + 1:
            raise ValueError("band array must have 2s+1 rows")
    else:
        if pad:
            A = pad_to_power_of_two(A, stream=stream)
        if A.dim() != 2 or A.shape[0] != A.shape[1]:
            raise ValueError("A must be square")
        N = A.shape[0]
    n = _nqubits(N)
    if hermitian:
        flags |= HERMITIAN
    if compact:
        if structure is None:
            raise ValueError("compact=True needs a structure")
        flags |= COMPACT
    if compensated:
        flags |= COMPENSATED
    if adjoint:
        flags |= ADJOINT
    lda = _rows(A, "A")
    rows = num_nonempty_x(n, structure, sv) if compact else N
    odt = _real_dtype(code) if hermitian else _complex_dtype(code)
    if out is None:
        out = torch.empty((rows, N), dtype=odt, device=A.device)
    elif out.shape != (rows, N) or out.dtype != odt or not out.is_contiguous():
        raise ValueError("out must be a contiguous %s tensor of shape %r" % (odt, (rows, N)))
    L = _native.lib()
    wsb = L.ptd_workspace_bytes(n, code, flags, sv)
    ws = torch.empty(wsb, dtype=torch.uint8, device=A.device) if wsb else None
    sh = _stream_handle(A.device, stream)
    st = L.pauli_decompose(n, code, flags, sv, _ptr(A), lda, _ptr(out), _ptr(ws) if ws is not None else None,
                           wsb, sh)
    _native.check(st, "pauli_decompose")
    if check:
        _native.check(L.ptd_workspace_status(_ptr(ws) if ws is not None else None, wsb, sh), "pauli_decompose")
    return out


@_on_stream
def reconstruct(c: torch.Tensor, *, hermitian: bool = False, adjoint: bool = False, dtype: torch.dtype | None = None,
                out: torch.Tensor | None = None, check: bool = False, stream=None) -> torch.Tensor:
    """A = sum_P c_P P from dense coefficients c[x, z] (adjoint: times 2^-n).

    With hermitian=True, c is real (float64/float32) and A is Hermitian.
    check: wait and raise if the one-launch schedule's exchange did not
    complete (as for decompose).
    """
    _require_device(c, "c")
    if hermitian:
        if c.dtype == torch.float64:
            code = C128
        elif c.dtype == torch.float32:
            code = C64
        else:
            raise TypeError("hermitian reconstruct takes real float64/float32 coefficients")
    else:
        code = _dtype_code(c.dtype)
    if c.dim() != 2 or c.shape[0] != c.shape[1] or not c.is_contiguous():
        raise ValueError("c must be a contiguous square (2^n, 2^n) tensor")
    N = c.shape[0]
    n = _nqubits(N)
    flags = (HERMITIAN if hermitian else 0) | (ADJOINT if adjoint else 0)
    adt = _complex_dtype(code)
    if out is None:
        out = torch.empty((N, N), dtype=adt, device=c.device)
    elif out.dim() != 2 or out.shape != (N, N) or out.dtype != adt or out.stride(1) != 1:
        raise ValueError("out must be a (2^n, 2^n) %s tensor with contiguous rows" % adt)
    L = _native.lib()
    wsb = L.ptd_reconstruct_workspace_bytes(n, code, flags)
    ws = torch.empty(wsb, dtype=torch.uint8, device=c.device) if wsb else None
    sh = _stream_handle(c.device, stream)
    st = L.pauli_reconstruct(n, code, flags, _ptr(c), _ptr(out), out.stride(0),
                             _ptr(ws) if ws is not None else None, wsb, sh)
    _native.check(st, "pauli_reconstruct")
    if check:
        _native.check(L.ptd_workspace_status(_ptr(ws) if ws is not None else None, wsb, sh), "pauli_reconstruct")
    return out


@_on_stream
def parseval(A: torch.Tensor, c: torch.Tensor, *, hermitian: bool = False, stream=None):
    """(||A||_F^2, 2^n sum|c|^2, relative residual), reduced in float64 on the GPU."""
    import numpy as np

    _require_device(A, "A")
    code = _dtype_code(A.dtype)
    n = _nqubits(A.shape[0])
    L = _native.lib()
    wsb = L.ptd_reduce_workspace_bytes()
    ws = torch.empty(wsb, dtype=torch.uint8, device=A.device)
    res = np.zeros(3, dtype=np.float64)
    st = L.ptd_parseval_residual(n, code, HERMITIAN if hermitian else 0, _ptr(A), _rows(A, "A"), _ptr(c),
                                 ctypes.c_void_p(res.ctypes.data), _ptr(ws), wsb, _stream_handle(A.device, stream))
    _native.check(st, "ptd_parseval_residual")
    return float(res[0]), float(res[1]), float(res[2])


# --------------------------------------------------------------------------
# combinations of decompositions (Sec. IV-B): new coefficients from known ones

def _coeff_square(c: torch.Tensor, name: str) -> int:
    _require_device(c, name)
    if c.dim() != 2 or c.shape[0] != c.shape[1] or not c.is_contiguous():
        raise ValueError("%s must be a contiguous square (2^n, 2^n) coefficient tensor" % name)
    return _nqubits(c.shape[0])


def _check_out(out, shape, dtype, device):
    if out is None:
        return torch.empty(shape, dtype=dtype, device=device)
    if tuple(out.shape) != tuple(shape) or out.dtype != dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous %s tensor of shape %r" % (dtype, tuple(shape)))
    return out


@_on_stream
def block_diagonal(blocks, *, compact: bool = False, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Coefficients of diag(A_0, ..., A_{2^m - 1}) from those of its blocks.

    blocks: a (2^m, 2^k, 2^k) tensor (block i = blocks[i]) or a list of 2^m
    (2^k, 2^k) tensors (stacked first), 1 <= m <= 5.  Returns
    (2^(k+m), 2^(k+m)) coefficients, or with compact=True only the first 2^k
    rows (the others are zero: those strings have X or Y on a new qubit)."""
    if isinstance(blocks, (list, tuple)):
        blocks = torch.stack(list(blocks))
    _require_device(blocks, "blocks")
    if blocks.dim() != 3 or blocks.shape[1] != blocks.shape[2] or not blocks.is_contiguous():
        raise ValueError("blocks must be a contiguous (2^m, 2^k, 2^k) tensor")
    k = _nqubits(blocks.shape[1])
    m = _nqubits(blocks.shape[0]) if blocks.shape[0] > 1 else 0
    code = _dtype_code(blocks.dtype)
    W = 1 << (k + m)
    out = _check_out(out, ((1 << k) if compact else W, W), blocks.dtype, blocks.device)
    st = _native.lib().ptd_block_diagonal(k, m, code, COMPACT if compact else 0, _ptr(blocks), _ptr(out),
                                          _stream_handle(blocks.device, stream))
    _native.check(st, "ptd_block_diagonal")
    return out


@_on_stream
def direct_sum(ca: torch.Tensor, cb: torch.Tensor, *, compact: bool = False, out: torch.Tensor | None = None,
               stream=None) -> torch.Tensor:
    """Coefficients of A (+) B = [[A, 0], [0, B]] from those of A and B."""
    n = _coeff_square(ca, "ca")
    if _coeff_square(cb, "cb") != n or cb.dtype != ca.dtype:
        raise ValueError("ca and cb must have the same size and dtype")
    code = _dtype_code(ca.dtype)
    W = 2 << n
    out = _check_out(out, ((1 << n) if compact else W, W), ca.dtype, ca.device)
    st = _native.lib().ptd_direct_sum(n, code, COMPACT if compact else 0, _ptr(ca), _ptr(cb), _ptr(out),
                                      _stream_handle(ca.device, stream))
    _native.check(st, "ptd_direct_sum")
    return out


@_on_stream
def hermitian_augment(c: torch.Tensor, *, compact: bool = False, out: torch.Tensor | None = None,
                      stream=None) -> torch.Tensor:
    """Real coefficients of [[0, A^H], [A, 0]] on n + 1 qubits from those of A:
    X on the new qubit carries Re c, Y carries Im c.  compact=True returns
    only the rows 2^n .. 2^(n+1) - 1 (the others are zero)."""
    n = _coeff_square(c, "c")
    code = _dtype_code(c.dtype)
    W = 2 << n
    out = _check_out(out, ((1 << n) if compact else W, W), _real_dtype(code), c.device)
    st = _native.lib().ptd_hermitian_augment(n, code, COMPACT if compact else 0, _ptr(c), _ptr(out),
                                             _stream_handle(c.device, stream))
    _native.check(st, "ptd_hermitian_augment")
    return out


@_on_stream
def linear_combination(mu, ca: torch.Tensor, cb: torch.Tensor, *, out: torch.Tensor | None = None,
                       stream=None) -> torch.Tensor:
    """Coefficients of mu A + B: mu * ca + cb elementwise (out may be ca or cb)."""
    n = _coeff_square(ca, "ca")
    if _coeff_square(cb, "cb") != n or cb.dtype != ca.dtype:
        raise ValueError("ca and cb must have the same size and dtype")
    code = _dtype_code(ca.dtype)
    out = _check_out(out, tuple(ca.shape), ca.dtype, ca.device)
    mu = complex(mu)
    st = _native.lib().ptd_linear_combination(n, code, mu.real, mu.imag, _ptr(ca), _ptr(cb), _ptr(out),
                                              _stream_handle(ca.device, stream))
    _native.check(st, "ptd_linear_combination")
    return out


@_on_stream
def decompose_sparse(rows: torch.Tensor, cols: torch.Tensor, vals: torch.Tensor, n: int, *, compact: bool = False,
                     out: torch.Tensor | None = None, stream=None):
    """Coefficients of a sparse 2^n x 2^n matrix given by coordinate entries
    (int32 rows and cols, complex vals, all on the GPU; repeated coordinates
    are summed).  Only the X-patterns r ^ c of its entries can be nonzero;
    returns (coefficients, xs): the dense (2^n, 2^n) array, or with
    compact=True the rows of those X-patterns only, and their ascending list
    xs (an int64 tensor on the device)."""
    import numpy as np

    for t, name in ((rows, "rows"), (cols, "cols"), (vals, "vals")):
        _require_device(t, name)
        if t.dim() != 1 or not t.is_contiguous():
            raise ValueError("%s must be a contiguous 1-D tensor" % name)
    if rows.dtype != torch.int32 or cols.dtype != torch.int32:
        raise TypeError("rows and cols must be int32")
    nnz = rows.shape[0]
    if cols.shape[0] != nnz or vals.shape[0] != nnz:
        raise ValueError("rows, cols and vals must have the same length")
    code = _dtype_code(vals.dtype)
    N = 1 << n
    L = _native.lib()
    wsb = L.ptd_sparse_workspace_bytes(n)
    if wsb == 0:
        raise ValueError("n must lie in 1..16")
    ws = torch.empty(wsb, dtype=torch.uint8, device=vals.device)
    xs = torch.empty(max(1, min(nnz, N)), dtype=torch.int32, device=vals.device)
    cnt = ctypes.c_int()
    st = L.ptd_sparse_nonempty_x(n, nnz, _ptr(rows), _ptr(cols), _ptr(xs), ctypes.byref(cnt), _ptr(ws), wsb,
                                 _stream_handle(vals.device, stream))
    _native.check(st, "ptd_sparse_nonempty_x")
    count = cnt.value
    out = _check_out(out, ((count if compact else N), N), vals.dtype, vals.device)
    if compact and count == 0:
        return out, xs[:0].to(torch.int64)
    st = L.pauli_decompose_sparse(n, code, COMPACT if compact else 0, nnz, _ptr(rows), _ptr(cols), _ptr(vals),
                                  _ptr(xs), count, _ptr(out), _ptr(ws), wsb, _stream_handle(vals.device, stream))
    _native.check(st, "pauli_decompose_sparse")
    return out, xs[:count].to(torch.int64)


@_on_stream
def decompose_csr(row_ptr: torch.Tensor, col_idx: torch.Tensor, vals: torch.Tensor, n: int, *,
                  compact: bool = False, out: torch.Tensor | None = None, stream=None):
    """Coefficients of a sparse 2^n x 2^n matrix in compressed-row form
    (int64 row_ptr of 2^n + 1 values, int32 col_idx, complex vals, all on
    the GPU; row r holds entries row_ptr[r] .. row_ptr[r + 1] - 1, clipped to
    the arrays; a column repeated within a row is summed).  Returns
    (coefficients, xs) as decompose_sparse does."""
    for t, name in ((row_ptr, "row_ptr"), (col_idx, "col_idx"), (vals, "vals")):
        _require_device(t, name)
        if t.dim() != 1 or not t.is_contiguous():
            raise ValueError("%s must be a contiguous 1-D tensor" % name)
    if row_ptr.dtype != torch.int64 or col_idx.dtype != torch.int32:
        raise TypeError("row_ptr must be int64 and col_idx int32")
    N = 1 << n
    if row_ptr.shape[0] != N + 1:
        raise ValueError("row_ptr must hold 2^n + 1 values")
    nnz = col_idx.shape[0]
    if vals.shape[0] != nnz:
        raise ValueError("col_idx and vals must have the same length")
    code = _dtype_code(vals.dtype)
    L = _native.lib()
    wsb = L.ptd_sparse_workspace_bytes(n)
    if wsb == 0:
        raise ValueError("n must lie in 1..16")
    ws = torch.empty(wsb, dtype=torch.uint8, device=vals.device)
    xs = torch.empty(max(1, min(nnz, N)), dtype=torch.int32, device=vals.device)
    cnt = ctypes.c_int()
    h = _stream_handle(vals.device, stream)
    st = L.ptd_csr_nonempty_x(n, nnz, _ptr(row_ptr), _ptr(col_idx), _ptr(xs), ctypes.byref(cnt), _ptr(ws), wsb, h)
    _native.check(st, "ptd_csr_nonempty_x")
    count = cnt.value
    out = _check_out(out, ((count if compact else N), N), vals.dtype, vals.device)
    if compact and count == 0:
        return out, xs[:0].to(torch.int64)
    st = L.pauli_decompose_csr(n, code, COMPACT if compact else 0, nnz, _ptr(row_ptr), _ptr(col_idx), _ptr(vals),
                               _ptr(xs), count, _ptr(out), _ptr(ws), wsb, h)
    _native.check(st, "pauli_decompose_csr")
    return out, xs[:count].to(torch.int64)


@_on_stream
def lcu_amplitudes(c: torch.Tensor, *, hermitian: bool = False, out: torch.Tensor | None = None, stream=None):
    """Amplitudes sqrt(|c_P| / lambda) of the ancilla state that prepares a
    block-encoding by a linear combination of the strings, and lambda =
    sum_P |c_P| (float64 sums on the device).  Returns (amplitudes, lambda);
    c is complex, or real with hermitian=True."""
    import numpy as np

    n = _coeff_square(c, "c")
    if hermitian:
        if c.dtype not in (torch.float64, torch.float32):
            raise TypeError("hermitian=True takes real float64/float32 coefficients")
        code = C128 if c.dtype == torch.float64 else C64
    else:
        code = _dtype_code(c.dtype)
    out = _check_out(out, tuple(c.shape), _real_dtype(code), c.device)
    L = _native.lib()
    wsb = L.ptd_reduce_workspace_bytes()
    ws = torch.empty(wsb, dtype=torch.uint8, device=c.device)
    lam = np.zeros(1, dtype=np.float64)
    st = L.ptd_lcu_amplitudes(n, code, HERMITIAN if hermitian else 0, _ptr(c), _ptr(out),
                              ctypes.c_void_p(lam.ctypes.data), _ptr(ws), wsb, _stream_handle(c.device, stream))
    _native.check(st, "ptd_lcu_amplitudes")
    return out, float(lam[0])


def _debug_decompose_path(A: torch.Tensor, path: int, hermitian: bool = False) -> torch.Tensor:
    """Run a specific dense schedule (1 = single pass, 2 = two passes); for tests."""
    code = _dtype_code(A.dtype)
    n = _nqubits(A.shape[0])
    odt = _real_dtype(code) if hermitian else _complex_dtype(code)
    out = torch.empty((A.shape[0], A.shape[0]), dtype=odt, device=A.device)
    st = _native.lib().ptd_debug_decompose_path(n, code, HERMITIAN if hermitian else 0, _ptr(A), _rows(A, "A"),
                                                _ptr(out), path, _stream_handle(A.device, None))
    _native.check(st, "ptd_debug_decompose_path")
    return out


def _debug_reconstruct_path(c: torch.Tensor, path: int, hermitian: bool = False, adjoint: bool = False):
    code = (C128 if c.dtype == torch.float64 else C64) if hermitian else _dtype_code(c.dtype)
    N = c.shape[0]
    n = _nqubits(N)
    out = torch.empty((N, N), dtype=_complex_dtype(code), device=c.device)
    flags = (HERMITIAN if hermitian else 0) | (ADJOINT if adjoint else 0)
    st = _native.lib().ptd_debug_reconstruct_path(n, code, flags, _ptr(c), _ptr(out), N, path,
                                                  _stream_handle(c.device, None))
    _native.check(st, "ptd_debug_reconstruct_path")
    return out


# --------------------------------------------------------------------------
# batched (many matrices of uneven size, n <= 10 each)

def _batch_layout(mats):
    """(base pointer, element offsets, n list) for same-dtype square GPU tensors."""
    import numpy as np

    if not mats:
        raise ValueError("empty batch")
    dt = mats[0].dtype
    esz = mats[0].element_size()
    ptrs = []
    ns = []
    for m in mats:
        _require_device(m, "batch matrix")
        if m.dtype != dt:
            raise TypeError("all batch matrices must share one dtype")
        if m.dim() != 2 or m.shape[0] != m.shape[1] or not m.is_contiguous():
            raise ValueError("batch matrices must be contiguous and square")
        ns.append(_nqubits(m.shape[0]))
        ptrs.append(m.data_ptr())
    base = min(ptrs)
    offs = np.array([(p - base) // esz for p in ptrs], dtype=np.int64)
    if any((p - base) % esz for p in ptrs):
        raise ValueError("batch matrices are not element-aligned relative to each other")
    return base, offs, np.array(ns, dtype=np.int32)


def _out_layout(ns, odt, device):
    import numpy as np

    sizes = np.array([1 << (2 * int(n)) for n in ns], dtype=np.int64)
    offs = np.zeros(len(ns), dtype=np.int64)
    offs[1:] = np.cumsum(sizes)[:-1]
    buf = torch.empty(int(sizes.sum()), dtype=odt, device=device)
    views = [buf[o:o + s].view(1 << int(n), 1 << int(n)) for o, s, n in zip(offs, sizes, ns)]
    return buf, offs, views


@_on_stream
def decompose_batched(mats, *, hermitian: bool = False, stream=None):
    """Decompose a list of square GPU matrices (n <= 10 each) in one launch.

    Returns a list of coefficient tensors (views of one packed buffer); an
    empty list gives an empty list."""
    import numpy as np

    if len(mats) == 0:
        return []
    base, in_offs, ns = _batch_layout(mats)
    code = _dtype_code(mats[0].dtype)
    odt = _real_dtype(code) if hermitian else _complex_dtype(code)
    obuf, out_offs, views = _out_layout(ns, odt, mats[0].device)
    L = _native.lib()
    nsp = ctypes.c_void_p(ns.ctypes.data)
    wsb = L.ptd_batched_workspace_bytes(len(ns), code, nsp)
    if wsb == 0:
        raise ValueError("batched decomposition needs 1 <= n <= 10 for every matrix")
    ws = torch.empty(wsb, dtype=torch.uint8, device=mats[0].device)
    st = L.pauli_decompose_batched(len(ns), code, HERMITIAN if hermitian else 0, nsp,
                                   ctypes.c_void_p(in_offs.ctypes.data), ctypes.c_void_p(out_offs.ctypes.data),
                                   ctypes.c_void_p(base), _ptr(obuf), _ptr(ws), wsb,
                                   _stream_handle(mats[0].device, stream))
    _native.check(st, "pauli_decompose_batched")
    return views


class BatchPlan:
    """A captured batched launch over fixed buffers (ptd_batch_plan_*).

    in_buf / out_buf are 1-D GPU tensors; ns, in_offsets, out_offsets are
    per-matrix qubit counts and element offsets into them."""

    def __init__(self, in_buf: torch.Tensor, ns, in_offsets, out_buf: torch.Tensor, out_offsets, *,
                 dtype_code: int, hermitian: bool = False, reconstruct: bool = False, adjoint: bool = False):
        import numpy as np

        self._ns = np.ascontiguousarray(ns, dtype=np.int32)
        self._io = np.ascontiguousarray(in_offsets, dtype=np.int64)
        self._oo = np.ascontiguousarray(out_offsets, dtype=np.int64)
        self._keep = (in_buf, out_buf)
        flags = (HERMITIAN if hermitian else 0) | (ADJOINT if adjoint else 0) | ((1 << 7) if reconstruct else 0)
        self._plan = ctypes.c_void_p()
        st = _native.lib().ptd_batch_plan_create(len(self._ns), dtype_code, flags, ctypes.c_void_p(self._ns.ctypes.data),
                                                 ctypes.c_void_p(self._io.ctypes.data),
                                                 ctypes.c_void_p(self._oo.ctypes.data), _ptr(in_buf), _ptr(out_buf),
                                                 ctypes.byref(self._plan))
        _native.check(st, "ptd_batch_plan_create")
        self.device = in_buf.device

    def launch(self, stream=None) -> None:
        _native.check(_native.lib().ptd_batch_plan_launch(self._plan, _stream_handle(self.device, stream)),
                      "ptd_batch_plan_launch")

    def close(self) -> None:
        if self._plan:
            _native.lib().ptd_batch_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
