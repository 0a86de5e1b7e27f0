"""pauli_decompose_noalloc (workspace in the library's fixed device array)
against pauli_decompose (caller's workspace): the same bits, on two calls in
a row, the second with a smaller input, through the C ABI."""
import ctypes

import numpy as np
import pytest

import synth
from tests.helpers import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_11644_amd import _native

    return _native.lib()


def _both(lib, A, flags=0):
    import torch

    from paper_2403_11644_amd import _native, api

    code = api._dtype_code(A.dtype)
    n = A.shape[0].bit_length() - 1
    odt = api._real_dtype(code) if flags & api.HERMITIAN else api._complex_dtype(code)
    sh = api._stream_handle(A.device, None)
    # output of the no-allocation call starts as garbage of its own
    got = torch.full(A.shape, float("nan"), dtype=odt, device=A.device)
    st = lib.pauli_decompose_noalloc(n, code, flags, 0, api._ptr(A), A.stride(0), api._ptr(got), sh)
    _native.check(st, "pauli_decompose_noalloc")
    want = torch.empty(A.shape, dtype=odt, device=A.device)
    wsb = lib.ptd_workspace_bytes(n, code, flags, 0)
    assert wsb <= 65536
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=A.device)
    st = lib.pauli_decompose(n, code, flags, 0, api._ptr(A), A.stride(0), api._ptr(want), api._ptr(ws), wsb, sh)
    _native.check(st, "pauli_decompose")
    torch.cuda.synchronize()
    return to_host(got), to_host(want)


@pytest.mark.parametrize("first,second", [((13, "c128", False), (11, "c128", False)),
                                          ((14, "c64", False), (12, "c64", True)),
                                          ((12, "c128", True), (8, "c64", False))])
def test_noalloc_matches_pauli_decompose(lib, first, second):
    for n, dt, herm in (first, second):
        print("noalloc case n=%d %s herm=%s" % (n, dt, herm), flush=True)
        npdt = np.complex128 if dt == "c128" else np.complex64
        A = synth.hermitian(n, seed=300 + n, dtype=npdt) if herm else synth.dense(n, seed=300 + n, dtype=npdt)
        got, want = _both(lib, to_dev(A), 1 if herm else 0)
        np.testing.assert_array_equal(got, want)
        assert np.isfinite(got).all()


def test_noalloc_argument_errors(lib):
    # validated before any HIP call, like pauli_decompose
    assert lib.pauli_decompose_noalloc(0, 0, 0, 0, ctypes.c_void_p(1 << 40), 1, ctypes.c_void_p(1 << 42), None) == -1
    assert lib.pauli_decompose_noalloc(4, 0, 0, 0, ctypes.c_void_p(1 << 40), 16, ctypes.c_void_p(1 << 40), None) == -1
    assert lib.pauli_decompose_noalloc(4, 0, 1 << 5, 0, ctypes.c_void_p(1 << 40), 16, ctypes.c_void_p(1 << 42),
                                       None) == -3
