"""Failure reporting of the one-launch schedules, and calls on side streams.

* A bounded wait that gives up must never leave finite wrong values: the
  test hook makes every wait of the launch give up after a few polls (no
  producer count can reach its target), with every kernel ending normally.
  The affected coefficients come out NaN and ptd_workspace_status reports
  PTD_EHIP; the next call on the same workspace starts clean.
* Calls on non-default streams allocate their workspace and outputs on that
  stream: two back-to-back calls on two side streams give the bits of the
  default stream.
"""
import ctypes

import numpy as np
import pytest

import synth
from tests.helpers import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ptd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_11644_amd as p

    return p


def _raw_decompose(A, flags=0):
    """pauli_decompose through the C ABI, returning (status, out, ws, wsb)."""
    import torch

    from paper_2403_11644_amd import _native, api

    L = _native.lib()
    code = api._dtype_code(A.dtype)
    n = A.shape[0].bit_length() - 1
    odt = api._real_dtype(code) if flags & api.HERMITIAN else api._complex_dtype(code)
    out = torch.empty(A.shape, dtype=odt, device=A.device)
    wsb = L.ptd_workspace_bytes(n, code, flags, 0)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=A.device)
    sh = api._stream_handle(A.device, None)
    st = L.pauli_decompose(n, code, flags, 0, api._ptr(A), A.stride(0), api._ptr(out), api._ptr(ws), wsb, sh)
    return st, out, ws, wsb


@pytest.mark.parametrize("n,dt,herm", [(11, "c128", False), (12, "c64", False), (13, "c128", True),
                                       (14, "c64", False)])
def test_wait_timeout_poisons_and_reports(ptd, n, dt, herm):
    import torch

    from paper_2403_11644_amd import _native, api

    L = _native.lib()
    npdt = np.complex128 if dt == "c128" else np.complex64
    A = to_dev(synth.hermitian(n, seed=40 + n, dtype=npdt) if herm else synth.dense(n, seed=40 + n, dtype=npdt))
    flags = api.HERMITIAN if herm else 0
    sh = api._stream_handle(A.device, None)
    print("wait-timeout case n=%d %s herm=%s" % (n, dt, herm), flush=True)
    L.ptd_debug_wait_test_mode(1)
    try:
        st, out, ws, wsb = _raw_decompose(A, flags)
        assert st == 0
        torch.cuda.synchronize()
        assert L.ptd_workspace_status(api._ptr(ws), wsb, sh) == -4
        assert L.ptd_last_hip_error() != 0
        got = to_host(out)
        # every phase-2 item timed out: no finite coefficient is left
        assert np.isnan(got).all()
    finally:
        L.ptd_debug_wait_test_mode(0)
    # the same workspace, normal limits: clean status and the right bits
    st = L.pauli_decompose(n, api._dtype_code(A.dtype), flags, 0, api._ptr(A), A.stride(0), api._ptr(out),
                           api._ptr(ws), wsb, sh)
    assert st == 0
    assert L.ptd_workspace_status(api._ptr(ws), wsb, sh) == 0
    want = to_host(ptd.decompose(A, hermitian=herm))
    np.testing.assert_array_equal(to_host(out), want)
    with pytest.raises(Exception):
        L.ptd_debug_wait_test_mode(1)
        try:
            ptd.decompose(A, hermitian=herm, check=True)
        finally:
            L.ptd_debug_wait_test_mode(0)
    assert np.array_equal(to_host(ptd.decompose(A, hermitian=herm, check=True)), want)


@pytest.mark.parametrize("n,dt", [(11, "c128"), (14, "c64")])
def test_reconstruct_wait_timeout(ptd, n, dt):
    from paper_2403_11644_amd import _native

    L = _native.lib()
    npdt = np.complex128 if dt == "c128" else np.complex64
    c = ptd.decompose(to_dev(synth.dense(n, seed=60 + n, dtype=npdt)))
    print("reconstruct wait-timeout case n=%d %s" % (n, dt), flush=True)
    L.ptd_debug_wait_test_mode(1)
    try:
        with pytest.raises(Exception):
            ptd.reconstruct(c, check=True)
    finally:
        L.ptd_debug_wait_test_mode(0)
    A = ptd.reconstruct(c, check=True)
    back = to_host(ptd.decompose(A))
    assert np.isfinite(back).all()


@pytest.mark.parametrize("n,dt", [(9, "c128"), (12, "c128"), (14, "c64")])
def test_side_streams(ptd, n, dt):
    import torch

    npdt = np.complex128 if dt == "c128" else np.complex64
    A = to_dev(synth.dense(n, seed=80 + n, dtype=npdt))
    B = to_dev(synth.dense(n, seed=81 + n, dtype=npdt))
    want_a = to_host(ptd.decompose(A))
    want_b = to_host(ptd.decompose(B))
    want_ra = to_host(ptd.reconstruct(ptd.decompose(A)))
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    print("side-stream case n=%d %s" % (n, dt), flush=True)
    for _ in range(3):
        ca = ptd.decompose(A, stream=s1)
        cb = ptd.decompose(B, stream=s2)
        cb2 = ptd.decompose(B, stream=s1)
        ra = ptd.reconstruct(ca, stream=s1)
        s1.synchronize()
        s2.synchronize()
        np.testing.assert_array_equal(to_host(ca), want_a)
        np.testing.assert_array_equal(to_host(cb), want_b)
        np.testing.assert_array_equal(to_host(cb2), want_b)
        np.testing.assert_array_equal(to_host(ra), want_ra)


def test_xcc_ids_match_queue_count(ptd):
    """The one-launch schedules keep one queue per XCD and send each
    workgroup to the queue of the die it reads from HW_REG_XCC_ID: the dies
    a wide launch observes must be exactly 0 .. count-1."""
    from paper_2403_11644_amd import _native

    L = _native.lib()
    mask, count = ctypes.c_uint(), ctypes.c_int()
    _native.check(L.ptd_debug_xcc_ids(ctypes.byref(mask), ctypes.byref(count)), "ptd_debug_xcc_ids")
    print("xcc mask %#x, count %d" % (mask.value, count.value), flush=True)
    assert count.value >= 1
    assert mask.value == (1 << count.value) - 1
