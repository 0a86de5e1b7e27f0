"""GPU parity of the batched persistent launch and its captured plan.

Each matrix of a batch must equal the single-matrix call bit for bit (both
run the same single-pass group routine) and match the oracle.
"""
import numpy as np
import pytest

import synth
from tests.helpers import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ptd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_11644_amd as p

    return p


def _mats(ns, dt, seed, hermitian=False):
    rng = np.random.default_rng(seed)
    out = []
    for n in ns:
        N = 1 << int(n)
        B = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))).astype(dt)
        out.append((B + B.conj().T) / 2 if hermitian else B)
    return out


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
@pytest.mark.parametrize("hermitian", [False, True])
def test_batched_matches_single_calls(ptd, oracle_mod, dt, hermitian):
    ns = np.random.default_rng(3).integers(1, 11, size=40)
    mats = _mats(ns, dt, seed=4, hermitian=hermitian)
    dev = [to_dev(m) for m in mats]
    got = ptd.decompose_batched(dev, hermitian=hermitian)
    for i, (m, g) in enumerate(zip(dev, got)):
        single = to_host(ptd.decompose(m, hermitian=hermitian))
        np.testing.assert_array_equal(to_host(g), single)
        if ns[i] <= 8:
            want = oracle_mod.decompose(mats[i].astype(np.complex128))
            if hermitian:
                want = want.real
            assert rel_err(to_host(g), want) <= (1e-12 if dt == np.complex128 else 1e-5)


def test_batched_integer_exact(ptd, oracle_mod):
    ns = [1, 2, 3, 5, 7, 9, 10, 4, 6, 8]
    mats = []
    want = []
    for i, n in enumerate(ns):
        re, im = synth.gaussian_int(n, seed=50 + i)
        mats.append(synth.int_to_complex(re, im, np.complex64))
        want.append(oracle_mod.decompose_int(re, im))
    got = ptd.decompose_batched([to_dev(m) for m in mats])
    for n, g, (cre, cim) in zip(ns, got, want):
        h = to_host(g) * (1 << n)
        np.testing.assert_array_equal(h.real.astype(np.int64), cre)
        np.testing.assert_array_equal(h.imag.astype(np.int64), cim)


def test_batched_reconstruct_round_trip(ptd):
    import ctypes

    import torch

    from paper_2403_11644_amd import _native, api

    ns = np.array([3, 10, 1, 7, 9, 2], dtype=np.int32)
    mats = _mats(ns, np.complex128, seed=8)
    coeffs = ptd.decompose_batched([to_dev(m) for m in mats])
    # coefficient views share one packed buffer: reconstruct them in one call
    base, in_offs, _ = api._batch_layout(coeffs)
    obuf, out_offs, views = api._out_layout(ns, torch.complex128, coeffs[0].device)
    L = _native.lib()
    wsb = L.ptd_batched_workspace_bytes(len(ns), 0, ctypes.c_void_p(ns.ctypes.data))
    ws = torch.empty(wsb, dtype=torch.uint8, device=coeffs[0].device)
    st = L.pauli_reconstruct_batched(len(ns), 0, 0, ctypes.c_void_p(ns.ctypes.data),
                                     ctypes.c_void_p(in_offs.ctypes.data), ctypes.c_void_p(out_offs.ctypes.data),
                                     ctypes.c_void_p(base), api._ptr(obuf), api._ptr(ws), wsb,
                                     api._stream_handle(coeffs[0].device, None))
    _native.check(st, "pauli_reconstruct_batched")
    for m, v in zip(mats, views):
        assert rel_err(to_host(v), m) <= 1e-13


def test_plan_replays(ptd):
    """The captured plan, replayed several times with eager work and
    synchronisations in between, matches the eager batched call each time."""
    import torch

    from paper_2403_11644_amd import api

    ns = np.array([10, 9, 2, 8, 5, 10, 3, 7], dtype=np.int32)
    buf, in_offs = synth.batched_hermitian(ns, seed=11, dtype=np.complex64)
    dbuf = to_dev(buf)
    sizes = np.array([1 << (2 * int(n)) for n in ns], dtype=np.int64)
    out_offs = np.zeros(len(ns), dtype=np.int64)
    out_offs[1:] = np.cumsum(sizes)[:-1]
    out = torch.empty(int(sizes.sum()), dtype=torch.float32, device=dbuf.device)
    plan = api.BatchPlan(dbuf, ns, in_offs, out, out_offs, dtype_code=api.C64, hermitian=True)
    mats = [dbuf[o:o + s].view(1 << int(n), 1 << int(n)) for o, s, n in zip(in_offs, sizes, ns)]
    eager = [to_host(v) for v in ptd.decompose_batched(mats, hermitian=True)]
    for rep in range(4):
        out.fill_(float("nan"))
        plan.launch()
        torch.cuda.synchronize()
        for o, s, e in zip(out_offs, sizes, eager):
            np.testing.assert_array_equal(to_host(out[o:o + s]).reshape(e.shape), e)
        _ = ptd.decompose(mats[0], hermitian=True)  # eager work between replays
        torch.cuda.synchronize()
    plan.close()


def test_batched_config_4096(ptd, oracle_mod):
    """4096 Hermitian complex64 matrices, n uniform in {2..10} (seeded), one
    launch: every matrix equals its single call; one matrix per n is checked
    against the oracle."""
    import torch

    from paper_2403_11644_amd import api

    ns = synth.batched_ns(4096, seed=0).astype(np.int32)
    buf, in_offs = synth.batched_hermitian(ns, seed=1, dtype=np.complex64)
    dbuf = to_dev(buf)
    sizes = np.array([1 << (2 * int(n)) for n in ns], dtype=np.int64)
    mats = [dbuf[o:o + s].view(1 << int(n), 1 << int(n)) for o, s, n in zip(in_offs, sizes, ns)]
    got = ptd.decompose_batched(mats, hermitian=True)
    torch.cuda.synchronize()
    checked = set()
    for i in range(len(ns)):
        n = int(ns[i])
        if i % 37 == 0 or n not in checked:
            single = to_host(ptd.decompose(mats[i], hermitian=True))
            np.testing.assert_array_equal(to_host(got[i]), single)
        if n not in checked:
            A = buf[in_offs[i]:in_offs[i] + sizes[i]].reshape(1 << n, 1 << n)
            want = oracle_mod.decompose(A.astype(np.complex128)).real
            assert rel_err(to_host(got[i]), want) <= 1e-5
            checked.add(n)
    assert checked == set(range(2, 11))
