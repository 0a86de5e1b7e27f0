"""Autotuner: candidates admitted only when bit-identical on integer input;
the chosen setting is used by pauli_decompose afterwards."""
import ctypes

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


def _check_report(rec, n, code, hermitian):
    """The kept setting is the default unless it beat the default's median by
    more than the larger run-to-run spread; the report says which."""
    from paper_2403_11644_amd import _native

    assert {"default_ms", "spread_ms", "kept"} <= set(rec)
    assert rec["spread_ms"] >= 0.0 and rec["default_ms"] > 0.0
    if rec["kept"]:
        assert rec["default_ms"] - rec["ms"] > rec["spread_ms"]
    else:
        assert rec["ms"] == rec["default_ms"]
        cfg, la = ctypes.c_int(), ctypes.c_int()
        L = _native.lib()
        assert L.ptd_get_tuning(n, code, 1 if hermitian else 0, ctypes.byref(cfg), ctypes.byref(la)) == 1
        L.ptd_clear_tuning()
        dcfg, dla = ctypes.c_int(), ctypes.c_int()
        assert L.ptd_get_tuning(n, code, 1 if hermitian else 0, ctypes.byref(dcfg), ctypes.byref(dla)) == 0
        assert (cfg.value, la.value) == (dcfg.value, dla.value)  # the default setting
        L.ptd_set_tuning(n, code, 1 if hermitian else 0, cfg.value, la.value)


@pytest.mark.parametrize("code,hermitian", [(0, False), (1, False), (1, True)])
def test_autotune_n11(ptd, oracle_mod, tmp_path, monkeypatch, code, hermitian):
    import ctypes

    from paper_2403_11644_amd import _native, tuning

    monkeypatch.setenv("PTD_AUTOTUNE_CACHE", str(tmp_path / "t.json"))
    L = _native.lib()
    L.ptd_clear_tuning()
    n = 11
    re, im = synth.gaussian_int(n, seed=1) if not hermitian else synth.gaussian_int_hermitian(n, seed=1)
    dt = np.complex128 if code == 0 else np.complex64
    A = to_dev(synth.int_to_complex(re, im, dt))
    before = to_host(ptd.decompose(A, hermitian=hermitian))
    rec = tuning.autotune(n, code, hermitian=hermitian, reps=2)
    assert rec["admitted"] >= 1 and rec["candidates"] >= rec["admitted"]
    _check_report(rec, n, code, hermitian)
    cfg, la = ctypes.c_int(), ctypes.c_int()
    assert L.ptd_get_tuning(n, code, 1 if hermitian else 0, ctypes.byref(cfg), ctypes.byref(la)) == 1
    assert (cfg.value, la.value) == (rec["cfg"], rec["lookahead"])
    after = to_host(ptd.decompose(A, hermitian=hermitian))
    np.testing.assert_array_equal(after, before)
    # cache round trip
    L.ptd_clear_tuning()
    assert tuning.load() == 1
    assert L.ptd_get_tuning(n, code, 1 if hermitian else 0, ctypes.byref(cfg), ctypes.byref(la)) == 1
    L.ptd_clear_tuning()
    # float input through the tuned setting stays within the bar
    L.ptd_set_tuning(n, code, 1 if hermitian else 0, rec["cfg"], rec["lookahead"])
    Af = synth.dense(n, seed=2, dtype=dt)
    got = to_host(ptd.decompose(to_dev(Af)))
    xs, zs = synth.sample_strings(n, 2000, seed=4)
    assert rel_err(got[xs, zs], oracle_mod.coeffs(Af, xs, zs)) <= (1e-12 if code == 0 else 1e-5)
    L.ptd_clear_tuning()


@pytest.mark.parametrize("code,hermitian,n", [(1, True, 10), (1, False, 9), (0, False, 10)])
def test_autotune_group_plan(ptd, oracle_mod, code, hermitian, n):
    """Sizes n <= 10 tune the group plan (workgroup size, radix) on a batch;
    every plan is admitted only if bit-identical on integer input, and single
    calls and batched launches keep agreeing bit for bit under the tuned plan
    and under every other plan."""
    import ctypes

    from paper_2403_11644_amd import _native, tuning

    L = _native.lib()
    L.ptd_clear_tuning()
    rec = tuning.autotune(n, code, hermitian=hermitian, reps=2, save=False)
    assert rec["admitted"] == rec["candidates"] >= 1
    assert rec["lookahead"] == 0
    _check_report(rec, n, code, hermitian)
    dt = np.complex128 if code == 0 else np.complex64
    plans = [0, 1] + ([2, 3] if code == 1 else [])
    mats = [synth.hermitian(n, seed=s, dtype=dt) if hermitian else synth.dense(n, seed=s, dtype=dt)
            for s in range(3)]
    dev = [to_dev(m) for m in mats]
    for plan in plans:
        assert L.ptd_set_tuning(n, code, 1 if hermitian else 0, plan, 0) == 0
        batched = [to_host(c) for c in ptd.decompose_batched(dev, hermitian=hermitian)]
        for m, d, b in zip(mats, dev, batched):
            np.testing.assert_array_equal(to_host(ptd.decompose(d, hermitian=hermitian)), b)
        want = oracle_mod.decompose(mats[0].astype(np.complex128))
        if hermitian:
            want = want.real
        assert rel_err(batched[0], want) <= (1e-12 if code == 0 else 1e-5)
    cfg, la = ctypes.c_int(), ctypes.c_int()
    L.ptd_clear_tuning()
    assert L.ptd_get_tuning(n, code, 1 if hermitian else 0, ctypes.byref(cfg), ctypes.byref(la)) == 0
