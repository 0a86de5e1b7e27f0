"""Compensated (TwoSum) complex64 butterflies against the float64 oracle."""
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


@pytest.mark.parametrize("n", [2, 5, 6, 7, 10, 12])
def test_compensated_beats_plain(ptd, oracle_mod, n):
    A = synth.dense(n, seed=20 + n, dtype=np.complex64)
    Ad = to_dev(A)
    plain = to_host(ptd.decompose(Ad))
    comp = to_host(ptd.decompose(Ad, compensated=True))
    if n <= 10:
        want = oracle_mod.decompose(A.astype(np.complex128))
        ep, ec = rel_err(plain, want), rel_err(comp, want)
    else:
        xs, zs = synth.sample_strings(n, 20000, seed=3)
        want = oracle_mod.coeffs(A, xs, zs)
        ep, ec = rel_err(plain[xs, zs], want), rel_err(comp[xs, zs], want)
    # one float32 rounding of the result (plus one at the pass boundary)
    assert ec <= 1.2e-7, ec
    assert ec <= ep * 1.05 + 1e-9, (ec, ep)


@pytest.mark.parametrize("n", [4, 9])
def test_compensated_integer_exact(ptd, oracle_mod, n):
    re, im = synth.gaussian_int(n, seed=n)
    cre, cim = oracle_mod.decompose_int(re, im)
    got = to_host(ptd.decompose(to_dev(synth.int_to_complex(re, im, np.complex64)), compensated=True)) * (1 << n)
    np.testing.assert_array_equal(got.real.astype(np.int64), cre)
    np.testing.assert_array_equal(got.imag.astype(np.int64), cim)


@pytest.mark.parametrize("n", [5, 11])
def test_compensated_hermitian(ptd, n):
    A = to_dev(synth.hermitian(n, seed=1, dtype=np.complex64))
    full = to_host(ptd.decompose(A, compensated=True))
    assert np.all(full.imag == 0.0)
    real = to_host(ptd.decompose(A, compensated=True, hermitian=True))
    np.testing.assert_array_equal(real, full.real)


def test_compensated_n15_sampled(ptd, oracle_mod):
    """n = 15 complex64 (the largest measured size): compensated vs plain on
    10^6 sampled coefficients against the float64 oracle, plus the float64
    Parseval residual of both."""
    n = 15
    A = synth.dense(n, seed=0, dtype=np.complex64)
    Ad = to_dev(A)
    xs, zs = synth.sample_strings(n, 1000000, seed=2)
    want = oracle_mod.coeffs(A, xs, zs)
    import torch

    ix = torch.from_numpy(xs.astype(np.int64)).cuda()
    iz = torch.from_numpy(zs.astype(np.int64)).cuda()
    c_plain = ptd.decompose(Ad)
    ep = rel_err(to_host(c_plain[ix, iz]), want)
    _, _, rp = ptd.parseval(Ad, c_plain)
    del c_plain
    c_comp = ptd.decompose(Ad, compensated=True)
    ec = rel_err(to_host(c_comp[ix, iz]), want)
    _, _, rc = ptd.parseval(Ad, c_comp)
    assert ec <= 1e-5 and ep <= 1e-5
    assert ec < ep
    assert rc <= 1e-6 and rp <= 1e-5
