"""GPU parity of the structured (diagonal / banded) paths against the oracle.

Only the nonempty X-patterns are computed (paper Sec. IV-A); the oracle
evaluates the same rows from the definition on the dense matrix, and the
rows it proves empty must come out exactly zero.
"""
import numpy as np
import pytest

import synth
from tests.helpers import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = {np.complex128: 1e-12, np.complex64: 1e-5}


@pytest.fixture(scope="module")
def ptd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_11644_amd as p

    return p


def _cases():
    # (name, n, s, builder) -> (bands array, dense matrix)
    def diag(n):
        d = synth.diagonal_real(n, seed=0)
        return synth.bands_from_diag(d), 0

    def tri(n):
        a, b = synth.tridiag_real_sym(n, seed=1)
        return synth.bands_from_tridiag(a, b), 1

    def band8(n):
        return synth.banded_complex(n, 8, seed=2), 8

    return {"diagonal": diag, "tridiagonal": tri, "band8": band8}


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
@pytest.mark.parametrize("kind,n", [("diagonal", 3), ("diagonal", 10), ("diagonal", 12), ("tridiagonal", 5),
                                    ("tridiagonal", 9), ("tridiagonal", 11), ("band8", 6), ("band8", 10),
                                    ("band8", 12), ("band8", 14), ("diagonal", 14), ("tridiagonal", 14)])
def test_structured_vs_oracle(ptd, oracle_mod, dt, kind, n):
    band, s = _cases()[kind](n)
    band = band.astype(dt)
    A = synth.dense_from_bands(band)
    structure = "diagonal" if s == 0 else "banded"
    xs = ptd.nonempty_x(n, structure, s if s else 0)
    Ad = to_dev(A)
    bd = to_dev(band)
    sv = None if s == 0 else s
    comp_dense_in = to_host(ptd.decompose(Ad, structure=structure, s=sv, compact=True))
    comp_bands_in = to_host(ptd.decompose(bd, structure=structure, s=sv, bands=True, compact=True))
    np.testing.assert_array_equal(comp_dense_in, comp_bands_in)
    assert comp_dense_in.shape == (len(xs), 1 << n)
    want = oracle_mod.rows(A.astype(np.complex128), np.array(xs, dtype=np.uint32))
    assert rel_err(comp_dense_in, want) <= TOL[dt]
    full = to_host(ptd.decompose(bd, structure=structure, s=sv, bands=True))
    np.testing.assert_array_equal(full[xs], comp_dense_in)
    mask = np.ones(1 << n, dtype=bool)
    mask[xs] = False
    assert np.all(full[mask] == 0)
    # the general dense path agrees on the listed rows and gives exact zeros
    # elsewhere (compared on the device: the dense output is 4 GiB at n = 14)
    import torch

    dense = ptd.decompose(Ad)
    ix = torch.tensor(xs, dtype=torch.int64, device=dense.device)
    assert rel_err(to_host(dense.index_select(0, ix)), comp_dense_in) <= TOL[dt]
    keep = torch.ones(1 << n, dtype=torch.bool, device=dense.device)
    keep[ix] = False
    assert float(dense[keep].abs().max()) == 0.0
    del dense


@pytest.mark.parametrize("n,s", [(6, 1), (8, 3), (11, 5), (12, 8)])
def test_structured_integer_exact(ptd, oracle_mod, n, s):
    rng = np.random.default_rng(n)
    band = (rng.integers(-8, 9, size=(2 * s + 1, 1 << n)) + 1j * rng.integers(-8, 9, size=(2 * s + 1, 1 << n)))
    k = np.arange(1 << n)
    for d in range(-s, s + 1):
        band[d + s][(k + d < 0) | (k + d >= (1 << n))] = 0
    A = synth.dense_from_bands(band)
    xs = ptd.nonempty_x(n, "banded", s)
    got = to_host(ptd.decompose(to_dev(band), structure="banded", s=s, bands=True, compact=True)) * (1 << n)
    if n <= 11:
        cre, cim = oracle_mod.decompose_int(A.real.astype(np.int64), A.imag.astype(np.int64))
        np.testing.assert_array_equal(got.real, cre[xs].astype(np.float64))
        np.testing.assert_array_equal(got.imag, cim[xs].astype(np.float64))
    else:
        want = oracle_mod.rows(A, np.array(xs, dtype=np.uint32)) * (1 << n)
        np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
@pytest.mark.parametrize("n", [7, 12, 14])
def test_structured_hermitian(ptd, oracle_mod, dt, n):
    # real symmetric tridiagonal is Hermitian: real coefficients
    a, b = synth.tridiag_real_sym(n, seed=4)
    band = synth.bands_from_tridiag(a, b).astype(dt)
    bd = to_dev(band)
    cplx = to_host(ptd.decompose(bd, structure="banded", s=1, bands=True, compact=True))
    assert np.all(cplx.imag == 0.0)
    real = to_host(ptd.decompose(bd, structure="banded", s=1, bands=True, compact=True, hermitian=True))
    np.testing.assert_array_equal(real, cplx.real)
    full = to_host(ptd.decompose(bd, structure="banded", s=1, bands=True, hermitian=True))
    xs = ptd.nonempty_x(n, "banded", 1)
    np.testing.assert_array_equal(full[xs], real)
    assert full.dtype == (np.float64 if dt == np.complex128 else np.float32)


def test_large_band_edge(ptd, oracle_mod):
    # s close to 2^n: nearly every X-pattern is nonempty
    n, s = 9, 500
    band = synth.banded_complex(n, s, seed=3)
    A = synth.dense_from_bands(band)
    xs = ptd.nonempty_x(n, "banded", s)
    assert xs == oracle_mod.nonempty_x_bruteforce(n, s)
    got = to_host(ptd.decompose(to_dev(band), structure="banded", s=s, bands=True, compact=True))
    want = oracle_mod.decompose(A)[xs]
    assert rel_err(got, want) <= 1e-12


# --------------------------------------------------------------------------
# anti-diagonal input: the one X-pattern 2^n - 1 (remark in Sec. IV-A)

@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
@pytest.mark.parametrize("n", [1, 2, 4, 8, 10, 11, 13])
@pytest.mark.parametrize("hermitian", [False, True])
def test_antidiagonal_vs_oracle(ptd, oracle_mod, dt, n, hermitian):
    N = 1 << n
    ad = synth.antidiagonal_complex(n, seed=90 + n, dtype=dt, hermitian=hermitian)
    A = synth.dense_from_antidiagonal(ad)
    assert ptd.nonempty_x(n, "antidiagonal") == [N - 1]
    want = oracle_mod.rows(A.astype(np.complex128), np.array([N - 1], dtype=np.uint32))
    if hermitian:
        want = want.real
    Ad, vd = to_dev(A), to_dev(ad[None, :])
    comp_dense = to_host(ptd.decompose(Ad, structure="antidiagonal", hermitian=hermitian, compact=True))
    comp_vec = to_host(ptd.decompose(vd, structure="antidiagonal", hermitian=hermitian, bands=True, compact=True))
    np.testing.assert_array_equal(comp_dense, comp_vec)
    assert comp_dense.shape == (1, N)
    assert rel_err(comp_dense, want) <= TOL[dt]
    full = to_host(ptd.decompose(vd, structure="antidiagonal", hermitian=hermitian, bands=True))
    np.testing.assert_array_equal(full[N - 1], comp_dense[0])
    assert np.all(full[:N - 1] == 0)
    # the dense path: same row, zeros elsewhere
    dense = to_host(ptd.decompose(Ad, hermitian=hermitian))
    assert rel_err(dense[N - 1:], comp_dense) <= TOL[dt]
    assert np.all(dense[:N - 1] == 0)


@pytest.mark.parametrize("n", [3, 9, 12])
def test_antidiagonal_integer_exact(ptd, oracle_mod, n):
    N = 1 << n
    re, im = synth.gaussian_int(n, seed=95)
    ad_int = (re[0], im[0])  # first row of a Gaussian-integer matrix as the anti-diagonal
    A_re = np.zeros((N, N), dtype=np.int64)
    A_im = np.zeros((N, N), dtype=np.int64)
    k = np.arange(N)
    A_re[k, N - 1 - k] = ad_int[0]
    A_im[k, N - 1 - k] = ad_int[1]
    want_re, want_im = oracle_mod.decompose_int(A_re, A_im) if n <= 9 else (None, None)
    vec = (ad_int[0] + 1j * ad_int[1]).astype(np.complex64)
    got = to_host(ptd.decompose(to_dev(vec[None, :]), structure="antidiagonal", bands=True, compact=True))
    scaled = got[0].astype(np.complex128) * N
    if want_re is not None:
        np.testing.assert_array_equal(scaled.real, want_re[N - 1].astype(np.float64))
        np.testing.assert_array_equal(scaled.imag, want_im[N - 1].astype(np.float64))
    else:
        rows = oracle_mod.rows((A_re + 1j * A_im).astype(np.complex128), np.array([N - 1], dtype=np.uint32))[0]
        np.testing.assert_array_equal(scaled, np.round(rows * N))
