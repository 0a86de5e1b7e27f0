"""Parity at the headline size, covering every X-pattern row and every
work item of the one-launch schedule.

* n = 14 complex128 (the headline workload, seed 0): for every X-pattern x,
  four strings whose low Z-positions fall in the four quarters of
  [0, 512), so every row and every phase-2 block of low positions is
  compared with the float64 oracle (65,536 strings, 1.1e9 oracle terms);
  plus the float64 Parseval residual over all 4^14 coefficients.
* n = 14 complex64, the cast of the same matrix: the same strings, within
  the complex64 bound.
* n = 14 Gaussian-integer input (re, im uniform integers in [-8, 8]):
  2^n c must be integers everywhere (Alg. 2 sums integers), equal to the
  oracle's exact integers on the sampled strings, satisfy Parseval exactly
  in int64 over all 4^14 coefficients (Theorem 1: sum |2^n c|^2 =
  2^n ||A||_F^2), and equal the two-pass schedule bit for bit over the
  whole array.
* The 4096-matrix batch (n uniform in {2..10}): every matrix equals its
  single call bit for bit and is compared with the oracle on 64 strings
  (all of them below n = 4).
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


def _gather(c, xs, zs):
    return to_host(c[to_dev(xs.astype(np.int64)), to_dev(zs.astype(np.int64))])


@pytest.fixture(scope="module")
def headline():
    """The n = 14 complex128 headline matrix on host and device."""
    A = synth.dense(14, seed=0)
    return A, to_dev(A)


def test_n14_c128_every_row(ptd, oracle_mod, headline):
    A, Ad = headline
    print("n=14 complex128, every row", flush=True)
    c = ptd.decompose(Ad, check=True)
    xs, zs = synth.sample_every_row(14, 4, seed=21)
    want = oracle_mod.coeffs(A, xs, zs)
    got = _gather(c, xs, zs)
    assert rel_err(got, want) <= 1e-12
    # also no row may be far off on its own: per-row error against the row's scale
    err_rows = np.abs(got - want).reshape(-1, 4).max(axis=1)
    scale = np.linalg.norm(A) / (1 << 14)
    assert err_rows.max() <= 1e-12 * scale * 1e3
    _, _, res = ptd.parseval(Ad, c)
    assert res <= 1e-12
    del c


def test_n14_c64_every_row(ptd, oracle_mod, headline):
    import torch

    A, Ad = headline
    print("n=14 complex64, every row", flush=True)
    A64 = Ad.to(torch.complex64)
    c = ptd.decompose(A64, check=True)
    xs, zs = synth.sample_every_row(14, 4, seed=22)
    want = oracle_mod.coeffs(A, xs, zs)
    got = _gather(c, xs, zs).astype(np.complex128)
    assert rel_err(got, want) <= 1e-5
    _, _, res = ptd.parseval(A64, c)
    assert res <= 1e-5
    del c, A64


def test_n14_gaussian_integer_exact(ptd, oracle_mod):
    import torch

    from paper_2403_11644_amd import api

    n = 14
    N = 1 << n
    re, im = synth.gaussian_int(n, seed=1)
    A = synth.int_to_complex(re, im)
    Ad = to_dev(A)
    print("n=14 Gaussian integers, exact", flush=True)
    c = ptd.decompose(Ad, check=True)
    scaled = c * float(N)
    # 2^n c is an integer everywhere (exact in float64: |2^n c| < 2^53)
    assert bool(torch.equal(scaled, torch.round(scaled.real) + 1j * torch.round(scaled.imag)))
    # sampled strings: the oracle's sums are exact integers as well
    xs, zs = synth.sample_every_row(n, 4, seed=23)
    want = np.rint(oracle_mod.coeffs(A, xs, zs) * N)
    got = _gather(scaled, xs, zs)
    np.testing.assert_array_equal(got.real.astype(np.int64), want.real.astype(np.int64))
    np.testing.assert_array_equal(got.imag.astype(np.int64), want.imag.astype(np.int64))
    # Parseval over all 4^n coefficients, in exact int64 on the host
    lhs = 0
    for r0 in range(0, N, 2048):
        blk = to_host(scaled[r0:r0 + 2048])
        bre = blk.real.astype(np.int64)
        bim = blk.imag.astype(np.int64)
        lhs += int((bre * bre).sum()) + int((bim * bim).sum())
    rhs = N * (int((re.astype(np.int64) ** 2).sum()) + int((im.astype(np.int64) ** 2).sum()))
    assert lhs == rhs
    # the two-pass schedule gives the same bits over the whole array
    two = api._debug_decompose_path(Ad, 2)
    assert bool(torch.equal(two, c))
    del c, scaled, two, Ad


def test_batched_4096_every_matrix(ptd, oracle_mod):
    import torch

    ns = synth.batched_ns(4096, seed=0).astype(np.int32)
    buf, in_offs = synth.batched_hermitian(ns, seed=1, dtype=np.complex64)
    dbuf = to_dev(buf)
    sizes = np.array([1 << (2 * int(n)) for n in ns], dtype=np.int64)
    mats = [dbuf[o:o + s].view(1 << int(n), 1 << int(n)) for o, s, n in zip(in_offs, sizes, ns)]
    print("batched 4096, every matrix", flush=True)
    got = ptd.decompose_batched(mats, hermitian=True)
    torch.cuda.synchronize()
    worst = 0.0
    for i in range(len(ns)):
        n = int(ns[i])
        g = to_host(got[i])
        np.testing.assert_array_equal(g, to_host(ptd.decompose(mats[i], hermitian=True)))
        A = buf[in_offs[i]:in_offs[i] + sizes[i]].reshape(1 << n, 1 << n).astype(np.complex128)
        xs, zs = synth.sample_strings(n, 64, seed=1000 + i)
        want = oracle_mod.coeffs(A, xs, zs, nthreads=1)
        err = rel_err(g[xs, zs], want.real)
        worst = max(worst, err)
        assert err <= 1e-5, (i, n, err)
    print("worst relative error over 4096 matrices: %.2e" % worst, flush=True)
