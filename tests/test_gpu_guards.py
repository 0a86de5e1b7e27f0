"""Guard canaries, determinism and exact zeros on the device.

* Every kernel family writes exactly its output: outputs are views into
  larger buffers whose surrounding elements hold a sentinel, unchanged
  after the call.
* Two calls on the same input give the same bits (no atomics in the data
  path of the dense, structured, batched and matrix-free kernels).
* Real symmetric input: the strings with an odd number of Y have exactly
  zero coefficients (Theorem 2 makes them real, the odd power of i makes
  them imaginary), and the complex output has exactly zero imaginary parts.
"""
import numpy as np
import pytest

import synth
from tests.helpers import to_dev

pytestmark = pytest.mark.gpu

GUARD = 4096  # elements on each side


@pytest.fixture(scope="module")
def ptd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_11644_amd as p

    return p


def _guarded(shape, dtype):
    import torch

    n = int(np.prod(shape))
    buf = torch.empty(n + 2 * GUARD, dtype=dtype, device="cuda")
    sentinel = complex(1234.5, -987.25) if dtype.is_complex else 1234.5
    buf.fill_(sentinel)
    return buf, buf[GUARD:GUARD + n].view(*shape), sentinel


def _guards_intact(buf, sentinel):
    import torch

    lo, hi = buf[:GUARD], buf[-GUARD:]
    want = torch.full_like(lo, sentinel)
    return bool(torch.equal(lo, want)) and bool(torch.equal(hi, want))


@pytest.mark.parametrize("n,dt,herm", [(3, "c128", False), (8, "c64", True), (10, "c128", False),
                                       (11, "c64", False), (12, "c128", True), (13, "c128", False),
                                       (14, "c64", False)])
def test_dense_writes_only_its_output(ptd, n, dt, herm):
    import torch

    tdt = torch.complex128 if dt == "c128" else torch.complex64
    A = to_dev(synth.hermitian(n, seed=900 + n, dtype=np.complex128 if dt == "c128" else np.complex64))
    odt = (torch.float64 if dt == "c128" else torch.float32) if herm else tdt
    N = 1 << n
    buf, out, s = _guarded((N, N), odt)
    ptd.decompose(A, hermitian=herm, out=out)
    torch.cuda.synchronize()
    assert _guards_intact(buf, s)
    assert bool(torch.equal(out, ptd.decompose(A, hermitian=herm)))


def test_reconstruct_writes_only_its_output(ptd):
    import torch

    for n in (6, 12):
        N = 1 << n
        c = to_dev(synth.complex_normal((N, N), seed=910 + n))
        buf, out, s = _guarded((N, N), torch.complex128)
        ptd.reconstruct(c, out=out)
        torch.cuda.synchronize()
        assert _guards_intact(buf, s)
        assert bool(torch.equal(out, ptd.reconstruct(c)))


def test_structured_and_matrix_free_write_only_their_output(ptd):
    import torch

    # banded, compact output
    n, sb = 12, 3
    N = 1 << n
    bands = to_dev(synth.banded_complex(n, sb, seed=920))  # band[d + s][k] = A[k][k + d]
    rows = ptd.num_nonempty_x(n, "banded", sb)
    buf, out, s = _guarded((rows, N), torch.complex128)
    ptd.decompose(bands, structure="banded", s=sb, bands=True, compact=True, out=out)
    torch.cuda.synchronize()
    assert _guards_intact(buf, s)
    # matrix-free: one-row kernel (n = 13 complex64) and two-halves kernel
    # (n = 14 complex128, real output)
    t = to_dev(synth.complex_normal(2 * 8192 - 1, seed=921, dtype=np.complex64))
    buf, out, s = _guarded((8192, 8192), torch.complex64)
    ptd.decompose(t, toeplitz=True, out=out)
    torch.cuda.synchronize()
    assert _guards_intact(buf, s)
    psi = to_dev(synth.complex_normal(1 << 14, seed=922))
    buf, out, s = _guarded((1 << 14, 1 << 14), torch.float64)
    ptd.decompose(psi, pure_state=True, hermitian=True, out=out)
    torch.cuda.synchronize()
    assert _guards_intact(buf, s)
    del buf, out
    torch.cuda.empty_cache()


def test_algebra_writes_only_its_output(ptd):
    import torch

    n = 9
    N = 1 << n
    ca = to_dev(synth.complex_normal((N, N), seed=930))
    cb = to_dev(synth.complex_normal((N, N), seed=931))
    buf, out, s = _guarded((N, 2 * N), torch.complex128)
    ptd.direct_sum(ca, cb, compact=True, out=out)
    torch.cuda.synchronize()
    assert _guards_intact(buf, s)
    buf, out, s = _guarded((2 * N, 2 * N), torch.float64)
    ptd.hermitian_augment(ca, out=out)
    torch.cuda.synchronize()
    assert _guards_intact(buf, s)
    buf, out, s = _guarded((N, N), torch.float64)
    ptd.lcu_amplitudes(ca, out=out)
    torch.cuda.synchronize()
    assert _guards_intact(buf, s)


@pytest.mark.parametrize("n,dt", [(7, "c128"), (11, "c64"), (14, "c128")])
def test_two_calls_give_the_same_bits(ptd, n, dt):
    import torch

    A = to_dev(synth.dense(n, seed=940 + n, dtype=np.complex128 if dt == "c128" else np.complex64))
    a = ptd.decompose(A)
    b = ptd.decompose(A)
    assert bool(torch.equal(a, b))
    del a, b
    t = to_dev(synth.complex_normal(2 * (1 << n) - 1, seed=941, dtype=np.complex128 if dt == "c128" else np.complex64))
    assert bool(torch.equal(ptd.decompose(t, toeplitz=True), ptd.decompose(t, toeplitz=True)))
    torch.cuda.empty_cache()


def test_batched_repeat_gives_the_same_bits(ptd):
    import torch

    mats = [to_dev(synth.dense(k, seed=950 + k, dtype=np.complex64)) for k in (2, 5, 8, 9, 10, 7, 10)]
    a = ptd.decompose_batched(mats)
    b = ptd.decompose_batched(mats)
    assert all(bool(torch.equal(x, y)) for x, y in zip(a, b))


@pytest.mark.parametrize("n,dt", [(5, "c128"), (9, "c64"), (12, "c128"), (13, "c64")])
def test_real_symmetric_odd_y_exactly_zero(ptd, n, dt):
    import torch

    N = 1 << n
    rng = np.random.default_rng(960 + n)
    B = rng.standard_normal((N, N))
    S = ((B + B.T) / 2).astype(np.complex128 if dt == "c128" else np.complex64)
    c = ptd.decompose(to_dev(S))
    assert float(c.imag.abs().max()) == 0.0
    x = torch.arange(N, device="cuda")
    pc = torch.zeros((N, N), dtype=torch.int64, device="cuda")
    xz = x[:, None] & x[None, :]
    for q in range(n):
        pc += (xz >> q) & 1
    odd = (pc & 1) == 1
    assert float(c.real[odd].abs().max()) == 0.0
    assert float(c.real[~odd].abs().max()) > 0.0
