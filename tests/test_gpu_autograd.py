"""Autograd through the hand-written adjoints: finite differences
(torch.autograd.gradcheck) and the oracle's gradient 2^-n sum_P w_P P."""
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


def test_gradcheck_n6(ptd):
    import torch

    A = to_dev(synth.dense(6, seed=3)).requires_grad_(True)
    assert torch.autograd.gradcheck(ptd.PauliDecompose.apply, (A,), eps=1e-6, atol=1e-8, rtol=1e-6,
                                    fast_mode=True)


def test_gradcheck_small_full(ptd):
    import torch

    A = to_dev(synth.dense(3, seed=5)).requires_grad_(True)
    assert torch.autograd.gradcheck(ptd.PauliDecompose.apply, (A,), eps=1e-6, atol=1e-8, rtol=1e-6)
    c = to_dev(synth.dense(3, seed=6)).requires_grad_(True)
    assert torch.autograd.gradcheck(ptd.PauliReconstruct.apply, (c,), eps=1e-6, atol=1e-8, rtol=1e-6)


@pytest.mark.parametrize("n", [6, 12, 14])
def test_oracle_gradient(ptd, oracle_mod, n):
    A = to_dev(synth.dense(n, seed=3)).requires_grad_(True)
    w = synth.dense(n, seed=9)
    c = ptd.pauli_decompose(A)
    c.backward(to_dev(w))
    got = to_host(A.grad)
    if n <= 7:
        want = oracle_mod.reconstruct(w) / (1 << n)
    else:
        # the adjoint of decompose is 2^-n reconstruct; check it through the
        # inverse relation decompose(2^n grad) = w on the GPU and on sampled
        # oracle coefficients
        back = to_host(ptd.decompose(to_dev(got * (1 << n))))
        assert rel_err(back, w) <= 1e-12
        xs, zs = synth.sample_strings(n, 500, seed=1)
        coef = oracle_mod.coeffs(got * (1 << n), xs, zs)
        assert rel_err(coef, w[xs, zs]) <= 1e-12
        return
    assert rel_err(got, want) <= 1e-12


def test_real_loss_gradient(ptd):
    # L = sum |c|^2 = 2^-n ||A||_F^2 (Parseval) => dL/dconj(A) = 2^-n A
    import torch

    n = 5
    A = to_dev(synth.dense(n, seed=12)).requires_grad_(True)
    L = (ptd.pauli_decompose(A).abs() ** 2).sum()
    L.backward()
    np.testing.assert_allclose(to_host(A.grad), to_host(A.detach()) * 2.0 / (1 << n), rtol=1e-12, atol=1e-14)
    torch.cuda.synchronize()


@pytest.mark.parametrize("n,dt,herm", [(3, "c128", False), (8, "c64", False), (10, "c128", True), (11, "c128", False),
                                       (13, "c64", True), (14, "c128", False), (15, "c128", False)])
def test_decompose_adjoint_is_unscaled(ptd, n, dt, herm):
    """PTD_ADJOINT of pauli_decompose: Tr(P A) without the 2^-n, i.e. the
    scaled coefficients times 2^n bit for bit (the scale is an exact power
    of two), on every dense schedule (group n <= 10, one launch n = 11..14,
    two-pass complex128 n = 15)."""
    import torch

    npdt = np.complex128 if dt == "c128" else np.complex64
    A = synth.hermitian(n, seed=70 + n, dtype=npdt) if herm else synth.dense(n, seed=70 + n, dtype=npdt)
    Ad = to_dev(A)
    c = ptd.decompose(Ad, hermitian=herm)
    u = ptd.decompose(Ad, hermitian=herm, adjoint=True, check=True)
    assert torch.equal(u, c * float(1 << n))
    del c, u, Ad
    torch.cuda.empty_cache()
