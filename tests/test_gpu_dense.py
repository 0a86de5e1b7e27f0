"""GPU parity of the dense decompose/reconstruct kernels against the CPU oracle.

Bars: exact int64 equality of 2^n c_P on Gaussian-integer inputs; relative
error in norm <= 1e-12 for the float64 path and <= 1e-5 for complex64.
"""
import numpy as np
import pytest

import synth
from tests.helpers import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


@pytest.fixture(scope="module")
def ptd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_11644_amd as p

    return p


def _tdtype(name):
    import torch

    return torch.complex128 if name == "c128" else torch.complex64


def _np_dtype(name):
    return np.complex128 if name == "c128" else np.complex64


# --------------------------------------------------------------------------
# float inputs, full oracle, every n and both schedules

@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", list(range(1, 11)))
def test_dense_fwd_group_vs_oracle(ptd, oracle_mod, dt, n):
    A = synth.dense(n, seed=100 + n, dtype=_np_dtype(dt))
    want = oracle_mod.decompose(A.astype(np.complex128))
    got = to_host(ptd.decompose(to_dev(A)))
    assert got.dtype == _np_dtype(dt)
    assert rel_err(got, want) <= TOL[dt], (n, dt, rel_err(got, want))


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [7, 8, 9, 10, 11])
def test_dense_fwd_two_pass_vs_oracle(ptd, oracle_mod, dt, n):
    from paper_2403_11644_amd import api

    A = synth.dense(n, seed=200 + n, dtype=_np_dtype(dt))
    want = oracle_mod.decompose(A.astype(np.complex128))
    got = to_host(api._debug_decompose_path(to_dev(A), 2))
    assert rel_err(got, want) <= TOL[dt], (n, dt, rel_err(got, want))


def test_padded_row_pitch(ptd, oracle_mod):
    # lda > 2^n: a view of the top-left block of a larger matrix
    import torch

    n = 7
    big = synth.dense(8, seed=7)
    Ad = to_dev(big)[: 1 << n, : 1 << n]
    assert Ad.stride(0) == 256
    want = oracle_mod.decompose(big[: 1 << n, : 1 << n])
    got = to_host(ptd.decompose(Ad))
    assert rel_err(got, want) <= 1e-12
    for path in (1, 2):
        from paper_2403_11644_amd import api

        g2 = to_host(api._debug_decompose_path(Ad, path))
        assert rel_err(g2, want) <= 1e-12
    torch.cuda.synchronize()


# --------------------------------------------------------------------------
# Gaussian integers: bit-exact through int64

@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n,path", [(3, 1), (6, 1), (9, 1), (10, 1), (7, 2), (10, 2), (11, 2)])
def test_dense_integer_exact(ptd, oracle_mod, dt, n, path):
    from paper_2403_11644_amd import api

    re, im = synth.gaussian_int(n, seed=300 + n)
    cre, cim = oracle_mod.decompose_int(re, im)
    A = synth.int_to_complex(re, im, _np_dtype(dt))
    got = to_host(api._debug_decompose_path(to_dev(A), path)) * (1 << n)
    np.testing.assert_array_equal(got.real.astype(np.int64), cre)
    np.testing.assert_array_equal(got.imag.astype(np.int64), cim)
    assert np.all(got.real == cre) and np.all(got.imag == cim)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n,path", [(4, 1), (5, 1), (7, 1), (8, 1), (10, 1), (8, 2), (11, 2)])
def test_hermitian_integer_exact(ptd, oracle_mod, dt, n, path):
    from paper_2403_11644_amd import api

    re, im = synth.gaussian_int_hermitian(n, seed=1)
    cre, cim = oracle_mod.decompose_int(re, im)
    assert np.all(cim == 0)
    A = to_dev(synth.int_to_complex(re, im, _np_dtype(dt)))
    real = to_host(api._debug_decompose_path(A, path, hermitian=True)) * (1 << n)
    np.testing.assert_array_equal(real, cre.astype(real.dtype))
    full = to_host(api._debug_decompose_path(A, path))
    assert np.all(full.imag == 0.0)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n,path", [(6, 1), (9, 1), (7, 2), (10, 2), (12, 2)])
def test_hermitian_float(ptd, oracle_mod, dt, n, path):
    from paper_2403_11644_amd import api

    A = synth.hermitian(n, seed=2, dtype=_np_dtype(dt))
    Ad = to_dev(A)
    full = to_host(api._debug_decompose_path(Ad, path))
    # Theorem 2, exactly in the butterfly network
    assert np.all(full.imag == 0.0)
    real = to_host(api._debug_decompose_path(Ad, path, hermitian=True))
    np.testing.assert_array_equal(real, full.real)
    if n <= 10:
        want = oracle_mod.decompose(A.astype(np.complex128))
        assert rel_err(real, want.real) <= TOL[dt]


# --------------------------------------------------------------------------
# reconstruction (the expansion A = sum_P c_P P) and its adjoint scaling

@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n,path", [(1, 1), (2, 1), (4, 1), (5, 1), (8, 1), (10, 1), (7, 2), (10, 2), (11, 2)])
def test_reconstruct_vs_oracle(ptd, oracle_mod, dt, n, path):
    from paper_2403_11644_amd import api

    c = synth.dense(n, seed=400 + n, dtype=_np_dtype(dt))
    cd = to_dev(c)
    got = to_host(api._debug_reconstruct_path(cd, path))
    if n <= 7:
        want = oracle_mod.reconstruct(c.astype(np.complex128))
        assert rel_err(got, want) <= TOL[dt]
    # round trip through the decomposition (exact inverse up to rounding)
    back = to_host(ptd.decompose(to_dev(got)))
    assert rel_err(back, c) <= 4 * TOL[dt]
    adj = to_host(api._debug_reconstruct_path(cd, path, adjoint=True))
    np.testing.assert_array_equal(adj, got / (1 << n))


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n,path", [(6, 1), (9, 2)])
def test_reconstruct_hermitian(ptd, oracle_mod, dt, n, path):
    from paper_2403_11644_amd import api

    c = np.random.default_rng(n).standard_normal((1 << n, 1 << n)).astype(
        np.float64 if dt == "c128" else np.float32)
    A = to_host(api._debug_reconstruct_path(to_dev(c), path, hermitian=True))
    np.testing.assert_array_equal(A, A.conj().T)
    want = oracle_mod.reconstruct(c.astype(np.complex128))
    assert rel_err(A, want) <= TOL[dt]


def test_reconstruct_integer_exact(ptd, oracle_mod):
    n = 6
    re, im = synth.gaussian_int(n, seed=9)
    c = synth.int_to_complex(re, im)
    A = to_host(ptd.reconstruct(to_dev(c)))
    want = oracle_mod.reconstruct(c)
    np.testing.assert_array_equal(A, want)


# --------------------------------------------------------------------------
# Parseval residual in float64 (Theorem 1)

# the single-launch reconstruction (n = 11..14) behind the public call

@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [11, 12, 13, 14])
def test_reconstruct_single_launch_integer(ptd, dt, n):
    """Gaussian-integer A: c = decompose(A) holds exact multiples of 2^-n, so
    the reconstruction must give A back bit for bit, and it must equal the
    two-pass schedule (checked against the oracle at n <= 11) exactly."""
    from paper_2403_11644_amd import api

    re, im = synth.gaussian_int(n, seed=700 + n)
    A = to_dev(synth.int_to_complex(re, im, _np_dtype(dt)))
    c = ptd.decompose(A)
    back = ptd.reconstruct(c)
    assert torch_equal(back, A)
    two = api._debug_reconstruct_path(c, 2)
    assert torch_equal(back, two)
    adj = ptd.reconstruct(c, adjoint=True)
    assert torch_equal(adj * (1 << n), back)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [11, 13])
def test_reconstruct_single_launch_float(ptd, dt, n):
    from paper_2403_11644_amd import api

    c = synth.dense(n, seed=800 + n, dtype=_np_dtype(dt))
    cd = to_dev(c)
    got = to_host(ptd.reconstruct(cd))
    two = to_host(api._debug_reconstruct_path(cd, 2))
    assert rel_err(got, two) <= TOL[dt]
    # A = sum_P c_P P  <=>  decompose(A) = c
    back = to_host(ptd.decompose(to_dev(got)))
    assert rel_err(back, c) <= (1e-12 if dt == "c128" else 2e-5)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [11, 12, 14])
def test_reconstruct_single_launch_hermitian(ptd, dt, n):
    from paper_2403_11644_amd import api

    re, im = synth.gaussian_int_hermitian(n, seed=900 + n)
    A = to_dev(synth.int_to_complex(re, im, _np_dtype(dt)))
    ch = ptd.decompose(A, hermitian=True)
    back = ptd.reconstruct(ch, hermitian=True)
    assert torch_equal(back, A)
    two = api._debug_reconstruct_path(ch, 2, hermitian=True)
    assert torch_equal(back, two)


def torch_equal(a, b):
    import torch

    return bool(torch.equal(a, b))


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_parseval(ptd, oracle_mod, dt):
    n = 9
    A = synth.dense(n, seed=11, dtype=_np_dtype(dt))
    Ad = to_dev(A)
    c = ptd.decompose(Ad)
    fa, fc, res = ptd.parseval(Ad, c)
    np.testing.assert_allclose(fa, oracle_mod.frobenius_sq(A), rtol=1e-13)
    np.testing.assert_allclose(fc, oracle_mod.coeff_energy(to_host(c), n), rtol=1e-12)
    assert res <= (1e-13 if dt == "c128" else 1e-6)
    H = to_dev(synth.hermitian(n, seed=3, dtype=_np_dtype(dt)))
    ch = ptd.decompose(H, hermitian=True)
    _, _, res_h = ptd.parseval(H, ch, hermitian=True)
    assert res_h <= (1e-13 if dt == "c128" else 1e-6)


# --------------------------------------------------------------------------
# full-size rows: sampled oracle coefficients and size-independent properties

@pytest.mark.parametrize("dt,n", [("c128", 13), ("c64", 13), ("c128", 14), ("c64", 14)])
def test_large_sampled(ptd, oracle_mod, dt, n):
    A = synth.dense(n, seed=0, dtype=_np_dtype(dt))
    Ad = to_dev(A)
    c = ptd.decompose(Ad)
    xs, zs = synth.sample_strings(n, 2000, seed=5)
    want = oracle_mod.coeffs(A, xs, zs)
    got = to_host(c[to_dev(xs.astype(np.int64)), to_dev(zs.astype(np.int64))])
    assert rel_err(got, want) <= TOL[dt]
    _, _, res = ptd.parseval(Ad, c)
    assert res <= (1e-12 if dt == "c128" else 1e-5)
    del c, Ad


# --------------------------------------------------------------------------
# the single-launch schedule (n = 11..15): parity, error flag, lookahead

def _fused(A, hermitian=False, lookahead=1, cfg=0):
    import torch

    from paper_2403_11644_amd import _native, api

    code = api._dtype_code(A.dtype)
    n = A.shape[0].bit_length() - 1
    odt = api._real_dtype(code) if hermitian else api._complex_dtype(code)
    out = torch.empty(A.shape, dtype=odt, device=A.device)
    L = _native.lib()
    wsb = L.ptd_workspace_bytes(n, code, api.HERMITIAN if hermitian else 0, 0)
    assert wsb > 0
    ws = torch.zeros(wsb, dtype=torch.uint8, device=A.device)
    st = L.ptd_debug_decompose_fused(n, code, api.HERMITIAN if hermitian else 0, api._ptr(A), A.stride(0),
                                     api._ptr(out), api._ptr(ws), wsb, lookahead, cfg,
                                     api._stream_handle(A.device, None))
    _native.check(st, "fused")
    torch.cuda.synchronize()
    words = ws.view(torch.int32).cpu().numpy()
    assert words[17] == 0, "a bounded wait ran out"
    return out


@pytest.mark.parametrize("dt", ["c128", "c64"])
# cfg: shape in bits 0-1, then non-temporal gathers (4), final stores (8),
# phase-2 loads (16)
@pytest.mark.parametrize("n,la,cfg", [(11, 1, 0), (11, 3, 1), (11, 2, 3), (12, 2, 7), (12, 4, 14), (12, 3, 17),
                                      (13, 1, 1), (13, 4, 0), (13, 2, 3), (13, 2, 30), (13, 3, 25)])
def test_fused_vs_oracle(ptd, oracle_mod, dt, n, la, cfg):
    A = synth.dense(n, seed=500 + n, dtype=_np_dtype(dt))
    got = to_host(_fused(to_dev(A), lookahead=la, cfg=cfg))
    if n <= 11:
        want = oracle_mod.decompose(A.astype(np.complex128))
        assert rel_err(got, want) <= TOL[dt]
    else:
        xs, zs = synth.sample_strings(n, 3000, seed=n)
        want = oracle_mod.coeffs(A, xs, zs)
        assert rel_err(got[xs, zs], want) <= TOL[dt]
    # the public entry point takes the same butterfly network: bit-identical
    np.testing.assert_array_equal(to_host(ptd.decompose(to_dev(A))), got)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [11, 12, 13])
def test_fused_integer_exact(ptd, oracle_mod, dt, n):
    from paper_2403_11644_amd import api

    re, im = synth.gaussian_int(n, seed=600 + n)
    A = to_dev(synth.int_to_complex(re, im, _np_dtype(dt)))
    got = to_host(_fused(A))
    # equal to the two-pass schedule bit for bit (both exact)
    two = to_host(api._debug_decompose_path(A, 2))
    np.testing.assert_array_equal(got, two)
    if n == 11:
        cre, cim = oracle_mod.decompose_int(re, im)
        np.testing.assert_array_equal((got.real * (1 << n)).astype(np.int64), cre)
        np.testing.assert_array_equal((got.imag * (1 << n)).astype(np.int64), cim)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n,cfg", [(11, 0), (11, 3), (12, 26), (12, 29), (13, 0), (13, 1), (13, 13), (13, 31),
                                   (14, 0), (14, 7), (14, 22)])
def test_fused_hermitian(ptd, oracle_mod, dt, n, cfg):
    re, im = synth.gaussian_int_hermitian(n, seed=1)
    A = to_dev(synth.int_to_complex(re, im, _np_dtype(dt)))
    full = to_host(_fused(A, cfg=cfg))
    assert np.all(full.imag == 0.0)
    real = to_host(_fused(A, hermitian=True, cfg=cfg))
    np.testing.assert_array_equal(real, full.real)
    if n == 11:
        cre, _ = oracle_mod.decompose_int(re, im)
        np.testing.assert_array_equal((real * (1 << n)).astype(np.int64), cre)
    else:
        A_h = synth.int_to_complex(re, im)
        xs, zs = synth.sample_strings(n, 2000, seed=3)
        want = oracle_mod.coeffs(A_h, xs, zs)
        np.testing.assert_array_equal(real[xs, zs], want.real)
    if n == 13:
        # every coefficient at once: 2^n c_P is an integer, and Parseval
        # (Theorem 1) holds exactly in integers, sum (2^n c_P)^2 = 2^n ||A||_F^2
        C = real.astype(np.float64) * (1 << n)
        assert np.all(C == np.round(C))
        Ci = C.astype(np.int64)
        rhs = (1 << n) * int((re.astype(np.int64) ** 2 + im.astype(np.int64) ** 2).sum())
        assert int((Ci * Ci).sum()) == rhs


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_hermitian_n13_float(ptd, oracle_mod, dt):
    """The n = 13 Hermitian workload, (B + B^H)/2 with complex N(0, 1) B from
    seed 0, through the public call: sampled strings against the oracle and
    bit-identical to the real part of the general path."""
    n = 13
    A = synth.hermitian(n, seed=0, dtype=_np_dtype(dt))
    Ad = to_dev(A)
    real = ptd.decompose(Ad, hermitian=True)
    full = ptd.decompose(Ad)
    assert float(full.imag.abs().max()) == 0.0
    assert bool((full.real == real).all())
    del full
    xs, zs = synth.sample_strings(n, 3000, seed=13)
    want = oracle_mod.coeffs(A, xs, zs)
    assert np.max(np.abs(want.imag)) <= 1e-12 * np.max(np.abs(want.real))
    assert rel_err(to_host(real)[xs, zs], want.real) <= TOL[dt]


def test_fused_n15_c64(ptd, oracle_mod):
    n = 15
    A = synth.dense(n, seed=0, dtype=np.complex64)
    Ad = to_dev(A)
    got = _fused(Ad)
    xs, zs = synth.sample_strings(n, 3000, seed=2)
    want = oracle_mod.coeffs(A, xs, zs)
    g = to_host(got[to_dev(xs.astype(np.int64)), to_dev(zs.astype(np.int64))])
    assert rel_err(g, want) <= 1e-5


@pytest.mark.parametrize("shape,pitch", [((1, 1), 1), ((3, 3), 3), ((5, 7), 9), ((100, 64), 64), ((70, 130), 200)])
@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_zero_pad_kernel(ptd, shape, pitch, dt):
    """ptd_zero_pad: A top-left in the next 2^n zero square, any row pitch."""
    import torch

    from paper_2403_11644_amd import api

    tdt = torch.complex128 if dt == "c128" else torch.complex64
    r, c = shape
    base = torch.arange(r * pitch, dtype=torch.float64).reshape(r, pitch).to(tdt) * (1 + 1j) + 1
    A = base.cuda()[:, :c]
    P = api.pad_to_power_of_two(A)
    N = 2
    while N < max(r, c):
        N *= 2
    assert P.shape == (N, N)
    want = torch.zeros((N, N), dtype=tdt)
    want[:r, :c] = base[:, :c]
    assert torch.equal(P.cpu(), want)


@pytest.mark.parametrize("size", [3, 100, 1500])
def test_pad_non_power_of_two(ptd, oracle_mod, size):
    """pad=True: the coefficients are those of A embedded top-left in the
    next 2^n zero matrix."""
    rng = np.random.default_rng(size)
    A = (rng.standard_normal((size, size)) + 1j * rng.standard_normal((size, size)))
    got = to_host(ptd.decompose(to_dev(A), pad=True))
    N = 1 << (size - 1).bit_length()
    P = np.zeros((N, N), dtype=np.complex128)
    P[:size, :size] = A
    n = N.bit_length() - 1
    if n <= 8:
        want = oracle_mod.decompose(P)
        assert rel_err(got, want) <= 1e-12
    else:
        xs, zs = synth.sample_strings(n, 3000, seed=1)
        assert rel_err(got[xs, zs], oracle_mod.coeffs(P, xs, zs)) <= 1e-12


# --------------------------------------------------------------------------
# the largest size the library takes: n = 16, 2^32 elements per matrix

@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_max_size_n16_strings(ptd, oracle_mod, dt):
    """A = 3 P1 - 5 P2 + 0.5 P3 at n = 16 (the sparse forms of the three
    strings come from the oracle's PauliComposer and are scattered into a
    zero matrix on the device).  Theorem 1: the coefficients are exactly
    those three numbers at those three strings and zero elsewhere (every
    partial sum is a small multiple of the scalar, exact in either
    precision), and the reconstruction returns exactly the scattered
    entries.  Offsets past 2^31 elements are exercised throughout."""
    import torch

    n, N = 16, 1 << 16
    tdt = torch.complex128 if dt == "c128" else torch.complex64
    strings = [(0xBEEF, 0x1234, 3.0), (0x8001, 0xFFFF, -5.0), (0x0000, 0x7A5C, 0.5)]
    rows = torch.arange(N, device="cuda")
    sparse = []
    A = torch.zeros((N, N), dtype=tdt, device="cuda")
    for x, z, alpha in strings:
        k, m = oracle_mod.pauli_sparse(oracle_mod.label(x, z, n))
        assert np.array_equal(k, np.arange(N) ^ x)
        kd, md = to_dev(k), to_dev(alpha * m, tdt)
        A[rows, kd] = md  # distinct X-patterns: no two strings share an entry
        sparse.append((kd, md))
    c = ptd.decompose(A)
    del A
    torch.cuda.synchronize()
    for x, z, alpha in strings:
        assert complex(c[x, z].item()) == alpha
    assert int((c != 0).sum().item()) == len(strings)
    R = ptd.reconstruct(c)
    del c
    for kd, md in sparse:
        assert bool(torch.equal(R[rows, kd], md))
    assert int((R != 0).sum().item()) == len(strings) * N
    del R, rows
    torch.cuda.empty_cache()


# --------------------------------------------------------------------------
# matrix-free Toeplitz input (PTD_TOEPLITZ): A[r][c] = t[c - r + 2^n - 1]

def _toeplitz_vec(n, seed, dt, hermitian):
    N = 1 << n
    t = synth.complex_normal(2 * N - 1, seed=seed, dtype=dt)
    if hermitian:
        t[N - 1] = t[N - 1].real
        t[:N - 1] = np.conj(t[N:][::-1])  # t[N-1-d] = conj(t[N-1+d])
    return t


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 3, 6, 10, 11, 12, 13, 14])
@pytest.mark.parametrize("hermitian", [False, True])
def test_toeplitz_matches_dense(ptd, oracle_mod, dt, n, hermitian):
    """The matrix-free path gathers the same values as the dense path and
    runs the same butterflies, so it equals the dense decomposition of the
    materialised matrix bit for bit; sampled coefficients against the oracle."""
    import torch

    N = 1 << n
    t = _toeplitz_vec(n, 300 + n, _np_dtype(dt), hermitian)
    td = to_dev(t)
    got = ptd.decompose(td, toeplitz=True, hermitian=hermitian)
    idx = torch.arange(N, device="cuda")[None, :] - torch.arange(N, device="cuda")[:, None] + (N - 1)
    Ad = td[idx]
    del idx
    dense = ptd.decompose(Ad, hermitian=hermitian)
    assert bool(torch.equal(got, dense))
    del dense
    if n <= 12:
        A = oracle_mod.toeplitz_matrix(t.astype(np.complex128))
        xs, zs = synth.sample_strings(n, 500, seed=11)
        want = oracle_mod.coeffs(A, xs, zs)
        if hermitian:
            want = want.real
        g = to_host(got[to_dev(xs.astype(np.int64)), to_dev(zs.astype(np.int64))])
        assert rel_err(g, want) <= TOL[dt]
    del got, Ad
    torch.cuda.empty_cache()


def test_toeplitz_n15_complex64(ptd):
    import torch

    n, N = 15, 1 << 15
    t = _toeplitz_vec(n, 315, np.complex64, False)
    td = to_dev(t)
    got = ptd.decompose(td, toeplitz=True)
    idx = torch.arange(N, device="cuda")[None, :] - torch.arange(N, device="cuda")[:, None] + (N - 1)
    Ad = td[idx]
    del idx
    assert bool(torch.equal(got, ptd.decompose(Ad)))
    del got, Ad
    torch.cuda.empty_cache()


def test_toeplitz_n15_complex64_hermitian(ptd):
    """Real output at n = 15 (complex64, two halves per row): the real part
    of the complex call bit for bit, and exactly real there."""
    import torch

    t = _toeplitz_vec(15, 316, np.complex64, True)
    td = to_dev(t)
    full = ptd.decompose(td, toeplitz=True)
    assert float(full.imag.abs().max()) == 0.0
    re = ptd.decompose(td, toeplitz=True, hermitian=True)
    assert bool(torch.equal(re, full.real))
    del full, re
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n", [2, 5, 8])
def test_toeplitz_integer_exact(ptd, oracle_mod, n):
    N = 1 << n
    rng = np.random.default_rng(330 + n)
    tre = rng.integers(-8, 9, size=2 * N - 1)
    tim = rng.integers(-8, 9, size=2 * N - 1)
    t = (tre + 1j * tim).astype(np.complex64)
    got = to_host(ptd.decompose(to_dev(t), toeplitz=True)).astype(np.complex128) * N
    A = oracle_mod.toeplitz_matrix(t.astype(np.complex128))
    wr, wi = oracle_mod.decompose_int(A.real.astype(np.int64), A.imag.astype(np.int64))
    np.testing.assert_array_equal(got.real, wr.astype(np.float64))
    np.testing.assert_array_equal(got.imag, wi.astype(np.float64))



# --------------------------------------------------------------------------
# matrix-free pure-state input (PTD_PURE_STATE): A = |psi><psi|

@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 4, 7, 10, 11, 13, 14])
@pytest.mark.parametrize("hermitian", [False, True])
def test_pure_state_expectations(ptd, oracle_mod, dt, n, hermitian):
    """Pauli expectation values <psi|P|psi> / 2^n: sampled against the oracle
    on |psi><psi|, real (imaginary parts exactly zero in the complex output),
    and against the dense decomposition of the materialised density matrix."""
    import torch

    N = 1 << n
    psi = synth.complex_normal(N, seed=700 + n, dtype=_np_dtype(dt))
    pd = to_dev(psi)
    got = ptd.decompose(pd, pure_state=True, hermitian=hermitian)
    if not hermitian:
        assert float(got.imag.abs().max()) == 0.0
    xs, zs = synth.sample_strings(n, 500, seed=13)
    ix, iz = to_dev(xs.astype(np.int64)), to_dev(zs.astype(np.int64))
    g = to_host(got[ix, iz])
    if n <= 12:
        want = oracle_mod.coeffs(oracle_mod.pure_density(psi), xs, zs)
        assert rel_err(g, want.real if hermitian else want) <= TOL[dt]
    # the same butterflies on the materialised matrix (formed by torch, whose
    # products may round differently, so within the bar rather than bit for bit)
    rho = torch.outer(pd, pd.conj())
    dense = ptd.decompose(rho, hermitian=hermitian)
    assert rel_err(to_host(got), to_host(dense)) <= TOL[dt]
    del rho, dense, got
    torch.cuda.empty_cache()


def test_pure_state_basis_state(ptd):
    """|k><k| for a basis state k: the coefficient of (x, z) is
    (-1)^popcount(z & k) / 2^n for x = 0 and zero otherwise, exactly."""
    import torch

    n, k = 9, 0b101100110
    N = 1 << n
    psi = torch.zeros(N, dtype=torch.complex128, device="cuda")
    psi[k] = 1.0
    got = to_host(ptd.decompose(psi, pure_state=True, hermitian=True))
    z = np.arange(N)
    sign = 1.0 - 2.0 * (np.array([bin(v & k).count("1") for v in z]) & 1)
    np.testing.assert_array_equal(got[0], sign / N)
    assert np.all(got[1:] == 0)


# --------------------------------------------------------------------------
# matrix-free mixed-state input (PTD_LOW_RANK): A = U U^*

@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n,R", [(1, 1), (3, 2), (6, 5), (10, 3), (11, 4), (12, 32), (13, 2), (14, 3)])
@pytest.mark.parametrize("hermitian", [False, True])
def test_mixed_state_expectations(ptd, oracle_mod, dt, n, R, hermitian):
    """sum_j <u_j|P|u_j> / 2^n over the factor's columns: sampled against the
    oracle on U U^* (n <= 12), real (imaginary parts exactly zero), and equal
    within the bar to the sum of the columns' pure-state decompositions."""
    import torch

    N = 1 << n
    U = synth.complex_normal((N, R), seed=800 + n, dtype=_np_dtype(dt))
    Ud = to_dev(U)
    got = ptd.decompose(Ud, low_rank=True, hermitian=hermitian)
    if not hermitian:
        assert float(got.imag.abs().max()) == 0.0
    xs, zs = synth.sample_strings(n, 500, seed=17)
    ix, iz = to_dev(xs.astype(np.int64)), to_dev(zs.astype(np.int64))
    if n <= 12:
        want = oracle_mod.coeffs(oracle_mod.mixed_density(U), xs, zs)
        assert rel_err(to_host(got[ix, iz]), want.real if hermitian else want) <= TOL[dt]
    acc = None
    for j in range(min(R, 4)):
        cj = ptd.decompose(Ud[:, j].contiguous(), pure_state=True, hermitian=True).to(torch.float64)
        acc = cj if acc is None else acc + cj
    if R <= 4:
        ref = got if hermitian else got.real
        assert rel_err(to_host(ref.to(torch.float64)), to_host(acc)) <= TOL[dt]
    del got, acc
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [4, 9, 12, 14])
def test_rank_one_is_the_pure_state(ptd, dt, n):
    """A one-column factor forms each entry with the pure state's products
    (plus an exact zero), so both calls agree bit for bit; and a factor with
    a row pitch wider than its rank reads the same values."""
    import torch

    N = 1 << n
    psi = synth.complex_normal(N, seed=820 + n, dtype=_np_dtype(dt))
    pd = to_dev(psi)
    a = ptd.decompose(pd[:, None], low_rank=True, hermitian=True)
    b = ptd.decompose(pd, pure_state=True, hermitian=True)
    assert bool(torch.equal(a, b))
    wide = torch.zeros((N, 5), dtype=pd.dtype, device=pd.device)
    wide[:, 1] = pd
    wide[:, 2] = 2 * pd
    c1 = ptd.decompose(wide[:, 1:3], low_rank=True)  # row pitch 5, rank 2
    c2 = ptd.decompose(wide[:, 1:3].contiguous(), low_rank=True)
    assert bool(torch.equal(c1, c2))
    del a, b, c1, c2, wide
    torch.cuda.empty_cache()


def test_mixed_state_n15_complex64(ptd):
    """n = 15 complex64 (two halves per row) for the state-vector sources: a
    one-column factor gives the pure-state bits, and a two-column factor the
    sum of its columns' expectation values within the bar."""
    import torch

    n, N = 15, 1 << 15
    U = to_dev(synth.complex_normal((N, 2), seed=830, dtype=np.complex64))
    p0 = ptd.decompose(U[:, 0].contiguous(), pure_state=True, hermitian=True)
    a = ptd.decompose(U[:, :1], low_rank=True, hermitian=True)
    assert bool(torch.equal(a, p0))
    del a
    p1 = ptd.decompose(U[:, 1].contiguous(), pure_state=True, hermitian=True)
    both = ptd.decompose(U, low_rank=True, hermitian=True)
    xs, zs = synth.sample_strings(n, 4000, seed=19)
    ix, iz = to_dev(xs.astype(np.int64)), to_dev(zs.astype(np.int64))
    want = p0[ix, iz].double() + p1[ix, iz].double()
    assert rel_err(to_host(both[ix, iz].double()), to_host(want)) <= TOL["c64"]
    del p0, p1, both
    torch.cuda.empty_cache()


# --------------------------------------------------------------------------
# the n = 13 Hermitian workload against the full oracle (every coefficient;
# about 50 s of host time each on 16 cores)

@pytest.mark.slow
def test_n13_hermitian_every_coefficient(ptd, oracle_mod):
    n = 13
    A = synth.hermitian(n, seed=0)
    Ad = to_dev(A)
    real = to_host(ptd.decompose(Ad, hermitian=True))
    full = to_host(ptd.decompose(Ad))
    del Ad
    want = oracle_mod.decompose(A)
    assert rel_err(real, want.real) <= 1e-12
    assert rel_err(full, want) <= 1e-12
    assert np.all(full.imag == 0.0)


@pytest.mark.slow
def test_n13_gaussian_integer_every_coefficient(ptd, oracle_mod):
    """2^n c_P as exact int64 for all 4^13 strings, through the complex128 and
    complex64 Hermitian paths."""
    import torch

    n = 13
    re, im = synth.gaussian_int_hermitian(n, seed=1)
    Ad = to_dev(synth.int_to_complex(re, im, np.complex128))
    g128 = to_host(ptd.decompose(Ad, hermitian=True)) * (1 << n)
    g64 = to_host(ptd.decompose(Ad.to(torch.complex64), hermitian=True)).astype(np.float64) * (1 << n)
    del Ad
    cre, cim = oracle_mod.decompose_int(re, im)
    assert np.all(cim == 0)
    np.testing.assert_array_equal(g128, cre.astype(np.float64))
    np.testing.assert_array_equal(g64, cre.astype(np.float64))
