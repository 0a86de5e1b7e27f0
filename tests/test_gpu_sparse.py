"""GPU parity of the sparse-input path: the X-pattern set r ^ c of the
entries, and the coefficients of those rows, against the oracle on the
assembled matrix (rows not listed must be exactly zero)."""
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


def _entries(n, nnz, seed, dt, clustered=False):
    N = 1 << n
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, N, size=nnz).astype(np.int32)
    if clustered:  # a band-like pattern plus scattered entries: few X-patterns
        cols = np.clip(rows + rng.integers(-3, 4, size=nnz), 0, N - 1).astype(np.int32)
    else:
        cols = rng.integers(0, N, size=nnz).astype(np.int32)
    vals = synth.complex_normal(nnz, seed=seed + 1, dtype=dt)
    return rows, cols, vals


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
@pytest.mark.parametrize("n,clustered", [(1, False), (2, False), (5, False), (9, True), (10, False), (11, True),
                                         (12, False), (13, True)])
@pytest.mark.parametrize("compact", [True, False])
def test_sparse_vs_oracle(ptd, oracle_mod, dt, n, clustered, compact):
    N = 1 << n
    rows, cols, vals = _entries(n, 3 * N, 500 + n, dt, clustered)
    got, xs = ptd.decompose_sparse(to_dev(rows), to_dev(cols), to_dev(vals), n, compact=compact)
    want_xs = oracle_mod.sparse_nonempty_x(n, rows, cols)
    assert to_host(xs).tolist() == want_xs
    A = oracle_mod.sparse_to_dense(n, rows, cols, vals)
    # rows of the listed X-patterns (a sample of them beyond n = 10)
    pick = np.array(want_xs, dtype=np.uint32)
    if n > 10:
        pick = pick[np.random.default_rng(7).choice(len(pick), size=min(len(pick), 24), replace=False)]
    want = oracle_mod.rows(A, pick)
    g = to_host(got)
    if compact:
        assert g.shape == (len(want_xs), N)
        idx = np.searchsorted(np.array(want_xs), pick)
        assert rel_err(g[idx], want) <= TOL[dt]
    else:
        assert rel_err(g[pick.astype(np.int64)], want) <= TOL[dt]
        mask = np.ones(N, dtype=bool)
        mask[want_xs] = False
        assert np.all(g[mask] == 0)


@pytest.mark.parametrize("n", [3, 8, 11])
def test_sparse_integer_exact_with_repeats(ptd, oracle_mod, n):
    """Gaussian-integer entries, with repeated coordinates (summed) and
    entries outside the matrix (ignored): exact against the oracle."""
    N = 1 << n
    rng = np.random.default_rng(600 + n)
    nnz = 2 * N
    rows = rng.integers(0, N, size=nnz)
    cols = rng.integers(0, N, size=nnz)
    rows[:8] = rows[8:16]  # repeats
    cols[:8] = cols[8:16]
    rows[-3:] = [N, -1, 2]  # out of range
    cols[-3:] = [0, 1, N + 5]
    vals = (rng.integers(-8, 9, size=nnz) + 1j * rng.integers(-8, 9, size=nnz)).astype(np.complex64)
    got, xs = ptd.decompose_sparse(to_dev(rows.astype(np.int32)), to_dev(cols.astype(np.int32)), to_dev(vals), n)
    A = oracle_mod.sparse_to_dense(n, rows, cols, vals)
    wr, wi = oracle_mod.decompose_int(A.real.astype(np.int64), A.imag.astype(np.int64)) if n <= 8 else (None, None)
    g = to_host(got).astype(np.complex128) * N
    if wr is not None:
        np.testing.assert_array_equal(g.real, wr.astype(np.float64))
        np.testing.assert_array_equal(g.imag, wi.astype(np.float64))
    else:
        pick = to_host(xs)[:16].astype(np.uint32)
        np.testing.assert_array_equal(g[pick.astype(np.int64)], np.round(oracle_mod.rows(A, pick) * N))


def test_sparse_empty_and_bad_list(ptd):
    import torch

    from paper_2403_11644_amd import _native, api

    e32 = torch.empty(0, dtype=torch.int32, device="cuda")
    ev = torch.empty(0, dtype=torch.complex128, device="cuda")
    got, xs = ptd.decompose_sparse(e32, e32, ev, 4)
    assert xs.numel() == 0 and float(got.abs().max()) == 0.0
    got, xs = ptd.decompose_sparse(e32, e32, ev, 4, compact=True)
    assert got.shape == (0, 16) and xs.numel() == 0
    # a list that is not strictly ascending, or leaves the matrix, is refused
    # by the device-side check before anything is written
    L = _native.lib()
    wsb = L.ptd_sparse_workspace_bytes(4)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    out = torch.empty((16, 16), dtype=torch.complex128, device="cuda")
    for bad in ([3, 3], [5, 2], [1, 16]):
        xs_bad = torch.tensor(bad, dtype=torch.int32, device="cuda")
        st = L.pauli_decompose_sparse(4, api.C128, 0, 0, None, None, None, api._ptr(xs_bad), len(bad),
                                      api._ptr(out), api._ptr(ws), wsb, None)
        assert st == -1


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
def test_sparse_band_matches_structured(ptd, dt):
    """A band matrix given as sparse entries: the same X-patterns and the
    same rows as the band path (within rounding)."""
    n, s = 10, 3
    band = synth.banded_complex(n, s, seed=12, dtype=dt)
    A = synth.dense_from_bands(band)
    r, c = np.nonzero(A)
    v = A[r, c]
    got, xs = ptd.decompose_sparse(to_dev(r.astype(np.int32)), to_dev(c.astype(np.int32)), to_dev(v), n, compact=True)
    want = to_host(ptd.decompose(to_dev(band), structure="banded", s=s, bands=True, compact=True))
    assert to_host(xs).tolist() == ptd.nonempty_x(n, "banded", s)
    assert rel_err(to_host(got), want) <= TOL[dt]


# -- compressed-row (CSR) input ------------------------------------------------

def _csr(n, seed, dt, clustered=False, repeats=False, long_row=True):
    """A compressed-row matrix: row lengths 0..6 (some rows empty), one row
    longer than a wave (so a wave loops over it), columns near the diagonal
    when clustered; with repeats, row 0 repeats a column."""
    N = 1 << n
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, 7, size=N)
    if long_row and N >= 4:
        counts[N // 2] = min(N, 150)
    if repeats:
        counts[0] = max(counts[0], 3)
    row_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    nnz = int(row_ptr[-1])
    rows = np.repeat(np.arange(N), counts)
    if clustered:
        cols = np.clip(rows + rng.integers(-3, 4, size=nnz), 0, N - 1)
    else:
        cols = rng.integers(0, N, size=nnz)
    if repeats:
        cols[1] = cols[0]
    vals = synth.complex_normal(nnz, seed=seed + 1, dtype=dt)
    return row_ptr, cols.astype(np.int32), vals


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
@pytest.mark.parametrize("n,clustered", [(1, False), (2, False), (5, False), (9, True), (10, False), (11, True),
                                         (12, False), (13, True)])
@pytest.mark.parametrize("compact", [True, False])
def test_csr_vs_oracle(ptd, oracle_mod, dt, n, clustered, compact):
    N = 1 << n
    row_ptr, cols, vals = _csr(n, 700 + n, dt, clustered, repeats=True)
    got, xs = ptd.decompose_csr(to_dev(row_ptr), to_dev(cols), to_dev(vals), n, compact=compact)
    want_xs = oracle_mod.csr_nonempty_x(n, row_ptr, cols)
    assert to_host(xs).tolist() == want_xs
    A = oracle_mod.csr_to_dense(n, row_ptr, cols, vals)
    pick = np.array(want_xs, dtype=np.uint32)
    if n > 10:
        pick = pick[np.random.default_rng(8).choice(len(pick), size=min(len(pick), 24), replace=False)]
    want = oracle_mod.rows(A, pick)
    g = to_host(got)
    if compact:
        assert g.shape == (len(want_xs), N)
        idx = np.searchsorted(np.array(want_xs), pick)
        assert rel_err(g[idx], want) <= TOL[dt]
    else:
        assert rel_err(g[pick.astype(np.int64)], want) <= TOL[dt]
        mask = np.ones(N, dtype=bool)
        mask[want_xs] = False
        assert np.all(g[mask] == 0)


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
@pytest.mark.parametrize("n", [6, 12])
def test_csr_equals_coordinates(ptd, dt, n):
    """The same entries (no repeated coordinate) given as compressed rows and
    as coordinates: each output element receives one value either way, so
    the two calls agree bit for bit."""
    N = 1 << n
    rng = np.random.default_rng(710 + n)
    dense_mask = rng.random((N, N)) < min(1.0, 5.0 / N)
    dense_mask[N // 3, :] = True  # one full row
    r, c = np.nonzero(dense_mask)
    vals = synth.complex_normal(len(r), seed=711, dtype=dt)
    row_ptr = np.concatenate([[0], np.cumsum(dense_mask.sum(axis=1))]).astype(np.int64)
    a, xa = ptd.decompose_csr(to_dev(row_ptr), to_dev(c.astype(np.int32)), to_dev(vals), n)
    b, xb = ptd.decompose_sparse(to_dev(r.astype(np.int32)), to_dev(c.astype(np.int32)), to_dev(vals), n)
    assert to_host(xa).tolist() == to_host(xb).tolist()
    np.testing.assert_array_equal(to_host(a), to_host(b))


@pytest.mark.parametrize("n", [3, 8, 11])
def test_csr_integer_exact(ptd, oracle_mod, n):
    """Gaussian-integer entries with a repeated column and out-of-range
    columns: exact against the oracle."""
    N = 1 << n
    row_ptr, cols, _ = _csr(n, 720 + n, np.complex64, repeats=True)
    rng = np.random.default_rng(721 + n)
    nnz = len(cols)
    cols[-2:] = [N, -4]  # ignored
    vals = (rng.integers(-8, 9, size=nnz) + 1j * rng.integers(-8, 9, size=nnz)).astype(np.complex64)
    got, xs = ptd.decompose_csr(to_dev(row_ptr), to_dev(cols), to_dev(vals), n)
    A = oracle_mod.csr_to_dense(n, row_ptr, cols, vals)
    g = to_host(got).astype(np.complex128) * N
    if n <= 8:
        wr, wi = oracle_mod.decompose_int(A.real.astype(np.int64), A.imag.astype(np.int64))
        np.testing.assert_array_equal(g.real, wr.astype(np.float64))
        np.testing.assert_array_equal(g.imag, wi.astype(np.float64))
    else:
        pick = to_host(xs)[:16].astype(np.uint32)
        np.testing.assert_array_equal(g[pick.astype(np.int64)], np.round(oracle_mod.rows(A, pick) * N))


def test_csr_clipped_pointers(ptd, oracle_mod):
    """Row pointers outside [0, nnz) or decreasing: every range is clipped
    to the arrays on the device as the oracle defines it (the worked n = 2
    case of the oracle's pins, and pointers drawn at random at n = 8)."""
    import torch

    rp = np.array([0, 2, 5, -3, 9], dtype=np.int64)
    ci = np.array([1, 2, 0, 7], dtype=np.int32)
    va = np.array([1, 2j, 3, 4], dtype=np.complex128)
    got, xs = ptd.decompose_csr(to_dev(rp), to_dev(ci), to_dev(va), 2)
    assert to_host(xs).tolist() == [1, 2, 3]
    np.testing.assert_allclose(to_host(got), oracle_mod.decompose(oracle_mod.csr_to_dense(2, rp, ci, va)),
                               rtol=0, atol=1e-15)
    n = 8
    N = 1 << n
    rng = np.random.default_rng(730)
    nnz = 600
    rp = rng.integers(-50, nnz + 50, size=N + 1).astype(np.int64)
    rp[5], rp[6] = -(1 << 40), 1 << 40  # far outside: row 5 takes every entry
    ci = rng.integers(0, N, size=nnz).astype(np.int32)
    va = synth.complex_normal(nnz, seed=731, dtype=np.complex128)
    got, xs = ptd.decompose_csr(to_dev(rp), to_dev(ci), to_dev(va), n)
    assert to_host(xs).tolist() == oracle_mod.csr_nonempty_x(n, rp, ci)
    want = oracle_mod.decompose(oracle_mod.csr_to_dense(n, rp, ci, va))
    assert rel_err(to_host(got), want) <= 1e-12
    # nothing at all: an empty matrix, dense zeros or no compact rows
    rp0 = torch.zeros(N + 1, dtype=torch.int64, device="cuda")
    e32 = torch.empty(0, dtype=torch.int32, device="cuda")
    ev = torch.empty(0, dtype=torch.complex64, device="cuda")
    got, xs = ptd.decompose_csr(rp0, e32, ev, n)
    assert xs.numel() == 0 and float(got.abs().max()) == 0.0
    got, xs = ptd.decompose_csr(rp0, e32, ev, n, compact=True)
    assert got.shape == (0, N)


@pytest.mark.parametrize("dt", [np.complex128, np.complex64])
def test_sparse_and_csr_at_n16(ptd, oracle_mod, dt):
    """The largest size (n = 16): a tridiagonal matrix plus 64 scattered
    entries, as coordinates and as compressed rows, compact output.  The
    X-pattern lists equal the oracle's, the two forms agree bit for bit (no
    repeated coordinate), and sampled strings of every listed row equal the
    oracle's sum over the stored entries."""
    n = 16
    N = 1 << n
    rng = np.random.default_rng(740)
    r = np.repeat(np.arange(N), 3)
    c = r + np.tile(np.array([-1, 0, 1]), N)
    keep = (c >= 0) & (c < N)
    r, c = r[keep], c[keep]
    sr = rng.integers(0, N, size=64)
    sc = (sr + rng.integers(2, N - 2, size=64)) % N  # off the three diagonals
    pairs = sorted(set(zip(sr.tolist(), sc.tolist())))
    r = np.append(r, [p[0] for p in pairs])
    c = np.append(c, [p[1] for p in pairs])
    vals = synth.complex_normal(len(r), seed=741, dtype=dt)
    want_xs = oracle_mod.sparse_nonempty_x(n, r, c)
    got, xs = ptd.decompose_sparse(to_dev(r.astype(np.int32)), to_dev(c.astype(np.int32)), to_dev(vals), n,
                                   compact=True)
    assert to_host(xs).tolist() == want_xs
    order = np.argsort(r, kind="stable")
    row_ptr = np.concatenate([[0], np.cumsum(np.bincount(r, minlength=N))]).astype(np.int64)
    got_csr, xs_csr = ptd.decompose_csr(to_dev(row_ptr), to_dev(c[order].astype(np.int32)), to_dev(vals[order]), n,
                                        compact=True)
    assert to_host(xs_csr).tolist() == want_xs
    g = to_host(got)
    np.testing.assert_array_equal(to_host(got_csr), g)
    zs = rng.integers(0, N, size=(len(want_xs), 4))
    xq = np.repeat(np.array(want_xs), 4)
    zq = zs.reshape(-1)
    want = oracle_mod.sparse_coeffs(n, r, c, vals, xq, zq)
    idx = np.repeat(np.arange(len(want_xs)), 4)
    assert rel_err(g[idx, zq], want) <= TOL[dt]
