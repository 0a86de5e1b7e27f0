"""Pins for the CPU oracle: values and identities fixed by the paper and by
mathematics, independent of the oracle's own code.  CPU only.

Each test names the passage of the paper it follows.  Together they catch the
plausible slips: a wrong letter table or Y sign (n=1 closed forms, worked
examples), a transposed operand in the trace (worked example with an
asymmetric corner entry, textbook comparison), a wrong qubit order (Kronecker
factorisation, direct sum, labels), a dropped or mis-scaled term (Parseval,
one-hot, reconstruction) and a wrong structured support (diagonal,
tridiagonal and band tests).
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


def _index_of_label(lab):
    n = len(lab)
    x = z = 0
    for j, ch in enumerate(lab):
        q = n - 1 - j
        xb, zb = {"I": (0, 0), "X": (1, 0), "Y": (1, 1), "Z": (0, 1)}[ch]
        x |= xb << q
        z |= zb << q
    return x, z


# -- Sec. I letter matrices and the Sec. II-A formula, by hand ---------------

def test_worked_examples(oracle_mod):
    data = json.load(open(GOLDEN))
    for ex in data["examples"]:
        M = np.array(ex["matrix"], dtype=np.float64)
        A = M[..., 0] + 1j * M[..., 1]
        n = A.shape[0].bit_length() - 1
        want = np.zeros((1 << n, 1 << n), dtype=np.complex128)
        for lab, (re, im) in ex["coefficients"].items():
            x, z = _index_of_label(lab)
            want[x, z] = re + 1j * im
        got = oracle_mod.decompose(A, nthreads=1)
        np.testing.assert_array_equal(got, want, err_msg=ex["name"])
        np.testing.assert_allclose(oracle_mod.decompose_textbook(A), want, atol=0, rtol=0,
                                   err_msg=ex["name"])


def test_n1_closed_forms(oracle_mod):
    rng = np.random.default_rng(5)
    for _ in range(20):
        a, b, c, d = rng.standard_normal(4) + 1j * rng.standard_normal(4)
        A = np.array([[a, b], [c, d]])
        got = oracle_mod.decompose(A, nthreads=1)
        # c[x, z]: I=(0,0), Z=(0,1), X=(1,0), Y=(1,1)
        np.testing.assert_allclose(got[0, 0], (a + d) / 2, rtol=1e-15, atol=1e-15)
        np.testing.assert_allclose(got[0, 1], (a - d) / 2, rtol=1e-15, atol=1e-15)
        np.testing.assert_allclose(got[1, 0], (b + c) / 2, rtol=1e-15, atol=1e-15)
        np.testing.assert_allclose(got[1, 1], 1j * (b - c) / 2, rtol=1e-15, atol=1e-15)


def test_labels():
    from oracle import oracle as O

    assert O.label(1, 3, 2) == "ZY"
    assert O.label(0, 0, 3) == "III"
    assert O.label(4, 0, 3) == "XII"
    assert O.label(1, 1, 3) == "IIY"
    for n in (1, 2, 3):
        for x in range(1 << n):
            for z in range(1 << n):
                assert _index_of_label(O.label(x, z, n)) == (x, z)


# -- Sec. II-B PauliComposer vs the Kronecker definition ---------------------

@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_composer_matches_kron(oracle_mod, n):
    N = 1 << n
    for x in range(N):
        for z in range(N):
            lab = oracle_mod.label(x, z, n)
            k1, m1 = oracle_mod.pauli_sparse(lab, "composer")
            k2, m2 = oracle_mod.pauli_sparse(lab, "kron")
            np.testing.assert_array_equal(k1, k2)
            np.testing.assert_array_equal(m1, m2)
            P = oracle_mod.pauli_matrix(lab)
            rows = np.arange(N)
            np.testing.assert_array_equal(P[rows, k1], m1)
            assert np.count_nonzero(P) == N
            # every row's nonzero sits at column j ^ x (the d-bits of the string)
            np.testing.assert_array_equal(k1, rows ^ x)


# -- the C oracle against np.kron + np.trace (Sec. II-A straightforward) -----

@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_oracle_vs_textbook(oracle_mod, n):
    A = synth.dense(n, seed=10 + n)
    got = oracle_mod.decompose(A)
    want = oracle_mod.decompose_textbook(A)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)


# -- Theorem 1: orthogonality -> one-hot, reconstruction, Parseval ----------

@pytest.mark.parametrize("n", [1, 2, 3])
def test_one_hot(oracle_mod, n):
    N = 1 << n
    for x in range(N):
        for z in range(N):
            P = oracle_mod.pauli_matrix(oracle_mod.label(x, z, n))
            c = oracle_mod.decompose(P, nthreads=1)
            want = np.zeros((N, N), dtype=np.complex128)
            want[x, z] = 1.0
            np.testing.assert_array_equal(c, want)


def test_reconstruction(oracle_mod):
    for n in (2, 3, 5):
        A = synth.dense(n, seed=20 + n)
        c = oracle_mod.decompose(A)
        np.testing.assert_allclose(oracle_mod.reconstruct(c), A, rtol=0, atol=1e-13)
    A = synth.dense(2, seed=3)
    c = oracle_mod.decompose(A)
    np.testing.assert_allclose(oracle_mod.reconstruct_textbook(c), A, rtol=0, atol=1e-14)
    np.testing.assert_allclose(oracle_mod.reconstruct(c), oracle_mod.reconstruct_textbook(c),
                               rtol=0, atol=1e-14)


@pytest.mark.parametrize("n", [4, 7])
def test_parseval(oracle_mod, n):
    A = synth.dense(n, seed=30 + n)
    c = oracle_mod.decompose(A)
    lhs = oracle_mod.frobenius_sq(A)
    rhs = oracle_mod.coeff_energy(c, n)
    assert abs(lhs - rhs) <= 1e-12 * lhs


# -- Theorem 2: Hermitian -> real coefficients -------------------------------

def test_hermitian_real(oracle_mod):
    n = 6
    A = synth.hermitian(n, seed=0)
    c = oracle_mod.decompose(A)
    # sequential float64 sums: |Im c| bounded by 2^-n * N * eps * sum|A| per row
    bound = 2.0 ** -n * (1 << n) * np.finfo(np.float64).eps * np.abs(A).sum()
    assert np.max(np.abs(c.imag)) <= bound
    assert np.max(np.abs(c.real)) > 0.01


def test_hermitian_int_exact(oracle_mod):
    n = 5
    re, im = synth.gaussian_int_hermitian(n, seed=1)
    A = synth.int_to_complex(re, im)
    np.testing.assert_array_equal(A, A.conj().T)
    cre, cim = oracle_mod.decompose_int(re, im)
    assert np.all(cim == 0)
    np.testing.assert_array_equal(cre.astype(np.float64), np.round(oracle_mod.decompose(A).real * (1 << n)))


def test_real_symmetric_odd_y_vanish(oracle_mod):
    # a real symmetric matrix has no strings with an odd number of Y letters
    n = 5
    rng = np.random.default_rng(4)
    B = rng.standard_normal((1 << n, 1 << n))
    A = (B + B.T).astype(np.complex128)
    c = oracle_mod.decompose(A)
    N = 1 << n
    odd = np.array([[bin(x & z).count("1") & 1 for z in range(N)] for x in range(N)], dtype=bool)
    assert np.max(np.abs(c[odd])) <= 1e-13
    assert np.max(np.abs(c[~odd].imag)) <= 1e-13


# -- integer mode ------------------------------------------------------------

def test_integer_mode_matches_float(oracle_mod):
    n = 6
    re, im = synth.gaussian_int(n, seed=7)
    cre, cim = oracle_mod.decompose_int(re, im)
    c = oracle_mod.decompose(synth.int_to_complex(re, im))
    np.testing.assert_array_equal(cre, np.round(c.real * (1 << n)).astype(np.int64))
    np.testing.assert_array_equal(cim, np.round(c.imag * (1 << n)).astype(np.int64))
    # the float result is itself exact here (small integers, power-of-two scale)
    np.testing.assert_array_equal(c.real * (1 << n), cre.astype(np.float64))


def test_sampled_mode(oracle_mod):
    n = 6
    A = synth.dense(n, seed=8)
    full = oracle_mod.decompose(A)
    xs, zs = synth.sample_strings(n, 500, seed=2)
    got = oracle_mod.coeffs(A, xs, zs)
    np.testing.assert_array_equal(got, full[xs, zs])
    # unsorted, repeated order
    perm = np.random.default_rng(1).permutation(len(xs))
    got2 = oracle_mod.coeffs(A, xs[perm], zs[perm])
    np.testing.assert_array_equal(got2, full[xs[perm], zs[perm]])


def test_row_mode(oracle_mod):
    n = 5
    A = synth.dense(n, seed=9)
    full = oracle_mod.decompose(A)
    xs = np.array([3, 0, 31, 3], dtype=np.uint32)
    np.testing.assert_array_equal(oracle_mod.rows(A, xs), full[xs])


# -- Sec. IV-A structured supports ------------------------------------------

def test_diagonal_is_walsh_hadamard(oracle_mod):
    n = 6
    d = synth.diagonal_real(n, seed=0)
    A = np.diag(d).astype(np.complex128)
    c = oracle_mod.decompose(A)
    N = 1 << n
    assert np.all(c[1:, :] == 0)
    H = scipy.linalg.hadamard(N)  # H[i, j] = (-1)^{popcount(i & j)}
    np.testing.assert_allclose(c[0, :], H @ d / N, rtol=0, atol=1e-14)


def test_tridiagonal_support(oracle_mod):
    n = 6
    a, b = synth.tridiag_real_sym(n, seed=1)
    A = synth.dense_from_bands(synth.bands_from_tridiag(a, b))
    c = oracle_mod.decompose(A)
    N = 1 << n
    nz_rows = sorted(set(np.nonzero(np.abs(c) > 1e-13)[0].tolist()))
    # Gamma_n: I/Z on the high qubits, X/Y on a block of low qubits -> x = 2^m - 1
    assert nz_rows == [(1 << m) - 1 for m in range(n + 1)]
    assert len(nz_rows) * N == (n + 1) * N  # at most (n+1) 2^n terms
    assert np.count_nonzero(np.abs(c) > 1e-13) <= (n + 1) * N


@pytest.mark.parametrize("n,s", [(5, 1), (6, 2), (6, 3), (7, 5), (8, 8)])
def test_band_support(oracle_mod, n, s):
    band = synth.banded_complex(n, s, seed=2)
    A = synth.dense_from_bands(band)
    c = oracle_mod.decompose(A)
    allowed = oracle_mod.nonempty_x_bruteforce(n, s)
    nz_rows = sorted(set(np.nonzero(np.abs(c) > 1e-13)[0].tolist()))
    assert set(nz_rows) <= set(allowed)
    # generic entries: every allowed x carries a nonzero coefficient
    assert nz_rows == allowed
    # the paper's bound (s n - c(s)) 2^n is attained by the support size
    assert len(allowed) * (1 << n) == oracle_mod.band_term_bound(n, s)


def test_antidiagonal_support(oracle_mod):
    # remark after the diagonal case (Sec. IV-A): replacing I, Z by X, Y, an
    # anti-diagonal matrix has coefficients only on strings with X or Y on
    # every qubit, x = 2^n - 1; brute force over the entries agrees
    n = 4
    N = 1 << n
    ad = synth.antidiagonal_complex(n, seed=80)
    c = oracle_mod.decompose(synth.dense_from_antidiagonal(ad))
    assert np.all(c[:N - 1] == 0) and np.any(c[N - 1] != 0)
    k = np.arange(N)
    xs = sorted({int(x) for x in (k ^ (N - 1 - k))})
    assert xs == [N - 1]


# -- Sec. IV-B combinations --------------------------------------------------

def test_kronecker_factorisation(oracle_mod):
    # Tr(A1^* B1 (x) ...) factorises (proof of Theorem 1): c(A (x) B) = c(A) (x) c(B)
    A = synth.dense(2, seed=40)
    B = synth.dense(3, seed=41)
    cA = oracle_mod.decompose(A)
    cB = oracle_mod.decompose(B)
    cAB = oracle_mod.decompose(np.kron(A, B))
    np.testing.assert_allclose(cAB, np.kron(cA, cB), rtol=0, atol=1e-14)


def _embed(blocks):
    """diag(blocks...) as a dense matrix."""
    N = blocks[0].shape[0]
    M = np.zeros((N * len(blocks), N * len(blocks)), dtype=np.complex128)
    for i, b in enumerate(blocks):
        M[i * N:(i + 1) * N, i * N:(i + 1) * N] = b
    return M


def test_direct_sum(oracle_mod):
    # the identity of Sec. IV-B (oracle.direct_sum) against the definition on
    # the assembled matrix
    n = 3
    A = synth.dense(n, seed=42)
    B = synth.dense(n, seed=43)
    N = 1 << n
    cA, cB, cC = (oracle_mod.decompose(M) for M in (A, B, _embed([A, B])))
    got = oracle_mod.direct_sum(cA, cB)
    np.testing.assert_allclose(got, cC, rtol=0, atol=1e-15)
    # I (x) (a+b)/2 + Z (x) (a-b)/2; the new qubit is the most significant one
    np.testing.assert_allclose(cC[:N, :N], (cA + cB) / 2, atol=1e-15)
    np.testing.assert_allclose(cC[:N, N:], (cA - cB) / 2, atol=1e-15)
    assert np.all(cC[N:, :] == 0) and np.all(got[N:, :] == 0)


@pytest.mark.parametrize("nblocks,k", [(2, 2), (4, 2), (8, 2), (8, 1), (32, 1)])
def test_block_diagonal_exact(oracle_mod, nblocks, k):
    # the paper's N = 8 example and others: pairwise direct sums of the
    # blocks' coefficients equal the decomposition of the assembled matrix,
    # exactly for Gaussian-integer blocks (2^(k+m) c is an integer)
    blocks_int = [synth.gaussian_int(k, seed=60 + i) for i in range(nblocks)]
    blocks = [synth.int_to_complex(re, im) for re, im in blocks_int]
    cs = [oracle_mod.decompose(b) for b in blocks]
    got = oracle_mod.block_diagonal(cs)
    M = _embed(blocks)
    re, im = oracle_mod.decompose_int(M.real.astype(np.int64), M.imag.astype(np.int64))
    scale = float(M.shape[0])
    np.testing.assert_array_equal(got.real * scale, re.astype(np.float64))
    np.testing.assert_array_equal(got.imag * scale, im.astype(np.float64))


def test_block_diagonal_is_a_transform_over_the_block_index(oracle_mod):
    # unrolled, the recursion is c'[x][(t << k) | z] = 2^-m sum_i
    # (-1)^popcount(t & i) c_i[x][z] (a Sylvester Hadamard transform over i,
    # scipy.linalg.hadamard), rows x >= 2^k zero
    from scipy.linalg import hadamard

    k, m = 2, 3
    K = 1 << k
    cs = [synth.complex_normal((K, K), seed=70 + i) for i in range(1 << m)]
    got = oracle_mod.block_diagonal(cs)
    H = hadamard(1 << m)
    stack = np.stack(cs)                          # [i][x][z]
    want = np.einsum("ti,ixz->xtz", H, stack) / (1 << m)
    np.testing.assert_allclose(got[:K].reshape(K, 1 << m, K), want, rtol=0, atol=1e-15)
    assert np.all(got[K:] == 0)


def test_hermitian_augmentation(oracle_mod):
    n = 3
    A = synth.dense(n, seed=44)
    N = 1 << n
    At = np.zeros((2 * N, 2 * N), dtype=np.complex128)
    At[:N, N:] = A.conj().T
    At[N:, :N] = A
    cA = oracle_mod.decompose(A)
    cT = oracle_mod.decompose(At)
    # X (x) Re(alpha) + Y (x) Im(alpha)
    np.testing.assert_allclose(oracle_mod.hermitian_augment(cA), cT.real, rtol=0, atol=1e-15)
    np.testing.assert_allclose(cT.imag, 0, atol=1e-15)
    np.testing.assert_allclose(cT[N:, :N], cA.real, atol=1e-15)
    np.testing.assert_allclose(cT[N:, N:], cA.imag, atol=1e-15)
    assert np.all(cT[:N, :] == 0)


def test_linearity(oracle_mod):
    n = 4
    A = synth.dense(n, seed=45)
    B = synth.dense(n, seed=46)
    mu = 0.3 - 1.7j
    cA, cB = oracle_mod.decompose(A), oracle_mod.decompose(B)
    np.testing.assert_allclose(oracle_mod.decompose(mu * A + B), mu * cA + cB, rtol=0, atol=1e-13)
    np.testing.assert_allclose(oracle_mod.linear_combination(mu, cA, cB), oracle_mod.decompose(mu * A + B),
                               rtol=0, atol=1e-13)
    # float32 arrays stay float32, with mu rounded to it
    got32 = oracle_mod.linear_combination(mu, cA.astype(np.complex64), cB.astype(np.complex64))
    assert got32.dtype == np.complex64
    np.testing.assert_allclose(got32, mu * cA + cB, rtol=0, atol=1e-5)


# -- Sec. VI-C: block-encoding by a linear combination of the strings --------

@pytest.mark.parametrize("hermitian", [False, True])
def test_lcu_amplitudes_block_encode(oracle_mod, hermitian):
    # PREP prepares sum_i sqrt(|alpha_i|/lambda) |i>, SELECT applies
    # (alpha_i/|alpha_i|) P_i; the top-left block of PREP^H SELECT PREP is
    # sum_i (|alpha_i|/lambda) (alpha_i/|alpha_i|) P_i = A / lambda.  So the
    # squared amplitudes, with the coefficients' phases put back and scaled by
    # lambda, must rebuild A by the textbook Kronecker expansion, and they
    # must form a unit vector.
    n = 3
    A = synth.hermitian(n, seed=81) if hermitian else synth.dense(n, seed=81)
    c = oracle_mod.decompose(A)
    amp, lam = oracle_mod.lcu_amplitudes(c.real if hermitian else c)
    assert abs(float(np.sum(amp ** 2)) - 1.0) <= 1e-14
    assert lam == pytest.approx(float(np.abs(c).sum()), rel=1e-15)
    phase = np.where(np.abs(c) > 0, c / np.where(np.abs(c) > 0, np.abs(c), 1), 0)
    back = oracle_mod.reconstruct_textbook(amp ** 2 * phase) * lam
    np.testing.assert_allclose(back, A, rtol=0, atol=1e-13)
    # an all-zero array has no normalisation: amplitudes zero, lambda zero
    z, lz = oracle_mod.lcu_amplitudes(np.zeros((4, 4), dtype=np.complex128))
    assert lz == 0.0 and np.all(z == 0)


def test_toeplitz_matrix(oracle_mod):
    # A[r][c] = t[c - r + N - 1] is scipy's Toeplitz matrix with first column
    # t[N-1], t[N-2], ..., t[0] and first row t[N-1], ..., t[2N-2]; its
    # decomposition has the Toeplitz structure's symmetry: conj-reversing t
    # gives A^H, whose coefficients are the conjugates (P Hermitian)
    n = 3
    N = 1 << n
    t = synth.complex_normal(2 * N - 1, seed=85)
    A = oracle_mod.toeplitz_matrix(t)
    np.testing.assert_array_equal(A, scipy.linalg.toeplitz(t[N - 1::-1], t[N - 1:]))
    cA = oracle_mod.decompose(A)
    cH = oracle_mod.decompose(oracle_mod.toeplitz_matrix(np.conj(t[::-1])))
    np.testing.assert_allclose(cH, np.conj(cA), rtol=0, atol=1e-15)


def test_sparse_support(oracle_mod):
    # any sparsity pattern: the rows x of nonzero coefficients are exactly the
    # r ^ c of the entries (generic values), the others are exactly zero
    n = 5
    N = 1 << n
    rng = np.random.default_rng(86)
    rows = rng.integers(0, N, size=12)
    cols = rng.integers(0, N, size=12)
    vals = rng.standard_normal(12) + 1j * rng.standard_normal(12)
    A = oracle_mod.sparse_to_dense(n, np.append(rows, [N, -1]), np.append(cols, [0, 3]), np.append(vals, [1, 1]))
    assert np.count_nonzero(A) == len({(r, c) for r, c in zip(rows, cols)})
    c = oracle_mod.decompose(A)
    nz = [x for x in range(N) if np.any(c[x] != 0)]
    assert nz == oracle_mod.sparse_nonempty_x(n, rows, cols)


def test_sparse_coeffs_from_entries(oracle_mod):
    # the sum over stored entries equals the dense oracle on the assembled
    # matrix (repeats, out-of-range entries, every string of a small case)
    n = 5
    N = 1 << n
    rng = np.random.default_rng(89)
    rows = rng.integers(0, N, size=40)
    cols = rng.integers(0, N, size=40)
    rows[:3], cols[:3] = rows[3:6], cols[3:6]  # repeats
    rows = np.append(rows, [N, -2])
    cols = np.append(cols, [1, 0])
    vals = rng.standard_normal(42) + 1j * rng.standard_normal(42)
    A = oracle_mod.sparse_to_dense(n, rows, cols, vals)
    xs, zs = np.divmod(np.arange(N * N), N)
    got = oracle_mod.sparse_coeffs(n, rows, cols, vals, xs, zs)
    np.testing.assert_allclose(got, oracle_mod.coeffs(A, xs, zs), rtol=0, atol=1e-14)


def test_csr_matches_scipy(oracle_mod):
    # compressed rows: the assembled matrix equals scipy's own conversion of
    # the same arrays (repeated columns in a row summed), and the X-pattern
    # list equals the one of the same entries given as coordinates
    import scipy.sparse

    n = 5
    N = 1 << n
    rng = np.random.default_rng(88)
    counts = rng.integers(0, 6, size=N)
    counts[0] = 3  # row 0 holds a repeated column
    counts[3] = 0  # an empty row
    row_ptr = np.concatenate([[0], np.cumsum(counts)])
    nnz = int(row_ptr[-1])
    col_idx = rng.integers(0, N, size=nnz)
    col_idx[1] = col_idx[0]
    vals = rng.standard_normal(nnz) + 1j * rng.standard_normal(nnz)
    want = scipy.sparse.csr_matrix((vals, col_idx, row_ptr), shape=(N, N)).toarray()
    np.testing.assert_array_equal(oracle_mod.csr_to_dense(n, row_ptr, col_idx, vals), want)
    rows = np.repeat(np.arange(N), counts)
    assert oracle_mod.csr_nonempty_x(n, row_ptr, col_idx) == oracle_mod.sparse_nonempty_x(n, rows, col_idx)
    c = oracle_mod.decompose(want)
    assert [x for x in range(N) if np.any(c[x] != 0)] == oracle_mod.csr_nonempty_x(n, row_ptr, col_idx)


def test_csr_clipped_ranges(oracle_mod):
    # out-of-range pointers and columns, worked by hand (n = 2, nnz = 4,
    # row_ptr = [0, 2, 5, -3, 9]): row 0 takes entries 0, 1; row 1's range
    # [2, 5) clips to [2, 4), and entry 3's column 7 lies outside the
    # matrix; row 2's range [5, -3) clips to [4, 4), empty; row 3's range
    # [-3, 9) clips to [0, 4), all four entries again
    row_ptr = [0, 2, 5, -3, 9]
    col_idx = [1, 2, 0, 7]
    vals = np.array([1, 2j, 3, 4], dtype=np.complex128)
    rows, cols, vs = oracle_mod.csr_to_coo(2, row_ptr, col_idx, vals)
    assert rows.tolist() == [0, 0, 1, 1, 3, 3, 3, 3]
    assert cols.tolist() == [1, 2, 0, 7, 1, 2, 0, 7]
    assert vs.tolist() == [1, 2j, 3, 4, 1, 2j, 3, 4]
    want = np.zeros((4, 4), dtype=np.complex128)
    want[0, 1], want[0, 2], want[1, 0] = 1, 2j, 3
    want[3, 1], want[3, 2], want[3, 0] = 1, 2j, 3
    np.testing.assert_array_equal(oracle_mod.csr_to_dense(2, row_ptr, col_idx, vals), want)
    assert oracle_mod.csr_nonempty_x(2, row_ptr, col_idx) == [1, 2, 3]


def test_pure_state_expectations(oracle_mod):
    # the coefficients of |psi><psi| are <psi|P|psi> / 2^n (textbook: P from
    # np.kron applied to psi), real; c_I = |psi|^2 / 2^n and Parseval gives
    # 2^n sum |c|^2 = |psi|^4
    n = 3
    N = 1 << n
    psi = synth.complex_normal(N, seed=87)
    c = oracle_mod.decompose(oracle_mod.pure_density(psi))
    for x in range(N):
        for z in range(N):
            P = oracle_mod.pauli_matrix(oracle_mod.label(x, z, n))
            assert abs(c[x, z] - np.vdot(psi, P @ psi) / N) <= 1e-14
    np.testing.assert_allclose(c.imag, 0, atol=1e-15)
    nrm = float(np.vdot(psi, psi).real)
    assert c[0, 0].real == pytest.approx(nrm / N, rel=1e-14)
    assert N * float(np.sum(np.abs(c) ** 2)) == pytest.approx(nrm ** 2, rel=1e-13)


def test_mixed_state_expectations(oracle_mod):
    # U U^* over three columns: the coefficients are the sums over the
    # columns of <u_r|P|u_r> / 2^n (textbook P from np.kron), real; one column
    # gives the pure state's density matrix
    n, R = 3, 3
    N = 1 << n
    U = synth.complex_normal((N, R), seed=88)
    c = oracle_mod.decompose(oracle_mod.mixed_density(U))
    for x in range(N):
        for z in range(N):
            P = oracle_mod.pauli_matrix(oracle_mod.label(x, z, n))
            want = sum(np.vdot(U[:, r], P @ U[:, r]) for r in range(R)) / N
            assert abs(c[x, z] - want) <= 1e-14
    np.testing.assert_allclose(c.imag, 0, atol=1e-15)
    np.testing.assert_array_equal(oracle_mod.mixed_density(U[:, :1]), oracle_mod.pure_density(U[:, 0]))


def test_maximally_mixed_state(oracle_mod):
    # U = I / 2 on two qubits: rho = I / 4 exactly, so only the identity
    # string survives, with Tr(rho) / 2^n = 1/4
    n = 2
    U = np.eye(4, dtype=np.complex128) / 2
    c = oracle_mod.decompose(oracle_mod.mixed_density(U))
    want = np.zeros((4, 4), dtype=np.complex128)
    want[0, 0] = 0.25
    np.testing.assert_array_equal(c, want)
