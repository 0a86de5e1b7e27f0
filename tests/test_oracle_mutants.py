"""Planted mistakes: each mutant below is the oracle with one plausible slip
(a transposed operand in the trace of Algorithm 2, the Y phase of Sec. II-B
with the wrong sign, a dropped 2^-n, x and z swapped in the layout, the
qubit order reversed, a dropped term of the sum, a shifted instead of
XOR-ed column index, the Z sign taken from the column instead of the row).
The pins of the oracle (worked examples, n = 1 closed forms, one-hot
outputs of Theorem 1, Parseval, real coefficients of Hermitian input) must
reject every one of them, while the oracle itself passes.  The same holds
for the sparse-input functions: a compressed-row reader whose row ranges
end one short or are not clipped, and a sum over stored entries with the
sign taken from the column or without the i^p phase, each fail a pin
(scipy's compressed-row conversion, the hand-worked clipped case, the
dense oracle).  CPU only."""
import json
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")
LETTERS = {"I": (0, 0), "X": (1, 0), "Y": (1, 1), "Z": (0, 1)}


def _index_of_label(lab):
    n = len(lab)
    x = z = 0
    for j, ch in enumerate(lab):
        xb, zb = LETTERS[ch]
        x |= xb << (n - 1 - j)
        z |= zb << (n - 1 - j)
    return x, z


def _pc(v):
    return bin(int(v)).count("1")


# -- the pins, as predicates over a decomposition function -------------------

def pin_worked_examples(dec):
    for ex in json.load(open(GOLDEN))["examples"]:
        M = np.array(ex["matrix"], dtype=np.float64)
        A = M[..., 0] + 1j * M[..., 1]
        n = A.shape[0].bit_length() - 1
        want = np.zeros((1 << n, 1 << n), dtype=np.complex128)
        for lab, (re, im) in ex["coefficients"].items():
            want[_index_of_label(lab)] = re + 1j * im
        if not np.allclose(dec(A), want, rtol=0, atol=1e-14):
            return False
    return True


def pin_n1_closed_forms(dec):
    a, b, c, d = 0.3 - 1.1j, 2.0 + 0.5j, -0.7 + 0.2j, 1.5 - 0.4j
    got = dec(np.array([[a, b], [c, d]]))
    want = np.array([[(a + d) / 2, (a - d) / 2], [(b + c) / 2, 1j * (b - c) / 2]])
    return np.allclose(got, want, rtol=0, atol=1e-15)


def pin_one_hot(oracle_mod, dec):
    for n in (1, 2, 3):
        N = 1 << n
        for x in range(N):
            for z in range(N):
                want = np.zeros((N, N), dtype=np.complex128)
                want[x, z] = 1.0
                if not np.allclose(dec(oracle_mod.pauli_matrix(oracle_mod.label(x, z, n))), want, atol=1e-15):
                    return False
    return True


def pin_parseval(dec):
    A = synth.dense(3, seed=41)
    c = dec(A)
    return abs(8 * np.sum(np.abs(c) ** 2) - np.sum(np.abs(A) ** 2)) <= 1e-12 * np.sum(np.abs(A) ** 2)


def pin_hermitian_real(dec):
    A = synth.hermitian(3, seed=42)
    return np.max(np.abs(dec(A).imag)) <= 1e-14


def all_pins(oracle_mod, dec):
    return {
        "worked_examples": pin_worked_examples(dec),
        "n1_closed_forms": pin_n1_closed_forms(dec),
        "one_hot": pin_one_hot(oracle_mod, dec),
        "parseval": pin_parseval(dec),
        "hermitian_real": pin_hermitian_real(dec),
    }


# -- the mutants --------------------------------------------------------------

def _closed_form(A, col, sign_index):
    """2^-n i^popcount(x&z) sum_k (-1)^popcount(z & sign_index(k, x)) A[k][col(k, x)],
    with the column and the sign's index as given (the right ones are
    col = k ^ x and sign_index = k)."""
    N = A.shape[0]
    n = N.bit_length() - 1
    c = np.zeros((N, N), dtype=np.complex128)
    for x in range(N):
        for z in range(N):
            s = sum((-1) ** _pc(z & sign_index(k, x)) * A[k, col(k, x)] for k in range(N))
            c[x, z] = (1j ** (_pc(x & z) % 4)) * s / N
    return c


def _bitrev(v, n):
    return int(format(v, "0%db" % n)[::-1], 2) if n else v


def mutants(oracle_mod):
    O = oracle_mod

    def transposed(A):
        return O.decompose(np.ascontiguousarray(np.asarray(A).T), nthreads=1)

    def y_phase_sign(A):
        c = O.decompose(A, nthreads=1)
        N = c.shape[0]
        s = np.array([[(-1) ** _pc(x & z) for z in range(N)] for x in range(N)])
        return c * s

    def no_scale(A):
        c = O.decompose(A, nthreads=1)
        return c * c.shape[0]

    def swapped_xz(A):
        return np.ascontiguousarray(O.decompose(A, nthreads=1).T)

    def reversed_qubits(A):
        c = O.decompose(A, nthreads=1)
        N = c.shape[0]
        n = N.bit_length() - 1
        r = [_bitrev(v, n) for v in range(N)]
        return c[np.ix_(r, r)]

    def dropped_term(A):
        B = np.array(A, dtype=np.complex128)
        B[-1, :] = 0  # the sum over rows stops one short
        return O.decompose(B, nthreads=1)

    def shifted_column(A):
        A = np.asarray(A, dtype=np.complex128)
        N = A.shape[0]
        return _closed_form(A, lambda k, x: (k + x) % N, lambda k, x: k)

    def sign_from_column(A):
        A = np.asarray(A, dtype=np.complex128)
        return _closed_form(A, lambda k, x: k ^ x, lambda k, x: k ^ x)

    return {
        "transposed operand": transposed,
        "Y phase sign": y_phase_sign,
        "dropped 2^-n": no_scale,
        "x and z swapped": swapped_xz,
        "qubit order reversed": reversed_qubits,
        "dropped term": dropped_term,
        "shifted column index": shifted_column,
        "sign from the column index": sign_from_column,
    }


def test_the_oracle_passes_every_pin(oracle_mod):
    res = all_pins(oracle_mod, lambda A: oracle_mod.decompose(A, nthreads=1))
    assert all(res.values()), res


def test_the_closed_form_helper_is_the_oracle(oracle_mod):
    # with the right column and sign index the mutant generator is the oracle
    A = synth.dense(2, seed=43)
    np.testing.assert_allclose(_closed_form(A, lambda k, x: k ^ x, lambda k, x: k), oracle_mod.decompose(A),
                               rtol=0, atol=1e-15)


@pytest.mark.parametrize("name", ["transposed operand", "Y phase sign", "dropped 2^-n", "x and z swapped",
                                  "qubit order reversed", "dropped term", "shifted column index",
                                  "sign from the column index"])
def test_every_mutant_is_caught(oracle_mod, name):
    dec = mutants(oracle_mod)[name]
    res = all_pins(oracle_mod, dec)
    assert not all(res.values()), "%s passed every pin: %r" % (name, res)


# -- sparse input: the entry-based oracle functions and their pins -------------

def pin_csr_scipy(oracle_mod, to_coo):
    import scipy.sparse

    n, N = 5, 32
    rng = np.random.default_rng(90)
    counts = rng.integers(0, 6, size=N)
    counts[0], counts[3] = 3, 0
    row_ptr = np.concatenate([[0], np.cumsum(counts)])
    col = rng.integers(0, N, size=int(row_ptr[-1]))
    col[1] = col[0]
    vals = rng.standard_normal(len(col)) + 1j * rng.standard_normal(len(col))
    want = scipy.sparse.csr_matrix((vals, col, row_ptr), shape=(N, N)).toarray()
    return np.array_equal(oracle_mod.sparse_to_dense(n, *to_coo(n, row_ptr, col, vals)), want)


def pin_csr_clipped(oracle_mod, to_coo):
    rows, cols, _ = to_coo(2, [0, 2, 5, -3, 9], [1, 2, 0, 7], np.array([1, 2j, 3, 4], dtype=np.complex128))
    return rows.tolist() == [0, 0, 1, 1, 3, 3, 3, 3] and cols.tolist() == [1, 2, 0, 7, 1, 2, 0, 7]


def pin_sparse_coeffs(oracle_mod, coeffs):
    n, N = 4, 16
    rng = np.random.default_rng(91)
    rows, cols = rng.integers(0, N, size=30), rng.integers(0, N, size=30)
    vals = rng.standard_normal(30) + 1j * rng.standard_normal(30)
    xs, zs = np.divmod(np.arange(N * N), N)
    want = oracle_mod.coeffs(oracle_mod.sparse_to_dense(n, rows, cols, vals), xs, zs)
    return np.allclose(coeffs(n, rows, cols, vals, xs, zs), want, rtol=0, atol=1e-14)


def _csr_mutant(end_shift=0, clip_start=True):
    def to_coo(n, row_ptr, col_idx, vals):
        row_ptr = np.asarray(row_ptr, dtype=np.int64)
        col_idx = np.asarray(col_idx, dtype=np.int64)
        vals = np.asarray(vals)
        nnz = len(col_idx)
        rows, cols, vs = [], [], []
        for r in range(1 << n):
            lo = min(max(int(row_ptr[r]), 0), nnz) if clip_start else min(int(row_ptr[r]), nnz)
            hi = min(max(int(row_ptr[r + 1]) + end_shift, lo), nnz)
            for e in range(lo, hi):
                rows.append(r)
                cols.append(int(col_idx[e]))
                vs.append(vals[e])
        return np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64), np.array(vs, dtype=np.complex128)
    return to_coo


def _sparse_coeffs_mutant(sign_from_col=False, no_phase=False):
    def coeffs(n, rows, cols, vals, xs, zs):
        N = 1 << n
        rows, cols = np.asarray(rows, dtype=np.int64), np.asarray(cols, dtype=np.int64)
        vals = np.asarray(vals).astype(np.complex128)
        out = np.empty(len(xs), dtype=np.complex128)
        for i, (x, z) in enumerate(zip(xs, zs)):
            sel = (rows ^ cols) == int(x)
            idx = cols[sel] if sign_from_col else rows[sel]
            sgn = np.array([(-1) ** _pc(int(z) & int(k)) for k in idx])
            total = np.sum(sgn * vals[sel]) if len(idx) else 0.0
            ph = 1 if no_phase else 1j ** (_pc(int(x) & int(z)) % 4)
            out[i] = ph * total / N
        return out
    return coeffs


def test_sparse_oracle_passes_its_pins(oracle_mod):
    assert pin_csr_scipy(oracle_mod, oracle_mod.csr_to_coo)
    assert pin_csr_clipped(oracle_mod, oracle_mod.csr_to_coo)
    assert pin_sparse_coeffs(oracle_mod, oracle_mod.sparse_coeffs)
    # the mutant generators with no slip are the oracle
    assert pin_csr_scipy(oracle_mod, _csr_mutant()) and pin_csr_clipped(oracle_mod, _csr_mutant())
    assert pin_sparse_coeffs(oracle_mod, _sparse_coeffs_mutant())


@pytest.mark.parametrize("slip", ["row end one short", "start not clipped"])
def test_csr_mutants_are_caught(oracle_mod, slip):
    to_coo = _csr_mutant(end_shift=-1) if slip == "row end one short" else _csr_mutant(clip_start=False)
    assert not (pin_csr_scipy(oracle_mod, to_coo) and pin_csr_clipped(oracle_mod, to_coo))


@pytest.mark.parametrize("slip", ["sign from the column", "no i^p phase"])
def test_sparse_coeffs_mutants_are_caught(oracle_mod, slip):
    coeffs = _sparse_coeffs_mutant(sign_from_col=slip == "sign from the column", no_phase=slip == "no i^p phase")
    assert not pin_sparse_coeffs(oracle_mod, coeffs)
