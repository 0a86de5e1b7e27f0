"""Planted mistakes: each mutant below is the oracle with one plausible slip
(a transposed operand in the trace of Algorithm 2, the Y phase of Sec. II-B
with the wrong sign, a dropped 2^-n, x and z swapped in the layout, the
qubit order reversed, a dropped term of the sum, a shifted instead of
XOR-ed column index, the Z sign taken from the column instead of the row).
The pins of the oracle (worked examples, n = 1 closed forms, one-hot
outputs of Theorem 1, Parseval, real coefficients of Hermitian input) must
reject every one of them, while the oracle itself passes.  CPU only."""
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
