"""The oracle's pins must be able to fail.

Plausible mistakes are planted in small CPU stand-ins of the MTTKRP
definition (a dropped factor, a wrong index, a transposed operand, a sign
error, an accumulate-instead-of-overwrite), and each must be rejected by at
least one of the closed-form pins used on the oracle.
"""
import numpy as np


def nrel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def correct(X, U, n):
    return np.einsum("ijk,ja,ka->ia", X, U[1], U[2])


MUTANTS = {
    "dropped_factor": lambda X, U, n: np.einsum("ijk,ja->ia", X, U[1]),
    "wrong_index": lambda X, U, n: np.einsum("ijk,ka,ka->ia", X, U[1][: X.shape[2]], U[2]),
    "transposed_operand": lambda X, U, n: np.einsum("ikj,ja,ka->ia", X, U[1], U[2]),
    "sign_error": lambda X, U, n: -np.einsum("ijk,ja,ka->ia", X, U[1], U[2]),
    "accumulates_into_output": lambda X, U, n: 1.0 + np.einsum("ijk,ja,ka->ia", X, U[1], U[2]),
}


def rank1_pin(fn):
    rng = np.random.default_rng(1)
    a, b, c = rng.standard_normal(6), rng.standard_normal(6), rng.standard_normal(6)
    X = np.multiply.outer(np.multiply.outer(a, b), c)
    U = [None, rng.standard_normal((6, 3)), rng.standard_normal((6, 3))]
    return nrel(fn(X, U, 0), np.outer(a, (b @ U[1]) * (c @ U[2]))) <= 1e-12


def kruskal_pin(fn):
    rng = np.random.default_rng(2)
    A1, B1, C1 = (rng.standard_normal((6, 2)) for _ in range(3))
    X = np.einsum("iq,jq,kq->ijk", A1, B1, C1)
    U = [None, rng.standard_normal((6, 3)), rng.standard_normal((6, 3))]
    return nrel(fn(X, U, 0), A1 @ ((B1.T @ U[1]) * (C1.T @ U[2]))) <= 1e-12


def test_pins_accept_the_definition():
    assert rank1_pin(correct) and kruskal_pin(correct)


def test_pins_reject_planted_mistakes():
    for name, fn in MUTANTS.items():
        assert not (rank1_pin(fn) and kruskal_pin(fn)), name
