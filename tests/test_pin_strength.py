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


# CP-ALS update: planted mistakes in a stand-in of the normal-equations step must fail
# the explicit Khatri-Rao least-squares pin.
def als_correct(X, U, n):
    M = correct(X, U, 0)
    V = (U[1].T @ U[1]) * (U[2].T @ U[2])
    A = np.linalg.solve(V, M.T).T
    return A / np.sqrt(np.sum(A * A, axis=0))


def _als_with(gram_fn, solve_fn):
    def fn(X, U, n):
        M = correct(X, U, 0)
        A = solve_fn(gram_fn(U), M)
        return A / np.sqrt(np.sum(A * A, axis=0))
    return fn


ALS_MUTANTS = {
    "gram_dropped": _als_with(lambda U: U[1].T @ U[1], lambda V, M: np.linalg.solve(V, M.T).T),
    "gram_sum_not_hadamard": _als_with(lambda U: U[1].T @ U[1] + U[2].T @ U[2], lambda V, M: np.linalg.solve(V, M.T).T),
    "gram_outer_not_inner": _als_with(lambda U: (U[1] @ U[1].T)[:3, :3] * (U[2] @ U[2].T)[:3, :3],
                                      lambda V, M: np.linalg.solve(V, M.T).T),
    "multiplies_not_solves": _als_with(lambda U: (U[1].T @ U[1]) * (U[2].T @ U[2]), lambda V, M: M @ V),
    "solve_transposed_side": _als_with(lambda U: (U[1].T @ U[1]) * (U[2].T @ U[2]) + np.triu(np.ones((3, 3)), 1),
                                       lambda V, M: np.linalg.solve(V, M.T).T),
}


def lstsq_pin(fn):
    rng = np.random.default_rng(3)
    X = rng.standard_normal((6, 5, 7))
    U = [None, rng.standard_normal((5, 3)), rng.standard_normal((7, 3))]
    KR = (U[1][:, None, :] * U[2][None, :, :]).reshape(-1, 3)
    A = np.linalg.lstsq(KR, X.reshape(6, -1).T, rcond=None)[0].T
    return nrel(fn(X, U, 0), A / np.sqrt(np.sum(A * A, axis=0))) <= 1e-10


def test_als_pin_accepts_the_definition():
    assert lstsq_pin(als_correct)


def test_als_pin_rejects_planted_mistakes():
    for name, fn in ALS_MUTANTS.items():
        assert not lstsq_pin(fn), name
