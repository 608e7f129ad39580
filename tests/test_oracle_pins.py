"""Pins for the CPU oracle: each check is fixed by the paper or by mathematics,
not by re-running the oracle's own formula.

  * hand-worked examples from the definitions (tests/golden/hand_examples.json)
  * brute force (pure-Python loops) and numpy.einsum on the Tab. IV strings
  * rank-1 and Kruskal closed forms, order-2 = GEMM, linearity
  * cross-mode invariant, MTTKRP vs TTMc relation, TTMc special cases
  * exact integer arithmetic, and the long-double bound on the oracle's own error
  * CP-ALS update: exact recovery of a Kruskal tensor's factor, and the same
    least-squares problem solved by numpy.linalg.lstsq on the explicit
    Khatri-Rao matrix (no normal equations)
"""
import itertools
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def nrel(a, b):
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm((np.asarray(a, dtype=np.float64) - b).ravel())
    s = np.linalg.norm(b.ravel())
    return d / s if s > 0 else d


def factors(rng, dims, R, skip):
    return [None if m == skip else rng.standard_normal((d, R)) for m, d in enumerate(dims)]


# ---------------------------------------------------------------- hand-worked
def test_hand_examples(oracle_mod):
    g = json.load(open(os.path.join(GOLDEN, "hand_examples.json")))
    X = np.array(g["X"], dtype=np.float64)
    for case in g["cases"]:
        n = case["mode"]
        U = [None] * 3
        for m, f in case["factors"].items():
            U[int(m)] = np.array(f, dtype=np.float64)
        if case["kind"] == "mttkrp":
            got = oracle_mod.mttkrp(X, U, n)
        else:
            got = oracle_mod.ttmc(X, U, n)
        assert np.array_equal(got, np.array(case["expect"], dtype=np.float64)), case["spec"]


# ---------------------------------------------------------------- brute force
def brute_mttkrp(X, U, n):
    dims = X.shape
    R = next(U[m].shape[1] for m in range(len(dims)) if m != n)
    M = [[0.0] * R for _ in range(dims[n])]
    for idx in itertools.product(*[range(d) for d in dims]):
        for r in range(R):
            p = X[idx]
            for m in range(len(dims)):
                if m != n:
                    p *= U[m][idx[m], r]
            M[idx[n]][r] += p
    return np.array(M)


def brute_ttmc(X, U, n):
    dims = X.shape
    N = len(dims)
    out_shape = [dims[m] if m == n else U[m].shape[1] for m in range(N)]
    Y = np.zeros(out_shape)
    for idx in itertools.product(*[range(d) for d in dims]):
        for ridx in itertools.product(*[range(out_shape[m]) if m != n else [None] for m in range(N)]):
            p = X[idx]
            for m in range(N):
                if m != n:
                    p *= U[m][idx[m], ridx[m]]
            o = tuple(idx[n] if m == n else ridx[m] for m in range(N))
            Y[o] += p
    return Y


TINY = [(3, 4), (3, 4, 5), (2, 3, 2, 3), (2, 3, 2, 3, 2)]


@pytest.mark.parametrize("dims", TINY)
@pytest.mark.parametrize("R", [1, 3])
def test_mttkrp_brute_force(oracle_mod, dims, R):
    rng = np.random.default_rng(11 + len(dims) + R)
    X = rng.uniform(-1, 1, dims)
    for n in range(len(dims)):
        U = factors(rng, dims, R, n)
        assert nrel(oracle_mod.mttkrp(X, U, n), brute_mttkrp(X, U, n)) <= 1e-14


@pytest.mark.parametrize("dims", [(3, 4, 5), (2, 3, 2, 3)])
def test_mttkrp_gemm_chain_brute_force(oracle_mod, dims):
    """Y[i_n, l] = sum over every other index and the rank of X * prod U * C[r, l], by loops;
    an identity C returns the MTTKRP itself."""
    rng = np.random.default_rng(21 + len(dims))
    X = rng.uniform(-1, 1, dims)
    R, L = 3, 2
    for n in range(len(dims)):
        U = factors(rng, dims, R, n)
        C = rng.standard_normal((R, L))
        Y = np.zeros((dims[n], L))
        for idx in np.ndindex(*dims):
            for r in range(R):
                p = X[idx]
                for m in range(len(dims)):
                    if m != n:
                        p *= U[m][idx[m], r]
                for l in range(L):
                    Y[idx[n], l] += p * C[r, l]
        assert nrel(oracle_mod.mttkrp_mm(X, U, n, C), Y) <= 1e-14
        assert np.array_equal(oracle_mod.mttkrp_mm(X, U, n, np.eye(R)), oracle_mod.mttkrp(X, U, n))


@pytest.mark.parametrize("dims", [(3, 4), (3, 4, 5), (2, 3, 2, 3)])
def test_ttmc_brute_force(oracle_mod, dims):
    rng = np.random.default_rng(5 + len(dims))
    X = rng.uniform(-1, 1, dims)
    for n in range(len(dims)):
        U = [None if m == n else rng.standard_normal((d, 2 + m % 2)) for m, d in enumerate(dims)]
        assert nrel(oracle_mod.ttmc(X, U, n), brute_ttmc(X, U, n)) <= 1e-14


# The einsum strings of Tab. IV, evaluated by numpy.einsum.
TAB4_MTTKRP = [
    ("ijk,ja,ka->ia", 0), ("ijk,ia,ka->ja", 1), ("ijk,ia,ja->ka", 2),
    ("ijklm,ja,ka,la,ma->ia", 0), ("ijklm,ia,ja,la,ma->ka", 2), ("ijklm,ia,ja,ka,la->ma", 4),
]


@pytest.mark.parametrize("spec,n", TAB4_MTTKRP)
def test_mttkrp_tab4_einsum(oracle_mod, spec, n):
    N = spec.index(",")
    dims = [5, 4, 6, 3, 7][:N] if N == 5 else [9, 7, 8]
    rng = np.random.default_rng(N * 10 + n)
    X = rng.uniform(-1, 1, dims)
    U = factors(rng, dims, 5, n)
    ref = np.einsum(spec, X, *[U[m] for m in range(N) if m != n], optimize=False)
    assert nrel(oracle_mod.mttkrp(X, U, n), ref) <= 1e-13


def test_ttmc_tab4_einsum(oracle_mod):
    dims = [4, 5, 3, 4, 3]
    rng = np.random.default_rng(77)
    X = rng.uniform(-1, 1, dims)
    U = [None] + [rng.standard_normal((d, r)) for d, r in zip(dims[1:], [2, 3, 2, 3])]
    ref = np.einsum("ijklm,jb,kc,ld,me->ibcde", X, *U[1:], optimize=False)
    assert nrel(oracle_mod.ttmc(X, U, 0), ref) <= 1e-13


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("dims", [(6, 5, 7), (4, 3, 5, 2), (3, 4, 2, 3, 2)])
def test_rank1_closed_form(oracle_mod, dims):
    """X = u_0 o u_1 o ... : M^(n) = u_n (x) prod_{m != n} (u_m^T U^m)."""
    rng = np.random.default_rng(3)
    u = [rng.standard_normal(d) for d in dims]
    X = u[0]
    for v in u[1:]:
        X = np.multiply.outer(X, v)
    R = 4
    for n in range(len(dims)):
        U = factors(rng, dims, R, n)
        h = np.ones(R)
        for m in range(len(dims)):
            if m != n:
                h = h * (u[m] @ U[m])
        assert nrel(oracle_mod.mttkrp(X, U, n), np.outer(u[n], h)) <= 1e-13


def test_kruskal_identity(oracle_mod):
    """X = sum_q a_q o b_q o c_q : M^(0) = A' ((B'^T B) * (C'^T C)), and cyclically."""
    rng = np.random.default_rng(4)
    I, J, K, Rp, R = 7, 6, 5, 3, 4
    A1, B1, C1 = rng.standard_normal((I, Rp)), rng.standard_normal((J, Rp)), rng.standard_normal((K, Rp))
    X = np.zeros((I, J, K))
    for q in range(Rp):
        X += np.multiply.outer(np.multiply.outer(A1[:, q], B1[:, q]), C1[:, q])
    A, B, C = rng.standard_normal((I, R)), rng.standard_normal((J, R)), rng.standard_normal((K, R))
    assert nrel(oracle_mod.mttkrp(X, [None, B, C], 0), A1 @ ((B1.T @ B) * (C1.T @ C))) <= 1e-13
    assert nrel(oracle_mod.mttkrp(X, [A, None, C], 1), B1 @ ((A1.T @ A) * (C1.T @ C))) <= 1e-13
    assert nrel(oracle_mod.mttkrp(X, [A, B, None], 2), C1 @ ((A1.T @ A) * (B1.T @ B))) <= 1e-13


def test_order2_is_gemm(oracle_mod):
    rng = np.random.default_rng(5)
    X = rng.standard_normal((13, 11))
    U0, U1 = rng.standard_normal((13, 6)), rng.standard_normal((11, 6))
    assert nrel(oracle_mod.mttkrp(X, [None, U1], 0), X @ U1) <= 1e-14
    assert nrel(oracle_mod.mttkrp(X, [U0, None], 1), X.T @ U0) <= 1e-14


def test_two_step_equivalence(oracle_mod):
    """Sec. II-A: MTTKRP equals the mode-0 unfolding of X times the Khatri-Rao product
    of the other factors, formed here as an explicit (J*K) x R matrix whose row j*K + k
    is the elementwise product of row j of B and row k of C."""
    rng = np.random.default_rng(6)
    I, J, K, R = 6, 5, 4, 3
    X = rng.standard_normal((I, J, K))
    B, C = rng.standard_normal((J, R)), rng.standard_normal((K, R))
    krp = np.empty((J * K, R))
    for j in range(J):
        for k in range(K):
            krp[j * K + k] = B[j] * C[k]
    assert nrel(oracle_mod.mttkrp(X, [None, B, C], 0), X.reshape(I, J * K) @ krp) <= 1e-14


def test_linearity(oracle_mod):
    rng = np.random.default_rng(7)
    dims = (5, 6, 4)
    X1, X2 = rng.standard_normal(dims), rng.standard_normal(dims)
    U = factors(rng, dims, 3, 1)
    a, b = 0.75, -1.5
    lhs = oracle_mod.mttkrp(a * X1 + b * X2, U, 1)
    rhs = a * oracle_mod.mttkrp(X1, U, 1) + b * oracle_mod.mttkrp(X2, U, 1)
    assert nrel(lhs, rhs) <= 1e-14
    V = [u.copy() if u is not None else None for u in U]
    W = [u.copy() if u is not None else None for u in U]
    W[2] = rng.standard_normal(U[2].shape)
    S = [u.copy() if u is not None else None for u in U]
    S[2] = a * V[2] + b * W[2]
    lhs = oracle_mod.mttkrp(X1, S, 1)
    rhs = a * oracle_mod.mttkrp(X1, V, 1) + b * oracle_mod.mttkrp(X1, W, 1)
    assert nrel(lhs, rhs) <= 1e-14


def test_cross_mode_invariant(oracle_mod):
    """sum_{i_n, r} M^(n)[i_n, r] U^n[i_n, r] = <X, [[U^0..U^{N-1}]]> for every n."""
    rng = np.random.default_rng(8)
    dims = (4, 5, 3, 6)
    X = rng.standard_normal(dims)
    R = 3
    U = [rng.standard_normal((d, R)) for d in dims]
    full = np.einsum("ijkl,ia,ja,ka,la->", X, *U)
    for n in range(4):
        Un = list(U)
        Un[n] = None
        v = float(np.sum(oracle_mod.mttkrp(X, Un, n) * U[n]))
        assert abs(v - full) <= 1e-12 * max(1.0, abs(full))


def test_mttkrp_equals_ttmc_diagonal(oracle_mod):
    """Order 3, shared factors: M[i, r] = Y[i, r, r]."""
    rng = np.random.default_rng(9)
    X = rng.standard_normal((6, 7, 5))
    B, C = rng.standard_normal((7, 4)), rng.standard_normal((5, 4))
    M = oracle_mod.mttkrp(X, [None, B, C], 0)
    Y = oracle_mod.ttmc(X, [None, B, C], 0)
    assert nrel(M, np.einsum("irr->ir", Y)) <= 1e-14


# ---------------------------------------------------------------- TTM / TTMc special cases
def test_ttm_is_tensordot(oracle_mod):
    rng = np.random.default_rng(10)
    X = rng.standard_normal((4, 5, 6))
    for m in range(3):
        Um = rng.standard_normal((X.shape[m], 3))
        ref = np.moveaxis(np.tensordot(X, Um, axes=([m], [0])), -1, m)
        assert nrel(oracle_mod.ttm(X, Um, m), ref) <= 1e-14


def test_ttmc_identity_returns_x(oracle_mod):
    rng = np.random.default_rng(12)
    X = rng.standard_normal((4, 5, 3, 2))
    for n in range(4):
        U = [None if m == n else np.eye(d) for m, d in enumerate(X.shape)]
        assert np.array_equal(oracle_mod.ttmc(X, U, n), X)


def test_ttmc_permutation_factors(oracle_mod):
    rng = np.random.default_rng(13)
    X = rng.standard_normal((4, 5, 6))
    p1, p2 = rng.permutation(5), rng.permutation(6)
    P1, P2 = np.eye(5)[:, p1], np.eye(6)[:, p2]  # P[i, r] = 1 iff i == p[r]
    Y = oracle_mod.ttmc(X, [None, P1, P2], 0)
    assert np.array_equal(Y, X[:, p1][:, :, p2])


def test_ttmc_orthogonal_preserves_norm(oracle_mod):
    rng = np.random.default_rng(14)
    X = rng.standard_normal((5, 6, 7))
    Q1, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    Q2, _ = np.linalg.qr(rng.standard_normal((7, 7)))
    Y = oracle_mod.ttmc(X, [None, Q1, Q2], 0)
    assert abs(np.linalg.norm(Y) - np.linalg.norm(X)) <= 1e-13 * np.linalg.norm(X)


def test_ttmc_tucker_closed_form(oracle_mod):
    """X = G x_0 V0 x_1 V1 x_2 V2 with orthonormal V: TTMc(X, V1, V2; mode 0) = G x_0 V0."""
    rng = np.random.default_rng(15)
    G = rng.standard_normal((3, 4, 2))
    V = [np.linalg.qr(rng.standard_normal((d, r)))[0] for d, r in [(7, 3), (9, 4), (8, 2)]]
    X = np.einsum("abc,ia,jb,kc->ijk", G, *V)
    Y = oracle_mod.ttmc(X, [None, V[1], V[2]], 0)
    assert nrel(Y, np.einsum("abc,ia->ibc", G, V[0])) <= 1e-13


def test_ttmc_rank1_closed_form(oracle_mod):
    rng = np.random.default_rng(16)
    a, b, c = rng.standard_normal(5), rng.standard_normal(6), rng.standard_normal(7)
    X = np.multiply.outer(np.multiply.outer(a, b), c)
    B, C = rng.standard_normal((6, 3)), rng.standard_normal((7, 4))
    ref = np.multiply.outer(np.multiply.outer(a, b @ B), c @ C)
    assert nrel(oracle_mod.ttmc(X, [None, B, C], 0), ref) <= 1e-13


# ---------------------------------------------------------------- exact arithmetic
def test_integer_inputs_exact(oracle_mod):
    """Integer X, U in {-2..2}: every partial sum is a small integer, so FP64 is exact."""
    rng = np.random.default_rng(17)
    dims = (9, 8, 7)
    X = rng.integers(-2, 3, dims)
    U = [rng.integers(-2, 3, (d, 4)) for d in dims]
    for n in range(3):
        Un = [None if m == n else U[m] for m in range(3)]
        spec = {0: "ijk,ja,ka->ia", 1: "ijk,ia,ka->ja", 2: "ijk,ia,ja->ka"}[n]
        exact = np.einsum(spec, X, *[U[m] for m in range(3) if m != n])  # int64, exact
        got = oracle_mod.mttkrp(X.astype(float), [u.astype(float) if u is not None else None for u in Un], n)
        assert np.array_equal(got, exact.astype(float))


def test_long_double_bounds_oracle_error(oracle_mod, synth):
    """Small-config MTTKRP (64^3, R=16): FP64 oracle within 1e-14 of the 80-bit version."""
    dims = (64, 64, 64)
    X = synth.x_tensor(synth.config_seed(1, 0), dims)
    U = [None] + [synth.normal_factor(synth.config_seed(1, 1 + m), 64, 16) for m in (1, 2)]
    a = oracle_mod.mttkrp(X, U, 0)
    b = oracle_mod.mttkrp(X, U, 0, long_double=True)
    assert nrel(a, b) <= 1e-14


# ---------------------------------------------------------------- input generator
def test_splitmix64_known_answers(synth):
    g = json.load(open(os.path.join(GOLDEN, "splitmix64_kat.json")))
    s0 = g["streams"][0]
    got = synth.splitmix64_at(s0["seed"], np.arange(3, dtype=np.uint64))
    assert [int(v) for v in got] == [int(h, 16) for h in s0["outputs_hex"]]
    s1 = g["streams"][1]
    got = synth.splitmix64_at(s1["seed"], np.arange(5, dtype=np.uint64))
    assert [int(v) for v in got] == [int(d) for d in s1["outputs_dec"]]


def test_uniform_values_exact_and_in_range(synth):
    idx = np.arange(100000, dtype=np.uint64)
    x = synth.x_values(123, idx)
    assert x.min() >= -1.0 and x.max() < 1.0
    z = synth.splitmix64_at(123, idx) >> np.uint64(11)
    # x = (2u - 2^53) / 2^53 exactly
    assert np.array_equal(x * 2.0 ** 53, 2.0 * z.astype(np.float64) - 2.0 ** 53)
    xi = synth.x_values(123, idx, "int5")
    assert set(np.unique(xi)) == {-2.0, -1.0, 0.0, 1.0, 2.0}


def test_slab_matches_full_tensor(synth):
    dims = (5, 6, 7)
    full = synth.x_tensor(99, dims)
    for mode in range(3):
        for i in (0, dims[mode] - 1):
            slab = synth.x_slab(99, dims, mode, i)
            assert np.array_equal(slab, np.take(full, [i], axis=mode))


# ---------------------------------------------------------------- CP-ALS update
def _unit_columns(A):
    return A / np.sqrt(np.sum(A * A, axis=0))


def _khatri_rao_rows(U, skip):
    """Rows of the Khatri-Rao product of the factors other than ``skip``, indexed by the
    other modes' indices flattened in increasing mode order (C order)."""
    mats = [U[m] for m in range(len(U)) if m != skip]
    K = mats[0]
    for B in mats[1:]:
        K = (K[:, None, :] * B[None, :, :]).reshape(-1, K.shape[1])
    return K


@pytest.mark.parametrize("n", [0, 1, 2])
def test_als_update_recovers_kruskal_factor(oracle_mod, n):
    """X = [[A, B, C]] exactly: the update with the true other factors returns the true
    factor of mode n with unit columns."""
    rng = np.random.default_rng(40 + n)
    dims, R = (9, 8, 10), 4
    F = [rng.standard_normal((d, R)) for d in dims]
    X = np.einsum("ir,jr,kr->ijk", *F)
    U = [None if m == n else F[m] for m in range(3)]
    got = oracle_mod.als_update(X, U, n)
    assert nrel(got, _unit_columns(F[n])) <= 1e-10


@pytest.mark.parametrize("dims,n", [((6, 5, 7), 0), ((6, 5, 7), 2), ((4, 3, 5, 4), 1), ((4, 3, 5, 4), 3)])
def test_als_update_matches_lstsq(oracle_mod, dims, n):
    """General X: the update solves min ||X_(n) - A KR^T||; lstsq on the explicit KR matrix."""
    rng = np.random.default_rng(sum(dims) + n)
    R = 3
    X = rng.standard_normal(dims)
    U = [rng.standard_normal((d, R)) for d in dims]
    Xn = np.moveaxis(X, n, 0).reshape(dims[n], -1)
    KR = _khatri_rao_rows(U, n)
    A = np.linalg.lstsq(KR, Xn.T, rcond=None)[0].T
    got = oracle_mod.als_update(X, [None if m == n else U[m] for m in range(len(dims))], n)
    assert nrel(got, _unit_columns(A)) <= 1e-10
    assert np.allclose(np.sqrt(np.sum(got * got, axis=0)), 1.0, rtol=0, atol=1e-14)


# ------------------------------------------------------------------ CP-ALS and HOOI (Sec. I consumers)
def _orth(rng, n, r):
    q, _ = np.linalg.qr(rng.standard_normal((n, r)))
    return q


def test_cp_als_rank1_exact_in_one_sweep(oracle_mod):
    """X = a o b o c: the first mode-0 update is a scaled a (M = a (b^T B)*(c^T C)), and
    the next two make the reconstruction exact, so one sweep gives fit 1."""
    rng = np.random.default_rng(11)
    a, b, c = rng.standard_normal(7), rng.standard_normal(6), rng.standard_normal(5)
    X = np.einsum("i,j,k->ijk", a, b, c)
    U0 = [rng.standard_normal((d, 1)) for d in X.shape]
    U, lam, fits = oracle_mod.cp_als(X, U0, 1)
    assert fits[0] == pytest.approx(1.0, abs=1e-12)
    for u, v in zip(U, (a, b, c)):
        assert abs(abs(u[:, 0] @ v) / np.linalg.norm(v) - 1.0) < 1e-12
    assert lam[0] == pytest.approx(np.linalg.norm(a) * np.linalg.norm(b) * np.linalg.norm(c), rel=1e-12)


def test_cp_als_recovers_planted_kruskal(oracle_mod):
    rng = np.random.default_rng(12)
    dims, R = (14, 12, 10), 3
    A = [rng.standard_normal((d, R)) for d in dims]
    lam = np.array([3.0, 2.0, 1.5])
    X = oracle_mod.kruskal_full(lam, A)
    U0 = [a + 0.2 * rng.standard_normal(a.shape) for a in A]
    U, lam_hat, fits = oracle_mod.cp_als(X, U0, 300, tol=1e-15)
    assert fits[-1] > 1.0 - 1e-8
    assert np.linalg.norm(oracle_mod.kruskal_full(lam_hat, U) - X) <= 1e-7 * np.linalg.norm(X)


def test_cp_als_first_update_is_least_squares(oracle_mod):
    """The mode-0 update minimises ||X_(0) - A (C kr B)^T||: compare with lstsq on the
    explicit Khatri-Rao product (columns normalised the same way)."""
    rng = np.random.default_rng(13)
    X = rng.standard_normal((6, 5, 4))
    U0 = [rng.standard_normal((d, 3)) for d in X.shape]
    U, _, _ = oracle_mod.cp_als(X, U0, 1)
    # After a full sweep U[0] is the first update; recompute it from U0 directly.
    K = np.einsum("jr,kr->jkr", U0[1], U0[2]).reshape(-1, 3)
    A = np.linalg.lstsq(K, X.reshape(6, -1).T, rcond=None)[0].T
    A /= np.linalg.norm(A, axis=0)
    assert np.allclose(U[0], A, atol=1e-12)


def test_cp_als_fit_does_not_decrease(oracle_mod):
    rng = np.random.default_rng(14)
    X = rng.standard_normal((9, 8, 7))
    U0 = [rng.standard_normal((d, 4)) for d in X.shape]
    _, _, fits = oracle_mod.cp_als(X, U0, 15)
    assert all(f2 >= f1 - 1e-12 for f1, f2 in zip(fits, fits[1:]))


def test_hooi_matrix_is_truncated_svd(oracle_mod):
    """Order 2: HOOI is subspace iteration on X X^T, converging to the truncated SVD;
    the fit is then Eckart-Young's 1 - sqrt(sum_{i>r} s_i^2) / ||X||."""
    rng = np.random.default_rng(15)
    sv = np.array([10.0, 7.0, 5.0, 1.0, 0.7, 0.4, 0.2, 0.1, 0.05])
    X = _orth(rng, 12, 9) @ np.diag(sv) @ _orth(rng, 9, 9).T
    U0 = [_orth(rng, 12, 3), _orth(rng, 9, 3)]
    U, G, fits = oracle_mod.tucker_hooi(X, U0, 40)
    left, s, right = np.linalg.svd(X)
    assert fits[-1] == pytest.approx(1 - np.sqrt(np.sum(s[3:] ** 2)) / np.linalg.norm(X), abs=1e-12)
    assert np.allclose(U[0] @ U[0].T, left[:, :3] @ left[:, :3].T, atol=1e-10)
    assert np.allclose(np.abs(np.diag(G)), s[:3], atol=1e-10)


def test_hooi_recovers_planted_tucker(oracle_mod):
    """X = G x_m V_m with orthonormal V_m: exact multilinear rank, so one sweep from a
    random orthonormal start gives the subspaces of V_m and fit 1."""
    rng = np.random.default_rng(16)
    dims, ranks = (10, 9, 8, 7), (3, 2, 4, 2)
    V = [_orth(rng, d, r) for d, r in zip(dims, ranks)]
    G0 = rng.standard_normal(ranks)
    X = oracle_mod.tucker_full(G0, V)
    U0 = [_orth(rng, d, r) for d, r in zip(dims, ranks)]
    U, G, fits = oracle_mod.tucker_hooi(X, U0, 1)
    assert fits[0] == pytest.approx(1.0, abs=1e-12)
    for u, v in zip(U, V):
        assert np.allclose(u @ u.T, v @ v.T, atol=1e-12)
        assert np.allclose(u.T @ u, np.eye(u.shape[1]), atol=1e-12)
    assert np.linalg.norm(G) == pytest.approx(np.linalg.norm(X), rel=1e-12)


def test_hooi_fit_does_not_decrease_and_core_norm(oracle_mod):
    """Orthonormal factors: ||X - [[G; U]]||^2 = ||X||^2 - ||G||^2 at every sweep, and
    the fit of HOOI does not decrease."""
    rng = np.random.default_rng(17)
    X = rng.standard_normal((8, 7, 6))
    U0 = [_orth(rng, d, 3) for d in X.shape]
    U, G, fits = oracle_mod.tucker_hooi(X, U0, 6)
    assert all(f2 >= f1 - 1e-12 for f1, f2 in zip(fits, fits[1:]))
    xn, gn = np.linalg.norm(X), np.linalg.norm(G)
    assert fits[-1] == pytest.approx(1 - np.sqrt(xn ** 2 - gn ** 2) / xn, abs=1e-12)


def test_sign_fix_convention(oracle_mod):
    Q = np.array([[0.1, -0.9], [-0.8, 0.2], [0.3, 0.9]])
    F = oracle_mod.sign_fix(Q)
    assert np.array_equal(F, np.array([[-0.1, 0.9], [0.8, -0.2], [-0.3, -0.9]]))
