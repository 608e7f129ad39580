"""Plain FP64 CPU oracle for MTTKRP and TTMc (Deinsum, arXiv 2206.08301).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  The
product library never links or calls it, and it shares no code with the HIP
path.

The arithmetic lives in ``oracle.c`` (plain loops, FP64, no FMA contraction):
  * ``mttkrp``  -- the MTTKRP einsum of Tab. IV summed term by term
                   (Sec. III-B, "tensor operations");
  * ``ttm``     -- one mode product (Sec. III-B);
  * ``ttmc``    -- the TTM chain over all modes but one (Sec. III-B).
This module only marshals numpy arrays to that library, except for
  * ``mttkrp_mm`` -- the MTTKRP followed by a matrix product, the chain of the
    paper's running example (Sec. II-A, ``ijk,ja,ka,al->il``): ``mttkrp``
    then one numpy matrix product, in that order;
  * ``als_update`` -- one CP-ALS factor update built on ``mttkrp`` (numpy).
    The paper names MTTKRP as the main kernel of the CP decomposition (Sec. I)
    but does not state the update; this is the textbook alternating
    least-squares step (Kolda & Bader, SIAM Review 51(3), 2009, Sec. 3.4);
  * ``cp_als`` and ``tucker_hooi`` -- the textbook CP-ALS sweep loop and the
    higher-order orthogonal iteration (Kolda & Bader, Sec. 3.4 and 4.2) on top
    of ``mttkrp`` / ``ttmc`` with numpy's dense solve and SVD, fits from the
    explicitly formed reconstructions.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i64p = ctypes.POINTER(ctypes.c_int64)
    dpp = ctypes.POINTER(ctypes.c_void_p)
    lib.oracle_num_threads.restype = ctypes.c_int
    for name in ("oracle_mttkrp", "oracle_mttkrp_ld"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int64,
                      ctypes.c_void_p, dpp, ctypes.c_void_p]
    lib.oracle_ttm.restype = ctypes.c_int
    lib.oracle_ttm.argtypes = [ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int64,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_ttmc.restype = ctypes.c_int
    lib.oracle_ttmc.argtypes = [ctypes.c_int, i64p, ctypes.c_int, i64p,
                                ctypes.c_void_p, dpp, ctypes.c_void_p]
    _lib = lib
    return lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dims(shape):
    return (ctypes.c_int64 * len(shape))(*[int(s) for s in shape])


def _factor_table(U, N, skip):
    """U: sequence of N entries indexed by mode (entry ``skip`` ignored)."""
    keep = []
    ptrs = (ctypes.c_void_p * N)()
    for m in range(N):
        if m == skip or U[m] is None:
            ptrs[m] = None
            continue
        a = _f64(U[m])
        keep.append(a)
        ptrs[m] = a.ctypes.data
    return ptrs, keep


def mttkrp(X, U, n, long_double=False):
    """M[i_n, r] = sum over the other indices of X[i] * prod_{m != n} U[m][i_m, r].

    ``U`` holds one matrix per mode (``U[n]`` is ignored).
    """
    X = _f64(X)
    N = X.ndim
    R = None
    for m in range(N):
        if m != n:
            R = np.shape(U[m])[1]
            if np.shape(U[m])[0] != X.shape[m]:
                raise ValueError(f"factor of mode {m} has {np.shape(U[m])[0]} rows, X has {X.shape[m]}")
    if R is None:
        raise ValueError("MTTKRP needs at least one contracted mode")
    ptrs, keep = _factor_table(U, N, n)
    M = np.empty((X.shape[n], R), dtype=np.float64)
    fn = _load().oracle_mttkrp_ld if long_double else _load().oracle_mttkrp
    rc = fn(N, _dims(X.shape), n, R, X.ctypes.data, ptrs, M.ctypes.data)
    if rc:
        raise RuntimeError(f"oracle_mttkrp failed with {rc}")
    return M


def ttm(X, Um, m):
    """Mode-m product: Y[.., r, ..] = sum_{i_m} X[.., i_m, ..] * Um[i_m, r]."""
    X = _f64(X)
    Um = _f64(Um)
    if Um.shape[0] != X.shape[m]:
        raise ValueError("factor rows must equal the contracted dimension")
    shape = list(X.shape)
    shape[m] = Um.shape[1]
    Y = np.empty(shape, dtype=np.float64)
    rc = _load().oracle_ttm(X.ndim, _dims(X.shape), m, Um.shape[1], X.ctypes.data,
                            Um.ctypes.data, Y.ctypes.data)
    if rc:
        raise RuntimeError(f"oracle_ttm failed with {rc}")
    return Y


def ttmc(X, U, n):
    """TTM chain over every mode except ``n`` (``U[n]`` is ignored)."""
    X = _f64(X)
    N = X.ndim
    ranks = [0] * N
    shape = list(X.shape)
    for m in range(N):
        if m == n:
            continue
        if np.shape(U[m])[0] != X.shape[m]:
            raise ValueError(f"factor of mode {m} has wrong row count")
        ranks[m] = np.shape(U[m])[1]
        shape[m] = ranks[m]
    ptrs, keep = _factor_table(U, N, n)
    Y = np.empty(shape, dtype=np.float64)
    rc = _load().oracle_ttmc(N, _dims(X.shape), n, _dims(ranks), X.ctypes.data, ptrs,
                             Y.ctypes.data)
    if rc:
        raise RuntimeError(f"oracle_ttmc failed with {rc}")
    return Y


def mttkrp_mm(X, U, n, C):
    """Y[i_n, l] = sum_r M[i_n, r] C[r, l] with M = mttkrp(X, U, n) (Sec. II-A chain)."""
    C = _f64(C)
    M = mttkrp(X, U, n)
    if C.ndim != 2 or C.shape[0] != M.shape[1]:
        raise ValueError("C must be R x L")
    return M @ C


def als_update(X, U, n):
    """One CP-ALS update of the mode-n factor.

    The least-squares problem  min_A || X_(n) - A (KR of the other factors)^T ||
    has the normal-equations solution  A = M V^{-1}  with M the mode-n MTTKRP
    and V the Hadamard product of the Gram matrices U[m]^T U[m], m != n.  The
    columns of A are then scaled to unit 2-norm (zero columns are left as
    they are).  ``U`` holds one matrix per mode; ``U[n]`` is ignored.
    Returns the new factor (FP64).
    """
    X = _f64(X)
    M = mttkrp(X, U, n)
    R = M.shape[1]
    V = np.ones((R, R), dtype=np.float64)
    for m in range(X.ndim):
        if m != n:
            Um = _f64(U[m])
            V = V * (Um.T @ Um)
    A = np.linalg.solve(V, M.T).T
    norms = np.sqrt(np.sum(A * A, axis=0))
    norms[norms == 0] = 1.0
    return A / norms


# --------------------------------------------------------------------------- decompositions
# The paper motivates MTTKRP and TTMc by the CP and Tucker decompositions that
# consume them (Sec. I).  It does not state the outer algorithms; these are the
# textbook ones (Kolda & Bader, SIAM Review 51(3), 2009): CP-ALS (Sec. 3.4) and
# the higher-order orthogonal iteration, HOOI (Sec. 4.2), written plainly on
# top of ``mttkrp`` and ``ttmc`` with numpy's dense solvers.

def _letters(N):
    return "abcdefgh"[:N]


def kruskal_full(lam, U):
    """The dense tensor sum_r lam_r U[0][:, r] o U[1][:, r] o ... (outer products)."""
    N = len(U)
    t = _letters(N)
    spec = "z," + ",".join(f"{t[m]}z" for m in range(N)) + "->" + t
    return np.einsum(spec, _f64(lam), *[_f64(u) for u in U])


def tucker_full(G, U):
    """The dense tensor G x_0 U[0] x_1 U[1] ... (each U[m] is I_m x R_m)."""
    Y = _f64(G)
    for m, u in enumerate(U):
        Y = ttm(Y, _f64(u).T, m)
    return Y


def cp_als(X, U0, sweeps, tol=0.0, with_fit=True):
    """CP-ALS from the starting factors ``U0`` (one I_m x R matrix per mode).

    A sweep updates the modes in increasing order; the mode-n update solves the
    normal equations A V = M, M = mttkrp(X, U, n), V = Hadamard product of the
    Grams U[m]^T U[m] (m != n), then stores U[n] = A with unit 2-norm columns and
    lam = the column norms of A.  After each sweep the fit
    1 - ||X - [[lam; U]]||_F / ||X||_F is computed from the explicitly formed
    reconstruction (skipped, and ``tol`` ignored, with ``with_fit=False``).
    Stops after ``sweeps`` sweeps, or earlier when the fit changes by less than
    ``tol``.  Returns (U, lam, fits).
    """
    X = _f64(X)
    N = X.ndim
    U = [_f64(u).copy() for u in U0]
    R = U[0].shape[1]
    lam = np.ones(R)
    fits = []
    xnorm = np.linalg.norm(X.ravel())
    for _ in range(sweeps):
        for n in range(N):
            M = mttkrp(X, [None if m == n else U[m] for m in range(N)], n)
            V = np.ones((R, R))
            for m in range(N):
                if m != n:
                    V = V * (U[m].T @ U[m])
            A = np.linalg.solve(V, M.T).T
            lam = np.sqrt(np.sum(A * A, axis=0))
            U[n] = A / np.where(lam > 0, lam, 1.0)
        if not with_fit:
            continue
        fits.append(1.0 - np.linalg.norm((X - kruskal_full(lam, U)).ravel()) / xnorm)
        if len(fits) > 1 and abs(fits[-1] - fits[-2]) < tol:
            break
    return U, lam, fits


def sign_fix(Q):
    """Columns scaled by +-1 so that each column's entry of largest magnitude (the
    first one on ties) is positive: the convention that makes singular vectors unique."""
    Q = _f64(Q).copy()
    for r in range(Q.shape[1]):
        k = int(np.argmax(np.abs(Q[:, r])))
        if Q[k, r] < 0:
            Q[:, r] = -Q[:, r]
    return Q


def tucker_hooi(X, U0, sweeps, tol=0.0):
    """HOOI from the starting factors ``U0`` (I_m x R_m, orthonormal columns).

    A sweep updates the modes in increasing order: Y = ttmc(X, U, n) (every mode
    but n), then U[n] = the R_n leading left singular vectors of the mode-n
    unfolding of Y (numpy SVD, columns by decreasing singular value, sign_fix).
    After each sweep the core G = Y x_n U[n]^T of the last mode and the fit
    1 - ||X - G x_0 U[0] ... ||_F / ||X||_F (explicit reconstruction) are formed.
    Stops after ``sweeps`` sweeps or when the fit changes by less than ``tol``.
    Returns (U, G, fits).
    """
    X = _f64(X)
    N = X.ndim
    U = [_f64(u).copy() for u in U0]
    fits = []
    xnorm = np.linalg.norm(X.ravel())
    G = None
    for _ in range(sweeps):
        for n in range(N):
            Y = ttmc(X, U, n)
            Yn = np.moveaxis(Y, n, 0).reshape(X.shape[n], -1)
            left, _, _ = np.linalg.svd(Yn, full_matrices=False)
            U[n] = sign_fix(left[:, :U[n].shape[1]])
        G = ttm(Y, U[N - 1], N - 1)
        fits.append(1.0 - np.linalg.norm((X - tucker_full(G, U)).ravel()) / xnorm)
        if len(fits) > 1 and abs(fits[-1] - fits[-2]) < tol:
            break
    return U, G, fits
