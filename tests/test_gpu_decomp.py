"""CP-ALS and Tucker-HOOI on the device (deinsum_cp_als, deinsum_tucker_hooi) against
the oracle's textbook loops run from the same starting factors for the same number of
sweeps: factors, lambda / core and the fit of every sweep."""
import numpy as np
import pytest
import torch

from gpu_common import flush, nrel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dn():
    import paper_2206_08301_amd as m
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    m._lib.load()
    return m


def orth(rng, n, r):
    q, _ = np.linalg.qr(rng.standard_normal((n, r)))
    return q


def planted_kruskal(oracle_mod, rng, dims, R, noise):
    A = [rng.standard_normal((d, R)) for d in dims]
    lam = np.linspace(2.0, 1.0, R)
    X = oracle_mod.kruskal_full(lam, A)
    return X + noise * np.linalg.norm(X) / np.sqrt(X.size) * rng.standard_normal(dims)


def planted_tucker(oracle_mod, rng, dims, ranks, noise):
    core = rng.standard_normal(ranks) * np.linspace(3.0, 1.0, ranks[0]).reshape((-1,) + (1,) * (len(ranks) - 1))
    X = oracle_mod.tucker_full(core, [orth(rng, d, r) for d, r in zip(dims, ranks)])
    return X + noise * np.linalg.norm(X) / np.sqrt(X.size) * rng.standard_normal(dims)


def same_columns_up_to_sign(a, b, tol):
    s = np.sign(np.sum(a * b, axis=0))
    return np.max(np.abs(a - b * s)) <= tol * max(1.0, np.max(np.abs(b)))


@pytest.mark.parametrize("dims,R", [((40, 36, 32), 4), ((12, 10, 14, 9), 3), ((30, 25), 5)])
def test_cp_als_fp64_matches_oracle(dn, oracle_mod, dims, R):
    rng = np.random.default_rng(900 + len(dims))
    X = planted_kruskal(oracle_mod, rng, dims, R, 0.05)
    U0 = [rng.standard_normal((d, R)) for d in dims]
    sweeps = 8
    U_ref, lam_ref, fits_ref = oracle_mod.cp_als(X, U0, sweeps)
    Xd = torch.from_numpy(X).cuda()
    Ud = [torch.from_numpy(u.copy()).cuda() for u in U0]
    flush(f"cp_als fp64 dims={dims} R={R}")
    lam, info = dn.cp_als(Xd, Ud, max_sweeps=sweeps, tol=0.0)
    torch.cuda.synchronize()
    assert info["sweeps"] == sweeps and not info["regularised"]
    assert np.allclose(info["fits"], fits_ref, atol=1e-9, rtol=0)
    assert np.allclose(lam.cpu().numpy(), lam_ref, rtol=1e-9, atol=0)
    for m in range(len(dims)):
        assert nrel(Ud[m].cpu().numpy(), U_ref[m]) <= 1e-9


def test_cp_als_fp32_form(dn, oracle_mod):
    rng = np.random.default_rng(910)
    dims, R = (48, 40, 36), 6
    X = planted_kruskal(oracle_mod, rng, dims, R, 0.05).astype(np.float32).astype(np.float64)
    U0 = [rng.standard_normal((d, R)).astype(np.float32).astype(np.float64) for d in dims]
    U_ref, lam_ref, fits_ref = oracle_mod.cp_als(X, U0, 5)
    Xd = torch.from_numpy(X).float().cuda()
    Ud = [torch.from_numpy(u).float().cuda() for u in U0]
    lam, info = dn.cp_als(Xd, Ud, precision="fp32", max_sweeps=5, tol=0.0)
    torch.cuda.synchronize()
    assert np.allclose(info["fits"], fits_ref, atol=1e-5, rtol=0)
    for m in range(3):
        assert nrel(Ud[m].double().cpu().numpy(), U_ref[m]) <= 1e-4


def test_cp_als_converges_on_planted_kruskal(dn, oracle_mod):
    """Exact rank-4 data, start near the truth: the fit reaches 1 (within the 1e-7 the
    norm identity resolves) and the run stops on tol before max_sweeps."""
    rng = np.random.default_rng(920)
    dims, R = (30, 28, 26), 4
    A = [rng.standard_normal((d, R)) for d in dims]
    X = oracle_mod.kruskal_full(np.ones(R), A)
    Ud = [torch.from_numpy(a + 0.05 * rng.standard_normal(a.shape)).cuda() for a in A]
    lam, info = dn.cp_als(torch.from_numpy(X).cuda(), Ud, max_sweeps=200, tol=1e-12)
    flush(f"cp_als planted: sweeps {info['sweeps']}, fit {info['fit']:.12f}")
    assert info["fit"] > 1 - 1e-6 and info["sweeps"] < 200
    rec = oracle_mod.kruskal_full(lam.cpu().numpy(), [u.cpu().numpy() for u in Ud])
    assert nrel(rec, X) <= 1e-6


def test_cp_als_flags_rank_deficient_update(dn):
    rng = np.random.default_rng(930)
    dims, R = (3, 3, 40), 16
    X = torch.from_numpy(rng.standard_normal(dims)).cuda()
    Ud = [torch.from_numpy(rng.standard_normal((d, R))).cuda() for d in dims]
    _, info = dn.cp_als(X, Ud, max_sweeps=2, tol=0.0)
    assert info["regularised"]


@pytest.mark.parametrize("dims,ranks", [((30, 28, 26), (4, 3, 5)), ((12, 11, 10, 9), (3, 2, 3, 2)),
                                        ((40, 30), (4, 4))])
def test_hooi_fp64_matches_oracle(dn, oracle_mod, dims, ranks):
    rng = np.random.default_rng(940 + len(dims))
    X = planted_tucker(oracle_mod, rng, dims, ranks, 0.02)
    U0 = [orth(rng, d, r) for d, r in zip(dims, ranks)]
    sweeps = 3
    U_ref, G_ref, fits_ref = oracle_mod.tucker_hooi(X, U0, sweeps)
    Xd = torch.from_numpy(X).cuda()
    Ud = [torch.from_numpy(u.copy()).cuda() for u in U0]
    flush(f"hooi fp64 dims={dims} ranks={ranks}")
    G, info = dn.tucker_hooi(Xd, Ud, max_sweeps=sweeps, tol=0.0)
    torch.cuda.synchronize()
    flush(f"  fits {info['fits']} vs {fits_ref}, iters {info['iters']}")
    assert info["sweeps"] == sweeps and not info["max_iters_hit"] and not info["rank_deficient"]
    assert np.allclose(info["fits"], fits_ref, atol=1e-9, rtol=0)
    for m in range(len(dims)):
        Um = Ud[m].cpu().numpy()
        assert np.max(np.abs(Um - U_ref[m])) <= 1e-8, m
        assert np.allclose(Um.T @ Um, np.eye(ranks[m]), atol=1e-12)
    assert nrel(G.cpu().numpy(), G_ref) <= 1e-8


def test_hooi_recovers_planted_subspaces(dn, oracle_mod):
    rng = np.random.default_rng(950)
    dims, ranks = (36, 34, 32), (5, 4, 3)
    V = [orth(rng, d, r) for d, r in zip(dims, ranks)]
    X = oracle_mod.tucker_full(rng.standard_normal(ranks), V)
    Ud = [torch.from_numpy(orth(rng, d, r)).cuda() for d, r in zip(dims, ranks)]
    G, info = dn.tucker_hooi(torch.from_numpy(X).cuda(), Ud, max_sweeps=3, tol=0.0)
    assert info["fit"] > 1 - 1e-7
    for u, v in zip(Ud, V):
        u = u.cpu().numpy()
        assert np.allclose(u @ u.T, v @ v.T, atol=1e-10)
    assert np.linalg.norm(G.cpu().numpy()) == pytest.approx(np.linalg.norm(X), rel=1e-12)


def test_hooi_fp32_form(dn, oracle_mod):
    rng = np.random.default_rng(960)
    dims, ranks = (40, 36, 30), (4, 4, 3)
    X = planted_tucker(oracle_mod, rng, dims, ranks, 0.02).astype(np.float32).astype(np.float64)
    U0 = [orth(rng, d, r).astype(np.float32).astype(np.float64) for d, r in zip(dims, ranks)]
    U_ref, G_ref, fits_ref = oracle_mod.tucker_hooi(X, U0, 2)
    Ud = [torch.from_numpy(u).float().cuda() for u in U0]
    G, info = dn.tucker_hooi(torch.from_numpy(X).float().cuda(), Ud, precision="fp32", max_sweeps=2, tol=0.0)
    assert np.allclose(info["fits"], fits_ref, atol=1e-5, rtol=0)
    for m in range(3):
        assert np.max(np.abs(Ud[m].double().cpu().numpy() - U_ref[m])) <= 1e-4
    assert nrel(G.cpu().numpy(), G_ref) <= 1e-4


def test_hooi_rejects_bad_ranks(dn):
    X = torch.zeros((6, 5, 4), dtype=torch.float64, device="cuda")
    U = [torch.zeros((6, 2), dtype=torch.float64, device="cuda"), torch.zeros((5, 2), dtype=torch.float64, device="cuda"),
         torch.zeros((4, 4), dtype=torch.float64, device="cuda")]  # 4 > 2 * 2 is fine; 5 would not be
    U[2] = torch.zeros((4, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(dn.DeinsumError) as ei:
        dn.tucker_hooi(X, U, max_sweeps=1)
    assert ei.value.status == -4


def test_cp_als_full_size_one_sweep(dn, synth, oracle_mod):
    """The 1024^3 R = 24 workload (uniform X, N(0,1) starting factors): one sweep on the
    device against the oracle's sweep (factors and lambda; the oracle's explicit-fit
    reconstruction is skipped at this size)."""
    dims, R = (1024, 1024, 1024), 24
    seed = synth.config_seed(2, 0)
    flush("cp_als 1024^3: host generation")
    X = synth.x_range(seed, 0, 1 << 30).reshape(dims)
    U0 = [synth.normal_factor(synth.config_seed(2, 1 + m), 1024, R) for m in range(3)]
    flush("cp_als 1024^3: oracle sweep")
    U_ref, lam_ref, _ = oracle_mod.cp_als(X, U0, 1, with_fit=False)
    Xd = torch.from_numpy(X).cuda()
    del X
    Ud = [torch.from_numpy(u.copy()).cuda() for u in U0]
    flush("cp_als 1024^3: device sweep")
    lam, info = dn.cp_als(Xd, Ud, max_sweeps=1, tol=0.0)
    torch.cuda.synchronize()
    assert np.allclose(lam.cpu().numpy(), lam_ref, rtol=1e-10, atol=0)
    for m in range(3):
        assert nrel(Ud[m].cpu().numpy(), U_ref[m]) <= 1e-10
    del Xd
    torch.cuda.empty_cache()


def test_hooi_full_size_one_sweep(dn, synth, oracle_mod):
    """The Tucker-step workload's shape (1024^3, ranks 32): a planted multilinear-rank-32
    tensor plus 1 % noise from the counter generator, one HOOI sweep from the same
    orthonormal start on the device and in the oracle: factors, core and fit."""
    dims, ranks = (1024, 1024, 1024), (32, 32, 32)
    rng = np.random.default_rng(970)
    V = [orth(rng, d, r) for d, r in zip(dims, ranks)]
    core = rng.standard_normal(ranks) * np.linspace(3.0, 1.0, 32)[:, None, None]
    flush("hooi 1024^3: host generation")
    X = oracle_mod.tucker_full(core, V)
    X += 0.01 * np.linalg.norm(X) / np.sqrt(X.size) * synth.x_range(2206083971, 0, 1 << 30).reshape(dims)
    U0 = [orth(rng, d, r) for d, r in zip(dims, ranks)]
    flush("hooi 1024^3: oracle sweep")
    U_ref, G_ref, fits_ref = oracle_mod.tucker_hooi(X, U0, 1)
    Xd = torch.from_numpy(X).cuda()
    del X
    Ud = [torch.from_numpy(u.copy()).cuda() for u in U0]
    flush("hooi 1024^3: device sweep")
    G, info = dn.tucker_hooi(Xd, Ud, max_sweeps=1, tol=0.0)
    torch.cuda.synchronize()
    flush(f"  fit {info['fit']:.12f} vs {fits_ref[0]:.12f}, iters {info['iters']}")
    assert abs(info["fit"] - fits_ref[0]) <= 1e-9
    for m in range(3):
        assert np.max(np.abs(Ud[m].cpu().numpy() - U_ref[m])) <= 1e-8, m
    assert nrel(G.cpu().numpy(), G_ref) <= 1e-8
    del Xd
    torch.cuda.empty_cache()
