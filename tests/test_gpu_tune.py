"""GPU tests of the autotuner: tuned plans are cached, used by later calls, and
their results still match the oracle."""
import numpy as np
import pytest
import torch

from gpu_common import flush, mttkrp_spec, nrel, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dn():
    import paper_2206_08301_amd as m
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    m._lib.load()
    return m


@pytest.mark.parametrize("n,prec", [(0, "fp64"), (2, "fp64"), (1, "fp32")])
def test_tuned_plan_is_cached_and_correct(dn, oracle_mod, n, prec):
    rng = np.random.default_rng(70 + n)
    dims, R = (96, 80, 130), 20
    X = rng.uniform(-1, 1, dims)
    U = [rng.standard_normal((d, R)) for d in dims]
    dt = torch.float64 if prec == "fp64" else torch.float32
    Xd = to_dev(X, dt)
    Ud = [to_dev(U[m], dt) for m in range(3) if m != n]
    spec = mttkrp_spec(3, n)
    dn.tune_clear()
    rep = dn.tune_mttkrp(spec, Xd, Ud, precision=prec, out_dtype=torch.float64, reps=3)
    flush(f"tuned mode {n} {prec}: {rep.plan_name.decode()} {rep.tuned_us:.1f} us")
    assert rep.tuned_us > 0 and rep.plan_name
    assert dn.tune_entries() == 1
    used = dn.Report()
    M = dn.mttkrp(spec, Xd, Ud, precision=prec, out_dtype=torch.float64, report=used)
    torch.cuda.synchronize()
    assert used.plan_name == rep.plan_name and used.groups == rep.groups
    ref = oracle_mod.mttkrp(X, [None if m == n else U[m] for m in range(3)], n)
    assert nrel(M.cpu().numpy(), ref) <= (1e-12 if prec == "fp64" else 1e-5)
    dn.tune_clear()


def test_tuned_batch_job_is_cached_and_correct(dn, oracle_mod):
    rng = np.random.default_rng(77)
    dims, R, n = (64, 120, 90), 40, 1
    X = rng.uniform(-1, 1, dims)
    U = [rng.standard_normal((d, R)) for d in dims]
    Xd = to_dev(X, torch.float64)
    Ud = [to_dev(U[m], torch.float64) for m in range(3) if m != n]
    spec = mttkrp_spec(3, n)
    dn.tune_clear()
    rep = dn.tune_mttkrp(spec, Xd, Ud, reps=3, batched=True)
    flush(f"tuned batch job: {rep.plan_name.decode()} {rep.tuned_us:.1f} us")
    assert rep.tuned_us > 0 and dn.tune_entries() == 1
    b = dn.Batch(4)
    _, M = b.add(spec, Xd, Ud)
    b.launch()
    torch.cuda.synchronize()
    ref = oracle_mod.mttkrp(X, [None if m == n else U[m] for m in range(3)], n)
    assert nrel(M.cpu().numpy(), ref) <= 1e-12
    b.close()
    dn.tune_clear()


def test_tuned_ttmc_variant_is_cached_and_correct(dn, oracle_mod):
    from gpu_common import ttmc_spec
    rng = np.random.default_rng(78)
    dims, ranks = (40, 70, 130), (8, 32, 24)
    X = rng.uniform(-1, 1, dims)
    U = [None] + [rng.standard_normal((d, ranks[m])) for m, d in enumerate(dims) if m > 0]
    Xd = to_dev(X)
    Ud = [to_dev(u) for u in U if u is not None]
    dn.tune_clear()
    Y = dn.ttmc(ttmc_spec(3, 0), Xd, Ud, tune_reps=2)
    torch.cuda.synchronize()
    assert dn.tune_entries() == 1
    ref = oracle_mod.ttmc(X, U, 0)
    assert nrel(Y.cpu().numpy(), ref) <= 1e-12
    dn.tune_clear()
