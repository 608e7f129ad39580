"""Tolerance-driven form choice on the GPU, against the oracle.

* 1024^3, R = 24, every mode: for tol 1e-12, 1e-5 and 1e-2 `prepare` stores X in the
  storage deinsum_choose_storage names (F64, FX20, BF16), the call with
  DEINSUM_PREC_AUTO reports the form it ran and its estimate, and the whole output's
  error against the oracle is at most that estimate, which is at most tol.
* The same on FP32 storage, where the tolerance picks between FP32 and BF16x3.
* The statistics the estimates use: deinsum_tensor_stats against numpy, and the FX20
  header's storage error against a host decode of the buffer.
"""
import numpy as np
import pytest
import torch

from gpu_common import SPEC3, flush, nrel, to_dev, ttmc_spec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dn():
    import paper_2206_08301_amd as m
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    m._lib.load()
    return m


@pytest.fixture(scope="module")
def bench_problem(synth, oracle_mod):
    """The benchmark's 1024^3 X (host copy dropped after upload), factors and whole
    oracle outputs of the three modes."""
    dims, R = (1024, 1024, 1024), 24
    seed = synth.config_seed(2, 0)
    flush(f"auto 1024^3 seed={seed}: host generation")
    X = synth.x_range(seed, 0, 1 << 30).reshape(dims)
    U = [synth.normal_factor(synth.config_seed(2, 1 + m), 1024, R) for m in range(3)]
    refs = {}
    for n in range(3):
        flush(f"auto 1024^3: oracle mode {n}")
        refs[n] = oracle_mod.mttkrp(X, [None if m == n else U[m] for m in range(3)], n)
    host_max = float(np.abs(X).max())
    host_rms = float(np.sqrt(np.mean(X * X)))
    Xd = torch.from_numpy(X).cuda()
    del X
    yield Xd, U, refs, R, (host_max, host_rms)
    del Xd
    torch.cuda.empty_cache()


def test_tensor_stats_match_host(dn, bench_problem):
    Xd, _, _, _, (hmax, hrms) = bench_problem
    mx, rms = dn.tensor_stats(Xd)
    assert mx == hmax
    assert rms == pytest.approx(hrms, rel=1e-9)


@pytest.mark.parametrize("tol,storage,form", [(1e-12, "f64", "fp64"), (1e-5, "fx20", "fx20"), (1e-2, "bf16", "bf16")])
def test_auto_1024cubed_whole_output(dn, bench_problem, tol, storage, form):
    Xd, U, refs, R, _ = bench_problem
    for n in range(3):
        flush(f"auto 1024^3 tol={tol} mode {n}: prepare + deinsum_mttkrp(AUTO)")
        Xs, st = dn.prepare(Xd, SPEC3[n], [R], tol)
        assert st == storage
        udt = torch.float64 if storage == "f64" else torch.float32
        ops = [to_dev(U[m], udt) for m in range(3) if m != n]
        rep = dn.Report()
        M = dn.mttkrp(SPEC3[n], Xs, ops, precision="auto", tol=tol, out_dtype=torch.float64, report=rep)
        torch.cuda.synchronize()
        err = nrel(M.cpu().numpy(), refs[n])
        flush(f"  form {dn.PRECISION_NAMES[rep.precision]}, est {rep.est_err:.3e}, oracle error {err:.3e}")
        assert dn.PRECISION_NAMES[rep.precision] == form
        assert err <= rep.est_err <= tol
        del Xs
    torch.cuda.empty_cache()


@pytest.mark.parametrize("tol,form", [(1e-5, "fp32"), (1e-4, "bf16x3")])
def test_auto_fp32_storage(dn, bench_problem, tol, form):
    Xd, U, refs, R, _ = bench_problem
    X32 = torch.empty(Xd.shape, dtype=torch.float32, device="cuda")
    dn.convert(Xd, X32)
    for n in range(3):
        ops = [to_dev(U[m], torch.float32) for m in range(3) if m != n]
        rep = dn.Report()
        M = dn.mttkrp(SPEC3[n], X32, ops, precision="auto", tol=tol, out_dtype=torch.float64, report=rep)
        torch.cuda.synchronize()
        err = nrel(M.cpu().numpy(), refs[n])
        flush(f"auto f32 tol={tol} mode {n}: form {dn.PRECISION_NAMES[rep.precision]}, est {rep.est_err:.3e}, "
              f"oracle error {err:.3e}")
        assert dn.PRECISION_NAMES[rep.precision] == form
        assert err <= rep.est_err <= tol
    with pytest.raises(dn.DeinsumError) as ei:  # no FP32-storage form meets 1e-12
        dn.mttkrp(SPEC3[0], X32, [to_dev(U[m], torch.float32) for m in (1, 2)], precision="auto", tol=1e-12)
    assert ei.value.status == -3
    del X32
    torch.cuda.empty_cache()


def test_explicit_forms_within_estimate(dn, bench_problem):
    """Every explicit form's report carries its estimate; the oracle error is below it."""
    Xd, U, refs, R, _ = bench_problem
    X32 = torch.empty(Xd.shape, dtype=torch.float32, device="cuda")
    dn.convert(Xd, X32)
    Xb = torch.empty(Xd.shape, dtype=torch.bfloat16, device="cuda")
    dn.convert(Xd, Xb)
    Xf = dn.to_fx20(Xd)
    copies = {"fp64": Xd, "fp32": X32, "bf16x3": X32, "bf16": Xb, "fx20": Xf}
    for prec, Xp in copies.items():
        udt = torch.float64 if prec == "fp64" else torch.float32
        for n in range(3):
            ops = [to_dev(U[m], udt) for m in range(3) if m != n]
            rep = dn.Report()
            M = dn.mttkrp(SPEC3[n], Xp, ops, precision=prec, out_dtype=torch.float64, report=rep)
            torch.cuda.synchronize()
            err = nrel(M.cpu().numpy(), refs[n])
            flush(f"explicit {prec} mode {n}: est {rep.est_err:.3e}, oracle error {err:.3e}")
            assert dn.PRECISION_NAMES[rep.precision] == prec
            assert err <= rep.est_err
    del copies, X32, Xb, Xf
    torch.cuda.empty_cache()


@pytest.mark.parametrize("scale,dist", [(1.0, "uniform"), (37.5, "cubed")])
def test_fx20_header_storage_error_matches_host_decode(dn, synth, scale, dist):
    """The encoder's recorded storage error ||X - X_fx20|| / ||X|| and rms against the
    buffer decoded on the host."""
    n = 3 * (1 << 20) + 17
    x = synth.x_range(2206083555, 0, n) * scale
    if dist == "cubed":
        x = x ** 3  # heavier tail: larger max / rms
    Xd = torch.from_numpy(x).cuda()
    F = dn.to_fx20(Xd)
    h = F.header()
    buf = F.buf.cpu().numpy()
    hi = buf[256:256 + 2 * n].view(np.float16).astype(np.float64)
    lo_off = 256 + (2 * n + 255) // 256 * 256
    lo = buf[lo_off:lo_off + n].view(np.int8).astype(np.float64)
    dec = (256.0 * hi + lo) * 2.0 ** h["exp2"]
    rel = np.linalg.norm(x - dec) / np.linalg.norm(x)
    assert h["count"] == n and h["max_abs"] == float(np.abs(x).max())
    assert h["storage_rel_err"] == pytest.approx(rel, rel=1e-6)
    assert h["rms"] == pytest.approx(float(np.sqrt(np.mean(x * x))), rel=1e-6)


def test_auto_ttmc_fp32_storage(dn, synth, oracle_mod):
    dims, ranks = (64, 48, 200), (8, 12)
    rng = np.random.default_rng(2206083556)
    X = synth.x_tensor(2206083557, dims)
    U = [None, rng.standard_normal((48, 8)), rng.standard_normal((200, 12))]
    ref = oracle_mod.ttmc(X, U, 0)
    rep = dn.Report()
    Y = dn.ttmc(ttmc_spec(3, 0), to_dev(X, torch.float32), [to_dev(u, torch.float32) for u in U[1:]],
                precision="auto", tol=1e-5, out_dtype=torch.float64, report=rep)
    torch.cuda.synchronize()
    err = nrel(Y.cpu().numpy(), ref)
    assert dn.PRECISION_NAMES[rep.precision] == "fp32"
    assert err <= rep.est_err <= 1e-5
