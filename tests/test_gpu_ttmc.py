"""GPU parity of the HIP TTMc path against the CPU oracle (through the C ABI)."""
import numpy as np
import pytest
import torch

from gpu_common import flush, nrel, to_dev, ttmc_spec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dn():
    import paper_2206_08301_amd as m
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    m._lib.load()
    return m


CASES = [
    ((20, 30, 40), (5, 7, 9)),
    ((64, 70, 130), (16, 32, 24)),
    ((9, 11, 13, 17), (3, 4, 5, 6)),
    ((6, 7, 5, 8, 9), (2, 3, 4, 3, 2)),
    ((33, 47), (5, 6)),
    # remaining product over a 900-long mode: its factor is read from global memory, not LDS
    ((3, 900, 20, 24), (2, 8, 8, 8)),
    # mode 0: a remaining product over 288,000 fibres, more than the pipelined row walk
    # takes (factor in LDS for rank 5; as scalar operands for exactly 8 ranks)
    ((2000, 10, 12, 16), (3, 5, 12, 12)),
    ((2000, 10, 12, 16), (3, 8, 12, 12)),
    # several c-groups per slab (partials reduced) before the remaining products; ragged last tile
    ((5, 6, 7, 300), (3, 4, 5, 6)),
]


@pytest.mark.parametrize("dims,ranks", CASES)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_ttmc_all_modes(dn, oracle_mod, dims, ranks, precision, tol):
    rng = np.random.default_rng(sum(dims) + len(precision))
    X = rng.uniform(-1, 1, dims)
    dt = torch.float64 if precision == "fp64" else torch.float32
    Xd = to_dev(X, dt)
    for n in range(len(dims)):
        flush(f"ttmc {precision} dims={dims} n={n}")
        U = [None if m == n else rng.standard_normal((d, ranks[m])) for m, d in enumerate(dims)]
        ref = oracle_mod.ttmc(X, U, n)
        got = dn.einsum(ttmc_spec(len(dims), n), Xd, *[to_dev(u, dt) for u in U if u is not None],
                        precision=precision, out_dtype=torch.float64)
        torch.cuda.synchronize()
        assert nrel(got.cpu().numpy(), ref) <= tol, (dims, n)


@pytest.mark.parametrize("dims,ranks", CASES)
def test_ttmc_bf16_all_modes(dn, synth, oracle_mod, dims, ranks):
    """BF16 form on inputs already representable in BF16 (X and factors rounded on the host):
    what remains is FP32 accumulation inside a matrix-core step, FP64 beyond."""
    rng = np.random.default_rng(sum(dims) + 16)
    X = synth.bf16_round(rng.uniform(-1, 1, dims)).astype(np.float64)
    Xd = to_dev(X, torch.float32).to(torch.bfloat16)
    for n in range(len(dims)):
        flush(f"ttmc bf16 dims={dims} n={n}")
        U = [None if m == n else synth.bf16_round(rng.standard_normal((d, ranks[m]))).astype(np.float64)
             for m, d in enumerate(dims)]
        ref = oracle_mod.ttmc(X, U, n)
        got = dn.einsum(ttmc_spec(len(dims), n), Xd, *[to_dev(u, torch.float32) for u in U if u is not None],
                        precision="bf16", out_dtype=torch.float64)
        torch.cuda.synchronize()
        assert nrel(got.cpu().numpy(), ref) <= 1e-5, (dims, n)


def test_ttmc_integer_exact(dn, synth, oracle_mod):
    dims = (40, 64, 96)
    X = synth.x_tensor(99, dims, "int5")
    rng = np.random.default_rng(1)
    for precision, dt in [("fp64", torch.float64), ("fp32", torch.float32), ("bf16", torch.bfloat16)]:
        udt = torch.float64 if precision == "fp64" else torch.float32
        for n in range(3):
            U = [None if m == n else rng.integers(-2, 3, (d, 16)).astype(np.float64) for m, d in enumerate(dims)]
            ref = oracle_mod.ttmc(X, U, n)
            Xd = to_dev(X, torch.float32).to(torch.bfloat16) if dt == torch.bfloat16 else to_dev(X, dt)
            got = dn.einsum(ttmc_spec(3, n), Xd, *[to_dev(u, udt) for u in U if u is not None],
                            precision=precision, out_dtype=torch.float64)
            torch.cuda.synchronize()
            assert np.array_equal(got.cpu().numpy(), ref), (precision, n)


def test_ttmc_identity_factors_return_x(dn):
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, (12, 16, 20))
    Xd = to_dev(X)
    got = dn.einsum("ijk,jb,kc->ibc", Xd, to_dev(np.eye(16)), to_dev(np.eye(20)))
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), X)


def test_mttkrp_equals_ttmc_diagonal(dn):
    rng = np.random.default_rng(3)
    X = to_dev(rng.uniform(-1, 1, (50, 60, 70)))
    B, C = to_dev(rng.standard_normal((60, 16))), to_dev(rng.standard_normal((70, 16)))
    M = dn.einsum("ijk,ja,ka->ia", X, B, C)
    Y = dn.einsum("ijk,jb,kc->ibc", X, B, C)
    torch.cuda.synchronize()
    assert nrel(M.cpu().numpy(), torch.diagonal(Y, dim1=1, dim2=2).cpu().numpy()) <= 1e-12


@pytest.mark.parametrize("dims,rank", [((1024, 1024, 1024), 32), ((192, 192, 192, 192), 16)])
def test_full_size_sampled_slabs(dn, synth, oracle_mod, dims, rank):
    """TTMc mode 0 at the full Tucker-step sizes (orthonormal factors), sampled slabs."""
    N = len(dims)
    cfg = 4
    seed = synth.config_seed(cfg, 0) + (0 if N == 3 else 50)
    X = torch.empty(dims, dtype=torch.float64, device="cuda")
    dn.synth_fill(X, seed)
    U = [None] + [synth.orthonormal_factor(synth.config_seed(cfg, 1 + m) + (0 if N == 3 else 50), dims[m], rank)
                  for m in range(1, N)]
    flush(f"ttmc full {dims}")
    Y = dn.einsum(ttmc_spec(N, 0), X, *[to_dev(u) for u in U[1:]])
    torch.cuda.synchronize()
    for i in (0, dims[0] // 2 + 1, dims[0] - 1):
        slab = synth.x_slab(seed, dims, 0, i)
        ref = oracle_mod.ttmc(slab, U, 0)[0]
        assert nrel(Y[i].cpu().numpy(), ref) <= 1e-12, i
    del X
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dims,ranks", [((40, 70, 130), (8, 32, 24)), ((24, 60, 50, 70), (3, 40, 20, 64))])
def test_ttmc_every_kernel_variant(dn, oracle_mod, dims, ranks):
    """Every compiled fused-kernel variant for the ranks (plan_hint = 0, 1, ...) matches the oracle."""
    rng = np.random.default_rng(sum(dims))
    X = rng.uniform(-1, 1, dims)
    Xd = to_dev(X)
    n = 0
    U = [None if m == n else rng.standard_normal((d, ranks[m])) for m, d in enumerate(dims)]
    ref = oracle_mod.ttmc(X, U, n)
    Ud = [to_dev(u) for u in U if u is not None]
    seen = 0
    for v in range(8):
        try:
            got = dn.ttmc(ttmc_spec(len(dims), n), Xd, Ud, variant=v)
        except dn.DeinsumError as e:
            assert e.status == -1  # no such variant
            break
        torch.cuda.synchronize()
        flush(f"ttmc variant {v} dims={dims}: {nrel(got.cpu().numpy(), ref):.2e}")
        assert nrel(got.cpu().numpy(), ref) <= 1e-12, v
        seen += 1
    assert seen >= 1


@pytest.mark.parametrize("dims,ranks", [((40, 70, 130), (8, 32, 24)), ((24, 60, 50, 70), (3, 40, 20, 64)),
                                        ((6, 33, 70), (4, 16, 16))])
def test_ttmc_bf16_every_kernel_variant(dn, synth, oracle_mod, dims, ranks):
    """Every compiled BF16 fused-kernel variant for the ranks, on BF16-representable inputs."""
    rng = np.random.default_rng(sum(dims) + 3)
    X = synth.bf16_round(rng.uniform(-1, 1, dims)).astype(np.float64)
    Xd = to_dev(X, torch.float32).to(torch.bfloat16)
    U = [None] + [synth.bf16_round(rng.standard_normal((d, ranks[m]))).astype(np.float64)
                  for m, d in enumerate(dims) if m > 0]
    ref = oracle_mod.ttmc(X, U, 0)
    Ud = [to_dev(u, torch.float32) for u in U[1:]]
    seen = 0
    for v in range(8):
        try:
            got = dn.ttmc(ttmc_spec(len(dims), 0), Xd, Ud, precision="bf16", out_dtype=torch.float64, variant=v)
        except dn.DeinsumError as e:
            assert e.status == -1  # no such variant
            break
        torch.cuda.synchronize()
        err = nrel(got.cpu().numpy(), ref)
        flush(f"ttmc bf16 variant {v} dims={dims}: {err:.2e}")
        assert err <= 1e-5, v
        seen += 1
    assert seen >= 1


@pytest.mark.parametrize("dims,ranks", CASES)
def test_ttmc_fx20_all_modes(dn, oracle_mod, dims, ranks):
    """FX20 form (X in the 3-byte FX20 storage, FP32 factors): against the oracle on the
    FP64 inputs, within the call's own error estimate and within 1e-5."""
    rng = np.random.default_rng(sum(dims) + 20)
    X = rng.uniform(-1, 1, dims)
    Xf = dn.to_fx20(to_dev(X))
    for n in range(len(dims)):
        flush(f"ttmc fx20 dims={dims} n={n}")
        U = [None if m == n else rng.standard_normal((d, ranks[m])) for m, d in enumerate(dims)]
        ref = oracle_mod.ttmc(X, U, n)
        rep = dn.Report()
        got = dn.einsum(ttmc_spec(len(dims), n), Xf, *[to_dev(u, torch.float32) for u in U if u is not None],
                        precision="fx20", out_dtype=torch.float64, report=rep)
        torch.cuda.synchronize()
        err = nrel(got.cpu().numpy(), ref)
        assert err <= min(1e-5, rep.est_err), (dims, n, err, rep.est_err)


def test_ttmc_fx20_integer_exact(dn, synth, oracle_mod):
    """Integer X in {-2..2} and integer factors: the FX20 codes, the FP16 splits and every
    FP32 partial sum are exact, so the result equals the oracle bit for bit."""
    dims = (40, 64, 96)
    X = synth.x_tensor(98, dims, "int5")
    Xf = dn.to_fx20(to_dev(X))
    rng = np.random.default_rng(4)
    for n in range(3):
        U = [None if m == n else rng.integers(-2, 3, (d, 16)).astype(np.float64) for m, d in enumerate(dims)]
        ref = oracle_mod.ttmc(X, U, n)
        got = dn.einsum(ttmc_spec(3, n), Xf, *[to_dev(u, torch.float32) for u in U if u is not None],
                        precision="fx20", out_dtype=torch.float64)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), ref), n


@pytest.mark.parametrize("dims,ranks", [((40, 70, 132), (8, 32, 24)), ((24, 60, 50, 70), (3, 40, 20, 64)),
                                        ((6, 33, 70), (4, 16, 16))])
def test_ttmc_fx20_every_kernel_variant(dn, oracle_mod, dims, ranks):
    rng = np.random.default_rng(sum(dims) + 5)
    X = rng.uniform(-1, 1, dims)
    Xf = dn.to_fx20(to_dev(X))
    U = [None] + [rng.standard_normal((d, ranks[m])) for m, d in enumerate(dims) if m > 0]
    ref = oracle_mod.ttmc(X, U, 0)
    Ud = [to_dev(u, torch.float32) for u in U[1:]]
    seen = 0
    for v in range(8):
        try:
            got = dn.ttmc(ttmc_spec(len(dims), 0), Xf, Ud, precision="fx20", out_dtype=torch.float64, variant=v)
        except dn.DeinsumError as e:
            assert e.status == -1  # no such variant
            break
        torch.cuda.synchronize()
        err = nrel(got.cpu().numpy(), ref)
        flush(f"ttmc fx20 variant {v} dims={dims}: {err:.2e}")
        assert err <= 1e-5, v
        seen += 1
    assert seen >= 1
