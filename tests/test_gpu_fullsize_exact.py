"""Integer-valued inputs at the full one-GPU shapes in every precision form:
X in {-2..2} from the counter generator, integer factors.  Every product and
partial sum is an integer small enough for the form's arithmetic, so each
form must reproduce the oracle exactly on the sampled output rows / slabs."""
import numpy as np
import pytest
import torch

from gpu_common import SPEC3, flush, mttkrp_spec, to_dev, ttmc_spec

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def dn():
    import paper_2206_08301_amd as m
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    m._lib.load()
    return m


def test_mttkrp_1024cubed_integer_exact_every_form(dn, synth, oracle_mod):
    dims, R = (1024, 1024, 1024), 24
    seed = synth.config_seed(2, 50)
    X = torch.empty(dims, dtype=torch.float64, device="cuda")
    dn.synth_fill(X, seed, dist="int5")
    U = [synth.int_factor(seed + 1 + m, 1024, R) for m in range(3)]
    rows = {0: (0, 999), 1: (3, 512), 2: (1023, 64)}
    refs = {}
    for n in range(3):
        Un = [None if m == n else U[m] for m in range(3)]
        for i in rows[n]:
            refs[(n, i)] = oracle_mod.mttkrp(synth.x_slab(seed, dims, n, i, dist="int5"), Un, n)[0]
    X32 = torch.empty(dims, dtype=torch.float32, device="cuda")
    dn.convert(X, X32)
    forms = {"fp64": (X, torch.float64), "fp32": (X32, torch.float32), "bf16x3": (X32, torch.float32)}
    for prec, (Xp, udt) in forms.items():
        for n in range(3):
            flush(f"1024^3 integer {prec} mode {n}")
            ops = [to_dev(U[m], udt) for m in range(3) if m != n]
            M = dn.mttkrp(SPEC3[n], Xp, ops, precision=prec, out_dtype=torch.float64)
            torch.cuda.synchronize()
            Mh = M.cpu().numpy()
            for i in rows[n]:
                assert np.array_equal(Mh[i], refs[(n, i)]), (prec, n, i)
    del X32
    torch.cuda.empty_cache()
    Xb = torch.empty(dims, dtype=torch.bfloat16, device="cuda")
    dn.convert(X, Xb)
    Xf = dn.to_fx20(X)
    for prec, Xp in (("bf16", Xb), ("fx20", Xf)):
        for n in range(3):
            flush(f"1024^3 integer {prec} mode {n}")
            ops = [to_dev(U[m], torch.float32) for m in range(3) if m != n]
            M = dn.mttkrp(SPEC3[n], Xp, ops, precision=prec, out_dtype=torch.float64)
            torch.cuda.synchronize()
            Mh = M.cpu().numpy()
            for i in rows[n]:
                assert np.array_equal(Mh[i], refs[(n, i)]), (prec, n, i)
    del X, Xb, Xf
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dims,rank", [((1024, 1024, 1024), 32), ((192, 192, 192, 192), 16)])
def test_ttmc_full_size_integer_exact(dn, synth, oracle_mod, dims, rank):
    N = len(dims)
    seed = synth.config_seed(4, 60 + N)
    X = torch.empty(dims, dtype=torch.float64, device="cuda")
    dn.synth_fill(X, seed, dist="int3")
    U = [None] + [synth.int_factor(seed + 1 + m, dims[m], rank, -1, 1) for m in range(1, N)]
    spec = ttmc_spec(N, 0)
    X32 = torch.empty(dims, dtype=torch.float32, device="cuda")
    dn.convert(X, X32)
    Xf = dn.to_fx20(X)
    for prec, Xp, dt in (("fp64", X, torch.float64), ("fp32", X32, torch.float32), ("fx20", Xf, torch.float32)):
        flush(f"TTMc integer {prec} dims={dims}")
        Y = dn.ttmc(spec, Xp, [to_dev(u, dt) for u in U[1:]], precision=prec, out_dtype=torch.float64)
        torch.cuda.synchronize()
        for i in (0, dims[0] // 2 + 1):
            ref = oracle_mod.ttmc(synth.x_slab(seed, dims, 0, i, dist="int3"), U, 0)[0]
            assert np.array_equal(Y[i].cpu().numpy(), ref), (prec, i)
    del X, X32, Xf
    torch.cuda.empty_cache()


def test_order5_60_last_mode_and_ttmc(dn, synth, oracle_mod):
    """The paper's order-5 forms at I = 60, R = 24: MTTKRP in the last mode (FP64, sampled
    rows against the oracle) and TTMc in mode 0 (FP64 on integer inputs, sampled slabs
    exact; the FP32, BF16 and FX20 forms exact too on these integer inputs)."""
    dims, R = (60,) * 5, 24
    seed = synth.config_seed(3, 70)
    X = torch.empty(dims, dtype=torch.float64, device="cuda")
    dn.synth_fill(X, seed, dist="int3")
    U = [synth.int_factor(seed + 1 + m, 60, R, -1, 1) for m in range(5)]
    flush("60^5 MTTKRP mode 4")
    M = dn.mttkrp(mttkrp_spec(5, 4), X, [to_dev(U[m]) for m in range(4)])
    torch.cuda.synchronize()
    for i in (0, 37, 59):
        ref = oracle_mod.mttkrp(synth.x_slab(seed, dims, 4, i, dist="int3"), [U[0], U[1], U[2], U[3], None], 4)[0]
        assert np.array_equal(M[i].cpu().numpy(), ref), i
    flush("60^5 TTMc mode 0")
    Y = dn.ttmc(ttmc_spec(5, 0), X, [to_dev(U[m]) for m in range(1, 5)])
    torch.cuda.synchronize()
    for i in (1, 42):
        ref = oracle_mod.ttmc(synth.x_slab(seed, dims, 0, i, dist="int3"), [None] + U[1:], 0)[0]
        assert np.array_equal(Y[i].cpu().numpy(), ref), i
    X32 = torch.empty(dims, dtype=torch.float32, device="cuda")
    dn.convert(X, X32)
    X16 = torch.empty(dims, dtype=torch.bfloat16, device="cuda")
    dn.convert(X, X16)
    Xf = dn.to_fx20(X)
    for prec, Xp in (("fp32", X32), ("bf16", X16), ("fx20", Xf)):
        flush(f"60^5 TTMc mode 0 {prec}")
        Yp = dn.ttmc(ttmc_spec(5, 0), Xp, [to_dev(U[m], torch.float32) for m in range(1, 5)], precision=prec,
                     out_dtype=torch.float64)
        torch.cuda.synchronize()
        assert torch.equal(Yp, Y), prec  # integer inputs: exact in every form
    del X, X32, X16, Xf, Y
    torch.cuda.empty_cache()
