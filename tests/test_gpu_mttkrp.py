"""GPU parity of the HIP MTTKRP path against the CPU oracle (through the C ABI)."""
import numpy as np
import pytest
import torch

from gpu_common import SPEC3, flush, mttkrp_spec, nrel, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dn():
    import paper_2206_08301_amd as m
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    m._lib.load()
    return m


def run(dn, spec, X, U, **kw):
    out = dn.einsum(spec, X, *U, **kw)
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


def factors_for(rng, dims, R, n):
    return [None if m == n else rng.standard_normal((d, R)) for m, d in enumerate(dims)]


def operands(U, n):
    return [u for m, u in enumerate(U) if m != n]


# ------------------------------------------------------------------ input generator
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
@pytest.mark.parametrize("dist", ["uniform", "int5", "int3"])
def test_device_generator_matches_host(dn, synth, dtype, dist):
    n, off, seed = 300_001, 12345, 2206083111
    t = torch.empty(n, dtype=dtype, device="cuda")
    dn.synth_fill(t, seed, dist=dist, offset=off)
    host = synth.x_values(seed, np.arange(off, off + n, dtype=np.uint64), dist)
    got = t.cpu()
    if dtype == torch.float64:
        assert np.array_equal(got.numpy(), host)
    elif dtype == torch.float32:
        assert np.array_equal(got.numpy(), host.astype(np.float32))
    else:
        ref = synth.bf16_round(host.astype(np.float32))
        assert np.array_equal(got.float().numpy(), ref)


# ------------------------------------------------------------------ small config (64^3, R=16)
def test_small_config_mode0(dn, synth, oracle_mod):
    dims, R = (64, 64, 64), 16
    X = synth.x_tensor(synth.config_seed(1, 0), dims)
    U = [None] + [synth.normal_factor(synth.config_seed(1, 1 + m), 64, R) for m in (1, 2)]
    ref = oracle_mod.mttkrp(X, U, 0)
    got = run(dn, SPEC3[0], to_dev(X), [to_dev(u) for u in U[1:]])
    assert nrel(got, ref) <= 1e-12


SHAPES = [
    ((97, 80, 33), (1, 8, 24)),
    ((33, 17, 45), (16, 64)),
    ((16, 64, 128), (24, 100)),
    ((5, 3, 130), (3,)),
    ((40, 50), (24, 7)),
    ((12, 7, 9, 20), (24,)),
    ((6, 5, 4, 7, 80), (24,)),
    ((7, 9, 6, 8, 5), (5, 33)),
]


@pytest.mark.parametrize("dims,Rs", SHAPES)
def test_fp64_all_modes(dn, oracle_mod, dims, Rs):
    rng = np.random.default_rng(sum(dims))
    X = rng.uniform(-1, 1, dims)
    Xd = to_dev(X)
    for R in Rs:
        for n in range(len(dims)):
            flush(f"fp64 dims={dims} R={R} n={n}")
            U = factors_for(rng, dims, R, n)
            ref = oracle_mod.mttkrp(X, U, n)
            got = run(dn, mttkrp_spec(len(dims), n), Xd, [to_dev(u) for u in operands(U, n)])
            assert nrel(got, ref) <= 1e-12, (dims, R, n)


def test_operand_order_is_respected(dn, oracle_mod):
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (9, 10, 11))
    B, C = rng.standard_normal((10, 4)), rng.standard_normal((11, 4))
    ref = oracle_mod.mttkrp(X, [None, B, C], 0)
    got = run(dn, "ijk,ka,ja->ia", to_dev(X), [to_dev(C), to_dev(B)])
    assert nrel(got, ref) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16", "bf16x3"])
@pytest.mark.parametrize("dims,R", [((37, 64, 96), 20), ((16, 21, 130), 20), ((6, 5, 7, 48), 20), ((64, 64, 64), 20),
                                    ((40, 33, 80), 50), ((24, 96, 64), 64)])
def test_integer_inputs_exact_every_form(dn, synth, oracle_mod, precision, dims, R):
    """Entries in {-2..2}: every partial sum is an integer below 2^24, exact in all forms."""
    rng = np.random.default_rng(len(dims) * 7 + dims[0])
    X = synth.x_tensor(77, dims, "int5")
    xdt = {"fp64": torch.float64, "fp32": torch.float32, "bf16": torch.bfloat16, "bf16x3": torch.float32}[precision]
    udt = torch.float64 if precision == "fp64" else torch.float32
    Xd = to_dev(X, xdt)
    for n in range(len(dims)):
        flush(f"int {precision} dims={dims} n={n}")
        U = [None if m == n else rng.integers(-2, 3, (d, R)).astype(np.float64) for m, d in enumerate(dims)]
        ref = oracle_mod.mttkrp(X, U, n)
        got = run(dn, mttkrp_spec(len(dims), n), Xd, [to_dev(u, udt) for u in operands(U, n)],
                  precision=precision, out_dtype=torch.float64)
        assert np.array_equal(got, ref), (precision, dims, n)


def test_run_to_run_bitwise(dn):
    rng = np.random.default_rng(3)
    X = to_dev(rng.uniform(-1, 1, (128, 96, 160)))
    U = [to_dev(rng.standard_normal((d, 24))) for d in (128, 96, 160)]
    for n in range(3):
        ops = [U[m] for m in range(3) if m != n]
        a = dn.einsum(SPEC3[n], X, *ops)
        b = dn.einsum(SPEC3[n], X, *ops)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


def test_library_pool_per_stream(dn):
    """Calls without a workspace of their own on two streams, enqueued back to back with
    no synchronisation between them, each get their stream's pool buffer: every output
    equals the same call run alone."""
    rng = np.random.default_rng(11)
    probs = []
    for dims, R in (((96, 640, 320), 24), ((200, 48, 700), 40)):
        X = to_dev(rng.uniform(-1, 1, dims))
        U = [to_dev(rng.standard_normal((d, R))) for d in dims]
        probs.append((X, U))
    specs = [(p, n) for p in range(2) for n in range(3)]
    need = [dn.workspace_size(SPEC3[n], tuple(probs[p][0].shape), [probs[p][1][0].shape[1]]) for p, n in specs]
    assert sum(w > 0 for w in need) >= 2, need  # pool buffers are really in play on both streams
    alone = {}
    for p, n in specs:
        X, U = probs[p]
        alone[(p, n)] = dn.mttkrp(SPEC3[n], X, [U[m] for m in range(3) if m != n])
        torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    for rep in range(3):
        outs = {}
        for k, (p, n) in enumerate(specs):
            X, U = probs[p]
            outs[(p, n)] = dn.mttkrp(SPEC3[n], X, [U[m] for m in range(3) if m != n], stream=streams[k % 2])
        torch.cuda.synchronize()
        for key, out in outs.items():
            assert torch.equal(out, alone[key]), (rep, key)


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-6), ("bf16x3", 1e-5), ("bf16", 2e-2)])
def test_mixed_precision_error(dn, synth, oracle_mod, precision, tol):
    dims, R = (96, 128, 256), 24
    X = synth.x_tensor(4242, dims)
    rng = np.random.default_rng(9)
    xdt = torch.bfloat16 if precision == "bf16" else torch.float32
    Xd = to_dev(X, torch.float32) if xdt == torch.float32 else to_dev(X, torch.float32).to(torch.bfloat16)
    for n in range(3):
        U = factors_for(rng, dims, R, n)
        ref = oracle_mod.mttkrp(X, U, n)
        got = run(dn, SPEC3[n], Xd, [to_dev(u, torch.float32) for u in operands(U, n)], precision=precision)
        err = nrel(got, ref)
        flush(f"{precision} mode {n}: normwise error {err:.3e}")
        assert err <= tol


def test_degenerate_and_empty(dn, oracle_mod):
    rng = np.random.default_rng(4)
    for dims in [(1, 1, 1), (1, 5, 1), (3, 1, 7), (1, 1, 300)]:
        X = rng.uniform(-1, 1, dims)
        for n in range(3):
            U = factors_for(rng, dims, 1, n)
            got = run(dn, SPEC3[n], to_dev(X), [to_dev(u) for u in operands(U, n)])
            assert nrel(got, oracle_mod.mttkrp(X, U, n)) <= 1e-12
    # an empty contracted mode: the sum is empty, M = 0
    X = torch.empty((5, 0, 4), dtype=torch.float64, device="cuda")
    B = torch.empty((0, 3), dtype=torch.float64, device="cuda")
    C = torch.ones((4, 3), dtype=torch.float64, device="cuda")
    out = torch.full((5, 3), 7.0, dtype=torch.float64, device="cuda")
    dn.einsum(SPEC3[0], X, B, C, out=out)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0


def test_output_canaries_untouched(dn, oracle_mod):
    rng = np.random.default_rng(6)
    dims, R = (50, 40, 70), 24
    X = rng.uniform(-1, 1, dims)
    for n in range(3):
        U = factors_for(rng, dims, R, n)
        buf = torch.full((dims[n] * R + 2048,), -123.5, dtype=torch.float64, device="cuda")
        out = buf[1024:1024 + dims[n] * R].view(dims[n], R)
        dn.einsum(SPEC3[n], to_dev(X), *[to_dev(u) for u in operands(U, n)], out=out)
        torch.cuda.synchronize()
        assert torch.all(buf[:1024] == -123.5) and torch.all(buf[1024 + dims[n] * R:] == -123.5)
        assert nrel(out.cpu().numpy(), oracle_mod.mttkrp(X, U, n)) <= 1e-12


def test_full_size_1024cubed_sampled_rows(dn, synth, oracle_mod):
    """X 1024^3 FP64 generated on the device (8 GiB), R = 24, every mode, in the
    benchmark's launch configuration; sampled output rows against the oracle on
    host slabs produced by the host generator."""
    dims, R = (1024, 1024, 1024), 24
    seed = synth.config_seed(2, 0)
    X = torch.empty(dims, dtype=torch.float64, device="cuda")
    dn.synth_fill(X, seed)
    U = [synth.normal_factor(synth.config_seed(2, 1 + m), 1024, R) for m in range(3)]
    Ud = [to_dev(u) for u in U]
    for n in range(3):
        flush(f"1024^3 mode {n}")
        M = dn.einsum(SPEC3[n], X, *[Ud[m] for m in range(3) if m != n])
        torch.cuda.synchronize()
        Mh = M.cpu().numpy()
        for i in (0, 517, 1023):
            slab = synth.x_slab(seed, dims, n, i)
            Un = [None if m == n else U[m] for m in range(3)]
            ref = oracle_mod.mttkrp(slab, Un, n)[0]
            assert nrel(Mh[i], ref) <= 1e-12, (n, i)
    del X
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision,tol", [("fx20", 4e-6), ("bf16x3", 1e-5), ("bf16", 2e-2)])
@pytest.mark.parametrize("dims", [(9, 7, 10, 80), (5, 6, 4, 9, 80), (3, 4, 33, 50)])
def test_merged_last_modes_match_unmerged(dn, synth, oracle_mod, precision, tol, dims):
    """Free mode n <= N-3 in the 32-element K-step forms: the default plan runs the last two
    modes as one (their Khatri-Rao factor built per call, plan name ending " m2"); it and the
    unmerged heuristic plan (plan_hint 1) both meet the form's bound against the oracle."""
    N = len(dims)
    R = 24
    X = synth.x_tensor(4343 + N, dims)
    rng = np.random.default_rng(N)
    if precision == "fx20":
        Xd = dn.to_fx20(to_dev(X))
    elif precision == "bf16":
        Xd = to_dev(X, torch.float32).to(torch.bfloat16)
    else:
        Xd = to_dev(X, torch.float32)
    for n in range(N - 2):
        U = factors_for(rng, dims, R, n)
        U = [None if u is None else u.astype(np.float32).astype(np.float64) for u in U]
        ref = oracle_mod.mttkrp(X, U, n)
        ops = [to_dev(u, torch.float32) for u in operands(U, n)]
        rep = dn.Report()
        merged = dn.mttkrp(mttkrp_spec(N, n), Xd, ops, precision=precision, out_dtype=torch.float64, report=rep)
        plain = dn.mttkrp(mttkrp_spec(N, n), Xd, ops, precision=precision, out_dtype=torch.float64, plan_hint=1)
        torch.cuda.synchronize()
        name = rep.plan_name.decode()
        flush(f"{precision} dims={dims} n={n}: {name}")
        assert name.endswith(" m2"), name
        nx = float(np.prod(dims))
        assert rep.alg_bytes == pytest.approx(nx * {"fx20": 3, "bf16": 2, "bf16x3": 4}[precision]
                                              + sum(d * R * 4 for m, d in enumerate(dims) if m != n)
                                              + dims[n] * R * 8)
        assert nrel(merged.cpu().numpy(), ref) <= tol
        assert nrel(plain.cpu().numpy(), ref) <= tol


@pytest.mark.parametrize("dims,R", [((33, 70, 130), 24), ((20, 64, 300), 64), ((17, 9, 40), 5)])
def test_mode0_through_fused_ttmc_pass(dn, oracle_mod, tmp_path, dims, R):
    """Order-3 mode 0 in FP64 through the fused TTMc pass (selected here by a plan-cache
    entry with order 2), against the oracle and against the K-contiguous kernel."""
    rng = np.random.default_rng(R + dims[2])
    X = rng.uniform(-1, 1, dims)
    U = factors_for(rng, dims, R, 0)
    ref = oracle_mod.mttkrp(X, U, 0)
    Xd, ops = to_dev(X), [to_dev(u) for u in operands(U, 0)]
    dn.tune_clear()
    dn.tune_mttkrp(SPEC3[0], Xd, ops, reps=1)
    cache = tmp_path / "cache.txt"
    dn.tune_save(str(cache))
    key = [l.split()[0] for l in cache.read_text().splitlines() if l.strip() and not l.startswith("#")][0]
    for hint in (1, 2):
        cache.write_text(f"{key} 1 1 1 0 {hint - 1} 2 0 0\n")
        dn.tune_clear()
        dn.tune_load(str(cache))
        rep = dn.Report()
        got = dn.mttkrp(SPEC3[0], Xd, ops, report=rep)
        torch.cuda.synchronize()
        name = rep.plan_name.decode()
        flush(f"dims={dims} R={R}: {name}")
        assert name.startswith("mttkrp_via_ttmc"), name
        assert nrel(got.cpu().numpy(), ref) <= 1e-12
    dn.tune_clear()
    plain = dn.mttkrp(SPEC3[0], Xd, ops, plan_hint=1)
    torch.cuda.synchronize()
    assert nrel(plain.cpu().numpy(), ref) <= 1e-12


@pytest.mark.parametrize("dims,R,L", [((33, 70, 130), 24, 16), ((9, 11, 13, 17), 5, 3), ((64, 64, 64), 16, 40)])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("bf16x3", 1e-5), ("fx20", 4e-6)])
def test_mttkrp_gemm_chain(dn, oracle_mod, dims, R, L, precision, tol):
    """The MTTKRP-GEMM chain of the paper's running example through the C ABI, every mode."""
    N = len(dims)
    rng = np.random.default_rng(sum(dims) + R + L)
    X = rng.uniform(-1, 1, dims)
    if precision == "fp64":
        Xd, udt = to_dev(X), torch.float64
    elif precision == "fx20":
        Xd, udt = dn.to_fx20(to_dev(X)), torch.float32
    else:
        X = X.astype(np.float32).astype(np.float64)
        Xd, udt = to_dev(X, torch.float32), torch.float32
    letters = "ijklmnop"[:N]
    for n in range(N):
        U = factors_for(rng, dims, R, n)
        if udt == torch.float32:
            U = [None if u is None else u.astype(np.float32).astype(np.float64) for u in U]
        C = rng.standard_normal((R, L))
        if udt == torch.float32:
            C = C.astype(np.float32).astype(np.float64)
        spec = letters + "," + ",".join(letters[m] + "z" for m in range(N) if m != n) + ",zy->" + letters[n] + "y"
        got = dn.einsum(spec, Xd, *[to_dev(u, udt) for u in operands(U, n)], to_dev(C, udt), precision=precision,
                        out_dtype=torch.float64)
        torch.cuda.synchronize()
        ref = oracle_mod.mttkrp_mm(X, U, n, C)
        err = nrel(got.cpu().numpy(), ref)
        flush(f"chain {precision} dims={dims} n={n}: {err:.2e}")
        assert got.shape == (dims[n], L)
        assert err <= tol, (precision, dims, n)


def test_mttkrp_gemm_chain_1024cubed(dn, synth, oracle_mod):
    """"ijk,ja,ka,al->il" at the one-GPU tile shape (R=24, L=16), sampled rows."""
    dims, R, L = (1024, 1024, 1024), 24, 16
    seed = synth.config_seed(2, 80)
    X = torch.empty(dims, dtype=torch.float64, device="cuda")
    dn.synth_fill(X, seed)
    U = [synth.normal_factor(seed + 1 + m, 1024, R) for m in range(3)]
    C = np.random.default_rng(seed).standard_normal((R, L))
    Y = dn.einsum("ijk,ja,ka,al->il", X, to_dev(U[1]), to_dev(U[2]), to_dev(C))
    torch.cuda.synchronize()
    for i in (0, 777):
        ref = oracle_mod.mttkrp_mm(synth.x_slab(seed, dims, 0, i), [None, U[1], U[2]], 0, C)[0]
        assert nrel(Y[i].cpu().numpy(), ref) <= 1e-12, i
    del X
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", ["fx20", "bf16", "bf16x3"])
@pytest.mark.parametrize("dims", [(64, 64, 64), (20, 30, 45)])
def test_order3_mode0_never_merges_last_modes(dn, synth, oracle_mod, precision, dims):
    """Order 3, free mode 0, a short or ragged last mode: the two contracted modes are all
    the other modes, so merging them would store the whole Khatri-Rao product; the plan
    must stay unmerged (no " m2") and still meet the form's bound against the oracle."""
    R = 16
    X = synth.x_tensor(4545, dims)
    rng = np.random.default_rng(45)
    if precision == "fx20":
        Xd = dn.to_fx20(to_dev(X))
    elif precision == "bf16":
        Xd = to_dev(X, torch.float32).to(torch.bfloat16)
    else:
        Xd = to_dev(X, torch.float32)
    U = factors_for(rng, dims, R, 0)
    U = [None if u is None else u.astype(np.float32).astype(np.float64) for u in U]
    rep = dn.Report()
    got = dn.mttkrp(SPEC3[0], Xd, [to_dev(u, torch.float32) for u in operands(U, 0)], precision=precision,
                    out_dtype=torch.float64, report=rep)
    torch.cuda.synchronize()
    name = rep.plan_name.decode()
    flush(f"{precision} dims={dims}: {name}")
    assert not name.endswith(" m2"), name
    tol = {"fx20": 4e-6, "bf16x3": 1e-5, "bf16": 2e-2}[precision]
    assert nrel(got.cpu().numpy(), oracle_mod.mttkrp(X, U, 0)) <= tol


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("dims", [(30, 50, 60), (7, 9, 11, 64), (40, 33, 45), (20, 24, 17)])
def test_short_last_mode(dn, oracle_mod, prec, tol, dims):
    """Last-mode MTTKRP whose contiguous output mode has at most 64 elements: the default
    plan keeps each X row in one 64-index tile when 32 < I_last <= 64 (the FP64 form then
    scales the factor operand by the step weights and accumulates on the matrix cores);
    uniform inputs against the oracle, integer inputs exact."""
    rng = np.random.default_rng(sum(dims))
    N, n, R = len(dims), len(dims) - 1, 24
    dt = torch.float64 if prec == "fp64" else torch.float32
    for dist in ("uniform", "int"):
        if dist == "uniform":
            X = rng.uniform(-1, 1, dims)
            U = [rng.standard_normal((d, R)) for d in dims]
        else:
            X = rng.integers(-3, 4, dims).astype(np.float64)
            U = [rng.integers(-2, 3, (d, R)).astype(np.float64) for d in dims]
        rep = dn.Report()
        M = dn.mttkrp(mttkrp_spec(N, n), to_dev(X, dt), [to_dev(U[m], dt) for m in range(N - 1)], precision=prec,
                      out_dtype=torch.float64, report=rep)
        torch.cuda.synchronize()
        name = rep.plan_name.decode()
        flush(f"short last mode {dims} {prec} {dist}: {name}")
        if 32 < dims[-1] <= 64:
            assert ",mt4" in name, name
        ref = oracle_mod.mttkrp(X, U[:-1] + [None], n)
        if dist == "uniform":
            assert nrel(M.cpu().numpy(), ref) <= tol
        else:
            assert np.array_equal(M.cpu().numpy(), ref)


KOUT_FORMS = [("fp32", torch.float32, torch.float32, 1e-6), ("bf16x3", torch.float32, torch.float32, 1e-5),
              ("bf16", torch.bfloat16, torch.float32, 2e-2), ("fx20", None, torch.float32, 4e-6)]


@pytest.mark.parametrize("form,xdt,udt,tol", KOUT_FORMS)
@pytest.mark.parametrize("dims,R", [((40, 70, 200), 24), ((33, 45, 256), 20), ((20, 64, 130), 8), ((17, 48, 96), 40),
                                    ((9, 5, 40), 3)])
def test_mode0_row_walk_every_form(dn, oracle_mod, form, xdt, udt, tol, dims, R):
    """Order-3 mode 0 through the mode-1-tiled walk (plan_hint 3): ragged mode-1 tiles,
    slices past mode 2, one to four column blocks; uniform inputs within each form's
    bound of the oracle, integer inputs exact."""
    rng = np.random.default_rng(sum(dims) + R)
    for dist in ("uniform", "int"):
        if dist == "uniform":
            X = rng.uniform(-1, 1, dims)
            U = [rng.standard_normal((d, R)) for d in dims]
        else:
            X = rng.integers(-3, 4, dims).astype(np.float64)
            U = [rng.integers(-2, 3, (d, R)).astype(np.float64) for d in dims]
        Xd = dn.to_fx20(to_dev(X)) if form == "fx20" else to_dev(X, xdt)
        rep = dn.Report()
        M = dn.mttkrp(mttkrp_spec(3, 0), Xd, [to_dev(U[1], udt), to_dev(U[2], udt)], precision=form,
                      out_dtype=torch.float64, plan_hint=3, report=rep)
        torch.cuda.synchronize()
        name = rep.plan_name.decode()
        assert name.startswith("mttkrp_kout"), name
        ref = oracle_mod.mttkrp(X, [None, U[1], U[2]], 0)
        got = M.cpu().numpy()
        flush(f"row walk {form} {dims} R={R} {dist}: {name}, err {nrel(got, ref):.2e}")
        if dist == "int":
            assert np.array_equal(got, ref)
        else:
            assert nrel(got, ref) <= tol


def test_mode0_row_walk_is_default_for_far_rows(dn, synth):
    """1 MiB or more between consecutive mode-0 rows: the reduced forms take the walk by
    default (FP64 keeps the fused TTMc pass); a short tensor keeps the K-contiguous kernel."""
    big, small = (128, 1024, 1024), (64, 48, 64)
    assert dn.workspace_size(mttkrp_spec(3, 0), big, [24], "fp32") > 0
    for prec, dt in (("fp32", torch.float32), ("bf16x3", torch.float32), ("bf16", torch.bfloat16)):
        for dims, want in ((big, "mttkrp_kout"), (small, "mttkrp_kcontig")):
            X = torch.empty(dims, dtype=dt, device="cuda")
            X.zero_()
            U = [torch.zeros((d, 24), dtype=torch.float32, device="cuda") for d in dims[1:]]
            rep = dn.Report()
            dn.mttkrp(mttkrp_spec(3, 0), X, U, precision=prec, out_dtype=torch.float64, report=rep)
            torch.cuda.synchronize()
            assert rep.plan_name.decode().startswith(want), (prec, dims, rep.plan_name)


# The FP64 64-index last-mode variants: column tiles, K instructions per step, output
# indices per lane, non-temporal loads.
FP64_MT4 = [(2, 4, 4, 1), (2, 4, 4, 0), (2, 2, 4, 1)]


@pytest.mark.parametrize("dims", [(7, 9, 60), (5, 6, 7, 50), (3, 11, 13, 64)])
def test_fp64_short_last_mode_every_variant(dn, oracle_mod, tmp_path, dims):
    """Every FP64 64-index last-mode variant, each forced by a plan-cache entry, on short
    last modes (ragged and whole tiles, contracted extents that leave a partial K step);
    integer inputs, exact against the oracle."""
    rng = np.random.default_rng(sum(dims) + 1)
    N, R = len(dims), 24
    X = rng.integers(-3, 4, dims).astype(np.float64)
    U = [rng.integers(-2, 3, (d, R)).astype(np.float64) for d in dims]
    ref = oracle_mod.mttkrp(X, U[:-1] + [None], N - 1)
    Xd = to_dev(X)
    ops = [to_dev(U[m]) for m in range(N - 1)]
    key = f"s:N{N}:n{N - 1}:p0:R{R}:" + "x".join(str(d) for d in dims)
    cache = tmp_path / "fp64_mt4.txt"
    try:
        for nt, ni, mt, xnt in FP64_MT4:
            cache.write_text(f"{key} {nt} {ni} {mt} {xnt} 0 0 0 1.0\n")
            dn.tune_clear()
            dn.tune_load(cache)
            rep = dn.Report()
            M = dn.mttkrp(mttkrp_spec(N, N - 1), Xd, ops, precision="fp64", out_dtype=torch.float64, report=rep)
            torch.cuda.synchronize()
            name = rep.plan_name.decode()
            flush(f"fp64 short last mode dims={dims}: {name}")
            assert f"mcontig<p0,nt{nt},ni{ni},mt{mt}{',nt' if xnt else ''}>" in name, name
            assert np.array_equal(M.cpu().numpy(), ref), name
    finally:
        dn.tune_clear()
