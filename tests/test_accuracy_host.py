"""Host tests (no GPU) of the tolerance-driven form choice: deinsum_estimate_error,
DEINSUM_PREC_AUTO's selection table and deinsum_choose_storage.

The estimate is a stated model (include/deinsum.h): these tests check that the library
applies the rule as stated, that each storage offers exactly its forms, and that the
choice moves between forms and storages as the tolerance moves.  Whether the model holds
for real results is checked on the GPU against the oracle (test_gpu_auto.py)."""
import math

import pytest

S0, S1, S2 = "ijk,ja,ka->ia", "ijk,ia,ka->ja", "ijk,ia,ja->ka"
D3 = (1024, 1024, 1024)
U32, UBF, UH, U64 = 2.0 ** -24, 2.0 ** -8, 2.0 ** -11, 2.0 ** -53


@pytest.fixture(scope="module")
def dn():
    import paper_2206_08301_amd as m
    m._lib.load()
    return m


def documented_rule(prec, N, L, k, dx_fx20=None):
    """The estimate as include/deinsum.h states it, restated here independently."""
    r3 = math.sqrt(3.0)
    rnd = {"f32": U32 / r3, "bf": UBF / r3}
    split_bf, split_h = UBF ** 2 / 3, UH ** 2 / 3
    acc64 = U64 * math.sqrt(L / 3)
    acc32 = U32 * math.sqrt(k / 3)
    if prec == "fp64":
        terms = [acc64]
    elif prec == "fp32":
        terms = [rnd["f32"], rnd["f32"]] + [rnd["f32"]] * (N - 2) + [acc64 + acc32]
    elif prec == "bf16":
        terms = [rnd["bf"], math.hypot(rnd["f32"], rnd["bf"])] + [rnd["f32"]] * (N - 2) + [acc64 + acc32]
    elif prec == "bf16x3":
        s = math.hypot(rnd["f32"], split_bf)
        terms = [s, s] + [rnd["f32"]] * (N - 2) + [split_bf, acc64 + acc32]
    elif prec == "fx20":
        terms = [dx_fx20, math.hypot(rnd["f32"], split_h)] + [rnd["f32"]] * (N - 2) + [split_h, acc64 + 2 * acc32]
    return 2 * math.sqrt(sum(t * t for t in terms))


@pytest.mark.parametrize("spec", [S0, S1, S2])
def test_fp64_estimate_follows_rule(dn, spec):
    form, est = dn.estimate_error(spec, D3, [24], "fp64")
    assert form == "fp64"
    assert est == pytest.approx(documented_rule("fp64", 3, 1024.0 ** 2, 1), rel=1e-12)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3"])
def test_reduced_estimates_follow_rule_for_some_compiled_slice(dn, prec):
    """The FP32 chain length k is the plan's slice, a multiple of 32 up to 512: the
    estimate must equal the rule for one of those k."""
    _, est = dn.estimate_error(S1, D3, [24], prec)
    cands = [documented_rule(prec, 3, 1024.0 ** 2, k) for k in range(4, 1025, 4)]
    assert min(abs(est - c) / c for c in cands) < 1e-12


def test_estimates_order_by_form(dn):
    e = {p: dn.estimate_error(S0, D3, [24], p)[1] for p in ("fp64", "fp32", "bf16x3", "bf16")}
    assert e["fp64"] < 1e-12 < e["fp32"] < 1e-5 < e["bf16x3"] < 1e-4 < e["bf16"] < 1e-2


def test_fp64_estimate_grows_with_contraction_length(dn):
    _, small = dn.estimate_error(S0, (64, 64, 64), [16], "fp64")
    _, big = dn.estimate_error("abcde,bz,cz,dz,ez->az", (80,) * 5, [24], "fp64")
    assert small < big < 1e-12  # 80^5 mode 0 sums 80^4 terms and still meets 1e-12


@pytest.mark.parametrize("tol,x,u,want", [
    (1e-12, "F64", "F64", "fp64"),
    (1e-5, "F32", "F32", "fp32"),      # BF16X3's estimate (1.8e-5) is above 1e-5
    (1e-4, "F32", "F32", "bf16x3"),    # both meet it: the faster BF16X3
    (1e-2, "BF16", "F32", "bf16"),
])
def test_auto_selection_table(dn, tol, x, u, want):
    form, est = dn.estimate_error(S0, D3, [24], "auto", tol=tol, x_dtype=getattr(dn, x), u_dtype=getattr(dn, u))
    assert form == want and est <= tol


@pytest.mark.parametrize("tol,x,u", [
    (1e-12, "F32", "F32"),   # no FP32-storage form meets 1e-12
    (1e-3, "BF16", "F32"),   # BF16's estimate is above 1e-3
    (1e-2, "F64", "F32"),    # no compiled form reads F64 X with F32 factors
    (1e-2, "F32", "F64"),
])
def test_auto_rejects_storage_that_cannot_meet_tol(dn, tol, x, u):
    with pytest.raises(dn.DeinsumError) as ei:
        dn.estimate_error(S0, D3, [24], "auto", tol=tol, x_dtype=getattr(dn, x), u_dtype=getattr(dn, u))
    assert ei.value.status == -3


def test_auto_argument_errors(dn):
    with pytest.raises(dn.DeinsumError) as ei:
        dn.estimate_error(S0, D3, [24], "auto", tol=0.0, x_dtype=dn.F32, u_dtype=dn.F32)
    assert ei.value.status == -1
    with pytest.raises(dn.DeinsumError) as ei:
        dn.estimate_error(S0, D3, [24], "auto", tol=1e-3, x_dtype=9, u_dtype=dn.F32)
    assert ei.value.status == -1
    with pytest.raises(dn.DeinsumError) as ei:  # FX20's estimate needs the buffer's header
        dn.estimate_error(S0, D3, [24], "auto", tol=1e-3, x_dtype=dn.FX20_STORAGE, u_dtype=dn.F32)
    assert ei.value.status == -1


def test_ttmc_forms(dn):
    spec, ranks = "ijk,jb,kc->ibc", [32, 32]
    assert dn.estimate_error(spec, D3, ranks, "auto", tol=1e-5, x_dtype=dn.F32, u_dtype=dn.F32)[0] == "fp32"
    with pytest.raises(dn.DeinsumError):  # the FX20 estimate needs the buffer's header
        dn.estimate_error(spec, D3, ranks, "auto", tol=1e-5, x_dtype=dn.FX20_STORAGE, u_dtype=dn.F32)
    _, e32 = dn.estimate_error(spec, D3, ranks, "fp32")
    assert e32 == pytest.approx(documented_rule("fp32", 3, 1024.0 ** 2, 2048), rel=1e-12)


UNIFORM = (1.0 - 2.0 ** -30, 3 ** -0.5)  # max |x| and rms of uniform [-1, 1) data


@pytest.mark.parametrize("tol,want", [
    (1e-12, ("f64", "fp64")),
    (1e-7, ("f64", "fp64")),
    (1e-5, ("fx20", "fx20")),
    (1e-2, ("bf16", "bf16")),
])
def test_choose_storage_table(dn, tol, want):
    storage, form, est = dn.choose_storage(S0, D3, [24], tol, *UNIFORM)
    assert (storage, form) == want and est <= tol


def test_choose_storage_fx20_model(dn):
    """Uniform data: max just under 1 gives e = -19, element errors uniform in
    +-2^-20, so the storage error is 2^-20 / (sqrt(3) rms) = 2^-20."""
    _, _, est = dn.choose_storage(S0, D3, [24], 1e-5, *UNIFORM)
    cands = [documented_rule("fx20", 3, 1024.0 ** 2, k, dx_fx20=2.0 ** -20) for k in range(32, 1025, 32)]
    assert min(abs(est - c) / c for c in cands) < 1e-9


def test_choose_storage_without_stats_skips_fx20(dn):
    assert dn.choose_storage(S0, D3, [24], 1e-5)[:2] == ("f32", "fp32")
    assert dn.choose_storage(S0, D3, [24], 1e-4)[:2] == ("f32", "bf16x3")
    with pytest.raises(dn.DeinsumError) as ei:
        dn.choose_storage(S0, D3, [24], 1e-15)
    assert ei.value.status == -3


def test_choose_storage_heavy_tailed_data_avoids_fx20(dn):
    """A large max / rms (one big outlier) makes the one-exponent FX20 storage coarse:
    the choice moves to F32."""
    storage, _, _ = dn.choose_storage(S0, D3, [24], 1e-5, 1000.0, 1.0)
    assert storage == "f32"


def test_opts_defaults(dn):
    o = dn._lib.Opts()
    dn._lib.load().deinsum_opts_init(o)
    assert (o.precision, o.out_dtype, o.tol, o.x_dtype, o.u_dtype, o.deterministic) == (0, 0, 1e-12, 0, 0, 1)
