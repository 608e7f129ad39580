"""Full-size parity without sampling, and the order-5 80^5 workload against the oracle.

* 1024^3, R = 24: X is drawn in host RAM by the host generator, uploaded, and the
  oracle computes the WHOLE output of every mode (every one of the 1024 rows, so every
  16-row tile and every partial of the launch the benchmark times).  Integer-valued
  inputs must match exactly in all five forms; uniform inputs within the forms' bounds.
* 80^5, R = 24, modes 0 and 2 (the paper's MTTKRP-O5 forms, Tab. IV, at the size that
  fits one GPU): X is generated on the device (26.2 GB; the device generator is pinned
  bit-identical to the host one), output rows are compared with the oracle on host slabs.
  Mode-0 rows i >= 53 lie wholly past element 2^31 (53 * 80^4 > 2^31).
"""
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


def reduced_copies(dn, Xd, forms):
    """Device copies of X in the storage each form reads (rounded to nearest even)."""
    out = {"fp64": Xd}
    if "fp32" in forms or "bf16x3" in forms:
        X32 = torch.empty(Xd.shape, dtype=torch.float32, device="cuda")
        dn.convert(Xd, X32)
        out["fp32"] = out["bf16x3"] = X32
    if "bf16" in forms:
        Xb = torch.empty(Xd.shape, dtype=torch.bfloat16, device="cuda")
        dn.convert(Xd, Xb)
        out["bf16"] = Xb
    if "fx20" in forms:
        out["fx20"] = dn.to_fx20(Xd)
    return out


def per_row_rel(got, ref):
    d = np.linalg.norm(got - ref, axis=1)
    s = np.linalg.norm(ref, axis=1)
    return d / np.where(s > 0, s, 1.0)


FORMS5 = ("fp64", "fp32", "bf16x3", "bf16", "fx20")


def test_1024cubed_whole_output_integer_exact_every_form(dn, synth, oracle_mod):
    """X in {-2..2}, factors in {-2..2}: every partial sum is an integer below 2^24, so
    every form reproduces the whole oracle output bit for bit, in every mode."""
    dims, R = (1024, 1024, 1024), 24
    seed = synth.config_seed(2, 51)
    flush(f"1024^3 int5 seed={seed}: host generation")
    X = synth.x_range(seed, 0, 1 << 30, "int5").reshape(dims)
    U = [synth.int_factor(seed + 1 + m, 1024, R) for m in range(3)]
    refs = {}
    for n in range(3):
        flush(f"1024^3 int5: oracle mode {n}")
        refs[n] = oracle_mod.mttkrp(X, [None if m == n else U[m] for m in range(3)], n)
    flush("1024^3 int5: upload")
    Xd = torch.from_numpy(X).cuda()
    del X
    copies = reduced_copies(dn, Xd, FORMS5)
    for prec in FORMS5:
        udt = torch.float64 if prec == "fp64" else torch.float32
        for n in range(3):
            flush(f"1024^3 int5 {prec} mode {n}: deinsum_mttkrp")
            ops = [to_dev(U[m], udt) for m in range(3) if m != n]
            M = dn.mttkrp(SPEC3[n], copies[prec], ops, precision=prec, out_dtype=torch.float64)
            torch.cuda.synchronize()
            got = M.cpu().numpy()
            bad = np.argwhere(got != refs[n])
            assert bad.size == 0, (prec, n, bad[:5].tolist())
    del copies, Xd
    torch.cuda.empty_cache()


def test_1024cubed_whole_output_uniform(dn, synth, oracle_mod):
    """The benchmark's inputs (X uniform [-1, 1) from the config-2 seed, N(0,1) factors):
    FP64 within 1e-12 normwise in every output row; the FP32, BF16x3 and FX20 forms within
    1e-5 (whole output and every row); BF16 within 1e-2."""
    dims, R = (1024, 1024, 1024), 24
    seed = synth.config_seed(2, 0)
    flush(f"1024^3 uniform seed={seed}: host generation")
    X = synth.x_range(seed, 0, 1 << 30).reshape(dims)
    U = [synth.normal_factor(synth.config_seed(2, 1 + m), 1024, R) for m in range(3)]
    refs = {}
    for n in range(3):
        flush(f"1024^3 uniform: oracle mode {n}")
        refs[n] = oracle_mod.mttkrp(X, [None if m == n else U[m] for m in range(3)], n)
    flush("1024^3 uniform: upload")
    Xd = torch.from_numpy(X).cuda()
    del X
    copies = reduced_copies(dn, Xd, FORMS5)
    tol = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-5, "fx20": 1e-5, "bf16": 1e-2}
    for prec in FORMS5:
        udt = torch.float64 if prec == "fp64" else torch.float32
        for n in range(3):
            flush(f"1024^3 uniform {prec} mode {n}: deinsum_mttkrp")
            ops = [to_dev(U[m], udt) for m in range(3) if m != n]
            M = dn.mttkrp(SPEC3[n], copies[prec], ops, precision=prec, out_dtype=torch.float64)
            torch.cuda.synchronize()
            got = M.cpu().numpy()
            whole = nrel(got, refs[n])
            rows = per_row_rel(got, refs[n])
            flush(f"  normwise {whole:.3e}, worst row {rows.max():.3e} (row {int(rows.argmax())})")
            assert whole <= tol[prec], (prec, n, whole)
            assert rows.max() <= tol[prec], (prec, n, int(rows.argmax()), rows.max())
    del copies, Xd
    torch.cuda.empty_cache()


ROWS80 = {0: (0, 53, 79), 2: (1, 40, 79)}


def _order5_refs(oracle_mod, synth, seed, dims, U, dist):
    refs = {}
    for n, rows in ROWS80.items():
        flush(f"80^5 {dist}: oracle mode {n} rows {rows}")
        slab = synth.x_rows(seed, dims, n, rows, dist)
        refs[n] = oracle_mod.mttkrp(slab, [None if m == n else U[m] for m in range(5)], n)
    return refs


def test_order5_80_integer_exact_every_form(dn, synth, oracle_mod):
    """80^5, R = 24, modes 0 and 2, X and factors in {-1, 0, 1}: sums of at most 80^4
    integer terms are exact in FP64, and every reduced form keeps its matrix-core sums
    below 2^24, so all five forms must match the oracle exactly on the sampled rows."""
    dims, R = (80,) * 5, 24
    seed = synth.config_seed(3, 50)
    U = [synth.int_factor(seed + 1 + m, 80, R, -1, 1) for m in range(5)]
    refs = _order5_refs(oracle_mod, synth, seed, dims, U, "int3")
    flush(f"80^5 int3 seed={seed}: device generation")
    Xd = torch.empty(dims, dtype=torch.float64, device="cuda")
    dn.synth_fill(Xd, seed, dist="int3")
    copies = reduced_copies(dn, Xd, FORMS5)
    for prec in FORMS5:
        udt = torch.float64 if prec == "fp64" else torch.float32
        for n, rows in ROWS80.items():
            flush(f"80^5 int3 {prec} mode {n}: deinsum_mttkrp")
            ops = [to_dev(U[m], udt) for m in range(5) if m != n]
            rep = dn.Report()
            M = dn.mttkrp(mttkrp_spec(5, n), copies[prec], ops, precision=prec, out_dtype=torch.float64,
                          report=rep)
            torch.cuda.synchronize()
            got = M.cpu().numpy()[list(rows)]
            flush(f"  plan {rep.plan_name.decode()}")
            assert np.array_equal(got, refs[n]), (prec, n)
    del copies, Xd
    torch.cuda.empty_cache()


def test_order5_80_uniform_against_oracle(dn, synth, oracle_mod):
    """The order-5 benchmark inputs (config-3 seeds, X uniform, N(0,1) factors), modes 0
    and 2: FP64 within 1e-12 of the oracle per sampled row; FP32, BF16x3 and FX20 within
    1e-5 of the oracle (not of the GPU's FP64 result)."""
    dims, R = (80,) * 5, 24
    seed = synth.config_seed(3, 0)
    U = [synth.normal_factor(synth.config_seed(3, 1 + m), 80, R) for m in range(5)]
    refs = _order5_refs(oracle_mod, synth, seed, dims, U, "uniform")
    flush(f"80^5 uniform seed={seed}: device generation")
    Xd = torch.empty(dims, dtype=torch.float64, device="cuda")
    dn.synth_fill(Xd, seed)
    forms = ("fp64", "fp32", "bf16x3", "fx20")
    copies = reduced_copies(dn, Xd, forms)
    tol = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-5, "fx20": 1e-5}
    for prec in forms:
        udt = torch.float64 if prec == "fp64" else torch.float32
        for n, rows in ROWS80.items():
            flush(f"80^5 uniform {prec} mode {n}: deinsum_mttkrp")
            ops = [to_dev(U[m], udt) for m in range(5) if m != n]
            M = dn.mttkrp(mttkrp_spec(5, n), copies[prec], ops, precision=prec, out_dtype=torch.float64)
            torch.cuda.synchronize()
            got = M.cpu().numpy()[list(rows)]
            err = per_row_rel(got, refs[n])
            flush(f"  per-row error {np.array2string(err, precision=3)}")
            assert err.max() <= tol[prec], (prec, n, err.tolist())
    del copies, Xd
    torch.cuda.empty_cache()
