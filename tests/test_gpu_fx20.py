"""GPU tests of the FX20 form (20-bit fixed point in an FP16 and an int8 plane): the encoder against a plain numpy encoding of the
format, and MTTKRP on FX20 storage against the FP64 oracle."""
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


def encode_np(x):
    """The FX20 format written out in numpy: e, m, h (FP16 plane), l (int8 plane)."""
    x = np.asarray(x, dtype=np.float64).ravel()
    mx = float(np.max(np.abs(x))) if x.size else 0.0
    e = (np.frexp(mx)[1] - 19) if mx > 0 else 0
    m = np.clip(np.rint(np.ldexp(x, -e)), -(2 ** 19), 2 ** 19).astype(np.int64)
    h = np.floor_divide(m + 128, 256)
    l = m - 256 * h
    assert np.all(np.abs(h) <= 2048) and np.all((l >= -128) & (l <= 127))
    hi = h.astype(np.float16).view(np.uint16)
    lo = l.astype(np.int8).view(np.uint8)
    return e, mx, m, hi, lo


def planes(dn, f):
    n = f.numel()
    raw = f.buf.cpu().numpy()
    hi = raw[256:256 + 2 * n].view(np.uint16)
    lo_off = 256 + (2 * n + 255) // 256 * 256
    lo = raw[lo_off:lo_off + n]
    return hi, lo


@pytest.mark.parametrize("shape,scale", [((7, 5, 9), 1.0), ((64, 33, 17), 1e-3), ((1,), 3.0), ((300,), 1e6)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_encoder_matches_format(dn, shape, scale, dtype):
    rng = np.random.default_rng(len(shape) + int(scale))
    x = rng.uniform(-scale, scale, shape)
    if dtype == torch.float32:
        x = x.astype(np.float32).astype(np.float64)
    f = dn.to_fx20(to_dev(x, dtype))
    torch.cuda.synchronize()
    e, mx, m, hi, lo = encode_np(x)
    h = f.header()
    assert h["magic"] == 0x30325846 and h["exp2"] == e and h["count"] == x.size and h["max_abs"] == mx
    ghi, glo = planes(dn, f)
    assert np.array_equal(ghi, hi) and np.array_equal(glo, lo)
    # decoding the planes gives back m = 256 h + l, and |x - m 2^e| <= 2^(e-1)
    dec = 256 * ghi.view(np.float16).astype(np.int64) + glo.view(np.int8).astype(np.int64)
    assert np.array_equal(dec, m)
    assert np.max(np.abs(x.ravel() - np.ldexp(dec.astype(np.float64), e))) <= 2.0 ** (e - 1)


def test_encoder_zero_tensor(dn):
    f = dn.to_fx20(torch.zeros((4, 4, 4), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    h = f.header()
    assert h["exp2"] == 0 and h["max_abs"] == 0.0
    ghi, glo = planes(dn, f)
    assert not ghi.any() and not glo.any()


SHAPES = [((64, 64, 64), 24), ((37, 45, 96), 20), ((16, 21, 130), 40), ((6, 5, 7, 48), 16), ((40, 33, 80), 64)]


@pytest.mark.parametrize("dims,R", SHAPES)
def test_fx20_integer_exact(dn, oracle_mod, synth, dims, R):
    """Integer X in [-2, 2] and integer factors: encoding and arithmetic are exact."""
    rng = np.random.default_rng(sum(dims))
    X = rng.integers(-2, 3, dims).astype(np.float64)
    U = [rng.integers(-2, 3, (d, R)).astype(np.float64) for d in dims]
    f = dn.to_fx20(to_dev(X))
    for n in range(len(dims)):
        flush(f"fx20 exact dims={dims} R={R} n={n}")
        ops = [to_dev(U[m], torch.float32) for m in range(len(dims)) if m != n]
        M = dn.mttkrp(mttkrp_spec(len(dims), n), f, ops, precision="fx20", out_dtype=torch.float64)
        torch.cuda.synchronize()
        ref = oracle_mod.mttkrp(X, [None if m == n else U[m] for m in range(len(dims))], n)
        assert np.array_equal(M.cpu().numpy(), ref), (dims, n)


@pytest.mark.parametrize("dims,R", SHAPES)
def test_fx20_uniform_error(dn, oracle_mod, dims, R):
    rng = np.random.default_rng(7 + sum(dims))
    X = rng.uniform(-1, 1, dims)
    U = [rng.standard_normal((d, R)).astype(np.float32).astype(np.float64) for d in dims]
    f = dn.to_fx20(to_dev(X))
    for n in range(len(dims)):
        ops = [to_dev(U[m], torch.float32) for m in range(len(dims)) if m != n]
        M = dn.mttkrp(mttkrp_spec(len(dims), n), f, ops, precision="fx20", out_dtype=torch.float64)
        torch.cuda.synchronize()
        ref = oracle_mod.mttkrp(X, [None if m == n else U[m] for m in range(len(dims))], n)
        err = nrel(M.cpu().numpy(), ref)
        flush(f"fx20 uniform dims={dims} R={R} n={n}: {err:.2e}")
        assert err <= 4e-6  # X carries 20 bits: about 1e-6 for uniform data


def test_fx20_header_mismatch_gives_nan(dn):
    """A buffer encoded for more elements than the call's dims is rejected in the output."""
    X = torch.rand((8, 8, 9), dtype=torch.float64, device="cuda")
    f = dn.to_fx20(X)
    small = dn.FX20(f.buf, (8, 8, 8))  # fewer elements than encoded: reads stay inside the buffer
    U = [torch.rand((8, 4), dtype=torch.float32, device="cuda") for _ in range(2)]
    M = dn.mttkrp(mttkrp_spec(3, 0), small, U, precision="fx20", out_dtype=torch.float64)
    torch.cuda.synchronize()
    assert torch.isnan(M).all()


def test_fx20_tuned_plan(dn, oracle_mod):
    rng = np.random.default_rng(99)
    dims, R = (96, 80, 128), 24
    X = rng.uniform(-1, 1, dims)
    U = [rng.standard_normal((d, R)).astype(np.float32).astype(np.float64) for d in dims]
    f = dn.to_fx20(to_dev(X))
    for n in (0, 2):
        ops = [to_dev(U[m], torch.float32) for m in range(3) if m != n]
        dn.tune_clear()
        rep = dn.tune_mttkrp(mttkrp_spec(3, n), f, ops, precision="fx20", out_dtype=torch.float64, reps=2)
        assert rep.tuned_us > 0
        M = dn.mttkrp(mttkrp_spec(3, n), f, ops, precision="fx20", out_dtype=torch.float64)
        torch.cuda.synchronize()
        ref = oracle_mod.mttkrp(X, [None if m == n else U[m] for m in range(3)], n)
        assert nrel(M.cpu().numpy(), ref) <= 4e-6
    dn.tune_clear()


# Every compiled FX20 last-mode (M-contiguous) kernel variant: column tiles, K
# instructions per step, output indices per lane, non-temporal loads.
FX20_MCONTIG = [(2, 1, 4, 0), (2, 1, 4, 1), (2, 1, 2, 0), (2, 1, 2, 1), (2, 2, 2, 0), (1, 1, 4, 0),
                (1, 2, 2, 0), (1, 2, 2, 1), (4, 1, 1, 0)]


@pytest.mark.parametrize("dims", [(7, 9, 60), (5, 6, 7, 50), (3, 5, 130)])
def test_fx20_last_mode_every_variant(dn, oracle_mod, tmp_path, dims):
    """Ragged last modes on every FX20 last-mode variant, each forced by a plan-cache
    entry.  In a ragged tile the lanes whose indices all exist take vector loads when the
    rows are whole runs of the lane's width (60 for every width, 50 and 130 for 2-index
    runs), element loads otherwise; integer inputs, exact against the oracle."""
    rng = np.random.default_rng(sum(dims))
    N, R = len(dims), 24
    X = rng.integers(-2, 3, dims).astype(np.float64)
    U = [rng.integers(-2, 3, (d, R)).astype(np.float64) for d in dims]
    ref = oracle_mod.mttkrp(X, U[:-1] + [None], N - 1)
    f = dn.to_fx20(to_dev(X))
    ops = [to_dev(U[m], torch.float32) for m in range(N - 1)]
    key = f"s:N{N}:n{N - 1}:p4:R{R}:" + "x".join(str(d) for d in dims)
    cache = tmp_path / "fx20_mcontig.txt"
    try:
        for nt, ni, mt, xnt in FX20_MCONTIG:
            cache.write_text(f"{key} {nt} {ni} {mt} {xnt} 0 0 0 1.0\n")
            dn.tune_clear()
            dn.tune_load(cache)
            rep = dn.Report()
            M = dn.mttkrp(mttkrp_spec(N, N - 1), f, ops, precision="fx20", out_dtype=torch.float64, report=rep)
            torch.cuda.synchronize()
            name = rep.plan_name.decode()
            flush(f"fx20 last mode dims={dims}: {name}")
            assert f"mcontig<p4,nt{nt},ni{ni},mt{mt}{',nt' if xnt else ''}>" in name, name
            assert np.array_equal(M.cpu().numpy(), ref), name
    finally:
        dn.tune_clear()
