"""deinsum_mttkrp_noalloc (workspace in the library's fixed per-device scratch array)
against deinsum_mttkrp (library pool), both called through the raw C ABI.

Two calls in a row on the same stream, the second on a smaller problem, so the second
runs over the first one's leftovers in the shared array: outputs must be bitwise equal to
deinsum_mttkrp's (same plan, same kernels, fixed reduction order) and within 1e-12 of
the oracle.  A problem whose plan needs more workspace than the array holds is rejected
before anything is enqueued.
"""
import ctypes

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


def raw_call(dn, entry, spec, X, ops, M, prec):
    """One call of `entry` through the C ABI: parsed spec, host dims, device pointers."""
    lib = dn._lib.load()
    sp = dn._lib.Spec()
    assert lib.deinsum_parse(spec.encode(), ctypes.byref(sp)) == 0
    o = dn._lib.Opts()
    lib.deinsum_opts_init(ctypes.byref(o))
    o.precision = dn.PRECISIONS[prec]
    o.out_dtype = dn._DT_CODE[M.dtype]
    dims = (ctypes.c_int64 * X.dim())(*X.shape)
    ptrs = (ctypes.c_void_p * len(ops))(*[u.data_ptr() for u in ops])
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return getattr(lib, entry)(ctypes.byref(sp), dims, ctypes.c_int64(ops[0].shape[1]), ctypes.c_void_p(X.data_ptr()),
                               ptrs, ctypes.c_void_p(M.data_ptr()), ctypes.byref(o), stream)


CASES = [
    # (dims, R, mode, precision): the first of each pair is the larger problem
    (((96, 200, 520), 40, 1, "fp64"), ((33, 47, 70), 16, 1, "fp64")),
    (((128, 96, 1000), 24, 2, "fp64"), ((40, 30, 65), 8, 2, "fp64")),
    (((64, 48, 40, 96), 24, 0, "fp32"), ((9, 10, 11, 17), 5, 0, "fp32")),
]


@pytest.mark.parametrize("pair", CASES, ids=lambda p: f"{len(p[0][0])}d-mode{p[0][2]}-{p[0][3]}")
def test_noalloc_matches_mttkrp_two_calls(dn, synth, oracle_mod, pair):
    rng = np.random.default_rng(2206083777)
    for step, (dims, R, n, prec) in enumerate(pair):
        N = len(dims)
        spec = mttkrp_spec(N, n)
        X = synth.x_tensor(2206083700 + step, dims)
        U = [None if m == n else rng.standard_normal((d, R)) for m, d in enumerate(dims)]
        xdt = torch.float64 if prec == "fp64" else torch.float32
        Xd = to_dev(X, xdt)
        ops = [to_dev(U[m], xdt) for m in range(N) if m != n]
        need = dn.workspace_size(spec, dims, [R], precision=prec)
        assert 0 < need <= dn.NOALLOC_SCRATCH_BYTES
        M_pool = torch.full((dims[n], R), np.nan, dtype=torch.float64, device="cuda")
        M_none = torch.full((dims[n], R), np.nan, dtype=torch.float64, device="cuda")
        flush(f"noalloc step {step}: dims={dims} R={R} mode={n} {prec} workspace={need}")
        assert raw_call(dn, "deinsum_mttkrp_noalloc", spec, Xd, ops, M_none, prec) == 0, dn.last_error()
        assert raw_call(dn, "deinsum_mttkrp", spec, Xd, ops, M_pool, prec) == 0, dn.last_error()
        torch.cuda.synchronize()
        a, b = M_none.cpu().numpy(), M_pool.cpu().numpy()
        assert np.array_equal(a, b), f"step {step}: max diff {np.nanmax(np.abs(a - b))}"
        Xr = X if prec == "fp64" else X.astype(np.float32).astype(np.float64)
        Ur = [None if u is None else (u if prec == "fp64" else u.astype(np.float32).astype(np.float64)) for u in U]
        ref = oracle_mod.mttkrp(Xr, Ur, n)
        assert nrel(a, ref) <= (1e-12 if prec == "fp64" else 1e-6)


def test_noalloc_rejects_workspace_beyond_scratch(dn):
    """80^5 FP64, R = 24, mode 0 needs more than the fixed array: NO_MEMORY, nothing run
    (X and the factors are never touched, so small stand-in buffers suffice)."""
    dims, R = (80,) * 5, 24
    spec = mttkrp_spec(5, 0)
    need = dn.workspace_size(spec, dims, [R])
    assert need > dn.NOALLOC_SCRATCH_BYTES
    lib = dn._lib.load()
    sp = dn._lib.Spec()
    assert lib.deinsum_parse(spec.encode(), ctypes.byref(sp)) == 0
    stand_in = torch.zeros(1 << 10, dtype=torch.float64, device="cuda")
    M = torch.full((80, R), 7.0, dtype=torch.float64, device="cuda")
    ptrs = (ctypes.c_void_p * 4)(*([stand_in.data_ptr()] * 4))
    d = (ctypes.c_int64 * 5)(*dims)
    st = lib.deinsum_mttkrp_noalloc(ctypes.byref(sp), d, R, ctypes.c_void_p(stand_in.data_ptr()), ptrs,
                                    ctypes.c_void_p(M.data_ptr()), None, None)
    assert st == -5 and "scratch" in dn.last_error()
    torch.cuda.synchronize()
    assert bool((M == 7.0).all())


def test_noalloc_rejects_caller_workspace(dn):
    lib = dn._lib.load()
    sp = dn._lib.Spec()
    assert lib.deinsum_parse(b"ijk,ja,ka->ia", ctypes.byref(sp)) == 0
    o = dn._lib.Opts()
    lib.deinsum_opts_init(ctypes.byref(o))
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    o.workspace = ws.data_ptr()
    o.workspace_bytes = ws.numel()
    X = torch.zeros((4, 4, 4), dtype=torch.float64, device="cuda")
    U = torch.zeros((4, 2), dtype=torch.float64, device="cuda")
    M = torch.zeros((4, 2), dtype=torch.float64, device="cuda")
    ptrs = (ctypes.c_void_p * 2)(U.data_ptr(), U.data_ptr())
    d = (ctypes.c_int64 * 3)(4, 4, 4)
    st = lib.deinsum_mttkrp_noalloc(ctypes.byref(sp), d, 2, ctypes.c_void_p(X.data_ptr()), ptrs,
                                    ctypes.c_void_p(M.data_ptr()), ctypes.byref(o), None)
    assert st == -1
