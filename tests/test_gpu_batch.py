"""GPU tests of the persistent batched MTTKRP launch (deinsum_batch_*)."""
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


def make_jobs(seed, count):
    """Uneven CP-ALS-style jobs: order 3 (and a few order 4), dims 32..300, R in {8,16,32,64}."""
    rng = np.random.default_rng(seed)
    jobs = []
    for t in range(count):
        N = 3 if t % 5 else 4
        dims = tuple(int(d) for d in rng.integers(32, 300 if N == 3 else 60, N))
        R = int(rng.choice([8, 16, 32, 64]))
        n = int(rng.integers(0, N))
        prec = "fp32" if rng.random() < 0.7 else "fp64"
        X = rng.uniform(-1, 1, dims)
        U = [rng.standard_normal((d, R)) for d in dims]
        jobs.append((dims, R, n, prec, X, U))
    return jobs


def add_job(batch, job):
    dims, R, n, prec, X, U = job
    dt = torch.float64 if prec == "fp64" else torch.float32
    Xd = to_dev(X, dt)
    Ud = [to_dev(U[m], dt) for m in range(len(dims)) if m != n]
    return batch.add(mttkrp_spec(len(dims), n), Xd, Ud, precision=prec, out_dtype=torch.float64)


def test_batch_matches_oracle(dn, oracle_mod):
    jobs = make_jobs(1, 12)
    b = dn.Batch(8)
    outs = [add_job(b, j)[1] for j in jobs]
    b.launch()
    torch.cuda.synchronize()
    for (dims, R, n, prec, X, U), M in zip(jobs, outs):
        Un = [None if m == n else U[m] for m in range(len(dims))]
        ref = oracle_mod.mttkrp(X, Un, n)
        tol = 1e-12 if prec == "fp64" else 1e-5
        err = nrel(M.cpu().numpy(), ref)
        flush(f"batch job dims={dims} R={R} n={n} {prec}: {err:.2e}")
        assert err <= tol
    assert b.info()["graph_captures"] == 1
    b.close()


def test_batch_alone_vs_mix_bitwise(dn):
    jobs = make_jobs(2, 9)
    mix = dn.Batch()
    mix_out = [add_job(mix, j)[1] for j in jobs]
    mix.launch()
    torch.cuda.synchronize()
    alone = dn.Batch()
    for j, ref in zip(jobs, mix_out):
        alone.reset()
        _, M = add_job(alone, j)
        alone.launch()
        torch.cuda.synchronize()
        assert torch.equal(M, ref)
    assert alone.info()["graph_captures"] == 1  # one capture, replayed for every job
    mix.close()
    alone.close()


def test_batch_graph_replays_are_identical(dn):
    jobs = make_jobs(3, 6)
    b = dn.Batch()
    outs = [add_job(b, j)[1] for j in jobs]
    b.launch()
    torch.cuda.synchronize()
    first = [o.clone() for o in outs]
    for rep in range(4):
        for o in outs:
            o.fill_(-1.0)  # eager work between replays
        torch.cuda.synchronize()
        b.launch()
        torch.cuda.synchronize()
        for o, f in zip(outs, first):
            assert torch.equal(o, f), rep
    info = b.info()
    assert info["graph_captures"] == 1 and info["launches"] == 5
    b.close()


def test_batch_rejects_unsupported(dn):
    b = dn.Batch()
    X = torch.zeros((8, 8, 8), dtype=torch.float32, device="cuda")
    U = [torch.zeros((8, 4), dtype=torch.float32, device="cuda")] * 2
    with pytest.raises(dn.DeinsumError):
        b.add("ijk,ja,ka->ia", X, U, precision="bf16x3")
    b.close()


def test_batch_add_validates_like_mttkrp(dn):
    """deinsum_batch_add_mttkrp rejects what deinsum_mttkrp rejects, before planning: a
    hand-built spec whose free mode or factor modes are out of range or inconsistent,
    misaligned pointers, and an output overlapping X or a factor.  Nothing is queued."""
    import ctypes
    lib = dn._lib.load()
    b = dn.Batch()
    X = torch.zeros((8, 8, 8), dtype=torch.float64, device="cuda")
    U = [torch.zeros((8, 4), dtype=torch.float64, device="cuda") for _ in range(2)]
    M = torch.zeros((8, 4), dtype=torch.float64, device="cuda")
    dims = (ctypes.c_int64 * 3)(8, 8, 8)
    o = dn._opts("fp64", torch.float64, None, 0, 0, None)

    def add(sp, Xp=X.data_ptr(), Up=None, Mp=M.data_ptr()):
        Up = Up or [u.data_ptr() for u in U]
        ptrs = (ctypes.c_void_p * 2)(*Up)
        return lib.deinsum_batch_add_mttkrp(b._h, ctypes.byref(sp), dims, 4, ctypes.c_void_p(Xp), ptrs,
                                            ctypes.c_void_p(Mp), ctypes.byref(o), None)

    good = dn.parse("ijk,ja,ka->ia")
    bad = []
    s = dn.parse("ijk,ja,ka->ia"); s.free_mode = 3; bad.append(s)
    s = dn.parse("ijk,ja,ka->ia"); s.factor_mode[1] = 1; bad.append(s)           # mode 1 twice
    s = dn.parse("ijk,ja,ka->ia"); s.factor_mode[0] = 0; bad.append(s)           # the free mode
    s = dn.parse("ijk,ja,ka->ia"); s.factor_mode[1] = 7; bad.append(s)           # out of range
    s = dn.parse("ijk,ja,ka->ia"); s.n_factors = 3; bad.append(s)
    for sp in bad:
        assert add(sp) == -1, dn.last_error()
    assert add(good, Mp=X.data_ptr()) == -1                      # output is X
    assert add(good, Mp=U[1].data_ptr()) == -1                   # output is a factor
    assert add(good, Xp=X.data_ptr() + 4) == -1                  # misaligned X
    assert add(good, Mp=M.data_ptr() + 4) == -1                  # misaligned M
    assert add(good, Up=[U[0].data_ptr(), U[1].data_ptr() + 2]) == -1
    assert b.info()["jobs"] == 0
    assert add(good) == 0                                        # the well-formed call is accepted
    assert b.info()["jobs"] == 1
    b.close()
