"""GPU tests of the CP-ALS request server (deinsum_server_*): results against the
oracle's ALS update, per-tensor ordering, and that a tensor's results are the
same alone and in any mix of concurrent requests."""
import numpy as np
import pytest
import torch

from gpu_common import flush, nrel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dn():
    import paper_2206_08301_amd as m
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    m._lib.load()
    return m


def host_tensor(seed, dims, R, prec):
    """Seeded X ~ U[-1,1] and N(0,1) factors, rounded to the storage precision."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, dims)
    U = [rng.standard_normal((d, R)) for d in dims]
    if prec == "fp32":
        X = X.astype(np.float32).astype(np.float64)
        U = [u.astype(np.float32).astype(np.float64) for u in U]
    return X, U


def device_copy(X, U, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    return (torch.from_numpy(X).to(dt).cuda().contiguous(),
            [torch.from_numpy(u).to(dt).cuda().contiguous() for u in U])


def oracle_sweeps(oracle_mod, X, U, modes):
    U = [u.copy() for u in U]
    for n in modes:
        U[n] = oracle_mod.als_update(X, [None if m == n else U[m] for m in range(X.ndim)], n)
    return U


def run_server(dn, tensors, requests, batched=True, arrivals=None, max_jobs=64, direct_max_jobs=4):
    """tensors: list of (X, U, prec) host arrays; requests: list of (tensor, mode).
    Returns the device factors after serving, the server's results and stats."""
    srv = dn.Server(batched=batched, max_jobs_per_epoch=max_jobs, max_requests=len(requests) + 8,
                    direct_max_jobs=direct_max_jobs)
    dev = []
    for X, U, prec in tensors:
        Xd, Ud = device_copy(X, U, prec)
        srv.add_tensor(Xd, Ud, precision=prec)
        dev.append(Ud)
    srv.start()
    if arrivals is None:
        for t, n in requests:
            srv.submit(t, n)
    else:
        srv.replay(arrivals, [t for t, _ in requests], [n for _, n in requests])
    srv.drain()
    arr, done, ep = srv.results()
    stats = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    return [[u.double().cpu().numpy() for u in Ud] for Ud in dev], (arr, done, ep), stats


def round_robin(order_of, sweeps):
    """Requests assigned round-robin over tensors, each tensor cycling through its modes."""
    reqs = []
    for s in range(sweeps):
        for n in range(max(order_of)):
            for t, N in enumerate(order_of):
                if n < N:
                    reqs.append((t, n))
    return reqs


SPECS_FP64 = [((40, 33, 50), 8), ((64, 48, 36), 16), ((90, 100, 120), 64), ((20, 18, 16, 22), 6)]


@pytest.mark.parametrize("batched", [True, False])
def test_server_matches_oracle_fp64(dn, oracle_mod, batched):
    tensors = []
    for k, (dims, R) in enumerate(SPECS_FP64):
        X, U = host_tensor(500 + k, dims, R, "fp64")
        tensors.append((X, U, "fp64"))
    reqs = round_robin([len(d) for d, _ in SPECS_FP64], 2)
    flush(f"server fp64 batched={batched}: {len(reqs)} requests")
    got, (arr, done, ep), stats = run_server(dn, tensors, reqs, batched=batched)
    assert stats["completed"] == len(reqs)
    for k, (X, U, _) in enumerate(tensors):
        modes = [n for t, n in reqs if t == k]
        ref = oracle_sweeps(oracle_mod, X, U, modes)
        for m in range(X.ndim):
            err = nrel(got[k][m], ref[m])
            flush(f"  tensor {k} dims={X.shape} mode {m}: {err:.2e}")
            assert err <= 1e-10


def test_server_matches_oracle_fp32(dn, oracle_mod):
    specs = [((48, 40, 56), 8), ((64, 60, 50), 32)]
    tensors = [(*host_tensor(600 + k, d, R, "fp32"), "fp32") for k, (d, R) in enumerate(specs)]
    reqs = round_robin([3, 3], 1)
    got, _, stats = run_server(dn, tensors, reqs)
    assert stats["completed"] == len(reqs)
    for k, (X, U, _) in enumerate(tensors):
        ref = oracle_sweeps(oracle_mod, X, U, [0, 1, 2])
        for m in range(3):
            err = nrel(got[k][m], ref[m])
            flush(f"  fp32 tensor {k} mode {m}: {err:.2e}")
            assert err <= 2e-4


def c5_like(seed, count):
    """Uneven tensors as in the serving workload, scaled down: R in {8,16,32,64}, each dim
    between R+16 and R+80 (so the normal equations stay well conditioned), 70% FP32."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        R = int(rng.choice([8, 16, 32, 64]))
        dims = tuple(int(d) for d in rng.integers(max(32, R + 16), R + 81, 3))
        prec = "fp32" if rng.random() < 0.7 else "fp64"
        X, U = host_tensor(seed * 100 + k, dims, R, prec)
        out.append((X, U, prec))
    return out


def test_server_alone_vs_mix_bitwise(dn):
    """With direct launches off (direct_max_jobs 0), each tensor's factors after its requests are bitwise the
    same served alone, in the full mix submitted at once, and in the mix arriving over
    time (different epochs)."""
    tensors = c5_like(7, 10)
    reqs = round_robin([3] * len(tensors), 2)
    mix, (_, _, ep_mix), st_mix = run_server(dn, tensors, reqs, direct_max_jobs=0)
    arrivals = np.arange(len(reqs)) * 2e-4
    spread, (_, _, ep_sp), st_sp = run_server(dn, tensors, reqs, arrivals=arrivals, direct_max_jobs=0)
    flush(f"mix epochs={st_mix['epochs']} max_batch={st_mix['max_batch']}; "
          f"spread epochs={st_sp['epochs']} max_batch={st_sp['max_batch']}")
    assert st_mix["max_batch"] > 1
    for k in (0, 3, 9):
        alone, _, _ = run_server(dn, [tensors[k]], [(0, n) for t, n in reqs if t == k], direct_max_jobs=0)
        for m in range(3):
            assert np.array_equal(alone[0][m], mix[k][m]), (k, m)
    for k in range(len(tensors)):
        for m in range(3):
            assert np.array_equal(spread[k][m], mix[k][m]), (k, m)


def test_server_alone_vs_mix_direct(dn, oracle_mod):
    """With direct launches for small epochs (the default), a tensor served alone runs every request with
    the per-request launches; its factors match the mix (batched epochs) within the
    form's tolerance, and both match the oracle's sweeps."""
    tensors = c5_like(7, 10)
    reqs = round_robin([3] * len(tensors), 2)
    mix, _, st_mix = run_server(dn, tensors, reqs)
    assert st_mix["max_batch"] > 1
    for k in (0, 3, 9):
        alone, (_, _, ep), st = run_server(dn, [tensors[k]], [(0, n) for t, n in reqs if t == k])
        assert st["max_batch"] == 1
        X, U, prec = tensors[k]
        ref = oracle_sweeps(oracle_mod, X, U, [n for t, n in reqs if t == k])
        tol = 1e-10 if prec == "fp64" else 5e-4
        for m in range(3):
            flush(f"  tensor {k} ({prec}) mode {m}: alone vs mix {nrel(alone[0][m], mix[k][m]):.2e}, "
                  f"alone vs oracle {nrel(alone[0][m], ref[m]):.2e}")
            assert nrel(alone[0][m], mix[k][m]) <= tol, (k, m)
            assert nrel(alone[0][m], ref[m]) <= tol, (k, m)


def test_server_batched_matches_per_request(dn):
    tensors = c5_like(8, 6)
    reqs = round_robin([3] * len(tensors), 1)
    a, _, _ = run_server(dn, tensors, reqs, batched=True)
    b, _, _ = run_server(dn, tensors, reqs, batched=False)
    for k, (_, _, prec) in enumerate(tensors):
        tol = 1e-10 if prec == "fp64" else 1e-4
        for m in range(3):
            assert nrel(a[k][m], b[k][m]) <= tol, (k, m, prec)


@pytest.mark.parametrize("batched", [True, False])
def test_server_fifo_per_tensor(dn, batched):
    tensors = c5_like(9, 5)
    reqs = round_robin([3] * len(tensors), 2)
    arrivals = np.arange(len(reqs)) * 1e-4
    _, (arr, done, ep), stats = run_server(dn, tensors, reqs, batched=batched, arrivals=arrivals)
    assert stats["completed"] == len(reqs)
    assert np.all(done >= arr)
    for k in range(len(tensors)):
        idx = [i for i, (t, _) in enumerate(reqs) if t == k]
        assert np.all(np.diff(ep[idx]) > 0), k
        assert np.all(np.diff(done[idx]) >= 0), k


def test_server_rejects_bad_input(dn):
    srv = dn.Server()
    X = torch.zeros((8, 8, 8), dtype=torch.float64, device="cuda")
    U = [torch.zeros((8, 65), dtype=torch.float64, device="cuda") for _ in range(3)]
    with pytest.raises(dn.DeinsumError):
        srv.add_tensor(X, U)
    U = [torch.ones((8, 4), dtype=torch.float64, device="cuda") for _ in range(3)]
    t = srv.add_tensor(X, U)
    srv.start()
    with pytest.raises(dn.DeinsumError):
        srv.submit(t, 3)
    with pytest.raises(dn.DeinsumError):
        srv.submit(t + 1, 0)
    srv.drain()
    srv.close()


@pytest.mark.parametrize("batched", [True, False])
def test_request_over_budget_fails_alone(dn, oracle_mod, batched):
    """A request whose MTTKRP workspace alone exceeds the HBM budget ends with
    NO_MEMORY; the other tensor's requests, interleaved with it, are served and match
    the oracle, and the server keeps accepting work."""
    small = host_tensor(710, (24, 20, 28), 8, "fp64")
    big = host_tensor(711, (200, 220, 240), 64, "fp64")
    ws_small = max(dn.workspace_size(s, small[0].shape, [8]) for s in ("ijk,ja,ka->ia", "ijk,ia,ka->ja", "ijk,ia,ja->ka"))
    ws_big = dn.workspace_size("ijk,ja,ka->ia", big[0].shape, [64])
    budget = (ws_small + ws_big) // 2
    assert ws_small <= budget < ws_big
    srv = dn.Server(batched=batched, max_requests=64, hbm_budget_bytes=budget)
    devs = []
    for X, U in (small, big):
        Xd, Ud = device_copy(X, U, "fp64")
        srv.add_tensor(Xd, Ud, precision="fp64")
        devs.append(Ud)
    srv.start()
    ids = []
    for n in range(3):
        ids.append((0, n, srv.submit(0, n)))
        ids.append((1, 0, srv.submit(1, 0)))  # mode 0 of the big tensor needs more than the budget
    st = srv.drain(check=False)
    assert st == -5, dn.last_error()
    for t, n, rid in ids:
        p = srv.poll(rid)
        if t == 0:
            assert p["status"] == "done" and p["done"] >= 0, p
        else:
            assert p["status"] == "NO_MEMORY" and p["code"] == -5, p
    assert srv.stats()["completed"] == 3
    rid = srv.submit(0, 0)  # the server still serves
    srv.drain(check=False)
    assert srv.poll(rid)["status"] == "done"
    srv.close()
    torch.cuda.synchronize()
    ref = oracle_sweeps(oracle_mod, small[0], small[1], [0, 1, 2, 0])
    for m in range(3):
        assert nrel(devs[0][m].cpu().numpy(), ref[m]) <= 1e-10


def test_regularised_update_is_flagged(dn):
    """R = 32 with two modes of extent 3: V = G^0 * G^1 (Hadamard) for the mode-2 update
    has rank at most 9 < 32, so the Gauss-Jordan pivots fall below the floor and the
    request is flagged; a well-conditioned tensor's requests are not."""
    sing = host_tensor(720, (3, 3, 90), 32, "fp64")
    good = host_tensor(721, (60, 50, 70), 8, "fp64")
    srv = dn.Server(batched=True, max_requests=16)
    for X, U in (sing, good):
        Xd, Ud = device_copy(X, U, "fp64")
        srv.add_tensor(Xd, Ud, precision="fp64")
    srv.start()
    r_sing = srv.submit(0, 2)
    r_good = [srv.submit(1, n) for n in range(3)]
    srv.drain()
    assert srv.poll(r_sing)["flags"] == {"regularised"}
    for r in r_good:
        p = srv.poll(r)
        assert p["status"] == "done" and p["flags"] == set(), p
    srv.close()


def test_poll_states_and_errors(dn):
    X, U = host_tensor(730, (30, 20, 25), 8, "fp64")
    srv = dn.Server(batched=True, max_requests=8)
    Xd, Ud = device_copy(X, U, "fp64")
    srv.add_tensor(Xd, Ud, precision="fp64")
    srv.start()
    rid = srv.submit(0, 1)
    assert srv.poll(rid)["status"] in ("pending", "running", "done")
    srv.drain()
    p = srv.poll(rid)
    assert p["status"] == "done" and p["code"] == 0 and p["done"] > 0
    with pytest.raises(dn.DeinsumError):
        srv.poll(rid + 100)
    srv.close()


def test_server_small_epochs_direct(dn, oracle_mod):
    """direct_max_jobs = 4: epochs of up to four requests run the per-request launches
    one after the other; the factors match the all-batched server within the form's
    tolerance and, for FP64 tensors, the oracle.  Out-of-range values are rejected."""
    tensors = c5_like(7, 10)
    reqs = round_robin([3] * len(tensors), 2)
    arrivals = np.arange(len(reqs)) * 5e-5  # small epochs
    batched, _, _ = run_server(dn, tensors, reqs, arrivals=arrivals, direct_max_jobs=0)
    direct, _, st = run_server(dn, tensors, reqs, arrivals=arrivals, direct_max_jobs=4)
    assert st["completed"] == len(reqs)
    for k, (X, U, prec) in enumerate(tensors):
        tol = 1e-10 if prec == "fp64" else 5e-4
        ref = oracle_sweeps(oracle_mod, X, U, [n for t, n in reqs if t == k]) if prec == "fp64" else None
        for m in range(3):
            assert nrel(direct[k][m], batched[k][m]) <= tol, (k, m)
            if ref is not None:
                assert nrel(direct[k][m], ref[m]) <= tol, (k, m)
    for bad in (-1, 65):
        with pytest.raises(dn.DeinsumError):
            dn.Server(max_jobs_per_epoch=64, direct_max_jobs=bad)
