"""Synthetic CP-ALS serving workload and its measurement (continuous batching vs
one launch per request), driven through the library's request server.

Workload: ``n_requests`` mode-n CP-ALS updates (MTTKRP + factor update) over
ceil(n_requests / (order * sweeps)) resident order-3 tensors.  Each dim is
uniform on [32, 512], the rank uniform on {8, 16, 32, 64}, FP32 with
probability 0.7 else FP64; X ~ U[-1, 1] from the counter generator, factors
N(0, 1).  Request q goes to tensor q mod T and cycles through that tensor's
modes.  Arrivals are a Poisson process of rate ``rate`` per second.

Latency = host-observed completion - scheduled arrival.  Two kinds of run per
server mode: open loop at the Poisson arrivals (``repeats`` runs, the two modes
alternating, after an untimed warm-up of both on the first 512 requests; p50/p99
of the pooled latencies with a 95 % bootstrap interval), and
saturation with every request released at t = 0 (throughput in requests/s and
algorithmic GB/s).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import synth as _synth

ARRIVAL_SEED = 2206083599
TENSOR_SEED = 2206090000
RANKS = (8, 16, 32, 64)


def make_workload(n_requests=4096, rate=2000.0, sweeps=10, order=3, lo=32, hi=512, fp32_share=0.7,
                  seed=ARRIVAL_SEED):
    rng = np.random.default_rng(seed)
    n_tensors = math.ceil(n_requests / (order * sweeps))
    tensors = []
    for t in range(n_tensors):
        dims = tuple(int(d) for d in rng.integers(lo, hi + 1, order))
        R = int(rng.choice(RANKS))
        prec = "fp32" if rng.random() < fp32_share else "fp64"
        tensors.append({"dims": dims, "R": R, "prec": prec, "seed": TENSOR_SEED + 10 * t})
    q = np.arange(n_requests)
    tensor_of = (q % n_tensors).astype(np.int32)
    mode_of = ((q // n_tensors) % order).astype(np.int32)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    return {"tensors": tensors, "tensor_of": tensor_of, "mode_of": mode_of, "arrivals": arrivals,
            "rate": rate, "order": order}


def materialise(dn, wl, device="cuda"):
    """Device X and initial factors for every tensor (X from the counter generator)."""
    state = []
    for t in wl["tensors"]:
        dt = torch.float64 if t["prec"] == "fp64" else torch.float32
        X = torch.empty(t["dims"], dtype=dt, device=device)
        dn.synth_fill(X, t["seed"])
        U0 = [torch.from_numpy(_synth.normal_factor(t["seed"] + 1 + m, d, t["R"])).to(dt).to(device)
              for m, d in enumerate(t["dims"])]
        state.append({"X": X, "U0": U0, "U": [u.clone() for u in U0], "prec": t["prec"]})
    torch.cuda.synchronize()
    return state


def request_bytes(wl):
    """Algorithmic HBM bytes of each request's MTTKRP: X once, the other factors, the output."""
    out = np.zeros(len(wl["tensor_of"]))
    for q, (t, n) in enumerate(zip(wl["tensor_of"], wl["mode_of"])):
        spec = wl["tensors"][t]
        e = 8 if spec["prec"] == "fp64" else 4
        vol = int(np.prod(spec["dims"]))
        fac = sum(spec["dims"][m] for m in range(len(spec["dims"])) if m != n) * spec["R"] * e
        out[q] = vol * e + fac + spec["dims"][n] * spec["R"] * 8
    return out


def serve_once(dn, wl, state, batched, open_loop, max_jobs=256, epochs_in_flight=2, **server_kw):
    for s in state:
        for u, u0 in zip(s["U"], s["U0"]):
            u.copy_(u0)
    torch.cuda.synchronize()
    n = len(wl["tensor_of"])
    srv = dn.Server(batched=batched, max_jobs_per_epoch=max_jobs, epochs_in_flight=epochs_in_flight,
                    max_requests=n + 16, **server_kw)
    for s in state:
        srv.add_tensor(s["X"], s["U"], precision=s["prec"])
    srv.start()
    arrivals = wl["arrivals"] if open_loop else np.zeros(n)
    srv.replay(arrivals, wl["tensor_of"], wl["mode_of"])
    srv.drain()
    arr, done, ep = srv.results()
    stats = srv.stats()
    srv.close()
    lat = done - arr
    span = float(done.max() - arr.min())
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "max_ms": float(lat.max() * 1e3), "req_per_s": n / span, "span_s": span,
            "epochs": stats["epochs"], "max_batch": stats["max_batch"], "completed": stats["completed"],
            "lat": lat}


def percentile_ci(runs, q, n_boot=1000, seed=2206083600):
    """Percentile q of the latencies pooled over the runs, with a 95 % bootstrap interval
    (each resample redraws every run's latencies with replacement, run sizes kept)."""
    rng = np.random.default_rng(seed)
    pooled = np.concatenate(runs)
    est = float(np.percentile(pooled, q))
    boots = np.empty(n_boot)
    for b in range(n_boot):
        boots[b] = np.percentile(np.concatenate([r[rng.integers(0, len(r), len(r))] for r in runs]), q)
    lo, hi = np.percentile(boots, [2.5, 97.5])
    return est, float(lo), float(hi)


def measure(dn, n_requests=4096, rate=2000.0, sweeps=10, repeats=3, log=None):
    wl = make_workload(n_requests=n_requests, rate=rate, sweeps=sweeps)
    state = materialise(dn, wl)
    total_bytes = float(request_bytes(wl).sum())
    out = {"workload": f"{n_requests} CP-ALS requests (MTTKRP + factor update), {len(wl['tensors'])} order-3 "
                       f"tensors, dims U[32,512], R in {{8,16,32,64}}, 70% FP32, Poisson {rate:g}/s, "
                       f"{sweeps} sweeps",
           "resident_gb": sum(s["X"].numel() * s["X"].element_size() for s in state) / 1e9,
           "statistic": f"p50 / p99 of the latencies pooled over {repeats} open-loop runs per server mode "
                        "(the two modes alternate run by run), 95 % bootstrap interval over the pooled runs"}
    modes = (("batched", True), ("per_request", False))
    # Untimed warm-up of both servers on the first 512 requests: the first launches of the
    # batch graph, the update kernels and every plan in the process load their code.
    warm = dict(wl, tensor_of=wl["tensor_of"][:512], mode_of=wl["mode_of"][:512], arrivals=wl["arrivals"][:512])
    for _, batched in modes:
        serve_once(dn, warm, state, batched, open_loop=True)
    runs = {name: [] for name, _ in modes}
    for r in range(repeats):
        for name, batched in (modes if r % 2 == 0 else modes[::-1]):
            runs[name].append(serve_once(dn, wl, state, batched, open_loop=True))
            if log:
                log(f"serving {name} open-loop run {r}: p50 {runs[name][-1]['p50_ms']:.3f} ms "
                    f"p99 {runs[name][-1]['p99_ms']:.3f} ms epochs {runs[name][-1]['epochs']}")
    for name, batched in modes:
        lats = [d["lat"] for d in runs[name]]
        p50 = percentile_ci(lats, 50)
        p99 = percentile_ci(lats, 99)
        sat = serve_once(dn, wl, state, batched, open_loop=False)
        if log:
            log(f"serving {name} saturation: {sat['req_per_s']:.0f} req/s, max batch {sat['max_batch']}")
        out[name] = {"p50_ms": p50[0] * 1e3, "p50_ci95_ms": [p50[1] * 1e3, p50[2] * 1e3],
                     "p99_ms": p99[0] * 1e3, "p99_ci95_ms": [p99[1] * 1e3, p99[2] * 1e3],
                     "runs_p50_ms": [d["p50_ms"] for d in runs[name]],
                     "runs_p99_ms": [d["p99_ms"] for d in runs[name]],
                     "open_loop_req_per_s": float(np.median([d["req_per_s"] for d in runs[name]])),
                     "epochs": int(np.median([d["epochs"] for d in runs[name]])),
                     "saturation_req_per_s": sat["req_per_s"],
                     "saturation_GBps": total_bytes / sat["span_s"] / 1e9,
                     "saturation_p99_ms": sat["p99_ms"], "saturation_max_batch": sat["max_batch"]}
    b, p = out["batched"], out["per_request"]
    out["p99_ratio"] = p["p99_ms"] / b["p99_ms"]
    out["p50_ratio"] = p["p50_ms"] / b["p50_ms"]
    out["p99_ci_disjoint"] = b["p99_ci95_ms"][1] < p["p99_ci95_ms"][0]
    out["throughput_ratio"] = b["saturation_req_per_s"] / p["saturation_req_per_s"]
    return out
