"""Benchmark: dense MTTKRP on one MI355X at the one-GPU tile shape.

Workload (one step): X of shape 1024 x 1024 x 1024, FP64, entries uniform in
[-1, 1) from the counter-based generator; three factors 1024 x 24, N(0,1);
MTTKRP in every mode (0, 1, 2) in the plain FP64 form.  X and the factors are
resident in HBM before the timed region.  The JSON line reports GFLOP/s of the
two-stage method, the HBM roofline of the dominant kernel, the mixed-precision
forms (X stored FP32 / BF16) with their error against the FP64 oracle on
sampled rows, the Tucker-step TTMc (1024^3, ranks 32; FP64, FP32, BF16) and the CPU oracle timed
on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DIMS = (1024, 1024, 1024)
R = 24
SPECS = {0: "ijk,ja,ka->ia", 1: "ijk,ia,ka->ja", 2: "ijk,ia,ja->ka"}


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true", help="skip the mixed-precision and TTMc fields")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serving", action="store_true", help="skip the CP-ALS serving measurement")
    ap.add_argument("--no-tune", action="store_true", help="use the heuristic plans instead of autotuning first")
    ap.add_argument("--no-more", action="store_true", help="skip the order-5 MTTKRP and order-4 TTMc workloads")
    ap.add_argument("--copy-probe", action="store_true",
                    help="profiling: run one plain 1 GiB device copy first (calibrates HBM byte counters)")
    ap.add_argument("--only", default="", help="profiling: run just one part (fp64|fx20|fp32|bf16|bf16x3|ttmc|more|serving)")
    ap.add_argument("--summarize-trace", default="", metavar="CSV",
                    help="print a kernel-time table from a rocprofv3 kernel_trace.csv and exit (no GPU)")
    ap.add_argument("--summarize-pmc", default="", metavar="CSV",
                    help="print a per-kernel counter table from a rocprofv3 counter_collection.csv and exit")
    ap.add_argument("--summarize-workloads", nargs=4, default=None, metavar=("TRACE", "FETCH", "WRITE", "MFMA"),
                    help="print per-workload kernel time, HBM bytes and matrix-core use from a kernel_trace.csv and "
                         "three counter_collection.csv files (FETCH_SIZE, WRITE_SIZE, MfmaUtil passes) and exit")
    ap.add_argument("--last", type=int, default=0, help="--summarize-*: steady state = the last N launches per kernel")
    ap.add_argument("--first-run", action="store_true",
                    help="--summarize-*: the dominant kernel's launches are those of its first run (a stretch "
                         "of launches at most 50 dispatches apart: the MTTKRP step's calls, when a later "
                         "workload launches the same kernel)")
    ap.add_argument("--bytes", type=float, default=0.0,
                    help="--summarize-trace: algorithmic bytes per launch of the kernel named by --kernel")
    ap.add_argument("--kernel", default="", help="--summarize-*: substring naming the dominant kernel")
    return ap.parse_args()


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "mttkrp_1024cubed_R24_fp64_hbm_traffic.txt")
# Sources of the dominant call's kernels (mode 0 through the fused TTMc pass).
KERNEL_SOURCES = ("paper_2206_08301_amd/csrc/ttmc.hip", "paper_2206_08301_amd/csrc/ttmc.h",
                  "paper_2206_08301_amd/csrc/kernels.h")


def measured_traffic(plan_name):
    """HBM bytes per launch of the dominant kernel from the committed PMC summary (FETCH_SIZE
    and WRITE_SIZE, copy-calibrated), or None once the kernel sources differ from the ones
    the counters were taken with or the timed call ran another plan family."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    mb = re.search(r"^traffic_bytes_per_launch: (\d+)", text, re.M)
    mh = re.search(r"^kernel_sources_sha256: ([0-9a-f]{64})", text, re.M)
    mp = re.search(r"^plan_family: (\S+)", text, re.M)
    if not (mb and mh and mp) or not plan_name.startswith(mp.group(1)):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return int(mb.group(1)) if h.hexdigest() == mh.group(1) else None


def boot_ci(samples, n=2000, seed=2206083010):
    """95 % bootstrap confidence interval of the median (percentile method)."""
    import numpy as np
    a = np.asarray(samples, dtype=np.float64)
    if a.size < 2:
        return [float(a[0]), float(a[0])] if a.size else [None, None]
    rng = np.random.default_rng(seed)
    meds = np.median(a[rng.integers(0, a.size, (n, a.size))], axis=1)
    return [round(float(np.percentile(meds, 2.5)), 4), round(float(np.percentile(meds, 97.5)), 4)]


def event_samples(torch, stream, fn, reps=10):
    """Durations (ms) of `reps` back-to-back calls, HIP events on the launch stream."""
    fn()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    evs[0].record(stream)
    for k in range(reps):
        fn()
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    return [evs[k].elapsed_time(evs[k + 1]) for k in range(reps)]


def timed(torch, stream, fn, reps=10):
    """{"ms": median, "ci95_ms": bootstrap CI of the median} of `reps` event-timed calls."""
    t = event_samples(torch, stream, fn, reps)
    return statistics.median(t), boot_ci(t)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def rel_rows(got_rows, ref_rows):
    """Largest normwise relative error over the sampled rows / slabs."""
    import numpy as np
    errs = []
    for g, r in zip(got_rows, ref_rows):
        errs.append(float(np.linalg.norm(np.ravel(g) - np.ravel(r)) / np.linalg.norm(np.ravel(r))))
    return max(errs)


def more_workloads(dn, synth, torch, stream, tune):
    """Order-5 MTTKRP (80^5, R=24, modes 0 and 2: FP64, FP32, FX20), order-4 TTMc (192^4,
    ranks 16, mode 0: FP64, FP32, BF16), and the paper's order-5 forms at 60^5, R=24
    (MTTKRP mode 4: FP64, FP32, FX20; TTMc mode 0: FP64, FP32, BF16).  Every form reports
    its error against the oracle on sampled output rows / slabs, and its median time with
    a 95 % bootstrap CI."""
    import numpy as np

    import oracle
    dev = torch.device("cuda:0")
    out = {}

    def entry(t_ci, byts, flops=None):
        t, ci = t_ci
        e = {"ms": round(t, 4), "ci95_ms": ci, "GB/s": round(byts / (t / 1e3) / 1e9, 1),
             "frac_hbm": round(byts / (t / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        if flops:
            e["GFLOP/s"] = round(flops / (t / 1e3) / 1e9, 1)
        return e

    D5, R5 = (80,) * 5, 24
    seed5 = synth.config_seed(3, 0)
    X = torch.empty(D5, dtype=torch.float64, device=dev)
    dn.synth_fill(X, seed5)
    Uh = [synth.normal_factor(synth.config_seed(3, 1 + m), 80, R5) for m in range(5)]
    U = [torch.from_numpy(u).to(dev) for u in Uh]
    X32 = torch.empty(D5, dtype=torch.float32, device=dev)
    dn.convert(X, X32)
    Xf = dn.to_fx20(X)
    nx = 80 ** 5
    res = {}
    rows5 = {0: (0, 53, 79), 2: (1, 40, 79)}
    for n in (0, 2):
        spec = "abcde," + ",".join(f"{l}z" for i, l in enumerate("abcde") if i != n) + "->" + "abcde"[n] + "z"
        ops = [U[m] for m in range(5) if m != n]
        ops32 = [u.float() for u in ops]
        ref = oracle.mttkrp(synth.x_rows(seed5, D5, n, rows5[n]), [None if m == n else Uh[m] for m in range(5)], n)
        M = torch.empty((80, R5), dtype=torch.float64, device=dev)
        row = {}
        for form, Xp, opsp in (("fp64", X, ops), ("fp32", X32, ops32), ("fx20", Xf, ops32)):
            if tune:
                dn.tune_mttkrp(spec, Xp, opsp, precision=form, out=M, reps=2)
            tc = timed(torch, stream, lambda: dn.mttkrp(spec, Xp, opsp, precision=form, out=M))
            xb = {"fp64": 8, "fp32": 4, "fx20": 3}[form]
            byts = nx * xb + 4 * 80 * R5 * (8 if form == "fp64" else 4) + 80 * R5 * 8
            flops = 2 * nx * R5 + 2 * (nx // 80) * R5 * 3
            e = entry(tc, byts, flops)
            torch.cuda.synchronize()
            e["rel_err_vs_oracle_sampled_rows"] = rel_rows(M.cpu().numpy()[list(rows5[n])], ref)
            if form != "fp64":
                e["speedup_vs_fp64"] = round(row["fp64"]["ms"] / tc[0], 3)
            row[form] = e
        res[str(n)] = row
        print(f"[bench] order-5 mode {n}: {row}", file=sys.stderr, flush=True)
    out["mttkrp_order5"] = {"workload": "MTTKRP order 5, X 80^5 FP64 (26.2 GB), R=24, modes 0 and 2", "modes": res}
    del X, X32, Xf, U
    torch.cuda.empty_cache()

    D4, R4 = (192,) * 4, 16
    seed4 = synth.config_seed(4, 0)
    X = torch.empty(D4, dtype=torch.float64, device=dev)
    dn.synth_fill(X, seed4)
    Bh = [synth.orthonormal_factor(synth.config_seed(4, 1 + m), 192, R4) for m in (1, 2, 3)]
    B = [torch.from_numpy(b).to(dev) for b in Bh]
    X32 = torch.empty(D4, dtype=torch.float32, device=dev)
    dn.convert(X, X32)
    X16 = torch.empty(D4, dtype=torch.bfloat16, device=dev)
    dn.convert(X, X16)
    Xf = dn.to_fx20(X)
    Y = torch.empty((192, R4, R4, R4), dtype=torch.float64, device=dev)
    slabs4 = (0, 77, 191)
    ref4 = [oracle.ttmc(synth.x_slab(seed4, D4, 0, i), [None] + Bh, 0)[0] for i in slabs4]
    row = {}
    nx = 192 ** 4
    B32 = [b.float() for b in B]
    for form, Xp, Bp in (("fp64", X, B), ("fp32", X32, B32), ("bf16", X16, B32), ("fx20", Xf, B32)):
        if tune:
            dn.ttmc("abcd,bx,cy,dz->axyz", Xp, Bp, precision=form, out=Y, tune_reps=2)
        tc = timed(torch, stream, lambda: dn.ttmc("abcd,bx,cy,dz->axyz", Xp, Bp, precision=form, out=Y))
        xb = {"fp64": 8, "fp32": 4, "bf16": 2, "fx20": 3}[form]
        byts = nx * xb + 3 * 192 * R4 * (8 if form == "fp64" else 4) + 192 * R4 ** 3 * 8
        e = entry(tc, byts)
        torch.cuda.synchronize()
        Yh = Y.cpu().numpy()
        e["rel_err_vs_oracle_sampled_slabs"] = rel_rows([Yh[i] for i in slabs4], ref4)
        if form != "fp64":
            e["speedup_vs_fp64"] = round(row["fp64"]["ms"] / tc[0], 3)
        row[form] = e
    print(f"[bench] ttmc order-4: {row}", file=sys.stderr, flush=True)
    out["ttmc_order4"] = {"workload": "TTMc order 4 mode 0, X 192^4 FP64 (10.9 GB), ranks 16, orthonormal factors",
                          "forms": row}
    del X, X32, X16, Xf, Y
    torch.cuda.empty_cache()

    # The paper's order-5 forms at I = 60, R = 24: MTTKRP in the last mode, TTMc in mode 0.
    D6, R6 = (60,) * 5, 24
    nx = 60 ** 5
    seed6 = synth.config_seed(3, 60)
    X = torch.empty(D6, dtype=torch.float64, device=dev)
    dn.synth_fill(X, seed6)
    Uh = [synth.normal_factor(synth.config_seed(3, 61 + m), 60, R6) for m in range(5)]
    U = [torch.from_numpy(u).to(dev) for u in Uh]
    U32 = [u.float() for u in U]
    X32 = torch.empty(D6, dtype=torch.float32, device=dev)
    dn.convert(X, X32)
    X16 = torch.empty(D6, dtype=torch.bfloat16, device=dev)
    dn.convert(X, X16)
    Xf = dn.to_fx20(X)
    spec = "abcde,az,bz,cz,dz->ez"
    rows6 = (0, 31, 59)
    ref6 = oracle.mttkrp(synth.x_rows(seed6, D6, 4, rows6), Uh[:4] + [None], 4)
    M = torch.empty((60, R6), dtype=torch.float64, device=dev)
    row = {}
    for form, Xp, opsp in (("fp64", X, U[:4]), ("fp32", X32, U32[:4]), ("fx20", Xf, U32[:4])):
        if tune:
            dn.tune_mttkrp(spec, Xp, opsp, precision=form, out=M, reps=3)
        tc = timed(torch, stream, lambda: dn.mttkrp(spec, Xp, opsp, precision=form, out=M))
        xb = {"fp64": 8, "fp32": 4, "fx20": 3}[form]
        byts = nx * xb + 4 * 60 * R6 * (8 if form == "fp64" else 4) + 60 * R6 * 8
        e = entry(tc, byts)
        torch.cuda.synchronize()
        e["rel_err_vs_oracle_sampled_rows"] = rel_rows(M.cpu().numpy()[list(rows6)], ref6)
        if form != "fp64":
            e["speedup_vs_fp64"] = round(row["fp64"]["ms"] / tc[0], 3)
        row[form] = e
    print(f"[bench] order-5 60^5 mttkrp mode 4: {row}", file=sys.stderr, flush=True)
    out["mttkrp_order5_last_mode"] = {"workload": "MTTKRP order 5, X 60^5 FP64 (6.2 GB), R=24, mode 4 (last)",
                                      "forms": row}
    tspec = "abcde,bw,cx,dy,ez->awxyz"
    Y = torch.empty((60, R6, R6, R6, R6), dtype=torch.float64, device=dev)
    slabs6 = (0, 29, 59)
    ref6t = [oracle.ttmc(synth.x_slab(seed6, D6, 0, i), [None] + Uh[1:], 0)[0] for i in slabs6]
    row = {}
    for form, Xp, Bp in (("fp64", X, U[1:]), ("fp32", X32, U32[1:]), ("bf16", X16, U32[1:]), ("fx20", Xf, U32[1:])):
        if tune:
            dn.ttmc(tspec, Xp, Bp, precision=form, out=Y, tune_reps=3)
        tc = timed(torch, stream, lambda: dn.ttmc(tspec, Xp, Bp, precision=form, out=Y))
        xb = {"fp64": 8, "fp32": 4, "bf16": 2, "fx20": 3}[form]
        byts = nx * xb + 4 * 60 * R6 * (8 if form == "fp64" else 4) + 60 * R6 ** 4 * 8
        e = entry(tc, byts)
        torch.cuda.synchronize()
        Yh = Y.cpu().numpy()
        e["rel_err_vs_oracle_sampled_slabs"] = rel_rows([Yh[i] for i in slabs6], ref6t)
        if form != "fp64":
            e["speedup_vs_fp64"] = round(row["fp64"]["ms"] / tc[0], 3)
        row[form] = e
    print(f"[bench] order-5 60^5 ttmc mode 0: {row}", file=sys.stderr, flush=True)
    out["ttmc_order5"] = {"workload": "TTMc order 5 mode 0, X 60^5 FP64 (6.2 GB), ranks 24, N(0,1) factors",
                          "forms": row}
    del X, X32, X16, Xf, Y
    torch.cuda.empty_cache()
    return out


def alg_counts(dims, R, n, xbytes):
    """Algorithmic bytes (X once, factors once, output once) and two-stage flops."""
    nx = 1
    for d in dims:
        nx *= d
    fac = sum(d for m, d in enumerate(dims) if m != n) * R
    ub = 8 if xbytes == 8 else 4
    byts = nx * xbytes + fac * ub + dims[n] * R * 8
    g = len(dims) - 2 if n == len(dims) - 1 else len(dims) - 1
    flops = 2 * nx * R + 2 * (nx // dims[g]) * R * max(1, len(dims) - 2)
    return byts, flops


def _csv_rows(path):
    import csv
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(f"none of {names} in {sorted(row)}")


def _short(name):
    """Kernel name without the return type, namespaces and argument list."""
    name = re.sub(r"^void ", "", name)
    name = name.replace("deinsum::(anonymous namespace)::", "").replace("deinsum::", "")
    return re.sub(r"\((?![^()]*\)\s*$).*$|\([^()]*\)\s*$", "", name).strip()


def _first_run(ids):
    """Indices of the first run of a kernel's dispatches (ids ascending): the stretch before
    the first gap of more than 50 dispatches."""
    n = 1
    while n < len(ids) and ids[n] - ids[n - 1] <= 50:
        n += 1
    return n


def summarize_trace(path, last, dominant, alg_bytes, first_run=False):
    """Kernel-time table from a rocprofv3 kernel_trace.csv: per kernel, launches, mean, and
    the median over the last `last` launches (the steady state of a run whose tuning and
    warm-up launches come first); for the kernel matching `dominant`, bytes / that median
    (first_run: the last `last` launches of its first run)."""
    rows = sorted(_csv_rows(path), key=lambda r: int(_col(r, "Dispatch_Id", "Dispatch_ID")))
    per, ids = {}, {}
    for r in rows:
        name = _short(_col(r, "Kernel_Name", "KernelName", "Name"))
        d = (int(_col(r, "End_Timestamp", "EndNs")) - int(_col(r, "Start_Timestamp", "BeginNs"))) / 1e3
        per.setdefault(name, []).append(d)
        ids.setdefault(name, []).append(int(_col(r, "Dispatch_Id", "Dispatch_ID")))
    tot = sum(sum(v) for v in per.values())
    print(f"{'kernel':<56} {'calls':>6} {'mean us':>9} {'median us':>10} {'steady med':>10} {'min us':>9} {'% time':>7}")
    for name, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        ss = v[-last:] if last else v
        print(f"{name[:56]:<56} {len(v):>6} {statistics.mean(v):>9.1f} {statistics.median(v):>10.1f} "
              f"{statistics.median(ss):>10.1f} {min(v):>9.1f} {100 * sum(v) / tot:>7.2f}")
    if dominant:
        hits = [n for n in per if dominant in n]
        if len(hits) == 1:
            v = per[hits[0]]
            if first_run:
                n = _first_run(ids[hits[0]])
                ss = v[:n][-last:] if last else v[:n]
                which = f"the last {len(ss)} of the {n} launches of its first run; {len(v)} in all"
            else:
                ss = v[-last:] if last else v
                which = f"the last {len(ss)} of {len(v)}"
            med = statistics.median(ss)
            print(f"\ndominant kernel: {hits[0]}")
            print(f"steady-state launches: {len(ss)} ({which}); median {med:.1f} us")
            if alg_bytes:
                gbs = alg_bytes / (med * 1e-6) / 1e9
                print(f"algorithmic bytes per launch {alg_bytes:.0f} / median = {gbs:.1f} GB/s "
                      f"= {gbs / HBM_PEAK_GBS:.4f} of {HBM_PEAK_GBS:.0f} GB/s")
        else:
            print(f"\ndominant kernel: {len(hits)} names match {dominant!r}: {hits}")


def summarize_pmc(path, dominant, first_run=False):
    """Per-kernel counter table from a rocprofv3 counter_collection.csv: each counter summed
    per dispatch, then averaged over the dispatches of a kernel.  The runtime's copy kernel
    (bench.py --copy-probe: 1 GiB read and written) calibrates FETCH_SIZE / WRITE_SIZE."""
    rows = _csv_rows(path)
    disp = {}
    for r in rows:
        key = (int(_col(r, "Dispatch_Id", "Dispatch_ID", "dispatch")), _short(_col(r, "Kernel_Name", "KernelName", "Name")))
        cname = _col(r, "Counter_Name", "CounterName")
        disp.setdefault(key, {}).setdefault(cname, 0.0)
        disp[key][cname] += float(_col(r, "Counter_Value", "CounterValue"))
    per, ids = {}, {}
    for (d, name), cs in sorted(disp.items(), key=lambda kv: kv[0][0]):  # dispatch order
        ids.setdefault(name, []).append(d)
        for c, v in cs.items():
            per.setdefault(name, {}).setdefault(c, []).append(v)
    # The calibration copy: the runtime copy dispatches issued before the first kernel of
    # the library (the 1 GiB probe runs before X is generated); later copies are uploads.
    first_lib = min((d for d, name in disp if "copyBuffer" not in name and "at::" not in name), default=None)
    probe = {c: sum(cs.get(c, 0.0) for (d, name), cs in disp.items()
                    if "copyBuffer" in name and (first_lib is None or d < first_lib))
             for c in ("FETCH_SIZE", "WRITE_SIZE")}
    counters = sorted({c for cs in per.values() for c in cs})
    print(f"{'kernel':<70} {'n':>4} " + " ".join(f"{c:>14}" for c in counters))
    for name, cs in sorted(per.items(), key=lambda kv: kv[0]):
        n = max(len(v) for v in cs.values())
        print(f"{name[:70]:<70} {n:>4} " + " ".join(f"{statistics.mean(cs[c]) if c in cs else 0.0:>14.1f}"
                                                    for c in counters))
    if dominant and any(probe.values()):
        gib_kib = float(1 << 20)
        scale = {c: gib_kib / v for c, v in probe.items() if v > 0}
        for c, v in probe.items():
            if v > 0:
                print(f"calibration copy (1 GiB read + 1 GiB written): {c} {v:.1f} KiB -> scale {gib_kib / v:.4f}")
        hits = [n for n in per if dominant in n]
        for h in hits:
            for c, sc in scale.items():
                if c in per[h]:
                    n = _first_run(ids[h]) if first_run else len(per[h][c])
                    vals = per[h][c][:n]
                    kib = statistics.mean(vals)
                    sel = f" (the {n} dispatches of its first run, of {len(per[h][c])})" if first_run else ""
                    print(f"{h[:60]}: {c} {kib:.1f} KiB per dispatch{sel} x {sc:.4f} (copy calibration) = "
                          f"{kib * sc * 1024:.0f} bytes")


def _launch_groups(path, is_trace):
    """Dispatches of the matrix-core kernels grouped by (kernel, grid size, run): a run is a
    stretch of launches of one kernel and grid no more than 50 dispatches apart, so the
    calls of one workload and form (its warm-up launch first) form one group."""
    rows = _csv_rows(path)
    per = {}
    for r in rows:
        d = int(_col(r, "Dispatch_Id", "Dispatch_ID"))
        name = _short(_col(r, "Kernel_Name", "KernelName"))
        if not any(k in name for k in ("stream_kernel", "ttmc_fused", "small_ttm")):
            continue
        grid = int(_col(r, "Grid_Size_X", "Grid_Size")) if is_trace else int(_col(r, "Grid_Size"))
        e = per.setdefault(d, {"name": name, "grid": grid, "c": {}})
        if is_trace:
            e["c"]["us"] = (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) / 1e3
        else:
            c = _col(r, "Counter_Name")
            e["c"][c] = e["c"].get(c, 0.0) + float(_col(r, "Counter_Value"))
    groups = {}
    for d in sorted(per):
        e = per[d]
        runs = groups.setdefault((e["name"], e["grid"]), [])
        if not runs or d - runs[-1][-1][0] > 50:
            runs.append([])
        runs[-1].append((d, e["c"]))
    return groups


def summarize_workloads(trace, fetch, write, mfma):
    """Per (kernel, grid, run): launches, steady-state median duration (the run without its
    first launch), HBM bytes per launch from FETCH_SIZE / WRITE_SIZE scaled by the 1 GiB
    calibration copy, matrix-core utilisation and executed matrix-core GFLOP per launch."""
    def probe_scale(path, c):
        rows = _csv_rows(path)
        first_lib, tot = None, 0.0
        disp = {}
        for r in rows:
            d = int(_col(r, "Dispatch_Id")); name = _col(r, "Kernel_Name")
            if _col(r, "Counter_Name") == c:
                disp[d] = (name, disp.get(d, (name, 0.0))[1] + float(_col(r, "Counter_Value")))
        libs = [d for d, (n, _) in disp.items() if "copyBuffer" not in n and "at::" not in n]
        first_lib = min(libs) if libs else None
        tot = sum(v for d, (n, v) in disp.items() if "copyBuffer" in n and (first_lib is None or d < first_lib))
        return float(1 << 30) / (tot * 1024) if tot else None
    sf, sw = probe_scale(fetch, "FETCH_SIZE"), probe_scale(write, "WRITE_SIZE")
    print(f"calibration: FETCH_SIZE x {sf:.4f}, WRITE_SIZE x {sw:.4f} (1 GiB device copy before the first library kernel)")
    gt, gf, gw, gm = (_launch_groups(trace, True), _launch_groups(fetch, False), _launch_groups(write, False),
                      _launch_groups(mfma, False))
    print(f"{'kernel':<52} {'grid':>8} {'run':>3} {'n':>3} {'steady us':>10} {'HBM GB':>8} {'GB/s':>7} "
          f"{'MfmaUtil':>8} {'F64 GF':>7} {'F16 GF':>7}")
    for key in sorted(gf, key=lambda k: gf[k][0][0][0]):
        for ri, run in enumerate(gf[key]):
            fb = statistics.mean(c.get("FETCH_SIZE", 0.0) for _, c in run) * 1024 * sf
            wr = gw.get(key, [])
            wb = statistics.mean(c.get("WRITE_SIZE", 0.0) for _, c in wr[ri]) * 1024 * sw if ri < len(wr) else float("nan")
            tr = gt.get(key, [])
            us = statistics.median([c["us"] for _, c in tr[ri][1:]] or [c["us"] for _, c in tr[ri]]) if ri < len(tr) else float("nan")
            mr = gm.get(key, [])
            mu = statistics.mean(c.get("MfmaUtil", 0.0) for _, c in mr[ri]) if ri < len(mr) else float("nan")
            f64 = statistics.mean(c.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) for _, c in mr[ri]) * 512 / 1e9 if ri < len(mr) else float("nan")
            f16 = statistics.mean(c.get("SQ_INSTS_VALU_MFMA_MOPS_F16", 0.0) for _, c in mr[ri]) * 512 / 1e9 if ri < len(mr) else float("nan")
            hbm = fb + wb
            print(f"{key[0][:52]:<52} {key[1]:>8} {ri:>3} {len(run):>3} {us:>10.1f} {hbm / 1e9:>8.3f} "
                  f"{hbm / (us * 1e-6) / 1e9:>7.0f} {mu:>8.1f} {f64:>7.2f} {f16:>7.2f}")


def main():
    args = parse_args()
    if args.summarize_workloads:
        summarize_workloads(*args.summarize_workloads)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.last, args.kernel, args.bytes, args.first_run)
        return
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc, args.kernel, args.first_run)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; sharding across GPUs is not implemented",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2206_08301_amd as dn
    from paper_2206_08301_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    seed = synth.config_seed(2, 0)

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print(f"[bench] generating X {DIMS} fp64 on the device", file=sys.stderr, flush=True)
    X = torch.empty(DIMS, dtype=torch.float64, device=dev)
    dn.synth_fill(X, seed)
    U = [synth.normal_factor(synth.config_seed(2, 1 + m), DIMS[m], R) for m in range(3)]
    Ud = [torch.from_numpy(u).to(dev) for u in U]
    Uf = [u.float() for u in Ud]
    ops = {n: [Ud[m] for m in range(3) if m != n] for n in range(3)}
    opsf = {n: [Uf[m] for m in range(3) if m != n] for n in range(3)}
    outs = {n: torch.empty((DIMS[n], R), dtype=torch.float64, device=dev) for n in range(3)}
    reports = {n: dn.Report() for n in range(3)}
    torch.cuda.synchronize()

    def step():
        for n in range(3):
            dn.mttkrp(SPECS[n], X, ops[n], out=outs[n])

    # ---- the timed step (FP64, three modes)
    steps, warmup = args.steps, args.warmup
    if args.only and args.only != "fp64":
        steps = 0
    ms_step = float("nan")
    per_mode_ms = {0: [], 1: [], 2: []}
    kernel_ms = {0: [], 1: [], 2: []}   # each call's main kernel alone (library HIP events)
    step_ms = []
    tune = not args.no_tune
    if steps:
        for n in range(3):
            if tune:  # the library's autotuner picks each mode's plan (untimed, cached)
                dn.tune_mttkrp(SPECS[n], X, ops[n], out=outs[n], reps=5)
            dn.mttkrp(SPECS[n], X, ops[n], out=outs[n], report=reports[n])
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        # The timed region: K steps, bracketed by device synchronisation.  The library
        # records HIP events around each call's main kernel on the launch stream
        # (deinsum_kernel_timing), which gives the dominant kernel's own duration.
        dn.kernel_timing(True, 3 * steps + 16)
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms_step = (time.perf_counter() - t0) * 1e3 / steps
        dn.kernel_timing(False)
        kt = dn.kernel_times()
        if len(kt) == 3 * steps:  # one main kernel per call, calls in mode order
            for i, (_, ms) in enumerate(kt):
                kernel_ms[i % 3].append(ms)
        # per-call durations with HIP events on the launch stream
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        for s in range(steps):
            ev[s][0].record(stream)
            for n in range(3):
                dn.mttkrp(SPECS[n], X, ops[n], out=outs[n])
                ev[s][n + 1].record(stream)
        torch.cuda.synchronize()
        for s in range(steps):
            step_ms.append(ev[s][0].elapsed_time(ev[s][3]))
            for n in range(3):
                per_mode_ms[n].append(ev[s][n].elapsed_time(ev[s][n + 1]))

    flops_step = sum(alg_counts(DIMS, R, n, 8)[1] for n in range(3))
    bytes_mode = {n: alg_counts(DIMS, R, n, 8)[0] for n in range(3)}
    result = {
        "metric": "MTTKRP/TTMc GFLOP/s & %roofline (FP64 vs mixed); p99 latency batched",
        "value": round(flops_step / (ms_step / 1e3) / 1e9, 1) if steps else None,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_step, 4) if steps else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (counter-based SplitMix64 X, uniform [-1,1); N(0,1) factors)",
        "config": {"workload": "MTTKRP order 3, X 1024x1024x1024 FP64, R=24, modes 0+1+2 per step",
                   "global_batch": 1, "parallelism": "single GPU"},
    }
    if steps:
        med = {n: statistics.median(per_mode_ms[n]) for n in range(3)}
        gbs = {n: bytes_mode[n] / (med[n] / 1e3) / 1e9 for n in range(3)}
        result["step_ms_event"] = {"median": round(statistics.median(step_ms), 4), "ci95": boot_ci(step_ms)}
        # Dominant kernel: the main kernel of the step's longest call, mode 0 (the fused
        # TTMc pass unless the tuner picked the K-contiguous kernel); its duration is the
        # median over the timed steps of the library's HIP events around that kernel.
        plan0 = reports[0].plan_name.decode()
        kname = ("ttmc_fused_kernel (MTTKRP mode 0 through the fused TTMc pass)" if plan0.startswith("mttkrp_via_ttmc")
                 else "mttkrp_stream_kernel (K-contiguous MTTKRP, mode 0)")
        if kernel_ms[0]:
            k0 = statistics.median(kernel_ms[0])
            how = ("median over the timed steps of the kernel's own duration, HIP events recorded by the "
                   "library on the launch stream around that kernel")
        else:
            k0 = med[0]
            how = "median call duration (HIP events around the whole call)"
        dom_gbs = bytes_mode[0] / (k0 / 1e3) / 1e9
        # Streaming peak of this machine: a plain full read of the same 8 GiB X (torch's sum,
        # the runtime's own reduction), median of 10, against which the fraction is also given.
        probe_ms = event_samples(torch, stream, lambda: X.sum(), 10)
        probe_gbs = X.numel() * 8 / (statistics.median(probe_ms) / 1e3) / 1e9
        result["roofline"] = {"bound": "hbm", "achieved": round(dom_gbs, 1), "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": round(dom_gbs / HBM_PEAK_GBS, 4),
                              "traffic": measured_traffic(plan0),
                              "kernel": kname, "kernel_ms": round(k0, 4),
                              "kernel_ms_ci95": boot_ci(kernel_ms[0]) if kernel_ms[0] else None,
                              "alg_bytes_per_launch": bytes_mode[0], "duration": how,
                              "measured_stream_GBps": round(probe_gbs, 1),
                              "frac_of_measured_stream": round(dom_gbs / probe_gbs, 4),
                              "stream_probe": "full read of the 8 GiB FP64 X by torch.sum, median of 10 event-timed runs"}
        result["modes"] = {}
        for n in range(3):
            e = {"ms": round(med[n], 4), "ci95_ms": boot_ci(per_mode_ms[n]), "GB/s": round(gbs[n], 1),
                 "frac_hbm": round(gbs[n] / HBM_PEAK_GBS, 4),
                 "GFLOP/s": round(alg_counts(DIMS, R, n, 8)[1] / (med[n] / 1e3) / 1e9, 1),
                 "plan": reports[n].plan_name.decode()}
            if kernel_ms[n]:
                km = statistics.median(kernel_ms[n])
                e["kernel_ms"] = round(km, 4)
                e["kernel_frac_hbm"] = round(bytes_mode[n] / (km / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
            result["modes"][str(n)] = e

    # ---- parity spot check of the timed outputs (sampled rows against the oracle)
    import oracle
    checks = {}

    def sampled_error(Mdev_by_mode, rows=(3, 700)):
        errs = []
        for n, Md in Mdev_by_mode.items():
            Mh = Md.double().cpu().numpy()
            Un = [None if m == n else U[m] for m in range(3)]
            for i in rows:
                ref = oracle.mttkrp(synth.x_slab(seed, DIMS, n, i), Un, n)[0]
                errs.append(float(np.linalg.norm(Mh[i] - ref) / np.linalg.norm(ref)))
        return max(errs)

    if steps:
        checks["fp64_max_rel_err_sampled"] = sampled_error(outs)

    # ---- mixed-precision forms and TTMc (extras)
    if not args.no_extras:
        forms = {}
        X32 = torch.empty(DIMS, dtype=torch.float32, device=dev)
        dn.convert(X, X32)
        Xb = None
        Xf = None
        forms_all = ("fx20", "fp32", "bf16x3", "bf16")
        todo = list(forms_all) if not args.only else ([args.only] if args.only in forms_all else [])
        # One-off cost of storing X in each form's storage (paid once per tensor, then
        # amortised over modes and sweeps): median of 3 event-timed conversions.
        storage_ms = {}
        if todo:
            storage_ms["f32"] = timed(torch, stream, lambda: dn.convert(X, X32), 3)
        for prec in todo:
            if prec == "bf16" and Xb is None:
                Xb = torch.empty(DIMS, dtype=torch.bfloat16, device=dev)
                storage_ms["bf16"] = timed(torch, stream, lambda: dn.convert(X, Xb), 3)
            if prec == "fx20" and Xf is None:
                storage_ms["fx20"] = timed(torch, stream, lambda: dn.to_fx20(X), 3)
                Xf = dn.to_fx20(X)
            Xp = Xb if prec == "bf16" else (Xf if prec == "fx20" else X32)
            skey = {"bf16": "bf16", "fx20": "fx20"}.get(prec, "f32")
            modes = [0, 1, 2]
            o32 = {n: torch.empty((DIMS[n], R), dtype=torch.float32, device=dev) for n in modes}
            if tune:
                for n in modes:
                    dn.tune_mttkrp(SPECS[n], Xp, opsf[n], precision=prec, out=o32[n], reps=3)
            preps = {n: dn.Report() for n in modes}
            for n in modes:
                dn.mttkrp(SPECS[n], Xp, opsf[n], precision=prec, out=o32[n], report=preps[n])
            torch.cuda.synchronize()
            res = {}
            for n in modes:
                t, ci = timed(torch, stream, lambda: dn.mttkrp(SPECS[n], Xp, opsf[n], precision=prec, out=o32[n]))
                xb = {"bf16": 2, "fx20": 3}.get(prec, 4)
                b, f = alg_counts(DIMS, R, n, xb)
                res[str(n)] = {"ms": round(t, 4), "ci95_ms": ci, "GB/s": round(b / (t / 1e3) / 1e9, 1),
                               "frac_hbm": round(b / (t / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                               "GFLOP/s": round(f / (t / 1e3) / 1e9, 1), "plan": preps[n].plan_name.decode(),
                               "est_err": preps[n].est_err}
                if steps:
                    res[str(n)]["speedup_vs_fp64"] = round(med[n] / t, 3)
            err = sampled_error(o32)
            st_ms = storage_ms[skey][0]
            forms[prec] = {"x_storage": {"bf16": "bf16", "fx20": "fx20 (20-bit fixed point: FP16 + int8 planes, 3 bytes)"}.get(prec, "f32"),
                           "storage_conversion_ms": round(st_ms, 4),
                           "storage_conversion_ci95_ms": storage_ms[skey][1],
                           "modes": res,
                           "max_rel_err_sampled_vs_fp64_oracle": err}
            if steps:
                # speedup of one 3-mode step with the conversion paid once in it, and the
                # number of steps after which the form has paid for its conversion
                t_form = sum(res[str(n)]["ms"] for n in modes)
                t64 = sum(med[n] for n in modes)
                forms[prec]["step_speedup_incl_conversion"] = round(t64 / (t_form + st_ms), 3)
                forms[prec]["steps_to_amortise_conversion"] = (round(st_ms / (t64 - t_form), 2)
                                                               if t64 > t_form else None)
            print(f"[bench] {prec}: {res} err {err:.2e} conversion {st_ms:.3f} ms", file=sys.stderr, flush=True)
        if forms:
            result["mixed_forms"] = forms
        del X32, Xb, Xf
        torch.cuda.empty_cache()
        if not args.only or args.only == "ttmc":
            Rt = 32
            Bt = [torch.from_numpy(synth.orthonormal_factor(synth.config_seed(4, 1 + m), 1024, Rt)).to(dev)
                  for m in (1, 2)]
            Y = torch.empty((1024, Rt, Rt), dtype=torch.float64, device=dev)
            if tune:
                dn.ttmc("ijk,jb,kc->ibc", X, Bt, out=Y, tune_reps=7)
            t, ci = timed(torch, stream, lambda: dn.ttmc("ijk,jb,kc->ibc", X, Bt, out=Y))
            nx = 1024 ** 3
            b = nx * 8 + 2 * 1024 * Rt * 8 + 1024 * Rt * Rt * 8
            f = 2 * nx * Rt + 2 * 1024 * 1024 * Rt * Rt
            Bh = [None] + [b_.cpu().numpy() for b_ in Bt]
            tslabs = (5, 512, 999)
            tref = [oracle.ttmc(synth.x_slab(seed, DIMS, 0, i), Bh, 0)[0] for i in tslabs]
            torch.cuda.synchronize()
            result["ttmc"] = {"workload": "TTMc order 3 mode 0, X 1024^3 FP64, B and C 1024x32 orthonormal",
                              "ms": round(t, 4), "ci95_ms": ci, "GB/s": round(b / (t / 1e3) / 1e9, 1),
                              "frac_hbm": round(b / (t / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                              "GFLOP/s": round(f / (t / 1e3) / 1e9, 1),
                              "max_rel_err_sampled": rel_rows([Y[i].cpu().numpy() for i in tslabs], tref)}
            # reduced-precision forms of the same TTMc: X stored FP32 / BF16, FP32 factors
            tforms = {}
            B32 = [b_.float() for b_ in Bt]
            for form, tdt in (("fp32", torch.float32), ("bf16", torch.bfloat16), ("fx20", None)):
                if form == "fx20":
                    Xt = dn.to_fx20(X)
                else:
                    Xt = torch.empty(DIMS, dtype=tdt, device=dev)
                    dn.convert(X, Xt)
                Yt = torch.empty_like(Y)
                if tune:
                    dn.ttmc("ijk,jb,kc->ibc", Xt, B32, precision=form, out=Yt, tune_reps=7)
                tt, tci = timed(torch, stream, lambda: dn.ttmc("ijk,jb,kc->ibc", Xt, B32, precision=form, out=Yt))
                xb = {"fp32": 4, "bf16": 2, "fx20": 3}[form]
                bt = nx * xb + 2 * 1024 * Rt * 4 + 1024 * Rt * Rt * 8
                torch.cuda.synchronize()
                tforms[form] = {"ms": round(tt, 4), "ci95_ms": tci, "GB/s": round(bt / (tt / 1e3) / 1e9, 1),
                                "frac_hbm": round(bt / (tt / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                                "speedup_vs_fp64": round(t / tt, 3),
                                "rel_err_vs_oracle_sampled_slabs": rel_rows([Yt[i].cpu().numpy() for i in tslabs],
                                                                            tref)}
                del Xt, Yt
                torch.cuda.empty_cache()
            result["ttmc"]["forms"] = tforms
            print(f"[bench] ttmc forms: {tforms}", file=sys.stderr, flush=True)
    result["checks"] = checks

    # ---- the other single-GPU workloads: order-5 MTTKRP and order-4 TTMc (extras)
    if not args.no_extras and not args.no_more and (not args.only or args.only == "more"):
        X = None  # the 1024^3 tensor is no longer needed
        torch.cuda.empty_cache()
        result["more_workloads"] = more_workloads(dn, synth, torch, stream, tune)

    # ---- CP-ALS serving: continuous batching vs one launch per request (extras)
    if not args.no_extras and not args.no_serving and (not args.only or args.only == "serving"):
        from paper_2206_08301_amd import serve_workload
        X = None
        torch.cuda.empty_cache()
        result["serving"] = serve_workload.measure(
            dn, repeats=int(os.environ.get("BENCH_SERVE_REPEATS", "5")),
            log=lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))

    # ---- CPU oracle on a bounded sample of the same workload: all three modes over
    # 64-row slabs of the benchmark's own X (the same counter-based values the GPU read,
    # drawn in host RAM; generation not timed) until about BENCH_CPU_SECONDS of oracle time.
    if not args.no_cpu:
        budget = float(os.environ.get("BENCH_CPU_SECONDS", "12"))
        t, rows, f = 0.0, 0, 0
        slab = DIMS[1] * DIMS[2]
        while rows < DIMS[0] and t < budget:
            Xs = synth.x_range(seed, rows * slab, 64 * slab).reshape(64, DIMS[1], DIMS[2])
            for n in range(3):
                Un = [None if m == n else U[m][rows:rows + 64] if m == 0 else U[m] for m in range(3)]
                t0 = time.perf_counter()
                oracle.mttkrp(Xs, Un, n)
                t += time.perf_counter() - t0
                f += alg_counts((64, DIMS[1], DIMS[2]), R, n, 8)[1]
            rows += 64
            del Xs
        # The 64^3 R=16 mode-0 workload on one thread (median of 3 runs, in a process of
        # its own that loads no other OpenMP runtime, so that OpenMP starts with one thread).
        single = None
        try:
            import subprocess
            code = ("import time, statistics, sys, importlib.util; sys.path.insert(0, %r); import oracle; "
                    "sp = importlib.util.spec_from_file_location('synth', oracle.__file__.rsplit('/', 2)[0] + "
                    "'/paper_2206_08301_amd/synth.py'); synth = importlib.util.module_from_spec(sp); "
                    "sp.loader.exec_module(synth); "
                    "X = synth.x_tensor(synth.config_seed(1, 0), (64, 64, 64)); "
                    "U = [None] + [synth.normal_factor(synth.config_seed(1, 1 + m), 64, 16) for m in (1, 2)]; "
                    "ts = []\n"
                    "for _ in range(3):\n"
                    "    t0 = time.perf_counter(); oracle.mttkrp(X, U, 0); ts.append(time.perf_counter() - t0)\n"
                    "print(oracle.num_threads(), statistics.median(ts))") % ROOT
            env = dict(os.environ, OMP_NUM_THREADS="1")
            r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120)
            th, sec = r.stdout.split()[-2:]
            flops1 = alg_counts((64, 64, 64), 16, 0, 8)[1]
            single = {"workload": "MTTKRP order 3, X 64^3 FP64, R=16, mode 0", "threads": int(th),
                      "ms": round(float(sec) * 1e3, 3), "GFLOP/s": round(flops1 / float(sec) / 1e9, 3)}
        except Exception as exc:  # reported, not fatal: the baseline above stands on its own
            single = {"error": str(exc)[:200]}
        result["cpu_baseline"] = {"value": round(f / t / 1e9, 3), "unit": "GFLOP/s", "cores": oracle.num_threads(),
                                  "kind": "oracle", "cpu_model": cpu_model(),
                                  "sample": f"MTTKRP modes 0, 1 and 2 of the 1024^3 R=24 FP64 step restricted to "
                                            f"{rows} of the 1024 mode-0 slices (64 at a time; X the benchmark's "
                                            f"own counter-based values, drawn in host RAM, generation excluded), "
                                            f"{t:.1f} s of oracle time; flops counted as for the GPU",
                                  "single_thread_small": single}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
