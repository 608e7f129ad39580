"""Host tests (no GPU) of bench.py's profile summaries: the dominant kernel's steady state
and HBM bytes are taken from its first run of launches when a later workload launches the
same kernel variant, and the copy probe calibrates the byte counters."""
import csv

import pytest

import bench

KERNEL = "void deinsum::(anonymous namespace)::ttmc_fused_kernel<0, 2, 2, 4, true, 2, 3, true>(deinsum::TkArgs)"
OTHER = "void deinsum::(anonymous namespace)::reduce_strided_kernel(deinsum::ReduceArgs)"


def test_first_run_splits_at_gaps_over_50_dispatches():
    assert bench._first_run([3]) == 1
    assert bench._first_run([3, 10, 60, 110]) == 4    # gaps of 7, 50, 50: one run
    assert bench._first_run([3, 10, 61, 70]) == 2     # gap of 51 ends the first run
    assert bench._first_run([5, 200, 201]) == 1


def write_trace(path, launches):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        t = 0
        for d, name, us in launches:
            w.writerow([d, name, t, t + int(us * 1000)])
            t += int(us * 1000) + 1000


def test_trace_first_run_keeps_later_workload_out(tmp_path, capsys):
    # the MTTKRP step's mode-0 calls (dispatches 10-18, every third), then 300 dispatches
    # later the TTMc workload's slower calls of the same kernel
    step = [(10 + 3 * k, KERNEL, us) for k, us in enumerate([1500, 1400, 1340, 1330, 1335, 1338])]
    others = [(11 + 3 * k, OTHER, 10) for k in range(6)]
    ttmc = [(330 + 2 * k, KERNEL, 1600) for k in range(5)]
    p = tmp_path / "trace.csv"
    write_trace(p, sorted(step + others + ttmc))
    alg = 8590524416
    bench.summarize_trace(str(p), 5, "ttmc_fused_kernel<0, 2, 2, 4", alg, first_run=True)
    out = capsys.readouterr().out
    assert "the last 5 of the 6 launches of its first run; 11 in all" in out
    assert "median 1338.0 us" in out  # the last 5 of the step's 6 calls
    frac = alg / 1338e-6 / 8e12
    assert f"= {frac:.4f} of 8000 GB/s" in out
    bench.summarize_trace(str(p), 5, "ttmc_fused_kernel<0, 2, 2, 4", alg)
    assert "median 1600.0 us" in capsys.readouterr().out  # without it: the TTMc calls


def write_pmc(path, dispatches):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for d, name, counter, v in dispatches:
            w.writerow([d, name, counter, v])


@pytest.mark.parametrize("first_run,expect_kib", [(True, 4000.0), (False, 4200.0)])
def test_pmc_calibration_and_first_run(tmp_path, capsys, first_run, expect_kib):
    copy = "__amd_rocclr_copyBuffer"
    rows = [(1, copy, "FETCH_SIZE", 262144.0), (2, copy, "FETCH_SIZE", 262144.0)]  # 1 GiB read as 512 MiB
    rows += [(5, KERNEL, "FETCH_SIZE", 4000.0), (9, KERNEL, "FETCH_SIZE", 4000.0)]
    rows += [(400, KERNEL, "FETCH_SIZE", 4600.0), (402, KERNEL, "FETCH_SIZE", 4200.0)]
    rows += [(450, copy, "FETCH_SIZE", 99.0)]  # a later upload: not part of the calibration
    p = tmp_path / "pmc.csv"
    write_pmc(p, rows)
    bench.summarize_pmc(str(p), "ttmc_fused_kernel<0, 2, 2, 4", first_run=first_run)
    out = capsys.readouterr().out
    assert "scale 2.0000" in out
    line = [ln for ln in out.splitlines() if ln.startswith("ttmc_fused_kernel") and "KiB per dispatch" in ln][0]
    assert f"FETCH_SIZE {expect_kib:.1f} KiB per dispatch" in line
    assert line.endswith(f"= {expect_kib * 2.0 * 1024:.0f} bytes")
