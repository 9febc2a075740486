"""Host-side pieces of bench.py (no GPU): the one-GPU guard and the kernel-trace
summary that the committed profiles are made with."""
import csv
import os
import subprocess
import sys

import pytest

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, REPO)

import bench  # noqa: E402

FIELDS = ["Kind", "Kernel_Name", "Start_Timestamp", "End_Timestamp"]


def _write_trace(path, launches):
    """launches: (name, duration_ns) in launch order, 1 us apart; names as
    rocprofv3 -T writes them (truncated: no namespace or arguments)."""
    t = 1_000_000
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for name, d in launches:
            w.writerow({"Kind": "KERNEL_DISPATCH", "Kernel_Name": name,
                        "Start_Timestamp": t, "End_Timestamp": t + d})
            t += d + 1000


def test_gpus_above_one_exit_with_message():
    r = subprocess.run([sys.executable, os.path.join(REPO, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=REPO, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_trace_summary_splits_calls_and_idle_launches(tmp_path, capsys):
    # call 0: three live sweeps (300 us) and two that return at once (10 us);
    # call 1: two live sweeps (600 us), one live and one idle panel update
    launches = [("k_init", 3000)]
    launches += [("k_sweep", 300_000), ("k_finalize", 7000)] * 3
    launches += [("k_sweep", 10_000), ("k_finalize", 4000)] * 2
    launches += [("k_panel_gemm", 800_000), ("k_colreduce", 30_000)]
    launches += [("k_init", 3000)]
    launches += [("k_sweep", 600_000), ("k_finalize", 7000)] * 2
    launches += [("k_panel_gemm", 1_500_000), ("k_panel_gemm", 15_000)]
    p = tmp_path / "run_kernel_trace.csv"
    _write_trace(str(p), launches)
    bench.summarize_trace(str(p))
    out = capsys.readouterr().out
    lines = out.splitlines()
    # whole-trace table: every k_sweep launch counted; live ones are those
    # above 0.3 of the longest (180 us here)
    sweep = next(ln for ln in lines if ln.startswith("k_sweep "))
    assert int(sweep.split()[1]) == 7
    assert "k_sweep live launches: 5 of 7" in out
    hdr = next(i for i, ln in enumerate(lines) if ln.lstrip().startswith("call"))
    c0 = lines[hdr + 1].split()
    c1 = lines[hdr + 2].split()
    # call, sweep_live, avg_us, idle, finalize_us, fold_us, gemm_live, avg_us, colred_us
    assert c0[:4] == ["0", "3", "300.0", "2"]
    assert float(c0[4]) == pytest.approx((3 * 7.0 + 2 * 4.0) / 5, abs=0.01)
    assert c0[6:8] == ["1", "800.0"]
    assert c1[:4] == ["1", "2", "600.0", "0"]
    assert c1[6:8] == ["1", "1500.0"]
