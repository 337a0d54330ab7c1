"""Host logic of the benchmark script, without a GPU: the one-GPU guard, the
algorithmic byte count of the fused step kernels against a hand count, the
rule that a committed counter summary is used only while it was taken on the
current kernel sources, and the counter and trace summaries built from small
synthetic rocprofv3 CSV files."""
import csv
import json
import os
import shutil
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_cpu_workers_stay_within_the_host_share():
    w = bench.cpu_workers()
    assert 1 <= w <= 16
    assert w <= (os.cpu_count() or 1)


def test_fused_bytes_hand_count():
    # m = 2 rows, n = 3 columns, 4 nonzeros, B = 2 LPs, 8-byte values and iterates
    m, n, nnz, B = 2, 3, 4, 2
    # primal: A' (4 values + 4 indices, 4 row pointers of A'), gather Y once (m B),
    # read Xbar and X0, write Xbar (3 n B)
    primal = 4 * 8 + 4 * 4 + 4 * (n + 1) + 8 * B * m + 8 * 3 * n * B
    # dual: A (values, indices, 3 row pointers), gather Xbar once (n B), read Y and
    # Y0, write Y (3 m B)
    dual = 4 * 8 + 4 * 4 + 4 * (m + 1) + 8 * B * n + 8 * 3 * m * B
    assert bench.fused_bytes(0, m, n, nnz, B, 8, 8) == primal
    assert bench.fused_bytes(1, m, n, nnz, B, 8, 8) == dual
    # affine in the live column count (the benchmark's per-launch mean relies on it)
    b0, b1, b5 = (bench.fused_bytes(1, m, n, nnz, k, 8, 8) for k in (0, 1, 5))
    assert b5 - b0 == 5 * (b1 - b0)


@pytest.fixture()
def fake_root(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2601_21990_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("kernels.hip", "pdlpb_internal.h", "pdlpb.cpp"):
        shutil.copy(os.path.join(ROOT, "paper_2601_21990_amd", "csrc", f), csrc / f)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return tmp_path


def test_traffic_summary_is_used_only_on_the_same_sources(fake_root):
    sha = bench.kernel_source_sha()
    path = fake_root / "profiles" / "t.json"
    path.write_text(json.dumps({"kernel": "k_dual", "kernels_sha256": sha, "bytes_per_launch": 123}))
    assert bench.measured_traffic("t.json", "k_dual") == 123
    assert bench.measured_traffic("t.json", "k_primal") is None
    assert bench.measured_traffic("missing.json", "k_dual") is None
    with open(fake_root / "paper_2601_21990_amd" / "csrc" / "kernels.hip", "a") as fh:
        fh.write("\n// changed\n")
    assert bench.kernel_source_sha() != sha
    assert bench.measured_traffic("t.json", "k_dual") is None


def _write_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_pmc_summary_scales_and_selects_solves(fake_root, tmp_path):
    # dispatches: solve 1 = begin, dual (10 KiB); solve 2 = begin, dual (20), dual (40), primal
    seq = [("k_begin_solve", 0), ("k_dual", 10), ("k_begin_solve", 0), ("k_dual", 20),
           ("k_dual", 40), ("k_primal", 99)]
    for counter, scale in (("FETCH_SIZE", 1.0), ("WRITE_SIZE", 0.5)):
        d = tmp_path / counter
        d.mkdir()
        _write_csv(d / "x_counter_collection.csv",
                   [{"Dispatch_Id": i, "Kernel_Name": f"pdlpb::{k}(args)", "Counter_Name": counter,
                     "Counter_Value": v * scale} for i, (k, v) in enumerate(seq)])
    out = tmp_path / "s.json"
    args = SimpleNamespace(pmc_solves="2", pmc_fetch=str(tmp_path / "FETCH_SIZE"),
                           pmc_write=str(tmp_path / "WRITE_SIZE"), pmc_kernel="k_dual",
                           pmc_out=str(out), pmc_command="cmd")
    bench.run_pmc_summary(args)
    s = json.loads(out.read_text())
    assert s["dispatches"] == 2
    assert s["fetch_kib_per_dispatch"] == 30.0 and s["write_kib_per_dispatch"] == 15.0
    # HBM bytes = 2 x FETCH_SIZE + 1 x WRITE_SIZE (KiB) per dispatch
    assert s["bytes_per_launch"] == (2 * 30 + 15) * 1024
    assert s["kernels_sha256"] == bench.kernel_source_sha()


def test_trace_summary_averages_the_chosen_solves(tmp_path):
    # kernel names as rocprofv3 -T writes them (truncated; template arguments may remain)
    d = tmp_path / "trace"
    d.mkdir()
    seq = [("k_begin_solve", 0, 1000), ("k_dual", 1000, 6000), ("k_begin_solve", 7000, 8000),
           ("k_dual", 8000, 12000), ("k_dual", 13000, 19000), ("k_primal", 20000, 23000)]
    _write_csv(d / "x_kernel_trace.csv",
               [{"Dispatch_Id": i, "Kernel_Name": k if k != "k_primal" else "k_primal<double, 16, 1, 0>",
                 "Start_Timestamp": a, "End_Timestamp": b} for i, (k, a, b) in enumerate(seq)])
    _write_csv(d / "x_kernel_stats.csv",
               [{"Name": "k_dual", "Calls": 3, "TotalDurationNs": 15000, "AverageNs": 5000.0,
                 "Percentage": 75.0}])
    out = tmp_path / "t.md"
    args = SimpleNamespace(trace_dir=str(d), trace_solves="2", trace_out=str(out),
                           trace_title="T", trace_command="cmd", trace_top=4)
    bench.run_trace_summary(args)
    text = out.read_text()
    assert "| k_dual | 2 | 5.000 |" in text          # (4000 + 6000) ns / 2
    assert "| k_primal | 1 | 3.000 |" in text
    assert "| k_dual | 3 | 0.015 | 5.000 | 75.00 |" in text


def test_sweep_refuses_iteration_counts_that_leave_dead_launches():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "sweep",
                        "--sweep-iters", "33"], capture_output=True, text=True, timeout=300)
    assert r.returncode != 0 and "64 k + 1" in r.stderr
