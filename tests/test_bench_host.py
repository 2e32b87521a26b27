"""Host logic of bench.py (no GPU): the one-GPU guard, the profile summarizer
on a synthetic rocprofv3 trace, and the lookup of committed HBM traffic."""
import csv
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stdout


def _write_csv(path, fields, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        w.writerows(rows)


def test_summarizer_splits_kernel_variants(tmp_path):
    """Dispatches after the last initialisation kernel form the timed run, one
    line per kernel variant, with the mean of end - start."""
    fields = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    rows, t = [], 0

    def add(name, ns):
        nonlocal t
        rows.append({"Kernel_Name": name, "Start_Timestamp": t, "End_Timestamp": t + ns})
        t += ns + 10

    add("void qew::k_step_fused<0, 8, false>(...)", 5_000_000)  # warm-up, before the last init
    add("void qew::k_init_split<0>(...)", 1000)
    for ns in (1_000_000, 3_000_000):
        add("void qew::k_step_fused<0, 8, false>(...)", ns)
    for ns in (4_000_000, 4_000_000, 7_000_000):
        add("void qew::k_step_fused<0, 8, true>(...)", ns)
    add("void qew::k_meas_split<0>(...)", 500)
    _write_csv(tmp_path / "run_kernel_trace.csv", fields, rows)
    text = bench.summarize_profile(str(tmp_path))
    assert "timed run: `qew::k_step_fused<0, 8, false>` 2 launches, average 2.00000 ms" in text
    assert "timed run: `qew::k_step_fused<0, 8, true>` 3 launches, average 5.00000 ms" in text
    assert "timed run: `qew::k_meas_split<0>` 1 launches" in text


def test_summarizer_counters_per_variant(tmp_path):
    fields = ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp", "Counter_Name",
              "Counter_Value"]
    rows = []
    for d, (name, v) in enumerate([("qew::k_init_split<0>()", 0.0),
                                   ("qew::k_step_fused<0, 8, false>()", 10.0),
                                   ("qew::k_step_fused<0, 8, false>()", 30.0),
                                   ("qew::k_step_fused<0, 8, true>()", 7.0)]):
        for part in (0.25, 0.75):  # per-XCD records of one dispatch are summed
            rows.append({"Dispatch_Id": d, "Kernel_Name": name, "Start_Timestamp": 100 * d,
                         "End_Timestamp": 100 * d + 50, "Counter_Name": "FETCH_SIZE",
                         "Counter_Value": v * part})
    _write_csv(tmp_path / "run_counter_collection.csv", fields, rows)
    text = bench.summarize_profile(str(tmp_path))
    assert "| `qew::k_step_fused<0, 8, false>` | FETCH_SIZE | 2 | 20 | 40 |" in text
    assert "| `qew::k_step_fused<0, 8, true>` | FETCH_SIZE | 1 | 7 | 7 |" in text


def test_traffic_lookup_needs_the_measured_kernel_code(monkeypatch, tmp_path):
    summary = tmp_path / "traffic.md"
    summary.write_text("traffic_per_launch fused k=56 tile=2048 source=00aa bytes=123\n"
                       "traffic_per_launch plain source=00cc bytes=45\n")
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(summary))
    hashes = {bench.FUSED_SYMBOLS: "00aa", bench.PLAIN_SYMBOLS: "00cc"}
    monkeypatch.setattr(bench, "kernel_source_hash", lambda pattern=bench.FUSED_SYMBOLS: hashes[pattern])
    assert bench.committed_traffic(56, 2048) == 123
    assert bench.committed_traffic(48, 2048) is None
    assert bench.committed_traffic(plain=True) == 45
    hashes[bench.FUSED_SYMBOLS] = "00bb"  # the fused kernel changed since
    assert bench.committed_traffic(56, 2048) is None
    assert bench.committed_traffic(plain=True) == 45
    hashes[bench.PLAIN_SYMBOLS] = "00dd"  # and the plain one
    assert bench.committed_traffic(plain=True) is None


def test_benchmark_problem_is_the_whole_workload():
    """The timed run is the 10^6-step workload with its 200 log-spaced
    measurements; a cut keeps the measurements inside it; the FP64 plain
    window has the run's measurement density (200 per 10^6 steps)."""
    p = bench.bench_problem(bench.HORIZON)
    assert p["n_steps"] == 10**6 and len(p["meas_steps"]) == 200
    assert p["meas_steps"][0] == 1 and p["meas_steps"][-1] == 10**6
    assert list(p["L"]) == [1 << 22] * 4 and p["kind"] == 0 and p["f"][0] == 1.0
    cut = bench.bench_problem(1000)
    assert cut["n_steps"] == 1000 and np.all(cut["meas_steps"] <= 1000)
    assert np.array_equal(cut["meas_steps"], p["meas_steps"][p["meas_steps"] <= 1000])
    w = bench.window_problem(20_000)
    assert w["n_steps"] == 20_000 and len(w["meas_steps"]) == 4 and w["meas_steps"][-1] == 20_000


def test_error_metric_floors():
    """v and ubar errors are relative to max(|x|, floor); w2 where positive."""
    assert bench._rel([1.0 + 1e-9], [1.0], 1e-3) == pytest.approx(1e-9)
    assert bench._rel([2e-6], [1e-6], 1e-3) == pytest.approx(1e-3)
    assert bench._rel([], [], 1e-3) == 0.0
