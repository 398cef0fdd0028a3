"""The benchmark's measurement helpers, on synthetic rocprofv3 outputs (CPU).

Iteration passes queued past convergence exit at their first instruction;
the trace summary's working columns and the per-launch traffic must leave
them out, and the committed traffic figures must only be used for the
kernel sources they were taken from.
"""
import csv
import json

import bench

AC = "void wfa::k_march<double, true, 2, wfa::PhAC<double>, wfa::FinAC>(wfa::Geo, int)"
B2 = "void wfa::k_march<double, true, 2, wfa::PhB2<double>, wfa::FinB2>(wfa::Geo, int)"
COPY = "wfa::k_copy(unsigned long, unsigned int const*, unsigned int*)"


def _write(path, fields, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_trace_summary_working_columns(tmp_path):
    durs = {AC: [250.0] * 10 + [2.0] * 3, B2: [120.0] * 9 + [1.5] * 4}
    trace, t = [], 0
    for name, ds in durs.items():
        for d in ds:
            trace.append({"Kernel_Name": name, "Start_Timestamp": t, "End_Timestamp": t + int(d * 1000)})
            t += int(d * 1000) + 500
    _write(tmp_path / "run_kernel_trace.csv", ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], trace)
    stats = []
    for name, ds in durs.items():
        stats.append({"Name": name, "Calls": len(ds), "TotalDurationNs": sum(ds) * 1000,
                      "AverageNs": sum(ds) / len(ds) * 1000, "Percentage": 50.0})
    _write(tmp_path / "run_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs",
                                               "Percentage"], stats)
    md = bench.summarize_trace(str(tmp_path / "run_kernel_stats.csv"), "title", "cmd")
    rows = {line.split("`")[1]: line for line in md.splitlines() if line.startswith("| `")}
    ac = rows["k_march<double, true, 2, PhAC<double>, FinAC>"].split("|")
    b2 = rows["k_march<double, true, 2, PhB2<double>, FinB2>"].split("|")
    assert int(ac[2]) == 13 and int(ac[6]) == 10 and float(ac[7]) == 250.0
    assert int(b2[2]) == 13 and int(b2[6]) == 9 and float(b2[7]) == 120.0
    # all-call average still reported as the profiler gave it
    assert abs(float(ac[4]) - sum(durs[AC]) / 13) < 0.01


def test_counter_means_leave_out_skipped_dispatches(tmp_path):
    rows, did = [], 0
    # FETCH_SIZE arrives as one row per XCD-level block: the dispatch's value is their sum
    for value in [1000.0] * 5 + [0.5] * 3:
        did += 1
        for part in (0.25, 0.75):
            rows.append({"Counter_Name": "FETCH_SIZE", "Kernel_Name": AC, "Dispatch_Id": did,
                         "Counter_Value": value * part})
    did += 1
    rows.append({"Counter_Name": "FETCH_SIZE", "Kernel_Name": COPY, "Dispatch_Id": did,
                 "Counter_Value": 524288.0})
    rows.append({"Counter_Name": "WRITE_SIZE", "Kernel_Name": COPY, "Dispatch_Id": did,
                 "Counter_Value": 7.0})
    _write(tmp_path / "c.csv", ["Counter_Name", "Kernel_Name", "Dispatch_Id", "Counter_Value"], rows)
    means = bench.counter_means(str(tmp_path / "c.csv"), "FETCH_SIZE")
    assert means["phase_ac"] == (1000.0, 5)
    assert means["copy"] == (524288.0, 1)
    assert "phase_ac" not in bench.counter_means(str(tmp_path / "c.csv"), "WRITE_SIZE")


def test_traffic_figures_gated_by_source_hash(tmp_path, monkeypatch):
    path = tmp_path / "traffic.json"
    monkeypatch.setitem(bench.TRAFFIC_FILES, "headline", str(path))
    assert bench.load_traffic("phase_ac", "headline") is None          # no file
    body = {"kernels": {"phase_ac": {"hbm_bytes_per_launch": 123}}}
    path.write_text(json.dumps(dict(body, source_hash="0" * 16)))
    assert bench.load_traffic("phase_ac", "headline") is None          # other sources
    path.write_text(json.dumps(dict(body, source_hash=bench.kernel_source_hash())))
    assert bench.load_traffic("phase_ac", "headline") == 123
    assert bench.load_traffic("phase_b2", "headline") is None


def test_gpus_other_than_one_refused():
    import subprocess
    import sys
    res = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stdout


def test_gpu_busy_union_of_intervals():
    """Busy time is the union of the kernel intervals over the span from the
    first start to the last end (overlapping kernels of concurrent streams
    count once), and the gaps are those between merged intervals."""
    us = 1000
    spans = [(0, 10 * us), (5 * us, 12 * us),      # overlap: one interval 0..12
             (40 * us, 50 * us),                   # gap 28 us
             (55 * us, 60 * us), (58 * us, 59 * us)]  # gap 5 us; nested interval
    busy, gaps = bench.gpu_busy(spans)
    assert abs(busy - (12 + 10 + 5) / 60) < 1e-12
    assert gaps["over_20us"] == 1 and abs(gaps["over_20us_total_ms"] - 0.028) < 1e-12
    assert gaps["median_us"] in (5.0, 28.0)
    assert gaps["over_1ms"] == 0 and gaps["busy_without_over_1ms"] == busy
    assert bench.gpu_busy([(3, 9)])[0] == 1.0
    # a gap over 1 ms (nothing queued) is left out of the second figure
    ms = 1000 * us
    busy, gaps = bench.gpu_busy([(0, 1 * ms), (3 * ms, 4 * ms), (4 * ms + 10 * us, 5 * ms)])
    assert abs(busy - (3 * ms - 10 * us) / (5 * ms)) < 1e-12
    assert gaps["over_1ms"] == 1 and abs(gaps["over_1ms_total_ms"] - 2.0) < 1e-12
    assert abs(gaps["busy_without_over_1ms"] - (3 * ms - 10 * us) / (3 * ms)) < 1e-12


def test_pmc_summary_means_per_working_dispatch(tmp_path):
    """Counter means per kernel over working dispatches: a dispatch under a
    fifth of the kernel's 90th percentile (a pass skipped after the solve
    stopped) is left out, and every counter of every file gets a row."""
    rows = []
    for did, (name, v) in enumerate([(AC, 100.0)] * 5 + [(AC, 1.0)] + [(B2, 40.0)] * 4):
        for c, scale in (("SQ_INSTS_VALU", 1.0), ("SQ_WAVES", 0.5)):
            rows.append({"Dispatch_Id": did, "Kernel_Name": name, "Counter_Name": c,
                         "Counter_Value": v * scale})
    _write(tmp_path / "c.csv", ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], rows)
    md = bench.summarize_pmc([str(tmp_path / "c.csv")], "t", ["cmd"])
    lines = {l.split("|")[1].strip(): l for l in md.splitlines() if l.startswith("| SQ_")}
    assert set(lines) == {"SQ_INSTS_VALU", "SQ_WAVES"}
    cols = [c.strip() for c in md.splitlines()[[i for i, l in enumerate(md.splitlines())
                                                 if l.startswith("| counter")][0]].split("|")[2:-1]]
    valu = [c.strip() for c in lines["SQ_INSTS_VALU"].split("|")[2:-1]]
    assert dict(zip(cols, valu)) == {"phase_ac": "100", "phase_b2": "40"}
