"""The profiler-summary helpers that feed the benchmark line (CPU): per-dispatch counters, the HBM
traffic of a sweep launch scaled by a plain copy's readings, the replay window of a batched graph,
and that the committed counter summaries were taken on the sources the kernels are built from now
(the bench line reports their figures only then)."""
import csv
import json
import os

import pytest

from paper_1006_0252_amd import profile_summary as ps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def write_counters(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for did, name, counter, value in rows:
            w.writerow({"Dispatch_Id": did, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


SWEEP = "void pa::colour::k_sweep16c<0>(pa_state const*, pa::SweepParams, pa::words::Lane)"


def test_dispatch_counters_sum_rows_per_dispatch(tmp_path):
    d = str(tmp_path / "c")
    # a counter may come in several rows per dispatch (one per hardware block): they add up
    write_counters(d, [(7, SWEEP, "SQ_INSTS_VALU", 10), (7, SWEEP, "SQ_INSTS_VALU", 5), (7, SWEEP, "SQ_WAVES", 3),
                       (3, SWEEP, "SQ_INSTS_VALU", 2), (5, "pa::k_hist(pa_state*, int)", "SQ_INSTS_VALU", 99)])
    got = ps.dispatch_counters(d, "k_sweep16c")
    assert list(got) == [3, 7]  # dispatch order
    assert got[7] == {"SQ_INSTS_VALU": 15.0, "SQ_WAVES": 3.0} and got[3] == {"SQ_INSTS_VALU": 2.0}
    assert list(ps.dispatch_counters(d, "")) == [3, 5, 7]


def test_traffic_scales_by_the_copy_calibration(tmp_path):
    f, w, cf, cw = (str(tmp_path / n) for n in ("f", "w", "cf", "cw"))
    write_counters(f, [(1, SWEEP, "FETCH_SIZE", 1000), (2, SWEEP, "FETCH_SIZE", 3000)])
    write_counters(w, [(1, SWEEP, "WRITE_SIZE", 400), (2, SWEEP, "WRITE_SIZE", 600)])
    # the copy moves 1 GiB each way; its counters read 2 GiB fetched (scale 1/2) and 1 GiB written
    write_counters(cf, [(1, "small", "FETCH_SIZE", 10), (2, "copy", "FETCH_SIZE", 2 * (1 << 20))])
    write_counters(cw, [(1, "small", "WRITE_SIZE", 10), (2, "copy", "WRITE_SIZE", 1 << 20)])
    out = str(tmp_path / "t.json")
    ps.traffic(f, w, cf, cw, out)
    res = json.load(open(out))
    assert res["fetch_kib_per_dispatch"] == 2000 and res["write_kib_per_dispatch"] == 500
    assert res["dispatches"] == [2, 2]
    assert res["copy_calibration"]["fetch_scale"] == 0.5 and res["copy_calibration"]["write_scale"] == 1.0
    assert res["bytes_per_launch"] == 2000 * 1024 * 0.5 + 500 * 1024 * 1.0
    assert res["source_digest"] == ps.sweep_source_digest()


def test_replay_window_counts_kernels_between_first_and_last_sweep(tmp_path, capsys):
    d = tmp_path / "r"
    d.mkdir()
    rows = [("setup", 0, 50), ("k_sweep_a", 100, 200), ("k_gather", 210, 240), ("k_sweep_b", 250, 400),
            ("after", 500, 600)]
    with open(d / "run_kernel_trace.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for name, s, e in rows:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": s * 1000, "End_Timestamp": e * 1000})
    ps.replay(str(d), 2)
    text = capsys.readouterr().out
    assert "2 sweep dispatches" in text
    assert "kernel time 0.000 s" in text  # 100 + 30 + 150 us
    lines = [ln for ln in text.splitlines() if ln.startswith("| `")]
    assert [ln.split("`")[1] for ln in lines] == ["k_sweep_b", "k_sweep_a", "k_gather"]
    assert "| 0.150 |" in lines[0] and "| 0.030 |" in lines[2]


@pytest.mark.parametrize("name,sources", [("sweep_L16_R1e6_traffic.json", ps.SWEEP_SOURCES),
                                          ("sweep_L16_R1e6_counters.json", ps.SWEEP_SOURCES),
                                          ("batched_256runs_L6-10_counters.json", ps.STRING_SOURCES)])
def test_committed_counter_summaries_match_the_sources(name, sources):
    with open(os.path.join(ROOT, "profiles", name)) as f:
        res = json.load(f)
    assert res["source_digest"] == ps.sweep_source_digest(sources), (
        f"{name} was taken on other sources than the kernel's current ones; retake it")
