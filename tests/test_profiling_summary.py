"""The rocprofv3 summary code on synthetic trace and counter files: the
average duration of the last timed launches, the copy-kernel scale factors
and the HBM bytes per launch, for both tiers of the benchmark line."""
import csv
import json

import pytest

from paper_2210_01076_amd import profiling


def _write_csv(path, header, rows):
    path.parent.mkdir(parents=True, exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def _fixture(tmp_path, kernel, block):
    # trace: 3 early launches (tuning) of 900 ns, then 4 timed ones of 100..400 ns
    durs = [900, 900, 900, 100, 200, 300, 400]
    trace_rows = [[i + 1, "void qtask::%s(void*)" % kernel, block, 1000 * i, 1000 * i + d]
                  for i, d in enumerate(durs)]
    trace_rows.append([100, "qtask::qk_copy(void*)", 256, 0, 50])
    _write_csv(tmp_path / "trace" / "run_kernel_trace.csv",
               ["Dispatch_Id", "Kernel_Name", "Workgroup_Size_X", "Start_Timestamp", "End_Timestamp"], trace_rows)
    _write_csv(tmp_path / "trace" / "run_kernel_stats.csv",
               ["Name", "Calls", "AverageNs", "TotalDurationNs", "Percentage"],
               [["void qtask::%s(void*)" % kernel, 7, 500, 3700, 99.0], ["qtask::qk_copy(void*)", 1, 50, 50, 1.0]])
    # counters: the copy kernel reads 2 KiB of FETCH_SIZE and writes 1 KiB of
    # WRITE_SIZE per KiB moved; the kernel's last 2 launches are the timed ones
    gib = 1 << 30
    for name, copy_kib, kib in (("FETCH_SIZE", gib / 1024 / 2, [7, 7, 10, 20]),
                                ("WRITE_SIZE", gib / 1024, [7, 7, 30, 40])):
        rows = [[i + 1, "void qtask::%s(void*)" % kernel, block, name, v] for i, v in enumerate(kib)]
        rows.append([100, "qtask::qk_copy(void*)", 256, name, copy_kib])
        d = "fetch" if name == "FETCH_SIZE" else "write"
        _write_csv(tmp_path / d / "run_counter_collection.csv",
                   ["Dispatch_Id", "Kernel_Name", "Workgroup_Size", "Counter_Name", "Counter_Value"], rows)


def _bench(path, launches, nbytes, ms, block_bits):
    line = {"config": {"workload": "synthetic layered circuit; complex128"},
            "roofline": {"bytes_per_launch": nbytes, "launches_timed": launches, "avg_launch_ms": ms,
                         "block": 1 << (block_bits - 4)},
            "c64": {"launch_bytes": nbytes, "launches": launches, "launch_ms": ms, "tile_bits": block_bits}}
    path.write_text("log line\n" + json.dumps(line) + "\n")


@pytest.mark.parametrize("tier,kernel", [("c128", "qk_pass<double, false>"), ("c64", "qk_pass<float, false>")])
def test_traffic_summary(tmp_path, tier, kernel):
    _fixture(tmp_path, kernel, 256)
    _bench(tmp_path / "b.json", 4, 1000.0, 0.00025, 12)       # traced run: 4 timed launches
    _bench(tmp_path / "c.json", 2, 1000.0, 0.00025, 12)       # counter runs: 2 timed launches
    rec, txt = profiling.summarize(str(tmp_path / "trace"), str(tmp_path / "fetch"), str(tmp_path / "write"),
                                   str(tmp_path / "b.json"), str(tmp_path / "c.json"), 1 << 30,
                                   {"trace": "t", "fetch": "f", "write": "w"}, kernel, "qk_copy", tier)
    assert rec["dispatches_traced"] == 4
    assert rec["avg_duration_us"] == pytest.approx(0.25)       # mean of 100..400 ns
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["fetch_kib_per_launch"] == pytest.approx(15.0) and rec["write_kib_per_launch"] == pytest.approx(35.0)
    assert rec["hbm_bytes_per_launch"] == pytest.approx((15.0 * 2 + 35.0) * 1024)
    assert rec["traffic_over_algorithmic"] == pytest.approx((15.0 * 2 + 35.0) * 1024 / 1000.0)
    assert rec["kernel_source_hash"] == profiling.kernel_source_hash()
    assert ("complex64 tier" in rec["workload"]) == (tier == "c64")
    assert "achieved (algorithmic / traced avg): 4.0 GB/s" in txt     # 1000 B / 0.25 us
