"""The rocprofv3 summary code on synthetic trace and counter files: the
average duration of the last timed launches, the copy-kernel scale factors
and the HBM bytes per launch, for both tiers of the benchmark line; the
matrix-core rate and busy fraction; the instruction-mix ratios."""
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


def _counter_fixture(tmp_path, kernel, durs, counters):
    """Trace of `durs` (ns) launches of `kernel` and one counter file with
    counters[name] = per-launch values."""
    _write_csv(tmp_path / "trace" / "run_kernel_trace.csv",
               ["Dispatch_Id", "Kernel_Name", "Workgroup_Size_X", "Start_Timestamp", "End_Timestamp"],
               [[i + 1, "void qtask::%s(void*)" % kernel, 256, 1000 * i, 1000 * i + d] for i, d in enumerate(durs)])
    _write_csv(tmp_path / "trace" / "run_kernel_stats.csv",
               ["Name", "Calls", "AverageNs", "TotalDurationNs", "Percentage"],
               [["void qtask::%s(void*)" % kernel, len(durs), sum(durs) / len(durs), sum(durs), 100.0]])
    rows = [[i + 1, "void qtask::%s(void*)" % kernel, 256, name, v]
            for name, vals in counters.items() for i, v in enumerate(vals)]
    _write_csv(tmp_path / "pmc" / "run_counter_collection.csv",
               ["Dispatch_Id", "Kernel_Name", "Workgroup_Size", "Counter_Name", "Counter_Value"], rows)


def test_mfma_summary_uses_the_last_dispatches(tmp_path):
    kernel = "qk_pass<double, true>"
    # two runs of two launches; the measured run is the last two: 1000 ns each,
    # 2e6 MOPS (x 512 flops) and 8e6 busy cycles over 8e3 GRBM cycles (8 XCDs)
    _counter_fixture(tmp_path, kernel, [5000, 5000, 1000, 1000],
                     {"SQ_INSTS_VALU_MFMA_MOPS_F64": [1, 1, 2e6, 2e6], "SQ_INSTS_VALU_MFMA_MOPS_F32": [0] * 4,
                      "SQ_VALU_MFMA_BUSY_CYCLES": [1, 1, 8e6, 8e6], "GRBM_GUI_ACTIVE": [8, 8, 8e3, 8e3]})
    rec, txt = profiling.summarize_mfma(str(tmp_path / "trace"), str(tmp_path / "pmc"), kernel,
                                        {"trace": "t", "pmc": "p"}, last=2)
    assert rec["dispatches_traced"] == 2 and rec["avg_duration_us"] == pytest.approx(1.0)
    assert rec["mfma_flops_per_dispatch"] == pytest.approx(2e6 * 512)
    assert rec["mfma_tflops"] == pytest.approx(2e6 * 512 / 1000 / 1e3)   # flops / ns / 1e3
    assert rec["frac_of_peak"] == pytest.approx(rec["mfma_tflops"] / 78.6)
    assert rec["mfma_busy_frac"] == pytest.approx(8e6 / (1e3 * 256 * 4))
    assert "dense F64 matrix peak" in txt


def test_issue_summary_ratios(tmp_path):
    kernel = "qk_pass<double, false>"
    # 4 waves per launch; 400 VALU and 200 SALU instructions; 1024 GRBM
    # cycles per XCD; wave cycles 1000, of which 250 waiting
    _counter_fixture(tmp_path, kernel, [2000, 2000],
                     {"SQ_WAVES": [4, 4], "SQ_INSTS_VALU": [400, 400], "SQ_INSTS_SALU": [200, 200],
                      "SQ_ACTIVE_INST_VALU": [400, 400], "SQ_WAVE_CYCLES": [1000, 1000],
                      "SQ_WAIT_INST_ANY": [250, 250], "GRBM_GUI_ACTIVE": [8 * 1024, 8 * 1024]})
    rec, txt = profiling.summarize_issue(str(tmp_path / "trace"), str(tmp_path / "pmc"), kernel,
                                         {"trace": "t", "pmc": "p"}, block=256)
    assert rec["dispatches_traced"] == 2 and rec["avg_duration_us"] == pytest.approx(2.0)
    assert rec["per_wave"]["SQ_INSTS_VALU"] == pytest.approx(100) and rec["per_wave"]["SQ_INSTS_SALU"] == 50
    assert rec["valu_issue_share"] == pytest.approx(400 * 4 / (1024 * 256 * 4))
    assert rec["wait_inst_any_over_wave_cycles"] == pytest.approx(0.25)
    assert rec["valu_bound_us"] == pytest.approx(rec["valu_issue_share"] * 2.0)
    assert rec["kernel_source_hash"] == profiling.kernel_source_hash()
    assert "VALU issue share of SIMD time" in txt
