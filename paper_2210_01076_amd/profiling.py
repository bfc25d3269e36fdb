"""Summaries of rocprofv3 output for the pass kernel.

Reads a kernel-trace directory (``--kernel-trace --stats --output-format
csv``) and two counter directories (``--pmc FETCH_SIZE`` and ``--pmc
WRITE_SIZE``, one pass each) of the same benchmark command, and writes

* a short text summary: the kernel statistics, the average duration of the
  pass launches of the benchmark's timed steps (the last N launches of the
  kernel with the benchmark's workgroup size, N as the benchmark reports),
  and the HBM bytes per launch from the two counters, each scaled by what the
  same counter reads for the plain copy kernel of known size;
* a JSON record of the traffic figures, keyed to a hash of the kernel source
  so that a consumer can tell when the kernel changed after the counters
  were taken.

Usage::

    python -m paper_2210_01076_amd.profiling mfma --trace DIR --pmc DIR --kernel NAME --out-txt FILE
    python -m paper_2210_01076_amd.profiling issue --trace DIR --pmc DIR --kernel NAME [--block N] --out-txt FILE \\
        [--out-json FILE]
    python -m paper_2210_01076_amd.profiling --trace DIR --fetch DIR --write DIR \\
        --bench-json FILE --counter-bench-json FILE --out-txt FILE --out-json FILE \\
        --cmd-trace "..." --cmd-fetch "..." --cmd-write "..."
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "kernels.hip")


def kernel_source_hash() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _one(dirpath: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(dirpath, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError("no *%s under %s" % (suffix, dirpath))
    return hits[0]


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "").replace("qtask::", "")


def kernel_stats(trace_dir: str):
    rows = []
    with open(_one(trace_dir, "kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            rows.append((_short(r["Name"]), int(r["Calls"]), float(r["AverageNs"]), float(r["TotalDurationNs"]),
                         float(r["Percentage"])))
    rows.sort(key=lambda x: -x[3])
    return rows


def dispatches(trace_dir: str, kernel: str, block: int):
    """Durations (ns) of the kernel's dispatches with this workgroup size, in
    dispatch order."""
    rows = []
    with open(_one(trace_dir, "kernel_trace.csv")) as f:
        for r in csv.DictReader(f):
            if _short(r["Kernel_Name"]) == kernel and int(r["Workgroup_Size_X"]) == block:
                rows.append((int(r["Dispatch_Id"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    return [d for _, d in sorted(rows)]


def counters(counter_dir: str, name: str):
    """Counter values (KiB) per dispatch in dispatch order, by (kernel, workgroup)."""
    rows = defaultdict(list)
    with open(_one(counter_dir, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != name:
                continue
            key = (_short(r["Kernel_Name"]), int(r["Workgroup_Size"]))
            rows[key].append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
    return {k: [v for _, v in sorted(x)] for k, x in rows.items()}


def _mean(xs):
    return sum(xs) / len(xs) if xs else float("nan")


def _bench_line(path):
    with open(path) as f:
        return json.loads([ln for ln in f.read().splitlines() if ln.startswith("{")][-1])


def _tier(bench, tier):
    """Pass-launch figures of one tier of a benchmark line: the complex128
    tier's are its roofline record, the complex64 tier's its own record."""
    if tier == "c128":
        return bench["roofline"]
    r = bench["c64"]
    return {"bytes_per_launch": r["launch_bytes"], "launches_timed": r["launches"], "avg_launch_ms": r["launch_ms"],
            "block": 1 << (r["tile_bits"] - 4)}


def summarize(trace, fetch, write, bench_json, counter_bench_json, copy_bytes, command, kernel, copy_kernel,
              tier="c128"):
    bench = _bench_line(bench_json)
    cbench = _bench_line(counter_bench_json)
    counter_launches = _tier(cbench, tier)["launches_timed"]
    counter_alg = _tier(cbench, tier)["bytes_per_launch"]
    roof = _tier(bench, tier)
    block, n_timed = roof["block"], roof["launches_timed"]
    stats = kernel_stats(trace)
    durs = dispatches(trace, kernel, block)[-n_timed:]
    fc = counters(fetch, "FETCH_SIZE")
    wc = counters(write, "WRITE_SIZE")
    key = (kernel, block)
    ckey = [k for k in fc if k[0] == copy_kernel]
    copy_f = _mean([v for k in ckey for v in fc[k]])
    copy_w = _mean([v for k in ckey for v in wc.get(k, [])])
    f_scale = (copy_bytes / 1024.0) / copy_f
    w_scale = (copy_bytes / 1024.0) / copy_w
    # the counter runs use their own (shorter) benchmark command: their
    # timed launches are the last ones of the kernel as well
    n_cnt = counter_launches
    f_kib = _mean(fc.get(key, [])[-n_cnt:])
    w_kib = _mean(wc.get(key, [])[-n_cnt:])
    hbm = (f_kib * f_scale + w_kib * w_scale) * 1024.0
    rec = {
        "kernel": kernel,
        "workload": bench["config"]["workload"],
        "block": block,
        "dispatches_traced": len(durs),
        "avg_duration_us": _mean(durs) / 1e3,
        "bench_avg_launch_ms": roof["avg_launch_ms"],
        "algorithmic_bytes_per_launch": roof["bytes_per_launch"],
        "fetch_kib_per_launch": f_kib,
        "write_kib_per_launch": w_kib,
        "copy_fetch_kib": copy_f,
        "copy_write_kib": copy_w,
        "copy_bytes": copy_bytes,
        "fetch_scale": f_scale,
        "write_scale": w_scale,
        "hbm_bytes_per_launch": hbm,
        "counter_run_algorithmic_bytes_per_launch": counter_alg,
        "traffic_over_algorithmic": hbm / counter_alg,
        "kernel_source_hash": kernel_source_hash(),
        "command": command,
    }
    if tier != "c128":
        rec["workload"] = rec["workload"].replace("complex128", "complex64 tier")
    lines = ["# %s -- %s" % (kernel, rec["workload"]), ""]
    for k, v in command.items():
        lines.append("%s: %s" % (k, v))
    lines += ["", "kernel statistics (rocprofv3 --stats):", "%-44s %7s %12s %12s %6s" % (
        "kernel", "calls", "avg_us", "total_ms", "pct")]
    for name, calls, avg, tot, p in stats[:8]:
        lines.append("%-44s %7d %12.2f %12.2f %6.2f" % (name[:44], calls, avg / 1e3, tot / 1e6, p))
    lines += [
        "",
        "timed pass launches (%d threads per workgroup): %d dispatches, avg %.2f us "
        "(bench, HIP events: %.2f us)" % (block, len(durs), rec["avg_duration_us"], roof["avg_launch_ms"] * 1e3),
        "algorithmic bytes per launch: %.0f" % roof["bytes_per_launch"],
        "achieved (algorithmic / traced avg): %.1f GB/s" % (roof["bytes_per_launch"] / (rec["avg_duration_us"] * 1e3)),
        "",
        "FETCH_SIZE: %.1f KiB/launch; copy kernel %.1f KiB for %d bytes read -> scale %.4f" % (
            f_kib, copy_f, copy_bytes, f_scale),
        "WRITE_SIZE: %.1f KiB/launch; copy kernel %.1f KiB for %d bytes written -> scale %.4f" % (
            w_kib, copy_w, copy_bytes, w_scale),
        "HBM bytes per launch (scaled): %.0f = %.3f x the algorithmic %.0f of the counter runs" % (
            hbm, rec["traffic_over_algorithmic"], counter_alg),
        "kernel source hash: %s" % rec["kernel_source_hash"],
    ]
    return rec, "\n".join(lines) + "\n"


MFMA_PEAK_TFLOPS = {"F32": 157.3, "F64": 78.6}


def summarize_mfma(trace, pmc, kernel, command, last=0, cus=256, simds=4, xcds=8):
    """Matrix-core figures of one kernel: average duration from the trace,
    MFMA flops from SQ_INSTS_VALU_MFMA_MOPS_* (units of 512 flops), and the
    busy fraction SQ_VALU_MFMA_BUSY_CYCLES / (cycles x CUs x SIMDs), where the
    kernel's cycles are GRBM_GUI_ACTIVE / XCDs (the GRBM counter is summed
    over the eight XCDs)."""
    stats = kernel_stats(trace)
    rows = []
    with open(_one(trace, "kernel_trace.csv")) as f:
        for r in csv.DictReader(f):
            if _short(r["Kernel_Name"]) == kernel:
                rows.append((int(r["Dispatch_Id"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    durs = [d for _, d in sorted(rows)]
    per = defaultdict(list)
    with open(_one(pmc, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if _short(r["Kernel_Name"]) == kernel:
                per[r["Counter_Name"]].append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
    per = {k: [v for _, v in sorted(x)] for k, x in per.items()}
    if last:
        # only the measured run's dispatches: the last `last` of the kernel
        durs = durs[-last:]
        per = {k: v[-last:] for k, v in per.items()}
    avg = {k: _mean(v) for k, v in per.items()}
    prec = "F64" if "<double" in kernel else "F32"
    flops = avg.get("SQ_INSTS_VALU_MFMA_MOPS_" + prec, float("nan")) * 512.0
    dur_ns = _mean(durs)
    tflops = flops / dur_ns / 1e3
    cycles = avg.get("GRBM_GUI_ACTIVE", float("nan")) / xcds
    busy = avg.get("SQ_VALU_MFMA_BUSY_CYCLES", float("nan")) / (cycles * cus * simds)
    rec = {"kernel": kernel, "dispatches_traced": len(durs), "avg_duration_us": dur_ns / 1e3,
           "mfma_flops_per_dispatch": flops, "mfma_tflops": tflops, "peak_tflops": MFMA_PEAK_TFLOPS[prec],
           "frac_of_peak": tflops / MFMA_PEAK_TFLOPS[prec], "mfma_busy_frac": busy, "counters": avg,
           "command": command}
    lines = ["# %s -- matrix-core use" % kernel, ""]
    for k, v in command.items():
        lines.append("%s: %s" % (k, v))
    lines += ["", "kernel statistics (rocprofv3 --stats):", "%-44s %7s %12s %12s %6s" % (
        "kernel", "calls", "avg_us", "total_ms", "pct")]
    for name, calls, a, tot, p in stats[:8]:
        lines.append("%-44s %7d %12.2f %12.2f %6.2f" % (name[:44], calls, a / 1e3, tot / 1e6, p))
    lines += ["", "%s: %d dispatches used%s, avg %.2f us" % (
        kernel, len(durs), " (the last %d of the kernel: the measured run)" % last if last else "", dur_ns / 1e3),
              "counters per dispatch (averages):"]
    for k in sorted(avg):
        lines.append("  %-32s %.6g" % (k, avg[k]))
    lines += ["MFMA flops per dispatch (MOPS x 512): %.4g" % flops,
              "achieved: %.1f TFLOP/s = %.3f of the %.1f TFLOP/s dense %s matrix peak" % (
                  tflops, tflops / MFMA_PEAK_TFLOPS[prec], MFMA_PEAK_TFLOPS[prec], prec),
              "kernel cycles: GRBM_GUI_ACTIVE / %d XCDs = %.4g (%.2f GHz over the traced duration)" % (
                  xcds, cycles, cycles / dur_ns),
              "MFMA busy: SQ_VALU_MFMA_BUSY_CYCLES / (cycles x %d CUs x %d SIMDs) = %.3f" % (cus, simds, busy)]
    return rec, "\n".join(lines) + "\n"


def summarize_issue(trace, pmc, kernel, command, block=0, cus=256, simds=4, xcds=8):
    """Instruction mix and issue of one kernel from SQ counters: per-wave
    instruction counts (SQ_INSTS_* / SQ_WAVES), the share of SIMD time the
    VALU instructions occupy (a wave64 VALU instruction holds a 16-lane SIMD
    for 4 cycles: SQ_INSTS_VALU x 4 / (cycles x CUs x SIMDs), cycles =
    GRBM_GUI_ACTIVE / XCDs), and the wave-time ratios SQ_ACTIVE_INST_VALU /
    SQ_WAVE_CYCLES and SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES.  Averages over all
    dispatches of the kernel (with workgroup size `block` when given)."""
    stats = kernel_stats(trace)
    durs = []
    with open(_one(trace, "kernel_trace.csv")) as f:
        for r in csv.DictReader(f):
            if _short(r["Kernel_Name"]) == kernel and (not block or int(r["Workgroup_Size_X"]) == block):
                durs.append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    per = defaultdict(list)
    with open(_one(pmc, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if _short(r["Kernel_Name"]) == kernel and (not block or int(r["Workgroup_Size"]) == block):
                per[r["Counter_Name"]].append(float(r["Counter_Value"]))
    avg = {k: _mean(v) for k, v in per.items()}
    waves = avg.get("SQ_WAVES", float("nan"))
    cycles = avg.get("GRBM_GUI_ACTIVE", float("nan")) / xcds
    wave_cycles = avg.get("SQ_WAVE_CYCLES", float("nan"))
    valu_share = avg.get("SQ_INSTS_VALU", float("nan")) * 4.0 / (cycles * cus * simds)
    rec = {"kernel": kernel, "dispatches_traced": len(durs), "avg_duration_us": _mean(durs) / 1e3,
           "counters": avg, "per_wave": {k: v / waves for k, v in avg.items() if k.startswith("SQ_INSTS_")},
           "valu_issue_share": valu_share,
           "valu_bound_us": valu_share * _mean(durs) / 1e3,
           "kernel_source_hash": kernel_source_hash(),
           "active_valu_over_wave_cycles": avg.get("SQ_ACTIVE_INST_VALU", float("nan")) / wave_cycles,
           "wait_inst_any_over_wave_cycles": avg.get("SQ_WAIT_INST_ANY", float("nan")) / wave_cycles,
           "command": command}
    lines = ["# %s -- instruction mix and issue" % kernel, ""]
    for k, v in command.items():
        lines.append("%s: %s" % (k, v))
    lines += ["", "kernel statistics (rocprofv3 --stats):", "%-44s %7s %12s %12s %6s" % (
        "kernel", "calls", "avg_us", "total_ms", "pct")]
    for name, calls, a, tot, p in stats[:8]:
        lines.append("%-44s %7d %12.2f %12.2f %6.2f" % (name[:44], calls, a / 1e3, tot / 1e6, p))
    lines += ["", "%s%s: %d dispatches traced, avg %.2f us; %d with counters" % (
        kernel, " (%d threads per workgroup)" % block if block else "", len(durs), _mean(durs) / 1e3,
        len(next(iter(per.values()), []))), "counters per dispatch (averages):"]
    for k in sorted(avg):
        lines.append("  %-28s %.6g" % (k, avg[k]))
    lines.append("per wave:")
    for k, v in sorted(rec["per_wave"].items()):
        lines.append("  %-28s %.1f" % (k, v))
    lines += ["kernel cycles: GRBM_GUI_ACTIVE / %d XCDs = %.4g" % (xcds, cycles),
              "VALU issue share of SIMD time: SQ_INSTS_VALU x 4 / (cycles x %d CUs x %d SIMDs) = %.3f" % (
                  cus, simds, valu_share),
              "SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES = %.3f" % rec["active_valu_over_wave_cycles"],
              "SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES = %.3f" % rec["wait_inst_any_over_wave_cycles"],
              "time the VALU instructions alone take: %.2f of the %.2f us average launch" % (
                  rec["valu_bound_us"], rec["avg_duration_us"]),
              "kernel source hash: %s" % rec["kernel_source_hash"]]
    return rec, "\n".join(lines) + "\n"


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "issue":
        ap = argparse.ArgumentParser()
        ap.add_argument("mode")
        ap.add_argument("--trace", required=True)
        ap.add_argument("--pmc", required=True)
        ap.add_argument("--kernel", required=True)
        ap.add_argument("--block", type=int, default=0)
        ap.add_argument("--cmd-trace", default="")
        ap.add_argument("--cmd-pmc", default="")
        ap.add_argument("--out-txt", required=True)
        ap.add_argument("--out-json", default="")
        a = ap.parse_args()
        rec, txt = summarize_issue(a.trace, a.pmc, a.kernel, {"trace": a.cmd_trace, "pmc": a.cmd_pmc}, block=a.block)
        with open(a.out_txt, "w") as f:
            f.write(txt)
        if a.out_json:
            with open(a.out_json, "w") as f:
                json.dump(rec, f, indent=1)
        print(txt)
        return
    if len(sys.argv) > 1 and sys.argv[1] == "mfma":
        ap = argparse.ArgumentParser()
        ap.add_argument("mode")
        ap.add_argument("--trace", required=True)
        ap.add_argument("--pmc", required=True)
        ap.add_argument("--kernel", required=True)
        ap.add_argument("--last", type=int, default=0, help="use only the kernel's last N dispatches")
        ap.add_argument("--cmd-trace", default="")
        ap.add_argument("--cmd-pmc", default="")
        ap.add_argument("--out-txt", required=True)
        a = ap.parse_args()
        rec, txt = summarize_mfma(a.trace, a.pmc, a.kernel, {"trace": a.cmd_trace, "pmc": a.cmd_pmc}, last=a.last)
        with open(a.out_txt, "w") as f:
            f.write(txt)
        print(txt)
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--bench-json", required=True, help="output of the traced benchmark run")
    ap.add_argument("--counter-bench-json", required=True, help="output of the counter benchmark runs")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--kernel", default="qk_pass<double, false>")
    ap.add_argument("--tier", default="c128", choices=["c128", "c64"],
                    help="which tier of the benchmark line the pass launches belong to")
    ap.add_argument("--copy-kernel", default="qk_copy")
    ap.add_argument("--cmd-trace", default="")
    ap.add_argument("--cmd-fetch", default="")
    ap.add_argument("--cmd-write", default="")
    ap.add_argument("--out-txt", required=True)
    ap.add_argument("--out-json", required=True)
    a = ap.parse_args()
    command = {"trace": a.cmd_trace, "fetch": a.cmd_fetch, "write": a.cmd_write}
    rec, txt = summarize(a.trace, a.fetch, a.write, a.bench_json, a.counter_bench_json, a.copy_bytes, command,
                         a.kernel, a.copy_kernel, a.tier)
    with open(a.out_txt, "w") as f:
        f.write(txt)
    with open(a.out_json, "w") as f:
        json.dump(rec, f, indent=1)
    print(txt)


if __name__ == "__main__":
    main()
