"""Summaries of rocprofv3 output for the pass kernel.

Reads a kernel-trace directory (``--kernel-trace --stats --output-format
csv``) and two counter directories (``--pmc FETCH_SIZE`` and ``--pmc
WRITE_SIZE``, one pass each) of the same benchmark command, and writes

* a short text summary: the kernel statistics, the average duration of the
  full-simulation pass launches (selected by their grid and workgroup size),
  and the HBM bytes per launch from the two counters, each scaled by what the
  same counter reads for the plain copy kernel of known size;
* a JSON record of the traffic figures, keyed to a hash of the kernel source
  so that a consumer can tell when the kernel changed after the counters
  were taken.

Usage::

    python -m paper_2210_01076_amd.profiling --trace DIR --fetch DIR --write DIR \\
        --bench-json FILE --copy-bytes N --out-txt FILE --out-json FILE --command "..."
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
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


def dispatches(trace_dir: str, kernel: str):
    """Durations (ns) of the kernel's dispatches, grouped by (grid, workgroup)."""
    out = defaultdict(list)
    with open(_one(trace_dir, "kernel_trace.csv")) as f:
        for r in csv.DictReader(f):
            if _short(r["Kernel_Name"]) != kernel:
                continue
            key = (int(r["Grid_Size_X"]), int(r["Workgroup_Size_X"]))
            out[key].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return out


def counters(counter_dir: str, name: str):
    """Counter values (KiB) per dispatch, grouped by (kernel, grid, workgroup)."""
    out = defaultdict(list)
    with open(_one(counter_dir, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != name:
                continue
            key = (_short(r["Kernel_Name"]), int(r["Grid_Size"]), int(r["Workgroup_Size"]))
            out[key].append(float(r["Counter_Value"]))
    return out


def _mean(xs):
    return sum(xs) / len(xs) if xs else float("nan")


def summarize(trace, fetch, write, bench_json, copy_bytes, command, kernel, copy_kernel):
    with open(bench_json) as f:
        bench = json.loads([ln for ln in f.read().splitlines() if ln.startswith("{")][-1])
    roof = bench["roofline"]
    launch = roof["launch"]          # {"grid": workgroups, "block": threads}
    grid_threads = launch["grid"] * launch["block"]
    stats = kernel_stats(trace)
    d = dispatches(trace, kernel)
    durs = d.get((grid_threads, launch["block"]), [])
    fc = counters(fetch, "FETCH_SIZE")
    wc = counters(write, "WRITE_SIZE")
    key = (kernel, grid_threads, launch["block"])
    ckey = [k for k in fc if k[0] == copy_kernel]
    copy_f = _mean([v for k in ckey for v in fc[k]])
    copy_w = _mean([v for k in ckey for v in wc.get(k, [])])
    f_scale = (copy_bytes / 1024.0) / copy_f
    w_scale = (copy_bytes / 1024.0) / copy_w
    f_kib = _mean(fc.get(key, []))
    w_kib = _mean(wc.get(key, []))
    hbm = (f_kib * f_scale + w_kib * w_scale) * 1024.0
    rec = {
        "kernel": kernel,
        "workload": bench["config"]["workload"],
        "launch": launch,
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
        "traffic_over_algorithmic": hbm / roof["bytes_per_launch"],
        "kernel_source_hash": kernel_source_hash(),
        "command": command,
    }
    lines = ["# %s -- %s" % (kernel, rec["workload"]), ""]
    for k, v in command.items():
        lines.append("%s: %s" % (k, v))
    lines += ["", "kernel statistics (rocprofv3 --stats):", "%-44s %7s %12s %12s %6s" % (
        "kernel", "calls", "avg_us", "total_ms", "pct")]
    for name, calls, avg, tot, p in stats[:8]:
        lines.append("%-44s %7d %12.2f %12.2f %6.2f" % (name[:44], calls, avg / 1e3, tot / 1e6, p))
    lines += [
        "",
        "full-simulation pass launches (%d workgroups x %d threads): %d dispatches, avg %.2f us "
        "(bench, HIP events: %.2f us)" % (launch["grid"], launch["block"], len(durs), rec["avg_duration_us"],
                                         roof["avg_launch_ms"] * 1e3),
        "algorithmic bytes per launch: %.0f" % roof["bytes_per_launch"],
        "achieved (algorithmic / traced avg): %.1f GB/s" % (roof["bytes_per_launch"] / (rec["avg_duration_us"] * 1e3)),
        "",
        "FETCH_SIZE: %.1f KiB/launch; copy kernel %.1f KiB for %d bytes read -> scale %.4f" % (
            f_kib, copy_f, copy_bytes, f_scale),
        "WRITE_SIZE: %.1f KiB/launch; copy kernel %.1f KiB for %d bytes written -> scale %.4f" % (
            w_kib, copy_w, copy_bytes, w_scale),
        "HBM bytes per launch (scaled): %.0f = %.3f x algorithmic" % (hbm, rec["traffic_over_algorithmic"]),
        "kernel source hash: %s" % rec["kernel_source_hash"],
    ]
    return rec, "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--bench-json", required=True)
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--kernel", default="qk_pass_pf<double>")
    ap.add_argument("--copy-kernel", default="qk_copy")
    ap.add_argument("--cmd-trace", default="")
    ap.add_argument("--cmd-fetch", default="")
    ap.add_argument("--cmd-write", default="")
    ap.add_argument("--out-txt", required=True)
    ap.add_argument("--out-json", required=True)
    a = ap.parse_args()
    command = {"trace": a.cmd_trace, "fetch": a.cmd_fetch, "write": a.cmd_write}
    rec, txt = summarize(a.trace, a.fetch, a.write, a.bench_json, a.copy_bytes, command, a.kernel, a.copy_kernel)
    with open(a.out_txt, "w") as f:
        f.write(txt)
    with open(a.out_json, "w") as f:
        json.dump(rec, f, indent=1)
    print(txt)


if __name__ == "__main__":
    main()
