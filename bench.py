"""Benchmark: full simulation and incremental update of a 24-qubit layered
random circuit (200 levels of RX/RY/RZ on every qubit + a random CNOT
matching; 100 batches of 1-4 random gate inserts/removals at uniform levels).

A step = one modifier batch: apply the edits, run the incremental update
(timed), then a full re-simulation of the modified circuit (timed) whose
bytes must equal the incremental result.  ``value`` is the full simulation's
achieved HBM throughput (algorithmic bytes / wall time of the full
re-simulations).  The JSON line also carries the incremental p50/p99 latency
and speedup, the complex64 tier, the pass kernel's roofline, and these
legs (each can be switched off):
  * append protocol: the same circuit built net by net with an update after
    each, compared with full re-simulations at the same depth;
  * large state: the layered family at 28 qubits (4 GiB, far above the
    Infinity Cache) for an HBM-only figure;
  * serving: 256 sessions of 12-28 qubits with Poisson modify+update
    requests, both precisions;
  * cpu baseline: the CPU oracle on a bounded sample, all threads and one.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def pct(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * p / 100.0
    lo, hi = int(math.floor(k)), int(math.ceil(k))
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fidelity(a, b):
    """|<a|b>|^2 / (<a|a><b|b>) in FP64."""
    import numpy as np
    return float(abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real))


def run_tier(Q, W, wl, dtype, steps, warmup, shape=None):
    nets = [list(x) for x in wl.nets]
    if shape:  # a pinned tile shape (b, c) instead of the autotuner's pick
        sim = Q.Simulator(wl.n, dtype, device=0, ckpt_interval=wl.ckpt_levels, autotune=0,
                          tile_bits=shape[0], low_bits=shape[1])
    else:
        sim = Q.Simulator(wl.n, dtype, device=0, ckpt_interval=wl.ckpt_levels, autotune=1)
    sim.build(nets)
    t0 = time.perf_counter()
    st = sim.update()          # first update: autotune + full simulation
    tune_s = time.perf_counter() - t0
    first_full = st
    o = Q.qtask_get_opts(sim.h)
    log("%s tile shape b=%d c=%d (autotune + first full %.2f s)" % (dtype, o.tile_bits, o.low_bits, tune_s))
    for _ in range(warmup):
        sim.update(full=True)
    inc_ms, full_ms, speed, bound = [], [], [], []
    full_bytes = full_wall = 0.0
    pass_ms, passes = 0.0, 0
    # every pass launch of the timed region (incremental and full): the
    # roofline figure of the pass kernel
    all_bytes, all_kernel_ms, all_launches = 0.0, 0.0, 0
    mismatches = 0
    gate_amp = 0
    t0 = time.perf_counter()
    for step in range(steps):
        batch = wl.batches[step % len(wl.batches)]
        for e in batch:
            W.apply_edit(nets, e)
            sim.apply_edit(e)
        si = sim.update()
        h_inc = sim.hash()
        sf = sim.update(full=True)
        h_full = sim.hash()
        mismatches += int(h_inc != h_full)
        inc_ms.append(si["wall_ms"])
        full_ms.append(sf["wall_ms"])
        speed.append(sf["wall_ms"] / max(si["wall_ms"], 1e-9))
        bound.append(si["levels_total"] / max(si["levels_replayed"], 1))
        full_bytes += sf["bytes"]
        full_wall += sf["wall_ms"]
        for s_ in (si, sf):
            all_bytes += s_["bytes"]
            all_kernel_ms += s_["kernel_ms"]
            all_launches += s_["passes"]
        pass_ms += sf["kernel_ms"]
        passes += sf["passes"]
        gate_amp += sf["gate_amp_updates"]
        if step % 20 == 0:
            log("%s step %d inc %.2f ms full %.2f ms mode %d" % (dtype, step, si["wall_ms"], sf["wall_ms"], si["mode"]))
    t1 = time.perf_counter()
    out = {
        "dtype": dtype,
        "timed_s": t1 - t0,
        "full_gbs": full_bytes / (full_wall * 1e-3) / 1e9,
        "full_ms_p50": pct(full_ms, 50),
        "inc_ms_p50": pct(inc_ms, 50),
        "inc_ms_p99": pct(inc_ms, 99),
        "speedup_p50": pct(speed, 50),
        "speedup_bound_p50": pct(bound, 50),
        "updates_per_s": steps / sum(x * 1e-3 for x in inc_ms),
        "mismatches": mismatches,
        "passes_per_full": passes / max(steps, 1),
        "pass_avg_ms": pass_ms / max(passes, 1),
        "pass_bytes": full_bytes / max(passes, 1),
        "gate_amp_updates_per_s": gate_amp / (full_wall * 1e-3),
        "first_full_ms": first_full["wall_ms"],
        "tile_bits": o.tile_bits,
        "low_bits": o.low_bits,
        "launches": all_launches,
        "launch_bytes": all_bytes / max(all_launches, 1),
        "launch_ms": all_kernel_ms / max(all_launches, 1),
    }
    return sim, nets, out


def run_serving(Q, W, dtype, specs, keep_n=20, order=0):
    """Serve the sessions on one device: open all, run each one's initial
    simulation (warm-up, untimed), then replay the Poisson request stream at
    its arrival times and report request latency and throughput."""
    import threading

    dt = Q.QTASK_C128 if dtype == "c128" else Q.QTASK_C64
    sv = Q.qtask_server_create(Q.qtask_server_opts_default(order=order))
    try:
        t0 = time.perf_counter()
        sids = [Q.qtask_server_open(sv, s.n, dt, Q.qtask_opts_default(device=0), s.nets) for s in specs]
        open_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        warm = [Q.qtask_server_submit(sv, sid, []) for sid in sids]
        Q.qtask_server_drain(sv)
        warm_s = time.perf_counter() - t0
        bad = sum(Q.qtask_server_wait(sv, t, 0.0)["status"] != Q.QTASK_OK for t in warm)
        log("serving %s: opened %d sessions in %.1f s, initial simulations %.1f s" % (dtype, len(sids), open_s, warm_s))
        events = sorted((a, i, r) for i, s in enumerate(specs) for r, a in enumerate(s.arrivals))
        recs = {(i, r): [c for e in specs[i].requests[r] for c in Q.make_edits(e)] for _, i, r in events}
        tickets = []

        def feed():
            start = time.perf_counter()
            for a, i, r in events:
                d = a - (time.perf_counter() - start)
                if d > 0:
                    time.sleep(d)
                tickets.append(Q.qtask_server_submit(sv, sids[i], recs[(i, r)]))

        t0 = time.perf_counter()
        th = threading.Thread(target=feed)
        th.start()
        th.join()
        Q.qtask_server_drain(sv)
        wall = time.perf_counter() - t0
        res = [Q.qtask_server_wait(sv, t, 0.0) for t in tickets]
        bad += sum(r["status"] != Q.QTASK_OK for r in res)
        lat = [r["latency_ms"] for r in res]
        svc = [r["done_ms"] - r["start_ms"] for r in res]
        used, resident = Q.qtask_server_usage(sv)
        kept = {}
        for i, sid in enumerate(sids):
            if specs[i].n <= keep_n:
                h = Q.qtask_server_session(sv, sid)
                try:
                    kept[i] = Q.qtask_read_amplitudes(h, 0, 1 << specs[i].n, dt)
                except Q.QtaskError as e:
                    if e.code != Q.QTASK_E_STALE:  # evicted sessions hold no state
                        raise
        out = {
            "dtype": dtype,
            "sessions": len(sids),
            "requests": len(res),
            "failed": bad,
            "latency_ms_p50": pct(lat, 50),
            "latency_ms_p99": pct(lat, 99),
            "service_ms_p50": pct(svc, 50),
            "updates_per_s": len(res) / wall,
            "timed_s": wall,
            "initial_sim_s": warm_s,
            "device_bytes": used,
            "resident": resident,
        }
        return out, kept
    finally:
        Q.qtask_server_destroy(sv)


def run_serving_sweep(Q, W, dtype, rates, seed=4242):
    """Latency against offered load: one request (1-3 edits) per session,
    arriving as one Poisson stream of the given aggregate rate (requests/s)
    spread over the sessions in a random order."""
    import numpy as np

    base = W.serving_sessions(requests=1)
    curve = []
    for rate in rates:
        rng = np.random.default_rng(seed)
        times = np.cumsum(rng.exponential(1.0 / rate, size=len(base)))
        order = rng.permutation(len(base))
        for k, i in enumerate(order):
            base[i].arrivals = [float(times[k])]
        res, _ = run_serving(Q, W, dtype, base, keep_n=0)
        point = {"offered_per_s": rate, "served_per_s": res["updates_per_s"], "latency_ms_p50": res["latency_ms_p50"],
                 "latency_ms_p99": res["latency_ms_p99"], "service_ms_p50": res["service_ms_p50"],
                 "failed": res["failed"], "requests": res["requests"]}
        log("serving sweep %s offered %.0f/s: served %.1f/s, p50 %.0f ms, p99 %.0f ms" % (
            dtype, rate, point["served_per_s"], point["latency_ms_p50"], point["latency_ms_p99"]))
        curve.append(point)
    return curve


def run_append(Q, wl, dtype, tile_bits, low_bits, every=25, ckpt_nets=10):
    """The paper's append protocol: build the circuit net by net and update
    the state after each; every `every` nets also time a full
    re-simulation at the same depth and compare the two bitwise.  The
    session keeps a checkpoint every `ckpt_nets` nets (2.5 GiB at 24 qubits
    for the 400 nets), so an update replays at most that many nets."""
    s = Q.Simulator(wl.n, dtype, device=0, ckpt_interval=ckpt_nets, tile_bits=tile_bits, low_bits=low_bits)
    inc, pairs, mismatches = [], [], 0
    try:
        for i, net in enumerate(wl.nets):
            s.add_level(i)
            for g in net:
                s.add_gate(i, g)
            st = s.update()
            inc.append(st["wall_ms"])
            if (i + 1) % every == 0:
                h = s.hash()
                sf = s.update(full=True)
                mismatches += int(s.hash() != h)
                pairs.append(sf["wall_ms"] / max(st["wall_ms"], 1e-9))
    finally:
        s.close()
    return {"dtype": dtype, "nets": len(wl.nets), "ckpt_nets": ckpt_nets,
            "update_ms_p50": pct(inc, 50), "update_ms_p99": pct(inc, 99),
            "speedup_p50": pct(pairs, 50), "speedup_min": min(pairs), "speedup_at_full_depth": pairs[-1],
            "mismatches": mismatches, "compared_depths": len(pairs)}


def run_small(Q, W, repeats=20):
    """The 10-qubit dense random circuit (20 levels, 10 single-gate
    modifiers): the whole state (16 KiB) is one tile, so this is launch
    latency, not bandwidth.  Wall time of each call (host planning, launches
    and the wait), per modifier for the incremental update and for a full
    re-simulation of the same circuit, compared by hash."""
    wl = W.config(1)
    nets = [list(x) for x in wl.nets]
    first, inc, full, mismatches = [], [], [], 0
    for _ in range(repeats):
        s = Q.Simulator(wl.n, "c128", device=0, ckpt_interval=5)
        try:
            s.build(nets)
            first.append(s.update()["wall_ms"])
        finally:
            s.close()
    s = Q.Simulator(wl.n, "c128", device=0, ckpt_interval=5)
    work = [list(x) for x in nets]
    try:
        s.build(work)
        s.update()
        for _ in range(repeats // 2):
            for batch in wl.batches:
                for e in batch:
                    W.apply_edit(work, e)
                    s.apply_edit(e)
                inc.append(s.update()["wall_ms"])
                h = s.hash()
                full.append(s.update(full=True)["wall_ms"])
                mismatches += int(s.hash() != h)
            # undo: replaying the same batches again needs the original circuit
            s.close()
            s = Q.Simulator(wl.n, "c128", device=0, ckpt_interval=5)
            work = [list(x) for x in nets]
            s.build(work)
            s.update()
    finally:
        s.close()
    return {"workload": "dense random circuit, 10 qubits, 20 levels, 10 single-gate modifiers; complex128",
            "first_update_us_p50": 1e3 * pct(first, 50),
            "update_us_p50": 1e3 * pct(inc, 50), "update_us_p99": 1e3 * pct(inc, 99),
            "full_us_p50": 1e3 * pct(full, 50), "updates": len(inc), "mismatches": mismatches}


def run_protocols(Q, wl, dtype, tile_bits, low_bits, every=25, ckpt_nets=10, mixes=50, seed=77):
    """The paper's other incremental protocols on the same circuit (Section
    IV): insert the nets one at a time in random order until the circuit is
    complete, remove them one at a time in random order until it is empty,
    and a mix of random net inserts and removals.  The state is updated after
    every step; every `every` steps a full re-simulation is timed beside the
    update and the two are compared bitwise."""
    import numpy as np

    rng = np.random.default_rng(seed)
    out = {}

    def measure(name, steps):
        s = Q.Simulator(wl.n, dtype, device=0, ckpt_interval=ckpt_nets, tile_bits=tile_bits, low_bits=low_bits)
        inc, pairs, mismatches = [], [], 0
        try:
            for i, step in enumerate(steps(s)):
                st = s.update()
                inc.append(st["wall_ms"])
                if (i + 1) % every == 0:
                    h = s.hash()
                    sf = s.update(full=True)
                    mismatches += int(s.hash() != h)
                    pairs.append(sf["wall_ms"] / max(st["wall_ms"], 1e-9))
        finally:
            s.close()
        out[name] = {"steps": len(inc), "update_ms_p50": pct(inc, 50), "update_ms_p99": pct(inc, 99),
                     "speedup_p50": pct(pairs, 50) if pairs else None, "mismatches": mismatches,
                     "compared": len(pairs)}

    nets = wl.nets

    def insert_random(s):
        # nets enter in random order, each at its place among those present
        order = rng.permutation(len(nets))
        present = []
        for k in order:
            pos = int(np.searchsorted(present, k))
            present.insert(pos, int(k))
            s.add_level(pos)
            for g in nets[k]:
                s.add_gate(pos, g)
            yield k

    def remove_random(s):
        s.build(nets)
        s.update()
        left = len(nets)
        while left > 0:
            s.remove_level(int(rng.integers(left)))
            left -= 1
            yield left

    def mix(s):
        s.build(nets)
        s.update()
        pool = list(range(len(nets)))
        for _ in range(mixes):
            if rng.integers(2) == 0 and len(s.levels) > 1:
                s.remove_level(int(rng.integers(len(s.levels))))
            else:
                pos = int(rng.integers(len(s.levels) + 1))
                k = pool[int(rng.integers(len(pool)))]
                s.add_level(pos)
                for g in nets[k]:
                    s.add_gate(pos, g)
            yield len(s.levels)

    measure("insert_random_order", insert_random)
    measure("remove_until_empty", remove_random)
    measure("mixed_%d" % mixes, mix)
    out["dtype"] = dtype
    out["ckpt_nets"] = ckpt_nets
    return out


def run_large(Q, W, n=28, levels=100, dtype="c128"):
    """Full simulations of the layered family at a state far larger than the
    256 MB Infinity Cache: HBM-only throughput of the pass kernel."""
    wl = W.config(2, n=n, levels=levels, batches=1)
    s = Q.Simulator(n, dtype, device=0, ckpt_interval=wl.ckpt_levels, autotune=1)
    try:
        s.build(wl.nets)
        s.update()
        best = None
        for _ in range(3):
            st = s.update(full=True)
            if best is None or st["kernel_ms"] < best["kernel_ms"]:
                best = st
        o = Q.qtask_get_opts(s.h)
    finally:
        s.close()
    gbs = best["bytes"] / (best["kernel_ms"] * 1e-3) / 1e9
    return {"qubits": n, "levels": levels, "dtype": dtype, "state_gib": (1 << n) * (16 if dtype == "c128" else 8) / 2**30,
            "full_ms": best["kernel_ms"], "passes": best["passes"], "gbs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS,
            "tile_bits": o.tile_bits, "low_bits": o.low_bits}


def run_ladder32(Q, W, levels=60, edits=6, tile_bits=12, low_bits=3, ckpt_nets=45):
    """Configuration 5 at reduced depth: 32 qubits in complex128 (a 64 GiB
    state plus two 64 GiB checkpoints), rotations and controlled-phase
    ladders, then single-gate inserts alternating between gates inside one
    tile (all qubits below b) and gates with a qubit at or above b.  Each
    update is timed, then a full re-simulation of the same circuit, and the
    two states are compared by hash."""
    n = 32
    wl = W.config(5, levels=levels, batches=1)
    nets = [list(x) for x in wl.nets]
    batches = W.split_edits(n, nets, 5005, edits, tile_bits)
    s = Q.Simulator(n, "c128", device=0, ckpt_interval=ckpt_nets, max_ckpts=2, tile_bits=tile_bits,
                    low_bits=low_bits)
    try:
        s.build(nets)
        st = s.update()
        full0 = st
        rows = []
        for i, batch in enumerate(batches):
            for e in batch:
                W.apply_edit(nets, e)
                s.apply_edit(e)
            st = s.update()
            h = s.hash()
            sf = s.update(full=True)
            rows.append({"high": i % 2 == 1, "gate": batch[0].gate[0], "qubits": list(batch[0].gate[1]),
                         "mode": st["mode"], "first_level": st["first_level"], "inc_ms": st["kernel_ms"],
                         "full_ms": sf["kernel_ms"], "equal": h == s.hash()})
            log("ladder-32 edit %d (%s on %s): mode %d from net %d, %.0f ms vs full %.0f ms" % (
                i, batch[0].gate[0], batch[0].gate[1], st["mode"], st["first_level"], st["kernel_ms"], sf["kernel_ms"]))
    finally:
        s.close()
    gbs = full0["bytes"] / (full0["kernel_ms"] * 1e-3) / 1e9
    sp = [r["full_ms"] / r["inc_ms"] for r in rows]
    return {"qubits": n, "levels": levels, "nets": len(wl.nets), "dtype": "c128", "state_gib": 64,
            "tile_bits": tile_bits, "low_bits": low_bits, "ckpt_nets": ckpt_nets,
            "full_ms": full0["kernel_ms"], "passes": full0["passes"], "gbs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS,
            "edits": rows, "speedup_p50": pct(sp, 50), "mismatches": sum(not r["equal"] for r in rows)}


MFMA_PEAK_TFLOPS = {"c64": 157.3, "c128": 78.6}   # dense FP32 / FP64 matrix-core peaks


def run_fused(Q, W, n=30, levels=300, k=5, tile_bits=11, low_bits=4, sample=1 << 20, tuned=True):
    """Configuration 3: the layered family at 30 qubits with every stage fused
    into a dense k-qubit unitary on the matrix cores, complex64 (renormalised
    at every 50-level segment end) against complex128, both fused; then the
    same circuit in complex64 with the autotuner choosing the tile shape and
    whether to fuse (and how wide) for comparison."""
    import numpy as np

    wl = W.config(3, n=n, levels=levels)
    common = dict(device=0, ckpt_interval=50, max_ckpts=1)
    out = {"qubits": n, "levels": levels, "fuse_width": k, "tile_bits": tile_bits, "low_bits": low_bits}
    sims = {}
    try:
        for dt in ("c64", "c128"):
            s = Q.Simulator(n, dt, tile_bits=tile_bits, low_bits=low_bits, fusion=Q.QTASK_FUSE_DENSE,
                            fuse_width=k, **common)
            sims[dt] = s
            s.build(wl.nets)
            st = s.update()
            tflops = st["mfma_flops"] / (st["kernel_ms"] * 1e-3) / 1e12
            out[dt] = {"full_ms": st["kernel_ms"], "passes": st["passes"],
                       "gbs": st["bytes"] / (st["kernel_ms"] * 1e-3) / 1e9,
                       "mfma_flops": st["mfma_flops"], "mfma_tflops": tflops,
                       "frac_of_mfma_peak": tflops / MFMA_PEAK_TFLOPS[dt]}
        a, b = sims["c128"], sims["c64"]
        inner = Q.qtask_inner(a.h, b.h)
        out["fidelity_c64_vs_c128"] = abs(inner) ** 2 / (Q.qtask_norm(a.h) * Q.qtask_norm(b.h))
        # max-abs over a sample: the first amplitudes, and 4096 spread over the rest
        err = 0.0
        for lo in range(0, sample, 1 << 16):
            err = max(err, float(np.max(np.abs(a.state(lo, 1 << 16) - b.state(lo, 1 << 16).astype(np.complex128)))))
        for i in np.linspace(sample, (1 << n) - 1, 4096).astype(np.int64):
            err = max(err, float(abs(a.state(int(i), 1)[0] - complex(b.state(int(i), 1)[0]))))
        out["max_abs_c64_vs_c128_sampled"] = err
        out["sample"] = "first %d amplitudes and 4096 spread over the rest" % sample
    finally:
        for s in sims.values():
            s.close()
    if not tuned:
        return out
    s = Q.Simulator(n, "c64", autotune=1, **common)
    try:
        s.build(wl.nets)
        st = s.update()
        o = Q.qtask_get_opts(s.h)
        out["autotuned_c64"] = {"full_ms": st["kernel_ms"], "passes": st["passes"],
                                "gbs": st["bytes"] / (st["kernel_ms"] * 1e-3) / 1e9,
                                "tile_bits": o.tile_bits, "low_bits": o.low_bits,
                                "fusion": {0: "auto", 1: "none", 2: "dense"}[o.fusion], "fuse_width": o.fuse_width}
    finally:
        s.close()
    return out


def cpu_baseline(W, wl, full_bytes_per_gate, min_s=10.0, max_nets=150):
    """Time the CPU oracle (all host threads) on the first nets of the same
    circuit, adding nets until about min_s seconds of work."""
    from oracle import oracle

    threads = oracle.max_threads()
    psi = oracle.basis(wl.n)
    gates = 0
    used = 0
    t0 = time.perf_counter()
    for net in wl.nets[:max_nets]:
        oracle.apply_gates(wl.n, psi, list(net), threads)
        gates += len(net)
        used += 1
        if time.perf_counter() - t0 >= min_s:
            break
    dt = time.perf_counter() - t0
    # the same oracle on one thread, over the first nets (about 3 s)
    psi1 = oracle.basis(wl.n)
    g1 = 0
    t1 = time.perf_counter()
    for net in wl.nets[:max_nets]:
        oracle.apply_gates(wl.n, psi1, list(net), 1)
        g1 += len(net)
        if time.perf_counter() - t1 >= min_s / 3:
            break
    dt1 = time.perf_counter() - t1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": full_bytes_per_gate * gates / dt / 1e9,
        "unit": "GB/s",
        "cores": threads,
        "cpu_model": model,
        "host_cpus": os.cpu_count(),
        "kind": "oracle",
        "sample": "first %d nets (%d gates) of the %d-qubit circuit, complex128, %.1f s on %d threads; value = the "
                  "GPU plan's bytes for the same gates / oracle time" % (used, gates, wl.n, dt, threads),
        "gate_amp_updates_per_s": gates * (1 << wl.n) / dt,
        "full_sim_s_extrapolated": dt * W.count_gates(wl.nets) / gates,
        "value_1_thread": full_bytes_per_gate * g1 / dt1 / 1e9,
        "gate_amp_updates_per_s_1_thread": g1 * (1 << wl.n) / dt1,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-c64", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-append", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-fused", action="store_true")
    ap.add_argument("--ladder32", action="store_true",
                    help="only the 32-qubit controlled-phase ladder with single-gate edits (about a minute)")
    ap.add_argument("--serving-sweep", action="store_true",
                    help="only the serving latency-throughput sweep (several minutes), printed as one JSON line")
    ap.add_argument("--fused-qubits", type=int, default=30, help="state size of the fused-unitary leg")
    ap.add_argument("--fused-levels", type=int, default=300, help="depth of the fused-unitary leg")
    ap.add_argument("--no-fused-tuned", action="store_true",
                    help="skip the autotuned comparison run of the fused-unitary leg (its timing candidates "
                         "would mix into a profile of the fused kernels)")
    ap.add_argument("--tile-bits", type=int, default=0,
                    help="pin the complex128 tier's tile bits instead of autotuning (profiling runs: counter "
                         "collection slows kernels and would sway the tuner's timings)")
    ap.add_argument("--low-bits", type=int, default=3, help="contiguous low bits with --tile-bits")
    ap.add_argument("--c64-tile-bits", type=int, default=0, help="the same for the complex64 tier")
    ap.add_argument("--c64-low-bits", type=int, default=4, help="contiguous low bits with --c64-tile-bits")
    ap.add_argument("--traffic-c64", default=os.path.join(ROOT, "profiles", "traffic_layered_n24_c64.json"))
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic_layered_n24.json"))
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the state and the serving sessions are not sharded across GPUs "
              "(the design notes describe how they would be)", file=sys.stderr)
        sys.exit(2)

    from paper_2210_01076_amd import qtask as Q
    from paper_2210_01076_amd import workloads as W

    if args.ladder32:
        print(json.dumps({"metric": "32-qubit full simulation GB/s; single-gate update vs full re-simulation",
                          "ladder32": run_ladder32(Q, W)}))
        return

    if args.serving_sweep:
        sweep = {"metric": "serving request latency against offered load", "unit": "ms",
                 "workload": "256 sessions, qubits log-uniform in [12,28], depth U{50..400} layered levels, "
                             "one request of 1-3 edits each, Poisson arrivals at the offered rate",
                 "c64": run_serving_sweep(Q, W, "c64", [8, 16, 32, 48]),
                 "c128": run_serving_sweep(Q, W, "c128", [8, 16, 24])}
        print(json.dumps(sweep))
        return

    copy_gbs = Q.qtask_copy_bandwidth(0, 1 << 30, 20)
    log("copy kernel ceiling %.1f GB/s" % copy_gbs)
    wl = W.config(2)
    shape = (args.tile_bits, args.low_bits) if args.tile_bits else None
    sim128, nets, r128 = run_tier(Q, W, wl, "c128", args.steps, args.warmup, shape)
    r64 = None
    if not args.no_c64:
        shape64 = (args.c64_tile_bits, args.c64_low_bits) if args.c64_tile_bits else None
        sim64, _, r64 = run_tier(Q, W, wl, "c64", args.steps, args.warmup, shape64)
        import numpy as np
        a = sim128.state()
        b = sim64.state().astype(np.complex128)
        r64["max_abs_vs_c128"] = float(np.max(np.abs(a - b)))
        r64["fidelity_vs_c128"] = fidelity(a, b)
        sim64.close()
    sim128.close()

    # before the serving leg: autotuner picks are cached per (qubits, dtype,
    # gate mix), and the serving sessions tune while other sessions run, so
    # a 28-qubit pick made there would be timed under contention
    small = run_small(Q, W)
    log("10-qubit circuit: update p50 %.0f us p99 %.0f us, full re-simulation p50 %.0f us, mismatches %d" % (
        small["update_us_p50"], small["update_us_p99"], small["full_us_p50"], small["mismatches"]))

    large = None
    if not args.no_large:
        large = run_large(Q, W)
        log("28-qubit complex128 full simulation: %.1f ms, %.0f GB/s (%.2f of peak)" % (
            large["full_ms"], large["gbs"], large["frac_of_peak"]))

    serving = None
    if not args.no_serving:
        import numpy as np
        specs = W.serving_sessions()
        s128, kept128 = run_serving(Q, W, "c128", specs)
        s64, kept64 = run_serving(Q, W, "c64", specs)
        errs = [float(np.max(np.abs(kept128[i] - kept64[i].astype(np.complex128)))) for i in kept128 if i in kept64]
        s64["max_abs_vs_c128"] = max(errs) if errs else None
        s64["compared_sessions"] = len(errs)
        # the same streams with the expected-shortest request started first
        sf = {}
        for dt in ("c128", "c64"):
            r, _ = run_serving(Q, W, dt, specs, keep_n=0, order=1)
            sf[dt] = {k: r[k] for k in ("latency_ms_p50", "latency_ms_p99", "service_ms_p50", "updates_per_s",
                                        "failed")}
        serving = {"workload": "256 sessions, qubits log-uniform in [12,28], depth U{50..400} layered levels, "
                               "Poisson requests of 1-3 edits (4 per session); sessions under 16 qubits batched",
                   "order": "oldest request first",
                   "c128": s128, "c64": s64,
                   "shortest_first": sf}
        log("serving, expected-shortest first: c128 p50 %.1f ms p99 %.1f ms | c64 p50 %.1f ms p99 %.1f ms" % (
            sf["c128"]["latency_ms_p50"], sf["c128"]["latency_ms_p99"],
            sf["c64"]["latency_ms_p50"], sf["c64"]["latency_ms_p99"]))
        log("serving c128 p50 %.1f ms p99 %.1f ms %.1f upd/s | c64 p50 %.1f ms p99 %.1f ms %.1f upd/s" % (
            s128["latency_ms_p50"], s128["latency_ms_p99"], s128["updates_per_s"],
            s64["latency_ms_p50"], s64["latency_ms_p99"], s64["updates_per_s"]))

    append = None
    if not args.no_append:
        append = run_append(Q, wl, "c128", r128["tile_bits"], r128["low_bits"])
        log("append protocol: update p50 %.2f ms, speedup vs full p50 %.1f (at full depth %.1f)" % (
            append["update_ms_p50"], append["speedup_p50"], append["speedup_at_full_depth"]))
    protocols = None
    if not args.no_append:
        protocols = run_protocols(Q, wl, "c128", r128["tile_bits"], r128["low_bits"])
        for k in ("insert_random_order", "remove_until_empty", "mixed_50"):
            p = protocols[k]
            log("%s: %d steps, update p50 %.2f ms p99 %.2f ms, speedup vs full p50 %s, mismatches %d" % (
                k, p["steps"], p["update_ms_p50"], p["update_ms_p99"],
                "%.1f" % p["speedup_p50"] if p["speedup_p50"] else "-", p["mismatches"]))
    fused = None
    if not args.no_fused:
        fused = run_fused(Q, W, n=args.fused_qubits, levels=args.fused_levels, tuned=not args.no_fused_tuned)
        log("%d-qubit fused k=5: complex64 %.0f ms (%.1f TFLOP/s on the matrix cores), complex128 %.0f ms "
            "(%.1f TFLOP/s); fidelity %.12f, sampled max-abs %.2e" % (
                fused["qubits"], fused["c64"]["full_ms"], fused["c64"]["mfma_tflops"], fused["c128"]["full_ms"],
                fused["c128"]["mfma_tflops"], fused["fidelity_c64_vs_c128"], fused["max_abs_c64_vs_c128_sampled"]))
        if "autotuned_c64" in fused:
            log("autotuned complex64 on the same circuit: %.0f ms (fusion %s)" % (
                fused["autotuned_c64"]["full_ms"], fused["autotuned_c64"]["fusion"]))

    per_gate = r128["pass_bytes"] * r128["passes_per_full"] / W.count_gates(nets)
    cpu = None if args.no_cpu else cpu_baseline(W, wl, per_gate)

    # HBM bytes per launch from the committed counter summary, dropped once
    # the kernel source no longer matches the one the counters were taken on
    def load_traffic(path):
        if not os.path.exists(path):
            return None
        from paper_2210_01076_amd import profiling
        with open(path) as f:
            rec = json.load(f)
        if rec.get("kernel_source_hash") != profiling.kernel_source_hash():
            return None
        return rec.get("hbm_bytes_per_launch")

    traffic = load_traffic(args.traffic)
    if r64 is not None:
        # the complex64 pass kernel's HBM bytes per launch, from its own summary
        r64["traffic"] = load_traffic(args.traffic_c64)
    achieved = r128["launch_bytes"] / (r128["launch_ms"] * 1e-3) / 1e9
    line = {
        "metric": "full-sim HBM GB/s vs peak; incremental update p50/p99 latency and speedup vs full re-sim",
        "value": round(r128["full_gbs"], 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r128["timed_s"] * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "layered random circuit, 24 qubits, 200 levels (RX/RY/RZ on every qubit + random "
                               "CNOT matching), 100 batches of 1-4 random gate inserts/removals; complex128",
                   "qubits": 24, "levels": 200, "batches": 100, "ckpt_levels": wl.ckpt_levels,
                   "tile_bits": r128["tile_bits"], "low_bits": r128["low_bits"]},
        "frac_of_peak": round(r128["full_gbs"] / HBM_PEAK_GBS, 4),
        "copy_ceiling_gbs": round(copy_gbs, 1),
        "frac_of_copy_ceiling": round(r128["full_gbs"] / copy_gbs, 4),
        "full_ms_p50": r128["full_ms_p50"],
        "incremental_ms_p50": r128["inc_ms_p50"],
        "incremental_ms_p99": r128["inc_ms_p99"],
        "incremental_speedup_p50": r128["speedup_p50"],
        "replay_bound_speedup_p50": r128["speedup_bound_p50"],
        "incremental_mismatches": r128["mismatches"],
        "updates_per_s": {"c128": r128["updates_per_s"], "c64": r64["updates_per_s"] if r64 else None},
        "gate_amp_updates_per_s": r128["gate_amp_updates_per_s"],
        "passes_per_full_sim": r128["passes_per_full"],
        "c64": r64,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "qk_pass<double, false>", "bytes_per_launch": r128["launch_bytes"],
                     "avg_launch_ms": r128["launch_ms"], "launches_timed": r128["launches"],
                     "block": 1 << (r128["tile_bits"] - 4),
                     "scope": "every pass launch of the timed steps (incremental and full), complex128",
                     "note": "cache-assisted: the 24-qubit complex128 state (256 MiB) is about the size of the "
                             "256 MB Infinity Cache; large_state is the HBM-only figure (28 qubits, 4 GiB)"},
        "append_protocol": append,
        "other_protocols": protocols,
        "small_circuit": small,
        "large_state": large,
        "fused_dense": fused,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
