"""Benchmark, headline: configuration 5 -- a 32-qubit complex128 state
(64 GiB) under a 500-level controlled-phase ladder circuit (RX/RY/RZ on every
qubit, then CP on even and on odd adjacent pairs), with checkpoints every 50
levels (three stored, as many as fit beside the state in 288 GB).

A step = one single-gate insert at a uniformly random level (alternately a
gate inside one tile and a gate across tiles) and its incremental update.
``value`` is the HBM throughput of the timed steps (algorithmic bytes of
their pass launches / wall time of the steps); ``roofline`` is the pass
kernel's bytes per launch over its average launch time.  After the timed
steps a full re-simulation checks the result bitwise, and two more edits are
each compared with their own full re-simulation (speedup p50 against the
replay bound of uniform edits).

Also in the line (each can be switched off): the 10-qubit launch-latency
circuit, the 24-qubit layered configuration in complex128 and complex64
(cache-assisted), the serving curve (256 sessions, two Poisson loads and a
saturating burst, both precisions) and the CPU oracle on a bounded sample of
the headline workload with its max-abs against the device.  ``--extras``
runs the 28-qubit state, the paper's other incremental protocols and the
30-qubit fused-unitary configuration instead.
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
        sim = Q.Simulator(wl.n, dtype, device=0, ckpt_interval=wl.ckpt_nets, autotune=0,
                          tile_bits=shape[0], low_bits=shape[1])
    else:
        sim = Q.Simulator(wl.n, dtype, device=0, ckpt_interval=wl.ckpt_nets, autotune=1)
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
        paths = Q.qtask_server_paths(sv)
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
            "batched_requests": paths["batched"],
            "stream_requests": paths["streamed"],
        }
        return out, kept
    finally:
        Q.qtask_server_destroy(sv)


def run_serving_curve(Q, W, dtype, rates, per_phase=128, keep_n=20, seed=4242):
    """Latency against offered load on one server: the 256 sessions are
    opened and simulated once (untimed), then each phase submits requests of
    1-3 edits as one Poisson stream at the offered rate (requests/s) over
    `per_phase` sessions in random order, and a last phase submits one
    request to every session at once (the saturation point).  Each phase is
    drained before the next; a request's latency is submit to done."""
    import threading

    import numpy as np

    dt = Q.QTASK_C128 if dtype == "c128" else Q.QTASK_C64
    specs = W.serving_sessions(requests=len(rates) + 1)
    budget = Q.qtask_server_opts_default().budget_bytes
    sv = Q.qtask_server_create(Q.qtask_server_opts_default())
    rng = np.random.default_rng(seed)
    try:
        t0 = time.perf_counter()
        sids = [Q.qtask_server_open(sv, sp.n, dt, Q.qtask_opts_default(device=0), sp.nets) for sp in specs]
        warm = [Q.qtask_server_submit(sv, sid, []) for sid in sids]
        Q.qtask_server_drain(sv)
        bad = sum(Q.qtask_server_wait(sv, t, 0.0)["status"] != Q.QTASK_OK for t in warm)
        log("serving %s: 256 sessions opened and simulated in %.1f s" % (dtype, time.perf_counter() - t0))
        nreq = [0] * len(specs)  # requests used per session
        curve = []
        for ph, rate in enumerate(list(rates) + [None]):
            if rate is None:
                order = list(range(len(specs)))
                times = [0.0] * len(order)
            else:
                order = [int(i) for i in rng.permutation(len(specs))[:per_phase]]
                times = list(np.cumsum(rng.exponential(1.0 / rate, size=len(order))))
            recs = []
            for i in order:
                recs.append([c for e in specs[i].requests[nreq[i]] for c in Q.make_edits(e)])
                nreq[i] += 1
            tickets = []

            def feed():
                start = time.perf_counter()
                for k, i in enumerate(order):
                    d = times[k] - (time.perf_counter() - start)
                    if d > 0:
                        time.sleep(d)
                    tickets.append(Q.qtask_server_submit(sv, sids[i], recs[k]))

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
            point = {"offered_per_s": rate if rate is not None else "all at once", "requests": len(res),
                     "served_per_s": len(res) / wall, "latency_ms_p50": pct(lat, 50),
                     "latency_ms_p99": pct(lat, 99), "service_ms_p50": pct(svc, 50)}
            log("serving %s offered %s: served %.1f/s, p50 %.0f ms, p99 %.0f ms" % (
                dtype, point["offered_per_s"], point["served_per_s"], point["latency_ms_p50"],
                point["latency_ms_p99"]))
            curve.append(point)
        used, resident = Q.qtask_server_usage(sv)
        peak = Q.qtask_server_peak_bytes(sv)
        paths = Q.qtask_server_paths(sv)
        kept = {}
        for i, sid in enumerate(sids):
            if specs[i].n <= keep_n:
                h = Q.qtask_server_session(sv, sid)
                try:
                    kept[i] = Q.qtask_read_amplitudes(h, 0, 1 << specs[i].n, dt)
                except Q.QtaskError as e:
                    if e.code != Q.QTASK_E_STALE:  # evicted sessions hold no state
                        raise
        sat = curve[-1]
        return {"dtype": dtype, "sessions": len(sids), "failed": bad, "curve": curve,
                "updates_per_s": sat["served_per_s"], "latency_ms_p50": sat["latency_ms_p50"],
                "latency_ms_p99": sat["latency_ms_p99"], "budget_bytes": budget, "peak_bytes": peak,
                "device_bytes": used, "resident": resident, "batched_requests": paths["batched"],
                "stream_requests": paths["streamed"], "batched_ticks": paths["ticks"]}, kept
    finally:
        Q.qtask_server_destroy(sv)


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
    and the wait).  Two sessions receive the same modifiers: one runs the
    incremental update, the other a full re-simulation of the modified
    circuit (which plans the edited segment too, as any simulation of the
    new circuit must); their states are compared by hash.  The same
    session's full re-simulation right after its update, which finds the
    edited segment's plan already made, is reported beside it."""
    wl = W.config(1)
    nets = [list(x) for x in wl.nets]
    first, inc, full, full_cached, plan, modes, mismatches = [], [], [], [], [], [], 0
    for _ in range(repeats):
        s = Q.Simulator(wl.n, "c128", device=0, ckpt_interval=5)
        try:
            s.build(nets)
            first.append(s.update()["wall_ms"])
        finally:
            s.close()
    for _ in range(repeats // 2):
        a = Q.Simulator(wl.n, "c128", device=0, ckpt_interval=5)
        b = Q.Simulator(wl.n, "c128", device=0, ckpt_interval=5)
        try:
            wa = [list(x) for x in nets]
            wb = [list(x) for x in nets]
            a.build(wa)
            b.build(wb)
            a.update()
            b.update()
            for batch in wl.batches:
                for e in batch:
                    W.apply_edit(wa, e)
                    a.apply_edit(e)
                    W.apply_edit(wb, e)
                    b.apply_edit(e)
                st = a.update()
                inc.append(st["wall_ms"])
                plan.append(st["plan_ms"])
                modes.append(st["mode"])
                full.append(b.update(full=True)["wall_ms"])
                h = a.hash()
                mismatches += int(b.hash() != h)
                full_cached.append(a.update(full=True)["wall_ms"])
                mismatches += int(a.hash() != h)
        finally:
            a.close()
            b.close()
    return {"workload": "dense random circuit, 10 qubits, 20 levels, 10 single-gate modifiers; complex128",
            "first_update_us_p50": 1e3 * pct(first, 50),
            "update_us_p50": 1e3 * pct(inc, 50), "update_us_p99": 1e3 * pct(inc, 99),
            "full_us_p50": 1e3 * pct(full, 50), "full_us_p99": 1e3 * pct(full, 99),
            "full_plans_cached_us_p50": 1e3 * pct(full_cached, 50),
            "update_plan_us_p50": 1e3 * pct(plan, 50),
            "update_modes": {str(m): modes.count(m) for m in sorted(set(modes))},
            "updates": len(inc), "mismatches": mismatches}


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
    s = Q.Simulator(n, dtype, device=0, ckpt_interval=wl.ckpt_nets, autotune=1)
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


HEADLINE = dict(n=32, levels=500, ckpt_nets=150, max_ckpts=3, tile_bits=12, low_bits=4)


def run_headline(Q, W, steps, warmup, tile_bits=None, low_bits=None, levels=None, verify_edits=1):
    """Configuration 5, the headline: 32 qubits in complex128 (a 64 GiB state
    and three 64 GiB checkpoints: of the segment boundaries every 50 levels,
    every third one is stored, at levels 150, 300 and 450 of 500), 500
    levels of RX/RY/RZ on every qubit plus controlled-phase ladders on even
    and odd adjacent pairs.

    After the first (full) simulation, `warmup` untimed steps insert a gate
    in the circuit's last segment; then `steps` timed steps each insert one
    gate at a uniformly random net, alternating between gates whose qubits
    all lie below the tile bits (inside one tile) and gates with a qubit at
    or above them, and run the incremental update.  A full re-simulation
    then checks the result bitwise (state hash), and `verify_edits` more
    edits (one inside a tile, one across) are each timed as an update and
    compared with their own full re-simulation."""
    n = HEADLINE["n"]
    levels = levels or HEADLINE["levels"]
    b = tile_bits or HEADLINE["tile_bits"]
    c = low_bits or HEADLINE["low_bits"]
    K = HEADLINE["ckpt_nets"]
    wl = W.config(5, levels=levels, batches=1)
    nets = [list(x) for x in wl.nets]
    sim = Q.Simulator(n, "c128", device=0, ckpt_interval=K, max_ckpts=HEADLINE["max_ckpts"], tile_bits=b,
                      low_bits=c, relabel=1, autotune=0)
    rows = []
    try:
        sim.build(nets)
        t0 = time.perf_counter()
        first = sim.update()
        log("headline: 32-qubit ladder, %d levels (%d nets): first full simulation %.0f ms (%d passes, "
            "plan %.0f ms, wall %.1f s)" % (levels, len(nets), first["kernel_ms"], first["passes"], first["plan_ms"],
                                           time.perf_counter() - t0))
        for i, batch in enumerate(W.split_edits(n, nets, 5004, warmup, b, tail=K)):
            for e in batch:
                W.apply_edit(nets, e)
                sim.apply_edit(e)
            st = sim.update()
            log("headline warm-up %d: %.0f ms from net %d" % (i, st["wall_ms"], st["first_level"]))
        timed = W.split_edits(n, nets, 5005, steps, b)
        t0 = time.perf_counter()
        for i, batch in enumerate(timed):
            for e in batch:
                W.apply_edit(nets, e)
                sim.apply_edit(e)
            st = sim.update()
            rows.append({"high": i % 2 == 1, "gate": batch[0].gate[0], "qubits": list(batch[0].gate[1]),
                         "mode": st["mode"], "first_level": st["first_level"], "wall_ms": st["wall_ms"],
                         "kernel_ms": st["kernel_ms"], "plan_ms": st["plan_ms"], "bytes": st["bytes"],
                         "passes": st["passes"], "levels_replayed": st["levels_replayed"],
                         "levels_total": st["levels_total"], "gate_amp_updates": st["gate_amp_updates"]})
            log("headline step %d (%s on %s): mode %d from net %d, %.0f ms, %d passes" % (
                i, batch[0].gate[0], batch[0].gate[1], st["mode"], st["first_level"], st["wall_ms"], st["passes"]))
        timed_s = time.perf_counter() - t0
        # the timed steps' result against a full re-simulation, bitwise
        h_inc = sim.hash()
        full = sim.update(full=True)
        mismatches = int(sim.hash() != h_inc)
        fulls = [full]
        verify = []
        for i, batch in enumerate(W.split_edits(n, nets, 5006, verify_edits, b)):
            for e in batch:
                W.apply_edit(nets, e)
                sim.apply_edit(e)
            si = sim.update()
            h = sim.hash()
            sf = sim.update(full=True)
            fulls.append(sf)
            eq = h == sim.hash()
            mismatches += int(not eq)
            verify.append({"high": i % 2 == 1, "gate": batch[0].gate[0], "qubits": list(batch[0].gate[1]),
                           "mode": si["mode"], "first_level": si["first_level"], "inc_ms": si["wall_ms"],
                           "full_ms": sf["wall_ms"], "speedup": sf["wall_ms"] / si["wall_ms"], "equal": eq})
            log("headline check %d (%s on %s): update %.0f ms from net %d, full %.0f ms, equal %s" % (
                i, batch[0].gate[0], batch[0].gate[1], si["wall_ms"], si["first_level"], sf["wall_ms"], eq))
        o = Q.qtask_get_opts(sim.h)
    finally:
        sim.close()
    full_ms = pct([f["wall_ms"] for f in fulls], 50)
    inc = [r["wall_ms"] for r in rows]
    byt = sum(r["bytes"] for r in rows)
    kms = sum(r["kernel_ms"] for r in rows)
    launches = sum(r["passes"] for r in rows)
    lo = [r for r in rows if not r["high"]]
    hi = [r for r in rows if r["high"]]
    return {
        "qubits": n, "levels": levels, "nets": len(wl.nets), "dtype": "c128", "state_gib": 64,
        "tile_bits": o.tile_bits, "low_bits": o.low_bits, "relabel": o.relabel,
        "ckpt_levels": K // 3, "ckpts_stored": HEADLINE["max_ckpts"],
        "first_full_ms": first["wall_ms"], "first_full_kernel_ms": first["kernel_ms"],
        "full_passes": first["passes"], "full_bytes": first["bytes"],
        "full_gbs": first["bytes"] / (first["kernel_ms"] * 1e-3) / 1e9,
        "full_ms_p50": full_ms,
        "timed_s": timed_s, "steps": rows,
        "inc_ms_p50": pct(inc, 50), "inc_ms_p99": pct(inc, 99),
        "inc_ms_p50_inside_tile": pct([r["wall_ms"] for r in lo], 50),
        "inc_ms_p50_across_tiles": pct([r["wall_ms"] for r in hi], 50),
        "speedup_p50": full_ms / pct(inc, 50), "speedup_p99": full_ms / pct(inc, 99),
        "replay_bound_speedup_p50": pct([r["levels_total"] / max(r["levels_replayed"], 1) for r in rows], 50),
        "timed_gbs": byt / (kms * 1e-3) / 1e9 if kms else None,
        "timed_wall_gbs": byt / timed_s / 1e9,
        "launches": launches, "launch_bytes": byt / max(launches, 1), "launch_ms": kms / max(launches, 1),
        "gate_amp_updates_per_s": sum(r["gate_amp_updates"] for r in rows) / timed_s,
        "verify": verify, "mismatches": mismatches,
    }


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


def run_fusion_wins(Q, W, n=28, levels=96):
    """Dense fusion where it pays: the blocked family (blocks of 5 adjacent
    qubits, RX/RY/RZ on every qubit and CZ inside the blocks each level, a
    CNOT between neighbouring blocks every 16 levels) at 28 qubits.  Each
    dtype runs twice with the autotuner choosing the tile shape: once with
    gate lists only (QTASK_FUSE_NONE) and once under QTASK_FUSE_AUTO, where
    it may also fuse every stage into a dense k-qubit unitary on the matrix
    cores.  Full simulations (best of two re-runs after the tuned first
    one); the results of the two plans are compared amplitude by amplitude,
    and complex64 against the complex128 gate-list result."""
    import numpy as np

    nets = W.blocked_circuit(n, levels, 7)
    out = {"workload": "blocked circuit, %d qubits, %d levels (blocks of 5 adjacent qubits; each level RX/RY/RZ on "
                       "every qubit then CZ on even and odd pairs inside each block; a CNOT between neighbouring "
                       "blocks every 16 levels)" % (n, levels), "qubits": n, "levels": levels}
    states = {}
    for dt in ("c128", "c64"):
        r = {}
        for name, fusion in (("lists", Q.QTASK_FUSE_NONE), ("auto", Q.QTASK_FUSE_AUTO)):
            s = Q.Simulator(n, dt, device=0, ckpt_interval=10 ** 6, autotune=1, fusion=fusion)
            try:
                s.build(nets)
                s.update()
                best = None
                for _ in range(2):
                    st = s.update(full=True)
                    if best is None or st["kernel_ms"] < best["kernel_ms"]:
                        best = st
                o = Q.qtask_get_opts(s.h)
                states[(dt, name)] = s.state()
            finally:
                s.close()
            r[name] = {"full_ms": best["kernel_ms"], "passes": best["passes"], "tile_bits": o.tile_bits,
                       "low_bits": o.low_bits, "fusion": {0: "auto", 1: "none", 2: "dense"}[o.fusion],
                       "fuse_width": o.fuse_width,
                       "mfma_tflops": best["mfma_flops"] / (best["kernel_ms"] * 1e-3) / 1e12,
                       "frac_of_mfma_peak": best["mfma_flops"] / (best["kernel_ms"] * 1e-3) / 1e12 /
                                            MFMA_PEAK_TFLOPS[dt]}
        r["speedup_auto_over_lists"] = r["lists"]["full_ms"] / r["auto"]["full_ms"]
        a = states[(dt, "lists")].astype(np.complex128)
        b = states[(dt, "auto")].astype(np.complex128)
        r["max_abs_auto_vs_lists"] = float(np.max(np.abs(a - b)))
        out[dt] = r
        log("blocked %d qubits %s: gate lists %.1f ms (b=%d c=%d), auto %.1f ms (%s k=%d b=%d, %.1f TFLOP/s), "
            "%.2fx" % (n, dt, r["lists"]["full_ms"], r["lists"]["tile_bits"], r["lists"]["low_bits"],
                       r["auto"]["full_ms"], r["auto"]["fusion"], r["auto"]["fuse_width"], r["auto"]["tile_bits"],
                       r["auto"]["mfma_tflops"], r["speedup_auto_over_lists"]))
    ref = states[("c128", "lists")]
    out["c64"]["max_abs_auto_vs_c128"] = float(np.max(np.abs(states[("c64", "auto")].astype(np.complex128) - ref)))
    return out


def run_sparse_ckpt(Q, W, n=24, levels=400, interval=20, full_ckpts=4, edits=20):
    """Sparse checkpoints (the paper's copy-on-write blocks) at a fixed
    checkpoint budget.  The top-controlled circuit (each level changes only
    the blocks whose top bit is 1) runs in two sessions with a checkpoint
    boundary every `interval` levels: one storing whole copies, at most
    `full_ckpts` of them; one storing each boundary's rewritable blocks, with
    as many boundaries as fit in the same bytes.  The same random
    single-gate inserts go to both; each update is compared with the other
    session's by state hash, and the restart levels and update times are
    reported.  The layered circuit's ratio of stored to whole-copy bytes is
    given beside it (every segment rewrites every block there)."""
    rng = __import__("numpy").random.default_rng(808)
    nets = W.top_controlled_circuit(n, levels, 17)
    out = {"workload": "top-controlled circuit, %d qubits, %d levels (an H layer, then one CX/CCX/CP/CZ per level "
                       "on the top qubit and qubits below it), complex128, a checkpoint boundary every %d levels, "
                       "%d random single-gate inserts" % (n, levels, interval, edits)}
    a = Q.Simulator(n, "c128", device=0, ckpt_interval=interval, max_ckpts=full_ckpts)
    try:
        a.build(nets)
        sa = a.update()
        ratio = sa["ckpt_bytes"] / max(sa["ckpt_full_bytes"], 1)
        # the most sparse checkpoints that fit in the bytes of the whole copies
        # (found on plan-only sessions, which lay out the same checkpoints)
        k_delta, delta_ratio = full_ckpts, 1.0
        for k in range(4 * full_ckpts, full_ckpts - 1, -1):
            probe = Q.Simulator(n, "c128", device=Q.QTASK_DEVICE_NONE, ckpt_interval=interval, ckpt_delta=1,
                                max_ckpts=k)
            try:
                probe.build(nets)
                sp = probe.update()
            finally:
                probe.close()
            if sp["ckpt_bytes"] <= sa["ckpt_bytes"]:
                k_delta, delta_ratio = k, sp["ckpt_bytes"] / max(sp["ckpt_full_bytes"], 1)
                break
        b = Q.Simulator(n, "c128", device=0, ckpt_interval=interval, ckpt_delta=1, max_ckpts=k_delta)
        try:
            b.build(nets)
            sb = b.update()
            rows, mism = [], 0
            work = [list(x) for x in nets]
            for i in range(edits):
                li = int(rng.integers(1, len(work)))
                used = {q for g in work[li] for q in g[1]}
                free = [q for q in range(n - 1) if q not in used]
                g = ("cx", (n - 1, free[int(rng.integers(len(free)))]), ()) if n - 1 not in used else \
                    ("t", (free[int(rng.integers(len(free)))],), ())
                e = W.Edit("insert", li, g)
                W.apply_edit(work, e)
                a.apply_edit(e)
                b.apply_edit(e)
                ra, rb = a.update(), b.update()
                mism += int(a.hash() != b.hash())
                rows.append((ra["first_level"], rb["first_level"], ra["wall_ms"], rb["wall_ms"]))
            hb = b.hash()
            b.update(full=True)
            mism += int(b.hash() != hb)
            out.update({
                "ckpt_bytes_full_copies": sa["ckpt_bytes"], "ckpts_full": full_ckpts,
                "ckpt_bytes_sparse": sb["ckpt_bytes"], "ckpt_full_bytes_sparse_session": sb["ckpt_full_bytes"],
                "ckpts_sparse": k_delta, "stored_over_whole_copy_bytes": sb["ckpt_bytes"] / max(sb["ckpt_full_bytes"], 1),
                "restart_level_mean_full": sum(r[0] for r in rows) / len(rows),
                "restart_level_mean_sparse": sum(r[1] for r in rows) / len(rows),
                "update_ms_p50_full": pct([r[2] for r in rows], 50),
                "update_ms_p50_sparse": pct([r[3] for r in rows], 50),
                "mismatches": mism})
        finally:
            b.close()
    finally:
        a.close()
    lay = Q.Simulator(n, "c128", device=0, ckpt_interval=100, ckpt_delta=1)
    try:
        lay.build(W.config(2, n=n, levels=100, batches=1).nets)
        sl = lay.update()
        out["layered_stored_over_whole_copy_bytes"] = sl["ckpt_bytes"] / max(sl["ckpt_full_bytes"], 1)
    finally:
        lay.close()
    log("sparse checkpoints: %.2f of whole-copy bytes, %d boundaries in %.2f GB against %d in %.2f GB; restart "
        "level mean %.0f vs %.0f, update p50 %.1f vs %.1f ms, mismatches %d; layered %.2f" % (
            out["stored_over_whole_copy_bytes"], out["ckpts_sparse"], out["ckpt_bytes_sparse"] / 1e9, full_ckpts,
            out["ckpt_bytes_full_copies"] / 1e9, out["restart_level_mean_sparse"],
            out["restart_level_mean_full"], out["update_ms_p50_sparse"], out["update_ms_p50_full"],
            out["mismatches"], out["layered_stored_over_whole_copy_bytes"]))
    return out


def cpu_baseline(Q, W, full_bytes_per_gate, min_s=10.0):
    """The CPU oracle (all host threads, then one) on a bounded sample of the
    headline workload: the 32-qubit circuit's first gates, one at a time,
    until about min_s seconds of work (the oracle holds the whole 64 GiB
    state in host memory; its pages are touched before the timing).  The
    same gates then run on the device and the two states are compared on
    the first 2^20 amplitudes and 4096 spread over the rest."""
    import numpy as np

    from oracle import oracle

    n = HEADLINE["n"]
    wl = W.config(5, levels=1, batches=1)
    gates = [g for net in wl.nets for g in net]
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    psi = np.empty(1 << n, dtype=np.complex128)
    psi.fill(0)
    psi[0] = 1
    touch_s = time.perf_counter() - t0
    used = 0
    t0 = time.perf_counter()
    for g in gates:
        oracle.apply_gates(n, psi, [g], threads)
        used += 1
        if time.perf_counter() - t0 >= min_s:
            break
    dt = time.perf_counter() - t0
    # the device on the same first `used` gates (they lie in the first net)
    err = 0.0
    idx = np.linspace(1 << 20, (1 << n) - 1, 4096).astype(np.int64)
    s = Q.Simulator(n, "c128", device=0, tile_bits=HEADLINE["tile_bits"], low_bits=HEADLINE["low_bits"],
                    relabel=1)
    try:
        s.build([gates[:used]])
        s.update()
        for lo in range(0, 1 << 20, 1 << 18):
            err = max(err, float(np.max(np.abs(s.state(lo, 1 << 18) - psi[lo:lo + (1 << 18)]))))
        for i in idx:
            err = max(err, float(abs(s.state(int(i), 1)[0] - psi[int(i)])))
    finally:
        s.close()
    # one thread, on the next gates (about min_s / 3)
    g1 = 0
    t1 = time.perf_counter()
    for g in gates[used:]:
        if time.perf_counter() - t1 >= min_s / 3:
            break
        oracle.apply_gates(n, psi, [g], 1)
        g1 += 1
    dt1 = time.perf_counter() - t1
    del psi
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": full_bytes_per_gate * used / dt / 1e9,
        "unit": "GB/s",
        "cores": threads,
        "cpu_model": model,
        "host_cpus": os.cpu_count(),
        "kind": "oracle",
        "sample": "the first %d gates of the 32-qubit, 500-level ladder circuit (complex128, the whole 64 GiB state "
                  "in host memory), %.1f s on %d threads; value = the device plan's bytes per gate (full "
                  "simulation average) times the gates, divided by the oracle time" % (used, dt, threads),
        "gate_amp_updates_per_s": used * float(1 << n) / dt,
        "value_1_thread": full_bytes_per_gate * g1 / dt1 / 1e9 if g1 else None,
        "gate_amp_updates_per_s_1_thread": g1 * float(1 << n) / dt1 if g1 else None,
        "first_touch_s": touch_s,
        "max_abs_device_c128_vs_oracle": err,
        "compared": "first 2^20 amplitudes and 4096 spread over the rest, after the sampled gates",
    }


def load_traffic(path):
    """HBM bytes per launch from a committed counter summary, or None once the
    kernel source no longer matches the one the counters were taken on."""
    if not path or not os.path.exists(path):
        return None
    from paper_2210_01076_amd import profiling
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != profiling.kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def load_issue(path, launch_ms):
    """The VALU-issue bound of the pass kernel from a committed SQ-counter
    summary (the share of SIMD time its VALU instructions take, times the
    traced launch time), beside the live launch time; None once the kernel
    source no longer matches."""
    if not path or not os.path.exists(path):
        return None
    from paper_2210_01076_amd import profiling
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != profiling.kernel_source_hash():
        return None
    bound_ms = rec["valu_bound_us"] / 1e3
    return {"valu_issue_share": round(rec["valu_issue_share"], 4), "valu_bound_ms": round(bound_ms, 2),
            "frac_of_valu_bound": round(bound_ms / launch_ms, 4) if launch_ms else None,
            "source": os.path.relpath(path, ROOT)}


def run_extras(Q, W, args):
    """The legs that do not fit the default run's time: the paper's other
    incremental protocols on the 24-qubit circuit, the 28-qubit layered
    state, and the 30-qubit fused-unitary configuration."""
    wl = W.config(2)
    out = {"metric": "extra legs (see each entry)"}
    out["large_state"] = run_large(Q, W)
    log("28-qubit complex128 full simulation: %.1f ms, %.0f GB/s" % (out["large_state"]["full_ms"],
                                                                   out["large_state"]["gbs"]))
    sim, _, r = run_tier(Q, W, wl, "c128", 2, 0)
    sim.close()
    out["append_protocol"] = run_append(Q, wl, "c128", r["tile_bits"], r["low_bits"])
    out["other_protocols"] = run_protocols(Q, wl, "c128", r["tile_bits"], r["low_bits"])
    out["fused_dense"] = run_fused(Q, W, n=args.fused_qubits, levels=args.fused_levels,
                                   tuned=not args.no_fused_tuned)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tier24", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the 32-qubit headline (profiling runs)")
    ap.add_argument("--headline-levels", type=int, default=0,
                    help="depth of the headline circuit (default 500; profiling runs may shorten it)")
    ap.add_argument("--verify-edits", type=int, default=1,
                    help="headline edits after the timed steps that are each compared with a full re-simulation")
    ap.add_argument("--tile-bits", type=int, default=0, help="headline tile bits (default 12)")
    ap.add_argument("--low-bits", type=int, default=0, help="headline contiguous low bits (default 4)")
    ap.add_argument("--budget-s", type=float, default=480.0,
                    help="wall-clock budget: the legs after the headline that would not fit are skipped "
                         "(and named in the line)")
    ap.add_argument("--extras", action="store_true",
                    help="instead of the default run: the 28-qubit state, the paper's other incremental "
                         "protocols and the 30-qubit fused-unitary legs, printed as one JSON line")
    ap.add_argument("--serving-sweep", action="store_true",
                    help="only the serving latency-throughput sweep (several minutes), printed as one JSON line")
    ap.add_argument("--fusion-only", action="store_true",
                    help="only the blocked-circuit leg where dense fusion pays, printed as one JSON line")
    ap.add_argument("--fusion-profile", nargs="?", const="c64:10", default=None, metavar="DTYPE:B",
                    help="only the dense k=5 plan of that leg in one dtype and tile size (default c64:10, c=4), "
                         "two full simulations (for counter runs of the matrix-core kernel)")
    ap.add_argument("--fused-qubits", type=int, default=30, help="state size of the fused-unitary leg")
    ap.add_argument("--fused-levels", type=int, default=300, help="depth of the fused-unitary leg")
    ap.add_argument("--no-fused-tuned", action="store_true",
                    help="skip the autotuned comparison run of the fused-unitary leg (its timing candidates "
                         "would mix into a profile of the fused kernels)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic_ladder_n32.json"))
    ap.add_argument("--issue", default=os.path.join(ROOT, "profiles", "issue_ladder_n32.json"))
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the state and the serving sessions are not sharded across GPUs "
              "(the design notes describe how they would be)", file=sys.stderr)
        sys.exit(2)

    from paper_2210_01076_amd import qtask as Q
    from paper_2210_01076_amd import workloads as W

    if args.extras:
        print(json.dumps(run_extras(Q, W, args)))
        return
    if args.fusion_only:
        print(json.dumps(run_fusion_wins(Q, W)))
        return
    if args.fusion_profile:
        dt, tb = args.fusion_profile.split(":")
        if dt not in ("c64", "c128"):
            raise SystemExit("--fusion-profile: dtype must be c64 or c128")
        nets = W.blocked_circuit(28, 96, 7)
        s = Q.Simulator(28, dt, device=0, ckpt_interval=10 ** 6, fusion=Q.QTASK_FUSE_DENSE, fuse_width=5,
                        tile_bits=int(tb), low_bits=4, autotune=0)
        try:
            s.build(nets)
            runs = [s.update(), s.update(full=True)]
        finally:
            s.close()
        print(json.dumps({"workload": "blocked circuit, 28 qubits, 96 levels, %s, every stage a dense 5-qubit "
                                      "unitary on the matrix cores (b=%s, c=4)" % ({"c64": "complex64",
                                                                                     "c128": "complex128"}[dt], tb),
                          "runs": [{"kernel_ms": r["kernel_ms"], "passes": r["passes"], "mfma_flops": r["mfma_flops"]}
                                   for r in runs]}))
        return
    if args.serving_sweep:
        sweep = {"metric": "serving request latency against offered load", "unit": "ms",
                 "workload": "256 sessions, qubits log-uniform in [12,28], depth U{50..400} layered levels; "
                             "per offered rate one Poisson stream of 128 requests of 1-3 edits over 128 sessions, "
                             "then one request to every session at once",
                 "c64": run_serving_curve(Q, W, "c64", [8, 16, 32, 48])[0],
                 "c128": run_serving_curve(Q, W, "c128", [8, 16, 24])[0]}
        print(json.dumps(sweep))
        return

    t_start = time.perf_counter()
    copy_gbs = Q.qtask_copy_bandwidth(0, 1 << 30, 20)
    log("copy kernel ceiling %.1f GB/s" % copy_gbs)
    head = run_headline(Q, W, args.steps, args.warmup, args.tile_bits or None, args.low_bits or None,
                        args.headline_levels or None, args.verify_edits)
    log("headline: update p50 %.0f ms p99 %.0f ms, full %.0f ms, speedup p50 %.2f (bound %.2f), %.0f GB/s per "
        "launch, mismatches %d (%.0f s so far)" % (
            head["inc_ms_p50"], head["inc_ms_p99"], head["full_ms_p50"], head["speedup_p50"],
            head["replay_bound_speedup_p50"], head["launch_bytes"] / head["launch_ms"] / 1e6, head["mismatches"],
            time.perf_counter() - t_start))

    tier24 = None
    small = None
    serving = None
    cpu = None
    fusion_wins = None
    sparse_ckpt = None
    skipped = []

    def fits(name, est_s):
        """Whether a leg estimated at est_s seconds still fits the wall budget."""
        if time.perf_counter() - t_start + est_s <= args.budget_s:
            return True
        skipped.append(name)
        log("skipping %s: %.0f s used of the %.0f s budget" % (name, time.perf_counter() - t_start, args.budget_s))
        return False

    if not args.headline_only:
        if not args.no_cpu and fits("cpu_baseline", 40):
            per_gate = head["full_bytes"] / W.count_gates(W.config(5, levels=head["levels"], batches=1).nets)
            cpu = cpu_baseline(Q, W, per_gate)
            log("cpu oracle: %.2f GB/s equivalent on %d threads; device vs oracle max-abs %.2e" % (
                cpu["value"], cpu["cores"], cpu["max_abs_device_c128_vs_oracle"]))
        if fits("small_circuit", 10):
            small = run_small(Q, W)
            log("10-qubit circuit: update p50 %.0f us p99 %.0f us, full re-simulation p50 %.0f us (%.0f us with the "
                "edited segment's plan already made), mismatches %d" % (
                    small["update_us_p50"], small["update_us_p99"], small["full_us_p50"],
                    small["full_plans_cached_us_p50"], small["mismatches"]))
        if not args.no_serving and fits("serving", 80):
            import numpy as np
            s128, kept128 = run_serving_curve(Q, W, "c128", [11, 20])
            s64, kept64 = run_serving_curve(Q, W, "c64", [23, 41])
            errs = [float(np.max(np.abs(kept128[i] - kept64[i].astype(np.complex128)))) for i in kept128
                    if i in kept64]
            s64["max_abs_vs_c128"] = max(errs) if errs else None
            s64["compared_sessions"] = len(errs)
            serving = {"workload": "256 sessions, qubits log-uniform in [12,28], depth U{50..400} layered levels; "
                                   "requests of 1-3 edits: Poisson streams at about 50% and 90% of the saturated "
                                   "rate over 128 sessions each, then one request to every session at once; "
                                   "sessions under 16 qubits batched",
                       "c128": s128, "c64": s64}
        if fits("fusion_wins", 40):
            fusion_wins = run_fusion_wins(Q, W)
        if fits("sparse_ckpt", 20):
            sparse_ckpt = run_sparse_ckpt(Q, W)
        if not args.no_tier24 and fits("tier24", 10 + 1.5 * (args.steps + args.warmup)):
            import numpy as np
            wl = W.config(2)
            sim128, _, r128 = run_tier(Q, W, wl, "c128", args.steps, args.warmup)
            sim64, _, r64 = run_tier(Q, W, wl, "c64", args.steps, args.warmup)
            a = sim128.state()
            b = sim64.state().astype(np.complex128)
            r64["max_abs_vs_c128"] = float(np.max(np.abs(a - b)))
            r64["fidelity_vs_c128"] = fidelity(a, b)
            sim64.close()
            sim128.close()
            tier24 = {"workload": "layered random circuit, 24 qubits, 200 levels (RX/RY/RZ on every qubit + random "
                                  "CNOT matching), modifier batches of 1-4 random gate inserts/removals; checkpoints "
                                  "every 50 levels; cache-assisted (the 256 MiB state is about the size of the "
                                  "Infinity Cache)",
                      "batches": args.steps, "ckpt_levels": wl.ckpt_nets // 2, "c128": r128, "c64": r64}
            log("24-qubit tier: c128 update p50 %.1f ms vs full %.1f ms; c64 %.1f ms vs %.1f ms" % (
                r128["inc_ms_p50"], r128["full_ms_p50"], r64["inc_ms_p50"], r64["full_ms_p50"]))

    achieved = head["launch_bytes"] / (head["launch_ms"] * 1e-3) / 1e9
    b = head["tile_bits"]
    line = {
        "metric": "full-sim HBM GB/s vs peak; incremental update p50/p99 latency and speedup vs full re-sim",
        "value": round(head["timed_wall_gbs"], 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["timed_s"] * 1e3 / max(args.steps, 1), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "controlled-phase ladder circuit, 32 qubits, %d levels (RX/RY/RZ on every qubit, "
                               "then CP on even and on odd adjacent pairs); one step = one single-gate insert at a "
                               "uniformly random level (alternately inside one tile and across tiles) and its "
                               "incremental update; complex128, 64 GiB state, checkpoints every 50 levels, 3 "
                               "stored" % head["levels"],
                   "qubits": 32, "levels": head["levels"], "edits": args.steps, "ckpt_levels": head["ckpt_levels"],
                   "ckpts_stored": head["ckpts_stored"], "tile_bits": b, "low_bits": head["low_bits"],
                   "relabel": head["relabel"]},
        "frac_of_peak": round(head["timed_wall_gbs"] / HBM_PEAK_GBS, 4),
        "copy_ceiling_gbs": round(copy_gbs, 1),
        "full_sim_gbs": round(head["full_gbs"], 1),
        "full_ms_p50": head["full_ms_p50"],
        "incremental_ms_p50": head["inc_ms_p50"],
        "incremental_ms_p99": head["inc_ms_p99"],
        "incremental_speedup_p50": head["speedup_p50"],
        "replay_bound_speedup_p50": head["replay_bound_speedup_p50"],
        "incremental_mismatches": head["mismatches"],
        "headline": head,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": load_traffic(args.traffic),
                     "kernel": "qk_pass<double, false>", "bytes_per_launch": head["launch_bytes"],
                     "avg_launch_ms": head["launch_ms"], "launches_timed": head["launches"],
                     "block": 1 << (b - 4),
                     "scope": "every pass launch of the timed steps (32 qubits, complex128)",
                     "issue": load_issue(args.issue, head["launch_ms"])},
        "tier24": tier24,
        "fusion_wins": fusion_wins,
        "sparse_ckpt": sparse_ckpt,
        "small_circuit": small,
        "serving": serving,
        "cpu_baseline": cpu,
        "skipped_for_budget": skipped,
        "run_s": time.perf_counter() - t_start,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
