"""Serving loop on the GPU: every request's result is the same alone and in
the mix (bitwise: the batched kernel runs the same pass body as the per-session
launch), for small sessions batched into graph-replayed rounds and large ones
on their own streams, and memory admission evicts and restores sessions."""
import numpy as np
import pytest

from oracle import oracle
from paper_2210_01076_amd import qtask as Q
from paper_2210_01076_amd import workloads as W
from tests.gpu_util import bytes_equal, check_state, log

pytestmark = pytest.mark.gpu


def _specs(seed, count, n_lo, n_hi, depth, requests, dtype=None):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        dt = dtype or ("c128" if i % 2 == 0 else "c64")
        nets = W.layered_circuit(n, depth, seed + i)
        reqs = W.modifier_batches(n, nets, seed + 1000 + i, requests, 1, 3, W.LAYERED_EDIT_KINDS)
        out.append((n, dt, nets, reqs))
    return out


def _alone(n, dtype, nets, reqs, opts):
    """Hash and final state of each request when the session runs alone."""
    hashes = []
    nets = [list(x) for x in nets]
    with Q.Simulator(n, dtype, device=0, **opts) as s:
        s.build(nets)
        s.update()
        hashes.append(s.hash())
        for batch in reqs:
            for e in batch:
                W.apply_edit(nets, e)
                s.apply_edit(e)
            s.update()
            hashes.append(s.hash())
        return hashes, s.state(), nets


def _serve(specs, opts, phases, read_states=True, **sopts):
    """Open every session, submit its initial simulation, then the requests
    of each phase (lists of (request, session)), draining after each."""
    sv = Q.qtask_server_create(Q.qtask_server_opts_default(**sopts))
    try:
        sids, tickets = [], {}
        for i, (n, dtype, nets, _) in enumerate(specs):
            dt = Q.QTASK_C128 if dtype == "c128" else Q.QTASK_C64
            o = opts[i] if isinstance(opts, list) else opts
            sids.append(Q.qtask_server_open(sv, n, dt, Q.qtask_opts_default(device=0, **o), nets))
        for i, sid in enumerate(sids):
            tickets[(i, 0)] = Q.qtask_server_submit(sv, sid, [])
        usage = []
        for order in phases:
            for r, i in order:
                edits = [c for e in specs[i][3][r] for c in Q.make_edits(e)]
                tickets[(i, r + 1)] = Q.qtask_server_submit(sv, sids[i], edits)
            Q.qtask_server_drain(sv)
            usage.append(Q.qtask_server_usage(sv))
        results = {k: Q.qtask_server_wait(sv, t, 0.0) for k, t in tickets.items()}
        _serve.paths = Q.qtask_server_paths(sv)
        states = []
        if read_states:
            for i, sid in enumerate(sids):
                h = Q.qtask_server_session(sv, sid)
                dt = Q.QTASK_C128 if specs[i][1] == "c128" else Q.QTASK_C64
                states.append(Q.qtask_read_amplitudes(h, 0, 1 << specs[i][0], dt))
        return results, states, usage
    finally:
        Q.qtask_server_destroy(sv)


def _interleaved(specs, requests):
    return [(r, i) for r in range(requests) for i in range(len(specs))]


@pytest.mark.parametrize("use_graph", [1, 0])
def test_small_sessions_alone_equals_mix(use_graph):
    """Sessions of 6..15 qubits, both dtypes, all in the batched path."""
    specs = _specs(41, 12, 6, 15, 12, 3)
    opts = dict(ckpt_interval=5)
    alone = [_alone(n, d, nets, reqs, opts) for n, d, nets, reqs in specs]
    results, states, usage = _serve(specs, opts, [_interleaved(specs, 3)], use_graph=use_graph)
    assert _serve.paths["streamed"] == 0 and _serve.paths["batched"] == len(results), _serve.paths
    for (i, r), res in sorted(results.items()):
        assert res["status"] == Q.QTASK_OK, (i, r, res["status"])
        assert res["state_hash"] == alone[i][0][r], "session %d request %d differs from its run alone" % (i, r)
        assert res["done_ms"] >= res["start_ms"] >= res["submit_ms"] - 1e-6
    for i, (n, d, _, _) in enumerate(specs):
        assert bytes_equal(states[i], alone[i][1])
        check_state(states[i], oracle.simulate(n, alone[i][2]), d, "session %d" % i)
    log("small mix ok, usage", usage)


@pytest.mark.parametrize("use_graph", [1, 0])
def test_fused_small_sessions_stay_batched(use_graph):
    """Small sessions whose plans have dense fused stages (on the matrix
    cores at 10 qubits and up, on the vector ALU below) share batched ticks
    with unfused ones: the batched kernel runs each pass in the variant the
    session's own launch would use, so every result equals the run alone
    and no request leaves the batched path."""
    specs = _specs(53, 12, 6, 15, 12, 3)
    opts = []
    for i, (n, _, _, _) in enumerate(specs):
        if i % 3 == 2:
            opts.append(dict(ckpt_interval=5))
        elif n >= 10:
            opts.append(dict(ckpt_interval=5, fusion=Q.QTASK_FUSE_DENSE, fuse_width=5, tile_bits=10))
        else:
            opts.append(dict(ckpt_interval=5, fusion=Q.QTASK_FUSE_DENSE, fuse_width=4))
    alone = [_alone(n, d, nets, reqs, opts[i]) for i, (n, d, nets, reqs) in enumerate(specs)]
    results, states, _ = _serve(specs, opts, [_interleaved(specs, 3)], use_graph=use_graph)
    paths = _serve.paths
    assert paths["streamed"] == 0 and paths["batched"] == len(results), paths
    for (i, r), res in sorted(results.items()):
        assert res["status"] == Q.QTASK_OK, (i, r, res["status"])
        assert res["state_hash"] == alone[i][0][r], "session %d request %d differs from its run alone" % (i, r)
    for i, (n, d, _, _) in enumerate(specs):
        assert bytes_equal(states[i], alone[i][1])
        check_state(states[i], oracle.simulate(n, alone[i][2]), d, "session %d" % i)
    log("fused small mix ok, paths", paths)


@pytest.mark.parametrize("order", [0, 1])
def test_mixed_sizes_alone_equals_mix(order):
    """Small batched sessions beside large ones on their own streams, with
    requests started oldest first or expected-shortest first."""
    small = _specs(77, 6, 8, 14, 10, 2)
    large = _specs(88, 3, 17, 19, 10, 2)
    specs = small + large
    opts = dict(ckpt_interval=4)
    alone = [_alone(n, d, nets, reqs, opts) for n, d, nets, reqs in specs]
    results, states, _ = _serve(specs, opts, [_interleaved(specs, 2)], max_inflight=2, order=order)
    for (i, r), res in sorted(results.items()):
        assert res["status"] == Q.QTASK_OK
        assert res["state_hash"] == alone[i][0][r], "session %d request %d" % (i, r)
    for i in range(len(specs)):
        assert bytes_equal(states[i], alone[i][1])



def test_admission_evicts_and_restores():
    """A budget that holds two of four sessions: every request still
    finishes, sessions evicted in the first phase are re-simulated from the
    start by their requests of the second, and every result equals the run
    alone."""
    specs = _specs(99, 4, 18, 18, 8, 3, dtype="c128")
    opts = dict(ckpt_interval=100)
    alone = [_alone(n, d, nets, reqs, opts) for n, d, nets, reqs in specs]
    state_bytes = (1 << 18) * 16
    budget = 2 * state_bytes + 4 * (1 << 20)
    phase1 = [(0, i) for i in range(4)]
    phase2 = [(r, i) for r in (1, 2) for i in range(4)]
    results, _, usage = _serve(specs, opts, [phase1, phase2], read_states=False, budget_bytes=budget,
                               max_inflight=4)
    for (i, r), res in sorted(results.items()):
        assert res["status"] == Q.QTASK_OK, (i, r, res["status"])
        assert res["state_hash"] == alone[i][0][r], "session %d request %d" % (i, r)
    for used, resident in usage:
        assert used <= budget and resident <= 2
    log("admission usage per phase", usage)


def test_request_that_cannot_fit_fails_cleanly():
    nets = W.layered_circuit(16, 4, 5)
    sv = Q.qtask_server_create(Q.qtask_server_opts_default(budget_bytes=1 << 20))
    try:
        sid = Q.qtask_server_open(sv, 16, Q.QTASK_C128, Q.qtask_opts_default(device=0), nets)
        t = Q.qtask_server_submit(sv, sid, [])
        res = Q.qtask_server_wait(sv, t, 60000.0)
        assert res["status"] == Q.QTASK_E_NOMEM
        h = Q.qtask_server_session(sv, sid)
        with pytest.raises(Q.QtaskError) as ei:
            Q.qtask_update_state(h)
        assert ei.value.code == Q.QTASK_E_BUSY
    finally:
        Q.qtask_server_destroy(sv)


def test_bad_edit_reports_status_and_session_recovers():
    n = 10
    nets = W.layered_circuit(n, 6, 6)
    sv = Q.qtask_server_create()
    try:
        sid = Q.qtask_server_open(sv, n, Q.QTASK_C128, Q.qtask_opts_default(device=0), nets)
        t0 = Q.qtask_server_submit(sv, sid, [])
        bad = Q.qtask_edit(op=0, kind=Q.KIND["h"], level=999, nq=1)
        t1 = Q.qtask_server_submit(sv, sid, [bad])
        t2 = Q.qtask_server_submit(sv, sid, [])
        r0, r1, r2 = (Q.qtask_server_wait(sv, t, 60000.0) for t in (t0, t1, t2))
        assert r0["status"] == Q.QTASK_OK
        assert r1["status"] == Q.QTASK_E_NOTFOUND
        assert r2["status"] == Q.QTASK_OK and r2["state_hash"] == r0["state_hash"]
    finally:
        Q.qtask_server_destroy(sv)


def _growing_specs(seed, count, n, depth, requests, inserts):
    """Sessions whose every request inserts new nets (each with one random
    gate): the circuit grows, and with it the number of checkpoints."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        nets = W.layered_circuit(n, depth, seed + i)
        cur = [list(x) for x in nets]
        reqs = []
        for _ in range(requests):
            batch = []
            for _ in range(inserts):
                li = int(rng.integers(len(cur)))
                kind = W.LAYERED_EDIT_KINDS[int(rng.integers(len(W.LAYERED_EDIT_KINDS)))]
                qs = tuple(int(q) for q in rng.choice(n, size=2 if kind == "cx" else 1, replace=False))
                ps = (float(rng.uniform(0, 2 * np.pi)),) if kind in ("rx", "ry", "rz") else ()
                e = W.Edit("insert", li, (kind, qs, ps), new_net=True)
                W.apply_edit(cur, e)
                batch.append(e)
            reqs.append(batch)
        out.append((n, "c128", nets, reqs))
    return out


def test_admission_holds_budget_while_sessions_grow():
    """Requests that insert nets add segments and so checkpoints.  Admission
    charges each session's bytes after its update (state, checkpoints, plans
    and scratch), so under a budget of about two and a half final footprints
    the admitted bytes never exceed the budget, even at their peak, every
    request finishes and every result equals the session run alone."""
    specs = _growing_specs(123, 4, 16, 6, 3, 3)
    opts = dict(ckpt_interval=2)
    alone = [_alone(n, d, nets, reqs, opts) for n, d, nets, reqs in specs]
    # the largest footprint any session reaches alone
    peak_alone = 0
    for n, d, nets, reqs in specs[:1]:
        nets = [list(x) for x in nets]
        with Q.Simulator(n, d, device=0, **opts) as s:
            s.build(nets)
            s.update()
            for batch in reqs:
                for e in batch:
                    W.apply_edit(nets, e)
                    s.apply_edit(e)
                s.update()
                peak_alone = max(peak_alone, Q.qtask_device_bytes(s.h))
    budget = int(2.5 * peak_alone)
    sv = Q.qtask_server_create(Q.qtask_server_opts_default(budget_bytes=budget, max_inflight=4))
    try:
        sids, tickets, usage = [], {}, []
        for n, dtype, nets, _ in specs:
            sids.append(Q.qtask_server_open(sv, n, Q.QTASK_C128, Q.qtask_opts_default(device=0, **opts), nets))
        for i, sid in enumerate(sids):
            tickets[(i, 0)] = Q.qtask_server_submit(sv, sid, [])
        Q.qtask_server_drain(sv)
        usage.append(Q.qtask_server_usage(sv))
        for r in range(3):
            for i, sid in enumerate(sids):
                edits = [c for e in specs[i][3][r] for c in Q.make_edits(e)]
                tickets[(i, r + 1)] = Q.qtask_server_submit(sv, sid, edits)
            Q.qtask_server_drain(sv)
            usage.append(Q.qtask_server_usage(sv))
        peak = Q.qtask_server_peak_bytes(sv)
        for (i, r), t in sorted(tickets.items()):
            res = Q.qtask_server_wait(sv, t, 0.0)
            assert res["status"] == Q.QTASK_OK, (i, r, res["status"])
            assert res["state_hash"] == alone[i][0][r], "session %d request %d" % (i, r)
        for used, resident in usage:
            assert used <= budget, (used, budget)
        assert peak <= budget, (peak, budget)
        log("growing sessions: budget", budget, "peak", peak, "usage", usage)
    finally:
        Q.qtask_server_destroy(sv)


def test_request_is_undone_when_it_can_never_fit():
    """A request whose inserted nets would need more checkpoints than the
    budget holds fails with QTASK_E_NOMEM and is undone: the session keeps
    its previous state and circuit, and its next request runs normally."""
    n = 14
    nets = W.layered_circuit(n, 4, 7)
    opts = dict(ckpt_interval=2)
    with Q.Simulator(n, "c128", device=0, **opts) as s:
        s.build([list(x) for x in nets])
        s.update()
        fits = Q.qtask_device_bytes(s.h)
        want = s.hash()
    budget = fits + (1 << n) * 16 // 2   # room for less than one more checkpoint
    sv = Q.qtask_server_create(Q.qtask_server_opts_default(budget_bytes=budget))
    try:
        sid = Q.qtask_server_open(sv, n, Q.QTASK_C128, Q.qtask_opts_default(device=0, **opts), nets)
        r0 = Q.qtask_server_wait(sv, Q.qtask_server_submit(sv, sid, []), 60000.0)
        assert r0["status"] == Q.QTASK_OK and r0["state_hash"] == want
        grow = [Q.qtask_edit(op=2, level=len(nets) - 1) for _ in range(6)]
        r1 = Q.qtask_server_wait(sv, Q.qtask_server_submit(sv, sid, grow), 60000.0)
        assert r1["status"] == Q.QTASK_E_NOMEM
        h = Q.qtask_server_session(sv, sid)
        assert Q.qtask_num_levels(h) == len(nets)
        assert Q.qtask_state_hash(h) == want
        r2 = Q.qtask_server_wait(sv, Q.qtask_server_submit(sv, sid, []), 60000.0)
        assert r2["status"] == Q.QTASK_OK and r2["state_hash"] == want
        assert Q.qtask_server_peak_bytes(sv) <= budget
    finally:
        Q.qtask_server_destroy(sv)
