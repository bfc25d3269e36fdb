"""Host-side logic of the library, run without a GPU: the C ABI's exports and
error semantics, the planner (checked by emulating its dumped plans on the
CPU against the oracle) and the affected-block tracker (the paper's worked
example, and soundness against oracle snapshots).  Sessions here are
plan-only (device QTASK_DEVICE_NONE): no device memory, no kernels."""
import json
import os
import re

import numpy as np
import pytest

from oracle import oracle
from paper_2210_01076_amd import qtask as Q
from paper_2210_01076_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def plan_only(n, dtype="c128", **kw):
    return Q.Simulator(n, dtype, device=Q.QTASK_DEVICE_NONE, **kw)


# ------------------------------------------------------------------- ABI

def test_library_exports_every_declared_symbol():
    lib = Q.load()
    with open(os.path.join(ROOT, "include", "qtask.h")) as f:
        header = f.read()
    names = set(re.findall(r"^\s*(?:const\s+char\s*\*|int)\s*(qtask_\w+)\s*\(", header, re.M))
    assert len(names) >= 30
    for name in sorted(names):
        assert hasattr(lib, name), name
        assert name in Q._SIGS, name


def test_status_strings_and_version():
    lib = Q.load()
    for code in range(9):
        assert lib.qtask_status_string(code)
    import ctypes
    a, b = ctypes.c_int(), ctypes.c_int()
    assert lib.qtask_version(ctypes.byref(a), ctypes.byref(b)) == 0 and a.value >= 1


def test_create_argument_errors():
    lib = Q.load()
    import ctypes
    h = ctypes.c_void_p()
    o = Q.qtask_opts_default(device=Q.QTASK_DEVICE_NONE)
    assert lib.qtask_create(0, 0, ctypes.byref(o), ctypes.byref(h)) == Q.QTASK_E_ARG
    assert lib.qtask_create(35, 0, ctypes.byref(o), ctypes.byref(h)) == Q.QTASK_E_ARG
    assert lib.qtask_create(5, 7, ctypes.byref(o), ctypes.byref(h)) == Q.QTASK_E_ARG
    bad = Q.qtask_opts_default(device=Q.QTASK_DEVICE_NONE, tile_bits=20)
    assert lib.qtask_create(5, 0, ctypes.byref(bad), ctypes.byref(h)) == Q.QTASK_E_ARG
    bad = Q.qtask_opts_default(device=Q.QTASK_DEVICE_NONE, ckpt_interval=-3)
    assert lib.qtask_create(5, 0, ctypes.byref(bad), ctypes.byref(h)) == Q.QTASK_E_ARG
    assert lib.qtask_create(5, 0, ctypes.byref(o), None) == Q.QTASK_E_ARG


def test_circuit_store_errors_keep_state():
    with plan_only(5) as sim:
        sim.build([[("h", (0,), ())], [("cx", (4, 3), ())]])
        lib = Q.load()
        import ctypes
        n_before = ctypes.c_uint64()
        lib.qtask_num_gates(sim.h, ctypes.byref(n_before))
        with pytest.raises(Q.QtaskError) as e:          # shares q4 with the CX: paper's conflict
            Q.qtask_insert_gate(sim.h, sim.levels[1], "cx", (4, 1))
        assert e.value.code == Q.QTASK_E_CONFLICT
        for qs, ps, kind in [((5,), (), "h"), ((1, 1), (), "cx"), ((0,), (), "rx"), ((0,), (1.0, 2.0), "rz"),
                             ((-1,), (), "x"), ((0,), (float("nan"),), "ry")]:
            with pytest.raises(Q.QtaskError) as e:
                Q.qtask_insert_gate(sim.h, sim.levels[0], kind, qs, ps)
            assert e.value.code == Q.QTASK_E_ARG, (kind, qs, ps)
        with pytest.raises(Q.QtaskError) as e:
            Q.qtask_remove_gate(sim.h, 999999)
        assert e.value.code == Q.QTASK_E_NOTFOUND
        with pytest.raises(Q.QtaskError) as e:
            Q.qtask_insert_gate(sim.h, 424242, "h", (1,))
        assert e.value.code == Q.QTASK_E_NOTFOUND
        n_after = ctypes.c_uint64()
        lib.qtask_num_gates(sim.h, ctypes.byref(n_after))
        assert n_after.value == n_before.value == 2
        # reads are unsupported on a plan-only session
        with pytest.raises(Q.QtaskError) as e:
            sim.state()
        assert e.value.code in (Q.QTASK_E_UNSUPPORTED, Q.QTASK_E_STALE)


def test_level_ids_are_stable():
    with plan_only(4) as sim:
        a = sim.add_level()
        b = sim.add_level()
        c = sim.add_level(1)            # between a and b
        assert [Q.qtask_level_at(sim.h, i) for i in range(3)] == [a, c, b]
        Q.qtask_remove_level(sim.h, c)
        assert [Q.qtask_level_at(sim.h, i) for i in range(2)] == [a, b]
        with pytest.raises(Q.QtaskError):
            Q.qtask_remove_level(sim.h, c)


# ----------------------------------------------------------- plan emulation

def _apply_local(psi, n, qs, m):
    """Apply matrix m (first-listed qubit = high local bit) on qubits qs."""
    k = len(qs)
    t = psi.reshape([2] * n)  # axis a <-> qubit n-1-a
    axes = [n - 1 - q for q in qs]
    t = np.moveaxis(t, axes, range(k))
    shp = t.shape
    t = (m @ t.reshape(1 << k, -1)).reshape(shp)
    return np.moveaxis(t, range(k), axes).reshape(-1)


def _relabel(psi, n, qin, qout):
    """Move the amplitude bit at position qin[p] to position qout[p] (a pass
    that stores its tile with the qubits permuted)."""
    if list(qin) == list(qout):
        return psi
    i = np.arange(1 << n, dtype=np.int64)
    j = i.copy()
    for p in qin:
        j &= ~(np.int64(1) << p)
    for p, o in zip(qin, qout):
        j |= ((i >> p) & 1) << o
    out = np.empty_like(psi)
    out[j] = psi
    return out


def emulate(dump, n):
    """Run the dumped plan of every segment on the CPU in complex128: ops on
    the positions they name, then each pass's store permutation; every
    segment must end in the plain layout."""
    for seg in dump["segments"]:
        where = list(range(n))  # circuit qubit at each position
        for ps in seg["passes"]:
            if ps["out"] != ps["qubits"]:
                moved = {o: where[q] for q, o in zip(ps["qubits"], ps["out"])}
                for o, q in moved.items():
                    where[o] = q
        assert where == list(range(n)), "segment does not end in the plain layout"
    return _emulate_ops(dump, n)


def _emulate_ops(dump, n):
    psi = oracle.basis(n).astype(np.complex128)
    for seg in dump["segments"]:
        assert seg["check"] == "", seg["check"]
        for ps in seg["passes"]:
            for st in ps["stages"]:
                if st["dense"]:
                    qs = st["qubits"]
                    U = np.array([complex(a, b) for a, b in st["U"]]).reshape(1 << len(qs), 1 << len(qs))
                    # register convention: bit j of the index <-> qs[j]; as a
                    # local matrix the first-listed qubit is the high bit
                    psi = _apply_local(psi, n, list(reversed(qs)), U)
                else:
                    for op in st["ops"]:
                        m = np.array([complex(a, b) for a, b in op["m"]])
                        d = int(round(np.sqrt(m.size)))
                        psi = _apply_local(psi, n, op["q"], m.reshape(d, d))
            psi = _relabel(psi, n, ps["qubits"], ps["out"])
    return psi


@pytest.mark.parametrize("relabel", [0, 1])
@pytest.mark.parametrize("n,b,c,seed,fam", [
    (5, 4, 2, 1, "dense"), (6, 5, 3, 2, "dense"), (8, 6, 4, 3, "layered"), (9, 6, 3, 4, "dense"),
    (10, 7, 4, 5, "layered"), (10, 10, 4, 6, "dense"), (7, 4, 0, 7, "ladder"), (11, 7, 4, 8, "ladder"),
    (12, 8, 5, 9, "layered")])
def test_planner_emulation_matches_oracle(n, b, c, seed, fam, relabel):
    if fam == "dense":
        nets = W.dense_random_circuit(n, 12, seed, kinds=W.GATE_KINDS)
    elif fam == "layered":
        nets = W.layered_circuit(n, 6, seed)
    else:
        nets = W.cp_ladder_circuit(n, 5, seed)
    with plan_only(n, tile_bits=b, low_bits=c, ckpt_interval=7, relabel=relabel) as sim:
        sim.build(nets)
        sim.update()
        dump = sim.dump()
    got = emulate(dump, n)
    want = oracle.simulate(n, nets)
    np.testing.assert_allclose(got, want, atol=1e-12)
    # every source gate lands in exactly one pass
    assert sum(seg["gates"] for seg in dump["segments"]) == W.count_gates(nets)
    if not relabel:
        assert all(p["out"] == p["qubits"] for seg in dump["segments"] for p in seg["passes"])


def _passes(n, nets, **kw):
    with plan_only(n, **kw) as sim:
        sim.build(nets)
        sim.update()
        return sim.stats()["passes"], sim.dump()


@pytest.mark.parametrize("fam,n,ratio", [("ladder", 32, 0.8), ("layered", 28, 0.95)])
def test_relabelling_lets_wide_low_runs_keep_few_passes(fam, n, ratio):
    """With relabelling, six contiguous low bits (1 KiB runs of complex128)
    cost clearly fewer passes than without, and no more than a quarter above the
    three-bit tiles without relabelling; every pass's store map is a
    permutation of its tile positions, and every tile holds the low
    positions (the emulation test above checks the arithmetic)."""
    nets = W.cp_ladder_circuit(n, 20, 11) if fam == "ladder" else W.layered_circuit(n, 30, 12)
    k = 150 if fam == "ladder" else 100
    plain3, _ = _passes(n, nets, tile_bits=12, low_bits=3, ckpt_interval=k, relabel=0)
    plain6, _ = _passes(n, nets, tile_bits=12, low_bits=6, ckpt_interval=k, relabel=0)
    rel6, dump = _passes(n, nets, tile_bits=12, low_bits=6, ckpt_interval=k, relabel=1)
    assert rel6 < ratio * plain6 and rel6 <= 1.25 * plain3, (plain3, plain6, rel6)
    moved = 0
    for seg in dump["segments"]:
        for p in seg["passes"]:
            assert sorted(p["out"]) == sorted(p["qubits"])
            assert all(q in p["qubits"] for q in range(6))
            moved += p["out"] != p["qubits"]
    assert moved > 0


def test_relabel_default_follows_state_size():
    with plan_only(25) as s:
        assert Q.qtask_get_opts(s.h).relabel == 0
    with plan_only(26) as s:
        assert Q.qtask_get_opts(s.h).relabel == 1
    with pytest.raises(Q.QtaskError):
        plan_only(12, relabel=2)


def test_planner_factors_diagonal_phases():
    """Every one-qubit diagonal runs as diag(1, p); each segment that had one
    ends with a single scalar op holding the product of the factored d0, and
    the plan still reproduces the oracle's state."""
    n = 9
    nets = W.layered_circuit(n, 8, 31)
    with plan_only(n, tile_bits=6, low_bits=2, ckpt_interval=3) as sim:
        sim.build(nets)
        sim.update()
        dump = sim.dump()
    kop_d1, kop_p1, kop_gph = 2, 14, 16
    for seg in dump["segments"]:
        ops = [op for p in seg["passes"] for st in p["stages"] for op in st["ops"]]
        assert not any(op["kop"] == kop_d1 for op in ops)
        gph = [op for op in ops if op["kop"] == kop_gph]
        # the layered family has no native phase gates: every P1 is a factored RZ
        if not any(op["kop"] == kop_p1 for op in ops):
            assert not gph
            continue
        assert len(gph) == 1 and gph[0]["q"] == []
        assert seg["passes"][-1]["stages"][-1]["ops"][-1]["kop"] == kop_gph
        g = complex(*gph[0]["m"][0])
        assert abs(abs(g) - 1.0) < 1e-13
        for op in ops:
            if op["kop"] == kop_p1:
                assert complex(*op["m"][0]) == 1 and abs(abs(complex(*op["m"][3])) - 1.0) < 1e-13
    np.testing.assert_allclose(emulate(dump, n), oracle.simulate(n, nets), atol=1e-12)


@pytest.mark.parametrize("k,b", [(4, 10), (5, 10), (6, 11), (5, 12), (4, 6)])
def test_planner_dense_fusion_emulation(k, b):
    n = 13
    nets = W.layered_circuit(n, 5, 21) + W.dense_random_circuit(n, 4, 22, kinds=W.GATE_KINDS)
    with plan_only(n, tile_bits=b, low_bits=3, fusion=Q.QTASK_FUSE_DENSE, fuse_width=k, ckpt_interval=6) as sim:
        sim.build(nets)
        sim.update()
        dump = sim.dump()
    stages = [st for seg in dump["segments"] for p in seg["passes"] for st in p["stages"]]
    dense = [st for st in stages if st["dense"]]
    assert dense and all(len(st["qubits"]) == k for st in dense)
    if b >= 10:
        assert all(st["mfma"] for st in dense)
    for st in dense:
        U = np.array([complex(a, c) for a, c in st["U"]]).reshape(1 << k, 1 << k)
        np.testing.assert_allclose(U @ U.conj().T, np.eye(1 << k), atol=1e-13)
    np.testing.assert_allclose(emulate(dump, n), oracle.simulate(n, nets), atol=1e-12)


def test_dense_fusion_needs_large_tiles():
    with pytest.raises(Q.QtaskError) as e:
        plan_only(8, fusion=Q.QTASK_FUSE_DENSE, fuse_width=5)
    assert e.value.code == Q.QTASK_E_UNSUPPORTED


def test_planner_auto_fusion_makes_dense_stages():
    # deep circuit on 4 qubits: every stage is long enough to fuse
    rng = np.random.default_rng(11)
    nets = []
    for _ in range(40):
        nets.append([("ry", (q,), (float(rng.uniform(0, 6)),)) for q in range(4)])
        nets.append([("cx", (0, 1), ()), ("cx", (2, 3), ())])
        nets.append([("cz", (1, 2), ())])
    with plan_only(4, tile_bits=4, low_bits=0, ckpt_interval=1000) as sim:
        sim.build(nets)
        sim.update()
        dump = sim.dump()
    dense = [st for seg in dump["segments"] for p in seg["passes"] for st in p["stages"] if st["dense"]]
    assert dense, "expected fused dense stages"
    np.testing.assert_allclose(emulate(dump, 4), oracle.simulate(4, nets), atol=1e-12)


# ------------------------------------------------------------------ tracker

def _worked():
    with open(os.path.join(GOLDEN, "worked_example.json")) as f:
        gold = json.load(f)
    nets = [[(g[0], tuple(g[1]), ()) for g in net] for net in gold["nets"]]
    return gold, nets


def test_worked_example_dirty_blocks():
    gold, nets = _worked()
    with plan_only(gold["n"], block_bits=gold["block_bits"], ckpt_interval=1) as sim:
        sim.build(nets)
        st = sim.update()
        assert st["mode"] == 1
        i, j = gold["gate_names"]["G8"]
        sim.apply_edit(W.Edit("remove", i, pos=j))
        sim.apply_edit(W.Edit("insert", i, (gold["g10"][0], tuple(gold["g10"][1]), ())))
        st = sim.update()
        assert st["mode"] == 3
        assert st["dirty_blocks"] == len(gold["dirty_blocks_after_edits"])
        dump = sim.dump()
        assert dump["dirty_block_list"] == gold["dirty_blocks_after_edits"]
        # updated amplitudes = the paper's 24
        bb = gold["block_bits"]
        amps = [a for blk in dump["dirty_block_list"] for a in range(blk << bb, (blk + 1) << bb)]
        assert len(amps) == gold["updated_amplitude_count"]
        # replay starts at the checkpoint right before the edited net
        assert st["first_level"] == i


def test_worked_example_without_checkpoints_replays_everything():
    gold, nets = _worked()
    with plan_only(gold["n"], block_bits=gold["block_bits"], ckpt_interval=1, max_ckpts=0) as sim:
        sim.build(nets)
        sim.update()
        i, j = gold["gate_names"]["G8"]
        sim.apply_edit(W.Edit("remove", i, pos=j))
        st = sim.update()
        # the Hadamard net couples every block, so without a checkpoint after
        # it the affected set is not closed and the whole state is redone
        assert st["mode"] == 2 and st["first_level"] == 0


def test_cancelling_edits_redo_nothing():
    gold, nets = _worked()
    with plan_only(gold["n"], block_bits=2, ckpt_interval=1) as sim:
        sim.build(nets)
        sim.update()
        sim.apply_edit(W.Edit("remove", 3, pos=0))
        sim.apply_edit(W.Edit("insert", 3, nets[3][0]))
        st = sim.update()
        assert st["mode"] == 3 and st["dirty_blocks"] == 0 and st["tiles"] == 0


@pytest.mark.parametrize("relabel", [0, 1])
@pytest.mark.parametrize("seed", range(6))
def test_tracker_sound_against_oracle(seed, relabel):
    """Blocks whose amplitudes actually change (at every checkpoint boundary
    and at the end) lie inside the tracker's affected set (with and without
    relabelling passes, whose store permutations move amplitude between
    blocks)."""
    rng = np.random.default_rng(seed)
    n, bb, K = 7, 3, 2
    kinds = ("x", "cx", "ccx", "swap", "z", "s", "t", "cz", "cp", "h", "rx")
    nets = W.dense_random_circuit(n, 10, 50 + seed, kinds=("x", "cx", "z", "s", "cz", "swap", "t"))
    with plan_only(n, block_bits=bb, ckpt_interval=K, tile_bits=5, low_bits=2, relabel=relabel) as sim:
        sim.build(nets)
        sim.update()
        for trial in range(4):
            old = [list(x) for x in nets]
            li = int(rng.integers(len(nets)))
            if nets[li] and rng.random() < 0.5:
                e = W.Edit("remove", li, pos=int(rng.integers(len(nets[li]))))
            else:
                free = [q for q in range(n) if all(q not in g[1] for g in nets[li])]
                kind = kinds[int(rng.integers(len(kinds)))]
                k = W.N_QUBITS[kind]
                if len(free) < k:
                    continue
                qs = tuple(int(q) for q in rng.choice(free, size=k, replace=False))
                e = W.Edit("insert", li, (kind, qs, tuple(rng.uniform(0, 6, W.N_PARAMS[kind]))))
            W.apply_edit(nets, e)
            sim.apply_edit(e)
            st = sim.update()
            a = oracle.snapshots(n, old)
            b = oracle.snapshots(n, nets)
            if st["mode"] == 3:
                dirty = set(sim.dump()["dirty_block_list"])
                for lv in range(len(nets) + 1):
                    if lv % K == 0 or lv == len(nets):
                        assert oracle.changed_blocks(a[lv], b[lv], bb) <= dirty, (trial, lv)
            else:
                assert st["mode"] == 2


@pytest.mark.parametrize("seed", range(6))
def test_tracker_sound_under_level_removal(seed):
    """Removing whole levels, including the ones that end a segment (which
    merges two segments): the blocks that actually change still lie inside
    the affected set whenever the update restricts itself to it."""
    rng = np.random.default_rng(seed)
    n, bb, K = 7, 3, 2
    nets = W.dense_random_circuit(n, 14, 70 + seed, kinds=("x", "cx", "z", "s", "cz", "swap", "t", "h"))
    with plan_only(n, block_bits=bb, ckpt_interval=K, tile_bits=5, low_bits=2) as sim:
        sim.build(nets)
        sim.update()
        modes = []
        for trial in range(8):
            if len(nets) < 2:
                break
            old = [list(x) for x in nets]
            li = int(rng.integers(len(nets)))
            del nets[li]
            sim.remove_level(li)
            st = sim.update()
            modes.append(st["mode"])
            if st["mode"] == 3:
                a = oracle.snapshots(n, old)[-1]
                b = oracle.snapshots(n, nets)[-1]
                dirty = set(sim.dump()["dirty_block_list"])
                assert oracle.changed_blocks(a, b, bb) <= dirty, (trial, li)
            else:
                assert st["mode"] == 2


def test_level_removal_inside_a_segment_stays_closed():
    """Removing a level that does not end its segment keeps the restricted
    replay available, and its affected set covers what actually changes."""
    n, bb = 7, 3
    nets = [[("h", (q,), ()) for q in range(n)]]
    nets += [[("cx", (6, 5), ())], [("z", (1,), ()), ("t", (4,), ())], [("cz", (2, 6), ())], [("s", (3,), ())],
             [("t", (5,), ())], [("cz", (0, 4), ())], [("z", (6,), ())], [("s", (5,), ())]]
    with plan_only(n, block_bits=bb, ckpt_interval=4, tile_bits=5, low_bits=2) as sim:
        sim.build(nets)
        sim.update()
        old = [list(x) for x in nets]
        del nets[4]
        sim.remove_level(4)
        st = sim.update()
        assert st["mode"] == 3
        dirty = set(sim.dump()["dirty_block_list"])
        changed = oracle.changed_blocks(oracle.snapshots(n, old)[-1], oracle.snapshots(n, nets)[-1], bb)
        assert changed and changed <= dirty and len(dirty) < 1 << (n - bb)


def test_tracker_sees_a_merged_phase_change_sign():
    """Removing a Z from a qubit that also carries a T turns their merged phase
    e^{i pi/4} * -1 into e^{i pi/4}: real and imaginary parts both change
    sign.  The per-block identities must tell the two plans apart (a hash
    whose step is xor-then-multiply does not: the two top-bit flips cancel),
    so the restricted replay covers the blocks that change."""
    n, bb = 7, 3
    nets = [[("h", (q,), ()) for q in range(n)]]
    nets += [[("cx", (6, 5), ())], [("s", (3,), ())], [("cz", (0, 4), ())], [("t", (6,), ())],
             [("z", (6,), ())], [("t", (5,), ())], [("z", (2,), ())], [("s", (5,), ())]]
    with plan_only(n, block_bits=bb, ckpt_interval=4, tile_bits=5, low_bits=2) as sim:
        sim.build(nets)
        sim.update()
        old = [list(x) for x in nets]
        del nets[5]
        sim.remove_level(5)
        st = sim.update()
        assert st["mode"] == 3
        dirty = set(sim.dump()["dirty_block_list"])
        changed = oracle.changed_blocks(oracle.snapshots(n, old)[-1], oracle.snapshots(n, nets)[-1], bb)
        assert changed and changed <= dirty


def test_tracker_couples_blocks_through_a_fused_near_identity():
    """Two H on a block qubit fuse into one real 2x2 whose off-diagonal
    entries are exactly zero.  The kernel still reads the partner amplitude
    (0 * x decides the sign of a zero result), so a restricted replay must not
    pair a recomputed block with a partner it leaves stale: after the CZ on
    that qubit is removed, either the replay is not restricted or its block
    set is closed under the pairing and covers what changed."""
    n, bb = 7, 3
    nets = [[("h", (q,), ()) for q in range(n)]]
    nets += [[("cx", (5, 4), ())], [("s", (3,), ())], [("cz", (0, 4), ())], [("h", (6,), ())],
             [("h", (6,), ())], [("cz", (6, 1), ())], [("t", (2,), ())], [("s", (5,), ())]]
    with plan_only(n, block_bits=bb, ckpt_interval=4, tile_bits=5, low_bits=2) as sim:
        sim.build(nets)
        sim.update()
        ops = [(o["kop"], o["gate"], o["q"]) for seg in sim.dump()["segments"] for p in seg["passes"]
               for st in p["stages"] for o in st["ops"]]
        assert (12, 0, [6]) in ops  # the fused H.H
        old = [list(x) for x in nets]
        del nets[6]
        sim.remove_level(6)
        st = sim.update()
        if st["mode"] == 3:
            dirty = set(sim.dump()["dirty_block_list"])
            pair = 1 << (6 - bb)
            assert all(j ^ pair in dirty for j in dirty)
            changed = oracle.changed_blocks(oracle.snapshots(n, old)[-1], oracle.snapshots(n, nets)[-1], bb)
            assert changed <= dirty


def test_segments_survive_a_full_rerun_after_level_removal():
    """The segment cut depends on the circuit and the anchor set only and is
    stable under a second run: after levels are inserted and the last one is
    removed (leaving an anchor on the new last level), the incremental update
    and the full re-simulation after it plan the same segments, which is what
    keeps their results bitwise equal."""
    n = 6
    nets = [[("h", (q % n,), ())] for q in range(7)]
    with plan_only(n, ckpt_interval=2, tile_bits=5, low_bits=2) as sim:
        sim.build(nets)
        sim.update()
        g = ("rz", (1,), (0.3,))
        nets.insert(5, [g])
        sim.add_level(5)
        sim.add_gate(5, g)
        sim.update()
        del nets[7]
        sim.remove_level(7)
        sim.update()
        inc = json.dumps(sim.dump()["segments"])
        sim.update(full=True)
        assert json.dumps(sim.dump()["segments"]) == inc
    # random edit sequences with level removals
    for seed in (28, 40, 209, 224):
        rng = np.random.default_rng(seed)
        nets = W.cp_ladder_circuit(8, 6, 903 + seed)
        with plan_only(8, ckpt_interval=2 + seed % 3, tile_bits=6, low_bits=3) as sim:
            sim.build(nets)
            sim.update()
            for _ in range(20):
                if rng.random() < 0.3 and len(nets) > 2:
                    li = int(rng.integers(len(nets)))
                    del nets[li]
                    sim.remove_level(li)
                else:
                    e = W.random_edit(rng, 8, nets, ("rx", "rz", "cp"))
                    W.apply_edit(nets, e)
                    sim.apply_edit(e)
                sim.update()
                inc = json.dumps(sim.dump()["segments"])
                sim.update(full=True)
                assert json.dumps(sim.dump()["segments"]) == inc


def test_plan_dump_as_graphviz(tmp_path):
    """A dump path ending in .dot gives the pass graph: one cluster per
    segment, one node per pass (the same passes as the JSON dump), edges in
    execution order, and the segment boundaries marked as checkpoints."""
    wl = W.config(2, n=12, levels=20, batches=1)
    with plan_only(12, ckpt_interval=8, tile_bits=8, low_bits=3) as sim:
        sim.build(wl.nets)
        sim.update()
        segs = sim.dump()["segments"]
        path = str(tmp_path / "plan.dot")
        Q.qtask_dump_plan(sim.h, path)
        txt = open(path).read()
    assert txt.startswith("digraph qtask {") and txt.rstrip().endswith("}")
    n_pass = sum(len(s["passes"]) for s in segs)
    assert txt.count("subgraph cluster_s") == len(segs)
    assert len(re.findall(r'p\d+_\d+ \[label="pass', txt)) == n_pass
    assert len(re.findall(r"p\d+_\d+ -> p\d+_\d+", txt)) == n_pass - 1
    assert txt.count('label="checkpoint"') == len(segs) - 1
    for s, seg in enumerate(segs):
        for p, ps in enumerate(seg["passes"]):
            line = next(l for l in txt.splitlines() if l.strip().startswith("p%d_%d [" % (s, p)))
            assert "qubits " + " ".join(str(q) for q in ps["qubits"]) in line
            assert line.count("ops\\l") == len(ps["stages"])


def test_abi_from_plain_c(tmp_path):
    """A C11 program includes the header and links the library directly:
    the modifier, update and query cycle of a plan-only session, with the
    documented status codes."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    libdir = os.path.dirname(Q.LIB_PATH)
    exe = str(tmp_path / "abi")
    subprocess.run([cc, "-std=c11", "-Wall", "-Werror", "-I", os.path.join(root, "include"),
                    os.path.join(root, "tests", "abi_plan_only.c"), "-L", libdir, "-lqtask",
                    "-Wl,-rpath," + libdir, "-o", exe], check=True)
    dot = str(tmp_path / "plan.dot")
    out = subprocess.run([exe, dot], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "FAIL" not in out.stdout and out.stdout.count("ok ") >= 20
    assert open(dot).read().startswith("digraph qtask {")


def test_server_opts_and_edit_records():
    o = Q.qtask_server_opts_default()
    assert o.struct_size == Q.ctypes.sizeof(Q.qtask_server_opts)
    assert o.budget_bytes == 256 << 30 and o.small_qubits == 16 and o.max_inflight >= 1 and o.use_graph == 1
    assert o.order == 0
    ins = W.Edit(op="insert", net=3, gate=("cp", (1, 4), (0.5,)), new_net=True)
    recs = Q.make_edits(ins)
    assert [r.op for r in recs] == [2, 0]
    assert recs[0].level == 3 and recs[1].level == 4
    assert recs[1].kind == Q.KIND["cp"] and recs[1].nq == 2 and list(recs[1].qubits)[:2] == [1, 4]
    assert recs[1].np == 1 and recs[1].params[0] == 0.5
    rem = Q.make_edits(W.Edit(op="remove", net=7, pos=2))
    assert len(rem) == 1 and rem[0].op == 1 and rem[0].level == 7 and rem[0].gate_index == 2


def test_server_needs_a_device():
    if Q.qtask_device_count() > 0:
        pytest.skip("a device is present")
    with pytest.raises(Q.QtaskError) as ei:
        Q.qtask_server_create()
    assert ei.value.code == Q.QTASK_E_DEVICE
    bad = Q.qtask_server_opts_default(max_inflight=0)
    with pytest.raises(Q.QtaskError) as ei:
        Q.qtask_server_create(bad)
    assert ei.value.code == Q.QTASK_E_ARG


# ------------------------------------------------- kernel-side emulation

def _xor_bits(vals, idx, nbits):
    """XOR (or OR: the contributions are disjoint) of vals[k] over the set
    bits k of idx (vectorised over idx)."""
    out = np.zeros_like(idx, dtype=np.int64)
    for k in range(nbits):
        out ^= np.where((idx >> k) & 1, np.int64(vals[k]), np.int64(0))
    return out


def _site_rows(site, t, base, nthr):
    """Lanes where a phase op's lane or origin site holds."""
    if site == 255:
        return np.ones(nthr, dtype=bool)
    if site < 64:
        return ((t.ravel() >> (site - 16)) & 1) == 1
    return np.full(nthr, bool((base >> (site - 64)) & 1))


def _apply_kop(a, op, coefs, t=None, base=0, ph=None):
    """One op record on the register block a (threads x 16), as the pass
    kernel's op switch applies it (register bits A, B, C; coefficients at
    `coef` in the coefficient array; t the thread indices, base the tile
    origin, for phases conditioned on lane or origin bits; ph the lanes'
    pending phase factors)."""
    ty, A, B, Cb, off = op
    c = coefs[off:off + 512]
    idx = np.arange(16)
    cx = lambda k: complex(c[2 * k], c[2 * k + 1])
    if ty == 16:  # GPH
        a *= cx(0)
        return
    if ty == 17:  # PC: phase on the registers with bit A set, where site B holds
        rows = _site_rows(B, t, base, a.shape[0])
        a[np.ix_(rows, ((idx >> A) & 1) == 1)] *= cx(0)
        return
    if ty == 18:  # PCL: phase into the pending factor of the lanes where both sites hold
        rows = _site_rows(A, t, base, a.shape[0]) & _site_rows(B, t, base, a.shape[0])
        ph["f"][rows] *= cx(0)
        ph["hit"] |= rows
        return
    if ty == 19:  # PHI: apply and reset the pending factors
        a[ph["hit"]] *= ph["f"][ph["hit"], None]
        ph["f"][:] = 1
        ph["hit"][:] = False
        return
    if ty == 11:  # DENSE
        U = (c[0:512:2] + 1j * c[1:512:2]).reshape(16, 16)
        a[:] = a @ U.T
        return
    bitA = (idx >> A) & 1
    if ty in (12, 13, 1):  # UR, UX, U1 on pairs
        lo = idx[bitA == 0]
        hi = lo | (1 << A)
        x, y = a[:, lo].copy(), a[:, hi].copy()
        if ty == 12:
            m = [c[0], c[1], c[2], c[3]]
        elif ty == 13:
            m = [c[0], 1j * c[1], 1j * c[2], c[3]]
        else:
            m = [cx(0), cx(1), cx(2), cx(3)]
        a[:, lo] = m[0] * x + m[1] * y
        a[:, hi] = m[2] * x + m[3] * y
    elif ty == 2:  # D1
        a[:, bitA == 0] *= cx(0)
        a[:, bitA == 1] *= cx(1)
    elif ty == 14:  # P1
        a[:, bitA == 1] *= cx(0)
    elif ty == 15:  # P2
        a[:, (bitA == 1) & (((idx >> B) & 1) == 1)] *= cx(0)
    elif ty in (3, 4):  # A1, X1
        lo = idx[bitA == 0]
        hi = lo | (1 << A)
        x, y = a[:, lo].copy(), a[:, hi].copy()
        if ty == 4:
            a[:, lo], a[:, hi] = y, x
        else:
            a[:, lo], a[:, hi] = cx(0) * y, cx(1) * x
    elif ty == 6:  # CX: control A, target B
        sel = idx[(bitA == 1) & (((idx >> B) & 1) == 0)]
        x, y = a[:, sel].copy(), a[:, sel | (1 << B)].copy()
        a[:, sel], a[:, sel | (1 << B)] = y, x
    elif ty == 8:  # SWAP
        sel = idx[(bitA == 1) & (((idx >> B) & 1) == 0)]
        oth = (sel & ~(1 << A)) | (1 << B)
        x, y = a[:, sel].copy(), a[:, oth].copy()
        a[:, sel], a[:, oth] = y, x
    elif ty == 10:  # CCX: controls A, B, target C
        sel = idx[(bitA == 1) & (((idx >> B) & 1) == 1) & (((idx >> Cb) & 1) == 0)]
        x, y = a[:, sel].copy(), a[:, sel | (1 << Cb)].copy()
        a[:, sel], a[:, sel | (1 << Cb)] = y, x
    else:
        raise AssertionError("op type %d" % ty)


def _mfma_operand(coefs, off, k):
    """The complex unitary of a matrix-core stage, decoded from its operand:
    the real block matrix M = [[Ur, -Ui], [Ui, Ur]] in the order the 16x16x4
    matrix instructions read it (in inner step s, lane l holds row
    16 rb + l % 16, column 4 s + l // 16 of M for each row block rb, stored
    at (s * 64 + l) * RB + rb).  Checks the block structure on the way."""
    dim = 1 << k
    mr = 2 * dim
    rbn, steps = mr // 16, mr // 4
    assert off % 16 == 0, "operand offset must allow aligned vector loads"
    blk = np.asarray(coefs[off:off + mr * mr], dtype=np.float64)
    assert blk.size == mr * mr
    M = np.full((mr, mr), np.nan)
    lane = np.arange(64)
    for s_ in range(steps):
        for rb in range(rbn):
            M[16 * rb + (lane & 15), 4 * s_ + (lane >> 4)] = blk[(s_ * 64 + lane) * rbn + rb]
    assert not np.isnan(M).any()
    Ur, Ui = M[:dim, :dim], M[dim:, :dim]
    assert np.array_equal(M[dim:, dim:], Ur) and np.array_equal(M[:dim, dim:], -Ui)
    return Ur + 1j * Ui


def emulate_kernel(dump, n):
    """Run the plan blobs the way the pass kernel does, tile by tile: the
    tile origin from the deposit runs, the first stage's registers loaded
    through its global maps, the op records on registers, LDS exchanges
    through the swizzled slot maps, matrix-core stages on LDS, and the last
    stage's registers stored through its own global maps.  Every load and
    store address is checked to lie inside the state, and every state slot
    to be written exactly once per pass."""
    psi = oracle.basis(n).astype(np.complex128)
    for seg in dump["segments"]:
        b = seg["b"]
        coefs = np.array(seg["coefs"], dtype=np.float64)
        nthr = 1 << (b - 4)
        t = np.arange(nthr, dtype=np.int64)[:, None]
        reg = np.arange(16, dtype=np.int64)[None, :]
        for ps in seg["passes"]:
            kp = ps["kernel"]
            out = np.zeros_like(psi)
            written = np.zeros(psi.size, dtype=np.int64)
            stages = kp["stages"]
            for tile in range(1 << (n - b)):
                base = 0
                for r in kp["runs"]:
                    src, ln, dst = r & 0xFF, (r >> 8) & 0xFF, r >> 16
                    base |= ((tile >> src) & ((1 << ln) - 1)) << dst
                lds = np.zeros(1 << b, dtype=np.complex128)
                ph = {"f": np.ones(nthr, dtype=np.complex128), "hit": np.zeros(nthr, dtype=bool)}
                for si, S in enumerate(stages):
                    if S["kind"] == 1:  # dense unitary on LDS
                        U = _mfma_operand(coefs, S["coef"], S["k"])
                        cols = _xor_bits(S["col_off"], np.arange(1 << len(S["col_off"]), dtype=np.int64),
                                         len(S["col_off"]))
                        slots = np.array(S["row_off"], dtype=np.int64)[:, None] ^ cols[None, :]
                        lds[slots] = U @ lds[slots]
                        continue
                    bt = _xor_bits(S["thr_off"], t, kp["n_thr"])
                    sl = bt ^ _xor_bits(S["reg_bit"], reg, 4)
                    if si == 0:
                        g = base | _xor_bits(S["g_thr"], t, kp["n_thr"]) | _xor_bits(S["g_bit"], reg, 4)
                        assert g.min() >= 0 and g.max() < psi.size
                        a = psi[g].copy()
                    else:
                        a = lds[sl].copy()
                    for op in S["ops"]:
                        _apply_kop(a, op, coefs, t, base, ph)
                    assert not ph["hit"].any(), "a pending phase outlives its stage"
                    if si + 1 == len(stages):
                        g = base | _xor_bits(S["g_thr"], t, kp["n_thr"]) | _xor_bits(S["g_bit"], reg, 4)
                        assert g.min() >= 0 and g.max() < psi.size
                        out[g] = a
                        np.add.at(written, g.ravel(), 1)
                    else:
                        lds[sl] = a
            assert np.all(written == 1), "a pass must write every amplitude exactly once"
            psi = out
    return psi


@pytest.mark.parametrize("relabel", [0, 1])
@pytest.mark.parametrize("n,b,c,fam,fusion,k", [
    (8, 6, 2, "dense", 1, 0), (9, 6, 3, "layered", 1, 0), (10, 7, 4, "ladder", 1, 0), (11, 7, 5, "layered", 1, 0),
    (10, 6, 4, "dense", 0, 0), (12, 10, 3, "layered", 2, 5), (11, 10, 3, "layered", 2, 4),
    (12, 11, 3, "dense", 2, 6)])
def test_kernel_emulation_of_plan_blobs_matches_oracle(n, b, c, fam, fusion, k, relabel):
    """The blobs the kernel reads (maps, op records, coefficients) give the
    oracle's state when run as the kernel runs them, with and without
    relabelling passes, for list stages, dense 16x16 stages and matrix-core
    stages."""
    if fam == "dense":
        nets = W.dense_random_circuit(n, 10, 90 + n, kinds=W.GATE_KINDS)
    elif fam == "layered":
        nets = W.layered_circuit(n, 6, 91 + n)
    else:
        nets = W.cp_ladder_circuit(n, 4, 92 + n)
    kw = dict(tile_bits=b, low_bits=c, ckpt_interval=5, relabel=relabel, fusion=fusion)
    if fusion == 2:
        kw["fuse_width"] = k
    with plan_only(n, **kw) as sim:
        sim.build(nets)
        sim.update()
        dump = sim.dump()
    np.testing.assert_allclose(emulate_kernel(dump, n), oracle.simulate(n, nets), atol=1e-12)


# ------------------------------------------------------ sparse checkpoints

def _sparse_net(rng, n):
    """One gate controlled on (or a phase with) the top qubit n-1, its other
    qubits drawn below: it changes only the blocks whose top bit is 1."""
    kind = ("ccx", "cx", "cp", "cz")[int(rng.integers(4))]
    rest = [int(q) for q in rng.choice(n - 1, size=2 if kind == "ccx" else 1, replace=False)]
    return [(kind, tuple([n - 1] + rest), (float(rng.uniform(0, 6)),) if kind == "cp" else ())]


@pytest.mark.parametrize("seed,max_ckpts", [(0, -1), (1, -1), (2, 2), (3, 3)])
def test_sparse_checkpoints_hold_every_changed_block(seed, max_ckpts):
    """With sparse checkpoints on, each stored boundary's checkpoint lists
    the blocks the segments since the previous stored boundary can change;
    the blocks that actually change between consecutive stored boundaries
    (oracle snapshots) lie among them, and the checkpoints hold fewer bytes
    than whole copies.  With max_ckpts the stored boundaries thin out and
    each checkpoint covers several segments."""
    rng = np.random.default_rng(40 + seed)
    n, bb, K = 9, 3, 3
    prep = [[("h", (q,), ()) for q in range(n)]]
    nets = prep + [_sparse_net(rng, n) for _ in range(20)]
    with plan_only(n, block_bits=bb, ckpt_interval=K, tile_bits=6, low_bits=2, ckpt_delta=1,
                   max_ckpts=max_ckpts) as sim:
        sim.build(nets)
        st = sim.update()
        dump = sim.dump()
    snaps = oracle.snapshots(n, nets)
    cks = dump["checkpoints"]
    if max_ckpts < 0:
        assert len(cks) == len(dump["segments"]) - 1
    else:
        assert 0 < len(cks) <= max_ckpts
    sparse = 0
    prev = 0
    for ck in cks:
        lvl = ck["level"]
        changed = oracle.changed_blocks(snaps[prev], snaps[lvl], bb)
        held = set(range(1 << (n - bb))) if ck["full"] else set(ck["blocks"])
        assert changed <= held, (ck["boundary"], sorted(changed - held))
        sparse += not ck["full"]
        prev = lvl
    assert sparse > 0
    assert st["ckpt_bytes"] < st["ckpt_full_bytes"]


def test_sparse_checkpoints_are_whole_on_layered_circuits():
    n = 10
    nets = W.layered_circuit(n, 8, 5)
    with plan_only(n, block_bits=4, ckpt_interval=4, ckpt_delta=1) as sim:
        sim.build(nets)
        st = sim.update()
        dump = sim.dump()
    assert all(ck["full"] for ck in dump["checkpoints"])
    assert st["ckpt_bytes"] == st["ckpt_full_bytes"] > 0
