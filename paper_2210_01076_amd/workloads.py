"""Seeded synthetic circuits and modifier streams.

This module only draws random structure (gate kinds, qubits, angles, edit
positions) and keeps the circuit as nested lists; it performs none of the
simulation arithmetic.  Both the CPU oracle (through the tests) and the GPU
library (through the binding) consume what it produces, so the two sides see
the same inputs without sharing any code.

A circuit is a list of nets (the paper's "net": a set of gates on disjoint
qubits, Section III-B).  A gate is a tuple ``(kind, qubits, params)``:

* ``kind`` is a lower-case name from ``GATE_KINDS``;
* ``qubits`` lists controls first, then the target(s), as in OpenQASM;
* ``params`` holds the rotation angles in radians.

Qubit ``k`` is bit ``k`` of the amplitude index (the paper makes the last
qubit the most significant bit, Section III-B).

The workload recipes follow the benchmark configurations of this project:
layered random circuits (rotation net + CNOT matching net), controlled-phase
ladders, and random insert/remove modifiers at uniform levels.  The paper's
own QASMBench circuits are not available; these seeded circuits stand in for
them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

Gate = Tuple[str, Tuple[int, ...], Tuple[float, ...]]
Net = List[Gate]

ONE_QUBIT = ("h", "x", "y", "z", "s", "sdg", "t", "tdg", "rx", "ry", "rz")
TWO_QUBIT = ("cx", "cz", "swap", "cp")
THREE_QUBIT = ("ccx",)
GATE_KINDS = ONE_QUBIT + TWO_QUBIT + THREE_QUBIT
N_PARAMS = {k: 0 for k in GATE_KINDS}
N_PARAMS.update({"rx": 1, "ry": 1, "rz": 1, "cp": 1})
N_QUBITS = {k: 1 for k in ONE_QUBIT}
N_QUBITS.update({k: 2 for k in TWO_QUBIT})
N_QUBITS.update({k: 3 for k in THREE_QUBIT})

#: gate kinds drawn by the small dense configuration (n=10, 20 levels)
CFG1_KINDS = ("h", "x", "y", "z", "s", "t", "rx", "ry", "rz", "cx", "cz", "swap")
#: gate kinds drawn by modifiers on layered circuits
LAYERED_EDIT_KINDS = ("rx", "ry", "rz", "cx")

TWO_PI = 2.0 * math.pi


def seed_for(cfg: int, kind: str = "circuit") -> int:
    """Seeds: 1000+cfg for circuits, 2000+cfg for modifiers, 3000+s for
    serving session s."""
    base = {"circuit": 1000, "modifier": 2000, "session": 3000}[kind]
    return base + cfg


def _gate(rng: np.random.Generator, kind: str, qubits: Sequence[int]) -> Gate:
    params = tuple(float(rng.uniform(0.0, TWO_PI)) for _ in range(N_PARAMS[kind]))
    return (kind, tuple(int(q) for q in qubits), params)


# --------------------------------------------------------------------------
# circuit families
# --------------------------------------------------------------------------

def dense_random_circuit(n: int, levels: int, seed: int,
                         kinds: Sequence[str] = CFG1_KINDS) -> List[Net]:
    """Every qubit gets one gate per net.  Qubits are visited in a seeded
    random order; a drawn multi-qubit kind also takes the next unvisited
    qubits (control first); when too few qubits are left a one-qubit kind is
    drawn instead."""
    rng = np.random.default_rng(seed)
    one = [k for k in kinds if N_QUBITS[k] == 1]
    nets: List[Net] = []
    for _ in range(levels):
        order = [int(q) for q in rng.permutation(n)]
        net: Net = []
        i = 0
        while i < n:
            kind = str(kinds[int(rng.integers(len(kinds)))])
            if i + N_QUBITS[kind] > n:
                kind = str(one[int(rng.integers(len(one)))])
            k = N_QUBITS[kind]
            net.append(_gate(rng, kind, order[i:i + k]))
            i += k
        nets.append(net)
    return nets


def layered_circuit(n: int, levels: int, seed: int) -> List[Net]:
    """Each level: RX/RY/RZ with uniform angles on every qubit (one net), then
    CNOTs on a random perfect matching (a second net: a random permutation
    paired consecutively, control first).  With odd n one qubit idles."""
    rng = np.random.default_rng(seed)
    nets: List[Net] = []
    for _ in range(levels):
        rot: Net = []
        for q in range(n):
            kind = ("rx", "ry", "rz")[int(rng.integers(3))]
            rot.append(_gate(rng, kind, (q,)))
        perm = [int(q) for q in rng.permutation(n)]
        ent: Net = [("cx", (perm[2 * i], perm[2 * i + 1]), ()) for i in range(n // 2)]
        nets.append(rot)
        nets.append(ent)
    return nets


def cp_ladder_circuit(n: int, levels: int, seed: int) -> List[Net]:
    """Each level: RX/RY/RZ on every qubit, then controlled-phase gates on
    adjacent pairs, split into an even-pair net and an odd-pair net (the
    phases commute, so the split is exact).  Angles are uniform."""
    rng = np.random.default_rng(seed)
    nets: List[Net] = []
    for _ in range(levels):
        rot: Net = []
        for q in range(n):
            kind = ("rx", "ry", "rz")[int(rng.integers(3))]
            rot.append(_gate(rng, kind, (q,)))
        even = [_gate(rng, "cp", (q, q + 1)) for q in range(0, n - 1, 2)]
        odd = [_gate(rng, "cp", (q, q + 1)) for q in range(1, n - 1, 2)]
        nets.extend([rot, even, odd])
    return nets


def brickwork_circuit(n: int, layers: int, seed: int) -> List[Net]:
    """Random two-qubit unitaries on adjacent pairs, in bricks: even pairs
    (0,1), (2,3), ... in even layers, odd pairs (1,2), (3,4), ... in odd
    layers.  Each brick is a generic two-qubit unitary written with
    rotations and CNOTs (Z-Y-Z rotations on both qubits, three CNOTs
    alternating in direction with RY/RZ between them, Z-Y-Z rotations
    again), uniform angles; the bricks of a layer run in parallel, 9 nets
    per layer.  Many non-diagonal gates act on few qubits between their
    couplings to the rest: the workload where dense fusion pays."""
    rng = np.random.default_rng(seed)
    nets: List[Net] = []

    def zyz(qs):
        return [[_gate(rng, k, (q,)) for q in qs] for k in ("rz", "ry", "rz")]

    for layer in range(layers):
        pairs = [(q, q + 1) for q in range(layer % 2, n - 1, 2)]
        lo = [q for a, b in pairs for q in (a, b)]
        body: List[Net] = zyz(lo)
        body.append([("cx", (a, b), ()) for a, b in pairs])
        body.append([g for a, b in pairs for g in (_gate(rng, "ry", (a,)), _gate(rng, "rz", (b,)))])
        body.append([("cx", (b, a), ()) for a, b in pairs])
        body.append([_gate(rng, "ry", (a,)) for a, b in pairs])
        body.append([("cx", (a, b), ()) for a, b in pairs])
        body += zyz(lo)
        nets.extend(body)
    return nets


def blocked_circuit(n: int, levels: int, seed: int, block: int = 5, mix_every: int = 16) -> List[Net]:
    """Qubits in blocks of `block` neighbours.  Each level: a random RX/RY/RZ
    on every qubit, then CZ on the even and then the odd adjacent pairs
    inside each block; every `mix_every` levels a CNOT joins each block's
    last qubit to the next block's first.  Blocks evolve on their own for
    long stretches, as in circuits built from subsystem unitaries with
    sparse couplings: a dense unitary over one block absorbs many levels."""
    rng = np.random.default_rng(seed)
    nets: List[Net] = []
    starts = list(range(0, n, block))
    for lv in range(levels):
        nets.append([_gate(rng, ("rx", "ry", "rz")[int(rng.integers(3))], (q,)) for q in range(n)])
        for par in (0, 1):
            net = [("cz", (q, q + 1), ()) for s0 in starts for q in range(s0 + par, min(s0 + block, n) - 1, 2)]
            if net:
                nets.append(net)
        if (lv + 1) % mix_every == 0:
            nets.append([("cx", (s0 + block - 1, s0 + block), ()) for s0 in starts if s0 + block < n])
    return nets


def top_controlled_circuit(n: int, levels: int, seed: int) -> List[Net]:
    """An H layer, then one gate per level that hinges on the top qubit: a CX
    or CCX controlled on it, or a CP or CZ with it, the other qubits drawn
    below.  Each level changes only the amplitudes whose top bit is 1 (half
    of the blocks), the case sparse checkpoints are for."""
    rng = np.random.default_rng(seed)
    nets: List[Net] = [[("h", (q,), ()) for q in range(n)]]
    for _ in range(levels):
        kind = ("ccx", "cx", "cp", "cz")[int(rng.integers(4))]
        rest = [int(q) for q in rng.choice(n - 1, size=2 if kind == "ccx" else 1, replace=False)]
        nets.append([_gate(rng, kind, [n - 1] + rest)])
    return nets


def ghz_circuit(n: int) -> List[Net]:
    """H on the top qubit, then a CNOT chain from it to every other qubit."""
    top = n - 1
    nets: List[Net] = [[("h", (top,), ())]]
    for q in range(n - 2, -1, -1):
        nets.append([("cx", (top, q), ())])
    return nets


def basis_prep(n: int, x: int) -> List[Net]:
    """X gates that turn |0...0> into the basis state |x>."""
    net = [("x", (q,), ()) for q in range(n) if (x >> q) & 1]
    return [net] if net else []


def qft_circuit(n: int) -> List[Net]:
    """Textbook QFT: for the top qubit down, H then controlled phases
    pi/2^m from the lower qubits, then swaps that reverse the qubit order."""
    nets: List[Net] = []
    for j in range(n - 1, -1, -1):
        nets.append([("h", (j,), ())])
        for m, k in enumerate(range(j - 1, -1, -1), start=1):
            nets.append([("cp", (k, j), (math.pi / (2 ** m),))])
    swaps = [("swap", (q, n - 1 - q), ()) for q in range(n // 2)]
    if swaps:
        nets.append(swaps)
    return nets


INVERSE_KIND = {"h": "h", "x": "x", "y": "y", "z": "z", "s": "sdg", "sdg": "s",
                "t": "tdg", "tdg": "t", "rx": "rx", "ry": "ry", "rz": "rz",
                "cx": "cx", "cz": "cz", "swap": "swap", "cp": "cp", "ccx": "ccx"}


def inverse_circuit(nets: List[Net]) -> List[Net]:
    """Nets in reverse order with every gate replaced by its inverse (angles
    negated).  This is structure only: the kinds' inverses are the textbook
    ones."""
    out: List[Net] = []
    for net in reversed(nets):
        inv: Net = []
        for kind, qs, ps in net:
            if kind in ("rx", "ry", "rz", "cp"):
                inv.append((kind, qs, tuple(-p for p in ps)))
            else:
                inv.append((INVERSE_KIND[kind], qs, ps))
        out.append(inv)
    return out


# --------------------------------------------------------------------------
# modifiers
# --------------------------------------------------------------------------

@dataclass
class Edit:
    """One circuit modifier, expressed on the circuit as it stands when the
    edit is applied.

    ``op == "insert"``: put ``gate`` into net ``net``; when ``new_net`` is
    true, first insert an empty net right after net ``net`` and put the gate
    there (the paper's insert_net + insert_gate).
    ``op == "remove"``: remove gate number ``pos`` of net ``net``.
    """
    op: str
    net: int
    gate: Gate = None
    pos: int = -1
    new_net: bool = False


def apply_edit(nets: List[Net], e: Edit) -> None:
    """Apply an edit to the nested-list circuit model (structure only)."""
    if e.op == "insert":
        if e.new_net:
            nets.insert(e.net + 1, [e.gate])
        else:
            nets[e.net].append(e.gate)
    elif e.op == "remove":
        del nets[e.net][e.pos]
    else:
        raise ValueError(e.op)


def _free_qubits(n: int, net: Net) -> List[int]:
    used = set()
    for _, qs, _ in net:
        used.update(qs)
    return [q for q in range(n) if q not in used]


def random_edit(rng: np.random.Generator, n: int, nets: List[Net],
                kinds: Sequence[str]) -> Edit:
    """Insert or remove with probability 1/2 each.  Insert: uniform net,
    uniform kind, uniform angle, qubits drawn from the net's free qubits; if
    too few are free, the gate goes into a new net right after it.  Remove:
    uniform non-empty net, then a uniform gate of it."""
    nonempty = [i for i, net in enumerate(nets) if net]
    do_insert = (not nonempty) or bool(rng.integers(2) == 0)
    if do_insert:
        li = int(rng.integers(len(nets)))
        kind = str(kinds[int(rng.integers(len(kinds)))])
        k = N_QUBITS[kind]
        free = _free_qubits(n, nets[li])
        if len(free) >= k:
            qs = [free[int(i)] for i in rng.choice(len(free), size=k, replace=False)]
            return Edit("insert", li, _gate(rng, kind, qs))
        qs = [int(q) for q in rng.choice(n, size=k, replace=False)]
        return Edit("insert", li, _gate(rng, kind, qs), new_net=True)
    li = nonempty[int(rng.integers(len(nonempty)))]
    return Edit("remove", li, pos=int(rng.integers(len(nets[li]))))


def modifier_batches(n: int, nets: List[Net], seed: int, batches: int,
                     min_edits: int, max_edits: int,
                     kinds: Sequence[str]) -> List[List[Edit]]:
    """Draw ``batches`` batches of U{min..max} edits.  The edits are drawn
    against a private copy of the circuit so positions stay valid when the
    batches are applied in order to the original."""
    rng = np.random.default_rng(seed)
    model = [list(net) for net in nets]
    out: List[List[Edit]] = []
    for _ in range(batches):
        m = int(rng.integers(min_edits, max_edits + 1))
        batch = []
        for _ in range(m):
            e = random_edit(rng, n, model, kinds)
            apply_edit(model, e)
            batch.append(e)
        out.append(batch)
    return out


def split_edits(n: int, nets: List[Net], seed: int, count: int, b: int,
                kinds: Sequence[str] = ("rx", "ry", "rz", "cp"), tail: int = 0) -> List[List[Edit]]:
    """``count`` single-gate inserts at uniform nets, alternating between
    gates whose qubits all lie below ``b`` (inside one tile) and gates with a
    qubit at or above ``b``.  The qubits come from the net's free qubits when
    enough are free; otherwise the gate goes into a new net right after it.
    With ``tail`` > 0 the nets are drawn among the last ``tail`` nets only.
    Drawn against a private copy of the circuit, like modifier_batches."""
    rng = np.random.default_rng(seed)
    model = [list(net) for net in nets]
    out: List[List[Edit]] = []
    for i in range(count):
        high = i % 2 == 1
        lo = max(0, len(model) - tail) if tail > 0 else 0
        li = int(rng.integers(lo, len(model)))
        kind = str(kinds[int(rng.integers(len(kinds)))])
        k = N_QUBITS[kind]
        free = _free_qubits(n, model[li])
        pool_lo = [q for q in range(b)]
        pool_hi = [q for q in range(b, n)]
        cand_lo = [q for q in free if q < b]
        cand_hi = [q for q in free if q >= b]
        new_net = False
        if high and cand_hi and len(free) >= k:
            q0 = cand_hi[int(rng.integers(len(cand_hi)))]
            rest = [q for q in free if q != q0]
        elif not high and len(cand_lo) >= k:
            q0, rest = None, cand_lo
        else:
            new_net = True
            if high:
                q0 = pool_hi[int(rng.integers(len(pool_hi)))]
                rest = [q for q in range(n) if q != q0]
            else:
                q0, rest = None, pool_lo
        if q0 is None:
            qs = [rest[int(j)] for j in rng.choice(len(rest), size=k, replace=False)]
        else:
            qs = [q0] + [rest[int(j)] for j in rng.choice(len(rest), size=k - 1, replace=False)]
        e = Edit("insert", li, _gate(rng, kind, qs), new_net=new_net)
        apply_edit(model, e)
        out.append([e])
    return out


# --------------------------------------------------------------------------
# the benchmark configurations
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    n: int
    nets: List[Net]
    batches: List[List[Edit]] = field(default_factory=list)
    ckpt_nets: int = 0  # nets per checkpoint segment (0 = library default); 50 levels in every family


def config(cfg: int, *, levels: int = None, n: int = None, batches: int = None) -> Workload:
    """The five configurations.  ``levels``/``n``/``batches`` shrink a
    configuration for tests; by default the full sizes are produced.  A
    "level" of the layered families is two (or three) nets, see the circuit
    family docstrings."""
    if cfg == 1:
        n = n or 10
        nets = dense_random_circuit(n, levels or 20, seed_for(1))
        b = modifier_batches(n, nets, seed_for(1, "modifier"), batches or 10, 1, 1, CFG1_KINDS)
        return Workload("dense_random_n%d_l%d" % (n, levels or 20), n, nets, b)
    if cfg == 2:
        n = n or 24
        nets = layered_circuit(n, levels or 200, seed_for(2))
        b = modifier_batches(n, nets, seed_for(2, "modifier"), batches or 100, 1, 4,
                             LAYERED_EDIT_KINDS)
        return Workload("layered_n%d_l%d" % (n, levels or 200), n, nets, b, ckpt_nets=100)
    if cfg == 3:
        n = n or 30
        nets = layered_circuit(n, levels or 300, seed_for(3))
        b = modifier_batches(n, nets, seed_for(3, "modifier"), batches or 0, 1, 4,
                             LAYERED_EDIT_KINDS) if batches else []
        return Workload("layered_n%d_l%d" % (n, levels or 300), n, nets, b, ckpt_nets=100)
    if cfg == 5:
        n = n or 32
        nets = cp_ladder_circuit(n, levels or 500, seed_for(5))
        b = modifier_batches(n, nets, seed_for(5, "modifier"), batches or 50, 1, 1,
                             ("rx", "ry", "rz", "cp"))
        return Workload("cp_ladder_n%d_l%d" % (n, levels or 500), n, nets, b, ckpt_nets=150)
    raise ValueError("configuration %d is a serving workload; use serving_sessions()" % cfg)


@dataclass
class SessionSpec:
    sid: int
    n: int
    nets: List[Net]
    requests: List[List[Edit]]
    arrivals: List[float]  # seconds from start, Poisson process


def serving_sessions(count: int = 256, n_lo: int = 12, n_hi: int = 28,
                     d_lo: int = 50, d_hi: int = 400, requests: int = 4,
                     rate_hz: float = 50.0, seed0: int = 3000) -> List[SessionSpec]:
    """Sessions with n = floor(exp(U[ln n_lo, ln(n_hi+1)))), depth U{d_lo..d_hi}
    layered levels, and a Poisson stream of requests of U{1,2,3} edits each."""
    out = []
    for s in range(count):
        rng = np.random.default_rng(seed0 + s)
        n = int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi + 1)))))
        n = max(n_lo, min(n_hi, n))
        depth = int(rng.integers(d_lo, d_hi + 1))
        nets = layered_circuit(n, depth, seed0 + s)
        reqs = modifier_batches(n, nets, seed0 + 100000 + s, requests, 1, 3, LAYERED_EDIT_KINDS)
        gaps = rng.exponential(1.0 / rate_hz, size=requests)
        arrivals = list(np.cumsum(gaps))
        out.append(SessionSpec(s, n, nets, reqs, [float(a) for a in arrivals]))
    return out


def count_gates(nets: List[Net]) -> int:
    return sum(len(net) for net in nets)
