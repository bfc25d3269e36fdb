"""Pins for the CPU oracle: each check compares it with something other than
itself (the paper's printed matrices and worked example, textbook closed
forms, library routines, brute force, classical bit logic)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import bruteforce, oracle
from paper_2210_01076_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

PAULI_X = np.array([[0, 1], [1, 0]], dtype=complex)
PAULI_Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
PAULI_Z = np.array([[1, 0], [0, -1]], dtype=complex)
EYE2 = np.eye(2, dtype=complex)


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _nets_from_json(nets):
    return [[(g[0], tuple(g[1]), tuple(g[2]) if len(g) > 2 else ()) for g in net] for net in nets]


# ---------------------------------------------------------------- gate table

def test_paper_printed_matrices():
    gold = _load("paper_matrices.json")
    for kind in ("x", "h", "cx"):
        want = gold[kind]["scale"] * np.array(gold[kind]["rows"], dtype=complex)
        np.testing.assert_allclose(oracle.gate_matrix(kind), want, atol=0, rtol=1e-15)


@pytest.mark.parametrize("kind", W.GATE_KINDS)
def test_gate_unitary(kind):
    rng = np.random.default_rng(7)
    for _ in range(5):
        ps = tuple(rng.uniform(0, 2 * np.pi, W.N_PARAMS[kind]))
        m = oracle.gate_matrix(kind, ps)
        np.testing.assert_allclose(m @ m.conj().T, np.eye(m.shape[0]), atol=1e-15)


@pytest.mark.parametrize("kind,pauli", [("rx", PAULI_X), ("ry", PAULI_Y), ("rz", PAULI_Z)])
def test_rotations_are_exponentials(kind, pauli):
    for th in (0.0, 0.3, np.pi / 2, np.pi, 2.5, 5.9):
        want = scipy.linalg.expm(-0.5j * th * pauli)
        np.testing.assert_allclose(oracle.gate_matrix(kind, (th,)), want, atol=2e-16)


def test_table_one_relations():
    g = oracle.gate_matrix
    np.testing.assert_allclose(g("y"), PAULI_Y, atol=0)
    np.testing.assert_allclose(g("z"), PAULI_Z, atol=0)
    np.testing.assert_allclose(g("s") @ g("s"), g("z"), atol=1e-16)      # S = sqrt(Z)
    np.testing.assert_allclose(g("t") @ g("t"), g("s"), atol=2e-16)      # T = sqrt(S)
    np.testing.assert_allclose(g("sdg"), g("s").conj().T, atol=0)
    np.testing.assert_allclose(g("tdg"), g("t").conj().T, atol=0)
    np.testing.assert_allclose(g("h") @ g("x") @ g("h"), g("z"), atol=1e-15)
    # CZ = (I (x) H) CX (I (x) H); CP(pi) = CZ; SWAP = CX . CX' . CX
    ih = np.kron(EYE2, g("h"))
    np.testing.assert_allclose(ih @ g("cx") @ ih, g("cz"), atol=1e-15)
    np.testing.assert_allclose(g("cp", (np.pi,)), g("cz"), atol=2e-16)
    swap_cx = np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0], [0, 1, 0, 0]], dtype=complex)
    np.testing.assert_allclose(g("cx") @ swap_cx @ g("cx"), g("swap"), atol=0)
    # CCX: identity on the first six basis states, X on the last two
    want = np.eye(8, dtype=complex)
    want[6:, 6:] = PAULI_X
    np.testing.assert_allclose(g("ccx"), want, atol=0)


# ------------------------------------------------------- whole-circuit pins

def _random_circuit(rng, n, nets, kinds=W.GATE_KINDS):
    out = []
    for _ in range(nets):
        perm = list(rng.permutation(n))
        net = []
        while perm:
            kind = kinds[int(rng.integers(len(kinds)))]
            k = W.N_QUBITS[kind]
            if k > len(perm):
                continue
            qs = tuple(int(perm.pop()) for _ in range(k))
            net.append((kind, qs, tuple(rng.uniform(0, 2 * np.pi, W.N_PARAMS[kind]))))
        out.append(net)
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_oracle_matches_bruteforce(n):
    rng = np.random.default_rng(100 + n)
    for trial in range(3):
        nets = _random_circuit(rng, n, 6)
        want = bruteforce.simulate(n, nets)
        got = oracle.simulate(n, nets)
        np.testing.assert_allclose(got, want, atol=1e-13, rtol=0)
        # a random input state too (the unitary, not only its first column)
        psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
        psi0 /= np.linalg.norm(psi0)
        np.testing.assert_allclose(oracle.simulate(n, nets, psi0),
                                   bruteforce.circuit_unitary(n, nets) @ psi0, atol=1e-13)


@pytest.mark.parametrize("n", [1, 3, 5, 6])
def test_entrywise_matches_literal_kronecker(n):
    rng = np.random.default_rng(200 + n)
    for _ in range(4):
        net = []
        for q in range(n):
            if rng.random() < 0.8:
                kind = W.ONE_QUBIT[int(rng.integers(len(W.ONE_QUBIT)))]
                net.append((kind, (q,), tuple(rng.uniform(0, 2 * np.pi, W.N_PARAMS[kind]))))
        np.testing.assert_allclose(bruteforce.net_matrix(n, net),
                                   bruteforce.kron_net_matrix(n, net), atol=1e-15)
        np.testing.assert_allclose(oracle.simulate(n, [net]),
                                   bruteforce.kron_net_matrix(n, net)[:, 0], atol=1e-15)


@pytest.mark.parametrize("n", [2, 3, 7, 12])
def test_ghz(n):
    psi = oracle.simulate(n, W.ghz_circuit(n))
    want = np.zeros(1 << n, dtype=complex)
    want[0] = want[-1] = 1 / math.sqrt(2)
    np.testing.assert_allclose(psi, want, atol=1e-15)


@pytest.mark.parametrize("n", [3, 5, 8])
def test_qft_of_basis_state(n):
    N = 1 << n
    for x in (0, 1, N // 3, N - 1):
        psi = oracle.simulate(n, W.basis_prep(n, x) + W.qft_circuit(n))
        np.testing.assert_allclose(np.abs(psi), np.full(N, N ** -0.5), atol=1e-14)
        y = np.arange(N)
        np.testing.assert_allclose(psi, np.exp(2j * np.pi * x * y / N) / math.sqrt(N), atol=1e-14)
        # the same closed form is sqrt(N) * inverse DFT of e_x
        e = np.zeros(N, dtype=complex)
        e[x] = 1
        np.testing.assert_allclose(psi, np.fft.ifft(e) * math.sqrt(N), atol=1e-14)


@pytest.mark.parametrize("n", [4, 9])
def test_circuit_then_inverse(n):
    rng = np.random.default_rng(300 + n)
    nets = _random_circuit(rng, n, 20)
    psi = oracle.simulate(n, nets + W.inverse_circuit(nets))
    depth = 2 * len(nets)
    want = oracle.basis(n)
    assert np.max(np.abs(psi - want)) <= depth * 1e-15 * 4


def test_norm_preserved():
    for n, seed in ((10, 1), (13, 2)):
        psi = oracle.simulate(n, W.layered_circuit(n, 10, seed))
        assert abs(oracle.norm2(psi) - 1.0) < 1e-13


def test_permutation_only_matches_bit_logic():
    rng = np.random.default_rng(400)
    n = 9
    for _ in range(10):
        x = int(rng.integers(1 << n))
        nets = _random_circuit(rng, n, 8, kinds=("x", "cx", "swap", "ccx"))
        y = x
        for net in nets:
            for kind, qs, _ in net:
                bit = lambda q: (y >> q) & 1
                if kind == "x":
                    y ^= 1 << qs[0]
                elif kind == "cx":
                    if bit(qs[0]):
                        y ^= 1 << qs[1]
                elif kind == "ccx":
                    if bit(qs[0]) and bit(qs[1]):
                        y ^= 1 << qs[2]
                elif kind == "swap":
                    a, b = bit(qs[0]), bit(qs[1])
                    if a != b:
                        y ^= (1 << qs[0]) | (1 << qs[1])
        psi = oracle.simulate(n, nets, oracle.basis(n, x))
        want = oracle.basis(n, y)
        assert np.array_equal(psi, want)


def test_diagonal_only_closed_form():
    rng = np.random.default_rng(500)
    n = 7
    N = 1 << n
    hadamards = [[("h", (q,), ()) for q in range(n)]]
    nets = _random_circuit(rng, n, 6, kinds=("z", "s", "sdg", "t", "tdg", "rz", "cz", "cp"))
    psi = oracle.simulate(n, hadamards + nets)
    phase = np.ones(N, dtype=complex)
    ys = np.arange(N)
    for net in nets:
        for kind, qs, ps in net:
            b0 = (ys >> qs[0]) & 1
            if kind == "z":
                phase *= (-1.0) ** b0
            elif kind in ("s", "sdg"):
                phase *= (1j if kind == "s" else -1j) ** b0
            elif kind in ("t", "tdg"):
                phase *= np.exp((1 if kind == "t" else -1) * 1j * np.pi / 4 * b0)
            elif kind == "rz":
                phase *= np.exp(1j * ps[0] / 2 * (2 * b0 - 1))
            else:
                b1 = (ys >> qs[1]) & 1
                lam = np.pi if kind == "cz" else ps[0]
                phase *= np.exp(1j * lam * (b0 & b1))
    np.testing.assert_allclose(psi, phase / math.sqrt(N), atol=1e-14)


# ---------------------------------------------------------- worked example

def test_worked_example_state_and_touched_blocks():
    gold = _load("worked_example.json")
    n, bb = gold["n"], gold["block_bits"]
    nets = _nets_from_json(gold["nets"])
    u = gold["uniform_amplitude"]
    before = oracle.simulate(n, nets)
    np.testing.assert_allclose(before, np.full(1 << n, u), atol=1e-15)
    edited = [list(net) for net in nets]
    del edited[3][0]                                    # remove G8
    g10 = gold["g10"]
    edited[3].append((g10[0], tuple(g10[1]), ()))       # insert G10
    after = oracle.simulate(n, edited)
    np.testing.assert_allclose(after, np.full(1 << n, u), atol=1e-15)

    rng = np.random.default_rng(600)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    gates = {name: nets[i][j] for name, (i, j) in gold["gate_names"].items()}
    gates["G10"] = (g10[0], tuple(g10[1]), ())
    for name, gate in gates.items():
        out = oracle.apply_gates(n, psi.copy(), [gate])
        assert oracle.changed_blocks(psi, out, bb) == set(gold["touched_blocks"][name]), name
    # the paper's dirty set is the union of the removed and inserted gates'
    # blocks, and G9 (its successor) keeps every block in place
    dirty = set(gold["touched_blocks"]["G8"]) | set(gold["touched_blocks"]["G10"])
    assert sorted(dirty) == gold["dirty_blocks_after_edits"]
    amps = [a for blk in sorted(dirty) for a in range(blk << bb, (blk + 1) << bb)]
    ranges = gold["updated_amplitude_ranges"]
    assert amps == [a for lo, hi in ranges for a in range(lo, hi + 1)]
    assert len(amps) == gold["updated_amplitude_count"]


def test_worked_example_paper_ranges_cover_exact_blocks():
    """The paper's interval partitions (hulls of the blocks a gate reads and
    writes) contain the exact touched blocks."""
    gold = _load("worked_example.json")
    for name, ranges in gold["paper_block_ranges"].items():
        key = name.split("_")[0]
        if isinstance(ranges[0], int):
            ranges = [ranges]
        hull = set(b for lo, hi in ranges for b in range(lo, hi + 1))
        exact = set(gold["touched_blocks"][key])
        if name.endswith("_first"):
            exact = {b for b in exact if b <= ranges[0][1]}
        assert exact <= hull, name


# ------------------------------------------- reductions and helper functions
# The state is a unit vector of 2^n amplitudes (Section II-A); the helpers
# below are the plain definitions the parity tests lean on: the squared norm,
# the inner product <a|b> (conjugate-linear in its first argument), fidelity
# |<a|b>|^2 / (<a|a><b|b>), per-net snapshots and changed-block sets.

KET0 = np.array([1, 0], dtype=complex)
KET1 = np.array([0, 1], dtype=complex)
PLUS = np.array([1, 1], dtype=complex) / math.sqrt(2)
MINUS = np.array([1, -1], dtype=complex) / math.sqrt(2)


def _rand_state(rng, n):
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / math.sqrt(sum(abs(complex(z)) ** 2 for z in v))


def test_norm2_closed_forms():
    # amplitudes k + i k: sum of 2 k^2 over k < 2^n is (2^n - 1) 2^n (2^(n+1) - 1) / 3
    for n in (1, 3, 6):
        k = np.arange(1 << n, dtype=float)
        want = (2 ** n - 1) * 2 ** n * (2 ** (n + 1) - 1) / 3
        assert oracle.norm2(k + 1j * k) == want
    assert oracle.norm2(PLUS) == pytest.approx(1.0, abs=4e-16)
    # complex64 input is widened before squaring
    assert oracle.norm2(np.array([3 + 4j], dtype=np.complex64)) == 25.0


def test_inner_conjugates_its_first_argument():
    rng = np.random.default_rng(31)
    psi = _rand_state(rng, 5)
    n2 = oracle.norm2(psi)
    # <psi|i psi> = i <psi|psi> and <i psi|psi> = -i <psi|psi>: fixes which side is conjugated
    assert abs(oracle.inner(psi, 1j * psi) - 1j * n2) < 1e-15
    assert abs(oracle.inner(1j * psi, psi) + 1j * n2) < 1e-15
    # textbook values on one qubit
    assert abs(oracle.inner(KET0, PLUS) - 2 ** -0.5) < 3e-16
    assert abs(oracle.inner(PLUS, MINUS)) < 1e-16
    assert abs(oracle.inner(KET1, MINUS) + 2 ** -0.5) < 3e-16
    # <0|(a|0> + b|1>)> picks a; as a bra, a|0> + b|1> gives conj(b) against |1>
    a, b = 0.6 + 0.2j, -0.3 + 0.7j
    assert oracle.inner(KET0, a * KET0 + b * KET1) == a
    assert oracle.inner(a * KET0 + b * KET1, KET1) == b.conjugate()
    assert oracle.inner(a * KET0, KET0) == a.conjugate()


def test_inner_against_python_sum_and_symmetry():
    rng = np.random.default_rng(32)
    for n in (1, 2, 4):
        x, y = _rand_state(rng, n), _rand_state(rng, n)
        want = sum(complex(p).conjugate() * complex(q) for p, q in zip(x, y))
        assert abs(oracle.inner(x, y) - want) < 1e-15
        assert abs(oracle.inner(y, x) - want.conjugate()) < 1e-15
        # linear in the second argument, index by index (a transposed or
        # reversed operand would break this)
        e = np.zeros(1 << n, dtype=complex)
        for k in range(1 << n):
            e[:] = 0
            e[k] = 1
            assert oracle.inner(e, y) == complex(y[k])


def test_fidelity_closed_forms():
    rng = np.random.default_rng(33)
    psi = _rand_state(rng, 4)
    for phi in (0.0, 0.7, math.pi, 4.0):
        assert oracle.fidelity(psi, np.exp(1j * phi) * psi) == pytest.approx(1.0, abs=1e-15)
    assert oracle.fidelity(KET0, KET1) == 0.0
    assert oracle.fidelity(KET0, PLUS) == pytest.approx(0.5, abs=1e-16)   # a missing square would give 2^-1/2
    assert oracle.fidelity(PLUS, MINUS) == pytest.approx(0.0, abs=1e-32)
    for th in (0.1, 0.9, 1.3):
        v = math.cos(th) * KET0 + math.sin(th) * KET1
        assert oracle.fidelity(KET0, v) == pytest.approx(math.cos(th) ** 2, abs=1e-16)
    # invariant under rescaling either argument (the norms are divided out)
    phi = _rand_state(rng, 4)
    f = oracle.fidelity(psi, phi)
    assert 0.0 < f < 1.0
    assert oracle.fidelity(3.0 * psi, phi) == pytest.approx(f, rel=1e-14)
    assert oracle.fidelity(psi, (0.25 - 2j) * phi) == pytest.approx(f, rel=1e-14)
    assert oracle.fidelity(phi, psi) == pytest.approx(f, rel=1e-14)


def test_snapshots_step_by_brute_force():
    rng = np.random.default_rng(34)
    for n in (1, 3, 5):
        nets = _random_circuit(rng, n, 5)
        snaps = oracle.snapshots(n, nets)
        assert len(snaps) == len(nets) + 1
        e0 = np.zeros(1 << n, dtype=complex)
        e0[0] = 1
        assert np.array_equal(snaps[0], e0)
        for i, net in enumerate(nets):
            np.testing.assert_allclose(snaps[i + 1], bruteforce.net_matrix(n, net) @ snaps[i], atol=1e-14)
        np.testing.assert_array_equal(snaps[-1], oracle.simulate(n, nets))


def test_changed_blocks_by_hand():
    a = np.zeros(16, dtype=complex)
    b = a.copy()
    b[5] = 1e-300      # block 1 of 4-amplitude blocks
    b[15] = -0.0 + 1j  # block 3
    assert oracle.changed_blocks(a, b, 2) == {1, 3}
    assert oracle.changed_blocks(a, b, 0) == {5, 15}
    assert oracle.changed_blocks(a, b, 4) == {0}
    assert oracle.changed_blocks(a, a.copy(), 1) == set()
