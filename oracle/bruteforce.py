"""Brute-force whole-circuit unitaries for tiny circuits (n <= 6).  TEST
INFRASTRUCTURE ONLY.

Two independent constructions of a net's 2^n x 2^n matrix, both written
straight from Section II-A of the paper:

* ``gate_full_matrix`` builds a gate's full matrix entry by entry:
  <r|G|c> = M[loc(r), loc(c)] when r and c agree on every qubit outside the
  gate, 0 otherwise;
* ``kron_net_matrix`` is the paper's literal form for a net of one-qubit
  gates: the Kronecker product of the gate matrices with identities padded
  into empty spots, most significant qubit first.

The circuit unitary is the product of the net matrices in order.  Neither
routine shares index arithmetic with the C oracle; they share only its gate
table, which the tests pin separately against the paper and against matrix
exponentials.
"""
from __future__ import annotations

from functools import reduce

import numpy as np

from . import oracle


def local_index(state: int, qubits) -> int:
    """Local index of a basis state for a gate on ``qubits``: the first-listed
    qubit is the most significant bit (the paper's CX has its control on the
    high bit)."""
    k = len(qubits)
    loc = 0
    for j, q in enumerate(qubits):
        loc |= ((state >> q) & 1) << (k - 1 - j)
    return loc


def gate_full_matrix(n: int, gate) -> np.ndarray:
    kind, qs, ps = gate
    m = oracle.gate_matrix(kind, ps)
    dim = 1 << n
    off_mask = ~sum(1 << q for q in qs)
    full = np.zeros((dim, dim), dtype=np.complex128)
    for r in range(dim):
        for c in range(dim):
            if (r & off_mask) == (c & off_mask):
                full[r, c] = m[local_index(r, qs), local_index(c, qs)]
    return full


def net_matrix(n: int, net) -> np.ndarray:
    """Product of the net's gate matrices (gates in a net commute)."""
    u = np.eye(1 << n, dtype=np.complex128)
    for g in net:
        u = gate_full_matrix(n, g) @ u
    return u


def kron_net_matrix(n: int, net) -> np.ndarray:
    """G_{n-1} (x) ... (x) G_0 for a net of one-qubit gates, identity where a
    qubit has no gate."""
    per_qubit = [np.eye(2, dtype=np.complex128) for _ in range(n)]
    for kind, qs, ps in net:
        assert len(qs) == 1, "literal Kronecker form is for one-qubit nets"
        per_qubit[qs[0]] = oracle.gate_matrix(kind, ps)
    return reduce(np.kron, [per_qubit[q] for q in range(n - 1, -1, -1)])


def circuit_unitary(n: int, nets) -> np.ndarray:
    u = np.eye(1 << n, dtype=np.complex128)
    for net in nets:
        u = net_matrix(n, net) @ u
    return u


def simulate(n: int, nets) -> np.ndarray:
    """Brute-force state: the circuit unitary's first column (input |0...0>)."""
    return circuit_unitary(n, nets)[:, 0].copy()
