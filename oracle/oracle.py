"""Python face of the CPU oracle.  TEST INFRASTRUCTURE ONLY: the tests, the
smoke check and the benchmark's CPU-baseline leg use it; the product library
never does.

It wraps ``qtask_oracle.c`` (a plain complex128 simulator, see that file for
the conventions) and adds the plain-definition helpers the tests need:
per-net snapshots, norms, inner products, fidelity, and the changed-block sets
used to check the affected-block tracker.

The oracle simulates a circuit given as nets of ``(kind, qubits, params)``
tuples (the layout the workload generator produces).  Its incremental
"update" is, by definition, a fresh full simulation of the modified circuit:
the paper's incremental result must equal that (Section I, Section III-E).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qtask_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

#: oracle-private gate codes; the order matches the enum in qtask_oracle.c
KIND_CODE = {name: i for i, name in enumerate(
    ["h", "x", "y", "z", "s", "sdg", "t", "tdg", "rx", "ry", "rz",
     "cx", "cz", "swap", "cp", "ccx"])}

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, -O2, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                        "-fPIC", "-shared", "-std=c11", "-Wall", "-Werror",
                        _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_apply.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int]
        lib.oracle_apply.restype = ctypes.c_int
        lib.oracle_gate_matrix.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_gate_matrix.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def gate_matrix(kind: str, params: Sequence[float] = ()) -> np.ndarray:
    """The oracle's matrix for a gate kind (dim x dim complex128)."""
    lib = _load()
    p = np.zeros(3, dtype=np.float64)
    p[:len(params)] = params
    m = np.zeros(2 * 64, dtype=np.float64)
    dim = lib.oracle_gate_matrix(KIND_CODE[kind], p.ctypes.data, m.ctypes.data)
    if dim < 0:
        raise ValueError(kind)
    return m[: 2 * dim * dim].view(np.complex128).reshape(dim, dim).copy()


def _flatten(gates):
    g = len(gates)
    kinds = np.zeros(max(g, 1), dtype=np.int32)
    qubits = np.zeros(3 * max(g, 1), dtype=np.int32)
    params = np.zeros(3 * max(g, 1), dtype=np.float64)
    for i, (kind, qs, ps) in enumerate(gates):
        kinds[i] = KIND_CODE[kind]
        qubits[3 * i:3 * i + len(qs)] = qs
        params[3 * i:3 * i + len(ps)] = ps
    return kinds, qubits, params


def apply_gates(n: int, psi: np.ndarray, gates, nthreads: int = 1) -> np.ndarray:
    """Apply a flat gate list to ``psi`` (complex128, modified in place)."""
    assert psi.dtype == np.complex128 and psi.size == (1 << n) and psi.flags.c_contiguous
    if not gates:
        return psi
    kinds, qubits, params = _flatten(gates)
    rc = _load().oracle_apply(n, psi.ctypes.data, len(gates), kinds.ctypes.data,
                              qubits.ctypes.data, params.ctypes.data, max(1, nthreads))
    if rc != 0:
        raise ValueError("oracle rejected a gate")
    return psi


def basis(n: int, x: int = 0) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[x] = 1.0
    return psi


def simulate(n: int, nets, psi0: np.ndarray = None, nthreads: int = 1) -> np.ndarray:
    """Full simulation: the ordered product of the nets applied to |0...0>
    (or to a copy of ``psi0``)."""
    psi = basis(n) if psi0 is None else np.array(psi0, dtype=np.complex128, copy=True)
    flat = [g for net in nets for g in net]
    return apply_gates(n, psi, flat, nthreads)


def snapshots(n: int, nets, nthreads: int = 1) -> List[np.ndarray]:
    """States after each net: snapshots[0] is the input, snapshots[i] the
    state after nets[:i]."""
    psi = basis(n)
    out = [psi.copy()]
    for net in nets:
        apply_gates(n, psi, list(net), nthreads)
        out.append(psi.copy())
    return out


def norm2(psi: np.ndarray) -> float:
    """sum_b |alpha_b|^2 in float64 (Section II-A normalisation)."""
    p = psi.astype(np.complex128)
    return float(np.sum(p.real * p.real + p.imag * p.imag))


def inner(a: np.ndarray, b: np.ndarray) -> complex:
    """<a|b> in complex128."""
    return complex(np.vdot(a.astype(np.complex128), b.astype(np.complex128)))


def fidelity(ref: np.ndarray, psi: np.ndarray) -> float:
    """|<ref|psi>|^2 / (<ref|ref><psi|psi>), all in float64."""
    return abs(inner(ref, psi)) ** 2 / (norm2(ref) * norm2(psi))


def changed_blocks(before: np.ndarray, after: np.ndarray, block_bits: int) -> set:
    """Indices of the 2^block_bits-amplitude blocks whose values differ."""
    d = (before != after).reshape(-1, 1 << block_bits).any(axis=1)
    return set(int(i) for i in np.nonzero(d)[0])
