"""Helpers shared by the GPU tests (they drive the library through the C ABI
and compare with the CPU oracle)."""
import sys

import numpy as np

from oracle import oracle
from paper_2210_01076_amd import qtask as Q

TOL = {"c128": 1e-12, "c64": 1e-5}


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sim(n, nets, dtype="c128", **opts):
    s = Q.Simulator(n, dtype, device=0, **opts)
    s.build(nets)
    return s


def check_state(got, want, dtype, what=""):
    got = np.asarray(got).astype(np.complex128)
    err = float(np.max(np.abs(got - want))) if got.size else 0.0
    assert err <= TOL[dtype], "%s max-abs error %.3e > %.1e" % (what, err, TOL[dtype])
    if dtype == "c64":
        f = oracle.fidelity(want, got)
        assert f >= 1 - 1e-6, "%s fidelity %.9f" % (what, f)
    return err


def bytes_equal(a, b):
    return np.asarray(a).view(np.uint8).tobytes() == np.asarray(b).view(np.uint8).tobytes()


def generic_prep(n, seed):
    """A net of random RY/RZ on every qubit plus a CX chain: a state with no
    zero amplitudes and no symmetry, to start single-gate tests from."""
    rng = np.random.default_rng(seed)
    rot1 = [("ry", (q,), (float(rng.uniform(0.3, 2.8)),)) for q in range(n)]
    rot2 = [("rz", (q,), (float(rng.uniform(0.3, 2.8)),)) for q in range(n)]
    chain1 = [("cx", (q, q + 1), ()) for q in range(0, n - 1, 2)]
    chain2 = [("cx", (q, q + 1), ()) for q in range(1, n - 1, 2)]
    rot3 = [("rx", (q,), (float(rng.uniform(0.3, 2.8)),)) for q in range(n)]
    return [rot1, rot2, chain1, chain2, rot3]
