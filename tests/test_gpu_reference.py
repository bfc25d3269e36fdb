"""The device paths that serve as references at 30 and 32 qubits, checked
against the CPU oracle over the whole state at 24 qubits (the largest size
the oracle runs in seconds):

 - the precision-tier reference: the layered family with every stage fused
   into a dense 5-qubit unitary on the matrix cores (tile bits 11, low bits
   4, a renormalisation point every 50 layered levels), in complex128
   (max-abs 1e-12) and complex64 (max-abs 1e-5, fidelity 1 - 1e-6);
 - the controlled-phase ladder family with single-gate edits inside one
   tile and across tiles: every incremental update bitwise equal to a full
   re-simulation, and the final state within 1e-12 of the oracle."""
import numpy as np
import pytest

from oracle import oracle
from paper_2210_01076_amd import qtask as Q
from paper_2210_01076_amd import workloads as W
from tests.gpu_util import bytes_equal, check_state, log, sim

pytestmark = pytest.mark.gpu

N = 24
_cache = {}


def _layered_oracle():
    if "layered" not in _cache:
        nets = W.layered_circuit(N, 60, 3003)
        _cache["layered"] = (nets, oracle.simulate(N, nets, nthreads=oracle.max_threads()))
    return _cache["layered"]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fused_k5_reference_against_oracle(dtype):
    """60 layered levels (120 nets) in segments of 100 nets, so the complex64
    run renormalises after level 50 and at the end."""
    nets, want = _layered_oracle()
    opts = dict(tile_bits=11, low_bits=4, fusion=Q.QTASK_FUSE_DENSE, fuse_width=5, ckpt_interval=100)
    with sim(N, nets, dtype, **opts) as s:
        st = s.update()
        assert st["segments_replayed"] == 2 and st["mfma_flops"] > 0
        got = s.state()
        err = check_state(got, want, dtype, "fused k=5 %s" % dtype)
        f = oracle.fidelity(want, got.astype(np.complex128))
        log("fused k=5 n=%d %s: max-abs %.3e fidelity 1-%.2e (%d passes, %.1f ms)" % (
            N, dtype, err, 1 - f, st["passes"], st["kernel_ms"]))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_gate_list_reference_against_oracle(dtype):
    """The same circuit with the autotuner free to choose the tile shape and
    whether to fuse (the 30-qubit complex64 leg's configuration)."""
    nets, want = _layered_oracle()
    with sim(N, nets, dtype, autotune=1, ckpt_interval=100) as s:
        s.update()
        check_state(s.state(), want, dtype, "autotuned %s" % dtype)


def test_ladder_edits_inside_and_across_tiles_against_oracle():
    """20 ladder levels (60 nets), tile bits 12 and low bits 3, checkpoints
    every 15 nets; four single-gate inserts alternating between gates whose
    qubits all lie below 12 and gates with a qubit at or above 12."""
    b = 12
    nets = [list(x) for x in W.cp_ladder_circuit(N, 20, 5005)]
    batches = W.split_edits(N, nets, 5006, 4, b)
    with sim(N, nets, "c128", tile_bits=b, low_bits=3, ckpt_interval=15) as s:
        s.update()
        for i, batch in enumerate(batches):
            for e in batch:
                W.apply_edit(nets, e)
                s.apply_edit(e)
            st = s.update()
            inc = s.state()
            s.update(full=True)
            assert bytes_equal(inc, s.state()), "edit %d: incremental != full" % i
            qs = batch[0].gate[1]
            assert (max(qs) >= b) == (i % 2 == 1)
            log("ladder edit %d %s on %s: mode %d from net %d" % (i, batch[0].gate[0], qs, st["mode"],
                                                                 st["first_level"]))
        check_state(s.state(), oracle.simulate(N, nets, nthreads=oracle.max_threads()), "c128", "ladder")


def _blocked_oracle():
    if "blocked" not in _cache:
        nets = W.blocked_circuit(N, 40, 7)
        _cache["blocked"] = (nets, oracle.simulate(N, nets, nthreads=oracle.max_threads()))
    return _cache["blocked"]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("plan", ["dense5", "auto"])
def test_blocked_circuit_fused_against_oracle(dtype, plan):
    """The blocked family (blocks of 5 adjacent qubits coupled every 16
    levels; the circuit whose dense fusion beats its gate lists at 28
    qubits), 40 levels at 24 qubits: every stage fused into a dense 5-qubit
    unitary on the matrix cores, and the plan the autotuner picks under
    automatic fusion, each against the oracle over the whole state."""
    nets, want = _blocked_oracle()
    if plan == "dense5":
        opts = dict(tile_bits=11, low_bits=4, fusion=Q.QTASK_FUSE_DENSE, fuse_width=5, ckpt_interval=60)
    else:
        opts = dict(autotune=1, fusion=Q.QTASK_FUSE_AUTO, ckpt_interval=60)
    with sim(N, nets, dtype, **opts) as s:
        st = s.update()
        if plan == "dense5":
            assert st["mfma_flops"] > 0
        o = Q.qtask_get_opts(s.h)
        got = s.state()
        err = check_state(got, want, dtype, "blocked %s %s" % (plan, dtype))
        log("blocked n=%d %s %s: fusion %d k=%d b=%d c=%d, max-abs %.3e (%d passes)" % (
            N, plan, dtype, o.fusion, o.fuse_width, o.tile_bits, o.low_bits, err, st["passes"]))
