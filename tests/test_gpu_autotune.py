"""Autotuner on the GPU: the pick is a valid shape (and, under automatic
fusion, possibly a dense fusion width), it is frozen for the session and
cached per key, and whatever it picks the results match the oracle and
incremental updates stay bitwise equal to a full re-simulation."""
import numpy as np
import pytest

from oracle import oracle
from paper_2210_01076_amd import qtask as Q
from paper_2210_01076_amd import workloads as W
from tests.gpu_util import bytes_equal, check_state, log, sim

pytestmark = pytest.mark.gpu


def _valid(o, n):
    assert 4 <= o.tile_bits <= 13 and o.tile_bits <= max(n, 4)
    assert 0 <= o.low_bits <= o.tile_bits - 3
    assert o.fusion in (Q.QTASK_FUSE_AUTO, Q.QTASK_FUSE_DENSE)
    if o.fusion == Q.QTASK_FUSE_DENSE:
        assert 4 <= o.fuse_width <= 6 and o.tile_bits - o.fuse_width >= 4


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_autotuned_layered_matches_oracle_and_stays_frozen(dtype):
    n = 16
    nets = W.layered_circuit(n, 30, 71)
    batches = W.modifier_batches(n, nets, 72, 3, 1, 3, W.LAYERED_EDIT_KINDS)
    with sim(n, nets, dtype, autotune=1, ckpt_interval=10) as s:
        s.update()
        o = Q.qtask_get_opts(s.h)
        _valid(o, n)
        log("%s layered-16 pick: b=%d c=%d fusion=%d k=%d" % (dtype, o.tile_bits, o.low_bits, o.fusion, o.fuse_width))
        check_state(s.state(), oracle.simulate(n, nets), dtype, "autotuned")
        for batch in batches:
            for e in batch:
                W.apply_edit(nets, e)
                s.apply_edit(e)
            s.update()
            inc = s.state()
            s.update(full=True)
            assert bytes_equal(inc, s.state())
            o2 = Q.qtask_get_opts(s.h)
            assert (o2.tile_bits, o2.low_bits, o2.fusion, o2.fuse_width) == (
                o.tile_bits, o.low_bits, o.fusion, o.fuse_width)
        check_state(s.state(), oracle.simulate(n, nets), dtype, "autotuned after edits")


def test_autotune_pick_is_cached_per_key():
    n = 14
    nets = W.layered_circuit(n, 20, 81)
    picks = []
    for _ in range(2):
        with sim(n, nets, autotune=1) as s:
            s.update()
            o = Q.qtask_get_opts(s.h)
            picks.append((o.tile_bits, o.low_bits, o.fusion, o.fuse_width))
    assert picks[0] == picks[1]


def test_autotuned_deep_dense_circuit_matches_oracle():
    """A deep circuit on 10 qubits: every tile holds the whole state, the
    case where fused dense stages can win; the result matches the oracle
    whatever the tuner picks."""
    n = 10
    nets = W.dense_random_circuit(n, 120, 91, kinds=W.GATE_KINDS)
    with sim(n, nets, autotune=1) as s:
        s.update()
        o = Q.qtask_get_opts(s.h)
        _valid(o, n)
        log("deep-10 pick: b=%d c=%d fusion=%d k=%d" % (o.tile_bits, o.low_bits, o.fusion, o.fuse_width))
        check_state(s.state(), oracle.simulate(n, nets), "c128", "autotuned deep")


def test_explicit_shape_is_not_retuned():
    n = 12
    nets = W.layered_circuit(n, 6, 95)
    with sim(n, nets, autotune=0, tile_bits=9, low_bits=3) as s:
        s.update()
        o = Q.qtask_get_opts(s.h)
        assert (o.tile_bits, o.low_bits, o.fusion) == (9, 3, Q.QTASK_FUSE_AUTO)
        check_state(s.state(), oracle.simulate(n, nets), "c128")
