"""Incremental update on the GPU: equal to the oracle's full simulation of the
modified circuit, and bitwise equal to a full GPU re-simulation."""
import json
import os

import numpy as np
import pytest

from oracle import oracle
from paper_2210_01076_amd import workloads as W
from tests.gpu_util import bytes_equal, check_state, log, sim

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _check_incremental(s, nets, n, dtype, with_oracle=True):
    inc = s.state()
    h_inc = s.hash()
    st = s.stats()
    s.update(full=True)
    full = s.state()
    assert bytes_equal(inc, full), "incremental != full re-simulation (mode %d)" % st["mode"]
    assert h_inc == s.hash()
    if with_oracle:
        check_state(inc, oracle.simulate(n, nets, nthreads=oracle.max_threads()), dtype)
    return st


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_dense_random_config_small(dtype):
    """n=10, 20 levels of random gates, 10 single-gate modifiers."""
    wl = W.config(1)
    nets = [list(x) for x in wl.nets]
    with sim(wl.n, nets, dtype, ckpt_interval=5) as s:
        s.update()
        check_state(s.state(), oracle.simulate(wl.n, nets), dtype)
        for bi, batch in enumerate(wl.batches):
            for e in batch:
                W.apply_edit(nets, e)
                s.apply_edit(e)
            s.update()
            st = _check_incremental(s, nets, wl.n, dtype)
            log("cfg1", dtype, bi, "mode", st["mode"], "first", st["first_level"])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_layered_batches(dtype):
    n = 17
    nets = W.layered_circuit(n, 30, 9)
    batches = W.modifier_batches(n, nets, 19, 8, 1, 4, W.LAYERED_EDIT_KINDS)
    with sim(n, nets, dtype, ckpt_interval=10) as s:
        s.update()
        for bi, batch in enumerate(batches):
            for e in batch:
                W.apply_edit(nets, e)
                s.apply_edit(e)
            s.update()
            st = _check_incremental(s, nets, n, dtype, with_oracle=bi % 3 == 0)
            log("layered", dtype, bi, "mode", st["mode"], "first", st["first_level"])


def test_remove_then_reinsert_restores_bits():
    n = 14
    nets = W.layered_circuit(n, 12, 4)
    with sim(n, nets, ckpt_interval=6) as s:
        s.update()
        before = s.state()
        gate = nets[9][2]
        s.apply_edit(W.Edit("remove", 9, pos=2))
        s.update()
        assert not bytes_equal(before, s.state())
        s.apply_edit(W.Edit("insert", 9, gate))
        s.update()
        assert bytes_equal(before, s.state())


def test_closed_mode_on_permutation_circuit():
    """Mostly-classical circuit: the affected set stays closed, so only its
    tiles are re-run; the result still equals a full re-simulation."""
    n = 16
    kinds = ("x", "cx", "ccx", "swap", "z", "s", "t", "cz")
    nets = [[("h", (q,), ()) for q in range(4)]] + W.dense_random_circuit(n, 30, 8, kinds=kinds)
    rng = np.random.default_rng(3)
    modes = []
    with sim(n, nets, block_bits=8, ckpt_interval=4) as s:
        s.update()
        for trial in range(10):
            li = int(rng.integers(len(nets) - 10, len(nets)))
            if nets[li]:
                e = W.Edit("remove", li, pos=int(rng.integers(len(nets[li]))))
            else:
                e = W.Edit("insert", li, ("x", (int(rng.integers(n)),), ()))
            W.apply_edit(nets, e)
            s.apply_edit(e)
            s.update()
            st = _check_incremental(s, nets, n, "c128")
            modes.append(st["mode"])
            log("closed", trial, st["mode"], st["dirty_blocks"], st["tiles"])
    assert 3 in modes


def test_worked_example_on_device():
    with open(os.path.join(GOLDEN, "worked_example.json")) as f:
        gold = json.load(f)
    nets = [[(g[0], tuple(g[1]), ()) for g in net] for net in gold["nets"]]
    with sim(gold["n"], nets, block_bits=gold["block_bits"], ckpt_interval=1) as s:
        s.update()
        np.testing.assert_allclose(s.state(), gold["uniform_amplitude"], atol=1e-15)
        i, j = gold["gate_names"]["G8"]
        s.apply_edit(W.Edit("remove", i, pos=j))
        s.apply_edit(W.Edit("insert", i, (gold["g10"][0], tuple(gold["g10"][1]), ())))
        s.update()
        st = s.stats()
        assert st["mode"] == 3 and st["dirty_blocks"] == 6
        np.testing.assert_allclose(s.state(), gold["uniform_amplitude"], atol=1e-15)
        _check_incremental(s, [[g for g in net] for net in nets], gold["n"], "c128", with_oracle=False)
