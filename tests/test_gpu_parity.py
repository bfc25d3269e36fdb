"""Parity of the HIP path with the CPU oracle (element by element)."""
import math

import numpy as np
import pytest

from oracle import oracle
from paper_2210_01076_amd import qtask as Q
from paper_2210_01076_amd import workloads as W
from tests.gpu_util import TOL, bytes_equal, check_state, generic_prep, log, sim

pytestmark = pytest.mark.gpu

DTYPES = ["c128", "c64"]


def test_device_visible():
    assert Q.qtask_device_count() >= 1


@pytest.mark.parametrize("dtype", DTYPES)
def test_every_gate_kind_at_edge_positions(dtype):
    n = 15  # several tiles at the default tile size, plus qubits above it
    prep = generic_prep(n, 1)
    base = oracle.simulate(n, prep)
    # qubits inside the contiguous low bits, at the tile-size edges of both
    # default tile shapes, and at the top of the state
    positions = sorted({0, 1, 3, 4, 10, 11, 12, n - 2, n - 1})
    cases = []
    for kind in W.GATE_KINDS:
        k = W.N_QUBITS[kind]
        for p in positions:
            qs = [p] + [q for q in positions if q != p][: k - 1]
            cases.append((kind, tuple(qs)))
            if k >= 2:
                cases.append((kind, tuple(reversed(qs))))
    for kind, qs in cases:
        ps = (1.2345,) * W.N_PARAMS[kind]
        nets = prep + [[(kind, qs, ps)]]
        want = oracle.apply_gates(n, base.copy(), [(kind, qs, ps)])
        log("gate", dtype, kind, qs)
        with sim(n, nets, dtype) as s:
            s.update()
            check_state(s.state(), want, dtype, "%s %s" % (kind, qs))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 10, 13, 16])
def test_random_circuits_small(dtype, n):
    nets = W.dense_random_circuit(n, 12, 40 + n, kinds=W.GATE_KINDS)
    want = oracle.simulate(n, nets)
    log("random", dtype, n)
    with sim(n, nets, dtype, ckpt_interval=5) as s:
        s.update()
        check_state(s.state(), want, dtype, "n=%d" % n)
        assert abs(s.norm() - 1.0) < (1e-12 if dtype == "c128" else 1e-5)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("b,c", [(12, 4), (10, 3), (13, 6), (8, 2), (6, 1)])
def test_layered_tile_shapes(dtype, b, c):
    n = 18
    nets = W.layered_circuit(n, 8, 77)
    want = oracle.simulate(n, nets, nthreads=oracle.max_threads())
    log("layered", dtype, b, c)
    with sim(n, nets, dtype, tile_bits=b, low_bits=c, ckpt_interval=4) as s:
        s.update()
        check_state(s.state(), want, dtype, "b=%d c=%d" % (b, c))


def test_ghz_and_qft_closed_forms():
    n = 20
    with sim(n, W.ghz_circuit(n)) as s:
        s.update()
        psi = s.state()
        want = np.zeros(1 << n, dtype=complex)
        want[0] = want[-1] = 1 / math.sqrt(2)
        check_state(psi, want, "c128", "ghz")
    x = 12345
    N = 1 << n
    with sim(n, W.basis_prep(n, x) + W.qft_circuit(n)) as s:
        s.update()
        psi = s.state()
        y = np.arange(N)
        want = np.exp(2j * np.pi * ((x * y) % N) / N) / math.sqrt(N)
        check_state(psi, want, "c128", "qft")


def test_ragged_reads_and_empty_circuit():
    n = 9
    nets = W.dense_random_circuit(n, 6, 5)
    want = oracle.simulate(n, nets)
    with sim(n, nets) as s:
        s.update()
        for first, count in [(0, 1), (3, 17), (511, 1), (100, 0), (0, 512)]:
            np.testing.assert_allclose(s.state(first, count), want[first:first + count], atol=1e-12)
        with pytest.raises(Q.QtaskError) as e:
            s.state(500, 13)
        assert e.value.code == Q.QTASK_E_NOTFOUND
        # stale after a modifier
        s.add_level()
        s.add_gate(len(s.levels) - 1, ("x", (0,), ()))
        with pytest.raises(Q.QtaskError) as e:
            s.state()
        assert e.value.code == Q.QTASK_E_STALE
    with sim(6, []) as s:
        s.update()
        assert bytes_equal(s.state(), oracle.basis(6))


def test_inverse_returns_input():
    n = 16
    nets = W.layered_circuit(n, 10, 3)
    with sim(n, nets + W.inverse_circuit(nets)) as s:
        s.update()
        psi = s.state()
        assert abs(psi[0] - 1) < 1e-12
        assert np.max(np.abs(psi[1:])) < 1e-12


@pytest.mark.parametrize("dtype", DTYPES)
def test_inner_product_and_norm(dtype):
    n = 12
    a_nets = W.layered_circuit(n, 5, 1)
    b_nets = W.layered_circuit(n, 5, 2)
    with sim(n, a_nets, dtype) as a, sim(n, b_nets, dtype) as b:
        a.update()
        b.update()
        got = Q.qtask_inner(a.h, b.h)
        want = oracle.inner(oracle.simulate(n, a_nets), oracle.simulate(n, b_nets))
        assert abs(got - want) < TOL[dtype] * 10
        assert Q.qtask_compare_states(a.h, a.h) == 0
        assert Q.qtask_compare_states(a.h, b.h) > 0


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("k,b", [(4, 10), (5, 10), (6, 11), (5, 12)])
def test_dense_fusion_on_matrix_cores(dtype, k, b):
    n = 15
    nets = W.layered_circuit(n, 6, 31) + W.dense_random_circuit(n, 4, 32, kinds=W.GATE_KINDS)
    want = oracle.simulate(n, nets, nthreads=oracle.max_threads())
    log("dense", dtype, k, b)
    with sim(n, nets, dtype, tile_bits=b, low_bits=3, fusion=Q.QTASK_FUSE_DENSE, fuse_width=k,
             ckpt_interval=6) as s:
        st = s.update()
        assert st["mfma_flops"] > 0
        check_state(s.state(), want, dtype, "dense k=%d b=%d" % (k, b))
