"""32 qubits in complex128 (a 64 GiB state): closed forms the oracle cannot
reach at this size, and incremental == full re-simulation."""
import math

import numpy as np
import pytest

from paper_2210_01076_amd import workloads as W
from tests.gpu_util import bytes_equal, log, sim

pytestmark = pytest.mark.gpu

N = 32


def test_ghz_32():
    with sim(N, W.ghz_circuit(N), ckpt_interval=8, max_ckpts=1) as s:
        st = s.update()
        log("ghz-32: %d passes %.1f ms" % (st["passes"], st["kernel_ms"]))
        r = 1 / math.sqrt(2)
        head = s.state(0, 4096)
        tail = s.state((1 << N) - 4096, 4096)
        assert abs(head[0] - r) < 1e-15 and abs(tail[-1] - r) < 1e-15
        assert np.max(np.abs(head[1:])) == 0 and np.max(np.abs(tail[:-1])) == 0
        assert abs(s.norm() - 1.0) < 1e-13


def test_qft_32_of_basis_state():
    x = 0x9E3779B9
    M = 1 << N
    with sim(N, W.basis_prep(N, x) + W.qft_circuit(N), ckpt_interval=1000) as s:
        st = s.update()
        log("qft-32: %d passes %.1f ms" % (st["passes"], st["kernel_ms"]))
        rng = np.random.default_rng(7)
        for first in [0, M - 2048] + [int(v) for v in rng.integers(0, M - 2048, size=6)]:
            amp = s.state(first, 2048)
            y = np.arange(first, first + 2048, dtype=np.uint64)
            phase = (np.uint64(x) * y) % np.uint64(M)           # exact integer phase
            want = np.exp(2j * np.pi * phase.astype(np.float64) / M) / 65536.0
            err = float(np.max(np.abs(amp - want)))
            assert err < 1e-12, (first, err)
        assert abs(s.norm() - 1.0) < 1e-12


def test_cp_ladder_32_incremental_equals_full():
    nets = W.cp_ladder_circuit(N, 4, 505)
    batches = W.modifier_batches(N, nets, 606, 3, 1, 1, ("rx", "ry", "rz", "cp"))
    with sim(N, nets, ckpt_interval=3, max_ckpts=2) as s:
        st = s.update()
        log("ladder-32 full: %d passes %.1f ms" % (st["passes"], st["kernel_ms"]))
        for batch in batches:
            for e in batch:
                W.apply_edit(nets, e)
                s.apply_edit(e)
            st = s.update()
            h_inc = s.hash()
            head = s.state(0, 1024)
            sf = s.update(full=True)
            log("ladder-32 inc mode %d from level %d: %.1f ms; full %.1f ms" % (
                st["mode"], st["first_level"], st["kernel_ms"], sf["kernel_ms"]))
            assert h_inc == s.hash()
            assert bytes_equal(head, s.state(0, 1024))
        assert abs(s.norm() - 1.0) < 1e-12
