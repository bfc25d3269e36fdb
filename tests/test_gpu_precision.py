"""The complex64 tier: FP32 amplitudes with renormalisation at segment ends
and FP64 reductions, checked against the complex128 path (itself checked
against the oracle) and against the oracle directly."""
import math

import numpy as np
import pytest

from oracle import oracle
from paper_2210_01076_amd import qtask as Q
from paper_2210_01076_amd import workloads as W
from tests.gpu_util import check_state, log, sim

pytestmark = pytest.mark.gpu


def _fidelity_device(a, b):
    ab = Q.qtask_inner(a.h, b.h)
    return abs(ab) ** 2 / (a.norm() * b.norm())


def test_c64_renormalised_vs_c128_and_oracle():
    n = 20
    nets = W.layered_circuit(n, 60, 44)
    want = oracle.simulate(n, nets, nthreads=oracle.max_threads())
    with sim(n, nets, "c128", ckpt_interval=20) as s128, sim(n, nets, "c64", ckpt_interval=20) as s64:
        s128.update()
        st = s64.update()
        assert st["segments_replayed"] == 6
        a = s128.state()
        check_state(a, want, "c128", "c128 vs oracle")
        b = s64.state()
        check_state(b, want, "c64", "c64 vs oracle")
        err = float(np.max(np.abs(a - b.astype(np.complex128))))
        f = _fidelity_device(s64, s128)
        log("c64 vs c128: max-abs %.3e fidelity %.12f norm %.9f" % (err, f, s64.norm()))
        assert err <= 1e-5 and f >= 1 - 1e-6
        assert abs(s64.norm() - 1.0) < 1e-6   # renormalised at the last segment end


def test_c64_without_renorm_drifts_less_than_tolerance_but_renorm_is_tighter():
    n = 18
    nets = W.layered_circuit(n, 40, 45)
    with sim(n, nets, "c64", ckpt_interval=10, renorm=0) as raw, sim(n, nets, "c64", ckpt_interval=10) as ren:
        raw.update()
        ren.update()
        d_raw = abs(raw.norm() - 1.0)
        d_ren = abs(ren.norm() - 1.0)
        log("norm drift raw %.3e renormalised %.3e" % (d_raw, d_ren))
        assert d_ren <= max(d_raw, 1e-7)


@pytest.mark.parametrize("n", [26, 30])
def test_fused_k5_c64_vs_c128_large(n):
    """Configuration-3 shape at reduced depth: dense 5-qubit fused unitaries
    on the matrix cores, complex64 against complex128 on the device."""
    nets = W.layered_circuit(n, 6, 303)
    opts = dict(tile_bits=11, low_bits=4, fusion=Q.QTASK_FUSE_DENSE, fuse_width=5, ckpt_interval=4)
    with sim(n, nets, "c128", **opts) as s128:
        st = s128.update()
        log("n=%d c128 fused: %d passes %.1f ms mfma %.2e flops" % (n, st["passes"], st["kernel_ms"], st["mfma_flops"]))
        with sim(n, nets, "c64", **opts) as s64:
            st64 = s64.update()
            log("n=%d c64 fused: %d passes %.1f ms" % (n, st64["passes"], st64["kernel_ms"]))
            f = _fidelity_device(s64, s128)
            a = s128.state(0, 1 << 16)
            b = s64.state(0, 1 << 16).astype(np.complex128)
            err = float(np.max(np.abs(a - b)))
            log("n=%d c64 vs c128 fidelity %.12f sampled max-abs %.3e" % (n, f, err))
            assert f >= 1 - 1e-6 and err <= 1e-5
        # the same circuit without fusion agrees with the fused result
        with sim(n, nets, "c128", tile_bits=11, low_bits=4, ckpt_interval=4) as plain:
            plain.update()
            np.testing.assert_allclose(plain.state(0, 1 << 16), s128.state(0, 1 << 16), atol=1e-12, rtol=0)
            assert abs(_fidelity_device(plain, s128) - 1.0) < 1e-12
