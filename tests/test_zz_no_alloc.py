"""The no-allocation entry point (dclbm_balance_static) against the
entry point it is a variant of (dclbm_balance), through the C ABI, on two
calls in a row, the second on a smaller simulation (run with -m gpu).

The static scratch array keeps the first call's partial sums; the second
call, with fewer levels and fewer nodes, must not see them.  The bar is bit
equality: both run the same kernels over the same blocks."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2004_14887_amd import workloads as W  # noqa: E402

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


def _static_balance(sim):
    from paper_2004_14887_amd import _lib
    out = torch.full((5,), float("nan"), dtype=torch.float64, device=sim.device)
    sim._sync_torch()
    _lib.check(sim.lib.dclbm_balance_static(sim.h, C.c_void_p(out.data_ptr())))
    sim.stream.synchronize()
    return out.cpu().numpy()


@requires_gpu
def test_static_balance_equals_balance_on_consecutive_calls():
    from paper_2004_14887_amd.sim import Simulation

    cases = [(W.pulse_vortices_3level(seed=2, n0=256, steps=6), "fp32"),   # 3 levels, larger
             (W.vortex_2level(seed=1, n0=64, steps=4), "fp64"),            # 2 levels, smaller
             (W.pulse_ring_3d(seed=3, n0=32, steps=3), "fp16")]            # 3-D, smallest
    for wl, prec in cases:
        print(f"[gpu] static balance {wl.name} {prec}", flush=True)
        sim = Simulation(wl, prec, probe_capacity=wl.steps)
        sim.init_from_workload()
        sim.step(wl.steps)
        got = _static_balance(sim)
        ref = np.array(sim.balance())
        sim.check()
        assert np.array_equal(got, ref), (wl.name, got, ref)
        # a second call on the same state gives the same bits
        assert np.array_equal(_static_balance(sim), ref)
        sim.close()


@requires_gpu
def test_static_balance_rejects_null_output():
    from paper_2004_14887_amd import _lib
    from paper_2004_14887_amd.sim import Simulation

    wl = W.vortex_2level(seed=1, n0=64, steps=1)
    sim = Simulation(wl, "fp64", probe_capacity=1)
    sim.init_from_workload()
    assert sim.lib.dclbm_balance_static(sim.h, None) == -1
    assert b"null" in _lib.load().dclbm_last_error()
    sim.close()
