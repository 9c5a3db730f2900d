"""The CPU-baseline build of the oracle (-O3 for the host, OpenMP over the
node loops) computes exactly what the checking build computes: every
node's arithmetic is unchanged and no FMA contraction is allowed, so a
multi-threaded run equals the checking build bit for bit (CPU only)."""
import os
import tempfile

import numpy as np
import pytest

import oracle as O
from paper_2004_14887_amd import workloads as W


@pytest.fixture(scope="module")
def baseline_lib():
    d = tempfile.mkdtemp(prefix="oracle_baseline_")
    try:
        return O.build_baseline(d)
    except Exception as e:   # no OpenMP runtime or compiler on this host
        pytest.skip(f"baseline build unavailable: {e}")


def _run(wl, steps, lib_path=None):
    o = O.Oracle(wl.lattice, wl.n0, wl.boxes, wl.tau0, wl.coupling, wl.eq_order, wl.probes, steps, lib_path=lib_path)
    for l in range(wl.n_levels):
        rho, u = W.initial_fields(wl, l)
        o.init(l, rho, u)
    o.run(steps)
    return o


@pytest.mark.parametrize("make", [lambda: W.pulse_vortices_3level(seed=2, n0=64, steps=6),
                                  lambda: W.pulse_ring_3d(seed=3, n0=24, steps=3, coupling=1)])
def test_baseline_build_equals_checking_build(baseline_lib, make):
    wl = make()
    os.environ.setdefault("OMP_NUM_THREADS", "4")
    a = _run(wl, wl.steps)
    b = _run(wl, wl.steps, baseline_lib)
    assert b.threads() >= 1 and a.threads() == 1
    for l in range(wl.n_levels):
        assert np.array_equal(a.f(l), b.f(l), equal_nan=True)
        assert np.array_equal(a.X(l), b.X(l), equal_nan=True)
    assert np.array_equal(a.probes(), b.probes())
    assert a.newton_stats() == b.newton_stats()
