"""CPU pins of the two acoustic studies (Sec. 4.1.1, Sec. 4.2.1): the OASPL
reduction and the uniform-fine reference of the reflection study.

* OASPL of a sinusoid of amplitude a (Pa) is 20 log10(a / sqrt(2) / 2e-5) dB,
  whatever its mean; both the oracle's reduction and the product's, the
  latter also from running sums of p' and p'^2 about the first sample (over
  whole periods).
* The reflection study's reference (one periodic level at the fine spacing,
  tau from Eq.(rescTau), twice the steps) must equal the refined run on the
  fine region until the pulse reaches the interfaces: with the oracle, after
  5 coarse steps the velocity divergences agree to 1e-10 of the signal
  (measured 1e-11; a reference with the coarse tau, or run for as many steps
  as the coarse level, is off by about 1e-2)."""
import numpy as np
import pytest

import oracle as O
from paper_2004_14887_amd import workloads as W

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("mean", [0.0, 3e-4])
def test_oaspl_of_a_sinusoid(mean):
    a_pa = 0.05
    t = np.arange(400)
    drho = mean + a_pa / W.C0 ** 2 * np.sin(2 * np.pi * t / 40.0)
    series = np.stack([CS2 * drho, 2 * CS2 * drho], axis=1)
    expect = 20 * np.log10(np.array([a_pa, 2 * a_pa]) / np.sqrt(2) / 2e-5)
    assert np.abs(O.oaspl(series, 0, 400) - expect).max() < 1e-9
    studies = pytest.importorskip("paper_2004_14887_amd.studies")
    assert np.abs(studies.oaspl(series, 0, 400) - expect).max() < 1e-9
    # from the running sums the device keeps: the same level
    d = series[100:380] - series[100]
    sums = np.stack([d.sum(axis=0), (d * d).sum(axis=0), series[100]])
    assert np.abs(studies.oaspl_from_sums(sums, 280) - expect).max() < 1e-6
    assert np.abs(studies.oaspl_from_sums(sums, 280) - O.oaspl(series, 100, 380)).max() < 1e-9


def _divergence_run(wl, steps):
    o = O.Oracle(wl.lattice, wl.n0, wl.boxes, wl.tau0, wl.coupling, wl.eq_order, [], 1)
    for l in range(wl.n_levels):
        rho, u = W.initial_fields(wl, l)
        o.init(l, rho, u)
    o.run(steps)
    return o


def _reflected(wl, ref, steps, ref_steps):
    a = _divergence_run(wl, steps)
    b = _divergence_run(ref, ref_steps)
    d1 = O.velocity_divergence(wl.lattice, a.f(1), wl.dims(1), False).reshape(wl.dims(1)[1], wl.dims(1)[0])
    dr = O.velocity_divergence(ref.lattice, b.f(0), ref.dims(0), True).reshape(ref.dims(0)[1], ref.dims(0)[0])
    lo = wl.boxes[0][0]
    ny, nx = d1.shape
    delta = d1 - dr[2 * lo[1]:2 * lo[1] + ny, 2 * lo[0]:2 * lo[0] + nx]
    return np.nanmax(np.abs(delta)) / np.abs(dr).max()


def test_reference_equals_refined_run_before_the_pulse_arrives():
    wl = W.pulse_plane(steps=5)
    ref = W.uniform_fine_reference(wl)
    assert ref.tau0 == pytest.approx(2 * wl.tau0 - 0.5) and ref.n0 == (300, 300)
    assert _reflected(wl, ref, 5, 10) < 1e-10
    # the reference at the coarse tau, or at the coarse step count, is not the fine run
    bad = W.uniform_fine_reference(wl)
    bad.tau0 = wl.tau0
    assert _reflected(wl, bad, 5, 10) > 1e-3
    assert _reflected(wl, ref, 5, 5) > 1e-3
