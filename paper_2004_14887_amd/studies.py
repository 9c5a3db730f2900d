"""The paper's studies of the interface's acoustic behaviour, run on the GPU
path:

* the reflection of an acoustic pulse at plane (Sec. 4.1.1) and circular
  (Sec. 4.1.2) refinement interfaces: the velocity divergence of the refined
  run against a uniform-fine reference run, on the fine region, after the
  pulse has crossed the interface;
* the spurious noise of a vortex convected across a plane (Sec. 4.2.1) or a
  30-degree-inclined (Sec. 4.2.2) interface: the overall sound pressure level
  (OASPL) at 36 far-field probes, from the FP64 running sums of the
  probes that the device keeps over the window.

Both compare the couplings DC1 and DC2.  Every step of both runs is the
library's (through Simulation); what is done here on the host is reading
back the probe series or the divergence fields and reducing them.
"""
from __future__ import annotations

from typing import Optional, Tuple

import numpy as np
import torch

from . import workloads as W
from .sim import Simulation


def oaspl(series: np.ndarray, start: int, stop: int, c0: float = W.C0) -> np.ndarray:
    """OASPL in dB re 2e-5 Pa of each probe (columns) of a series of
    p' = c_s^2 (rho - 1) in lattice units over coarse steps [start, stop):
    pascals are c0^2 rho0 (rho - 1) with rho0 = 1 kg/m^3; the window's mean
    is removed before the root mean square."""
    p = np.asarray(series, dtype=np.float64)[start:stop] * (c0 * c0 / W.CS2)
    p = p - p.mean(axis=0)
    prms = np.sqrt((p * p).mean(axis=0))
    return 20.0 * np.log10(prms / 2e-5)


def oaspl_from_sums(sums: np.ndarray, n: int, c0: float = W.C0) -> np.ndarray:
    """The OASPL of `oaspl` from the running sums of n coarse steps about a
    shift K per probe (rows: sum (p' - K), sum (p' - K)^2, and K, which
    the mean square does not depend on): the mean square about the
    window's mean is sum d^2 / n - (sum d / n)^2."""
    s1, s2 = np.asarray(sums, dtype=np.float64)[:2]
    mean = s1 / n
    prms = np.sqrt(np.maximum(s2 / n - mean * mean, 0.0)) * (c0 * c0 / W.CS2)
    return 20.0 * np.log10(prms / 2e-5)


def _run(wl: W.Workload, precision: str, device: str, steps: Optional[int] = None,
         window: Optional[Tuple[int, int]] = None) -> Simulation:
    sim = Simulation(wl, precision, device=device, probe_capacity=max(1, wl.steps))
    sim.init_from_workload()
    if window is not None:
        sim.set_probe_window(*window)
    sim.step(wl.steps if steps is None else steps)
    sim.check()
    return sim


def reflection(n0: int = 150, steps: int = 90, coupling: int = 2, collision: str = "bgk", tau0: float = 0.51,
               precision: str = "fp64", device: str = "cuda:0", shape: str = "plane") -> dict:
    """Reflected field of the acoustic pulse at the refinement interface of
    workloads.pulse_plane (shape "plane", Sec. 4.1.1) or pulse_circle
    ("circle", Sec. 4.1.2) after `steps` coarse steps: (div u - div u_ref) on
    the refined level's nodes, divided by max |div u_ref| over the reference
    domain.  Returns the field [ny, nx] (NaN where the centred difference is
    undefined: the level's outermost nodes, and nodes next to a region's
    missing nodes), its largest magnitude ("max") and its root mean square
    over the defined nodes ("l2")."""
    if shape == "circle":
        wl = W.pulse_circle(n0=n0, coupling=coupling, tau0=tau0, steps=steps)
        wl.collision = collision
    else:
        wl = W.pulse_plane(n0=n0, coupling=coupling, tau0=tau0, steps=steps, collision=collision)
    ref = W.uniform_fine_reference(wl)
    a = _run(wl, precision, device)
    d1 = a.divergence(1)
    ny, nx = wl.dims(1)[1], wl.dims(1)[0]
    a.close()
    b = _run(ref, precision, device)
    dr = b.divergence(0).reshape(ref.dims(0)[1], ref.dims(0)[0])
    b.close()
    lo = wl.boxes[0][0]
    sub = dr[2 * lo[1]:2 * lo[1] + ny, 2 * lo[0]:2 * lo[0] + nx]
    scale = dr.abs().max()
    rel = ((d1.reshape(ny, nx) - sub) / scale).cpu().numpy()
    m = ~np.isnan(rel)
    return {"field": rel, "max": float(np.abs(rel[m]).max()), "l2": float(np.sqrt((rel[m] ** 2).mean())),
            "div_ref_max": float(scale), "workload": wl.name, "steps": steps}


def vortex_oaspl(n0: int = 150, steps: int = 650, coupling: int = 2, precision: str = "fp64",
                 window: Tuple[int, int] = (200, 650), device: str = "cuda:0", boxes=None,
                 shape: str = "plane") -> dict:
    """OASPL of the spurious noise of workloads.vortex_plane (shape "plane",
    Sec. 4.2.1) or vortex_inclined ("inclined", Sec. 4.2.2), absorbing layers
    included, at its 36 probes over the coarse-step window, from the device's
    running sums ("per_probe"; "per_probe_series" is the same from the
    series); `boxes=[]` runs the same flow without the refinement (the level
    of noise the interface adds to)."""
    make = W.vortex_inclined if shape == "inclined" else W.vortex_plane
    wl = make(n0=n0, coupling=coupling, steps=steps)
    if boxes is not None:
        wl.boxes = boxes
        wl.region = None
    sim = _run(wl, precision, device, window=window)
    series = sim.probes().cpu().numpy()
    sums, n = sim.probe_sums()
    sums = sums.cpu().numpy()
    sim.close()
    L = oaspl_from_sums(sums, n)
    return {"per_probe": L, "max": float(L.max()), "mean": float(L.mean()), "series": series,
            "per_probe_series": oaspl(series, *window), "sums": sums, "n_summed": n,
            "workload": wl.name, "window": list(window)}
