"""Writes vortex_plane_oaspl.json: the FP64 oracle's OASPL of the convected
vortex across a plane refinement interface (Sec. 4.2.1) and across a
30-degree-inclined one (Sec. 4.2.2), DC1 and DC2, at the full size of
workloads.vortex_plane and vortex_inclined (150^2 coarse cells with absorbing
layers, 650 coarse steps, H-RR at the physical viscosity), over the probe
window [200, 650).  Calls only the oracle (and the seeded input generators);
takes a few minutes on 8 cores.

    python tests/golden/make_vortex_plane_oaspl.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2004_14887_amd import workloads as W  # noqa: E402

WINDOW = (200, 650)


def main():
    out = {"workloads": "vortex_plane / vortex_inclined n0=150 layer=12 sigma=0.3 steps=650 H-RR sigma=0.98 psi "
                        "eq_order=3", "window": list(WINDOW), "unit": "dB re 2e-5 Pa", "cases": {}}
    for case, make in (("plane", W.vortex_plane), ("inclined", W.vortex_inclined)):
        res = {"per_probe": {}, "max": {}, "mean": {}}
        for cp in (1, 2):
            wl = make(coupling=cp, steps=WINDOW[1])
            o = O.Oracle(wl.lattice, wl.n0, wl.boxes, wl.tau0, wl.coupling, wl.eq_order, wl.probes, wl.steps)
            if wl.region is not None:
                o.set_region(wl.region)
            o.set_collision("hrr", wl.hrr_sigma, wl.hrr_psi)
            o.set_sponge(wl.sponge_cells, wl.sponge_sigma, wl.background)
            for l in range(wl.n_levels):
                rho, u = W.initial_fields(wl, l)
                o.init(l, rho, u)
            o.run(wl.steps)
            L = O.oaspl(o.probes(), *WINDOW)
            key = f"DC{cp}"
            res["per_probe"][key] = [round(float(v), 4) for v in L]
            res["max"][key] = round(float(L.max()), 4)
            res["mean"][key] = round(float(L.mean()), 4)
            print(case, key, res["max"][key], res["mean"][key], flush=True)
        out["cases"][case] = res
    with open(os.path.join(HERE, "vortex_plane_oaspl.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
