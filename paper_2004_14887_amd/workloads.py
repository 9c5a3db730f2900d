"""Seeded synthetic workloads: mesh layouts and analytic initial fields.

This module holds no part of the lattice Boltzmann method or of the grid
coupling.  It only describes meshes (a periodic coarse domain and nested
refined boxes) and evaluates the paper's analytic initial fields at node
positions, so that the HIP library and the CPU oracle start from the same
numbers:

* the barotropic convected vortex, an exact steady solution of the isothermal
  Euler equations (Sec. 4.2, Eq.(init_COVO));
* the Gaussian acoustic pulse (Sec. 4.1, Eq.(init_Pulse)), read with a radial
  distance r^2 = x^2 + y^2 (+ z^2);
* a divergence-free vortex ring for 3-D cases (curl of an azimuthal vector
  potential), a synthetic stand-in for 3-D vortical structures.

All lengths are in coarse (level-0) cells, all velocities in lattice units;
under acoustic scaling velocities are the same on every level.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

CS2 = 1.0 / 3.0
CS = math.sqrt(CS2)


@dataclasses.dataclass
class Workload:
    name: str
    lattice: str                      # "D2Q9" | "D3Q19"
    n0: Tuple[int, ...]               # periodic coarse domain, nodes per axis
    boxes: List[Tuple[Tuple[int, ...], Tuple[int, ...]]]  # per refined level: (lo, hi) in parent node coords
    tau0: float
    steps: int
    coupling: int = 2                 # 1 = DC1, 2 = DC2
    eq_order: int = 2
    probes: List[Tuple[int, ...]] = dataclasses.field(default_factory=list)
    background: Tuple[float, ...] = (0.0, 0.0, 0.0)
    vortices: List[dict] = dataclasses.field(default_factory=list)   # 2-D barotropic vortices
    pulses: List[dict] = dataclasses.field(default_factory=list)
    rings: List[dict] = dataclasses.field(default_factory=list)      # 3-D vortex rings
    seed: int = 0
    collision: str = "bgk"            # "bgk" | "hrr" (Sec. 2; Sec. 3.3 and 3.5 on refined meshes)
    hrr_sigma: float = 0.98
    hrr_psi: bool = True
    sponge_cells: int = 0             # absorbing layer on level 0 (width in cells; 0: none)
    sponge_sigma: float = 0.0
    region: Optional[np.ndarray] = None   # level 1 as a [ny, nx] mask of level-0 cells over its box (None: the box)

    @property
    def D(self) -> int:
        return 2 if self.lattice == "D2Q9" else 3

    @property
    def Q(self) -> int:
        return 9 if self.lattice == "D2Q9" else 19

    @property
    def n_levels(self) -> int:
        return 1 + len(self.boxes)

    def dims(self, l: int) -> Tuple[int, int, int]:
        return level_dims(self)[l]

    def n_nodes(self, l: int) -> int:
        d = self.dims(l)
        return d[0] * d[1] * d[2]


def level_dims(wl: Workload) -> List[Tuple[int, int, int]]:
    """Dense node counts per level: level 0 is n0; level l+1 has 2*(hi-lo)+1
    nodes per axis (cell-vertex, both box faces included)."""
    out = []
    d0 = list(wl.n0[:wl.D]) + [1] * (3 - wl.D)
    out.append(tuple(d0))
    for lo, hi in wl.boxes:
        d = [2 * (hi[a] - lo[a]) + 1 for a in range(wl.D)] + [1] * (3 - wl.D)
        out.append(tuple(d))
    return out


def level_origin(wl: Workload, l: int) -> np.ndarray:
    """Level-0 coordinate of node 0 of level l."""
    off = np.zeros(3)
    for k in range(1, l + 1):
        lo = wl.boxes[k - 1][0]
        for a in range(wl.D):
            off[a] += lo[a] / float(2 ** (k - 1))
    return off


def node_positions(wl: Workload, l: int) -> np.ndarray:
    """[3, n] level-0 coordinates of the dense nodes of level l, x fastest."""
    d = wl.dims(l)
    off = level_origin(wl, l)
    h = 1.0 / 2 ** l
    z, y, x = np.meshgrid(np.arange(d[2]), np.arange(d[1]), np.arange(d[0]), indexing="ij")
    pos = np.stack([off[0] + h * x.ravel(), off[1] + h * y.ravel(), off[2] + h * z.ravel()])
    if wl.D == 2:
        pos[2] = 0.0
    return pos


def _min_image(d: np.ndarray, L: float) -> np.ndarray:
    return d - L * np.round(d / L)


def initial_fields(wl: Workload, l: int) -> Tuple[np.ndarray, np.ndarray]:
    """(rho[n], u[D, n]) of the analytic initial state on level l."""
    pos = node_positions(wl, l)
    n = pos.shape[1]
    rho = np.ones(n)
    u = np.zeros((3, n))
    for a in range(3):
        u[a] += wl.background[a] if a < len(wl.background) else 0.0
    L = [float(wl.n0[a]) if a < wl.D else 1.0 for a in range(3)]
    for v in wl.vortices:
        dx = _min_image(pos[0] - v["xc"], L[0])
        dy = _min_image(pos[1] - v["yc"], L[1])
        r2 = (dx * dx + dy * dy) / (v["Rc"] ** 2)
        g = np.exp(-0.5 * r2)
        u[0] += -v["eps"] * (dy / v["Rc"]) * g
        u[1] += v["eps"] * (dx / v["Rc"]) * g
        rho *= np.exp(-(v["eps"] ** 2) / (2.0 * CS2) * np.exp(-r2))
    for p in wl.pulses:
        r2 = np.zeros(n)
        for a in range(wl.D):
            d = _min_image(pos[a] - p["c"][a], L[a])
            r2 += d * d
        rho *= 1.0 + p["A"] * np.exp(-r2 / (2.0 * p["Rc"] ** 2))
    for rg in wl.rings:
        u += _ring_velocity(pos, rg, L)
    return rho, u[:wl.D].copy()


def _ring_frame(axis):
    n = np.asarray(axis, float)
    n = n / np.linalg.norm(n)
    t = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(n, t)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(n, e1)
    return n, e1, e2


def _ring_profile(r, z, R, s):
    """(u_r, u_z) for the potential A(r,z) = (r/R) exp(-((r-R)^2+z^2)/(2 s^2)),
    u = curl(A e_phi), with unit amplitude."""
    E = np.exp(-((r - R) ** 2 + z ** 2) / (2.0 * s * s))
    ur = (r / R) * E * z / (s * s)
    uz = (E / R) * (2.0 - r * (r - R) / (s * s))
    return ur, uz


def _ring_velocity(pos, rg, L):
    n, e1, e2 = _ring_frame(rg["axis"])
    d = np.stack([_min_image(pos[a] - rg["c"][a], L[a]) for a in range(3)])
    zc = n @ d
    rvec = d - np.outer(n, zc)
    r = np.sqrt((rvec * rvec).sum(0))
    ur, uz = _ring_profile(r, zc, rg["R"], rg["core"])
    # unit amplitude -> peak speed rg["peak"], peak taken on a fixed fine sample
    rr, zz = np.meshgrid(np.linspace(0, 3 * rg["R"], 601), np.linspace(-3 * rg["R"], 3 * rg["R"], 601))
    a, b = _ring_profile(rr, zz, rg["R"], rg["core"])
    scale = rg["peak"] / np.sqrt(a * a + b * b).max()
    safe = np.where(r > 1e-12, r, 1.0)
    er = np.where(r > 1e-12, rvec / safe, 0.0)
    return scale * (er * ur + np.outer(n, uz))


# --------------------------------------------------------------------------
# The same fields evaluated with torch on a device, for meshes whose finest
# level holds ~1e9 nodes.  Every vortex, pulse and ring decays like a
# Gaussian away from its core, so each is evaluated only on the nodes within
# `cut` core radii of it (outside, its contribution is below e^(-cut^2/2)
# of its peak, 1.3e-14 at cut = 8); inside, the formulas and their order are
# those of initial_fields.
# --------------------------------------------------------------------------

def _axis_runs(wl, l, a, c, ext):
    """Contiguous index runs of level l along axis a whose min-image distance
    to coordinate c is at most ext."""
    d = wl.dims(l)[a]
    L = float(wl.n0[a]) if a < wl.D else 1.0
    pos = level_origin(wl, l)[a] + np.arange(d) / 2.0 ** l
    near = np.abs(_min_image(pos - c, L)) <= ext
    runs, i = [], 0
    while i < d:
        if near[i]:
            j = i
            while j < d and near[j]:
                j += 1
            runs.append((i, j))
            i = j
        else:
            i += 1
    return runs


def _boxes(wl, l, c, ext):
    """Sub-boxes ((z0, z1), (y0, y1), (x0, x1)) of level l within ext of point c."""
    rx = _axis_runs(wl, l, 0, c[0], ext)
    ry = _axis_runs(wl, l, 1, c[1], ext)
    rz = _axis_runs(wl, l, 2, c[2], ext) if wl.D == 3 else [(0, 1)]
    return [(z, y, x) for z in rz for y in ry for x in rx]


def _box_displacements(torch, wl, l, box, c, device, zs):
    """Min-image displacements (dx, dy, dz) from c over box rows zs."""
    off = level_origin(wl, l)
    h = 1.0 / 2 ** l
    L = [float(wl.n0[a]) if a < wl.D else 1.0 for a in range(3)]
    (_, _), (y0, y1), (x0, x1) = box
    f64 = torch.float64

    def axis(a, lo, hi):
        p = off[a] + h * torch.arange(lo, hi, dtype=f64, device=device)
        dd = p - c[a]
        return dd - L[a] * torch.round(dd / L[a])

    dx = axis(0, x0, x1).view(1, 1, -1)
    dy = axis(1, y0, y1).view(1, -1, 1)
    if wl.D == 3:
        dz = axis(2, zs[0], zs[1]).view(-1, 1, 1)
    else:
        dz = torch.zeros((1, 1, 1), dtype=f64, device=device)
    return dx, dy, dz


def initial_fields_device(wl: Workload, l: int, device, cut: float = 8.0, slab_nodes: int = 1 << 25):
    """(rho[n], u[D, n]) of level l as float64 torch tensors on `device`, the
    fields of initial_fields evaluated on each structure's bounding box."""
    import torch

    d = wl.dims(l)
    n = d[0] * d[1] * d[2]
    rho = torch.ones(n, dtype=torch.float64, device=device)
    u = torch.empty((wl.D, n), dtype=torch.float64, device=device)
    for a in range(wl.D):
        u[a].fill_(wl.background[a] if a < len(wl.background) else 0.0)
    rho3 = rho.view(d[2], d[1], d[0])
    u3 = [u[a].view(d[2], d[1], d[0]) for a in range(wl.D)]

    def slabs(box):
        (z0, z1), (y0, y1), (x0, x1) = box
        per = max(1, slab_nodes // max(1, (y1 - y0) * (x1 - x0)))
        for z in range(z0, z1, per):
            yield (z, min(z1, z + per))

    for v in wl.vortices:
        c = (v["xc"], v["yc"], 0.0)
        for box in _boxes(wl, l, c, cut * v["Rc"]):
            (_, _), (y0, y1), (x0, x1) = box
            for zs in slabs(box):
                dx, dy, _ = _box_displacements(torch, wl, l, box, c, device, zs)
                r2 = (dx * dx + dy * dy) / (v["Rc"] ** 2)
                g = torch.exp(-0.5 * r2)
                u3[0][zs[0]:zs[1], y0:y1, x0:x1] += -v["eps"] * (dy / v["Rc"]) * g
                u3[1][zs[0]:zs[1], y0:y1, x0:x1] += v["eps"] * (dx / v["Rc"]) * g
                rho3[zs[0]:zs[1], y0:y1, x0:x1] *= torch.exp(-(v["eps"] ** 2) / (2.0 * CS2) * torch.exp(-r2))
    for p in wl.pulses:
        c = tuple(p["c"]) + (0.0,) * (3 - len(p["c"]))
        for box in _boxes(wl, l, c, cut * p["Rc"]):
            (_, _), (y0, y1), (x0, x1) = box
            for zs in slabs(box):
                dx, dy, dz = _box_displacements(torch, wl, l, box, c, device, zs)
                r2 = dx * dx + dy * dy
                if wl.D == 3:
                    r2 = r2 + dz * dz
                rho3[zs[0]:zs[1], y0:y1, x0:x1] *= 1.0 + p["A"] * torch.exp(-r2 / (2.0 * p["Rc"] ** 2))
    for rg in wl.rings:
        nax, _, _ = _ring_frame(rg["axis"])
        rr, zz = np.meshgrid(np.linspace(0, 3 * rg["R"], 601), np.linspace(-3 * rg["R"], 3 * rg["R"], 601))
        a_, b_ = _ring_profile(rr, zz, rg["R"], rg["core"])
        scale = rg["peak"] / np.sqrt(a_ * a_ + b_ * b_).max()
        c = tuple(rg["c"])
        for box in _boxes(wl, l, c, rg["R"] + cut * rg["core"]):
            (_, _), (y0, y1), (x0, x1) = box
            for zs in slabs(box):
                dx, dy, dz = _box_displacements(torch, wl, l, box, c, device, zs)
                shape = (zs[1] - zs[0], y1 - y0, x1 - x0)
                dd = [dx.expand(shape), dy.expand(shape), dz.expand(shape)]
                zc = nax[0] * dd[0] + nax[1] * dd[1] + nax[2] * dd[2]
                rv = [dd[a] - nax[a] * zc for a in range(3)]
                r = torch.sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2])
                E = torch.exp(-((r - rg["R"]) ** 2 + zc ** 2) / (2.0 * rg["core"] * rg["core"]))
                ur = (r / rg["R"]) * E * zc / (rg["core"] * rg["core"])
                uz = (E / rg["R"]) * (2.0 - r * (r - rg["R"]) / (rg["core"] * rg["core"]))
                big = r > 1e-12
                safe = torch.where(big, r, torch.ones_like(r))
                for a in range(3):
                    er = torch.where(big, rv[a] / safe, torch.zeros_like(r))
                    u3[a][zs[0]:zs[1], y0:y1, x0:x1] += scale * (er * ur + nax[a] * uz)
    return rho, u


# --------------------------------------------------------------------------
# The configurations
# --------------------------------------------------------------------------

def _ring_probes(center, radius, count, D):
    out = []
    for k in range(count):
        a = 2.0 * math.pi * k / count
        p = [int(round(center[0] + radius * math.cos(a))), int(round(center[1] + radius * math.sin(a)))]
        out.append(tuple(p[:D]))
    return out


def _sphere_probes(center, radius, count):
    out = []
    g = math.pi * (3.0 - math.sqrt(5.0))
    for k in range(count):
        z = 1.0 - 2.0 * (k + 0.5) / count
        r = math.sqrt(1.0 - z * z)
        t = g * k
        out.append(tuple(int(round(center[a] + radius * v))
                         for a, v in enumerate((r * math.cos(t), r * math.sin(t), z))))
    return out


def vortex_2level(seed: int = 1, n0: int = 128, steps: int = 200, coupling: int = 2) -> Workload:
    """D2Q9 BGK FP64: periodic n0^2 with a centred n0/2 patch refined x2;
    two barotropic vortices (Mach 0.1 background, strength 0.1 U0, radius 8)
    positioned to cross the coarse->fine and fine->coarse faces; 16 probes."""
    rng = np.random.default_rng(seed)
    U0 = 0.1 * CS
    jit = rng.uniform(-0.5, 0.5, size=2)
    q = n0 // 4
    c = n0 / 2.0
    vort = [dict(xc=q - 6 + jit[0], yc=c + jit[1], eps=0.1 * U0, Rc=8.0),
            dict(xc=3 * q - 6 + jit[0], yc=c + jit[1], eps=0.1 * U0, Rc=8.0)]
    probes = _ring_probes((c, c), 0.375 * n0, 8, 2) + _ring_probes((c, c), 0.15625 * n0, 8, 2)
    return Workload(name=f"vortex_2level_{n0}", lattice="D2Q9", n0=(n0, n0),
                    boxes=[((q, q), (3 * q, 3 * q))], tau0=0.55, steps=steps, coupling=coupling,
                    probes=probes, background=(U0, 0.0, 0.0), vortices=vort, seed=seed)


def pulse_plane(n0: int = 150, coupling: int = 2, tau0: float = 0.51, steps: int = 90,
                lattice: str = "D2Q9", collision: str = "bgk") -> Workload:
    """The acoustic pulse across plane refinement interfaces (Sec. 4.1.1) at
    the paper's resolution: a 3 m periodic square of 150 coarse cells
    (dx^c = 0.02 m), the Gaussian pulse of Eq.(init_Pulse) at its centre
    (A = 1e-3, R_c = 0.1 m = 5 cells), and a refined band whose x faces lie
    37 cells (0.74 m) either side of the centre.  The paper's band is periodic
    in y; a nested box cannot touch the periodic boundary, so the band stops
    3 cells short of it, and the y faces are first reached by the pulse's
    front after about 100 coarse steps, after the 90 steps used here."""
    c = n0 / 2.0
    half = int(round(0.74 / 3.0 * n0))
    lo = int(round(c)) - half
    boxes = [((lo, 3), (lo + 2 * half, n0 - 3))]
    return Workload(name=f"pulse_plane_{n0}_dc{coupling}", lattice=lattice, n0=(n0, n0), boxes=boxes, tau0=tau0,
                    steps=steps, coupling=coupling, pulses=[dict(c=(c, c, 0.0), A=1e-3, Rc=0.1 / 3.0 * n0)],
                    collision=collision)


# Physical scales of the convected-vortex study (Sec. 4.2): speed of sound,
# kinematic viscosity and the coarse spacing, which fix the lattice time step
# dt = dx / (sqrt(3) c0) and tau0 - 1/2 = 3 nu dt / dx^2.
C0 = 347.3
NU = 1.49e-5
DX_COARSE = 0.02


def physical_tau0(dx: float = DX_COARSE) -> float:
    dt = dx / (math.sqrt(3.0) * C0)
    return 0.5 + 3.0 * NU * dt / dx ** 2


def vortex_plane(n0: int = 150, coupling: int = 2, steps: int = 650, collision: str = "hrr",
                 tau0: float = None, layer: int = 12, layer_sigma: float = 0.3) -> Workload:
    """The barotropic vortex convected across a plane refinement interface
    (Sec. 4.2.1, Eq.(init_COVO)) at the paper's resolution and domain: a 3 m
    square of 150 coarse cells (dx^c = 0.02 m, dx^f = 0.01 m), U_x = 0.1 c0,
    eps = 0.15 U_x, R_c = 0.06 m = 3 coarse cells, the vortex starting 6 R_c
    upstream of the interface, inside the fine region, with the physical
    viscosity (tau0 - 1/2 = 3.7e-6) and the H-RR collision the paper uses for
    it.  36 probes on a circle of 1.2 m (60 coarse cells) around the
    interface's centre, at the nearest coarse nodes.  The paper bounds the
    domain with absorbing layers; here a layer of `layer` cells (0.24 m) at
    the periodic seam absorbs what would come back.  The refined region is
    the box left of the interface, from the layer's inner edge (plus the
    2-cell margin) to the interface, over the height between the layers; the
    vortex crosses only its right face."""
    c = n0 // 2
    U = 0.1 * CS
    Rc = 0.06 / DX_COARSE
    m = layer + 2
    boxes = [((m, m), (c, n0 - m))]
    probes = []
    for k in range(36):
        th = 2.0 * math.pi * k / 36.0
        probes.append((int(round(c + 60.0 * math.cos(th))), int(round(c + 60.0 * math.sin(th)))))
    vort = [dict(xc=c - 6.0 * Rc, yc=float(c), eps=0.15 * U, Rc=Rc)]
    return Workload(name=f"vortex_plane_{n0}_dc{coupling}", lattice="D2Q9", n0=(n0, n0), boxes=boxes,
                    tau0=physical_tau0() if tau0 is None else tau0, steps=steps, coupling=coupling, eq_order=3,
                    probes=probes, background=(U, 0.0, 0.0), vortices=vort, collision=collision,
                    sponge_cells=layer, sponge_sigma=layer_sigma if layer else 0.0)


def circle_region(box, centre, radius: float) -> np.ndarray:
    """[ny, nx] mask of the level-0 cells of box = ((lo), (hi)) whose centres
    lie within `radius` cells of `centre`: a stair-stepped circular refined
    region (Sec. 4.1.2, Fig. PulseCir_mesh)."""
    (lx, ly), (hx, hy) = box[0][:2], box[1][:2]
    cy, cx = np.mgrid[0:hy - ly, 0:hx - lx]
    px, py = lx + cx + 0.5, ly + cy + 0.5
    return ((px - centre[0]) ** 2 + (py - centre[1]) ** 2 <= radius * radius).astype(np.uint8)


def pulse_circle(n0: int = 150, coupling: int = 2, tau0: float = 0.51, steps: int = 90) -> Workload:
    """The acoustic pulse across a circular refinement interface (Sec. 4.1.2)
    at the paper's resolution: the domain and pulse of pulse_plane, the
    refined region the level-0 cells within 1 m (50 cells) of the pulse's
    centre, stair-stepped as in Fig. PulseCir_mesh."""
    c = n0 / 2.0
    R = 1.0 / 3.0 * n0
    lo, hi = int(math.floor(c - R)) - 1, int(math.ceil(c + R)) + 1
    box = ((lo, lo), (hi, hi))
    wl = Workload(name=f"pulse_circle_{n0}_dc{coupling}", lattice="D2Q9", n0=(n0, n0), boxes=[box], tau0=tau0,
                  steps=steps, coupling=coupling, pulses=[dict(c=(c, c, 0.0), A=1e-3, Rc=0.1 / 3.0 * n0)])
    wl.region = circle_region(box, (c, c), R)
    return wl


def vortex_inclined(n0: int = 150, coupling: int = 2, steps: int = 650, collision: str = "hrr",
                    tau0: float = None, layer: int = 12, layer_sigma: float = 0.3) -> Workload:
    """The convected vortex of vortex_plane across a 30-degree-inclined
    interface (Sec. 4.2.2, Fig. COVO_inclined_mesh): the refined region is the
    stair-stepped set of level-0 cells left of the line through the domain's
    centre leaning 30 degrees from the vertical (x = c + tan(30) (y - c)),
    within the layers; the vortex crosses it at the centre.  Same flow,
    collision, probes, layers and steps as the plane case."""
    wl = vortex_plane(n0=n0, coupling=coupling, steps=steps, collision=collision, tau0=tau0, layer=layer,
                      layer_sigma=layer_sigma)
    c = n0 // 2
    m = layer + 2
    t = math.tan(math.radians(30.0))
    hi_x = int(math.ceil(c + t * (n0 - m - c))) + 2
    box = ((m, m), (min(hi_x, n0 - m), n0 - m))
    wl.boxes = [box]
    cy, cx = np.mgrid[0:box[1][1] - box[0][1], 0:box[1][0] - box[0][0]]
    px, py = box[0][0] + cx + 0.5, box[0][1] + cy + 0.5
    wl.region = (px < c + t * (py - c)).astype(np.uint8)
    wl.name = f"vortex_inclined_{n0}_dc{coupling}"
    return wl


def uniform_fine_reference(wl: Workload) -> Workload:
    """The reference of the reflection study (Sec. 4.1.1): the same domain and
    fields on one periodic level at the resolution of wl's first refined
    level (twice as many nodes per axis, tau from Eq.(rescTau)), run for
    twice as many steps.  Its node i (per axis) sits at coarse coordinate
    i / 2, so wl's level-1 node k matches reference node 2 lo + k."""
    assert wl.n_levels >= 2
    scale = lambda v: tuple(2.0 * x for x in v)
    pulses = [dict(c=scale(p["c"]), A=p["A"], Rc=2.0 * p["Rc"]) for p in wl.pulses]
    vort = [dict(xc=2.0 * v["xc"], yc=2.0 * v["yc"], eps=v["eps"], Rc=2.0 * v["Rc"]) for v in wl.vortices]
    assert not wl.rings
    return Workload(name=wl.name + "_reference", lattice=wl.lattice, n0=tuple(2 * n for n in wl.n0), boxes=[],
                    tau0=2.0 * wl.tau0 - 0.5, steps=2 * wl.steps, coupling=wl.coupling, eq_order=wl.eq_order,
                    background=wl.background, vortices=vort, pulses=pulses, collision=wl.collision,
                    hrr_sigma=wl.hrr_sigma, hrr_psi=wl.hrr_psi)


def pulse_vortices_3level(seed: int = 2, n0: int = 2048, steps: int = 1000, coupling: int = 2,
                          tau0: float = 0.55) -> Workload:
    """D2Q9, 3 levels: periodic n0^2, nested x2 patch over 25% and x4 patch over
    6.25% of the domain; Gaussian pulse (1e-3, half-width 6) plus 16 seeded
    barotropic vortices (swirl Mach 0.05-0.2, radius 8); 16 probes."""
    assert n0 % 16 == 0
    rng = np.random.default_rng(seed)
    q = n0 // 4
    c = n0 / 2.0
    vort = []
    for _ in range(16):
        xc, yc = rng.uniform(0, n0, size=2)
        vort.append(dict(xc=float(xc), yc=float(yc), eps=float(rng.uniform(0.05, 0.2)) * CS, Rc=8.0))
    pulses = [dict(c=(c, c, 0.0), A=1e-3, Rc=6.0)]
    probes = _ring_probes((c, c), 0.375 * n0, 16, 2)
    return Workload(name=f"pulse_vortices_3level_{n0}", lattice="D2Q9", n0=(n0, n0),
                    boxes=[((q, q), (3 * q, 3 * q)), ((q, q), (3 * q, 3 * q))], tau0=tau0,
                    steps=steps, coupling=coupling, probes=probes, vortices=vort, pulses=pulses,
                    seed=seed)


def pulse_ring_3d(seed: int = 3, n0: int = 256, steps: int = 500, coupling: int = 2,
                  tau0: float = 0.52) -> Workload:
    """D3Q19, 2 levels: periodic n0^3 with the central (n0/2)^3 region refined
    x2; spherical pulse (1e-3, half-width 6) plus a vortex ring convected along
    a seeded axis (background Mach 0.1, ring radius 12, core 3, peak 0.1 U0)."""
    assert n0 % 8 == 0
    rng = np.random.default_rng(seed)
    q = n0 // 4
    c = n0 / 2.0
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    U0 = 0.1 * CS
    R = min(12.0, n0 / 10.0)
    rings = [dict(c=tuple(c - 0.3 * n0 * axis), axis=tuple(axis), R=R, core=R / 4.0, peak=0.1 * U0)]
    pulses = [dict(c=(c, c, c), A=1e-3, Rc=min(6.0, n0 / 16.0))]
    probes = _sphere_probes((c, c, c), 0.46875 * n0, 16)
    return Workload(name=f"pulse_ring_3d_{n0}", lattice="D3Q19", n0=(n0, n0, n0),
                    boxes=[((q, q, q), (3 * q, 3 * q, 3 * q))], tau0=tau0, steps=steps,
                    coupling=coupling, probes=probes, background=tuple(U0 * axis), rings=rings,
                    pulses=pulses, seed=seed)


def uniform_state(lattice: str, n0, boxes, rho0: float = 1.0, u0=(0.0, 0.0, 0.0), tau0: float = 0.6,
                  coupling: int = 2, steps: int = 10) -> Workload:
    """A uniform state (rest or uniform flow) on any mesh."""
    return Workload(name="uniform", lattice=lattice, n0=tuple(n0), boxes=list(boxes), tau0=tau0,
                    steps=steps, coupling=coupling, background=tuple(u0), pulses=[])


def serving_requests(seed: int = 4, n: int = 256, max_levels: int = 3, min_side: int = 64, max_side: int = 1024,
                     min_steps: int = 100, max_steps: int = 2000, n_probes: int = 4):
    """A stream of D2Q9 requests for the serving loop, and their unit-rate
    Poisson inter-arrival gaps (scale by 1 / rate).

    Per request: periodic side S = 2^U(log2 min_side, log2 max_side), a
    multiple of 16; 1..max_levels levels, each refined box U(0.25, 0.5) of its
    parent's extent per axis, placed uniformly at least 4 parent cells from
    the parent's boundary; a background flow of Mach U(0.05, 0.2) in a random
    direction; tau0 ~ U(0.51, 0.6); U_int[min_steps, max_steps] coarse steps;
    one barotropic vortex (strength 0.1 U0, radius max(4, S/16)) and one
    Gaussian pulse (1e-3, half-width 6) at uniform positions; n_probes probes
    at uniform level-0 nodes."""
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(n):
        S = int(round(2.0 ** rng.uniform(math.log2(min_side), math.log2(max_side)) / 16.0)) * 16
        S = max(S, min_side)
        L = int(rng.integers(1, max_levels + 1))
        boxes = []
        ext = (S, S)
        for _ in range(1, L):
            lo, hi = [], []
            for a in range(2):
                side = max(3, int(round(rng.uniform(0.25, 0.5) * ext[a])))
                side = min(side, ext[a] - 8)
                s0 = int(rng.integers(4, ext[a] - 4 - side + 1))
                lo.append(s0)
                hi.append(s0 + side)
            boxes.append((tuple(lo), tuple(hi)))
            ext = (2 * (hi[0] - lo[0]), 2 * (hi[1] - lo[1]))
        mach = float(rng.uniform(0.05, 0.2))
        ang = float(rng.uniform(0.0, 2.0 * math.pi))
        U0 = mach * CS
        bg = (U0 * math.cos(ang), U0 * math.sin(ang), 0.0)
        tau0 = float(rng.uniform(0.51, 0.6))
        steps = int(rng.integers(min_steps, max_steps + 1))
        vc = rng.uniform(0, S, size=2)
        pc = rng.uniform(0, S, size=2)
        vort = [dict(xc=float(vc[0]), yc=float(vc[1]), eps=0.1 * U0, Rc=max(4.0, S / 16.0))]
        pulses = [dict(c=(float(pc[0]), float(pc[1]), 0.0), A=1e-3, Rc=6.0)]
        probes = [tuple(int(v) for v in rng.integers(0, S, size=2)) for _ in range(n_probes)]
        reqs.append(Workload(name=f"request_{k}_S{S}_L{L}", lattice="D2Q9", n0=(S, S), boxes=boxes, tau0=tau0,
                             steps=steps, probes=probes, background=bg, vortices=vort, pulses=pulses, seed=seed))
    gaps = rng.exponential(1.0, size=n)
    return reqs, gaps


def rings_4level(seed: int = 5, n0: int = 512, sides=(344, 476, 544), steps: int = 200, n_rings: int = 64,
                 n_pulses: int = 8, tau0: float = 0.52) -> Workload:
    """D3Q19, 4 levels: periodic n0^3 with three nested centred boxes (sides
    in parent cells; the default 344 / 476 / 544 covers 30.3%, 10.0% and 1.87%
    of the volume, about 206 GB of FP16 storage: a finest box of 3% would
    need about 270 GB); seeded vortex rings
    (radius U(8, 16), core radius/4, peak swirl U(0.05, 0.2) c_s, random axes,
    no background) and Gaussian pulses (1e-3, half-width 6); 16 probes on a
    sphere of radius 0.375 n0.  Replicas keep the layout with smaller n0 and
    sides."""
    rng = np.random.default_rng(seed)
    boxes = []
    ext = n0
    for sd in sides:
        lo = (ext - sd) // 2
        boxes.append(((lo, lo, lo), (lo + sd, lo + sd, lo + sd)))
        ext = 2 * sd
    c = n0 / 2.0
    scale = n0 / 512.0
    rings = []
    for _ in range(n_rings):
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        R = float(rng.uniform(8.0, 16.0)) * max(scale, 0.25)
        rings.append(dict(c=tuple(rng.uniform(0, n0, size=3)), axis=tuple(axis), R=R, core=R / 4.0,
                          peak=float(rng.uniform(0.05, 0.2)) * CS))
    pulses = [dict(c=tuple(rng.uniform(0, n0, size=3)), A=1e-3, Rc=6.0 * max(scale, 0.25))
              for _ in range(n_pulses)]
    probes = _sphere_probes((c, c, c), 0.375 * n0, 16)
    return Workload(name=f"rings_4level_{n0}", lattice="D3Q19", n0=(n0, n0, n0), boxes=boxes, tau0=tau0,
                    steps=steps, probes=probes, rings=rings, pulses=pulses, seed=seed)
