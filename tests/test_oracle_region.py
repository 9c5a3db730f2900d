"""Pins of the oracle's refined regions of any shape made of level-0 cells
(Sec. 3.4 closing paragraph, App. B; the node classes, the hanging-node
stencil rule and the H-RR gradients on them are readings R30-R32).

* A mask covering the whole box gives the box path bit for bit, and a mask
  covering a rectangle inside a larger box gives the path of that smaller box
  bit for bit (level 0 everywhere, level 1 on the shared nodes): the classes
  derived from the mask and the stencil rule reduce to the box's.
* A stair-stepped circle (Sec. 4.1.2) and an L-shaped region (a concave
  corner) admit valid couples at every co-located node under DC1 and DC2,
  keep a uniform flow, and, with a centred pulse in a centred circle, keep
  the square's symmetry (transposition and mirror images) to rounding.
* Every level-0 co-located node has its level-1 partner, and holes are
  exactly the nodes whose four cells are refined."""
import numpy as np
import pytest

import oracle as O
from paper_2004_14887_amd import workloads as W

N = 64
BOX = ((12, 12), (52, 52))
HOLE, BULK, TFC, TFF, IE = 0, 1, 2, 3, 4


def run(wl, region=None, steps=10, coupling=2):
    o = O.Oracle("D2Q9", wl.n0, wl.boxes, wl.tau0, coupling, wl.eq_order, [], 1)
    if region is not None:
        o.set_region(region)
    for l in range(wl.n_levels):
        rho, u = W.initial_fields(wl, l)
        o.init(l, rho, u)
    o.run(steps)
    return o


def pulse(boxes, c=(30.0, 33.0)):
    return W.Workload("p", "D2Q9", (N, N), boxes, 0.55, 10, pulses=[dict(c=(c[0], c[1], 0.0), A=1e-3, Rc=3.0)],
                      background=(0.03, 0.01, 0.0))


def same(a, b):
    return np.array_equal(np.nan_to_num(a, nan=7.0), np.nan_to_num(b, nan=7.0))


@pytest.mark.parametrize("coupling", [1, 2])
def test_full_mask_is_the_box(coupling):
    a = run(pulse([BOX]), np.ones((40, 40), np.uint8), coupling=coupling)
    b = run(pulse([BOX]), None, coupling=coupling)
    for l in range(2):
        assert same(a.f(l), b.f(l))


@pytest.mark.parametrize("coupling", [1, 2])
def test_rectangle_in_a_larger_box_is_the_smaller_box(coupling):
    big, small = ((10, 11), (54, 53)), ((14, 16), (47, 49))
    m = np.zeros((53 - 11, 54 - 10), np.uint8)
    m[16 - 11:49 - 11, 14 - 10:47 - 10] = 1
    a = run(pulse([big]), m, coupling=coupling)
    b = run(pulse([small]), None, coupling=coupling)
    assert same(a.f(0), b.f(0))
    fa = a.f(1).reshape(9, 2 * (53 - 11) + 1, 2 * (54 - 10) + 1)
    fb = b.f(1).reshape(9, 2 * (49 - 16) + 1, 2 * (47 - 14) + 1)
    oy, ox = 2 * (16 - 11), 2 * (14 - 10)
    sub = fa[:, oy:oy + fb.shape[1], ox:ox + fb.shape[2]]
    assert same(sub, fb)
    assert np.isnan(np.delete(fa, np.s_[ox:ox + fb.shape[2]], axis=2)).all()


def circle():
    return W.circle_region(BOX, (32.0, 32.0), 16.0)


def l_shape():
    m = np.ones((40, 40), np.uint8)
    m[20:, 20:] = 0
    return m


@pytest.mark.parametrize("region", [circle, l_shape])
@pytest.mark.parametrize("coupling", [1, 2])
def test_uniform_flow_is_kept(region, coupling):
    wl = W.Workload("u", "D2Q9", (N, N), [BOX], 0.55, 10, background=(0.04, -0.02, 0.0))
    o = run(wl, region(), coupling=coupling)
    fe = O.feq("D2Q9", 1.0, np.array([0.04, -0.02, 0.0]))
    for l in range(2):
        f = o.f(l)
        m = ~np.isnan(f[0])
        assert m.sum() > 1000
        assert np.abs(f[:, m] - fe[:, None]).max() < 1e-14


@pytest.mark.parametrize("coupling", [1, 2])
def test_centred_pulse_in_a_circle_keeps_the_square_symmetry(coupling):
    wl = pulse([BOX], c=(32.0, 32.0))
    wl.background = (0.0, 0.0, 0.0)
    o = run(wl, circle(), steps=40, coupling=coupling)
    r0 = o.f(0).sum(0).reshape(N, N)
    r1 = o.f(1).sum(0).reshape(81, 81)
    assert np.nanmax(np.abs(r1 - 1)) > 1e-5
    assert np.nanmax(np.abs(r0 - r0.T)) < 1e-13
    assert np.nanmax(np.abs(r0 - np.roll(r0[:, ::-1], 1, axis=1))) < 1e-13
    assert np.nanmax(np.abs(r1 - r1.T)) < 1e-13
    assert np.nanmax(np.abs(r1 - r1[:, ::-1])) < 1e-13


def test_classes_pair_up():
    o = O.Oracle("D2Q9", (N, N), [BOX], 0.55, 2, 2, [], 1)
    m = circle()
    o.set_region(m)
    c0 = o.classes(0).reshape(N, N)
    c1 = o.classes(1).reshape(81, 81)
    ys, xs = np.nonzero(c0 == TFC)
    assert len(xs) > 50
    assert (c1[2 * (ys - 12), 2 * (xs - 12)] == TFF).all()
    assert (c1 == TFF).sum() == len(xs)
    # holes: all four incident cells refined
    pad = np.zeros((42, 42), np.uint8)
    pad[1:41, 1:41] = m
    four = pad[:-1, :-1] & pad[:-1, 1:] & pad[1:, :-1] & pad[1:, 1:]
    assert np.array_equal(c0[12:53, 12:53] == HOLE, four.astype(bool))


def test_region_validation():
    o3 = O.Oracle("D2Q9", (N, N), [BOX, ((10, 10), (30, 30))], 0.55, 2, 2, [], 1)
    with pytest.raises(ValueError):
        o3.set_region(circle())
    o = O.Oracle("D2Q9", (N, N), [BOX], 0.55, 2, 2, [], 1)
    o.set_region(circle())
    o.set_collision("hrr", 0.98, True)


# ---------------------------------------------------------------- H-RR on regions
# The gradients of Sec. 3.3 on a stair-stepped interface (reading R32): a
# point of a fine co-located node's coarse stencil that is not a node of the
# fine level is a parent node, and that parent node is then a bulk node (its
# fine partner would exist if it were co-located or a hole), so the parent's
# ring of complete macroscopic fields serves it as on a box.

def hrr_run(wl, region, steps, coupling=2):
    o = O.Oracle("D2Q9", wl.n0, wl.boxes, wl.tau0, coupling, 3, [], 1)
    if region is not None:
        o.set_region(region)
    o.set_collision("hrr", 0.98, True)
    for l in range(wl.n_levels):
        rho, u = W.initial_fields(wl, l)
        o.init(l, rho, u)
    o.run(steps)
    return o


@pytest.mark.parametrize("coupling", [1, 2])
def test_hrr_full_mask_is_the_box(coupling):
    a = hrr_run(pulse([BOX]), np.ones((40, 40), np.uint8), 6, coupling)
    b = hrr_run(pulse([BOX]), None, 6, coupling)
    for l in range(2):
        assert same(a.f(l), b.f(l))


@pytest.mark.parametrize("region", [circle, l_shape])
def test_hrr_uniform_flow_and_symmetry(region):
    wl = W.Workload("u", "D2Q9", (N, N), [BOX], 0.55, 6, background=(0.04, -0.02, 0.0))
    o = hrr_run(wl, region(), 6)
    fe = O.feq("D2Q9", 1.0, np.array([0.04, -0.02, 0.0]), 3)
    for l in range(2):
        assert np.nanmax(np.abs(o.f(l) - fe[:, None])) < 1e-14
    if region is circle:
        wl = pulse([BOX], c=(32.0, 32.0))
        wl.background = (0.0, 0.0, 0.0)
        o = hrr_run(wl, circle(), 30)
        r0, r1 = o.f(0).sum(0).reshape(N, N), o.f(1).sum(0).reshape(81, 81)
        assert np.nanmax(np.abs(r0 - r0.T)) < 1e-13
        assert np.nanmax(np.abs(r1 - r1.T)) < 1e-13 and np.nanmax(np.abs(r1 - r1[:, ::-1])) < 1e-13


@pytest.mark.parametrize("region", [circle, l_shape])
@pytest.mark.parametrize("substep", [1, 2])
def test_hrr_linear_field_gradients_on_a_region(region, substep):
    """A linear velocity field's gradient is A / 2^l at every node class of a
    stair-stepped interface: bulk, TF^c (hole neighbours from the child),
    TF^f (coarse stencil, missing fine points from the parent) and IE
    (interpolated with weights summing to one)."""
    wl = W.Workload("lin", "D2Q9", (N, N), [BOX], 0.55, 1)
    rng = np.random.default_rng(3)
    A = 1e-3 * (2 * rng.random((2, 2)) - 1)
    c = np.array([32.0, 32.0])
    o = O.Oracle("D2Q9", wl.n0, wl.boxes, 0.55, 2, 3, [], 1)
    o.set_region(region())
    o.set_collision("hrr", 0.98, True)
    for l in range(2):
        pos = W.node_positions(wl, l)
        o.init(l, np.ones(pos.shape[1]), A @ (pos[:2] - c[:, None]))
    for l in range(2):
        G = o.hrr_gradients(l, substep)[0][:2, :2]
        cls = o.classes(l)
        idx = np.indices((wl.dims(l)[1], wl.dims(l)[0])).reshape(2, -1)
        m = (cls != HOLE) & (idx[0] >= 2) & (idx[0] <= wl.dims(l)[1] - 3) & (idx[1] >= 2) & \
            (idx[1] <= wl.dims(l)[0] - 3) if l == 0 else (cls != HOLE)
        assert {TFF, IE} <= set(np.unique(cls[m])) if l == 1 else TFC in set(np.unique(cls[m]))
        err = np.abs(G[:, :, m] - (A / 2.0 ** l)[:, :, None]).max() / np.abs(A).max()
        assert err < 1e-10, (l, err)


def test_l_shape_inner_corner_is_the_convex_corner_of_appendix_b():
    """App. B prints the sets of a convex corner (fine grid on three
    quadrants, coarse grid on the upper-right one): an L-shaped region
    missing its upper-right block has that corner, and the sets its
    co-located node gets from the region's occupancy are the printed ones."""
    rows = {}
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "index_sets.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                p = line.split()
                rows.setdefault(p[0], {})[p[1]] = {int(v) for v in p[2:]}
    m = np.ones((40, 40), np.uint8)
    m[20:, 20:] = 0                       # the block above-right of cell corner (20, 20) is coarse
    for coupling in (1, 2):
        o = O.Oracle("D2Q9", (N, N), [BOX], 0.55, coupling, 2, [], 1)
        o.set_region(m)
        assert o.classes(1).reshape(81, 81)[40, 40] == TFF
        Kf, Kc = o.node_masks(1, (40, 40))
        rc, s = O.sets("D2Q9", Kf, Kc, coupling)
        assert rc == 0
        for key in ("P", "Qf", "Mf"):
            assert s[key] == rows["convex"][key], (coupling, key)
        # and the outer corners of the same region are the concave corner, rotated
        Kf, Kc = o.node_masks(1, (80, 0))
        rc, s = O.sets("D2Q9", Kf, Kc, coupling)
        assert rc == 0 and len(s["Mf"]) == len(rows["concave"]["Mf"])
