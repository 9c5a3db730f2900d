"""GPU parity on the mesh shapes, options and failure paths that the main
parity cases do not reach (run with -m gpu): boxes placed off centre with
unequal sides, unequal 3-D extents with probes on the x-face buffers, DC1 on
three levels, the third-order equilibrium on D2Q9, and the instability latch
(a non-finite density found while stepping) for single simulations and for a
served request whose neighbours must finish unchanged.

Bar: FP64 populations within 1e-12 relative of the FP64 oracle on every node
of every level, probes within 1e-13 absolute."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import Oracle  # noqa: E402
from paper_2004_14887_amd import workloads as W  # noqa: E402

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")

ERR_NEWTON, ERR_UNSTABLE = -4, -5


def gpu_run(wl, steps, precision="fp64", fields=None, **kw):
    from paper_2004_14887_amd.sim import Simulation

    print(f"[gpu] {wl.name} {precision} steps={steps} coupling={wl.coupling} eq={wl.eq_order}", flush=True)
    sim = Simulation(wl, precision, probe_capacity=max(1, steps), **kw)
    if fields is None:
        sim.init_from_workload()
    else:
        for l, (rho, u) in enumerate(fields):
            sim.init(l, torch.from_numpy(rho), torch.from_numpy(u))
    sim.step(steps)
    return sim


def oracle_run(wl, steps):
    o = Oracle(wl.lattice, wl.n0, wl.boxes, wl.tau0, wl.coupling, wl.eq_order, wl.probes, max(1, steps))
    for l in range(wl.n_levels):
        rho, u = W.initial_fields(wl, l)
        o.init(l, rho, u)
    o.run(steps)
    return o


def max_rel(g, r):
    m = ~np.isnan(r)
    assert np.array_equal(m, ~np.isnan(g)), "hole pattern differs"
    return float(np.max(np.abs(g[m] - r[m]) / np.abs(r[m])))


def assert_parity(sim, o, wl, tol=1e-12, probe_tol=1e-13):
    worst = 0.0
    for l in range(wl.n_levels):
        e = max_rel(sim.populations(l).cpu().numpy(), o.f(l))
        print(f"  level {l}: max rel err {e:.3e}", flush=True)
        worst = max(worst, e)
    assert worst <= tol
    if wl.probes:
        pg, po = sim.probes().cpu().numpy(), o.probes()
        assert pg.shape == po.shape
        assert np.abs(pg - po).max() <= probe_tol
    return worst


def offcentre_3level(coupling=2, steps=30):
    """72 x 56 periodic level 0; a level-1 box [9, 40) x [14, 27) (31 x 13
    parent cells, off centre); inside it an off-centre level-2 box
    [7, 30) x [4, 21) of level-1 cells.  A pulse, two vortices and a mean
    flow cross the interfaces; probes on every level, on box faces and
    corners."""
    vort = [dict(xc=20.3, yc=20.6, eps=0.04, Rc=4.0), dict(xc=40.7, yc=16.2, eps=-0.03, Rc=3.0)]
    probes = [(9, 14), (40, 27), (24, 20), (12, 16), (13, 23), (60, 40), (30, 14), (9, 20)]
    return W.Workload(name="offcentre_3level", lattice="D2Q9", n0=(72, 56),
                      boxes=[((9, 14), (40, 27)), ((7, 4), (30, 21))], tau0=0.56, steps=steps, coupling=coupling,
                      probes=probes, background=(0.04, -0.015, 0.0), vortices=vort,
                      pulses=[dict(c=(25.0, 19.5, 0.0), A=1e-3, Rc=2.5)])


@requires_gpu
@pytest.mark.parametrize("coupling", [1, 2])
def test_offcentre_unequal_boxes_three_levels_fp64(coupling):
    wl = offcentre_3level(coupling)
    sim = gpu_run(wl, wl.steps)
    sim.check()
    assert_parity(sim, oracle_run(wl, wl.steps), wl)


@requires_gpu
def test_3d_unequal_extents_xface_probes_fp64():
    """D3Q19 on a 28 x 24 x 20 periodic level 0 with a box of 15 x 9 x 10
    parent cells: every side and every extent differs.  Probes sit on both
    x faces of the box (nodes kept in the face-contiguous buffers), on a y
    face, on a z edge, inside and outside."""
    probes = [(5, 10, 9), (20, 8, 7), (12, 6, 9), (5, 6, 4), (12, 10, 9), (25, 2, 17), (20, 15, 14)]
    wl = W.Workload(name="box_3d_unequal", lattice="D3Q19", n0=(28, 24, 20), boxes=[((5, 6, 4), (20, 15, 14))],
                    tau0=0.54, steps=12, probes=probes, background=(0.03, 0.012, -0.02),
                    pulses=[dict(c=(11.3, 10.2, 8.7), A=1e-3, Rc=2.0)],
                    rings=[dict(c=(14.0, 11.0, 9.0), axis=(0.3, 0.8, 0.52), R=3.0, core=0.8, peak=0.02)])
    sim = gpu_run(wl, wl.steps)
    sim.check()
    assert_parity(sim, oracle_run(wl, wl.steps), wl)


@requires_gpu
def test_dc1_three_levels_2d_fp64():
    wl = W.pulse_vortices_3level(seed=2, n0=128, steps=40, coupling=1)
    sim = gpu_run(wl, wl.steps)
    sim.check()
    assert_parity(sim, oracle_run(wl, wl.steps), wl)


@requires_gpu
def test_dc1_three_levels_3d_fp64():
    wl = W.Workload("ring3_3lvl_dc1", "D3Q19", (32, 32, 32), [((8, 8, 8), (24, 24, 24)), ((8, 8, 8), (24, 24, 24))],
                    0.52, 6, coupling=1, pulses=[dict(c=(15.5, 16.0, 16.5), A=1e-3, Rc=3.0)],
                    background=(0.03, -0.02, 0.01), probes=[(16, 16, 16), (4, 4, 4), (8, 12, 16)])
    sim = gpu_run(wl, wl.steps)
    sim.check()
    assert_parity(sim, oracle_run(wl, wl.steps), wl)


@requires_gpu
@pytest.mark.parametrize("coupling", [1, 2])
def test_d2q9_third_order_equilibrium_fp64(coupling):
    """D2Q9 with the H3 terms of the equilibrium (the xxy and xyy terms),
    two levels, vortices crossing both faces with a Mach-0.1 mean flow."""
    wl = W.vortex_2level(seed=1, n0=64, steps=60, coupling=coupling)
    wl.eq_order = 3
    sim = gpu_run(wl, wl.steps)
    sim.check()
    assert_parity(sim, oracle_run(wl, wl.steps), wl)


@requires_gpu
def test_d2q9_third_order_equilibrium_fp32_probe_error():
    """The same in FP32 (the generic equilibrium path of the shifted form):
    probe error against the FP64 oracle within 1e-4 of the signal peak."""
    wl = W.vortex_2level(seed=1, n0=64, steps=60)
    wl.eq_order = 3
    wl.pulses = [dict(c=(32.0, 32.0, 0.0), A=1e-3, Rc=3.0)]
    g = gpu_run(wl, wl.steps, "fp32").probes().cpu().numpy()
    r = oracle_run(wl, wl.steps).probes()
    e = float(np.abs(g - r).max() / np.abs(r).max())
    print(f"  eq3 fp32 probe error {e:.3e}", flush=True)
    assert e <= 1e-4


def _fields_with(wl, level, node, value):
    out = [W.initial_fields(wl, l) for l in range(wl.n_levels)]
    out[level][0][node] = value
    return out


@requires_gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_non_finite_density_latches_unstable_single_level(precision, bad):
    """One periodic level (no interface, so no Newton): a non-finite density
    at one node must surface as DCLBM_ERR_UNSTABLE from dclbm_check."""
    from paper_2004_14887_amd._lib import DclbmError

    wl = W.Workload(name="single_nan", lattice="D2Q9", n0=(70, 53), boxes=[], tau0=0.6, steps=3,
                    background=(0.02, 0.0, 0.0))
    sim = gpu_run(wl, wl.steps, precision, fields=_fields_with(wl, 0, 70 * 20 + 33, bad))
    with pytest.raises(DclbmError) as ei:
        sim.check()
    assert ei.value.status == ERR_UNSTABLE


@requires_gpu
@pytest.mark.parametrize("lattice,precision", [("D2Q9", "fp64"), ("D2Q9", "fp16"), ("D3Q19", "fp32"),
                                               ("D3Q19", "fp16")])
def test_non_finite_density_on_refined_mesh_is_unstable_not_newton(lattice, precision):
    """A NaN inside the refined level reaches the interface: the cause is
    reported as an instability (not as a Newton failure)."""
    from paper_2004_14887_amd._lib import DclbmError

    if lattice == "D2Q9":
        wl = W.vortex_2level(seed=1, n0=64, steps=4)
    else:
        wl = W.pulse_ring_3d(seed=3, n0=32, steps=4)
    d = wl.dims(1)
    node = (d[2] // 2 * d[1] + 2) * d[0] + d[0] // 2   # two nodes inside the box edge
    sim = gpu_run(wl, wl.steps, precision, fields=_fields_with(wl, 1, node, float("nan")))
    with pytest.raises(DclbmError) as ei:
        sim.check()
    assert ei.value.status == ERR_UNSTABLE


@requires_gpu
def test_stable_runs_do_not_latch():
    for prec in ("fp64", "fp32", "fp16"):
        wl = W.pulse_vortices_3level(seed=2, n0=64, steps=20)
        gpu_run(wl, wl.steps, prec).check()


@requires_gpu
def test_serving_failed_requests_leave_others_unchanged():
    """In one mix: a 1-level request whose initial field holds a NaN (fails
    with DCLBM_ERR_UNSTABLE), a 2-level request whose Newton is allowed one
    iteration at an unreachable tolerance (fails with DCLBM_ERR_NEWTON), and
    healthy requests.  The failures are reported, and every healthy request's
    probe series equals, bit for bit, the same request served alone."""
    from paper_2004_14887_amd.server import Server, request_fields

    reqs, _ = W.serving_requests(seed=4, n=10, min_side=64, max_side=160, min_steps=10, max_steps=40)
    one_level = next(k for k, r in enumerate(reqs) if r.n_levels == 1)
    two_level = next(k for k, r in enumerate(reqs) if r.n_levels >= 2)
    fields = [request_fields(r) for r in reqs]
    bad_fields = [(rho.copy(), u.copy()) for rho, u in fields[one_level]]
    bad_fields[0][0][bad_fields[0][0].size // 3] = float("nan")

    def server(slots):
        return Server(1 << 30, precision="fp32", max_levels=3, max_slots=slots, steps_per_tick=2, max_probes=8,
                      max_probe_steps=2000, max_level_nodes=400 * 400)

    print(f"[gpu] serving failure isolation: nan in request {one_level}, newton failure in {two_level}", flush=True)
    srv = server(6)
    ids = []
    for k, r in enumerate(reqs):
        if k == one_level:
            ids.append(srv.submit(r, fields=bad_fields))
        elif k == two_level:
            ids.append(srv.submit(r, fields=fields[k], newton_max_iter=1, newton_tol=1e-300))
        else:
            ids.append(srv.submit(r, fields=fields[k]))
    srv.drain()
    assert srv.poll(ids[one_level]) == "failed"
    assert srv.info(ids[one_level])["status"] == ERR_UNSTABLE
    assert srv.poll(ids[two_level]) == "failed"
    assert srv.info(ids[two_level])["status"] == ERR_NEWTON
    mix = {k: srv.result(ids[k])[0] for k in range(len(reqs)) if k not in (one_level, two_level)}
    srv.close()
    for k, got in mix.items():
        one = server(1)
        rid = one.submit(reqs[k], fields=fields[k])
        one.drain()
        assert one.poll(rid) == "done"
        alone = one.result(rid)[0]
        one.close()
        assert np.array_equal(got, alone), f"request {k} changed by the failing neighbours"
