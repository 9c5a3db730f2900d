"""GPU parity of refined regions of any shape made of level-0 cells
(Sec. 3.4 closing paragraph, App. B), run with -m gpu.

* A stair-stepped circle and an L-shaped region (a concave corner) under DC1
  and DC2: every node of both levels against the oracle after several coarse
  steps, from a pulse on a mean flow and from random fields (FP64 1e-12
  relative; FP32 1e-7 and FP16 2e-4 absolute, as for boxes); the NaN pattern
  (holes, and level-1 nodes outside the region) identical.
* A mask covering the whole box gives the box path's populations bit for bit.
* A uniform flow is kept exactly in every storage form.
* Probes inside the box but outside the region are read on level 0, as the
  oracle reads them.
* The pulse across the circular interface of Sec. 4.1.2 at the paper's
  resolution: the reflected field against oracle runs (1e-9 of the
  reference's peak), DC1 and DC2."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
from paper_2004_14887_amd import workloads as W  # noqa: E402

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")

N = 64
BOX = ((12, 12), (52, 52))


def circle():
    return W.circle_region(BOX, (31.0, 33.5), 16.5)


def l_shape():
    m = np.ones((40, 40), np.uint8)
    m[21:, 19:] = 0
    return m


def workload(region, coupling, steps=8, probes=()):
    wl = W.Workload("region", "D2Q9", (N, N), [BOX], 0.56, steps, coupling=coupling,
                    pulses=[dict(c=(29.0, 34.0, 0.0), A=1e-3, Rc=3.0)], background=(0.03, 0.01, 0.0),
                    probes=list(probes))
    wl.region = region
    return wl


def random_fields(wl, seed):
    rng = np.random.default_rng(seed)
    out = []
    for l in range(wl.n_levels):
        n = int(np.prod(wl.dims(l)))
        out.append((1.0 + 1e-2 * (2.0 * rng.random(n) - 1.0), 5e-2 * (2.0 * rng.random((2, n)) - 1.0)))
    return out


def both(wl, precision, fields=None):
    from paper_2004_14887_amd.sim import Simulation

    print(f"[gpu] region DC{wl.coupling} {precision} {'random' if fields else 'pulse'}, {wl.steps} steps", flush=True)
    sim = Simulation(wl, precision, probe_capacity=max(1, wl.steps))
    o = O.Oracle(wl.lattice, wl.n0, wl.boxes, wl.tau0, wl.coupling, wl.eq_order, wl.probes, max(1, wl.steps))
    if wl.region is not None:
        o.set_region(wl.region)
    for l in range(wl.n_levels):
        rho, u = fields[l] if fields else W.initial_fields(wl, l)
        sim.init(l, torch.from_numpy(rho), torch.from_numpy(u))
        o.init(l, rho, u)
    sim.step(wl.steps)
    sim.check()
    o.run(wl.steps)
    return sim, o


def errors(sim, o, wl, relative):
    worst = 0.0
    for l in range(wl.n_levels):
        g, r = sim.populations(l).cpu().numpy(), o.f(l)
        m = ~np.isnan(r)
        assert np.array_equal(m, ~np.isnan(g)), f"level {l}: NaN pattern differs"
        d = np.abs(g[m] - r[m])
        e = float(d.max() / np.abs(r[m]).max()) if relative else float(d.max())
        print(f"  level {l}: {'rel' if relative else 'abs'} err {e:.2e}", flush=True)
        worst = max(worst, e)
    return worst


@requires_gpu
@pytest.mark.parametrize("region", [circle, l_shape])
@pytest.mark.parametrize("coupling", [1, 2])
def test_region_fp64_every_node(region, coupling):
    wl = workload(region(), coupling)
    sim, o = both(wl, "fp64")
    assert errors(sim, o, wl, True) < 1e-12


@requires_gpu
@pytest.mark.parametrize("region", [circle, l_shape])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-7), ("fp16", 2e-4)])
def test_region_random_fields(region, precision, tol):
    wl = workload(region(), 2, steps=3)
    sim, o = both(wl, precision, random_fields(wl, 17))
    assert errors(sim, o, wl, precision == "fp64") < tol


@requires_gpu
def test_full_mask_is_the_box_path():
    from paper_2004_14887_amd.sim import Simulation

    out = []
    for region in (np.ones((40, 40), np.uint8), None):
        wl = workload(region, 2)
        sim = Simulation(wl, "fp32", probe_capacity=wl.steps)
        sim.init_from_workload()
        sim.step(wl.steps)
        out.append([sim.populations(l).cpu() for l in range(2)])
    for a, b in zip(*out):
        assert torch.equal(torch.nan_to_num(a, nan=-7.0), torch.nan_to_num(b, nan=-7.0))


@requires_gpu
def test_uniform_flow_kept_in_every_form():
    from paper_2004_14887_amd.sim import Simulation

    for prec in ("fp64", "fp32", "fp16"):
        wl = workload(circle(), 2, steps=5)
        wl.pulses = []
        sim = Simulation(wl, prec, probe_capacity=5)
        sim.init_from_workload()
        sim.step(5)
        for l in range(2):
            rho, u = sim.macros(l)
            m = ~torch.isnan(rho)
            assert (rho[m] - 1).abs().max().item() < 1e-14, prec
            assert (u[0][m] - 0.03).abs().max().item() < 1e-14 and (u[1][m] - 0.01).abs().max().item() < 1e-14


@requires_gpu
def test_probes_follow_the_region():
    # (20, 20) and (40, 40) lie in the box but outside the circle; (31, 33) inside
    wl = workload(circle(), 2, steps=6, probes=[(20, 20), (40, 40), (31, 33), (5, 60)])
    sim, o = both(wl, "fp64")
    g = sim.probes().cpu().numpy()
    assert np.abs(g - o.probes()).max() < 1e-15


@requires_gpu
@pytest.mark.parametrize("coupling", [1, 2])
def test_circular_interface_reflection_matches_oracle(coupling):
    from paper_2004_14887_amd import studies

    print(f"[gpu] circular interface reflection DC{coupling}", flush=True)
    res = studies.reflection(steps=90, coupling=coupling, shape="circle")
    wl = W.pulse_circle(coupling=coupling, steps=90)
    ref = W.uniform_fine_reference(wl)
    a = O.Oracle(wl.lattice, wl.n0, wl.boxes, wl.tau0, coupling, wl.eq_order, [], 1)
    a.set_region(wl.region)
    b = O.Oracle(ref.lattice, ref.n0, ref.boxes, ref.tau0, coupling, ref.eq_order, [], 1)
    for o, w in ((a, wl), (b, ref)):
        for l in range(w.n_levels):
            rho, u = W.initial_fields(w, l)
            o.init(l, rho, u)
        o.run(w.steps)
    d1 = O.velocity_divergence(wl.lattice, a.f(1), wl.dims(1), False).reshape(wl.dims(1)[1], wl.dims(1)[0])
    dr = O.velocity_divergence(ref.lattice, b.f(0), ref.dims(0), True).reshape(ref.dims(0)[1], ref.dims(0)[0])
    lo = wl.boxes[0][0]
    ny, nx = d1.shape
    r = (d1 - dr[2 * lo[1]:2 * lo[1] + ny, 2 * lo[0]:2 * lo[0] + nx]) / np.abs(dr).max()
    g = res["field"]
    assert np.array_equal(np.isnan(g), np.isnan(r))
    m = ~np.isnan(r)
    e = np.abs(g[m] - r[m]).max()
    print(f"  rate max {res['max']:.3e} l2 {res['l2']:.3e}; field error {e:.2e}", flush=True)
    assert e < 1e-9


@requires_gpu
@pytest.mark.parametrize("region", [circle, l_shape])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-7)])
def test_region_hrr_random_fields(region, precision, tol):
    """H-RR on a refined region (R32): every node against the oracle."""
    wl = workload(region(), 2, steps=3)
    wl.collision, wl.eq_order = "hrr", 3
    from paper_2004_14887_amd.sim import Simulation

    fields = random_fields(wl, 23)
    print(f"[gpu] region H-RR {precision}", flush=True)
    sim = Simulation(wl, precision, probe_capacity=3)
    o = O.Oracle(wl.lattice, wl.n0, wl.boxes, wl.tau0, wl.coupling, wl.eq_order, [], 1)
    o.set_region(wl.region)
    o.set_collision("hrr", wl.hrr_sigma, wl.hrr_psi)
    for l in range(2):
        rho, u = fields[l]
        sim.init(l, torch.from_numpy(rho), torch.from_numpy(u))
        o.init(l, rho, u)
    sim.step(3)
    sim.check()
    o.run(3)
    assert errors(sim, o, wl, precision == "fp64") < tol


@requires_gpu
@pytest.mark.parametrize("collision", ["bgk", "hrr"])
def test_region_checkpoint_resume_is_bitwise(collision):
    """A refined region with an absorbing layer, BGK or H-RR: stepping on from
    a checkpoint loaded into a fresh simulation gives the same populations,
    bit for bit, as stepping on from the state that was saved."""
    from paper_2004_14887_amd.sim import Simulation

    wl = workload(circle(), 2, steps=7)
    wl.collision, wl.eq_order = collision, 3
    wl.sponge_cells, wl.sponge_sigma = 8, 0.3
    print(f"[gpu] region checkpoint {collision}", flush=True)
    a = Simulation(wl, "fp32", probe_capacity=7)
    a.init_from_workload()
    a.step(3)
    blob = a.save()
    a.step(4)
    b = Simulation(wl, "fp32", probe_capacity=7)
    b.load(blob)
    b.step(4)
    for l in range(2):
        x, y = a.populations(l).cpu(), b.populations(l).cpu()
        assert torch.equal(torch.nan_to_num(x, nan=-7.0), torch.nan_to_num(y, nan=-7.0)), f"level {l} differs"
    assert torch.equal(a.probes().cpu(), b.probes().cpu())
