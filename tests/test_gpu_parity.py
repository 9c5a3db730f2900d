"""GPU parity: the HIP library against the FP64 oracle, element by element,
on the same seeded inputs (needs an MI355X; run with -m gpu).

Bar: FP64 populations within 1e-12 relative of the oracle after the stated
number of coarse steps, every level, every direction; holes NaN on both
sides.  FP32 / FP16-storage forms: probe pressure error against the FP64
oracle within 1e-4 / 1e-3 of the probe signal's peak (max norm).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import Oracle  # noqa: E402
from paper_2004_14887_amd import workloads as W  # noqa: E402

CS2 = 1.0 / 3.0


def _gpu_ok():
    return torch.cuda.is_available()


requires_gpu = pytest.mark.skipif(not _gpu_ok(), reason="no GPU")


def gpu_run(wl, steps, precision="fp64", **kw):
    from paper_2004_14887_amd.sim import Simulation

    print(f"[gpu] {wl.name} {precision} steps={steps} coupling={wl.coupling} eq={wl.eq_order}", flush=True)
    sim = Simulation(wl, precision, probe_capacity=max(1, steps), **kw)
    sim.init_from_workload()
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


def assert_population_parity(sim, o, wl, tol=1e-12):
    worst = 0.0
    for l in range(wl.n_levels):
        e = max_rel(sim.populations(l).cpu().numpy(), o.f(l))
        print(f"  level {l}: max rel err {e:.3e}", flush=True)
        worst = max(worst, e)
    assert worst <= tol
    return worst


@requires_gpu
@pytest.mark.parametrize("coupling", [1, 2])
def test_vortex_2level_200_steps_fp64(coupling):
    """128^2 periodic, centred 64^2-cell patch refined x2, two vortices crossing
    both faces, tau 0.55, 200 coarse steps: populations within 1e-12."""
    wl = W.vortex_2level(seed=1, n0=128, steps=200, coupling=coupling)
    sim = gpu_run(wl, wl.steps)
    sim.check()
    o = oracle_run(wl, wl.steps)
    assert_population_parity(sim, o, wl)
    # probes and the shared macroscopic state at co-located nodes
    pg, po = sim.probes().cpu().numpy(), o.probes()
    assert pg.shape == po.shape == (200, 16)
    assert np.abs(pg - po).max() <= 1e-13
    Xg, Xo = sim.shared(1).cpu().numpy(), o.X(1)
    assert max_rel(Xg[:1], Xo[:1]) <= 1e-12
    m = ~np.isnan(Xo[1])
    assert np.abs(Xg[1:3][:, m] - Xo[1:3][:, m]).max() <= 1e-13


@requires_gpu
def test_pulse_vortices_3level_fp64_parity():
    """3 levels (reduced 128^2 replica of the 2048^2 nesting), 40 coarse steps."""
    wl = W.pulse_vortices_3level(seed=2, n0=128, steps=40)
    sim = gpu_run(wl, wl.steps)
    sim.check()
    o = oracle_run(wl, wl.steps)
    assert_population_parity(sim, o, wl)
    assert np.abs(sim.probes().cpu().numpy() - o.probes()).max() <= 1e-13


@requires_gpu
@pytest.mark.parametrize("coupling,eq_order", [(2, 2), (1, 2), (2, 3)])
def test_pulse_ring_3d_fp64_parity(coupling, eq_order):
    """D3Q19, 2 levels (32^3 replica of the 256^3 nesting), faces, edges and
    corners of the refined box, 12 coarse steps."""
    wl = W.pulse_ring_3d(seed=3, n0=32, steps=12, coupling=coupling)
    wl.eq_order = eq_order
    sim = gpu_run(wl, wl.steps)
    sim.check()
    o = oracle_run(wl, wl.steps)
    assert_population_parity(sim, o, wl)


@requires_gpu
def test_3d_three_levels_fp64_parity():
    wl = W.Workload("ring3_3lvl", "D3Q19", (32, 32, 32), [((8, 8, 8), (24, 24, 24)), ((8, 8, 8), (24, 24, 24))],
                    0.52, 6, pulses=[dict(c=(15.5, 16.0, 16.5), A=1e-3, Rc=3.0)],
                    background=(0.03, -0.02, 0.01), probes=[(16, 16, 16), (4, 4, 4)])
    sim = gpu_run(wl, wl.steps)
    o = oracle_run(wl, wl.steps)
    assert_population_parity(sim, o, wl)


@requires_gpu
def test_balance_matches_oracle():
    wl = W.vortex_2level(seed=4, n0=64, steps=10)
    sim = gpu_run(wl, wl.steps)
    o = oracle_run(wl, wl.steps)
    bg, bo = np.array(sim.balance()), o.balance()
    assert abs(bg[0] - bo[0]) <= 1e-12 * abs(bo[0])
    assert np.abs(bg[1:] - bo[1:]).max() <= 1e-12 * abs(bo[0])


@requires_gpu
def test_graph_replay_equals_eager_and_is_deterministic():
    wl = W.pulse_vortices_3level(seed=5, n0=64, steps=9)
    a = gpu_run(wl, wl.steps)
    b = gpu_run(wl, wl.steps)
    from paper_2004_14887_amd.sim import Simulation

    e = Simulation(wl, "fp64", probe_capacity=wl.steps)
    e.set_timing(True)          # eager launches, no graph
    e.init_from_workload()
    e.step(wl.steps)
    for l in range(wl.n_levels):
        fa, fb, fe = a.populations(l), b.populations(l), e.populations(l)
        assert torch.equal(torch.nan_to_num(fa, 7.0), torch.nan_to_num(fb, 7.0))
        assert torch.equal(torch.nan_to_num(fa, 7.0), torch.nan_to_num(fe, 7.0))


@requires_gpu
def test_newton_failure_is_latched():
    from paper_2004_14887_amd._lib import DclbmError

    wl = W.vortex_2level(seed=1, n0=64, steps=2)
    sim = gpu_run(wl, 1, newton_max_iter=1, newton_tol=1e-300)
    with pytest.raises(DclbmError) as ei:
        sim.check()
    assert ei.value.status == -4


@requires_gpu
def test_uniform_flow_stays_uniform_all_precisions():
    """A uniform flow stays uniform on a 3-level mesh in every form.  With the
    storage reference at the flow itself (the default, u_ref = background)
    the reduced forms carry exact zeros; with u_ref = 0 they carry the flow's
    deviation from rest and keep it to their storage precision."""
    u0 = (0.05, -0.03)
    for prec, u_ref, tol in (("fp64", None, 1e-15), ("fp32", None, 1e-15), ("fp16", None, 1e-15),
                             ("fp32", (0.0, 0.0), 1e-7), ("fp16", (0.0, 0.0), 2e-4)):
        wl = W.uniform_state("D2Q9", (64, 64), [((16, 16), (48, 48)), ((16, 16), (48, 48))], u0=u0)
        sim = gpu_run(wl, 4, prec, u_ref=u_ref)
        for l in range(3):
            rho, u = sim.macros(l)
            m = ~torch.isnan(rho)
            assert (rho[m] - 1).abs().max().item() <= tol, (prec, u_ref)
            assert (u[0][m] - u0[0]).abs().max().item() <= tol * 4, (prec, u_ref)
            assert (u[1][m] - u0[1]).abs().max().item() <= tol * 4, (prec, u_ref)


def _probe_error(wl, steps, precision):
    g = gpu_run(wl, steps, precision).probes().cpu().numpy()
    r = oracle_run(wl, steps).probes()
    return float(np.abs(g - r).max() / np.abs(r).max())


def _three_level_replica(steps):
    # 128^2 replica of the 2048^2 three-level nesting: pulse + 16 vortices, no background flow
    return W.pulse_vortices_3level(seed=2, n0=128, steps=steps)


@requires_gpu
def test_fp32_probe_error_within_1e_4():
    """FP32 arithmetic with FP32 storage of f - w against the FP64 oracle:
    max-norm probe pressure error relative to the signal peak <= 1e-4."""
    wl = _three_level_replica(400)
    e = _probe_error(wl, wl.steps, "fp32")
    print(f"fp32 probe error {e:.3e}")
    assert e <= 1e-4


FP16_FLOOR = ("binary16 storage of 256 (f - E) misses the 1e-3 target where a probe sits near a Mach-0.05-0.2 "
              "vortex: the probe density sums nine stored values whose rounding step is 2^-11 of |f - E| ~ 0.02; "
              "about 14 mantissa bits would be needed")


@requires_gpu
@pytest.mark.xfail(strict=True, reason="measured about 3e-3 on this replica; " + FP16_FLOOR)
def test_fp16_storage_probe_error_within_1e_3():
    """FP16 storage of 256 (f - w) against the FP64 oracle on the three-level
    replica: probe error within 1e-3 of the signal peak (not met)."""
    wl = _three_level_replica(400)
    e = _probe_error(wl, wl.steps, "fp16")
    print(f"fp16 probe error {e:.3e}")
    assert e <= 1e-3


@requires_gpu
def test_reduced_precision_with_background_flow():
    """Mach-0.1 background flow (vortices crossing both faces of a 2-level
    mesh, plus a pulse).  Storing deviations from the background equilibrium
    (u_ref = background, the default) keeps FP32 within 1e-4 of the FP64
    oracle; deviations from the rest state (u_ref = 0) are O(0.17 w) and
    their rounding floor is far higher (measured, bounded)."""
    wl = W.vortex_2level(seed=1, n0=128, steps=200)
    wl.pulses = [dict(c=(64.0, 64.0, 0.0), A=1e-3, Rc=6.0)]
    r = oracle_run(wl, wl.steps).probes()

    def err(prec, u_ref):
        g = gpu_run(wl, wl.steps, prec, u_ref=u_ref).probes().cpu().numpy()
        return float(np.abs(g - r).max() / np.abs(r).max())

    e32 = err("fp32", None)
    e32_rest = err("fp32", (0.0, 0.0))
    print(f"background flow: fp32 {e32:.3e} (rest reference {e32_rest:.3e})")
    assert e32 <= 1e-4
    assert e32 < e32_rest


@requires_gpu
@pytest.mark.xfail(strict=True, reason="measured about 1.25e-2 (small probe signal); " + FP16_FLOOR)
def test_fp16_with_background_flow_within_1e_3():
    """FP16 storage on the vortex pair with a Mach-0.1 mean flow and a pulse,
    against the FP64 oracle: within 1e-3 (not met)."""
    wl = W.vortex_2level(seed=1, n0=128, steps=200)
    wl.pulses = [dict(c=(64.0, 64.0, 0.0), A=1e-3, Rc=6.0)]
    r = oracle_run(wl, wl.steps).probes()
    g = gpu_run(wl, wl.steps, "fp16").probes().cpu().numpy()
    e16 = float(np.abs(g - r).max() / np.abs(r).max())
    print(f"background flow: fp16 {e16:.3e}")
    assert e16 <= 1e-3


@requires_gpu
def test_fp32_3d_ring_with_background_flow_within_1e_4():
    """D3Q19 two-level replica of the ring workload (Mach-0.1 flow along a
    seeded axis, pulse, vortex ring): FP32 probe error against the oracle."""
    wl = W.pulse_ring_3d(seed=3, n0=64, steps=60)
    e = _probe_error(wl, wl.steps, "fp32")
    print(f"3-D ring fp32 probe error {e:.3e}")
    assert e <= 1e-4


@requires_gpu
@pytest.mark.parametrize("lattice,n0", [("D2Q9", (70, 53)), ("D3Q19", (20, 17, 13))])
def test_single_level_periodic_fp64_parity(lattice, n0):
    """One periodic level (the plain scheme the refined step reduces to), on
    ragged sizes that leave partial 64 x 4 tiles: every population against
    the oracle after 10 steps."""
    wl = W.Workload(name=f"single_{lattice}", lattice=lattice, n0=n0, boxes=[], tau0=0.6, steps=10,
                    pulses=[dict(c=tuple(v / 2.0 for v in n0) + (0.0,) * (3 - len(n0)), A=1e-3, Rc=3.0)],
                    background=(0.02, -0.01, 0.005)[:len(n0)] + (0.0,) * (3 - len(n0)))
    sim = gpu_run(wl, wl.steps)
    sim.check()
    assert_population_parity(sim, oracle_run(wl, wl.steps), wl)


@requires_gpu
@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
def test_smallest_legal_box_fp64_parity(lattice):
    """The smallest legal refinement: an 8-node periodic level 0 and a box of
    3 parent cells at the minimum margin of 2 (7 fine nodes per axis, so every
    hanging node uses the one-sided line-end stencil)."""
    D = 2 if lattice == "D2Q9" else 3
    wl = W.Workload(name=f"smallest_{lattice}", lattice=lattice, n0=(8,) * D,
                    boxes=[((2,) * D, (5,) * D)], tau0=0.58, steps=20,
                    pulses=[dict(c=(3.5, 3.5, 3.5 if D == 3 else 0.0), A=1e-3, Rc=1.5)],
                    background=(0.03, 0.01, -0.02)[:D] + (0.0,) * (3 - D), probes=[(3,) * D, (6,) * D])
    sim = gpu_run(wl, wl.steps)
    sim.check()
    o = oracle_run(wl, wl.steps)
    assert_population_parity(sim, o, wl)
    assert np.abs(sim.probes().cpu().numpy() - o.probes()).max() <= 1e-15


@requires_gpu
def test_zero_steps_and_no_probes():
    """Degenerate calls: zero coarse steps leave the initial state, a
    configuration without probes steps and reports an empty series."""
    wl = W.vortex_2level(seed=1, n0=64, steps=4)
    wl.probes = []
    from paper_2004_14887_amd.sim import Simulation
    sim = Simulation(wl, "fp64", probe_capacity=1)
    sim.init_from_workload()
    f0 = sim.populations(1).cpu().numpy()
    sim.step(0)
    assert np.array_equal(sim.populations(1).cpu().numpy(), f0, equal_nan=True)
    sim.step(4)
    sim.check()
    assert sim.probes().shape[0] == 0 or sim.probes().numel() == 0
    assert_population_parity(sim, oracle_run(wl, 4), wl)


def _four_level_replica(steps, n0=32):
    # the 4-level 512^3 nesting at n0 = 32: centred boxes of 22, 30, 32 parent cells
    return W.rings_4level(seed=5, n0=n0, sides=(22, 30, 32), steps=steps, n_rings=4, n_pulses=2)


@requires_gpu
def test_four_levels_d3q19_fp64_parity():
    """Four nested levels (three interfaces, 15 level substeps per coarse
    step), D3Q19, vortex rings and pulses: every population of every level
    against the oracle."""
    wl = _four_level_replica(6)
    sim = gpu_run(wl, wl.steps)
    sim.check()
    assert_population_parity(sim, oracle_run(wl, wl.steps), wl)


@requires_gpu
@pytest.mark.xfail(strict=True, reason="measured about 1.3e-3; " + FP16_FLOOR)
def test_four_levels_fp16_storage_against_fp64():
    """FP16 storage on the 4-level replica, 60 coarse steps (480 finest
    substeps), probe error against the FP64 GPU path (which the previous test
    ties to the oracle): within 1e-3 (not met)."""
    wl = _four_level_replica(60)
    ref = gpu_run(wl, wl.steps, "fp64").probes().cpu().numpy()
    got = gpu_run(wl, wl.steps, "fp16").probes().cpu().numpy()
    e = float(np.abs(got - ref).max() / np.abs(ref).max())
    print(f"4-level fp16 probe error {e:.3e}")
    assert e <= 1e-3


@requires_gpu
@pytest.mark.slow
def test_four_levels_full_size_uniform_flow_is_exact():
    """The 4-level 512^3 D3Q19 mesh at full size in FP16 storage (about
    193 GB of workspace, 1041^3 finest nodes, 64-bit element offsets): a
    uniform flow with the storage reference at the flow is carried as exact
    zeros through 2 coarse steps (30 level substeps), so the FP64 balances
    equal the exact totals."""
    wl = W.rings_4level(seed=5, steps=2)
    wl.rings, wl.pulses = [], []
    u0 = (0.03, -0.02, 0.01)
    wl.background = u0
    from paper_2004_14887_amd.sim import Simulation
    torch.cuda.empty_cache()   # blocks cached by earlier tests
    print(f"[gpu] {wl.name} fp16 full size", flush=True)
    sim = Simulation(wl, "fp16", probe_capacity=4)
    for l in range(wl.n_levels):
        n = sim.n_dense(l)
        rho = torch.ones(n, dtype=torch.float64, device="cuda")
        u = torch.empty((3, n), dtype=torch.float64, device="cuda")
        for a in range(3):
            u[a].fill_(u0[a])
        sim.init(l, rho, u)
        del rho, u
    sim.step(wl.steps)
    sim.check()
    bal = sim.balance()
    # owned volume: each level's dense nodes minus the closed box of its
    # child (owned by the child), weighted 2^(-3 l)
    vol = 0.0
    for l in range(wl.n_levels):
        d = wl.dims(l)
        own = d[0] * d[1] * d[2]
        if l + 1 < wl.n_levels:
            lo, hi = wl.boxes[l]
            own -= (hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1)
        vol += own * 0.125 ** l
    print(f"  balances {bal}, owned volume {vol}", flush=True)
    assert abs(bal[0] - vol) <= 1e-12 * vol
    for a in range(3):
        assert abs(bal[1 + a] - u0[a] * vol) <= 1e-12 * vol
    sim.close()


@requires_gpu
@pytest.mark.slow
def test_full_size_2048_three_levels_sampled():
    """The 2048^2 three-level workload at full size, in the graph-replay launch
    configuration the benchmark times, against the oracle after 2 coarse
    steps: every node of every level compared."""
    wl = W.pulse_vortices_3level(seed=2, n0=2048, steps=2)
    sim = gpu_run(wl, wl.steps)
    sim.check()
    o = oracle_run(wl, wl.steps)
    assert_population_parity(sim, o, wl)


@requires_gpu
@pytest.mark.slow
def test_full_size_256_cubed_two_levels():
    """The 256^3 D3Q19 two-level workload at full size, 1 coarse step, every node."""
    wl = W.pulse_ring_3d(seed=3, n0=256, steps=1)
    sim = gpu_run(wl, wl.steps)
    sim.check()
    o = oracle_run(wl, wl.steps)
    assert_population_parity(sim, o, wl)
