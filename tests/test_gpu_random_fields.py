"""Every node of every level against the FP64 oracle, from random initial
fields (run with -m gpu).

The density and velocity of every node are drawn independently (seeded), so
the populations a node pulls come from unrelated neighbours: a node that a
launch skips, updates twice or pulls from the wrong place differs from the
oracle by about the field amplitude (1e-2 in f), while the storage rounding of
the reduced forms stays orders of magnitude below it.  The meshes are ragged
(rows that end mid-block, tile counts per XCD that are odd, so the two-tile
bulk workgroups of 2-D FP16 meet a missing second tile), refined (holes,
interface tiles on every face, x-face buffers in 3-D) and run several coarse
steps under DC2.

Bars (|f_gpu - f_oracle| over all nodes and directions): FP64 1e-12
relative; FP32 1e-7 absolute; FP16 storage 2e-4 absolute.  Measured: about
1.5e-15, 1e-8 and 2.2e-5; a misplaced node gives about 1e-2."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import Oracle  # noqa: E402
from paper_2004_14887_amd import workloads as W  # noqa: E402

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


def ragged_2d_3level():
    """130 x 24 periodic level 0 (3 bulk tiles per XCD row slot); a level-1
    box [8, 70) x [6, 18) (125 x 25 nodes); inside it a level-2 box
    [20, 100) x [4, 20) of level-1 cells (161 x 33 nodes)."""
    return W.Workload(name="ragged_2d_3level", lattice="D2Q9", n0=(130, 24),
                      boxes=[((8, 6), (70, 18)), ((20, 4), (100, 20))], tau0=0.58, steps=3)


def ragged_3d_2level():
    """72 x 40 x 36 periodic level 0; an off-centre level-1 box
    [10, 43) x [8, 30) x [8, 26) (67 x 45 x 37 nodes)."""
    return W.Workload(name="ragged_3d_2level", lattice="D3Q19", n0=(72, 40, 36),
                      boxes=[((10, 8, 8), (43, 30, 26))], tau0=0.56, steps=3)


def random_fields(wl, seed):
    """Per level: density 1 +- 1e-2 and velocity components +- 5e-2, drawn
    independently at every node (hole values are never read)."""
    rng = np.random.default_rng(seed)
    out = []
    for l in range(wl.n_levels):
        n = int(np.prod(wl.dims(l)))
        rho = 1.0 + 1e-2 * (2.0 * rng.random(n) - 1.0)
        u = 5e-2 * (2.0 * rng.random((wl.D, n)) - 1.0)
        out.append((rho, u))
    return out


def run_both(wl, precision, fields, steps):
    from paper_2004_14887_amd.sim import Simulation

    print(f"[gpu] {wl.name} {precision} random fields, {steps} steps", flush=True)
    sim = Simulation(wl, precision, probe_capacity=max(1, steps))
    for l, (rho, u) in enumerate(fields):
        sim.init(l, torch.from_numpy(rho), torch.from_numpy(u))
    sim.step(steps)
    sim.check()
    o = Oracle(wl.lattice, wl.n0, wl.boxes, wl.tau0, wl.coupling, wl.eq_order, [], 1)
    for l, (rho, u) in enumerate(fields):
        o.init(l, rho, u)
    o.run(steps)
    return sim, o


@requires_gpu
@pytest.mark.parametrize("mesh", [ragged_2d_3level, ragged_3d_2level])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-7), ("fp16", 2e-4)])
def test_random_fields_every_node(mesh, precision, tol):
    wl = mesh()
    fields = random_fields(wl, seed=11)
    sim, o = run_both(wl, precision, fields, wl.steps)
    worst = 0.0
    for l in range(wl.n_levels):
        g = sim.populations(l).cpu().numpy()
        r = o.f(l)
        m = ~np.isnan(r)
        assert np.array_equal(m, ~np.isnan(g)), f"level {l}: hole pattern differs"
        d = np.abs(g[m] - r[m])
        e = float(d.max() / np.abs(r[m]).max()) if precision == "fp64" else float(d.max())
        print(f"  level {l}: {'max rel' if precision == 'fp64' else 'max abs'} err {e:.3e}", flush=True)
        worst = max(worst, e)
    assert worst <= tol
