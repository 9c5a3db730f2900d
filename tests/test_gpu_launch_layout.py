"""Launch layouts of a 3-D FP16 level substep (run with -m gpu).

A refined level's substep runs either as one launch, its interface segments
interleaved over the front of the grid, or as two kernels side by side (the
bulk alone, and the probe, capture and segment workgroups on a second
stream); dclbm_set_split picks one.  The layouts must give the same
populations and probe series bit for bit, through graph replays and eager
launches alike, and switching layout in the middle of a run must rebuild the
cached graphs.  The default choice follows the weight of the bulk against
the segments, so on the small meshes of the other tests it is the single
launch; this test is what runs the split layout against it.
"""
import copy

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2004_14887_amd import workloads as W  # noqa: E402

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


def meshes():
    a = W.pulse_ring_3d(seed=3, n0=48, steps=8)
    b = W.pulse_ring_3d(seed=3, n0=64, steps=8)
    b.boxes = [((16, 16, 16), (48, 48, 48)), ((20, 20, 20), (44, 44, 44))]
    c = copy.deepcopy(b)
    c.n0 = (96, 48, 40)
    c.boxes = [((10, 12, 9), (74, 30, 27))]
    c.probes = [(10, 20, 18), (74, 13, 10), (40, 20, 20), (5, 5, 5)]
    return {"ring_48_2level": a, "ring_64_3level": b, "offcentre_96x48x40": c}


def run(wl, plan, timing=False):
    from paper_2004_14887_amd.sim import Simulation
    sim = Simulation(wl, "fp16", probe_capacity=wl.steps)
    sim.init_from_workload()
    sim.set_timing(timing)
    for mode, n in plan:
        sim.set_split(mode)
        sim.step(n)
    sim.check()
    out = [torch.nan_to_num(sim.populations(l), nan=-7.0).cpu() for l in range(wl.n_levels)], sim.probes().cpu()
    sim.close()
    return out


def same(a, b, what):
    pa, sa = a
    pb, sb = b
    assert torch.equal(sa, sb), f"{what}: probe series differ"
    for l, (x, y) in enumerate(zip(pa, pb)):
        assert torch.equal(x, y), f"{what}: level {l} differs"


@requires_gpu
@pytest.mark.parametrize("name", list(meshes()))
def test_split_and_single_launch_agree_bitwise(name):
    wl = meshes()[name]
    print(f"[gpu] launch layouts {name}", flush=True)
    ref = run(wl, [(0, 8)])
    same(ref, run(wl, [(1, 8)]), "split, graphs")
    same(ref, run(wl, [(1, 3), (0, 3), (-1, 2)]), "switched mid-run")
    same(ref, run(wl, [(1, 8)], timing=True), "split, eager")
    same(ref, run(wl, [(0, 8)], timing=True), "single launch, eager")


@requires_gpu
def test_split_mode_is_validated():
    from paper_2004_14887_amd._lib import DclbmError
    from paper_2004_14887_amd.sim import Simulation
    wl = W.pulse_ring_3d(seed=3, n0=48, steps=2)
    sim = Simulation(wl, "fp16", probe_capacity=2)
    for bad in (-2, 2):
        with pytest.raises(DclbmError):
            sim.set_split(bad)
    sim.close()
