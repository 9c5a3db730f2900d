"""Checkpoint and resume through the C ABI (run with -m gpu).

Stepping on from a restored checkpoint gives the same populations, probe
series and running probe sums, bit for bit, as stepping on from the state that was saved.
This holds when the checkpoint goes back into the simulation that wrote it,
and when it goes into a fresh simulation of the same configuration.  It is
checked for every storage form, in 2-D and 3-D, and for a checkpoint taken
during the first coarse step's special time interpolation as well as after
the steps have moved to graph replays.  Checkpoints of another
configuration, truncated buffers and blobs that are not checkpoints are
rejected.
"""
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2004_14887_amd import workloads as W  # noqa: E402

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")

CASES = [
    ("vortices_3level_128", "fp64"),
    ("vortices_3level_128", "fp32"),
    ("vortices_3level_128", "fp16"),
    ("ring_3d_48", "fp32"),
    ("ring_3d_48", "fp16"),
]


def workload(name, steps):
    if name == "vortices_3level_128":
        return W.pulse_vortices_3level(seed=2, n0=128, steps=steps)
    return W.pulse_ring_3d(seed=3, n0=48, steps=steps)


def state(sim):
    pops = [sim.populations(l).cpu() for l in range(sim.wl.n_levels)]
    sums, n = sim.probe_sums()
    return pops, sim.probes().cpu(), sums.cpu(), n


def same(a, b):
    pa, sa, ua, na = a
    pb, sb, ub, nb = b
    assert sa.shape == sb.shape and torch.equal(sa, sb), "probe series differ"
    assert na == nb and torch.equal(torch.nan_to_num(ua, nan=-7.0), torch.nan_to_num(ub, nan=-7.0)), \
        "probe sums differ"
    for l, (x, y) in enumerate(zip(pa, pb)):
        assert torch.equal(torch.nan_to_num(x, nan=-7.0), torch.nan_to_num(y, nan=-7.0)), f"level {l} differs"


@requires_gpu
@pytest.mark.parametrize("name,precision", CASES)
@pytest.mark.parametrize("at", [1, 4])
def test_resume_is_bitwise(name, precision, at):
    from paper_2004_14887_amd.sim import Simulation
    more = 5
    wl = workload(name, at + more)
    print(f"[gpu] checkpoint {name} {precision} at step {at}", flush=True)
    a = Simulation(wl, precision, probe_capacity=at + more)
    a.init_from_workload()
    a.set_probe_window(at - 1, at + more - 1)   # spans the checkpoint
    a.step(at)
    blob = a.save()
    assert blob.numel() == a.checkpoint_bytes()
    a.step(more)
    a.check()
    ref = state(a)
    assert ref[1].shape[0] == at + more and ref[3] == more
    # into a fresh simulation of the same configuration
    b = Simulation(wl, precision, probe_capacity=at + more)
    b.load(blob)
    b.step(more)
    b.check()
    same(ref, state(b))
    b.close()
    # back into the one that wrote it, from a host copy
    a.load(blob.cpu())
    a.step(more)
    a.check()
    same(ref, state(a))
    a.close()


@requires_gpu
def test_load_rejects_what_is_not_its_checkpoint():
    from paper_2004_14887_amd._lib import DclbmError
    from paper_2004_14887_amd.sim import Simulation
    wl = workload("vortices_3level_128", 4)
    a = Simulation(wl, "fp32", probe_capacity=4)
    a.init_from_workload()
    a.step(2)
    blob = a.save()
    for other in (Simulation(wl, "fp32", probe_capacity=5), Simulation(wl, "fp16", probe_capacity=4)):
        with pytest.raises(DclbmError) as ei:
            other.load(blob)
        assert ei.value.status == -1 and "another configuration" in str(ei.value)
        other.close()
    with pytest.raises(DclbmError):
        a.load(blob[: blob.numel() - 256].clone())
    with pytest.raises(DclbmError) as ei:
        a.load(torch.zeros(blob.numel(), dtype=torch.uint8, device=blob.device))
    assert "not a checkpoint" in str(ei.value)
    import ctypes as C
    small = torch.empty(blob.numel(), dtype=torch.uint8, device=blob.device)
    ptr = small.data_ptr()
    assert ptr % 256 == 0
    assert a.lib.dclbm_save(a.h, C.c_void_p(ptr), blob.numel() - 1) == -1
    # the rejected loads changed nothing: the state still steps like the saved one
    a.step(2)
    b = Simulation(wl, "fp32", probe_capacity=4)
    b.load(blob)
    b.step(2)
    same(state(a), state(b))
    a.close()
    b.close()
