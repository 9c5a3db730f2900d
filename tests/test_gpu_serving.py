"""The serving runtime on the GPU (run with -m gpu): continuous batching of
many simulations through the C ABI.

* Each request's probe series is bit-identical alone and in a mix where
  requests arrive while others run, queue for slots and memory, and share
  every launch with whatever else is resident.
* A served request equals the same workload stepped alone through the
  single-simulation entry points (within the FP32 form's own error in 2-D,
  bit for bit in 3-D, where both kernels order Newton alike).
* FP64 serving matches the FP64 oracle.
* Admission never exceeds the arena: requests wait for memory and slots,
  and all complete.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2004_14887_amd import workloads as W  # noqa: E402

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")


def small_requests(n=12, seed=4, max_steps=60):
    reqs, _ = W.serving_requests(seed=seed, n=n, min_side=64, max_side=192, min_steps=10, max_steps=max_steps)
    return reqs


def make_server(precision="fp32", arena=1 << 30, **kw):
    from paper_2004_14887_amd.server import Server
    kw.setdefault("max_levels", 3)
    kw.setdefault("max_slots", 4)
    kw.setdefault("max_probes", 8)
    kw.setdefault("max_probe_steps", 2000)
    kw.setdefault("max_level_nodes", 400 * 400)
    return Server(arena, precision=precision, **kw)


def drain_all(srv, ids):
    srv.drain()
    out = {}
    for rid in ids:
        assert srv.poll(rid) == "done", (rid, srv.info(rid))
        out[rid] = srv.result(rid)
    return out


@requires_gpu
def test_serving_alone_equals_mix():
    from paper_2004_14887_amd.server import request_fields
    reqs = small_requests()
    fields = [request_fields(r) for r in reqs]
    print(f"[gpu] serving mix of {len(reqs)}: sides {[r.n0[0] for r in reqs]} levels {[r.n_levels for r in reqs]}",
          flush=True)
    # the mix: 4 slots, requests arrive in three waves while others run
    srv = make_server(max_slots=4, steps_per_tick=1)
    ids = []
    for k in range(5):
        ids.append(srv.submit(reqs[k], fields=fields[k]))
    for _ in range(7):
        srv.tick()
    for k in range(5, 9):
        ids.append(srv.submit(reqs[k], fields=fields[k]))
    for _ in range(3):
        srv.tick()
    for k in range(9, len(reqs)):
        ids.append(srv.submit(reqs[k], fields=fields[k]))
    mix = drain_all(srv, ids)
    srv.close()
    # alone: one slot, one request at a time, several steps per tick
    for k, r in enumerate(reqs):
        one = make_server(max_slots=1, steps_per_tick=3)
        rid = one.submit(r, fields=fields[k])
        alone = drain_all(one, [rid])[rid][0]
        one.close()
        got = mix[ids[k]][0]
        assert got.shape == (r.steps, len(r.probes))
        assert np.array_equal(got, alone), f"request {k} differs alone vs in the mix"


@requires_gpu
def test_serving_equals_single_simulation():
    """A served FP32 request against the same workload stepped alone through
    the single-simulation entry points.  In 2-D the two kernels order the
    Newton loop differently (rolled in the serving kernel, for its register
    budget); FP32 Newton stops at |dX| < 2e-6, so the two may stop one
    iteration apart and agree only within the FP32 form's own error: their
    difference must stay within twice the single path's error against the
    FP64 path (and is often zero)."""
    from paper_2004_14887_amd.sim import Simulation
    reqs = small_requests(n=6)
    srv = make_server(max_slots=6, steps_per_tick=2)
    ids = [srv.submit(r) for r in reqs]
    res = drain_all(srv, ids)
    srv.close()

    def single(r, prec):
        sim = Simulation(r, prec, probe_capacity=r.steps)
        sim.init_from_workload()
        sim.step(r.steps)
        sim.check()
        p = sim.probes().cpu().numpy()
        sim.close()
        return p

    for k, r in enumerate(reqs):
        print(f"[gpu] single {r.name} steps={r.steps}", flush=True)
        ref32, ref64 = single(r, "fp32"), single(r, "fp64")
        got = res[ids[k]][0]
        peak = max(np.abs(ref64).max(), 1e-30)
        d = float(np.abs(got - ref32).max() / peak)
        e32 = float(np.abs(ref32 - ref64).max() / peak)
        e_srv = float(np.abs(got - ref64).max() / peak)
        print(f"  {r.name}: served vs single {d:.2e}; vs FP64: single {e32:.2e}, served {e_srv:.2e}", flush=True)
        assert d <= max(2.0 * e32, 1e-6), f"request {k}"
        assert e_srv <= max(2.0 * e32, 1e-6), f"request {k}"


@requires_gpu
def test_serving_fp64_matches_oracle():
    from oracle import Oracle
    reqs = [r for r in small_requests(n=10, max_steps=30) if r.n0[0] <= 128][:3]
    assert len(reqs) >= 2
    srv = make_server(precision="fp64", max_slots=3)
    ids = [srv.submit(r) for r in reqs]
    res = drain_all(srv, ids)
    srv.close()
    for k, r in enumerate(reqs):
        o = Oracle(r.lattice, r.n0, r.boxes, r.tau0, r.coupling, r.eq_order, r.probes, r.steps)
        for l in range(r.n_levels):
            rho, u = W.initial_fields(r, l)
            o.init(l, rho, u)
        o.run(r.steps)
        ref = o.probes()
        got = res[ids[k]][0]
        err = float(np.abs(got - ref).max())
        print(f"  {r.name}: max |dp'| {err:.2e} (peak {np.abs(ref).max():.2e})", flush=True)
        assert err <= 1e-13


@requires_gpu
def test_admission_by_footprint():
    from paper_2004_14887_amd.sim import workspace_bytes
    reqs = small_requests(n=8)
    need = [workspace_bytes(r, "fp32") for r in reqs]
    two = sum(sorted(need)[-2:])
    arena = two + 4096
    srv = make_server(arena=arena, max_slots=8, steps_per_tick=2)
    ids = [srv.submit(r) for r in reqs]
    waited_for_memory = False
    for _ in range(100000):
        nr, nq = srv.tick()
        st = srv.stats()
        resident = [srv.info(i) for i in ids if srv.poll(i) == "running"]
        assert sum(r["workspace_bytes"] for r in resident) <= st["arena_bytes"]
        assert len(resident) <= 8
        if nq > 0 and len(resident) < 8:
            waited_for_memory = True
        if nr == 0 and nq == 0:
            break
    assert waited_for_memory
    infos = [srv.result(i)[1] for i in ids]
    assert all(i["state"] == 2 for i in infos)
    # some request was admitted only after another finished
    assert any(b["t_admit"] >= min(a["t_done"] for a in infos) for b in infos)
    srv.close()


@requires_gpu
def test_server_rejects_what_it_cannot_serve():
    from paper_2004_14887_amd._lib import DclbmError
    reqs = small_requests(n=6)
    srv = make_server(arena=64 << 20, max_levels=2, max_probe_steps=40)
    two_level = next(r for r in reqs if r.n_levels <= 2)
    three_level = next(r for r in reqs if r.n_levels == 3)
    with pytest.raises(DclbmError) as ei:
        srv.submit(three_level, steps=10)
    assert ei.value.status == -1
    with pytest.raises(DclbmError) as ei:
        srv.submit(two_level, steps=41)
    assert ei.value.status == -1
    big = W.serving_requests(seed=5, n=1, min_side=1024, max_side=1024)[0][0]
    big.boxes = big.boxes[:1]
    with pytest.raises(DclbmError) as ei:
        srv.submit(big, steps=10)
    assert ei.value.status in (-1, -2)
    srv.precision = "fp64"   # a request of another class than the server's FP32
    with pytest.raises(DclbmError) as ei:
        srv.submit(two_level, steps=10)
    assert ei.value.status == -1
    srv.close()


@requires_gpu
def test_serving_d3q19_equals_single_simulation():
    """A D3Q19 FP32 server (2-level meshes of different sizes, background
    flows): each served request equals the same workload stepped alone
    through the single-simulation entry points, bit for bit (in 3-D both
    kernels run the same Newton loop)."""
    from paper_2004_14887_amd.server import Server
    from paper_2004_14887_amd.sim import Simulation
    reqs = [W.pulse_ring_3d(seed=s, n0=n0, steps=st) for s, n0, st in ((3, 32, 12), (4, 48, 7), (5, 40, 10))]
    srv = Server(1 << 30, lattice="D3Q19", precision="fp32", max_levels=2, max_slots=2, steps_per_tick=3,
                 max_probes=16, max_probe_steps=64, max_level_nodes=100 ** 3)
    ids = [srv.submit(r) for r in reqs]
    srv.drain()
    for k, r in enumerate(reqs):
        assert srv.poll(ids[k]) == "done"
        got = srv.result(ids[k])[0]
        sim = Simulation(r, "fp32", probe_capacity=r.steps)
        sim.init_from_workload()
        sim.step(r.steps)
        sim.check()
        ref = sim.probes().cpu().numpy()
        sim.close()
        assert np.array_equal(got, ref), f"request {k}: max diff {np.abs(got - ref).max()}"
    srv.close()
