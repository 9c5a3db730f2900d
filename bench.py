#!/usr/bin/env python3
"""Benchmark: refined-mesh LBM step with direct coupling on one MI355X.

One "step" is one coarse time step of the whole hot path: every level's
fused stream-and-collide with 2:1 sub-cycling, the coarse history capture,
the Newton reconstruction at co-located nodes, hanging-node interpolation,
restriction, and the probe sample.

`value` is the default workload: D2Q9, 3 levels, 2048^2 periodic coarse grid
with nested x2 (25%) and x4 (6.25%) patches, Gaussian pulse plus 16 seeded
vortices, FP32 arithmetic with FP32 deviation storage (the production form).
Beside it, in the same run:
  * the FP64 and FP16-storage forms of that workload, and the probe errors of
    FP32 and FP16 against the FP64 GPU path over all 1000 coarse steps of it;
  * the 2-level 256^3 D3Q19 workload (pulse and vortex ring, Mach-0.1 mean
    flow) in all three forms, with errors over its 500 coarse steps;
  * the 4-level 512^3 D3Q19 workload (64 vortex rings, 8 pulses; refined
    boxes of 30.3%, 10.0% and 1.87% of the volume, about 206 GB) in FP16
    storage;
  * the H-RR collision of Sec. 2 on the 2048^2 3-level mesh (with the
    interface gradients of Sec. 3.3), FP32 and FP64;
  * the reflection and spurious-noise studies of Sec. 4.1.1 and 4.2.1, DC1
    against DC2;
  * the serving loop (256 seeded requests);
  * the FP64 CPU oracle (single thread and all host cores) on bounded samples.

Prints ONE JSON line (see the keys at the bottom).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline, FP32/FP16-store vs FP64 at stated error; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
BYTES = {"fp64": 8, "fp32": 4, "fp16": 2}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "fp16"])
    ap.add_argument("--n0", type=int, default=2048)
    ap.add_argument("--latency-steps", type=int, default=200)
    ap.add_argument("--timing-steps", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=2, help="coarse steps of the single-thread oracle sample")
    ap.add_argument("--cpu-steps-parallel", type=int, default=8, help="coarse steps of the all-core oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 / FP16 side runs")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the full-length accuracy runs")
    ap.add_argument("--no-3d", action="store_true", help="skip the 256^3 D3Q19 workload")
    ap.add_argument("--no-4level", action="store_true", help="skip the 4-level 512^3 D3Q19 workload")
    ap.add_argument("--no-hrr", action="store_true", help="skip the H-RR collision on the 2048^2 3-level mesh")
    ap.add_argument("--no-studies", action="store_true", help="skip the reflection and spurious-noise studies")
    ap.add_argument("--workload", default="pulse_vortices_3level",
                    choices=["pulse_vortices_3level", "pulse_ring_3d", "rings_4level"],
                    help="workload of `value`: 3-level 2048^2 D2Q9 (default), 2-level 256^3 D3Q19, or the "
                         "4-level 512^3 D3Q19 mesh (FP16 storage only)")
    ap.add_argument("--copy-only", action="store_true", help="only run the plain copy kernel (counter calibration)")
    ap.add_argument("--serving-requests", type=int, default=256, help="requests in the serving run (0: skip it)")
    ap.add_argument("--serving-only", action="store_true", help="only the serving run")
    ap.add_argument("--serving-slots", type=int, default=128)
    ap.add_argument("--serving-steps-per-tick", type=int, default=4)
    ap.add_argument("--serving-loads", default="0.5,0.9", help="offered loads of the open-loop runs ('' for none)")
    ap.add_argument("--serving-grid", type=int, default=0, help="workgroups of the persistent launches (0: resident)")
    ap.add_argument("--serving-steady-only", action="store_true", help="only the steady-state part of the serving run")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name, steps, n0=None):
    from paper_2004_14887_amd import workloads as W

    if name == "pulse_ring_3d":
        return W.pulse_ring_3d(seed=3, n0=n0 or 256, steps=steps)
    if name == "rings_4level":
        return W.rings_4level(seed=5, steps=steps)
    return W.pulse_vortices_3level(seed=2, n0=n0 or 2048, steps=steps)


def new_sim(wl, prec, capacity, on_device):
    from paper_2004_14887_amd.sim import Simulation

    log(f"{wl.name} {prec}: create + init")
    sim = Simulation(wl, prec, probe_capacity=capacity)
    sim.init_from_workload(on_device=on_device)
    return sim


def run_form(wl, prec, steps, warmup, latency_steps, timing_steps, on_device=False):
    """Time `steps` coarse steps (graph replays) after `warmup`, then per-step
    latencies, then an instrumented pass with in-dispatch events around every
    level-substep launch."""
    import torch

    sim = new_sim(wl, prec, warmup + steps + latency_steps + timing_steps + 2, on_device)
    sim.step(warmup)
    sim.synchronize()
    sim.check()
    ups = sim.updates_per_step()
    # timed region: exactly `steps` coarse steps
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(sim.stream)
    t0 = time.perf_counter()
    sim.step(steps)
    ev1.record(sim.stream)
    sim.synchronize()
    t1 = time.perf_counter()
    wall_ms = (t1 - t0) * 1e3
    gpu_ms = ev0.elapsed_time(ev1)
    log(f"{wl.name} {prec}: {steps} steps in {wall_ms:.2f} ms wall ({gpu_ms:.2f} ms events)")
    lat = []
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(latency_steps + 1)]
    evs[0].record(sim.stream)
    for k in range(latency_steps):
        sim.step(1)
        evs[k + 1].record(sim.stream)
    sim.synchronize()
    for k in range(latency_steps):
        lat.append(evs[k].elapsed_time(evs[k + 1]))
    sim.set_timing(True)
    sim.step(timing_steps)
    sim.synchronize()
    sim.set_timing(False)
    bulk = []
    for l in range(wl.n_levels):
        ms, n, nodes = sim.bulk_time(l)
        bulk.append(dict(level=l, ms=ms, launches=n, nodes_per_launch=nodes, iface_bytes=sim.interface_bytes(l)))
    sim.check()
    out = dict(prec=prec, steps=steps, wall_ms=wall_ms, gpu_ms=gpu_ms, updates_per_step=ups,
               mlups=ups * steps / (wall_ms * 1e3), p50=float(np.percentile(lat, 50)) if lat else None,
               p99=float(np.percentile(lat, 99)) if lat else None, bulk=bulk, workspace_gb=sim.bytes / 1e9)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def probe_series(wl, prec, on_device=False):
    """Probe series of every coarse step of the workload's full length."""
    import torch

    sim = new_sim(wl, prec, wl.steps, on_device)
    sim.step(wl.steps)
    sim.check()
    p = sim.probes().cpu().numpy()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return p


def accuracy(wl, precs, on_device=False):
    """Probe errors e_p = max|p' - p'_FP64| / max|p'_FP64| (and the L2 form)
    of each reduced form against the FP64 GPU path, over all wl.steps coarse
    steps.  The FP64 GPU path matches the FP64 oracle to 1e-12 (parity tests)."""
    ref = probe_series(wl, "fp64", on_device)
    out = {"steps": wl.steps, "reference": "FP64 GPU path", "peak_abs_p": float(np.abs(ref).max())}
    for p in precs:
        g = probe_series(wl, p, on_device)
        d = g - ref
        out[p] = {"e_p_max": float(np.abs(d).max() / np.abs(ref).max()),
                  "e_p_l2": float(np.linalg.norm(d) / np.linalg.norm(ref)),
                  "target": 1e-4 if p == "fp32" else 1e-3}
        log(f"{wl.name} accuracy {p}: {out[p]}")
    return out


def roofline(form, Q, workload):
    """Dominant launch (longest total time): algorithmic bytes per launch
    (updated nodes x 2Q values) over its mean in-dispatch duration, against
    8 TB/s; the interface bytes of that launch are stated separately."""
    bpv = BYTES[form["prec"]]
    per_node = 2 * Q * bpv
    best = max(form["bulk"], key=lambda b: b["ms"])
    avg_ms = best["ms"] / max(1, best["launches"])
    algo = best["nodes_per_launch"] * per_node
    achieved = algo / (avg_ms * 1e-3) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        rec = json.load(open(tfile))
        key = f"{workload}/{form['prec']}/level{best['level']}"
        src = open(os.path.join(ROOT, "paper_2004_14887_amd", "csrc", "kernels.hpp"), "rb").read()
        if rec.get("kernels_sha256") == hashlib.sha256(src).hexdigest() and key in rec.get("bytes_per_launch", {}):
            traffic = rec["bytes_per_launch"][key]
    per_level = [{"level": b["level"], "launches": b["launches"], "nodes_per_launch": b["nodes_per_launch"],
                  "avg_launch_ms": round(b["ms"] / max(1, b["launches"]), 5),
                  "gbs": round(b["nodes_per_launch"] * per_node / (b["ms"] / max(1, b["launches"]) * 1e-3) / 1e9, 1),
                  "interface_bytes_per_launch": round(b["iface_bytes"])}
                 for b in form["bulk"]]
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": f"k_level (level {best['level']} substep)", "algorithmic_bytes_per_launch": algo,
            "interface_bytes_per_launch": round(best["iface_bytes"]),
            "frac_with_interface_bytes": round((algo + best["iface_bytes"]) / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "avg_launch_ms": round(avg_ms, 5), "per_level": per_level}


def form_summary(f, Q, ref_mlups=None, err=None):
    bpv = BYTES[f["prec"]]
    return {"mlups": round(f["mlups"], 1), "ms_per_step": round(f["wall_ms"] / f["steps"], 5),
            "pct_hbm_roofline": round(100.0 * f["mlups"] * 1e6 * 2 * Q * bpv / (HBM_PEAK_GBS * 1e9), 2),
            "p50_ms": None if f["p50"] is None else round(f["p50"], 5),
            "p99_ms": None if f["p99"] is None else round(f["p99"], 5),
            "speedup_vs_fp64": round(f["mlups"] / ref_mlups, 3) if ref_mlups else None,
            "error_vs_fp64": err, "workspace_gb": round(f["workspace_gb"], 2)}


def serving_run(n_requests, slots, steps_per_tick, loads=(0.5, 0.9), seed=4, grid=0, steady_only=False):
    """Continuous batching of a seeded Poisson stream of D2Q9 FP32 requests
    (side 64-1024, 1-3 levels, 100-2000 steps) on one long-lived server.

    * warm-up: the whole stream once, closed loop (fills the pinned pool);
    * capacity: the stream again, every request queued at once (8 submitting
      threads): aggregate MLUPS = updates / (last completion - first arrival);
    * steady state: `slots` resident copies of one 3-level request, MLUPS
      over 20 ticks, beside the same request stepped alone through the
      single-simulation path;
    * open loop at `loads` of the capacity: the seeded unit-rate gaps
      rescaled; latency = completion - arrival (the library's clock)."""
    import threading
    from concurrent.futures import ThreadPoolExecutor

    import torch

    from paper_2004_14887_amd import workloads as W
    from paper_2004_14887_amd.server import Server, request_fields
    from paper_2004_14887_amd.sim import Simulation

    reqs, gaps = W.serving_requests(seed=seed, n=n_requests)
    log(f"serving: generating initial fields of {len(reqs)} requests")
    with ThreadPoolExecutor(8) as ex:
        fields = list(ex.map(request_fields, reqs))
    max_nodes = max(r.n_nodes(l) for r in reqs for l in range(r.n_levels))
    arena = 24 << 30
    srv = Server(arena, precision="fp32", max_levels=3, max_slots=slots, steps_per_tick=steps_per_tick,
                 max_probes=8, max_probe_steps=max(r.steps for r in reqs), max_level_nodes=max_nodes, grid=grid)

    def one_run(arrivals, producers=1):
        torch.cuda.synchronize()
        ticks0 = srv.stats()["ticks"]
        ids = [None] * len(reqs)
        left = [producers]
        lock = threading.Lock()

        def producer(part):
            t0 = time.perf_counter()
            for k in part:
                if arrivals is not None:
                    dt = t0 + arrivals[k] - time.perf_counter()
                    if dt > 0:
                        time.sleep(dt)
                ids[k] = srv.submit(reqs[k], fields=fields[k])
            with lock:
                left[0] -= 1

        ths = [threading.Thread(target=producer, args=(list(range(j, len(reqs), producers)),))
               for j in range(producers)]
        for th in ths:
            th.start()
        while True:
            nr, nq = srv.tick()
            if nr == 0 and nq == 0:
                with lock:
                    if left[0] == 0:
                        break
                time.sleep(5e-5)
        for th in ths:
            th.join()
        nr, nq = srv.tick()
        assert nr == 0 and nq == 0
        infos = [srv.result(i)[1] if srv.poll(i) == "done" else srv.info(i) for i in ids]
        for i in ids:
            srv.release(i)
        ok = [i for i in infos if i["state"] == 2]
        lat = np.array([i["t_done"] - i["t_submit"] for i in ok])
        qd = np.array([i["t_admit"] - i["t_submit"] for i in ok])
        span = max(i["t_done"] for i in ok) - min(i["t_submit"] for i in infos)
        ups = sum(i["updates"] for i in ok)
        return {"mlups": round(ups / span / 1e6, 1), "makespan_s": round(span, 3),
                "latency_p50_s": round(float(np.percentile(lat, 50)), 4),
                "latency_p99_s": round(float(np.percentile(lat, 99)), 4),
                "queue_p50_s": round(float(np.percentile(qd, 50)), 4),
                "queue_p99_s": round(float(np.percentile(qd, 99)), 4),
                "completed": len(ok), "failed": len(infos) - len(ok),
                "ticks": srv.stats()["ticks"] - ticks0, "updates": int(ups)}

    cap = None
    if not steady_only:
        log("serving: warm-up (closed loop)")
        one_run(None, producers=8)
        log("serving: closed loop (capacity)")
        cap = one_run(None, producers=8)
        log(f"serving: capacity {cap['mlups']} MLUPS over {cap['makespan_s']} s")

    # steady state: `slots` resident copies of one 3-level request
    tmpl = next(r for r in reqs if r.n_levels == 3 and 400 <= r.n0[0] <= 640)
    ticks = 20
    steps = steps_per_tick * (ticks + 4)
    tf = request_fields(tmpl)
    ids = [srv.submit(tmpl, steps=steps, fields=tf) for _ in range(slots)]
    srv.tick()
    srv.tick()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(ticks):
        srv.tick()
    srv.stream.synchronize()
    dt = time.perf_counter() - t0
    per_step = srv.info(ids[0])["updates"] // steps
    srv.drain()
    for i in ids:
        srv.release(i)
    sim = Simulation(tmpl, "fp32", probe_capacity=steps + 8)
    sim.init_from_workload()
    sim.step(4)
    sim.synchronize()
    t1 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    dt1 = time.perf_counter() - t1
    sim.close()
    steady = {"request": tmpl.name, "resident": slots, "updates_per_step_each": int(per_step),
              "mlups": round(slots * per_step * steps_per_tick * ticks / dt / 1e6, 1),
              "alone_single_simulation_mlups": round(per_step * steps / dt1 / 1e6, 1)}
    log(f"serving: steady state {steady}")
    if steady_only:
        g = srv.stats()["grid"]
        srv.close()
        return {"steady_state": steady, "grid": g}

    out = {"requests": len(reqs), "precision": "fp32", "slots": slots, "steps_per_tick": steps_per_tick,
           "arena_gb": arena / 2 ** 30, "capacity": cap, "steady_state": steady, "loads": {}}
    mean_updates = cap["updates"] / max(1, cap["completed"])
    for load in loads:
        rate = load * cap["mlups"] * 1e6 / mean_updates      # requests per second
        arrivals = np.cumsum(gaps) / rate
        arrivals -= arrivals[0]
        log(f"serving: open loop at load {load} ({rate:.1f} requests/s)")
        out["loads"][str(load)] = one_run(arrivals)
        log(f"serving: load {load}: {out['loads'][str(load)]}")
    srv.close()
    return out


def _oracle_mlups(lib_path, wl, steps, threads):
    from oracle import Oracle
    from paper_2004_14887_amd import workloads as W

    o = Oracle(wl.lattice, wl.n0, wl.boxes, wl.tau0, wl.coupling, wl.eq_order, wl.probes, steps, lib_path=lib_path)
    o.set_threads(threads)
    for l in range(wl.n_levels):
        rho, u = W.initial_fields(wl, l)
        o.init(l, rho, u)
    used = o.threads()
    t0 = time.perf_counter()
    o.run(steps)
    dt = time.perf_counter() - t0
    ups = sum(int((o.classes(l) != 0).sum()) << l for l in range(wl.n_levels))
    del o
    return ups * steps / dt / 1e6, dt, used


def cpu_baseline(name, n0, steps_single, steps_all):
    """The FP64 oracle as it stands, built for this host (-O3 -march=native,
    OpenMP over its node loops; same arithmetic as the checking build) and
    timed on bounded samples of the benchmark workload: the first coarse steps,
    on one thread and on all host cores; plus the 128^2 two-level vortex
    workload over all its 200 coarse steps."""
    from oracle import build_baseline
    from paper_2004_14887_amd import workloads as W

    d = tempfile.mkdtemp(prefix="oracle_baseline_")
    lib = build_baseline(d)
    nproc = os.cpu_count() or 1
    threads = int(os.environ.get("OMP_NUM_THREADS", nproc))
    wl = make_workload(name, steps_all, n0)
    one, dt1, _ = _oracle_mlups(lib, wl, steps_single, 1)
    log(f"cpu baseline: {one:.2f} MLUPS single thread ({dt1:.1f} s)")
    allc, dta, used = _oracle_mlups(lib, wl, steps_all, threads)
    log(f"cpu baseline: {allc:.2f} MLUPS on {used} threads ({dta:.1f} s)")
    c1 = W.vortex_2level(seed=1, n0=128, steps=200)
    c1_one, c1_dt1, _ = _oracle_mlups(lib, c1, 200, 1)
    c1_all, c1_dta, c1_used = _oracle_mlups(lib, c1, 200, threads)
    return {"value": round(allc, 3), "unit": "MLUPS", "cores": used, "kind": "oracle",
            "sample": f"first {steps_all} coarse steps of {wl.name}, FP64, {used} OpenMP threads ({dta:.1f} s); "
                      f"single thread over the first {steps_single} steps ({dt1:.1f} s)",
            "single_thread_mlups": round(one, 3), "nproc": nproc,
            "build": "gcc -O3 -march=native -fopenmp -ffp-contract=off",
            "vortex_2level_128_full_200_steps": {"single_thread_mlups": round(c1_one, 3), "single_thread_s": round(c1_dt1, 2),
                                                 "all_core_mlups": round(c1_all, 3), "all_core_s": round(c1_dta, 2),
                                                 "threads": c1_used}}


def workload_block(name, steps, warmup, latency_steps, timing_steps, precs, with_accuracy, on_device):
    """Timed forms, roofline and full-length accuracy of one extra workload."""
    wl = make_workload(name, steps)
    Q = wl.Q
    forms = {p: run_form(wl, p, steps, warmup, latency_steps, timing_steps, on_device) for p in precs}
    acc = None
    if with_accuracy and "fp64" in precs:
        acc = accuracy(_full_length(name), [p for p in precs if p != "fp64"], on_device)
    ref = forms["fp64"]["mlups"] if "fp64" in forms else None
    main = "fp32" if "fp32" in forms else precs[0]
    out = {"config": {"workload": wl.name, "lattice": wl.lattice, "levels": wl.n_levels, "n0": list(wl.n0),
                      "boxes": [list(map(list, b)) for b in wl.boxes], "tau0": wl.tau0,
                      "updates_per_step": forms[main]["updates_per_step"]},
           "forms": {p: form_summary(f, Q, ref, (acc or {}).get(p)) for p, f in forms.items()},
           "roofline": roofline(forms[main], Q, wl.name)}
    if acc:
        out["accuracy"] = {k: v for k, v in acc.items() if k in ("steps", "reference", "peak_abs_p")}
    return out


def _full_length(name):
    """The workload at its configured number of coarse steps."""
    from paper_2004_14887_amd import workloads as W

    if name == "pulse_ring_3d":
        return W.pulse_ring_3d(seed=3, n0=256)
    return W.pulse_vortices_3level(seed=2, n0=2048)


def four_level_block(steps, warmup):
    """The 4-level 512^3 D3Q19 workload at full size, FP16 storage: 64 seeded
    vortex rings and 8 pulses evaluated on the device."""
    wl = make_workload("rings_4level", steps)
    f = run_form(wl, "fp16", steps, warmup, min(steps, 5), 1, on_device=True)
    sides = [wl.boxes[0][1][0] - wl.boxes[0][0][0]] + \
        [(wl.boxes[k][1][0] - wl.boxes[k][0][0]) / 2 ** k for k in (1, 2)]
    return {"config": {"workload": wl.name, "lattice": wl.lattice, "levels": wl.n_levels, "n0": list(wl.n0),
                       "boxes": [list(map(list, b)) for b in wl.boxes], "tau0": wl.tau0,
                       "box_sides_coarse_cells": sides,
                       "volume_fractions": [round((s / 512.0) ** 3, 4) for s in sides],
                       "rings": len(wl.rings), "pulses": len(wl.pulses),
                       "updates_per_step": f["updates_per_step"]},
            "forms": {"fp16": form_summary(f, wl.Q)},
            "roofline": roofline(f, wl.Q, wl.name)}


def hrr_block(steps, warmup, bgk_mlups):
    """The H-RR collision (Sec. 2) on the 2048^2 3-level mesh with the
    interface gradients of Sec. 3.3: FP32 and FP64, eager launches (four per
    refined level substep, two on level 0).  Minimum HBM traffic per node
    update: the populations read twice (the macroscopic pass and the
    collision) and written once, and the D + 1 macroscopic values written
    and read once: 3 Q + 2 (D + 1) values."""
    wl = make_workload("pulse_vortices_3level", steps)
    wl.collision = "hrr"
    forms = {p: run_form(wl, p, steps, warmup, min(steps, 20), 0, True) for p in ("fp32", "fp64")}
    out = {}
    for p, f in forms.items():
        bpv = BYTES[p]
        gbs = f["mlups"] * 1e6 * (3 * wl.Q + 2 * (wl.D + 1)) * bpv / 1e9
        out[p] = {"mlups": round(f["mlups"], 1), "ms_per_step": round(f["wall_ms"] / f["steps"], 5),
                  "min_traffic_gbs": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                  "vs_bgk_same_form": round(f["mlups"] / bgk_mlups[p], 3) if bgk_mlups.get(p) else None}
    return {"config": {"workload": wl.name + "_hrr", "sigma": wl.hrr_sigma, "psi": wl.hrr_psi,
                       "updates_per_step": forms["fp32"]["updates_per_step"]}, "forms": out}


def studies_block():
    """The paper's acoustic studies on the GPU path, DC1 against DC2 (FP64):
    the pulse reflected by plane interfaces (Sec. 4.1.1) and by a
    stair-stepped circular interface (Sec. 4.1.2; largest and RMS reflected
    velocity divergence relative to the uniform-fine reference's peak, after
    90 coarse steps) and the spurious noise of a vortex convected across a
    plane and a 30-degree-inclined interface (Sec. 4.2.1, 4.2.2; OASPL over
    36 probes, H-RR at the physical viscosity, the paper's 3 m domain of
    150^2 coarse cells with absorbing layers, coarse steps 200-650), with the
    same vortex on the unrefined mesh beside it."""
    from paper_2004_14887_amd import studies

    refl, refl_c, noise = {}, {}, {}
    for cp in (1, 2):
        t0 = time.perf_counter()
        r = studies.reflection(steps=90, coupling=cp)
        refl[f"DC{cp}"] = {"max": float(f"{r['max']:.4g}"), "l2": float(f"{r['l2']:.4g}")}
        r = studies.reflection(steps=90, coupling=cp, shape="circle")
        refl_c[f"DC{cp}"] = {"max": float(f"{r['max']:.4g}"), "l2": float(f"{r['l2']:.4g}")}
        v = studies.vortex_oaspl(coupling=cp)
        noise[f"DC{cp}"] = {"max_db": round(v["max"], 2), "mean_db": round(v["mean"], 2)}
        log(f"studies DC{cp}: reflection {r['max']:.3e}, OASPL max {v['max']:.2f} dB "
            f"({time.perf_counter() - t0:.1f} s)")
    v = studies.vortex_oaspl(coupling=2, boxes=[])
    noise["no_refinement"] = {"max_db": round(v["max"], 2), "mean_db": round(v["mean"], 2)}
    inclined = {}
    for cp in (1, 2):
        v = studies.vortex_oaspl(coupling=cp, shape="inclined")
        inclined[f"DC{cp}"] = {"max_db": round(v["max"], 2), "mean_db": round(v["mean"], 2)}
    inclined["paper_table"] = {"note": "context only", "STD": {"max_db": 85.1, "mean_db": 82.6},
                               "DC1": {"max_db": 84.5, "mean_db": 80.9}, "DC2": {"max_db": 82.1, "mean_db": 79.6}}
    noise["paper_table"] = {"note": "context only: its absorbing layers and probe window are not given",
                            "STD": {"max_db": 80.7, "mean_db": 77.0}, "DC1": {"max_db": 68.9, "mean_db": 65.6},
                            "DC2": {"max_db": 69.8, "mean_db": 66.5}}
    return {"reflection_pulse_plane_150": refl, "reflection_pulse_circle_150": refl_c, "oaspl_vortex_plane_150": noise,
            "oaspl_vortex_inclined_150": inclined}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only: a multi-GPU run is not part of it; "
                                   "run with --gpus 1"}))
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    from paper_2004_14887_amd.sim import copy_calibration

    copy_gbs, copy_ms = copy_calibration()
    log(f"copy kernel: {copy_gbs:.1f} GB/s ({copy_ms:.4f} ms per 512 MiB copy)")
    if args.copy_only:
        print(json.dumps({"copy_gbs": round(copy_gbs, 1), "copy_ms": copy_ms}))
        return
    if args.serving_only:
        print(json.dumps(serving_run(args.serving_requests, args.serving_slots, args.serving_steps_per_tick,
                        tuple(float(x) for x in args.serving_loads.split(",") if x), grid=args.serving_grid,
                        steady_only=args.serving_steady_only)))
        return
    name = args.workload
    # initial fields evaluated on the device (outside every timed region)
    on_device = True
    if name == "rings_4level" and args.precision != "fp16":
        sys.exit("rings_4level: only --precision fp16 fits one GPU")
    wl = make_workload(name, args.steps, args.n0 if name == "pulse_vortices_3level" else None)
    main_form = run_form(wl, args.precision, args.steps, args.warmup, args.latency_steps, args.timing_steps,
                         on_device)
    forms = {args.precision: main_form}
    if not args.no_compare and name != "rings_4level":
        for p in ("fp64", "fp32", "fp16"):
            if p != args.precision:
                forms[p] = run_form(wl, p, args.steps, args.warmup, args.latency_steps, args.timing_steps, on_device)
    acc = {}
    if not args.no_accuracy and "fp64" in forms and args.n0 == 2048 and name != "rings_4level":
        acc = accuracy(_full_length(name), [p for p in forms if p != "fp64"], on_device)
    extra = {}
    if name == "pulse_vortices_3level" and not args.no_3d:
        extra["pulse_ring_3d_256"] = workload_block("pulse_ring_3d", args.steps, min(args.warmup, 5),
                                                    min(args.latency_steps, 50), min(args.timing_steps, 5),
                                                    ["fp32", "fp16", "fp64"], not args.no_accuracy, True)
    if name == "pulse_vortices_3level" and not args.no_4level:
        torch.cuda.empty_cache()
        extra["rings_4level_512"] = four_level_block(min(args.steps, 10), min(args.warmup, 2))
    if name == "pulse_vortices_3level" and args.n0 == 2048 and not args.no_hrr:
        torch.cuda.empty_cache()
        extra["hrr_pulse_vortices_3level_2048"] = hrr_block(min(args.steps, 100), min(args.warmup, 5),
                                                            {p: f["mlups"] for p, f in forms.items()})
    if name == "pulse_vortices_3level" and not args.no_studies:
        torch.cuda.empty_cache()
        extra["studies"] = studies_block()
    cpu = None
    if not args.no_cpu_baseline and name != "rings_4level":
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(name, args.n0 if name == "pulse_vortices_3level" else None, args.cpu_steps,
                           args.cpu_steps_parallel)
    serving = None
    if args.serving_requests > 0 and name == "pulse_vortices_3level":
        try:
            serving = serving_run(args.serving_requests, args.serving_slots, args.serving_steps_per_tick,
                                  tuple(float(x) for x in args.serving_loads.split(",") if x), grid=args.serving_grid,
                                  steady_only=args.serving_steady_only)
        except Exception as e:   # reported, never hides the main line
            serving = {"error": repr(e)}
    Q = wl.Q
    rl = roofline(main_form, Q, wl.name)
    mlups = main_form["mlups"]
    ref = forms["fp64"]["mlups"] if "fp64" in forms else None
    res = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_form["wall_ms"] / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f32 (f16 storage)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": wl.name, "lattice": wl.lattice, "levels": wl.n_levels, "n0": list(wl.n0),
                   "steps_per_run": args.steps,
                   "boxes": [list(map(list, b)) for b in wl.boxes], "tau0": wl.tau0, "coupling": "DC2",
                   "precision": args.precision, "updates_per_step": main_form["updates_per_step"]},
        "hbm_roofline_frac_of_mlups": round(mlups * 1e6 * 2 * Q * BYTES[args.precision] / (HBM_PEAK_GBS * 1e9), 4),
        "copy_kernel_gbs": round(copy_gbs, 1),
        "latency_ms": {"p50": main_form["p50"] and round(main_form["p50"], 5),
                       "p99": main_form["p99"] and round(main_form["p99"], 5)},
        "roofline": rl,
        "cpu_baseline": cpu,
        "forms": {p: form_summary(f, Q, ref, acc.get(p)) for p, f in forms.items()},
        "accuracy": {k: v for k, v in acc.items() if k in ("steps", "reference", "peak_abs_p")} or None,
        "workloads": extra or None,
        "serving": serving,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
