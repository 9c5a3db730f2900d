#!/usr/bin/env python3
"""Benchmark: refined-mesh LBM step with direct coupling on one MI355X.

One "step" is one coarse time step of the whole hot path: every level's
fused stream-and-collide with 2:1 sub-cycling, the coarse history capture,
the Newton reconstruction at co-located nodes, hanging-node interpolation,
restriction, and the probe sample.  Default workload: D2Q9, 3 levels,
2048^2 periodic coarse grid with nested x2 (25%) and x4 (6.25%) patches,
Gaussian pulse plus 16 seeded vortices, FP32 arithmetic with FP32 deviation
storage (the production form); the FP64 and FP16-storage forms are timed
beside it, and the FP64 CPU oracle on a bounded sample.

Prints ONE JSON line (see the keys at the bottom).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline, FP32/FP16-store vs FP64 at stated error; p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "fp16"])
    ap.add_argument("--n0", type=int, default=2048)
    ap.add_argument("--latency-steps", type=int, default=200)
    ap.add_argument("--timing-steps", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 / FP16 side runs")
    ap.add_argument("--workload", default="pulse_vortices_3level",
                    choices=["pulse_vortices_3level", "pulse_ring_3d", "rings_4level_uniform"],
                    help="3-level 2048^2 D2Q9 (default), 2-level 256^3 D3Q19, or the 4-level 512^3 D3Q19 mesh at "
                         "full size (FP16 storage only, about 194 GB) carrying a uniform flow")
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


def bytes_per_value(prec):
    return {"fp64": 8, "fp32": 4, "fp16": 2}[prec]


def run_form(wl, prec, steps, warmup, latency_steps, timing_steps):
    import torch

    from paper_2004_14887_amd.sim import Simulation

    log(f"{prec}: create + init ({wl.name})")
    sim = Simulation(wl, prec, probe_capacity=warmup + steps + latency_steps + timing_steps + 2)
    if getattr(wl, "device_uniform", False):
        # a uniform (rho = 1, u = background) state built on the device, level
        # by level: host-side fields of the 1.1e9-node finest level would not pay
        for l in range(wl.n_levels):
            n = sim.n_dense(l)
            rho = torch.ones(n, dtype=torch.float64, device=sim.device)
            u = torch.empty((3, n), dtype=torch.float64, device=sim.device)
            for a in range(3):
                u[a].fill_(wl.background[a])
            sim.init(l, rho, u)
            del rho, u
            torch.cuda.empty_cache()
    else:
        sim.init_from_workload()
    sim.step(warmup)
    sim.synchronize()
    sim.check()
    ups = sim.updates_per_step()
    # timed region: exactly `steps` coarse steps (graph replays after the first step)
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
    log(f"{prec}: {steps} steps in {wall_ms:.2f} ms wall ({gpu_ms:.2f} ms events)")
    # per-step latency percentiles (events around each graph launch)
    lat = []
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(latency_steps + 1)]
    evs[0].record(sim.stream)
    for k in range(latency_steps):
        sim.step(1)
        evs[k + 1].record(sim.stream)
    sim.synchronize()
    for k in range(latency_steps):
        lat.append(evs[k].elapsed_time(evs[k + 1]))
    # instrumented pass: events around every bulk launch (eager launches)
    sim.set_timing(True)
    sim.step(timing_steps)
    sim.synchronize()
    sim.set_timing(False)
    bulk = []
    for l in range(wl.n_levels):
        ms, n, nodes = sim.bulk_time(l)
        bulk.append(dict(level=l, ms=ms, launches=n, nodes_per_launch=nodes))
    sim.check()
    probes = sim.probes().cpu().numpy()
    out = dict(prec=prec, steps=steps, wall_ms=wall_ms, gpu_ms=gpu_ms, updates_per_step=ups,
               mlups=ups * steps / (wall_ms * 1e3), p50=float(np.percentile(lat, 50)),
               p99=float(np.percentile(lat, 99)), bulk=bulk, probes=probes)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def roofline(form, Q, workload):
    bpv = bytes_per_value(form["prec"])
    per_node = 2 * Q * bpv                      # read Q + write Q values (A/B pull)
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
                  "gbs": round(b["nodes_per_launch"] * per_node / (b["ms"] / max(1, b["launches"]) * 1e-3) / 1e9, 1)}
                 for b in form["bulk"]]
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": f"k_level (level {best['level']} substep)", "algorithmic_bytes_per_launch": algo,
            "avg_launch_ms": round(avg_ms, 5), "per_level": per_level}


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


def cpu_baseline(wl_full, steps):
    """The FP64 oracle as it stands, single-threaded, on the first `steps`
    coarse steps of the same workload."""
    from oracle import Oracle
    from paper_2004_14887_amd import workloads as W

    o = Oracle(wl_full.lattice, wl_full.n0, wl_full.boxes, wl_full.tau0, wl_full.coupling, wl_full.eq_order,
               wl_full.probes, steps)
    for l in range(wl_full.n_levels):
        rho, u = W.initial_fields(wl_full, l)
        o.init(l, rho, u)
    t0 = time.perf_counter()
    o.run(steps)
    dt = time.perf_counter() - t0
    ups = 0
    for l in range(wl_full.n_levels):
        cls = o.classes(l)
        ups += int((cls != 0).sum()) << l
    return {"value": round(ups * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"first {steps} coarse steps of the same workload, FP64, single thread ({dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2004_14887_amd import workloads as W

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
    if args.workload == "pulse_ring_3d":
        n0 = args.n0 if args.n0 != 2048 else 256
        wl = W.pulse_ring_3d(seed=3, n0=n0, steps=args.steps)
        mk = lambda steps: W.pulse_ring_3d(seed=3, n0=n0, steps=steps)
    elif args.workload == "rings_4level_uniform":
        # only FP16 storage fits one GPU at this size; no FP64 side run, no
        # oracle baseline (its FP64 state would need about 0.8 TB)
        if args.precision != "fp16":
            sys.exit("rings_4level_uniform: only --precision fp16 fits one GPU")
        wl = W.rings_4level(seed=5, steps=args.steps)
        wl.rings, wl.pulses = [], []
        wl.background = (0.03, -0.02, 0.01)
        wl.name = "rings_4level_512_uniform"
        wl.device_uniform = True
        args.no_compare, args.no_cpu_baseline, args.serving_requests = True, True, 0
        mk = None
    else:
        wl = W.pulse_vortices_3level(seed=2, n0=args.n0, steps=args.steps)
        mk = lambda steps: W.pulse_vortices_3level(seed=2, n0=args.n0, steps=steps)
    main_form = run_form(wl, args.precision, args.steps, args.warmup, args.latency_steps, args.timing_steps)
    side = {}
    if not args.no_compare:
        for p in ("fp64", "fp32", "fp16"):
            if p != args.precision:
                side[p] = run_form(wl, p, args.steps, args.warmup, args.latency_steps, args.timing_steps)
    forms = dict(side)
    forms[args.precision] = main_form
    # accuracy of the reduced-precision forms against the FP64 GPU path
    # (which matches the FP64 oracle to 1e-12, see the parity tests)
    acc = {}
    if "fp64" in forms:
        ref = forms["fp64"]["probes"]
        n = min(len(ref), *(len(f["probes"]) for f in forms.values()))
        for p, f in forms.items():
            if p == "fp64":
                continue
            d = f["probes"][:n] - ref[:n]
            acc[p] = {"e_p_max": float(np.abs(d).max() / np.abs(ref[:n]).max()),
                      "e_p_l2": float(np.linalg.norm(d) / np.linalg.norm(ref[:n]))}
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(mk(args.cpu_steps), args.cpu_steps)
    serving = None
    if args.serving_requests > 0:
        try:
            serving = serving_run(args.serving_requests, args.serving_slots, args.serving_steps_per_tick,
                        tuple(float(x) for x in args.serving_loads.split(",") if x), grid=args.serving_grid,
                        steady_only=args.serving_steady_only)
        except Exception as e:   # reported, never hides the main line
            serving = {"error": repr(e)}
    Q = wl.Q
    rl = roofline(main_form, Q, wl.name)
    bpv = bytes_per_value(args.precision)
    mlups = main_form["mlups"]
    hbm_frac_mlups = mlups * 1e6 * 2 * Q * bpv / (HBM_PEAK_GBS * 1e9)
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
        "hbm_roofline_frac_of_mlups": round(hbm_frac_mlups, 4),
        "copy_kernel_gbs": round(copy_gbs, 1),
        "latency_ms": {"p50": round(main_form["p50"], 5), "p99": round(main_form["p99"], 5)},
        "roofline": rl,
        "cpu_baseline": cpu,
        "serving": serving,
        "forms": {p: {"mlups": round(f["mlups"], 1), "ms_per_step": round(f["wall_ms"] / f["steps"], 5),
                      "p50_ms": round(f["p50"], 5), "p99_ms": round(f["p99"], 5),
                      "speedup_vs_fp64": (round(f["mlups"] / forms["fp64"]["mlups"], 3) if "fp64" in forms else None),
                      "error_vs_fp64": acc.get(p)} for p, f in forms.items()},
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
