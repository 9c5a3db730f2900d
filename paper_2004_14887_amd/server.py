"""Python face of the serving runtime (dclbm_server_* in include/dclbm.h).

A Server owns a torch-allocated device workspace (fixed tables plus the
arena requests are admitted into) and a HIP stream, and forwards every call
to the C ABI.  submit() may run on another thread than tick(): the library
serialises them, and ctypes releases the GIL during each call.

    srv = Server(precision="fp32", max_levels=3, max_slots=64, arena_bytes=8 << 30)
    rid = srv.submit(workload)            # initial fields from the workload
    while srv.poll(rid) not in ("done", "failed"):
        srv.tick()
    probes, info = srv.result(rid)
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from .sim import make_config
from .workloads import Workload, initial_fields


def server_config(lattice="D2Q9", precision="fp32", eq_order=2, max_levels=3, max_slots=64, steps_per_tick=1,
                  max_probes=8, max_probe_steps=2000, max_level_nodes=1 << 20, grid=0, max_inflight=2):
    c = _lib.ServerConfig()
    c.abi_version = _lib.ABI_VERSION
    c.lattice = _lib.LATTICE[lattice]
    c.precision = _lib.PRECISION[precision]
    c.eq_order = eq_order
    c.max_levels = max_levels
    c.max_slots = max_slots
    c.steps_per_tick = steps_per_tick
    c.max_probes = max_probes
    c.max_probe_steps = max_probe_steps
    c.max_level_nodes = max_level_nodes
    c.grid = grid
    c.max_inflight = max_inflight
    return c


def request_fields(wl: Workload):
    """Dense FP64 (rho, u) of every level of a workload, C-contiguous."""
    out = []
    for l in range(wl.n_levels):
        rho, u = initial_fields(wl, l)
        out.append((np.ascontiguousarray(rho, dtype=np.float64), np.ascontiguousarray(u, dtype=np.float64)))
    return out


class Server:
    def __init__(self, arena_bytes: int, device="cuda:0", stream: Optional[torch.cuda.Stream] = None, **cfg):
        self.lib = _lib.load()
        self.cfg = server_config(**cfg)
        self.precision = cfg.get("precision", "fp32")
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        total = C.c_size_t()
        _lib.check(self.lib.dclbm_server_workspace_bytes(C.byref(self.cfg), int(arena_bytes), C.byref(total)))
        self.bytes = total.value
        self._raw = torch.empty(self.bytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._raw.data_ptr() + 255) // 256 * 256
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self.lib.dclbm_server_create(C.byref(self.cfg), C.c_void_p(ptr), self.bytes,
                                                    C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self._n_probes = {}

    def close(self):
        if getattr(self, "h", None):
            self.lib.dclbm_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, wl: Workload, steps: Optional[int] = None, fields: Optional[Sequence] = None,
               newton_max_iter: int = 0, newton_tol: float = 0.0) -> int:
        steps = int(steps if steps is not None else wl.steps)
        cfg, keep = make_config(wl, self.precision, probe_capacity=steps, newton_max_iter=newton_max_iter,
                                newton_tol=newton_tol)
        if fields is None:
            fields = request_fields(wl)
        L = wl.n_levels
        prho = (C.c_void_p * L)(*[f[0].ctypes.data for f in fields])
        pu = (C.c_void_p * L)(*[f[1].ctypes.data for f in fields])
        rid = C.c_uint64()
        _lib.check(self.lib.dclbm_server_submit(self.h, C.byref(cfg), steps, prho, pu, C.byref(rid)))
        self._n_probes[rid.value] = len(wl.probes)
        return rid.value

    def tick(self):
        nr, nq = C.c_int32(), C.c_int32()
        _lib.check(self.lib.dclbm_server_tick(self.h, C.byref(nr), C.byref(nq)))
        return nr.value, nq.value

    def poll(self, rid: int) -> str:
        st = C.c_int32()
        _lib.check(self.lib.dclbm_server_poll(self.h, rid, C.byref(st)))
        return _lib.REQ_STATE[st.value]

    def info(self, rid: int) -> dict:
        inf = _lib.RequestInfo()
        n = C.c_int64()
        self.lib.dclbm_server_result(self.h, rid, None, C.byref(n), C.byref(inf))
        return {k: getattr(inf, k) for k, _ in inf._fields_}

    def result(self, rid: int):
        """(probe series [steps][n_probes] FP64, record) of a finished request."""
        inf = _lib.RequestInfo()
        n = C.c_int64()
        _lib.check(self.lib.dclbm_server_result(self.h, rid, None, C.byref(n), C.byref(inf)))
        npb = max(1, inf.n_probes)
        out = np.zeros((max(1, n.value), npb), dtype=np.float64)
        _lib.check(self.lib.dclbm_server_result(self.h, rid, C.c_void_p(out.ctypes.data), C.byref(n), C.byref(inf)))
        return out[:n.value, :inf.n_probes], {k: getattr(inf, k) for k, _ in inf._fields_}

    def release(self, rid: int):
        _lib.check(self.lib.dclbm_server_release(self.h, rid))

    def stats(self) -> dict:
        inf = _lib.ServerInfo()
        _lib.check(self.lib.dclbm_server_stats(self.h, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in inf._fields_}

    def drain(self, max_ticks: int = 10_000_000):
        """Tick until nothing is resident or queued."""
        for _ in range(max_ticks):
            nr, nq = self.tick()
            if nr == 0 and nq == 0:
                return
        raise RuntimeError("server did not drain")
