"""Python face of the library: a Simulation owns a torch-allocated device
workspace and a HIP stream (torch's), and forwards every call to the C ABI.

    from paper_2004_14887_amd import Simulation, workloads
    wl = workloads.vortex_2level()
    sim = Simulation(wl, precision="fp64")
    sim.init_from_workload()
    sim.step(wl.steps)
    f1 = sim.populations(1)        # torch float64 [Q, n] on the device
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import _lib
from .workloads import Workload, initial_fields, initial_fields_device


def make_config(wl: Workload, precision: str = "fp64", probe_capacity: Optional[int] = None,
                newton_max_iter: int = 0, newton_tol: float = 0.0, u_ref=None):
    """C configuration of a workload.  u_ref (reduced-precision storage
    reference velocity) defaults to the workload's background flow."""
    cfg = _lib.Config()
    cfg.abi_version = _lib.ABI_VERSION
    cfg.lattice = _lib.LATTICE[wl.lattice]
    cfg.precision = _lib.PRECISION[precision]
    cfg.coupling = wl.coupling
    cfg.eq_order = wl.eq_order
    for a in range(3):
        cfg.n0[a] = wl.n0[a] if a < wl.D else 1
    cfg.n_levels = wl.n_levels
    for k, (lo, hi) in enumerate(wl.boxes):
        for a in range(wl.D):
            cfg.box_lo[k][a] = lo[a]
            cfg.box_hi[k][a] = hi[a]
    cfg.tau0 = wl.tau0
    probes = (C.c_int32 * max(1, 3 * len(wl.probes)))()
    for k, p in enumerate(wl.probes):
        for a in range(wl.D):
            probes[3 * k + a] = p[a]
    cfg.n_probes = len(wl.probes)
    cfg.h_probe_xyz = C.cast(probes, C.POINTER(C.c_int32))
    cfg.probe_capacity = probe_capacity if probe_capacity is not None else max(1, wl.steps)
    cfg.newton_max_iter = newton_max_iter
    cfg.newton_tol = newton_tol
    ur = wl.background if u_ref is None else u_ref
    for a in range(3):
        cfg.u_ref[a] = float(ur[a]) if a < len(ur) and a < wl.D else 0.0
    cfg.collision = _lib.COLLISION[wl.collision]
    cfg.hrr_sigma = float(wl.hrr_sigma)
    cfg.hrr_psi = 1 if wl.hrr_psi else 0
    cfg.sponge_cells = int(wl.sponge_cells)
    cfg.sponge_sigma = float(wl.sponge_sigma)
    keep = [probes]
    if wl.region is not None:
        region = np.ascontiguousarray(np.asarray(wl.region, dtype=np.uint8))
        lo, hi = wl.boxes[0]
        assert region.shape == (hi[1] - lo[1], hi[0] - lo[0]), "region mask must cover level 1's box cells"
        cfg.h_region = region.ctypes.data_as(C.POINTER(C.c_uint8))
        keep.append(region)
    return cfg, keep


def workspace_bytes(wl: Workload, precision: str = "fp64", **kw) -> int:
    lib = _lib.load()
    cfg, _keep = make_config(wl, precision, **kw)
    out = C.c_size_t()
    _lib.check(lib.dclbm_workspace_bytes(C.byref(cfg), C.byref(out)))
    return out.value


class Simulation:
    def __init__(self, wl: Workload, precision: str = "fp64", device="cuda:0",
                 stream: Optional[torch.cuda.Stream] = None, probe_capacity: Optional[int] = None,
                 newton_max_iter: int = 0, newton_tol: float = 0.0, u_ref=None):
        self.lib = _lib.load()
        self.wl = wl
        self.precision = precision
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        cfg, self._probe_buf = make_config(wl, precision, probe_capacity, newton_max_iter, newton_tol, u_ref)
        self.cfg = cfg
        nbytes = C.c_size_t()
        _lib.check(self.lib.dclbm_workspace_bytes(C.byref(cfg), C.byref(nbytes)))
        self.bytes = nbytes.value
        # 256-byte aligned view into a torch-owned uint8 buffer
        self._raw = torch.empty(self.bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._raw.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self.lib.dclbm_create(C.byref(cfg), C.c_void_p(self._ws_ptr), self.bytes,
                                             C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.D, self.Q = wl.D, wl.Q

    def close(self):
        if getattr(self, "h", None):
            self.lib.dclbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- geometry
    def level_shape(self, l):
        dims = (C.c_int32 * 3)()
        n = C.c_int64()
        _lib.check(self.lib.dclbm_level_shape(self.h, l, dims, C.byref(n)))
        return tuple(dims), n.value

    def n_dense(self, l):
        d, _ = self.level_shape(l)
        return d[0] * d[1] * d[2]

    def updates_per_step(self):
        u = C.c_int64()
        _lib.check(self.lib.dclbm_updates_per_step(self.h, C.byref(u)))
        return u.value

    # ---------------------------------------------------------------- state
    def _sync_torch(self):
        # caller-side work (torch kernels on the current stream) must finish
        # before the library's stream reads it, and vice versa
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def init(self, level, rho: torch.Tensor, u: torch.Tensor):
        rho = rho.to(self.device, torch.float64).contiguous()
        u = u.to(self.device, torch.float64).contiguous()
        assert rho.numel() == self.n_dense(level) and u.shape[0] == self.D
        self._sync_torch()
        _lib.check(self.lib.dclbm_init_equilibrium(self.h, level, C.c_void_p(rho.data_ptr()),
                                                   C.c_void_p(u.data_ptr())))
        self.stream.synchronize()

    def init_from_workload(self, on_device: bool = False):
        """Initial equilibrium from the workload's analytic fields, evaluated
        on the host (numpy) or, for large meshes, on the device (each
        structure on its bounding box)."""
        for l in range(self.wl.n_levels):
            if on_device:
                rho, u = initial_fields_device(self.wl, l, self.device)
                self.init(l, rho, u)
                del rho, u
                torch.cuda.empty_cache()
            else:
                rho, u = initial_fields(self.wl, l)
                self.init(l, torch.from_numpy(rho), torch.from_numpy(u))

    def step(self, n: int = 1):
        _lib.check(self.lib.dclbm_step(self.h, int(n)))

    def synchronize(self):
        self.stream.synchronize()

    def check(self):
        _lib.check(self.lib.dclbm_check(self.h))

    def _out(self, shape):
        return torch.empty(shape, dtype=torch.float64, device=self.device)

    def populations(self, l) -> torch.Tensor:
        out = self._out((self.Q, self.n_dense(l)))
        self._sync_torch()
        _lib.check(self.lib.dclbm_read_populations(self.h, l, C.c_void_p(out.data_ptr())))
        self.stream.synchronize()
        return out

    def macros(self, l):
        n = self.n_dense(l)
        rho, u = self._out((n,)), self._out((self.D, n))
        _lib.check(self.lib.dclbm_read_macros(self.h, l, C.c_void_p(rho.data_ptr()), C.c_void_p(u.data_ptr())))
        self.stream.synchronize()
        return rho, u

    def divergence(self, l, u: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Centred-difference velocity divergence [n] of level l (NaN where a
        stencil point is a hole or beyond the level), from u [D][n] as
        macros() returns it (read here when not given)."""
        if u is None:
            u = self.macros(l)[1]
        u = u.to(self.device, torch.float64).contiguous()
        assert u.shape == (self.D, self.n_dense(l))
        out = self._out((self.n_dense(l),))
        self._sync_torch()
        _lib.check(self.lib.dclbm_velocity_divergence(self.h, l, C.c_void_p(u.data_ptr()),
                                                      C.c_void_p(out.data_ptr())))
        self.stream.synchronize()
        return out

    def shared(self, l) -> torch.Tensor:
        out = self._out((4, self.n_dense(l)))
        _lib.check(self.lib.dclbm_read_shared(self.h, l, C.c_void_p(out.data_ptr())))
        self.stream.synchronize()
        return out

    def probes(self) -> torch.Tensor:
        n = C.c_int64()
        _lib.check(self.lib.dclbm_read_probes(self.h, None, C.byref(n)))
        np_ = len(self.wl.probes)
        out = self._out((max(1, n.value), max(1, np_)))
        _lib.check(self.lib.dclbm_read_probes(self.h, C.c_void_p(out.data_ptr()), C.byref(n)))
        return out[:n.value, :np_]

    def set_probe_window(self, start: int, stop: int) -> None:
        """Running FP64 sums of p' and p'^2 over coarse steps [start, stop)
        from the steps enqueued after this call (dclbm_set_probe_window)."""
        _lib.check(self.lib.dclbm_set_probe_window(self.h, int(start), int(stop)))

    def probe_sums(self):
        """(sums [3][n_probes] FP64: sum (p' - K), sum (p' - K)^2, K the
        window's first sample; steps summed)."""
        n = C.c_int64()
        out = self._out((3, max(1, len(self.wl.probes))))
        _lib.check(self.lib.dclbm_read_probe_sums(self.h, C.c_void_p(out.data_ptr()), C.byref(n)))
        return out[:, :len(self.wl.probes)], n.value

    def balance(self):
        out = (C.c_double * 5)()
        _lib.check(self.lib.dclbm_balance(self.h, out))
        return list(out)

    # ---------------------------------------------------------------- checkpoints
    def checkpoint_bytes(self) -> int:
        n = C.c_size_t()
        _lib.check(self.lib.dclbm_checkpoint_bytes(self.h, C.byref(n)))
        return n.value

    def save(self) -> torch.Tensor:
        """Checkpoint of the current state as a uint8 device tensor."""
        n = self.checkpoint_bytes()
        raw = torch.empty(n + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        blob = raw[off:off + n]
        self._sync_torch()
        _lib.check(self.lib.dclbm_save(self.h, C.c_void_p(blob.data_ptr()), n))
        return blob

    def load(self, blob: torch.Tensor):
        """Restore a checkpoint written by save() for the same configuration
        (here or by another Simulation); a host tensor is copied over."""
        assert blob.dtype == torch.uint8 and blob.dim() == 1
        if blob.device != self.device or blob.data_ptr() % 256 or not blob.is_contiguous():
            raw = torch.empty(blob.numel() + 256, dtype=torch.uint8, device=self.device)
            off = (-raw.data_ptr()) % 256
            aligned = raw[off:off + blob.numel()]
            aligned.copy_(blob)
            blob = aligned
        self._sync_torch()
        _lib.check(self.lib.dclbm_load(self.h, C.c_void_p(blob.data_ptr()), blob.numel()))

    def set_split(self, mode: int):
        """3-D FP16 launch layout (dclbm_set_split): -1 by weight, 0 one
        launch, 1 bulk and segments as two kernels side by side."""
        _lib.check(self.lib.dclbm_set_split(self.h, int(mode)))

    def set_timing(self, on: bool):
        _lib.check(self.lib.dclbm_set_timing(self.h, 1 if on else 0))

    def interface_bytes(self, l) -> float:
        b = C.c_double()
        _lib.check(self.lib.dclbm_interface_bytes(self.h, l, C.byref(b)))
        return b.value

    def bulk_time(self, l):
        ms, n, nodes = C.c_double(), C.c_int64(), C.c_int64()
        _lib.check(self.lib.dclbm_bulk_time(self.h, l, C.byref(ms), C.byref(n), C.byref(nodes)))
        return ms.value, n.value, nodes.value


def lattice_table(lattice: str):
    lib = _lib.load()
    q = C.c_int32()
    xi = (C.c_int32 * 57)()
    w = (C.c_double * 19)()
    _lib.check(lib.dclbm_lattice_table(_lib.LATTICE[lattice], C.byref(q), xi, w))
    Q = q.value
    return [tuple(xi[3 * i:3 * i + 3]) for i in range(Q)], [w[i] for i in range(Q)]


def copy_calibration(nbytes: int = 512 << 20, repeats: int = 20, device="cuda:0", stream=None):
    """GB/s (read + write) of the library's plain 16-byte copy kernel."""
    lib = _lib.load()
    st = stream if stream is not None else torch.cuda.Stream(device=device)
    a = torch.empty(nbytes, dtype=torch.uint8, device=device)
    b = torch.empty(nbytes, dtype=torch.uint8, device=device)
    a.zero_()
    torch.cuda.synchronize(device)
    ms = C.c_double()
    _lib.check(lib.dclbm_copy_calibration(C.c_void_p(b.data_ptr()), C.c_void_p(a.data_ptr()), nbytes,
                                          C.c_void_p(st.cuda_stream), repeats, C.byref(ms)))
    return 2.0 * nbytes / (ms.value * 1e-3) / 1e9, ms.value
