"""ctypes wrapper of the C oracle (dclbm_oracle.c).

TEST INFRASTRUCTURE ONLY (see the package docstring).  The C file is the
oracle; this file only moves arrays in and out.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dclbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_libs = {}

LATTICES = {"D2Q9": 0, "D3Q19": 1}

# The checking build: -O2, no FMA contraction, so the C expression order is
# the arithmetic order.
CHECK_FLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]
# The CPU-baseline build (timed beside the GPU on the host that runs it):
# -O3 for that host's own instruction set, OpenMP over the node loops.  Still
# no FMA contraction and no fast math, so every node's arithmetic, and hence
# every result, is the same as the checking build's.
BASELINE_FLAGS = ["-O3", "-march=native", "-fopenmp", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                  "-fno-fast-math"]


def build_oracle(force: bool = True, path: str = _LIB, flags=None) -> str:
    """Compile the oracle with gcc into `path` (default: the checking build)."""
    if force or not os.path.exists(path):
        tmp = path + ".tmp"
        cmd = ["gcc", *(flags or CHECK_FLAGS), "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, path)
    return path


def build_baseline(directory: str) -> str:
    """The CPU-baseline build of the same source, for the host it runs on."""
    return build_oracle(True, os.path.join(directory, "liboracle_baseline.so"), BASELINE_FLAGS)


def load_library(path: str = None):
    path = path or _LIB
    with _lock:
        if path not in _libs:
            if path == _LIB and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
                build_oracle(force=True)
            lib = C.CDLL(path)
            P = C.c_void_p
            dp = C.POINTER(C.c_double)
            ip = C.POINTER(C.c_int)
            lib.orc_create.restype = P
            lib.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, ip, C.c_int, ip, C.c_double,
                                       C.c_int, ip, C.c_longlong, C.c_char_p, C.c_int]
            lib.orc_destroy.argtypes = [P]
            lib.orc_level_dims.argtypes = [P, C.c_int, ip]
            lib.orc_level_tau.argtypes = [P, C.c_int, dp]
            lib.orc_classes.argtypes = [P, C.c_int, C.POINTER(C.c_ubyte)]
            lib.orc_set_newton.argtypes = [P, C.c_double, C.c_int]
            lib.orc_plant_R.argtypes = [P, C.c_double]
            lib.orc_set_collision.argtypes = [P, C.c_int, C.c_double, C.c_int]
            lib.orc_set_sponge.argtypes = [P, C.c_int, C.c_double, dp]
            lib.orc_set_region.argtypes = [P, C.POINTER(C.c_ubyte)]
            lib.orc_hrr_gradients.argtypes = [P, C.c_int, C.c_int, dp]
            lib.orc_init.argtypes = [P, C.c_int, dp, dp]
            lib.orc_run.argtypes = [P, C.c_longlong]
            for name in ("orc_get_f", "orc_get_pre", "orc_get_x", "orc_set_f"):
                getattr(lib, name).argtypes = [P, C.c_int, dp]
            lib.orc_get_probes.restype = C.c_longlong
            lib.orc_get_probes.argtypes = [P, dp]
            lib.orc_balance.argtypes = [P, dp]
            lib.orc_newton_stats.argtypes = [P, C.POINTER(C.c_longlong), ip, C.POINTER(C.c_longlong)]
            lib.orc_threads.restype = C.c_int
            lib.orc_threads.argtypes = []
            lib.orc_set_threads.argtypes = [C.c_int]
            lib.orc_lattice.argtypes = [C.c_int, ip, ip, ip, dp]
            lib.orc_feq.argtypes = [C.c_int, C.c_int, C.c_double, dp, dp]
            lib.orc_newton.argtypes = [C.c_int, C.c_int, dp, dp, C.c_double, C.c_int, dp, ip]
            lib.orc_residual.argtypes = [C.c_int, C.c_int, dp, dp, dp, dp]
            lib.orc_sets.argtypes = [C.c_int, C.c_uint, C.c_uint, C.c_int, C.POINTER(C.c_uint)]
            lib.orc_node_masks.argtypes = [P, C.c_int, ip, C.POINTER(C.c_uint), C.POINTER(C.c_uint)]
            lib.orc_line_stencil.argtypes = [C.c_int, C.c_int, ip, dp]
            lib.orc_time_interp.restype = C.c_double
            lib.orc_time_interp.argtypes = [C.c_longlong, C.c_int, C.c_double, C.c_double, C.c_double]
            _libs[path] = lib
    return _libs[path]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def lattice_table(lattice: str):
    lib = load_library()
    Q, D = C.c_int(), C.c_int()
    xi = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    lib.orc_lattice(LATTICES[lattice], C.byref(Q), C.byref(D), _ip(xi), _dp(w))
    return xi[:Q.value].copy(), w[:Q.value].copy()


def feq(lattice: str, rho: float, u, eq_order: int = 2) -> np.ndarray:
    lib = load_library()
    uu = np.zeros(3)
    uu[:len(u)] = u
    out = np.zeros(19)
    lib.orc_feq(LATTICES[lattice], eq_order, float(rho), _dp(uu), _dp(out))
    return out[:(9 if lattice == "D2Q9" else 19)].copy()


def newton(lattice: str, h, G, eq_order: int = 2, tol: float = 1e-12, maxit: int = 20):
    """Solve F(X)=0 for one co-located node; returns (rc, X[D+1], iterations)."""
    lib = load_library()
    h = np.ascontiguousarray(h, np.float64)
    G = np.ascontiguousarray(G, np.float64)
    X = np.zeros(4)
    it = C.c_int()
    rc = lib.orc_newton(LATTICES[lattice], eq_order, _dp(h), _dp(G), tol, maxit, _dp(X), C.byref(it))
    D = 2 if lattice == "D2Q9" else 3
    return rc, X[:D + 1].copy(), it.value


def residual(lattice: str, h, G, X, eq_order: int = 2):
    lib = load_library()
    h = np.ascontiguousarray(h, np.float64)
    G = np.ascontiguousarray(G, np.float64)
    XX = np.zeros(4)
    XX[:len(X)] = X
    F = np.zeros(4)
    lib.orc_residual(LATTICES[lattice], eq_order, _dp(h), _dp(G), _dp(XX), _dp(F))
    D = 2 if lattice == "D2Q9" else 3
    return F[:D + 1].copy()


def _bits_to_set(m):
    return {i for i in range(19) if (m >> i) & 1}


def sets(lattice: str, Kf, Kc, coupling: int = 2):
    """Index sets from the known-direction sets; returns (rc, dict)."""
    lib = load_library()
    kf = sum(1 << i for i in Kf)
    kc = sum(1 << i for i in Kc)
    out = (C.c_uint * 6)()
    rc = lib.orc_sets(LATTICES[lattice], kf, kc, coupling, out)
    names = ["P", "Qf", "Qc", "Mf", "Mc", "gammaR"]
    return rc, {n: _bits_to_set(out[k]) for k, n in enumerate(names)}


def line_stencil(k: int, N: int):
    lib = load_library()
    pos = np.zeros(4, np.int32)
    w = np.zeros(4)
    lib.orc_line_stencil(k, N, _ip(pos), _dp(w))
    return pos, w


def time_interp(captures: int, substep: int, Hm: float, H0: float, Hp: float) -> float:
    return load_library().orc_time_interp(captures, substep, Hm, H0, Hp)


class Oracle:
    """One simulation held by the C oracle.

    boxes: list of ((lo...), (hi...)) per refined level, each in the parent
    level's node coordinates.  probes: list of level-0 node coordinates.
    """

    def __init__(self, lattice: str, n0, boxes=(), tau0: float = 0.55, coupling: int = 2,
                 eq_order: int = 2, probes=(), probe_capacity: int = 0, lib_path: str = None):
        self.lib = load_library(lib_path)
        self.lattice = lattice
        self.D = 2 if lattice == "D2Q9" else 3
        self.Q = 9 if lattice == "D2Q9" else 19
        n0a = np.zeros(3, np.int32)
        n0a[:self.D] = n0[:self.D]
        self.n_levels = 1 + len(boxes)
        b = np.zeros(max(1, 6 * len(boxes)), np.int32)
        for k, (lo, hi) in enumerate(boxes):
            b[6 * k:6 * k + self.D] = lo[:self.D]
            b[6 * k + 3:6 * k + 3 + self.D] = hi[:self.D]
        pr = np.zeros(max(1, 3 * len(probes)), np.int32)
        for k, p in enumerate(probes):
            pr[3 * k:3 * k + self.D] = p[:self.D]
        err = C.create_string_buffer(256)
        self.h = self.lib.orc_create(LATTICES[lattice], eq_order, coupling, _ip(n0a), self.n_levels,
                                     _ip(b), float(tau0), len(probes), _ip(pr), int(probe_capacity),
                                     err, 256)
        if not self.h:
            raise ValueError("oracle: " + err.value.decode())
        self.n_probes = len(probes)
        self.dims = []
        for l in range(self.n_levels):
            d = np.zeros(3, np.int32)
            self.lib.orc_level_dims(self.h, l, _ip(d))
            self.dims.append(tuple(int(x) for x in d))

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_destroy(h)
            self.h = None

    def n(self, l):
        d = self.dims[l]
        return d[0] * d[1] * d[2]

    def tau(self, l):
        t = C.c_double()
        self.lib.orc_level_tau(self.h, l, C.byref(t))
        return t.value

    def classes(self, l):
        out = np.zeros(self.n(l), np.uint8)
        self.lib.orc_classes(self.h, l, out.ctypes.data_as(C.POINTER(C.c_ubyte)))
        return out

    def set_newton(self, tol, maxit):
        self.lib.orc_set_newton(self.h, tol, maxit)

    def plant_R(self, R):
        self.lib.orc_plant_R(self.h, R)

    def set_collision(self, kind: str = "bgk", sigma: float = 0.98, psi: bool = True):
        """'bgk' or 'hrr' (Sec. 2, with the interface gradients of Sec. 3.3 on
        refined meshes); call before init."""
        if self.lib.orc_set_collision(self.h, {"bgk": 0, "hrr": 1}[kind], float(sigma), int(bool(psi))) != 0:
            raise ValueError("oracle: invalid collision setting (0 <= sigma <= 1)")

    def set_sponge(self, width: int, sigma_max: float, u_target=(0.0, 0.0, 0.0)):
        """Absorbing layer on level 0 (width cells at the periodic seam)."""
        u = np.zeros(3)
        u[:len(u_target)] = u_target
        if self.lib.orc_set_sponge(self.h, int(width), float(sigma_max), _dp(u)) != 0:
            raise ValueError("oracle: invalid absorbing layer")

    def set_region(self, mask):
        """Refined region of level 1 as a [ny, nx] mask of level-0 cells over
        its box (1 = refined)."""
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        r = self.lib.orc_set_region(self.h, m.ctypes.data_as(C.POINTER(C.c_ubyte)))
        if r != 0:
            raise ValueError("oracle: invalid refined region" + (" (interface sets)" if r == -2 else ""))

    def hrr_gradients(self, l, substep=2):
        """H-RR gradient tensors of level l from the current state:
        [2][3][3][n] (d_b u_a, then sum_g d_g Psi_abg; node index last)."""
        out = np.zeros((self.n(l), 2, 3, 3))
        if self.lib.orc_hrr_gradients(self.h, l, int(substep), _dp(out)) != 0:
            raise RuntimeError("oracle: H-RR gradients need collision 'hrr'")
        return np.moveaxis(out, 0, -1)

    def init(self, l, rho, u):
        rho = np.ascontiguousarray(rho, np.float64).reshape(-1)
        u = np.ascontiguousarray(u, np.float64).reshape(self.D, -1)
        assert rho.size == self.n(l) and u.shape[1] == self.n(l)
        if self.lib.orc_init(self.h, l, _dp(rho), _dp(u)) != 0:
            raise RuntimeError("oracle init failed")

    def run(self, n_steps):
        rc = self.lib.orc_run(self.h, int(n_steps))
        if rc != 0:
            raise RuntimeError("oracle: Newton did not converge")

    def f(self, l):
        out = np.zeros((self.Q, self.n(l)))
        self.lib.orc_get_f(self.h, l, _dp(out))
        return out

    def pre(self, l):
        out = np.zeros((self.Q, self.n(l)))
        self.lib.orc_get_pre(self.h, l, _dp(out))
        return out

    def X(self, l):
        out = np.zeros((4, self.n(l)))
        self.lib.orc_get_x(self.h, l, _dp(out))
        return out

    def set_f(self, l, f):
        f = np.ascontiguousarray(f, np.float64).reshape(self.Q, self.n(l))
        self.lib.orc_set_f(self.h, l, _dp(f))

    def probes(self):
        n = self.lib.orc_get_probes(self.h, None)
        out = np.zeros((max(n, 1), max(self.n_probes, 1)))
        self.lib.orc_get_probes(self.h, _dp(out))
        return out[:n, :self.n_probes].copy()

    def balance(self):
        out = np.zeros(5)
        self.lib.orc_balance(self.h, _dp(out))
        return out

    def threads(self):
        return int(self.lib.orc_threads())

    def set_threads(self, n: int):
        self.lib.orc_set_threads(int(n))

    def newton_stats(self):
        calls, mx = C.c_longlong(), C.c_int()
        hist = (C.c_longlong * 8)()
        self.lib.orc_newton_stats(self.h, C.byref(calls), C.byref(mx), hist)
        return calls.value, mx.value, list(hist)

    def node_masks(self, l, k):
        kk = np.zeros(3, np.int32)
        kk[:len(k)] = k
        kf, kc = C.c_uint(), C.c_uint()
        rc = self.lib.orc_node_masks(self.h, l, _ip(kk), C.byref(kf), C.byref(kc))
        if rc != 0:
            raise ValueError("not a co-located fine node")
        return _bits_to_set(kf.value), _bits_to_set(kc.value)


def oaspl(series, start: int, stop: int, c0: float = 347.3, cs2: float = 1.0 / 3.0):
    """Overall sound pressure level in dB re 2e-5 Pa of each column of a probe
    series of p' = c_s^2 (rho - 1) (lattice units, rho0 = 1 kg/m^3), over rows
    [start, stop): pressure in pascals c0^2 (rho - 1), its mean over the
    window removed, root mean square, 20 log10(p_rms / 2e-5)."""
    p = np.asarray(series, dtype=np.float64)[start:stop] * (c0 * c0 / cs2)
    p = p - p.mean(axis=0)
    return 20.0 * np.log10(np.sqrt((p * p).mean(axis=0)) / 2e-5)


def velocity_divergence(lattice: str, f, dims, periodic: bool):
    """Centred-difference velocity divergence of a level's populations
    f [Q, n] (x fastest over dims = (nx, ny, nz)): u = sum_i xi_i f_i / sum_i f_i,
    then sum over the D axes of (u_a(x + e_a) - u_a(x - e_a)) / 2.  Periodic
    levels wrap; otherwise nodes whose stencil leaves the level are NaN, and
    NaN populations (holes) propagate."""
    xi, _ = lattice_table(lattice)
    D = 2 if lattice == "D2Q9" else 3
    f = np.asarray(f, dtype=np.float64)
    rho = f.sum(axis=0)
    shape = (dims[2], dims[1], dims[0])
    div = np.zeros(shape)
    for a in range(D):
        u = ((xi[:, a].astype(np.float64) @ f) / rho).reshape(shape)
        ax = 2 - a
        if periodic:
            div += 0.5 * (np.roll(u, -1, axis=ax) - np.roll(u, 1, axis=ax))
        else:
            d = np.full(shape, np.nan)
            hi = [slice(None)] * 3
            lo = [slice(None)] * 3
            mid = [slice(None)] * 3
            hi[ax], lo[ax], mid[ax] = slice(2, None), slice(None, -2), slice(1, -1)
            d[tuple(mid)] = 0.5 * (u[tuple(hi)] - u[tuple(lo)])
            div += d
    return div.reshape(-1)
