"""Build the HIP library (gfx950) in-tree with hipcc.

Each translation unit is compiled to an object in parallel (engine_inst.hip
once per lattice / equilibrium-order / storage class, twelve in all), then
the objects are linked into libdclbm.so.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdclbm.so")
CSRC = os.path.join(HERE, "csrc")
# (source, object name, extra defines): the host code, the serving runtime,
# and engine_inst.hip once per (lattice, equilibrium order, storage form)
UNITS = [(os.path.join(CSRC, "dclbm.hip"), "dclbm", []), (os.path.join(CSRC, "server.hip"), "server", [])] + [
    (os.path.join(CSRC, "engine_inst.hip"), f"engine_d{d}{eq}_{p}",
     [f"-DDCLBM_DIM={d}", f"-DDCLBM_EQ={eq}", f"-DDCLBM_P={p}"])
    for d in (3, 2) for eq in (2, 3) for p in (1, 2, 0)]
SOURCES = sorted({u[0] for u in UNITS})
HEADERS = [os.path.join(CSRC, f) for f in ("kernels.hpp", "engine.hpp", "engine_impl.hpp", "lattice.hpp")] + \
    [os.path.join(ROOT, "include", "dclbm.h")]
OBJDIR = os.path.join(HERE, "_build")

FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         # packed FP32 instructions are kept out of generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-munsafe-fp-atomics", "-Wno-unused-result"]


def _compile(unit, verbose: bool) -> str:
    src, name, defs = unit
    obj = os.path.join(OBJDIR, name + ".o")
    cmd = ["hipcc", *FLAGS, *defs, "-I", os.path.join(ROOT, "include"), "-c", "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build_library(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(len(UNITS), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, verbose), UNITS))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
