"""MI355X-native lattice Boltzmann step on nested-box refined meshes with the
cell-vertex direct grid coupling of Astoul et al. (arXiv:2004.14887).

The compute path is the HIP library libdclbm.so (C ABI in include/dclbm.h);
this package holds its ctypes binding, the Simulation wrapper (torch owns the
device memory and stream) and the seeded synthetic workloads.
"""
from . import workloads  # noqa: F401


def __getattr__(name):
    # the HIP-backed classes load the library lazily, so that importing the
    # package (e.g. for workloads) works on a machine without the built library
    if name in ("Simulation", "workspace_bytes", "make_config", "lattice_table"):
        from . import sim
        return getattr(sim, name)
    raise AttributeError(name)
