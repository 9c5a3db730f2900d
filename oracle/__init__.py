"""FP64 CPU oracle of the direct-coupling LBM step (arXiv:2004.14887).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg.  The product library never imports it.
"""
from .oracle import Oracle, build_oracle, build_baseline, lattice_table, feq, newton, residual, sets, \
    line_stencil, time_interp, load_library, oaspl, velocity_divergence

__all__ = ["Oracle", "build_oracle", "build_baseline", "lattice_table", "feq", "newton", "residual", "sets",
           "line_stencil", "time_interp", "load_library", "oaspl", "velocity_divergence"]
