"""Plain FP64 CPU oracle for the staggered-leapfrog lattice evolution.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only code allowed to import this package.  The GPU
library never imports it and shares no code with it.

The arithmetic lives in ``oracle.c`` (plain loops, FP64, built with
``-O2 -ffp-contract=off``); this module builds and loads it and converts
between NumPy arrays and its C structs.
"""
from .oracle import (  # noqa: F401
    OracleParams,
    OracleState,
    Oracle,
    build,
    laplacian,
    grad_energy,
    mean_potential,
    potential_point,
    dpotential_point,
    solve_adot,
    philox4x64_10,
    grf_normals,
    grf_modes,
    grf_mode_parts,
    grf_field,
    grf_sites,
    grf_initial,
    spectrum,
    spectrum_bins,
)
