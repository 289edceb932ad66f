"""Seeded synthetic workloads for the BCC EAM lattice MD path.

This package generates inputs only: lattice geometry in a plain (non-canonical)
atom order, seeded random displacements, velocities and recoil atoms, and
samples of the synthetic analytic potential.  It holds none of the method's
arithmetic (no lattice-id map, no neighbour stencil, no spline, no EAM sums,
no integrator), so both the CPU oracle and the GPU path can consume it.
"""
from .synth import (  # noqa: F401
    A_FE, RC, DELTA, MASS_FE, KB_EV, ACC_A_FS2, N_TABLE, RHO_MAX,
    CONFIGS, Config, BATCH_CONFIGS, BatchConfig, bcc_positions, thermal_state, add_recoils, make_state,
    make_batch,
    potential_samples, analytic_potential_params,
)
