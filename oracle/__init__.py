"""CPU oracle for the EAM lattice MD hot path (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library.
Every function here is a thin ctypes wrapper over ``oracle.c`` (FP64, OpenMP),
which cites the passages of the paper it follows; ``oracle.mlp`` is the numpy
float64 reference of the surrogate networks' training arithmetic.
"""
from .oracle import (  # noqa: F401
    ANALYTIC, ANALYTIC_SF, MLP, MLP_PARAMS, TABLE, Potential, mlp_eval, acc_unit, build, eam, eam_sampled, hash_site,
    kinetic, lattice_coords, lattice_id, library_path, nearest_site_brute, neighbours,
    num_threads, place, rehash, run, site_position, spline_eval, spline_slopes, stencil, wigner_seitz,
)
