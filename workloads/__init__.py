"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package builds the linear systems (SPD matrices in CSR, right-hand
sides, manufactured solutions, coefficient fields) that the solver is run on.
It holds none of the solver's arithmetic: no PCG step, no precision control,
no preconditioner.  Every random draw goes through
``numpy.random.default_rng([workload, stream])`` so that both sides of a
parity test see bit-identical inputs.
"""

from .problems import (  # noqa: F401
    CSR,
    stencil_poisson2d,
    fv_diffusion,
    q1_anisotropic,
    q1_anisotropic_bounds,
    spectrum_matrix,
    dense_to_csr,
    paper_spectrum,
    poisson2d_system,
    blocky_diffusion3d_system,
    q1_system,
    batched_systems,
    adjoint_inputs,
)
