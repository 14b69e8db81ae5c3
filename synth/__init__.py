"""Seeded synthetic inputs for sketched GMRES.

This package holds only input generators: sparse test operators in CSR form and
right-hand sides.  It performs none of the solver's arithmetic, so both the CPU
oracle and the HIP path may take their inputs from it.
"""

from .problems import (  # noqa: F401
    CSR,
    convection_diffusion,
    random_dominant,
    rhs,
    batched_random_systems,
    batch_workload,
    block_rhs_workload,
    diagonal,
    WORKLOADS,
    workload,
)
