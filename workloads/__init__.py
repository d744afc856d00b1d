"""Seeded synthetic inputs shared by the oracle-side tests and the HIP path.

This package holds no arithmetic of the group-shared-exponent method: it only
builds sparse matrices in FP64 CSR form, right-hand sides and request streams
from seeded random draws.  Both the CPU oracle and the GPU library consume
exactly these arrays, so neither depends on the other for its inputs.
"""
from .generators import (  # noqa: F401
    CSR,
    poisson2d,
    diffusion3d,
    layered3d,
    block_sample_rows,
    diffusion2d,
    convdiff2d,
    powerlaw,
    random_sparse,
    diagonal,
    fixed_rows,
    rhs_from_solution,
    serving_stream,
    serving_request_matrix,
    make_config,
    CONFIGS,
)
