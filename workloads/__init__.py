"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and the benchmark.

This package holds no step of the solver: it only builds CSR matrices, right-hand sides and request
streams from fixed seeds, so that the CPU oracle and the HIP library see byte-identical inputs.
"""
from .stencils import (  # noqa: F401
    CSR,
    poisson2d,
    poisson3d,
    varcoef3d,
    convdiff3d,
    permute_symmetric,
    rcm_permutation,
    tridiag1d,
    config_system,
    serve_stream,
    random_csr,
)
