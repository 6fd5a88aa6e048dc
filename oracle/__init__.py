"""CPU FP64 oracle for the eigenvalue-count estimator.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.
"""
from .oracle import (CountResult, LanczosResult, build, count, dense_operator, host_threads,
                     jacobi_matrix, lanczos, negcount, probe_quadrature, quadrature, step)

__all__ = ["CountResult", "LanczosResult", "build", "count", "dense_operator", "host_threads",
           "jacobi_matrix", "lanczos", "negcount", "probe_quadrature", "quadrature", "step"]
