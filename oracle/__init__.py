"""CPU FP64 oracle for the eigenvalue-count estimator.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.
"""
from .block import (BlockCountResult, BlockLanczosResult, block_count, block_lanczos,
                    block_negcount, block_quadrature, block_rule_matrix, block_tridiagonal)
from .oracle import (ArnoldiResult, CountResult, ILDLFactor, LanczosResult, abs_invsqrt_blocks,
                     arnoldi, arnoldi_quadrature, build, count, count_arnoldi, count_tangent,
                     dense_operator, dense_operator_ldl, ildl, lanczos_ldl,
                     divided_difference, host_threads, jacobi_matrix, lanczos, lanczos_tangent,
                     apply_operator, negcount, probe_quadrature, probe_quadrature_tangent, quadrature, step,
                     step_deriv)

__all__ = ["BlockCountResult", "BlockLanczosResult", "block_count", "block_lanczos",
           "block_negcount", "block_quadrature", "block_rule_matrix", "block_tridiagonal",
           "apply_operator", "ArnoldiResult", "CountResult", "ILDLFactor", "LanczosResult", "abs_invsqrt_blocks",
           "arnoldi", "arnoldi_quadrature", "build", "count", "count_arnoldi", "count_tangent",
           "dense_operator", "dense_operator_ldl", "ildl", "lanczos_ldl",
           "divided_difference", "host_threads", "jacobi_matrix", "lanczos", "lanczos_tangent",
           "negcount", "probe_quadrature", "probe_quadrature_tangent", "quadrature", "step",
           "step_deriv"]
