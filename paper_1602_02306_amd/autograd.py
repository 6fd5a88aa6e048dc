"""torch.autograd.Function for the erf-smoothed eigenvalue count.

    count = SmoothCount.apply(V, xi, eta, problem)

V: the diagonal potential (CUDA float64, n), xi / eta: 0-dim float64
tensors, problem: a SmoothProblem (the Laplacian part of A on the device,
the preconditioner, the probe block, k, the smoothing width and the
checkpoint mode).  A = L + diag(V) is assembled on the device (a scatter of V
into the diagonal entries of L's CSR values); forward and backward are the
library's ecnt_smooth_fwd / ecnt_smooth_bwd.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import ecount as ec


@dataclass
class SmoothProblem:
    L: ec.DeviceCSR          # A without the potential (values of L; diagonal entries present)
    diag_pos: torch.Tensor   # int64 positions of the diagonal entries in L's CSR arrays
    prec: object             # workloads.PrecSpec (Laplacian polynomial)
    probes: torch.Tensor     # n x m, float64, device
    k: int
    smooth_w: float = 0.05
    ckpt: str = "keep"       # 'keep' the basis between forward and backward, or 'recompute'

    @staticmethod
    def from_host(L_csr, prec, probes_np, k, smooth_w=0.05, ckpt="keep", device="cuda"):
        rows = np.repeat(np.arange(L_csr.n), np.diff(L_csr.row_ptr))
        pos = np.nonzero(L_csr.col_idx == rows)[0]
        if len(pos) != L_csr.n:
            raise ValueError("every diagonal entry of L must be stored")
        return SmoothProblem(ec.upload_csr(L_csr, device=device),
                             torch.from_numpy(pos.astype(np.int64)).to(device), prec,
                             torch.from_numpy(np.ascontiguousarray(probes_np)).to(device, torch.float64),
                             int(k), float(smooth_w), ckpt)

    def assemble(self, V: torch.Tensor) -> ec.DeviceCSR:
        val = self.L.val.clone()
        val.index_add_(0, self.diag_pos, V.detach().to(val.dtype))
        return ec.DeviceCSR(self.L.n, self.L.nnz, self.L.row_ptr, self.L.col_idx, val)


class SmoothCount(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V, xi, eta, problem: SmoothProblem):
        A = problem.assemble(V)
        res, ws = ec.smooth_forward(A, problem.prec, float(xi), float(eta), problem.probes,
                                    problem.k, problem.smooth_w)
        ctx.problem = problem
        ctx.A = A
        ctx.shifts = (float(xi), float(eta))
        ctx.ws = ws if problem.ckpt == "keep" else None
        return torch.tensor(res.estimate, dtype=torch.float64, device=V.device)

    @staticmethod
    def backward(ctx, g):
        pb = ctx.problem
        xi, eta = ctx.shifts
        dV, dxi, deta = ec.smooth_backward(ctx.A, pb.prec, xi, eta, pb.probes, pb.k, pb.smooth_w,
                                           g_est=float(g), ckpt=pb.ckpt, workspace=ctx.ws)
        ctx.ws = None
        dev = dV.device
        return (dV, torch.tensor(dxi, dtype=torch.float64, device=dev),
                torch.tensor(deta, dtype=torch.float64, device=dev), None)
