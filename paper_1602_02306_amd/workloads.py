"""Seeded synthetic inputs for the eigenvalue-count estimator.

This module only *builds inputs*: sparse matrices, potentials, random probe
vectors and the coefficients that define the preconditioner M.  It holds none
of the estimator's arithmetic (no operator application, no Lanczos, no
quadrature), so that the GPU library and the CPU oracle can both be fed from
it without sharing any computational code.

Problem family (stands in for the paper's DFT Hamiltonians, Section 7, whose
matrices are not available): A = L + diag(V), where L is the unscaled
Dirichlet finite-difference Laplacian on a regular grid (diagonal 2*ndim,
off-diagonal -1) and V is a local potential.

Grid ordering: a 3D point (x, y, z) of a grid with dims (d0, d1, d2) is row
r = (x*d1 + y)*d2 + z; a 2D point (x, y) is r = x*d1 + y.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Sequence

import numpy as np

# ---------------------------------------------------------------------------
# Sparse matrices
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class CSR:
    """Symmetric sparse matrix in CSR form (both triangles, sorted columns,
    diagonal always stored).  int32 indices, float64 values."""
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        d[rows, self.col_idx] = self.val
        return d

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.n))


def grid_strides(dims: Sequence[int]) -> list[int]:
    strides = [1] * len(dims)
    for a in range(len(dims) - 2, -1, -1):
        strides[a] = strides[a + 1] * dims[a + 1]
    return strides


def laplacian_csr(dims: Sequence[int], diag_extra: np.ndarray | None = None) -> CSR:
    """Dirichlet Laplacian on a grid of shape `dims` (1 to 3 axes) plus an
    optional diagonal term.  Diagonal 2*ndim, neighbours -1; columns sorted."""
    dims = tuple(int(d) for d in dims)
    nd = len(dims)
    n = int(np.prod(dims))
    strides = grid_strides(dims)
    coords = np.unravel_index(np.arange(n, dtype=np.int64), dims)
    # offsets in ascending column order: -s0, -s1, ..., -1, 0, +1, ..., +s0
    offs = []
    for a in range(nd):
        offs.append((a, -1))
    offs.append((None, 0))
    for a in reversed(range(nd)):
        offs.append((a, +1))
    # reorder negative part so that strides descend (most negative first)
    neg = sorted([o for o in offs if o[1] == -1], key=lambda o: -strides[o[0]])
    pos = sorted([o for o in offs if o[1] == +1], key=lambda o: strides[o[0]])
    offs = neg + [(None, 0)] + pos
    ncol = len(offs)
    cols = np.empty((n, ncol), dtype=np.int64)
    vals = np.empty((n, ncol), dtype=np.float64)
    valid = np.empty((n, ncol), dtype=bool)
    rows = np.arange(n, dtype=np.int64)
    diag = np.full(n, 2.0 * nd)
    if diag_extra is not None:
        diag = diag + np.asarray(diag_extra, dtype=np.float64)
    for t, (a, sgn) in enumerate(offs):
        if a is None:
            cols[:, t] = rows
            vals[:, t] = diag
            valid[:, t] = True
        else:
            c = coords[a] + sgn
            valid[:, t] = (c >= 0) & (c < dims[a])
            cols[:, t] = rows + sgn * strides[a]
            vals[:, t] = -1.0
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = cols[valid].astype(np.int32)
    val = vals[valid]
    return CSR(n, row_ptr.astype(np.int32), col_idx, val)


# ---------------------------------------------------------------------------
# Potentials
# ---------------------------------------------------------------------------


def uniform_potential(n: int, seed: int) -> np.ndarray:
    """V_r ~ U[0, 1), drawn as numpy.random.default_rng(seed).random(n)."""
    return np.random.default_rng(seed).random(n)


def gaussian_wells(dims: Sequence[int], rng: np.random.Generator, nwells: int = 32,
                   sigma: float = 3.0, depth: tuple[float, float] = (5.0, 15.0)) -> np.ndarray:
    """Sum of attractive Gaussian wells on the grid:
    V(r) = -sum_w d_w exp(-|r - c_w|^2 / (2 sigma^2)), centres c_w uniform in
    the continuous box [0, d_a - 1] per axis, depths d_w ~ U[depth].  Draw
    order from `rng`: all centres (nwells x ndim), then all depths."""
    dims = tuple(int(d) for d in dims)
    nd = len(dims)
    centres = rng.uniform(0.0, 1.0, size=(nwells, nd)) * (np.array(dims, dtype=np.float64) - 1.0)
    depths = rng.uniform(depth[0], depth[1], size=nwells)
    axes = [np.arange(d, dtype=np.float64) for d in dims]
    V = np.zeros(dims, dtype=np.float64)
    inv = 1.0 / (2.0 * sigma * sigma)
    for w in range(nwells):
        # separable: exp(-sum_a (x_a - c_a)^2 * inv) = prod_a exp(-(x_a - c_a)^2 * inv)
        f = None
        for a in range(nd):
            g = np.exp(-((axes[a] - centres[w, a]) ** 2) * inv)
            shape = [1] * nd
            shape[a] = dims[a]
            g = g.reshape(shape)
            f = g if f is None else f * g
        V -= depths[w] * f
    return V.reshape(-1)


# ---------------------------------------------------------------------------
# Probe vectors (counter-based, so any entry can be regenerated anywhere)
# ---------------------------------------------------------------------------

_GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014)."""
    z = x.astype(np.uint64, copy=True)
    z ^= z >> np.uint64(30)
    z *= _MIX1
    z ^= z >> np.uint64(27)
    z *= _MIX2
    z ^= z >> np.uint64(31)
    return z


def rademacher(n: int, m: int, seed: int, dtype=np.float64, row_block: int = 1 << 16) -> np.ndarray:
    """n x m row-major block of +-1 probes.  Entry (r, j) is the sign of
    splitmix64(seed + (j*n + r + 1) * golden_gamma): +1 if its top bit is 0."""
    out = np.empty((n, m), dtype=dtype)
    j = np.arange(m, dtype=np.uint64)[None, :]
    seed_u = np.uint64(seed % (1 << 64))
    with np.errstate(over="ignore"):
        for r0 in range(0, n, row_block):
            r1 = min(n, r0 + row_block)
            r = np.arange(r0, r1, dtype=np.uint64)[:, None]
            ctr = (j * np.uint64(n) + r + np.uint64(1)) * _GOLDEN_GAMMA + seed_u
            z = splitmix64(ctr)
            out[r0:r1] = np.where((z >> np.uint64(63)) == 0, 1.0, -1.0).astype(dtype)
    return out


def rademacher_torch(n: int, m: int, seed: int, device="cuda", dtype=None, row_block: int = 1 << 15):
    """The same +-1 block as `rademacher`, generated with torch on `device`
    (SplitMix64 in wrapping int64 arithmetic; logical shifts emulated by
    masking).  Bitwise identical to the numpy version."""
    import torch
    dtype = dtype or torch.float64

    def as_i64(u: int) -> int:
        u &= (1 << 64) - 1
        return u - (1 << 64) if u >= 1 << 63 else u

    def lsr(x, sh):
        return (x >> sh) & ((1 << (64 - sh)) - 1)

    gamma, mix1, mix2 = as_i64(0x9E3779B97F4A7C15), as_i64(0xBF58476D1CE4E5B9), as_i64(0x94D049BB133111EB)
    out = torch.empty((n, m), dtype=dtype, device=device)
    j = torch.arange(m, dtype=torch.int64, device=device)[None, :]
    seed_i = as_i64(seed)
    for r0 in range(0, n, row_block):
        r1 = min(n, r0 + row_block)
        r = torch.arange(r0, r1, dtype=torch.int64, device=device)[:, None]
        z = (j * n + r + 1) * gamma + seed_i
        z = z ^ lsr(z, 30)
        z = z * mix1
        z = z ^ lsr(z, 27)
        z = z * mix2
        z = z ^ lsr(z, 31)
        out[r0:r1] = torch.where(z >= 0, 1.0, -1.0).to(dtype)
    return out


def identity_probes(n: int) -> np.ndarray:
    """sqrt(n) * I: n probes with sum_j v_j v_j^T = n I and |v_j|^2 = n."""
    return np.sqrt(float(n)) * np.eye(n)


def hadamard_probes(n: int) -> np.ndarray:
    """Columns of the Sylvester-Hadamard matrix of order n (a power of 2):
    +-1 entries, sum_j v_j v_j^T = n I."""
    if n < 1 or n & (n - 1):
        raise ValueError("n must be a power of two")
    H = np.ones((1, 1))
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    return H


# ---------------------------------------------------------------------------
# Preconditioner definitions (inputs of the method, T = M^* M)
# ---------------------------------------------------------------------------


def cheb_interp_coeffs(f, lo: float, hi: float, degree: int) -> np.ndarray:
    """Coefficients c_0..c_d of the degree-d Chebyshev interpolant of f at the
    d+1 first-kind Chebyshev points of [lo, hi]: p(x) = sum_j c_j T_j(t),
    t = (2x - lo - hi)/(hi - lo)."""
    d = int(degree)
    kk = np.arange(d + 1)
    theta = np.pi * (kk + 0.5) / (d + 1)
    x = 0.5 * (lo + hi) + 0.5 * (hi - lo) * np.cos(theta)
    fx = np.array([f(xi) for xi in x], dtype=np.float64)
    c = np.array([(2.0 / (d + 1)) * np.sum(fx * np.cos(j * theta)) for j in range(d + 1)])
    c[0] *= 0.5
    return c


@dataclasses.dataclass
class PrecSpec:
    """kind: 'none' (M = I), 'jacobi' (M_tau = |diag(A) - tau|^(-1/2), per shift),
    'cheb' (M = sum_j coef[j] T_j((2(L + s I) - (lo + hi) I)/(hi - lo)) with
    L the Dirichlet Laplacian of `dims`, shared by all shifts), or 'ildl'
    (M_tau = |D|^(-1/2) L^{-1} P from an ILDL(droptol) factorization of
    A - tau I, one per shift)."""
    kind: str
    dims: tuple = ()
    s: float = 0.0
    lo: float = 0.0
    hi: float = 0.0
    coef: np.ndarray | None = None
    droptol: float = 0.0

    @property
    def degree(self) -> int:
        return 0 if self.coef is None else len(self.coef) - 1


def cheb_invsqrt_prec(dims: Sequence[int], s: float = 1.0, degree: int = 4) -> PrecSpec:
    """M = c_d(L + sI): Chebyshev interpolant of x^(-1/2) on the Gershgorin
    interval [s, s + 4*ndim] of L + sI, so that T = M^2 approximates
    (L + sI)^(-1) and is SPD."""
    nd = len(dims)
    lo, hi = float(s), float(s + 4 * nd)
    coef = cheb_interp_coeffs(lambda x: x ** -0.5, lo, hi, degree)
    return PrecSpec("cheb", tuple(int(d) for d in dims), float(s), lo, hi, coef)


def cheb_inverse_prec(dims: Sequence[int], s: float = 1.0, degree: int = 8) -> PrecSpec:
    """T = c_d(L + sI): Chebyshev interpolant of 1/x on [s, s + 4*ndim], an
    unfactored HPD approximation of (L + sI)^(-1) (degree 8: positive on the
    interval, relative error 1.2% for s = 1 in 3-D)."""
    nd = len(dims)
    lo, hi = float(s), float(s + 4 * nd)
    coef = cheb_interp_coeffs(lambda x: 1.0 / x, lo, hi, degree)
    return PrecSpec("cheb", tuple(int(d) for d in dims), float(s), lo, hi, coef)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    dims: tuple
    potential: str          # 'uniform' | 'wells'
    seed: int               # potential seed
    xi: float
    eta: float
    prec: str               # 'none' | 'jacobi' | 'cheb' (M = c4 of x^-1/2) | 'cheb_inv' (T = c8 of 1/x)
    m: int
    k: int
    probe_seed: int = 12345
    vec: str = "f64"        # storage type of A values and Lanczos vectors
    smooth_w: float = 0.0   # width of the erf-smoothed step (0: the paper's step)
    method: str = "lanczos" # 'lanczos' (Algorithm 2 on M(A - tau I)M) | 'arnoldi' (Algorithm 4 on T(A - tau I))
                            # | 'block' (block Lanczos on blocks of 16 probes, block Gauss rule)
    scale: float = 1.0      # A = scale * L + diag(potential)
    droptol: float = 0.0    # ILDL drop tolerance (prec 'ildl')
    taus: tuple = ()        # non-empty: the workload is n_(A - tau I) at these shifts

    @property
    def n(self) -> int:
        return int(np.prod(self.dims))


WORKLOADS = {
    # 2D 30x30, V ~ U[0,1] seed 0, Jacobi, [0.5, 1.5], 40 probes, k = 20
    "c1": Workload("c1", (30, 30), "uniform", 0, 0.5, 1.5, "jacobi", 40, 20),
    # 3D 64^3 + 32 Gaussian wells (seed 1), Chebyshev M, [-8, -2], 256 probes, k = 30
    "c2": Workload("c2", (64, 64, 64), "wells", 1, -8.0, -2.0, "cheb", 256, 30),
    # 128^3, FP32 storage, 512 probes
    "c3": Workload("c3", (128, 128, 128), "wells", 1, -8.0, -2.0, "cheb", 512, 30, vec="f32"),
    # the 64^3 problem in the FP32 storage form (its exact count is known)
    "c2_f32": Workload("c2_f32", (64, 64, 64), "wells", 1, -8.0, -2.0, "cheb", 256, 30, vec="f32"),
    # the 64^3 problem with the unfactored T = c8(L+I) ~ (L+I)^-1 and the Arnoldi estimator
    "c2_arn": Workload("c2_arn", (64, 64, 64), "wells", 1, -8.0, -2.0, "cheb_inv", 256, 30,
                       method="arnoldi"),
    # the 64^3 problem of c2 in the block-Lanczos form (blocks of 16 probes)
    "c2_blk": Workload("c2_blk", (64, 64, 64), "wells", 1, -8.0, -2.0, "cheb", 256, 30,
                       method="block"),
    # 96^3, erf-smoothed count of width 0.05, 128 probes
    "c5": Workload("c5", (96, 96, 96), "wells", 1, -8.0, -2.0, "cheb", 128, 30, smooth_w=0.05),
    # small cases that the oracle finishes in seconds
    "c2_small": Workload("c2_small", (16, 16, 16), "wells", 1, -8.0, -2.0, "cheb", 24, 12),
    "c2_ragged": Workload("c2_ragged", (13, 11, 9), "wells", 7, -60.0, -30.0, "cheb", 37, 9),
    # Table 1 "Laplace": (1/h^2) x 5-point Laplacian, h = 2^-7, n_(A - 3000 I) = 226, m = 50,
    # ILDL(t) preconditioner; k = 6 Lanczos steps
    "t1": Workload("t1", (127, 127), "zero", 0, 0.0, 3000.0, "ildl", 50, 6, scale=16384.0,
                   droptol=1e-6, taus=(3000.0,)),
    # its small counterpart (h = 2^-5) for parity tests
    "t1_small": Workload("t1_small", (31, 31), "zero", 0, 0.0, 300.0, "ildl", 37, 8, scale=1024.0,
                         droptol=1e-3, taus=(300.0,)),
}


@dataclasses.dataclass
class Problem:
    A: CSR
    V: np.ndarray
    prec: PrecSpec
    xi: float
    eta: float
    dims: tuple


def make_potential(wl: Workload) -> np.ndarray:
    if wl.potential == "uniform":
        return uniform_potential(wl.n, wl.seed)
    if wl.potential == "wells":
        return gaussian_wells(wl.dims, np.random.default_rng(wl.seed))
    if wl.potential == "zero":
        return np.zeros(wl.n)
    raise ValueError(wl.potential)


def make_prec(kind: str, dims, droptol: float = 0.0) -> PrecSpec:
    if kind == "ildl":
        return PrecSpec("ildl", tuple(dims), droptol=float(droptol))
    if kind == "cheb":
        return cheb_invsqrt_prec(dims)
    if kind == "cheb_inv":
        return cheb_inverse_prec(dims)
    if kind in ("jacobi", "none"):
        return PrecSpec(kind, tuple(dims))
    raise ValueError(kind)


def make_problem(wl: Workload) -> Problem:
    V = make_potential(wl)
    if wl.scale == 1.0:
        A = laplacian_csr(wl.dims, V)
    else:
        A = laplacian_csr(wl.dims)
        A.val = A.val * wl.scale
        if np.any(V != 0.0):
            raise ValueError("a scaled Laplacian takes no potential")
    return Problem(A, V, make_prec(wl.prec, wl.dims, wl.droptol), wl.xi, wl.eta, tuple(wl.dims))


def make_probes(wl: Workload, dtype=np.float64) -> np.ndarray:
    return rademacher(wl.n, wl.m, wl.probe_seed, dtype=dtype)


# ---------------------------------------------------------------------------
# Batched family: many Hamiltonians of uneven size, 3 contiguous slices each
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class BatchItem:
    index: int
    dims: tuple
    V: np.ndarray
    A: CSR
    prec: PrecSpec
    shifts: np.ndarray      # 4 sorted endpoints -> 3 contiguous intervals


def block_diag_csr(mats: Sequence[CSR]) -> CSR:
    """The block-diagonal matrix diag(mats[0], mats[1], ...) in CSR form (rows
    and column indices of block b offset by the sizes of the blocks before
    it): how a batch of independent problems is handed over as one matrix."""
    n = sum(int(a.n) for a in mats)
    nnz = sum(a.nnz for a in mats)
    if n >= 2 ** 31 or nnz >= 2 ** 31:
        raise ValueError("block-diagonal matrix exceeds int32 indexing")
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col_idx = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    r = 0
    e = 0
    for a in mats:
        row_ptr[r + 1:r + a.n + 1] = e + a.row_ptr[1:].astype(np.int64)
        col_idx[e:e + a.nnz] = a.col_idx.astype(np.int64) + r
        val[e:e + a.nnz] = a.val
        r += int(a.n)
        e += a.nnz
    return CSR(n, row_ptr.astype(np.int32), col_idx, val)


def batched_item(b: int, nmin: int = 16, nmax: int = 64, base_seed: int = 1000,
                 lo: float = -8.0, hi: float = -2.0, nshift: int = 4) -> BatchItem:
    """Problem b of the batched family: rng = default_rng(base_seed + b); draw
    the grid edge N ~ U{nmin..nmax}, then `nshift` endpoints ~ U[lo, hi]
    (sorted), then the wells (centres, depths) on the N^3 grid."""
    rng = np.random.default_rng(base_seed + b)
    N = int(rng.integers(nmin, nmax + 1))
    shifts = np.sort(rng.uniform(lo, hi, size=nshift))
    dims = (N, N, N)
    V = gaussian_wells(dims, rng)
    return BatchItem(b, dims, V, laplacian_csr(dims, V), cheb_invsqrt_prec(dims), shifts)
