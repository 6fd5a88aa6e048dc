"""Exact eigenvalue counts (negative inertia) used to check the oracle.

TEST INFRASTRUCTURE ONLY.  The traditional way to count eigenvalues below a
shift is Sylvester's law of inertia applied to an LDL^T factorization of
A - tau I (Section 1 of the paper); for small matrices a dense symmetric
eigendecomposition gives the same count, and for the Dirichlet Laplacian the
spectrum is known in closed form.

All functions count #{lambda < tau}; a count on [xi, eta) is the difference.
"""
from __future__ import annotations

import numpy as np


def dense_negcount(A_dense: np.ndarray, tau: float) -> int:
    lam = np.linalg.eigvalsh(A_dense)
    return int(np.sum(lam < tau))


def laplacian_eigenvalues(dims, h: float | None = None) -> np.ndarray:
    """Closed-form spectrum of the Dirichlet Laplacian on a grid with `dims`
    interior points per axis (diagonal 2*ndim, neighbours -1):
    lambda = sum_a 4 sin^2(pi i_a / (2 (N_a + 1))), i_a = 1..N_a; multiplied by
    1/h^2 when a mesh width h is given."""
    lam = np.zeros(1)
    for N in dims:
        i = np.arange(1, N + 1, dtype=np.float64)
        l1 = 4.0 * np.sin(np.pi * i / (2.0 * (N + 1))) ** 2
        lam = (lam[:, None] + l1[None, :]).reshape(-1)
    if h is not None:
        lam = lam / (h * h)
    return lam


def laplacian_negcount(dims, tau: float, h: float | None = None) -> int:
    return int(np.sum(laplacian_eigenvalues(dims, h) < tau))


def sparse_negcount(A_csr, tau: float) -> int:
    """Negative inertia of A - tau I from a sparse symmetric factorization
    P (A - tau I) P^T = L D L^T (SuperLU with a fill-reducing symmetric
    ordering and diagonal pivots only; D = diag(U)).  By Sylvester's law the
    count of negative pivots equals the count of eigenvalues below tau."""
    import scipy.sparse as sp
    from scipy.sparse.linalg import splu
    n = A_csr.shape[0]
    M = (A_csr - tau * sp.identity(n, format="csr")).tocsc()
    lu = splu(M, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
              options=dict(SymmetricMode=True))
    if not np.array_equal(lu.perm_r, lu.perm_c):
        raise RuntimeError("factorization used off-diagonal pivots; inertia not available")
    d = lu.U.diagonal()
    if np.any(d == 0.0):
        raise RuntimeError("zero pivot: tau is (numerically) an eigenvalue")
    return int(np.sum(d < 0.0))


def planewise_negcount(dims, diag: np.ndarray, tau: float) -> int:
    """Negative inertia of A - tau I for A = L + diag(V) on a 3D grid
    (x slowest), by block Gaussian elimination over x-planes.  The plane
    blocks couple through -I, so the Schur complements are
    S_0 = D_0 - tau I, S_x = D_x - tau I - S_{x-1}^{-1}, and by the
    Haynsworth inertia additivity n_(A - tau I) = sum_x n_(S_x)."""
    d0, d1, d2 = dims
    p = d1 * d2
    # in-plane block of the 3D stencil: diagonal 6, in-plane neighbours -1
    T1 = 2.0 * np.eye(d2) - np.eye(d2, k=1) - np.eye(d2, k=-1)
    T0 = 2.0 * np.eye(d1) - np.eye(d1, k=1) - np.eye(d1, k=-1)
    Lp = np.kron(T0, np.eye(d2)) + np.kron(np.eye(d1), T1) + 2.0 * np.eye(p)
    count = 0
    Sinv = None
    diag = np.asarray(diag).reshape(d0, p)
    for x in range(d0):
        S = Lp + np.diag(diag[x]) - tau * np.eye(p)
        if Sinv is not None:
            S = S - Sinv
        lam, U = np.linalg.eigh(S)
        count += int(np.sum(lam < 0.0))
        Sinv = (U / lam) @ U.T
    return count
