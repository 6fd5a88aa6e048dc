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


# ---------------------------------------------------------------------------
# Nested dissection: inertia of A - tau I for large 3D grids
# ---------------------------------------------------------------------------

def _inertia_from_sytrf(f: np.ndarray, ipiv: np.ndarray) -> int:
    """Number of negative eigenvalues of D from LAPACK's Bunch-Kaufman
    factorization (dsytrf, lower): a 1 x 1 block where ipiv > 0, a 2 x 2
    block at rows (i, i+1) where ipiv[i] = ipiv[i+1] < 0."""
    s = f.shape[0]
    neg = 0
    i = 0
    while i < s:
        if ipiv[i] > 0:
            neg += int(f[i, i] < 0.0)
            i += 1
        else:
            a, b, c = f[i, i], f[i + 1, i], f[i + 1, i + 1]
            det = a * c - b * b
            if det < 0.0:
                neg += 1                      # one eigenvalue of each sign
            elif det > 0.0:
                neg += 2 if a + c < 0.0 else 0
            else:
                raise RuntimeError("singular 2 x 2 pivot")
            i += 2
    return neg


def _eliminate(F: np.ndarray, s: int):
    """Eliminate the first s variables of the symmetric front F:
    F = [[F_SS, F_SB], [F_BS, F_BB]].  By Haynsworth's inertia additivity
    In(F) = In(F_SS) + In(F_BB - F_BS F_SS^{-1} F_SB); returns the negative
    inertia of F_SS (from a Bunch-Kaufman LDL^T, Sylvester's law) and the
    Schur complement on the remaining variables."""
    import scipy.linalg.lapack as lapack
    FSS = np.asfortranarray(F[:s, :s])
    if F.shape[0] == s:
        f, ipiv, info = lapack.dsytrf(FSS, lower=1)
        if info > 0:
            raise RuntimeError("singular pivot: tau is (numerically) an eigenvalue of a front")
        return _inertia_from_sytrf(f, ipiv), None
    FSB = np.asfortranarray(F[:s, s:])
    lw = max(int(lapack.dsysv_lwork(s, lower=1)[0]), s * 64)
    f, ipiv, X, info = lapack.dsysv(FSS, FSB, lower=1, lwork=lw,
                                    overwrite_a=True, overwrite_b=False)
    if info > 0:
        raise RuntimeError("singular pivot: tau is (numerically) an eigenvalue of a front")
    U = F[s:, s:] - F[:s, s:].T @ X
    return _inertia_from_sytrf(f, ipiv), U


def nd_negcount(dims, diag: np.ndarray, tau: float, leaf: int = 1024) -> int:
    """Negative inertia n_(A - tau I) of A = L + diag(V) on a 3D grid (L the
    Dirichlet 7-point Laplacian, diagonal 6, neighbours -1; row
    r = (x*d1 + y)*d2 + z; `diag` = V) by a multifrontal symmetric-indefinite
    LDL^T in nested-dissection order (Section 1 of the paper: eigenvalue
    counts from Sylvester's law of inertia).

    The grid box is split recursively by the middle plane of its longest
    axis; boxes of at most `leaf` points are eliminated whole.  Each node
    eliminates its separator (or its whole leaf box) from a dense front that
    holds those variables and their neighbours outside the box (points of
    ancestor separators); the front is A's entries among them plus the
    children's Schur complements.  Haynsworth additivity makes the count the
    sum of the negative pivots over all fronts."""
    d = tuple(int(t) for t in dims)
    if len(d) != 3:
        raise ValueError("3D grids only")
    n = d[0] * d[1] * d[2]
    diag = np.asarray(diag, dtype=np.float64).reshape(n)
    loc = np.full(n, -1, dtype=np.int64)     # global row -> position in the current front

    def rows_of(lo, hi):
        xs, ys, zs = (np.arange(lo[a], hi[a]) for a in range(3))
        return ((xs[:, None, None] * d[1] + ys[None, :, None]) * d[2] + zs[None, None, :]).reshape(-1)

    def boundary(lo, hi):
        """Face neighbours of the box that lie in the grid but outside it."""
        parts = []
        for a in range(3):
            for plane in (lo[a] - 1, hi[a]):
                if 0 <= plane < d[a]:
                    l2, h2 = list(lo), list(hi)
                    l2[a], h2[a] = plane, plane + 1
                    parts.append(rows_of(l2, h2))
        return np.unique(np.concatenate(parts)) if parts else np.zeros(0, dtype=np.int64)

    def coords(r):
        return r // (d[1] * d[2]), (r // d[2]) % d[1], r % d[2]

    def front(S, B, updates):
        """Dense front on S (eliminated) then B, from A's entries that touch S
        and the children's Schur complements."""
        idx = np.concatenate([S, B])
        f = len(idx)
        F = np.zeros((f, f))
        loc[idx] = np.arange(f)
        pS = np.arange(len(S))
        F[pS, pS] = 6.0 + diag[S] - tau
        x, y, z = coords(S)
        for a, c in enumerate((x, y, z)):
            for step in (-1, 1):
                ok = (c + step >= 0) & (c + step < d[a])
                q = S[ok] + step * (d[1] * d[2], d[2], 1)[a]
                pq = loc[q]
                keep = pq >= 0
                F[pS[ok][keep], pq[keep]] = -1.0
                F[pq[keep], pS[ok][keep]] = -1.0
        for Bc, Uc in updates:
            pc = loc[Bc]
            F[np.ix_(pc, pc)] += Uc
        loc[idx] = -1
        return F

    def solve(lo, hi):
        """Eliminate every point of the box; returns (negatives, boundary rows,
        Schur complement on them)."""
        size = [hi[a] - lo[a] for a in range(3)]
        B = boundary(lo, hi)
        if size[0] * size[1] * size[2] <= leaf:
            S = rows_of(lo, hi)
            updates = []
            neg = 0
        else:
            a = int(np.argmax(size))
            mid = lo[a] + size[a] // 2
            l1, h1 = list(lo), list(hi)
            h1[a] = mid
            l2, h2 = list(lo), list(hi)
            l2[a] = mid + 1
            ls, hs = list(lo), list(hi)
            ls[a], hs[a] = mid, mid + 1
            S = rows_of(ls, hs)
            updates = []
            neg = 0
            for cl, ch in ((l1, h1), (l2, h2)):
                if all(ch[t] > cl[t] for t in range(3)):
                    c_neg, c_B, c_U = solve(cl, ch)
                    neg += c_neg
                    updates.append((c_B, c_U))
        F = front(S, B, updates)
        del updates
        f_neg, U = _eliminate(F, len(S))
        return neg + f_neg, B, U

    neg, _, _ = solve([0, 0, 0], list(d))
    return neg
