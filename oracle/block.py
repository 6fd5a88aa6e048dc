"""Oracle for the block-Lanczos form of the eigenvalue-count estimator.

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.

The paper runs one Lanczos process per probe (Section 3.1, Algorithm 1) and
averages the Gauss-rule quadratic forms v_j^T h(C) v_j (Section 3.2, eq.
rand_prec_quad, Algorithm 2).  This variant is not in the paper: the probes
are taken P at a time, V_b = [v_j ... v_{j+P-1}], and the block Lanczos
method (Golub and Underwood, 1977) builds one block-tridiagonal matrix per
block; the block Gauss rule (Golub and Meurant, "Matrices, Moments and
Quadrature with Applications", 2010, Chapter 7) then gives the P x P matrix

    V_b^T h(C) V_b  ~  R_0^T E_1^T h(T_k) E_1 R_0,

whose diagonal holds the per-probe estimates s_j and whose trace is their sum.
With P = 1 this is the paper's estimator.  The rule is exact for polynomials
of degree <= 2k - 1 (in place of h), and exact for h itself once the block
Krylov space is invariant.

Steps for one block (every line a plain numpy operation):
    V_b = Q_1 R_0                     (QR, diagonal of R_0 made positive)
    for i = 1..k:
        W   = C Q_i
        H_l = Q_l^T W,  l = 1..i      (one classical Gram-Schmidt pass
        W   = W - sum_l Q_l H_l        against the whole basis: two matrix
                                       products with [Q_1 .. Q_i])
        A_i = (H_i + H_i^T) / 2       (the diagonal block, symmetric part)
        W   = Q_{i+1} B_{i+1}         (QR, diagonal of B_{i+1} positive)
        stop with k_used = i when min diag(B_{i+1}) <= 1e3 eps rm, rm the
        largest |entry| of A_1..A_i and B_2..B_i   (invariant space)
    T_k: A_i on the diagonal, B_{i+1} below it and B_{i+1}^T above it
    theta, Y = eigh(T_k);  Z = Y[:P, :]
    S = R_0^T Z diag(h(theta)) Z^T R_0;   s_j = S[j, j]

The positive-diagonal QR is unique for a block of full column rank, so any
other way of orthonormalizing (for instance Cholesky QR) gives the same basis
up to rounding.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .oracle import _mean, apply_operator, step


@dataclass
class BlockLanczosResult:
    A: np.ndarray       # nblk x k x P x P, A_1..A_k of each block
    B: np.ndarray       # nblk x (k+1) x P x P, B[:, 0] = 0, B[:, i] = B_{i+1}
    R0: np.ndarray      # nblk x P x P
    k_used: np.ndarray  # nblk


def qr_pos(W: np.ndarray):
    """Thin QR with a non-negative diagonal of R (Householder QR, then signs;
    LAPACK takes the column-major copy without transposing it)."""
    Q, R = np.linalg.qr(np.asfortranarray(W))
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d, R * d[:, None]


def block_lanczos(A, prec, tau: float, V: np.ndarray, k: int, P: int = 16,
                  nthreads: int | None = None) -> BlockLanczosResult:
    """Block Lanczos with full reorthogonalization for every block of P
    consecutive columns of V (n x m, m a multiple of P)."""
    V = np.asarray(V, dtype=np.float64)
    n, m = V.shape
    if m % P:
        raise ValueError("the number of probes must be a multiple of the block size")
    nblk = m // P
    Ab = np.zeros((nblk, k, P, P))
    Bb = np.zeros((nblk, k + 1, P, P))
    R0s = np.zeros((nblk, P, P))
    kused = np.zeros(nblk, dtype=np.int32)
    eps = np.finfo(np.float64).eps
    for b in range(nblk):
        Q1, R0 = qr_pos(V[:, b * P:(b + 1) * P])
        R0s[b] = R0
        Q = np.zeros((n, (k + 1) * P))      # [Q_1 Q_2 ...], block l in columns (l-1)P..lP-1
        Q[:, :P] = Q1
        rm = 0.0
        kused[b] = k
        for i in range(1, k + 1):
            Qi = Q[:, :i * P]
            W = apply_operator(A, prec, tau, Q[:, (i - 1) * P:i * P], nthreads)
            H = Qi.T @ W                     # stacked H_1..H_i
            W = W - Qi @ H
            Hi = H[(i - 1) * P:i * P]
            Ai = 0.5 * (Hi + Hi.T)
            Qn, Bn = qr_pos(W)
            Ab[b, i - 1] = Ai
            Bb[b, i] = Bn
            rm = max(rm, float(np.max(np.abs(Ai))))
            if i > 1:
                rm = max(rm, float(np.max(np.abs(Bb[b, i - 1]))))
            if float(np.min(np.diag(Bn))) <= 1e3 * eps * rm:
                kused[b] = i
                break
            Q[:, i * P:(i + 1) * P] = Qn
    return BlockLanczosResult(Ab, Bb, R0s, kused)


def block_tridiagonal(Ab: np.ndarray, Bb: np.ndarray, k: int) -> np.ndarray:
    """Dense T_k of one block from A_1..A_k and B_2..B_k."""
    P = Ab.shape[-1]
    T = np.zeros((k * P, k * P))
    for i in range(k):
        T[i * P:(i + 1) * P, i * P:(i + 1) * P] = Ab[i]
        if i + 1 < k:
            T[(i + 1) * P:(i + 2) * P, i * P:(i + 1) * P] = Bb[i + 1]
            T[i * P:(i + 1) * P, (i + 1) * P:(i + 2) * P] = Bb[i + 1].T
    return T


def block_rule_matrix(res: BlockLanczosResult, b: int, smooth_w: float = 0.0):
    """(S, min |theta|): S = R_0^T E_1^T h(T_k) E_1 R_0 for block b."""
    P = res.R0.shape[-1]
    T = block_tridiagonal(res.A[b], res.B[b], int(res.k_used[b]))
    theta, Y = np.linalg.eigh(T)
    Z = Y[:P, :]
    F = (Z * step(theta, smooth_w)) @ Z.T
    R0 = res.R0[b]
    return R0.T @ F @ R0, float(np.min(np.abs(theta)))


def block_quadrature(res: BlockLanczosResult, smooth_w: float = 0.0):
    """Per-probe estimates s_j (diagonal of each block's S) and min |theta| per probe."""
    nblk, P = res.R0.shape[0], res.R0.shape[-1]
    s = np.zeros(nblk * P)
    mins = np.zeros(nblk * P)
    for b in range(nblk):
        S, mn = block_rule_matrix(res, b, smooth_w)
        s[b * P:(b + 1) * P] = np.diag(S)
        mins[b * P:(b + 1) * P] = mn
    return s, mins


def block_negcount(A, prec, tau, V, k, P=16, smooth_w=0.0, nthreads=None):
    """(1/m) sum_j s_j(tau) with the block rule, plus s, the Lanczos data, min |theta|."""
    res = block_lanczos(A, prec, tau, V, k, P, nthreads)
    s, mins = block_quadrature(res, smooth_w)
    return _mean(s), s, res, float(np.min(mins))


@dataclass
class BlockCountResult:
    estimate: float
    variance: float
    neg_xi: float
    neg_eta: float
    s_xi: np.ndarray
    s_eta: np.ndarray
    min_abs_ritz: float
    lan_xi: BlockLanczosResult
    lan_eta: BlockLanczosResult


def block_count(A, prec, xi, eta, V, k, P=16, smooth_w=0.0, nthreads=None) -> BlockCountResult:
    """Number of eigenvalues of A in [xi, eta) with the block rule, both shifts
    on the same probes; variance as in the single-vector form (sample
    variance of the per-probe differences over m)."""
    if not (xi < eta):
        raise ValueError("need xi < eta")
    _, s_xi, lx, mx = block_negcount(A, prec, xi, V, k, P, smooth_w, nthreads)
    _, s_eta, le, me = block_negcount(A, prec, eta, V, k, P, smooth_w, nthreads)
    m = len(s_xi)
    d = s_eta - s_xi
    est = _mean(d)
    if m > 1:
        acc = 0.0
        for v in d:
            acc += (float(v) - est) ** 2
        var = acc / ((m - 1) * m)
    else:
        var = float("nan")
    return BlockCountResult(est, var, _mean(s_xi), _mean(s_eta), s_xi, s_eta, min(mx, me), lx, le)
