"""Pins of the oracle's Arnoldi estimator (Section 4, Algorithms 3 and 4)
against what the mathematics fixes.

C = T (A - tau I) with an unfactored HPD T is similar to
T^(1/2) (A - tau I) T^(1/2), so it has the inertia of A - tau I (eq. negi_T),
real eigenvalues, and h(C) is the spectral projector on its negative
eigenvalues.  The Arnoldi quadrature |v|^2 e_1^T h(H_k) e_1 (eq.
arnoldi_quad) is therefore checked against: the exact count for a full
Krylov space, the Lanczos estimator when T = I (C symmetric), the matrix sign
function of H_k computed by an independent library routine, the ideal
preconditioner (two steps), and the moments v^T C^p v, p <= k.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_1602_02306_amd import workloads as W


def small_problem(dims=(4, 4, 4), seed=3):
    wl = W.Workload("t", dims, "wells", seed, -5.0, 1.0, "none", 4, 4)
    return W.make_problem(wl)


def t_spec(kind, dims):
    if kind == "cheb":
        return W.cheb_inverse_prec(dims, degree=8)
    return W.PrecSpec(kind, ())


def dense_T(A, spec, tau):
    """T as a dense matrix, built here from its definition."""
    n = A.n
    if spec.kind == "none":
        return np.eye(n)
    if spec.kind == "jacobi":
        return np.diag(1.0 / np.abs(np.diag(A.to_dense()) - tau))
    L = W.laplacian_csr(spec.dims).to_dense()
    B = (2.0 * (L + spec.s * np.eye(n)) - (spec.lo + spec.hi) * np.eye(n)) / (spec.hi - spec.lo)
    Tj_1, Tj = np.eye(n), B
    out = spec.coef[0] * Tj_1 + spec.coef[1] * Tj
    for j in range(2, len(spec.coef)):
        Tj_1, Tj = Tj, 2.0 * B @ Tj - Tj_1
        out += spec.coef[j] * Tj
    return out


def mid_gaps(lam, i):
    lam = np.sort(lam)
    return 0.5 * (lam[i] + lam[i + 1])


@pytest.mark.parametrize("kind", ["none", "jacobi", "cheb"])
def test_full_krylov_exact_count(kind):
    """k = n with Hadamard probes: every quadrature is exact and the average is
    tr h(C) = n_(A - tau I)."""
    dims = (4, 4, 4)
    P = small_problem(dims)
    n = P.A.n
    lam = np.linalg.eigvalsh(P.A.to_dense())
    xi, eta = mid_gaps(lam, 5), mid_gaps(lam, 40)
    r = oracle.count_arnoldi(P.A, t_spec(kind, dims), xi, eta, W.hadamard_probes(n), n)
    assert abs(r.neg_xi - 6.0) < 1e-8 and abs(r.neg_eta - 41.0) < 1e-8
    assert abs(r.estimate - 35.0) < 1e-8


def test_identity_preconditioner_is_lanczos():
    """T = I: C = A - tau I is symmetric, Arnoldi reduces to Lanczos with full
    reorthogonalization, and eq. arnoldi_quad to eq. gauss_quad probe by probe."""
    dims = (5, 4, 3)
    P = small_problem(dims, seed=4)
    n = P.A.n
    lam = np.linalg.eigvalsh(P.A.to_dense())
    xi, eta = mid_gaps(lam, 9), mid_gaps(lam, 30)
    V = W.rademacher(n, 9, 2)
    ra = oracle.count_arnoldi(P.A, W.PrecSpec("none", ()), xi, eta, V, 12)
    rl = oracle.count(P.A, W.PrecSpec("none", ()), xi, eta, V, 12)
    assert np.max(np.abs(ra.s_xi - rl.s_xi)) <= 1e-8 * n
    assert np.max(np.abs(ra.s_eta - rl.s_eta)) <= 1e-8 * n
    # H is tridiagonal up to rounding
    H = ra.lan_xi.H
    for j in range(H.shape[0]):
        upper = np.triu(H[j, :12, :12], 2)
        assert np.max(np.abs(upper)) <= 1e-10 * np.max(np.abs(H[j]))


def test_quadrature_is_the_spectral_projector():
    """e_1^T h(H) e_1 = (1 - sign(H)_11)/2 for any H without eigenvalues on the
    imaginary axis, complex pairs included (scipy's matrix sign function)."""
    rng = np.random.default_rng(7)
    for trial in range(20):
        k = int(rng.integers(2, 12))
        H = np.triu(rng.standard_normal((k, k)), -1)   # upper Hessenberg
        H[np.arange(1, k), np.arange(k - 1)] = np.abs(H[np.arange(1, k), np.arange(k - 1)]) + 0.1
        theta = np.linalg.eigvals(H)
        if np.min(np.abs(theta.real)) < 1e-2:
            continue
        Hx = np.zeros((k + 1, k))
        Hx[:k] = H
        s, mins = oracle.arnoldi_quadrature(Hx, k, 3.0)
        ref = 3.0 * 0.5 * (1.0 - scipy.linalg.signm(H)[0, 0].real)
        assert abs(s - ref) <= 1e-9 * (1.0 + abs(ref)), (trial, s, ref)
        assert abs(mins - np.min(np.abs(theta.real))) < 1e-12


def test_ideal_preconditioner_two_steps():
    """Diagonal A with T = |A - tau I|^(-1): C = sign(A - tau I) has
    eigenvalues -1 and +1, the Krylov space is invariant after 2 steps, and
    the quadrature counts the negative entries exactly for +-1 probes."""
    rng = np.random.default_rng(5)
    d = rng.uniform(-3.0, 3.0, 200)
    A = W.CSR(200, np.arange(201, dtype=np.int32), np.arange(200, dtype=np.int32), d)
    V = W.rademacher(200, 7, 11)
    tau = 0.25
    res = oracle.arnoldi(A, W.PrecSpec("jacobi", ()), tau, V, 5)
    assert np.all(res.k_used <= 2)
    for j in range(7):
        s, _ = oracle.arnoldi_quadrature(res.H[j], res.k_used[j], res.nu[j])
        assert abs(s - np.sum(d < tau)) < 1e-9


@pytest.mark.parametrize("kind", ["none", "jacobi", "cheb"])
def test_moments(kind):
    """Arnoldi quadrature is exact for polynomials of degree <= k:
    |v|^2 e_1^T H_k^p e_1 = v^T C^p v, C built here as dense T (A - tau I)."""
    dims = (4, 3, 5)
    P = small_problem(dims, seed=6)
    n = P.A.n
    tau = -1.3
    spec = t_spec(kind, dims)
    Cd = dense_T(P.A, spec, tau) @ (P.A.to_dense() - tau * np.eye(n))
    V = W.rademacher(n, 3, 9)
    k = 7
    res = oracle.arnoldi(P.A, spec, tau, V, k)
    for j in range(3):
        v = V[:, j]
        Hk = res.H[j, :k, :k]
        Cp_v, Hp = v.copy(), np.eye(k)
        for p in range(k + 1):
            lhs = res.nu[j] * Hp[0, 0]
            rhs = v @ Cp_v
            assert abs(lhs - rhs) <= 1e-9 * max(1.0, abs(rhs)), (kind, j, p, lhs, rhs)
            Cp_v = Cd @ Cp_v
            Hp = Hp @ Hk
        # Hessenberg below the first subdiagonal, positive subdiagonal
        assert np.all(res.H[j][np.tril_indices(k + 1, -2, k)] == 0.0)
        assert np.all(np.diag(res.H[j], -1) > 0.0)


def test_cheb_inverse_is_positive_on_the_spectrum():
    """The unfactored T of the 64^3 family is HPD: its series is positive on
    [1, 13], which holds the spectrum of L + I for every 3-D grid."""
    spec = W.cheb_inverse_prec((8, 8, 8))
    x = np.linspace(spec.lo, spec.hi, 20001)
    t = (2.0 * x - spec.lo - spec.hi) / (spec.hi - spec.lo)
    val = np.polynomial.chebyshev.chebval(t, spec.coef)
    assert np.min(val) > 0.05
    assert np.max(np.abs(val * x - 1.0)) < 0.02
