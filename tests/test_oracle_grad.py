"""Pins of the oracle's derivative of the erf-smoothed count.

The smoothed estimator replaces h(theta) by S_w(theta) = erfc(theta/w)/2 at
the Ritz values (the paper notes that the rule only sees h at the Ritz
values, Section 3.3); its derivative with respect to the diagonal potential V
and the endpoints is computed by the oracle in forward mode (Algorithm 1
differentiated line by line, Daleckii-Krein for the tridiagonal step).  It is
pinned here by (i) central finite differences of the oracle's own estimate
and (ii) at k = n, where the Gauss rule is exact, the closed-form derivative
of v^T S_w(C) v from the eigendecomposition of the dense C.
"""
import numpy as np
import pytest

import oracle
from paper_1602_02306_amd import workloads as W

SW = 0.05


def problem(dims=(6, 6, 6), seed=1, xi=-160.0, eta=-120.0, m=6, k=8, prec="cheb"):
    wl = W.Workload("t", dims, "wells", seed, xi, eta, prec, m, k)
    return wl, W.make_problem(wl), W.make_probes(wl)


def smoothed(P, wl, V, V_pot, xi, eta, k):
    A = W.laplacian_csr(wl.dims, V_pot)
    return oracle.count(A, P.prec, xi, eta, V, k, smooth_w=SW).estimate


@pytest.mark.parametrize("prec", ["cheb", "none"])
def test_tangent_matches_finite_differences(prec):
    wl, P, V = problem(prec=prec)
    rng = np.random.default_rng(3)
    u = rng.standard_normal(P.A.n)
    _, d = oracle.count_tangent(P.A, P.prec, wl.xi, wl.eta, V, wl.k, u, 0.0, 0.0, SW)
    h = 1e-4
    fd = (smoothed(P, wl, V, P.V + h * u, wl.xi, wl.eta, wl.k)
          - smoothed(P, wl, V, P.V - h * u, wl.xi, wl.eta, wl.k)) / (2 * h)
    assert abs(fd - d) <= 1e-6 * abs(d) + 1e-8
    for dxi, deta in ((1.0, 0.0), (0.0, 1.0)):
        _, d = oracle.count_tangent(P.A, P.prec, wl.xi, wl.eta, V, wl.k, np.zeros(P.A.n), dxi, deta, SW)
        fd = (smoothed(P, wl, V, P.V, wl.xi + h * dxi, wl.eta + h * deta, wl.k)
              - smoothed(P, wl, V, P.V, wl.xi - h * dxi, wl.eta - h * deta, wl.k)) / (2 * h)
        assert abs(fd - d) <= 1e-6 * abs(d) + 1e-8  # FD rounding floor ~ eps*|f|/h


def test_tangent_closed_form_full_krylov():
    """k = n: s_j = v^T S_w(C) v exactly, and with C = M(A - tau I)M,
    d s_j = sum_{a,b} (u_a^T v)(u_b^T v) S[1](mu_a, mu_b) u_a^T dC u_b,
    dC = M diag(du) M - dtau M^2 ((mu, u) the eigenpairs of C)."""
    dims = (3, 3, 3)
    wl, P, V = problem(dims=dims, seed=2, m=3, k=27)
    lam = np.linalg.eigvalsh(P.A.to_dense())
    tau = 0.5 * (lam[10] + lam[11])
    n = P.A.n
    C = oracle.dense_operator(P.A, P.prec, tau)
    # M from the eigendecomposition of L (independent of the oracle's Clenshaw)
    L = W.laplacian_csr(dims).to_dense()
    ll, UL = np.linalg.eigh(L)
    t = (2 * (ll + P.prec.s) - (P.prec.lo + P.prec.hi)) / (P.prec.hi - P.prec.lo)
    M = (UL * np.polynomial.chebyshev.chebval(t, P.prec.coef)) @ UL.T
    mu, U = np.linalg.eigh(0.5 * (C + C.T))
    D = oracle.divided_difference(mu, SW)
    rng = np.random.default_rng(9)
    du = rng.standard_normal(n)
    for dtau in (0.0, 0.7):
        dC = M @ np.diag(du) @ M - dtau * (M @ M)
        T = oracle.lanczos_tangent(P.A, P.prec, tau, V, n, du, dtau)
        for j in range(V.shape[1]):
            assert T.lan.k_used[j] >= n - 1
            c = U.T @ V[:, j]
            exact = float(c @ (D * (U.T @ dC @ U)) @ c)
            s, ds = oracle.probe_quadrature_tangent(T.lan.alpha[j], T.lan.beta[j], T.dalpha[j],
                                                    T.dbeta[j], T.lan.k_used[j], T.lan.nu[j], SW)
            assert abs(s - float(c @ (oracle.step(mu, SW) * c))) <= 1e-9 * n
            assert abs(ds - exact) <= 1e-7 * max(1.0, abs(exact))


def test_divided_difference_limits():
    th = np.array([-0.1, -0.1 + 1e-12, 0.0, 0.3])
    D = oracle.divided_difference(th, SW)
    assert np.allclose(np.diag(D), oracle.step_deriv(th, SW))
    assert abs(D[0, 1] - oracle.step_deriv(np.array([-0.1]), SW)[0]) < 1e-6
    S = oracle.step(th, SW)
    assert abs(D[2, 3] - (S[2] - S[3]) / (th[2] - th[3])) < 1e-15
