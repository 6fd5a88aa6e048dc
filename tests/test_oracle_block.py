"""Pins of the block-Lanczos oracle (block Gauss rule on blocks of P probes)
against what the mathematics fixes: the paper's single-vector estimator at
P = 1 (Section 3.1 eq. gauss_quad, Section 3.2 Algorithm 2), the degree of
exactness 2k - 1 of the block Gauss rule, exactness once the block Krylov
space is invariant (then the count is the inertia, Section 2 eq. negi_T),
and the rule's dependence on the probe block only through its span."""
import numpy as np
import pytest

import oracle
from paper_1602_02306_amd import workloads as W


def problem(dims, seed=3, prec="cheb"):
    wl = W.Workload("t", dims, "wells", seed, -5.0, 1.0, prec, 4, 4)
    return W.make_problem(wl)


def mid_gap(lam, i):
    lam = np.sort(lam)
    return 0.5 * (lam[i] + lam[i + 1])


@pytest.mark.parametrize("prec", ["none", "jacobi", "cheb"])
def test_block_size_one_is_the_paper_estimator(prec):
    """P = 1: the block recurrence is Algorithm 1 and S = |v|^2 e_1^T h(J_k) e_1."""
    P = problem((5, 4, 4), prec=prec)
    lam = np.linalg.eigvalsh(P.A.to_dense())
    tau = mid_gap(lam, 20)
    V = W.rademacher(P.A.n, 6, 11)
    mean_s, s_scalar, res, _ = oracle.negcount(P.A, P.prec, tau, V, 9)
    mean_b, s_block, bres, _ = oracle.block_negcount(P.A, P.prec, tau, V, 9, P=1)
    assert np.array_equal(bres.k_used, res.k_used)
    assert np.allclose(s_block, s_scalar, rtol=1e-11, atol=1e-11)
    # the 1 x 1 blocks are alpha_i and beta_{i+1}
    assert np.allclose(bres.A[:, :, 0, 0], res.alpha, rtol=1e-11, atol=1e-12)
    assert np.allclose(bres.B[:, 1:, 0, 0], res.beta[:, 1:], rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("Pb,k", [(16, 4), (4, 6)])
def test_block_gauss_rule_degree_of_exactness(Pb, k):
    """R_0^T E_1^T T_k^p E_1 R_0 = V_b^T C^p V_b for p <= 2k - 1 and not for
    p = 2k (block Gauss rule)."""
    P = problem((6, 5, 4), seed=5)
    lam = np.linalg.eigvalsh(P.A.to_dense())
    tau = mid_gap(lam, 30)
    C = oracle.dense_operator(P.A, P.prec, tau)
    V = W.rademacher(P.A.n, 2 * Pb, 4)
    res = oracle.block_lanczos(P.A, P.prec, tau, V, k, P=Pb)
    assert np.all(res.k_used == k)
    for b in range(2):
        Vb = V[:, b * Pb:(b + 1) * Pb]
        T = oracle.block_tridiagonal(res.A[b], res.B[b], k)
        R0 = res.R0[b]
        Tp = np.eye(k * Pb)
        Cp = np.eye(C.shape[0])
        for p in range(2 * k + 1):
            lhs = R0.T @ Tp[:Pb, :Pb] @ R0
            rhs = Vb.T @ Cp @ Vb
            err = np.abs(lhs - rhs).max() / np.abs(rhs).max()
            if p <= 2 * k - 1:
                assert err < 1e-10, (p, err)
            else:
                assert err > 1e-6, (p, err)
            Tp = Tp @ T
            Cp = Cp @ C


def test_block_rule_exact_when_space_exhausted():
    """n = 3P: after three blocks the Krylov space is the whole space, the
    fourth residual vanishes (k_used = 3) and S = V_b^T h(C) V_b exactly;
    with the scaled identity as probe matrix (sum_j v_j v_j^T = n I) the mean
    of the s_j is the inertia n_(A - tau I) (eq. negi_T)."""
    P = problem((4, 4, 3), seed=7)
    n = P.A.n
    lam = np.linalg.eigvalsh(P.A.to_dense())
    tau = mid_gap(lam, 12)
    C = oracle.dense_operator(P.A, P.prec, tau)
    ev, U = np.linalg.eigh(0.5 * (C + C.T))
    Pm = (U * (ev < 0)) @ U.T
    V = W.identity_probes(n)
    res = oracle.block_lanczos(P.A, P.prec, tau, V, 5, P=16)
    assert np.all(res.k_used == 3)
    s, _ = oracle.block_quadrature(res)
    assert abs(float(np.mean(s)) - 13.0) < 1e-9
    Vr = W.rademacher(n, 16, 9)
    rr = oracle.block_lanczos(P.A, P.prec, tau, Vr, 5, P=16)
    assert rr.k_used[0] == 3
    S, _ = oracle.block_rule_matrix(rr, 0)
    assert np.abs(S - Vr.T @ Pm @ Vr).max() < 1e-9 * np.abs(Vr.T @ Vr).max()


def test_block_rule_depends_on_the_span_only():
    """V_b -> V_b U (U orthogonal) maps S to U^T S U: the rule sees the block
    Krylov space, not the basis of the probe block."""
    P = problem((6, 5, 4), seed=5)
    lam = np.linalg.eigvalsh(P.A.to_dense())
    tau = mid_gap(lam, 30)
    V = W.rademacher(P.A.n, 16, 2)
    U, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((16, 16)))
    r1 = oracle.block_lanczos(P.A, P.prec, tau, V, 4, P=16)
    r2 = oracle.block_lanczos(P.A, P.prec, tau, V @ U, 4, P=16)
    S1, _ = oracle.block_rule_matrix(r1, 0)
    S2, _ = oracle.block_rule_matrix(r2, 0)
    assert np.abs(S2 - U.T @ S1 @ U).max() < 1e-10 * np.abs(S1).max()


def test_block_count_is_difference_of_shifts():
    P = problem((5, 4, 4), seed=2)
    lam = np.linalg.eigvalsh(P.A.to_dense())
    xi, eta = mid_gap(lam, 5), mid_gap(lam, 30)
    V = W.rademacher(P.A.n, 32, 6)
    r = oracle.block_count(P.A, P.prec, xi, eta, V, 4, P=16)
    assert r.estimate == pytest.approx(r.neg_eta - r.neg_xi, abs=1e-12)
    with pytest.raises(ValueError):
        oracle.block_lanczos(P.A, P.prec, xi, V[:, :20], 3, P=16)


def test_oracle_at_the_largest_k_against_the_block_transcription():
    """k = 512 on n = 640 (shift near the bottom of the spectrum and inside it):
    the C oracle (alpha first, then one Gram-Schmidt pass) and the numpy block
    oracle at P = 1 (one pass from C q_i) sum in different orders; both keep the
    basis orthogonal to rounding, so their per-probe values agree to 1e-12 n
    and both estimates lie within a few units of the exact count."""
    P = problem((10, 8, 8), seed=3)
    n = P.A.n
    lam = np.sort(np.linalg.eigvalsh(P.A.to_dense()))
    xi, eta = mid_gap(lam, 40), mid_gap(lam, 300)
    V = W.rademacher(n, 2, 17)
    ref = oracle.count(P.A, P.prec, xi, eta, V, 512)
    blk = oracle.block_count(P.A, P.prec, xi, eta, V, 512, P=1)
    s1 = np.concatenate([ref.s_xi, ref.s_eta])
    s2 = np.concatenate([blk.s_xi, blk.s_eta])
    assert np.max(np.abs(s1 - s2)) <= 1e-12 * n
    exact = int(np.sum((lam >= xi) & (lam < eta)))
    assert exact == 260
    assert abs(ref.estimate - exact) < 30 and abs(blk.estimate - exact) < 30
