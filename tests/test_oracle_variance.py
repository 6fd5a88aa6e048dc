"""Pins of the oracle's `variance` output (the sampling variance of the
Hutchinson mean, Section 2, eq. traceT: the m probe values d_j are i.i.d., so
the variance of their mean is Var(d)/m, estimated without bias by the sample
variance of the d_j divided by m).

  * m = 2: the unbiased estimate has the closed form (d_0 - d_1)^2 / 4.
  * m = 1: undefined (NaN).
  * Statistical: over many independent probe blocks (disjoint seeds) the
    reported variances must average to the empirical variance of the
    estimates themselves.  The comparison uses a z-score whose standard error
    is estimated from the same samples (fourth moments included, so no
    normality is assumed), and the test also shows that the two plausible
    mistakes (the division by m forgotten; the biased 1/m sample variance in
    place of 1/(m-1)) would fail it.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1602_02306_amd import workloads as W


def _c1():
    wl = W.WORKLOADS["c1"]
    return wl, W.make_problem(wl)


def test_variance_closed_form_two_probes():
    wl, P = _c1()
    V = W.rademacher(P.A.n, 2, 31)
    r = oracle.count(P.A, P.prec, wl.xi, wl.eta, V, wl.k)
    d0 = r.s_eta[0] - r.s_xi[0]
    d1 = r.s_eta[1] - r.s_xi[1]
    assert r.estimate == pytest.approx(0.5 * (d0 + d1), rel=1e-15, abs=1e-13)
    assert r.variance == pytest.approx(0.25 * (d0 - d1) ** 2, rel=1e-13, abs=1e-13)
    assert r.variance > 0.0


def test_variance_single_probe_nan():
    wl, P = _c1()
    r = oracle.count(P.A, P.prec, wl.xi, wl.eta, W.rademacher(P.A.n, 1, 3), wl.k)
    assert math.isnan(r.variance)


def _zscore(est, var):
    """z of (empirical variance of the estimates) - (mean reported variance),
    with the standard error of both terms estimated from the samples."""
    S = len(est)
    e = np.asarray(est) - np.mean(est)
    v_emp = float(np.sum(e ** 2) / (S - 1))
    mu4 = float(np.mean(e ** 4))
    var_vemp = (mu4 - (S - 3) / (S - 1) * v_emp ** 2) / S
    v_rep = float(np.mean(var))
    var_vrep = float(np.var(var, ddof=1)) / S
    return (v_emp - v_rep) / math.sqrt(var_vemp + var_vrep), v_emp, v_rep


@pytest.mark.parametrize("m,S", [(40, 300), (2, 600)])
def test_variance_matches_spread_of_estimates(m, S):
    """c1 at k = 20: S independent probe blocks of m probes (seeds 1000 + s).
    The reported variance is the variance of the estimate."""
    wl, P = _c1()
    est, var = [], []
    for s in range(S):
        V = W.rademacher(P.A.n, m, 1000 + s)
        r = oracle.count(P.A, P.prec, wl.xi, wl.eta, V, wl.k)
        est.append(r.estimate)
        var.append(r.variance)
    var = np.asarray(var)
    z, v_emp, v_rep = _zscore(est, var)
    print("m=%d S=%d: empirical var of estimates %.4f, mean reported %.4f, z = %.2f" % (m, S, v_emp, v_rep, z))
    assert abs(z) <= 4.0
    # the same test rejects the plausible mistakes
    z_no_m, _, _ = _zscore(est, var * m)               # /m forgotten
    assert abs(z_no_m) > 4.0
    if m == 2:
        z_ddof, _, _ = _zscore(est, var * (m - 1) / m)  # 1/m sample variance
        assert abs(z_ddof) > 4.0
