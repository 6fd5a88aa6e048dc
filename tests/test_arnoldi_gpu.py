"""GPU parity of the Arnoldi estimator (Section 4, Algorithm 4) against the
oracle on the same seeded probes.

The GPU orthogonalizes by two classical Gram-Schmidt passes and evaluates
e_1^T h(H_k) e_1 through the matrix sign function; the oracle follows
Algorithm 3 (modified Gram-Schmidt) and Algorithm 4 (eigendecomposition of
H_k, first column of its inverse).  The two agree in exact arithmetic; the
tolerances are those of the Lanczos parity tests: the estimate within
1e-10 * max(|ref|, 1) and every per-probe value within 1e-10 * max(|s_j|, 1).
"""
import numpy as np
import pytest

import oracle
from paper_1602_02306_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def ec():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_02306_amd import ecount
    ecount.load()
    return ecount


def t_spec(kind, dims):
    return W.cheb_inverse_prec(dims, degree=8) if kind == "cheb" else W.PrecSpec("none", ())


def run(ec, A, T, xi, eta, V, k, **kw):
    Ad = ec.upload_csr(A, val_dtype=kw.pop("val", "f64"))
    vec = kw.get("vec", "f64")
    Vd = torch.from_numpy(V).to("cuda", torch.float32 if vec == "f32" else torch.float64)
    return ec.count_arnoldi(Ad, T, xi, eta, Vd, k, **kw)


def check(r, ref, n, tol=TOL):
    s = r.per_probe.cpu().numpy()
    s_ref = np.concatenate([ref.s_xi, ref.s_eta])
    d = np.max(np.abs(s - s_ref) / np.maximum(1.0, np.abs(s_ref)))
    print("gpu %.15f oracle %.15f | max |ds|/max(|s|,1) %.2e" % (r.estimate, ref.estimate, d), flush=True)
    assert abs(r.estimate - ref.estimate) <= tol * max(1.0, abs(ref.estimate))
    assert d <= tol
    assert abs(r.neg_xi - ref.neg_xi) <= tol * max(1.0, abs(ref.neg_xi))
    assert abs(r.neg_eta - ref.neg_eta) <= tol * max(1.0, abs(ref.neg_eta))


@pytest.mark.parametrize("kind", ["cheb", "none"])
@pytest.mark.parametrize("name", ["c2_small", "c2_ragged"])
def test_arnoldi_parity(ec, name, kind):
    wl = W.WORKLOADS[name]
    P = W.make_problem(wl)
    V = W.make_probes(wl)
    T = t_spec(kind, wl.dims)
    r = run(ec, P.A, T, wl.xi, wl.eta, V, wl.k)
    ref = oracle.count_arnoldi(P.A, T, wl.xi, wl.eta, V, wl.k)
    check(r, ref, P.A.n)
    assert np.all(r.k_used.cpu().numpy() == np.concatenate([ref.lan_xi.k_used, ref.lan_eta.k_used]))


def test_arnoldi_more_steps_and_waves(ec):
    """k = 40 (two basis chunks per pass) and column waves with a ragged last wave."""
    wl = W.WORKLOADS["c2_ragged"]
    P = W.make_problem(wl)
    V = W.make_probes(wl)[:, :11]
    T = t_spec("cheb", wl.dims)
    ref = oracle.count_arnoldi(P.A, T, wl.xi, wl.eta, V, 40)
    r = run(ec, P.A, T, wl.xi, wl.eta, V, 40)
    check(r, ref, P.A.n, tol=1e-9)
    r = run(ec, P.A, T, wl.xi, wl.eta, V, 40, max_cols=7)
    check(r, ref, P.A.n, tol=1e-9)


def test_arnoldi_full_krylov_exact(ec):
    """k = n with Hadamard probes gives the exact inertia on the GPU as well."""
    dims = (4, 4, 4)
    wl = W.Workload("t", dims, "wells", 3, -5.0, 1.0, "none", 4, 4)
    P = W.make_problem(wl)
    n = P.A.n
    lam = np.sort(np.linalg.eigvalsh(P.A.to_dense()))
    xi, eta = 0.5 * (lam[5] + lam[6]), 0.5 * (lam[40] + lam[41])
    T = t_spec("cheb", dims)
    r = run(ec, P.A, T, xi, eta, W.hadamard_probes(n), 64)
    assert abs(r.neg_xi - 6.0) < 1e-8 and abs(r.neg_eta - 41.0) < 1e-8
    assert abs(r.estimate - 35.0) < 1e-8


def test_arnoldi_fp32_bound(ec):
    wl = W.WORKLOADS["c2_small"]
    P = W.make_problem(wl)
    V = W.make_probes(wl)
    T = t_spec("cheb", wl.dims)
    r = run(ec, P.A, T, wl.xi, wl.eta, V, wl.k, vec="f32", val="f32")
    ref = oracle.count_arnoldi(P.A, T, wl.xi, wl.eta, V, wl.k)
    check(r, ref, P.A.n, tol=1e-4)


def test_arnoldi_rejects_unsupported(ec):
    wl = W.WORKLOADS["c1"]
    P = W.make_problem(wl)
    V = W.make_probes(wl)
    with pytest.raises(ec.EcntError) as e:
        run(ec, P.A, W.PrecSpec("jacobi", ()), wl.xi, wl.eta, V, wl.k)
    assert e.value.status == ec.ECNT_EUNSUPPORTED


def test_arnoldi_one_step_one_probe(ec):
    """k = 1 (H_1 is a scalar: sign of the Rayleigh quotient) and m = 1
    (variance NaN) against the oracle."""
    wl = W.WORKLOADS["c2_small"]
    P = W.make_problem(wl)
    V = W.make_probes(wl)[:, :1]
    T = t_spec("cheb", wl.dims)
    for k in (1, 2):
        r = run(ec, P.A, T, wl.xi, wl.eta, V, k)
        ref = oracle.count_arnoldi(P.A, T, wl.xi, wl.eta, V, k)
        check(r, ref, P.A.n)
        assert np.isnan(r.variance)


def test_arnoldi_deterministic(ec):
    wl = W.WORKLOADS["c2_ragged"]
    P = W.make_problem(wl)
    V = W.make_probes(wl)
    T = t_spec("cheb", wl.dims)
    a = run(ec, P.A, T, wl.xi, wl.eta, V, wl.k)
    b = run(ec, P.A, T, wl.xi, wl.eta, V, wl.k)
    assert a.estimate == b.estimate and torch.equal(a.per_probe, b.per_probe)


@pytest.mark.parametrize("kind", ["none", "cheb"])
def test_arnoldi_maximum_k(ec, kind):
    """k = 64, the largest the Arnoldi estimator takes, on n = 640 with one shift
    near the bottom of the spectrum and one inside it."""
    wl = W.Workload("t", (10, 8, 8), "wells", 3, -5.0, 1.0, "cheb", 4, 64)
    P = W.make_problem(wl)
    lam = np.sort(np.linalg.eigvalsh(P.A.to_dense()))
    xi, eta = 0.5 * (lam[40] + lam[41]), 0.5 * (lam[300] + lam[301])
    V = W.rademacher(P.A.n, 4, 17)
    T = t_spec(kind, wl.dims)
    print("arnoldi maximum k", kind, flush=True)
    r = run(ec, P.A, T, xi, eta, V, 64)
    ref = oracle.count_arnoldi(P.A, T, xi, eta, V, 64)
    check(r, ref, P.A.n)
