"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Tolerances for FP64 (stated):
  * the estimate within 1e-10 * max(|ref|, 1);
  * every per-probe quadrature value s_j, and the per-shift means, within
    1e-10 * max(|ref|, 1) of the oracle's;
  * alpha/beta within 1e-8 * max|alpha| (diagnostics only).
Two correct implementations of Algorithm 1 that differ only in rounding
(summation order, the fused Gram-Schmidt pass) agree to about 1e-13 at the
workloads' k; once Ritz values converge next to 0 the quadrature and the late
coefficients become ill-conditioned (measured on the CPU for the 30x30
problem at k = 40: per-probe s_j move by up to 2e-8 = 2e-11 |v|^2 and late
alpha/beta by 1.6e-7 under 1e-16 perturbations of the operator).  The k = 40
cases on that problem therefore bound s_j by 1e-10 * |v_j|^2 (s_j lies in
[0, |v_j|^2], a sum of Gauss weights times |v_j|^2) and alpha/beta by 1e-6.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1602_02306_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = 1e-10


@pytest.fixture(scope="module")
def ec():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_02306_amd import ecount
    ecount.load()
    return ecount


def gpu_count(ec, A, prec, xi, eta, V, k, **kw):
    Ad = ec.upload_csr(A, val_dtype=kw.pop("val", "f64"))
    vec = kw.get("vec", "f64")
    Vd = torch.from_numpy(V).to("cuda", torch.float32 if vec == "f32" else torch.float64)
    return ec.count(Ad, prec, xi, eta, Vd, k, **kw)


def rel(a, b):
    return abs(a - b) / max(1.0, abs(b))


def assert_parity(r, ref, k=None, coef_tol=1e-8, probe_scale="rel"):
    """probe_scale 'rel': s_j within TOL * max(|s_j|, 1); 'nu': within
    TOL * |v_j|^2 (the ill-conditioned k = 40 cases only, see the header)."""
    s = r.per_probe.cpu().numpy()
    s_ref = np.concatenate([ref.s_xi, ref.s_eta])
    nu = np.concatenate([ref.lan_xi.nu, ref.lan_eta.nu])
    scale = np.maximum(1.0, np.abs(s_ref)) if probe_scale == "rel" else nu
    print("gpu %.15f oracle %.15f | rel est %.2e | max |ds|/nu %.2e | max |ds|/max(|s|,1) %.2e"
          % (r.estimate, ref.estimate, rel(r.estimate, ref.estimate),
             np.max(np.abs(s - s_ref) / nu), np.max(np.abs(s - s_ref) / np.maximum(1, np.abs(s_ref)))),
          flush=True)
    assert rel(r.estimate, ref.estimate) <= TOL
    if probe_scale == "rel":
        assert abs(r.neg_xi - ref.neg_xi) <= TOL * max(1.0, abs(ref.neg_xi))
        assert abs(r.neg_eta - ref.neg_eta) <= TOL * max(1.0, abs(ref.neg_eta))
    else:
        nu_mean = float(np.mean(nu))
        assert abs(r.neg_xi - ref.neg_xi) <= TOL * nu_mean
        assert abs(r.neg_eta - ref.neg_eta) <= TOL * nu_mean
    assert np.all(np.abs(s - s_ref) <= TOL * scale)
    if not math.isnan(ref.variance):
        assert abs(r.variance - ref.variance) <= 1e-8 * max(ref.variance, 1e-12)
    ku = r.k_used.cpu().numpy()
    ku_ref = np.concatenate([ref.lan_xi.k_used, ref.lan_eta.k_used])
    assert np.array_equal(ku, ku_ref)
    if k is not None:
        al = r.alpha.cpu().numpy().T
        be = r.beta.cpu().numpy().T
        al_ref = np.concatenate([ref.lan_xi.alpha, ref.lan_eta.alpha])
        be_ref = np.concatenate([ref.lan_xi.beta, ref.lan_eta.beta])
        scale = max(1.0, np.abs(al_ref).max())
        print("max |d alpha| %.2e  max |d beta| %.2e" % (
            max(np.max(np.abs(al[c, :ku_ref[c]] - al_ref[c, :ku_ref[c]])) for c in range(al.shape[0])),
            max(np.max(np.abs(be[c, :ku_ref[c] + 1] - be_ref[c, :ku_ref[c] + 1])) for c in range(al.shape[0]))),
            flush=True)
        for c in range(al.shape[0]):
            kk = ku_ref[c]
            assert np.all(np.abs(al[c, :kk] - al_ref[c, :kk]) <= coef_tol * scale)
            assert np.all(np.abs(be[c, :kk + 1] - be_ref[c, :kk + 1]) <= coef_tol * scale)


def run_workload(ec, name, **over):
    wl = W.WORKLOADS[name]
    P = W.make_problem(wl)
    V = W.make_probes(wl)
    k = over.pop("k", wl.k)
    rule = over.pop("rule", "gauss")
    sw = over.pop("smooth_w", wl.smooth_w)
    r = gpu_count(ec, P.A, P.prec, wl.xi, wl.eta, V, k, rule=rule, smooth_w=sw, **over)
    ref = oracle.count(P.A, P.prec, wl.xi, wl.eta, V, k, rule=rule, smooth_w=sw)
    return r, ref, k


@pytest.mark.parametrize("name", ["c1", "c2_small", "c2_ragged"])
def test_parity_small_workloads(ec, name):
    print("case", name, flush=True)
    r, ref, k = run_workload(ec, name)
    assert_parity(r, ref, k)


def test_parity_ga_rule(ec):
    r, ref, k = run_workload(ec, "c1", rule="ga")
    assert_parity(r, ref, k)


def test_parity_ga_rule_cheb(ec):
    r, ref, k = run_workload(ec, "c2_ragged", rule="ga")
    assert_parity(r, ref, k)


def test_parity_smoothed(ec):
    r, ref, k = run_workload(ec, "c2_small", smooth_w=0.05)
    assert_parity(r, ref, k)


def test_parity_more_than_one_basis_chunk(ec):
    # k = 40 > 32: the reorthogonalization runs over two basis chunks
    r, ref, k = run_workload(ec, "c1", k=40)
    assert_parity(r, ref, k, coef_tol=1e-6, probe_scale="nu")


@pytest.mark.parametrize("prec", ["none", "jacobi", "cheb"])
def test_full_krylov_exact_count_gpu(ec, prec):
    """k = n with Hadamard probes: the estimate is the exact integer count
    (Proposition 1 and eq. negi_T), for every preconditioner."""
    dims = (4, 4, 4)
    wl = W.Workload("t", dims, "wells", 3, -5.0, 1.0, prec, 64, 64)
    P = W.make_problem(wl)
    lam = np.linalg.eigvalsh(P.A.to_dense())
    xi, eta = 0.5 * (lam[5] + lam[6]), 0.5 * (lam[40] + lam[41])
    V = W.hadamard_probes(64)
    r = gpu_count(ec, P.A, P.prec, xi, eta, V, 64)
    assert abs(r.estimate - 35.0) < 1e-9
    ref = oracle.count(P.A, P.prec, xi, eta, V, 64)
    assert rel(r.estimate, ref.estimate) <= TOL


FORMS = {"fused": {}, "waves": {"fused": "off"}}


@pytest.mark.parametrize("form", list(FORMS))
def test_ideal_preconditioner_breakdown_gpu(ec, form):
    """Diagonal A with |A - tau I|^(-1/2): two distinct eigenvalues of C, the
    Lanczos run stops after 2 steps and s_j equals the count (Section 6).
    Both the one-launch form of small problems and the column waves."""
    rng = np.random.default_rng(5)
    d = rng.uniform(-3.0, 3.0, 300)
    A = W.CSR(300, np.arange(301, dtype=np.int32), np.arange(300, dtype=np.int32), d)
    V = W.rademacher(300, 70, 11)
    r = gpu_count(ec, A, W.PrecSpec("jacobi", ()), -0.5, 0.7, V, 6, tune=FORMS[form])
    ku = r.k_used.cpu().numpy()
    assert np.all(ku == 2)
    s = r.per_probe.cpu().numpy()
    assert np.allclose(s[:70], np.sum(d < -0.5), atol=1e-9)
    assert np.allclose(s[70:], np.sum(d < 0.7), atol=1e-9)
    assert abs(r.estimate - np.sum((d >= -0.5) & (d < 0.7))) < 1e-9


@pytest.mark.parametrize("form", list(FORMS))
def test_breakdown_mixed_within_a_wave(ec, form):
    """Diagonal A without preconditioner: probes that are unit vectors span an
    invariant space at once (k_used = 1), a probe on two coordinates after two
    steps, Rademacher probes run to k; all in one wave, each column against the
    oracle (its k_used and s_j) while the others keep iterating.  Both the
    one-launch form of small problems and the column waves."""
    rng = np.random.default_rng(8)
    n = 300
    d = np.sort(rng.uniform(-3.0, 3.0, n))
    A = W.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    V = W.rademacher(n, 6, 21)
    V[:, 0] = 0.0
    V[7, 0] = 1.0
    V[:, 3] = 0.0
    V[200, 3] = 1.0
    V[:, 4] = 0.0
    V[10, 4] = 1.0
    V[250, 4] = -1.0
    print("mixed breakdown", form, flush=True)
    r = gpu_count(ec, A, W.PrecSpec("none", ()), -0.5, 0.7, V, 12, tune=FORMS[form])
    ref = oracle.count(A, W.PrecSpec("none", ()), -0.5, 0.7, V, 12)
    ku = np.concatenate([ref.lan_xi.k_used, ref.lan_eta.k_used])
    assert set(ku.tolist()) >= {1, 2, 12}
    assert_parity(r, ref)


def test_single_probe_variance_nan(ec):
    wl = W.WORKLOADS["c1"]
    P = W.make_problem(wl)
    V = W.rademacher(P.A.n, 1, 5)
    r = gpu_count(ec, P.A, P.prec, wl.xi, wl.eta, V, 7)
    ref = oracle.count(P.A, P.prec, wl.xi, wl.eta, V, 7)
    assert math.isnan(r.variance) and math.isnan(ref.variance)
    assert rel(r.estimate, ref.estimate) <= TOL


def max_k_problem():
    wl = W.Workload("t", (10, 8, 8), "wells", 3, -5.0, 1.0, "cheb", 4, 512)
    P = W.make_problem(wl)
    lam = np.sort(np.linalg.eigvalsh(P.A.to_dense()))
    return P, 0.5 * (lam[40] + lam[41]), 0.5 * (lam[300] + lam[301])


@pytest.mark.parametrize("rule,k", [("gauss", 512), ("ga", 256)])
def test_parity_maximum_k(ec, rule, k):
    """The largest k the library takes (512 for the Gauss rule, 256 for the
    GA rule) on n = 640: a 513-slot basis and the largest tridiagonal
    eigenproblem.  Two FP64 oracles that differ only in rounding order (the C
    oracle and the block oracle at P = 1) agree to 1e-14 |v|^2 here."""
    P, xi, eta = max_k_problem()
    V = W.rademacher(P.A.n, 4, 17)
    print("maximum k", rule, k, flush=True)
    r = gpu_count(ec, P.A, P.prec, xi, eta, V, k, rule=rule)
    ref = oracle.count(P.A, P.prec, xi, eta, V, k, rule=rule)
    assert np.all(ref.lan_xi.k_used == k) and np.all(ref.lan_eta.k_used == k)
    assert_parity(r, ref)


def test_one_step(ec):
    r, ref, k = run_workload(ec, "c2_ragged", k=1)
    assert_parity(r, ref, k)


def test_negcounts_four_shifts(ec):
    """Spectrum slicing: 4 shifts, 3 contiguous intervals in one call."""
    wl = W.WORKLOADS["c2_ragged"]
    P = W.make_problem(wl)
    V = W.make_probes(wl)
    taus = np.array([-70.0, -55.0, -41.0, -30.0])
    Ad = ec.upload_csr(P.A)
    Vd = torch.from_numpy(V).cuda()
    r = ec.negcounts(Ad, P.prec, taus, Vd, wl.k)
    s_gpu = r.per_probe.cpu().numpy().reshape(4, -1)
    for i, tau in enumerate(taus):
        mean, s, _, _ = oracle.negcount(P.A, P.prec, tau, V, wl.k)
        assert rel(r.negcounts[i], mean) <= TOL
        assert np.all(np.abs(s_gpu[i] - s) <= TOL * np.maximum(1.0, np.abs(s)))
    for t in range(3):
        d = s_gpu[t + 1] - s_gpu[t]
        assert rel(r.counts[t], d.mean()) <= 1e-12


def test_jacobi_singular_reported(ec):
    d = np.array([1.0, 0.5, 3.0, -1.0] * 16)
    A = W.CSR(64, np.arange(65, dtype=np.int32), np.arange(64, dtype=np.int32), d)
    V = W.rademacher(64, 3, 1)
    with pytest.raises(ec.EcntError) as e:
        gpu_count(ec, A, W.PrecSpec("jacobi", ()), 0.5, 2.0, V, 3)
    assert e.value.status == ec.ECNT_ENOTHPD


def test_deterministic_bitwise(ec):
    wl = W.WORKLOADS["c2_small"]
    P = W.make_problem(wl)
    V = W.make_probes(wl)
    a = gpu_count(ec, P.A, P.prec, wl.xi, wl.eta, V, wl.k)
    b = gpu_count(ec, P.A, P.prec, wl.xi, wl.eta, V, wl.k)
    assert a.estimate == b.estimate and a.variance == b.variance
    assert torch.equal(a.per_probe, b.per_probe)


def test_bench_configuration_sampled(ec):
    """The benchmark workload at full size (64^3 wells, Chebyshev M, 256
    probes, k = 30), in the launch configuration the benchmark times; the
    oracle recomputes a sample of probes one by one (each probe's Lanczos run
    is independent, so a column subset reproduces its s_j exactly)."""
    wl = W.WORKLOADS["c2"]
    P = W.make_problem(wl)
    V = W.make_probes(wl)
    print("case c2 full", flush=True)
    r = gpu_count(ec, P.A, P.prec, wl.xi, wl.eta, V, wl.k)
    s = r.per_probe.cpu().numpy().reshape(2, -1)
    sample = [0, 101, 255]
    ref = oracle.count(P.A, P.prec, wl.xi, wl.eta, V[:, sample], wl.k)
    for t, (sx, se) in enumerate(zip(ref.s_xi, ref.s_eta)):
        j = sample[t]
        assert abs(s[0, j] - sx) <= TOL * max(1.0, abs(sx))
        assert abs(s[1, j] - se) <= TOL * max(1.0, abs(se))
    # whole-run properties: estimate is the mean of the per-probe differences
    d = s[1] - s[0]
    assert rel(r.estimate, d.mean()) <= 1e-12
    exact = json.load(open(os.path.join(GOLDEN, "exact_counts.json"))).get("c2", {}).get("count")
    print("c2 estimate %.4f +- %.4f exact %s" % (r.estimate, math.sqrt(r.variance), exact), flush=True)


def test_bench_configuration_sampled_fp32(ec):
    """The benchmark workload at full size in the FP32 storage form (the
    launch configuration of its bench line): sampled probes against the FP64
    oracle and the estimate against the FP64 path, within the FP32 bound."""
    wl = W.WORKLOADS["c2"]
    P = W.make_problem(wl)
    V = W.make_probes(wl)
    print("case c2 full fp32", flush=True)
    r = gpu_count(ec, P.A, P.prec, wl.xi, wl.eta, V, wl.k, vec="f32", val="f32")
    s = r.per_probe.cpu().numpy().reshape(2, -1)
    sample = [3, 128]
    ref = oracle.count(P.A, P.prec, wl.xi, wl.eta, V[:, sample], wl.k)
    nu = float(P.A.n)   # |v_j|^2 of a Rademacher probe
    for t, (sx, se) in enumerate(zip(ref.s_xi, ref.s_eta)):
        j = sample[t]
        print("probe %d: fp32 %.6f %.6f oracle %.6f %.6f" % (j, s[0, j], s[1, j], sx, se), flush=True)
        assert abs(s[0, j] - sx) <= FP32_BOUND * nu
        assert abs(s[1, j] - se) <= FP32_BOUND * nu
    r64 = gpu_count(ec, P.A, P.prec, wl.xi, wl.eta, V, wl.k)
    print("estimate fp32 %.8f fp64 %.8f" % (r.estimate, r64.estimate), flush=True)
    assert rel(r.estimate, r64.estimate) <= FP32_BOUND


@pytest.mark.parametrize("name", ["c2_small", "c2_ragged"])
def test_parity_clenshaw_evaluation(ec, name):
    """M evaluated by Clenshaw's recurrence instead of the product of its
    quadratic factors: same polynomial, same parity bar."""
    r, ref, k = run_workload(ec, name, eval="clenshaw")
    assert_parity(r, ref, k)


@pytest.mark.parametrize("max_cols", [30, 37, 1])
def test_parity_column_waves(ec, max_cols):
    """Columns run in waves of at most max_cols (ragged last wave; odd widths
    take the one-column-per-lane kernels); results equal the oracle's."""
    r, ref, k = run_workload(ec, "c2_ragged", max_cols=max_cols)
    assert_parity(r, ref, k)


def test_parity_column_waves_two_basis_chunks(ec):
    """k = 40 (two basis chunks per pass, alpha_i from the second) in column
    waves of 30 (a ragged last wave): every wave against the oracle."""
    r, ref, k = run_workload(ec, "c1", k=40, max_cols=30)
    assert_parity(r, ref, k, coef_tol=1e-6, probe_scale="nu")


@pytest.mark.parametrize("vec", ["f64", "f32"])
def test_parity_padded_slots_in_waves(ec, vec):
    """A block vector of 4096 rows x 32 columns is a power of two in bytes, so
    the basis slots are padded; two waves of 32 columns (m = 32, both shifts)."""
    wl = W.WORKLOADS["c2_small"]
    P = W.make_problem(wl)
    V = W.rademacher(P.A.n, 32, 17)
    ref = oracle.count(P.A, P.prec, wl.xi, wl.eta, V, wl.k)
    r = gpu_count(ec, P.A, P.prec, wl.xi, wl.eta, V, wl.k, vec=vec, max_cols=32)
    if vec == "f64":
        assert_parity(r, ref, wl.k)
    else:
        s = r.per_probe.cpu().numpy()
        s_ref = np.concatenate([ref.s_xi, ref.s_eta])
        assert abs(r.estimate - ref.estimate) <= 1e-4 * max(1.0, abs(ref.estimate))
        assert np.max(np.abs(s - s_ref)) <= 1e-4 * P.A.n


def test_parity_column_waves_jacobi(ec):
    r, ref, k = run_workload(ec, "c1", max_cols=48)
    assert_parity(r, ref, k)


@pytest.mark.parametrize("tune", [{"tile": "2x4"}, {"tile": "1x8"}, {"tile": "4x4"},
                                  {"tile": "4x4-unfused"}, {"tile": "8x8-wg"},
                                  {"red_waves": 64}, {"red_waves": 65536}, {"csr_vw": 1},
                                  {"tile": "2x4", "red_waves": 8192, "csr_vw": 1}])
def test_parity_launch_shapes(ec, tune):
    """Every launch shape the autotuner may pick gives the oracle's results."""
    r, ref, k = run_workload(ec, "c2_ragged", tune=tune)
    assert_parity(r, ref, k)
    r, ref, k = run_workload(ec, "c2_small", tune=tune)
    assert_parity(r, ref, k)


def test_stencil_tile_shapes_bitwise(ec):
    """The plain stencil sweep computes each grid point the same way whatever
    the line block, so the tile shape alone changes no bit of the result."""
    wl = W.WORKLOADS["c2_ragged"]
    P = W.make_problem(wl)
    V = W.make_probes(wl)
    outs = [gpu_count(ec, P.A, P.prec, wl.xi, wl.eta, V, wl.k, tune={"tile": t})
            for t in ("4x4-unfused", "2x4", "1x8")]
    for o in outs[1:]:
        assert o.estimate == outs[0].estimate
        assert torch.equal(o.per_probe, outs[0].per_probe)


@pytest.mark.parametrize("tile", ["4x4", "8x8-wg"])
@pytest.mark.parametrize("name", ["c2_small", "c2_ragged"])
def test_fused_quadratic_sweep_matches_two_sweeps(ec, name, tile):
    """Each quadratic factor of the preconditioner in one fused sweep against
    the same factor as two plain sweeps: the same values up to rounding (the
    fused form sums in the same order; only FMA contraction may differ)."""
    wl = W.WORKLOADS[name]
    P = W.make_problem(wl)
    V = W.make_probes(wl)
    a = gpu_count(ec, P.A, P.prec, wl.xi, wl.eta, V, wl.k, tune={"tile": tile})
    b = gpu_count(ec, P.A, P.prec, wl.xi, wl.eta, V, wl.k, tune={"tile": "4x4-unfused"})
    nu = float(P.A.n)
    assert abs(a.estimate - b.estimate) <= 1e-12 * max(1.0, abs(b.estimate))
    assert float((a.per_probe - b.per_probe).abs().max()) <= 1e-12 * nu


# FP32 storage form: A values, probes, Lanczos vectors and basis in FP32;
# alpha/beta, every dot product and norm and the tridiagonal eigensolve in
# FP64.  Parity with the FP64 oracle is not expected to 1e-10; the stated
# bound is 1e-4 * max(|estimate|, 1) on the estimate and 1e-4 * |v_j|^2 on each
# per-probe value.
FP32_BOUND = 1e-4


@pytest.mark.parametrize("name", ["c2_small", "c2_ragged", "c1"])
def test_fp32_form_within_stated_bound(ec, name):
    wl = W.WORKLOADS[name]
    P = W.make_problem(wl)
    V = W.make_probes(wl)
    r = gpu_count(ec, P.A, P.prec, wl.xi, wl.eta, V, wl.k, vec="f32", val="f32")
    ref = oracle.count(P.A, P.prec, wl.xi, wl.eta, V, wl.k)
    s = r.per_probe.cpu().numpy()
    s_ref = np.concatenate([ref.s_xi, ref.s_eta])
    nu = np.concatenate([ref.lan_xi.nu, ref.lan_eta.nu])
    e_est = rel(r.estimate, ref.estimate)
    e_probe = float(np.max(np.abs(s - s_ref) / nu))
    print("fp32 %s: est %.10f oracle %.10f rel %.2e  max|ds|/nu %.2e" % (name, r.estimate, ref.estimate, e_est, e_probe), flush=True)
    assert e_est <= FP32_BOUND
    assert e_probe <= FP32_BOUND


@pytest.mark.parametrize("name,max_cols", [("c2_small", 0), ("c2_ragged", 0), ("c2_ragged", 37)])
def test_fp32_workgroup_sweep_within_stated_bound(ec, name, max_cols):
    """The FP32 form with the preconditioner's quadratic factors in the
    workgroup sweep on 8 x 8 line blocks: an even wave width (two columns per
    lane) and an odd one (waves of 37 columns, one per lane), each within the
    FP32 bound of the FP64 oracle."""
    wl = W.WORKLOADS[name]
    P = W.make_problem(wl)
    V = W.make_probes(wl)
    kw = {"max_cols": max_cols} if max_cols else {}
    r = gpu_count(ec, P.A, P.prec, wl.xi, wl.eta, V, wl.k, vec="f32", val="f32",
                  tune={"tile": "8x8-wg"}, **kw)
    ref = oracle.count(P.A, P.prec, wl.xi, wl.eta, V, wl.k)
    s = r.per_probe.cpu().numpy()
    s_ref = np.concatenate([ref.s_xi, ref.s_eta])
    nu = np.concatenate([ref.lan_xi.nu, ref.lan_eta.nu])
    e_est = rel(r.estimate, ref.estimate)
    e_probe = float(np.max(np.abs(s - s_ref) / nu))
    print("fp32 wg %s/%d: rel %.2e  max|ds|/nu %.2e" % (name, max_cols, e_est, e_probe), flush=True)
    assert e_est <= FP32_BOUND
    assert e_probe <= FP32_BOUND


@pytest.mark.parametrize("prec_kind", ["none", "jacobi"])
@pytest.mark.parametrize("n", [1, 2, 3])
def test_tiny_problems(ec, n, prec_kind):
    """n = 1..3 rows (far below one tile or wavefront), k = n: the Krylov
    space is the whole space, so every s_j is v_j^T h(C) v_j exactly
    (eq. gauss_quad with k = n)."""
    rng = np.random.default_rng(40 + n)
    d = np.sort(rng.uniform(-3.0, 3.0, n)) + np.arange(n)
    e = rng.uniform(0.2, 0.6, max(n - 1, 0))
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    rows, cols, vals = [], [], []
    for r in range(n):
        for c in range(max(0, r - 1), min(n, r + 2)):
            rows.append(r)
            cols.append(c)
            vals.append(T[r, c])
    rp = np.searchsorted(np.array(rows), np.arange(n + 1)).astype(np.int32)
    A = W.CSR(n, rp, np.array(cols, dtype=np.int32), np.array(vals))
    lam = np.linalg.eigvalsh(T)
    xi = lam[0] - 0.5 if n == 1 else 0.5 * (lam[0] + lam[1])
    eta = lam[-1] + 0.5
    prec = W.PrecSpec(prec_kind, ())
    V = W.rademacher(n, 3, 7 + n)
    print("tiny n=%d %s" % (n, prec_kind), flush=True)
    r = gpu_count(ec, A, prec, xi, eta, V, n)
    ref = oracle.count(A, prec, xi, eta, V, n)
    assert_parity(r, ref)
    s = r.per_probe.cpu().numpy()
    for t, tau in enumerate((xi, eta)):
        Cd = oracle.dense_operator(A, prec, tau)
        ev, U = np.linalg.eigh(0.5 * (Cd + Cd.T))
        Pm = (U * (ev < 0)) @ U.T
        exact = np.einsum("ij,ik,kj->j", V, Pm, V)
        assert np.all(np.abs(s[3 * t:3 * t + 3] - exact) <= 1e-10 * n)


@pytest.mark.parametrize("k", [40, 128])
def test_fp32_form_more_than_one_basis_chunk(ec, k):
    """FP32 storage past one basis chunk (the Gram column with one column per
    lane beyond 24 basis vectors, alpha_i from the launch that holds q_i):
    within the FP32 bound of the FP64 oracle."""
    if k == 40:
        wl = W.WORKLOADS["c2_small"]
        P = W.make_problem(wl)
        V, xi, eta = W.make_probes(wl), wl.xi, wl.eta
    else:
        P, xi, eta = max_k_problem()
        V = W.rademacher(P.A.n, 4, 17)
    r = gpu_count(ec, P.A, P.prec, xi, eta, V, k, vec="f32", val="f32")
    ref = oracle.count(P.A, P.prec, xi, eta, V, k)
    s = r.per_probe.cpu().numpy()
    s_ref = np.concatenate([ref.s_xi, ref.s_eta])
    nu = np.concatenate([ref.lan_xi.nu, ref.lan_eta.nu])
    e_est = rel(r.estimate, ref.estimate)
    e_probe = float(np.max(np.abs(s - s_ref) / nu))
    print("fp32 k=%d: est %.10f oracle %.10f rel %.2e  max|ds|/nu %.2e" % (k, r.estimate, ref.estimate, e_est, e_probe), flush=True)
    assert e_est <= FP32_BOUND
    assert e_probe <= FP32_BOUND


# ---------------------------------------------------------------------------
# Differentiated form: gradient of the erf-smoothed count
# ---------------------------------------------------------------------------

GRAD_CASES = {
    "wells6": W.Workload("wells6", (6, 6, 6), "wells", 1, -160.0, -120.0, "cheb", 6, 8),
    "c2_small": W.WORKLOADS["c2_small"],
    "ragged": W.Workload("ragged", (7, 5, 6), "wells", 4, -120.0, -60.0, "cheb", 9, 10),
}


def grad_setup(ec, name, w=0.05):
    wl = GRAD_CASES[name]
    P = W.make_problem(wl)
    V = W.make_probes(wl)
    Ad = ec.upload_csr(P.A)
    Vd = torch.from_numpy(V).cuda()
    return wl, P, V, Ad, Vd


@pytest.mark.parametrize("name", ["wells6", "c2_small", "ragged"])
def test_smooth_gradient_matches_oracle_tangents(ec, name):
    """<dV, u>, d/dxi and d/deta against the oracle's forward-mode tangents
    (Algorithm 1 differentiated in its literal order), relative 1e-8."""
    w = 0.05
    wl, P, V, Ad, Vd = grad_setup(ec, name, w)
    print("case grad", name, flush=True)
    res, ws = ec.smooth_forward(Ad, P.prec, wl.xi, wl.eta, Vd, wl.k, w)
    ref = oracle.count(P.A, P.prec, wl.xi, wl.eta, V, wl.k, smooth_w=w)
    assert rel(res.estimate, ref.estimate) <= TOL
    dV, dxi, deta = ec.smooth_backward(Ad, P.prec, wl.xi, wl.eta, Vd, wl.k, w, workspace=ws)
    dV = dV.cpu().numpy()
    rng = np.random.default_rng(11)
    for t in range(2):
        u = rng.standard_normal(P.A.n)
        _, d_ref = oracle.count_tangent(P.A, P.prec, wl.xi, wl.eta, V, wl.k, u, 0.0, 0.0, w)
        d_gpu = float(np.dot(dV, u))
        print("  <dV,u> gpu %.12e oracle %.12e" % (d_gpu, d_ref), flush=True)
        assert abs(d_gpu - d_ref) <= 1e-8 * max(abs(d_ref), 1e-12 * np.abs(dV).sum())
    _, dxi_ref = oracle.count_tangent(P.A, P.prec, wl.xi, wl.eta, V, wl.k, np.zeros(P.A.n), 1.0, 0.0, w)
    _, deta_ref = oracle.count_tangent(P.A, P.prec, wl.xi, wl.eta, V, wl.k, np.zeros(P.A.n), 0.0, 1.0, w)
    print("  dxi %.12e / %.12e  deta %.12e / %.12e" % (dxi, dxi_ref, deta, deta_ref), flush=True)
    assert abs(dxi - dxi_ref) <= 1e-8 * max(abs(dxi_ref), 1e-10)
    assert abs(deta - deta_ref) <= 1e-8 * max(abs(deta_ref), 1e-10)


def _grad_vs_oracle(ec, P, xi, eta, V, k, w, seed):
    """Forward per probe at 1e-10 * max(|s_j|, 1) and <dV, u>, dxi, deta
    against the oracle's forward-mode tangents at 1e-8 relative."""
    Ad = ec.upload_csr(P.A)
    Vd = torch.from_numpy(V).cuda()
    res, ws = ec.smooth_forward(Ad, P.prec, xi, eta, Vd, k, w, details=True)
    ref = oracle.count(P.A, P.prec, xi, eta, V, k, smooth_w=w)
    s = res.per_probe.cpu().numpy()
    s_ref = np.concatenate([ref.s_xi, ref.s_eta])
    ds = np.max(np.abs(s - s_ref) / np.maximum(1.0, np.abs(s_ref)))
    print("  estimate gpu %.15f oracle %.15f rel %.2e | max |ds|/max(|s|,1) %.2e"
          % (res.estimate, ref.estimate, rel(res.estimate, ref.estimate), ds), flush=True)
    assert rel(res.estimate, ref.estimate) <= TOL
    assert ds <= TOL
    dV, dxi, deta = ec.smooth_backward(Ad, P.prec, xi, eta, Vd, k, w, workspace=ws)
    dV = dV.cpu().numpy()
    u = np.random.default_rng(seed).standard_normal(P.A.n)
    _, d_ref = oracle.count_tangent(P.A, P.prec, xi, eta, V, k, u, 0.0, 0.0, w)
    _, dxi_ref = oracle.count_tangent(P.A, P.prec, xi, eta, V, k, np.zeros(P.A.n), 1.0, 0.0, w)
    _, deta_ref = oracle.count_tangent(P.A, P.prec, xi, eta, V, k, np.zeros(P.A.n), 0.0, 1.0, w)
    d_gpu = float(np.dot(dV, u))
    print("  <dV,u> gpu %.12e oracle %.12e | dxi %.12e / %.12e | deta %.12e / %.12e"
          % (d_gpu, d_ref, dxi, dxi_ref, deta, deta_ref), flush=True)
    assert abs(d_gpu - d_ref) <= 1e-8 * abs(d_ref)
    assert abs(dxi - dxi_ref) <= 1e-8 * max(abs(dxi_ref), 1e-10)
    assert abs(deta - deta_ref) <= 1e-8 * max(abs(deta_ref), 1e-10)


@pytest.mark.parametrize("k", [30, 32])
def test_smooth_gradient_at_largest_k_several_tiles(ec, k):
    """The differentiated form at the workload's k = 30 and at its limit
    k = 32, with 64 probes (128 columns: two 64-column tiles) on the 16^3
    wells problem."""
    wl = W.Workload("g16", (16, 16, 16), "wells", 1, -8.0, -2.0, "cheb", 64, k, smooth_w=0.05)
    P = W.make_problem(wl)
    print("case grad 16^3 m=64 k=%d" % k, flush=True)
    _grad_vs_oracle(ec, P, wl.xi, wl.eta, W.make_probes(wl), k, 0.05, 21)


def test_smooth_gradient_hard_shift_k32(ec):
    """k = 32, 128 columns, on the n = 640 problem with xi just above the 41st
    eigenvalue (near the bottom of the spectrum, where a Gram-Schmidt pass
    that took alpha_i from the same vector as the other coefficients loses
    orthogonality fastest)."""
    P, xi, eta = max_k_problem()
    V = W.rademacher(P.A.n, 64, 23)
    print("case grad n=640 hard shift k=32", flush=True)
    _grad_vs_oracle(ec, P, xi, eta, V, 32, 0.05, 22)


def test_smooth_gradient_finite_differences_gpu(ec):
    """Central differences of the GPU's own smoothed estimate."""
    w = 0.05
    wl, P, V, Ad, Vd = grad_setup(ec, "wells6", w)
    _, ws = ec.smooth_forward(Ad, P.prec, wl.xi, wl.eta, Vd, wl.k, w)
    dV, dxi, deta = ec.smooth_backward(Ad, P.prec, wl.xi, wl.eta, Vd, wl.k, w, workspace=ws)
    u = np.random.default_rng(5).standard_normal(P.A.n)
    h = 1e-4

    def est(Vpot, xi, eta):
        A2 = ec.upload_csr(W.laplacian_csr(wl.dims, Vpot))
        return ec.smooth_forward(A2, P.prec, xi, eta, Vd, wl.k, w)[0].estimate

    fd = (est(P.V + h * u, wl.xi, wl.eta) - est(P.V - h * u, wl.xi, wl.eta)) / (2 * h)
    g = float(np.dot(dV.cpu().numpy(), u))
    assert abs(fd - g) <= 1e-6 * abs(g) + 1e-8
    fd = (est(P.V, wl.xi + h, wl.eta) - est(P.V, wl.xi - h, wl.eta)) / (2 * h)
    assert abs(fd - dxi) <= 1e-6 * abs(dxi) + 1e-8
    fd = (est(P.V, wl.xi, wl.eta + h) - est(P.V, wl.xi, wl.eta - h)) / (2 * h)
    assert abs(fd - deta) <= 1e-6 * abs(deta) + 1e-8


def test_smooth_keep_and_recompute_agree(ec):
    w = 0.05
    wl, P, V, Ad, Vd = grad_setup(ec, "c2_small", w)
    res, ws = ec.smooth_forward(Ad, P.prec, wl.xi, wl.eta, Vd, wl.k, w)
    cnt = ec.count(Ad, P.prec, wl.xi, wl.eta, Vd, wl.k, smooth_w=w)
    # the differentiated forward is the count's forward (alpha_i first, then
    # the Gram-Schmidt pass): the same kernels, the same estimate
    assert abs(res.estimate - cnt.estimate) <= 1e-15 * abs(cnt.estimate)
    a = ec.smooth_backward(Ad, P.prec, wl.xi, wl.eta, Vd, wl.k, w, g_est=2.0, workspace=ws)
    b = ec.smooth_backward(Ad, P.prec, wl.xi, wl.eta, Vd, wl.k, w, g_est=2.0, ckpt="recompute")
    assert torch.equal(a[0], b[0]) and a[1] == b[1] and a[2] == b[2]
    c = ec.smooth_backward(Ad, P.prec, wl.xi, wl.eta, Vd, wl.k, w, g_est=1.0, ckpt="recompute")
    assert torch.allclose(a[0], 2.0 * c[0], rtol=1e-14, atol=0)


def test_smooth_autograd_function(ec):
    from paper_1602_02306_amd.autograd import SmoothCount, SmoothProblem
    w = 0.05
    wl = GRAD_CASES["wells6"]
    P = W.make_problem(wl)
    V = W.make_probes(wl)
    L = W.laplacian_csr(wl.dims)
    pb = SmoothProblem.from_host(L, P.prec, V, wl.k, w)
    Vt = torch.from_numpy(P.V).cuda().requires_grad_(True)
    xi = torch.tensor(wl.xi, dtype=torch.float64, device="cuda", requires_grad=True)
    eta = torch.tensor(wl.eta, dtype=torch.float64, device="cuda", requires_grad=True)
    out = SmoothCount.apply(Vt, xi, eta, pb)
    (3.0 * out).backward()
    ref = oracle.count(P.A, P.prec, wl.xi, wl.eta, V, wl.k, smooth_w=w)
    assert rel(out.item(), ref.estimate) <= TOL
    u = np.random.default_rng(2).standard_normal(P.A.n)
    _, d_ref = oracle.count_tangent(P.A, P.prec, wl.xi, wl.eta, V, wl.k, u, 0.0, 0.0, w)
    assert abs(float(np.dot(Vt.grad.cpu().numpy(), u)) - 3.0 * d_ref) <= 1e-8 * abs(3.0 * d_ref)


def test_smooth_rejects_unsupported(ec):
    wl = W.WORKLOADS["c1"]
    P = W.make_problem(wl)
    Ad = ec.upload_csr(P.A)
    Vd = torch.from_numpy(W.make_probes(wl)).cuda()
    with pytest.raises(ec.EcntError) as e:
        ec.smooth_forward(Ad, P.prec, wl.xi, wl.eta, Vd, wl.k, 0.05)   # Jacobi M depends on A
    assert e.value.status == ec.ECNT_EUNSUPPORTED


# ---------------------------------------------------------------------------
# A as a grid stencil (a_form auto) against the CSR sweep (a_form csr)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,vec", [("c2_small", "f64"), ("c2_ragged", "f64"), ("c2_ragged", "f32")])
def test_a_stencil_form_equals_csr_form(ec, name, vec):
    """When A is the grid stencil plus a diagonal, the stencil sweep applies it;
    it sums each row as the CSR sweep does, so both forms agree bitwise."""
    wl = W.WORKLOADS[name]
    P = W.make_problem(wl)
    V = W.make_probes(wl)
    print("case a-form", name, vec, flush=True)
    ec.profile_enable(True)
    a = gpu_count(ec, P.A, P.prec, wl.xi, wl.eta, V, wl.k, vec=vec, val=vec)
    prof = ec.profile_read()
    ec.profile_enable(False)
    b = gpu_count(ec, P.A, P.prec, wl.xi, wl.eta, V, wl.k, vec=vec, val=vec, tune={"a_form": "csr"})
    assert prof["op_a_stencil"]["bytes"] > 0 and prof["op_csr"]["bytes"] == 0
    assert a.estimate == b.estimate
    assert torch.equal(a.per_probe, b.per_probe)
    assert torch.equal(a.alpha, b.alpha) and torch.equal(a.beta, b.beta)


def _perturbed(A, rng, how):
    """A copy of A (CSR, both triangles) that is not of the stencil form:
    'coef' scales every symmetric off-diagonal pair by its own factor in
    [0.9, 1.1]; 'extra' adds one symmetric pair of long-range entries."""
    import scipy.sparse as sp
    S = A.to_scipy().tocoo()
    r, c, v = S.row.copy(), S.col.copy(), S.data.copy()
    if how == "coef":
        lo, hi = np.minimum(r, c), np.maximum(r, c)
        f = 1.0 + 0.1 * (2.0 * rng.random(A.n * 8) - 1.0)
        key = (lo * 7919 + hi) % f.size
        v = np.where(r != c, v * f[key], v)
    else:
        i, j = 3, A.n - 5
        r = np.concatenate([r, [i, j]])
        c = np.concatenate([c, [j, i]])
        v = np.concatenate([v, [-0.25, -0.25]])
    M = sp.csr_matrix((v, (r, c)), shape=(A.n, A.n))
    M.sort_indices()
    return W.CSR(A.n, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64))


@pytest.mark.parametrize("how", ["coef", "extra"])
def test_a_not_a_stencil_falls_back_to_csr(ec, how):
    """Variable off-diagonal coefficients, or a coupling outside the stencil:
    the device check rejects the stencil form and the CSR sweep applies A
    (parity with the oracle on the perturbed matrix)."""
    wl = W.WORKLOADS["c2_ragged"]
    P = W.make_problem(wl)
    A2 = _perturbed(P.A, np.random.default_rng(3), how)
    V = W.make_probes(wl)
    print("case a-form fallback", how, flush=True)
    ec.profile_enable(True)
    r = gpu_count(ec, A2, P.prec, wl.xi, wl.eta, V, wl.k)
    prof = ec.profile_read()
    ec.profile_enable(False)
    assert prof["op_csr"]["bytes"] > 0 and prof["op_a_stencil"]["bytes"] == 0
    ref = oracle.count(A2, P.prec, wl.xi, wl.eta, V, wl.k)
    assert_parity(r, ref, wl.k)


def test_hbm_probes_plausible(ec):
    """The stream probes report GB/s between a slow and an impossible rate."""
    for kind in ("copy", "read", "update_mix"):
        g = ec.hbm_probe(kind, 1 << 30, reps=3)
        print("probe", kind, g, flush=True)
        assert 500.0 < g < 9000.0


@pytest.mark.parametrize("prec,k,rule", [("jacobi", 20, "gauss"), ("none", 12, "gauss"),
                                         ("jacobi", 30, "ga"), ("jacobi", 64, "gauss")])
def test_fused_small_form_against_oracle_and_waves(ec, prec, k, rule):
    """c1 (900 rows) runs by default in the one-launch form of small problems
    (M = I or Jacobi, FP64 vectors, k <= 64): against the oracle to the stated
    bar, and against the column-wave kernels (opts.fused = 1), which sum in
    another order, to the same bar.  The profile shows which kernels ran."""
    wl = W.WORKLOADS["c1"]
    P = W.make_problem(wl)
    V = W.make_probes(wl)
    pr = P.prec if prec == "jacobi" else W.PrecSpec("none", ())
    print("case fused", prec, k, rule, flush=True)
    ec.profile_enable(True)
    a = gpu_count(ec, P.A, pr, wl.xi, wl.eta, V, k, rule=rule)
    pa = ec.profile_read()
    ec.profile_enable(True)
    b = gpu_count(ec, P.A, pr, wl.xi, wl.eta, V, k, rule=rule, tune={"fused": "off"})
    pb = ec.profile_read()
    ec.profile_enable(False)
    assert pa["lz_fused"]["launches"] == 1 and pa["lz_dots"]["launches"] == 0
    assert pb["lz_fused"]["launches"] == 0 and pb["lz_dots"]["launches"] >= k
    ref = oracle.count(P.A, pr, wl.xi, wl.eta, V, k, rule=rule)
    scale = "nu" if k >= 40 else "rel"
    assert_parity(a, ref, k, probe_scale=scale)
    assert_parity(b, ref, k, probe_scale=scale)
    assert np.array_equal(a.k_used.cpu().numpy(), b.k_used.cpu().numpy())
    sa, sb = a.per_probe.cpu().numpy(), b.per_probe.cpu().numpy()
    bound = TOL * (np.maximum(1.0, np.abs(sb)) if scale == "rel" else
                   np.concatenate([ref.lan_xi.nu, ref.lan_eta.nu]))
    assert np.all(np.abs(sa - sb) <= bound)


@pytest.mark.parametrize("side,fused", [(40, True), (44, False)])
def test_fused_form_lds_limit(ec, side, fused):
    """The one-launch form holds a column's operator, q and w in LDS (at most
    150 KiB: 28 bytes per row and 12 per nonzero): a 40 x 40 five-point
    operator (1600 rows, 136 KiB) runs in it, 44 x 44 (1936 rows, 164 KiB) in
    the column waves.  Both against the oracle, Jacobi, k = 24."""
    rng = np.random.default_rng(side)
    A = W.laplacian_csr((side, side), rng.uniform(0.0, 1.0, side * side))
    prec = W.PrecSpec("jacobi", ())
    V = W.rademacher(A.n, 8, 77)
    print("case fused limit", side, flush=True)
    ec.profile_enable(True)
    r = gpu_count(ec, A, prec, 0.5, 1.5, V, 24)
    prof = ec.profile_read()
    ec.profile_enable(False)
    assert (prof["lz_fused"]["launches"] == 1) == fused
    assert (prof["lz_dots"]["launches"] > 0) == (not fused)
    ref = oracle.count(A, prec, 0.5, 1.5, V, 24)
    assert_parity(r, ref, 24)
