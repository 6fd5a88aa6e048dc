"""GPU parity of the block-Lanczos form (blocks of 16 probes, block Gauss
rule) against the block oracle on the same seeded probes.

The GPU orthonormalizes each block by Cholesky QR applied twice and keeps the
basis as X_l with Q_l = X_l S_l; the oracle uses Householder QR with a
positive diagonal.  Both give the same basis up to rounding (the positive-
diagonal QR is unique), so the tolerances are those of the Lanczos parity
tests: the estimate within 1e-10 * max(|ref|, 1) and every per-probe value
within 1e-10 * max(|s_j|, 1).
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


def prec_of(kind, dims):
    if kind == "cheb":
        return W.cheb_invsqrt_prec(dims)
    return W.PrecSpec(kind, ())


def run(ec, A, prec, xi, eta, V, k, **kw):
    Ad = ec.upload_csr(A)
    Vd = torch.from_numpy(np.ascontiguousarray(V)).to("cuda", torch.float64)
    return ec.count_block(Ad, prec, xi, eta, Vd, k, **kw)


def check(r, ref, n, tol=TOL):
    s = r.per_probe.cpu().numpy()
    s_ref = np.concatenate([ref.s_xi, ref.s_eta])
    d = np.max(np.abs(s - s_ref) / np.maximum(1.0, np.abs(s_ref)))
    print("gpu %.15f oracle %.15f | max |ds|/max(|s|,1) %.2e" % (r.estimate, ref.estimate, d), flush=True)
    assert abs(r.estimate - ref.estimate) <= tol * max(1.0, abs(ref.estimate))
    assert d <= tol
    assert abs(r.neg_xi - ref.neg_xi) <= tol * max(1.0, abs(ref.neg_xi))
    assert abs(r.neg_eta - ref.neg_eta) <= tol * max(1.0, abs(ref.neg_eta))


def kused_ref(ref, m):
    ku = [np.repeat(x.k_used, 16) for x in (ref.lan_xi, ref.lan_eta)]
    return np.concatenate(ku)


@pytest.mark.parametrize("kind", ["cheb", "none", "jacobi"])
@pytest.mark.parametrize("name", ["c2_small", "c2_ragged"])
def test_block_parity(ec, name, kind):
    wl = W.WORKLOADS[name]
    P = W.make_problem(wl)
    prec = prec_of(kind, wl.dims) if kind != "cheb" else P.prec
    V = W.rademacher(P.A.n, 32, 5)
    print("block parity", name, kind, P.A.n, flush=True)
    r = run(ec, P.A, prec, wl.xi, wl.eta, V, wl.k)
    ref = oracle.block_count(P.A, prec, wl.xi, wl.eta, V, wl.k)
    check(r, ref, P.A.n)
    assert np.array_equal(r.k_used.cpu().numpy(), kused_ref(ref, 32))


def test_block_column_waves_and_basis_chunks(ec):
    """k = 20 (three launches of at most 8 basis blocks per Gram-Schmidt pass)
    and column waves of one block each."""
    wl = W.WORKLOADS["c2_ragged"]
    P = W.make_problem(wl)
    V = W.rademacher(P.A.n, 32, 8)
    ref = oracle.block_count(P.A, P.prec, wl.xi, wl.eta, V, 20)
    print("block waves/chunks", flush=True)
    r = run(ec, P.A, P.prec, wl.xi, wl.eta, V, 20)
    check(r, ref, P.A.n, tol=1e-9)
    r = run(ec, P.A, P.prec, wl.xi, wl.eta, V, 20, max_cols=16)
    check(r, ref, P.A.n, tol=1e-9)


def test_block_smoothed_step(ec):
    wl = W.WORKLOADS["c2_small"]
    P = W.make_problem(wl)
    V = W.rademacher(P.A.n, 16, 3)
    ref = oracle.block_count(P.A, P.prec, wl.xi, wl.eta, V, wl.k, smooth_w=0.3)
    print("block smoothed", flush=True)
    r = run(ec, P.A, P.prec, wl.xi, wl.eta, V, wl.k, smooth_w=0.3)
    check(r, ref, P.A.n)


def test_block_exhausted_space_is_exact(ec):
    """n = 48, identity probes (3 blocks): the fourth residual vanishes,
    k_used = 3 and the counts are the exact inertias."""
    wl = W.Workload("t", (4, 4, 3), "wells", 7, -5.0, 1.0, "cheb", 4, 4)
    P = W.make_problem(wl)
    n = P.A.n
    lam = np.sort(np.linalg.eigvalsh(P.A.to_dense()))
    xi, eta = 0.5 * (lam[5] + lam[6]), 0.5 * (lam[30] + lam[31])
    V = W.identity_probes(n)
    print("block exhausted", flush=True)
    r = run(ec, P.A, P.prec, xi, eta, V, 5)
    ref = oracle.block_count(P.A, P.prec, xi, eta, V, 5)
    assert np.all(r.k_used.cpu().numpy() == 3)
    check(r, ref, n, tol=1e-9)
    assert abs(r.neg_xi - 6.0) < 1e-8 and abs(r.neg_eta - 31.0) < 1e-8
    assert abs(r.estimate - 25.0) < 1e-8


def test_block_several_tiles_ragged_tail(ec):
    """30,690 rows (a ragged last tile of 2 rows in each row chunk's grid),
    4 blocks per shift, k = 10."""
    wl = W.Workload("b", (33, 31, 30), "wells", 1, -8.0, -2.0, "cheb", 64, 10)
    P = W.make_problem(wl)
    V = W.rademacher(P.A.n, 64, 21)
    print("block tiles", P.A.n, flush=True)
    r = run(ec, P.A, P.prec, wl.xi, wl.eta, V, wl.k)
    ref = oracle.block_count(P.A, P.prec, wl.xi, wl.eta, V, wl.k)
    check(r, ref, P.A.n)


def test_block_bench_configuration_sampled(ec):
    """The c2_blk bench configuration (64^3, m = 256, k = 30, both shifts in one
    wave, default launch shapes): the first probe block against the oracle,
    per probe and k_used; the estimate is the mean of the per-probe values."""
    wl = W.WORKLOADS["c2_blk"]
    P = W.make_problem(wl)
    Vd = W.rademacher_torch(wl.n, wl.m, wl.probe_seed, device="cuda", dtype=torch.float64)
    print("block bench configuration", wl.n, wl.m, wl.k, flush=True)
    r = ec.count_block(ec.upload_csr(P.A), P.prec, wl.xi, wl.eta, Vd, wl.k)
    s = r.per_probe.cpu().numpy()
    V0 = Vd[:, :16].cpu().numpy()
    ref = oracle.block_count(P.A, P.prec, wl.xi, wl.eta, V0, wl.k)
    d = max(np.max(np.abs(s[:16] - ref.s_xi) / np.maximum(1.0, np.abs(ref.s_xi))),
            np.max(np.abs(s[wl.m:wl.m + 16] - ref.s_eta) / np.maximum(1.0, np.abs(ref.s_eta))))
    print("sampled block: max |ds|/max(|s|,1) %.2e" % d, flush=True)
    assert d <= TOL
    ku = r.k_used.cpu().numpy()
    assert np.all(ku[:16] == ref.lan_xi.k_used[0]) and np.all(ku[wl.m:wl.m + 16] == ref.lan_eta.k_used[0])
    mean = np.mean(s[wl.m:]) - np.mean(s[:wl.m])
    assert abs(r.estimate - mean) <= 1e-12 * max(1.0, abs(mean))


def test_block_ragged_last_column_wave(ec):
    """m = 48 probes (96 columns) in waves of 64: the last wave holds 2 blocks."""
    wl = W.WORKLOADS["c2_ragged"]
    P = W.make_problem(wl)
    V = W.rademacher(P.A.n, 48, 13)
    ref = oracle.block_count(P.A, P.prec, wl.xi, wl.eta, V, wl.k)
    print("block ragged wave", flush=True)
    r = run(ec, P.A, P.prec, wl.xi, wl.eta, V, wl.k, max_cols=64)
    check(r, ref, P.A.n)
    assert np.array_equal(r.k_used.cpu().numpy(), kused_ref(ref, 48))


def test_block_maximum_k(ec):
    """k = 32, the largest block count of steps: T_k of order 512 (the
    quadrature's largest band matrix) on n = 640."""
    wl = W.Workload("t", (10, 8, 8), "wells", 3, -5.0, 1.0, "cheb", 16, 32)
    P = W.make_problem(wl)
    lam = np.sort(np.linalg.eigvalsh(P.A.to_dense()))
    xi, eta = 0.5 * (lam[40] + lam[41]), 0.5 * (lam[300] + lam[301])
    V = W.rademacher(P.A.n, 16, 19)
    ref = oracle.block_count(P.A, P.prec, xi, eta, V, 32)
    assert ref.lan_xi.k_used[0] == 32 and ref.lan_eta.k_used[0] == 32
    print("block maximum k", flush=True)
    r = run(ec, P.A, P.prec, xi, eta, V, 32)
    check(r, ref, P.A.n)
    assert np.all(r.k_used.cpu().numpy() == 32)
