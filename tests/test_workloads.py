"""The seeded input builders (no arithmetic of the method lives there)."""
import numpy as np

from paper_1602_02306_amd import workloads as W


def test_laplacian_csr_matches_dense_kron():
    for dims in [(5,), (4, 6), (3, 4, 5)]:
        A = W.laplacian_csr(dims).to_dense()
        Ts = [2.0 * np.eye(d) - np.eye(d, k=1) - np.eye(d, k=-1) for d in dims]
        ref = np.zeros_like(A)
        for a in range(len(dims)):
            term = np.ones((1, 1))
            for b in range(len(dims)):
                term = np.kron(term, Ts[b] if a == b else np.eye(dims[b]))
            ref += term
        assert np.array_equal(A, ref)


def test_csr_sorted_with_diagonal():
    A = W.laplacian_csr((7, 3, 5), np.arange(105.0))
    for r in range(A.n):
        cols = A.col_idx[A.row_ptr[r]:A.row_ptr[r + 1]]
        assert np.all(np.diff(cols) > 0) and r in cols
    assert A.nnz == 7 * 105 - 2 * (3 * 5 + 7 * 5 + 7 * 3)


def test_rademacher_counter_based_and_torch_identical():
    import torch
    a = W.rademacher(3000, 9, 77)
    assert set(np.unique(a)) == {-1.0, 1.0}
    # entry (r, j) depends only on (seed, j, r): a sub-block regenerates identically
    assert np.array_equal(W.rademacher(3000, 9, 77)[:, 4], a[:, 4])
    b = W.rademacher_torch(3000, 9, 77, device="cpu").numpy()
    assert np.array_equal(a, b)
    assert abs(a.mean()) < 0.05


def test_hadamard_and_identity_probes_resolve_identity():
    for V in (W.hadamard_probes(16), W.identity_probes(16)):
        assert np.allclose(V @ V.T, 16 * np.eye(16))


def test_chebyshev_interpolant_nodes():
    c = W.cheb_interp_coeffs(lambda x: x ** -0.5, 1.0, 13.0, 4)
    k = np.arange(5)
    t = np.cos(np.pi * (k + 0.5) / 5)
    x = 7.0 + 6.0 * t
    assert np.allclose(np.polynomial.chebyshev.chebval(t, c), x ** -0.5, rtol=1e-13)


def test_wells_reading():
    rng = np.random.default_rng(1)
    V = W.gaussian_wells((10, 11, 12), rng)
    rng = np.random.default_rng(1)
    cen = rng.uniform(0, 1, size=(32, 3)) * (np.array([10, 11, 12]) - 1.0)
    dep = rng.uniform(5, 15, size=32)
    x, y, z = 3, 7, 2
    r = (x * 11 + y) * 12 + z
    ref = -np.sum(dep * np.exp(-((cen - [x, y, z]) ** 2).sum(1) / 18.0))
    assert abs(V[r] - ref) < 1e-12


def test_batched_item_draws():
    it = W.batched_item(5)
    assert 16 <= it.dims[0] <= 64 and it.dims[0] == it.dims[1] == it.dims[2]
    assert np.all(np.diff(it.shifts) > 0) and it.shifts[0] >= -8 and it.shifts[-1] <= -2
