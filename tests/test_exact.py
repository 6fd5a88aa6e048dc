"""Exact eigenvalue counts: closed form, dense, sparse LDL^T and plane-wise
inertia agree, and reproduce the paper's printed exact count."""
import json
import os

import numpy as np
import pytest

from oracle import exact
from paper_1602_02306_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_table1_laplace_exact_count():
    """Table 1: Laplace, h = 2^-7, n = 16129, n_(A - 3000 I) = 226."""
    g = json.load(open(os.path.join(GOLDEN, "paper_table1.json")))["laplace"]
    assert g["grid"][0] * g["grid"][1] == g["n"]
    assert exact.laplacian_negcount(g["grid"], g["tau"], h=g["h"]) == g["exact_negcount"]
    A = W.laplacian_csr(g["grid"]).to_scipy() / g["h"] ** 2
    assert exact.sparse_negcount(A, g["tau"]) == g["exact_negcount"]


def test_closed_form_matches_dense():
    for dims in [(7,), (5, 6), (4, 3, 5)]:
        L = W.laplacian_csr(dims).to_dense()
        assert np.allclose(np.sort(exact.laplacian_eigenvalues(dims)), np.linalg.eigvalsh(L),
                           atol=1e-12)


@pytest.mark.parametrize("N", [6, 9])
def test_inertia_methods_agree(N):
    wl = W.Workload("t", (N, N, N), "wells", 1, -8.0, -2.0, "cheb", 1, 1)
    P = W.make_problem(wl)
    Ad = P.A.to_dense()
    for tau in (-8.0, -2.0, -20.0):
        d = exact.dense_negcount(Ad, tau)
        assert exact.sparse_negcount(P.A.to_scipy(), tau) == d
        assert exact.planewise_negcount(P.dims, P.V, tau) == d


@pytest.mark.parametrize("dims,leaves", [((6, 6, 6), (4, 10 ** 6)), ((9, 8, 11), (40,)),
                                         ((13, 11, 9), (64,)), ((2, 17, 3), (4, 10 ** 6))])
def test_nested_dissection_inertia_matches_dense(dims, leaves):
    """The multifrontal nested-dissection LDL^T count equals the dense
    eigenvalue count, with leaf boxes small enough that every kind of front
    (separator with ancestors on several faces, a ragged split, a leaf) occurs,
    and with the whole grid as one leaf."""
    wl = W.Workload("t", dims, "wells", 3, -8.0, -2.0, "cheb", 1, 1)
    P = W.make_problem(wl)
    lam = np.linalg.eigvalsh(P.A.to_dense())
    for tau in (-30.0, -8.0, -2.0, 0.5, 7.0, 20.0):
        d = int(np.sum(lam < tau))
        for leaf in leaves:
            assert exact.nd_negcount(P.dims, P.V, tau, leaf=leaf) == d, (tau, leaf)


def test_nested_dissection_closed_form():
    """V = 0: the count of the Dirichlet Laplacian below tau from its
    closed-form spectrum."""
    dims = (14, 12, 13)
    lam = np.sort(exact.laplacian_eigenvalues(dims))
    for tau in (0.37, 2.0, 6.05, 11.3):
        assert exact.nd_negcount(dims, np.zeros(int(np.prod(dims))), tau) == int(np.sum(lam < tau))


def test_stored_exact_counts_small():
    data = json.load(open(os.path.join(GOLDEN, "exact_counts.json")))
    for name in ("c1", "c2_small", "c2_ragged"):
        wl = W.WORKLOADS[name]
        Ad = W.make_problem(wl).A.to_dense()
        assert data[name]["count"] == exact.dense_negcount(Ad, wl.eta) - exact.dense_negcount(Ad, wl.xi)
    assert data["c1"]["count"] == 72


def test_stored_batch_exact_counts_consistent():
    """The 64 stored counts of the batched family: each item's grid and shifts
    are those the generator draws for it, its slice counts are differences of
    its stored inertia counts, and the smallest item (16^3) recomputes by the
    dense eigenvalue count."""
    data = json.load(open(os.path.join(GOLDEN, "exact_counts.json")))["c4"]
    items = data["items"]
    assert [it["problem"] for it in items] == list(range(64))
    for it in items:
        B = W.batched_item(it["problem"], base_seed=data["base_seed"])
        assert list(B.dims) == it["dims"]
        np.testing.assert_array_equal(np.asarray(it["shifts"]), B.shifts)
        neg = it["negcounts"]
        assert it["counts"] == [neg[i + 1] - neg[i] for i in range(len(neg) - 1)]
        assert all(c >= 0 for c in it["counts"])
    small = min(items, key=lambda it: it["dims"][0])
    B = W.batched_item(small["problem"], base_seed=data["base_seed"])
    lam = np.linalg.eigvalsh(B.A.to_dense())
    assert small["negcounts"] == [int(np.sum(lam < t)) for t in B.shifts]
