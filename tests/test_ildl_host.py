"""Host side of the ILDL preconditioner: the library's factorization
(ecnt_ildl_factor, sparse rows) against the oracle's (dense), argument
checks, and the validation of LDL factors before any device work."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1602_02306_amd import ecount as ec
from paper_1602_02306_amd import workloads as W


def scaled_laplacian(dims, scale):
    A = W.laplacian_csr(dims)
    A.val = A.val * scale
    return A


def random_indefinite(n, band, density, seed):
    rng = np.random.default_rng(seed)
    K = np.zeros((n, n))
    for i in range(n):
        for j in range(max(0, i - band), i):
            if rng.random() < density:
                K[i, j] = K[j, i] = rng.standard_normal()
        K[i, i] = 0.2 * rng.standard_normal()
    rp, ci, va = [0], [], []
    for i in range(n):
        nz = np.nonzero(K[i])[0]
        ci += list(nz)
        va += list(K[i, nz])
        rp.append(len(ci))
    return W.CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va)), K


CASES = [
    ("laplace_9x7", lambda: W.laplacian_csr((9, 7)), 2.5),
    ("laplace_31", lambda: scaled_laplacian((31, 31), 1024.0), 300.0),
    ("random", lambda: random_indefinite(300, 12, 0.3, 11)[0], 0.05),
]


@pytest.mark.parametrize("name,make,tau", CASES)
@pytest.mark.parametrize("t", [0.0, 1e-6, 1e-3, 1e-1])
def test_library_factor_equals_oracle_bitwise(name, make, tau, t):
    """Both follow the same elimination, pivot and drop rules with the same
    per-entry update order, so the factors agree to the last bit."""
    A = make()
    H = ec.ildl_factor(A, tau, t)
    F = oracle.ildl(A, tau, t)
    assert np.array_equal(H.perm, F.perm)
    assert np.array_equal(H.l_rp, F.l_rp)
    assert np.array_equal(H.l_ci, F.l_ci)
    assert np.array_equal(H.l_val, F.l_val)
    assert np.array_equal(H.d_diag, F.d_diag)
    assert np.array_equal(H.d_off, F.d_off)
    rows = np.repeat(np.arange(A.n), np.diff(H.l_rp))
    assert H.bandwidth == (int(np.max(rows - H.l_ci)) if len(H.l_ci) else 0)
    assert H.n2x2 == int(np.count_nonzero(H.d_off))


def test_library_inertia_count():
    A, K = random_indefinite(200, 10, 0.3, 4)
    H = ec.ildl_factor(A, 0.1, 0.0)
    assert H.nneg == int(np.sum(np.linalg.eigvalsh(K - 0.1 * np.eye(200)) < 0))


def test_structurally_unsymmetric_input_is_symmetrized():
    """An explicit zero stored in one triangle only does not change the factor."""
    A = W.laplacian_csr((6, 5))
    K = np.zeros((A.n, A.n))
    for i in range(A.n):
        for p in range(A.row_ptr[i], A.row_ptr[i + 1]):
            K[i, A.col_idx[p]] = A.val[p]
    rp, ci, va = [0], [], []
    for i in range(A.n):
        cols = list(np.nonzero(K[i])[0])
        if i + 7 < A.n:
            cols.append(i + 7)   # explicit zero above the diagonal only
        cols.sort()
        ci += cols
        va += [K[i, c] for c in cols]
        rp.append(len(ci))
    B = W.CSR(A.n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va))
    Ha, Hb = ec.ildl_factor(A, 3.1, 0.0), ec.ildl_factor(B, 3.1, 0.0)
    assert np.array_equal(Ha.perm, Hb.perm)
    assert np.array_equal(Ha.d_diag, Hb.d_diag)


def test_ildl_rejects_bad_arguments():
    lib = ec.load()
    A = W.laplacian_csr((4, 4))
    rp = np.ascontiguousarray(A.row_ptr, np.int32)
    ci = np.ascontiguousarray(A.col_idx, np.int32)
    va = np.ascontiguousarray(A.val)
    h = ctypes.c_void_p()
    for args, code in [((0, rp, ci, va, 0.0, 0.0), ec.ECNT_EINVAL),
                       ((A.n, rp, ci, va, float("nan"), 0.0), ec.ECNT_EINVAL),
                       ((A.n, rp, ci, va, 0.0, -1.0), ec.ECNT_EINVAL)]:
        n, a, b, c, tau, t = args
        rc = lib.ecnt_ildl_factor(n, a.ctypes.data, b.ctypes.data, c.ctypes.data, tau, t,
                                  ctypes.byref(h))
        assert rc == code, ec.last_error()
    bad = ci.copy()
    bad[3] = 99
    rc = lib.ecnt_ildl_factor(A.n, rp.ctypes.data, bad.ctypes.data, va.ctypes.data, 0.0, 0.0,
                              ctypes.byref(h))
    assert rc == ec.ECNT_EINVAL
    # a zero matrix has only zero pivots
    z = W.CSR(3, np.array([0, 1, 2, 3], np.int32), np.array([0, 1, 2], np.int32), np.zeros(3))
    with pytest.raises(ec.EcntError) as e:
        ec.ildl_factor(z, 0.0, 0.0)
    assert e.value.status == ec.ECNT_ENOTHPD


def _fake_factor(bandwidth, nnz=10):
    return ec.LdlFactorT(*([0x1000] * 6), nnz, bandwidth, 0)


class _FakePrec:
    kind = "ldl"

    def __init__(self, fs):
        self.factors = fs


class _F:
    def __init__(self, st):
        self.st = st

    def struct(self):
        return self.st


@pytest.mark.parametrize("bw,nfac,code", [(300, 1, ec.ECNT_EUNSUPPORTED), (-1, 1, ec.ECNT_EINVAL),
                                          (10, 1, ec.ECNT_OK)])
def test_ldl_factor_validated_on_host(bw, nfac, code):
    lib = ec.load()
    cs = ec.CsrT(1000, 5000, 0x3000, 0x4000, 0x5000, 0, 0)
    prec = _FakePrec([_F(_fake_factor(bw)) for _ in range(nfac)])
    ps, keep = ec.prec_struct(prec)
    o = ec.opts_struct(3)
    taus = np.array([0.5])
    out = np.zeros(1)
    if code == ec.ECNT_OK:
        # a valid description sizes its workspace (two scratch blocks, |D|^-1/2)
        assert lib.ecnt_workspace_bytes(1000, 4, 1, ctypes.byref(ps), ctypes.byref(o)) > 0
        return
    rc = lib.ecnt_negcounts(ctypes.byref(cs), ctypes.byref(ps), taus.ctypes.data, 1, 0x1000, 4,
                            ctypes.byref(o), 0x2000, 1 << 40, None, out.ctypes.data, None, None,
                            None)
    assert rc == code, ec.last_error()


def test_ldl_null_factor_array_rejected():
    lib = ec.load()
    cs = ec.CsrT(1000, 5000, 0x3000, 0x4000, 0x5000, 0, 0)
    ps = ec.PrecT(3, 0, (ctypes.c_int32 * 3)(0, 0, 0), 0, 0, 0.0, 0.0, 0.0, None, None)
    o = ec.opts_struct(3)
    taus = np.array([0.5])
    out = np.zeros(1)
    rc = lib.ecnt_negcounts(ctypes.byref(cs), ctypes.byref(ps), taus.ctypes.data, 1, 0x1000, 4,
                            ctypes.byref(o), 0x2000, 1 << 40, None, out.ctypes.data, None, None,
                            None)
    assert rc == ec.ECNT_EINVAL


def test_ldl_batches_rejected():
    lib = ec.load()
    cs = ec.CsrT(128, 640, 0x3000, 0x4000, 0x5000, 0, 0)
    prec = _FakePrec([_F(_fake_factor(10))])
    ps, keep = ec.prec_struct(prec)
    o = ec.opts_struct(3)
    taus = [np.array([0.5]), np.array([0.5])]
    items = (ec.BatchItemT * 2)()
    for b in range(2):
        items[b] = ec.BatchItemT(64, (ctypes.c_int32 * 3)(1, 1, 64), 0, taus[b].ctypes.data)
    assert lib.ecnt_batch_workspace_bytes(items, 2, 1, 4, ctypes.byref(ps), ctypes.byref(o)) == 0
    assert "LDL" in ec.last_error()
