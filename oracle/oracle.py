"""Oracle for the preconditioned Lanczos eigenvalue-count estimator.

TEST INFRASTRUCTURE ONLY.  A plain FP64 CPU implementation, written from the
paper (Vecharynski & Yang, "Preconditioned iterative methods for eigenvalue
counts"), against which the GPU library is checked.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may use it; the product path
never does.  It shares no code with the GPU library: the Lanczos recurrence
lives in `lanczos_oracle.c` (plain C, built with gcc), the quadrature below
uses numpy's dense symmetric eigensolver.

Estimator (one shift tau; Section 3.2, eq. rand_prec_quad and Algorithm 2):
    s_j(tau) = |v_j|^2 * sum_{i : theta_i < 0} z_i(1)^2
where theta_i, z_i are the eigenpairs of the k x k Lanczos matrix J_k of
probe v_j (Section 3.1, eq. gauss_quad), and
    n_(A - tau I) ~ (1/m) sum_j s_j(tau).
Interval count (end of Section 3.2): c(xi, eta) = n_(A - eta I) - n_(A - xi I),
run on the same probe block for both shifts.

Generalized averaged Gauss rule (Section 3.4, eq. GA_Tk): J_k is replaced by
the (2k-1) x (2k-1) tridiagonal matrix with diagonal
(alpha_1..alpha_k, alpha_{k-1}..alpha_1) and off-diagonal
(beta_2..beta_k, beta_{k+1}, beta_{k-1}..beta_2).

Readings where the paper is silent (each listed in the design notes):
  * the returned count is the unrounded mean (the brackets of Algorithm 2's
    last step are display rounding);
  * `variance` is the sample variance of the per-probe differences
    d_j = s_j(eta) - s_j(xi) divided by m (NaN for m = 1);
  * h(0) = 0 (strict theta < 0, eq. h), so the count is #{xi <= lambda < eta};
  * smooth_w > 0 replaces h(theta) by S_w(theta) = erfc(theta / w) / 2
    (an erf-smoothed step; w -> 0 recovers the paper's estimator).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lanczos_oracle.c")
_SRC_ILDL = os.path.join(_HERE, "ildl_oracle.c")
_LIB = os.path.join(_HERE, "liblanczos_oracle.so")
_lib = None

PREC_KINDS = {"none": 0, "jacobi": 1, "cheb": 2, "ildl": 3}


def build(force: bool = True) -> str:
    """Compile the C half of the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-Wall", "-o", tmp, _SRC, _SRC_ILDL, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_lanczos.restype = ctypes.c_int
        lib.oracle_lanczos.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int, ctypes.c_int, P,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int, P, ctypes.c_double, P, ctypes.c_int64,
                                       ctypes.c_int, ctypes.c_int, P, P, P, P]
        lib.oracle_dense_operator.restype = ctypes.c_int
        lib.oracle_dense_operator.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int, ctypes.c_int,
                                              P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_int, P, ctypes.c_double, P]
        lib.oracle_lanczos_tangent.restype = ctypes.c_int
        lib.oracle_lanczos_tangent.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int, ctypes.c_int,
                                               P, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_int, P, ctypes.c_double,
                                               P, ctypes.c_double, P, ctypes.c_int64, ctypes.c_int,
                                               ctypes.c_int, P, P, P, P, P, P]
        lib.oracle_arnoldi.restype = ctypes.c_int
        lib.oracle_arnoldi.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int, ctypes.c_int, P,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int, P, ctypes.c_double, P, ctypes.c_int64,
                                       ctypes.c_int, ctypes.c_int, P, P, P]
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_apply_operator.restype = ctypes.c_int
        lib.oracle_apply_operator.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int, ctypes.c_int,
                                              P, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_int, P, ctypes.c_double,
                                              P, ctypes.c_int64, ctypes.c_int, P]
        PP = ctypes.POINTER(ctypes.c_void_p)
        lib.oracle_ildl.restype = ctypes.c_int
        lib.oracle_ildl.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_double, ctypes.c_double,
                                    P, P, P, ctypes.POINTER(ctypes.c_int64), PP, PP, PP]
        lib.oracle_free.restype = None
        lib.oracle_free.argtypes = [ctypes.c_void_p]
        lib.oracle_lanczos_ldl.restype = ctypes.c_int
        lib.oracle_lanczos_ldl.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_double, P, P, P, P,
                                           P, P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                           P, P, P, P]
        lib.oracle_dense_operator_ldl.restype = ctypes.c_int
        lib.oracle_dense_operator_ldl.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_double, P, P,
                                                  P, P, P, P, P]
        lib.oracle_abs_invsqrt_blocks.restype = ctypes.c_int
        lib.oracle_abs_invsqrt_blocks.argtypes = [ctypes.c_int64, P, P, P, P]
        _lib = lib
    return _lib


def host_threads() -> int:
    return len(os.sched_getaffinity(0))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _prec_args(prec, n):
    kind = PREC_KINDS[prec.kind]
    dims = np.zeros(3, dtype=np.int32)
    nd = len(prec.dims) if prec.dims else 0
    dims[:nd] = prec.dims
    if kind == 2:
        coef = np.ascontiguousarray(prec.coef, dtype=np.float64)
        if int(np.prod(prec.dims)) != n:
            raise ValueError("preconditioner grid does not match n")
    else:
        coef = np.zeros(1)
    return kind, nd, dims, coef


# ---------------------------------------------------------------------------
# ILDL(t) preconditioner of one shift (Section 6)
# ---------------------------------------------------------------------------


@dataclass
class ILDLFactor:
    """P (A - tau I) P^T ~ L D L^T.  perm[i]: the row of A - tau I placed at
    row i; L strictly lower (unit diagonal implied) in CSR (l_rp, l_ci, l_val);
    D block diagonal: d_diag, and d_off[i] = D_{i+1,i} at the first row of a
    2 x 2 block (0 elsewhere)."""
    perm: np.ndarray
    l_rp: np.ndarray
    l_ci: np.ndarray
    l_val: np.ndarray
    d_diag: np.ndarray
    d_off: np.ndarray

    @property
    def n(self) -> int:
        return len(self.perm)

    def dense_L(self) -> np.ndarray:
        n = self.n
        L = np.eye(n)
        for i in range(n):
            for p in range(self.l_rp[i], self.l_rp[i + 1]):
                L[i, self.l_ci[p]] = self.l_val[p]
        return L

    def dense_D(self) -> np.ndarray:
        D = np.diag(self.d_diag)
        for i in np.nonzero(self.d_off)[0]:
            D[i + 1, i] = D[i, i + 1] = self.d_off[i]
        return D

    def bandwidth(self) -> int:
        rows = np.repeat(np.arange(self.n), np.diff(self.l_rp))
        return int(np.max(rows - self.l_ci)) if len(self.l_ci) else 0


def _csr_args(A):
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
    va = np.ascontiguousarray(A.val, dtype=np.float64)
    return rp, ci, va


def ildl(A, tau: float, droptol: float) -> ILDLFactor:
    """ILDL(t) of A - tau I with Bunch-Kaufman pivoting (oracle_ildl in
    ildl_oracle.c: natural order, dense right-looking)."""
    lib = _load()
    n = A.n
    rp, ci, va = _csr_args(A)
    perm = np.zeros(n, dtype=np.int32)
    dd = np.zeros(n)
    do = np.zeros(n)
    nnz = ctypes.c_int64(0)
    prp, pci, pval = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    rc = lib.oracle_ildl(n, _ptr(rp), _ptr(ci), _ptr(va), float(tau), float(droptol), _ptr(perm),
                         _ptr(dd), _ptr(do), ctypes.byref(nnz), ctypes.byref(prp),
                         ctypes.byref(pci), ctypes.byref(pval))
    if rc == -3:
        raise ZeroDivisionError("ILDL: zero pivot (A - tau I singular in the factorization)")
    if rc != 0:
        raise ValueError("oracle_ildl failed (%d)" % rc)
    try:
        nz = int(nnz.value)
        l_rp = np.ctypeslib.as_array(ctypes.cast(prp, ctypes.POINTER(ctypes.c_int32)), (n + 1,)).copy()
        l_ci = np.ctypeslib.as_array(ctypes.cast(pci, ctypes.POINTER(ctypes.c_int32)), (max(nz, 1),))[:nz].copy()
        l_val = np.ctypeslib.as_array(ctypes.cast(pval, ctypes.POINTER(ctypes.c_double)), (max(nz, 1),))[:nz].copy()
    finally:
        for p in (prp, pci, pval):
            lib.oracle_free(p)
    return ILDLFactor(perm, l_rp, l_ci, l_val, dd, do)


def abs_invsqrt_blocks(F: ILDLFactor):
    """|D|^(-1/2) by blocks as the oracle forms it: (e_diag, e_off)."""
    lib = _load()
    n = F.n
    ed = np.zeros(n)
    eo = np.zeros(n)
    dd = np.ascontiguousarray(F.d_diag)
    do = np.ascontiguousarray(F.d_off)
    lib.oracle_abs_invsqrt_blocks(n, _ptr(dd), _ptr(do), _ptr(ed), _ptr(eo))
    return ed, eo


def _ldl_args(F: ILDLFactor):
    return [np.ascontiguousarray(a) for a in (F.perm, F.l_rp, F.l_ci, F.l_val, F.d_diag, F.d_off)]


@dataclass
class LanczosResult:
    alpha: np.ndarray   # m x k
    beta: np.ndarray    # m x (k+1), beta[:, 0] = beta_1 = 0
    k_used: np.ndarray  # m
    nu: np.ndarray      # m, |v_j|^2


def lanczos(A, prec, tau: float, V: np.ndarray, k: int, nthreads: int | None = None) -> LanczosResult:
    """Algorithm 1 on C = M (A - tau I) M^* for every column of V (n x m).
    For prec.kind == 'ildl' the factor of this shift is built first (ildl)."""
    lib = _load()
    V = np.ascontiguousarray(V, dtype=np.float64)
    n, m = V.shape
    if A.n != n:
        raise ValueError("probe block does not match A")
    if prec.kind == "ildl":
        return lanczos_ldl(A, ildl(A, tau, prec.droptol), tau, V, k, nthreads)
    kind, nd, dims, coef = _prec_args(prec, n)
    alpha = np.zeros((m, k))
    beta = np.zeros((m, k + 1))
    k_used = np.zeros(m, dtype=np.int32)
    nu = np.zeros(m)
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
    va = np.ascontiguousarray(A.val, dtype=np.float64)
    rc = lib.oracle_lanczos(n, _ptr(rp), _ptr(ci), _ptr(va), kind, nd, _ptr(dims),
                            float(prec.s), float(prec.lo), float(prec.hi), len(coef) - 1,
                            _ptr(coef), float(tau), _ptr(V), m, int(k),
                            int(nthreads or host_threads()), _ptr(alpha), _ptr(beta),
                            _ptr(k_used), _ptr(nu))
    if rc == -2:
        raise ZeroDivisionError("Jacobi preconditioner is singular: a_rr == tau")
    if rc != 0:
        raise ValueError("oracle_lanczos failed (%d)" % rc)
    return LanczosResult(alpha, beta, k_used, nu)


def lanczos_ldl(A, F: ILDLFactor, tau: float, V: np.ndarray, k: int,
                nthreads: int | None = None) -> LanczosResult:
    """Algorithm 1 on C = M (A - tau I) M^*, M = |D|^(-1/2) L^{-1} P from the
    factor F of this shift."""
    lib = _load()
    V = np.ascontiguousarray(V, dtype=np.float64)
    n, m = V.shape
    rp, ci, va = _csr_args(A)
    perm, lrp, lci, lval, dd, do = _ldl_args(F)
    alpha = np.zeros((m, k))
    beta = np.zeros((m, k + 1))
    k_used = np.zeros(m, dtype=np.int32)
    nu = np.zeros(m)
    rc = lib.oracle_lanczos_ldl(n, _ptr(rp), _ptr(ci), _ptr(va), float(tau), _ptr(perm),
                                _ptr(lrp), _ptr(lci), _ptr(lval), _ptr(dd), _ptr(do), _ptr(V), m,
                                int(k), int(nthreads or host_threads()), _ptr(alpha), _ptr(beta),
                                _ptr(k_used), _ptr(nu))
    if rc == -2:
        raise ZeroDivisionError("ILDL factor has a zero pivot")
    if rc != 0:
        raise ValueError("oracle_lanczos_ldl failed (%d)" % rc)
    return LanczosResult(alpha, beta, k_used, nu)


def dense_operator_ldl(A, F: ILDLFactor, tau: float) -> np.ndarray:
    """C = M (A - tau I) M^* with the ILDL preconditioner (small n only)."""
    lib = _load()
    n = A.n
    rp, ci, va = _csr_args(A)
    perm, lrp, lci, lval, dd, do = _ldl_args(F)
    C = np.zeros((n, n))
    lib.oracle_dense_operator_ldl(n, _ptr(rp), _ptr(ci), _ptr(va), float(tau), _ptr(perm),
                                  _ptr(lrp), _ptr(lci), _ptr(lval), _ptr(dd), _ptr(do), _ptr(C))
    return C


def dense_operator(A, prec, tau: float) -> np.ndarray:
    """C = M (A - tau I) M^* as a dense matrix (small n only)."""
    if prec.kind == "ildl":
        return dense_operator_ldl(A, ildl(A, tau, prec.droptol), tau)
    lib = _load()
    n = A.n
    kind, nd, dims, coef = _prec_args(prec, n)
    C = np.zeros((n, n))
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
    va = np.ascontiguousarray(A.val, dtype=np.float64)
    lib.oracle_dense_operator(n, _ptr(rp), _ptr(ci), _ptr(va), kind, nd, _ptr(dims),
                              float(prec.s), float(prec.lo), float(prec.hi), len(coef) - 1,
                              _ptr(coef), float(tau), _ptr(C))
    return C


def apply_operator(A, prec, tau: float, X: np.ndarray, nthreads: int | None = None) -> np.ndarray:
    """Y = C X, C = M (A - tau I) M^*, for an n x m block X (preconditioner
    kinds none, jacobi, cheb), column by column with the oracle's operator."""
    if prec.kind == "ildl":
        raise ValueError("apply_operator takes the preconditioners none, jacobi and cheb")
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    n, m = X.shape
    if A.n != n:
        raise ValueError("block does not match A")
    kind, nd, dims, coef = _prec_args(prec, n)
    Y = np.zeros((n, m))
    rp, ci, va = _csr_args(A)
    rc = lib.oracle_apply_operator(n, _ptr(rp), _ptr(ci), _ptr(va), kind, nd, _ptr(dims),
                                   float(prec.s), float(prec.lo), float(prec.hi), len(coef) - 1,
                                   _ptr(coef), float(tau), _ptr(X), m,
                                   int(nthreads or host_threads()), _ptr(Y))
    if rc == -2:
        raise ZeroDivisionError("Jacobi preconditioner is singular: a_rr == tau")
    if rc != 0:
        raise ValueError("oracle_apply_operator failed (%d)" % rc)
    return Y


# ---------------------------------------------------------------------------
# Quadrature (Section 3.1 eq. gauss_quad; Section 3.4 eq. GA_Tk)
# ---------------------------------------------------------------------------


def jacobi_matrix(alpha: np.ndarray, beta: np.ndarray, k: int, rule: str = "gauss") -> np.ndarray:
    """Dense tridiagonal matrix of the rule.  alpha: alpha_1..alpha_k (at least),
    beta: beta_1..beta_{k+1} (beta[0] = beta_1 = 0)."""
    a = np.asarray(alpha[:k], dtype=np.float64)
    b = np.asarray(beta[1:k], dtype=np.float64)          # beta_2..beta_k
    if rule == "ga" and k >= 2:
        diag = np.concatenate([a, a[:k - 1][::-1]])
        off = np.concatenate([b, [beta[k]], b[:k - 2][::-1]])
    elif rule in ("gauss", "ga"):
        diag, off = a, b
    else:
        raise ValueError(rule)
    return np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)


def step(theta: np.ndarray, smooth_w: float = 0.0) -> np.ndarray:
    """h(theta) = 1 for theta < 0 else 0 (eq. h); or erfc(theta/w)/2 if w > 0."""
    if smooth_w > 0.0:
        return np.array([0.5 * math.erfc(t / smooth_w) for t in theta])
    return (theta < 0.0).astype(np.float64)


def probe_quadrature(alpha_j, beta_j, k_used: int, nu: float, rule: str = "gauss",
                     smooth_w: float = 0.0):
    """Return (s_j, min |theta|) for one probe: s_j = nu * sum_i z_i(1)^2 h(theta_i)."""
    J = jacobi_matrix(alpha_j, beta_j, int(k_used), rule if k_used == len(alpha_j) else "gauss")
    theta, Z = np.linalg.eigh(J)
    w = Z[0, :] ** 2
    return nu * float(np.dot(w, step(theta, smooth_w))), float(np.min(np.abs(theta)))


def quadrature(res: LanczosResult, rule: str = "gauss", smooth_w: float = 0.0):
    m = res.alpha.shape[0]
    s = np.zeros(m)
    mins = np.zeros(m)
    for j in range(m):
        s[j], mins[j] = probe_quadrature(res.alpha[j], res.beta[j], res.k_used[j], res.nu[j],
                                         rule, smooth_w)
    return s, mins


def _mean(x) -> float:
    acc = 0.0
    for v in x:              # index order
        acc += float(v)
    return acc / len(x)


@dataclass
class CountResult:
    estimate: float
    variance: float
    neg_xi: float
    neg_eta: float
    s_xi: np.ndarray
    s_eta: np.ndarray
    min_abs_ritz: float
    lan_xi: LanczosResult
    lan_eta: LanczosResult


def negcount(A, prec, tau, V, k, rule="gauss", smooth_w=0.0, nthreads=None):
    """Algorithm 2: (1/m) sum_j s_j(tau), plus the per-probe s_j."""
    res = lanczos(A, prec, tau, V, k, nthreads)
    s, mins = quadrature(res, rule, smooth_w)
    return _mean(s), s, res, float(np.min(mins))


def count(A, prec, xi, eta, V, k, rule="gauss", smooth_w=0.0, nthreads=None) -> CountResult:
    """Estimate the number of eigenvalues of A in [xi, eta)."""
    if not (xi < eta):
        raise ValueError("need xi < eta")
    _, s_xi, lx, mx = negcount(A, prec, xi, V, k, rule, smooth_w, nthreads)
    _, s_eta, le, me = negcount(A, prec, eta, V, k, rule, smooth_w, nthreads)
    m = len(s_xi)
    d = s_eta - s_xi
    est = _mean(d)
    if m > 1:
        acc = 0.0
        for v in d:
            acc += (float(v) - est) ** 2
        var = acc / ((m - 1) * m)
    else:
        var = float("nan")
    return CountResult(est, var, _mean(s_xi), _mean(s_eta), s_xi, s_eta, min(mx, me), lx, le)


# ---------------------------------------------------------------------------
# Derivatives of the erf-smoothed estimator (forward mode)
# ---------------------------------------------------------------------------


def step_deriv(theta: np.ndarray, smooth_w: float) -> np.ndarray:
    """d/dtheta of erfc(theta / w) / 2."""
    return -np.exp(-(theta / smooth_w) ** 2) / (smooth_w * math.sqrt(math.pi))


def divided_difference(theta: np.ndarray, smooth_w: float) -> np.ndarray:
    """S[1](a, b) = (S(a) - S(b)) / (a - b), S'(a) on (near-)coincident pairs."""
    S = step(theta, smooth_w)
    ta, tb = theta[:, None], theta[None, :]
    diff = ta - tb
    close = np.abs(diff) < 1e-8 * (1.0 + np.abs(ta))
    with np.errstate(divide="ignore", invalid="ignore"):
        D = (S[:, None] - S[None, :]) / diff
    D[close] = step_deriv(0.5 * (ta + tb), smooth_w)[close]
    return D


@dataclass
class TangentResult:
    lan: LanczosResult
    dalpha: np.ndarray
    dbeta: np.ndarray


def lanczos_tangent(A, prec, tau, V, k, du, dtau, nthreads=None) -> TangentResult:
    """Algorithm 1 and its forward-mode derivative along A -> A + t diag(du),
    tau -> tau + t dtau (M fixed)."""
    lib = _load()
    V = np.ascontiguousarray(V, dtype=np.float64)
    n, m = V.shape
    kind, nd, dims, coef = _prec_args(prec, n)
    du = np.ascontiguousarray(du, dtype=np.float64)
    alpha, beta = np.zeros((m, k)), np.zeros((m, k + 1))
    dalpha, dbeta = np.zeros((m, k)), np.zeros((m, k + 1))
    k_used = np.zeros(m, dtype=np.int32)
    nu = np.zeros(m)
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
    va = np.ascontiguousarray(A.val, dtype=np.float64)
    rc = lib.oracle_lanczos_tangent(n, _ptr(rp), _ptr(ci), _ptr(va), kind, nd, _ptr(dims),
                                    float(prec.s), float(prec.lo), float(prec.hi), len(coef) - 1,
                                    _ptr(coef), float(tau), _ptr(du), float(dtau), _ptr(V), m,
                                    int(k), int(nthreads or host_threads()), _ptr(alpha),
                                    _ptr(beta), _ptr(dalpha), _ptr(dbeta), _ptr(k_used), _ptr(nu))
    if rc != 0:
        raise ValueError("oracle_lanczos_tangent failed (%d)" % rc)
    return TangentResult(LanczosResult(alpha, beta, k_used, nu), dalpha, dbeta)


def probe_quadrature_tangent(alpha_j, beta_j, dalpha_j, dbeta_j, k_used, nu, smooth_w):
    """(s_j, ds_j): s = nu e1^T S(J) e1 and its derivative
    ds = nu sum_{a,b} z_a z_b S[1](theta_a, theta_b) (Z^T dJ Z)_{ab}
    (Daleckii-Krein), z = first row of the eigenvector matrix Z of J."""
    k = int(k_used)
    J = jacobi_matrix(alpha_j, beta_j, k)
    dJ = jacobi_matrix(dalpha_j, dbeta_j, k)
    theta, Z = np.linalg.eigh(J)
    z = Z[0, :]
    s = nu * float(np.dot(z * z, step(theta, smooth_w)))
    D = divided_difference(theta, smooth_w)
    ds = nu * float(z @ (D * (Z.T @ dJ @ Z)) @ z)
    return s, ds


def count_tangent(A, prec, xi, eta, V, k, du, dxi=0.0, deta=0.0, smooth_w=0.05, nthreads=None):
    """(estimate, directional derivative) of the smoothed interval count along
    V -> V + t du, xi -> xi + t dxi, eta -> eta + t deta."""
    m = V.shape[1]
    out = []
    for tau, dtau in ((xi, dxi), (eta, deta)):
        T = lanczos_tangent(A, prec, tau, V, k, du, dtau, nthreads)
        sd = [probe_quadrature_tangent(T.lan.alpha[j], T.lan.beta[j], T.dalpha[j], T.dbeta[j],
                                       T.lan.k_used[j], T.lan.nu[j], smooth_w) for j in range(m)]
        out.append(np.array(sd))
    d = out[1] - out[0]
    return _mean(d[:, 0]), _mean(d[:, 1])


# ---------------------------------------------------------------------------
# Arnoldi estimator for an unfactored preconditioner T (Section 4)
# ---------------------------------------------------------------------------
# C = T (A - tau I); `prec` describes T itself: "none" T = I, "jacobi"
# T = |diag(A) - tau|^(-1), "cheb" T = sum_j c_j T_j(B) with the given series.
# Per probe (Algorithm 4): k Arnoldi steps (Algorithm 3, modified
# Gram-Schmidt) give H_k; with H_k = Z Theta Z^(-1),
#     s_j(tau) = |v_j|^2 Re sum_{i : Re theta_i < 0} z_i(1) t_i,
# t_i the i-th entry of the FIRST COLUMN of Z^(-1) (eq. arnoldi_quad; this is
# e_1^T h(H_k) e_1 with h = 1 on the open left half-plane, whatever the
# eigenvector scaling).  Algorithm 4 writes the first row; the equation and
# the identity fix the first column.


@dataclass
class ArnoldiResult:
    H: np.ndarray       # m x (k+1) x k, H[j, i, l] = h_{i+1, l+1} of probe j
    k_used: np.ndarray  # m
    nu: np.ndarray      # m


def arnoldi(A, prec, tau: float, V: np.ndarray, k: int, nthreads: int | None = None) -> ArnoldiResult:
    """Algorithm 3 on C = T (A - tau I) for every column of V (n x m)."""
    lib = _load()
    V = np.ascontiguousarray(V, dtype=np.float64)
    n, m = V.shape
    if A.n != n:
        raise ValueError("probe block does not match A")
    kind, nd, dims, coef = _prec_args(prec, n)
    H = np.zeros((m, k + 1, k))
    k_used = np.zeros(m, dtype=np.int32)
    nu = np.zeros(m)
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
    va = np.ascontiguousarray(A.val, dtype=np.float64)
    rc = lib.oracle_arnoldi(n, _ptr(rp), _ptr(ci), _ptr(va), kind, nd, _ptr(dims),
                            float(prec.s), float(prec.lo), float(prec.hi), len(coef) - 1,
                            _ptr(coef), float(tau), _ptr(V), m, int(k),
                            int(nthreads or host_threads()), _ptr(H), _ptr(k_used), _ptr(nu))
    if rc == -2:
        raise ZeroDivisionError("T = |diag(A) - tau|^-1 is singular: a_rr == tau")
    if rc != 0:
        raise ValueError("oracle_arnoldi failed (%d)" % rc)
    return ArnoldiResult(H, k_used, nu)


def arnoldi_quadrature(Hj: np.ndarray, k_used: int, nu: float):
    """Return (s_j, min |Re theta|) for one probe (Algorithm 4, eq. arnoldi_quad)."""
    Hk = Hj[:k_used, :k_used]
    theta, Z = np.linalg.eig(Hk)
    S = np.linalg.inv(Z)
    neg = theta.real < 0.0
    val = np.sum(Z[0, neg] * S[neg, 0])
    return nu * float(val.real), float(np.min(np.abs(theta.real)))


def count_arnoldi(A, prec, xi, eta, V, k, nthreads=None) -> CountResult:
    """Interval count with the Arnoldi estimator at xi and eta on the same probes."""
    if not (xi < eta):
        raise ValueError("need xi < eta")
    out = []
    for tau in (xi, eta):
        res = arnoldi(A, prec, tau, V, k, nthreads)
        m = res.H.shape[0]
        sv = np.zeros(m)
        mins = np.zeros(m)
        for j in range(m):
            sv[j], mins[j] = arnoldi_quadrature(res.H[j], res.k_used[j], res.nu[j])
        out.append((sv, res, float(np.min(mins))))
    (s_xi, rx, mx), (s_eta, re_, me) = out
    m = len(s_xi)
    d = s_eta - s_xi
    est = _mean(d)
    if m > 1:
        acc = 0.0
        for v in d:
            acc += (float(v) - est) ** 2
        var = acc / ((m - 1) * m)
    else:
        var = float("nan")
    return CountResult(est, var, _mean(s_xi), _mean(s_eta), s_xi, s_eta, min(mx, me), rx, re_)
