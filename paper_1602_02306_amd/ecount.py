"""Python binding of libecount.so (the C ABI in include/ecount.h).

Argument marshalling only: every step of the estimator runs in the HIP
kernels of the library.  PyTorch provides device memory (the CSR arrays, the
probe block, the workspace, the optional per-probe outputs) and the current
stream.  There is no CPU fallback: if the library is not built, or no GPU is
present, the calls raise.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libecount.so")

ECNT_OK, ECNT_EINVAL, ECNT_ENOTHPD, ECNT_EWORKSPACE, ECNT_EDEVICE, ECNT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "ECNT_OK", -1: "ECNT_EINVAL", -2: "ECNT_ENOTHPD", -3: "ECNT_EWORKSPACE",
                -4: "ECNT_EDEVICE", -5: "ECNT_EUNSUPPORTED"}
DTYPES = {"f64": 0, "f32": 1}
PREC_KINDS = {"none": 0, "jacobi": 1, "cheb": 2, "ldl": 3}
RULES = {"gauss": 0, "ga": 1}


class EcntError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


class CsrT(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("val_type", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class PrecT(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("ndim", ctypes.c_int32), ("dims", ctypes.c_int32 * 3),
                ("degree", ctypes.c_int32), ("eval", ctypes.c_int32), ("s", ctypes.c_double),
                ("lo", ctypes.c_double), ("hi", ctypes.c_double), ("coef", ctypes.c_void_p),
                ("ldl", ctypes.c_void_p)]


class LdlFactorT(ctypes.Structure):
    _fields_ = [("perm", ctypes.c_void_p), ("l_row_ptr", ctypes.c_void_p),
                ("l_col_idx", ctypes.c_void_p), ("l_val", ctypes.c_void_p),
                ("d_diag", ctypes.c_void_p), ("d_off", ctypes.c_void_p),
                ("nnz", ctypes.c_int64), ("bandwidth", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class OptsT(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("vec_type", ctypes.c_int32), ("rule", ctypes.c_int32),
                ("max_cols", ctypes.c_int32), ("smooth_w", ctypes.c_double),
                ("tile", ctypes.c_int32), ("red_waves", ctypes.c_int32), ("csr_vw", ctypes.c_int32),
                ("a_form", ctypes.c_int32), ("fused", ctypes.c_int32)]


TILES = {"auto": 0, "4x4": 1, "2x4": 2, "1x8": 3, "4x4-unfused": 4, "8x8-wg": 5}
A_FORMS = {"auto": 0, "csr": 1}
FUSED = {"auto": 0, "off": 1}


class InfoT(ctypes.Structure):
    _fields_ = [("neg_xi", ctypes.c_double), ("neg_eta", ctypes.c_double),
                ("min_abs_ritz", ctypes.c_double), ("per_probe", ctypes.c_void_p),
                ("k_used", ctypes.c_void_p), ("alpha", ctypes.c_void_p), ("beta", ctypes.c_void_p)]


class BatchItemT(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("dims", ctypes.c_int32 * 3), ("reserved", ctypes.c_int32),
                ("taus", ctypes.c_void_p)]


class KernelStatT(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]


_lib = None


def load():
    """Load libecount.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libecount.so is not built (run __graft_entry__.build() or "
                               "python -m paper_1602_02306_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        lib.ecnt_workspace_bytes.restype = ctypes.c_size_t
        lib.ecnt_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                             ctypes.POINTER(PrecT), ctypes.POINTER(OptsT)]
        lib.ecnt_count.restype = ctypes.c_int32
        lib.ecnt_count.argtypes = [ctypes.POINTER(CsrT), ctypes.POINTER(PrecT), ctypes.c_double,
                                   ctypes.c_double, P, ctypes.c_int64, ctypes.POINTER(OptsT), P,
                                   ctypes.c_size_t, P, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(InfoT)]
        lib.ecnt_count_noalloc.restype = ctypes.c_int32
        lib.ecnt_count_noalloc.argtypes = [ctypes.POINTER(CsrT), ctypes.POINTER(PrecT),
                                           ctypes.c_double, ctypes.c_double, P, ctypes.c_int64,
                                           ctypes.POINTER(OptsT), P,
                                           ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(InfoT)]
        lib.ecnt_negcounts.restype = ctypes.c_int32
        lib.ecnt_negcounts.argtypes = [ctypes.POINTER(CsrT), ctypes.POINTER(PrecT), P,
                                       ctypes.c_int32, P, ctypes.c_int64, ctypes.POINTER(OptsT), P,
                                       ctypes.c_size_t, P, P, P, P, ctypes.POINTER(InfoT)]
        lib.ecnt_last_error.restype = ctypes.c_char_p
        lib.ecnt_last_error.argtypes = []
        lib.ecnt_version.restype = ctypes.c_char_p
        lib.ecnt_version.argtypes = []
        lib.ecnt_smooth_workspace_bytes.restype = ctypes.c_size_t
        lib.ecnt_smooth_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64,
                                                    ctypes.POINTER(PrecT), ctypes.POINTER(OptsT)]
        lib.ecnt_smooth_fwd.restype = ctypes.c_int32
        lib.ecnt_smooth_fwd.argtypes = lib.ecnt_count.argtypes
        lib.ecnt_smooth_bwd.restype = ctypes.c_int32
        lib.ecnt_smooth_bwd.argtypes = [ctypes.POINTER(CsrT), ctypes.POINTER(PrecT), ctypes.c_double,
                                        ctypes.c_double, P, ctypes.c_int64, ctypes.POINTER(OptsT),
                                        ctypes.c_int32, ctypes.c_double, P, ctypes.c_size_t, P, P,
                                        ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]
        BI = ctypes.POINTER(BatchItemT)
        lib.ecnt_batch_workspace_bytes.restype = ctypes.c_size_t
        lib.ecnt_batch_workspace_bytes.argtypes = [BI, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                                   ctypes.POINTER(PrecT), ctypes.POINTER(OptsT)]
        batch_args = [ctypes.POINTER(CsrT), ctypes.POINTER(PrecT), BI, ctypes.c_int32,
                      ctypes.c_int32, P, ctypes.c_int64, ctypes.POINTER(OptsT), P, ctypes.c_size_t, P]
        for name in ("ecnt_batch_prepare", "ecnt_batch_enqueue"):
            getattr(lib, name).restype = ctypes.c_int32
            getattr(lib, name).argtypes = batch_args
        lib.ecnt_batch_results.restype = ctypes.c_int32
        lib.ecnt_batch_results.argtypes = [BI, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                           ctypes.POINTER(PrecT), ctypes.POINTER(OptsT), P,
                                           ctypes.c_size_t, P, P, P, P, ctypes.POINTER(InfoT)]
        lib.ecnt_count_batched.restype = ctypes.c_int32
        lib.ecnt_count_batched.argtypes = batch_args + [P, P, P, ctypes.POINTER(InfoT)]
        lib.ecnt_arnoldi_workspace_bytes.restype = ctypes.c_size_t
        lib.ecnt_arnoldi_workspace_bytes.argtypes = lib.ecnt_smooth_workspace_bytes.argtypes
        lib.ecnt_count_arnoldi.restype = ctypes.c_int32
        lib.ecnt_count_arnoldi.argtypes = lib.ecnt_count.argtypes
        lib.ecnt_block_workspace_bytes.restype = ctypes.c_size_t
        lib.ecnt_block_workspace_bytes.argtypes = lib.ecnt_smooth_workspace_bytes.argtypes
        lib.ecnt_count_block.restype = ctypes.c_int32
        lib.ecnt_count_block.argtypes = lib.ecnt_count.argtypes
        lib.ecnt_profile_enable.restype = ctypes.c_int32
        lib.ecnt_ildl_factor.restype = ctypes.c_int32
        lib.ecnt_ildl_factor.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_double, ctypes.c_double,
                                         ctypes.POINTER(ctypes.c_void_p)]
        lib.ecnt_ildl_sizes.restype = ctypes.c_int32
        lib.ecnt_ildl_sizes.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)]
        lib.ecnt_ildl_export.restype = ctypes.c_int32
        lib.ecnt_ildl_export.argtypes = [ctypes.c_void_p] + [P] * 6
        lib.ecnt_ildl_free.restype = None
        lib.ecnt_ildl_free.argtypes = [ctypes.c_void_p]
        lib.ecnt_profile_enable.argtypes = [ctypes.c_int32]
        lib.ecnt_hbm_probe.restype = ctypes.c_int32
        lib.ecnt_hbm_probe.argtypes = [ctypes.c_int32, P, ctypes.c_size_t, ctypes.c_int32, P,
                                       ctypes.POINTER(ctypes.c_double)]
        lib.ecnt_profile_read.restype = ctypes.c_int32
        lib.ecnt_profile_read.argtypes = [ctypes.POINTER(KernelStatT), ctypes.c_int32]
        _lib = lib
    return _lib


def last_error() -> str:
    return load().ecnt_last_error().decode()


def _check(rc: int):
    if rc != ECNT_OK:
        raise EcntError(rc, last_error())


# ---------------------------------------------------------------------------
# Device-side inputs
# ---------------------------------------------------------------------------


@dataclass
class DeviceCSR:
    n: int
    nnz: int
    row_ptr: object   # torch int32 (device)
    col_idx: object   # torch int32 (device)
    val: object       # torch float64/float32 (device)

    def struct(self) -> CsrT:
        import torch
        vt = DTYPES["f32"] if self.val.dtype == torch.float32 else DTYPES["f64"]
        return CsrT(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                    self.val.data_ptr(), vt, 0)


def upload_csr(A, val_dtype: str = "f64", device: str = "cuda") -> DeviceCSR:
    """Copy a host CSR (workloads.CSR) to device memory."""
    import torch
    tdt = torch.float32 if val_dtype == "f32" else torch.float64
    return DeviceCSR(int(A.n), int(A.nnz),
                     torch.from_numpy(np.ascontiguousarray(A.row_ptr, dtype=np.int32)).to(device),
                     torch.from_numpy(np.ascontiguousarray(A.col_idx, dtype=np.int32)).to(device),
                     torch.from_numpy(np.ascontiguousarray(A.val, dtype=np.float64)).to(device, tdt))


# ---------------------------------------------------------------------------
# ILDL(t) preconditioner (factored on the host by the library, applied on the GPU)
# ---------------------------------------------------------------------------


@dataclass
class HostLDL:
    """P (A - tau I) P^T ~ L D L^T as ecnt_ildl_export lays it out (host arrays)."""
    n: int
    perm: np.ndarray
    l_rp: np.ndarray
    l_ci: np.ndarray
    l_val: np.ndarray
    d_diag: np.ndarray
    d_off: np.ndarray
    bandwidth: int
    n2x2: int
    nneg: int


def ildl_factor(A, tau: float, droptol: float) -> HostLDL:
    """ILDL(droptol) of A - tau I (ecnt_ildl_factor; host CSR `A`, host work)."""
    lib = load()
    n = int(A.n)
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
    va = np.ascontiguousarray(A.val, dtype=np.float64)
    h = ctypes.c_void_p()
    _check(lib.ecnt_ildl_factor(n, rp.ctypes.data, ci.ctypes.data, va.ctypes.data, float(tau),
                                float(droptol), ctypes.byref(h)))
    try:
        nnz, bw, n2, nneg = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib.ecnt_ildl_sizes(h, ctypes.byref(nnz), ctypes.byref(bw), ctypes.byref(n2),
                                   ctypes.byref(nneg)))
        z = int(nnz.value)
        a = dict(perm=np.zeros(n, np.int32), l_rp=np.zeros(n + 1, np.int32),
                 l_ci=np.zeros(z, np.int32), l_val=np.zeros(z), d_diag=np.zeros(n),
                 d_off=np.zeros(n))
        _check(lib.ecnt_ildl_export(h, *[a[k].ctypes.data for k in (
            "perm", "l_rp", "l_ci", "l_val", "d_diag", "d_off")]))
    finally:
        lib.ecnt_ildl_free(h)
    return HostLDL(n, bandwidth=int(bw.value), n2x2=int(n2.value), nneg=int(nneg.value), **a)


@dataclass
class DeviceLDL:
    n: int
    nnz: int
    bandwidth: int
    t: dict   # torch device tensors

    def struct(self) -> LdlFactorT:
        t = self.t
        return LdlFactorT(*[t[k].data_ptr() for k in ("perm", "l_rp", "l_ci", "l_val", "d_diag",
                                                      "d_off")],
                          self.nnz, self.bandwidth, 0)


def upload_ldl(F: HostLDL, device: str = "cuda") -> DeviceLDL:
    import torch
    t = {}
    for k in ("perm", "l_rp", "l_ci", "l_val", "d_diag", "d_off"):
        a = getattr(F, k)
        if a.size == 0:   # keep a valid pointer for empty entry arrays
            a = np.zeros(1, dtype=a.dtype)
        t[k] = torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return DeviceLDL(F.n, int(F.l_val.size), F.bandwidth, t)


@dataclass
class LDLPrecond:
    """ECNT_PREC_LDL: one device factor per shift, in shift order."""
    factors: list
    kind: str = "ldl"


def ildl_precond(A, taus, droptol: float, device: str = "cuda") -> LDLPrecond:
    """Factor A - tau I for every shift on the host and upload the factors."""
    return LDLPrecond([upload_ldl(ildl_factor(A, float(t), droptol), device) for t in taus])


EVALS = {"auto": 0, "clenshaw": 1}


def prec_struct(prec, eval: str = "auto"):
    """ecnt_prec from a workloads.PrecSpec or an LDLPrecond; returns (struct,
    keep-alive array)."""
    kind = PREC_KINDS[prec.kind]
    if kind == 3:
        arr = (LdlFactorT * len(prec.factors))(*[f.struct() for f in prec.factors])
        st = PrecT(3, 0, (ctypes.c_int32 * 3)(0, 0, 0), 0, EVALS[eval], 0.0, 0.0, 0.0, None,
                   ctypes.addressof(arr))
        return st, arr
    dims = (ctypes.c_int32 * 3)(0, 0, 0)
    coef = np.zeros(1)
    ndim = 0
    if kind == 2:
        ndim = len(prec.dims)
        for a, d in enumerate(prec.dims):
            dims[a] = int(d)
        coef = np.ascontiguousarray(prec.coef, dtype=np.float64)
    st = PrecT(kind, ndim, dims, max(len(coef) - 1, 0) if kind == 2 else 0, EVALS[eval],
               float(prec.s), float(prec.lo), float(prec.hi), coef.ctypes.data if kind == 2 else None)
    return st, coef


def _check_factors(prec, nshift: int):
    # the library reads one factor per shift from the host array
    if prec.kind == "ldl" and len(prec.factors) != nshift:
        raise ValueError("the LDL preconditioner needs one factor per shift (%d, got %d)"
                         % (nshift, len(prec.factors)))


def opts_struct(k: int, vec: str = "f64", rule: str = "gauss", smooth_w: float = 0.0,
                max_cols: int = 0, tune: dict | None = None) -> OptsT:
    """ecnt_opts; `tune` holds optional launch-shape tunables:
    {"tile": "4x4"|"2x4"|"1x8", "red_waves": int, "csr_vw": int, "a_form": "auto"|"csr",
    "fused": "auto"|"off"}."""
    t = tune or {}
    return OptsT(int(k), DTYPES[vec], RULES[rule], int(max_cols), float(smooth_w),
                 TILES[t.get("tile", "auto")], int(t.get("red_waves", 0)), int(t.get("csr_vw", 0)),
                 A_FORMS[t.get("a_form", "auto")], FUSED[t.get("fused", "auto")])


def workspace_bytes(n: int, m: int, nshift: int, prec, k: int, vec: str = "f64",
                    rule: str = "gauss", smooth_w: float = 0.0, max_cols: int = 0,
                    tune: dict | None = None) -> int:
    _check_factors(prec, nshift)
    ps, _coef = prec_struct(prec)
    o = opts_struct(k, vec, rule, smooth_w, max_cols, tune)
    return int(load().ecnt_workspace_bytes(int(n), int(m), int(nshift), ctypes.byref(ps),
                                           ctypes.byref(o)))


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Workspace:
    """A reusable device workspace (torch uint8 buffer)."""

    def __init__(self, nbytes: int, device: str = "cuda"):
        import torch
        self.buf = torch.empty(int(nbytes), dtype=torch.uint8, device=device)

    @property
    def nbytes(self) -> int:
        return self.buf.numel()

    def ensure(self, nbytes: int):
        if self.nbytes < nbytes:
            import torch
            dev = self.buf.device
            # release the old buffer first: old and new together may not fit
            self.buf = None
            torch.cuda.empty_cache()
            self.buf = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
        return self


@dataclass
class CountResult:
    estimate: float
    variance: float
    neg_xi: float
    neg_eta: float
    min_abs_ritz: float
    per_probe: object = None   # torch (2m,) float64: s_j(xi) then s_j(eta)
    k_used: object = None      # torch (2m,) int32
    alpha: object = None       # torch (k, 2m)
    beta: object = None        # torch (k+1, 2m)


def _info(C: int, k: int, want: bool, device):
    import torch
    if not want:
        return InfoT(), {}
    t = {"per_probe": torch.empty(C, dtype=torch.float64, device=device),
         "k_used": torch.empty(C, dtype=torch.int32, device=device),
         "alpha": torch.empty((k, C), dtype=torch.float64, device=device),
         "beta": torch.empty((k + 1, C), dtype=torch.float64, device=device)}
    info = InfoT(0.0, 0.0, 0.0, t["per_probe"].data_ptr(), t["k_used"].data_ptr(),
                 t["alpha"].data_ptr(), t["beta"].data_ptr())
    return info, t


def count(A: DeviceCSR, prec, xi: float, eta: float, probes, k: int, vec: str = "f64",
          rule: str = "gauss", smooth_w: float = 0.0, workspace: Workspace | None = None,
          stream=None, details: bool = True, eval: str = "auto", max_cols: int = 0,
          tune: dict | None = None) -> CountResult:
    """Interval count on [xi, eta) (ecnt_count).  `probes`: torch device tensor
    n x m (float64 for vec='f64', float32 for vec='f32')."""
    lib = load()
    n, m = probes.shape
    _check_factors(prec, 2)
    ps, _coef = prec_struct(prec, eval)
    o = opts_struct(k, vec, rule, smooth_w, max_cols, tune)
    need = lib.ecnt_workspace_bytes(n, m, 2, ctypes.byref(ps), ctypes.byref(o))
    ws = (workspace or Workspace(max(need, 1), probes.device)).ensure(need)
    info, keep = _info(2 * m, k, details, probes.device)
    est, var = ctypes.c_double(), ctypes.c_double()
    cs = A.struct()
    # a request the library cannot size is passed on so that it reports its own status
    rc = lib.ecnt_count(ctypes.byref(cs), ctypes.byref(ps), float(xi), float(eta),
                        probes.data_ptr(), m, ctypes.byref(o), ws.buf.data_ptr(), ws.nbytes,
                        _stream_handle(stream), ctypes.byref(est), ctypes.byref(var),
                        ctypes.byref(info))
    _check(rc)
    return CountResult(est.value, var.value, info.neg_xi, info.neg_eta, info.min_abs_ritz,
                       keep.get("per_probe"), keep.get("k_used"), keep.get("alpha"),
                       keep.get("beta"))


NOALLOC_SCRATCH_BYTES = 64 << 20   # ECNT_NOALLOC_SCRATCH_BYTES


def count_noalloc(A: DeviceCSR, prec, xi: float, eta: float, probes, k: int, vec: str = "f64",
                  rule: str = "gauss", smooth_w: float = 0.0, stream=None, details: bool = True,
                  eval: str = "auto", max_cols: int = 0, tune: dict | None = None) -> CountResult:
    """Interval count through ecnt_count_noalloc: as `count`, with the scratch in
    the library's fixed device array instead of a workspace (problems whose
    workspace exceeds NOALLOC_SCRATCH_BYTES are refused).  With details=True
    the optional per-probe outputs are torch tensors the caller allocates."""
    lib = load()
    n, m = probes.shape
    _check_factors(prec, 2)
    ps, _coef = prec_struct(prec, eval)
    o = opts_struct(k, vec, rule, smooth_w, max_cols, tune)
    info, keep = _info(2 * m, k, details, probes.device)
    est, var = ctypes.c_double(), ctypes.c_double()
    cs = A.struct()
    _check(lib.ecnt_count_noalloc(ctypes.byref(cs), ctypes.byref(ps), float(xi), float(eta),
                                  probes.data_ptr(), m, ctypes.byref(o), _stream_handle(stream),
                                  ctypes.byref(est), ctypes.byref(var), ctypes.byref(info)))
    return CountResult(est.value, var.value, info.neg_xi, info.neg_eta, info.min_abs_ritz,
                       keep.get("per_probe"), keep.get("k_used"), keep.get("alpha"),
                       keep.get("beta"))


def arnoldi_workspace_bytes(n: int, m: int, T, k: int, vec: str = "f64", max_cols: int = 0,
                            tune: dict | None = None) -> int:
    ps, _coef = prec_struct(T)
    o = opts_struct(k, vec, "gauss", 0.0, max_cols, tune)
    return int(load().ecnt_arnoldi_workspace_bytes(int(n), int(m), ctypes.byref(ps), ctypes.byref(o)))


def count_arnoldi(A: DeviceCSR, T, xi: float, eta: float, probes, k: int, vec: str = "f64",
                  workspace: Workspace | None = None, stream=None, details: bool = True,
                  max_cols: int = 0, tune: dict | None = None) -> CountResult:
    """Interval count with the Arnoldi estimator on T (A - tau I)
    (ecnt_count_arnoldi); `T` is the preconditioner itself (PrecSpec "none"
    or "cheb")."""
    lib = load()
    n, m = probes.shape
    ps, _coef = prec_struct(T)
    o = opts_struct(k, vec, "gauss", 0.0, max_cols, tune)
    need = lib.ecnt_arnoldi_workspace_bytes(n, m, ctypes.byref(ps), ctypes.byref(o))
    ws = (workspace or Workspace(max(need, 1), probes.device)).ensure(need)
    info, keep = _info(2 * m, k, details, probes.device)
    if details:
        info.alpha = None
        info.beta = None
    est, var = ctypes.c_double(), ctypes.c_double()
    cs = A.struct()
    rc = lib.ecnt_count_arnoldi(ctypes.byref(cs), ctypes.byref(ps), float(xi), float(eta),
                                probes.data_ptr(), m, ctypes.byref(o), ws.buf.data_ptr(), ws.nbytes,
                                _stream_handle(stream), ctypes.byref(est), ctypes.byref(var),
                                ctypes.byref(info))
    _check(rc)
    return CountResult(est.value, var.value, info.neg_xi, info.neg_eta, info.min_abs_ritz,
                       keep.get("per_probe"), keep.get("k_used"))


def block_workspace_bytes(n: int, m: int, prec, k: int, smooth_w: float = 0.0, max_cols: int = 0,
                          eval: str = "auto") -> int:
    ps, _coef = prec_struct(prec, eval)
    o = opts_struct(k, "f64", "gauss", smooth_w, max_cols, None)
    return int(load().ecnt_block_workspace_bytes(int(n), int(m), ctypes.byref(ps), ctypes.byref(o)))


def count_block(A: DeviceCSR, prec, xi: float, eta: float, probes, k: int, smooth_w: float = 0.0,
                workspace: Workspace | None = None, stream=None, details: bool = True,
                eval: str = "auto", max_cols: int = 0) -> CountResult:
    """Interval count with the block-Lanczos form (ecnt_count_block): probes
    in blocks of 16 columns (m a multiple of 16), FP64, k <= 32."""
    lib = load()
    n, m = probes.shape
    _check_factors(prec, 2)
    ps, _coef = prec_struct(prec, eval)
    o = opts_struct(k, "f64", "gauss", smooth_w, max_cols, None)
    need = lib.ecnt_block_workspace_bytes(n, m, ctypes.byref(ps), ctypes.byref(o))
    ws = (workspace or Workspace(max(need, 1), probes.device)).ensure(need)
    info, keep = _info(2 * m, k, details, probes.device)
    if details:
        info.alpha = None
        info.beta = None
    est, var = ctypes.c_double(), ctypes.c_double()
    cs = A.struct()
    rc = lib.ecnt_count_block(ctypes.byref(cs), ctypes.byref(ps), float(xi), float(eta),
                              probes.data_ptr(), m, ctypes.byref(o), ws.buf.data_ptr(), ws.nbytes,
                              _stream_handle(stream), ctypes.byref(est), ctypes.byref(var),
                              ctypes.byref(info))
    _check(rc)
    return CountResult(est.value, var.value, info.neg_xi, info.neg_eta, info.min_abs_ritz,
                       keep.get("per_probe"), keep.get("k_used"))


@dataclass
class NegcountsResult:
    negcounts: np.ndarray
    counts: np.ndarray
    variances: np.ndarray
    min_abs_ritz: float
    per_probe: object = None
    k_used: object = None
    alpha: object = None
    beta: object = None


def negcounts(A: DeviceCSR, prec, taus, probes, k: int, vec: str = "f64", rule: str = "gauss",
              smooth_w: float = 0.0, workspace: Workspace | None = None, stream=None,
              details: bool = True, eval: str = "auto", max_cols: int = 0,
              tune: dict | None = None) -> NegcountsResult:
    """Algorithm 2 at several shifts on one probe block (ecnt_negcounts)."""
    lib = load()
    n, m = probes.shape
    taus = np.ascontiguousarray(taus, dtype=np.float64)
    S = len(taus)
    _check_factors(prec, S)
    ps, _coef = prec_struct(prec, eval)
    o = opts_struct(k, vec, rule, smooth_w, max_cols, tune)
    need = lib.ecnt_workspace_bytes(n, m, S, ctypes.byref(ps), ctypes.byref(o))
    ws = (workspace or Workspace(max(need, 1), probes.device)).ensure(need)
    info, keep = _info(S * m, k, details, probes.device)
    neg = np.zeros(S)
    cnt = np.zeros(max(S - 1, 1))
    var = np.zeros(max(S - 1, 1))
    cs = A.struct()
    rc = lib.ecnt_negcounts(ctypes.byref(cs), ctypes.byref(ps), taus.ctypes.data, S,
                            probes.data_ptr(), m, ctypes.byref(o), ws.buf.data_ptr(), ws.nbytes,
                            _stream_handle(stream), neg.ctypes.data, cnt.ctypes.data,
                            var.ctypes.data, ctypes.byref(info))
    _check(rc)
    return NegcountsResult(neg, cnt[:S - 1], var[:S - 1], info.min_abs_ritz,
                           keep.get("per_probe"), keep.get("k_used"), keep.get("alpha"),
                           keep.get("beta"))


def version() -> str:
    return load().ecnt_version().decode()


def profile_enable(on: bool = True):
    """Start (and reset) or stop per-kernel-family HIP-event timing."""
    _check(load().ecnt_profile_enable(1 if on else 0))


PROBES = {"copy": 0, "read": 1, "update_mix": 2}


def hbm_probe(kind: str, nbytes: int = 18 << 30, reps: int = 10, stream=None) -> float:
    """Effective GB/s of a tuned stream (ecnt_hbm_probe): 'copy', 'read' or
    'update_mix' (16 vectors read, one read and written in place)."""
    import torch
    buf = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
    g = ctypes.c_double()
    _check(load().ecnt_hbm_probe(PROBES[kind], buf.data_ptr(), buf.numel(), int(reps),
                                 _stream_handle(stream), ctypes.byref(g)))
    del buf
    return g.value


def profile_read() -> dict:
    """{family: {launches, ms, bytes}} accumulated since profile_enable(True)."""
    arr = (KernelStatT * 64)()
    n = load().ecnt_profile_read(arr, 64)
    return {arr[i].name.decode(): {"launches": int(arr[i].launches), "ms": float(arr[i].total_ms),
                                   "bytes": float(arr[i].bytes)} for i in range(n)}


# ---------------------------------------------------------------------------
# Differentiated form (erf-smoothed count)
# ---------------------------------------------------------------------------

CKPT = {"keep": 0, "recompute": 1}


def smooth_workspace_bytes(n: int, m: int, prec, k: int, smooth_w: float) -> int:
    ps, _coef = prec_struct(prec)
    o = opts_struct(k, "f64", "gauss", smooth_w)
    return int(load().ecnt_smooth_workspace_bytes(int(n), int(m), ctypes.byref(ps), ctypes.byref(o)))


def smooth_forward(A: DeviceCSR, prec, xi: float, eta: float, probes, k: int, smooth_w: float,
                   workspace: Workspace | None = None, stream=None, details: bool = False):
    """Smoothed interval count (ecnt_smooth_fwd).  Returns (CountResult, workspace);
    the workspace holds the state that smooth_backward(..., ckpt='keep') uses."""
    lib = load()
    n, m = probes.shape
    ps, _coef = prec_struct(prec)
    o = opts_struct(k, "f64", "gauss", smooth_w)
    need = lib.ecnt_smooth_workspace_bytes(n, m, ctypes.byref(ps), ctypes.byref(o))
    ws = (workspace or Workspace(max(need, 1), probes.device)).ensure(need)
    info, keep = _info(2 * m, k, details, probes.device)
    est, var = ctypes.c_double(), ctypes.c_double()
    cs = A.struct()
    rc = lib.ecnt_smooth_fwd(ctypes.byref(cs), ctypes.byref(ps), float(xi), float(eta),
                             probes.data_ptr(), m, ctypes.byref(o), ws.buf.data_ptr(), ws.nbytes,
                             _stream_handle(stream), ctypes.byref(est), ctypes.byref(var),
                             ctypes.byref(info))
    _check(rc)
    res = CountResult(est.value, var.value, info.neg_xi, info.neg_eta, info.min_abs_ritz,
                      keep.get("per_probe"), keep.get("k_used"), keep.get("alpha"), keep.get("beta"))
    return res, ws


def smooth_backward(A: DeviceCSR, prec, xi: float, eta: float, probes, k: int, smooth_w: float,
                    g_est: float = 1.0, ckpt: str = "keep", workspace: Workspace | None = None,
                    stream=None):
    """Gradient of g_est * estimate: (dV (torch, device, n), dxi, deta)."""
    import torch
    lib = load()
    n, m = probes.shape
    ps, _coef = prec_struct(prec)
    o = opts_struct(k, "f64", "gauss", smooth_w)
    need = lib.ecnt_smooth_workspace_bytes(n, m, ctypes.byref(ps), ctypes.byref(o))
    if need and ckpt == "keep" and (workspace is None or workspace.nbytes < need):
        raise ValueError("ckpt='keep' needs the workspace returned by smooth_forward")
    ws = (workspace or Workspace(max(need, 1), probes.device)).ensure(need)
    dV = torch.empty(n, dtype=torch.float64, device=probes.device)
    dxi, deta = ctypes.c_double(), ctypes.c_double()
    cs = A.struct()
    rc = lib.ecnt_smooth_bwd(ctypes.byref(cs), ctypes.byref(ps), float(xi), float(eta),
                             probes.data_ptr(), m, ctypes.byref(o), CKPT[ckpt], float(g_est),
                             ws.buf.data_ptr(), ws.nbytes, _stream_handle(stream), dV.data_ptr(),
                             ctypes.byref(dxi), ctypes.byref(deta))
    _check(rc)
    return dV, dxi.value, deta.value


# ---------------------------------------------------------------------------
# Batches of independent problems (block-diagonal A)
# ---------------------------------------------------------------------------


@dataclass
class BatchResult:
    negcounts: np.ndarray      # (nprob, nshift)
    counts: np.ndarray         # (nprob, nshift - 1)
    variances: np.ndarray      # (nprob, nshift - 1)
    per_probe: object = None   # torch (nprob, nshift * m) float64
    k_used: object = None      # torch (nprob, nshift * m) int32


class Batch:
    """A batch of independent problems run as one launch sequence
    (ecnt_batch_prepare / ecnt_batch_enqueue / ecnt_batch_results).

    A: DeviceCSR of the block-diagonal matrix (workloads.block_diag_csr);
    sizes: rows per problem; taus: (nprob, nshift) shifts; dims: per-problem
    grids (needed with the Laplacian preconditioner); probes: torch device
    tensor A.n x m.  `enqueue` only launches kernels, so it can be captured
    in a torch.cuda.CUDAGraph (see `capture`)."""

    def __init__(self, A: DeviceCSR, prec, sizes, taus, probes, k: int, dims=None,
                 vec: str = "f64", rule: str = "gauss", smooth_w: float = 0.0,
                 max_cols: int = 0, eval: str = "auto", workspace: Workspace | None = None,
                 stream=None, details: bool = False, tune: dict | None = None):
        self.lib = load()
        self.A, self.probes = A, probes
        self.n, self.m = probes.shape
        taus = np.ascontiguousarray(np.atleast_2d(taus), dtype=np.float64)
        self.nprob, self.nshift = taus.shape
        if len(sizes) != self.nprob:
            raise ValueError("sizes and taus disagree on the number of problems")
        self._taus = taus
        self._items = (BatchItemT * self.nprob)()
        for b in range(self.nprob):
            d = dims[b] if dims is not None else (1, 1, int(sizes[b]))
            d = tuple(int(x) for x in d)
            d = (1,) * (3 - len(d)) + d
            self._items[b] = BatchItemT(int(sizes[b]), (ctypes.c_int32 * 3)(*d), 0,
                                        taus[b].ctypes.data)
        self._ps, self._coef = prec_struct(prec, eval)
        if self._ps.kind == PREC_KINDS["cheb"]:
            self._ps.ndim = 3
        self._o = opts_struct(k, vec, rule, smooth_w, max_cols, tune)
        self._cs = A.struct()
        need = self.lib.ecnt_batch_workspace_bytes(self._items, self.nprob, self.nshift, self.m,
                                                   ctypes.byref(self._ps), ctypes.byref(self._o))
        self.ws = (workspace or Workspace(max(need, 1), probes.device)).ensure(need)
        self.details = details
        self._keep = {}
        if details:
            import torch
            C = self.nshift * self.m
            self._keep = {"per_probe": torch.empty((self.nprob, C), dtype=torch.float64,
                                                   device=probes.device),
                          "k_used": torch.empty((self.nprob, C), dtype=torch.int32,
                                                device=probes.device)}
        self.prepare(stream)

    def _args(self, stream):
        return (ctypes.byref(self._cs), ctypes.byref(self._ps), self._items, self.nprob,
                self.nshift, self.probes.data_ptr(), self.m, ctypes.byref(self._o),
                self.ws.buf.data_ptr(), self.ws.nbytes, _stream_handle(stream))

    def prepare(self, stream=None):
        _check(self.lib.ecnt_batch_prepare(*self._args(stream)))

    def enqueue(self, stream=None):
        _check(self.lib.ecnt_batch_enqueue(*self._args(stream)))

    def results(self, stream=None) -> BatchResult:
        S = self.nshift
        neg = np.zeros((self.nprob, S))
        cnt = np.zeros((self.nprob, max(S - 1, 1)))
        var = np.zeros((self.nprob, max(S - 1, 1)))
        info = InfoT()
        if self.details:
            info = InfoT(0.0, 0.0, 0.0, self._keep["per_probe"].data_ptr(),
                         self._keep["k_used"].data_ptr(), None, None)
        _check(self.lib.ecnt_batch_results(self._items, self.nprob, S, self.m,
                                           ctypes.byref(self._ps), ctypes.byref(self._o),
                                           self.ws.buf.data_ptr(), self.ws.nbytes,
                                           _stream_handle(stream), neg.ctypes.data,
                                           cnt.ctypes.data, var.ctypes.data, ctypes.byref(info)))
        return BatchResult(neg, cnt[:, :S - 1], var[:, :S - 1],
                           self._keep["per_probe"].clone() if self.details else None,
                           self._keep["k_used"].clone() if self.details else None)

    def run(self, stream=None) -> BatchResult:
        self.enqueue(stream)
        return self.results(stream)

    def capture(self):
        """Capture `enqueue` into a torch.cuda.CUDAGraph (returned); replay it and
        then call `results`."""
        import torch
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.enqueue(s)   # warm-up outside the capture (first-launch code-object loads)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            self.enqueue()
        return g


def batch_workspace_bytes(sizes, dims, nshift: int, m: int, prec, k: int, vec: str = "f64",
                          rule: str = "gauss", smooth_w: float = 0.0, max_cols: int = 0,
                          tune: dict | None = None) -> int:
    """Workspace bytes of a batch (ecnt_batch_workspace_bytes); 0 if invalid."""
    taus = np.zeros((len(sizes), nshift))
    items = (BatchItemT * len(sizes))()
    for b, n in enumerate(sizes):
        d = tuple(int(x) for x in (dims[b] if dims is not None else (1, 1, n)))
        d = (1,) * (3 - len(d)) + d
        items[b] = BatchItemT(int(n), (ctypes.c_int32 * 3)(*d), 0, taus[b].ctypes.data)
    ps, _coef = prec_struct(prec)
    if ps.kind == PREC_KINDS["cheb"]:
        ps.ndim = 3
    o = opts_struct(k, vec, rule, smooth_w, max_cols, tune)
    return int(load().ecnt_batch_workspace_bytes(items, len(sizes), int(nshift), int(m),
                                                 ctypes.byref(ps), ctypes.byref(o)))


def count_batched(A: DeviceCSR, prec, sizes, taus, probes, k: int, dims=None, **kw) -> BatchResult:
    """One-shot batched run (prepare + enqueue + results)."""
    return Batch(A, prec, sizes, taus, probes, k, dims=dims, **kw).run(kw.get("stream"))
