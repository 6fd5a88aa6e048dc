"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, sizes its workspace, and rejects invalid calls before any
device work (these calls never reach the GPU)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1602_02306_amd import ecount as ec
from paper_1602_02306_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ecount.h")


def declared_symbols():
    txt = open(HEADER).read()
    return re.findall(r"ECNT_API\s+[\w\s\*]+?\b(ecnt_\w+)\s*\(", txt)


def test_header_declares_entry_points():
    names = declared_symbols()
    for n in ["ecnt_count", "ecnt_negcounts", "ecnt_workspace_bytes", "ecnt_last_error",
              "ecnt_version"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ec.load()
    nm = subprocess.run(["nm", "-D", "--defined-only", ec.LIB_PATH], capture_output=True,
                        text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(ecnt_\w+)", nm))
    for name in declared_symbols():
        assert name in exported, name
        assert hasattr(lib, name)
    assert ec.version().startswith("ecount-mi355x")


def test_workspace_bytes():
    prec = W.cheb_invsqrt_prec((64, 64, 64))
    b = ec.workspace_bytes(64 ** 3, 256, 2, prec, 30)
    # basis (k+1 blocks) + 3 Chebyshev scratch blocks, FP64
    blk = 64 ** 3 * 512 * 8
    assert 34 * blk <= b <= 34 * blk + 256 * 2 ** 20
    b32 = ec.workspace_bytes(64 ** 3, 256, 2, prec, 30, vec="f32")
    assert abs(b32 - b / 2) < 256 * 2 ** 20
    jac = W.PrecSpec("jacobi", ())
    assert ec.workspace_bytes(900, 40, 2, jac, 20) > 21 * 900 * 80 * 8
    # invalid requests size to 0
    assert ec.workspace_bytes(900, 40, 2, jac, 901) == 0
    assert ec.workspace_bytes(900, 0, 2, jac, 20) == 0
    assert ec.workspace_bytes(900, 40, 0, jac, 20) == 0
    assert ec.workspace_bytes(900, 40, 2, W.cheb_invsqrt_prec((10, 10, 10)), 20) == 0


def _call_count(A=True, prec=None, xi=0.0, eta=1.0, probes=0x1000, m=4, k=3, ws=0x2000,
                ws_bytes=1 << 40, n=64, opts=None, est=True):
    lib = ec.load()
    cs = ec.CsrT(n, 5 * n, 0x3000, 0x4000, 0x5000, 0, 0)
    if prec is None:
        prec = W.PrecSpec("none", ())
    ps, keep = ec.prec_struct(prec)
    o = opts or ec.opts_struct(k)
    e, v = ctypes.c_double(), ctypes.c_double()
    rc = lib.ecnt_count(ctypes.byref(cs) if A else None, ctypes.byref(ps), xi, eta, probes, m,
                        ctypes.byref(o), ws, ws_bytes, None,
                        ctypes.byref(e) if est else None, ctypes.byref(v), None)
    return rc, ec.last_error()


@pytest.mark.parametrize("kw,code", [
    (dict(A=False), ec.ECNT_EINVAL),
    (dict(xi=1.0, eta=1.0), ec.ECNT_EINVAL),
    (dict(xi=2.0, eta=1.0), ec.ECNT_EINVAL),
    (dict(xi=float("nan")), ec.ECNT_EINVAL),
    (dict(eta=float("inf")), ec.ECNT_EINVAL),
    (dict(probes=None), ec.ECNT_EINVAL),
    (dict(m=0), ec.ECNT_EINVAL),
    (dict(k=0), ec.ECNT_EINVAL),
    (dict(k=65), ec.ECNT_EINVAL),
    (dict(n=0), ec.ECNT_EINVAL),
    (dict(est=False), ec.ECNT_EINVAL),
    (dict(ws=None), ec.ECNT_EWORKSPACE),
    (dict(ws_bytes=1024), ec.ECNT_EWORKSPACE),
    (dict(n=1000, k=600), ec.ECNT_EUNSUPPORTED),
    (dict(prec=W.PrecSpec("cheb", (4, 4, 5), 1.0, 1.0, 13.0, np.ones(3))), ec.ECNT_EINVAL),
    (dict(prec=W.PrecSpec("cheb", (4, 4, 4), 1.0, 13.0, 1.0, np.ones(3))), ec.ECNT_EINVAL),
    (dict(prec=W.PrecSpec("cheb", (4, 4, 4), 1.0, 1.0, 13.0, np.array([1.0, np.nan]))), ec.ECNT_EINVAL),
    (dict(opts=ec.OptsT(3, 7, 0, 0, 0.0)), ec.ECNT_EINVAL),
    (dict(opts=ec.OptsT(3, 0, 5, 0, 0.0)), ec.ECNT_EINVAL),
    (dict(opts=ec.OptsT(3, 0, 0, -1, 0.0)), ec.ECNT_EINVAL),
    (dict(opts=ec.OptsT(3, 0, 0, 0, -1.0)), ec.ECNT_EINVAL),
    (dict(opts=ec.OptsT(3, 0, 0, 0, 0.0, 6)), ec.ECNT_EINVAL),
    (dict(opts=ec.OptsT(3, 0, 0, 0, 0.0, 0, 32)), ec.ECNT_EINVAL),
    (dict(opts=ec.OptsT(3, 0, 0, 0, 0.0, 0, 0, 3)), ec.ECNT_EINVAL),
    (dict(opts=ec.OptsT(3, 0, 0, 0, 0.0, 0, 0, 0, 2)), ec.ECNT_EINVAL),
    (dict(opts=ec.OptsT(3, 0, 0, 0, 0.0, 0, 0, 0, 0, 2)), ec.ECNT_EINVAL),
])
def test_invalid_calls_rejected_on_host(kw, code):
    rc, msg = _call_count(**kw)
    assert rc == code, msg
    assert msg


def test_negcounts_rejects_bad_shift_counts():
    lib = ec.load()
    cs = ec.CsrT(64, 320, 0x3000, 0x4000, 0x5000, 0, 0)
    ps, keep = ec.prec_struct(W.PrecSpec("none", ()))
    o = ec.opts_struct(3)
    taus = np.array([0.0, np.nan])
    out = np.zeros(4)
    for S, code in [(0, ec.ECNT_EINVAL), (65, ec.ECNT_EINVAL), (2, ec.ECNT_EINVAL)]:
        rc = lib.ecnt_negcounts(ctypes.byref(cs), ctypes.byref(ps), taus.ctypes.data, S, 0x1000, 4,
                                ctypes.byref(o), 0x2000, 1 << 40, None, out.ctypes.data, None,
                                None, None)
        assert rc == code, ec.last_error()


def _items(sizes, dims, taus):
    arr = (ec.BatchItemT * len(sizes))()
    for b, (n, d) in enumerate(zip(sizes, dims)):
        arr[b] = ec.BatchItemT(n, (ctypes.c_int32 * 3)(*d), 0, taus[b].ctypes.data)
    return arr


def test_batch_workspace_bytes():
    lib = ec.load()
    prec = W.cheb_invsqrt_prec((4, 4, 4))
    ps, keep = ec.prec_struct(prec)
    o = ec.opts_struct(5)
    taus = np.tile(np.array([-3.0, -2.0, -1.0]), (3, 1))
    sizes, dims = [64, 125, 60], [(4, 4, 4), (5, 5, 5), (3, 4, 5)]
    it = _items(sizes, dims, taus)
    b = lib.ecnt_batch_workspace_bytes(it, 3, 3, 8, ctypes.byref(ps), ctypes.byref(o))
    # basis (k+1 blocks) and 3 scratch blocks of 249 rows x 24 columns, FP64
    assert b >= 9 * 249 * 24 * 8
    # a grid that does not match its problem's rows, k above a problem's size,
    # no problems, too many shifts: size 0
    bad = _items(sizes, [(4, 4, 4), (5, 5, 4), (3, 4, 5)], taus)
    assert lib.ecnt_batch_workspace_bytes(bad, 3, 3, 8, ctypes.byref(ps), ctypes.byref(o)) == 0
    o70 = ec.opts_struct(61)
    assert lib.ecnt_batch_workspace_bytes(it, 3, 3, 8, ctypes.byref(ps), ctypes.byref(o70)) == 0
    assert lib.ecnt_batch_workspace_bytes(it, 0, 3, 8, ctypes.byref(ps), ctypes.byref(o)) == 0
    assert lib.ecnt_batch_workspace_bytes(it, 3, 65, 8, ctypes.byref(ps), ctypes.byref(o)) == 0
    # without the stencil preconditioner the grids are ignored
    pj, keepj = ec.prec_struct(W.PrecSpec("jacobi", ()))
    assert lib.ecnt_batch_workspace_bytes(bad, 3, 3, 8, ctypes.byref(pj), ctypes.byref(o)) > 0


def test_batch_rejects_invalid_calls_on_host():
    lib = ec.load()
    ps, keep = ec.prec_struct(W.PrecSpec("none", ()))
    o = ec.opts_struct(3)
    taus = np.tile(np.array([0.0, 1.0]), (2, 1))
    it = _items([32, 32], [(1, 1, 32)] * 2, taus)
    out = np.zeros(4)
    cases = [(ec.CsrT(65, 320, 0x3000, 0x4000, 0x5000, 0, 0), it, 2, ec.ECNT_EINVAL),   # A.n != sum n
             (ec.CsrT(64, 320, 0x3000, 0x4000, 0x5000, 0, 0), None, 2, ec.ECNT_EINVAL),
             (ec.CsrT(64, 320, 0x3000, 0x4000, 0x5000, 0, 0), it, 0, ec.ECNT_EINVAL)]
    for cs, items, nshift, code in cases:
        rc = lib.ecnt_count_batched(ctypes.byref(cs), ctypes.byref(ps), items, 2, nshift, 0x1000, 4,
                                    ctypes.byref(o), 0x2000, 1 << 40, None, out.ctypes.data, None,
                                    None, None)
        assert rc == code, ec.last_error()
    cs = ec.CsrT(64, 320, 0x3000, 0x4000, 0x5000, 0, 0)
    rc = lib.ecnt_count_batched(ctypes.byref(cs), ctypes.byref(ps), it, 2, 2, 0x1000, 4,
                                ctypes.byref(o), 0x2000, 1024, None, out.ctypes.data, None, None,
                                None)
    assert rc == ec.ECNT_EWORKSPACE
    taus_nan = np.array([[0.0, np.nan], [0.0, 1.0]])
    it2 = _items([32, 32], [(1, 1, 32)] * 2, taus_nan)
    rc = lib.ecnt_count_batched(ctypes.byref(cs), ctypes.byref(ps), it2, 2, 2, 0x1000, 4,
                                ctypes.byref(o), 0x2000, 1 << 40, None, out.ctypes.data, None,
                                None, None)
    assert rc == ec.ECNT_EINVAL


def _call_noalloc(n=64, m=4, k=3, prec=None, xi=0.0, eta=1.0, probes=0x1000, opts=None):
    lib = ec.load()
    cs = ec.CsrT(n, 7 * n, 0x3000, 0x4000, 0x5000, 0, 0)
    ps, keep = ec.prec_struct(prec or W.PrecSpec("none", ()))
    o = opts or ec.opts_struct(k)
    e, v = ctypes.c_double(), ctypes.c_double()
    rc = lib.ecnt_count_noalloc(ctypes.byref(cs), ctypes.byref(ps), xi, eta, probes, m,
                                ctypes.byref(o), None, ctypes.byref(e), ctypes.byref(v), None)
    return rc, ec.last_error()


def test_noalloc_refuses_oversized_count_on_host():
    """A count whose workspace exceeds the fixed array is refused before any
    device call (this process has no GPU)."""
    prec = W.cheb_invsqrt_prec((64, 64, 64))
    rc, msg = _call_noalloc(n=64 ** 3, m=256, k=30, prec=prec, xi=-8.0, eta=-2.0)
    assert rc == ec.ECNT_EWORKSPACE, msg
    assert "fixed" in msg and str(ec.NOALLOC_SCRATCH_BYTES) in msg
    # the limit is the workspace size of ecnt_count: just above it is refused
    jac = W.PrecSpec("jacobi", ())
    n, m = 4096, 64
    k = next(k for k in range(1, 200) if ec.workspace_bytes(n, m, 2, jac, k) > ec.NOALLOC_SCRATCH_BYTES)
    rc, msg = _call_noalloc(n=n, m=m, k=k, prec=jac)
    assert rc == ec.ECNT_EWORKSPACE, msg


@pytest.mark.parametrize("kw,code", [
    (dict(xi=1.0, eta=1.0), ec.ECNT_EINVAL),
    (dict(xi=float("nan")), ec.ECNT_EINVAL),
    (dict(probes=None), ec.ECNT_EINVAL),
    (dict(m=0), ec.ECNT_EINVAL),
    (dict(k=65), ec.ECNT_EINVAL),
    (dict(n=1000, k=600), ec.ECNT_EUNSUPPORTED),
])
def test_noalloc_invalid_calls_rejected_on_host(kw, code):
    rc, msg = _call_noalloc(**kw)
    assert rc == code, msg


def test_hbm_probe_rejects_bad_arguments_on_host():
    lib = ec.load()
    g = ctypes.c_double()
    for kind, buf, nbytes, reps in [(3, 0x1000, 1 << 30, 1), (0, None, 1 << 30, 1),
                                    (0, 0x1000, 1 << 20, 1), (1, 0x1000, 1 << 30, 0)]:
        rc = lib.ecnt_hbm_probe(kind, buf, nbytes, reps, None, ctypes.byref(g))
        assert rc == ec.ECNT_EINVAL, ec.last_error()
