"""Host-side checks of the block-Lanczos entry point: workspace sizing and
rejection of unsupported calls before any device work."""
import ctypes

import pytest

from paper_1602_02306_amd import ecount as ec
from paper_1602_02306_amd import workloads as W


def test_block_workspace_bytes():
    prec = W.cheb_invsqrt_prec((64, 64, 64))
    n = 64 ** 3
    b = ec.block_workspace_bytes(n, 256, prec, 30)
    blk = n * 512 * 8
    # basis (k+1 slots) + 3 Chebyshev scratch blocks + small per-block matrices
    assert 34 * blk <= b <= 34 * blk + 512 * 2 ** 20
    assert ec.block_workspace_bytes(n, 256, prec, 30, max_cols=128) < b


@pytest.mark.parametrize("n,m,k,kw", [
    (4096, 24, 4, {}),                 # m not a multiple of 16
    (4096, 32, 33, {}),                # k above 32
    (40, 32, 41, {}),                  # k > n
    (4096, 32, 4, dict(max_cols=24)),  # wave width not a multiple of 16
])
def test_block_workspace_rejects(n, m, k, kw):
    assert ec.block_workspace_bytes(n, m, W.PrecSpec("none", ()), k, **kw) == 0


def _call(m=32, k=4, vec=0, rule=0, n=4096, ldl=False):
    lib = ec.load()
    cs = ec.CsrT(n, 5 * n, 0x3000, 0x4000, 0x5000, 0, 0)
    ps, keep = ec.prec_struct(W.PrecSpec("none", ()))
    if ldl:
        f = (ec.LdlFactorT * 2)()
        for s in range(2):
            f[s] = ec.LdlFactorT(0x100, 0x200, 0x300, 0x400, 0x500, 0x600, 0, 0, 0)
        ps.kind = ec.PREC_KINDS["ldl"]
        ps.ldl = ctypes.cast(f, ctypes.c_void_p)
        keep = (keep, f)
    o = ec.OptsT(k, vec, rule, 0, 0.0)
    e, v = ctypes.c_double(), ctypes.c_double()
    rc = lib.ecnt_count_block(ctypes.byref(cs), ctypes.byref(ps), 0.0, 1.0, 0x1000, m,
                              ctypes.byref(o), 0x2000, 1 << 40, None, ctypes.byref(e),
                              ctypes.byref(v), None)
    return rc, ec.last_error()


@pytest.mark.parametrize("kw,code", [
    (dict(m=24), ec.ECNT_EINVAL),
    (dict(k=33), ec.ECNT_EUNSUPPORTED),
    (dict(vec=1), ec.ECNT_EUNSUPPORTED),
    (dict(rule=1), ec.ECNT_EUNSUPPORTED),
    (dict(n=20, k=21), ec.ECNT_EINVAL),
    (dict(ldl=True), ec.ECNT_EUNSUPPORTED),
])
def test_block_rejected_on_host(kw, code):
    rc, msg = _call(**kw)
    assert rc == code, msg
    assert msg
