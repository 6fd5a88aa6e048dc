"""The product path has no CPU fallback: the package never imports the oracle,
and without the built HIP library every call fails loudly."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_package_does_not_import_the_oracle():
    code = ("import sys; import paper_1602_02306_amd.ecount, paper_1602_02306_amd.autograd, "
            "paper_1602_02306_amd.autotune, paper_1602_02306_amd.workloads; "
            "print(any(m == 'oracle' or m.startswith('oracle.') for m in sys.modules))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         check=True).stdout.strip()
    assert out == "False"


def test_missing_library_fails_loudly(monkeypatch):
    from paper_1602_02306_amd import ecount as ec
    monkeypatch.setattr(ec, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libecount.so"))
    monkeypatch.setattr(ec, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        ec.load()
