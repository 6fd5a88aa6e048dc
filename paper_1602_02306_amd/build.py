"""Build the HIP library libecount.so in-tree for gfx950 with hipcc.

Each source is compiled to an object in parallel (no device code crosses
files: every kernel is launched from its own file), then the objects are
linked into the shared library."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libecount.so")
OBJ = os.path.join(PKG, "_build")
SOURCES = ["ecount_api.hip", "k_operator.hip", "k_lanczos.hip", "k_quad.hip", "k_backward.hip", "k_arnoldi.hip",
           "ildl_factor.hip", "k_ldl.hip", "k_block.hip", "k_probe.hip", "k_small.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # packed-FP32 instructions stay disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden",
]


def _jobs() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16, len(SOURCES)))


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(src):
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + FLAGS + inc + ["-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        return src, obj, r

    with ThreadPoolExecutor(_jobs()) as ex:
        results = list(ex.map(compile_one, SOURCES))
    failed = False
    for src, obj, r in results:
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                        if "packed-fp32-ops" not in l)
        if msg.strip():
            print(msg, file=sys.stderr, flush=True)
        if r.returncode != 0:
            print("compiling %s failed" % src, file=sys.stderr, flush=True)
            failed = True
    if failed:
        raise subprocess.CalledProcessError(1, "hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for _, o, _ in results]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
