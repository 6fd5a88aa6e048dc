"""Launch-shape autotuner.

The estimator's kernels are cut into workgroups by a few shape parameters that
do not change what is computed (ecnt_opts.tile, red_waves, csr_vw, and the
column-wave width max_cols): the stencil's line block, the rows per chunk of
the two-phase column sums, the columns per lane of the CSR sweep, and how many
Lanczos columns run together.  Their best values depend on the problem's size
class (rows, problems per batch, columns, steps, precision), so they are
searched per class by timing short runs on the real inputs and cached in a
JSON file (path: $ECNT_TUNE_CACHE, else ~/.cache/ecount/tune.json).

Search: coordinate descent from the built-in defaults, one parameter at a
time, keeping a change only if it is at least 2% faster; each trial is the
median of a few event-timed runs with k_tune Lanczos steps (32 by default, so
the full run for k <= 32: the reorthogonalization sweeps and the partial sums
they reduce grow with the step, and a short trial undervalues them).
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Callable

DEFAULTS = {"tile": "auto", "red_waves": 0, "csr_vw": 0}


SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def cache_path() -> str:
    return os.environ.get("ECNT_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ecount", "tune.json"))


def lookup(key: str, cache: str | None = None):
    """Tuned entry for a size class: the user cache first, then the table
    shipped with the package (measured on an MI355X); None if neither has it."""
    for path, src in ((cache or cache_path(), "cache"), (SHIPPED, "shipped")):
        e = load_cache(path).get(key)
        if e:
            e = dict(e)
            e["source"] = src
            return e
    return None


def size_class(n: int, nprob: int, cols: int, k: int, vec: str, prec_kind: str) -> str:
    """Key of a size class: rows and problems in powers of two, exact columns and k."""
    lg = lambda x: int(round(math.log2(max(1, x))))
    return "%s/%s/rows2^%d/prob2^%d/cols%d/k%d" % (prec_kind, vec, lg(n), lg(nprob), cols, k)


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(entries: dict, path: str | None = None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def coordinate_search(run_ms: Callable[[dict], float], space: dict, start: dict,
                      min_gain: float = 0.02, log=None):
    """Minimise run_ms over `space` ({param: [values]}) by coordinate descent
    from `start`.  Returns (best config, its ms, list of (config, ms))."""
    best = dict(start)
    best_ms = run_ms(best)
    trials = [(dict(best), best_ms)]
    if log:
        log("tune start %s: %.3f ms" % (best, best_ms))
    for key, values in space.items():
        for v in values:
            if v == best.get(key):
                continue
            cfg = dict(best)
            cfg[key] = v
            ms = run_ms(cfg)
            trials.append((dict(cfg), ms))
            if log:
                log("tune %s=%s: %.3f ms" % (key, v, ms))
            if ms < best_ms * (1.0 - min_gain):
                best, best_ms = cfg, ms
    return best, best_ms, trials


def _timed(fn, reps: int) -> float:
    import torch
    fn()   # warm
    out = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    out.sort()
    return out[len(out) // 2]


def tune_batch(A, prec, sizes, taus, probes, k: int, dims=None, vec: str = "f64",
               mem_bytes: int | None = None, k_tune: int = 32, reps: int = 3,
               cache: str | None = None, retune: bool = False, log=None) -> dict:
    """Best launch shape for a batch (ecount.Batch arguments).  Returns
    {"max_cols", "tile", "red_waves", "csr_vw", "key", "ms", "source"}.
    mem_bytes bounds the workspace of the full-k run (column waves are
    narrowed until it fits)."""
    import numpy as np
    from . import ecount as ec

    taus = np.atleast_2d(taus)
    nprob, S = taus.shape
    m = probes.shape[1]
    Ct = S * m
    key = size_class(int(probes.shape[0]), nprob, Ct, k, vec, prec.kind)
    if not retune:
        e = lookup(key, cache)
        if e:
            return e
    kt = max(2, min(k, k_tune))

    def need_bytes(kk, w):
        return ec.batch_workspace_bytes(sizes, dims, S, m, prec, kk, vec=vec,
                                        max_cols=0 if w == Ct else w)

    def make_run(ws):
        def run_ms(cfg):
            tune = {x: cfg[x] for x in DEFAULTS}
            bt = ec.Batch(A, prec, sizes, taus, probes, kt, dims=dims, vec=vec, workspace=ws,
                          max_cols=0 if cfg["max_cols"] == Ct else cfg["max_cols"], tune=tune)
            return _timed(lambda: bt.run(), reps) * k / kt
        return run_ms

    return _search(key, Ct, k, kt, vec, need_bytes, make_run, mem_bytes, probes.device, cache, log)


def _search(key, Ct, k, kt, vec, need_bytes, make_run, mem_bytes, device, cache, log):
    import torch
    from . import ecount as ec
    # column-wave widths whose full-k workspace fits
    widths = []
    w = Ct
    while w >= 32:
        need = need_bytes(k, w)
        if need and (mem_bytes is None or need <= mem_bytes):
            widths.append(w)
        if len(widths) == 3:
            break
        w //= 2
    if not widths:
        raise RuntimeError("no column-wave width fits the memory budget")
    ws = ec.Workspace(max(max(need_bytes(kt, w) for w in widths), 1), device)
    space = {"max_cols": widths,
             "tile": ["4x4", "8x8-wg", "4x4-unfused", "2x4", "1x8"],
             "red_waves": [1024, 2048, 4096, 8192],
             "csr_vw": [1, 2] + ([4] if vec == "f32" else [])}
    start = {"max_cols": widths[0], "tile": "auto", "red_waves": 0, "csr_vw": 0}
    t0 = time.perf_counter()
    best, best_ms, trials = coordinate_search(make_run(ws), space, start, log=log)
    del ws
    torch.cuda.empty_cache()
    entry = dict(best)
    entry.update({"key": key, "ms": best_ms, "k_tune": kt, "trials": len(trials),
                  "tune_seconds": time.perf_counter() - t0})
    entries = load_cache(cache)
    entries[key] = entry
    try:
        save_cache(entries, cache)
    except OSError:
        pass
    entry = dict(entry)
    entry["source"] = "search"
    return entry


def tune_count(A, prec, xi: float, eta: float, probes, k: int, vec: str = "f64",
               mem_bytes: int | None = None, k_tune: int = 32, reps: int = 3,
               cache: str | None = None, retune: bool = False, log=None) -> dict:
    """Best launch shape for an interval count (ecount.count arguments), as
    tune_batch for a single problem."""
    from . import ecount as ec
    n, m = probes.shape
    Ct = 2 * m
    key = size_class(int(n), 1, Ct, k, vec, prec.kind)
    if not retune:
        e = lookup(key, cache)
        if e:
            return e
    kt = max(2, min(k, k_tune))

    def need_bytes(kk, w):
        return ec.workspace_bytes(n, m, 2, prec, kk, vec=vec, max_cols=0 if w == Ct else w)

    def make_run(ws):
        def run_ms(cfg):
            tune = {x: cfg[x] for x in DEFAULTS}
            mc = 0 if cfg["max_cols"] == Ct else cfg["max_cols"]
            return _timed(lambda: ec.count(A, prec, xi, eta, probes, kt, vec=vec, workspace=ws,
                                           details=False, max_cols=mc, tune=tune), reps) * k / kt
        return run_ms

    return _search(key, Ct, k, kt, vec, need_bytes, make_run, mem_bytes, probes.device, cache, log)
