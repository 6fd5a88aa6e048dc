"""Benchmark: Lanczos probe-steps/s of the eigenvalue-count estimator on one GPU.

One step = one interval count (Algorithm 2 at tau = xi and tau = eta on one
probe block): 2 * m * k probe-steps (one Lanczos step of one probe at one
shift each).  Inputs are synthetic (64^3 Gaussian-well Hamiltonian, CSR,
Chebyshev preconditioner, 256 Rademacher probes, k = 30, FP64) and resident in
HBM before timing starts.  Prints ONE JSON line.

  python bench.py [--steps K] [--warmup W] [--workload c2] [--no-cpu-baseline]
  python bench.py --copy-calib     (a plain device copy of known size, for
                                    scaling rocprofv3 FETCH_SIZE/WRITE_SIZE)
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, AMD public specification

WORKLOAD_TEXT = {
    "c1": "2D 5-pt 30x30 + V~U[0,1] (seed 0), CSR, Jacobi M per shift, [0.5,1.5], m=40, k=20, FP64",
    "c2": "3D 7-pt 64^3 CSR + 32 Gaussian wells (seed 1), Chebyshev M=c4(L+I), [-8,-2], m=256, k=30, FP64",
    "c3": "3D 7-pt 128^3 CSR + 32 Gaussian wells (seed 1), Chebyshev M=c4(L+I), [-8,-2], m=512, k=30, FP32 vectors",
    "c2_f32": "the 64^3 problem of c2 with A values and all Lanczos vectors in FP32 (FP64 alpha/beta, dots, eigensolve)",
    "c2_arn": "the 64^3 problem of c2 with the unfactored T = degree-8 Chebyshev approximation of (L+I)^-1 "
              "and the Arnoldi estimator (Algorithm 4), m=256, k=30, FP64",
    "c2_blk": "the 64^3 problem of c2 in the block-Lanczos form: blocks of 16 probes, one block "
              "Lanczos process per block (MFMA f64 dots and updates, Cholesky QR twice), block Gauss "
              "rule, m=256, k=30, FP64",
    "c5": "3D 7-pt 96^3 CSR + 32 Gaussian wells (seed 1), Chebyshev M, erf-smoothed count w=0.05, [-8,-2], m=128, k=30",
    "t1": "Table 1 Laplace: (1/h^2) 2D 5-pt Laplacian, h=2^-7 (127x127, n=16129), n_(A-3000I), "
          "ILDL(1e-6) preconditioner with |D| (library factorization, 2x2 pivots), m=50, k=6, FP64",
    "c4": "64 independent 3D 7-pt Gaussian-well Hamiltonians, N^3 grids with N~U{16..64} (seeds 1000+b), "
          "4 sorted shifts ~U[-8,-2] each (3 intervals), Chebyshev M=c4(L+I), m=64, k=25, one "
          "block-diagonal launch sequence replayed from a captured graph",
}
BATCH = {"c4": "f64", "c4_f32": "f32"}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _code_only(text: str) -> str:
    """Source text without comments and trailing blanks (the kernels' code:
    counters taken on it stay valid when only a comment changes)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in text.split("\n"))
    return "\n".join(ln for ln in lines if ln)


def kernel_sources_sha(csrc: str | None = None) -> str:
    h = hashlib.sha256()
    csrc = csrc or os.path.join(ROOT, "paper_1602_02306_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            h.update(_code_only(open(os.path.join(csrc, f), encoding="utf-8").read()).encode())
    return h.hexdigest()[:16]


def copy_calib(nbytes: int = 1 << 30):
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calib_bytes_each_way": nbytes, "launches": 3}), flush=True)


def cpu_baseline(P, V, wl, target_s: float, gpu_per_probe=None):
    """The oracle timed on a bounded sample of the probes (whole probes, both
    shifts).  With the GPU's per-probe values of the same run, also how far
    they are from the oracle's on the sampled probes (relative to |v|^2 = n)."""
    import oracle
    threads = oracle.host_threads()
    m = V.shape[1]
    done, t_tot, batch = 0, 0.0, max(1, min(threads, m))
    if wl.method == "block":
        batch = 16
    worst, worst_rel = 0.0, 0.0

    def run(lo, s):
        if wl.method == "arnoldi":
            return oracle.count_arnoldi(P.A, P.prec, wl.xi, wl.eta, V[:, lo:lo + s], wl.k,
                                        nthreads=threads)
        if wl.method == "block":
            return oracle.block_count(P.A, P.prec, wl.xi, wl.eta, V[:, lo:lo + s], wl.k,
                                      nthreads=threads)
        return oracle.count(P.A, P.prec, wl.xi, wl.eta, V[:, lo:lo + s], wl.k,
                            nthreads=threads, smooth_w=wl.smooth_w)

    while done < m:
        s = min(batch, m - done)
        t0 = time.perf_counter()
        ref = run(done, s)
        dt = time.perf_counter() - t0
        if gpu_per_probe is not None:
            gx, ge = gpu_per_probe[done:done + s], gpu_per_probe[m + done:m + done + s]
            worst = max(worst, float(np.max(np.abs(gx - ref.s_xi))), float(np.max(np.abs(ge - ref.s_eta))))
            worst_rel = max(worst_rel,
                            float(np.max(np.abs(gx - ref.s_xi) / np.maximum(1.0, np.abs(ref.s_xi)))),
                            float(np.max(np.abs(ge - ref.s_eta) / np.maximum(1.0, np.abs(ref.s_eta)))))
        t_tot += dt
        done += s
        log("cpu oracle: %d probes in %.1f s (total %.1f s)" % (s, dt, t_tot))
        if t_tot >= target_s:
            break
        per = t_tot / done
        batch = max(1, min(m - done, int((target_s - t_tot) / per) + 1, 4 * threads))
        if wl.method == "block":   # whole blocks of 16 probes
            batch = min(m - done, max(16, (batch + 15) // 16 * 16))
    # a whole workload that runs in far less than a second is timed over
    # repeated passes (about 2 s), so that thread start-up does not dominate
    passes = 1
    if done == m and t_tot < 2.0:
        t0 = time.perf_counter()
        while t_tot + (time.perf_counter() - t0) < 2.0:
            run(0, m)
            passes += 1
        t_tot += time.perf_counter() - t0
    steps = 2 * done * wl.k * passes
    out = {"value": steps / t_tot, "unit": "probe-steps/s", "cores": threads, "kind": "oracle",
           "sample": "%d of %d probes x 2 shifts x k=%d, %d pass%s (%d probe-steps, %.1f s)"
                     % (done, m, wl.k, passes, "" if passes == 1 else "es", steps, t_tot)}
    if gpu_per_probe is not None:
        out["gpu_vs_oracle_max_abs_per_probe_over_n"] = worst / wl.n
        out["gpu_vs_oracle_max_rel_per_probe"] = worst_rel
    return out


def grad_check_sample(ec, A, P, wl, Vd, nprobe: int = 1, seed: int = 5):
    """Sampled check of the differentiated form at full size: the GPU's smoothed
    forward + backward on the first `nprobe` probes (the estimator on that
    probe subset) against the oracle's forward-mode tangents on the same
    subset: <dV, u> for a random direction u, d/dxi and d/deta."""
    import oracle
    import torch
    Vs = Vd[:, :nprobe].contiguous()
    res, ws = ec.smooth_forward(A, P.prec, wl.xi, wl.eta, Vs, wl.k, wl.smooth_w)
    dV, dxi, deta = ec.smooth_backward(A, P.prec, wl.xi, wl.eta, Vs, wl.k, wl.smooth_w, workspace=ws)
    dV = dV.cpu().numpy()
    del ws
    torch.cuda.empty_cache()
    V = Vs.cpu().double().numpy()
    u = np.random.default_rng(seed).standard_normal(wl.n)
    t0 = time.perf_counter()
    est_ref, d_ref = oracle.count_tangent(P.A, P.prec, wl.xi, wl.eta, V, wl.k, u, 0.0, 0.0, wl.smooth_w)
    _, dxi_ref = oracle.count_tangent(P.A, P.prec, wl.xi, wl.eta, V, wl.k, np.zeros(wl.n), 1.0, 0.0,
                                      wl.smooth_w)
    _, deta_ref = oracle.count_tangent(P.A, P.prec, wl.xi, wl.eta, V, wl.k, np.zeros(wl.n), 0.0, 1.0,
                                       wl.smooth_w)
    dt = time.perf_counter() - t0
    d_gpu = float(np.dot(dV, u))
    out = {"probes": nprobe, "oracle_s": dt,
           "estimate_rel": abs(res.estimate - est_ref) / max(1.0, abs(est_ref)),
           "dV_dot_u_rel": abs(d_gpu - d_ref) / abs(d_ref),
           "dxi_rel": abs(dxi - dxi_ref) / max(abs(dxi_ref), 1e-300),
           "deta_rel": abs(deta - deta_ref) / max(abs(deta_ref), 1e-300)}
    log("sampled gradient check (%d probe): %s" % (nprobe, out))
    return out


def cpu_baseline_batch(items, V, off, k: int, target_s: float, m_total: int, gpu_per_probe=None):
    """The oracle on a bounded sample of the batch: problems in order, all
    shifts, the first few probes of each, until about target_s seconds; with
    the GPU's per-probe values (nprob x nshift*m) also their largest distance
    from the oracle's on the sample (relative to |v|^2 = n of the problem)."""
    import oracle
    threads = oracle.host_threads()
    m = V.shape[1]
    mp = min(m, threads)
    steps, t_tot, nprob = 0, 0.0, 0
    worst = 0.0
    for b, it in enumerate(items):
        Vb = np.ascontiguousarray(V[off[b]:off[b + 1], :mp])
        t0 = time.perf_counter()
        for si, tau in enumerate(it.shifts):
            _, s_ref, _, _ = oracle.negcount(it.A, it.prec, float(tau), Vb, k, nthreads=threads)
            if gpu_per_probe is not None:
                g = gpu_per_probe[b, si * m_total:si * m_total + mp]
                worst = max(worst, float(np.max(np.abs(g - s_ref))) / it.A.n)
        t_tot += time.perf_counter() - t0
        steps += len(it.shifts) * mp * k
        nprob += 1
        log("cpu oracle: problem %d (n=%d) done, total %.1f s" % (b, it.A.n, t_tot))
        if t_tot >= target_s:
            break
    out = {"value": steps / t_tot, "unit": "probe-steps/s", "cores": threads, "kind": "oracle",
           "sample": "problems 0..%d of %d, all %d shifts, first %d of %d probes, k=%d "
                     "(%d probe-steps, %.1f s)" % (nprob - 1, len(items), len(items[0].shifts), mp,
                                                  m_total, k, steps, t_tot)}
    if gpu_per_probe is not None:
        out["gpu_vs_oracle_max_abs_per_probe_over_n"] = worst
    return out


def bench_negcount_ldl(args, wl, ceilings=None):
    """n_(A - tau I) with the factored ILDL preconditioner (Table 1 Laplace):
    the library factors A - tau I on the host once (outside the timed
    region); one step = one ecnt_negcounts over the m probes."""
    import torch
    from paper_1602_02306_amd import ecount as ec
    from paper_1602_02306_amd import workloads as W
    P = W.make_problem(wl)
    A = ec.upload_csr(P.A)
    Vd = W.rademacher_torch(wl.n, wl.m, wl.probe_seed, device="cuda", dtype=torch.float64)
    taus = list(wl.taus)
    S = len(taus)
    t0 = time.perf_counter()
    host = [ec.ildl_factor(P.A, t, wl.droptol) for t in taus]
    t_fac = time.perf_counter() - t0
    prec = ec.LDLPrecond([ec.upload_ldl(h) for h in host])
    log("ILDL(%g): %.2f s on the host, nnz(L) %s, bandwidth %s, 2x2 blocks %s" % (
        wl.droptol, t_fac, [h.l_val.size for h in host], [h.bandwidth for h in host],
        [h.n2x2 for h in host]))
    # the exact count: Sylvester inertia of the exact factorization (no dropping)
    exact = [ec.ildl_factor(P.A, t, 0.0).nneg for t in taus]
    need = ec.workspace_bytes(wl.n, wl.m, S, prec, wl.k)
    ws = ec.Workspace(need)

    def one(details=False):
        return ec.negcounts(A, prec, taus, Vd, wl.k, workspace=ws, details=details)

    for i in range(args.warmup):
        r = one()
        log("warmup %d: negcounts %s" % (i, r.negcounts))
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ec.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        r = one()
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ec.profile_enable(False)
    prof = ec.profile_read()
    ms = max((t1 - t0) * 1e3 / args.steps, ev0.elapsed_time(ev1) / args.steps)
    probe_steps = S * wl.m * wl.k
    value = probe_steps / (ms / 1e3)
    log("timed %d steps: %.3f ms/step, %.0f probe-steps/s" % (args.steps, ms, value))
    fams = {k: v for k, v in prof.items() if v["launches"] > 0}
    total_kernel_ms = sum(v["ms"] for v in fams.values())
    dom = max((f for f in fams if fams[f]["bytes"] > 0), key=lambda f: fams[f]["ms"])
    d = fams[dom]
    per_launch_bytes = d["bytes"] / d["launches"]
    per_launch_ms = d["ms"] / d["launches"]
    achieved = per_launch_bytes / (per_launch_ms / 1e3) / 1e9
    kernels = {f: {"launches_per_step": v["launches"] / args.steps, "ms_per_step": v["ms"] / args.steps,
                   "share": v["ms"] / total_kernel_ms if total_kernel_ms else None,
                   "gbs": (v["bytes"] / (v["ms"] / 1e3) / 1e9) if v["ms"] > 0 and v["bytes"] > 0 else None}
               for f, v in fams.items()}
    est = float(r.negcounts[0])
    out = {
        "metric": "Lanczos probe-steps/s + HBM GB/s at fixed count error vs LDLᵀ inertia",
        "value": value, "unit": "probe-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl.name + ": " + WORKLOAD_TEXT.get(wl.name, ""), "n": wl.n,
                   "probes": wl.m, "shifts": S, "columns": S * wl.m, "k": wl.k,
                   "probe_steps_per_step": probe_steps, "droptol": wl.droptol,
                   "factor_seconds_host": t_fac},
        "hbm_gbs_algorithmic": sum(v["bytes"] for v in fams.values()) / args.steps / (ms / 1e3) / 1e9,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": per_launch_bytes, "avg_launch_ms": per_launch_ms,
                     "note": "the triangular solves walk the rows in sequence (the columns are the "
                             "parallel dimension), so this path is bound by the per-row latency "
                             "chain, not by HBM"},
        "kernels": kernels,
        "accuracy": {"estimate": est, "std_error": None, "exact_count": exact[0],
                     "method_exact": "LDL^T Sylvester inertia (library, exact factorization)",
                     "abs_error": abs(est - exact[0]), "rel_error": abs(est - exact[0]) / exact[0]},
        "kernel_sources_sha": kernel_sources_sha(),
    }
    rd = one(details=True)
    gpu_pp = rd.per_probe.cpu().numpy()
    if not args.no_cpu_baseline:
        import oracle
        V = Vd.cpu().double().numpy()
        threads = oracle.host_threads()
        t0 = time.perf_counter()
        F = oracle.ildl(P.A, taus[0], wl.droptol)
        t_ofac = time.perf_counter() - t0
        done, t_tot, worst = 0, 0.0, 0.0
        batch = min(threads, wl.m)
        while done < wl.m and t_tot < args.cpu_seconds:
            s_ = min(batch, wl.m - done)
            t0 = time.perf_counter()
            res = oracle.lanczos_ldl(P.A, F, taus[0], V[:, done:done + s_], wl.k, nthreads=threads)
            s_ref, _ = oracle.quadrature(res)
            t_tot += time.perf_counter() - t0
            worst = max(worst, float(np.max(np.abs(gpu_pp[done:done + s_] - s_ref))))
            done += s_
        # a whole workload that runs in far less than a second is timed over
        # repeated passes (about 2 s), so that thread start-up does not dominate
        passes = 1
        if done == wl.m and t_tot < 2.0:
            t0 = time.perf_counter()
            while t_tot + (time.perf_counter() - t0) < 2.0:
                oracle.quadrature(oracle.lanczos_ldl(P.A, F, taus[0], V, wl.k, nthreads=threads))
                passes += 1
            t_tot += time.perf_counter() - t0
        steps_ = done * wl.k * passes
        out["cpu_baseline"] = {"value": steps_ / t_tot, "unit": "probe-steps/s", "cores": threads,
                               "kind": "oracle",
                               "sample": "%d of %d probes x 1 shift x k=%d, %d pass%s (%d probe-steps, "
                                         "%.1f s; the oracle's own ILDL factorization, %.1f s, not "
                                         "counted)" % (done, wl.m, wl.k, passes, "" if passes == 1 else "es",
                                                       steps_, t_tot, t_ofac),
                               "gpu_vs_oracle_max_abs_per_probe_over_n": worst / wl.n}
    print(json.dumps(out), flush=True)


def bench_graph_single(args, name: str):
    """One small interval count (the 30x30 problem) as a graph replay: the
    count's launch sequence (a batch of one problem) captured once into a
    hipGraph and replayed, each replay followed by the results copy.  One
    step = one whole count; the eager single-problem call is timed beside it."""
    import torch
    from paper_1602_02306_amd import ecount as ec
    from paper_1602_02306_amd import workloads as W
    wl = W.WORKLOADS[name]
    P = W.make_problem(wl)
    A = ec.upload_csr(P.A)
    Vd = W.rademacher_torch(wl.n, wl.m, wl.probe_seed, device="cuda", dtype=torch.float64)
    dims = [wl.dims] if P.prec.kind == "cheb" else None
    bt = ec.Batch(A, P.prec, [wl.n], np.array([[wl.xi, wl.eta]]), Vd, wl.k, dims=dims, details=True)
    steps = max(args.steps, 200)
    for _ in range(max(args.warmup, 3)):
        r = bt.run()
    g = bt.capture()
    g.replay()
    r = bt.results()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
        r = bt.results()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    # the eager single-problem call, same inputs
    ws = ec.Workspace(ec.workspace_bytes(wl.n, wl.m, 2, P.prec, wl.k))
    for _ in range(3):
        re = ec.count(A, P.prec, wl.xi, wl.eta, Vd, wl.k, workspace=ws, details=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        re = ec.count(A, P.prec, wl.xi, wl.eta, Vd, wl.k, workspace=ws, details=False)
    ms_eager = (time.perf_counter() - t0) * 1e3 / steps
    rd = ec.count(A, P.prec, wl.xi, wl.eta, Vd, wl.k, workspace=ws, details=True)
    same = bool(torch.equal(rd.per_probe, r.per_probe[0]))
    est, var = float(r.counts[0, 0]), float(r.variances[0, 0])
    probe_steps = 2 * wl.m * wl.k
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "exact_counts.json")))
    exact = golden.get(wl.name, {}).get("count")
    log("graph replay %.3f ms per count, eager %.3f ms; estimate %.6f (eager %.6f, per-probe bitwise %s)"
        % (ms, ms_eager, est, re.estimate, same))
    out = {
        "metric": "Lanczos probe-steps/s + HBM GB/s at fixed count error vs LDLᵀ inertia",
        "value": probe_steps / (ms / 1e3), "unit": "probe-steps/s", "n_gpus": 1, "steps": steps,
        "warmup": max(args.warmup, 3), "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": name + "_graph: " + WORKLOAD_TEXT.get(name, "") +
                   "; one count = one hipGraph replay of its launch sequence + the results copy",
                   "n": wl.n, "probes": wl.m, "shifts": 2, "k": wl.k, "probe_steps_per_step": probe_steps},
        "latency": {"graph_ms_per_count": ms, "eager_ms_per_count": ms_eager,
                    "graph_equals_eager_bitwise": same},
        "roofline": {"bound": "latency", "kernel": None, "achieved": None, "peak": None, "unit": None,
                     "frac": None, "traffic": None,
                     "note": "the 30x30 working set (12 MB) stays in cache: launch- and latency-bound"},
        "accuracy": {"estimate": est, "std_error": math.sqrt(var), "exact_count": exact,
                     "method_exact": "dense eigendecomposition",
                     "abs_error": abs(est - exact) if exact is not None else None,
                     "rel_error": abs(est - exact) / exact if exact else None},
        "kernel_sources_sha": kernel_sources_sha(),
    }
    if not args.no_cpu_baseline:
        V = Vd.cpu().double().numpy()
        out["cpu_baseline"] = cpu_baseline(P, V, wl, args.cpu_seconds, r.per_probe[0].cpu().numpy())
    print(json.dumps(out), flush=True)


def bench_batched(args, name: str, ceilings=None):
    """The batched form: 64 problems of uneven size in one launch sequence,
    captured once into a graph and replayed; one step = one whole batch."""
    import torch
    from paper_1602_02306_amd import autotune
    from paper_1602_02306_amd import ecount as ec
    from paper_1602_02306_amd import workloads as W
    vec = BATCH[name]
    nprob, m, k = 64, 64, 25
    t0 = time.perf_counter()
    items = [W.batched_item(b) for b in range(nprob)]
    sizes = [it.A.n for it in items]
    dims = [it.dims for it in items]
    taus = np.stack([it.shifts for it in items])
    S = taus.shape[1]
    Abd = W.block_diag_csr([it.A for it in items])
    off = np.concatenate([[0], np.cumsum(sizes)])
    log("built %d problems, %d rows, %d nonzeros in %.1f s" % (nprob, Abd.n, Abd.nnz,
                                                              time.perf_counter() - t0))
    prec = items[0].prec
    A = ec.upload_csr(Abd, val_dtype=vec)
    del Abd
    tdt = torch.float32 if vec == "f32" else torch.float64
    Vd = W.rademacher_torch(int(off[-1]), m, 4242, device="cuda", dtype=tdt)
    free, _total = torch.cuda.mem_get_info()
    budget = free - (16 << 30)
    if args.tune == "off":
        Ct = S * m
        w = Ct
        while w > 32 and ec.batch_workspace_bytes(sizes, dims, S, m, prec, k, vec=vec,
                                                  max_cols=0 if w == Ct else w) > budget:
            w //= 2
        cfg = {"max_cols": w, "tile": "auto", "red_waves": 0, "csr_vw": 0, "source": "defaults"}
    else:
        cfg = autotune.tune_batch(A, prec, sizes, taus, Vd, k, dims=dims, vec=vec,
                                  mem_bytes=budget, retune=args.tune == "search", log=log)
    log("launch shape (%s): %s" % (cfg["source"], {x: cfg[x] for x in ("max_cols", "tile",
                                                                      "red_waves", "csr_vw")}))
    Ct = S * m
    tune = {x: cfg[x] for x in autotune.DEFAULTS}
    max_cols = 0 if cfg["max_cols"] == Ct else cfg["max_cols"]
    bt = ec.Batch(A, prec, sizes, taus, Vd, k, dims=dims, vec=vec, max_cols=max_cols, tune=tune)
    log("workspace %.2f GiB" % (bt.ws.nbytes / 2 ** 30))
    for i in range(args.warmup):
        r = bt.run()
        log("warmup %d: sum of negcounts %.6f" % (i, float(r.negcounts.sum())))
    g = bt.capture()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        g.replay()
        r = bt.results()
    ev1.record(stream)
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    ms = max((w1 - w0) * 1e3 / args.steps, ev0.elapsed_time(ev1) / args.steps)
    probe_steps = nprob * S * m * k
    value = probe_steps / (ms / 1e3)
    log("timed %d graph replays: %.3f ms/batch, %.0f probe-steps/s" % (args.steps, ms, value))
    # per-family event timings from one eager run of the same launches
    ec.profile_enable(True)
    r2 = bt.run()
    ec.profile_enable(False)
    assert np.array_equal(r2.negcounts, r.negcounts)
    fams = {f: v for f, v in ec.profile_read().items() if v["launches"] > 0}
    total_kernel_ms = sum(v["ms"] for v in fams.values())
    dom = max((f for f in fams if fams[f]["bytes"] > 0), key=lambda f: fams[f]["ms"])
    d = fams[dom]
    per_launch_bytes = d["bytes"] / d["launches"]
    per_launch_ms = d["ms"] / d["launches"]
    achieved = per_launch_bytes / (per_launch_ms / 1e3) / 1e9
    algo_bytes = sum(v["bytes"] for v in fams.values())
    out = {
        "metric": "Lanczos probe-steps/s + HBM GB/s at fixed count error vs LDLᵀ inertia",
        "value": value, "unit": "probe-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if vec == "f64" else "f32-storage/f64-accumulate",
        "data": "synthetic",
        "config": {"workload": name + ": " + WORKLOAD_TEXT["c4"], "problems": nprob,
                   "rows": int(off[-1]), "probes": m, "shifts": S, "columns_per_problem": Ct,
                   "k": k, "probe_steps_per_step": probe_steps,
                   "launch_shape": {x: cfg[x] for x in ("max_cols", "tile", "red_waves", "csr_vw")},
                   "tuned": cfg["source"]},
        "hbm_gbs_algorithmic": algo_bytes / (total_kernel_ms / 1e3) / 1e9 if total_kernel_ms else None,
        "algorithmic_bytes_per_probe_step": algo_bytes / probe_steps,
        "roofline": add_ceiling({"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                                 "algorithmic_bytes_per_launch": per_launch_bytes,
                                 "avg_launch_ms": per_launch_ms}, ceilings),
        "kernels": {f: {"launches_per_step": v["launches"], "ms_per_step": v["ms"],
                        "share": v["ms"] / total_kernel_ms,
                        "gbs": (v["bytes"] / (v["ms"] / 1e3) / 1e9) if v["bytes"] > 0 else None}
                    for f, v in fams.items()},
        "eager_kernel_ms": total_kernel_ms,
        "result": {"sum_negcounts": float(r.negcounts.sum()),
                   "counts_first_problem": [float(x) for x in r.counts[0]]},
        "accuracy": batch_accuracy(r),
        "kernel_sources_sha": kernel_sources_sha(),
    }
    if not args.no_cpu_baseline:
        V = Vd[:, :16].cpu().double().numpy()
        # per-probe values of the same batch (one more eager run with details)
        btd = ec.Batch(A, prec, sizes, taus, Vd, k, dims=dims, vec=vec, max_cols=max_cols,
                       tune=tune, workspace=bt.ws, details=True)
        pp = btd.run().per_probe.cpu().numpy()
        out["cpu_baseline"] = cpu_baseline_batch(items, V, off, k, args.cpu_seconds, m, pp)
    print(json.dumps(out), flush=True)


def batch_accuracy(r):
    """The batch's slice counts against the exact counts of the 64 problems
    (LDL^T inertia at every shift, tests/golden/exact_counts.json)."""
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "exact_counts.json"))).get("c4")
    if not golden or len(golden["items"]) < r.counts.shape[0]:
        return None
    ex = np.array([it["counts"] for it in golden["items"][:r.counts.shape[0]]], dtype=np.float64)
    est = np.asarray(r.counts)
    rel = (est - ex) / np.maximum(ex, 1.0)
    tot_est, tot_ex = float(est.sum()), float(ex.sum())
    return {"slices": int(ex.size), "exact_total": tot_ex, "estimate_total": tot_est,
            "total_rel_error": (tot_est - tot_ex) / tot_ex,
            "median_abs_rel_error": float(np.median(np.abs(rel))),
            "mean_abs_rel_error": float(np.mean(np.abs(rel))),
            "slices_within_5pct": float(np.mean(np.abs(rel) <= 0.05)),
            "method_exact": "LDL^T Sylvester inertia (nested dissection)"}


CEILING_KIND = {"lz_update": "update_mix", "bw_update": "update_mix", "blk_update": "update_mix",
                "lz_dots": "read", "bw_dots": "read", "blk_dots": "read"}


def measure_ceilings(args):
    """Tuned streams on this device (ecnt_hbm_probe: 1 GiB streams), measured
    in the same run as the bench: what the sweeps' access mixes can reach."""
    if args.no_ceiling:
        return None
    import torch
    from paper_1602_02306_amd import ecount as ec
    free, _ = torch.cuda.mem_get_info()
    nbytes = 18 << 30 if free > (40 << 30) else 1 << 30
    out = {k: ec.hbm_probe(k, nbytes if k == "update_mix" else min(nbytes, 2 << 30))
           for k in ("copy", "read", "update_mix")}
    torch.cuda.empty_cache()
    log("HBM ceilings (GB/s): %s" % {k: round(v) for k, v in out.items()})
    return out


def add_ceiling(roof: dict, ceilings):
    """The dominant kernel's achieved GB/s against the tuned stream of its own
    access mix (besides the data-sheet peak in `frac`)."""
    if not ceilings or not roof.get("kernel"):
        return roof
    kind = CEILING_KIND.get(roof["kernel"], "copy")
    roof["ceiling"] = {"kind": kind, "gbs": ceilings[kind], "frac": roof["achieved"] / ceilings[kind],
                       "measured": {k: v for k, v in ceilings.items()}}
    return roof


def traffic_from_profiles(family: str, per_launch_algo: float, workload: str = "c2"):
    """HBM bytes per launch from committed rocprofv3 counter runs of this
    workload (profiles/counters.json for c2, counters_<workload>.json for the
    others), if they were taken on the current kernel sources."""
    name = "counters.json" if workload == "c2" else "counters_%s.json" % workload
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_sha") != kernel_sources_sha():
        return None
    ent = d.get("kernels", {}).get(family)
    if not ent:
        return None
    return ent.get("hbm_bytes_per_launch")


FAMILY_OF = [("k_blk_update<true>", "blk_normalize"), ("k_blk_update", "blk_update"),
             ("k_blk_dots_fin", "lz_finalize"), ("k_blk_norm_fin", "lz_finalize"),
             ("k_blk_dots", "blk_dots"), ("k_blk_quad", "blk_quadrature"),
             ("k_ldl_solve", "op_ldl_solve"), ("k_ldl_eapply", "op_ldl_elementwise"),
             ("k_ldl_permute", "op_ldl_elementwise"), ("k_ldl_band", "lz_setup"),
             ("k_ldl_eblocks", "lz_setup"),
             ("k_quad_sweep", "op_cheb_quad"), ("k_arn_quad", "quadrature"),
             ("k_arn_fin", "lz_finalize"), ("k_arn_norm_fin", "lz_finalize"),
             ("k_bdots_fin", "lz_finalize"),
             ("k_bnorm_fin", "lz_finalize"), ("k_rowsum", "lz_finalize"), ("k_vgrad", "bw_vgrad"),
             ("k_bdots", "bw_dots"), ("k_bupdate", "bw_update"), ("k_grad_", "lz_finalize"),
             ("k_stencil_check", "lz_setup"), ("k_stencil_a", "op_a_stencil"),
             ("k_stencil", "op_cheb_sweep"), ("k_csr_op", "op_csr"), ("k_dots_fin", "lz_finalize"),
             ("k_dots", "lz_dots"), ("k_update", "lz_update"), ("k_setup_fin", "lz_finalize"),
             ("k_setup", "lz_setup"), ("k_norm_fin", "lz_finalize"), ("k_jacobi_diag", "lz_setup"),
             ("k_tridiag", "quadrature"), ("k_reduce", "quadrature"), ("k_init", "lz_finalize"),
             ("k_probe", "hbm_probe"), ("k_lanczos_fused", "lz_fused"), ("copyBuffer", "copy"),
             ("FillFunc", "fill")]


def family(kernel_name: str) -> str:
    for key, fam in FAMILY_OF:
        if key in kernel_name:
            return fam
    return kernel_name[:48]


def summarize(trace_dir: str, pmc_dir: str | None, command: str, workload: str):
    """Markdown summary of rocprofv3 output: per kernel family, launches, total
    and average duration (kernel trace), and, when counter runs are given,
    calibrated HBM bytes per launch from FETCH_SIZE / WRITE_SIZE (scaled by
    what the same counters read for a plain device copy of known size)."""
    import csv
    import collections
    import glob

    def one(pattern):
        files = glob.glob(os.path.join(pattern), recursive=True)
        return files[0] if files else None

    trace = one(os.path.join(trace_dir, "**", "*kernel_trace.csv"))
    fams = collections.defaultdict(lambda: [0, 0.0])
    for r in csv.DictReader(open(trace)):
        f = family(r["Kernel_Name"])
        fams[f][0] += 1
        fams[f][1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
    total = sum(v[1] for v in fams.values())
    lines = ["# rocprofv3 summary: %s" % workload, "", "Command (from the repository root):", "",
             "    " + command, "",
             "| kernel family | launches | total ms | share | avg ms/launch |",
             "|---|---:|---:|---:|---:|"]
    for f, (n, ms) in sorted(fams.items(), key=lambda x: -x[1][1]):
        lines.append("| %s | %d | %.3f | %.1f%% | %.4f |" % (f, n, ms, 100 * ms / total, ms / n))
    counters = {}
    if pmc_dir:
        calib = {}
        per = {}
        for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
            cf = one(os.path.join(pmc_dir, "pmc_copy_" + ctr, "**", "*counter_collection.csv"))
            copies = [float(r["Counter_Value"]) for r in csv.DictReader(open(cf))
                      if "copyBuffer" in r["Kernel_Name"]]
            # each copy moves 1 GiB each way: KiB expected / KiB counted
            calib[ctr] = (2 ** 20) / (sum(copies) / len(copies))
            kf = one(os.path.join(pmc_dir, "pmc_" + ctr, "**", "*counter_collection.csv"))
            acc = collections.defaultdict(lambda: [0, 0.0])
            for r in csv.DictReader(open(kf)):
                a = acc[family(r["Kernel_Name"])]
                a[0] += 1
                a[1] += float(r["Counter_Value"])
            per[ctr] = acc
        lines += ["", "Counter calibration (plain 1 GiB device copy): FETCH_SIZE x %.3f, "
                      "WRITE_SIZE x %.3f" % (calib["FETCH_SIZE"], calib["WRITE_SIZE"]), "",
                  "| kernel family | fetch GiB/launch | write GiB/launch | HBM GiB/launch (calibrated) |",
                  "|---|---:|---:|---:|"]
        for f in sorted(per["FETCH_SIZE"], key=lambda f: -per["FETCH_SIZE"][f][1]):
            nf, vf = per["FETCH_SIZE"][f]
            nw, vw = per["WRITE_SIZE"].get(f, [1, 0.0])
            fg = vf / nf * calib["FETCH_SIZE"] / 2 ** 20
            wg = vw / max(nw, 1) * calib["WRITE_SIZE"] / 2 ** 20
            if fg + wg < 1e-3:
                continue
            counters[f] = {"fetch_bytes_per_launch": fg * 2 ** 30, "write_bytes_per_launch": wg * 2 ** 30,
                           "hbm_bytes_per_launch": (fg + wg) * 2 ** 30}
            lines.append("| %s | %.3f | %.3f | %.3f |" % (f, fg, wg, fg + wg))
    return "\n".join(lines) + "\n", counters


def k_sweep(args):
    """Accuracy against the exact count versus k: for each k (and rule), one
    warm-up and one event-timed count on the workload's probes; prints one
    JSON line per run.  Throughput at a stated count error is read off these
    lines (the smallest k whose error is below the target)."""
    import torch
    from paper_1602_02306_amd import ecount as ec
    from paper_1602_02306_amd import workloads as W
    wl = W.WORKLOADS[args.workload]
    P = W.make_problem(wl)
    A = ec.upload_csr(P.A)
    Vd = W.rademacher_torch(wl.n, wl.m, wl.probe_seed, device="cuda", dtype=torch.float64)
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "exact_counts.json")))
    base = wl.name.replace("_arn", "").replace("_blk", "")
    exact = golden.get(wl.name, golden.get(base, {})).get("count")
    rules = ["gauss"] if wl.method != "lanczos" else args.rules.split(",")
    ws = ec.Workspace(1)
    for k in [int(x) for x in args.k_sweep.split(",")]:
        for rule in rules:
            def run():
                if wl.method == "block":
                    need = ec.block_workspace_bytes(wl.n, wl.m, P.prec, k)
                    return ec.count_block(A, P.prec, wl.xi, wl.eta, Vd, k, workspace=ws.ensure(need),
                                          details=False)
                if wl.method == "arnoldi":
                    need = ec.arnoldi_workspace_bytes(wl.n, wl.m, P.prec, k)
                    return ec.count_arnoldi(A, P.prec, wl.xi, wl.eta, Vd, k, workspace=ws.ensure(need),
                                            details=False)
                need = ec.workspace_bytes(wl.n, wl.m, 2, P.prec, k, rule=rule)
                return ec.count(A, P.prec, wl.xi, wl.eta, Vd, k, rule=rule, workspace=ws.ensure(need),
                                details=False)
            run()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            r = run()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            rec = {"workload": wl.name, "form": wl.method, "rule": rule, "k": k, "estimate": r.estimate,
                   "std_error": math.sqrt(r.variance), "exact_count": exact,
                   "rel_error": (r.estimate - exact) / exact if exact else None,
                   "ms_per_count": ms, "probe_steps_per_s": 2 * wl.m * k / (ms / 1e3)}
            print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-ceiling", action="store_true", help="skip the HBM stream probes")
    ap.add_argument("--copy-calib", action="store_true")
    ap.add_argument("--k-sweep", metavar="K1,K2,...",
                    help="count error against the exact count and probe-steps/s at each k "
                    "(rules from --rules; one JSON line per run) and exit")
    ap.add_argument("--rules", default="gauss,ga", help="with --k-sweep: gauss, ga (single-vector form)")
    ap.add_argument("--summarize", metavar="TRACE_DIR",
                    help="print a markdown summary of a rocprofv3 kernel trace and exit")
    ap.add_argument("--pmc-dir", help="with --summarize: directory holding the counter runs")
    ap.add_argument("--command", default="", help="with --summarize: the profiled command")
    ap.add_argument("--counters-json", help="with --summarize: write calibrated per-launch bytes here")
    ap.add_argument("--tune", choices=["auto", "off", "search"], default="auto",
                    help="launch shapes: auto = tuned table (user cache, then the shipped one) or "
                    "a search if the size class is in neither; off = built-in defaults; search = "
                    "search again")
    args = ap.parse_args()

    if args.summarize:
        text, counters = summarize(args.summarize, args.pmc_dir, args.command, args.workload)
        print(text)
        if args.counters_json and counters:
            json.dump({"source_sha": kernel_sources_sha(), "workload": args.workload,
                       "command": args.command, "kernels": counters},
                      open(args.counters_json, "w"), indent=1)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs the estimator on a single "
              "MI355X (probe columns would shard across GPUs with one 32-byte all-reduce at the "
              "end, which is not implemented); got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.copy_calib:
        copy_calib()
        return

    if args.k_sweep:
        k_sweep(args)
        return
    ceilings = measure_ceilings(args)
    if args.workload in BATCH:
        bench_batched(args, args.workload, ceilings)
        return
    if args.workload == "c1_graph":
        bench_graph_single(args, "c1")
        return
    if args.workload == "t1":
        from paper_1602_02306_amd import workloads as W
        bench_negcount_ldl(args, W.WORKLOADS["t1"], ceilings)
        return

    from paper_1602_02306_amd import ecount as ec
    from paper_1602_02306_amd import workloads as W

    wl = W.WORKLOADS[args.workload]
    log("building inputs", wl.name, "n=%d m=%d k=%d" % (wl.n, wl.m, wl.k))
    P = W.make_problem(wl)
    vec = wl.vec
    tdt = torch.float32 if vec == "f32" else torch.float64
    A = ec.upload_csr(P.A, val_dtype=vec)
    # probes generated in HBM (bitwise the same block as workloads.rademacher)
    Vd = W.rademacher_torch(wl.n, wl.m, wl.probe_seed, device="cuda", dtype=tdt)
    S = 2
    grad = wl.smooth_w > 0.0
    # FP32 128^3 form: one shift (m columns) per wave bounds the basis to 124 GiB
    max_cols = wl.m if wl.name == "c3" else 0
    tune, tuned = None, None
    arn = wl.method == "arnoldi"
    blk = wl.method == "block"
    if not grad and not arn and not blk and args.tune != "off":
        from paper_1602_02306_amd import autotune
        free, _total = torch.cuda.mem_get_info()
        cfg = autotune.tune_count(A, P.prec, wl.xi, wl.eta, Vd, wl.k, vec=vec,
                                  mem_bytes=free - (16 << 30), retune=args.tune == "search",
                                  log=log)
        max_cols = 0 if cfg["max_cols"] == S * wl.m else cfg["max_cols"]
        tune = {x: cfg[x] for x in autotune.DEFAULTS}
        tuned = {"source": cfg["source"], "max_cols": cfg["max_cols"], **tune}
        log("launch shape (%s): %s" % (cfg["source"], tuned))
    if grad:
        need = ec.smooth_workspace_bytes(wl.n, wl.m, P.prec, wl.k, wl.smooth_w)
    elif arn:
        need = ec.arnoldi_workspace_bytes(wl.n, wl.m, P.prec, wl.k, vec=vec, max_cols=max_cols)
    elif blk:
        need = ec.block_workspace_bytes(wl.n, wl.m, P.prec, wl.k, max_cols=max_cols)
    else:
        need = ec.workspace_bytes(wl.n, wl.m, S, P.prec, wl.k, vec=vec, smooth_w=wl.smooth_w,
                                  max_cols=max_cols)
    ws = ec.Workspace(need)
    log("workspace %.2f GiB" % (need / 2 ** 30))
    grad_times = {}

    def one():
        if arn:
            return ec.count_arnoldi(A, P.prec, wl.xi, wl.eta, Vd, wl.k, vec=vec, workspace=ws,
                                    details=False, max_cols=max_cols)
        if blk:
            return ec.count_block(A, P.prec, wl.xi, wl.eta, Vd, wl.k, workspace=ws, details=False,
                                  max_cols=max_cols)
        if not grad:
            return ec.count(A, P.prec, wl.xi, wl.eta, Vd, wl.k, vec=vec, smooth_w=wl.smooth_w,
                            workspace=ws, details=False, max_cols=max_cols, tune=tune)
        # differentiated form: forward keeping the basis, then the backward
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        res, _ = ec.smooth_forward(A, P.prec, wl.xi, wl.eta, Vd, wl.k, wl.smooth_w, workspace=ws)
        e1.record()
        dV, dxi, deta = ec.smooth_backward(A, P.prec, wl.xi, wl.eta, Vd, wl.k, wl.smooth_w,
                                           workspace=ws)
        e2.record()
        torch.cuda.synchronize()
        grad_times.setdefault("fwd_ms", []).append(e0.elapsed_time(e1))
        grad_times.setdefault("bwd_ms", []).append(e1.elapsed_time(e2))
        grad_times["dxi"], grad_times["deta"] = dxi, deta
        grad_times["dV_norm"] = float(torch.linalg.vector_norm(dV))
        return res

    for i in range(args.warmup):
        r = one()
        log("warmup %d: estimate %.6f" % (i, r.estimate))
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ec.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        r = one()
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ec.profile_enable(False)
    prof = ec.profile_read()
    wall_ms = (t1 - t0) * 1e3 / args.steps
    ev_ms = ev0.elapsed_time(ev1) / args.steps
    ms = max(wall_ms, ev_ms)
    probe_steps = S * wl.m * wl.k
    value = probe_steps / (ms / 1e3)
    log("timed %d steps: %.3f ms/step (events %.3f), %.0f probe-steps/s" % (args.steps, ms, ev_ms, value))

    fams = {k: v for k, v in prof.items() if v["launches"] > 0}
    total_kernel_ms = sum(v["ms"] for v in fams.values())
    algo_bytes = sum(v["bytes"] for v in fams.values()) / args.steps
    # the dominant kernel: most time among the families that stream block vectors
    dom = max((f for f in fams if fams[f]["bytes"] > 0), key=lambda f: fams[f]["ms"])
    d = fams[dom]
    per_launch_bytes = d["bytes"] / d["launches"]
    per_launch_ms = d["ms"] / d["launches"]
    achieved = per_launch_bytes / (per_launch_ms / 1e3) / 1e9
    traffic = traffic_from_profiles(dom, per_launch_bytes, wl.name)
    kernels = {f: {"launches_per_step": v["launches"] / args.steps,
                   "ms_per_step": v["ms"] / args.steps,
                   "share": v["ms"] / total_kernel_ms if total_kernel_ms else None,
                   "gbs": (v["bytes"] / (v["ms"] / 1e3) / 1e9) if v["ms"] > 0 and v["bytes"] > 0 else None}
               for f, v in fams.items()}

    exact = None
    gpath = os.path.join(ROOT, "tests", "golden", "exact_counts.json")
    if os.path.exists(gpath):
        golden = json.load(open(gpath))
        # the FP32 storage form of a problem has the problem's exact count
        base = wl.name.replace("_f32", "").replace("_arn", "").replace("_blk", "")
        exact = golden.get(wl.name, golden.get(base, {})).get("count")
    accuracy = {"estimate": r.estimate, "std_error": math.sqrt(r.variance) if r.variance == r.variance else None,
                "exact_count": exact, "method_exact": "LDL^T Sylvester inertia" if exact is not None else None,
                "abs_error": abs(r.estimate - exact) if exact is not None else None,
                "rel_error": abs(r.estimate - exact) / exact if exact else None}

    out = {
        "metric": "Lanczos probe-steps/s + HBM GB/s at fixed count error vs LDLᵀ inertia",
        "value": value,
        "unit": "probe-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if vec == "f64" else "f32-storage/f64-accumulate",
        "data": "synthetic",
        "config": {"workload": wl.name + ": " + WORKLOAD_TEXT.get(wl.name, ""), "n": wl.n,
                   "probes": wl.m, "shifts": S, "columns": S * wl.m, "k": wl.k,
                   "probe_steps_per_step": probe_steps},
        "hbm_gbs_algorithmic": algo_bytes / (ms / 1e3) / 1e9,
        "algorithmic_bytes_per_probe_step": algo_bytes / probe_steps,
        "roofline": add_ceiling({"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                                 "algorithmic_bytes_per_launch": per_launch_bytes,
                                 "avg_launch_ms": per_launch_ms}, ceilings),
        "kernels": kernels,
        "accuracy": accuracy,
        "kernel_sources_sha": kernel_sources_sha(),
    }
    if grad:
        # the same number of timed steps with the basis recomputed inside the backward
        rec = []
        for i in range(max(1, args.steps // 2)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ec.smooth_backward(A, P.prec, wl.xi, wl.eta, Vd, wl.k, wl.smooth_w, ckpt="recompute",
                               workspace=ws)
            e1.record()
            torch.cuda.synchronize()
            rec.append(e0.elapsed_time(e1))
        f = grad_times["fwd_ms"][-args.steps:]
        b = grad_times["bwd_ms"][-args.steps:]
        out["differentiated"] = {
            "step": "smoothed forward + backward (dV in R^n, dxi, deta), basis kept",
            "fwd_ms": sum(f) / len(f), "bwd_keep_ms": sum(b) / len(b),
            "bwd_recompute_ms": sum(rec) / len(rec),
            "fwd_probe_steps_per_s": probe_steps / (sum(f) / len(f) / 1e3),
            "dxi": grad_times["dxi"], "deta": grad_times["deta"], "dV_norm": grad_times["dV_norm"],
            "workspace_gib": need / 2 ** 30}
    if blk:
        # the block form's 16 x 16 contractions on the FP64 matrix cores: G_l = X_l^T Y and
        # Y -= X_l K_l cost 2 * 16 * 16 * n flops per basis block per column block at step i
        nblk = S * wl.m // 16
        step_flops = 2.0 * 16 * 16 * wl.n * nblk * (wl.k * (wl.k + 1) // 2)
        mf = {}
        for fam in ("blk_dots", "blk_update"):
            if fam in fams and fams[fam]["ms"] > 0:
                ms_per_count = fams[fam]["ms"] / args.steps
                mf[fam] = step_flops / (ms_per_count / 1e3) / 1e12
        if mf:
            top = max(mf, key=mf.get)
            out["mfma"] = {"kernel": top, "achieved": mf[top], "peak": 78.6, "unit": "TFLOP/s",
                           "frac": mf[top] / 78.6, "dtype": "f64",
                           "per_kernel_tflops": mf,
                           "note": "secondary: these kernels are HBM-bound (4 flop per byte of "
                                   "basis read against a ridge of 78.6/8 = 9.8)"}
    if max_cols:
        out["config"]["column_waves"] = "%d columns per wave" % max_cols
    if tuned:
        out["config"]["launch_shape"] = tuned
    gpu_pp = None
    if grad:
        # untimed: per-probe smoothed values for the sampled oracle comparison
        rd, _ = ec.smooth_forward(A, P.prec, wl.xi, wl.eta, Vd, wl.k, wl.smooth_w, workspace=ws,
                                  details=True)
        gpu_pp = rd.per_probe.cpu().numpy()
        if not args.no_cpu_baseline:
            del ws
            torch.cuda.empty_cache()
            out["differentiated"]["sampled_check_vs_oracle"] = grad_check_sample(ec, A, P, wl, Vd)
    if not grad:
        # one more run with per-probe outputs (untimed): sampled parity against
        # the oracle below, and the FP32 form against the FP64 path
        if arn:
            rd = ec.count_arnoldi(A, P.prec, wl.xi, wl.eta, Vd, wl.k, vec=vec, workspace=ws,
                                  details=True, max_cols=max_cols)
        elif blk:
            rd = ec.count_block(A, P.prec, wl.xi, wl.eta, Vd, wl.k, workspace=ws, details=True,
                                max_cols=max_cols)
        else:
            rd = ec.count(A, P.prec, wl.xi, wl.eta, Vd, wl.k, vec=vec, workspace=ws, details=True,
                          max_cols=max_cols, tune=tune)
        gpu_pp = rd.per_probe.cpu().numpy()
        if not arn and not blk:
            # the generalized averaged Gauss rule on the same Lanczos coefficients
            # (an untimed run on the same probes: the Lanczos data are bitwise the same,
            # only the quadrature kernel differs)
            rga = ec.count(A, P.prec, wl.xi, wl.eta, Vd, wl.k, vec=vec, rule="ga", workspace=ws,
                           details=False, max_cols=max_cols, tune=tune)
            accuracy["ga_rule"] = {"estimate": rga.estimate,
                                   "std_error": math.sqrt(rga.variance) if rga.variance == rga.variance else None,
                                   "rel_error": abs(rga.estimate - exact) / exact if exact else None}
            log("GA rule on the same probes: %.4f" % rga.estimate)
        if vec == "f32":
            del ws
            torch.cuda.empty_cache()
            A64 = ec.upload_csr(P.A, val_dtype="f64")
            V64 = Vd.double()
            free, _total = torch.cuda.mem_get_info()
            w64 = 2 * wl.m
            while w64 > 16 and ec.workspace_bytes(wl.n, wl.m, 2, P.prec, wl.k,
                                                  max_cols=0 if w64 == 2 * wl.m else w64) > free - (8 << 30):
                w64 //= 2
            r64 = ec.count(A64, P.prec, wl.xi, wl.eta, V64, wl.k, details=True,
                           max_cols=0 if w64 == 2 * wl.m else w64)
            pp64 = r64.per_probe.cpu().numpy()
            accuracy["fp64_path_estimate"] = r64.estimate
            accuracy["fp32_minus_fp64_estimate"] = r.estimate - r64.estimate
            accuracy["fp32_minus_fp64_max_abs_per_probe_over_n"] = float(np.max(np.abs(gpu_pp - pp64))) / wl.n
            if exact is not None:
                accuracy["fp64_path_abs_error"] = abs(r64.estimate - exact)
                accuracy["fp64_path_rel_error"] = abs(r64.estimate - exact) / exact
            log("FP64 path on the same probes: %.6f (FP32 %.6f)" % (r64.estimate, r.estimate))
            del A64, V64
    if not args.no_cpu_baseline:
        V = Vd.cpu().double().numpy()
        out["cpu_baseline"] = cpu_baseline(P, V, wl, args.cpu_seconds, gpu_pp)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
