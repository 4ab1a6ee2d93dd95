"""Throughput of the damped Fisher solve (Algorithm 1 of arXiv 2310.17556) on one MI355X.

Workload (default): n = 4096 samples, m = 4,000,000 parameters, FP32 S = G / sqrt(n) with G iid
N(0,1), column-centered, v iid N(0,1), lambda in {1e-2, 1e-4, 1e-6}; the Gram in scaled FP8
(E4M3 with a power-of-two scale per 32 columns, FP32 accumulation, FP64 across k-slices, exact
FP64 diagonal), FP64 Cholesky / triangular solves and the library's automatic refinement sweep
count (two FP64 sweeps at this shape). One step = one independent one-shot solve per lambda
(three solves, each forming its own Gram). Inputs are drawn on the device before timing starts.

Also reported on the same line: the plain FP32 path and the split-BF16 path on the same workload;
an error table over Gram precision x sweeps x lambda (relative error of x, eps_Sy =
|S^T (y - y*)| / |S^T y*| and the final W-residual, all against FP64); the paper-scale plain FP32
workload (n = 1024, m = 1M, column-scaled S, v in the row space, lambda = 1e-3); the batched path
(n = 2048, m = 2M, 16 lambdas x 8 right-hand sides sharing one Gram) and the uneven batch
(64 problems of log-uniform sizes), each with the errors of every solve against FP64.

Printed: one JSON line with solves/s (value), the Gram kernel's roofline position (timed with
HIP events on the stream it runs on), and the FP64 CPU oracle's throughput on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "solves/s + SYRK MFMA% at n=4096,m=4M: mixed vs FP32, rel err ≤1e-6"
PEAK_TFLOPS = {"bf16x3": 2500.0, "fp32": 157.3, "mxfp8": 5000.0}   # dense MFMA peaks of MI355X
HBM_PEAK_GBS = 8000.0
PREC_CODE = {"fp32": 0, "bf16x3": 1, "mxfp8": 2}
DTYPE = {"fp32": "f32+f64", "bf16x3": "bf16x3+f64", "mxfp8": "fp8(e4m3,mx)+f64"}
PASSES = {"fp32": 1, "bf16x3": 3, "mxfp8": 1}   # matrix-core products per Gram term
CENTERED = True   # every workload's S is column-centered; passed to the library as DFISHER_CENTERED


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def fp64_reference(S, v, lams, chunk=131072):
    """x for each lambda from an FP64 Gram (torch/rocBLAS on the device, independent of the
    library's kernels) and an FP64 Cholesky; used only to report the error of the timed solves."""
    import torch

    n, m = S.shape
    G = torch.zeros((n, n), dtype=torch.float64, device=S.device)
    b = torch.zeros(n, dtype=torch.float64, device=S.device)
    v64 = v.double()
    for c0 in range(0, m, chunk):
        blk = S[:, c0:c0 + chunk].double()
        G += blk @ blk.T
        b += blk @ v64[c0:c0 + chunk]
        del blk
    xs = {}
    for lam in lams:
        L = torch.linalg.cholesky(G + lam * torch.eye(n, dtype=torch.float64, device=S.device))
        y = torch.cholesky_solve(b[:, None], L)[:, 0]
        x = torch.empty(m, dtype=torch.float64, device=S.device)
        for c0 in range(0, m, chunk):
            blk = S[:, c0:c0 + chunk].double()
            x[c0:c0 + chunk] = (v64[c0:c0 + chunk] - blk.T @ y) / lam
            del blk
        xs[lam] = x
    return xs


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ONE_CORE = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
import numpy as np
import oracle, synth
out = {"threads": oracle.num_threads()}
# smallest workload: n = 32, m = 1024, lambda = 1e-2, the whole solve
S = synth.make_S(32, 1024, synth.seed(1), "iid"); v = synth.make_v(S, synth.seed(1), "iid")
t0 = time.perf_counter(); reps = 0
while time.perf_counter() - t0 < 1.0:
    oracle.solve(S, v, 1e-2); reps += 1
out["c1_solves_per_s"] = reps / (time.perf_counter() - t0)
# paper-scale workload n = 1024, m = 1M: Gram, S v and the apply on a column sample (scaled by
# m / sample), the Cholesky and the triangular solves at full n
ms = int(sys.argv[2])
S = synth.make_S(1024, ms, synth.seed(2), "scaled"); v = synth.make_v(S, synth.seed(2), "scaled")
t0 = time.perf_counter(); W = oracle.gram(S, 1e-3); b = oracle.gemv(S, v); t1 = time.perf_counter()
L, info = oracle.cholesky(W); y = oracle.backward(L, oracle.forward(L, b)); t2 = time.perf_counter()
oracle.apply(S, v, y, 1e-3); t3 = time.perf_counter()
out["c2_seconds_estimate"] = (t1 - t0 + t3 - t2) * (1_000_000 / ms) + (t2 - t1)
out["c2_solves_per_s"] = 1.0 / out["c2_seconds_estimate"]
out["c2_sample_columns"] = ms
print(json.dumps(out))
"""


def cpu_one_core(m_sample=8192):
    """The oracle on one host core (OMP_NUM_THREADS=1, a child process that touches no GPU) for the
    smallest workload (whole solves) and the paper-scale workload (column sample, scaled)."""
    import subprocess

    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _ONE_CORE, ROOT, str(m_sample)], env=env, capture_output=True,
                       text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-500:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_baseline(S, v, lam, m_sample):
    """The FP64 oracle on the host on a column sample of the same workload: the Gram, S v and the
    final apply run on m_sample columns and are scaled by m / m_sample (they are linear in m); the
    Cholesky and triangular solves run once at full n."""
    import numpy as np

    import oracle

    oracle.build(force=False)
    n, m = S.shape
    Ss = S[:, :m_sample].cpu().numpy()
    vs = v[:m_sample].double().cpu().numpy()
    t0 = time.perf_counter()
    W = oracle.gram(Ss, lam)
    t1 = time.perf_counter()
    b = oracle.gemv(Ss, vs)
    t2 = time.perf_counter()
    L, info = oracle.cholesky(W + 0.0)
    t3 = time.perf_counter()
    y = oracle.backward(L, oracle.forward(L, b))
    t4 = time.perf_counter()
    oracle.apply(Ss, vs, y, lam)
    t5 = time.perf_counter()
    scale = m / m_sample
    t_full = (t1 - t0 + t2 - t1 + t5 - t4) * scale + (t3 - t2) + (t4 - t3)
    return {
        "value": 1.0 / t_full,
        "unit": "solves/s",
        "cores": oracle.num_threads(),
        "cpu_model": _cpu_model(),
        "kind": "oracle",
        "sample": (f"n={n}, first {m_sample} of m={m} columns: Gram+Sv+apply timed on the sample and "
                   f"scaled x{scale:.0f}; Cholesky and triangular solves timed at full n; lambda={lam}"),
        "seconds_measured": t5 - t0,
        "seconds_full_solve_estimate": t_full,
        "cholesky_info": int(info),
    }


SHIFT = {"on_failure": "DFISHER_SHIFT_ON_FAILURE", "always": "DFISHER_SHIFT_ALWAYS", "none": "DFISHER_SHIFT_NONE"}
GRAM_KERNEL = {"fp32": "gram_kernel_v2<0>", "bf16x3": "gram_kernel_split", "mxfp8": "gram_kernel_fp8"}


# HBM bytes per launch of the Gram tile kernel at the full workload, from rocprofv3 FETCH_SIZE /
# WRITE_SIZE passes (each scaled by the same counters' reading for a device copy of known size),
# valid only for the kernel source they were taken on (sha256 of csrc/gram.hip); see profiles/.
GRAM_TRAFFIC = {
    ("mxfp8", 4096, 4_000_000): {
        "gram_hip_sha256": "ed0e1b1b8a2c47d60e3da9db03f4f431d44327d15ac2ab86941abdc907a295a7",
        # FETCH_SIZE x 2 + WRITE_SIZE x 1 (KiB -> bytes), mean of 12 launches in the latest pair of
        # counter runs; the re-reads vary from box to box and run to run (75.8 to 116.5 GB over
        # four pairs)
        "bytes_per_launch": 116.47e9 + 1.14e9,
    },
}


def gram_traffic(prec, n, m):
    import hashlib

    rec = GRAM_TRAFFIC.get((prec, n, m))
    if rec is None:
        return None
    with open(os.path.join(ROOT, "paper_2310_17556_amd", "csrc", "gram.hip"), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if sha != rec["gram_hip_sha256"]:
        return None   # the kernel changed since the counters were taken
    return rec["bytes_per_launch"]


def run_path(dfl, ctx, S, v, lams, prec, sweeps, steps, warmup, xbuf, shift="on_failure"):
    import torch

    policy = getattr(dfl, SHIFT[shift])
    infos = []
    for _ in range(warmup):
        for lam in lams:
            dfl.dfisher_solve(ctx, S, v, lam, gram_prec=PREC_CODE[prec], centered=CENTERED, sweeps=sweeps, shift_policy=policy,
                              x=xbuf[lam])
    torch.cuda.synchronize()
    gram_ms, stage = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        for lam in lams:
            _, info = dfl.dfisher_solve(ctx, S, v, lam, gram_prec=PREC_CODE[prec], centered=CENTERED, sweeps=sweeps,
                                        shift_policy=policy, x=xbuf[lam])
            t = dfl.dfisher_ctx_last_timing(ctx)
            gram_ms.append(t["gram_ms"])
            stage.append(t)
            infos.append((lam, info))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    avg = {k: sum(s[k] for s in stage) / len(stage) for k in stage[0]} if stage else {}
    return elapsed, gram_ms, avg, infos


def _errs(x, xref, v, lam):
    """(|x - x*| / |x*|, eps_Sy) for one solve. S^T y = v - lambda x, so
    eps_Sy = |S^T (y - y*)| / |S^T y*| = lambda |x - x*| / |v - lambda x*| (meaningful for FP64 x)."""
    import torch

    d = torch.linalg.norm(x.double() - xref)
    return float(d / torch.linalg.norm(xref)), float(lam * d / torch.linalg.norm(v.double() - lam * xref))


def error_table(dfl, ctx, S, v, lams, xref, table, shift="on_failure"):
    """Untimed FP64-output solves for each (Gram precision, sweep count) and lambda: relative error of
    x, eps_Sy and the final residual |S v - lambda y - S S^T y| / |S v| (measured by the library)."""
    import torch

    policy = getattr(dfl, SHIFT[shift])
    x64 = torch.empty(S.shape[1], dtype=torch.float64, device=S.device)
    out = {}
    for prec, sweep_list in table:
        for sw in sweep_list:
            row = {}
            for lam in lams:
                # as called by default (the final step may take the last correction through the FP8
                # codes), then with the measured final residual (which takes the exact step)
                _, info = dfl.dfisher_solve(ctx, S, v, lam, gram_prec=PREC_CODE[prec], centered=CENTERED, sweeps=sw,
                                            shift_policy=policy, x=x64, x_fp64=True)
                rel, esy = _errs(x64, xref[lam], v, lam)
                _, infw = dfl.dfisher_solve(ctx, S, v, lam, gram_prec=PREC_CODE[prec], centered=CENTERED, sweeps=sw,
                                            shift_policy=policy, x=x64, x_fp64=True, final_resid=True)
                rel_x, esy_x = _errs(x64, xref[lam], v, lam)
                row[str(lam)] = {"rel_err": rel, "eps_Sy": esy, "w_resid": infw["w_resid"],
                                 "eps_Sy_exact_step": esy_x, "sweeps": info["sweeps_done"], "shift": info["shift"]}
            out[f"{prec}/{'auto' if sw < 0 else sw}"] = row
    del x64
    return out


def _fp64_x(S, v, lam, chunk=131072):
    """FP64 reference x for one (S, v, lambda) from torch FP64 products on the device."""
    import torch

    n, m = S.shape
    G = torch.zeros((n, n), dtype=torch.float64, device=S.device)
    b = torch.zeros(n, dtype=torch.float64, device=S.device)
    v64 = v.double()
    for c0 in range(0, m, chunk):
        blk = S[:, c0:c0 + chunk].double()
        G += blk @ blk.T
        b += blk @ v64[c0:c0 + chunk]
        del blk
    L = torch.linalg.cholesky(G + lam * torch.eye(n, dtype=torch.float64, device=S.device))
    y = torch.cholesky_solve(b[:, None], L)[:, 0]
    x = torch.empty(m, dtype=torch.float64, device=S.device)
    for c0 in range(0, m, chunk):
        x[c0:c0 + chunk] = (v64[c0:c0 + chunk] - S[:, c0:c0 + chunk].double().T @ y) / lam
    return x


def _summ(vals):
    vals = sorted(vals)
    return {"max": vals[-1], "median": vals[len(vals) // 2], "count": len(vals)}


def paper_scale_leg(dfl, dev, reps, n=1024, m=1_000_000, lam=1e-3, seed=2):
    """The paper-scale plain FP32 workload: column-scaled S (scales log-uniform in [1e-3, 1]), v in
    the row space of S plus N(0, 1e-6) noise, lambda = 1e-3; the plain FP32 path (no sweeps) and the
    mixed paths with their automatic sweep counts."""
    import torch

    import synth

    S = synth.make_S_torch(n, m, synth.seed(seed), dev, kind="scaled")
    v = synth.make_v_torch(S, synth.seed(seed), kind="scaled")
    ctx = dfl.dfisher_ctx_create(0)
    xref = _fp64_x(S, v, lam)
    out = {"workload": f"n={n} m={m}, column-scaled S, v = S^T u + N(0, 1e-6), lambda={lam}", "paths": {}}
    x = torch.empty(m, dtype=torch.float32, device=dev)
    x64 = torch.empty(m, dtype=torch.float64, device=dev)
    for prec, sw in [("fp32", 0), ("fp32", 1), ("mxfp8", -1), ("bf16x3", -1)]:
        dfl.dfisher_solve(ctx, S, v, lam, gram_prec=PREC_CODE[prec], centered=CENTERED, sweeps=sw, x=x)   # warmup
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            _, info = dfl.dfisher_solve(ctx, S, v, lam, gram_prec=PREC_CODE[prec], centered=CENTERED, sweeps=sw, x=x)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        rel32, _ = _errs(x, xref, v, lam)
        _, i64 = dfl.dfisher_solve(ctx, S, v, lam, gram_prec=PREC_CODE[prec], centered=CENTERED, sweeps=sw, x=x64, x_fp64=True,
                                   final_resid=True)
        rel64, esy = _errs(x64, xref, v, lam)
        out["paths"][f"{prec}/{'auto' if sw < 0 else sw}"] = {
            "solves_per_s": 1.0 / el, "ms_per_solve": el * 1e3, "sweeps": info["sweeps_done"],
            "shift": info["shift"], "rel_err_fp32_out": rel32, "rel_err": rel64, "eps_Sy": esy,
            "w_resid": i64["w_resid"]}
    dfl.dfisher_ctx_destroy(ctx)
    del S, v, x, x64, xref
    torch.cuda.empty_cache()
    return out


def _batched_ref(S, V, lams, chunk=131072):
    """FP64 x for every (lambda, rhs) pair: one FP64 Gram, B = S V^T, one Cholesky per lambda."""
    import torch

    n, m = S.shape
    G = torch.zeros((n, n), dtype=torch.float64, device=S.device)
    B = torch.zeros((n, V.shape[0]), dtype=torch.float64, device=S.device)
    for c0 in range(0, m, chunk):
        blk = S[:, c0:c0 + chunk].double()
        G += blk @ blk.T
        B += blk @ V[:, c0:c0 + chunk].double().T.contiguous()
        del blk
    Ys = []
    for lam in lams:
        L = torch.linalg.cholesky(G + lam * torch.eye(n, dtype=torch.float64, device=S.device))
        Ys.append(torch.cholesky_solve(B, L))   # n x nrhs
    return Ys


def batched_leg(dfl, dev, prec, sweeps, reps, n=2048, m=2_000_000, nlam=16, nrhs=8, seed=4):
    """Many lambdas x right-hand sides sharing one S: one dfisher_solve_batched call per step. The
    errors of all nlam x nrhs solves are measured against FP64 (x and eps_Sy from an FP64-output call)."""
    import torch

    import synth

    S = synth.make_S_torch(n, m, synth.seed(seed), dev, kind="iid")
    V = synth.make_V_torch(m, nrhs, synth.seed(seed), dev)
    lams = [float(x) for x in synth.lambdas_logspaced(1e-6, 1e-1, nlam)]
    ctx = dfl.dfisher_ctx_create(0)
    X = torch.empty((nlam, nrhs, m), dtype=torch.float32, device=dev)
    dfl.dfisher_solve_batched(ctx, S, lams, V, gram_prec=PREC_CODE[prec], centered=CENTERED, sweeps=sweeps, X=X)   # warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, infos = dfl.dfisher_solve_batched(ctx, S, lams, V, gram_prec=PREC_CODE[prec], centered=CENTERED, sweeps=sweeps, X=X)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    # the same call enqueued without any wait (DFISHER_ASYNC, statuses on the device), captured once
    # into a graph and replayed; no shift is needed at these lambdas, so X is bitwise the eager one
    Xg = torch.empty_like(X)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        _, dinf = dfl.dfisher_solve_batched(ctx, S, lams, V, gram_prec=PREC_CODE[prec], centered=CENTERED,
                                            sweeps=sweeps, X=Xg, shift_policy=dfl.DFISHER_SHIFT_NONE,
                                            enqueue_only=True)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    elg = (time.perf_counter() - t0) / reps
    ginfos = dfl.batch_infos(dinf)
    graph_ok = all(i["potrf_info"] == 0 for i in ginfos) and bool(torch.equal(Xg, X))
    del g, Xg, dinf
    X64 = torch.empty((nlam, nrhs, m), dtype=torch.float64, device=dev)
    dfl.dfisher_solve_batched(ctx, S, lams, V, gram_prec=PREC_CODE[prec], centered=CENTERED, sweeps=sweeps, X=X64, x_fp64=True)
    Ys = _batched_ref(S, V, lams)
    Yall = torch.stack([Y for Y in Ys], dim=1).reshape(n, nlam * nrhs)   # column l * nrhs + r
    lamv = torch.tensor(lams, dtype=torch.float64, device=dev)[:, None, None]
    acc = {k: torch.zeros((nlam, nrhs), dtype=torch.float64, device=dev) for k in ("d32", "d64", "x", "sty")}
    for c0 in range(0, m, 131072):
        c1 = min(m, c0 + 131072)
        T = (S[:, c0:c1].double().T @ Yall).T.reshape(nlam, nrhs, c1 - c0)   # S^T y* for every pair
        Xr = (V[:, c0:c1].double()[None] - T) / lamv
        acc["d32"] += ((X[:, :, c0:c1].double() - Xr) ** 2).sum(-1)
        acc["d64"] += ((X64[:, :, c0:c1] - Xr) ** 2).sum(-1)
        acc["x"] += (Xr ** 2).sum(-1)
        acc["sty"] += (T ** 2).sum(-1)
        del T, Xr
    rel32 = (acc["d32"].sqrt() / acc["x"].sqrt()).flatten().tolist()
    rel64 = (acc["d64"].sqrt() / acc["x"].sqrt()).flatten().tolist()
    esy = (lamv[:, :, 0] * acc["d64"].sqrt() / acc["sty"].sqrt()).flatten().tolist()
    dfl.dfisher_ctx_destroy(ctx)
    del S, V, X, X64, Ys
    torch.cuda.empty_cache()
    return {"workload": f"batched: n={n} m={m}, {nlam} lambdas log-spaced in [1e-6, 1e-1] x {nrhs} iid right-hand "
                        "sides, one shared Gram",
            "gram": prec, "sweeps": infos[0]["sweeps_done"], "solves_per_s": nlam * nrhs / el, "ms_per_call": el * 1e3,
            "graph_replay": {"solves_per_s": nlam * nrhs / elg, "ms_per_call": elg * 1e3,
                             "x_bitwise_equal_to_eager": graph_ok},
            "rel_err_fp32_out": _summ(rel32), "rel_err": _summ(rel64), "eps_Sy": _summ(esy),
            "max_shift": max(i["shift"] for i in infos)}


def uneven_leg(dfl, dev, prec, sweeps, reps, nprob=64, seed=5):
    """64 independent problems, n log-uniform in [256, 2048], m log-uniform in [1e5, 2e6],
    lambda log-uniform in [1e-5, 1e-2]: one dfisher_solve_uneven call per step. Every problem's
    error is measured against FP64 (x and eps_Sy from an FP64-output call as timed, and from one
    that also reports the final residual, which takes the exact final pass)."""
    import torch

    import synth

    ns, ms, lams = synth.uneven_shapes(nprob, synth.seed(seed))
    Ss, vs = [], []
    for p in range(nprob):
        n, m = int(ns[p]), int(ms[p])
        buf = synth.make_S_torch(n, m, synth.seed(seed, p), dev, kind="iid", ld=(m + 3) // 4 * 4)
        Ss.append(buf[:, :m])
        vs.append(synth.make_v_torch(buf, synth.seed(seed, p), kind="iid", m=m))
    lams = [float(x) for x in lams]
    ctx = dfl.dfisher_ctx_create(0)
    xs = [torch.empty(int(m), dtype=torch.float32, device=dev) for m in ms]
    dfl.dfisher_solve_uneven(ctx, Ss, vs, lams, gram_prec=PREC_CODE[prec], centered=CENTERED, sweeps=sweeps, xs=xs)   # capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, infos = dfl.dfisher_solve_uneven(ctx, Ss, vs, lams, gram_prec=PREC_CODE[prec], centered=CENTERED, sweeps=sweeps, xs=xs)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    # which problems took the final step through the FP8 codes: a call that forces the exact final
    # pass gives the same x exactly for the others
    xchk = [torch.empty(int(m), dtype=torch.float32, device=dev) for m in ms]
    dfl.dfisher_solve_uneven(ctx, Ss, vs, lams, gram_prec=PREC_CODE[prec], centered=CENTERED, sweeps=sweeps, xs=xchk,
                             exact_apply=True)
    fp8_final = [not bool(torch.equal(a, b)) for a, b in zip(xs, xchk)]
    del xchk
    # FP64 output as called (the errors of the timed configuration), then with the measured final
    # residual (which takes the exact final pass)
    x64s = [torch.empty(int(m), dtype=torch.float64, device=dev) for m in ms]
    dfl.dfisher_solve_uneven(ctx, Ss, vs, lams, gram_prec=PREC_CODE[prec], centered=CENTERED, sweeps=sweeps, xs=x64s,
                             x_fp64=True)
    x64w = [torch.empty(int(m), dtype=torch.float64, device=dev) for m in ms]
    _, inf64 = dfl.dfisher_solve_uneven(ctx, Ss, vs, lams, gram_prec=PREC_CODE[prec], centered=CENTERED, sweeps=sweeps, xs=x64w,
                                        x_fp64=True, final_resid=True)
    rel32, rel64, esy, esyx, per = [], [], [], [], []
    for p in range(nprob):
        xr = _fp64_x(Ss[p], vs[p], lams[p])
        r32, _ = _errs(xs[p], xr, vs[p], lams[p])
        r64, e = _errs(x64s[p], xr, vs[p], lams[p])
        _, ex = _errs(x64w[p], xr, vs[p], lams[p])
        rel32.append(r32)
        rel64.append(r64)
        esy.append(e)
        esyx.append(ex)
        per.append([int(ns[p]), int(ms[p]), lams[p], infos[p]["sweeps_done"], r32, e, inf64[p]["w_resid"], fp8_final[p]])
        del xr
    del x64w
    worst = max(range(nprob), key=lambda q: esy[q])
    dfl.dfisher_ctx_destroy(ctx)
    out = {"workload": f"uneven: {nprob} problems, n log-uniform [256, 2048], m log-uniform [1e5, 2e6], "
                       "lambda log-uniform [1e-5, 1e-2], one right-hand side each",
           "gram": prec, "sweeps": "auto" if sweeps < 0 else sweeps,
           "sweeps_per_problem": _summ([i["sweeps_done"] for i in infos]),
           "solves_per_s": nprob / el, "ms_per_call": el * 1e3,
           "S_GB": sum(4.0 * int(n) * int(m) for n, m in zip(ns, ms)) / 1e9,
           "gram_flops": float(sum(float(n) * (n + 1) * m for n, m in zip(ns, ms))),
           "rel_err_fp32_out": _summ(rel32), "rel_err": _summ(rel64), "eps_Sy": _summ(esy),
           "eps_Sy_exact_final_pass": _summ(esyx),
           "w_resid": _summ([i["w_resid"] for i in inf64]),
           "fp8_final_step_problems": sum(1 for f in fp8_final if f),
           "worst_problem": dict(zip(["n", "m", "lambda", "sweeps", "rel_err_fp32_out", "eps_Sy", "w_resid",
                                      "fp8_final_step"], per[worst])),
           "retried": sum(1 for i in infos if i["attempts"] > 1)}
    del Ss, vs, xs, x64s
    torch.cuda.empty_cache()
    return out


def _sweeps_arg(s):
    return -1 if s == "auto" else int(s)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--m", type=int, default=4_000_000)
    ap.add_argument("--prec", default="mxfp8", choices=sorted(PREC_CODE))
    ap.add_argument("--sweeps", type=_sweeps_arg, default=2,
                    help="refinement sweeps of the timed path, or 'auto' (default 2: the count at which every "
                         "solve of the workload meets 1e-6 in x and in eps_Sy, reported by the error table)")
    ap.add_argument("--shift", default="on_failure", choices=sorted(SHIFT),
                    help="Cholesky shift policy of the mixed path")
    ap.add_argument("--lams", default="1e-2,1e-4,1e-6")
    ap.add_argument("--fp32-steps", type=int, default=1, help="timed steps of the plain FP32 path (0: skip)")
    ap.add_argument("--no-ref", action="store_true", help="skip the FP64 error check")
    ap.add_argument("--no-table", action="store_true", help="skip the precision x sweeps error table")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-m", type=int, default=8192)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--alt-prec", default="bf16x3", choices=sorted(PREC_CODE) + ["none"],
                    help="second mixed precision timed for comparison (none: skip)")
    ap.add_argument("--no-paper-scale", action="store_true", help="skip the n=1024, m=1M plain FP32 workload")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched multi-lambda/RHS leg")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-batch leg")
    ap.add_argument("--leg-reps", type=int, default=3, help="timed calls of the batched and uneven legs")
    ap.add_argument("--leg-sweeps", type=_sweeps_arg, default=-1,
                    help="refinement sweeps of the batched and uneven legs (default 'auto': the a-priori count "
                         "per problem shape)")
    ap.add_argument("--no-auto", action="store_true", help="skip the DFISHER_SWEEPS_AUTO run of the main workload")
    ap.add_argument("--no-centered", action="store_true",
                    help="do not declare S centered (the workloads' S is column-centered; the declaration "
                         "makes the factored matrix exact along the all-ones direction)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run two device copies of 1 GiB (reference reading for the HBM byte counters)")
    args = ap.parse_args()
    global CENTERED
    CENTERED = not args.no_centered

    if args.gpus != 1:
        print(json.dumps({"error": f"--gpus {args.gpus}: this build runs on exactly one GPU; multi-GPU "
                                   "sharding (m split across GPUs + one all-reduce of the Gram) is not "
                                   "implemented"}))
        return 2

    import torch

    import paper_2310_17556_amd as dfl
    import synth

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU available"}))
        return 2
    if args.copy_calibration:
        # a plain device copy of known size: each launch reads 2^30 bytes and writes 2^30 bytes
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30, "launches": 2}))
        return 0
    n, m = args.n, args.m
    lams = [float(x) for x in args.lams.split(",")]
    dev = torch.device("cuda:0")
    log(f"[bench] generating S {n}x{m} ({4 * n * m / 1e9:.1f} GB) on the device")
    S = synth.make_S_torch(n, m, synth.seed(args.seed), dev, kind="iid")
    v = synth.make_v_torch(S, synth.seed(args.seed), kind="iid")
    torch.cuda.synchronize()
    ctx = dfl.dfisher_ctx_create(0)
    dfl.dfisher_ctx_enable_timing(ctx, True)
    xbuf = {lam: torch.empty(m, dtype=torch.float32, device=dev) for lam in lams}
    sweeps_resolved = dfl.dfisher_auto_sweeps(PREC_CODE[args.prec], n, m) if args.sweeps < 0 else args.sweeps

    log(f"[bench] mixed path: {args.prec} Gram + {args.sweeps} sweep(s) (a-priori rule {sweeps_resolved}), "
        f"{args.warmup} warmup + {args.steps} steps")
    elapsed, gram_ms, stage_avg, infos = run_path(dfl, ctx, S, v, lams, args.prec, args.sweeps, args.steps,
                                                  args.warmup, xbuf, args.shift)
    solves = args.steps * len(lams)
    value = solves / elapsed
    gram_avg_ms = sum(gram_ms) / len(gram_ms)
    algo_flops = float(n) * (n + 1) * m
    achieved = algo_flops / (gram_avg_ms * 1e-3) / 1e12
    passes = PASSES[args.prec]
    peak = PEAK_TFLOPS[args.prec]
    log(f"[bench] mixed: {value:.3f} solves/s, gram {gram_avg_ms:.2f} ms, stages {stage_avg}")

    x_mixed = {lam: xbuf[lam].clone() for lam in lams}
    # which final step each timed solve took: the last correction through the FP8 codes, or the
    # exact column pass over S (an untimed call that forces the latter gives the same x exactly then)
    final_step = {}
    xchk = torch.empty(m, dtype=torch.float32, device=dev)
    for lam in lams:
        dfl.dfisher_solve(ctx, S, v, lam, gram_prec=PREC_CODE[args.prec], centered=CENTERED, sweeps=args.sweeps,
                          shift_policy=getattr(dfl, SHIFT[args.shift]), x=xchk, exact_apply=True)
        final_step[str(lam)] = "exact" if bool(torch.equal(xchk, x_mixed[lam])) else "fp8"
    del xchk
    log(f"[bench] final step per lambda: {final_step}")

    fp32 = None
    if args.fp32_steps > 0:
        log(f"[bench] plain FP32 path: {args.fp32_steps} step(s)")
        xb32 = {lam: torch.empty(m, dtype=torch.float32, device=dev) for lam in lams}
        e32, g32, st32, inf32 = run_path(dfl, ctx, S, v, lams, "fp32", 0, args.fp32_steps, 0, xb32)
        g32avg = sum(g32) / len(g32)
        fp32 = {"solves_per_s": args.fp32_steps * len(lams) / e32, "gram_ms": g32avg,
                "gram_tflops_algorithmic": algo_flops / (g32avg * 1e-3) / 1e12,
                "gram_mfma_frac": algo_flops / (g32avg * 1e-3) / 1e12 / PEAK_TFLOPS["fp32"],
                "sweeps": 0, "stage_ms": st32,
                "shifts": {str(l): i["shift"] for l, i in inf32}}
        log(f"[bench] fp32: {fp32['solves_per_s']:.3f} solves/s, gram {g32avg:.2f} ms")

    auto = None
    if args.sweeps >= 0 and not args.no_auto:
        log("[bench] same path with DFISHER_SWEEPS_AUTO (measured residuals): 1 step")
        xba = {lam: torch.empty(m, dtype=torch.float32, device=dev) for lam in lams}
        eau, gau, stau, infau = run_path(dfl, ctx, S, v, lams, args.prec, -1, 1, 0, xba, args.shift)
        auto = {"solves_per_s": len(lams) / eau, "sweeps_done": {str(l): i["sweeps_done"] for l, i in infau},
                "resid": {str(l): i["resid"] for l, i in infau}, "stage_ms": stau}
        log(f"[bench] auto: {auto['solves_per_s']:.3f} solves/s, sweeps {auto['sweeps_done']}")

    alt = None
    if args.alt_prec != "none" and args.alt_prec != args.prec:
        log(f"[bench] {args.alt_prec} path: 1 step")
        xbalt = {lam: torch.empty(m, dtype=torch.float32, device=dev) for lam in lams}
        ea, ga, sta, infa = run_path(dfl, ctx, S, v, lams, args.alt_prec, args.sweeps, 1, 1, xbalt, args.shift)
        gaavg = sum(ga) / len(ga)
        alt = {"gram": args.alt_prec, "sweeps": infa[0][1]["sweeps_done"], "solves_per_s": len(lams) / ea,
               "gram_ms": gaavg, "gram_tflops_algorithmic": algo_flops / (gaavg * 1e-3) / 1e12,
               "gram_mfma_frac_hw": algo_flops * PASSES[args.alt_prec] / (gaavg * 1e-3) / 1e12
               / PEAK_TFLOPS[args.alt_prec],
               "stage_ms": sta, "shifts": {str(l): i["shift"] for l, i in infa}}
        log(f"[bench] {args.alt_prec}: {alt['solves_per_s']:.3f} solves/s, gram {gaavg:.2f} ms")

    errors = None
    table = None
    if not args.no_ref:
        log("[bench] FP64 reference for the error report")
        xref = fp64_reference(S, v, lams)
        errors = {"mixed": {}, "fp32": {}, "alt": {}}
        for lam in lams:
            errors["mixed"][str(lam)] = _errs(x_mixed[lam], xref[lam], v, lam)[0]
            if fp32 is not None:
                errors["fp32"][str(lam)] = _errs(xb32[lam], xref[lam], v, lam)[0]
            if alt is not None:
                errors["alt"][str(lam)] = _errs(xbalt[lam], xref[lam], v, lam)[0]
        log(f"[bench] errors (FP32 x) {errors}")
        if not args.no_table:
            log("[bench] error table: precision x sweeps x lambda, FP64 x")
            table = error_table(dfl, ctx, S, v, lams, xref,
                                [("mxfp8", [0, 1, 2, 3]), ("bf16x3", [0, 1, 2, 3]), ("fp32", [0, 1])], args.shift)
            log(f"[bench] table {json.dumps(table)}")
        del xref

    # stage bandwidths (algorithmic bytes): the prep pass reads S (+ v) and, for the scaled-FP8 Gram,
    # writes the codes and their scales; each refinement sweep reads S once (fused pass)
    ldq = (m + 127) // 128 * 128
    prep_write = {"mxfp8": n * ldq * (1 + 1 / 32), "bf16x3": 4.0 * n * ((m + 63) // 64 * 64), "fp32": 0.0}
    rowpass_bytes = 4.0 * n * m + 4.0 * m + 16.0 * n + prep_write[args.prec]
    apply_bytes = 4.0 * n * m + 8.0 * n + 8.0 * m
    if args.prec == "mxfp8" and all(f == "fp8" for f in final_step.values()):
        # the FP8 final step reads the codes and scales, T = S^T y, the column sums (centered), v,
        # and writes x
        apply_bytes = n * ldq * (1 + 1 / 32) + 8.0 * m * (2 if CENTERED else 1) + 4.0 * m + 4.0 * m + 8.0 * n
    timed = infos[-solves:]
    sweeps_done = {str(l): i["sweeps_done"] for l, i in timed[-len(lams):]}
    refine_bytes = sum(i["sweeps_done"] for _, i in timed) / len(timed) * (4.0 * n * m + 8.0 * n)

    def gbs(b, ms):
        return b / (ms * 1e-3) / 1e9 if ms else None

    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] FP64 CPU oracle on a {args.cpu_sample_m}-column sample")
        cpu = cpu_baseline(S, v, lams[-1], args.cpu_sample_m)
        log("[bench] FP64 CPU oracle on one core (smallest and paper-scale workloads)")
        cpu["one_core"] = cpu_one_core()
        log(f"[bench] cpu baseline {cpu}")
    dfl.dfisher_ctx_destroy(ctx)
    del S, v, xbuf, x_mixed
    if fp32 is not None:
        del xb32
    if auto is not None:
        del xba
    if alt is not None:
        del xbalt
    torch.cuda.empty_cache()

    paper = None
    if not args.no_paper_scale:
        log("[bench] paper-scale workload: n=1024 m=1M, column-scaled S, row-space v, lambda=1e-3")
        paper = paper_scale_leg(dfl, dev, args.leg_reps)
        log(f"[bench] paper scale {paper}")
    batched = None
    if not args.no_batched:
        log("[bench] batched leg: n=2048 m=2M, 16 lambdas x 8 right-hand sides")
        batched = batched_leg(dfl, dev, args.prec, args.leg_sweeps, args.leg_reps)
        log(f"[bench] batched {batched}")
    uneven = None
    if not args.no_uneven:
        log("[bench] uneven leg: 64 problems")
        uneven = uneven_leg(dfl, dev, args.prec, args.leg_sweeps, args.leg_reps)
        log(f"[bench] uneven {uneven}")

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.prec],
        "data": "synthetic",
        "config": {"workload": f"damped Fisher solve n={n} m={m} (iid N(0,1)/sqrt(n) column-centered S, iid v), "
                               f"one solve per lambda in {lams}",
                   "n": n, "m": m, "lambdas": lams, "gram": args.prec,
                   "sweeps": "auto" if args.sweeps < 0 else args.sweeps, "sweeps_a_priori_rule": sweeps_resolved,
                   "sweeps_done": sweeps_done, "shift": args.shift, "solves_per_step": len(lams),
                   "centered_flag": CENTERED},
        "roofline": {"bound": "mfma", "kernel": GRAM_KERNEL[args.prec], "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": gram_traffic(args.prec, n, m),
                     "algorithmic_flops_per_launch": algo_flops, "avg_launch_ms": gram_avg_ms,
                     "mfma_util_hw": achieved * passes / peak},
        "stage_ms": stage_avg,
        "hbm": {"rowpass_GBs": gbs(rowpass_bytes, stage_avg.get("rowpass_ms")),
                "rowpass_bytes": rowpass_bytes,
                "apply_GBs": gbs(apply_bytes, stage_avg.get("apply_ms")),
                "apply_bytes": apply_bytes,
                "final_step": final_step,
                "refine_GBs": gbs(refine_bytes, stage_avg.get("refine_ms")),
                "refine_note": "refine_ms includes the triangular solves of every sweep",
                "peak_GBs": HBM_PEAK_GBS},
        "fp32_path": fp32,
        "auto_sweeps_path": auto,
        "alt_path": alt,
        "rel_err_vs_fp64": errors,
        "error_table": table,
        "shifts": {str(l): i["shift"] for l, i in infos[-len(lams):]},
        "paper_scale": paper,
        "batched": batched,
        "uneven": uneven,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
