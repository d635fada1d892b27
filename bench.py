#!/usr/bin/env python
"""Benchmark of the Laplace-evidence hot path on one MI355X.

Metric: logL+grad evaluations per second and time-to-log Z at d = 1024, for
the mixed-precision path (BF16 discovery GEMM, FP32 L-BFGS bulk, FP64 polish,
Hessian, Cholesky and combine) against the plain FP64 path.

One step = one full evidence computation (discovery, batched L-BFGS, dedup,
Newton polish, Hessian, Cholesky, log det, combine) for each posterior of the
d = 1024 workload: (a) a dense-covariance Gaussian and (b) a K = 8 Gaussian
mixture, 16384 rays x 32 points and 16384 starts each.  Inputs are resident
in HBM when the timed region starts (sb_evidence_dev); the value is the
number of logL+grad evaluations performed per second of wall time.

Also reported: the roofline of the dominant kernel of the step, the batched
L-BFGS step of the FP32 bulk (HBM-bound; its launches timed with HIP events
on their stream at full batch), the roofline of the bulk's split-BF16
contraction at the mixture's shape (matrix cores), and the CPU oracle timed
on the host on a bounded sample of the workload.
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

PEAK = {"fp32": 157.3, "fp64": 78.6, "bf16": 2500.0, "hbm": 8000.0}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def workload(names, n_starts=None):
    from paper_2601_19957_amd import synth

    out = {}
    for nm in names:
        prob, cfg = synth.make_workload(nm, n_starts=n_starts)
        out[nm] = (prob, cfg)
    return out


def closed_form_logz(prob) -> float:
    """Laplace log Z of the synthetic problem from its generator data (box truncation aside)."""
    d = prob.d
    logv = float(sum(math.log(h - l) for l, h in zip(prob.lo, prob.hi)))
    if prob.norm == 0 and prob.K == 1:  # peak-zero Gaussian
        return 0.5 * d * math.log(2 * math.pi) + 0.5 * float(prob.sum_log_lambda[0]) - logv
    return -logv  # normalised mixture: total mass 1


def time_quadform(L, prob, B, reps=20, dtype=None):
    """Average duration of the A3 contraction at the bulk shape (the split-BF16 kernel the
    mixed bulk runs, or another dtype), HIP events on its stream."""
    import torch
    from paper_2601_19957_amd import synth

    m = L.DeviceModel(prob, low_precision=True)
    X = torch.as_tensor(synth.points_near_modes(prob, B, 5, scale=0.3), device="cuda").float()
    qf = L.QuadForm(m, X, dtype=L.DTYPE_F32_SPLIT if dtype is None else dtype)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        qf(stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        qf(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    avg_s = e0.elapsed_time(e1) * 1e-3 / reps
    d, K = prob.d, prob.K
    flops = 2.0 * B * K * d * d + 2.0 * B * K * d  # Y = delta P^T, q = delta . Y
    return avg_s, flops


def recorded_traffic(summary="profiles/quad_gemm_split_B16384_d1024_K8.md",
                     source="paper_2601_19957_amd/csrc/gemm_bf16.hip"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None when the
    kernel source changed since the counters were taken."""
    import hashlib
    import re

    try:
        txt = open(os.path.join(ROOT, summary)).read()
        sha = hashlib.sha256(open(os.path.join(ROOT, source), "rb").read()).hexdigest()
    except OSError:
        return None
    m_t = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    m_h = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", txt)
    if not m_t or not m_h or m_h.group(1) != sha:
        return None
    return float(m_t.group(1))


def a3_variants(L):
    """logL+grad (A3: contraction, epilogue and hand-written backward) per config and precision
    at the config's start count, HIP events on its stream: evals/s and the fraction of the
    peak of the arithmetic the contraction runs on (algorithmic flops 2 B K d^2 + 4 B K d)."""
    import torch
    from paper_2601_19957_amd import synth

    out = []
    cases = [("c1", [L.DTYPE_F64]), ("c2", [L.DTYPE_F64]),
             ("c4a", [L.DTYPE_F64, L.DTYPE_F32, L.DTYPE_F32_SPLIT]),
             ("c4b", [L.DTYPE_F64, L.DTYPE_F32, L.DTYPE_F32_SPLIT])]
    names = {L.DTYPE_F64: ("f64", "fp64"), L.DTYPE_F32: ("f32", "fp32"),
             L.DTYPE_F32_SPLIT: ("f32 as split bf16", "bf16")}
    for name, dts in cases:
        prob, cfg = synth.make_workload(name)
        B = cfg.n_starts
        m = L.DeviceModel(prob, low_precision=True)
        X64 = torch.as_tensor(synth.points_near_modes(prob, B, 11, scale=0.5), device="cuda")
        flops = 2.0 * B * prob.K * prob.d ** 2 + 4.0 * B * prob.K * prob.d
        for dt in dts:
            X = X64 if dt == L.DTYPE_F64 else X64.float()
            # small problems: many launches, so that the GPU time, not the host's submission
            # time, sets the pace (buffers and workspace allocated once)
            reps = 5 if prob.d * prob.K >= 4096 and dt == L.DTYPE_F64 else (
                10 if prob.d >= 1024 else 200)
            call = L.LoglGrad(m, X, dtype=dt)
            call()  # warm (code objects, tile cache)
            st = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(st)
            for _ in range(reps):
                call(st)
            e1.record(st)
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) / reps / 1e3
            del call
            lab, pk = names[dt]
            out.append(dict(config=name, d=prob.d, K=prob.K, batch=B, dtype=lab,
                            ms=sec * 1e3, evals_per_s=B / sec, tflops=flops / sec / 1e12,
                            peak_tflops=PEAK[pk], frac=flops / sec / 1e12 / PEAK[pk]))
            log(f"A3 {name} {lab}: {sec*1e3:.3f} ms, {B/sec:.3e} evals/s, "
                f"{flops/sec/1e12:.1f} TFLOP/s")
        del m, X64
        torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def recorded_lbfgs(summary="profiles/lbfgs_step_B16384_d1024_m8.md",
                   source="paper_2601_19957_amd/csrc/lbfgs.hip"):
    """HBM bytes per full-batch L-BFGS step launch (16384 starts, d = 1024, m = 8) and the
    plain-copy rate from the committed rocprofv3 counter summary, or None when the kernel
    source changed since the counters were taken."""
    import hashlib
    import re

    try:
        txt = open(os.path.join(ROOT, summary)).read()
        sha = hashlib.sha256(open(os.path.join(ROOT, source), "rb").read()).hexdigest()
    except OSError:
        return None
    m_h = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", txt)
    if not m_h or m_h.group(1) != sha:
        return None
    val = {}
    for key in ("lbfgs_traffic_bytes_per_launch", "copy_tbps"):
        m_v = re.search(key + r":\s*([0-9.eE+]+)", txt)
        if not m_v:
            return None
        val[key] = float(m_v.group(1))
    return val


def time_lbfgs_step(L, prob, cfg, n_timed=40, dtype="f32", box_starts=False, min_full=0.99,
                    hist_bf16=False):
    """The L-BFGS step (A4) as the mixed bulk runs it (FP32, one workgroup per start) at full
    batch: sb_lbfgs_timed_dev from the BF16 discovery starts, HIP events around each step
    launch on its stream.  Averaged over the full-batch launches in which every start either
    accepted its trial or halved its step, at least min_full accepting with a full history ring;
    their algorithmic bytes come from the library (sb_lbfgs_timed_dev's per-launch count): an
    accepting start with a full ring moves (2m + 6) d 4 bytes (the history pairs but the
    evicted one read, or all m when the curvature test keeps the new pair out and it is not
    written; x and g read at both slots; s, y, direction and trial point written), one with c
    pairs (2c + 6) d 4 plus 2 d 4 when it stores the new pair, a halving one 3 d 4 bytes (point
    and direction read, trial point written); with hist_bf16 the ring's vectors count 2 d
    bytes each instead of 4 d.  dtype "f64": the same step in FP64 (the plain
    path and the polish), 8-byte elements, from the FP64 discovery starts.  box_starts: from
    points one standard deviation around the modes instead, without a gradient stop (small
    problems' discovery starts converge before the history ring fills, and from far points
    the curvature test keeps pairs out of a non-convex region, so no launch would have every
    start accepting with a full ring)."""
    import numpy as np

    f64 = dtype == "f64"
    es = 8 if f64 else 4
    mdl = L.DeviceModel(prob, low_precision=not f64)
    disc = L.sb_discover_dev(mdl, cfg.n_rays, cfg.n_points, cfg.n_starts, cfg.seed,
                             dtype=L.DTYPE_F64 if f64 else L.DTYPE_BF16)
    X0 = disc["X0"] if f64 else disc["X0"].float()
    if box_starts:
        import torch
        from paper_2601_19957_amd import synth

        Xb = torch.as_tensor(synth.points_near_modes(prob, cfg.n_starts, 17, scale=1.0),
                             device="cuda")
        X0 = Xb if f64 else Xb.float()
    B, d = X0.shape
    # near starts: no gradient stop, so that every start is still stepping when its ring is full
    r = L.sb_lbfgs_timed_dev(mdl, X0, m=cfg.m, max_iter=n_timed + 8, n_timed=n_timed,
                             grad_tol=1e-300 if box_starts else 0.0,
                             hist_bf16=hist_bf16 and not f64)
    full, back = r["step_full"].astype(np.int64), r["step_back"].astype(np.int64)
    nbytes = r["step_bytes"]
    # steady-state full-batch launches: every start accepted or halved, at least min_full of
    # them accepting with a full ring; the library counts each one's bytes from the ring
    # counts before and after it
    sel = [i for i in range(n_timed) if int(r["step_rows"][i]) == B and nbytes[i] > 0
           and full[i] >= min_full * B]
    if not sel:
        log(f"L-BFGS step d={d} {dtype}: no full-batch launch in which every start accepted or "
            f"halved (rows {r['step_rows'].tolist()}, full {full.tolist()}, halving "
            f"{back.tolist()})")
        return None
    us = r["step_us"][sel].astype(np.float64)
    per_launch = nbytes[sel]
    alg = float(per_launch.mean())
    avg_us = float(us.mean())
    achieved = alg / avg_us / 1e3  # GB/s
    rec = recorded_lbfgs() if (d, cfg.m, B) == (1024, 8, 16384) and hist_bf16 and not f64 \
        else None
    h16 = hist_bf16 and not f64
    # the library's launch shape for this d (threads per start, values per thread)
    tpb = 64 if d <= 256 else (128 if d <= 512 else (256 if d <= 1024 else 512))
    ept = 1 if d <= 64 else (2 if d <= 128 else 4)
    if h16 and d > 256:
        tpb, ept = tpb // 2, 8
    out = dict(bound="hbm", achieved=achieved, peak=PEAK["hbm"], unit="GB/s",
               frac=achieved / PEAK["hbm"],
               traffic=rec["lbfgs_traffic_bytes_per_launch"] if rec else None,
               kernel=f"lbfgs_step_kernel<{'double' if f64 else 'float'},{tpb},{ept},true"
                      f"{',true' if h16 else ''}> (A4 batched L-BFGS step, "
                      f"{'FP64' if f64 else ('FP32 bulk, BF16 history ring' if h16 else 'FP32')})",
               shape=f"B={B} d={d} m={cfg.m}", algorithmic_bytes=alg, avg_launch_us=avg_us,
               launches=len(sel), launch_us_range=[float(us.min()), float(us.max())],
               timed_steps=[int(i) for i in sel],
               halving_starts=[int(back[i]) for i in sel],
               launch_bytes=[float(nbytes[i]) for i in sel],
               launch_us=[float(x) for x in us])
    if rec:
        out["copy_GBps"] = rec["copy_tbps"] * 1e3
        out["frac_of_copy"] = achieved / out["copy_GBps"]
    return out


def lbfgs_step_variants(L):
    """The L-BFGS step's HBM roofline at c1 (d = 64, 4096 starts), c2 (d = 256, 8192) and c4b
    (d = 1024, 16384) in FP32 (FP32 and BF16 history ring) and FP64 (algorithmic bytes per
    launch counted by the library from the starts' ring counts);
    c1 and c2 from points around the modes, c4b from its discovery starts."""
    from paper_2601_19957_amd import synth

    out = {}
    for name in ("c1", "c2", "c4b"):
        prob, cfg = synth.make_workload(name)
        for dt in ("f32", "f32_h16", "f64"):
            # (c1, c2: at least 90% with a full ring; their rings fill unevenly near the modes)
            r = time_lbfgs_step(L, prob, cfg, n_timed=24, dtype=dt[:3], box_starts=name != "c4b",
                                min_full=0.99 if name == "c4b" else 0.9,
                                hist_bf16=dt == "f32_h16")
            if r:
                out[f"{name}_{dt}"] = {k: r[k] for k in ("achieved", "frac", "avg_launch_us",
                                                         "algorithmic_bytes", "shape", "kernel",
                                                         "launches")}
                log(f"L-BFGS step {name} {dt}: {r['avg_launch_us']:.1f} us, "
                    f"{r['achieved']:.0f} GB/s = {r['frac']:.3f} of HBM peak")
            torch_empty_cache()
    return out


def torch_empty_cache():
    import torch

    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def time_quadform_pairs(L, prob, B, reps=20):
    """The bulk's screened mixture contraction as it runs near the modes: every start listed
    for the one component it sits at (the mixture's starts spread over its K components),
    split BF16, 128 x 128 tiles; average duration by HIP events on its stream, algorithmic
    FLOPs 2 d^2 + 2 d per listed pair."""
    import numpy as np
    import torch
    from paper_2601_19957_amd import synth

    m = L.DeviceModel(prob, low_precision=True)
    Xh = synth.points_near_modes(prob, B, 5, scale=0.3)
    comp = np.arange(B) % prob.K  # the component each start was drawn at
    counts = np.bincount(comp, minlength=prob.K).astype(np.int32)
    rows = np.zeros((prob.K, B), dtype=np.int32)
    for k in range(prob.K):
        idx = np.flatnonzero(comp == k).astype(np.int32)
        rows[k, :idx.size] = idx
    X = torch.as_tensor(Xh, device="cuda").float()
    g = torch.as_tensor(counts, device="cuda")
    rw = torch.as_tensor(rows, device="cuda")
    Y = torch.empty((B, prob.K * prob.d), dtype=torch.float32, device="cuda")
    qp = torch.empty((B, prob.K, (prob.d + 63) // 64), dtype=torch.float32, device="cuda")
    mv = m.view(L.DTYPE_F32_SPLIT)
    import ctypes as C
    nt = C.c_int32()
    stream = torch.cuda.current_stream()

    def launch():
        st = L.lib().sb_quadform_pairs_dev(C.byref(mv), B, X.data_ptr(), g.data_ptr(),
                                           rw.data_ptr(), B, Y.data_ptr(), qp.data_ptr(),
                                           C.byref(nt), stream.cuda_stream)
        L._check(st, "sb_quadform_pairs_dev")

    for _ in range(3):
        launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        launch()
    e1.record(stream)
    torch.cuda.synchronize()
    avg_s = e0.elapsed_time(e1) * 1e-3 / reps
    pairs = int(counts.sum())
    flops = 2.0 * pairs * prob.d * prob.d + 2.0 * pairs * prob.d
    achieved = flops / avg_s / 1e12
    return dict(bound="mfma", achieved=achieved, peak=PEAK["bf16"], unit="TFLOP/s",
                frac=achieved / PEAK["bf16"], executed_mfma_frac=3.0 * achieved / PEAK["bf16"],
                kernel="quad_gemm_bf16_kernel<3,0,128,128,...> grouped (screened mixture bulk)",
                pairs_per_launch=pairs, pairs_per_component=counts.tolist(),
                avg_launch_us=avg_s * 1e6, shape=f"B={B} d={prob.d} K={prob.K}")


def calibration_copy() -> int:
    """A plain device copy of known size (1 GiB read + 1 GiB written) that calibrates the HBM
    byte counters of a profiled run; a 1 GiB fill in between evicts the source from the 256 MB
    last-level cache.  Returns the bytes moved each way."""
    import torch

    n_copy = 256 << 20  # floats
    src = torch.ones(n_copy, dtype=torch.float32, device="cuda")
    flush = torch.full((n_copy,), 2.0, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del flush, src, dst
    torch.cuda.empty_cache()
    return 4 * n_copy


def cpu_baseline(prob, cfg, budget_s=20.0):
    """The oracle, as it stands, on a bounded sample: a few starts of the same workload."""
    import oracle

    threads = os.cpu_count() or 1
    ns = max(1, min(threads, 32))
    t0 = time.perf_counter()
    r = oracle.evidence(prob, cfg, n_threads=threads, n_starts=ns)
    dt = time.perf_counter() - t0
    if dt < 0.25 * budget_s and ns < 4 * threads:  # too short a sample: take more starts
        ns = min(int(ns * min(8.0, budget_s / max(dt, 1e-3))), 8 * threads)
        t0 = time.perf_counter()
        r = oracle.evidence(prob, cfg, n_threads=threads, n_starts=ns)
        dt = time.perf_counter() - t0
    # single-threaded, a smaller sample of the same workload
    ns1 = max(1, min(4, ns))
    t1 = time.perf_counter()
    r1 = oracle.evidence(prob, cfg, n_threads=1, n_starts=ns1)
    dt1 = time.perf_counter() - t1
    return dict(value=r.n_grad_evals / dt, unit="logL+grad evals/s", cores=threads, kind="oracle",
                sample=f"{prob.name}: whole path with {ns} starts "
                       f"({ns} rays x {cfg.n_points} points), {r.n_grad_evals} logL+grad evals "
                       f"in {dt:.2f} s, log Z {r.log_z:.6f}",
                seconds=dt, log_z=r.log_z, cpu_model=cpu_model(),
                single_thread=dict(value=r1.n_grad_evals / dt1, starts=ns1, seconds=dt1))


def precheck_leg(L, prob, name, reps=10):
    """Preprocessing probe (2d + 1 FP64 l evaluations in one batch, sensitivities, classes,
    marginal log-evidence): wall time per sb_precheck_dev call (it ends with a stream
    synchronisation) on the workload's posterior, and on a d = 1024 Gaussian with 64
    unconstrained and 32 weakly constrained coordinates against its closed form."""
    import numpy as np
    import torch
    from paper_2601_19957_amd import synth

    m = L.DeviceModel(prob)
    L.sb_precheck_dev(m)  # tile autotune
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = L.sb_precheck_dev(m)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    d, K = prob.d, prob.K
    flops = (2.0 * d + 1) * K * (2.0 * d * d + 3.0 * d)
    out = dict(workload=f"{name}: d={d} K={K}", ms=dt * 1e3, logl_evals=2 * d + 1,
               tflops=flops / dt / 1e12, frac_fp64_peak=flops / dt / 1e12 / PEAK["fp64"],
               n_flat=r["n_flat"], n_soft=r["n_soft"])
    nz = synth.nuisance_gaussian(1024, 64, 32, seed=2601199575)
    rz = L.sb_precheck_dev(L.DeviceModel(nz))
    cls = rz["cls"].cpu().numpy()
    D = 0.5 * (nz.hi - nz.lo)
    sig = 1.0 / np.sqrt(np.diag(nz.prec[0]))
    ref = float(np.sum(np.log(2 * D[:64])) + np.sum(0.5 * math.log(2 * math.pi) + np.log(sig[64:96])))
    out["degenerate_d1024"] = dict(
        classes_as_constructed=bool((cls[:64] == 1).all() and (cls[64:96] == 2).all()
                                    and (cls[96:] == 0).all()),
        logz_marginal=float(rz["logz_marginal"].cpu().numpy()[0]), closed_form=ref)
    return out


def chisao_leg(L, prob, name, reps=3):
    """ChiSao moves at the bulk's batch (16384 samples of the workload's posterior, every
    seventh stuck): one Hands Like Clouds step of four draws plus four anti-convergence steps,
    FP64 (8 batches of gradients), then stick detection on the result; wall time per call after
    a warm call, gradient evaluations per second and the contraction's FP64 rate; and reseeding
    rays (32 points each) from 2048 of the samples."""
    import numpy as np
    import torch
    from paper_2601_19957_amd import synth

    B, ns, n_anti = 16384, 4, 4
    d, K = prob.d, prob.K
    m = L.DeviceModel(prob)
    X0 = torch.as_tensor(synth.random_points(prob, B, seed=2601199576), device="cuda")
    g = torch.Generator(device="cuda").manual_seed(2601199577)
    Z = torch.randn((1, ns, B, d), generator=g, dtype=torch.float64, device="cuda")
    stuck = torch.zeros(B, dtype=torch.uint8, device="cuda")
    stuck[::7] = 1
    X = X0.clone()
    L.sb_chisao_explore_dev(m, X, stuck, Z, 0.1, 0.05, n_anti, 0.02, 0.9)  # tile autotune
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        X.copy_(X0)
        L.sb_chisao_explore_dev(m, X, stuck, Z, 0.1, 0.05, n_anti, 0.02, 0.9)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    l, gr = L.sb_logl_grad_dev(m, X)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sm = L.sb_chisao_stick_dev(l, gr, 1e-3)
    torch.cuda.synchronize()
    ds = time.perf_counter() - t1
    # reseeding rays from 2048 of the samples, 32 points each (65536 FP64 l evaluations)
    Br, npt = 2048, 32
    U = torch.randn((Br, d), generator=g, dtype=torch.float64, device="cuda")
    Xr = X[:Br].clone()
    L.sb_chisao_reseed_dev(m, Xr, U, npt)  # tile autotune at this row count
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(reps):
        Xr.copy_(X[:Br])
        L.sb_chisao_reseed_dev(m, Xr, U, npt)
    torch.cuda.synchronize()
    dr = (time.perf_counter() - t2) / reps
    n_ev = B * (ns + n_anti)
    flops = n_ev * K * 2.0 * d * d
    return dict(workload=f"{name}: B={B} d={d} K={K} n_smooth={ns} n_anti={n_anti}",
                ms=dt * 1e3, grad_evals=n_ev, grad_evals_per_s=n_ev / dt,
                contraction_tflops=flops / dt / 1e12,
                frac_fp64_peak=flops / dt / 1e12 / PEAK["fp64"], stick_ms=ds * 1e3,
                n_stuck_after=int(sm.sum().item()),
                reseed=dict(rays=Br, n_pts=npt, ms=dr * 1e3,
                            logl_evals_per_s=Br * npt / dr))


def chisao_cycle_leg(L):
    """The ChiSao oscillation cycle (sb_evidence_chisao_dev, FP64) beside the single
    convergence phase: on the hidden-mode mixture at d = 16 (a narrow heavy component the
    coarse rays miss beside a wide one: one phase finds one mode, the cycle both; 256 rays x
    32 points, 16 starts, three oscillations) and on c1's K = 4 mixture at d = 64 with its
    4096 starts (three oscillations): wall time of each after a warm call, modes found, and
    |log Z - the reference mode set's| (Newton from every component mean, on the host)."""
    import oracle as O
    from paper_2601_19957_amd import synth

    out = {}
    cases = [("hidden_d16", synth.hidden_mode_mixture(16, 13),
              synth.RunConfig(n_rays=256, n_points=32, n_starts=16, seed=79),
              L.ChiSaoConfig(n_osc=3, n_anti=10, alpha_anti=0.05))]
    p1, c1 = synth.make_workload("c1")
    cases.append(("c1", p1, c1, L.ChiSaoConfig(n_osc=3, n_anti=4, alpha_anti=0.01)))
    for name, prob, cfg, cc in cases:
        ref = O.reference_modes(prob)
        row = dict(d=prob.d, K=prob.K, n_starts=cfg.n_starts, n_osc=cc.n_osc,
                   reference_modes=int(ref.n_modes))
        for lab, run in (("single_phase", L.EvidenceRunner(prob, cfg)),
                         ("cycle", L.EvidenceRunner(prob, cfg, chisao=cc))):
            run.run()
            t0 = time.perf_counter()
            r = run.run()
            dt = time.perf_counter() - t0
            row[lab] = dict(ms=dt * 1e3, modes=int(r.n_modes), log_z=float(r.log_z),
                            dlogz_vs_reference=abs(float(r.log_z) - float(ref.log_z)),
                            grad_evals=int(r.n_grad_evals))
        out[name] = row
        log(f"ChiSao cycle {name}: single phase {row['single_phase']['modes']} modes in "
            f"{row['single_phase']['ms']:.1f} ms, cycle {row['cycle']['modes']} modes in "
            f"{row['cycle']['ms']:.1f} ms (reference {row['reference_modes']})")
    return out


def reduce_leg(L, prob, name):
    """Dimensional reduction at the modes (Jacobi eigendecomposition of the K mode Hessians,
    FP64; the precisions, to which the separated mixture's mode Hessians are equal to e^-60):
    wall time of one sb_eig_reduce_dev call after a warm call, sweeps, d_eff, and the largest
    eigenvalue difference against numpy.linalg.eigh on the host."""
    import numpy as np
    import torch

    H = torch.as_tensor(prob.prec, device="cuda")
    lo = torch.as_tensor(prob.lo, device="cuda")
    hi = torch.as_tensor(prob.hi, device="cuda")
    L.sb_eig_reduce_dev(H[:1], lo, hi, 10.0, 1.5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = L.sb_eig_reduce_dev(H, lo, hi, 10.0, 1.5)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ev = r["eigval"].cpu().numpy()
    err = max(float(np.max(np.abs(ev[k] - np.sort(np.linalg.eigvalsh(prob.prec[k]))[::-1])))
              for k in range(prob.K))
    return dict(workload=f"{name}: {prob.K} matrices of n={prob.d}", ms=dt * 1e3,
                sweeps=r["sweeps"], d_eff=r["d_eff"], max_abs_eig_err_vs_numpy=err,
                max_eig=float(ev.max()))


USER_GAUSS_SRC = r"""
__device__ double gauss(const double *x, int d, const double *p) {
  const double *P = p, *mu = p + d * d;
  double q = 0.0;
  for (int i = 0; i < d; ++i) {
    double r = 0.0;
    for (int j = 0; j < d; ++j) r += P[i * d + j] * (x[j] - mu[j]);
    q += (x[i] - mu[i]) * r;
  }
  return -0.5 * q;
}
"""


def user_fd_leg(L, reps=5):
    """Generic user likelihood (a d = 64 Gaussian written as HIP source, compiled at run time):
    finite-difference gradients of 4096 points (2d + 3 evaluations each) and full FD Hessians
    at 4 points (2d^2 + 3 each), HIP events on the stream, in user-function evaluations per
    second; then the whole evidence path on it (discovery, FD L-BFGS, dedup, FD Laplace) against
    the Gaussian's closed form."""
    import numpy as np
    import torch
    from paper_2601_19957_amd import synth

    d, B = 64, 4096
    rng = np.random.Generator(np.random.PCG64(2601199576))
    P, _ = synth.random_precision(rng, d, 0.05, 1.0)
    mu = rng.uniform(-8, 8, d)
    params = torch.as_tensor(np.concatenate([P.ravel(), mu]), device="cuda")
    X = torch.as_tensor(mu + rng.standard_normal((B, d)), device="cuda")
    t0 = time.perf_counter()
    fn = L.UserLogL(USER_GAUSS_SRC, "gauss")
    compile_s = time.perf_counter() - t0
    out = {"workload": f"d={d} Gaussian as user HIP source", "compile_ms": compile_s * 1e3}
    stream = torch.cuda.current_stream()
    for name, Xb, full in (("fd_grad", X, False), ("fd_hessian", X[:4], True)):
        fn.fd(Xb, 1e-4, params, full=full)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            r = fn.fd(Xb, 1e-4, params, full=full)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        n_ev = Xb.shape[0] * ((2 * d * d + 3) if full else (2 * d + 3))
        out[name] = dict(points=int(Xb.shape[0]), ms=ms, user_evals_per_s=n_ev / (ms * 1e-3))
    g = r["H"].cpu().numpy()
    out["fd_hessian"]["max_abs_err_vs_closed_form"] = float(np.max(np.abs(g + P[None])))
    # the whole evidence path on the user likelihood (1024 rays x 32 points, 1024 starts)
    lo = torch.full((d,), -30.0, dtype=torch.float64, device="cuda")
    hi = torch.full((d,), 30.0, dtype=torch.float64, device="cuda")
    cfg = synth.RunConfig(n_rays=1024, n_points=32, n_starts=1024, m=8, max_iter=0,
                          max_modes=16, precision=synth.PREC_FP64, grad_tol=1e-7, dedup_tol=0.0,
                          seed=2601199577)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev = fn.evidence(d, lo, hi, cfg, 1e-5, 1e-3, 1e-3, params)
    dt = time.perf_counter() - t0
    lam = np.linalg.eigvalsh(P)
    ref = 0.5 * d * math.log(2 * math.pi) - 0.5 * float(np.sum(np.log(lam))) - d * math.log(60.0)
    out["evidence_path"] = dict(status=ev.status, ms=dt * 1e3, n_modes=ev.n_modes,
                                iterations=ev.iterations, grad_rows=ev.n_grad_evals,
                                user_evals=ev.n_logl_evals + ev.n_grad_evals * (2 * d + 3),
                                log_z=ev.log_z, closed_form=ref,
                                abs_err=abs(ev.log_z - ref))
    return out


def uneven_batch(L, serial=False):
    """The 512-problem uneven workload (d log-uniform in 8..512, K in 1..4,
    1024 starts each, FP64) as one sb_evidence_batch call: one warm-up call,
    then one timed call; log Z checked against the closed form -log V."""
    import numpy as np
    from paper_2601_19957_amd import synth

    probs, cfg = synth.make_workload("c3")
    cfgs = [synth.make_run_config("c3", seed=cfg.seed + j) for j in range(len(probs))]
    log(f"uneven batch: {len(probs)} problems, sum d = {sum(p.d for p in probs)}")
    L.sb_evidence_batch(probs, cfgs)
    t0 = time.perf_counter()
    res = L.sb_evidence_batch(probs, cfgs)
    dt = time.perf_counter() - t0
    ok = sum(1 for p, r in zip(probs, res) if r.status == 0 and r.n_modes == p.K)
    gap = max(abs(r.log_z + float(np.sum(np.log(p.hi - p.lo)))) for p, r in zip(probs, res)
              if r.status == 0 and r.n_modes == p.K) if ok else None
    evals = sum(r.n_grad_evals for r in res)
    out = dict(problems=len(probs), starts=sum(c.n_starts for c in cfgs), seconds=dt,
               problems_per_s=len(probs) / dt, logl_grad_evals_per_s=evals / dt,
               all_modes_found=f"{ok}/{len(probs)}", max_dlogz_vs_closed_form=gap,
               phases_ms=[round(x * 1e3, 2) for x in res[0].seconds[:7]], dtype="f64")
    log(f"uneven batch: {dt*1e3:.1f} ms, {ok}/{len(probs)} complete, gap {gap}")
    if serial:
        t0 = time.perf_counter()
        for p, c in zip(probs, cfgs):
            L.sb_evidence(p, c)
        ds = time.perf_counter() - t0
        out["serial_seconds"] = ds
        out["speedup_vs_serial"] = ds / dt
        log(f"one call per problem: {ds*1e3:.1f} ms")
    return out


def path_only(L, wl, args):
    """Only the whole path (for profiling one step): warm-up calls, then the timed steps between
    two boundary kernels (a one-element fill and multiply before, the same after), so that a
    kernel trace can be cut to exactly the timed steps."""
    import torch

    stream = torch.cuda.Stream()
    ex = L.ExecContext()
    runners = {n: L.EvidenceRunner(p, c, exec=ex) for n, (p, c) in wl.items()}
    for w in range(args.warmup):
        for n, r in runners.items():
            res = r.run(stream)
            log(f"warmup {w} {n}: {res.seconds[7] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    mark = torch.full((1,), 7.0, device="cuda")
    mark.mul_(3.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        for n, r in runners.items():
            r.run(stream)
        log(f"step {k} done")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    mark.mul_(3.0)
    torch.cuda.synchronize()
    print(json.dumps(dict(path_only=True, steps=args.steps,
                          ms_per_step=total / max(1, args.steps) * 1e3)), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--workload", default="c4a,c4b")
    ap.add_argument("--starts", type=int, default=None, help="override the start count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the uneven-batch leg (512 problems, d in 8..512)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the uneven-batch leg (for profiling it)")
    ap.add_argument("--no-host", action="store_true",
                    help="skip the host-entry (sb_evidence) time-to-log Z")
    ap.add_argument("--no-a3", action="store_true",
                    help="skip the per-config logL+grad (A3) precision variants")
    ap.add_argument("--batch-serial", action="store_true",
                    help="also time the uneven batch as one call per problem")
    ap.add_argument("--no-precheck", action="store_true",
                    help="skip the preprocessing-probe measurement")
    ap.add_argument("--no-reduce", action="store_true",
                    help="skip the eigen-reduction measurement")
    ap.add_argument("--no-user", action="store_true",
                    help="skip the generic-likelihood finite-difference measurement")
    ap.add_argument("--no-chisao", action="store_true",
                    help="skip the ChiSao-moves measurement")
    ap.add_argument("--no-f32-bulk", action="store_true",
                    help="skip the whole path with the FP32 matrix-core bulk contraction")
    ap.add_argument("--path-only", action="store_true",
                    help="only the whole path between boundary kernels (for profiling one step)")
    ap.add_argument("--no-step-variants", action="store_true",
                    help="skip the L-BFGS step roofline at c1, c2, c4b in FP32 and FP64")
    ap.add_argument("--modules-only", action="store_true",
                    help="only the preprocessing, eigen-reduction, user-likelihood and ChiSao legs")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only the roofline kernel timing (for profiling that kernel)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with the 1 GiB device copy that calibrates HBM byte counters")
    ap.add_argument("--a3-only", action="store_true",
                    help="only the logL+grad legs (a3_variants) and the L-BFGS step variants")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for {max(args.gpus, world)}): the evidence "
              "path here runs on a single MI355X; see DESIGN.md for how it would shard.",
              file=sys.stderr)
        return 2

    import torch
    import numpy as np
    from paper_2601_19957_amd import _lib as L

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    L.lib()
    if args.batch_only:
        print(json.dumps(dict(batch_only=True, uneven_batch=uneven_batch(L, args.batch_serial))),
              flush=True)
        return 0
    if args.a3_only:
        print(json.dumps(dict(a3_only=True, a3_variants=a3_variants(L),
                              lbfgs_step_variants=None if args.no_step_variants
                              else lbfgs_step_variants(L))), flush=True)
        return 0
    names = [n.strip() for n in args.workload.split(",") if n.strip()]
    log(f"generating {names}")
    wl = workload(names, args.starts)
    big = names[-1]
    prob_big, cfg_big = wl[big]
    if args.modules_only:
        print(json.dumps(dict(modules_only=True, precheck=precheck_leg(L, prob_big, big),
                              eig_reduce=reduce_leg(L, prob_big, big), user_fd=user_fd_leg(L),
                              chisao=chisao_leg(L, prob_big, big))),
              flush=True)
        return 0

    if args.path_only:
        return path_only(L, wl, args)

    # ---- roofline of the dominant kernel: the L-BFGS step at full batch
    log("timing the L-BFGS step at full batch")
    roofline = time_lbfgs_step(L, prob_big, cfg_big, hist_bf16=True)

    # ---- the bulk contraction (split BF16) at the largest posterior's shape
    log("timing the A3 contraction (split BF16) at the bulk shape")
    kt_s, kflops = time_quadform(L, prob_big, cfg_big.n_starts)
    kt32_s, _ = time_quadform(L, prob_big, cfg_big.n_starts, reps=5, dtype=L.DTYPE_F32)
    traffic = recorded_traffic() if (prob_big.d, prob_big.K, cfg_big.n_starts) == (1024, 8, 16384) \
        else None
    achieved = kflops / kt_s / 1e12
    contraction = dict(bound="mfma", achieved=achieved, peak=PEAK["bf16"], unit="TFLOP/s",
                       frac=achieved / PEAK["bf16"], traffic=traffic,
                       kernel="quad_gemm_bf16_kernel<3,0,...> (A3 contraction, FP32 data as "
                              "split BF16: 3 MFMA products per multiply-add)",
                       shape=f"B={cfg_big.n_starts} d={prob_big.d} K={prob_big.K}",
                       avg_launch_us=kt_s * 1e6,
                       executed_mfma_frac=3.0 * achieved / PEAK["bf16"],
                       fp32_equivalent_frac=achieved / PEAK["fp32"],
                       fp32_kernel_us=kt32_s * 1e6)
    log("timing the screened mixture contraction (listed start-component pairs)")
    pairs = time_quadform_pairs(L, prob_big, cfg_big.n_starts) if prob_big.K > 1 else None
    if pairs:
        log(f"pairs contraction: {pairs['avg_launch_us']:.1f} us, "
            f"{pairs['achieved']:.1f} TFLOP/s = {pairs['frac']:.3f} of BF16 peak")
    if args.kernel_only:
        print(json.dumps(dict(kernel_only=True, roofline=roofline,
                              contraction_roofline=contraction, pairs_roofline=pairs,
                              copy_calibration_bytes=calibration_copy())), flush=True)
        return 0

    # ---- whole path, inputs resident in HBM, on one stream; the iteration blocks replay
    # the execution context's HIP graphs (captured in the first warm-up call)
    stream = torch.cuda.Stream()
    ex = L.ExecContext()
    runners = {n: L.EvidenceRunner(p, c, exec=ex) for n, (p, c) in wl.items()}
    ref = {n: closed_form_logz(p) for n, (p, _) in wl.items()}
    cold = {}
    for w in range(args.warmup):
        for n, r in runners.items():
            tc = time.perf_counter()
            res = r.run(stream)
            if w == 0:
                cold[n] = time.perf_counter() - tc
            log(f"warmup {w} {n}: status {res.status} log Z {res.log_z:.9f} "
                f"(closed form {ref[n]:.9f}) modes {res.n_modes} iters {res.iterations} "
                f"evals {res.n_grad_evals} t {res.seconds[7]*1e3:.1f} ms "
                f"phases {[round(s*1e3, 2) for s in res.seconds[:7]]}")
    torch.cuda.synchronize()
    exec_before = ex.stats()
    per = {n: [] for n in names}
    last = {}
    evals = 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        for n, r in runners.items():
            ts = time.perf_counter()
            res = r.run(stream)
            per[n].append(time.perf_counter() - ts)
            evals += res.n_grad_evals
            last[n] = res
            if res.status != 0:
                log(f"step {k} {n}: status {res.status} {L.last_error()}")
        log(f"step {k} done")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    exec_after = ex.stats()
    exec_stats = {"timed_region": {k: exec_after[k] - exec_before[k] for k in exec_after},
                  "total": exec_after}
    log(f"execution context: {exec_stats}")

    # ---- the same calls through sb_evidence_dev: no context, nothing allocated, the blocks
    # launched directly
    direct = {}
    for n, (p, c) in wl.items():
        rd = L.EvidenceRunner(p, c)
        rd.run(stream)
        ts = []
        for _ in range(3):
            t1 = time.perf_counter()
            resd = rd.run(stream)
            ts.append(time.perf_counter() - t1)
        direct[n] = float(np.median(ts)) * 1e3
        same = resd.log_z == last[n].log_z and np.array_equal(resd.modes, last[n].modes)
        log(f"direct launches {n}: {direct[n]:.1f} ms, same result as the graph path: {same}")
        del rd
        torch.cuda.empty_cache()

    # ---- the same mixed path with parts of the bulk in plain FP32 (the library reads the
    # switches at each call): the FP32 matrix-core contraction and the FP32 history ring
    # (SB_BULK_GEMM=f32, SB_BULK_HIST=f32), and the split contraction with the FP32 ring
    # (SB_BULK_HIST=f32)
    variants = {"f32_matrix_bulk": {"SB_BULK_GEMM": "f32", "SB_BULK_HIST": "f32"},
                "f32_history": {"SB_BULK_HIST": "f32"}}
    bulk_var = {}
    if not args.no_f32_bulk:
        for vname, env in variants.items():
            bulk_var[vname] = {}
            os.environ.update(env)
            try:
                for n, (p, c) in wl.items():
                    rf = L.EvidenceRunner(p, c)
                    rf.run(stream)
                    ts = []
                    for _ in range(3):
                        t1 = time.perf_counter()
                        resf = rf.run(stream)
                        ts.append(time.perf_counter() - t1)
                    bulk_var[vname][n] = dict(ms=float(np.median(ts)) * 1e3, log_z=resf.log_z,
                                              evals=resf.n_grad_evals,
                                              iterations=resf.iterations, status=resf.status)
                    log(f"{vname} {n}: {bulk_var[vname][n]['ms']:.1f} ms, log Z "
                        f"{resf.log_z:.9f}, iters {resf.iterations}")
                    del rf
                    torch.cuda.empty_cache()
            finally:
                for k in env:
                    del os.environ[k]
    f32_bulk = bulk_var.get("f32_matrix_bulk", {})

    # ---- plain FP64 path, same pipeline and starts
    t64 = {}
    res64 = {}
    if not args.no_fp64:
        from paper_2601_19957_amd import synth

        for n, (p, c) in wl.items():
            c64 = synth.RunConfig(**{**vars(c), "precision": synth.PREC_FP64})
            r64 = L.EvidenceRunner(p, c64, exec=ex)
            r64.run(stream)  # warm (code objects, tile cache, block graph)
            ts = []
            for _ in range(args.fp64_steps):
                t1 = time.perf_counter()
                res64[n] = r64.run(stream)
                ts.append(time.perf_counter() - t1)
            t64[n] = float(np.median(ts))
            log(f"fp64 {n}: {t64[n]*1e3:.1f} ms log Z {res64[n].log_z:.9f} "
                f"iters {res64[n].iterations} evals {res64[n].n_grad_evals}")
            del r64
            torch.cuda.empty_cache()

    # ---- parity against the oracle's reference mode set (Newton from each mean)
    import oracle

    dlogz, dmodes, refz = {}, {}, {}
    for n, (p, _) in wl.items():
        refm = oracle.reference_modes(p)
        refz[n] = refm.log_z
        dlogz[n] = abs(last[n].log_z - refm.log_z) if n in last else None
        if n in last and last[n].n_modes == refm.n_modes:
            dmodes[n] = float(np.max(np.abs(last[n].modes - refm.modes)))
        log(f"{n}: |dlogZ| vs oracle {dlogz[n]:.3e} (closed form gap "
            f"{abs(refm.log_z - ref[n]):.3e}), modes {last[n].n_modes}/{refm.n_modes}")

    # ---- time-to-log Z through the host entry point (upload of the problem and allocation
    # of the device workspace included)
    host = {}
    if not args.no_host:
        for n, (p, c) in wl.items():
            ts = []
            for _ in range(2):
                t1 = time.perf_counter()
                rh = L.sb_evidence(p, c)
                ts.append(time.perf_counter() - t1)
            host[n] = float(np.median(ts)) * 1e3
            log(f"host entry {n}: {host[n]:.1f} ms, log Z {rh.log_z:.9f}")

    batch = None
    if not args.no_batch:
        batch = uneven_batch(L, serial=args.batch_serial)

    pre = None
    if not args.no_precheck:
        pre = precheck_leg(L, prob_big, big)
        log(f"precheck {big}: {pre['ms']:.3f} ms, {pre['tflops']:.1f} TFLOP/s")

    red = None
    if not args.no_reduce:
        red = reduce_leg(L, prob_big, big)
        log(f"eigen reduction {big}: {red['ms']:.1f} ms, {red['sweeps']} sweeps")

    ufd = None
    if not args.no_user:
        ufd = user_fd_leg(L)
        log(f"user FD: grad {ufd['fd_grad']['ms']:.3f} ms, hessian {ufd['fd_hessian']['ms']:.3f} ms")

    chi = None
    if not args.no_chisao:
        chi = chisao_leg(L, prob_big, big)
        log(f"ChiSao moves {big}: {chi['ms']:.1f} ms, {chi['grad_evals_per_s']:.3g} grad evals/s")
        chi["cycle"] = chisao_cycle_leg(L)

    a3 = None
    if not args.no_a3:
        a3 = a3_variants(L)
    steps_v = None
    if not args.no_step_variants:
        steps_v = lbfgs_step_variants(L)

    cpu = None
    if not args.no_cpu_baseline:
        log("CPU baseline (oracle) on a bounded sample")
        cb = cpu_baseline(prob_big, cfg_big)
        cpu = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample", "cpu_model",
                                  "single_thread")}

    ms_per_step = total / max(1, args.steps) * 1e3
    out = {
        "metric": "logL+grad evals/s and time-to-log Z at d=1024 vs plain FP64 (|dlogZ|<=1e-6)",
        "value": evals / total,
        "unit": "logL+grad evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16/f32/f64 (mixed)",
        "data": "synthetic",
        "config": {
            "workload": " + ".join(f"{n}: d={wl[n][0].d} K={wl[n][0].K} "
                                   f"{'Gaussian' if wl[n][0].K == 1 else 'mixture'} "
                                   f"{wl[n][1].n_rays}x{wl[n][1].n_points} rays, "
                                   f"{wl[n][1].n_starts} starts" for n in names),
            "precision": "mixed",
        },
        "time_to_logz_ms": {n: float(np.median(per[n])) * 1e3 for n in names},
        "time_to_logz_range_ms": {n: [min(per[n]) * 1e3, max(per[n]) * 1e3] for n in names},
        "time_to_logz_cold_ms": {n: cold[n] * 1e3 for n in cold},
        "time_to_logz_host_entry_ms": host or None,
        "time_to_logz_direct_ms": direct,
        "time_to_logz_f32_matrix_bulk": f32_bulk or None,
        "time_to_logz_f32_history": bulk_var.get("f32_history") or None,
        "exec_context": exec_stats,
        "phases_ms": {n: dict(zip(("prep", "discovery", "bulk", "dedup_pre",
                                   "polish_hessian_chol", "dedup_combine"),
                                  [round(last[n].seconds[i] * 1e3, 2) for i in (0, 1, 2, 3, 4, 6)]))
                      for n in last},
        "time_to_logz_fp64_ms": {n: t64[n] * 1e3 for n in t64},
        "speedup_vs_fp64": {n: t64[n] / float(np.median(per[n])) for n in t64},
        "dlogz_vs_oracle": dlogz,
        "dlogz_fp64_vs_oracle": {n: abs(res64[n].log_z - refz[n]) for n in res64},
        "max_mode_dist_vs_oracle": dmodes,
        "uneven_batch": batch,
        "a3_variants": a3,
        "lbfgs_step_variants": steps_v,
        "pairs_contraction_roofline": pairs,
        "precheck": pre,
        "eig_reduce": red,
        "user_fd": ufd,
        "chisao": chi,
        "roofline": roofline,
        "contraction_roofline": contraction,
        "cpu_baseline": cpu,
    }
    if args.calibrate_copy:
        calibration_copy()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
