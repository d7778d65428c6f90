#!/usr/bin/env python3
"""Benchmark of the slimLS hot path on one MI355X.

Workload (the plain single-slice method on the GPU): a 1024 x 1024 image,
720 angles uniform on [0, pi) x 1449 rays, 20 random ellipses, 1% noise,
blocks of 8 angles (11,592 rays), memory r = 10, lambda = 1e-3.  The Gram
system of the full window (p = 127,512) is solved by conjugate gradients with
matrix-free projectors.  Inputs are seeded synthetic data resident in HBM
before timing.

A "step" is one slimLS iteration: residual of the sampled block, CG solve of
the Gram system, back-projection over the window and update of x.  `value`
is sampled rays per second through whole steps (block rays x steps / wall
time).  The line also carries:
  roofline      the dominant kernel (CG forward or back projector over the
                88-angle window), its algorithmic flops per launch (two per
                non-zero weight) over its average HIP-event launch time;
  projector     fwd, back and fwd+back rays/s of one 8-angle block;
  time_to_target  the plain method's stop rule (first k >= r+1 with
                ||s_k|| <= 1e-2 ||x_k||) fixes the target error e* (its error
                vs x_true there); time-to-target is the wall time to the
                first step with error <= e*;
  batched       the same parameters on B = 8 different 1024^2 slices in one
                context: wall time until every slice reaches the error its
                plain run had at its stop step, amortized over B, next to
                the plain runs' mean time-to-target;
  volume        512 slices of 512^2 (360 angles x 725 rays, 4 angles/block,
                r = 8): fwd/back rays/s of one block over all slices and
                the time of whole slimLS steps;
  mixed         64 x 256^2 + 32 x 512^2 + 8 x 1024^2 slices (360 angles, 4
                angles/block, r = 8): one context per size, stepped as one
                group with interleaved CG, vs the contexts one after another;
  gram_solve    explicit Gram mode on 256^2 (p = 2178): Gram update and FP64
                Cholesky + solves per step, the factorisation's FP64 TFLOP/s;
  warm_start    the learned warm start on 256^2 (180 angles, 1 angle/block,
                r = 5): steps to each held-out sample's e* from x0 = 0 and
                from x0 = CNN(u), single-slice wall-clock time-to-target with
                the warm start's cost included, CNN inference throughput;
  cpu_baseline  the FP64 oracle's steps of the same run on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP64_TFLOPS = 78.6

# HBM bytes per launch of the CG projector kernels on this workload, from
# rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch, mean over the
# 88-angle window launches that did work: launches enqueued past the CG stop
# return at entry and are left out; profiles/ has the summary and commands),
# each scaled by what the counter reads for a copy of 256 MiB (FETCH reads
# half: x2.0; WRITE x1.0), per kernel instance: the forward for every
# rays-per-lane count the autotuner can pick, the back-projector's one-slice
# tile.  Valid only for the projector code they were taken on (SHA-256 of
# the source without comments and layout, code_digest below); otherwise the
# line reports traffic as null.
PMC_TRAFFIC = {
    "source": "paper_1912_07962_amd/csrc/project.hip",
    "sha256": "675c893ad8e445ac5433b420f0e484f39f9e11cbad910a337370d682a9493ca4",
    "fetch_scale": 2.0,
    "write_scale": 1.0,
    # instance -> (FETCH_SIZE, WRITE_SIZE) KiB per dispatch
    "kib": {"cg_forward/2": (8294.6, 2008.5), "cg_forward/3": (8301.5, 3002.0),
            "cg_forward/4": (4213.9, 3984.8), "cg_forward/6": (6727.8, 5483.6),
            "cg_forward/8": (4236.4, 7969.5), "cg_back/1": (3051.0, 8192.0)},
}

# VALU wave instructions per launch of the same kernel instances, from
# rocprofv3 --pmc SQ_INSTS_VALU (median over the window launches of the same
# runs' kind; same source digest rule).  The FP32 vector peak (157.3 TFLOP/s
# = 256 CUs x 2.4 GHz x 128 FMA lanes) is two wave64 FP32 VALU instructions
# per CU and cycle: 1228.8 G instructions/s, the issue ceiling used here.
PMC_VALU = {
    "sha256": PMC_TRAFFIC["sha256"],
    "insts": {"cg_forward/8": 14363638, "cg_back/1": 13305856},
}
PEAK_VALU_GINST = 256 * 2.4 * 2


def pmc_valu(kind, avg_launch_s):
    """VALU issue of a kernel instance against the chip's VALU issue rate, or
    None when no counters were taken on this code and instance."""
    if kind not in PMC_VALU["insts"]:
        return None
    if code_digest(os.path.join(ROOT, PMC_TRAFFIC["source"])) != PMC_VALU["sha256"]:
        return None
    n = PMC_VALU["insts"][kind]
    rate = n / avg_launch_s / 1e9
    return {"insts_per_launch": n, "achieved_ginst_s": rate, "peak_ginst_s": PEAK_VALU_GINST,
            "frac": rate / PEAK_VALU_GINST}


def fwd_rays_per_lane(fwd_items, rays_in_group):
    """Rays per lane (the band kernel's IT) the library's launch plan uses for
    a one-slice forward: the tune's cap (0: the maximum, 8), limited to what
    the larger orientation group needs, rounded up to an instantiated value."""
    cap = min(fwd_items, 8) if fwd_items > 0 else 8
    want = max(1, min(cap, -(-rays_in_group // 512)))
    return want if want <= 6 else 8


def code_digest(path):
    """SHA-256 of a C++/HIP source with its comments and layout removed, so
    that edits to comments leave it unchanged (the code is what the counters
    measured)."""
    import hashlib
    import re
    with open(path, encoding="utf-8") as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    lines = (" ".join(line.split()) for line in text.splitlines())
    return hashlib.sha256("\n".join(l for l in lines if l).encode()).hexdigest()


def pmc_traffic(kind):
    """Scaled HBM bytes per launch of a kernel instance ("cg_forward/IT",
    "cg_back/BT"), or None."""
    t = PMC_TRAFFIC
    if t["sha256"] is None or kind not in t["kib"]:
        return None
    if code_digest(os.path.join(ROOT, t["source"])) != t["sha256"]:
        return None
    fetch, write = t["kib"][kind]
    return (fetch * t["fetch_scale"] + write * t["write_scale"]) * 1024.0


def window_nnz(N, thetas):
    """Non-zero Joseph weights of the listed angles: 2 d N^2 per angle."""
    return sum(2.0 * max(abs(math.cos(t)), abs(math.sin(t))) * N * N for t in thetas)


def cpu_baseline(cfg, b, sched, mean_cg_iters, budget_s):
    """Time the FP64 oracle on a full-window step of the same run (bounded).

    The oracle (scipy CSR products, FP64 CG) takes step r + 2 of the run, whose
    window holds the r + 1 = 11 blocks sched[1..r+1] (p = 127,512):
    the residual of the new block, CG iterations on the Gram system until the
    budget is spent, then s = M^T z and the update.  The step's cost is
    extrapolated to ``mean_cg_iters`` CG iterations (the GPU's mean per timed
    step at the same tolerance); building the CSR rows of the window is set
    up before timing and not counted."""
    import numpy as np
    from oracle import slimls, system

    N, na, g, r, lam = cfg["N"], cfg["n_angles"], cfg["g"], cfg["r"], cfg["lam"]
    P = system.Projector(N, na)
    T = slimls.Tomo(P, b, g, r, lam, chol_max_p=0, cg_tol=1e-6)
    window = [int(v) for v in sched[1:r + 2]]       # the window after step r + 2
    t_build = time.perf_counter()
    mats = [T.rows(beta) for beta in window]
    M = sp_vstack(mats)
    t_build = time.perf_counter() - t_build
    x = np.zeros(P.n)
    lam_k = lam
    t0 = time.perf_counter()
    res = np.asarray(mats[-1] @ x).reshape(-1) - T.data(window[-1])
    e = np.zeros(M.shape[0])
    e[-res.size:] = res
    t_res = time.perf_counter() - t0
    # bounded CG: the oracle's own routine with an iteration cap sized to the
    # budget from a two-iteration probe (the tolerance is never reached)
    apply = lambda v: M @ (M.T @ v) + lam_k * v
    t0 = time.perf_counter()
    slimls.cg(apply, e, 1e-300, max_iter=2)
    probe = (time.perf_counter() - t0) / 2.0
    its = int(max(2, min(200, budget_s / max(probe, 1e-6))))
    t0 = time.perf_counter()
    slimls.cg(apply, e, 1e-300, max_iter=its)
    t_it = (time.perf_counter() - t0) / its
    t0 = time.perf_counter()
    z = e * 0.0
    s_ = np.asarray(M.T @ z).reshape(-1)
    x = x - s_
    t_back = time.perf_counter() - t0
    step_s = t_res + mean_cg_iters * t_it + t_back
    ell = g * P.R
    return {"value": ell / step_s, "unit": "rays/s", "cores": 1, "kind": "oracle",
            "cpu": _cpu_model(), "nproc": os.cpu_count(),
            "sample": f"one full-window step of the same 1024^2 run (window of {r + 1} blocks, "
                      f"p = {M.shape[0]}): residual {t_res * 1e3:.0f} ms, {its} FP64 CG "
                      f"iterations at {t_it * 1e3:.0f} ms each extrapolated to the GPU's "
                      f"{mean_cg_iters:.1f} per step, back-projection and update "
                      f"{t_back * 1e3:.0f} ms; scipy CSR products (single-threaded), CSR "
                      f"rows of the window built beforehand in {t_build:.0f} s (not counted)"}


def sp_vstack(mats):
    import scipy.sparse as sp
    return sp.vstack(mats, format="csr")


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def plain_ttr(s, bd, x, xt, sched, g, r, M, nrm):
    """Plain run from x = 0 to the stop rule (first k >= r+1 with
    ||s_k|| <= 1e-2 ||x_k||, at most 3 epochs).  e* is the error there; the
    time-to-target is the wall time to the first step whose error is <= e*
    (the error is not monotone, so that step can come before the stop).
    Returns dict(stop_s, stop_steps, e_star, by_rule, s, steps)."""
    import torch
    x.zero_()
    torch.cuda.synchronize()          # x is zeroed on torch's stream, used on the library's
    s.set_data(bd, x, xt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k = 0
    trace = []
    while True:
        beta = int(sched[k % len(sched)])
        info = s.step(list(range(beta * g, beta * g + g)))
        k += 1
        trace.append((time.perf_counter() - t1, info["err_norm"] / nrm))
        if k >= r + 1 and info["step_norm"] <= 1e-2 * info["x_norm"]:
            break
        if k >= 3 * M:
            break
    torch.cuda.synchronize()
    stop_s = time.perf_counter() - t1
    e_star = trace[-1][1]
    first = next(i for i, (_, e) in enumerate(trace) if e <= e_star)
    return {"stop_s": stop_s, "stop_steps": k, "e_star": e_star, "by_rule": k < 3 * M,
            "s": trace[first][0], "steps": first + 1}


def batched_ttr(cfg, s1, sched, dev, B, autotune=True):
    """B different 1024^2 slices (phantom and noise seeds + slice index) under
    the plain parameters.  Each slice's plain run fixes its target e*_b (its
    error at its stop step); the batched context then steps all B slices
    together until every slice is within its own e*_b."""
    import numpy as np
    import torch
    import synth
    from paper_1912_07962_amd import Slim

    N, na, g, r, lam = cfg["N"], cfg["n_angles"], cfg["g"], cfg["r"], cfg["lam"]
    M = na // g
    print(f"bench: batched time-to-target, {B} slices", file=sys.stderr, flush=True)
    probs = [synth.make_slice_problem(N, na, cfg["n_ellipses"], cfg["noise"],
                                      cfg["phantom_seed"] + i, cfg["noise_seed"] + i)
             for i in range(B)]
    nrm = np.array([np.linalg.norm(p[0]) for p in probs])
    plain = []
    x1 = torch.zeros((N, N), dtype=torch.float32, device=dev)
    for i, (xt_i, b_i, _) in enumerate(probs):
        bd = torch.as_tensor(b_i, dtype=torch.float32, device=dev)
        xt = torch.as_tensor(xt_i, dtype=torch.float32, device=dev)
        plain.append(plain_ttr(s1, bd, x1, xt, sched, g, r, M, nrm[i]))
    e_star = np.array([p["e_star"] for p in plain])

    bd = torch.as_tensor(np.stack([p[1] for p in probs]), dtype=torch.float32, device=dev)
    xt = torch.as_tensor(np.stack([p[0] for p in probs]), dtype=torch.float32, device=dev)
    xb = torch.zeros((B, N, N), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    sb = Slim(N, na, r=r, lam=lam, n_slices=B, angles_per_block=g, gram_mode="pcg",
              pcg_tol=1e-6, stream=torch.cuda.Stream())
    tune = sb.autotune() if autotune else None
    sb.set_data(bd, xb, xt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k = 0
    iters = 0
    while True:
        beta = int(sched[k % len(sched)])
        info = sb.step(list(range(beta * g, beta * g + g)))
        iters += info["pcg_iters"]
        k += 1
        rel = sb.slice_norms()[:, 2] / nrm
        if np.all(rel <= e_star) or k >= 3 * M:
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    plain_mean = float(np.mean([p["s"] for p in plain]))
    out = {"slices": B, "plain_mean_s": plain_mean,
           "plain_steps": [p["steps"] for p in plain],
           "plain_stop_steps": [p["stop_steps"] for p in plain], "e_star": e_star.tolist(),
           "batched_wall_s": wall, "batched_amortized_s": wall / B, "batched_steps": k,
           "batched_cg_iters_per_step": iters / k,
           "reached": bool(np.all(rel <= e_star)),
           "speedup_vs_plain": plain_mean / (wall / B), "autotune": tune}
    print(f"bench: batched {wall:.2f} s for {B} slices ({wall / B:.3f} s each) vs plain "
          f"{plain_mean:.3f} s", file=sys.stderr, flush=True)
    sb.close()
    return out


def volume_bench(dev, B, steps, autotune=True):
    """512^2 slices of one ellipsoid volume sharing A (360 angles x 725 rays,
    4 angles/block, r = 8, lambda = 1e-3): one-block projector rays/s over
    all slices, then whole slimLS steps after the window has filled."""
    import numpy as np
    import torch
    import synth
    from paper_1912_07962_amd import Slim

    cfg = synth.get_config("c4")
    N, na, g, r, lam = cfg["N"], cfg["n_angles"], cfg["g"], cfg["r"], cfg["lam"]
    print(f"bench: volume {B} x {N}^2 inputs", file=sys.stderr, flush=True)
    xs, bs = synth.make_volume_problem(N, B, na, cfg["n_ellipsoids"], cfg["noise"],
                                       cfg["phantom_seed"], cfg["noise_seed"])
    xt = torch.as_tensor(xs, dtype=torch.float32, device=dev)
    bd = torch.as_tensor(bs, dtype=torch.float32, device=dev)
    del xs, bs
    torch.cuda.synchronize()
    vstream = torch.cuda.Stream()
    s = Slim(N, na, r=r, lam=lam, n_slices=B, angles_per_block=g, gram_mode="pcg", pcg_tol=1e-6,
             stream=vstream)
    tune = {"window": s.autotune(), "block": s.autotune(n_ids=g)} if autotune else None
    R = s.R
    ell = g * R
    theta = np.arange(na) * (np.pi / na)
    n_img = N * N

    def _time(fn, n=10):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(vstream)
        for _ in range(n):
            fn()
        e1.record(vstream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n * 1e-3

    proj = []
    v = torch.randn((B, g, R), device=dev)
    out_f = torch.empty((B, g, R), device=dev)
    out_b = torch.empty((B, N, N), device=dev)
    torch.cuda.synchronize()
    # a block of row-stepping angles (theta near 0) and one of column-stepping
    # angles (theta near pi/2; the public forward stages bands of columns of x
    # for those, transposed on their way into LDS)
    for blk in (list(range(0, g)), list(range(na // 2, na // 2 + g))):
        t_f = _time(lambda: s.project(blk, xt, out_f))
        t_b = _time(lambda: s.backproject(blk, v, out_b))
        nnz = window_nnz(N, theta[blk])
        byt = B * (8.0 * n_img + 8.0 * ell)     # fwd: x in, rays out; back: rays in, image out
        proj.append({"angles": blk, "fwd_us": t_f * 1e6, "back_us": t_b * 1e6,
                     "fwd_rays_per_s": ell * B / t_f, "back_rays_per_s": ell * B / t_b,
                     "fwd_back_rays_per_s": ell * B / (t_f + t_b),
                     "hbm_gbs_algorithmic": byt / (t_f + t_b) / 1e9,
                     "hbm_frac": byt / (t_f + t_b) / 1e9 / PEAK_HBM_GBS,
                     "alu_tflops": 2 * 2.0 * nnz * B / (t_f + t_b) / 1e12})
    del out_f, out_b, v

    x = torch.zeros((B, N, N), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    s.set_data(bd, x, xt)
    sched = synth.schedule(na // g, 1, cfg["schedule_seed"])
    for k in range(r + 1):
        beta = int(sched[k])
        s.step(list(range(beta * g, beta * g + g)))
    torch.cuda.synchronize()
    s.profile(True)
    t0 = time.perf_counter()
    iters = []
    flops = 0.0
    window = [int(sched[k]) for k in range(0, r + 1)]
    for k in range(r + 1, r + 1 + steps):
        beta = int(sched[k])
        info = s.step(list(range(beta * g, beta * g + g)))
        window = (window + [beta])[-(r + 1):]
        ids = [a for bb in window for a in range(bb * g, bb * g + g)]
        flops += info["pcg_iters"] * 2.0 * window_nnz(N, theta[ids]) * B
        iters.append(info["pcg_iters"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stats = s.kernel_stats()
    s.profile(False)
    # per CG iteration that did work: launches enqueued past the stop return
    # at entry, and their time is charged to the iterations that did work
    avg_f = stats["cg_forward"]["total_ms"] / max(sum(iters), 1) * 1e-3
    avg_b = stats["cg_back"]["total_ms"] / max(sum(iters), 1) * 1e-3
    fl = flops / max(sum(iters), 1)
    s.close()
    print(f"bench: volume step {wall / steps * 1e3:.1f} ms", file=sys.stderr, flush=True)
    return {"slices": B, "N": N, "block_rays": ell, "projector": proj, "autotune": tune,
            "ms_per_step": wall / steps * 1e3, "steps": steps,
            "slice_rays_per_s": ell * B * steps / wall,
            "cg_iters_per_step": float(np.mean(iters)),
            "cg_forward_us": avg_f * 1e6, "cg_back_us": avg_b * 1e6,
            "cg_forward_tflops": fl / avg_f / 1e12, "cg_back_tflops": fl / avg_b / 1e12,
            "kernel_ms": {k: v2["total_ms"] for k, v2 in stats.items()}}



def crossings3(N, n_det, w):
    """Ray-plane crossings inside the volume of one direction (each carries
    up to four non-zero bilinear weights): the walk of the 3D forward
    projector, counted on the host."""
    import numpy as np
    import synth
    w = np.asarray(w, np.float64)
    eu, ev = synth.detector_basis(w)
    m = int(np.argmax(np.abs(w)))
    a, b = [k for k in range(3) if k != m]
    hN, hn = (N - 1) / 2.0, (n_det - 1) / 2.0
    t = np.arange(n_det) - hn
    T, Q = np.meshgrid(t, t)
    lo = np.zeros_like(T)
    hi = np.full_like(T, N - 1.0)
    for ax in (a, b):
        s = w[ax] / w[m]
        f0 = hN + T * (eu[ax] - eu[m] * s) + Q * (ev[ax] - ev[m] * s) - hN * s
        if s != 0.0:
            e1, e2 = (-1.0 - f0) / s, (N - f0) / s
            lo = np.maximum(lo, np.minimum(e1, e2))
            hi = np.minimum(hi, np.maximum(e1, e2))
        else:
            hi = np.where((f0 > -1.0) & (f0 < N), hi, -1.0)
    return float(np.clip(np.floor(hi) - np.ceil(lo) + 1, 0, None).sum())


def proj3d_bench(dev, steps):
    """The paper's 3D experiment: a 511^3 volume, projection images of
    511 x 511 pixels from 1000 directions uniform on the sphere, one image per
    block, r = 0, alpha = 1 in unit-voxel scaling (lambda = h^2), 0.1% noise,
    CG to 1e-6: one-direction projector rays/s, then whole slimLS steps with
    the Jacobi-preconditioned CG (the library's default) and with plain CG."""
    import numpy as np
    import torch
    import synth
    from paper_1912_07962_amd import Slim3D

    cfg = synth.get_config("c3d")
    N, n, nd, r, lam = cfg["N"], cfg["n_det"], cfg["n_dirs"], cfg["r"], cfg["lam"]
    sched = synth.schedule(nd, 1, cfg["schedule_seed"])
    visit = [int(v) for v in sched[:steps + 1]]
    print(f"bench: 3D {N}^3 inputs ({len(visit)} directions)", file=sys.stderr, flush=True)
    x_true, b, dirs = synth.make_problem3(N, nd, n, cfg["n_ellipsoids"], cfg["noise"],
                                          cfg["phantom_seed"], cfg["dir_seed"], cfg["noise_seed"],
                                          dir_ids=visit)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        xt = torch.as_tensor(x_true, dtype=torch.float32, device=dev)
        bd = torch.as_tensor(b, dtype=torch.float32, device=dev)
        x = torch.zeros((N, N, N), dtype=torch.float32, device=dev)
        v = torch.randn((1, n, n), device=dev)
        out_f = torch.empty((1, n, n), device=dev)
        out_b = torch.empty((N, N, N), device=dev)
    st.synchronize()
    del x_true, b
    s = Slim3D(N, dirs, n_det=n, r=r, lam=lam, pcg_tol=1e-6, stream=st)

    def _time(fn, reps=10):
        fn()
        st.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        st.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    proj = []
    for d in visit[:2]:
        t_f = _time(lambda: s.project([d], xt, out_f))
        t_b = _time(lambda: s.backproject([d], v, out_b))
        cross = crossings3(N, n, dirs[d])
        w = np.abs(dirs[d])
        proj.append({"dir": d, "major_axis": "xyz"[int(np.argmax(w))],
                     "fwd_us": t_f * 1e6, "back_us": t_b * 1e6,
                     "fwd_rays_per_s": n * n / t_f, "back_rays_per_s": n * n / t_b,
                     "fwd_back_rays_per_s": n * n / (t_f + t_b),
                     # algorithmic traffic: the volume once and the image once each way
                     "fwd_hbm_frac": (4.0 * N ** 3 + 4.0 * n * n) / t_f / 1e9 / PEAK_HBM_GBS,
                     "back_hbm_frac": (4.0 * N ** 3 + 4.0 * n * n) / t_b / 1e9 / PEAK_HBM_GBS,
                     "crossings": cross,
                     "fwd_alu_tflops": 2 * 4.0 * cross / t_f / 1e12,
                     "back_alu_tflops": 2 * 4.0 * cross / t_b / 1e12})
    del out_f, out_b, v
    s.set_data(bd, x, xt)
    s.step([visit[0]])                          # first step: untimed
    st.synchronize()
    t0 = time.perf_counter()
    infos = []
    for d in visit[1:]:
        infos.append(s.step([d]))
    st.synchronize()
    wall = time.perf_counter() - t0
    # the same steps' kernels timed one by one on a second pass over fresh data
    s.set_data(bd, x.zero_(), xt)
    s.profile(True)
    for d in visit:
        s.step([d])
    stats = s.kernel_stats()
    s.profile(False)
    it = sum(i["pcg_iters"] for i in infos)
    cg_f = stats["cg_forward"]["total_ms"] / max(stats["cg_forward"]["launches"], 1)
    cg_b = stats["cg_back"]["total_ms"] / max(stats["cg_back"]["launches"], 1)
    s.close()
    # the same steps with plain (unpreconditioned) CG, for comparison
    s = Slim3D(N, dirs, n_det=n, r=r, lam=lam, pcg_tol=1e-6, stream=st, gram_mode="pcg")
    s.set_data(bd, x.zero_(), xt)
    s.step([visit[0]])
    st.synchronize()
    t0 = time.perf_counter()
    plain = [s.step([d]) for d in visit[1:]]
    st.synchronize()
    wall_plain = time.perf_counter() - t0
    s.close()
    it_plain = sum(i["pcg_iters"] for i in plain)
    print(f"bench: 3D step with plain CG {wall_plain / len(plain) * 1e3:.1f} ms, "
          f"{it_plain / len(plain):.1f} CG iterations", file=sys.stderr, flush=True)
    rel = [i["err_norm"] / float(np.linalg.norm(xt.cpu().numpy().astype(np.float64)))
           for i in infos[-1:]]
    print(f"bench: 3D step {wall / len(infos) * 1e3:.1f} ms, {it / len(infos):.1f} CG iterations",
          file=sys.stderr, flush=True)
    return {"N": N, "n_det": n, "n_dirs": nd, "r": r, "lambda": lam, "steps": len(infos),
            "ms_per_step": wall / len(infos) * 1e3, "rays_per_s": n * n * len(infos) / wall,
            "cg_iters_per_step": it / len(infos), "rel_err_last": rel[0],
            "cg_forward_us": cg_f * 1e3, "cg_back_us": cg_b * 1e3,
            "preconditioner": "jacobi",
            "plain_cg": {"ms_per_step": wall_plain / len(plain) * 1e3,
                         "cg_iters_per_step": it_plain / len(plain)},
            "kernel_ms": {k: v2["total_ms"] for k, v2 in stats.items()}, "projector": proj}


def precision_bench(dev, s_fp32_ms, steps=10):
    """The precision variant: the 64^2 workload's 20 epochs in FP32 and with
    bf16 storage (image shadow and sinogram), each epoch's error against the
    stored FP64 oracle run (tests/golden/c1_epochs.npz, written by the oracle
    alone) and against the oracle under the bf16 storage model; then the
    1024^2 workload's full-window steps with bf16 storage, timed against the
    FP32 steps of the headline."""
    import numpy as np
    import torch
    import synth
    from paper_1912_07962_amd import Slim

    gd = np.load(os.path.join(ROOT, "tests", "golden", "c1_epochs.npz"))
    cfg = synth.get_config("c3")
    N, na, r, lam, E = cfg["N"], cfg["n_angles"], cfg["r"], cfg["lam"], cfg["epochs"]
    x_true, b, _ = synth.make_slice_problem(N, na, cfg["n_ellipses"], cfg["noise"],
                                            cfg["phantom_seed"], cfg["noise_seed"])
    sched = gd["schedule"]   # the schedule the stored oracle run followed
    def rel(a, c):
        a = np.asarray(a, np.float64).reshape(-1)
        c = np.asarray(c, np.float64).reshape(-1)
        return float(np.linalg.norm(a - c) / np.linalg.norm(c))
    out = {"workload": "64^2, 90 angles x 91 rays, 1 angle/block, r = 5, lambda = 1e-2, 20 epochs"}
    for prec in ("fp32", "bf16"):
        st = torch.cuda.Stream()
        s = Slim(N, na, r=r, lam=lam, precision=prec, stream=st)
        with torch.cuda.stream(st):
            bd = torch.as_tensor(b, dtype=torch.float32, device=dev)
            if prec == "bf16":
                bd = bd.to(torch.bfloat16)
            x = torch.zeros((N, N), dtype=torch.float32, device=dev)
        st.synchronize()
        s.set_data(bd, x)
        e64, emod = [], []
        t0 = time.perf_counter()
        for k, beta in enumerate(sched, 1):
            s.step([int(beta)], read=False)
            if k % na == 0:
                st.synchronize()          # the steps run on the context's stream
                xe = x.cpu().numpy()
                e64.append(rel(xe, gd["x_fp64"][k // na - 1]))
                emod.append(rel(xe, gd["x_bf16"][k // na - 1]))
        wall = time.perf_counter() - t0
        out[prec] = {"rel_err_vs_fp64_per_epoch": e64, "rel_err_vs_bf16_model_per_epoch": emod,
                     "ms_per_step_incl_epoch_readback": wall / len(sched) * 1e3}
        s.close()
    out["rel_err_vs_x_true_fp64_oracle"] = [float(v) for v in gd["err_fp64"]]
    # 1024^2 full-window steps with bf16 storage
    cfg2 = synth.get_config("c2")
    N2, na2, g2, r2, lam2 = cfg2["N"], cfg2["n_angles"], cfg2["g"], cfg2["r"], cfg2["lam"]
    xt2, b2, _ = synth.make_slice_problem(N2, na2, cfg2["n_ellipses"], cfg2["noise"],
                                          cfg2["phantom_seed"], cfg2["noise_seed"])
    st = torch.cuda.Stream()
    s = Slim(N2, na2, r=r2, lam=lam2, angles_per_block=g2, gram_mode="pcg", pcg_tol=1e-6,
             precision="bf16", stream=st)
    s.autotune()
    with torch.cuda.stream(st):
        bd = torch.as_tensor(b2, dtype=torch.float32, device=dev).to(torch.bfloat16)
        x = torch.zeros((N2, N2), dtype=torch.float32, device=dev)
        xt = torch.as_tensor(xt2, dtype=torch.float32, device=dev)
    st.synchronize()
    s.set_data(bd, x, xt)
    sched2 = synth.schedule(na2 // g2, 1, cfg2["schedule_seed"])
    for k in range(r2 + 2):
        s.step(list(range(int(sched2[k]) * g2, int(sched2[k]) * g2 + g2)))
    st.synchronize()
    t0 = time.perf_counter()
    its = []
    for k in range(r2 + 2, r2 + 2 + steps):
        its.append(s.step(list(range(int(sched2[k]) * g2, int(sched2[k]) * g2 + g2)))["pcg_iters"])
    st.synchronize()
    wall = time.perf_counter() - t0
    s.close()
    out["bf16_1024"] = {"ms_per_step": wall / steps * 1e3, "fp32_ms_per_step": s_fp32_ms,
                        "cg_iters_per_step": float(np.mean(its)), "steps": steps}
    print(f"bench: precision variant: bf16 error vs FP64 {out['bf16']['rel_err_vs_fp64_per_epoch'][0]:.2e} "
          f"(epoch 1) .. {out['bf16']['rel_err_vs_fp64_per_epoch'][-1]:.2e} (epoch {E}); fp32 "
          f"{max(out['fp32']['rel_err_vs_fp64_per_epoch']):.2e} at most; 1024^2 bf16 "
          f"{out['bf16_1024']['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
    return out


def gram_bench(dev, steps):
    """Explicit Gram mode on the 256^2 workload (180 angles x 363 rays, 1
    angle/block, r = 5, lambda = 1e-2, p = 6 x 363 = 2178): per-step times of
    the Gram update (new block row of tiles + assembly of G) and of the FP64
    Cholesky with its two triangular solves, after the window has filled;
    the factorisation's p^3/3 flop against the FP64 peak."""
    import numpy as np
    import torch
    import synth
    from paper_1912_07962_amd import Slim

    cfg = synth.get_config("c5")
    N, na, g, r, lam = cfg["N"], cfg["n_angles"], cfg["g"], cfg["r"], cfg["lam"]
    x_true, b, _ = synth.make_slice_problem(N, na, cfg["n_ellipses"], cfg["noise"], 20000, 1020000)
    st = torch.cuda.Stream()
    s = Slim(N, na, r=r, lam=lam, angles_per_block=g, gram_mode="chol", stream=st)
    x = torch.zeros((N, N), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    s.set_data(torch.as_tensor(b, dtype=torch.float32, device=dev), x,
               torch.as_tensor(x_true, dtype=torch.float32, device=dev))
    sched = synth.schedule(na // g, 2, cfg["schedule_seed"])
    for k in range(r + 1):
        s.step([int(sched[k])])
    torch.cuda.synchronize()
    s.profile(True)
    t0 = time.perf_counter()
    for k in range(r + 1, r + 1 + steps):
        s.step([int(sched[k])])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stats = s.kernel_stats()
    s.profile(False)
    s.close()
    p = (r + 1) * g * s.R
    chol_ms = stats["cholesky"]["total_ms"] / steps
    gram_ms = stats["gram"]["total_ms"] / steps
    flops = p ** 3 / 3.0
    return {"workload": "256x256 image, 180 angles x 363 rays, 1 angle/block, r=5, lambda=1e-2",
            "p": p, "steps": steps, "ms_per_step": wall / steps * 1e3,
            "gram_ms_per_step": gram_ms, "cholesky_and_solves_ms_per_step": chol_ms,
            "factor_fp64_tflops": flops / (chol_ms * 1e-3) / 1e12,
            "factor_frac_fp64_peak": flops / (chol_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS}


def warm_bench(dev, n_test, n_timed):
    """Learned warm start on the 256^2 workload (180 angles x 363 rays, 1
    angle/block, r = 5, lambda = 1e-2) with the trained parameters shipped
    in the package: iterations to each test sample's e* from x0 = 0 and from
    x0 = CNN(u) over n_test held-out seeds (batched), then wall-clock
    time-to-target of single-slice runs for n_timed of them, the warm start's
    back-projection and CNN inference included."""
    import numpy as np
    import torch
    from paper_1912_07962_amd import Cnn, Slim
    from paper_1912_07962_amd import warmstart as ws

    cfg = ws.config()
    path = os.path.join(ROOT, "paper_1912_07962_amd", "weights", "warmstart_256.npy")
    net = Cnn(cfg["N"], ws.CHANNELS, max_batch=16, in_scale=ws.in_scale(cfg))
    net.set_params(np.load(path))
    seeds = range(cfg["test_seeds"][0], cfg["test_seeds"][0] + n_test)
    print(f"bench: warm start, {n_test} test samples", file=sys.stderr, flush=True)
    xte, bte = ws.make_samples(seeds, workers=min(16, os.cpu_count() or 1), cfg=cfg)
    plain = ws.plain_data(bte, xte, cfg)
    ev = ws.evaluate(net, bte, xte, plain, cfg)

    # error floor set by the null space of A: the part of x0 - x_true that no
    # update can remove (updates lie in R(A^T)), for the network's x0 and x0 = 0
    n_fl = min(32, n_test)
    x0_fl = ws.warm_start(net, plain["u"][:n_fl].contiguous(), net.max_batch)
    floors = []
    for lam_f in (1e-3, 1e-4):
        fl = ws.null_space_floor(x0_fl, xte[:n_fl], cfg, lam=lam_f, tol=1e-4, max_iter=4000)
        floors.append({"lambda": lam_f,
                       "net_x0_rel_mean": float(np.mean(fl["x0"]["rel_floor"])),
                       "net_x0_rel_max": float(np.max(fl["x0"]["rel_floor"])),
                       "zero_x0_rel_mean": float(np.mean(fl["zero"]["rel_floor"])),
                       "cg_iters": [fl["x0"]["cg_iters"], fl["zero"]["cg_iters"]],
                       "cg_relres": [fl["x0"]["cg_relres"], fl["zero"]["cg_relres"]]})
    ev["null_space_floor"] = {"samples": n_fl, "upper_bounds": floors,
                              "e_star_mean_same_samples": float(np.mean(plain["e_star"][:n_fl]))}
    print(f"bench: null-space floor <= {floors[-1]['net_x0_rel_mean']:.2e} (network x0), "
          f"{floors[-1]['zero_x0_rel_mean']:.2e} (x0 = 0) of ||x_true||; e* "
          f"{ev['null_space_floor']['e_star_mean_same_samples']:.3f}", file=sys.stderr, flush=True)
    del x0_fl

    # CNN inference throughput (batch 16)
    u16 = plain["u"][:16].contiguous()
    x16 = torch.empty_like(u16)
    net.forward(u16, x16)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        net.forward(u16, x16)
    e1.record()
    torch.cuda.synchronize()
    t_inf = e0.elapsed_time(e1) / 10 * 1e-3
    inf_tflops = net.forward_flops() * 16 / t_inf / 1e12

    # CNN training steps at batch 16 (loss, gradients, Adam) on a copy of the
    # network, targets the plain method's iterates; the convolution work of a
    # step is ~3x the forward's (forward, data and weight gradients)
    net_t = Cnn(cfg["N"], ws.CHANNELS, max_batch=16, in_scale=ws.in_scale(cfg))
    net_t.set_params(np.load(path))
    t16 = plain["target"][:16].contiguous()
    for _ in range(2):
        net_t.loss_grad(u16, t16)
        net_t.adam(1e-5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        net_t.loss_grad(u16, t16)
        net_t.adam(1e-5)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / 10
    net_t.close()
    train_tflops = 3.0 * net.forward_flops() * 16 / t_train / 1e12

    # single-slice wall clock
    N, g, r = cfg["N"], cfg["g"], cfg["r"]
    sched = ws.schedule(cfg)
    first = ws.first_angles(cfg)
    s = Slim(N, cfg["n_angles"], r=r, lam=cfg["lam"], angles_per_block=g, gram_mode="chol")
    x = torch.zeros((N, N), dtype=torch.float32, device=dev)
    t_plain, t_warm, st_plain, st_warm = [], [], [], []
    for i in range(n_timed):
        bd = torch.as_tensor(bte[i], device=dev)
        xt = torch.as_tensor(xte[i], device=dev)
        nrm = float(np.linalg.norm(xte[i]))
        e_star = float(plain["e_star"][i])
        for warm in (False, True):
            x.zero_()
            s.set_data(bd, x, xt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            k = 0
            if warm:
                s.warmstart(first, x0=x, net=net)  # into the bound x: restarts from x0
            err = float(torch.linalg.vector_norm(x - xt)) / nrm if warm else 1.0
            while err > e_star and k < len(sched):
                beta = int(sched[k])
                info = s.step(list(range(beta * g, beta * g + g)))
                k += 1
                err = info["err_norm"] / nrm
            torch.cuda.synchronize()
            (t_warm if warm else t_plain).append(time.perf_counter() - t0)
            (st_warm if warm else st_plain).append(k)
    s.close()
    ev.update({"test_samples": n_test, "timed_samples": n_timed,
               "plain_s_mean": float(np.mean(t_plain)), "warm_s_mean": float(np.mean(t_warm)),
               "timed_plain_steps_mean": float(np.mean(st_plain)),
               "timed_warm_steps_mean": float(np.mean(st_warm)),
               "speedup_vs_plain": float(np.mean(t_plain) / np.mean(t_warm)),
               "cnn_inference_ms_batch16": t_inf * 1e3, "cnn_inference_tflops": inf_tflops,
               "cnn_inference_mfma_frac": inf_tflops / PEAK_BF16_TFLOPS,
               "cnn_train_step_ms_batch16": t_train * 1e3, "cnn_train_tflops_3x_forward": train_tflops})
    net.close()
    print(f"bench: warm {ev['warm_s_mean']:.3f} s vs plain {ev['plain_s_mean']:.3f} s per slice",
          file=sys.stderr, flush=True)
    return ev



def stream_bench(s_res, cfg, x_true, b, sched, warmup, steps, stream, resident_ms):
    """The same 1024^2 steps with each block's rows handed over from pinned host
    memory (slim_step_data) instead of a resident sinogram: the PCIe-inclusive
    rate, read back every step, and read back only at the end (the copy of the
    next block then overlaps the current step)."""
    import numpy as np
    import torch
    from paper_1912_07962_amd import Slim

    N, na, g, r, lam = cfg["N"], cfg["n_angles"], cfg["g"], cfg["r"], cfg["lam"]
    dev = torch.device("cuda:0")
    t = s_res.get_tune()
    out = {"block_bytes": None}
    for mode in ("read_every_step", "read_at_end"):
        ss = Slim(N, na, r=r, lam=lam, angles_per_block=g, gram_mode="pcg", pcg_tol=1e-6,
                  stream=stream)
        ss.set_tune(fwd_bt=t["fwd_bt"], fwd_items=t["fwd_items"], fwd_slots=t["fwd_slots"],
                    back_bt=t["back_bt"])
        x = torch.zeros((N, N), dtype=torch.float32, device=dev)
        ss.set_data(None, x, torch.as_tensor(x_true, dtype=torch.float32, device=dev))
        bb = np.asarray(b, np.float32).reshape(na, -1)
        blocks = []
        for k in range(warmup + steps):
            beta = int(sched[k])
            ids = list(range(beta * g, beta * g + g))
            blocks.append((ids, torch.from_numpy(np.ascontiguousarray(bb[ids])).pin_memory()))
        out["block_bytes"] = blocks[0][1].numel() * 4
        for ids, blk in blocks[:warmup]:
            ss.step_data(ids, blk)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k, (ids, blk) in enumerate(blocks[warmup:]):
            ss.step_data(ids, blk, read=(mode == "read_every_step" or k == steps - 1))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[mode] = {"ms_per_step": wall / steps * 1e3,
                     "rays_per_s": g * ss.R * steps / wall}
        ss.close()
    out["resident_ms_per_step"] = resident_ms
    print(f"bench: streamed blocks {out['read_every_step']['ms_per_step']:.2f} / "
          f"{out['read_at_end']['ms_per_step']:.2f} ms/step (resident {resident_ms:.2f})",
          file=sys.stderr, flush=True)
    return out


def tik_bench(s_res, cfg, bd, xt, sched, warmup, steps, stream, resident_ms, resident_iters, tik):
    """The same 1024^2 steps as slimTik with L = I (one more forward projection
    of the window per step; the Tikhonov shift also changes the CG's
    conditioning): ms per step and CG iterations against plain slimLS."""
    import torch
    from paper_1912_07962_amd import Slim

    N, na, g, r, lam = cfg["N"], cfg["n_angles"], cfg["g"], cfg["r"], cfg["lam"]
    t = s_res.get_tune()
    st = Slim(N, na, r=r, lam=lam, angles_per_block=g, gram_mode="pcg", pcg_tol=1e-6,
              stream=stream, tikhonov=tik)
    st.set_tune(fwd_bt=t["fwd_bt"], fwd_items=t["fwd_items"], fwd_slots=t["fwd_slots"],
                back_bt=t["back_bt"])
    x = torch.zeros((N, N), dtype=torch.float32, device=bd.device)
    st.set_data(bd, x, xt)
    for k in range(warmup):
        beta = int(sched[k])
        st.step(list(range(beta * g, beta * g + g)))
    torch.cuda.synchronize()
    iters = []
    t0 = time.perf_counter()
    for k in range(warmup, warmup + steps):
        beta = int(sched[k])
        iters.append(st.step(list(range(beta * g, beta * g + g)))["pcg_iters"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st.close()
    out = {"tikhonov": tik, "ms_per_step": wall / steps * 1e3,
           "cg_iters_per_step": sum(iters) / steps, "plain_ms_per_step": resident_ms,
           "plain_cg_iters_per_step": resident_iters}
    print(f"bench: slimTik {out['ms_per_step']:.2f} ms/step, {out['cg_iters_per_step']:.1f} CG "
          f"iterations (plain {resident_ms:.2f}, {resident_iters:.1f})", file=sys.stderr, flush=True)
    return out


def mixed_bench(dev, steps, autotune=True):
    """Mixed batch: 64 slices of 256^2, 32 of 512^2 and 8 of 1024^2 (one
    ellipsoid volume sampled at three resolutions), 360 angles, 4 angles per
    block, r = 8, lambda = 1e-3, CG; one context per size on its own stream.
    Three identical sets of contexts take the same steps: stepped as one
    group whose CG solves run in shared launches (one launch per kernel per
    iteration over all sizes, chunks replayed as graphs), as one group with
    each context's own launches interleaved by the host, and one context
    after another.  All take the same r + 1 steps first, so every timed step
    has a full window."""
    import numpy as np
    import torch
    import synth
    from paper_1912_07962_amd import Group, Slim

    cfg = synth.get_config("c4m")
    na, g, r, lam = cfg["n_angles"], cfg["g"], cfg["r"], cfg["lam"]
    print("bench: mixed batch inputs", file=sys.stderr, flush=True)
    modes = ("shared", "interleaved", "sequential")
    sets = {m: [] for m in modes}
    keep, rays, tunes = [], 0, []
    for N, B in cfg["groups"]:
        xs, bs = synth.make_volume_problem(N, B, na, cfg["n_ellipsoids"], cfg["noise"],
                                           cfg["phantom_seed"], cfg["noise_seed"])
        tuned = None
        for m in modes:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                s = Slim(N, na, r=r, lam=lam, n_slices=B, angles_per_block=g, gram_mode="pcg",
                         pcg_tol=1e-6, stream=st)
                if autotune and tuned is None:
                    tuned = s.autotune()["chosen"]
                    tunes.append(tuned)
                elif tuned is not None:
                    s.set_tune(**tuned)
                bd = torch.as_tensor(bs, dtype=torch.float32, device=dev)
                xt = torch.as_tensor(xs, dtype=torch.float32, device=dev)
                x = torch.zeros((B, N, N), dtype=torch.float32, device=dev)
            st.synchronize()
            s.set_data(bd, x, xt)
            sets[m].append(s)
            keep.append((st, bd, xt, x))
        rays += B * g * sets["shared"][-1].R
    grp = {"shared": Group(sets["shared"], shared=True),
           "interleaved": Group(sets["interleaved"], shared=False)}
    sched = synth.schedule(na // g, 1, cfg["schedule_seed"])
    blk = lambda k: list(range(int(sched[k]) * g, int(sched[k]) * g + g))

    def run(m, k):
        if m in grp:
            return grp[m].step(blk(k))
        return [s.step(blk(k)) for s in sets[m]]

    for k in range(r + 1):
        for m in modes:
            run(m, k)
    torch.cuda.synchronize()
    ms, iters = {}, {}
    for m in modes:
        t0 = time.perf_counter()
        for k in range(r + 1, r + 1 + steps):
            infos = run(m, k)
        torch.cuda.synchronize()
        ms[m] = (time.perf_counter() - t0) / steps * 1e3
        iters[m] = [i["pcg_iters"] for i in infos]
    # per size: largest |x_shared - x_other| after the last step
    diff = {m: [(a[3] - b[3]).abs().max().item() for a, b in zip(keep[0::3], keep[j::3])]
            for j, m in ((1, "interleaved"), (2, "sequential"))}
    same = all(v == 0.0 for d in diff.values() for v in d)
    for gp in grp.values():
        gp.close()
    for m in modes:
        for s in sets[m]:
            s.close()
    print(f"bench: mixed batch {ms['shared']:.1f} ms/step shared launches, "
          f"{ms['interleaved']:.1f} interleaved, {ms['sequential']:.1f} sequential",
          file=sys.stderr, flush=True)
    return {"groups": [list(gp) for gp in cfg["groups"]], "steps": steps,
            "shared_ms_per_step": ms["shared"], "interleaved_ms_per_step": ms["interleaved"],
            "sequential_ms_per_step": ms["sequential"],
            "shared_speedup_vs_sequential": ms["sequential"] / ms["shared"],
            "shared_speedup_vs_interleaved": ms["interleaved"] / ms["shared"],
            "slice_rays_per_s": rays / (ms["shared"] * 1e-3),
            "same_steps": iters["shared"] == iters["interleaved"] == iters["sequential"],
            "results_identical": bool(same), "max_abs_diff_vs_shared": diff,
            "cg_iters_last_step": iters["shared"], "autotune": tunes}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=12)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ttr", action="store_true", help="skip the time-to-target run")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched time-to-target run")
    ap.add_argument("--batch", type=int, default=8, help="slices of the batched run")
    ap.add_argument("--volume-slices", type=int, default=512,
                    help="slices of the 512^2 volume workload (0 skips it)")
    ap.add_argument("--volume-steps", type=int, default=4, help="timed volume steps")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in projector launch shapes")
    ap.add_argument("--fix-tune", default=None, metavar="FB,FI,FS,BB",
                    help="launch shape of the 1024^2 context (fwd_bt, fwd_items, fwd_slots, "
                         "back_bt) instead of its autotuner search; profiling runs pin it, "
                         "since a profiler perturbs the search's timings")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="copy 256 MiB once before timing (a kernel of known traffic for "
                         "scaling hardware byte counters)")
    ap.add_argument("--stream-steps", type=int, default=20,
                    help="timed steps with blocks handed over from host memory (0: skip)")
    ap.add_argument("--tik-steps", type=int, default=20,
                    help="timed slimTik steps (L = I) of the same workload (0: skip)")
    ap.add_argument("--tikhonov", type=float, default=0.1,
                    help="Tikhonov parameter of the slimTik leg")
    ap.add_argument("--mixed-steps", type=int, default=3,
                    help="timed steps of the mixed batch (0 skips it)")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the precision-variant leg (bf16 storage)")
    ap.add_argument("--proj3d-steps", type=int, default=3,
                    help="timed steps of the 3D random-direction workload (0 skips it)")
    ap.add_argument("--gram-steps", type=int, default=20,
                    help="timed steps of the explicit-Gram (FP64 Cholesky) 256^2 run (0 skips it)")
    ap.add_argument("--warm-test", type=int, default=256,
                    help="held-out samples of the warm-start evaluation (0 skips it)")
    ap.add_argument("--warm-timed", type=int, default=8,
                    help="of those, samples timed as single-slice runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only; --gpus must be 1 (more GPUs would "
              "each take a share of the slices)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1912_07962_amd import Slim

    cfg = synth.get_config("c2")
    N, na, g, r, lam = cfg["N"], cfg["n_angles"], cfg["g"], cfg["r"], cfg["lam"]
    x_true, b, _ = synth.make_slice_problem(N, na, cfg["n_ellipses"], cfg["noise"],
                                            cfg["phantom_seed"], cfg["noise_seed"])
    dev = torch.device("cuda:0")
    bd = torch.as_tensor(b, dtype=torch.float32, device=dev)
    xt = torch.as_tensor(x_true, dtype=torch.float32, device=dev)
    x = torch.zeros((N, N), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    # the library's own stream (default priority): CG chunks replay as graphs
    main_stream = torch.cuda.Stream()
    s = Slim(N, na, r=r, lam=lam, angles_per_block=g, gram_mode="pcg", pcg_tol=1e-6,
             stream=main_stream)
    if args.fix_tune:
        fb, fi, fs, bb = (int(v) for v in args.fix_tune.split(","))
        s.set_tune(fwd_bt=fb, fwd_items=fi, fwd_slots=fs, back_bt=bb)
        tune = {"fixed": s.get_tune()}
    else:
        tune = None if args.no_autotune else s.autotune()
    R = s.R
    ell = g * R
    M = na // g
    sched = synth.schedule(M, 1 + (max(args.warmup, r + 2) + 2 * args.steps) // M + 1,
                           cfg["schedule_seed"])
    theta = np.arange(na) * (np.pi / na)

    if args.calibration_copy:
        # 256 MiB read + 256 MiB written by a blit copy and by an elementwise
        # kernel: known traffic for scaling the hardware byte counters
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    s.set_data(bd, x, xt)
    # the timed steps start with the memory window full (r + 1 blocks) whatever
    # --warmup says; steps r + 1 and r + 2 are checked against the FP64 oracle
    # run stored for this workload (same schedule, CG to 1e-12)
    warmup = max(args.warmup, r + 2)
    print(f"bench: warmup {warmup} steps", file=sys.stderr, flush=True)
    gold = np.load(os.path.join(ROOT, "tests", "golden", "c2_window.npz"))
    assert [int(v) for v in gold["blocks"]] == [int(v) for v in sched[:r + 2]]
    parity = {}
    for k in range(warmup):
        beta = int(sched[k])
        s.step(list(range(beta * g, beta * g + g)))
        if f"x{k + 1}" in gold.files:
            ref = gold[f"x{k + 1}"].astype(np.float64).reshape(-1)
            got = x.cpu().numpy().astype(np.float64).reshape(-1)
            parity[f"step_{k + 1}"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    torch.cuda.synchronize()

    # timed region: exactly `steps` steps, no instrumentation
    iters = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(main_stream)
    for k in range(warmup, warmup + args.steps):
        beta = int(sched[k])
        info = s.step(list(range(beta * g, beta * g + g)))
        iters.append(info["pcg_iters"])
    ev1.record(main_stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    print(f"bench: timed {args.steps} steps in {wall:.3f} s", file=sys.stderr, flush=True)

    # the next `steps` steps with HIP events around every kernel on the
    # library's stream (launched one by one): per-kernel times for the roofline
    s.profile(True)
    prof_iters = []
    flops_cg = 0.0
    k0 = warmup + args.steps
    window = [int(sched[k]) for k in range(max(0, k0 - r), k0)]
    for k in range(k0, k0 + args.steps):
        beta = int(sched[k])
        info = s.step(list(range(beta * g, beta * g + g)))
        window = (window + [beta])[-(r + 1):]
        ids = [a for bb in window for a in range(bb * g, bb * g + g)]
        flops_cg += info["pcg_iters"] * 2.0 * window_nnz(N, theta[ids])
        prof_iters.append(info["pcg_iters"])
    torch.cuda.synchronize()
    stats = s.kernel_stats()
    s.profile(False)

    # dominant kernel: CG forward or back over the window (same work per launch)
    dom = max(("cg_forward", "cg_back"), key=lambda k: stats[k]["total_ms"])
    shape = s.get_tune()
    n_row = sum(1 for a in ids if abs(np.cos(theta[a])) >= abs(np.sin(theta[a])))
    inst = (f"cg_forward/{fwd_rays_per_lane(shape['fwd_items'], max(n_row, len(ids) - n_row) * R)}"
            if dom == "cg_forward" else "cg_back/1")
    kernel_name = (f"fwd_band_kernel<{inst.split('/')[1]}, 1, float>" if dom == "cg_forward"
                   else "back_kernel<double, 1>")
    st = stats[dom]
    # per CG iteration that did work (launches enqueued past the stop return
    # at entry; their time is charged to the iterations that did work)
    avg_ms = st["total_ms"] / max(sum(prof_iters), 1)
    flops_per_launch = flops_cg / max(sum(prof_iters), 1)
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12

    # projector metric: one 8-angle block, fwd / back / fwd+back
    blk = list(range(8 * 37, 8 * 37 + 8))
    v = torch.randn((8, R), device=dev)

    def _time(fn, n=50):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(main_stream)
        for _ in range(n):
            fn()
        e1.record(main_stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n * 1e-3

    with torch.cuda.stream(main_stream):
        out_f = torch.empty((8, R), device=dev)
        out_b = torch.empty((N, N), device=dev)
    t_f = _time(lambda: s.project(blk, xt, out_f))
    t_b = _time(lambda: s.backproject(blk, v, out_b))
    projector = {"block_angles": 8, "rays": 8 * R, "fwd_rays_per_s": 8 * R / t_f,
                 "back_rays_per_s": 8 * R / t_b, "fwd_back_rays_per_s": 8 * R / (t_f + t_b),
                 "fwd_us": t_f * 1e6, "back_us": t_b * 1e6}

    streaming = None
    if args.stream_steps > 0:
        streaming = stream_bench(s, cfg, x_true, b, sched, warmup,
                                 min(args.stream_steps, len(sched) - warmup), main_stream,
                                 wall / args.steps * 1e3)

    tik = None
    if args.tik_steps > 0:
        tik = tik_bench(s, cfg, bd, xt, sched, warmup,
                        min(args.tik_steps, len(sched) - warmup), main_stream,
                        wall / args.steps * 1e3, sum(iters) / len(iters), args.tikhonov)

    ttr = None
    if not args.no_ttr:
        t = plain_ttr(s, bd, x, xt, sched, g, r, M, float(np.linalg.norm(x_true)))
        ttr = {"plain_s": t["s"], "plain_steps": t["steps"], "rel_err_target": t["e_star"],
               "stop_rule_s": t["stop_s"], "stop_rule_steps": t["stop_steps"],
               "stopped_by_rule": t["by_rule"]}
        print(f"bench: time-to-target {t['s']:.2f} s in {t['steps']} steps (stop rule at "
              f"{t['stop_steps']})", file=sys.stderr, flush=True)

    batched = None
    if not args.no_batched:
        batched = batched_ttr(cfg, s, sched, dev, args.batch, not args.no_autotune)

    gram = None
    if args.gram_steps > 0:
        print("bench: explicit Gram mode, 256^2", file=sys.stderr, flush=True)
        gram = gram_bench(dev, args.gram_steps)

    warm = None
    if args.warm_test > 0:
        warm = warm_bench(dev, args.warm_test, min(args.warm_timed, args.warm_test))

    mixed = None
    if args.mixed_steps > 0:
        mixed = mixed_bench(dev, args.mixed_steps, not args.no_autotune)

    volume = None
    if args.volume_slices > 0:
        volume = volume_bench(dev, args.volume_slices, args.volume_steps, not args.no_autotune)

    precision = None
    if not args.no_precision:
        precision = precision_bench(dev, wall / args.steps * 1e3)

    p3d = None
    if args.proj3d_steps > 0:
        p3d = proj3d_bench(dev, args.proj3d_steps)

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (FP64 oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cfg, b, sched, float(np.mean(iters)), args.cpu_budget)

    value = ell * args.steps / wall
    line = {
        "metric": "rays/s fwd+back + time-to-rel-err 1e-2, 1024^2 slice, plain",
        "value": value,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": warmup,
        "warmup_requested": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 CG scalars and norms)",
        "data": "synthetic: 20 random ellipses, exact line integrals + 1% Gaussian noise",
        "config": {"workload": "plain slimLS, 1024x1024 image, 720 angles x 1449 rays, "
                               "8 angles/block, r=10, lambda=1e-3, CG to 1e-6",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": f"{dom}: {kernel_name} (88-angle window)",
                     "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": pmc_traffic(inst),
                     "avg_launch_us": avg_ms * 1e3, "flops_per_launch": flops_per_launch,
                     "valu_issue": pmc_valu(inst, avg_ms * 1e-3)},
        "cpu_baseline": cpu,
        "autotune": tune,
        "projector": projector,
        "time_to_target": ttr,
        "batched": batched,
        "streaming": streaming,
        "slimtik": tik,
        "volume": volume,
        "mixed": mixed,
        "gram_solve": gram,
        "proj3d": p3d,
        "precision": precision,
        "warm_start": warm,
        "cg_iters_per_step": float(np.mean(iters)),
        "window_blocks_timed": r + 1,
        "parity_rel_err": {"vs": "FP64 oracle (CG to 1e-12), same schedule from x = 0",
                           "cg_tol": 1e-6, **parity},
        "event_ms_timed_region": ev_ms,
        "graphs": True,
        "kernel_ms": {k: v2["total_ms"] for k, v2 in stats.items()},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
