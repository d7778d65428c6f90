#!/usr/bin/env python3
"""Benchmark of the slimLS hot path on one MI355X.

Workload (the plain single-slice method on the GPU): a 1024 x 1024 image,
720 angles uniform on [0, pi) x 1449 rays, 20 random ellipses, 1% noise,
blocks of 8 angles (11,592 rays), memory r = 10, lambda = 1e-3.  The Gram
system of the full window (p = 127,512) is solved by Jacobi-PCG with
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
  time_to_target  wall time and steps of the plain method to its stop rule
                (first k >= r+1 with ||s_k|| <= 1e-2 ||x_k||) and the error
                vs x_true there;
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


def window_nnz(N, thetas):
    """Non-zero Joseph weights of the listed angles: 2 d N^2 per angle."""
    return sum(2.0 * max(abs(math.cos(t)), abs(math.sin(t))) * N * N for t in thetas)


def cpu_baseline(cfg, b, x_true, budget_s):
    """Time the FP64 oracle's first steps of the same run (bounded)."""
    import numpy as np
    from oracle import slimls, system
    import synth

    N, na, g, r, lam = cfg["N"], cfg["n_angles"], cfg["g"], cfg["r"], cfg["lam"]
    P = system.Projector(N, na)
    T = slimls.Tomo(P, b, g, r, lam, x_true=x_true, chol_max_p=0, cg_tol=1e-6)
    sched = synth.schedule(na // g, 1, cfg["schedule_seed"])
    t0 = time.perf_counter()
    steps = 0
    for beta in sched:
        T.step(int(beta))
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    ell = g * P.R
    return {"value": ell * steps / dt, "unit": "rays/s", "cores": 1, "kind": "oracle",
            "sample": f"first {steps} slimLS steps of the same 1024^2 run from x=0 (window "
                      f"filling, p up to {min(steps, r + 1) * ell}), scipy CSR products, FP64 "
                      f"CG to 1e-6, CSR build of each new block included; {dt:.1f} s, "
                      f"single-threaded sparse kernels"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=12)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ttr", action="store_true", help="skip the time-to-target run")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; --gpus must be 1 "
              "(the batched-slice path shards by slices, see DESIGN.md)", file=sys.stderr)
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
    s = Slim(N, na, r=r, lam=lam, angles_per_block=g, gram_mode="pcg", pcg_tol=1e-6)
    R = s.R
    ell = g * R
    M = na // g
    sched = synth.schedule(M, 1 + (args.warmup + args.steps) // M + 1, cfg["schedule_seed"])
    theta = np.arange(na) * (np.pi / na)

    s.set_data(bd, x, xt)
    print(f"bench: warmup {args.warmup} steps", file=sys.stderr, flush=True)
    for k in range(args.warmup):
        beta = int(sched[k])
        s.step(list(range(beta * g, beta * g + g)))
    torch.cuda.synchronize()

    s.profile(True)
    iters = []
    flops_cg = 0.0
    window = [int(sched[k]) for k in range(max(0, args.warmup - r), args.warmup)]
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for k in range(args.warmup, args.warmup + args.steps):
        beta = int(sched[k])
        info = s.step(list(range(beta * g, beta * g + g)))
        window = (window + [beta])[-(r + 1):]
        ids = [a for bb in window for a in range(bb * g, bb * g + g)]
        flops_cg += info["pcg_iters"] * 2.0 * window_nnz(N, theta[ids])
        iters.append(info["pcg_iters"])
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    stats = s.kernel_stats()
    s.profile(False)
    print(f"bench: timed {args.steps} steps in {wall:.3f} s", file=sys.stderr, flush=True)

    # dominant kernel: CG forward or back over the window (same work per launch)
    dom = max(("cg_forward", "cg_back"), key=lambda k: stats[k]["total_ms"])
    st = stats[dom]
    avg_ms = st["total_ms"] / max(st["launches"], 1)
    flops_per_launch = flops_cg / max(sum(iters), 1)
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12

    # projector metric: one 8-angle block, fwd / back / fwd+back
    blk = list(range(8 * 37, 8 * 37 + 8))
    v = torch.randn((8, R), device=dev)

    def _time(fn, n=50):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n * 1e-3

    t_f = _time(lambda: s.project(blk, xt))
    t_b = _time(lambda: s.backproject(blk, v))
    projector = {"block_angles": 8, "rays": 8 * R, "fwd_rays_per_s": 8 * R / t_f,
                 "back_rays_per_s": 8 * R / t_b, "fwd_back_rays_per_s": 8 * R / (t_f + t_b),
                 "fwd_us": t_f * 1e6, "back_us": t_b * 1e6}

    ttr = None
    if not args.no_ttr:
        x.zero_()
        s.set_data(bd, x, xt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        k = 0
        nrm = float(np.linalg.norm(x_true))
        while True:
            beta = int(sched[k % len(sched)])
            info = s.step(list(range(beta * g, beta * g + g)))
            k += 1
            if k >= r + 1 and info["step_norm"] <= 1e-2 * info["x_norm"]:
                break
            if k >= 3 * M:
                break
        torch.cuda.synchronize()
        ttr = {"plain_s": time.perf_counter() - t1, "plain_steps": k,
               "rel_err_at_stop": info["err_norm"] / nrm, "stopped_by_rule": k < 3 * M}
        print(f"bench: time-to-target {ttr['plain_s']:.2f} s in {k} steps", file=sys.stderr,
              flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (FP64 oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cfg, b, x_true, args.cpu_budget)

    value = ell * args.steps / wall
    line = {
        "metric": "rays/s fwd+back + time-to-rel-err 1e-2, 1024^2 slice, plain",
        "value": value,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 CG scalars and norms)",
        "data": "synthetic: 20 random ellipses, exact line integrals + 1% Gaussian noise",
        "config": {"workload": "plain slimLS, 1024x1024 image, 720 angles x 1449 rays, "
                               "8 angles/block, r=10, lambda=1e-3, Jacobi-PCG to 1e-6",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": f"{dom} (88-angle window)",
                     "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": None,
                     "avg_launch_us": avg_ms * 1e3, "flops_per_launch": flops_per_launch},
        "cpu_baseline": cpu,
        "projector": projector,
        "time_to_target": ttr,
        "cg_iters_per_step": float(np.mean(iters)),
        "event_ms_timed_region": ev_ms,
        "kernel_ms": {k: v2["total_ms"] for k, v2 in stats.items()},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
