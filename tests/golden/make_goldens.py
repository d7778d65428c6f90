"""Write the stored expected values of the full-size parity tests.

Every value stored here comes from the FP64 oracle (``oracle/``) run on the
seeded inputs of ``synth/``; nothing else is imported.  The runs are too slow
for a test (CG to a relative residual of 1e-12 on Gram systems of up to
127,512 rows), so they are made once on the CPU and stored as compressed
numpy archives next to this script.

  c2_window   the 1024^2 plain workload (720 angles x 1449 rays, 8 angles per
              block, r = 10, lambda = 1e-3) from x = 0 over the first 12 blocks
              of its schedule (synth.schedule(90, ., 3002)): the window is full
              (11 blocks, 127,512 rows) from step 11 on.  Stores x after steps
              11 and 12 (float32: the storage rounding, 6e-8 relative, is far
              below the tests' 1e-5) and the norms of every step.
  c4_slices   the 512-slice 512^2 volume (360 angles x 725 rays, 4 angles per
              block, r = 8, lambda = 1e-3): three slices, each its own 2D
              problem with the shared schedule (synth.schedule(90, ., 3004)),
              10 steps from x = 0 (window full, 26,100 rows, from step 9 on).
              Stores each slice's x after steps 9 and 10 (its data come from
              synth.volume_slice).

  c4m_slices  the mixed batch (360 angles, 4 angles per block, r = 8,
              lambda = 1e-3, schedule synth.schedule(90, ., 3004)): one slice
              of each size group -- slice 20 of the 64 256^2 slices, 13 of
              the 32 512^2 slices, 3 of the 8 1024^2 slices, each its own 2D
              problem (synth.volume_slice of that group's volume) -- 10 steps
              from x = 0 (window full from step 9 on).  Stores x after steps
              9 and 10.
  chol_cap    the explicit-Gram path at its size cap: a 362^2 image, 64
              angles x 512 rays (custom detector; 511 would be the default),
              2 angles per block, r = 7, lambda = 1e-2, so the full window
              has p = 8 x 2 x 512 = 8192 rows; 9 steps of dense Cholesky from
              x = 0 (schedule synth.schedule(32, ., 3101)).  Stores x after
              steps 8 and 9.
  cnn_256     the warm-start network at its deployed size: 4 levels,
              channels 32/64/128/256 on 256^2 images, seeded parameters
              (cnn_params), two inputs u = the data back-projection of the
              first 4 sampled blocks of the 256^2 warm-start workload (test
              seeds 20000 and 20001), computed by the oracle's projector.
              Stores u, the targets (x_true), the forward output x0 and the
              loss under bf16 storage (the oracle's store hook rounds where
              the kernels store bf16; conv weights rounded to bf16), the full
              gradient of every tensor of at most 20,000 entries, and for the
              larger ones 4,096 entries at seeded positions plus the norm.

  c1_epochs   the 64^2 workload (90 angles x 91 rays, one angle per block,
              r = 5, lambda = 1e-2) over its 20 epochs of the random-cyclic
              schedule (oracle.sampler.schedule(90, 20, 3001)) from x = 0,
              twice: in float64, and with the bf16 storage model of the
              precision variant (b and the image read by the residual rounded
              to bf16, nearest even).  Stores the schedule, x after every
              epoch (float32) and the errors vs x_true.

usage: python tests/golden/make_goldens.py [c2_window] [c4_slices] [c4m_slices] [chol_cap]
                                          [cnn_256] [c1_epochs]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import cnn as ocnn  # noqa: E402
from oracle import sampler  # noqa: E402
from oracle import slimls, system  # noqa: E402

CG_TOL = 1e-12
C4_SLICES = (160, 256, 352)


def _run(name, T, sched, keep, steps):
    out = {"step_norm": [], "x_norm": [], "err_norm": [], "cg_iters": [], "blocks": []}
    t0 = time.time()
    for k in range(1, steps + 1):
        beta = int(sched[k - 1])
        rec = T.step(beta)
        out["step_norm"].append(rec.step_norm)
        out["x_norm"].append(rec.x_norm)
        out["err_norm"].append(rec.err_norm)
        out["cg_iters"].append(rec.cg_iters)
        out["blocks"].append(beta)
        if k in keep:
            out[f"x{k}"] = T.x.astype(np.float32)
        print(f"{name}: step {k} block {beta} cg {rec.cg_iters} "
              f"rho {rec.step_norm / rec.x_norm:.3e} {time.time() - t0:.0f} s", flush=True)
    return out


def c2_window():
    cfg = synth.get_config("c2")
    N, na, g, r, lam = cfg["N"], cfg["n_angles"], cfg["g"], cfg["r"], cfg["lam"]
    x_true, b, _ = synth.make_slice_problem(N, na, cfg["n_ellipses"], cfg["noise"],
                                            cfg["phantom_seed"], cfg["noise_seed"])
    sched = synth.schedule(na // g, 1, cfg["schedule_seed"])
    T = slimls.Tomo(system.Projector(N, na), b, g, r, lam, x_true=x_true, chol_max_p=0,
                    cg_tol=CG_TOL)
    out = _run("c2_window", T, sched, (r + 1, r + 2), r + 2)
    np.savez_compressed(os.path.join(HERE, "c2_window.npz"), N=N, n_angles=na, g=g, r=r,
                        lam=lam, cg_tol=CG_TOL, schedule_seed=cfg["schedule_seed"],
                        **{k: np.asarray(v) for k, v in out.items()})


def c4_slices():
    cfg = synth.get_config("c4")
    N, B, na, g, r, lam = cfg["N"], cfg["n_slices"], cfg["n_angles"], cfg["g"], cfg["r"], cfg["lam"]
    sched = synth.schedule(na // g, 1, cfg["schedule_seed"])
    P = system.Projector(N, na)
    store = {}
    for j, k in enumerate(C4_SLICES):
        x_true, b = synth.volume_slice(N, B, k, na, cfg["n_ellipsoids"], cfg["noise"],
                                       cfg["phantom_seed"], cfg["noise_seed"])
        T = slimls.Tomo(P, b, g, r, lam, x_true=x_true, chol_max_p=0, cg_tol=CG_TOL)
        out = _run(f"c4_slices[{k}]", T, sched, (r + 1, r + 2), r + 2)
        for key, v in out.items():
            store[f"s{j}_{key}"] = np.asarray(v)
    np.savez_compressed(os.path.join(HERE, "c4_slices.npz"), N=N, n_slices=B, n_angles=na, g=g,
                        r=r, lam=lam, cg_tol=CG_TOL, slices=np.asarray(C4_SLICES),
                        schedule_seed=cfg["schedule_seed"], **store)


C4M_PICKS = ((256, 64, 20), (512, 32, 13), (1024, 8, 3))


def c4m_slices():
    cfg = synth.get_config("c4m")
    na, g, r, lam = cfg["n_angles"], cfg["g"], cfg["r"], cfg["lam"]
    sched = synth.schedule(na // g, 1, cfg["schedule_seed"])
    store = {}
    for j, (N, B, k) in enumerate(C4M_PICKS):
        x_true, b = synth.volume_slice(N, B, k, na, cfg["n_ellipsoids"], cfg["noise"],
                                       cfg["phantom_seed"], cfg["noise_seed"])
        T = slimls.Tomo(system.Projector(N, na), b, g, r, lam, x_true=x_true, chol_max_p=0,
                        cg_tol=CG_TOL)
        out = _run(f"c4m_slices[{N}]", T, sched, (r + 1, r + 2), r + 2)
        for key, v in out.items():
            store[f"s{j}_{key}"] = np.asarray(v)
    np.savez_compressed(os.path.join(HERE, "c4m_slices.npz"), n_angles=na, g=g, r=r, lam=lam,
                        cg_tol=CG_TOL, picks=np.asarray(C4M_PICKS),
                        schedule_seed=cfg["schedule_seed"], **store)


CHOL_CAP = dict(N=362, n_angles=64, R=512, g=2, r=7, lam=1e-2, n_ellipses=10, noise=0.01,
                phantom_seed=3102, noise_seed=3103, schedule_seed=3101)


def chol_cap_problem():
    """(x_true[N, N], b[n_angles, R]) of the Cholesky size-cap case."""
    c = CHOL_CAP
    theta, s, _ = synth.scan_geometry(c["N"], c["n_angles"], c["R"])
    ells = synth.random_ellipses(c["n_ellipses"], c["phantom_seed"])
    clean = synth.analytic_sinogram(ells, theta, s)
    return synth.rasterize(ells, c["N"]), synth.add_noise(clean, c["noise"], c["noise_seed"])


def chol_cap():
    c = CHOL_CAP
    x_true, b = chol_cap_problem()
    sched = synth.schedule(c["n_angles"] // c["g"], 1, c["schedule_seed"])
    T = slimls.Tomo(system.Projector(c["N"], c["n_angles"], R=c["R"]), b, c["g"], c["r"],
                    c["lam"], x_true=x_true, chol_max_p=8192)
    out = _run("chol_cap", T, sched, (c["r"] + 1, c["r"] + 2), c["r"] + 2)
    np.savez_compressed(os.path.join(HERE, "chol_cap.npz"), **c,
                        **{k: np.asarray(v) for k, v in out.items()})


CNN_CHANNELS = (32, 64, 128, 256)
CNN_SEEDS = (20000, 20001)
CNN_PARAM_SEED = 4242
CNN_FULL_MAX = 20000
CNN_SAMPLES = 4096


def cnn_params(seed=CNN_PARAM_SEED, channels=CNN_CHANNELS):
    """Seeded float32 parameters of the warm-start network: He-normal conv
    weights (ocnn.init_params), biases 0.05 N(0, 1), head bias 0.1, cu 0.8."""
    rng = np.random.default_rng(seed + 1)
    p = ocnn.init_params(channels, seed)
    for k in sorted(p):
        if k.endswith(".b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    p["head.b"] = np.array([0.1])
    p["head.cu"] = np.array([0.8])
    return {k: v.astype(np.float32) for k, v in p.items()}


def cnn_sample_positions(name, size):
    """The seeded entries of a large gradient tensor that are stored."""
    seed = sum(ord(ch) for ch in name)
    return np.sort(np.random.default_rng(seed).choice(size, CNN_SAMPLES, replace=False))


def cnn_256():
    cfg = synth.get_config("c5")
    N, na, g = cfg["N"], cfg["n_angles"], cfg["g"]
    first = [int(beta) * g + a for beta in synth.schedule(na // g, 1, cfg["schedule_seed"])[:4]
             for a in range(g)]
    P = system.Projector(N, na)
    us, ts = [], []
    for sd in CNN_SEEDS:
        x_true, b, _ = synth.make_slice_problem(N, na, cfg["n_ellipses"], cfg["noise"], sd,
                                                sd + 1_000_000)
        us.append(P.back(first, b[first]).reshape(N, N))
        ts.append(x_true)
    u = np.stack(us).astype(np.float32)
    t = np.stack(ts).astype(np.float32)
    in_scale = N / (2.0 * 4)
    p32 = cnn_params()
    p = {k: (slimls.round_bf16(v) if k.endswith(".w") and not k.startswith("head")
             else v.astype(np.float64)) for k, v in p32.items()}
    t0 = time.time()
    x0, _ = ocnn.forward(p, u.astype(np.float64), in_scale, levels=4, store=slimls.round_bf16)
    print(f"cnn_256: forward {time.time() - t0:.0f} s", flush=True)
    loss, grads, _ = ocnn.loss_and_grads(p, u.astype(np.float64), t.astype(np.float64), in_scale,
                                         levels=4, store=slimls.round_bf16)
    print(f"cnn_256: gradients {time.time() - t0:.0f} s", flush=True)
    store = {}
    for k, v in grads.items():
        v = np.asarray(v, np.float64).reshape(-1)
        if v.size <= CNN_FULL_MAX:
            store["g_" + k] = v
        else:
            pos = cnn_sample_positions(k, v.size)
            store["gpos_" + k] = pos
            store["gval_" + k] = v[pos]
            store["gnorm_" + k] = np.linalg.norm(v)
    np.savez_compressed(os.path.join(HERE, "cnn_256.npz"), u=u, target=t, in_scale=in_scale,
                        param_seed=CNN_PARAM_SEED, x0=x0.astype(np.float64), loss=loss, **store)


def c1_epochs():
    cfg = synth.get_config("c1")
    N, na, r, lam, E = cfg["N"], cfg["n_angles"], cfg["r"], cfg["lam"], cfg["epochs"]
    x_true, b, _ = synth.make_slice_problem(N, na, cfg["n_ellipses"], cfg["noise"],
                                            cfg["phantom_seed"], cfg["noise_seed"])
    sched = sampler.schedule(na, E, cfg["schedule_seed"])
    P = system.Projector(N, na)
    runs = {"fp64": slimls.Tomo(P, b, 1, r, lam, x_true=x_true),
            "bf16": slimls.Tomo(P, slimls.round_bf16(b), 1, r, lam, x_true=x_true,
                                x_store=slimls.round_bf16)}
    store = {}
    t0 = time.time()
    for name, T in runs.items():
        xs, errs = [], []
        for k, beta in enumerate(sched, 1):
            rec = T.step(int(beta))
            if k % na == 0:
                xs.append(T.x.astype(np.float32))
                errs.append(rec.err_norm / np.linalg.norm(x_true))
        store[f"x_{name}"] = np.stack(xs)
        store[f"err_{name}"] = np.asarray(errs)
        print(f"c1_epochs[{name}]: {len(xs)} epochs, {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "c1_epochs.npz"), N=N, n_angles=na, r=r, lam=lam,
                        epochs=E, schedule_seed=cfg["schedule_seed"],
                        schedule=np.asarray(sched, np.int32), **store)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c4_slices", "c2_window", "c4m_slices", "chol_cap", "cnn_256",
                             "c1_epochs"]
    for w in which:
        {"c2_window": c2_window, "c4_slices": c4_slices, "c4m_slices": c4m_slices,
         "chol_cap": chol_cap, "cnn_256": cnn_256, "c1_epochs": c1_epochs}[w]()
