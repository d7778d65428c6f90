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

usage: python tests/golden/make_goldens.py [c2_window] [c4_slices]
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


if __name__ == "__main__":
    which = sys.argv[1:] or ["c4_slices", "c2_window"]
    for w in which:
        {"c2_window": c2_window, "c4_slices": c4_slices}[w]()
