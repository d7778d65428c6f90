"""Learned warm start for slimLS: training data from the method itself,
training on the GPU, and the iterations it saves.

Workload: 256 x 256 images, 180 angles x 363 rays, 10 random ellipses, 1%
noise; blocks of one angle, memory r = 5, lambda = 1e-2; one shared block
schedule (seed 3005).  For every sample:

* u = sum_{j<=4} A_{tau_j}^T b_{tau_j} over the first 4 sampled blocks
  (``Slim.data_backprojection``);
* the plain method runs from x0 = 0 to its stop rule (first k >= r+1 with
  ||s_k|| <= 1e-2 ||x_k||, sec. 4.3) or 20 epochs; its iterate there is the
  training target and its error there is the sample's target error e*;
* the plain method's iterations to the target are the steps until its error
  first drops to e*; the warm start's are the steps from x0 = CNN(u) until
  the error first drops to e* (the iteration itself is unchanged: sec. 1
  allows any x0, and its updates lie in R(A^T)).

Every sample of a chunk runs as one batch of slices sharing A (one context
with n_slices = chunk size), so the Gram factorisation is shared.  The
network is the U-Net of ``include/slim_cnn.h``, trained with Adam on the
mean squared error to the targets by the library's own kernels.

Run ``python -m paper_1912_07962_amd.warmstart --help`` for the command line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np
import torch

import synth

from .slim import Cnn, Slim, SlimError

CHANNELS = (32, 64, 128, 256)
N_FIRST = 4          # blocks whose back-projection feeds the network
RHO_TOL = 1e-2       # stop rule tolerance


def config():
    return synth.get_config("c5")


def in_scale(cfg=None) -> float:
    """Input scale of the network: u sums N_FIRST back-projections whose
    weights are O(h) = O(2/N), so N / (2 N_FIRST) makes uh O(intensity)."""
    cfg = config() if cfg is None else cfg
    return cfg["N"] / (2.0 * N_FIRST)


def _sample(args):
    seed, N, n_angles, n_ellipses, noise = args
    x, b, _ = synth.make_slice_problem(N, n_angles, n_ellipses, noise, seed, seed + 1_000_000)
    return x, b


def make_samples(seeds, workers: int = 8, cfg=None):
    """(x_true [n,N,N], b [n,n_angles,R]) float32 for the given seeds
    (phantom seed s, noise seed s + 1e6)."""
    cfg = config() if cfg is None else cfg
    jobs = [(int(s), cfg["N"], cfg["n_angles"], cfg["n_ellipses"], cfg["noise"]) for s in seeds]
    if workers > 1 and len(jobs) > 8:
        with Pool(workers) as pool:
            out = pool.map(_sample, jobs, chunksize=max(1, len(jobs) // (4 * workers)))
    else:
        out = [_sample(j) for j in jobs]
    x = np.stack([o[0] for o in out]).astype(np.float32)
    b = np.stack([o[1] for o in out]).astype(np.float32)
    return x, b


def schedule(cfg=None):
    cfg = config() if cfg is None else cfg
    M = cfg["n_angles"] // cfg["g"]
    return synth.schedule(M, cfg["epochs"], cfg["schedule_seed"])


def first_angles(cfg=None):
    cfg = config() if cfg is None else cfg
    g = cfg["g"]
    return [int(beta) * g + a for beta in schedule(cfg)[:N_FIRST] for a in range(g)]


def _context(cfg, B):
    return Slim(cfg["N"], cfg["n_angles"], r=cfg["r"], lam=cfg["lam"], n_slices=B,
                angles_per_block=cfg["g"], gram_mode="chol")


def run_chunk(b, x_true, cfg, x0=None, e_star=None, target_steps=0, device="cuda"):
    """One batch of slices through the method.

    Without e_star (plain mode, x0 = 0): runs to every slice's stop rule and
    returns u, the targets (x at each slice's stop step, or after
    target_steps steps if that is > 0), e*, the stop step, the first step at
    which the error is <= e* and the mean error after every step.  With e_star (warm mode, x0
    given): runs until every slice's error is <= its e* and returns the first
    such step per slice.  Both cap at cfg["epochs"] epochs."""
    B, N = b.shape[0], cfg["N"]
    g, r = cfg["g"], cfg["r"]
    sched = schedule(cfg)
    s = _context(cfg, B)
    bd = torch.as_tensor(b, device=device)
    xt = torch.as_tensor(x_true, device=device)
    x = torch.zeros((B, N, N), dtype=torch.float32, device=device)
    if x0 is not None:
        x.copy_(x0)
    s.set_data(bd, x, xt)
    nrm = np.linalg.norm(x_true.reshape(B, -1).astype(np.float64), axis=1)
    nrm[nrm == 0] = 1.0
    out = {}
    if e_star is None:
        out["u"] = s.data_backprojection(first_angles(cfg)).clone()
        target = torch.zeros_like(x)
        stop = np.zeros(B, dtype=np.int64)
        errs = []
        done = np.zeros(B, dtype=bool)
    else:
        reach = np.zeros(B, dtype=np.int64)
        e0 = torch.linalg.vector_norm((x - xt).reshape(B, -1), dim=1).double().cpu().numpy() / nrm
        done = e0 <= e_star                     # x0 itself is within the target: 0 steps
    k = 0
    for beta in sched:
        s.step(list(range(int(beta) * g, int(beta) * g + g)))
        k += 1
        nr = s.slice_norms()
        err = nr[:, 2] / nrm
        if e_star is None:
            errs.append(err)
            rule = (k >= r + 1) & (nr[:, 0] <= RHO_TOL * nr[:, 1]) & ~done
            for i in np.nonzero(rule)[0]:
                if target_steps <= 0:
                    target[i].copy_(x[i])
                stop[i] = k
            done |= rule
            if target_steps > 0:
                if k == target_steps:
                    target.copy_(x)
                if k < target_steps:
                    continue
        else:
            hit = (err <= e_star) & ~done
            reach[hit] = k
            done |= hit
        if done.all():
            break
    if e_star is None:
        for i in np.nonzero(~done)[0]:          # epoch cap: the last iterate
            if target_steps <= 0:
                target[i].copy_(x[i])
            stop[i] = k
        errs = np.array(errs)
        es = errs[stop - 1, np.arange(B)]
        first = np.array([int(np.argmax(errs[:, i] <= es[i])) + 1 for i in range(B)])
        out.update(target=target, e_star=es, stop=stop, first=first, curve=errs.mean(axis=1))
    else:
        reach[~done] = k + 1                    # not reached within the cap
        out["reach"] = reach
        out["reached"] = done
    s.close()
    return out


def plain_data(b, x_true, cfg, chunk=512, target_steps=0):
    """Plain runs over all samples in chunks (see run_chunk)."""
    parts = [run_chunk(b[i:i + chunk], x_true[i:i + chunk], cfg, target_steps=target_steps)
             for i in range(0, b.shape[0], chunk)]
    L = min(len(p["curve"]) for p in parts)
    return {"u": torch.cat([p["u"] for p in parts]),
            "target": torch.cat([p["target"] for p in parts]),
            "e_star": np.concatenate([p["e_star"] for p in parts]),
            "stop": np.concatenate([p["stop"] for p in parts]),
            "first": np.concatenate([p["first"] for p in parts]),
            "curve": np.mean([p["curve"][:L] for p in parts], axis=0)}


def train(net: Cnn, u, target, epochs: int, batch: int, lr: float, seed: int = 0, log=None,
          lr_final: float | None = None):
    """Adam on mean((net(u) - target)^2), the step size decaying linearly
    from lr to lr_final over the epochs; returns the mean loss per epoch."""
    n = u.shape[0]
    rng = np.random.default_rng(seed)
    lr_final = lr if lr_final is None else lr_final
    hist = []
    for ep in range(epochs):
        lr_ep = lr + (lr_final - lr) * (ep / max(epochs - 1, 1))
        order = rng.permutation(n)
        tot, cnt = 0.0, 0
        for i in range(0, n - batch + 1, batch):
            idx = torch.as_tensor(order[i:i + batch], device=u.device)
            loss, _ = net.loss_grad(u.index_select(0, idx).contiguous(),
                                    target.index_select(0, idx).contiguous())
            net.adam(lr_ep)
            tot += loss
            cnt += 1
        hist.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep + 1}: loss {hist[-1]:.4e}")
    return hist


def warm_start(net: Cnn, u, batch: int):
    """x0 = net(u) in batches."""
    x0 = torch.empty_like(u)
    for i in range(0, u.shape[0], batch):
        net.forward(u[i:i + batch].contiguous(), x0[i:i + batch])
    return x0


def warm_steps(b, x_true, x0, e_star, cfg, chunk=512):
    """Steps from x0 until each slice's error is <= its e*."""
    reach, ok = [], []
    for i in range(0, b.shape[0], chunk):
        o = run_chunk(b[i:i + chunk], x_true[i:i + chunk], cfg, x0=x0[i:i + chunk],
                      e_star=e_star[i:i + chunk])
        reach.append(o["reach"])
        ok.append(o["reached"])
    return np.concatenate(reach), np.concatenate(ok)


def main(argv=None):
    ap = argparse.ArgumentParser(description="train and evaluate the slimLS warm start")
    ap.add_argument("--train", type=int, default=10000, help="training samples")
    ap.add_argument("--test", type=int, default=1000, help="test samples")
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=1e-4)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--chunk", type=int, default=512)
    ap.add_argument("--seed", type=int, default=0, help="initialisation and shuffling seed")
    ap.add_argument("--target-steps", type=int, default=180,
                    help="train on the plain iterate after this many steps (0: at the stop "
                         "rule; default one epoch)")
    ap.add_argument("--save", default=None, help="write the trained parameters (.npy)")
    ap.add_argument("--json", default=None, help="write the summary here")
    a = ap.parse_args(argv)
    cfg = config()

    def log(msg):
        print(f"warmstart: {msg}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    tr = np.arange(cfg["train_seeds"][0], cfg["train_seeds"][0] + a.train)
    te = np.arange(cfg["test_seeds"][0], cfg["test_seeds"][0] + a.test)
    xtr, btr = make_samples(tr, a.workers, cfg)
    xte, bte = make_samples(te, a.workers, cfg)
    log(f"{a.train} + {a.test} samples in {time.perf_counter() - t0:.1f} s")
    t1 = time.perf_counter()
    dtr = plain_data(btr, xtr, cfg, a.chunk, a.target_steps)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t1
    log(f"plain targets in {t_gen:.1f} s, mean stop step {dtr['stop'].mean():.1f}")
    dte = plain_data(bte, xte, cfg, a.chunk)

    net = Cnn(cfg["N"], CHANNELS, max_batch=max(a.batch, 16), in_scale=in_scale(cfg))
    net.set_params(init_params(CHANNELS, a.seed))
    t2 = time.perf_counter()
    hist = train(net, dtr["u"], dtr["target"], a.epochs, a.batch, a.lr, seed=a.seed, log=log,
                 lr_final=a.lr_final)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t2
    summary = evaluate(net, bte, xte, dte, cfg, a.chunk)
    curve = dtr["curve"]
    xt = torch.as_tensor(xtr, device="cuda").reshape(a.train, -1)
    t_err = torch.linalg.vector_norm(dtr["target"].reshape(a.train, -1) - xt, dim=1)
    summary.update(plain_err_curve={k: float(curve[k - 1])
                                    for k in (1, 4, 10, 20, 34, 60, 90, 180, 360, 900)
                                    if k <= len(curve)},
                   target_steps=a.target_steps,
                   target_rel_err=float((t_err / torch.linalg.vector_norm(xt, dim=1)).mean()),
                   train_samples=a.train, test_samples=a.test, epochs=a.epochs, batch=a.batch,
                   lr=a.lr, lr_final=a.lr_final, loss_per_epoch=hist, train_s=t_train,
                   targets_s=t_gen, train_samples_per_s=a.epochs * a.train / t_train,
                   train_tflops=3.0 * net.forward_flops() * a.epochs * a.train / t_train / 1e12)
    log(json.dumps(summary))
    if a.save:
        np.save(a.save, net.get_params())
    if a.json:
        with open(a.json, "w") as f:
            json.dump(summary, f)
    return summary


def init_params(channels=CHANNELS, seed: int = 0) -> np.ndarray:
    """Packed initial parameters: He-normal conv weights (std sqrt(2/(9 Cin))),
    zero biases, head weights N(0, 0.01/c_1), bh = 0, cu = 1 (so x0 starts as
    the scaled back-projection plus a small learned correction)."""
    from .slim import cnn_layout
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in cnn_layout(channels):
        if name == "head.cu":
            v = np.ones(shape)
        elif name == "head.w":
            v = rng.standard_normal(shape) * 0.1 / np.sqrt(shape[0])
        elif name.endswith(".w"):
            v = rng.standard_normal(shape) * np.sqrt(2.0 / (9 * shape[3]))
        else:
            v = np.zeros(shape)
        parts.append(v.reshape(-1))
    return np.concatenate(parts).astype(np.float32)


def null_space_floor(x0, x_true, cfg, lam: float = 1e-6, tol: float = 1e-6,
                     max_iter: int = 3000):
    """Error floor of a start x0: slimLS updates lie in R(A^T) (sec. 1), so
    the component of x0 - x_true in the null space of A (all angles) is never
    removed.  One step of the library with every angle in one block, b = 0
    and damping lam turns d = x0 - x_true into
        d - A^T (A A^T + lam I)^{-1} A d = lam (A^T A + lam I)^{-1} d,
    which is the null-space component of d plus what remains of its range
    component after the factors lam / (sigma^2 + lam); its norm bounds the
    floor from above and reaches it as lam -> 0 (CG to tol, at most max_iter
    iterations, the reached residual reported).  Returns per sample
    ||.|| / ||x_true|| for x0 (a tensor [n, N, N] on the GPU or None) and
    for x0 = 0, with the CG's iterations and residual."""
    N, na = cfg["N"], cfg["n_angles"]
    xt = torch.as_tensor(x_true, dtype=torch.float32, device="cuda").reshape(-1, N, N)
    n = xt.shape[0]
    s = Slim(N, na, r=0, lam=lam, n_slices=n, angles_per_block=na, gram_mode="pcg",
             pcg_tol=tol, pcg_max_iter=max_iter)
    b0 = torch.zeros((n, na, s.R), dtype=torch.float32, device="cuda")
    nrm = torch.linalg.vector_norm(xt.reshape(n, -1), dim=1).double().cpu().numpy()
    out = {"lambda": lam}
    for name, d in (("x0", None if x0 is None else x0 - xt), ("zero", -xt)):
        if d is None:
            continue
        x = d.contiguous().clone()
        s.set_data(b0, x)
        try:
            info = s.step(list(range(na)))
        except SlimError as e:          # the cap reached: still an upper bound
            if e.status != 5:
                raise
            info = {"pcg_iters": max_iter, "pcg_relres": float("nan")}
        rem = torch.linalg.vector_norm(x.reshape(n, -1), dim=1).double().cpu().numpy()
        out[name] = {"rel_floor": (rem / nrm).tolist(), "cg_iters": info["pcg_iters"],
                     "cg_relres": info["pcg_relres"]}
    s.close()
    return out


def evaluate(net: Cnn, b, x_true, plain, cfg, chunk=512):
    """Iterations to each test sample's e* from x0 = 0 (plain), from the
    scaled back-projection x0 = alpha u (alpha fitted by least squares to the
    plain targets) and from x0 = net(u)."""
    u, tgt = plain["u"], plain["target"]
    alpha = float((u * tgt).sum() / (u * u).sum())
    x_lin = alpha * u
    r_lin, ok_lin = warm_steps(b, x_true, x_lin, plain["e_star"], cfg, chunk)
    x0 = warm_start(net, u, net.max_batch)
    r_net, ok_net = warm_steps(b, x_true, x0, plain["e_star"], cfg, chunk)
    xt = torch.as_tensor(x_true, device=u.device)
    n = torch.linalg.vector_norm((xt).reshape(xt.shape[0], -1), dim=1)

    def rel(x):
        return float((torch.linalg.vector_norm((x - xt).reshape(xt.shape[0], -1), dim=1) / n).mean())

    first = plain["first"]
    return {"plain_steps_mean": float(first.mean()), "plain_stop_mean": float(plain["stop"].mean()),
            "e_star_mean": float(plain["e_star"].mean()),
            "scaled_u_steps_mean": float(r_lin.mean()), "scaled_u_reached": float(ok_lin.mean()),
            "net_steps_mean": float(r_net.mean()), "net_reached": float(ok_net.mean()),
            "net_fewer_steps_frac": float((r_net < first).mean()),
            "net_steps_saved_mean": float((first - r_net).mean()),
            "x0_rel_err_net": rel(x0), "x0_rel_err_scaled_u": rel(x_lin), "alpha": alpha}


if __name__ == "__main__":
    main()
