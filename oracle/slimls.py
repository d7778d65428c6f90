"""The slimLS iteration in float64 (test infrastructure only).

Paper: eq. (ram)   x_k = x_{k-1} - B_k A_k^T (A_k x_{k-1} - b_k)
       eq. (B_k)   B_k = (alpha_k^{-1} C_k + M_k^T M_k)^{-1},  M_k = [A_{k-r}; ...; A_k]
with C_k = I and alpha_k = 1/lam (sec. 1: C_k = I and r = 0 give damped block
Kaczmarz, eq. (dbK)).  alpha_k is constant, or ramped up over the first r+1
steps as in sec. 4.2 (alpha_k = k alpha / (r+1), used in sec. 4.3), which in
terms of lam is lam_k = lam (r+1) / k for k <= r+1; ``lam`` may also be
changed between steps (a caller-driven decay of alpha_k, end of sec. 3).
slimTik (sec. 2, eq. (slimTik)) with L = I is the same iteration with a
Tikhonov term; ``tik_mu`` states the reading of its shift.  Blocks with negative index are empty,
so M_k grows over the first r steps (sec. 1).

Three algebraically equal ways to form the step s_k = x_{k-1} - x_k:

* ``step_primal``   -- eq. (B_k) literally: solve (lam I + M^T M) s = A_k^T res
                       (dense n x n; tiny problems only);
* ``step_dual``     -- the Gram (push-through) form used for parity:
                       (lam I + M^T M)^{-1} M^T = M^T (lam I + M M^T)^{-1} and
                       A_k^T res = M^T [0; ...; 0; res], so
                       s = M^T z with (M M^T + lam I) z = [0; ...; 0; res];
                       the p x p system is solved by dense Cholesky (LAPACK)
                       for p <= chol_max_p, else by plain CG to a relative
                       residual of cg_tol;
* ``step_woodbury`` -- Sherman-Morrison-Woodbury (sec. 2 remark on exact
                       solves): s = (g - M^T (lam I + M M^T)^{-1} M g) / lam,
                       g = A_k^T res.

Pins (tests/test_oracle_*.py): the three forms agree; r = 0 is damped block
Kaczmarz (eq. dbK); lam -> 0 with one row per block is Kaczmarz (eq. Kacz);
the ramp's first steps against closed forms for one- and two-row windows
(Sherman-Morrison, Cramer's rule); slimTik equals plain slimLS on the stacked
blocks [A_k; (tik/sqrt(M)) I] and, with full memory, reaches the Tikhonov
solution of eq. (TLS1) after one epoch;
full memory over one epoch gives the Tikhonov solution at every k (the
induction of App. A with the damped Hessian); the residual identity after a
step; consistent data is a fixed point; Theorem 3.1(i) in expectation.
Full reconstructions at the workload sizes have no printed values: parity
beyond these pins is unpinned.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def _stack(mats):
    if any(sp.issparse(m) for m in mats):
        return sp.vstack([sp.csr_matrix(m) for m in mats], format="csr")
    return np.vstack(mats)


def _dense(a):
    return a.toarray() if sp.issparse(a) else np.asarray(a)


def cg(apply, rhs: np.ndarray, tol: float, max_iter: int = 100000):
    """Plain conjugate gradients (Hestenes-Stiefel) for an SPD operator.

    Stops when ||rhs - A z|| <= tol * ||rhs||.  Returns (z, iterations, relres)."""
    z = np.zeros_like(rhs)
    r = rhs.copy()
    p = r.copy()
    rr = r @ r
    nb = np.sqrt(rhs @ rhs)
    if nb == 0.0:
        return z, 0, 0.0
    it = 0
    while np.sqrt(rr) > tol * nb and it < max_iter:
        q = apply(p)
        a = rr / (p @ q)
        z += a * p
        r -= a * q
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return z, it, float(np.sqrt(rr) / nb)


def gram(window, lam: float) -> np.ndarray:
    """G = M M^T + lam I for M = vstack(window), dense float64."""
    M = _stack(window)
    G = _dense(M @ M.T).astype(np.float64)
    G[np.diag_indices_from(G)] += lam
    return G


def step_dual(window, res, lam, chol_max_p=8000, cg_tol=1e-12):
    """Returns (s, z, info).  ``window`` lists the blocks A_{k-r}..A_k, oldest first."""
    M = _stack(window)
    p = M.shape[0]
    e = np.zeros(p)
    e[p - res.size:] = res
    if p <= chol_max_p:
        G = _dense(M @ M.T).astype(np.float64)
        G[np.diag_indices_from(G)] += lam
        z = sla.cho_solve(sla.cho_factor(G, lower=True), e)
        info = {"mode": "chol", "iters": 0, "relres": 0.0}
    else:
        z, it, rel = cg(lambda v: M @ (M.T @ v) + lam * v, e, cg_tol)
        info = {"mode": "cg", "iters": it, "relres": rel}
    s = M.T @ z
    return np.asarray(s).reshape(-1), z, info


def step_primal(window, res, lam):
    """s = (lam I + M^T M)^{-1} A_k^T res, eq. (B_k) with C_k = I, alpha = 1/lam."""
    M = _dense(_stack(window))
    Ak = _dense(window[-1])
    H = M.T @ M
    H[np.diag_indices_from(H)] += lam
    return np.linalg.solve(H, Ak.T @ res)


def step_woodbury(window, res, lam):
    """s = (g - M^T (lam I + M M^T)^{-1} M g) / lam with g = A_k^T res."""
    M = _dense(_stack(window))
    g = _dense(window[-1]).T @ res
    G = M @ M.T
    G[np.diag_indices_from(G)] += lam
    return (g - M.T @ np.linalg.solve(G, M @ g)) / lam


# slimTik (sec. 2, eq. (slimTik)) with L = I: slimLS on the stacked problem
# [A; lam_t I] x ~ [b; 0] (eq. (TLS1)) whose block k is [A_k; (lam_t/sqrt(M)) I].
# With C_k = I the step is
#   s = (mu I + M^T M)^{-1} (A_k^T res + tau x_{k-1}),  tau = lam_t^2 / M,
#   mu = 1/alpha_k + W tau,
# W the number of blocks in the window (each stacked block adds tau I to
# M^T M).  The printed equation has r lam_t^2 / M; counting the window's
# blocks gives W = r + 1 once the window is full (the reading used here).

def tik_mu(lam: float, tik: float, n_blocks: int, W: int) -> tuple[float, float]:
    """(mu, tau) of the slimTik step for damping lam = 1/alpha_k and window W."""
    tau = tik * tik / n_blocks
    return lam + W * tau, tau


def step_tik_primal(window, res, x, lam, tik, n_blocks):
    """eq. (slimTik) literally (L = I): dense n x n solve."""
    M = _dense(_stack(window))
    mu, tau = tik_mu(lam, tik, n_blocks, len(window))
    H = M.T @ M
    H[np.diag_indices_from(H)] += mu
    return np.linalg.solve(H, _dense(window[-1]).T @ res + tau * x)


def step_tik_dual(window, res, x, lam, tik, n_blocks, chol_max_p=8000, cg_tol=1e-12):
    """The same step through the p x p Gram system: by Woodbury
    (mu I + M^T M)^{-1} = (I - M^T (mu I + M M^T)^{-1} M) / mu, so with
    c = tau / mu,  s = M^T z + c x  and  (M M^T + mu I) z = [0; ...; 0; res] - c M x."""
    M = _stack(window)
    mu, tau = tik_mu(lam, tik, n_blocks, len(window))
    c = tau / mu
    p = M.shape[0]
    e = -c * np.asarray(M @ x).reshape(-1)
    e[p - res.size:] += res
    if p <= chol_max_p:
        G = _dense(M @ M.T).astype(np.float64)
        G[np.diag_indices_from(G)] += mu
        z = sla.cho_solve(sla.cho_factor(G, lower=True), e)
        info = {"mode": "chol", "iters": 0, "relres": 0.0}
    else:
        z, it, rel = cg(lambda v: M @ (M.T @ v) + mu * v, e, cg_tol)
        info = {"mode": "cg", "iters": it, "relres": rel}
    s = np.asarray(M.T @ z).reshape(-1) + c * x
    return s, z, info


@dataclass
class StepRecord:
    k: int
    block: int
    step_norm: float
    x_norm: float
    err_norm: float
    mode: str = "chol"
    cg_iters: int = 0


@dataclass
class SlimLS:
    """Iterates of slimLS for a problem given block-wise.

    block_rows(beta) -> rows A_beta (sparse or dense), block_data(beta) -> b_beta.
    """
    block_rows: callable
    block_data: callable
    r: int
    lam: float
    x: np.ndarray
    x_true: np.ndarray | None = None
    form: str = "dual"
    chol_max_p: int = 8000
    cg_tol: float = 1e-12
    window: list = field(default_factory=list)     # block ids, oldest first
    k: int = 0
    history: list = field(default_factory=list)
    # x_store(x): the image as stored for the residual A_k x (identity; the
    # bf16-storage variant passes a rounding to bfloat16)
    x_store: callable = None
    # ramp: alpha_k = k alpha / (r+1) for k <= r+1 (sec. 4.2), else alpha
    ramp: bool = False
    # slimTik with L = I (eq. (slimTik)): Tikhonov parameter of eq. (TLS1)
    # (0: plain slimLS) and the number of blocks M
    tik: float = 0.0
    n_blocks: int = 0

    def lam_at(self, k: int) -> float:
        """Damping 1/alpha_k of the k-th step (1-based)."""
        alpha = 1.0 / self.lam
        if self.ramp and k <= self.r + 1:
            alpha = k * alpha / (self.r + 1)
        return 1.0 / alpha

    def step(self, beta: int) -> StepRecord:
        self.window.append(int(beta))
        if len(self.window) > self.r + 1:
            self.window.pop(0)
        mats = [self.block_rows(b) for b in self.window]
        Ak = mats[-1]
        xs = self.x if self.x_store is None else self.x_store(self.x)
        res = np.asarray(Ak @ xs).reshape(-1) - self.block_data(beta)
        info = {"mode": self.form, "iters": 0}
        lam = self.lam_at(self.k + 1)
        if self.tik > 0.0:
            xt = np.asarray(xs, np.float64).reshape(-1)
            if self.form == "dual":
                s, _, info = step_tik_dual(mats, res, xt, lam, self.tik, self.n_blocks,
                                           self.chol_max_p, self.cg_tol)
            else:
                s = step_tik_primal(mats, res, xt, lam, self.tik, self.n_blocks)
        elif self.form == "dual":
            s, _, info = step_dual(mats, res, lam, self.chol_max_p, self.cg_tol)
        elif self.form == "primal":
            s = step_primal(mats, res, lam)
        elif self.form == "woodbury":
            s = step_woodbury(mats, res, lam)
        else:
            raise ValueError(self.form)
        self.x = self.x - s
        self.k += 1
        err = float(np.linalg.norm(self.x - self.x_true)) if self.x_true is not None else float("nan")
        rec = StepRecord(self.k, int(beta), float(np.linalg.norm(s)), float(np.linalg.norm(self.x)),
                         err, info["mode"], info.get("iters", 0))
        self.history.append(rec)
        return rec


def round_bf16(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) and return as float64.

    bfloat16 keeps the upper 16 bits of an IEEE float32: the float32 value is
    rounded to 8 significand bits by adding 0x7FFF plus the lowest kept bit
    and truncating."""
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def stop_index(history, r: int, tol: float):
    """First step k >= r+1 with ||s_k|| / ||x_k|| <= tol (1-based), or None."""
    for rec in history:
        if rec.k >= r + 1 and rec.x_norm > 0 and rec.step_norm / rec.x_norm <= tol:
            return rec.k
    return None


class Tomo:
    """slimLS on a 2D parallel-beam problem: block beta = angles g*beta .. g*beta+g-1."""

    def __init__(self, projector, b: np.ndarray, g: int, r: int, lam: float,
                 x0: np.ndarray | None = None, x_true: np.ndarray | None = None,
                 chol_max_p: int = 8000, cg_tol: float = 1e-12, form: str = "dual",
                 x_store=None, ramp: bool = False, tik: float = 0.0):
        self.P = projector
        self.g = g
        self.n_blocks = projector.n_angles // g
        self.b = np.asarray(b, np.float64).reshape(projector.n_angles, projector.R)
        x0 = np.zeros(projector.n) if x0 is None else np.asarray(x0, np.float64).reshape(-1)
        xt = None if x_true is None else np.asarray(x_true, np.float64).reshape(-1)
        self.it = SlimLS(self.rows, self.data, r, lam, x0.copy(), xt, form, chol_max_p, cg_tol,
                         x_store=x_store, ramp=ramp, tik=tik, n_blocks=self.n_blocks)

    def angles_of(self, beta: int):
        return list(range(beta * self.g, beta * self.g + self.g))

    def rows(self, beta: int):
        return self.P.rows(self.angles_of(beta))

    def data(self, beta: int):
        return self.b[self.angles_of(beta)].reshape(-1)

    @property
    def x(self):
        return self.it.x

    def step(self, beta: int) -> StepRecord:
        return self.it.step(beta)

    def run(self, sched, tol: float | None = None, epoch_len: int | None = None):
        """Run the schedule; stop at the first k >= r+1 with rho_k <= tol if tol
        is given.  Returns (x at the end, list of x at epoch ends, stop step)."""
        epoch_len = self.n_blocks if epoch_len is None else epoch_len
        snaps = []
        for beta in sched:
            rec = self.step(int(beta))
            if rec.k % epoch_len == 0:
                snaps.append(self.x.copy())
            if tol is not None and stop_index([rec], self.it.r, tol) is not None:
                return self.x.copy(), snaps, rec.k
        return self.x.copy(), snaps, None
