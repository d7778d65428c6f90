"""Pins of the oracle's slimLS iteration (CPU only).

Every pin follows from the paper's definitions or from textbook linear
algebra, not from the oracle's own code path:

* the dual (Gram) step used for parity equals the primal eq. (B_k) solve and
  the Sherman-Morrison-Woodbury form;
* r = 0 is damped block Kaczmarz (sec. 1, eq. dbK); lam -> 0 with one row per
  block is randomized Kaczmarz (eq. Kacz); lam -> 0 with full-row-rank blocks
  is block Kaczmarz with the pseudo-inverse (eq. stochnewt1);
* with memory covering every block and x0 = 0, one epoch without replacement
  gives x_k = (lam I + sum_{i<=k} A_i^T A_i)^{-1} sum_{i<=k} A_i^T b_i for all k
  (App. A's induction with the damped Hessian), hence Tikhonov at k = M;
* after a step, A_k x_k - b_k = lam z_last and A_j x_k = A_j x_{k-1} + lam z_j;
* consistent data is a fixed point; updates stay in R(A^T);
* Theorem 3.1(i): E x_k obeys the exact first-moment recursion, contracts to
  x_hat at rate rho, and Monte Carlo means of the oracle follow it;
  Lemma B.1(iii) bounds ||B_k A_k^T A_k||.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import sampler, slimls, system


def _dense_problem(m=120, n=20, ell=10, seed=0, noise=0.01):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    x_true = np.ones(n)
    clean = A @ x_true
    e = rng.standard_normal(m)
    b = clean + noise * np.linalg.norm(clean) * e / np.linalg.norm(e)
    blocks = [np.arange(i * ell, (i + 1) * ell) for i in range(m // ell)]
    return A, b, x_true, blocks


def _runner(A, b, blocks, r, lam, form="dual", x0=None, x_true=None):
    x0 = np.zeros(A.shape[1]) if x0 is None else x0
    return slimls.SlimLS(lambda beta: A[blocks[beta]], lambda beta: b[blocks[beta]],
                         r, lam, x0.copy(), x_true, form)


@pytest.mark.parametrize("r", [0, 1, 3])
def test_dual_primal_woodbury_agree(r):
    A, b, _, blocks = _dense_problem()
    sched = np.random.default_rng(1).integers(0, len(blocks), 15)
    runs = {f: _runner(A, b, blocks, r, 0.3, f) for f in ("dual", "primal", "woodbury")}
    for beta in sched:
        for it in runs.values():
            it.step(beta)
        np.testing.assert_allclose(runs["dual"].x, runs["primal"].x, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(runs["woodbury"].x, runs["primal"].x, rtol=1e-9, atol=1e-11)


def test_dual_equals_primal_on_tomography():
    N, na = 10, 12
    P = system.Projector(N, na)
    x_true, b, _ = synth.make_slice_problem(N, na, 3, 0.01, 5, 6)
    sched = sampler.schedule(na // 2, 2, 11)
    t_d = slimls.Tomo(P, b, 2, 2, 1e-2, form="dual")
    t_p = slimls.Tomo(P, b, 2, 2, 1e-2, form="primal")
    for beta in sched:
        t_d.step(beta)
        t_p.step(beta)
    np.testing.assert_allclose(t_d.x, t_p.x, rtol=1e-10, atol=1e-12)


def test_r0_is_damped_block_kaczmarz():
    A, b, _, blocks = _dense_problem(seed=3)
    lam = 0.05
    it = _runner(A, b, blocks, 0, lam)
    x = np.zeros(A.shape[1])
    for beta in [3, 7, 1, 1, 0, 11, 5]:
        Ak, bk = A[blocks[beta]], b[blocks[beta]]
        # eq. (dbK) with the residual at x_{k-1}
        x = x - np.linalg.solve(np.eye(A.shape[1]) / (1 / lam) + Ak.T @ Ak, Ak.T @ (Ak @ x - bk))
        it.step(beta)
        np.testing.assert_allclose(it.x, x, rtol=1e-11, atol=1e-13)


def test_single_row_small_lambda_is_kaczmarz():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((30, 8))
    b = rng.standard_normal(30)
    blocks = [np.array([i]) for i in range(30)]
    it = _runner(A, b, blocks, 0, 1e-12)
    x = np.zeros(8)
    for tau in rng.integers(0, 30, 40):
        a = A[tau]
        x = x - (a @ x - b[tau]) / (a @ a) * a     # eq. (Kacz), alpha = 1
        it.step(tau)
    np.testing.assert_allclose(it.x, x, rtol=1e-8, atol=1e-9)


def test_small_lambda_r0_is_block_kaczmarz_pinv():
    A, b, _, blocks = _dense_problem(m=60, n=20, ell=5, seed=8)
    it = _runner(A, b, blocks, 0, 1e-11)
    x = np.zeros(20)
    for beta in [2, 9, 4, 4, 11, 0]:
        Ak = A[blocks[beta]]
        x = x - np.linalg.pinv(Ak) @ (Ak @ x - b[blocks[beta]])   # eq. (stochnewt1)
        it.step(beta)
    np.testing.assert_allclose(it.x, x, rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("kind", ["dense", "tomo"])
def test_full_memory_is_regularised_recursive_ls(kind):
    lam = 0.02
    if kind == "dense":
        A, b, _, blocks = _dense_problem(m=80, n=30, ell=8, seed=9)
        n = 30
    else:
        N, na, g = 12, 16, 2
        P = system.Projector(N, na)
        A = P.full().toarray()
        _, bb, _ = synth.make_slice_problem(N, na, 3, 0.01, 21, 22)
        b = bb.reshape(-1)
        R = P.R
        blocks = [np.arange(beta * g * R, (beta + 1) * g * R) for beta in range(na // g)]
        n = N * N
    M = len(blocks)
    order = sampler.epoch_permutation(M, 0, 123)
    it = _runner(A, b, blocks, M - 1, lam)
    H = lam * np.eye(n)
    rhs = np.zeros(n)
    for beta in order:
        it.step(beta)
        Ak = A[blocks[beta]]
        H += Ak.T @ Ak
        rhs += Ak.T @ b[blocks[beta]]
        np.testing.assert_allclose(it.x, np.linalg.solve(H, rhs), rtol=1e-9, atol=1e-11)
    x_tik = np.linalg.solve(A.T @ A + lam * np.eye(n), A.T @ b)
    np.testing.assert_allclose(it.x, x_tik, rtol=1e-9, atol=1e-11)


def test_post_step_residual_identity():
    N, na, g, r, lam = 14, 18, 3, 2, 1e-2
    P = system.Projector(N, na)
    _, b, _ = synth.make_slice_problem(N, na, 4, 0.01, 31, 32)
    T = slimls.Tomo(P, b, g, r, lam)
    for beta in [1, 4, 0, 5, 2]:
        x_prev = T.x.copy()
        T.it.window.append(beta)
        if len(T.it.window) > r + 1:
            T.it.window.pop(0)
        mats = [T.rows(w) for w in T.it.window]
        res = mats[-1] @ x_prev - T.data(beta)
        s, z, _ = slimls.step_dual(mats, res, lam)
        x_new = x_prev - s
        T.it.x = x_new
        off = 0
        for w, Mw in zip(T.it.window, mats):
            zw = z[off:off + Mw.shape[0]]
            off += Mw.shape[0]
            if w is T.it.window[-1]:
                np.testing.assert_allclose(Mw @ x_new - T.data(w), lam * zw, rtol=1e-10, atol=1e-14)
            else:
                np.testing.assert_allclose(Mw @ x_new, Mw @ x_prev + lam * zw, rtol=1e-10, atol=1e-14)


def test_consistent_data_is_fixed_point_and_updates_in_range():
    N, na = 16, 10     # underdetermined: m = 10*23 = 230 < n = 256
    P = system.Projector(N, na)
    A = P.full()
    x_true = synth.rasterize(synth.random_ellipses(3, 41), N).reshape(-1)
    b = A @ x_true
    T = slimls.Tomo(P, b, 1, 3, 1e-3, x0=x_true)
    for beta in sampler.schedule(na, 2, 5):
        T.step(beta)
    np.testing.assert_allclose(T.x, x_true, rtol=0, atol=1e-12)
    # from x0 = 0 with noisy data every iterate lies in R(A^T)
    rng = np.random.default_rng(2)
    T2 = slimls.Tomo(P, b + 0.01 * rng.standard_normal(b.size), 1, 3, 1e-3)
    for beta in sampler.schedule(na, 2, 6):
        T2.step(beta)
    Ad = A.toarray()
    coef, *_ = np.linalg.lstsq(Ad.T, T2.x, rcond=None)
    np.testing.assert_allclose(Ad.T @ coef, T2.x, rtol=0, atol=1e-9 * np.linalg.norm(T2.x))


def _expectation_pieces(A, b, blocks, alpha):
    n = A.shape[1]
    I = np.eye(n)
    Bs = [alpha * np.linalg.inv(I + alpha * A[i].T @ A[i]) for i in blocks]
    EBA = sum(B @ A[i].T @ A[i] for B, i in zip(Bs, blocks)) / len(blocks)
    EBb = sum(B @ A[i].T @ b[i] for B, i in zip(Bs, blocks)) / len(blocks)
    return Bs, EBA, EBb


def test_theorem_3_1_first_moment():
    # i.i.d. uniform sampling, r = 0, fixed alpha (sec. 3)
    A, b, _, blocks = _dense_problem(m=60, n=8, ell=6, seed=12, noise=0.05)
    alpha = 2.0
    n = A.shape[1]
    Bs, EBA, EBb = _expectation_pieces(A, b, blocks, alpha)
    x_hat = np.linalg.solve(EBA, EBb)                      # eq. (xhat)
    rho = np.linalg.norm(np.eye(n) - EBA, 2)                # ||E B_k / alpha||
    assert rho < 1.0                                        # Lemma B.1(i)
    # Lemma B.1(iii): ||B_k A_k^T A_k|| <= alpha A_max / (1 + alpha A_max)
    Amax = max(np.linalg.eigvalsh(A[i].T @ A[i]).max() for i in blocks)
    for B, i in zip(Bs, blocks):
        assert np.linalg.norm(B @ A[i].T @ A[i], 2) <= alpha * Amax / (1 + alpha * Amax) + 1e-12
    # exact first moment: E x_k = (I - E B A^T A) E x_{k-1} + E B A^T b
    K = 12
    Ex = [np.zeros(n)]
    for _ in range(K):
        Ex.append(Ex[-1] - EBA @ Ex[-1] + EBb)
    for k in range(K + 1):
        assert np.linalg.norm(Ex[k] - x_hat) <= rho ** k * np.linalg.norm(x_hat) * (1 + 1e-10)
    # Monte Carlo mean of the oracle's iterates follows E x_k
    rng = np.random.default_rng(99)
    runs = 600
    xs = np.zeros((runs, n))
    for j in range(runs):
        it = _runner(A, b, blocks, 0, 1.0 / alpha)
        for beta in rng.integers(0, len(blocks), K):
            it.step(beta)
        xs[j] = it.x
    mean = xs.mean(0)
    se = xs.std(0, ddof=1) / np.sqrt(runs)
    assert np.all(np.abs(mean - Ex[K]) <= 4.5 * se + 1e-12)


def test_bias_grows_with_alpha():
    # Lemma 3.2 / fig. (bound): x_hat -> x_LS as alpha -> 0
    A, b, _, blocks = _dense_problem(m=100, n=10, ell=10, seed=13, noise=0.05)
    x_ls = np.linalg.lstsq(A, b, rcond=None)[0]
    diffs = []
    for alpha in (1e-3, 1e-1, 10.0):
        _, EBA, EBb = _expectation_pieces(A, b, blocks, alpha)
        diffs.append(np.linalg.norm(np.linalg.solve(EBA, EBb) - x_ls) / np.linalg.norm(x_ls))
    # the bound of Lemma 3.2 is linear in alpha for small alpha
    assert diffs[0] < 1e-3 and diffs[0] < diffs[1] < diffs[2]


def test_memory_speeds_initial_convergence():
    # sec. 4.1: alpha = 1, 20 iterations, larger r converges faster initially
    A, b, _, blocks = _dense_problem(m=1000, n=100, ell=10, seed=14)
    x_ls = np.linalg.lstsq(A, b, rcond=None)[0]
    med = {}
    for r in (0, 4, 8):
        errs = []
        for run in range(15):
            it = _runner(A, b, blocks, r, 1.0)
            for beta in np.random.default_rng(run).integers(0, 100, 20):
                it.step(beta)
            errs.append(np.linalg.norm(it.x - x_ls) / np.linalg.norm(x_ls))
        med[r] = np.median(errs)
    assert med[0] > med[4] > med[8]


def test_cg_mode_matches_cholesky():
    N, na, g, r, lam = 16, 16, 2, 2, 1e-2
    P = system.Projector(N, na)
    _, b, _ = synth.make_slice_problem(N, na, 4, 0.01, 51, 52)
    t_c = slimls.Tomo(P, b, g, r, lam)
    t_g = slimls.Tomo(P, b, g, r, lam, chol_max_p=0, cg_tol=1e-13)
    for beta in sampler.schedule(na // g, 2, 7):
        t_c.step(beta)
        rec = t_g.step(beta)
        assert rec.mode == "cg"
    np.testing.assert_allclose(t_g.x, t_c.x, rtol=1e-10, atol=1e-12)


def test_stop_rule():
    H = [slimls.StepRecord(k, 0, s, 1.0, 0.0) for k, s in enumerate([1.0, 0.005, 0.5, 0.009, 0.001], 1)]
    assert slimls.stop_index(H, r=2, tol=1e-2) == 4     # k=2 is inside the first r+1 steps


def test_tomo_run_stops_where_stop_index_says():
    # Tomo.run's early termination (sec. 4.3) is the first k >= r+1 with
    # ||s_k|| <= tol ||x_k||: the same step as stop_index over the full history
    N, na, g, r, lam = 24, 30, 1, 3, 1e-2
    P = system.Projector(N, na)
    _, b, _ = synth.make_slice_problem(N, na, 5, 0.01, 61, 62)
    sched = sampler.schedule(na // g, 3, 8)
    full = slimls.Tomo(P, b, g, r, lam)
    full.run(sched)
    for tol in (0.3, 5e-2, 1e-2):
        k_ref = slimls.stop_index(full.it.history, r, tol)
        assert k_ref is not None and k_ref >= r + 1
        T = slimls.Tomo(P, b, g, r, lam)
        x, _, k = T.run(sched, tol=tol)
        assert k == k_ref and len(T.it.history) == k
        np.testing.assert_array_equal(x, T.x)
    # a tolerance never met runs the whole schedule
    T = slimls.Tomo(P, b, g, r, lam)
    assert T.run(sched, tol=1e-12)[2] is None and len(T.it.history) == len(sched)


def test_sparse_block_matches_dense_block():
    N, na = 9, 6
    P = system.Projector(N, na)
    ids = [4, 1]
    dense = system.dense_bruteforce(N, P.R, P.theta[ids])
    assert sp.issparse(P.rows(ids))
    np.testing.assert_allclose(P.rows(ids).toarray(), dense, rtol=1e-13, atol=1e-15)


def test_round_bf16_published_values():
    from oracle.slimls import round_bf16
    # bfloat16 has an 8-bit significand: 1 + 2^-8 is a tie -> even (1.0),
    # 1 + 3*2^-8 is a tie -> even (1 + 2^-6); pi -> 3.140625; 65504 (the
    # largest float16) rounds up to 2^16
    vals = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, np.pi, -np.pi, 65504.0])
    got = round_bf16(vals)
    np.testing.assert_array_equal(got, [1.0, 1.0, 1 + 2.0 ** -6, 3.140625, -3.140625, 65536.0])


def _cramer(G, rhs):
    """Solve G z = rhs by Cramer's rule (determinants; tiny systems only)."""
    d = np.linalg.det(G)
    z = np.empty(len(rhs))
    for i in range(len(rhs)):
        Gi = G.copy()
        Gi[:, i] = rhs
        z[i] = np.linalg.det(Gi) / d
    return z


def test_ramped_damping_first_steps_closed_forms():
    """Ramp of sec. 4.2: alpha_k = k alpha / (r+1) for k <= r+1, then alpha.

    Single-row blocks make each step a tiny Gram system: one row is
    Sherman-Morrison, x_1 = x_0 - a (a x_0 - b) / (1/alpha_1 + |a|^2); two to
    three rows are solved by Cramer's rule on (M M^T + I/alpha_k) z = [0; ...; res]
    with s = M^T z (the push-through identity of eq. (B_k)).  A wrong ramp
    index (k vs k+1, r vs r+1) or a ramp applied to lam instead of alpha
    moves every step below."""
    rng = np.random.default_rng(21)
    A = rng.standard_normal((12, 7))
    b = rng.standard_normal(12)
    blocks = [np.array([i]) for i in range(12)]
    r, lam = 2, 0.4
    alpha = 1.0 / lam
    it = slimls.SlimLS(lambda t: A[blocks[t]], lambda t: b[blocks[t]], r, lam, np.zeros(7),
                       ramp=True)
    plain = _runner(A, b, blocks, r, lam)
    x = np.zeros(7)
    sched = [4, 9, 0, 6, 2]
    for k, tau in enumerate(sched, 1):
        alpha_k = k * alpha / (r + 1) if k <= r + 1 else alpha
        win = sched[max(0, k - 1 - r):k]
        M = A[win]
        res = A[tau] @ x - b[tau]
        if len(win) == 1:
            a = A[tau]
            s = a * res / (1.0 / alpha_k + a @ a)
        else:
            e = np.zeros(len(win))
            e[-1] = res
            s = M.T @ _cramer(M @ M.T + np.eye(len(win)) / alpha_k, e)
        x = x - s
        it.step(tau)
        plain.step(tau)
        np.testing.assert_allclose(it.x, x, rtol=1e-11, atol=1e-13)
        if k == 1:   # the ramp changes the first step (alpha/3 instead of alpha)
            assert np.linalg.norm(plain.x - it.x) > 1e-3 * np.linalg.norm(x)


def test_damping_changed_between_steps():
    """A caller-driven schedule (end of sec. 3: alpha_k constant, then
    decaying): each r = 0 single-row step is Sherman-Morrison with the
    lam = 1/alpha_k in force."""
    rng = np.random.default_rng(22)
    A = rng.standard_normal((10, 6))
    b = rng.standard_normal(10)
    blocks = [np.array([i]) for i in range(10)]
    it = _runner(A, b, blocks, 0, 0.5)
    x = np.zeros(6)
    for k, tau in enumerate([3, 8, 1, 5, 0, 7], 1):
        lam_k = 0.5 if k <= 2 else 0.5 * k / 2.0   # alpha_k = 2 alpha / k after two steps
        it.lam = lam_k
        a = A[tau]
        x = x - a * (a @ x - b[tau]) / (lam_k + a @ a)
        it.step(tau)
        np.testing.assert_allclose(it.x, x, rtol=1e-11, atol=1e-13)


def _stacked_runner(A, b, blocks, r, lam, tik):
    """Plain slimLS (no Tikhonov term) on the stacked blocks [A_k; (tik/sqrt(M)) I]
    with data [b_k; 0]: the construction of sec. 2 that defines slimTik."""
    M, n = len(blocks), A.shape[1]
    reg = tik / np.sqrt(M) * np.eye(n)
    return slimls.SlimLS(lambda t: np.vstack([A[blocks[t]], reg]),
                         lambda t: np.concatenate([b[blocks[t]], np.zeros(n)]),
                         r, lam, np.zeros(n), None, "primal")


@pytest.mark.parametrize("form", ["dual", "primal"])
@pytest.mark.parametrize("r", [0, 2, 5])
def test_slimtik_is_slimls_on_the_stacked_system(form, r):
    """eq. (slimTik) with L = I equals slimLS run on eq. (TLS1)'s stacked rows,
    window by window (including the first r steps, whose windows hold fewer
    blocks), so the Tikhonov shift counts the blocks in the window."""
    A, b, _, blocks = _dense_problem(m=60, n=8, ell=5, seed=31)
    tik, lam = 0.7, 0.3
    it = slimls.SlimLS(lambda t: A[blocks[t]], lambda t: b[blocks[t]], r, lam, np.zeros(8),
                       form=form, tik=tik, n_blocks=len(blocks))
    ref = _stacked_runner(A, b, blocks, r, lam, tik)
    for tau in np.random.default_rng(32).integers(0, len(blocks), 20):
        it.step(tau)
        ref.step(tau)
        np.testing.assert_allclose(it.x, ref.x, rtol=1e-10, atol=1e-12)


def test_slimtik_full_memory_epoch_reaches_tikhonov():
    """With the window covering every block (r = M - 1), one epoch without
    replacement and a vanishing damping lam, the slimLS induction of App. A on
    the stacked system gives x_M = (A^T A + tik^2 I)^{-1} A^T b, the Tikhonov
    solution of eq. (TLS1) with L = I (textbook least squares on [A; tik I]).
    The printed shift r tik^2 / M would stop at (M-1)/M tik^2 instead."""
    A, b, _, blocks = _dense_problem(m=48, n=10, ell=6, seed=33)
    M, tik = len(blocks), 0.9
    it = slimls.SlimLS(lambda t: A[blocks[t]], lambda t: b[blocks[t]], M - 1, 1e-12,
                       np.zeros(10), tik=tik, n_blocks=M)
    for tau in sampler.epoch_permutation(M, 0, 34):
        it.step(tau)
    x_tik = np.linalg.lstsq(np.vstack([A, tik * np.eye(10)]),
                            np.concatenate([b, np.zeros(10)]), rcond=None)[0]
    np.testing.assert_allclose(it.x, x_tik, rtol=1e-9, atol=1e-11)
