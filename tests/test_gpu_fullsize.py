"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (library stream, CG graph replay, autotuned projector shapes),
against stored FP64 oracle runs (``tests/golden/make_goldens.py``, which
calls only ``oracle/`` and ``synth/``; CG to a relative residual of 1e-12).

* the 1024^2 plain workload (720 angles x 1449 rays, 8 angles per block,
  r = 10, lambda = 1e-3) with its memory window full: x after steps 11 and 12
  (p = 127,512 Gram rows), at CG tolerance 1e-9 and at the benchmark's 1e-6;
* the 512-slice 512^2 volume (360 x 725, 4 angles per block, r = 8): all 512
  slices stepped together, three slices checked after steps 9 and 10;
* the mixed batch (64 x 256^2, 32 x 512^2, 8 x 1024^2) stepped as one group:
  one slice of each context against its own oracle run after steps 9 and 10;
* the explicit-Gram FP64 Cholesky at its size cap, p = 8192, and at the
  256^2 warm-start workload's p = 2178 over r + 2 steps;
* the warm-start network at its deployed size (4 levels, 256^2), forward and
  gradients.

Bars: x rel. <= 1e-5 in norm (the reconstruction target; weights and x are
float32, Gram scalars float64) and element by element within 1e-5 of the
largest entry; step norms within 1e-5.  At the benchmark's CG tolerance 1e-6
the norm bar is the same and the elementwise bar 2e-5 (measured: 1.2e-6 in
norm and 4.5e-6 elementwise at 1024^2, 1.4e-6 and 3.9e-6 on the volume, against
2.9e-7 and 5e-7 at 1e-9).  The network's bars are those of its smaller-size
tests.
"""
import importlib.util
import os

import numpy as np
import pytest

import synth
from oracle import slimls, system

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    path = os.path.join(GOLDEN, name + ".npz")
    if not os.path.exists(path):
        pytest.skip(f"{name}.npz not generated (tests/golden/make_goldens.py {name})")
    return np.load(path)


def _rel(a, b):
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _max_rel(a, b):
    """Largest elementwise difference relative to the largest entry."""
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _block(beta, g):
    return list(range(int(beta) * g, int(beta) * g + g))


def _golden_script():
    spec = importlib.util.spec_from_file_location("make_goldens",
                                                  os.path.join(GOLDEN, "make_goldens.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


# --------------------------------------------------------- 1024^2 window
@pytest.mark.parametrize("tol", [1e-9, 1e-6])
def test_config2_full_window_matches_oracle(tol):
    from paper_1912_07962_amd import Slim
    gd = _golden("c2_window")
    cfg = synth.get_config("c2")
    N, na, g, r, lam = cfg["N"], cfg["n_angles"], cfg["g"], cfg["r"], cfg["lam"]
    assert (int(gd["N"]), int(gd["g"]), int(gd["r"])) == (N, g, r)
    x_true, b, _ = synth.make_slice_problem(N, na, cfg["n_ellipses"], cfg["noise"],
                                            cfg["phantom_seed"], cfg["noise_seed"])
    st = torch.cuda.Stream()
    s = Slim(N, na, r=r, lam=lam, angles_per_block=g, gram_mode="pcg", pcg_tol=tol, stream=st)
    s.autotune()
    with torch.cuda.stream(st):
        bd = torch.as_tensor(b, dtype=torch.float32, device="cuda")
        xt = torch.as_tensor(x_true, dtype=torch.float32, device="cuda")
        x = torch.zeros((N, N), dtype=torch.float32, device="cuda")
    st.synchronize()
    s.set_data(bd, x, xt)
    errs = {}
    for k, beta in enumerate(gd["blocks"], start=1):
        info = s.step(_block(beta, g))
        assert info["pcg_relres"] <= tol
        sn = float(gd["step_norm"][k - 1])
        if f"x{k}" in gd.files:
            xe = x.cpu().numpy()
            errs[k] = (_rel(xe, gd[f"x{k}"]), _max_rel(xe, gd[f"x{k}"]),
                       abs(info["step_norm"] - sn) / sn)
    print(f"1024^2 window, CG tol {tol:g}: (rel, max elementwise, step norm) after steps "
          + ", ".join(f"{k}: {e[0]:.2e} {e[1]:.2e} {e[2]:.2e}" for k, e in errs.items()))
    assert sorted(errs) == [r + 1, r + 2]
    for k, (rel, mx, dsn) in errs.items():
        if tol <= 1e-9:
            assert rel <= 1e-5 and mx <= 1e-5 and dsn <= 1e-5, (k, rel, mx, dsn)
        else:
            # the benchmark's tolerance: the reconstruction target still holds
            assert rel <= 1e-5 and mx <= 2e-5 and dsn <= 1e-5, (k, rel, mx, dsn)
    s.close()


# --------------------------------------------------------- 512-slice volume
@pytest.fixture(scope="module")
def volume_512():
    cfg = synth.get_config("c4")
    xs, bs = synth.make_volume_problem(cfg["N"], cfg["n_slices"], cfg["n_angles"],
                                       cfg["n_ellipsoids"], cfg["noise"], cfg["phantom_seed"],
                                       cfg["noise_seed"])
    bd = torch.as_tensor(bs, dtype=torch.float32, device="cuda")
    del xs, bs
    return cfg, bd


@pytest.mark.parametrize("tol", [1e-9, 1e-6])
def test_volume_512_full_window_sampled_slices(volume_512, tol):
    from paper_1912_07962_amd import Slim
    cfg, bd = volume_512
    gd = _golden("c4_slices")
    N, B, na, g, r, lam = (cfg[k] for k in ("N", "n_slices", "n_angles", "g", "r", "lam"))
    st = torch.cuda.Stream()
    s = Slim(N, na, r=r, lam=lam, n_slices=B, angles_per_block=g, gram_mode="pcg",
             pcg_tol=tol, stream=st)
    s.autotune()
    s.autotune(n_ids=g)
    with torch.cuda.stream(st):
        x = torch.zeros((B, N, N), dtype=torch.float32, device="cuda")
    st.synchronize()
    s.set_data(bd, x)
    picks = [int(v) for v in gd["slices"]]
    out = []
    for k, beta in enumerate(gd["s0_blocks"], start=1):
        s.step(_block(beta, g))
        if f"s0_x{k}" in gd.files:
            xe = x.cpu().numpy()
            for j, sl in enumerate(picks):
                ref = gd[f"s{j}_x{k}"]
                out.append((k, sl, _rel(xe[sl], ref), _max_rel(xe[sl], ref)))
    print(f"512 x 512^2 volume, CG tol {tol:g}: "
          + ", ".join(f"step {k} slice {sl}: {a:.2e} {m:.2e}" for k, sl, a, m in out))
    assert len(out) == 2 * len(picks)
    for k, sl, rel, mx in out:
        assert rel <= 1e-5, (k, sl, rel)
        assert mx <= (1e-5 if tol <= 1e-9 else 2e-5), (k, sl, mx)
    s.close()


# --------------------------------------------------------- mixed batch
@pytest.mark.parametrize("shared", [True, False])
def test_mixed_group_each_context_matches_its_oracle(shared):
    from paper_1912_07962_amd import Group, Slim
    gd = _golden("c4m_slices")
    cfg = synth.get_config("c4m")
    na, g, r, lam = cfg["n_angles"], cfg["g"], cfg["r"], cfg["lam"]
    picks = [tuple(int(v) for v in p) for p in gd["picks"]]
    assert [(N, B) for N, B, _ in picks] == [tuple(gp) for gp in cfg["groups"]]
    ctxs, xs, keep = [], [], []
    for N, B, _ in picks:
        _, bs = synth.make_volume_problem(N, B, na, cfg["n_ellipsoids"], cfg["noise"],
                                          cfg["phantom_seed"], cfg["noise_seed"])
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            s = Slim(N, na, r=r, lam=lam, n_slices=B, angles_per_block=g, gram_mode="pcg",
                     pcg_tol=1e-9, stream=st)
            s.autotune()
            bd = torch.as_tensor(bs, dtype=torch.float32, device="cuda")
            x = torch.zeros((B, N, N), dtype=torch.float32, device="cuda")
        st.synchronize()
        s.set_data(bd, x)
        ctxs.append(s)
        xs.append(x)
        keep.append((st, bd))
    grp = Group(ctxs, shared=shared)
    res = []
    for k, beta in enumerate(gd["s0_blocks"], start=1):
        grp.step(_block(beta, g))
        if f"s0_x{k}" in gd.files:
            torch.cuda.synchronize()
            for j, (N, B, sl) in enumerate(picks):
                xe = xs[j][sl].cpu().numpy()
                ref = gd[f"s{j}_x{k}"]
                res.append((k, N, _rel(xe, ref), _max_rel(xe, ref)))
    print("mixed group: " + ", ".join(f"step {k} N={N}: {a:.2e} {m:.2e}" for k, N, a, m in res))
    assert len(res) == 2 * len(picks)
    for k, N, rel, mx in res:
        assert rel <= 1e-5 and mx <= 1e-5, (k, N, rel, mx)
    grp.close()
    for s in ctxs:
        s.close()


# --------------------------------------------------------- explicit Gram
def test_cholesky_at_its_size_cap_matches_oracle():
    from paper_1912_07962_amd import Slim
    gd = _golden("chol_cap")
    mg = _golden_script()
    c = mg.CHOL_CAP
    assert (c["r"] + 1) * c["g"] * c["R"] == 8192
    x_true, b = mg.chol_cap_problem()
    s = Slim(c["N"], c["n_angles"], n_rays=c["R"], r=c["r"], lam=c["lam"],
             angles_per_block=c["g"], gram_mode="chol")
    bd = torch.as_tensor(b, dtype=torch.float32, device="cuda")
    xt = torch.as_tensor(x_true, dtype=torch.float32, device="cuda")
    x = torch.zeros((c["N"], c["N"]), dtype=torch.float32, device="cuda")
    s.set_data(bd, x, xt)
    res = []
    for k, beta in enumerate(gd["blocks"], start=1):
        info = s.step(_block(beta, c["g"]))
        sn = float(gd["step_norm"][k - 1])
        assert abs(info["step_norm"] - sn) <= 1e-5 * sn, k
        if f"x{k}" in gd.files:
            xe = x.cpu().numpy()
            res.append((k, _rel(xe, gd[f"x{k}"]), _max_rel(xe, gd[f"x{k}"])))
    print("Cholesky p = 8192: " + ", ".join(f"step {k}: {a:.2e} {m:.2e}" for k, a, m in res))
    assert len(res) == 2
    for k, rel, mx in res:
        assert rel <= 1e-5 and mx <= 1e-5, (k, rel, mx)
    s.close()


def test_cholesky_warmstart_workload_full_window():
    """256^2, 180 angles x 363 rays, one angle per block, r = 5,
    lambda = 1e-2: p = 2178 once the window is full; r + 2 steps against
    the oracle's dense Cholesky."""
    from paper_1912_07962_amd import Slim
    cfg = synth.get_config("c5")
    N, na, g, r, lam = cfg["N"], cfg["n_angles"], cfg["g"], cfg["r"], cfg["lam"]
    x_true, b = synth.warmstart_sample(20000)
    sched = synth.schedule(na // g, 1, cfg["schedule_seed"])[: r + 2]
    s = Slim(N, na, r=r, lam=lam, angles_per_block=g, gram_mode="chol")
    x = torch.zeros((N, N), dtype=torch.float32, device="cuda")
    s.set_data(torch.as_tensor(b, dtype=torch.float32, device="cuda"), x,
               torch.as_tensor(x_true, dtype=torch.float32, device="cuda"))
    T = slimls.Tomo(system.Projector(N, na), b, g, r, lam, x_true=x_true)
    for k, beta in enumerate(sched, start=1):
        info = s.step(_block(beta, g))
        rec = T.step(int(beta))
        xe = x.cpu().numpy()
        assert _rel(xe, T.x) <= 1e-5 and _max_rel(xe, T.x) <= 1e-5, k
        assert abs(info["step_norm"] - rec.step_norm) <= 1e-5 * rec.step_norm, k
    assert rec.mode == "chol" and T.it.window and len(T.it.window) == r + 1
    s.close()


# --------------------------------------------------------- network, 256^2
def test_cnn_256_forward_and_gradients_match_oracle():
    """Bars as in the smaller network tests: forward rel. <= 1e-2, loss
    <= 1e-3, each gradient tensor (all entries, or its stored sample and its
    norm for tensors over 20,000 entries) <= 5e-2."""
    from paper_1912_07962_amd import Cnn
    gd = _golden("cnn_256")
    mg = _golden_script()
    p = mg.cnn_params(int(gd["param_seed"]))
    u, t = gd["u"], gd["target"]
    B, N = u.shape[0], u.shape[1]
    net = Cnn(N, mg.CNN_CHANNELS, max_batch=B, in_scale=float(gd["in_scale"]))
    net.set_params(p)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    x0 = net.forward(dev(u)).cpu().numpy()
    fwd = _rel(x0, gd["x0"])
    loss, g = net.loss_grad(dev(u), dev(t), want_grad=True)
    gg = net.unpack(g)
    errs = {}
    for k, v in gg.items():
        v = np.asarray(v, np.float64).reshape(-1)
        if "g_" + k in gd.files:
            errs[k] = _rel(v, gd["g_" + k])
        else:
            pos = gd["gpos_" + k]
            nrm = float(gd["gnorm_" + k])
            errs[k] = max(_rel(v[pos], gd["gval_" + k]), abs(np.linalg.norm(v) - nrm) / nrm)
    print(f"cnn 256^2: forward {fwd:.2e}, loss {abs(loss - float(gd['loss'])) / float(gd['loss']):.2e},"
          f" gradient worst {max(errs.values()):.2e} ({max(errs, key=errs.get)})")
    assert fwd <= 1e-2
    assert abs(loss - float(gd["loss"])) <= 1e-3 * float(gd["loss"])
    assert len(errs) == len(mg.cnn_params()) and all(e <= 5e-2 for e in errs.values()), errs
    net.close()
