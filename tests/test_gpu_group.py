"""Mixed batches (contexts of different grid sizes stepped as one group) and
the graph replay of CG iteration chunks, both against the plain per-context
path they must reproduce bit for bit."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

NA, G = 24, 2


def _problem(N, B, seed):
    xs, bs = synth.make_volume_problem(N, B, NA, 8, 0.01, seed, seed + 1)
    extra = [synth.make_slice_problem(N, NA, 3, 0.01, seed + 10 + k, seed + 20 + k)
             for k in range(B)]
    return xs + np.stack([e[0] for e in extra]), bs + np.stack([e[1] for e in extra])


def _ctx(N, B, mode, b, stream=None, use_graph=True):
    from paper_1912_07962_amd import Slim
    s = Slim(N, NA, r=3, lam=1e-2, n_slices=B, angles_per_block=G, gram_mode=mode,
             pcg_tol=1e-10, pcg_max_iter=2000, stream=stream, use_graph=use_graph)
    x = torch.zeros((B, N, N), dtype=torch.float32, device="cuda")
    bd = torch.as_tensor(b, dtype=torch.float32, device="cuda")
    s.set_data(bd, x)
    return s, x, bd


SPECS = [(32, 3, "pcg"), (64, 2, "chol"), (48, 4, "pcg"), (40, 1, "pcg")]


@pytest.mark.parametrize("shared,streams", [(False, False), (True, False), (True, True)])
def test_group_step_equals_separate_steps(shared, streams):
    """Shared launches (one back-projection, forward and vector launch per
    CG iteration over all contexts; graph replay when the contexts have
    streams of their own) and interleaved per-context launches both equal
    the contexts stepped alone, bit for bit."""
    from paper_1912_07962_amd import Group
    probs = [_problem(N, B, 100 + i) for i, (N, B, _) in enumerate(SPECS)]
    sts = [torch.cuda.Stream() if streams else None for _ in SPECS]
    grp_ctx = [_ctx(N, B, m, probs[i][1], stream=sts[i]) for i, (N, B, m) in enumerate(SPECS)]
    torch.cuda.synchronize()
    solo = [_ctx(N, B, m, probs[i][1]) for i, (N, B, m) in enumerate(SPECS)]
    grp = Group([c[0] for c in grp_ctx], shared=shared)
    sched = synth.schedule(NA // G, 1, 17)
    for beta in sched:
        ids = list(range(int(beta) * G, int(beta) * G + G))
        infos = grp.step(ids)
        for i, (s, x, _) in enumerate(solo):
            inf = s.step(ids)
            assert infos[i]["step_norm"] == inf["step_norm"]
            assert infos[i]["pcg_iters"] == inf["pcg_iters"]
        torch.cuda.synchronize()
        for (_, xg, _), (_, xs, _) in zip(grp_ctx, solo):
            assert torch.equal(xg, xs)
    grp.close()


def test_graph_replay_equals_eager_launches():
    """Chunks of CG iterations replayed as graphs on a side stream, with eager
    work and synchronisations of the program between replays, against the
    same contexts launching every kernel on the default stream."""
    side = torch.cuda.Stream()
    N, B = 48, 3
    _, b = _problem(N, B, 7)
    eager, xe, _ = _ctx(N, B, "pcg", b, use_graph=False)
    with torch.cuda.stream(side):
        graph, xg, _ = _ctx(N, B, "pcg", b, stream=side, use_graph=True)
    side.synchronize()
    other = torch.randn((256, 256), device="cuda")
    sched = synth.schedule(NA // G, 1, 5)
    for k, beta in enumerate(sched):
        ids = list(range(int(beta) * G, int(beta) * G + G))
        ie = eager.step(ids)
        with torch.cuda.stream(side):
            ig = graph.step(ids)
        side.synchronize()
        other = other @ other.T / 256.0       # eager work between replays
        torch.cuda.synchronize()
        assert ig["pcg_iters"] == ie["pcg_iters"] and ig["pcg_iters"] > 8
        assert torch.equal(xg, xe), k


def test_group_argument_errors():
    from paper_1912_07962_amd import Group, Slim, SlimError
    a = Slim(32, NA, r=1, lam=1e-2, angles_per_block=G)
    b = Slim(32, NA + 2, r=1, lam=1e-2, angles_per_block=G)
    with pytest.raises(SlimError):
        Group([a, b])                 # different angle sets
    with pytest.raises(SlimError):
        Group([a, a])                 # listed twice
    g = Group([a])
    with pytest.raises(SlimError):
        g.step([0, 1])                # no data bound
    # a context bound to streaming data is refused before any context moves
    x1 = torch.zeros((32, 32), device="cuda")
    a.set_data(torch.zeros((NA, a.R), device="cuda"), x1)
    c = Slim(32, NA, r=1, lam=1e-2, angles_per_block=G)
    c.set_data(None, torch.zeros((32, 32), device="cuda"))
    g2 = Group([a, c])
    with pytest.raises(SlimError) as e:
        g2.step([0, 1])
    assert e.value.status == 6
    assert a.step([0, 1])["k"] == 1   # a's iteration did not advance
    g2.close()


def test_non_finite_data_is_reported():
    """NaN or Inf in b (or in x0) reaches the step norms: SLIM_ENUMERIC."""
    from paper_1912_07962_amd import Slim, SlimError
    N = 32
    for mode in ("chol", "pcg"):
        for where in ("b", "x"):
            s = Slim(N, NA, r=1, lam=1e-2, angles_per_block=G, gram_mode=mode)
            b = torch.zeros((NA, s.R), device="cuda")
            x = torch.zeros((N, N), device="cuda")
            if where == "b":
                b[0, s.R // 2] = float("nan")
            else:
                x[N // 2, N // 2] = float("inf")
            s.set_data(b, x)
            with pytest.raises(SlimError) as e:
                s.step([0, 1])
            assert e.value.status == 4, (mode, where)
            s.close()


def test_shared_launches_repeatable_at_scale():
    """Two identical groups of the mixed-batch sizes (64 slices of 256^2, 32
    of 512^2, 8 of 1024^2; 360 angles, 4 per block, r = 8) in shared launches
    give the same iterates bit for bit, step after step, and equal the
    contexts stepped alone.  At these sizes the CG vector launch holds
    thousands of workgroups, so a slice's stop flag is set while other
    workgroups of the same slice are starting: their stop decision must be
    the same for all of a workgroup's waves."""
    from paper_1912_07962_amd import Group, Slim
    cfg = synth.get_config("c4m")
    na, g, r, lam = cfg["n_angles"], cfg["g"], cfg["r"], cfg["lam"]
    sets = {"A": [], "B": [], "solo": []}
    for N, B in cfg["groups"]:
        xs, bs = synth.make_volume_problem(N, B, na, cfg["n_ellipsoids"], cfg["noise"],
                                           cfg["phantom_seed"], cfg["noise_seed"])
        for key in sets:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                s = Slim(N, na, r=r, lam=lam, n_slices=B, angles_per_block=g, gram_mode="pcg",
                         pcg_tol=1e-6, stream=st)
                bd = torch.as_tensor(bs, dtype=torch.float32, device="cuda")
                x = torch.zeros((B, N, N), dtype=torch.float32, device="cuda")
            st.synchronize()
            s.set_data(bd, x)
            sets[key].append((s, x, bd))
    grp = {k: Group([c[0] for c in sets[k]], shared=True) for k in ("A", "B")}
    sched = synth.schedule(na // g, 1, cfg["schedule_seed"])
    for k in range(r + 4):
        ids = list(range(int(sched[k]) * g, int(sched[k]) * g + g))
        ia = grp["A"].step(ids)
        ib = grp["B"].step(ids)
        assert [i["pcg_iters"] for i in ia] == [i["pcg_iters"] for i in ib]
        torch.cuda.synchronize()
        for (_, xa, _), (_, xb, _) in zip(sets["A"], sets["B"]):
            assert torch.equal(xa, xb), f"step {k + 1}"
    for k in range(r + 4):
        ids = list(range(int(sched[k]) * g, int(sched[k]) * g + g))
        for s, _, _ in sets["solo"]:
            s.step(ids)
    torch.cuda.synchronize()
    for (_, xa, _), (_, xs, _) in zip(sets["A"], sets["solo"]):
        assert torch.equal(xa, xs)
    for gp in grp.values():
        gp.close()
    for v in sets.values():
        for s, _, _ in v:
            s.close()
