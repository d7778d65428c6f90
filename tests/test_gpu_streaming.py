"""Streaming data: each block's sinogram rows are passed with its step
(slim_step_data) instead of a resident sinogram.  The step reads only b_k
(eq. (ram)), so the iterates must equal the resident path's bit for bit and
the FP64 oracle's to the float32 tolerance (x rel. <= 1e-5)."""
import numpy as np
import pytest

import synth
from oracle import sampler, slimls, system

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def _rel(a, b):
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("B,g,r,mode,where", [(2, 2, 3, "chol", "pinned"), (1, 1, 4, "pcg", "pinned"),
                                              (3, 2, 2, "pcg", "device"), (2, 3, 1, "chol", "pageable")])
def test_streamed_blocks_match_resident_and_oracle(B, g, r, mode, where):
    from paper_1912_07962_amd import Slim
    N, na, lam = 48, 36, 1e-2
    xs, bs = synth.make_volume_problem(N, B, na, 8, 0.01, 91, 92)
    extra = [synth.make_slice_problem(N, na, 3, 0.01, 900 + k, 950 + k) for k in range(B)]
    xs = xs + np.stack([e[0] for e in extra])
    bs = (bs + np.stack([e[1] for e in extra])).astype(np.float32)
    M = na // g
    sched = sampler.schedule(M, 1, 93)[:14]
    kw = dict(r=r, lam=lam, n_slices=B, angles_per_block=g, gram_mode=mode, pcg_tol=1e-11,
              pcg_max_iter=3000)
    res = Slim(N, na, **kw)
    x_res = torch.zeros((B, N, N), dtype=torch.float32, device="cuda")
    res.set_data(_dev(bs), x_res, _dev(xs))
    st = Slim(N, na, **kw)
    x_st = torch.zeros((B, N, N), dtype=torch.float32, device="cuda")
    st.set_data(None, x_st, _dev(xs))
    P = system.Projector(N, na)
    oracles = [slimls.Tomo(P, bs[k], g, r, lam, x_true=xs[k]) for k in range(B)]
    for k, beta in enumerate(sched, 1):
        ids = list(range(beta * g, beta * g + g))
        blk = torch.from_numpy(np.ascontiguousarray(bs[:, ids, :]))
        if where == "pinned":
            blk = blk.pin_memory()
        elif where == "device":
            blk = blk.cuda()
        read = k % 3 == 0 or k == len(sched)     # unread steps let copies run ahead
        info_s = st.step_data(ids, blk, read=read)
        info_r = res.step(ids)
        for o in oracles:
            o.step(beta)
        if read:
            assert info_s == info_r
            a, b = x_st.cpu().numpy(), x_res.cpu().numpy()
            assert np.array_equal(a, b), (k, np.abs(a - b).max())
            for s in range(B):
                assert _rel(a[s], oracles[s].x) < 1e-5, (k, s)
    # partial reconstructions are available on demand and unchanged by reading them
    assert np.array_equal(x_st.cpu().numpy(), x_res.cpu().numpy())


def test_streaming_state_errors():
    from paper_1912_07962_amd import Slim
    N, na = 32, 16
    _, b, _ = synth.make_slice_problem(N, na, 3, 0.01, 97, 98)
    s = Slim(N, na, r=1, lam=1e-2)
    x = torch.zeros((N, N), dtype=torch.float32, device="cuda")
    s.set_data(_dev(b), x)
    blk = torch.from_numpy(np.ascontiguousarray(np.asarray(b, np.float32).reshape(na, -1)[3]))
    with pytest.raises(Exception):      # resident data bound: no streaming steps
        s.step_data([3], blk)
    s.set_data(None, x)
    with pytest.raises(Exception):      # streaming bound: slim_step needs the block's data
        s.step([3])
    with pytest.raises(Exception):      # wrong size
        s.step_data([3], torch.zeros(5))
    s.step_data([3], blk)
