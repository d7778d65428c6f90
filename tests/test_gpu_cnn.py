"""Warm-start CNN on the GPU against the FP64 oracle.

The oracle runs with the GPU's storage precision: conv weights rounded to
bfloat16, and every tensor the kernels store in bfloat16 rounded there too
(the oracle's ``store`` hook).  What remains is fp32-vs-fp64 accumulation:
where the two sums straddle a bf16 rounding boundary the stored values differ
by one bf16 ulp (2^-8 relative), and such flips propagate through the
following layers.  With up to 17 stored layers the forward output differs by
a few 1e-3 in relative norm; the bounds are 1e-2 for outputs, 5e-2 for one
parameter's gradient (small tensors such as biases sum few terms) and 2e-2
for the whole gradient vector.  Index or layout mistakes give O(1) errors."""
import numpy as np
import pytest

import synth
from oracle import cnn as ocnn
from oracle import slimls, system

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _rel(a, b):
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _params(channels, seed):
    rng = np.random.default_rng(seed)
    p = ocnn.init_params(channels, seed)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    p["head.b"] = np.array([0.1])
    p["head.cu"] = np.array([0.8])
    return {k: v.astype(np.float32) for k, v in p.items()}


def _oracle_view(p32):
    """float64 parameters as the GPU uses them: conv weights in bf16."""
    out = {}
    for k, v in p32.items():
        v = v.astype(np.float64)
        out[k] = slimls.round_bf16(v) if (k.endswith(".w") and not k.startswith("head")) else v
    return out


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


CASES = [((32, 64), 16, 3), ((32, 64, 128), 32, 2), ((32, 64, 128, 256), 64, 2)]


@pytest.mark.parametrize("channels,N,B", CASES)
def test_forward_matches_oracle(channels, N, B):
    from paper_1912_07962_amd import Cnn
    p = _params(channels, 11)
    u = np.random.default_rng(1).uniform(0.0, 1.0, (B, N, N)).astype(np.float32)
    net = Cnn(N, channels, max_batch=B, in_scale=1.7)
    assert net.n_params == sum(v.size for v in p.values())
    net.set_params(p)
    x0 = net.forward(_dev(u)).cpu().numpy()
    ref, _ = ocnn.forward(_oracle_view(p), u.astype(np.float64), 1.7, levels=len(channels),
                          store=slimls.round_bf16)
    err = _rel(x0, ref)
    print(f"forward rel err {err:.2e}")
    assert err < 1e-2


@pytest.mark.parametrize("channels,N,B", CASES)
def test_gradients_match_oracle(channels, N, B):
    from paper_1912_07962_amd import Cnn
    p = _params(channels, 12)
    rng = np.random.default_rng(2)
    u = rng.uniform(0.0, 1.0, (B, N, N)).astype(np.float32)
    t = rng.uniform(0.0, 1.0, (B, N, N)).astype(np.float32)
    net = Cnn(N, channels, max_batch=B, in_scale=1.3)
    net.set_params(p)
    loss, g = net.loss_grad(_dev(u), _dev(t), want_grad=True)
    lo, go, _ = ocnn.loss_and_grads(_oracle_view(p), u.astype(np.float64), t.astype(np.float64),
                                    1.3, levels=len(channels), store=slimls.round_bf16)
    assert abs(loss - lo) <= 1e-3 * lo
    gd = net.unpack(g)
    errs = {k: _rel(gd[k], go[k]) for k in go}
    print("gradient rel err max", max(errs.values()), "whole", _rel(g, net.pack(go)))
    for k in go:
        assert errs[k] < 5e-2, (k, errs[k])
    assert _rel(g, net.pack(go)) < 2e-2
    # bitwise reproducible (fixed-order reductions)
    _, g2 = net.loss_grad(_dev(u), _dev(t), want_grad=True)
    assert np.array_equal(g, g2)


def test_adam_steps_match_oracle():
    from paper_1912_07962_amd import Cnn
    channels, N, B = (32, 64), 16, 2
    p = _params(channels, 13)
    rng = np.random.default_rng(3)
    u = rng.uniform(0.0, 1.0, (B, N, N)).astype(np.float32)
    t = rng.uniform(0.0, 1.0, (B, N, N)).astype(np.float32)
    net = Cnn(N, channels, max_batch=B)
    net.set_params(p)
    ref = {k: v.astype(np.float64) for k, v in p.items()}
    m = {k: np.zeros_like(v) for k, v in ref.items()}
    v = {k: np.zeros_like(v) for k, v in ref.items()}
    for step in (1, 2, 3):
        _, g = net.loss_grad(_dev(u), _dev(t), want_grad=True)
        net.adam(1e-3)
        ocnn.adam_step(ref, {k: a.astype(np.float64) for k, a in net.unpack(g).items()}, m, v,
                       step, 1e-3)
        got = net.unpack(net.get_params())
        for k in ref:
            np.testing.assert_allclose(got[k], ref[k], rtol=1e-6, atol=2e-7, err_msg=k)


def test_training_reduces_loss():
    from paper_1912_07962_amd import Cnn
    channels, N, B = (32, 64), 32, 8
    p = _params(channels, 14)
    rng = np.random.default_rng(4)
    u = _dev(rng.uniform(0.0, 1.0, (B, N, N)))
    t = _dev(rng.uniform(0.0, 1.0, (B, N, N)))
    net = Cnn(N, channels, max_batch=B)
    net.set_params(p)
    losses = []
    for _ in range(40):
        loss, _ = net.loss_grad(u, t)
        losses.append(loss)
        net.adam(3e-3)
    assert losses[-1] < 0.5 * losses[0], losses[::8]


def test_data_backprojection_and_warmstart():
    from paper_1912_07962_amd import Cnn, Slim, SlimError
    N, na, B = 64, 30, 2
    probs = [synth.make_slice_problem(N, na, 5, 0.01, 70 + k, 80 + k) for k in range(B)]
    b = np.stack([q[1] for q in probs])
    s = Slim(N, na, r=1, lam=1e-2, n_slices=B)
    x = torch.zeros((B, N, N), dtype=torch.float32, device="cuda")
    s.set_data(_dev(b), x)
    ids = [3, 17, 8, 25]
    u = s.data_backprojection(ids).cpu().numpy()
    P = system.Projector(N, na)
    for k in range(B):
        ref = P.back(ids, b[k][ids].astype(np.float32).astype(np.float64))
        assert _rel(u[k], ref) < 1e-6
    # no network: zeros, fallback flag
    x0, used = s.warmstart(ids)
    assert not used and not torch.any(x0)
    # invalid parameters: fallback
    net = Cnn(N, (32, 64), max_batch=1)
    bad = net.pack(_params((32, 64), 5))
    bad[7] = np.nan
    net.set_params(bad)
    x0, used = s.warmstart(ids, net=net)
    assert not used and not torch.any(x0)
    # a valid network, run in chunks of max_batch = 1
    net.set_params(_params((32, 64), 5))
    x0, used = s.warmstart(ids, net=net)
    assert used
    direct = net.forward(_dev(u[:1])).cpu().numpy()
    assert np.array_equal(x0[:1].cpu().numpy(), direct)
    direct = net.forward(_dev(u[1:])).cpu().numpy()
    assert np.array_equal(x0[1:].cpu().numpy(), direct)
    # into the bound x: the iteration restarts from x0 with fresh projector
    # copies, exactly as binding x0 with set_data
    s.warmstart(ids, x0=x, net=net)
    s.step([5])
    x_a = x.clone()
    x.copy_(x0)
    s.set_data(_dev(b), x)
    s.step([5])
    assert torch.equal(x, x_a)
    # size mismatch
    other = Cnn(32, (32, 64), max_batch=1)
    with pytest.raises(SlimError):
        s.warmstart(ids, net=other)


def test_cnn_call_errors():
    from paper_1912_07962_amd import Cnn, SlimError
    net = Cnn(16, (32, 64), max_batch=2)
    u = torch.zeros((3, 16, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(SlimError):
        net.forward(u)                        # batch above max_batch
    with pytest.raises(SlimError):
        net.adam(1e-3)                        # no gradient yet
    with pytest.raises(SlimError):
        net.set_params(np.zeros(5, np.float32))
    net.loss_grad(u[:2], u[:2])
    with pytest.raises(SlimError):
        net.adam(-1.0)
