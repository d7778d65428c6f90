"""The trained warm start saves iterations: a reduced version of the
warm-start workload (128^2, 90 angles x 181 rays, 1 angle/block, r = 5,
lambda = 1e-2) trained by the library's own kernels on targets the plain
method generates, evaluated on held-out seeds against x0 = 0."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def test_trained_network_reaches_the_plain_error_in_fewer_steps():
    from paper_1912_07962_amd import Cnn
    from paper_1912_07962_amd import warmstart as ws
    cfg = dict(ws.config(), N=128, n_angles=90)
    xtr, btr = ws.make_samples(range(50000, 50768), workers=8, cfg=cfg)
    xte, bte = ws.make_samples(range(60000, 60064), workers=8, cfg=cfg)
    dtr = ws.plain_data(btr, xtr, cfg, chunk=512, target_steps=90)
    dte = ws.plain_data(bte, xte, cfg, chunk=512)
    net = Cnn(cfg["N"], ws.CHANNELS, max_batch=16, in_scale=ws.in_scale(cfg))
    net.set_params(ws.init_params(ws.CHANNELS, 0))
    hist = ws.train(net, dtr["u"], dtr["target"], epochs=8, batch=16, lr=1e-3, lr_final=1e-4)
    assert hist[-1] < 0.5 * hist[0]
    res = ws.evaluate(net, bte, xte, dte, cfg)
    print(res)
    assert res["net_reached"] == 1.0
    assert res["net_steps_mean"] < res["plain_steps_mean"]
    assert res["net_fewer_steps_frac"] >= 0.6
    # the network does better than the best rescaled back-projection
    assert res["x0_rel_err_net"] < res["x0_rel_err_scaled_u"]
