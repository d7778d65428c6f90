"""The learned warm start in float64 (test infrastructure only).

A small CNN maps the back-projection of the first sampled blocks,
u = sum_{j<=4} A_{tau_j}^T b_{tau_j}, to a starting point x0 for slimLS; its
benefit is judged by the iterations the method needs from x0 to reach the
error of the plain run (the paper's iteration starts from any x0; its updates
lie in R(A^T), sec. 1, so the component of x0 outside R(A^T) is kept).

Network (a 4-level U-Net), layout [batch][channel][row][column]:

  in      uh = in_scale * u                                  (1 channel)
  enc 1   E1a = relu(conv(uh)),  E1 = relu(conv(E1a))        c0 channels, N x N
  enc l   El_a = relu(conv(pool(E_{l-1}))), El = relu(conv(El_a))   c_{l-1}, N/2^{l-1}
  dec l   U = relu(conv(up(D_{l+1})))  (D_4 = E4),  C = [U, E_l] (channels)
          Dl_a = relu(conv(C)),  D_l = relu(conv(Dl_a))      c_{l-1} channels
  head    x0 = sum_c wh[c] D1[c] + bh + cu * uh

conv is a 3x3 cross-correlation with zero padding and a bias, pool is a 2x2
average, up is nearest-neighbour x2.  Loss: mean squared error
L = mean((x0 - target)^2) over batch and pixels; optimizer: Adam
(Kingma & Ba 2015, Algorithm 1) with bias correction.

Conv weights are [Cout][3][3][Cin].  ``store`` (identity by default) is
applied wherever the GPU kernels store a tensor in bfloat16 (every
activation after bias and ReLU, pool outputs, and every activation gradient
after masking), so a run can follow the GPU's storage precision.

Pins (tests/test_oracle_cnn.py): conv against scipy's 2D correlation; pool
and up against their adjoints; the whole backward pass against central finite
differences; Adam's first step against its closed form lr * sign(g).
"""
from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------- layers
def conv3x3(x, w, b):
    """out[n,o,y,x] = b[o] + sum_{ky,kx,c} xpad[n,c,y+ky,x+kx] w[o,ky,kx,c]."""
    n, c, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    out = np.zeros((n, w.shape[0], H, W))
    for ky in range(3):
        for kx in range(3):
            out += np.einsum("nchw,oc->nohw", xp[:, :, ky:ky + H, kx:kx + W], w[:, ky, kx, :])
    return out + b[None, :, None, None]


def conv3x3_backward(x, w, dz):
    """Gradients of sum(dz * conv3x3(x, w, b)) wrt x, w and b."""
    n, c, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            dxp[:, :, ky:ky + H, kx:kx + W] += np.einsum("nohw,oc->nchw", dz, w[:, ky, kx, :])
            dw[:, ky, kx, :] = np.einsum("nohw,nchw->oc", dz, xp[:, :, ky:ky + H, kx:kx + W])
    return dxp[:, :, 1:-1, 1:-1], dw, dz.sum(axis=(0, 2, 3))


def pool(x):
    """2x2 average."""
    n, c, H, W = x.shape
    return x.reshape(n, c, H // 2, 2, W // 2, 2).mean(axis=(3, 5))


def pool_backward(dp):
    return np.repeat(np.repeat(dp, 2, axis=2), 2, axis=3) / 4.0


def up(x):
    """Nearest-neighbour x2."""
    return np.repeat(np.repeat(x, 2, axis=2), 2, axis=3)


def up_backward(du):
    n, c, H, W = du.shape
    return du.reshape(n, c, H // 2, 2, W // 2, 2).sum(axis=(3, 5))


def relu(z):
    return np.maximum(z, 0.0)


# ---------------------------------------------------------------- network
def layer_names(levels: int = 4):
    """Conv layers in forward order."""
    names = ["e1a", "e1b"]
    for l in range(2, levels + 1):
        names += [f"e{l}a", f"e{l}b"]
    for l in range(levels - 1, 0, -1):
        names += [f"u{l}", f"d{l}a", f"d{l}b"]
    return names


def layer_shapes(channels=(32, 64, 128, 256)):
    """{name: (Cout, Cin)} for every 3x3 conv layer."""
    L = len(channels)
    sh = {"e1a": (channels[0], 1), "e1b": (channels[0], channels[0])}
    for l in range(2, L + 1):
        c = channels[l - 1]
        sh[f"e{l}a"] = (c, channels[l - 2])
        sh[f"e{l}b"] = (c, c)
    for l in range(L - 1, 0, -1):
        c = channels[l - 1]
        sh[f"u{l}"] = (c, channels[l])
        sh[f"d{l}a"] = (c, 2 * c)
        sh[f"d{l}b"] = (c, c)
    return sh


def init_params(channels=(32, 64, 128, 256), seed: int = 0):
    """He-normal conv weights (std sqrt(2 / (9 Cin))), zero biases, head
    weights N(0, 1/c0), cu = 1 (x0 starts near uh plus a small correction)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, (co, ci) in layer_shapes(channels).items():
        p[name + ".w"] = rng.standard_normal((co, 3, 3, ci)) * np.sqrt(2.0 / (9 * ci))
        p[name + ".b"] = np.zeros(co)
    p["head.w"] = rng.standard_normal(channels[0]) / np.sqrt(channels[0])
    p["head.b"] = np.zeros(1)
    p["head.cu"] = np.ones(1)
    return p


def forward(p, u, in_scale: float, levels: int = 4, store=None):
    """x0 for u[n, N, N].  Returns (x0[n, N, N], cache)."""
    st = (lambda a: a) if store is None else store
    uh = in_scale * np.asarray(u, np.float64)[:, None]
    cache = {"uh": uh}

    def cv(name, x):
        z = conv3x3(x, p[name + ".w"], p[name + ".b"])
        y = st(relu(z))
        cache[name + ".in"] = x
        cache[name + ".out"] = y
        return y

    x = cv("e1b", cv("e1a", uh))
    enc = {1: x}
    for l in range(2, levels + 1):
        pl = st(pool(enc[l - 1]))
        x = cv(f"e{l}b", cv(f"e{l}a", pl))
        enc[l] = x
    d = enc[levels]
    for l in range(levels - 1, 0, -1):
        uu = cv(f"u{l}", up(d))
        cat = np.concatenate([uu, enc[l]], axis=1)
        d = cv(f"d{l}b", cv(f"d{l}a", cat))
    cache["d1"] = d
    x0 = np.einsum("nchw,c->nhw", d, p["head.w"]) + p["head.b"][0] + p["head.cu"][0] * uh[:, 0]
    return x0, cache


def loss_and_grads(p, u, target, in_scale: float, levels: int = 4, store=None):
    """MSE loss and its gradient wrt every parameter (manual backward)."""
    st = (lambda a: a) if store is None else store
    x0, c = forward(p, u, in_scale, levels, store)
    target = np.asarray(target, np.float64)
    diff = x0 - target
    loss = float(np.mean(diff * diff))
    dx0 = 2.0 * diff / diff.size
    g = {}
    g["head.w"] = np.einsum("nhw,nchw->c", dx0, c["d1"])
    g["head.b"] = np.array([dx0.sum()])
    g["head.cu"] = np.array([np.sum(dx0 * c["uh"][:, 0])])
    dy = st(dx0[:, None] * p["head.w"][None, :, None, None] * (c["d1"] > 0))

    def back(name, dz, mask_in=True):
        """dz: gradient at the pre-activation of layer `name`; returns the
        gradient at its input (masked by the input's ReLU if mask_in)."""
        x = c[name + ".in"]
        dx, dw, db = conv3x3_backward(x, p[name + ".w"], dz)
        g[name + ".w"] = dw
        g[name + ".b"] = db
        return dx * (x > 0) if mask_in else dx

    # decoder, top level first: dy is the gradient at the pre-activation of
    # d{l}b; each level hands the next-deeper one the gradient at the
    # pre-activation of the layer its up-sampling read
    skip = {}
    for l in range(1, levels):
        d_la = st(back(f"d{l}b", dy))
        dcat = st(back(f"d{l}a", d_la))
        cu = c[f"u{l}.out"].shape[1]
        skip[l] = dcat[:, cu:]                    # gradient reaching E_l via C
        dup = st(back(f"u{l}", dcat[:, :cu], mask_in=False))
        below = c[f"d{l + 1}b.out"] if l + 1 < levels else c[f"e{levels}b.out"]
        dy = st(up_backward(dup) * (below > 0))
    # encoder, bottom level first: dy is the gradient at the pre-activation
    # of e{l}b; E_{l-1} receives the pool path and the skip path
    for l in range(levels, 0, -1):
        d_la = st(back(f"e{l}b", dy))
        if l == 1:
            back("e1a", d_la, mask_in=False)
            break
        dp = st(back(f"e{l}a", d_la, mask_in=False))
        e_prev = c[f"e{l - 1}b.out"]
        dy = st((pool_backward(dp) + skip[l - 1]) * (e_prev > 0))
    return loss, g, x0


def adam_step(p, g, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1), in place; t >= 1."""
    for k in p:
        m[k] = beta1 * m[k] + (1 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1 - beta2) * g[k] * g[k]
        mh = m[k] / (1 - beta1 ** t)
        vh = v[k] / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
