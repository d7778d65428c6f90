"""Edge sizes through the C ABI against the FP64 oracle: the smallest grids
(N = 2, a single ray, one angle, one block holding every angle) and the
largest detector the library accepts (R = 4096) on 4096^2 and 8192^2 (the
largest) images, where
the oracle evaluates sampled rays one by one from the closed-form weight and
the adjoint identity covers every ray and pixel."""
import math

import numpy as np
import pytest

import synth
from oracle import geometry, slimls, system

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def _rel(a, b):
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def ray_sum(img, theta, t, R, rows=256):
    """One ray's sum over the whole image with the closed-form Joseph weight
    (pixel (i, j) at x = centre j, y = centre i), in float64."""
    N = img.shape[0]
    h = 2.0 / N
    xc = geometry.pixel_centres(N)
    s = geometry.ray_offsets(N, R)[t]
    tot = 0.0
    for i0 in range(0, N, rows):
        y = xc[i0:i0 + rows, None]
        tot += float(np.sum(geometry.joseph_weight(theta, s, xc[None, :], y, h)
                            * img[i0:i0 + rows]))
    return tot


def test_ray_sum_matches_the_oracle_projector():
    """The sampled-ray helper agrees with the oracle's CSR rows (CPU)."""
    N, na, R = 12, 7, 9
    P = system.Projector(N, na, R=R)
    img = np.random.default_rng(1).standard_normal((N, N))
    ref = P.forward(list(range(na)), img).reshape(na, R)
    th = geometry.angles(na)
    for a in range(na):
        for t in range(R):
            assert abs(ray_sum(img, th[a], t, R) - ref[a, t]) <= 1e-12 * np.abs(ref).max()


@gpu
@pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")
@pytest.mark.parametrize("N,na,R,g,r", [(2, 1, 1, 1, 0), (2, 3, 3, 3, 0), (3, 2, 1, 1, 1),
                                        (5, 4, 7, 4, 2), (4, 6, 5, 2, 3)])
def test_tiny_grids_step_like_the_oracle(N, na, R, g, r):
    from paper_1912_07962_amd import Slim
    rng = np.random.default_rng(N * 10 + na)
    x_true = rng.uniform(0.1, 1.0, (N, N))
    P = system.Projector(N, na, R=R)
    b = P.forward(list(range(na)), x_true).reshape(na, R)
    ids = list(range(na))
    s = Slim(N, na, n_rays=R, r=r, lam=1e-2, angles_per_block=g, gram_mode="chol")
    fwd = s.project(ids, _dev(x_true)).cpu().numpy().reshape(na, R)
    assert _rel(fwd, b) < 1e-6
    v = rng.standard_normal((na, R))
    back = s.backproject(ids, _dev(v)).cpu().numpy().reshape(N, N)
    assert _rel(back, P.back(ids, v).reshape(N, N)) < 1e-6
    T = slimls.Tomo(P, b, g, r, 1e-2, x_true=x_true)
    x = torch.zeros((N, N), dtype=torch.float32, device="cuda")
    s.set_data(_dev(b), x, _dev(x_true))
    M = na // g
    for k, beta in enumerate([j % M for j in range(3 * M)], 1):
        s.step(list(range(beta * g, beta * g + g)))
        T.step(beta)
        assert _rel(x.cpu().numpy(), T.x) < 1e-5, (k, _rel(x.cpu().numpy(), T.x))


@gpu
@pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")
@pytest.mark.parametrize("N", [4096, 8192])    # 8192: the largest image, one-row bands
def test_largest_detector_sampled_rays_and_adjoint(N):
    from paper_1912_07962_amd import Slim
    na, R = 8, 4096
    ids = list(range(na))                 # row- and column-stepping angles
    rng = np.random.default_rng(7)
    img = rng.uniform(0.0, 1.0, (N, N)).astype(np.float32)
    s = Slim(N, na, n_rays=R, r=0, lam=1.0)
    fwd = s.project(ids, _dev(img)).cpu().numpy().reshape(na, R).astype(np.float64)
    th = geometry.angles(na)
    img64 = img.astype(np.float64)
    for a, t in [(0, 0), (0, 2048), (1, 100), (2, 4095), (3, 1500), (4, 2047), (5, 3000),
                 (6, 777), (7, 3333)]:
        ref = ray_sum(img64, th[a], t, R)
        assert abs(fwd[a, t] - ref) <= 1e-6 * max(abs(ref), 1.0), (a, t, fwd[a, t], ref)
    v = rng.standard_normal((na, R)).astype(np.float32)
    back = s.backproject(ids, _dev(v)).cpu().numpy().astype(np.float64).reshape(N, N)
    lhs = float(np.sum(fwd * v.astype(np.float64)))
    rhs = float(np.sum(img64 * back))
    assert abs(lhs - rhs) <= 1e-6 * np.sqrt(np.sum(fwd ** 2) * np.sum(v.astype(np.float64) ** 2))
