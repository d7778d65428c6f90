"""Pins of the oracle's projection matrix (CPU only).

The paper gives no discretisation of its parallel-beam ray tracer (sec. 4.3);
the oracle's Joseph weight is pinned here against facts that do not depend on
its code: exact line integrals of ellipses and Gaussians (Kak & Slaney's
closed forms), a brute-force evaluation of the weight on every (ray, pixel)
pair, exact chord lengths, and the band structure of A_theta A_theta^T.
"""
import math

import numpy as np
import pytest

import synth
from oracle import geometry as geo
from oracle import system


def test_rays_per_config():
    # ray counts of the five workloads: 91, 1449, 725, 363 rays
    assert [geo.n_rays(N) for N in (64, 1024, 512, 256)] == [91, 1449, 725, 363]
    for N in (64, 256, 512, 1024):
        assert geo.n_rays(N) == math.ceil(N * math.sqrt(2))


@pytest.mark.parametrize("N,na", [(8, 12), (13, 16)])
def test_sparse_build_equals_bruteforce(N, na):
    P = system.Projector(N, na)
    dense = system.dense_bruteforce(N, P.R, P.theta)
    # equal up to rounding: at an exact tie |s - u| = h d the weight is 0,
    # which direct evaluation may round to ~1e-17 (e.g. cos(pi/2) != 0)
    np.testing.assert_allclose(P.full().toarray(), dense, rtol=1e-13, atol=1e-15)


def test_each_pixel_hits_at_most_two_rays_per_angle():
    P = system.Projector(24, 24)   # includes 0, pi/4, pi/2, 3pi/4
    for a in range(P.n_angles):
        Aa = P.angle(a).tocsc()
        assert np.diff(Aa.indptr).max() <= 2


def test_same_angle_gram_is_tridiagonal():
    P = system.Projector(16, 24)
    for a in range(P.n_angles):
        G = (P.angle(a) @ P.angle(a).T).toarray()
        band = np.abs(np.subtract.outer(np.arange(P.R), np.arange(P.R))) <= 1
        assert np.all(G[~band] == 0.0)
        assert np.all(np.diag(G)[np.diag(G) > 0] > 0)


def test_interior_chords_are_exact():
    # theta = 0: vertical rays x = s through the interior cross all N rows
    # and carry exactly h per row -> chord length 2.  theta = pi/4: the
    # central ray is the square's diagonal, chord 2*sqrt(2).
    N = 32
    P = system.Projector(N, 4)
    ones = np.ones(N * N)
    p0 = P.angle(0) @ ones
    s = geo.ray_offsets(N, P.R)
    h = 2.0 / N
    inner = np.abs(s) <= 1.0 - h / 2
    np.testing.assert_allclose(p0[inner], 2.0, rtol=0, atol=1e-13)
    p45 = P.angle(1) @ ones
    assert abs(p45[(P.R - 1) // 2] - 2.0 * math.sqrt(2.0)) < 1e-12


def _radon_error(N, na, image_fn, radon_fn):
    P = system.Projector(N, na)
    xc = geo.pixel_centres(N)
    X, Y = np.meshgrid(xc, xc)
    x = image_fn(X, Y).reshape(-1)
    s = geo.ray_offsets(N, P.R)
    ref = radon_fn(P.theta[:, None], s[None, :])
    got = P.full() @ x
    return np.linalg.norm(got - ref.reshape(-1)) / np.linalg.norm(ref)


def test_gaussian_radon_second_order():
    # f = exp(-|p - c|^2 / (2 sig^2)): every line integral is
    # sig sqrt(2 pi) exp(-(s - c.n)^2 / (2 sig^2)).
    cx, cy, sig = 0.13, -0.21, 0.18

    def img(X, Y):
        return np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * sig ** 2))

    def rad(T, S):
        return sig * math.sqrt(2 * math.pi) * np.exp(-(S - cx * np.cos(T) - cy * np.sin(T)) ** 2 / (2 * sig ** 2))

    errs = [_radon_error(N, 30, img, rad) for N in (16, 32, 64)]
    assert errs[2] < 5e-3
    # second order: halving h divides the error by about 4
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_ellipse_radon_first_order():
    ells = synth.random_ellipses(6, seed=7)
    errs = []
    for N in (32, 64, 128):
        theta, s, _ = synth.scan_geometry(N, 45)
        P = system.Projector(N, 45)
        got = P.full() @ synth.rasterize(ells, N).reshape(-1)
        ref = synth.analytic_sinogram(ells, theta, s)
        errs.append(np.linalg.norm(got - ref.reshape(-1)) / np.linalg.norm(ref))
    assert errs[2] < 3e-2
    # point-sampled discontinuities: first order, error roughly halves
    assert errs[0] / errs[1] > 1.4 and errs[1] / errs[2] > 1.4


def test_symmetry_of_opposite_angles():
    # theta and theta + pi/2 swap the roles of x and y: the block at angle
    # a + n/2 applied to the transposed image equals the block at a applied to
    # the image with rays reversed (rotation of the square by 90 degrees).
    N, na = 20, 8
    P = system.Projector(N, na)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((N, N))
    for a in range(na // 2):
        p = P.angle(a) @ x.reshape(-1)
        # rotating the image by -90 deg maps angle theta to theta + pi/2
        q = P.angle(a + na // 2) @ np.rot90(x, k=-1).reshape(-1)
        np.testing.assert_allclose(q, p, rtol=1e-12, atol=1e-12)
