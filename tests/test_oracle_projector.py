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


@pytest.mark.parametrize("N,na,ids", [
    (16, 12, [0, 3, 6, 9]),
    (21, 30, [29, 0, 7, 7, 15, 22]),          # any order, a repeated angle
    (64, 90, list(range(0, 90, 11))),
    (33, 7, [6, 2, 4]),
])
def test_back_is_adjoint_of_forward(N, na, ids):
    # <A_ids x, y> = <x, A_ids^T y> for random x, y: pins the layout of the
    # rays ([len(ids)][R], angle-major) in Projector.back against the forward
    # projector, which the Radon pins above fix.
    P = system.Projector(N, na)
    rng = np.random.default_rng(N * 1000 + na)
    x = rng.standard_normal(N * N)
    y = rng.standard_normal(len(ids) * P.R)
    lhs = float(P.forward(ids, x) @ y)
    rhs = float(x @ P.back(ids, y))
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(P.forward(ids, x)) * np.linalg.norm(y)


def test_back_equals_bruteforce_transpose():
    # A^T y with every (ray, pixel) weight evaluated directly
    N, na = 12, 10
    P = system.Projector(N, na)
    ids = [9, 1, 4]
    dense = system.dense_bruteforce(N, P.R, P.theta[ids])
    y = np.random.default_rng(1).standard_normal(len(ids) * P.R)
    np.testing.assert_allclose(P.back(ids, y), dense.T @ y, rtol=0, atol=1e-13)


def test_back_of_ones_at_zero_and_right_angle_is_h():
    # theta = 0 (rays x = s) and pi/2 (rays y = s): d = 1 and the rays are one
    # pixel apart, so the hat weights of a pixel sum to 1 (linear
    # interpolation is a partition of unity) and every pixel whose centre lies
    # between two rays of the detector gets exactly h from a row of ones.
    N = 24
    P = system.Projector(N, 2)          # angles 0 and pi/2
    h = 2.0 / N
    for a in (0, 1):
        out = P.back([a], np.ones(P.R)).reshape(N, N)
        np.testing.assert_allclose(out, h, rtol=0, atol=1e-15)
    # one ray on: its weights are the hat function of the distance to it
    v = np.zeros(P.R)
    t = (P.R - 1) // 2 + 3
    v[t] = 1.0
    out = P.back([0], v).reshape(N, N)
    xc = geo.pixel_centres(N)
    s_t = geo.ray_offsets(N, P.R)[t]
    ref = h * np.maximum(0.0, 1.0 - np.abs(s_t - xc) / h)
    np.testing.assert_allclose(out, np.tile(ref, (N, 1)), rtol=0, atol=1e-15)
