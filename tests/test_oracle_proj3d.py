"""Pins of the 3D parallel-beam oracle (oracle/proj3d.py), independent of any
implementation: the per-voxel candidate enumeration against the definition
evaluated on every (ray, voxel) pair, exact sums for axis-aligned and
interior rays, the mirror symmetry of opposite directions, analytic line
integrals of a Gaussian blob (second order in h) and of ellipsoids (first
order: point-sampled edges), the back-projector as the transpose, and the
slimLS iteration on 3D blocks against its primal form and the Tikhonov
solution (full memory)."""
import math

import numpy as np
import pytest

import synth
from oracle import proj3d, slimls

DIRS = np.array([
    [0.0, 0.0, 1.0], [0.0, 0.0, -1.0], [1.0, 0.0, 0.0], [0.0, -1.0, 0.0],
    [1e-9, 2e-9, 1.0],                      # near the z axis
    [1.0, 1.0, 1.0], [1.0, 1.0, 0.0],       # ties between |w| components
    [1.0, -2.0, 0.3], [-0.2, 0.5, -0.9], [0.7, 0.1, -0.4],
])
DIRS = DIRS / np.linalg.norm(DIRS, axis=1, keepdims=True)


@pytest.mark.parametrize("N,n_det", [(5, 5), (6, 9), (7, 4)])
def test_candidate_enumeration_equals_definition(N, n_det):
    dirs = np.concatenate([DIRS, synth.random_directions(6, 11)])
    dense = proj3d.dense_bruteforce(N, n_det, dirs)
    for d, w in enumerate(dirs):
        A = proj3d.dir_rows(N, n_det, w).toarray()
        ref = dense[d * n_det * n_det:(d + 1) * n_det * n_det]
        np.testing.assert_allclose(A, ref, rtol=1e-13, atol=1e-15)
        assert np.count_nonzero(ref) > 0


def test_axis_aligned_rays_sum_voxel_columns():
    N = 8
    h = 2.0 / N
    x = np.random.default_rng(3).standard_normal((N, N, N))       # [z][y][x]
    P = proj3d.Projector3D(N, [[0, 0, 1], [1, 0, 0]])
    # w = z: e_u = x, e_v = y, ray (q, t) is voxel column (., q, t)
    np.testing.assert_allclose(P.forward([0], x).reshape(N, N), h * x.sum(axis=0), rtol=1e-13)
    # w = x: e_u = z x x = y, e_v = x x y = z, ray (q, t) is voxel row (q, t, .)
    np.testing.assert_allclose(P.forward([1], x).reshape(N, N), h * x.sum(axis=2), rtol=1e-13)


def test_interior_rays_have_the_chord_length():
    """A ray whose crossing point lies inside the grid of voxel centres in
    every plane x_m = c_m sums weights N h / |w_m| = 2 / |w_m| (bilinear
    weights sum to one in each plane); no ray exceeds it."""
    N, n_det = 16, 16
    h = 2.0 / N
    for w in synth.random_directions(8, 5):
        w, eu, ev = proj3d.basis(w)
        m, a, b = proj3d.major_axis(w)
        A = proj3d.dir_rows(N, n_det, w)
        sums = np.asarray(A.sum(axis=1)).reshape(n_det, n_det)
        assert sums.max() <= 2.0 / abs(w[m]) * (1 + 1e-13)
        c = (np.arange(N) - (N - 1) / 2.0) * h
        s = (np.arange(n_det) - (n_det - 1) / 2.0) * h
        lo, hi = c[0], c[-1]
        n_in = 0
        for q in range(n_det):
            for t in range(n_det):
                o = s[t] * eu + s[q] * ev
                P = o[None, :] + ((c - o[m]) / w[m])[:, None] * w[None, :]
                if np.all((P[:, [a, b]] >= lo) & (P[:, [a, b]] <= hi)):
                    n_in += 1
                    assert abs(sums[q, t] - 2.0 / abs(w[m])) <= 1e-12 * sums[q, t]
        assert n_in > 0


def test_opposite_directions_mirror_the_detector():
    """-w gives e_u -> -e_u and the same e_v: the image is mirrored in t."""
    N = 12
    x = np.random.default_rng(8).uniform(size=(N, N, N))
    for w in synth.random_directions(4, 9):
        P = proj3d.Projector3D(N, [w, -w])
        a = P.forward([0], x).reshape(N, N)
        b = P.forward([1], x).reshape(N, N)
        np.testing.assert_allclose(b, a[:, ::-1], rtol=1e-12, atol=1e-14)


def _gauss(N, cen, sig):
    c = (np.arange(N) - (N - 1) / 2.0) * (2.0 / N)
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    r2 = (X - cen[0]) ** 2 + (Y - cen[1]) ** 2 + (Z - cen[2]) ** 2
    return np.exp(-r2 / (2 * sig * sig))


def test_gaussian_line_integrals_second_order():
    """Along any line at distance d from the centre the integral of
    exp(-|p - c|^2 / 2 s^2) is s sqrt(2 pi) exp(-d^2 / 2 s^2)."""
    cen, sig = np.array([0.1, -0.05, 0.07]), 0.2
    dirs = synth.random_directions(2, 21)
    errs = []
    for N in (16, 32, 64):
        h = 2.0 / N
        x = _gauss(N, cen, sig)
        e = []
        for w in dirs:
            w, eu, ev = proj3d.basis(w)
            s = (np.arange(N) - (N - 1) / 2.0) * h
            V, U = np.meshgrid(s, s, indexing="ij")
            O = U[..., None] * eu + V[..., None] * ev
            rel = O - cen
            d2 = np.einsum("...i,...i->...", rel, rel) - (rel @ w) ** 2
            exact = sig * math.sqrt(2 * math.pi) * np.exp(-d2 / (2 * sig * sig))
            got = (proj3d.dir_rows(N, N, w) @ x.reshape(-1)).reshape(N, N)
            e.append(np.linalg.norm(got - exact) / np.linalg.norm(exact))
        errs.append(max(e))
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs
    assert errs[2] < 5e-3


def test_ellipsoid_line_integrals_converge():
    ells = synth.random_ellipsoids3(6, 17)
    w = synth.random_directions(1, 23)[0]
    errs = []
    for N in (16, 32, 64):
        x = synth.rasterize3(ells, N)
        exact = synth.line_integrals(ells, w, N, N)
        got = (proj3d.dir_rows(N, N, w) @ x.reshape(-1)).reshape(N, N)
        errs.append(np.linalg.norm(got - exact) / np.linalg.norm(exact))
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[0] / errs[2] > 2.0 and errs[2] < 0.08, errs


def test_single_ray_and_back_projector_follow_the_definition():
    N, n_det = 6, 8
    dirs = np.concatenate([DIRS[[0, 5, 7]], synth.random_directions(2, 4)])
    dense = proj3d.dense_bruteforce(N, n_det, dirs)
    P = proj3d.Projector3D(N, dirs, n_det)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(N ** 3)
    v = rng.standard_normal(len(dirs) * n_det * n_det)
    ids = list(range(len(dirs)))
    np.testing.assert_allclose(P.back(ids, v), dense.T @ v, rtol=1e-12, atol=1e-13)
    ref = dense @ x
    for d in ids:
        for q, t in ((0, 0), (3, 4), (n_det - 1, 2), (5, n_det - 1)):
            got = proj3d.single_ray(N, n_det, dirs[d], q, t, x)
            assert abs(got - ref[(d * n_det + q) * n_det + t]) <= 1e-12 * (1 + abs(got))


def _tomo(N, n_dirs, g, r, lam, seed, **kw):
    x_true, b, dirs = synth.make_problem3(N, n_dirs, N, 4, 0.01, seed, seed + 1, seed + 2)
    P = proj3d.Projector3D(N, dirs)
    return P, b.reshape(n_dirs, -1), x_true, slimls.Tomo(P, b.reshape(n_dirs, -1), g, r, lam,
                                                          x_true=x_true, **kw)


@pytest.mark.parametrize("r", [0, 2])
def test_slimls_on_3d_blocks_dual_equals_primal(r):
    N, nd, lam = 5, 6, 1e-2
    _, b, x_true, Td = _tomo(N, nd, 1, r, lam, 31)
    _, _, _, Tp = _tomo(N, nd, 1, r, lam, 31, form="primal")
    for beta in (3, 0, 5, 1, 4, 2):
        Td.step(beta)
        Tp.step(beta)
        np.testing.assert_allclose(Td.x, Tp.x, rtol=1e-10, atol=1e-12)


def test_slimls_3d_full_memory_epoch_is_tikhonov():
    N, nd, lam = 5, 4, 5e-3
    P, b, _, T = _tomo(N, nd, 1, nd - 1, lam, 41)
    for beta in (2, 0, 3, 1):
        T.step(beta)
    A = P.rows(range(nd)).toarray()
    x_tik = np.linalg.solve(A.T @ A + lam * np.eye(N ** 3), A.T @ b.reshape(-1))
    np.testing.assert_allclose(T.x, x_tik, rtol=1e-9, atol=1e-11)
