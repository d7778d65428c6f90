"""3D phantoms and parallel-beam projection data from random directions.

Acquisition convention (the 3D experiment of the paper: projection images of
a volume taken from directions drawn uniformly on the unit sphere):

* the volume covers [-1, 1]^3 with N^3 cubic voxels of side h = 2/N, stored
  [k][i][j] (z, y, x; row-major), voxel (k, i, j) centred at
  (x_j, y_i, z_k) = ((j, i, k) - (N-1)/2) h;
* a direction w (unit vector) has the detector basis
  e_u = (z x w) / |z x w|, e_v = w x e_u  (e_u = x, e_v = w x x when w is
  +-z), and a projection image of n_det x n_det pixels of side h, pixel
  (q, t) (row q along e_v, column t along e_u) centred at
  u_t = (t - (n_det-1)/2) h, v_q = (q - (n_det-1)/2) h; its ray is the line
  {u_t e_u + v_q e_v + tau w};
* data are stored [direction][q][t].

Everything is float64 numpy and seeded.  Nothing here evaluates the discrete
projector or the reconstruction step.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def random_directions(n: int, seed: int) -> np.ndarray:
    """n directions uniform on the unit sphere (normalised Gaussian vectors):
    [n, 3] float64 (x, y, z)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def detector_basis(w) -> tuple[np.ndarray, np.ndarray]:
    """(e_u, e_v) of the convention above."""
    w = np.asarray(w, np.float64)
    zx = np.array([-w[1], w[0], 0.0])           # z x w
    nz = math.hypot(w[0], w[1])
    eu = np.array([1.0, 0.0, 0.0]) if nz < 1e-12 else zx / nz
    ev = np.cross(w, eu)
    return eu, ev


@dataclass(frozen=True)
class Ellipsoid3:
    centre: tuple      # (x, y, z)
    axes: tuple        # semi-axes (a, b, c) along the columns of rot
    rot: tuple         # 3x3 rotation matrix, row-major (columns = axes)
    rho: float         # additive density


def _rotation(rng: np.random.Generator) -> np.ndarray:
    """A rotation drawn uniformly (normalised Gaussian quaternion)."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([
        [a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
        [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
        [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


def random_ellipsoids3(n: int, seed: int) -> list[Ellipsoid3]:
    """n random ellipsoids, arbitrarily rotated: centre at radius U[0, 0.5]
    in a uniform direction, semi-axes U[0.05, 0.4], density U[0.1, 1],
    redrawn until the ellipsoid lies inside the ball of radius 0.95 (so its
    projections fall inside every detector of side 2)."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        rad = rng.uniform(0.0, 0.5)
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        ax = rng.uniform(0.05, 0.4, 3)
        rot = _rotation(rng)
        rho = rng.uniform(0.1, 1.0)
        if rad + ax.max() <= 0.95:
            out.append(Ellipsoid3(tuple(rad * d), tuple(ax), tuple(rot.reshape(-1)), rho))
    return out


def _frame(e: Ellipsoid3):
    """Map p -> D^-1 Q^T (p - c): the ellipsoid becomes the unit ball."""
    Q = np.asarray(e.rot, np.float64).reshape(3, 3)
    return np.asarray(e.centre, np.float64), Q.T / np.asarray(e.axes, np.float64)[:, None]


def rasterize3(ells: list[Ellipsoid3], N: int, k0: int = 0, k1: int | None = None) -> np.ndarray:
    """Point-sample the phantom at voxel centres: [k1 - k0, N, N] float64
    (z slices k0 .. k1-1 of the [k][i][j] volume)."""
    k1 = N if k1 is None else k1
    h = 2.0 / N
    c = (np.arange(N, dtype=np.float64) - (N - 1) / 2.0) * h
    out = np.zeros((k1 - k0, N, N))
    for e in ells:
        cen, F = _frame(e)
        # only voxels within the ellipsoid's bounding ball can be inside it
        rad = max(e.axes)
        lo = np.searchsorted(c, cen - rad, side="left")
        hi = np.searchsorted(c, cen + rad, side="right")
        kl, kh = max(lo[2], k0), min(hi[2], k1)
        if kl >= kh or lo[0] >= hi[0] or lo[1] >= hi[1]:
            continue
        Z, Y, X = np.meshgrid(c[kl:kh], c[lo[1]:hi[1]], c[lo[0]:hi[0]], indexing="ij")
        P = np.stack([X, Y, Z], axis=-1) - cen
        yv = P @ F.T
        out[kl - k0:kh - k0, lo[1]:hi[1], lo[0]:hi[0]] += \
            e.rho * (np.einsum("...i,...i->...", yv, yv) <= 1.0)
    return out


def line_integrals(ells: list[Ellipsoid3], w, n_det: int, N: int) -> np.ndarray:
    """Exact integrals of the phantom along the n_det x n_det rays of
    direction w: [n_det, n_det] float64 ([q][t]).

    In the frame where an ellipsoid is the unit ball the ray is y0 + tau y1
    (y1 = F w), and the chord length in tau is 2 sqrt(disc) / |y1|^2 with
    disc = (y0.y1)^2 - |y1|^2 (|y0|^2 - 1); |w| = 1 makes tau arc length."""
    h = 2.0 / N
    eu, ev = detector_basis(w)
    s = (np.arange(n_det, dtype=np.float64) - (n_det - 1) / 2.0) * h
    V, U = np.meshgrid(s, s, indexing="ij")
    O = U[..., None] * eu + V[..., None] * ev
    out = np.zeros((n_det, n_det))
    w = np.asarray(w, np.float64)
    for e in ells:
        cen, F = _frame(e)
        y1 = F @ w
        y0 = (O - cen) @ F.T
        a = y1 @ y1
        bq = y0 @ y1
        disc = bq * bq - a * (np.einsum("...i,...i->...", y0, y0) - 1.0)
        out += e.rho * 2.0 * np.sqrt(np.clip(disc, 0.0, None)) / a
    return out


def make_problem3(N: int, n_dirs: int, n_det: int, n_ellipsoids: int, noise: float,
                  phantom_seed: int, dir_seed: int, noise_seed: int, dir_ids=None):
    """A 3D problem: (x_true[N, N, N], b[n_dirs, n_det, n_det], dirs[n_dirs, 3]).

    The noise is eps = noise * ||b_clean|| e / ||e|| with one Gaussian draw
    over the data of the listed directions (all of them by default); the
    data of other directions are left zero (for runs that visit only some
    directions).  float64."""
    ells = random_ellipsoids3(n_ellipsoids, phantom_seed)
    dirs = random_directions(n_dirs, dir_seed)
    ids = range(n_dirs) if dir_ids is None else [int(d) for d in dir_ids]
    b = np.zeros((n_dirs, n_det, n_det))
    for d in ids:
        b[d] = line_integrals(ells, dirs[d], n_det, N)
    clean_norm = np.linalg.norm(b)
    if noise > 0.0 and clean_norm > 0.0:
        rng = np.random.default_rng(noise_seed)
        e = np.zeros_like(b)
        for d in ids:
            e[d] = rng.standard_normal((n_det, n_det))
        b = b + noise * clean_norm * e / np.linalg.norm(e)
    return rasterize3(ells, N), b, dirs
