"""Random ellipse phantoms, their exact sinograms, noise and block schedules.

Conventions (the acquisition geometry of a 2D parallel-beam scan):

* the image covers [-1, 1]^2 with N x N square pixels of side h = 2/N; pixel
  (i, j) (row i, column j, row-major) has centre x_j = (j - (N-1)/2) h,
  y_i = (i - (N-1)/2) h;
* projection angles are theta_a = a*pi/n_angles, a = 0..n_angles-1 (uniform
  on [0, pi));
* a projection has R = 2*floor(N/sqrt(2)) + 1 rays with spacing h, centred on
  the rotation axis: s_t = (t - (R-1)/2) h; ray (theta, s) is the line
  x cos(theta) + y sin(theta) = s.

Everything is float64 numpy and seeded.  Nothing here evaluates the discrete
projector or the reconstruction step.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def n_rays_for(N: int) -> int:
    """Number of detector rays R = 2*floor(N/sqrt 2) + 1 (= ceil(N*sqrt 2))."""
    return 2 * int(math.floor(N / math.sqrt(2.0))) + 1


def scan_geometry(N: int, n_angles: int, n_rays: int | None = None):
    """Return (theta[n_angles], s[n_rays], h) of the scan, float64."""
    R = n_rays_for(N) if n_rays is None else int(n_rays)
    h = 2.0 / N
    theta = np.arange(n_angles, dtype=np.float64) * (np.pi / n_angles)
    s = (np.arange(R, dtype=np.float64) - (R - 1) / 2.0) * h
    return theta, s, h


@dataclass(frozen=True)
class Ellipse:
    cx: float
    cy: float
    a: float      # semi-axis along the rotated x' direction
    b: float      # semi-axis along the rotated y' direction
    phi: float    # rotation of the x' axis from +x, radians
    rho: float    # additive density


def _draw_ellipse(rng: np.random.Generator) -> Ellipse:
    # centre radius U[0, 0.5], polar angle U[0, 2pi); semi-axes U[0.05, 0.4];
    # rotation U[0, pi); density U[0.1, 1]; redraw until the ellipse lies
    # inside the disc of radius 0.95 (so it is inside every projection).
    while True:
        rad = rng.uniform(0.0, 0.5)
        ang = rng.uniform(0.0, 2.0 * np.pi)
        a = rng.uniform(0.05, 0.4)
        b = rng.uniform(0.05, 0.4)
        phi = rng.uniform(0.0, np.pi)
        rho = rng.uniform(0.1, 1.0)
        if rad + max(a, b) <= 0.95:
            return Ellipse(rad * np.cos(ang), rad * np.sin(ang), a, b, phi, rho)


def random_ellipses(n: int, seed: int) -> list[Ellipse]:
    """n random ellipses from numpy's PCG64 stream ``seed``."""
    rng = np.random.default_rng(seed)
    return [_draw_ellipse(rng) for _ in range(n)]


@dataclass(frozen=True)
class Ellipsoid:
    cx: float
    cy: float
    cz: float
    a: float
    b: float
    c: float      # semi-axis along z (rotation is about z only)
    phi: float
    rho: float


def random_ellipsoids(n: int, seed: int) -> list[Ellipsoid]:
    """n random ellipsoids in [-1,1]^3, rotated about z only, so every z-slice
    is an ellipse.  Same laws as the 2D ellipses, with c ~ U[0.05, 0.4] and
    cz ~ U[-0.5, 0.5]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        e = _draw_ellipse(rng)
        c = rng.uniform(0.05, 0.4)
        cz = rng.uniform(-0.5, 0.5)
        out.append(Ellipsoid(e.cx, e.cy, cz, e.a, e.b, c, e.phi, e.rho))
    return out


def ellipsoid_slice(ells: list[Ellipsoid], z: float) -> list[Ellipse]:
    """Cross-sections of ellipsoids with the plane at height z."""
    out = []
    for e in ells:
        q = (z - e.cz) / e.c
        if abs(q) < 1.0:
            f = math.sqrt(1.0 - q * q)
            out.append(Ellipse(e.cx, e.cy, e.a * f, e.b * f, e.phi, e.rho))
    return out


def rasterize(ells: list[Ellipse], N: int) -> np.ndarray:
    """Point-sample the phantom at pixel centres: [N, N] float64, row i = y."""
    h = 2.0 / N
    c = (np.arange(N, dtype=np.float64) - (N - 1) / 2.0) * h
    X, Y = np.meshgrid(c, c)  # X[i, j] = x_j, Y[i, j] = y_i
    img = np.zeros((N, N), dtype=np.float64)
    for e in ells:
        cp, sp = np.cos(e.phi), np.sin(e.phi)
        dx, dy = X - e.cx, Y - e.cy
        u = (dx * cp + dy * sp) / e.a
        v = (-dx * sp + dy * cp) / e.b
        img += e.rho * ((u * u + v * v) <= 1.0)
    return img


def analytic_sinogram(ells: list[Ellipse], theta: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Exact line integrals of the phantom: [n_angles, n_rays] float64.

    For an ellipse with semi-axes a, b rotated by phi and centred at c, the
    integral along x cos(t) + y sin(t) = s is 2 rho a b sqrt(a_t^2 - s'^2) / a_t^2
    for |s'| < a_t, with s' = s - (cx cos t + cy sin t) and
    a_t^2 = a^2 cos^2(t - phi) + b^2 sin^2(t - phi) (Kak & Slaney, ch. 3).
    """
    T = theta[:, None]
    S = s[None, :]
    out = np.zeros((theta.size, s.size), dtype=np.float64)
    for e in ells:
        at2 = (e.a * np.cos(T - e.phi)) ** 2 + (e.b * np.sin(T - e.phi)) ** 2
        sp = S - (e.cx * np.cos(T) + e.cy * np.sin(T))
        q = np.clip(at2 - sp * sp, 0.0, None)
        out += 2.0 * e.rho * e.a * e.b * np.sqrt(q) / at2
    return out


def add_noise(clean: np.ndarray, level: float, seed: int) -> np.ndarray:
    """clean + eps with eps = level * ||clean|| * e / ||e||, e ~ N(0, I).

    One draw over every entry (rays that miss the phantom included)."""
    if level == 0.0:
        return clean.copy()
    rng = np.random.default_rng(seed)
    e = rng.standard_normal(clean.shape)
    return clean + level * np.linalg.norm(clean) * e / np.linalg.norm(e)


def make_slice_problem(N: int, n_angles: int, n_ellipses: int, noise: float,
                       phantom_seed: int, noise_seed: int):
    """One 2D problem: (x_true[N,N], b[n_angles, R], b_clean) as float64."""
    theta, s, _ = scan_geometry(N, n_angles)
    ells = random_ellipses(n_ellipses, phantom_seed)
    x_true = rasterize(ells, N)
    clean = analytic_sinogram(ells, theta, s)
    return x_true, add_noise(clean, noise, noise_seed), clean


def volume_slice(N: int, n_slices: int, k: int, n_angles: int, n_ellipsoids: int,
                 noise: float, phantom_seed: int, noise_seed: int, ells=None):
    """Slice k of the volume of ``make_volume_problem``: (x_true[N, N],
    b[n_angles, R]) float64.  The slice sits at z_k = (k - (B-1)/2) * 2/B and
    gets noise seed ``noise_seed + k``; an empty slice has b = 0."""
    theta, s, _ = scan_geometry(N, n_angles)
    if ells is None:
        ells = random_ellipsoids(n_ellipsoids, phantom_seed)
    z = (k - (n_slices - 1) / 2.0) * (2.0 / n_slices)
    sl = ellipsoid_slice(ells, z)
    clean = analytic_sinogram(sl, theta, s)
    b = add_noise(clean, noise, noise_seed + k) if np.any(clean) else clean
    return rasterize(sl, N), b


def make_volume_problem(N: int, n_slices: int, n_angles: int, n_ellipsoids: int,
                        noise: float, phantom_seed: int, noise_seed: int):
    """Independent z-slices of one random ellipsoid volume.

    Returns (x_true[B, N, N], b[B, n_angles, R]) float64; slice k is
    ``volume_slice(..., k, ...)``."""
    ells = random_ellipsoids(n_ellipsoids, phantom_seed)
    R = n_rays_for(N)
    xs = np.zeros((n_slices, N, N), dtype=np.float64)
    bs = np.zeros((n_slices, n_angles, R), dtype=np.float64)
    for k in range(n_slices):
        xs[k], bs[k] = volume_slice(N, n_slices, k, n_angles, n_ellipsoids, noise,
                                    phantom_seed, noise_seed, ells)
    return xs, bs


def schedule(n_blocks: int, epochs: int, seed: int) -> np.ndarray:
    """Random-cyclic block order: one permutation of the blocks per epoch,
    int32 [epochs * n_blocks]."""
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.permutation(n_blocks) for _ in range(epochs)]).astype(np.int32)
