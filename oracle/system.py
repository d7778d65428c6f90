"""Explicit rows of the projection matrix A, float64 CSR (test infrastructure only).

A has one row per (angle, ray), angle-major then ray, and one column per
pixel, row-major (column index i*N + j for row i / y, column j / x).  Rays
that miss the grid are all-zero rows and are kept, so block a occupies rows
a*R .. a*R+R-1.  Entries are the Joseph weights of ``geometry.joseph_weight``.

Sparse build: for each pixel the weight is non-zero only for rays with
|s_t - u| < h d, u = x_j cos + y_i sin.  With ray spacing h and d <= 1 these
are among t = floor(u/h + (R-1)/2) and that index + 1; the formula is
evaluated on both and zero entries are dropped.  ``dense_bruteforce``
evaluates the same formula on every (ray, pixel) pair and pins that
candidate rule on small grids.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import geometry as geo


def angle_rows(N: int, R: int, theta: float) -> sp.csr_matrix:
    """A_theta: the R x N^2 block of rays at one angle."""
    h = 2.0 / N
    xc = geo.pixel_centres(N)
    X = np.tile(xc, N)           # x_j of column i*N + j
    Y = np.repeat(xc, N)         # y_i of column i*N + j
    c, s = math.cos(theta), math.sin(theta)
    u = X * c + Y * s
    t0 = np.floor(u / h + (R - 1) / 2.0).astype(np.int64)
    rows, cols, vals = [], [], []
    pix = np.arange(N * N, dtype=np.int64)
    for t in (t0, t0 + 1):
        ok = (t >= 0) & (t < R)
        st = (t[ok] - (R - 1) / 2.0) * h
        w = geo.joseph_weight(theta, st, X[ok], Y[ok], h)
        nz = w > 0.0
        rows.append(t[ok][nz])
        cols.append(pix[ok][nz])
        vals.append(w[nz])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(R, N * N))


class Projector:
    """Per-angle CSR blocks of A, built on first use and cached."""

    def __init__(self, N: int, n_angles: int, R: int | None = None,
                 theta: np.ndarray | None = None):
        self.N = N
        self.n = N * N
        self.R = geo.n_rays(N) if R is None else R
        self.theta = geo.angles(n_angles) if theta is None else np.asarray(theta, np.float64)
        self.n_angles = self.theta.size
        self._cache: dict[int, sp.csr_matrix] = {}

    def angle(self, a: int) -> sp.csr_matrix:
        if a not in self._cache:
            self._cache[a] = angle_rows(self.N, self.R, float(self.theta[a]))
        return self._cache[a]

    def rows(self, angle_ids) -> sp.csr_matrix:
        """Stacked rows of the given angles, in the given order."""
        return sp.vstack([self.angle(int(a)) for a in angle_ids], format="csr")

    def full(self) -> sp.csr_matrix:
        return self.rows(range(self.n_angles))

    def forward(self, angle_ids, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, np.float64).reshape(-1)
        return np.concatenate([self.angle(int(a)) @ x for a in angle_ids])

    def back(self, angle_ids, v: np.ndarray) -> np.ndarray:
        v = np.asarray(v, np.float64).reshape(len(angle_ids), self.R)
        out = np.zeros(self.n)
        for k, a in enumerate(angle_ids):
            out += self.angle(int(a)).T @ v[k]
        return out


def dense_bruteforce(N: int, R: int, theta: np.ndarray) -> np.ndarray:
    """All (ray, pixel) weights by direct evaluation: [len(theta)*R, N*N]."""
    h = 2.0 / N
    xc = geo.pixel_centres(N)
    X = np.tile(xc, N)
    Y = np.repeat(xc, N)
    st = geo.ray_offsets(N, R)
    out = np.zeros((len(theta) * R, N * N))
    for k, th in enumerate(theta):
        for t in range(R):
            out[k * R + t] = geo.joseph_weight(float(th), st[t], X, Y, h)
    return out
