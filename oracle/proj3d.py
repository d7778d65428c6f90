"""Explicit rows of the 3D parallel-beam projection matrix, float64 CSR (test
infrastructure only).

The paper's 3D experiment (sec. 4.3, three-dimensional streaming tomography)
takes projection images of a volume from directions drawn uniformly on the
unit sphere, one image being one block of rows.  Conventions (restated from
the acquisition geometry, independently of the GPU path):

* volume [-1, 1]^3, N^3 voxels of side h = 2/N, stored [k][i][j] = (z, y, x),
  voxel centre c = ((j, i, k) - (N-1)/2) h, column index (k N + i) N + j;
* direction w, detector basis e_u = (z x w)/|z x w| (x when w = +-z),
  e_v = w x e_u; an n_det x n_det image with pixel (q, t) on the ray
  {u_t e_u + v_q e_v + tau w}, u_t = (t - (n_det-1)/2) h, v_q likewise; rows
  are direction-major, then q, then t.

Weights (Joseph's method in 3D, along the major axis): with m the axis of
the largest |w_m| (the first one on a tie) and a < b the other two, a ray
meets the plane of a voxel's centre, x_m = c_m, in one point P; the weight is

    a(ray, voxel) = (h / |w_m|) L((P_a - c_a)/h) L((P_b - c_b)/h),
    L(s) = max(0, 1 - |s|),

i.e. bilinear interpolation between the four voxel centres around P in each
plane, times the ray's length per plane.  ``dense_bruteforce`` evaluates
exactly this on every (ray, voxel) pair.  ``dir_rows`` uses that P - c is
linear in the detector offset between the ray and the voxel's own ray,
(du, dv) = (u - c.e_u, v - c.e_v) / h:

    (P - c)_x / h = (e_u[x] - e_u[m] w_x / w_m) du + (e_v[x] - e_v[m] w_x / w_m) dv,

and that only rays with |du| < |e_u[a]| + |e_u[b]| <= sqrt(2) (dv likewise)
can have a non-zero weight, so each voxel meets at most 4 x 4 candidate rays
around its own.  The brute force pins that enumeration on small volumes.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def basis(w) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(w, e_u, e_v) as float64 arrays."""
    w = np.asarray(w, np.float64).reshape(3)
    nz = math.hypot(w[0], w[1])
    eu = np.array([1.0, 0.0, 0.0]) if nz < 1e-12 else np.array([-w[1], w[0], 0.0]) / nz
    ev = np.cross(w, eu)
    return w, eu, ev


def major_axis(w) -> tuple[int, int, int]:
    """(m, a, b): the axis of the largest |w_m| (first on a tie), then the
    other two in increasing order."""
    aw = np.abs(np.asarray(w, np.float64))
    m = int(np.argmax(aw))
    a, b = [k for k in range(3) if k != m]
    return m, a, b


def _centres(N: int) -> np.ndarray:
    return (np.arange(N, dtype=np.float64) - (N - 1) / 2.0) * (2.0 / N)


def _tent(s):
    return np.maximum(0.0, 1.0 - np.abs(s))


def dir_rows(N: int, n_det: int, w, kslab: int = 8) -> sp.csr_matrix:
    """A_w: the n_det^2 x N^3 block of one direction (candidate enumeration)."""
    h = 2.0 / N
    w, eu, ev = basis(w)
    m, a, b = major_axis(w)
    La = (eu[a] - eu[m] * w[a] / w[m], ev[a] - ev[m] * w[a] / w[m])
    Lb = (eu[b] - eu[m] * w[b] / w[m], ev[b] - ev[m] * w[b] / w[m])
    scale = h / abs(w[m])
    c = _centres(N)
    off = (n_det - 1) / 2.0
    rows, cols, vals = [], [], []
    for k0 in range(0, N, kslab):
        k1 = min(N, k0 + kslab)
        Z, Y, X = np.meshgrid(c[k0:k1], c, c, indexing="ij")
        col = np.arange(k0 * N * N, k1 * N * N, dtype=np.int64)
        fu = ((X * eu[0] + Y * eu[1] + Z * eu[2]) / h + off).reshape(-1)
        fv = ((X * ev[0] + Y * ev[1] + Z * ev[2]) / h + off).reshape(-1)
        tu, tv = np.floor(fu), np.floor(fv)
        for ot in (-1, 0, 1, 2):
            t = tu + ot
            du = t - fu
            for oq in (-1, 0, 1, 2):
                q = tv + oq
                dv = q - fv
                wgt = scale * _tent(La[0] * du + La[1] * dv) * _tent(Lb[0] * du + Lb[1] * dv)
                ok = (wgt > 0.0) & (t >= 0) & (t < n_det) & (q >= 0) & (q < n_det)
                rows.append((q[ok] * n_det + t[ok]).astype(np.int64))
                cols.append(col[ok])
                vals.append(wgt[ok])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n_det * n_det, N ** 3))


def dense_bruteforce(N: int, n_det: int, dirs) -> np.ndarray:
    """Every (ray, voxel) weight by the plane-intersection definition:
    [len(dirs) * n_det^2, N^3]."""
    h = 2.0 / N
    c = _centres(N)
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    C = np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1)   # [N^3, 3]
    s = (np.arange(n_det, dtype=np.float64) - (n_det - 1) / 2.0) * h
    dirs = np.asarray(dirs, np.float64).reshape(-1, 3)
    out = np.zeros((len(dirs) * n_det * n_det, N ** 3))
    for d, wv in enumerate(dirs):
        w, eu, ev = basis(wv)
        m, a, b = major_axis(w)
        for q in range(n_det):
            for t in range(n_det):
                o = s[t] * eu + s[q] * ev
                tau = (C[:, m] - o[m]) / w[m]
                P = o[None, :] + tau[:, None] * w[None, :]
                wa = _tent((P[:, a] - C[:, a]) / h)
                wb = _tent((P[:, b] - C[:, b]) / h)
                out[(d * n_det + q) * n_det + t] = (h / abs(w[m])) * wa * wb
    return out


def single_ray(N: int, n_det: int, w, q: int, t: int, x: np.ndarray) -> float:
    """(A x) on one ray, from the definition: in every plane x_m = c_m the
    4 x 4 voxels around the ray's crossing point, weights evaluated
    directly (for checks at sizes where no CSR block is built)."""
    h = 2.0 / N
    w, eu, ev = basis(w)
    m, a, b = major_axis(w)
    c = _centres(N)
    o = (t - (n_det - 1) / 2.0) * h * eu + (q - (n_det - 1) / 2.0) * h * ev
    x = np.asarray(x).reshape(N, N, N)                 # [z][y][x], read entry by entry
    total = 0.0
    for km in range(N):
        tau = (c[km] - o[m]) / w[m]
        P = o + tau * w
        ia0 = int(math.floor(P[a] / h + (N - 1) / 2.0))
        ib0 = int(math.floor(P[b] / h + (N - 1) / 2.0))
        for ia in range(ia0 - 1, ia0 + 3):
            for ib in range(ib0 - 1, ib0 + 3):
                if not (0 <= ia < N and 0 <= ib < N):
                    continue
                wgt = (h / abs(w[m])) * _tent((P[a] - c[ia]) / h) * _tent((P[b] - c[ib]) / h)
                if wgt == 0.0:
                    continue
                idx = [0, 0, 0]
                idx[m], idx[a], idx[b] = km, ia, ib
                total += wgt * float(x[idx[2], idx[1], idx[0]])
    return total


class Projector3D:
    """Per-direction CSR blocks of A, built on first use and cached.  Exposes
    the interface of the 2D ``Projector`` (``R`` = rows per block = n_det^2,
    ``n_angles`` = directions, ``n`` = N^3), so the slimLS iteration runs on
    it unchanged."""

    def __init__(self, N: int, dirs, n_det: int | None = None):
        self.N = N
        self.n = N ** 3
        self.dirs = np.asarray(dirs, np.float64).reshape(-1, 3)
        self.n_angles = len(self.dirs)
        self.n_det = N if n_det is None else int(n_det)
        self.R = self.n_det ** 2
        self._cache: dict[int, sp.csr_matrix] = {}

    def angle(self, d: int) -> sp.csr_matrix:
        if d not in self._cache:
            self._cache[d] = dir_rows(self.N, self.n_det, self.dirs[d])
        return self._cache[d]

    def rows(self, ids) -> sp.csr_matrix:
        return sp.vstack([self.angle(int(d)) for d in ids], format="csr")

    def forward(self, ids, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, np.float64).reshape(-1)
        return np.concatenate([self.angle(int(d)) @ x for d in ids])

    def back(self, ids, v: np.ndarray) -> np.ndarray:
        v = np.asarray(v, np.float64).reshape(len(ids), self.R)
        out = np.zeros(self.n)
        for k, d in enumerate(ids):
            out += self.angle(int(d)).T @ v[k]
        return out
