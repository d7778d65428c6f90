"""Scan geometry and the Joseph weight, float64 (test infrastructure only).

The paper models the tomography problems with a parallel-beam ray-tracing
matrix (sec. 4.3, 2D limited-angle and 3D streaming experiments) and notes
that blocks of A may be produced by function evaluations instead of being
stored (sec. 4.2).  It does not fix the discretisation; this oracle takes
Joseph's method, written as one closed form for every (ray, pixel) pair:

    a[(theta, s), (i, j)] = (h/d) * max(0, 1 - |s - x_j cos(theta) - y_i sin(theta)| / (h d)),
    d = max(|cos(theta)|, |sin(theta)|),

with pixel centres x_j = (j-(N-1)/2) h, y_i = (i-(N-1)/2) h, h = 2/N, ray
offsets s_t = (t-(R-1)/2) h, R = 2 floor(N/sqrt 2) + 1 and theta_a = a pi / n_angles.
Along the major axis of a ray this is linear interpolation between the two
nearest pixel centres, times the path length h/d per row (or column) step.

Pins: analytic ellipse / Gaussian line integrals (discretisation order),
brute-force evaluation of the formula on every pair, row-sum identity.
"""
from __future__ import annotations

import math

import numpy as np


def n_rays(N: int) -> int:
    return 2 * int(math.floor(N / math.sqrt(2.0))) + 1


def angles(n_angles: int) -> np.ndarray:
    return np.arange(n_angles, dtype=np.float64) * (math.pi / n_angles)


def pixel_centres(N: int) -> np.ndarray:
    h = 2.0 / N
    return (np.arange(N, dtype=np.float64) - (N - 1) / 2.0) * h


def ray_offsets(N: int, R: int) -> np.ndarray:
    h = 2.0 / N
    return (np.arange(R, dtype=np.float64) - (R - 1) / 2.0) * h


def joseph_weight(theta: float, s, x, y, h: float):
    """The closed-form weight of ray (theta, s) on the pixel centred at (x, y)."""
    c, sn = math.cos(theta), math.sin(theta)
    d = max(abs(c), abs(sn))
    return (h / d) * np.maximum(0.0, 1.0 - np.abs(s - x * c - y * sn) / (h * d))
