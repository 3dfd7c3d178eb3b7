"""Brute-force ray/pixel intersection lengths (test infrastructure only).

Clips every ray of a tiny geometry against every pixel square with the Liang-Barsky
parametric slab test. This is independent of the closed-form trapezoid used by the
oracle projectors and serves to pin them. A ray lying exactly on a pixel edge (only
possible for axis-aligned rays) is credited with half its clipped length, the mean of
the two one-sided limits.
"""
from __future__ import annotations

import numpy as np

from .core import EDGE_TIE, Geometry


def _clip(o, d, lo, hi):
    """Parametric interval of the line o + t d inside the closed slab [lo, hi] (arrays)."""
    if d == 0.0:
        inside = (o >= lo - EDGE_TIE) & (o <= hi + EDGE_TIE)
        on_edge = (np.abs(o - lo) <= EDGE_TIE) | (np.abs(o - hi) <= EDGE_TIE)
        t0 = np.where(inside, -np.inf, np.inf)
        t1 = np.where(inside, np.inf, -np.inf)
        return t0, t1, on_edge
    ta = (lo - o) / d
    tb = (hi - o) / d
    return np.minimum(ta, tb), np.maximum(ta, tb), np.zeros(np.shape(lo), dtype=bool)


def ray_pixel_lengths(g: Geometry, a: int, i: int) -> np.ndarray:
    """Lengths of ray (a, i) inside each pixel, as an n-vector."""
    N = g.N
    c, s = g.cos[a], g.sin[a]
    si = g.s[i]
    ox, oy = si * c, si * s          # a point on the line <p, omega> = s_i
    dx, dy = -s, c                   # unit direction along the line
    cols = np.arange(N, dtype=np.float64)
    x0 = np.tile(cols - N / 2, N)
    y0 = np.repeat(cols - N / 2, N)
    tx0, tx1, ex = _clip(ox, dx, x0, x0 + 1.0)
    ty0, ty1, ey = _clip(oy, dy, y0, y0 + 1.0)
    t0 = np.maximum(tx0, ty0)
    t1 = np.minimum(tx1, ty1)
    length = np.where(t1 > t0, t1 - t0, 0.0)
    length = np.where(np.isfinite(length), length, 0.0)
    return np.where(ex | ey, 0.5 * length, length)


def brute_force_matrix(g: Geometry) -> np.ndarray:
    """Dense m x n matrix of intersection lengths by clipping."""
    A = np.zeros((g.m, g.n))
    for a in range(g.n_ang):
        for i in range(g.n_det):
            A[a * g.n_det + i] = ray_pixel_lengths(g, a, i)
    return A


def chord_length_in_square(g: Geometry, a: int, i: int) -> float:
    """Length of ray (a, i) inside the whole image square [-N/2, N/2]^2, by clipping;
    half of it when the ray runs along the square's boundary."""
    N = g.N
    c, s = g.cos[a], g.sin[a]
    si = g.s[i]
    ox, oy = si * c, si * s
    dx, dy = -s, c
    lo = np.array([-N / 2])
    hi = np.array([N / 2])
    tx0, tx1, ex = _clip(ox, dx, lo, hi)
    ty0, ty1, ey = _clip(oy, dy, lo, hi)
    t0 = max(tx0[0], ty0[0])
    t1 = min(tx1[0], ty1[0])
    L = t1 - t0 if (t1 > t0 and np.isfinite(t1 - t0)) else 0.0
    return 0.5 * L if (ex[0] or ey[0]) else L
