"""Brute-force projector matrices of tiny geometries (test infrastructure only).

* Line model: every ray is clipped against every pixel square with the Liang-Barsky
  parametric slab test. A ray lying exactly on a pixel edge (only possible for
  axis-aligned rays) is credited with half its clipped length, the mean of the two
  one-sided limits.
* Strip model: every pixel square is clipped (Sutherland-Hodgman) against the two
  half-planes bounding the strip of width ds around the ray, and the area of the
  remaining polygon is taken by the shoelace formula.
* Joseph's model: the ray's crossing of each row (or column) centre line, the two
  pixels of that row bracketing it, linear interpolation weights times the ray's
  length per row.

None of these uses the closed forms of the oracle projectors; they serve to pin them.
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


def _clip_halfplane(poly, nx, ny, c):
    """Part of polygon `poly` (list of (x, y)) with nx*x + ny*y <= c."""
    out = []
    n = len(poly)
    for k in range(n):
        P, Q = poly[k], poly[(k + 1) % n]
        fp = nx * P[0] + ny * P[1] - c
        fq = nx * Q[0] + ny * Q[1] - c
        if fp <= 0.0:
            out.append(P)
        if (fp < 0.0 < fq) or (fq < 0.0 < fp):
            r = fp / (fp - fq)
            out.append((P[0] + r * (Q[0] - P[0]), P[1] + r * (Q[1] - P[1])))
    return out


def _area(poly):
    if len(poly) < 3:
        return 0.0
    a = 0.0
    for k in range(len(poly)):
        x0, y0 = poly[k]
        x1, y1 = poly[(k + 1) % len(poly)]
        a += x0 * y1 - x1 * y0
    return 0.5 * abs(a)


def strip_area_matrix(g: Geometry) -> np.ndarray:
    """Dense m x n strip-model matrix: area of (pixel square) and (strip of width ds
    centred on the ray), divided by ds."""
    N = g.N
    A = np.zeros((g.m, g.n))
    for a in range(g.n_ang):
        c, s = g.cos[a], g.sin[a]
        for i in range(g.n_det):
            lo, hi = g.s[i] - 0.5 * g.ds, g.s[i] + 0.5 * g.ds
            for j in range(g.n):
                r, cc = divmod(j, N)
                x0, y0 = cc - N / 2, r - N / 2
                sq = [(x0, y0), (x0 + 1, y0), (x0 + 1, y0 + 1), (x0, y0 + 1)]
                poly = _clip_halfplane(sq, c, s, hi)            # <p, omega> <= hi
                poly = _clip_halfplane(poly, -c, -s, -lo)       # <p, omega> >= lo
                A[a * g.n_det + i, j] = _area(poly) / g.ds
    return A


def joseph_matrix(g: Geometry) -> np.ndarray:
    """Dense m x n matrix of Joseph's method: for a ray with |cos| >= |sin| (closer to
    the y axis) the image rows are sampled where the ray crosses their centre lines,
    else the columns; each sample interpolates linearly between the two pixel centres
    around the crossing (pixels outside the image are zero) and is weighted by the
    ray's length per row (or column), 1/max(|cos|, |sin|)."""
    N = g.N
    A = np.zeros((g.m, g.n))
    centres = np.arange(N) - N / 2 + 0.5
    for a in range(g.n_ang):
        c, s = g.cos[a], g.sin[a]
        rows = abs(c) >= abs(s)
        step = 1.0 / max(abs(c), abs(s))
        for i in range(g.n_det):
            row = a * g.n_det + i
            for b in range(N):
                if rows:
                    xs = (g.s[i] - centres[b] * s) / c       # crossing of row b's centre line
                else:
                    xs = (g.s[i] - centres[b] * c) / s       # crossing of column b's centre line
                k = int(np.floor(xs - centres[0]))           # centres[k] <= xs < centres[k+1]
                f = xs - centres[0] - k
                for kk, w in ((k, 1.0 - f), (k + 1, f)):
                    if 0 <= kk < N and w > 0.0:
                        j = b * N + kk if rows else kk * N + b
                        A[row, j] += w * step
    return A

