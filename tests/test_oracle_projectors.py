"""Pins of the oracle's projectors against facts that do not come from the oracle.

CPU only. Each test names the property it checks and where it comes from.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from oracle import brute
from oracle.core import assemble_dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

TINY = [
    dict(N=6, n_ang=12, n_det=11, ang_range=180.0),
    dict(N=5, n_ang=9, n_det=9, ang_range=120.0),
    dict(N=8, n_ang=16, n_det=12, ang_range=180.0),       # even n_det: half-integer bins
    dict(N=7, n_ang=0, n_det=11, angles_deg=[0.0, 90.0, 45.0, 13.7, 101.3, 179.9, 33.3333, 135.0]),
    dict(N=4, n_ang=6, n_det=7, ang_range=180.0, det_spacing=1.3),
    dict(N=30, n_ang=4, n_det=31, ang_range=180.0, det_spacing=1.3),  # edge rays at s = +-13
]


@pytest.mark.parametrize("kw", TINY)
def test_line_model_equals_brute_force_clipping(kw):
    """A's entries are exact ray/pixel intersection lengths: Liang-Barsky clipping of
    every ray against every pixel square gives the same matrix."""
    g = O.Geometry(**kw)
    A, AT, _ = assemble_dense(g)
    Ab = O.brute_force_matrix(g)
    assert np.abs(A - Ab).max() <= 1e-13
    assert np.array_equal(AT, A.T) or np.abs(AT - A.T).max() <= 1e-15


def test_row_sums_are_chord_lengths():
    """Sum over pixels of a ray's lengths = its chord through the image square."""
    g = O.Geometry(16, 45, 25)
    A, _, _ = assemble_dense(g)
    rows = A.sum(axis=1)
    chords = np.array([O.chord_length_in_square(g, a, i)
                       for a in range(g.n_ang) for i in range(g.n_det)])
    assert np.abs(rows - chords).max() <= 1e-12 * max(1.0, chords.max())
    assert chords.max() > 16.0  # some rays run along the diagonal


@pytest.mark.parametrize("n_det", [23, 24])
def test_zero_degree_rays_average_adjacent_columns(n_det):
    """At 0 degrees the rays are vertical lines x = s_i. With odd n_det they lie on
    pixel edges and see the mean of the two adjacent column sums; with even n_det they
    run through column centres and see one column sum."""
    N = 16
    g = O.Geometry(N, 4, n_det)  # angles 0, 45, 90, 135
    x = np.random.default_rng(3).uniform(size=N * N)
    y = g.A(x)[:n_det]
    col = x.reshape(N, N).sum(axis=0)
    for i, s in enumerate(g.s):
        u = s + N / 2
        if abs(u - round(u)) < 1e-12:
            c = int(round(u))
            left = col[c - 1] if 0 <= c - 1 < N else 0.0
            right = col[c] if 0 <= c < N else 0.0
            want = 0.5 * (left + right)
        else:
            c = int(math.floor(u))
            want = col[c] if 0 <= c < N else 0.0
        assert abs(y[i] - want) <= 1e-12 * max(1.0, abs(want))


def test_ninety_degree_rays_average_adjacent_rows():
    N = 12
    g = O.Geometry(N, 2, 17)  # 0 and 90 degrees
    x = np.random.default_rng(4).uniform(size=N * N)
    y = g.A(x)[17:]
    row = x.reshape(N, N).sum(axis=1)
    for i, s in enumerate(g.s):
        r = int(round(s + N / 2))
        want = 0.5 * ((row[r - 1] if 0 <= r - 1 < N else 0.0) + (row[r] if 0 <= r < N else 0.0))
        assert abs(y[i] - want) <= 1e-12 * max(1.0, abs(want))


def _disk_image(N, R, sub=16):
    """Area fraction of the disk |p| <= R in each pixel, by sub x sub sampling."""
    off = (np.arange(sub) + 0.5) / sub
    c = np.arange(N) - N / 2
    xs = (c[:, None] + off[None, :]).ravel()
    X2 = xs[None, :] ** 2
    inside = (X2 + X2.T) <= R * R          # [row samples, col samples]
    return inside.reshape(N, sub, N, sub).mean(axis=(1, 3)).ravel()


def test_disk_projection_converges_to_closed_form():
    """The projection of a uniform disk of radius R is 2 sqrt(R^2 - s^2) at every angle.
    The discretisation error of A applied to the disk's area-fraction image must shrink
    with the grid (fixed R/N; for a disk's jump the relative 2-norm error decays like
    N^-1/2) and stay under bounds frozen from a first run (0.0069, 0.0051, 0.0040)."""
    errs = []
    for N in (64, 128, 256):
        R = 0.3 * N
        g = O.Geometry(N, 30, N + 1)
        y = g.A(_disk_image(N, R)).reshape(g.n_ang, g.n_det)
        s = g.s
        exact = 2.0 * np.sqrt(np.maximum(R * R - s * s, 0.0))
        err = np.linalg.norm(y - exact[None, :]) / np.linalg.norm(np.broadcast_to(exact, y.shape))
        errs.append(err)
    assert errs[1] < 0.85 * errs[0] and errs[2] < 0.85 * errs[1], errs
    assert errs[0] < 0.0075 and errs[1] < 0.0055 and errs[2] < 0.0044, errs


def test_single_pixel_centroid_follows_projection_of_centre():
    """Orientation pin: the projection of one pixel with centre (xc, yc) is a profile
    of unit area centred at s = xc cos(theta) + yc sin(theta). Sampled on a fine
    detector (ds = 0.01) its discrete centroid and area match to O(ds^2)."""
    N = 20
    ds = 0.01
    g = O.Geometry(N, 37, 3001, det_spacing=ds)
    for (r, c) in [(0, 0), (3, 15), (19, 2), (10, 10)]:
        x = np.zeros(N * N)
        x[r * N + c] = 1.0
        y = g.A(x).reshape(g.n_ang, g.n_det)
        xc, yc = c - N / 2 + 0.5, r - N / 2 + 0.5
        cent = (y * g.s[None, :]).sum(axis=1) / y.sum(axis=1)
        want = xc * g.cos + yc * g.sin
        assert np.abs(cent - want).max() <= 1e-3
        assert np.abs(y.sum(axis=1) * ds - 1.0).max() <= 1e-3


def test_matched_adjoint_identity():
    g = O.Geometry(32, 45, 47)
    r = np.random.default_rng(5)
    x = r.standard_normal(g.n)
    y = r.standard_normal(g.m)
    lhs = g.A(x) @ y
    rhs = x @ g.AT(y)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs) + 1e-12


def test_hat_partition_of_unity():
    """B distributes each pixel over the detector with weights summing to 1/ds: B 1 =
    n_ang/ds wherever every pixel centre projects inside the detector."""
    for ds in (1.0, 1.25):
        g = O.Geometry(24, 33, 41, det_spacing=ds)
        x = g.B_hat(np.ones(g.m))
        assert np.abs(x - g.n_ang / ds).max() <= 1e-12


def test_hat_hand_computed_2x2():
    """B for a 2 x 2 image, angles 0, 90 and 45 degrees, three unit bins at s = -1, 0, 1,
    written out by hand from the interpolation weights."""
    g = O.Geometry(2, 0, 3, angles_deg=[0.0, 90.0, 45.0])
    _, _, B = assemble_dense(g)
    a = 1.0 / math.sqrt(2.0)
    want = np.zeros((4, 9))
    # 0 deg: pixel centre x-coordinates -1/2, +1/2, -1/2, +1/2 -> bins (0,1) or (1,2)
    want[0, 0:2] = 0.5; want[1, 1:3] = 0.5; want[2, 0:2] = 0.5; want[3, 1:3] = 0.5
    # 90 deg: y-coordinates -1/2, -1/2, +1/2, +1/2
    want[0, 3:5] = 0.5; want[1, 3:5] = 0.5; want[2, 4:6] = 0.5; want[3, 4:6] = 0.5
    # 45 deg: projections -1/sqrt2, 0, 0, +1/sqrt2 -> u = 1 - a, 1, 1, 1 + a
    want[0, 6] = a; want[0, 7] = 1 - a
    want[1, 7] = 1.0
    want[2, 7] = 1.0
    want[3, 7] = 1 - a; want[3, 8] = a
    assert np.abs(B - want).max() <= 1e-15


def test_unmatchedness_is_of_the_order_the_paper_reports():
    """Diagnostic: ||B - A^T||_F / ||A||_F for the line model and the interpolating
    back projector is nonzero and of the order of Table 6.2's 0.14-0.37 differences
    between discretisation models."""
    g = O.Geometry(32, 45, 47)
    A, AT, B = assemble_dense(g)
    ratio = np.linalg.norm(B - AT) / np.linalg.norm(A)
    assert 0.05 < ratio < 0.8, ratio


@pytest.mark.parametrize("kind", ["hat", "adj"])
def test_pixel_spot_checks_equal_full_back_projection(kind):
    """The per-pixel NumPy evaluation used for large-size spot checks agrees with the
    C back projectors on every pixel of a small geometry (incl. axis angles)."""
    g = O.Geometry(20, 24, 31, det_spacing=1.0)
    y = np.random.default_rng(6).standard_normal(g.m)
    full = g.back(kind)(y)
    pix = np.arange(g.n)
    assert np.abs(g.back_pixels(kind, y, pix) - full).max() <= 1e-12 * np.abs(full).max()


def test_storage_matches_table_6_3():
    """Every storage entry of Table 6.3 equals k*m (AB) or k*n (BA)."""
    with open(os.path.join(GOLDEN, "table_6_3_storage.json")) as f:
        gold = json.load(f)
    for e in gold["entries"]:
        sz = gold["sizes"][e["size"]]
        assert O.basis_storage(e["method"], e["k"], sz["m"], sz["n"]) == e["storage"], e


def test_angle_table_snaps_axis_angles():
    th, c, s = O.angle_table(720, 180.0)
    assert th[360] == 90.0 and c[360] == 0.0 and s[360] == 1.0
    assert c[0] == 1.0 and s[0] == 0.0
    th, c, s = O.angle_table(1800, 180.0)
    assert th[900] == 90.0 and c[900] == 0.0
    th, c, s = O.angle_table(60, 120.0)
    assert th[45] == 90.0 and c[45] == 0.0 and s[45] == 1.0


# ---- strip and Joseph (interpolation) models -------------------------------------------

MODEL_GEOMS = [
    dict(N=4, n_ang=7, n_det=7),                                   # 0 deg included
    dict(N=5, n_ang=6, n_det=9, det_spacing=0.8),
    dict(N=3, n_ang=8, n_det=5, det_spacing=1.3),                  # 0, 45, 90, 135 deg
    dict(N=6, n_ang=0, n_det=8, angles_deg=[0.0, 90.0, 45.0, 13.7, 101.3, 179.9, 33.3333]),
]


def _dense(g, f, n_in):
    return np.stack([f(e) for e in np.eye(n_in)], axis=1)


@pytest.mark.parametrize("kw", MODEL_GEOMS)
def test_strip_model_equals_polygon_clipping(kw):
    """Strip model (Sec. 6.1): the oracle's closed form (trapezoid integrated over the
    detector cell) equals the area of strip and pixel by polygon clipping, divided by
    ds; its transpose is the exact transpose."""
    g = O.Geometry(**kw)
    ref = brute.strip_area_matrix(g)
    A = _dense(g, lambda e: g.A_model("strip", e), g.n)
    AT = _dense(g, lambda e: g.AT_model("strip", e), g.m)
    assert np.abs(A - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    assert np.abs(AT - ref.T).max() <= 1e-13 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("kw", MODEL_GEOMS)
def test_joseph_model_equals_row_interpolation(kw):
    """Joseph's model (Sec. 6.1): the oracle's closed form (a triangle of half-width
    max(|cos|,|sin|) in detector coordinates) equals sampling the rows (or columns) at
    the ray's crossings with linear interpolation, weighted by the length per row."""
    g = O.Geometry(**kw)
    ref = brute.joseph_matrix(g)
    A = _dense(g, lambda e: g.A_model("joseph", e), g.n)
    AT = _dense(g, lambda e: g.AT_model("joseph", e), g.m)
    assert np.abs(A - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    assert np.abs(AT - ref.T).max() <= 1e-13 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("row", [0, 1])
def test_model_differences_match_table_6_2(row):
    """||As - Al||/||As||, ||As - Ai||/||As||, ||Al - Ai||/||Al|| (Frobenius) at the
    scan parameters of Table 6.1 reproduce Table 6.2 to the four printed digits."""
    with open(os.path.join(GOLDEN, "table_6_2_model_differences.json")) as f:
        gold = json.load(f)["rows"][row]
    g = O.Geometry(gold["N"], gold["n_ang"], gold["n_det"])
    G = g.model_gram()        # order: line, strip, Joseph
    d = lambda a, b: math.sqrt(G[a, a] + G[b, b] - 2.0 * G[a, b])
    got = {"s_l": d(1, 0) / math.sqrt(G[1, 1]), "s_i": d(1, 2) / math.sqrt(G[1, 1]),
           "l_i": d(0, 2) / math.sqrt(G[0, 0])}
    for k in ("s_l", "s_i", "l_i"):
        assert abs(got[k] - gold[k]) <= 0.5e-4, (gold["size"], k, got[k], gold[k])


def test_strip_columns_sum_to_the_pixel_area():
    """Summed over the bins of one angle, a strip-model column is the pixel's area over
    ds (every strip of the detector tiles the plane), for pixels whose footprint lies
    on the detector."""
    for ds in (1.0, 0.8, 1.25):
        g = O.Geometry(12, 17, 31, det_spacing=ds)
        A = _dense(g, lambda e: g.A_model("strip", e), g.n).reshape(g.n_ang, g.n_det, g.n)
        sums = A.sum(axis=1)                      # n_ang x n
        assert np.abs(sums - 1.0 / ds).max() <= 1e-13, ds


def test_joseph_is_exact_on_linear_images():
    """Linear interpolation reproduces a linear image, so for rays that stay inside the
    pixel centres' hull Joseph's ray sum is the exact line integral of the linear
    function across the image: the length of the segment times its midpoint value."""
    N = 24
    g = O.Geometry(N, 0, 9, angles_deg=[0.0, 10.0, 30.0, 44.0, 60.0, 80.0, 90.0, 125.0, 170.0],
                   det_spacing=1.0)
    al, be, ga = 0.37, -0.21, 1.5
    cen = np.arange(N) - N / 2 + 0.5
    X, Y = np.meshgrid(cen, cen)                      # X: column coordinate, Y: row
    x = (al * X + be * Y + ga).ravel()
    y = g.A_model("joseph", x).reshape(g.n_ang, g.n_det)
    checked = 0
    for a in range(g.n_ang):
        c, s = g.cos[a], g.sin[a]
        for i, si in enumerate(g.s):
            p0 = np.array([si * c, si * s])           # foot of the ray, its midpoint
            d = np.array([-s, c])
            if abs(c) >= abs(s):                      # rows: y from -N/2 to N/2
                tt = np.array([-N / 2, N / 2]) - p0[1]
                ends = [p0 + (t / d[1]) * d for t in tt]
                inner = all(abs(e[0]) <= N / 2 - 1.0 for e in ends)
            else:
                tt = np.array([-N / 2, N / 2]) - p0[0]
                ends = [p0 + (t / d[0]) * d for t in tt]
                inner = all(abs(e[1]) <= N / 2 - 1.0 for e in ends)
            if not inner:
                continue
            length = np.linalg.norm(ends[1] - ends[0])
            mid = 0.5 * (ends[0] + ends[1])
            exact = length * (al * mid[0] + be * mid[1] + ga)
            assert abs(y[a, i] - exact) <= 1e-12 * abs(exact), (a, i)
            checked += 1
    assert checked >= 30


def test_narrow_strips_tend_to_the_line_model():
    """As the strip width goes to zero the strip model becomes the line model (away
    from the axis-aligned edge case): one ray through the centre, error O(ds)."""
    angles = [7.0, 23.0, 45.0, 61.0, 118.0]
    x = np.random.default_rng(3).random(10 * 10)
    line = O.Geometry(10, 0, 1, angles_deg=angles, det_spacing=1.0).A(x)
    errs = []
    for ds in (1e-2, 1e-3):
        g = O.Geometry(10, 0, 1, angles_deg=angles, det_spacing=ds)
        errs.append(np.abs(g.A_model("strip", x) - line).max() / np.abs(line).max())
    assert errs[1] < 1e-2 and errs[1] < 0.2 * errs[0], errs


# ---- thresholded back projector B_tau (Sec. 6.5) ----------------------------------------

@pytest.mark.parametrize("row", [0, 1])
def test_b_tau_unmatchedness_matches_table_6_4(row):
    """||B_tau - As^T||_F / ||As||_F at the scan parameters of Table 6.1 reproduces Table 6.4
    for tau = 0.01, 0.1, 0.3, 0.5 to the four printed digits (max As = 1 there: at 0
    degrees a strip covers a pixel column exactly)."""
    with open(os.path.join(GOLDEN, "table_6_4_b_tau_unmatchedness.json")) as f:
        gold = json.load(f)
    r = gold["rows"][row]
    g = O.Geometry(r["N"], r["n_ang"], r["n_det"])
    assert g.strip_max() == pytest.approx(1.0, abs=1e-14)
    for tau, want in zip(gold["tau"], r["values"]):
        assert abs(g.strip_tau_unmatchedness(tau) - want) <= 0.5e-4, (r["size"], tau)


@pytest.mark.parametrize("kw", MODEL_GEOMS[:3])
def test_b_tau_equals_thresholded_clipping_matrix(kw):
    """B_tau is the transpose of the polygon-clipping strip matrix with the entries below
    tau * max dropped (entries within 1e-6 * max of the threshold kept), for several tau,
    including 0.5 where axis angles put entries exactly on the threshold."""
    g = O.Geometry(**kw)
    ref = brute.strip_area_matrix(g)
    mx = ref.max()
    assert abs(g.strip_max() - mx) <= 1e-13
    for tau in (0.0, 0.1, 0.3, 0.5, 0.9):
        want = np.where(ref >= tau * mx - 1e-6 * mx, ref, 0.0).T
        got = _dense(g, g.B_tau(tau), g.m)
        assert np.abs(got - want).max() <= 1e-13, tau
    # tau = 0 is the strip transpose itself
    y = np.random.default_rng(4).standard_normal(g.m)
    assert np.abs(g.B_tau(0.0)(y) - g.AT_model("strip", y)).max() <= 1e-13

