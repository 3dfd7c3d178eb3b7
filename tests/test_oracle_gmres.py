"""Pins of the oracle's AB-/BA-GMRES and stopping rules (CPU only).

The GMRES oracle is pinned by what Sec. 2 and Sec. 5 state about the iterates --
minimisers over a Krylov space, equal to LSQR/LSMR for B = A^T -- computed here by
other means (power-basis QR, Golub-Kahan with full reorthogonalisation, scipy), and
by the invariants of the Arnoldi process.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as sla

import oracle as O
import workloads as W
from oracle.core import assemble_dense


@pytest.fixture(scope="module")
def cfg1():
    w = W.CONFIG1
    g = O.Geometry(w.N, w.n_ang, w.n_det)
    xb = w.phantom()
    b, enorm = W.add_noise(g.A(xb), w.eta, w.noise_dir())
    return g, xb, b, enorm


@pytest.mark.parametrize("method", ["ab", "ba"])
@pytest.mark.parametrize("kind", ["hat", "adj"])
def test_iterates_minimise_over_krylov_space(cfg1, method, kind):
    """Sec. 2: x_k is the minimiser of ||b - A x|| (AB) or ||B(b - A x)|| (BA) over
    K_k(BA, Bb); the minimiser is recomputed from a QR of the power sequence."""
    g, _, b, _ = cfg1
    f = O.ab_gmres if method == "ab" else O.ba_gmres
    r = f(g.A, g.back(kind), b, 6, keep_iterates=True)
    for k in range(1, 7):
        xr = O.min_residual_iterate(method, g.A, g.back(kind), b, k)
        assert np.linalg.norm(xr - r.iterates[k - 1]) <= 1e-9 * np.linalg.norm(xr)


@pytest.mark.parametrize("method", ["ab", "ba"])
@pytest.mark.parametrize("kind", ["hat", "adj"])
def test_iterates_from_nonzero_x0_are_krylov_minimisers(cfg1, method, kind):
    """Sec. 2 with a starting guess: x_k lies in x_0 + K_k(BA, B r_0), r_0 = b - A x_0, and
    minimises ||b - A x|| (AB) or ||B(b - A x)|| (BA) there. The minimiser is recomputed
    from a QR of the power sequence; the starting guess is a seeded smooth image, and the
    iterates differ from those of x_0 = 0 (the start matters)."""
    g, xb, b, _ = cfg1
    f = O.ab_gmres if method == "ab" else O.ba_gmres
    x0 = 0.5 * xb + 0.05 * np.random.default_rng(31).uniform(size=g.n)
    r = f(g.A, g.back(kind), b, 6, x0=x0, keep_iterates=True)
    r0 = f(g.A, g.back(kind), b, 6, keep_iterates=True)
    for k in range(1, 7):
        xr = O.min_residual_iterate(method, g.A, g.back(kind), b, k, x0=x0)
        assert np.linalg.norm(xr - r.iterates[k - 1]) <= 1e-9 * np.linalg.norm(xr), k
        assert np.linalg.norm(r0.iterates[k - 1] - r.iterates[k - 1]) > 1e-3 * np.linalg.norm(xr)
    # the same minimiser with x_0 = 0 reproduces the zero-start run
    assert np.allclose(O.min_residual_iterate(method, g.A, g.back(kind), b, 4, x0=np.zeros(g.n)),
                       r0.iterates[3], rtol=0, atol=1e-9 * np.linalg.norm(r0.iterates[3]))


@pytest.mark.parametrize("method", ["ab", "ba"])
def test_matched_case_equals_lsqr_lsmr_full_reorth(cfg1, method):
    """Sec. 5: with B = A^T, AB-GMRES equals LSQR and BA-GMRES equals LSMR; in finite
    precision they agree with the full-reorthogonalisation variants."""
    g, _, b, _ = cfg1
    f = O.ab_gmres if method == "ab" else O.ba_gmres
    r = f(g.A, g.AT, b, 15, keep_iterates=True)
    gk = O.golub_kahan_lsqr if method == "ab" else O.golub_kahan_lsmr
    for k in (1, 5, 10, 15):
        xr = gk(g.A, g.AT, b, k)
        assert np.linalg.norm(xr - r.iterates[k - 1]) <= 1e-9 * np.linalg.norm(xr), k


@pytest.mark.parametrize("method", ["ab", "ba"])
def test_matched_case_vs_scipy(cfg1, method):
    """The same equivalence against scipy's LSQR / LSMR (no reorthogonalisation, so
    only the first iterations are compared)."""
    g, _, b, _ = cfg1
    A, AT, _ = assemble_dense(O.Geometry(16, 20, 23))
    gs = O.Geometry(16, 20, 23)
    bs = A @ np.random.default_rng(7).uniform(size=gs.n) + 0.01 * np.random.default_rng(8).standard_normal(gs.m)
    f = O.ab_gmres if method == "ab" else O.ba_gmres
    r = f(gs.A, gs.AT, bs, 8, keep_iterates=True)
    for k in (1, 3, 8):
        if method == "ab":
            xs = sla.lsqr(A, bs, damp=0.0, atol=0, btol=0, conlim=0, iter_lim=k)[0]
        else:
            xs = sla.lsmr(A, bs, damp=0.0, atol=0, btol=0, conlim=0, maxiter=k)[0]
        assert np.linalg.norm(xs - r.iterates[k - 1]) <= 1e-8 * np.linalg.norm(xs), k


@pytest.mark.parametrize("method", ["ab", "ba"])
@pytest.mark.parametrize("kind", ["hat", "adj"])
def test_arnoldi_relation_and_monotone_residuals(cfg1, method, kind):
    """M W_k = W_{k+1} H_k for M = AB or BA up to rounding; the minimised residual
    (||b - A x_k|| for AB, ||B(b - A x_k)|| for BA) never increases; the small least
    squares residual equals it."""
    g, _, b, _ = cfg1
    Bop = g.back(kind)
    f = O.ab_gmres if method == "ab" else O.ba_gmres
    K = 30
    r = f(g.A, Bop, b, K, keep_iterates=True, keep_basis=True)
    Wb = r.W
    M = (lambda v: g.A(Bop(v))) if method == "ab" else (lambda v: Bop(g.A(v)))
    MW = np.stack([M(Wb[j]) for j in range(K)], axis=1)
    rel = np.linalg.norm(MW - Wb[:K + 1].T @ r.H) / np.linalg.norm(MW)
    assert rel <= 10 * np.finfo(float).eps * math.sqrt(K) * 10, rel
    if method == "ab":
        minimised = np.array(r.res_norms)
    else:
        minimised = np.array([np.linalg.norm(Bop(b - g.A(x))) for x in r.iterates])
    assert np.all(np.diff(minimised) <= 1e-12 * minimised[:-1])
    assert np.allclose(np.array(r.ls_res), minimised, rtol=1e-9, atol=0)


def test_full_dimension_gmres_solves_tiny_systems():
    """With k = n on a tiny full-rank problem BA-GMRES returns the solution of the
    square system BA x = Bb (dense solve), and both methods recover x_bar from
    consistent data."""
    g = O.Geometry(5, 12, 9)
    A, AT, B = assemble_dense(g)
    rng = np.random.default_rng(11)
    xb = rng.uniform(size=g.n)
    noisy = A @ xb + 0.05 * rng.standard_normal(g.m)
    r = O.ba_gmres(g.A, g.B_hat, noisy, g.n)
    want = np.linalg.solve(B @ A, B @ noisy)
    assert np.linalg.norm(r.x - want) <= 1e-8 * np.linalg.norm(want)
    for f in (O.ab_gmres, O.ba_gmres):
        r = f(g.A, g.B_hat, A @ xb, g.m)
        assert r.status == "breakdown"
        assert np.linalg.norm(r.x - xb) <= 1e-8 * np.linalg.norm(xb)


def test_discrepancy_principle_picks_first_crossing(cfg1):
    g, _, b, enorm = cfg1
    full = O.ab_gmres(g.A, g.B_hat, b, 30)
    k = O.dp_index(full.res_norms, 1.0, enorm)
    assert k is not None and 1 < k < 30
    r = O.ab_gmres(g.A, g.B_hat, b, 30, stop="dp", tau=1.0, noise_norm=enorm, keep_iterates=True)
    assert r.k_stop == k and r.status == "ok"
    assert r.res_norms[k - 1] <= enorm < r.res_norms[k - 2]
    r2 = O.ab_gmres(g.A, g.B_hat, b, 3, stop="dp", tau=1.0, noise_norm=enorm)
    assert r2.status == "not_converged" and r2.k_stop == 3


def test_zero_rhs_returns_x0():
    g = O.Geometry(8, 10, 13)
    r = O.ba_gmres(g.A, g.B_hat, np.zeros(g.m), 5)
    assert r.k_stop == 0 and r.status == "zero_rhs" and not r.x.any()


def _direct_periodogram_ncp(r, n_ang, n_det):
    """NCP distance with the DFT written as an explicit sum (no FFT)."""
    q = n_det // 2
    i = np.arange(n_det)
    R = r.reshape(n_ang, n_det)
    white = np.arange(1, q + 1) / q
    C = []
    for row in R:
        p = []
        for j in range(1, q + 1):
            ang = -2.0 * math.pi * j * i / n_det
            p.append((row @ np.cos(ang)) ** 2 + (row @ np.sin(ang)) ** 2)
        p = np.array(p)
        C.append(np.cumsum(p) / p.sum() if p.sum() > 0 else white)
    return float(np.linalg.norm(np.mean(C, axis=0) - white))


def test_ncp_fft_equals_direct_dft():
    r = np.random.default_rng(2).standard_normal(5 * 37)
    assert abs(O.ncp_distance(r, 5, 37) - _direct_periodogram_ncp(r, 5, 37)) <= 1e-12
    r = np.random.default_rng(3).standard_normal(3 * 24)
    assert abs(O.ncp_distance(r, 3, 24) - _direct_periodogram_ncp(r, 3, 24)) <= 1e-12


def test_ncp_special_cases():
    """An impulse has a flat periodogram (distance 0); a pure tone at frequency j0 has a
    step NCP whose distance to the white line is a closed-form sum; white noise is
    close to the line."""
    n_det, n_ang = 41, 4
    q = n_det // 2
    r = np.zeros((n_ang, n_det))
    r[:, 7] = 3.0
    assert O.ncp_distance(r.ravel(), n_ang, n_det) <= 1e-13
    j0 = 6
    i = np.arange(n_det)
    tone = np.tile(np.cos(2 * math.pi * j0 * i / n_det), (n_ang, 1))
    want = math.sqrt(sum((j / q) ** 2 for j in range(1, j0)) + sum((1 - j / q) ** 2 for j in range(j0, q + 1)))
    assert abs(O.ncp_distance(tone.ravel(), n_ang, n_det) - want) <= 1e-10
    noise = np.random.default_rng(9).standard_normal(400 * 1001)
    assert O.ncp_distance(noise, 400, 1001) < 0.05
    assert O.ncp_distance(np.zeros(3 * 11), 3, 11) <= 1e-15


def test_ncp_index_rule():
    assert O.ncp_index([0.5, 0.4, 0.3, 0.35, 0.2]) == (3, True)
    assert O.ncp_index([0.5, 0.4, 0.3]) == (3, False)


def test_ncp_stop_returns_previous_iterate(cfg1):
    g, _, b, _ = cfg1
    full = O.ba_gmres(g.A, g.B_hat, b, 30, stop="ncp", ncp_shape=(g.n_ang, g.n_det),
                      keep_iterates=True)
    k, increased = O.ncp_index(full.ncp)
    assert full.k_stop == k
    assert np.array_equal(full.x, full.iterates[k - 1])


def test_bf16_rounding_known_values():
    """bfloat16 keeps 8 significant bits and rounds to nearest, ties to even."""
    ulp = 2.0 ** -7
    v = np.array([1.0, 1.0 + ulp / 2, 1.0 + 3 * ulp / 2, 1.0 + ulp / 4, 1.0 + 3 * ulp / 4,
                  -2.5, 3.0e38, 1e-40, np.inf, -np.inf])
    want = np.array([1.0, 1.0, 1.0 + 2 * ulp, 1.0, 1.0 + ulp, -2.5])
    got = O.bf16_round(v)
    assert np.array_equal(got[:6], want[:6])
    assert abs(got[6] / 3.0e38 - 1) < 2 ** -8
    assert got[7] != 0 and abs(got[7] / 1e-40 - 1) < 0.1   # subnormal: fewer bits
    assert np.isposinf(got[8]) and np.isneginf(got[9]) and np.isnan(O.bf16_round(np.array([np.nan])))[0]
