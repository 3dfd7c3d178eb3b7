"""GPU LSQR and LSMR (C ABI) -- the matched comparators of the paper (Sec. 5, 6.2).

* Against SciPy's LSQR / LSMR (the same short recurrences, no reorthogonalisation) on
  explicit matrices of tiny geometries, for the line, strip and Joseph models, with and
  without an initial guess: iterates at several k within 1e-9, or 1000x the change a
  1e-13 perturbation of b causes in SciPy's own iterate where that is larger (FP64).
* Sec. 5: with B = A^T, AB-GMRES is LSQR and BA-GMRES is LSMR; the GPU iterates agree
  with the FP64 oracle's matched GMRES at early k (before short recurrences lose
  orthogonality) and stop at the same DP iteration (FP32 projectors).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _dense_model(go, model):
    f = go.fwd(model)
    return np.stack([f(e) for e in np.eye(go.n)], axis=1)


@pytest.mark.parametrize("model", ["line", "strip", "joseph"])
@pytest.mark.parametrize("method", ["lsqr", "lsmr"])
@pytest.mark.parametrize("with_x0", [False, True])
def test_against_scipy(gpu_lib, model, method, with_x0):
    import torch
    import paper_2110_01481_amd as abg
    go = O.Geometry(14, 18, 21)
    A = _dense_model(go, model)
    rng = np.random.default_rng(21)
    b = A @ rng.uniform(size=go.n) + 0.02 * rng.standard_normal(go.m)
    x0 = 0.5 * rng.uniform(size=go.n) if with_x0 else None
    gg = abg.Geometry(14, 18, 21, model=model)
    bt = torch.tensor(b, device="cuda")
    x0t = torch.tensor(x0, device="cuda") if with_x0 else None
    def scipy_run(rhs, k):
        if method == "lsqr":
            return sla.lsqr(A, rhs, damp=0.0, atol=0, btol=0, conlim=0, iter_lim=k, x0=x0)[0]
        return sla.lsmr(A, rhs, damp=0.0, atol=0, btol=0, conlim=0, maxiter=k, x0=x0)[0]

    d = np.random.default_rng(5).standard_normal(go.m)
    bp = b + 1e-13 * np.linalg.norm(b) * d / np.linalg.norm(d)
    for k in (1, 2, 5, 12, 25):
        ref = scipy_run(b, k)
        # short recurrences lose orthogonality: from k ~ 10 on this problem a 1e-13
        # change of b moves SciPy's own iterate by 1e-7 .. 1e-3; the bound is 1000x that
        tol = max(1e-9, 1e3 * _rel(scipy_run(bp, k), ref))
        r = abg.lsq(method, gg, bt, k, x0=x0t)
        assert r.status == "ok" and r.k_done == k, (r.status, r.k_done)
        assert _rel(r.x.cpu().numpy(), ref) <= tol, (k, _rel(r.x.cpu().numpy(), ref), tol)
        # the explicit residual reported is ||b - A x_k||
        assert abs(r.res_norm - np.linalg.norm(b - A @ r.x.cpu().numpy())) <= 1e-10 * np.linalg.norm(b)


@pytest.fixture(scope="module")
def cfg1():
    w = W.CONFIG1
    go = O.Geometry(w.N, w.n_ang, w.n_det)
    xb = w.phantom()
    b, enorm = W.add_noise(go.A(xb), w.eta, w.noise_dir())
    return go, xb, b, enorm


@pytest.mark.parametrize("method", ["lsqr", "lsmr"])
def test_matched_gmres_equivalence(gpu_lib, cfg1, method):
    """Sec. 5: LSQR iterates are AB-GMRES(A, A^T) iterates and LSMR iterates BA-GMRES(A, A^T)
    iterates (FP64, k <= 10 on the 64^2 workload)."""
    import torch
    import paper_2110_01481_amd as abg
    go, _, b, _ = cfg1
    gg = abg.Geometry(go.N, go.n_ang, go.n_det)
    f = O.ab_gmres if method == "lsqr" else O.ba_gmres
    ref = f(go.A, go.AT, b, 10, keep_iterates=True)
    bt = torch.tensor(b, device="cuda")
    for k in (1, 3, 6, 10):
        r = abg.lsq(method, gg, bt, k)
        assert _rel(r.x.cpu().numpy(), ref.iterates[k - 1]) <= 1e-7, k


@pytest.mark.parametrize("method", ["lsqr", "lsmr"])
@pytest.mark.parametrize("model", ["line", "strip"])
def test_discrepancy_principle_fp32(gpu_lib, method, model):
    """FP32 projectors, DP (tau = 1.02): the same stopping iteration as the FP64 oracle's
    matched GMRES and an iterate within 1e-4 of it."""
    import torch
    import paper_2110_01481_amd as abg
    go = O.Geometry(48, 60, 69)
    xb = W.ellipse_phantom(48, 5, W.rng(61, 0, 0))
    b, enorm = W.add_noise(go.fwd(model)(xb), 0.02, W.rng(61, 0, 1).standard_normal(go.m))
    gg = abg.Geometry(48, 60, 69, model=model)
    f = O.ab_gmres if method == "lsqr" else O.ba_gmres
    back = go.AT if model == "line" else go.back(model + "_t")
    ref = f(go.fwd(model), back, b, 100, stop="dp", tau=1.02, noise_norm=enorm)
    r = abg.lsq(method, gg, torch.tensor(b, dtype=torch.float32, device="cuda"), 100, stop="dp",
                tau=1.02, noise_norm=enorm)
    assert r.status == "ok" and r.k_stop == ref.k_stop, (r.k_stop, ref.k_stop)
    assert r.res_norm <= 1.02 * enorm
    assert _rel(r.x.double().cpu().numpy(), ref.x) <= 1e-4


def test_zero_rhs_and_bad_arguments(gpu_lib):
    import torch
    import paper_2110_01481_amd as abg
    gg = abg.Geometry(16, 10, 23)
    z = torch.zeros(gg.m, device="cuda")
    for method in ("lsqr", "lsmr"):
        r = abg.lsq(method, gg, z, 5)
        assert r.status == "zero_rhs" and r.k_done == 0 and float(r.x.abs().max()) == 0.0
    with pytest.raises(abg.AbgError):
        abg.lsq("lsqr", gg, torch.ones(gg.m, device="cuda"), 5, stop="dp", tau=0.5, noise_norm=1.0)


@pytest.mark.parametrize("method", ["ab", "ba", "lsqr", "lsmr"])
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("stop", ["none", "dp"])
def test_workspace_contents_do_not_matter(gpu_lib, method, dt, stop):
    """Every solver initialises what it reads: a workspace whose bytes are all 0xFF (NaN in
    FP32 and FP64) gives bit-identical results to a zeroed one, for each stopping rule."""
    import torch
    import paper_2110_01481_amd as abg
    go = O.Geometry(48, 60, 69)
    xb = W.ellipse_phantom(48, 5, W.rng(61, 0, 0))
    b, enorm = W.add_noise(go.A(xb), 0.02, W.rng(61, 0, 1).standard_normal(go.m))
    gg = abg.Geometry(48, 60, 69)
    tdt = torch.float64 if dt == "f64" else torch.float32
    bt = torch.tensor(b, dtype=tdt, device="cuda")
    kw = dict(stop=stop, tau=1.02, noise_norm=enorm) if stop == "dp" else {}
    if method in ("ab", "ba"):
        nb = abg.workspace_bytes(gg, method, 40, proj=dt, basis=dt, stop=stop)
        run = lambda ws: abg.gmres(method, gg, bt, 40, workspace=ws, **kw)
    else:
        nb = abg.lsq_workspace_bytes(gg, method, dt)
        run = lambda ws: abg.lsq(method, gg, bt, 40, workspace=ws, **kw)
    outs = []
    for fill in (0x00, 0xFF):
        ws = torch.full((nb,), fill, dtype=torch.uint8, device="cuda")
        r = run(ws)
        outs.append((r.status, r.k_stop, r.x.cpu().numpy().copy(), r.res_hist.copy()))
    assert outs[0][0] == outs[1][0] and outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][2], outs[1][2]) and np.array_equal(outs[0][3], outs[1][3])
    assert np.all(np.isfinite(outs[1][2]))


def test_lsq_one_pixel_and_invalid_rules(gpu_lib):
    """A 1 x 1 image: the Krylov space has dimension one, so after the first step the
    iterate is the least-squares solution, and later steps keep it (FP64). The NCP rule
    needs at least two bins per projection; x_ref and err_hist come together."""
    import ctypes
    import torch
    import paper_2110_01481_amd as abg
    from paper_2110_01481_amd import _binding as B
    go = O.Geometry(1, 7, 3)
    A = np.stack([go.A(e) for e in np.eye(go.n)], axis=1)
    b = np.random.default_rng(3).uniform(size=go.m)
    xs = np.linalg.lstsq(A, b, rcond=None)[0]
    gg = abg.Geometry(1, 7, 3)
    for method in ("lsqr", "lsmr"):
        for k in (1, 3):
            r = abg.lsq(method, gg, torch.tensor(b, device="cuda"), k)
            assert r.status in ("ok", "breakdown")
            assert abs(float(r.x.cpu()[0]) - xs[0]) <= 1e-12 * abs(xs[0]), (method, k)
    g1 = abg.Geometry(8, 6, 1)
    with pytest.raises(abg.AbgError):
        abg.lsq("lsqr", g1, torch.ones(g1.m, device="cuda"), 5, stop="ncp")
    lib = B.load_library()
    bt = torch.ones(gg.m, dtype=torch.float64, device="cuda")
    x = torch.empty(gg.n, dtype=torch.float64, device="cuda")
    nb = abg.lsq_workspace_bytes(gg, "lsqr", "f64")
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    xr = torch.zeros(gg.n, dtype=torch.float64, device="cuda")
    err = np.zeros(5)
    for xref, eh in ((ctypes.c_void_p(xr.data_ptr()), None), (None, err.ctypes.data_as(B._dp))):
        rc = lib.abg_lsqr(gg.handle, ctypes.c_void_p(bt.data_ptr()), None,
                          ctypes.c_void_p(x.data_ptr()), 5, B.Stop(B.STOP_NONE, 1.0, 0.0), B.F64,
                          ctypes.c_void_p(ws.data_ptr()), nb, None, xref, eh, None)
        assert rc == -1
