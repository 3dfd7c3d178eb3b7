"""Deep Krylov runs against the FP64 oracle: the multi-block Gram-Schmidt forms and the
Givens forms that only long runs reach (Sec. 2 listing: MGS, Hessenberg least squares,
iterate).

Problem: 144^2 image, 360 angles x 205 bins, 8 ellipses, 1% noise, so that both basis
vector lengths (m = 73800 for AB-GMRES, n = 20736 for BA-GMRES) exceed what one block
holds (8192 elements in FP64, 16384 in FP32): every Gram-Schmidt step runs on a block
group with grid-wide reductions. 80 steps without a stopping rule cross every form a
single solve takes by step (the inverse compact WY form for steps 2-64, the plain sweep
from 65; the one-wave Givens update to k = 63, two entries per lane to 127). The 64^2
problem runs 140 steps, past k = 127, where the Givens update takes its block-wide form.
The batched engine (its own multi-block sweep) runs the same problems.

Oracle: tests/golden/oracle_deep.npz (make_oracle_golden.py deep): iterates at
k = 15, 32, 63, 64, 65, 80 (64^2: 64, 127, 128, 140), the GMRES residual history
|| ||r_0|| e_1 - H_k y_k || of every step, and two probes of the oracle itself:
  * sensitivity: the relative change of each x_k and each residual norm when b moves by
    1e-15 relative. Late iterates of these ill-posed problems amplify rounding-level
    changes of the data enormously (x_80 moves by ~1e-4 under the 1e-15 change).
  * FP32 storage: the relative change when every projector output, b and every stored
    basis vector are rounded to FP32 (dots, norms and the small problem in FP64) -- what
    FP32 storage alone does to the method (x_65 of BA-GMRES moves by 1.5e-3).
Bounds per step (probes taken as the largest over k-3..k+3 where every step is stored,
since one perturbation samples a spike):
  FP64 GPU vs FP64 oracle:  max(1e-9, 1e3 * sensitivity)  (GPU and oracle round
                            differently at every operation; the worst step seen is 136x
                            the one-direction probe);
  FP32 GPU vs FP64 oracle:  max(1e-4, 100 * FP32-storage change)  (the GPU also rounds
                            inside each projector sum of ~1000 terms, about sqrt(1000)
                            times more than the outputs' rounding alone: 25x at k = 15).
Up to k ~ 10 the 1e-4 target binds; beyond, FP32 iterates of these problems differ from
the FP64 ones by what FP32 rounding itself causes (1e-3 around k = 65), and the test holds
the GPU to that.
"""
import os

import numpy as np
import pytest

import oracle as O  # noqa: F401  (the golden file is the oracle's output)
import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "oracle_deep.npz")
DEEP = {"N": 144, "n_ang": 360, "eta": 0.01, "K": 80, "cfg": 94}


@pytest.fixture(scope="module")
def gold():
    z = np.load(GOLD)
    return {k: z[k] for k in z.files}


def _near(s):
    s = np.asarray(s)
    return np.array([np.nanmax(s[max(0, k - 3):k + 4]) for k in range(s.size)])


def _bound(g, pre, what, dt):
    """Per-step bounds for x_k (what = "x") or the GMRES residual norms ("ls")."""
    if dt == "f64":
        return np.maximum(1e-9, 1e3 * _near(g[pre + "sens_" + what]))
    # the FP32-storage probe of x_k exists at the stored steps only
    d = g[pre + "d32_" + what]
    return np.maximum(1e-4, 100.0 * (_near(d) if what == "ls" else d))


def _deep_inputs():
    """b = A x_bar + e with the oracle's A, as make_oracle_golden.py forms it."""
    d = DEEP
    n_det = W.n_det_for(d["N"])
    go = O.Geometry(d["N"], d["n_ang"], n_det)
    xb = W.ellipse_phantom(d["N"], 8, W.rng(d["cfg"], d["N"], W.STREAM_PHANTOM))
    b, _ = W.add_noise(go.A(xb), d["eta"], W.rng(d["cfg"], d["N"], W.STREAM_NOISE).standard_normal(go.m))
    return d["N"], d["n_ang"], n_det, b


@pytest.fixture(scope="module")
def deep(gpu_lib):
    N, n_ang, n_det, b = _deep_inputs()
    return gpu_lib.Geometry(N, n_ang, n_det), b


@pytest.fixture(scope="module")
def small(gpu_lib):
    w = W.CONFIG1
    go = O.Geometry(w.N, w.n_ang, w.n_det)
    b, _ = W.add_noise(go.A(w.phantom()), w.eta, w.noise_dir())
    return gpu_lib.Geometry(w.N, w.n_ang, w.n_det), b


def _t(a, dt):
    import torch
    return torch.tensor(a, dtype=torch.float64 if dt == "f64" else torch.float32, device="cuda")


def _check_iterate(x, ref, bound, what):
    x = np.asarray(x, dtype=np.float64)
    e_norm = np.linalg.norm(x - ref) / np.linalg.norm(ref)
    e_max = np.abs(x - ref).max() / np.abs(ref).max()
    print(f"{what}: ||x - x_ref||/||x_ref|| = {e_norm:.2e}, max|x - x_ref|/max|x_ref| = "
          f"{e_max:.2e} (bound {bound:.1e})")
    assert e_norm <= bound and e_max <= bound, (what, e_norm, e_max, bound)


def _check_ls(ls, g, pre, dt, what):
    ref = g[pre + "ls_res"]
    n = len(ls)
    dev = np.abs(np.asarray(ls) / ref[:n] - 1.0)
    bound = _bound(g, pre, "ls", dt)[:n]
    k = int(np.argmax(dev / bound))
    print(f"{what}: GMRES residual history, worst step {k + 1}: {dev[k]:.2e} (bound {bound[k]:.1e}); "
          f"largest deviation {dev.max():.2e}")
    assert np.all(dev <= bound), (what, k + 1, dev[k], bound[k])


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("method", ["ab", "ba"])
def test_single_solve_80_steps(gpu_lib, gold, deep, method, dt):
    """Single solves (multi-block Gram-Schmidt: the inverse compact WY form to step 64, the
    plain sweep after it): GMRES residual history of all 80 steps, and the iterates at
    k = 15, 32, 63, 64, 65 (solves with that k_max; stop rule NONE) and 80."""
    gg, b = deep
    pre = f"deep_{method}_"
    bt = _t(b, dt)
    r = gpu_lib.gmres(method, gg, bt, DEEP["K"])
    assert r.status == "ok" and r.k_done == DEEP["K"]
    _check_ls(r.ls_hist, gold, pre, dt, f"single {method} {dt}")
    xb = _bound(gold, pre, "x", dt)
    for k in gold[pre + "ks"]:
        k = int(k)
        rk = r if k == DEEP["K"] else gpu_lib.gmres(method, gg, bt, k)
        assert rk.k_done == k
        _check_iterate(rk.x.double().cpu().numpy(), gold[pre + f"x{k}"], xb[k - 1],
                       f"single {method} {dt} x_{k}")


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("method", ["ab", "ba"])
def test_engine_80_steps(gpu_lib, gold, deep, method, dt):
    """The batched engine's multi-block sweep (plain MGS every step) on the same problem:
    three copies with k_max = 32, 65 and 80 advanced together, round by round; their
    iterates against the oracle's at those k, and the residual history of all 80 steps."""
    gg, b = deep
    pre = f"deep_{method}_"
    bt = _t(b, dt)
    ks = (32, 65, 80)
    eng = gpu_lib.Engine(proj=dt, basis=dt, max_slots=len(ks))
    try:
        res = eng.run([gpu_lib.Problem(g=gg, method=method, b=bt, k_max=k, stop="none") for k in ks])
    finally:
        eng.close()
    xb = _bound(gold, pre, "x", dt)
    for k, r in zip(ks, res):
        assert r.status == "ok" and r.k_done == k
        _check_iterate(r.x.double().cpu().numpy(), gold[pre + f"x{k}"], xb[k - 1],
                       f"engine {method} {dt} x_{k}")
    _check_ls(res[-1].ls_hist, gold, pre, dt, f"engine {method} {dt}")


@pytest.mark.parametrize("method", ["ab", "ba"])
def test_givens_block_form_past_127(gpu_lib, gold, small, method):
    """64^2 problem, 140 steps in FP64: steps 128-140 take the block-wide Givens update
    (one-wave forms below). Residual history of every step and the iterates at
    k = 64, 127, 128 and 140, single solves and the engine."""
    gg, b = small
    pre = f"givens_{method}_"
    bt = _t(b, "f64")
    K = 140
    r = gpu_lib.gmres(method, gg, bt, K)
    assert r.status == "ok" and r.k_done == K
    _check_ls(r.ls_hist, gold, pre, "f64", f"single {method} 140")
    xb = _bound(gold, pre, "x", "f64")
    for k in gold[pre + "ks"]:
        k = int(k)
        rk = r if k == K else gpu_lib.gmres(method, gg, bt, k)
        _check_iterate(rk.x.cpu().numpy(), gold[pre + f"x{k}"], xb[k - 1], f"single {method} x_{k}")
    eng = gpu_lib.Engine(proj="f64", basis="f64", max_slots=2)
    try:
        e128, e140 = eng.run([gpu_lib.Problem(g=gg, method=method, b=bt, k_max=k, stop="none")
                              for k in (128, 140)])
    finally:
        eng.close()
    _check_ls(e140.ls_hist, gold, pre, "f64", f"engine {method} 140")
    _check_iterate(e128.x.cpu().numpy(), gold[pre + "x128"], xb[127], f"engine {method} x_128")
    _check_iterate(e140.x.cpu().numpy(), gold[pre + "x140"], xb[139], f"engine {method} x_140")
