"""Error histories and stopping-rule markers (Sec. 6.2 and 6.3).

The relative reconstruction error ||x_bar - x_k|| / ||x_bar|| of every iterate of one
solve, the point of semi-convergence (its minimum), and the iterations the discrepancy
principle and the NCP criterion choose with the error there -- the quantities the paper
plots in its error-history figures and tabulates as reconstruction errors. All device
work runs in the library: the error curve comes from the solver's own error-history
calls (abg_gmres_error_history for AB-/BA-GMRES, the x_ref argument of abg_lsqr /
abg_lsmr), the markers from solves with the DP and NCP rules on the same data.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import _binding as B


@dataclass
class History:
    method: str             # "ab", "ba", "lsqr" or "lsmr"
    rel_err: np.ndarray     # ||x_bar - x_k|| / ||x_bar||, k = 1..len
    k_min: int              # argmin of rel_err (1-based; first of equal values)
    err_min: float
    k_dp: int | None        # DP iteration (None: not met within k_max)
    err_dp: float | None
    k_ncp: int | None       # NCP iteration
    err_ncp: float | None


def markers(rel_err: np.ndarray, k_dp: int | None, k_ncp: int | None):
    """(k_min, err_min, err_dp, err_ncp) of an error curve; k = 0 stands for x_0 and has
    no entry (its error is None)."""
    rel_err = np.asarray(rel_err, dtype=np.float64)
    if rel_err.size == 0:
        return 0, float("nan"), None, None
    k_min = int(np.argmin(rel_err)) + 1

    def at(k):
        return float(rel_err[k - 1]) if k is not None and 1 <= k <= rel_err.size else None

    return k_min, float(rel_err[k_min - 1]), at(k_dp), at(k_ncp)


def error_history(method: str, g, b: np.ndarray, x_bar: np.ndarray, k_max: int,
                  noise_norm: float, tau: float = 1.0, bp: str = "hat", dtype: str = "f32",
                  ncp: bool = True, device: str = "cuda") -> History:
    """Semi-convergence record of one method on (g's model A, back projector bp) for
    right-hand side b (host array, m) and true image x_bar (host array, n). AB-/BA-GMRES
    keep their basis in `dtype` (FP32 projectors with an FP32 basis by default); LSQR and
    LSMR use A's exact transpose and ignore bp. noise_norm: ||e|| for the DP rule."""
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    bt = torch.tensor(np.ascontiguousarray(b), dtype=tdt, device=device)
    xr = torch.tensor(np.ascontiguousarray(x_bar), dtype=tdt, device=device)
    # the norm of the reference as the device holds it (rounded to dtype)
    nrm = float(np.linalg.norm(xr.cpu().numpy().astype(np.float64)))
    if method in ("ab", "ba"):
        def run(**kw):
            return B.gmres(method, g, bt, k_max, bp=bp, **kw)
    else:
        def run(**kw):
            return B.lsq(method, g, bt, k_max, **kw)
    full = run(x_ref=xr)
    rel = full.err_hist / nrm
    dp = run(stop="dp", tau=tau, noise_norm=noise_norm)
    k_dp = dp.k_stop if dp.status == "ok" else None
    k_ncp = None
    if ncp:
        k_ncp = run(stop="ncp").k_stop
    k_min, e_min, e_dp, e_ncp = markers(rel, k_dp, k_ncp)
    return History(method, rel, k_min, e_min, k_dp, e_dp, k_ncp, e_ncp)
