"""AB-GMRES and BA-GMRES, step by step as listed in Sec. 2 (test infrastructure only).

For k = 1, 2, ...:
  q_k = A B w_k (AB)  or  q_k = B A w_k (BA);
  modified Gram-Schmidt: for i = 1..k, h_{i,k} = q_k^T w_i, q_k <- q_k - h_{i,k} w_i
  (one pass, ascending i, no reorthogonalisation);
  h_{k+1,k} = ||q_k||_2, w_{k+1} = q_k / h_{k+1,k};
  y_k = argmin_y || ||r_0|| e_1 - H_k y ||_2, solved from scratch each k with
  numpy.linalg.lstsq on the (k+1) x k Hessenberg matrix;
  x_k = x_0 + B [w_1..w_k] y_k (AB)  or  x_0 + [w_1..w_k] y_k (BA);
  r_k = b - A x_k, then the stopping rule.
with r_0 = b - A x_0 (AB) and r_0 = B b - B A x_0 (BA), w_1 = r_0/||r_0||.

Optional `basis_round` rounds every stored basis vector w_k (e.g. bf16_round): the
reduced-precision storage variant, in which the operator is applied to the stored
vector; everything else stays FP64.

Readings where the listing is silent: x_0 = 0 unless given; the stopping rule is
checked from k = 1; a breakdown h_{k+1,k} <= 1e-14 ||A B w_k|| (resp. ||B A w_k||)
ends the iteration with y_k from the square k x k part of H_k; the discrepancy
principle without a crossing up to k_max returns x_{k_max} as "not_converged".
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .stopping import ncp_distance

BREAKDOWN_REL = 1e-14


@dataclass
class GmresResult:
    x: np.ndarray
    k_stop: int
    k_done: int
    status: str
    res_norms: list = field(default_factory=list)      # ||b - A x_k||, k = 1..k_done
    ls_res: list = field(default_factory=list)         # || ||r0|| e1 - H_k y_k ||
    ncp: list = field(default_factory=list)            # d_k (NCP runs only)
    dp_margin: list = field(default_factory=list)      # (||r_k|| - tau||e||)/(tau||e||)
    H: np.ndarray | None = None
    W: np.ndarray | None = None
    ys: list = field(default_factory=list)
    iterates: list = field(default_factory=list)
    beta: float = 0.0


def bf16_round(v: np.ndarray) -> np.ndarray:
    """Round to float32 (nearest), then to the nearest bfloat16 (8 significant bits,
    ties to even), returned as float64. Storage rounding of the reduced-precision basis
    variant, which is not part of the paper's method."""
    f = np.asarray(v, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def _gmres(method, A, B, b, k_max, stop="none", tau=1.0, noise_norm=0.0, x0=None,
           ncp_shape=None, keep_iterates=False, keep_basis=False, basis_round=None):
    b = np.asarray(b, dtype=np.float64)
    n = B(np.zeros_like(b)).size
    x0 = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64)
    rb0 = b - A(x0)
    r0 = rb0 if method == "ab" else B(rb0)
    beta = float(np.linalg.norm(r0))
    res = GmresResult(x=x0.copy(), k_stop=0, k_done=0, status="ok", beta=beta)
    if beta == 0.0:
        res.status = "zero_rhs"
        return res
    L = r0.size
    W = np.zeros((k_max + 1, L))
    H = np.zeros((k_max + 1, k_max))
    W[0] = r0 / beta
    if basis_round is not None:
        W[0] = basis_round(W[0])
    thr = tau * noise_norm
    prev_x = None
    best = (np.inf, 0, None)
    for k in range(1, k_max + 1):
        w = W[k - 1]
        q = A(B(w)) if method == "ab" else B(A(w))
        q_norm0 = float(np.linalg.norm(q))
        for i in range(k):
            h = float(q @ W[i])
            H[i, k - 1] = h
            q = q - h * W[i]
        hk = float(np.linalg.norm(q))
        H[k, k - 1] = hk
        breakdown = hk <= BREAKDOWN_REL * q_norm0
        rhs = np.zeros(k + 1)
        rhs[0] = beta
        if breakdown:
            y = np.linalg.lstsq(H[:k, :k], rhs[:k], rcond=None)[0]
        else:
            W[k] = q / hk
            if basis_round is not None:
                W[k] = basis_round(W[k])
            y = np.linalg.lstsq(H[:k + 1, :k], rhs, rcond=None)[0]
        t = W[:k].T @ y
        x = x0 + (B(t) if method == "ab" else t)
        r = b - A(x)
        rn = float(np.linalg.norm(r))
        res.res_norms.append(rn)
        res.ls_res.append(float(np.linalg.norm(rhs - H[:k + 1, :k] @ y)))
        res.ys.append(y.copy())
        if thr > 0:
            res.dp_margin.append((rn - thr) / thr)
        if keep_iterates:
            res.iterates.append(x.copy())
        res.k_done = k
        if stop == "dp" and rn <= thr:
            res.x, res.k_stop, res.status = x, k, "ok"
            break
        if stop == "ncp":
            d = ncp_distance(r, *ncp_shape)
            res.ncp.append(d)
            if k >= 2 and d > res.ncp[-2]:
                res.x, res.k_stop, res.status = prev_x, k - 1, "ok"
                break
            if d < best[0]:
                best = (d, k, x)
            prev_x = x
        if breakdown:
            res.x, res.k_stop, res.status = x, k, "breakdown"
            break
        if k == k_max:
            if stop == "ncp":
                res.x, res.k_stop, res.status = best[2], best[1], "ok"
            else:
                res.x, res.k_stop = x, k
                res.status = "not_converged" if stop == "dp" else "ok"
    res.H = H[:res.k_done + 1, :res.k_done]
    if keep_basis:
        res.W = W[:res.k_done + 1]
    return res


def ab_gmres(A, B, b, k_max, **kw) -> GmresResult:
    """AB-GMRES: GMRES on min_u ||b - A B u||, x = B u (B as right preconditioner)."""
    return _gmres("ab", A, B, b, k_max, **kw)


def ba_gmres(A, B, b, k_max, **kw) -> GmresResult:
    """BA-GMRES: GMRES on min_x ||B b - B A x|| (B as left preconditioner)."""
    return _gmres("ba", A, B, b, k_max, **kw)
