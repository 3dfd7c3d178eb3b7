"""Stopping rules of Sec. 6.3 (test infrastructure only).

Discrepancy principle (eq. 6.1): k_DP is the smallest k with ||b - A x_k||_2 <= tau ||e||_2.

NCP criterion: the paper defers its details to other sources. The reading used here is
the normalised cumulative periodogram of Hansen, Kilmer & Kjeldsen (BIT 2006), applied
to each projection (sinogram row) of the residual:
  1. r_hat = DFT of the row (length n_det); q = floor(n_det/2);
     p_j = |r_hat_j|^2 for j = 1..q (the constant term j = 0 is left out);
  2. c(j) = sum_{l<=j} p_l / sum_{l<=q} p_l (c = white-noise line if the row is zero);
  3. cbar = mean of c over the rows; d_k = ||cbar - c_white||_2 with c_white(j) = j/q;
  4. k_NCP = first k with d_{k+1} > d_k (the residual was closest to white noise at k);
     if d never increases up to k_max, the k of the smallest d.
"""
from __future__ import annotations

import numpy as np


def ncp_distance(r: np.ndarray, n_ang: int, n_det: int) -> float:
    R = np.asarray(r, dtype=np.float64).reshape(n_ang, n_det)
    F = np.fft.fft(R, axis=1)
    q = n_det // 2
    P = np.abs(F[:, 1:q + 1]) ** 2
    total = P.sum(axis=1, keepdims=True)
    white = np.arange(1, q + 1, dtype=np.float64) / q
    safe = np.where(total > 0.0, total, 1.0)
    C = np.where(total > 0.0, np.cumsum(P, axis=1) / safe, white[None, :])
    cbar = C.mean(axis=0)
    return float(np.linalg.norm(cbar - white))


def dp_index(res_norms, tau: float, noise_norm: float):
    """1-based smallest k with res_norms[k-1] <= tau*noise_norm, or None."""
    thr = tau * noise_norm
    for k, r in enumerate(res_norms, start=1):
        if r <= thr:
            return k
    return None


def ncp_index(dists):
    """1-based k_NCP from d_1, d_2, ...: first k with d_{k+1} > d_k, else argmin."""
    for k in range(1, len(dists)):
        if dists[k] > dists[k - 1]:
            return k, True
    return int(np.argmin(dists)) + 1, False
