"""Independent Krylov-subspace minimisers used to pin the GMRES oracle (test only).

Sec. 2 states what the k-th iterates are, independently of how Arnoldi builds them:
  AB-GMRES: x_k in x_0 + K_k(BA, B r_0) minimising ||b - A x||_2;
  BA-GMRES: x_k in x_0 + K_k(BA, B r_0) minimising ||B(b - A x)||_2.
Sec. 5 adds that with B = A^T these are the LSQR and LSMR iterates. The functions here
build an orthonormal basis of the Krylov space from the power sequence with a
Householder QR (numpy.linalg.qr) and minimise with numpy.linalg.lstsq, and run
Golub-Kahan bidiagonalisation with full reorthogonalisation for the matched case.
"""
from __future__ import annotations

import numpy as np


def krylov_basis(M, v0: np.ndarray, k: int) -> np.ndarray:
    """Orthonormal basis (columns) of span{v0, M v0, ..., M^{k-1} v0}.

    Each new power is normalised before the QR to keep the columns comparable; the
    span is unchanged."""
    cols = [v0 / np.linalg.norm(v0)]
    for _ in range(1, k):
        v = M(cols[-1])
        cols.append(v / np.linalg.norm(v))
    Q, _ = np.linalg.qr(np.stack(cols, axis=1))
    return Q


def min_residual_iterate(method: str, A, B, b: np.ndarray, k: int, x0=None) -> np.ndarray:
    """x_k of AB-/BA-GMRES by direct minimisation over x_0 + K_k(BA, B r_0), r_0 = b - A x_0
    (x_0 = 0 if not given): AB minimises ||b - A x||, BA ||B(b - A x)|| (Sec. 2)."""
    r0 = b if x0 is None else b - A(x0)
    Q = krylov_basis(lambda v: B(A(v)), B(r0), k)
    AQ = np.stack([A(Q[:, j]) for j in range(k)], axis=1)
    if method == "ab":
        c = np.linalg.lstsq(AQ, r0, rcond=None)[0]
    else:
        BAQ = np.stack([B(AQ[:, j]) for j in range(k)], axis=1)
        c = np.linalg.lstsq(BAQ, B(r0), rcond=None)[0]
    return Q @ c if x0 is None else x0 + Q @ c


def _golub_kahan(A, AT, b, k):
    """Lower-bidiagonalisation A V_k = U_{k+1} Bk with full reorthogonalisation."""
    m = b.size
    beta1 = np.linalg.norm(b)
    U = [b / beta1]
    v = AT(U[0])
    alpha = np.linalg.norm(v)
    V = [v / alpha]
    Bk = np.zeros((k + 1, k))
    Bk[0, 0] = alpha
    for j in range(k):
        u = A(V[j]) - Bk[j, j] * U[j]
        for ui in U:
            u -= (ui @ u) * ui
        beta = np.linalg.norm(u)
        U.append(u / beta)
        Bk[j + 1, j] = beta
        if j + 1 < k:
            v = AT(U[j + 1]) - beta * V[j]
            for vi in V:
                v -= (vi @ v) * vi
            alpha = np.linalg.norm(v)
            V.append(v / alpha)
            Bk[j + 1, j + 1] = alpha
    return beta1, np.stack(U, axis=1), np.stack(V, axis=1), Bk


def golub_kahan_lsqr(A, AT, b, k):
    """LSQR iterate x_k (minimises ||b - A x|| over K_k(A^T A, A^T b)) via GK with
    full reorthogonalisation."""
    beta1, U, V, Bk = _golub_kahan(A, AT, b, k)
    rhs = np.zeros(k + 1)
    rhs[0] = beta1
    y = np.linalg.lstsq(Bk, rhs, rcond=None)[0]
    return V @ y


def golub_kahan_lsmr(A, AT, b, k):
    """LSMR iterate x_k (minimises ||A^T(b - A x)|| over the same space)."""
    beta1, U, V, Bk = _golub_kahan(A, AT, b, k)
    ATAV = np.stack([AT(A(V[:, j])) for j in range(k)], axis=1)
    y = np.linalg.lstsq(ATAV, AT(b), rcond=None)[0]
    return V @ y
