"""Basis vectors longer than 2^21 elements: the streaming Gram-Schmidt variant (single
solves forced onto it, and the batched engine, which takes it for such vectors) and the
register variant agree with the FP64 oracle at a fixed iteration count."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

# (method, N, n_ang): BA has L = N^2 > 2^21, AB has L = n_ang * n_det > 2^21
CASES = [("ba", 1450, 30), ("ab", 96, 15400)]
K = 6


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("method,N,n_ang", CASES)
def test_streaming_gram_schmidt_matches_oracle(gpu_lib, method, N, n_ang):
    import torch
    abg = gpu_lib
    n_det = W.n_det_for(N)
    L = N * N if method == "ba" else n_ang * n_det
    assert L > 2 ** 21
    go = O.Geometry(N, n_ang, n_det)
    xb = W.ellipse_phantom(N, 6, W.rng(92, N, 0))
    b, _ = W.add_noise(go.A(xb), 0.01, W.rng(92, N, 1).standard_normal(go.m))
    f = O.ab_gmres if method == "ab" else O.ba_gmres
    ref = f(go.A, go.B_hat, b, K)
    gg = abg.Geometry(N, n_ang, n_det)
    bt = torch.tensor(b, dtype=torch.float64, device="cuda")
    reg = abg.gmres(method, gg, bt, K)
    abg.mgs_force_stream(True)
    try:
        stream = abg.gmres(method, gg, bt, K)
    finally:
        abg.mgs_force_stream(False)
    eng = abg.Engine(proj="f64", basis="f64", max_slots=1)
    batched = eng.run([abg.Problem(g=gg, method=method, b=bt, k_max=K, stop="none")])[0]
    eng.close()
    for name, r in (("register", reg), ("stream", stream), ("engine", batched)):
        err = _rel(r.x.cpu().numpy(), ref.x)
        ls = np.abs(np.asarray(r.ls_hist) - np.asarray(ref.ls_res[:K])).max() / ref.beta
        print(method, N, n_ang, name, r.k_done, f"{err:.2e}", f"{ls:.2e}")
        assert r.k_done == K and err <= 1e-9 and ls <= 1e-10
