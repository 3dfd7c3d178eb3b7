"""GPU tests of the request loop: continuous batching through few slots and a memory
budget that forces requests to wait; every result equals the same problem solved alone,
bit for bit (FP32 and BF16 basis)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _stream(abg, torch, n=20, rate=400.0, seed=3):
    g = np.random.default_rng(seed)
    t = np.cumsum(g.exponential(1.0 / rate, n))
    reqs = []
    from paper_2110_01481_amd.serving import Request
    for i in range(n):
        N = int(g.choice([24, 32, 48, 64]))
        n_ang = int(g.integers(20, 80))
        n_det = W.n_det_for(N)
        gg = abg.Geometry(N, n_ang, n_det, ang_range=180.0 if i % 3 else 120.0)
        x = torch.tensor(W.ellipse_phantom(N, 4, W.rng(91, i, 0)).ravel(), dtype=torch.float32,
                         device="cuda")
        bc = gg.fp(x).double().cpu().numpy()
        b, en = W.add_noise(bc, float(g.uniform(0.01, 0.03)), W.rng(91, i, 1).standard_normal(bc.size))
        p = abg.Problem(g=gg, method="ab" if i % 2 else "ba", b=torch.tensor(b, dtype=torch.float32, device="cuda"),
                        k_max=int(g.integers(8, 40)), stop="dp", tau=1.02, noise_norm=en,
                        bp="adj" if i % 5 == 0 else "hat")
        reqs.append(Request(float(t[i]), p, keep_result=True))
    return reqs


@pytest.mark.parametrize("basis", ["f32", "bf16"])
def test_served_equals_alone(gpu_lib, basis):
    import torch
    abg = gpu_lib
    from paper_2110_01481_amd.serving import Server, solve_alone
    reqs = _stream(abg, torch)
    need = [abg.request_bytes(r.problem.g, r.problem.method, r.problem.k_max, "f32", basis, "dp")
            for r in reqs]
    budget = 3 * max(need)
    srv = Server(proj="f32", basis=basis, max_slots=4, budget_bytes=budget)
    rep = srv.run(reqs)
    srv.close()
    assert rep.n == len(reqs) and sum(rep.statuses.values()) == len(reqs)
    assert rep.peak_bytes <= budget and rep.peak_active <= 4
    assert rep.latency_p99_s >= rep.latency_p50_s > 0
    for i, r in enumerate(reqs):
        got = rep.results[i]
        ref = solve_alone(r.problem, proj="f32", basis=basis)
        assert got.k_stop == ref.k_stop and got.status == ref.status, i
        assert torch.equal(got.x, ref.x), i
        if basis == "f32" and got.status == "ok":
            assert got.res_norm <= 1.02 * r.problem.noise_norm
