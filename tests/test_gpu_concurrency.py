"""Concurrent single solves: host threads, each on its own stream with its own
workspaces, give bit for bit the results of the same solves run one after another (the
library's pooled host state, its locks and the fixed-order reductions make a solve's
arithmetic independent of what else runs). Multi-block Gram-Schmidt groups of concurrent
solves and engine rounds are admitted on the host against what the device holds."""
import threading

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _problems():
    out = []
    for inst, (N, n_ang) in enumerate(((64, 90), (128, 180), (256, 90))):
        w = W.Workload(cfg=7, instance=inst, N=N, n_ang=n_ang, n_det=W.n_det_for(N),
                       n_ellipses=5, eta=0.02, k_max=40, stop="dp", tau=1.02)
        go = O.Geometry(w.N, w.n_ang, w.n_det)
        b, enorm = W.add_noise(go.A(w.phantom()), w.eta, w.noise_dir())
        out.append((w, b, enorm))
    return out


def test_two_threads_match_sequential(gpu_lib):
    import torch
    import paper_2110_01481_amd as abg
    probs = _problems()
    jobs = []
    for w, b, enorm in probs:
        gg = abg.Geometry(w.N, w.n_ang, w.n_det)
        bt = torch.tensor(b, dtype=torch.float32, device="cuda")
        for meth in ("ab", "ba"):
            jobs.append(("gmres", meth, gg, bt, enorm))
        jobs.append(("lsq", "lsqr", gg, bt, enorm))

    def run(job, stream=None):
        kind, meth, gg, bt, enorm = job
        if kind == "gmres":
            return abg.gmres(meth, gg, bt, 40, stop="dp", tau=1.02, noise_norm=enorm, stream=stream)
        return abg.lsq(meth, gg, bt, 40, stop="dp", tau=1.02, noise_norm=enorm, stream=stream)

    ref = [run(j) for j in jobs]
    results = [None] * len(jobs)
    errors = []

    def worker(idx):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for i in idx:
                    results[i] = run(jobs[i], stream=s)
            s.synchronize()
        except Exception as e:   # reported by the main thread
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(list(range(t, len(jobs), 2)),))
               for t in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not errors, errors
    for r, q in zip(results, ref):
        assert r is not None and r.status == q.status and r.k_stop == q.k_stop
        assert torch.equal(r.x, q.x)
        assert np.array_equal(r.res_hist, q.res_hist)


def test_large_concurrent_solves_and_engine_are_admitted(gpu_lib):
    """Four host threads each run a 2048^2 BA-GMRES solve (FP32; basis vectors of 4.2M
    elements: the streaming Gram-Schmidt variant, a group of 512 blocks that must be
    resident at once) while a fifth runs an engine round by round on four 512^2 problems
    (its Gram-Schmidt grids take the whole device). More groups than the device holds
    would wait on each other on the device; the host-side admission makes the launches
    wait for capacity instead, so every solve completes (no bounded-wait error) and gives
    bit for bit the result of the same solve run alone."""
    import torch
    import paper_2110_01481_amd as abg
    big = abg.Geometry(2048, 120, W.n_det_for(2048))
    small = abg.Geometry(512, 180, W.n_det_for(512))
    bb = [big.fp(torch.tensor(W.ellipse_phantom(2048, 8, W.rng(8, j, 0)), dtype=torch.float32,
                              device="cuda")) for j in range(4)]
    bs = [small.fp(torch.tensor(W.ellipse_phantom(512, 8, W.rng(8, 10 + j, 0)), dtype=torch.float32,
                                device="cuda")) for j in range(4)]
    torch.cuda.synchronize()
    K = 6
    ref_big = [abg.gmres("ba", big, b, K) for b in bb]
    eng = abg.Engine(proj="f32", basis="f32", max_slots=4, stream=torch.cuda.Stream())
    probs = [abg.Problem(g=small, method=m, b=b, k_max=K, stop="none")
             for b, m in zip(bs, ("ab", "ba", "ab", "ba"))]
    ref_small = eng.run(probs)
    out_big = [None] * 4
    out_small = []
    errors = []

    def solve(j):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                out_big[j] = abg.gmres("ba", big, bb[j], K, stream=s)
            s.synchronize()
        except Exception as e:   # reported by the main thread
            errors.append(e)

    def engine():
        try:
            out_small.extend(eng.run(probs))
        except Exception as e:   # reported by the main thread
            errors.append(e)

    threads = [threading.Thread(target=solve, args=(j,)) for j in range(4)]
    threads.append(threading.Thread(target=engine))
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=300)
    eng.close()
    assert not errors, errors
    for r, q in zip(out_big, ref_big):
        assert r is not None and r.status == "ok" and r.k_done == K
        assert torch.equal(r.x, q.x)
    assert len(out_small) == 4
    for r, q in zip(out_small, ref_small):
        assert r.status == q.status and torch.equal(r.x, q.x)
