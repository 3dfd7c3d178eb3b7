"""Concurrent single solves: two host threads, each on its own stream with its own
workspaces, give bit for bit the results of the same solves run one after another (the
library's per-thread host state, its locks and the fixed-order reductions make a solve's
arithmetic independent of what else runs). Problems are small enough that the
Gram-Schmidt groups of both solves fit on the device at once."""
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
