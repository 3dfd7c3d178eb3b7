"""Writes the oracle's reference results for the full-size workloads (CPU, FP64).

Calls only the oracle and the seeded input generators. Usage:
    python tests/golden/make_oracle_golden.py 2     # 512^2, 720 x 725, DP (minutes)
    python tests/golden/make_oracle_golden.py 3     # 2048^2, 1800 x 2897, NCP (an hour)

Output: tests/golden/oracle_config<N>.json with, per solve, the stopping iteration, the
residual / NCP histories, the error history against the phantom (config 2) and a
fingerprint of the returned iterate (norm, inner products with seeded vectors, values at
seeded pixels) that GPU tests compare with.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

N_PIX = 2000
N_PROBES = 4


def fingerprint(x: np.ndarray, seed: int = 99) -> dict:
    rng = np.random.default_rng(seed)
    pix = np.sort(rng.choice(x.size, size=min(N_PIX, x.size), replace=False))
    probes = [rng.standard_normal(x.size) for _ in range(N_PROBES)]
    return {"norm": float(np.linalg.norm(x)),
            "probe_dots": [float(v @ x) for v in probes],
            "pixels": pix.tolist(),
            "values": x[pix].tolist()}


def run_config2(out_path: str):
    w = W.CONFIG2
    g = O.Geometry(w.N, w.n_ang, w.n_det)
    xb = w.phantom()
    b, enorm = W.add_noise(g.A(xb), w.eta, w.noise_dir())
    res = {"workload": "512x512, 720 angles in [0,180), 725 bins, 20 ellipses, 2% noise",
           "noise_norm": enorm, "tau": w.tau, "k_max": w.k_max, "solves": {}}
    for method, f in (("ab", O.ab_gmres), ("ba", O.ba_gmres)):
        for kind in ("hat", "adj"):
            t0 = time.time()
            r = f(g.A, g.back(kind), b, w.k_max, stop="dp", tau=w.tau, noise_norm=enorm,
                  keep_iterates=True)
            res["solves"][f"{method}-{kind}"] = {
                "k_stop": r.k_stop, "status": r.status, "res_norms": r.res_norms,
                "dp_margin": r.dp_margin, "ls_res": r.ls_res,
                "error_vs_truth": float(np.linalg.norm(r.x - xb) / np.linalg.norm(xb)),
                # error history (Sec. 6.2): ||x_k - x_bar|| and ||x_k|| for k = 1..k_stop
                "err_norms": [float(np.linalg.norm(x - xb)) for x in r.iterates],
                "x_norms": [float(np.linalg.norm(x)) for x in r.iterates],
                "x": fingerprint(r.x), "seconds": time.time() - t0}
            print(method, kind, r.k_stop, r.status, f"{time.time() - t0:.1f}s", flush=True)
    with open(out_path, "w") as fh:
        json.dump(res, fh)


def run_config3(out_path: str, k_fixed=(3, 6)):
    w = W.CONFIG3
    g = O.Geometry(w.N, w.n_ang, w.n_det)
    xb = w.phantom()
    b, enorm = W.add_noise(g.A(xb), w.eta, w.noise_dir())
    t0 = time.time()
    r = O.ba_gmres(g.A, g.B_hat, b, w.k_max, stop="ncp", ncp_shape=(g.n_ang, g.n_det),
                   keep_iterates=True)
    fixed = {str(k): fingerprint(r.iterates[k - 1]) for k in k_fixed if k <= len(r.iterates)}
    res = {"workload": "2048x2048, 1800 angles in [0,180), 2897 bins, 50 ellipses, 1% noise",
           "noise_norm": enorm, "k_max": w.k_max,
           "solves": {"ba-hat": {"k_stop": r.k_stop, "status": r.status,
                                 "ncp": r.ncp, "res_norms": r.res_norms, "ls_res": r.ls_res,
                                 "error_vs_truth": float(np.linalg.norm(r.x - xb) / np.linalg.norm(xb)),
                                 "x": fingerprint(r.x), "fixed_k": fixed,
                                 "seconds": time.time() - t0}}}
    print("ba hat", r.k_stop, r.status, f"{time.time() - t0:.1f}s", flush=True)
    with open(out_path, "w") as fh:
        json.dump(res, fh)


if __name__ == "__main__":
    cfg = int(sys.argv[1])
    out = os.path.join(HERE, f"oracle_config{cfg}.json")
    {2: run_config2, 3: run_config3}[cfg](out)
    print("wrote", out)
