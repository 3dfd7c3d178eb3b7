"""Writes the oracle's reference results for the full-size workloads (CPU, FP64).

Calls only the oracle and the seeded input generators. Usage:
    python tests/golden/make_oracle_golden.py 2     # 512^2, 720 x 725, DP (minutes)
    python tests/golden/make_oracle_golden.py 3     # 2048^2, 1800 x 2897, NCP (an hour)
    python tests/golden/make_oracle_golden.py 4     # the mix's 128^2 / 256^2 problems, DP
    python tests/golden/make_oracle_golden.py deep  # 80- and 140-step runs, no stop rule

Output: tests/golden/oracle_config<N>.json with, per solve, the stopping iteration, the
residual / NCP histories, the error history against the phantom (config 2) and a
fingerprint of the returned iterate (norm, inner products with seeded vectors, values at
seeded pixels); and the returned iterates whole, for element-by-element comparison:
tests/golden/oracle_config2_x.npz (the four 512^2 solves, FP64) and
tests/golden/oracle_config3_x.npy (the 2048^2 NCP iterate, rounded to FP32 to halve its
size: a relative floor of 6e-8 per element, far below the 1e-4 comparisons it serves).
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
    whole = {}
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
            whole[f"{method}_{kind}"] = r.x
            print(method, kind, r.k_stop, r.status, f"{time.time() - t0:.1f}s", flush=True)
    with open(out_path, "w") as fh:
        json.dump(res, fh)
    np.savez_compressed(os.path.join(HERE, "oracle_config2_x.npz"), **whole)


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
    np.save(os.path.join(HERE, "oracle_config3_x.npy"), r.x.astype(np.float32))


def _perturbed(b: np.ndarray, eps: float, seed: int = 17) -> np.ndarray:
    d = np.random.default_rng(seed).standard_normal(b.size)
    return b + eps * np.linalg.norm(b) * d / np.linalg.norm(d)


def _deep_case(f, go, b, K, ks, eps=1e-15):
    """K steps of the oracle without a stopping rule, the iterates at the steps ks, the
    GMRES residual history, and the sensitivity probe: the relative change of every x_k
    and of every GMRES residual norm when b moves by eps relative (a rounding-level
    change of the data: GPU-vs-oracle differences of the arithmetic are of that kind)."""
    ref = f(go.A, go.B_hat, b, K, keep_iterates=True)
    per = f(go.A, go.B_hat, _perturbed(b, eps), K, keep_iterates=True)
    sens_x = [float(np.linalg.norm(p - r) / np.linalg.norm(r)) for p, r in zip(per.iterates, ref.iterates)]
    sens_ls = [float(abs(p / r - 1.0)) for p, r in zip(per.ls_res, ref.ls_res)]
    out = {"ls_res": np.asarray(ref.ls_res), "res_norms": np.asarray(ref.res_norms),
           "sens_x": np.asarray(sens_x), "sens_ls": np.asarray(sens_ls), "ks": np.asarray(ks),
           "beta": np.asarray(ref.beta), "status": np.asarray(ref.status)}
    for k in ks:
        out[f"x{k}"] = ref.iterates[k - 1]
    return out


def _f32(v):
    return np.asarray(v, dtype=np.float32).astype(np.float64)


def _f32_rounded_case(f, go, b, ref):
    """The same run with every projector output, the data b and every stored basis vector
    rounded to FP32 (dots, norms and the small problem stay FP64): how far FP32 storage
    alone moves x_k and the GMRES residual norms from the FP64 run `ref`."""
    r = f(lambda v: _f32(go.A(v)), lambda v: _f32(go.B_hat(v)), _f32(b), len(ref["ls_res"]),
          keep_iterates=True, basis_round=_f32)
    out = {"d32_ls": np.abs(np.asarray(r.ls_res) / ref["ls_res"] - 1.0)}
    x_all = {int(k): ref[f"x{int(k)}"] for k in ref["ks"]}
    out["d32_x"] = np.array([np.linalg.norm(r.iterates[k - 1] - x_all[k]) / np.linalg.norm(x_all[k])
                             if k in x_all else np.nan for k in range(1, len(ref["ls_res"]) + 1)])
    return out


# Deep Krylov runs: vectors long enough for the multi-block Gram-Schmidt paths (more than
# 16384 elements for both methods), 80 steps without a stopping rule so that the iterates
# cross every Gram-Schmidt and Givens form; and the 64^2 problem for 140 steps, past the
# register forms of the Givens update (k > 127).
DEEP = {"N": 144, "n_ang": 360, "eta": 0.01, "K": 80, "ks": (15, 32, 63, 64, 65, 80), "cfg": 94}
GIVENS = {"K": 140, "ks": (64, 127, 128, 140)}


def deep_problem():
    d = DEEP
    n_det = W.n_det_for(d["N"])
    go = O.Geometry(d["N"], d["n_ang"], n_det)
    xb = W.ellipse_phantom(d["N"], 8, W.rng(d["cfg"], d["N"], W.STREAM_PHANTOM))
    b, enorm = W.add_noise(go.A(xb), d["eta"], W.rng(d["cfg"], d["N"], W.STREAM_NOISE).standard_normal(go.m))
    return go, xb, b, enorm


def givens_problem():
    w = W.CONFIG1
    go = O.Geometry(w.N, w.n_ang, w.n_det)
    xb = w.phantom()
    b, enorm = W.add_noise(go.A(xb), w.eta, w.noise_dir())
    return go, xb, b, enorm


def run_deep(out_path: str):
    res = {}
    go, _, b, _ = deep_problem()
    for method, f in (("ab", O.ab_gmres), ("ba", O.ba_gmres)):
        t0 = time.time()
        case = _deep_case(f, go, b, DEEP["K"], DEEP["ks"])
        case.update(_f32_rounded_case(f, go, b, case))
        for k, v in case.items():
            res[f"deep_{method}_{k}"] = v
        print("deep", method, f"{time.time() - t0:.1f}s", flush=True)
    go, _, b, _ = givens_problem()
    for method, f in (("ab", O.ab_gmres), ("ba", O.ba_gmres)):
        t0 = time.time()
        for k, v in _deep_case(f, go, b, GIVENS["K"], GIVENS["ks"]).items():
            res[f"givens_{method}_{k}"] = v
        print("givens", method, f"{time.time() - t0:.1f}s", flush=True)
    np.savez_compressed(out_path, **res)


def run_batched(out_path: str):
    """The 128^2 and 256^2 problems of the 64-problem mix (DP, tau = 1.02, k_max = 100),
    b = A x_bar + e with the oracle's A: stopping iteration, status and iterate (FP32)."""
    res = {}
    for w in W.batched_workloads():
        if w.N > 256:
            continue
        t0 = time.time()
        go = O.Geometry(w.N, w.n_ang, w.n_det, ang_range=w.ang_range)
        b, enorm = W.add_noise(go.A(w.phantom()), w.eta, w.noise_dir())
        f = O.ab_gmres if w.method == "ab" else O.ba_gmres
        r = f(go.A, go.B_hat, b, w.k_max, stop="dp", tau=w.tau, noise_norm=enorm)
        res[f"i{w.instance}_k_stop"] = np.asarray(r.k_stop)
        res[f"i{w.instance}_status"] = np.asarray(r.status)
        res[f"i{w.instance}_res_norms"] = np.asarray(r.res_norms)
        res[f"i{w.instance}_x"] = r.x.astype(np.float32)
        print(w.instance, w.N, w.n_ang, w.method, r.k_stop, r.status, f"{time.time() - t0:.1f}s",
              flush=True)
    np.savez_compressed(out_path, **res)


if __name__ == "__main__":
    cfg = sys.argv[1]
    if cfg == "deep":
        out = os.path.join(HERE, "oracle_deep.npz")
        run_deep(out)
    elif cfg == "4":
        out = os.path.join(HERE, "oracle_config4_small.npz")
        run_batched(out)
    else:
        out = os.path.join(HERE, f"oracle_config{cfg}.json")
        {2: run_config2, 3: run_config3}[int(cfg)](out)
    print("wrote", out)
