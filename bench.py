"""Benchmark: GMRES iterations per second of AB- and BA-GMRES on one MI355X.

Workload (default): the single-solve case -- 512 x 512 image, 720 angles in [0,180),
725 bins, 20-ellipse phantom, 2% Gaussian noise, FP32 projectors with the FP64
Hessenberg/Givens solve, discrepancy-principle stop (tau = 1.02, k_max = 100), unmatched
pair (line-model A, interpolating B). One step = one AB-GMRES solve plus one BA-GMRES
solve; the metric counts their Arnoldi iterations.

Prints one JSON line. `roofline` covers the kernel with the largest share of the timed
region, measured with HIP events on the solver's stream; `cpu_baseline` times the FP64
oracle (AB-GMRES, literal algorithm) on a bounded number of iterations of the same
workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBPS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
_CSRC = "paper_2110_01481_amd/csrc/"
# kernels whose stored counter summaries (profiles/<kernel>_<workload>_counters.md) bench.py
# reads: the kernel-name prefix in rocprofv3's CSV and the sources whose change makes the
# stored readings stale
COUNTER_KERNELS = {
    "forward_kernel_f32": ("forward_kernel<float>",
                           [_CSRC + "fwd_body.h", _CSRC + "geometry.h", _CSRC + "projectors.hip"]),
    "forward_kernel_f64": ("forward_kernel<double>",
                           [_CSRC + "fwd_body.h", _CSRC + "geometry.h", _CSRC + "projectors.hip"]),
    "back_kernel_f64": ("back_kernel<double, false, false, true>",
                        [_CSRC + "back_body.h", _CSRC + "geometry.h", _CSRC + "projectors.hip"]),
    "back_kernel_f32": ("back_kernel<float, false, false, true>",
                        [_CSRC + "back_body.h", _CSRC + "geometry.h", _CSRC + "projectors.hip"]),
}
# kernels of a solve whose L2 hit rate the TCC pass reports
L2_KERNELS = ("forward_kernel", "back_kernel", "mgs_kernel", "mgs_stream_kernel",
              "combine_kernel", "ncp_fft_rows_kernel", "ncp_colsum_kernel")


def progress(msg: str):
    """One progress line on stderr (stdout carries only the result line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def source_hash(kernel_key: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in COUNTER_KERNELS[kernel_key][1]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def forward_source_hash() -> str:
    return source_hash("forward_kernel_f32")


def _counter_means(csv_path: str, kernel_prefix: str) -> dict:
    import csv
    sums, counts = {}, {}
    with open(csv_path) as fh:
        for r in csv.DictReader(fh):
            name = r["Kernel_Name"].replace("abg::(anonymous namespace)::", "").replace("void ", "")
            if not name.startswith(kernel_prefix):
                continue
            c = r["Counter_Name"]
            sums[c] = sums.get(c, 0.0) + float(r["Counter_Value"])
            counts[c] = counts.get(c, 0) + 1
    return {c: sums[c] / counts[c] for c in sums}


def summarize_counters(d: str, kernel_key: str = "forward_kernel_f32",
                       workload: str = "512x512, 720 x 725, FP32", bench_args: str = "") -> str:
    """Markdown summary of the FETCH_SIZE / WRITE_SIZE passes under directory d (sub-
    directories fetch, write, cfetch, cwrite, and optionally sq and l2, as written by the
    commands listed in it) for the kernel `kernel_key` of COUNTER_KERNELS."""
    kname = COUNTER_KERNELS[kernel_key][0]
    f = _counter_means(os.path.join(d, "fetch", "run_counter_collection.csv"), kname)
    w = _counter_means(os.path.join(d, "write", "run_counter_collection.csv"), kname)
    cf = _counter_means(os.path.join(d, "cfetch", "run_counter_collection.csv"), "__amd_rocclr_copyBuffer")
    cw = _counter_means(os.path.join(d, "cwrite", "run_counter_collection.csv"), "__amd_rocclr_copyBuffer")
    copy_kib = 1024 * 1024
    data = {"kernel": kname, "workload": workload,
            "fetch_kib_per_dispatch": round(f["FETCH_SIZE"], 1),
            "write_kib_per_dispatch": round(w["WRITE_SIZE"], 1),
            "copy_kib": copy_kib,
            "copy_fetch_kib": round(cf["FETCH_SIZE"], 1), "copy_write_kib": round(cw["WRITE_SIZE"], 1),
            "fetch_scale": round(copy_kib / cf["FETCH_SIZE"], 4),
            "write_scale": round(copy_kib / cw["WRITE_SIZE"], 4),
            "source_hash": source_hash(kernel_key)}
    data["traffic_bytes_per_launch"] = int(1024 * (data["fetch_kib_per_dispatch"] * data["fetch_scale"] +
                                                   data["write_kib_per_dispatch"] * data["write_scale"]))
    sq_csv = os.path.join(d, "sq", "run_counter_collection.csv")
    if os.path.exists(sq_csv):
        sq = _counter_means(sq_csv, kname)
        data["valu_wave_insts_per_dispatch"] = round(sq["SQ_INSTS_VALU"], 1)
        if "SQ_INSTS_VMEM_RD" in sq:
            data["vmem_read_wave_insts_per_dispatch"] = round(sq["SQ_INSTS_VMEM_RD"], 1)
    l2_csv = os.path.join(d, "l2", "run_counter_collection.csv")
    if os.path.exists(l2_csv):
        # L2 (TCC) hit rate = hits / (hits + misses) per kernel of the solve
        data["l2_hit_rate"] = {}
        for k in L2_KERNELS:
            m = _counter_means(l2_csv, k)
            hit, miss = m.get("TCC_HIT_sum", 0.0), m.get("TCC_MISS_sum", 0.0)
            if hit + miss > 0:
                data["l2_hit_rate"][k] = round(hit / (hit + miss), 4)
    b = "python -u bench.py " + (bench_args or "--config 2 --steps 2 --warmup 1 --quick")
    c = "python -u bench.py --copy-calibration-mib 1024"
    sqc = ("SQ_WAVES SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_INSTS_VALU SQ_INSTS_VMEM_RD "
           "SQ_ACTIVE_INST_VALU SQ_WAIT_ANY GRBM_GUI_ACTIVE")
    lines = [
        f"# HBM traffic of {kname} ({workload})",
        "",
        f"Counters per dispatch of `{kname}`, averaged over the dispatches of the",
        "run, and of the plain device copy of 1 GiB (`__amd_rocclr_copyBuffer`) that calibrates",
        "them: the copy reads and writes exactly 1 GiB, so each counter is scaled by",
        "1 GiB / (its reading on the copy).",
        "",
        "Commands (each a run of its own, from the repository root, `TMPDIR=/tmp`):",
        "",
        f"    rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/fetch -o run -- {b}",
        f"    rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/write -o run -- {b}",
        f"    rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/cfetch -o run -- {c}",
        f"    rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/cwrite -o run -- {c}",
        f"    rocprofv3 --pmc {sqc} --output-format csv -d <dir>/sq -o run -- {b}",
        f"    rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum --output-format csv -d <dir>/l2 -o run -- {b}",
        f"    python bench.py --summarize-counters <dir> --counter-kernel {kernel_key}",
        "",
        "The SQ pass gives the VALU instructions per dispatch (wave level; x 64 lanes for",
        "the lane operations that bench.py sets against the VALU issue rate); the TCC pass",
        "the L2 hit rate, hits / (hits + misses), of each kernel of the solve.",
        "",
        "`source_hash` covers the kernel's sources; bench.py reports `traffic` only while it",
        "matches.",
        "",
        "```json",
        json.dumps(data, indent=1),
        "```",
        ""]
    return "\n".join(lines)


def summarize_kernel_stats(d: str, title: str, command: str) -> str:
    """Text summary of a `rocprofv3 --kernel-trace --stats --output-format csv` run under
    directory d: calls, average and total time and share per kernel (run_kernel_stats.csv),
    and the average over launches longer than 20 us per kernel (run_kernel_trace.csv:
    launches of steps enqueued past a stop return at entry in a few microseconds)."""
    import csv
    import glob

    def find(name):
        hits = glob.glob(os.path.join(d, "**", name), recursive=True)
        if not hits:
            raise FileNotFoundError(f"{name} under {d}")
        return hits[0]

    def short(n):
        n = n.replace("abg::(anonymous namespace)::", "").replace("void ", "")
        return n.split("(")[0] if "(" in n else n

    rows = []
    with open(find("run_kernel_stats.csv")) as fh:
        for r in csv.DictReader(fh):
            rows.append((short(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                         float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    long_runs = {}
    with open(find("run_kernel_trace.csv")) as fh:
        for r in csv.DictReader(fh):
            us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            if us > 20.0:
                k = short(r["Kernel_Name"])
                n, t = long_runs.get(k, (0, 0.0))
                long_runs[k] = (n + 1, t + us)
    out = [f"# {title}", "", "Command (from the repository root, TMPDIR=/tmp):", "",
           f"    {command}", "",
           "Whole run (set-up, warm-up and the timed steps). Launches of steps enqueued past a",
           "stop return at entry (a few microseconds) and are counted in calls/avg of the table;",
           "the averages over launches longer than 20 us are listed below it.", "",
           f"{'kernel':<64s} {'calls':>7s} {'avg us':>9s} {'total ms':>9s} {'share':>6s}"]
    for name, calls, avg, tot, pct in sorted(rows, key=lambda r: -r[3]):
        out.append(f"{name[:64]:<64s} {calls:7d} {avg:9.1f} {tot:9.2f} {pct:5.1f}%")
    out.append("")
    for name, (n, t) in sorted(long_runs.items(), key=lambda kv: -kv[1][1]):
        out.append(f"{name}: {n} launches > 20 us, average {t / n:.1f} us")
    out.append("")
    return "\n".join(out)


def stored_counters(kernel_key: str, workload_tag: str) -> dict | None:
    """The stored counter summary of a kernel on a workload, if it was taken on the
    kernel's current sources."""
    path = os.path.join(PROFILES, f"{kernel_key}_{workload_tag}_counters.md")
    try:
        with open(path) as fh:
            text = fh.read()
        data = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    return data if data.get("source_hash") == source_hash(kernel_key) else None


FP32_VECTOR_PEAK_TFLOPS = 157.3
VALU_ISSUE_PEAK = 256 * 4 * 16 * 2.4e9   # lane operations per second
FP64_VECTOR_PEAK_TFLOPS = 78.6


def line_model_nnz(N: int, theta_deg: np.ndarray, n_det: int, ds: float = 1.0) -> int:
    """Expected number of (ray, pixel) pairs with positive intersection length: a chord
    of length L in direction (-sin, cos) crosses grid lines at rate |cos| + |sin| per
    unit length, so it touches 1 + L(|cos| + |sin|) pixels (axis-aligned edge rays touch
    two pixels per band). Used only to count the algorithmic work of a forward apply."""
    total = 0.0
    s = (np.arange(n_det) - 0.5 * (n_det - 1)) * ds
    h = N / 2.0
    for th in theta_deg:
        rad = th * math.pi / 180.0
        c, sn = abs(math.cos(rad)), abs(math.sin(rad))
        if min(c, sn) < 1e-15:
            on_edge = np.abs((s + h) - np.round(s + h)) < 1e-9
            inside = np.abs(s) <= h
            total += float(np.sum(np.where(inside, np.where(on_edge, 2 * N, N), 0)))
            continue
        # chord of the line x cos + y sin = s through the square [-h, h]^2
        px, py = s * math.cos(rad), s * math.sin(rad)
        dx, dy = -math.sin(rad), math.cos(rad)
        ta, tb = (-h - px) / dx, (h - px) / dx
        tc, td = (-h - py) / dy, (h - py) / dy
        t0 = np.maximum(np.minimum(ta, tb), np.minimum(tc, td))
        t1 = np.minimum(np.maximum(ta, tb), np.maximum(tc, td))
        L = np.maximum(t1 - t0, 0.0)
        total += float(np.sum(np.where(L > 0, 1.0 + L * (c + sn), 0.0)))
    return int(round(total))


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _stream_kernel_stats(ms_total, launches, bytes_total, reductions=None):
    """Achieved HBM rate of a bandwidth-bound kernel from its algorithmic bytes."""
    if not launches or ms_total <= 0:
        return None
    out = {"launches": launches, "avg_us": round(1e3 * ms_total / launches, 2),
           "alg_bytes_per_launch": int(bytes_total / launches),
           "GBps": round(bytes_total / (ms_total * 1e-3) / 1e9, 1)}
    out["frac_hbm"] = round(out["GBps"] / HBM_PEAK_GBPS, 4)
    if reductions:
        out["grid_reductions"] = reductions
        out["us_per_reduction_upper"] = round(1e3 * ms_total / reductions, 2)
    return out


def cpu_oracle_baseline(w, b_np, enorm, budget_s=15.0, max_iters=10):
    """Times the FP64 oracle's AB-GMRES (unmatched pair) on the 512^2 workload for as many
    Arnoldi iterations as fit in ~budget_s seconds (each run from scratch)."""
    import oracle as O
    from oracle.core import num_threads
    g = O.Geometry(w.N, w.n_ang, w.n_det)
    k = 1
    while True:
        t0 = time.perf_counter()
        O.ab_gmres(g.A, g.B_hat, b_np, k)
        dt = time.perf_counter() - t0
        if dt * 2.2 > budget_s or k >= max_iters:
            return {"value": round(k / dt, 4), "unit": "GMRES iters/s", "cores": num_threads(),
                    "kind": "oracle", "host_cpu": _cpu_model(),
                    "sample": f"FP64 oracle AB-GMRES, {k} Arnoldi iterations from x0=0 on the "
                              f"{w.N}^2 / {w.n_ang}x{w.n_det} workload (literal x_k and b-Ax_k "
                              f"each step), {dt:.2f} s; host {os.cpu_count()} logical CPUs"}
        k = min(max_iters, k * 2)


def cpu_oracle_baseline_ncp(w, b_np, xb, arnoldi_steps=0):
    """The FP64 oracle on the 2048^2 NCP workload, on the host cores. A BA-GMRES
    iteration with the NCP rule applies A and B once (q = B A w_k), forms x_k = W_k y_k,
    applies A once more for the literal residual b - A x_k and evaluates its periodogram
    distance; its Gram-Schmidt and least squares cost O(k L) and O(k^3). The bounded
    sample times one oracle A apply (on the phantom), one B apply (on b) and one NCP
    distance (of b - A x_bar) and gives value = 1 / (2 t_A + t_B + t_NCP) iterations per
    second, an upper bound on the oracle's rate (its Gram-Schmidt is left out).
    arnoldi_steps > 0 also runs the oracle's BA-GMRES for that many iterations with its
    operators wrapped in timers, and reports the time per iteration after the set-up
    applies (B of a zero vector for the size, A x_0, B r_0)."""
    import oracle as O
    from oracle.core import num_threads
    g = O.Geometry(w.N, w.n_ang, w.n_det)
    t0 = time.perf_counter()
    ax = g.A(xb)
    t_a = time.perf_counter() - t0
    t0 = time.perf_counter()
    g.B_hat(b_np)
    t_b = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.ncp_distance(b_np - ax, g.n_ang, g.n_det)
    t_ncp = time.perf_counter() - t0
    it = 2 * t_a + t_b + t_ncp
    out = {"value": round(1.0 / it, 5), "unit": "GMRES iters/s", "cores": num_threads(),
           "kind": "oracle", "host_cpu": _cpu_model(),
           "A_apply_s": round(t_a, 3), "B_apply_s": round(t_b, 3), "ncp_s": round(t_ncp, 3),
           "sample": f"FP64 oracle on the {w.N}^2 / {w.n_ang}x{w.n_det} workload: one A apply "
                     f"({t_a:.1f} s), one B apply ({t_b:.1f} s) and one NCP distance "
                     f"({t_ncp:.2f} s); value = 1/(2 t_A + t_B + t_NCP), the operator and "
                     f"stopping-rule cost of one BA-GMRES iteration; host {os.cpu_count()} "
                     "logical CPUs"}
    if arnoldi_steps > 0:
        calls = []

        def timed(name, f):
            def run(v):
                t1 = time.perf_counter()
                r = f(v)
                calls.append((name, time.perf_counter() - t1))
                return r
            return run

        t0 = time.perf_counter()
        O.ba_gmres(timed("A", g.A), timed("B", g.B_hat), b_np, arnoldi_steps, stop="ncp",
                   ncp_shape=(g.n_ang, g.n_det))
        total = time.perf_counter() - t0
        setup = sum(dt for _, dt in calls[:3])    # B(0) for the size, A x_0, B r_0
        out["arnoldi"] = {"steps": arnoldi_steps, "s": round(total, 2),
                          "s_per_iteration": round((total - setup) / arnoldi_steps, 2),
                          "iters_per_s": round(arnoldi_steps / (total - setup), 5)}
    return out


def _dp_problem(abg, torch, gg, w, xt, dev, seed):
    """b = A x + e for the workload's phantom x (device forward projector), e Gaussian
    from a seeded device generator, scaled to ||e|| = eta ||A x||."""
    bc = gg.fp(xt)
    gg.release_workspace()
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    e = torch.randn(bc.numel(), generator=gen, device=dev, dtype=bc.dtype)
    e *= w.eta * torch.linalg.vector_norm(bc) / torch.linalg.vector_norm(e)
    b = bc + e
    return abg.Problem(g=gg, method=w.method, b=b, k_max=w.k_max, stop="dp", tau=w.tau,
                       noise_norm=float(torch.linalg.vector_norm(e.double())))


def _concurrent_solves(abg, torch, probs, n_threads=3):
    """The same single solves (FP32) spread over n_threads host threads, each on its own
    stream (largest problems dealt out first); returns (s, errors). Three streams keep the
    Gram-Schmidt groups that run at once within what the device holds."""
    import threading
    bs = [p.b.float() for p in probs]
    order = sorted(range(len(probs)), key=lambda i: -probs[i].g.n * probs[i].g.n_ang)
    parts = [order[t::n_threads] for t in range(n_threads)]
    errors = []

    def worker(idx):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                for i in idx:
                    p = probs[i]
                    abg.gmres(p.method, p.g, bs[i], p.k_max, stop=p.stop, tau=p.tau,
                              noise_norm=p.noise_norm, bp=p.bp, stream=st)
            st.synchronize()
        except Exception as e:   # reported by the caller
            errors.append(repr(e))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ths = [threading.Thread(target=worker, args=(part,)) for part in parts]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, errors


def _single_solves(abg, torch, probs, dtype):
    """Sequential single solves (the plain method) of the problems; returns (s, results)."""
    bs = [p.b.to(dtype) for p in probs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = [abg.gmres(p.method, p.g, b, p.k_max, stop=p.stop, tau=p.tau, noise_norm=p.noise_norm,
                     bp=p.bp) for p, b in zip(probs, bs)]
    torch.cuda.synchronize()
    return time.perf_counter() - t0, out


PAIRS = [("strip", "adj"), ("strip", "joseph_t"), ("line", "strip_t"), ("line", "joseph_t"),
         ("joseph", "adj"), ("joseph", "strip_t")]


def bench_models(abg, torch, dev, w, xb, reps=20):
    """The three forward models and four back projectors of the workload (time per apply,
    FP32), the six unmatched pairs (A, B = A'^T) of the paper's Table 6.3 and the pairs
    (A_s, B_tau) of Sec. 6.5 for the thresholds of Table 6.4, solved with AB- and BA-GMRES
    under the DP rule on this workload: stopping iteration, solve time and relative
    reconstruction error ||x - x_true|| / ||x_true||."""
    geo = {m: abg.Geometry(w.N, w.n_ang, w.n_det, ang_range=w.ang_range, model=m)
           for m in ("line", "strip", "joseph")}
    x = torch.tensor(xb, dtype=torch.float32, device=dev)
    xt = torch.tensor(xb, dtype=torch.float64, device=dev)

    def timed(fn):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {"apply_ms": {}}
    y = geo["line"].fp(x)
    for m, g in geo.items():
        out["apply_ms"]["A_" + m] = round(timed(lambda: g.fp(x)), 4)
    for k in ("hat", "adj", "strip_t", "joseph_t"):
        out["apply_ms"]["B_" + k] = round(timed(lambda: geo["line"].bp(y, k)), 4)
    pairs = {}
    for m, k in PAIRS:
        g = geo[m]
        bc = g.fp(xt)
        gen = torch.Generator(device=dev)
        gen.manual_seed(7)
        e = torch.randn(bc.numel(), generator=gen, device=dev, dtype=bc.dtype)
        e *= w.eta * torch.linalg.vector_norm(bc) / torch.linalg.vector_norm(e)
        b = (bc + e).float()
        enorm = float(torch.linalg.vector_norm(e))
        for meth in ("ab", "ba"):
            abg.gmres(meth, g, b, w.k_max, stop="dp", tau=w.tau, noise_norm=enorm, bp=k)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = abg.gmres(meth, g, b, w.k_max, stop="dp", tau=w.tau, noise_norm=enorm, bp=k)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            err = float(torch.linalg.vector_norm(r.x.double() - xt) / torch.linalg.vector_norm(xt))
            pairs[f"{meth}:A_{m},B_{k}"] = {"k_stop": r.k_stop, "ms": round(1e3 * dt, 3),
                                           "iters_per_s": round(r.k_done / dt, 1),
                                           "rel_error": round(err, 4)}
    out["pairs_dp"] = pairs
    # Sec. 6.5: (A_s, B_tau) for the thresholds of Table 6.4
    sweep = {}
    g = geo["strip"]
    bc = g.fp(xt)
    gen = torch.Generator(device=dev)
    gen.manual_seed(8)
    e = torch.randn(bc.numel(), generator=gen, device=dev, dtype=bc.dtype)
    e *= w.eta * torch.linalg.vector_norm(bc) / torch.linalg.vector_norm(e)
    b = (bc + e).float()
    enorm = float(torch.linalg.vector_norm(e))
    for tau in (0.0, 0.01, 0.1, 0.3, 0.5):
        mx = g.set_strip_threshold(tau)
        for meth in ("ab", "ba"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = abg.gmres(meth, g, b, w.k_max, stop="dp", tau=w.tau, noise_norm=enorm, bp="strip_tau")
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            err = float(torch.linalg.vector_norm(r.x.double() - xt) / torch.linalg.vector_norm(xt))
            sweep[f"{meth}:tau={tau:g}"] = {"k_stop": r.k_stop, "ms": round(1e3 * dt, 3),
                                           "rel_error": round(err, 4)}
    out["strip_b_tau_dp"] = sweep
    out["strip_max_entry"] = mx
    for g in geo.values():
        g.release_workspace()
    return out


def bench_histories(abg, torch, dev, w, xb, eta=0.003, K=150):
    """Error histories of Sec. 6.2 with the markers of Sec. 6.3 on the workload's geometry
    with the strip model A_s and noise ||e|| / ||A_s x|| = eta (the paper's histories use
    0.3%): AB- and BA-GMRES for (A_s, A_l^T) and (A_s, A_i^T), LSQR and LSMR on A_s, FP32.
    Per run: the minimum of ||x_k - x|| / ||x|| over k <= K and its k, k_DP (tau = 1) and
    k_NCP with the errors there, the curve every 5 steps, and the time of its three solves
    (the full history, DP, NCP)."""
    from paper_2110_01481_amd import history as Hh
    g = abg.Geometry(w.N, w.n_ang, w.n_det, ang_range=w.ang_range, model="strip")
    bc = g.fp(torch.tensor(xb, dtype=torch.float64, device=dev)).cpu().numpy()
    b, enorm = W.add_noise(bc, eta, W.rng(w.cfg, w.instance, 11).standard_normal(bc.size))
    out = {"workload": f"{w.N}x{w.N}, {w.n_ang} angles, {w.n_det} bins, A_s (strip model), "
                       f"{100 * eta:g}% noise, K = {K}, FP32 projectors and basis"}
    runs = [("ab", "adj"), ("ba", "adj"), ("ab", "joseph_t"), ("ba", "joseph_t"),
            ("lsqr", None), ("lsmr", None)]
    for meth, bp in runs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = Hh.error_history(meth, g, b, xb, K, enorm, tau=1.0, bp=bp or "adj", dtype="f32")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        name = f"{meth}:A_s,B_{bp}" if bp else f"{meth}:A_s"

        def r4(v):
            return None if v is None else round(v, 4)

        out[name] = {"k_min": h.k_min, "err_min": r4(h.err_min), "k_dp": h.k_dp,
                     "err_dp": r4(h.err_dp), "k_ncp": h.k_ncp, "err_ncp": r4(h.err_ncp),
                     "curve_every_5": [r4(float(v)) for v in h.rel_err[4::5]],
                     "s": round(dt, 3)}
    g.release_workspace()
    return out


def bench_concurrent_pair(abg, torch, dev, gg, w, b32, enorm, basis, steps, warmup=50):
    """The timed step's two solves (AB and BA, same input and rule) run at the same time
    from two host threads, each on its own stream with its own workspace: Arnoldi
    iterations per second of the pair. The solves are the same as in the sequential
    step; only their overlap on the device differs."""
    import threading
    jobs = []
    for m in ("ab", "ba"):
        nb = abg.workspace_bytes(gg, m, w.k_max, proj="f32", basis=basis, stop="dp")
        jobs.append((m, torch.empty(nb, dtype=torch.uint8, device=dev),
                     torch.empty(gg.n, dtype=torch.float32, device=dev), torch.cuda.Stream()))
    n_steps = warmup + steps
    start = threading.Barrier(3)
    done = threading.Barrier(3)
    iters = [0, 0]
    errors = []

    def worker(j):
        m, ws, x, st = jobs[j]
        try:
            with torch.cuda.stream(st):
                for step in range(n_steps):
                    start.wait()
                    r = abg.gmres(m, gg, b32, w.k_max, stop="dp", tau=w.tau, noise_norm=enorm,
                                  basis=basis, workspace=ws, out=x, stream=st)
                    if step >= warmup:
                        iters[j] += r.k_done
                    done.wait()
        except Exception as e:   # reported below
            errors.append(repr(e))
            start.abort()
            done.abort()

    torch.cuda.synchronize()
    ths = [threading.Thread(target=worker, args=(j,)) for j in range(2)]
    for t in ths:
        t.start()
    t0 = None
    try:
        for step in range(n_steps):
            if step == warmup:
                t0 = time.perf_counter()
            start.wait()
            done.wait()
        t1 = time.perf_counter()
    except threading.BrokenBarrierError:
        pass
    for t in ths:
        t.join()
    if errors or t0 is None:
        return {"error": errors}
    return {"iters_per_s": round(sum(iters) / (t1 - t0), 1),
            "ms_per_step": round(1e3 * (t1 - t0) / steps, 3), "steps": steps}


def bench_lsq(abg, torch, dev, w, xb, b32, enorm, reps=5):
    """The matched comparators (Sec. 5, 6.2) on the timed workload's input: LSQR and LSMR
    with A and its exact transpose, FP32, under the same DP rule: stopping iteration,
    solve time (median of reps), iterations per second and ||x - x_true|| / ||x_true||.
    Each step is one forward and one transposed projection with short recurrences."""
    g = abg.Geometry(w.N, w.n_ang, w.n_det, ang_range=w.ang_range)
    xt = torch.tensor(xb, dtype=torch.float64, device=dev)
    out = {}
    for meth in ("lsqr", "lsmr"):
        nb = abg.lsq_workspace_bytes(g, meth, "f32")
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        x = torch.empty(g.n, dtype=torch.float32, device=dev)
        times = []
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = abg.lsq(meth, g, b32, w.k_max, stop="dp", tau=w.tau, noise_norm=enorm,
                        workspace=ws, out=x)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        dt = float(np.median(times[1:]))
        err = float(torch.linalg.vector_norm(r.x.double() - xt) / torch.linalg.vector_norm(xt))
        out[meth] = {"k_stop": r.k_stop, "ms": round(1e3 * dt, 3),
                     "iters_per_s": round(r.k_done / dt, 1), "n_literal": r.n_literal,
                     "rel_error": round(err, 4)}
    return out


def bench_few_view(abg, torch, dev):
    """Under-determined few-view scan (512^2, 180 angles: m = 0.5 n), AB- and BA-GMRES
    with the DP rule in FP32: stopping iteration, time, Krylov-basis bytes (k+1 vectors of
    length m for AB, n for BA) and relative reconstruction error."""
    w = W.CONFIG_FEW_VIEW
    g = abg.Geometry(w.N, w.n_ang, w.n_det, ang_range=w.ang_range)
    xt = torch.tensor(w.phantom(), dtype=torch.float64, device=dev)
    bc = g.fp(xt)
    gen = torch.Generator(device=dev)
    gen.manual_seed(9)
    e = torch.randn(bc.numel(), generator=gen, device=dev, dtype=bc.dtype)
    e *= w.eta * torch.linalg.vector_norm(bc) / torch.linalg.vector_norm(e)
    b = (bc + e).float()
    enorm = float(torch.linalg.vector_norm(e))
    out = {"workload": f"{w.N}x{w.N}, {w.n_ang} angles, {w.n_det} bins (m = {w.m}, n = {w.n}), "
                       f"{100 * w.eta:g}% noise, DP tau={w.tau}"}
    for meth in ("ab", "ba"):
        abg.gmres(meth, g, b, w.k_max, stop="dp", tau=w.tau, noise_norm=enorm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = abg.gmres(meth, g, b, w.k_max, stop="dp", tau=w.tau, noise_norm=enorm)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        L = w.m if meth == "ab" else w.n
        err = float(torch.linalg.vector_norm(r.x.double() - xt) / torch.linalg.vector_norm(xt))
        out[meth] = {"k_stop": r.k_stop, "ms": round(1e3 * dt, 3),
                     "iters_per_s": round(r.k_done / dt, 1),
                     "basis_bytes": (r.k_done + 1) * L * 4, "rel_error": round(err, 4)}
    g.release_workspace()
    return out


def bench_batched(abg, torch, dev, reps=3):
    """The 64-problem batched workload (N in {128..1024}, 60..720 angles, half limited
    angle, AB/BA alternating, per-problem DP): engine throughput after autotuning, next to
    the same 64 solves run one by one (FP32 and plain FP64)."""
    ws = W.batched_workloads()
    probs = []
    for w in ws:
        gg = abg.Geometry(w.N, w.n_ang, w.n_det, ang_range=w.ang_range)
        xt = torch.tensor(w.phantom().ravel(), dtype=torch.float32, device=dev)
        probs.append(_dp_problem(abg, torch, gg, w, xt, dev, 4_000_000 + w.instance))
    eng = abg.Engine(proj="f32", basis="f32", max_slots=len(probs))
    xs = [torch.empty(p.g.n, dtype=torch.float32, device=dev) for p in probs]
    wss = [torch.empty(abg.request_bytes(p.g, p.method, p.k_max, "f32", "f32", "dp"),
                       dtype=torch.uint8, device=dev) for p in probs]

    def run(tune=False):
        tags = [eng.submit(p, x=x, workspace=w_) for p, x, w_ in zip(probs, xs, wss)]
        tuned = eng.autotune(reps=3) if tune else None
        done = {}
        while len(done) < len(tags):
            eng.step()
            done.update(dict(eng.poll()))
        return [done[t] for t in tags], tuned

    run()                                   # warm-up (graph capture, allocations)
    _, tuned = run(tune=True)
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, _ = run()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    tb = float(np.median(times))
    t32, s32 = _single_solves(abg, torch, probs, torch.float32)
    t64, s64 = _single_solves(abg, torch, probs, torch.float64)
    _concurrent_solves(abg, torch, probs)            # warm-up
    conc = [_concurrent_solves(abg, torch, probs) for _ in range(reps)]
    tc = float(np.median([c[0] for c in conc]))
    conc_err = [e for c in conc for e in c[1]]
    same_k = sum(int(a.k_stop == b.k_stop) for a, b in zip(res, s64))
    err = max(float(torch.linalg.vector_norm(a.x.double() - b.x) / torch.linalg.vector_norm(b.x))
              for a, b in zip(res, s64))
    eng.close()
    return {"workload": "64 problems: N in {128,256,512,1024}, angles in {60,180,360,720}, "
                        "32 full-range [0,180) + 32 limited [0,120), eta U[0.005,0.03], AB/BA "
                        "alternating, DP tau=1.02, k_max=100; FP32 projectors and basis",
            "reconstructions_per_s": round(len(probs) / tb, 1), "ms_per_batch": round(1e3 * tb, 2),
            "arnoldi_iterations": int(sum(r.k_done for r in res)),
            "tiles": {"rays": tuned["rays"], "ang_block": tuned["ang_block"],
                      "sched": tuned["sched"]},
            "single_fp32_recon_per_s": round(len(probs) / t32, 1),
            "single_fp64_recon_per_s": round(len(probs) / t64, 1),
            "single_fp32_3_streams_recon_per_s": (round(len(probs) / tc, 1) if not conc_err
                                                  else {"error": conc_err[:2]}),
            "speedup_vs_single_fp64": round(t64 / tb, 2),
            "same_k_stop_as_fp64": f"{same_k}/{len(probs)}",
            "max_rel_diff_vs_fp64": float(f"{err:.3g}")}


def bench_serving(abg, torch, dev, seconds, bases, single_sample=160):
    """Poisson request stream (50/s; N in {256..2048}, 180-1800 angles, AB/BA, k_max in
    [30,120], DP) through the continuous-batching server under a 200 GB workspace budget,
    in real time and as a closed batch, per basis dtype; for comparison, the first
    `single_sample` requests as a closed batch and solved one by one (plain FP64 and FP32
    single solves)."""
    from paper_2110_01481_amd.serving import Request, Server
    stream = W.serving_requests(rate=50.0, duration=seconds)
    pool = {N: [torch.tensor(W.ellipse_phantom(N, 10, W.rng(5, 100000 + 10 * N + j, 0)).ravel(),
                             dtype=torch.float32, device=dev) for j in range(2)]
            for N in sorted({w.N for _, w in stream})}
    reqs = []
    for i, (t, w) in enumerate(stream):
        gg = abg.Geometry(w.N, w.n_ang, w.n_det, ang_range=w.ang_range)
        reqs.append(Request(t, _dp_problem(abg, torch, gg, w, pool[w.N][i % 2], dev, 5_000_000 + i)))
    out = {"workload": f"Poisson arrivals 50/s for {seconds:g} s ({len(reqs)} requests): N in "
                       "{256,512,1024,2048}, angles U{180..1800}, eta U[0.01,0.03], AB/BA 50/50, "
                       "k_max U{30..120}, DP tau=1.02; admission by request workspace bytes "
                       "against a 200 GB budget",
           "runs": {}}
    for basis in bases:
        srv = Server(proj="f32", basis=basis, max_slots=256, budget_bytes=200e9)
        tuned = srv.tune([r.problem for r in reqs[:32]])
        progress(f"serving {basis}: tuned, {len(reqs)} requests in real time")
        live = srv.run(reqs, realtime=True)
        progress(f"serving {basis}: real-time run done, closed batch")
        closed = srv.run(reqs, realtime=False)
        progress(f"serving {basis}: closed batch done")
        srv.close()
        out["runs"][basis] = {"realtime": live.as_dict(),
                              "closed_batch_reconstructions_per_s": round(closed.completed_per_s, 2),
                              "tuned_on_first_32": {k: tuned[k] for k in ("rays", "ang_block", "sched")}}
    sample = [r.problem for r in reqs[:single_sample]]
    srv = Server(proj="f32", basis="f32", max_slots=256, budget_bytes=200e9)
    srv.tune(sample[:32])
    srv.run(reqs[:single_sample], realtime=False)   # warm-up
    eng = srv.run(reqs[:single_sample], realtime=False)
    srv.close()
    _single_solves(abg, torch, sample[:8], torch.float32)   # warm-up
    t64, _ = _single_solves(abg, torch, sample, torch.float64)
    t32, _ = _single_solves(abg, torch, sample, torch.float32)
    out["sample"] = {"requests": f"the first {len(sample)} requests",
                     "engine_fp32_closed_batch_recon_per_s": round(eng.completed_per_s, 2),
                     "single_fp32_recon_per_s": round(len(sample) / t32, 2),
                     "single_fp64_recon_per_s": round(len(sample) / t64, 2)}
    return out


GOLDEN = os.path.join(ROOT, "tests", "golden")


def oracle_iterate(cfg: int):
    """The oracle's returned iterate of the workload, stored whole by
    tests/golden/make_oracle_golden.py (config 3: x_{k_NCP}, rounded to FP32), and its
    stopping iteration; None when absent."""
    try:
        with open(os.path.join(GOLDEN, f"oracle_config{cfg}.json")) as fh:
            meta = json.load(fh)
        if cfg == 3:
            return np.load(os.path.join(GOLDEN, "oracle_config3_x.npy")).astype(np.float64), meta
        z = np.load(os.path.join(GOLDEN, "oracle_config2_x.npz"))
        return {k: z[k] for k in z.files}, meta
    except (OSError, ValueError, KeyError):
        return None, None


class SingleRun:
    """Repeated single solves of one workload through the C ABI: untimed warm-up steps,
    a timed region without instrumentation, then (optionally) the same steps with every
    projector, Gram-Schmidt, basis-combination and NCP launch stamped with HIP events on
    the solver's stream (abg_profile_enable): the kernels' durations."""

    def __init__(self, abg, torch, gg, w, methods, b, basis, stop, tau, enorm):
        self.abg, self.torch, self.gg, self.w = abg, torch, gg, w
        self.methods, self.b, self.basis = methods, b, basis
        self.stop, self.tau, self.enorm = stop, tau, enorm
        proj = "f64" if b.dtype == torch.float64 else "f32"
        self.bufs = {}
        for m in methods:
            nb = abg.workspace_bytes(gg, m, w.k_max, proj=proj, basis=basis, stop=stop)
            self.bufs[m] = (torch.empty(nb, dtype=torch.uint8, device=b.device),
                            torch.empty(gg.n, dtype=b.dtype, device=b.device))

    def step(self):
        iters, res = 0, {}
        for m in self.methods:
            ws, out = self.bufs[m]
            r = self.abg.gmres(m, self.gg, self.b, self.w.k_max, stop=self.stop, tau=self.tau,
                               noise_norm=self.enorm, basis=self.basis, workspace=ws, out=out)
            iters += r.k_done
            res[m] = r
        return iters, res

    def run(self, steps, warmup, instrument=True):
        torch, abg = self.torch, self.abg
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters, last = 0, None
        for _ in range(steps):
            n, last = self.step()
            iters += n
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out = {"iters_per_s": iters / dt, "ms_per_step": 1e3 * dt / steps, "iters": iters,
               "last": last, "prof": None}
        if instrument:
            abg.profile_enable(True)
            abg.profile_read(reset=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n_i = 0
            for _ in range(steps):
                n_i += self.step()[0]
            torch.cuda.synchronize()
            out["instrumented"] = {"ms_per_step": round(1e3 * (time.perf_counter() - t0) / steps, 3),
                                   "iters": n_i}
            out["prof"] = abg.profile_read(reset=True)
            abg.profile_enable(False)
        return out


def _rel(a, b) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _work_per_launch(w, proj: str):
    """Algorithmic work of one launch of each compute-bound kernel on workload w: 2 flop per
    nonzero of A (forward), 4 flop per pixel-angle pair (back: two taps), 3 flop per
    Goertzel step (NCP: N_det steps for each of floor(N_det/2) frequencies of every row)."""
    th = (np.arange(w.n_ang) * w.ang_range) / w.n_ang
    nnz = line_model_nnz(w.N, th, w.n_det)
    q = w.n_det // 2
    return {"forward": (2.0 * nnz, f"{nnz} ray-pixel intersections x 2 flop"),
            "back": (4.0 * w.n * w.n_ang, f"{w.n * w.n_ang} pixel-angle pairs x 4 flop"),
            "ncp": (3.0 * w.n_ang * q * w.n_det,
                    f"{w.n_ang} rows x {q} frequencies x {w.n_det} Goertzel steps x 3 flop")}, nnz


def roofline_of(prof, w, proj: str, tag: str):
    """Roofline object of the kernel class with the largest share of the instrumented pass."""
    share = {k: v[1] for k, v in prof.items() if v[0] > 0}
    dominant = max(share, key=share.get)
    n, ms = prof[dominant]
    avg_ms = ms / n
    peak = FP64_VECTOR_PEAK_TFLOPS if proj == "f64" else FP32_VECTOR_PEAK_TFLOPS
    work, _ = _work_per_launch(w, proj)
    names = {"forward": f"forward_kernel<{'double' if proj == 'f64' else 'float'}> (ray-driven "
                        f"line model A, {proj.upper()})",
             "back": f"back_kernel (pixel-driven unmatched B, {proj.upper()})",
             "ncp": "ncp_fft_rows/colsum/dist/final kernels (periodogram of every sinogram row, FP64)",
             "mgs": "mgs kernels (Gram-Schmidt + Givens)", "combine": "combine_kernel"}
    roof = {"kernel": names[dominant], "avg_launch_ms": round(avg_ms, 4),
            "share_of_kernel_time": round(ms / sum(share.values()), 4)}
    if dominant in work:
        flops, desc = work[dominant]
        pk = FP64_VECTOR_PEAK_TFLOPS if dominant == "ncp" else peak
        ach = flops / (avg_ms * 1e-3) / 1e12
        roof.update({"bound": "alu", "achieved": round(ach, 3), "peak": pk, "unit": "TFLOP/s",
                     "frac": round(ach / pk, 4), "traffic": None, "work_per_launch": desc})
        key = f"{dominant}_kernel_{proj}"
        tr = stored_counters(key, tag) if key in COUNTER_KERNELS else None
        if tr:
            roof["traffic"] = tr["traffic_bytes_per_launch"]
            roof["traffic_note"] = (f"HBM bytes per launch from FETCH_SIZE x {tr['fetch_scale']} + "
                                    f"WRITE_SIZE x {tr['write_scale']} (copy-calibrated, "
                                    f"profiles/{key}_{tag}_counters.md); "
                                    f"{tr['traffic_bytes_per_launch'] / (avg_ms * 1e-3) / 1e9:.0f} GB/s")
            if "valu_wave_insts_per_dispatch" in tr:
                lane_ops = 64.0 * tr["valu_wave_insts_per_dispatch"]
                roof["valu_issue_frac"] = round(lane_ops / (avg_ms * 1e-3) / VALU_ISSUE_PEAK, 4)
            if tr.get("l2_hit_rate"):
                roof["l2_hit_rate"] = tr["l2_hit_rate"].get(dominant + "_kernel")
            if dominant == "forward" and "vmem_read_wave_insts_per_dispatch" in tr:
                # the forward walk issues one 64-lane gather per band and wave: its issue
                # rate per CU, in cycles of the 2.4 GHz peak clock (a texture path taking
                # four lane addresses per cycle needs 16)
                g = tr["vmem_read_wave_insts_per_dispatch"]
                roof["gathers"] = {
                    "wave_gathers_per_launch": int(g),
                    "cycles_per_gather_per_cu_at_2_4_ghz": round(avg_ms * 1e-3 * 2.4e9 / (g / 256), 1),
                    "note": "one 64-lane gather per band and wave; 16 cycles each at four lane "
                            "addresses per cycle"}
    else:
        roof.update({"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": None, "traffic": None})
    return roof


def krylov_bytes(methods, w, last, sv: int, sx: int):
    """Algorithmic HBM bytes of the Gram-Schmidt and basis-combination launches of one
    step. Step j (0..k_done) of a solve reads q and w_1..w_j and writes w_{j+1} and its
    copy; the residual form of step j reads j (BA: Z, plus b - A x_0) or j+1 (AB: W)
    vectors of m and writes one; forming the iterate reads k_done basis vectors."""
    mgs = comb = red = 0
    for m in methods:
        L = w.m if m == "ab" else w.n
        kd = last[m].k_done
        for j in range(kd + 1):
            mgs += j * L * sv + L * sv + 2 * L * sx
            red += j + 1
        for j in range(1, kd + 1):
            comb += ((j + 1) * w.m * sx + w.m * sx) if m == "ba" else ((j + 1) * w.m * sv + w.m * sx)
        comb += kd * L * sv + L * sx
    return mgs, comb, red


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 30 at 2048^2, 50 otherwise)")
    # after idle the device needs ~0.7 s under load before a timed region runs at its
    # steady rate (with too short a warm-up the first region ran up to 15% slower)
    ap.add_argument("--warmup", type=int, default=None,
                    help="warm-up steps (default 8 at 2048^2, 200 otherwise)")
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3],
                    help="3: 2048^2 BA-GMRES NCP (default); 2: 512^2 AB+BA DP; 1: 64^2")
    ap.add_argument("--proj", default=None, choices=["f64", "f32"],
                    help="projector dtype of the timed solves (default f64 at 2048^2, else f32)")
    ap.add_argument("--basis", default=None, choices=["f64", "f32", "bf16"],
                    help="basis storage dtype (default: the projector dtype)")
    ap.add_argument("--quick", action="store_true",
                    help="only the timed workload (no variants, 512^2 extras, batched mix, "
                         "serving or CPU baseline): for profiler runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-arnoldi-steps", type=int, default=0,
                    help="also time this many iterations of the oracle's BA-GMRES at 2048^2")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="seconds of Poisson arrivals for the serving run (0: skip)")
    ap.add_argument("--serve-basis", default="f32,bf16")
    ap.add_argument("--no-concurrent", action="store_true",
                    help="skip the 512^2 AB || BA run on two streams")
    ap.add_argument("--no-models", action="store_true",
                    help="skip the strip / Joseph models, the six unmatched pairs, few-view, "
                         "error histories and LSQR/LSMR")
    ap.add_argument("--summarize-counters", default="",
                    help="print the counter summary of the rocprofv3 passes under this directory")
    ap.add_argument("--counter-kernel", default="forward_kernel_f32", choices=sorted(COUNTER_KERNELS))
    ap.add_argument("--counter-workload", default="512x512, 720 x 725, FP32")
    ap.add_argument("--counter-bench-args", default="")
    ap.add_argument("--summarize-kernel-stats", default="",
                    help="print the kernel-time summary of a rocprofv3 --kernel-trace --stats "
                         "csv run under this directory (with --stats-title, --stats-command)")
    ap.add_argument("--stats-title", default="")
    ap.add_argument("--stats-command", default="")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run device-to-device copies of this many MiB (a plain copy "
                         "kernel whose HBM counters calibrate FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.summarize_counters:
        print(summarize_counters(args.summarize_counters, args.counter_kernel,
                                 args.counter_workload, args.counter_bench_args))
        return
    if args.summarize_kernel_stats:
        print(summarize_kernel_stats(args.summarize_kernel_stats, args.stats_title,
                                     args.stats_command))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the solver library runs on one GPU; --gpus N > 1 is not "
                                   "supported (how the path would shard is described, not "
                                   "implemented)"}))
        sys.exit(2)

    import torch
    import paper_2110_01481_amd as abg

    torch.cuda.set_device(0)
    if args.copy_calibration_mib > 0:
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nb, "copies": 3}))
        return
    abg.load_library()
    try:
        out = run_bench(args, abg, torch)
    finally:
        # release the library's process-wide resources before the interpreter and the
        # HIP runtime shut down
        abg.shutdown()
    print(json.dumps(out), flush=True)


def run_bench(args, abg, torch):
    big = args.config == 3
    steps = args.steps if args.steps is not None else (30 if big else 50)
    warmup = args.warmup if args.warmup is not None else (8 if big else 200)
    proj = args.proj or ("f64" if big else "f32")
    basis = args.basis or proj
    w = {1: W.CONFIG1, 2: W.CONFIG2, 3: W.CONFIG3}[args.config]
    tag = f"{w.N}x{w.N}_{w.n_ang}x{w.n_det}"
    dev = torch.device("cuda:0")
    gg = abg.Geometry(w.N, w.n_ang, w.n_det, ang_range=w.ang_range)
    xb = w.phantom()
    # b = A x_bar + e: A x_bar by the library's FP64 forward projector (the oracle's FP64
    # A gives the same vector to rounding), e the seeded noise direction scaled to eta
    bbar = gg.fp(torch.tensor(xb, dtype=torch.float64, device=dev)).cpu().numpy()
    gg.release_workspace()
    b_np, enorm = W.add_noise(bbar, w.eta, w.noise_dir())
    bt = {"f64": torch.tensor(b_np, dtype=torch.float64, device=dev),
          "f32": torch.tensor(b_np, dtype=torch.float32, device=dev)}
    stop = w.stop if w.stop != "none" else "dp"
    tau = w.tau if stop == "dp" else 1.0
    methods = ["ba"] if big else ["ab", "ba"]
    progress(f"timed workload {tag}, {'+'.join(methods)}, {stop}, proj {proj}, basis {basis}")
    main_run = SingleRun(abg, torch, gg, w, methods, bt[proj], basis, stop, tau, enorm)
    r = main_run.run(steps, warmup)
    value, last, prof = r["iters_per_s"], r["last"], r["prof"]
    progress(f"timed region: {value:.2f} iters/s ({r['ms_per_step']:.2f} ms per step)")
    roof = roofline_of(prof, w, proj, tag)
    work, nnz = _work_per_launch(w, proj)
    fwd_n, fwd_ms = prof["forward"]
    bck_n, bck_ms = prof["back"]
    fwd_avg, bck_avg = fwd_ms / max(fwd_n, 1), bck_ms / max(bck_n, 1)
    sx = 8 if proj == "f64" else 4
    sv = {"f64": 8, "f32": 4, "bf16": 2}[basis]
    spmv_bytes = nnz * (sx + 4) + (w.n + w.m) * sx
    extra = {
        "A_applies_per_s": round(1e3 / fwd_avg, 2) if fwd_n else None,
        "B_applies_per_s": round(1e3 / bck_avg, 2) if bck_n else None,
        "A_spmv_equiv_GBps": round(spmv_bytes / (fwd_avg * 1e-3) / 1e9, 1) if fwd_n else None,
        "B_spmv_equiv_GBps": round(spmv_bytes / (bck_avg * 1e-3) / 1e9, 1) if bck_n else None,
        "spmv_equiv_note": "bytes an explicit CSR product would stream: nnz x (value + 4-byte "
                           "index) + the two vectors",
        "nnz_A": nnz,
        "kernel_ms": {k: [v[0], round(v[1], 3)] for k, v in prof.items()},
        "instrumented_pass": r["instrumented"],
        "k_stop": {m: last[m].k_stop for m in methods},
        "k_done": {m: last[m].k_done for m in methods},
    }
    if fwd_n:
        extra["A_tflops"] = round(work["forward"][0] / (fwd_avg * 1e-3) / 1e12, 3)
    if bck_n:
        extra["B_tflops"] = round(work["back"][0] / (bck_avg * 1e-3) / 1e12, 3)
    if prof["ncp"][0]:
        extra["ncp_avg_ms"] = round(prof["ncp"][1] / prof["ncp"][0], 4)
    mgs_b, comb_b, red = krylov_bytes(methods, w, last, sv, sx)
    extra["mgs"] = _stream_kernel_stats(prof["mgs"][1], prof["mgs"][0], mgs_b * steps, red * steps)
    extra["combine"] = _stream_kernel_stats(prof["combine"][1], prof["combine"][0], comb_b * steps)

    if big:
        x_orc, meta = oracle_iterate(3)
        if meta is not None:
            sol = meta["solves"]["ba-hat"]
            extra["oracle"] = {"k_stop": sol["k_stop"], "ncp": sol["ncp"],
                               "stored": "tests/golden/oracle_config3_x.npy (x_kNCP, FP32-rounded)"}
        if x_orc is not None:
            extra["rel_error_vs_oracle"] = round(_rel(last["ba"].x.double().cpu().numpy(), x_orc), 9)
        extra["ncp_hist"] = [round(float(v), 6) for v in last["ba"].ncp_hist]
        extra["rel_error_vs_phantom"] = round(_rel(last["ba"].x.double().cpu().numpy(), xb), 5)
        if not args.quick:
            variants = {}
            for p_, b_ in (("f32", "f32"), ("f32", "bf16")):
                if (p_, b_) == (proj, basis):
                    continue
                progress(f"variant proj {p_} basis {b_}")
                vr = SingleRun(abg, torch, gg, w, methods, bt[p_], b_, stop, tau, enorm).run(
                    max(steps // 3, 3), 2, instrument=False)
                xv = vr["last"]["ba"].x.double().cpu().numpy()
                d = {"iters_per_s": round(vr["iters_per_s"], 2),
                     "ms_per_solve": round(vr["ms_per_step"], 2),
                     "k_stop": vr["last"]["ba"].k_stop, "k_done": vr["last"]["ba"].k_done,
                     "rel_error_vs_fp64_gpu": round(_rel(xv, last["ba"].x.double().cpu().numpy()), 7)}
                if x_orc is not None:
                    d["rel_error_vs_oracle"] = round(_rel(xv, x_orc), 7)
                variants[f"proj_{p_}_basis_{b_}"] = d
                torch.cuda.empty_cache()
            extra["variants"] = variants
    gg.release_workspace()

    if not args.quick and args.config != 1:
        extra["workload_512"] = bench_512(args, abg, torch, dev)

    if not args.quick and not args.no_batch:
        progress("batched mix")
        extra["batched"] = bench_batched(abg, torch, dev)
        progress("batched mix done")
    if not args.quick and args.serve_seconds > 0:
        extra["serving"] = bench_serving(abg, torch, dev, args.serve_seconds,
                                         [b for b in args.serve_basis.split(",") if b])

    cpu = None
    if not args.quick and not args.no_cpu_baseline:
        progress("CPU oracle baseline")
        if big:
            cpu = cpu_oracle_baseline_ncp(w, b_np, xb, args.cpu_arnoldi_steps)
        else:
            cpu = cpu_oracle_baseline(w, b_np, enorm)
        progress("CPU oracle baseline done")

    stop_desc = {"dp": f"DP stop (tau={tau})", "ncp": "NCP stop"}[stop]
    return {
        "metric": "GMRES iters/s", "value": round(value, 3), "unit": "iters/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": round(r["ms_per_step"], 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": proj if basis == proj else f"{proj}+{basis} basis",
        "data": "synthetic",
        "config": {"workload": f"{w.N}x{w.N} image, {w.n_ang} angles in [0,{w.ang_range:g}), "
                               f"{w.n_det} bins, {w.n_ellipses}-ellipse phantom, "
                               f"{100 * w.eta:g}% noise; " + "+".join(m.upper() for m in methods) +
                               f"-GMRES, {stop_desc}, k_max={w.k_max}, {proj.upper()} projectors, "
                               f"{basis.upper()} basis, FP64 Hessenberg/Givens, unmatched pair "
                               "(line-model A, interpolating B)",
                   "global_batch": len(methods), "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }


def bench_512(args, abg, torch, dev):
    """The 512^2 single-solve workload (AB- and BA-GMRES, DP tau = 1.02, k_max = 100):
    FP32 projectors and basis timed as in the main region, the plain FP64 solves, the two
    solves on two streams, and the strip / Joseph models, few-view, error histories and
    LSQR / LSMR on the same geometry."""
    w = W.CONFIG2
    gg = abg.Geometry(w.N, w.n_ang, w.n_det, ang_range=w.ang_range)
    xb = w.phantom()
    bbar = gg.fp(torch.tensor(xb, dtype=torch.float64, device=dev)).cpu().numpy()
    gg.release_workspace()
    b_np, enorm = W.add_noise(bbar, w.eta, w.noise_dir())
    b32 = torch.tensor(b_np, dtype=torch.float32, device=dev)
    b64 = torch.tensor(b_np, dtype=torch.float64, device=dev)
    progress("512^2 workload")
    r32 = SingleRun(abg, torch, gg, w, ["ab", "ba"], b32, "f32", "dp", w.tau, enorm).run(50, 200)
    r64 = SingleRun(abg, torch, gg, w, ["ab", "ba"], b64, "f64", "dp", w.tau, enorm).run(10, 5,
                                                                                      instrument=False)
    prof = r32["prof"]
    out = {"workload": "512x512, 720 angles, 725 bins, 20 ellipses, 2% noise; AB+BA-GMRES, DP "
                       "tau=1.02, k_max=100, unmatched pair",
           "fp32_iters_per_s": round(r32["iters_per_s"], 2),
           "fp32_ms_per_step": round(r32["ms_per_step"], 3),
           "fp64_iters_per_s": round(r64["iters_per_s"], 2),
           "k_stop_fp32": {m: r32["last"][m].k_stop for m in ("ab", "ba")},
           "k_stop_fp64": {m: r64["last"][m].k_stop for m in ("ab", "ba")},
           "kernel_ms_fp32": {k: [v[0], round(v[1], 3)] for k, v in prof.items()},
           "roofline_fp32": roofline_of(prof, w, "f32", f"{w.N}x{w.N}_{w.n_ang}x{w.n_det}"),
           "f32_vs_f64_iterate_rel": {
               m: _rel(r32["last"][m].x.double().cpu().numpy(), r64["last"][m].x.cpu().numpy())
               for m in ("ab", "ba")}}
    x_orc, _ = oracle_iterate(2)
    if x_orc is not None:
        out["rel_error_vs_oracle"] = {
            f"{m}_{dt}": round(_rel(rr["last"][m].x.double().cpu().numpy(), x_orc[f"{m}_hat"]), 9)
            for m in ("ab", "ba") for dt, rr in (("fp32", r32), ("fp64", r64))}
    if not args.no_concurrent:
        out["concurrent_ab_ba"] = bench_concurrent_pair(abg, torch, dev, gg, w, b32, enorm, "f32", 50)
    if not args.no_models:
        out["models"] = bench_models(abg, torch, dev, w, xb)
        progress("models done")
        out["few_view"] = bench_few_view(abg, torch, dev)
        out["histories"] = bench_histories(abg, torch, dev, w, xb)
        progress("few-view and histories done")
        out["lsq"] = bench_lsq(abg, torch, dev, w, xb, b32, enorm)
    gg.release_workspace()
    return out


if __name__ == "__main__":
    main()
