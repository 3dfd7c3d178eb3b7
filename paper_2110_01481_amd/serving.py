"""Request loop over the batched engine: reconstructions of mixed sizes arrive over time,
are admitted by the device memory their solve needs, and share the engine's rounds with
the solves already running (continuous batching).

Admission is first-come first-served: the oldest waiting request is admitted as soon as
an engine slot is free and its workspace (Krylov basis, Hessenberg state and scratch:
abg_request_bytes) fits in what is left of the memory budget; its workspace is released
when its result is returned. Every solve keeps its basis and Hessenberg state on the
device for its whole life. Latency is measured from arrival to the host seeing the
finished result.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from ._binding import Engine, Problem, SolveResult, request_bytes


@dataclass
class Request:
    arrival: float          # seconds after the start of the run
    problem: Problem        # inputs already on the device
    keep_result: bool = False


@dataclass
class ServeReport:
    n: int
    duration_s: float                       # first arrival to last completion
    offered_per_s: float                    # arrivals per second of the arrival window
    completed_per_s: float                  # reconstructions per second (whole run)
    latency_p50_s: float
    latency_p99_s: float
    latency_max_s: float
    wait_p50_s: float                       # arrival to admission
    peak_bytes: int
    peak_active: int
    rounds: int
    iterations: int
    statuses: dict
    latencies: np.ndarray = field(repr=False, default=None)
    results: dict = field(repr=False, default_factory=dict)
    tiles: tuple = (0, 0, 0)

    def as_dict(self) -> dict:
        return {"requests": self.n, "duration_s": round(self.duration_s, 3),
                "offered_req_per_s": round(self.offered_per_s, 2),
                "reconstructions_per_s": round(self.completed_per_s, 2),
                "latency_p50_s": round(self.latency_p50_s, 4),
                "latency_p99_s": round(self.latency_p99_s, 4),
                "latency_max_s": round(self.latency_max_s, 4),
                "admission_wait_p50_s": round(self.wait_p50_s, 4),
                "peak_workspace_GB": round(self.peak_bytes / 1e9, 2),
                "peak_active": self.peak_active, "rounds": self.rounds,
                "arnoldi_iterations": self.iterations, "statuses": self.statuses,
                "tiles": list(self.tiles)}


class Server:
    """Continuous-batching request loop on one device."""

    def __init__(self, proj: str = "f32", basis: str = "f32", max_slots: int = 256,
                 budget_bytes: float = 200e9, tiles: tuple | None = None, engine=None):
        self.proj, self.basis = proj, basis
        self.budget = int(budget_bytes)
        self.engine = engine if engine is not None else Engine(proj=proj, basis=basis,
                                                               max_slots=max_slots)
        if tiles:
            self.engine.set_tiles(*tiles)

    @staticmethod
    def _sync(device):
        import torch
        if getattr(device, "type", "cpu") == "cuda":
            torch.cuda.synchronize(device)

    @staticmethod
    def _alloc(p: Problem, nbytes: int):
        import torch
        ws = torch.empty(nbytes, dtype=torch.uint8, device=p.b.device)
        x = torch.empty(p.g.n, dtype=p.b.dtype, device=p.b.device)
        return ws, x

    def close(self):
        self.engine.close()

    def tune(self, problems: list, reps: int = 2, cache: str | None = None) -> dict:
        """Picks the engine's tile shapes and schedule on a closed batch of representative
        problems (the autotuner times them without advancing them), then solves them to
        completion. Call before run()."""
        eng = self.engine
        held = []
        for p in problems:
            ws, x = self._alloc(p, self.request_bytes(p))
            if eng.submit(p, x=x, workspace=ws) is None:
                break
            held.append((ws, x))
        out = eng.autotune(reps=reps, cache=cache)
        left = len(held)
        while left > 0:
            eng.step()
            left -= len(eng.poll())
        return out

    def request_bytes(self, p: Problem) -> int:
        return request_bytes(p.g, p.method, p.k_max, self.proj, self.basis, p.stop)

    def run(self, requests: list[Request], realtime: bool = True) -> ServeReport:
        """Serves the requests (sorted by arrival). With realtime=False every request is
        taken as arrived at time 0 (a closed batch through the same admission)."""
        eng = self.engine
        n = len(requests)
        need = [self.request_bytes(r.problem) for r in requests]
        if any(b > self.budget for b in need):
            raise ValueError("a request needs more device memory than the whole budget")
        arrivals = np.array([r.arrival if realtime else 0.0 for r in requests])
        admit_t = np.full(n, np.nan)
        done_t = np.full(n, np.nan)
        queue: deque[int] = deque()
        held: dict[int, tuple] = {}      # engine tag -> (request index, workspace, x)
        used = peak = peak_active = 0
        nxt = 0
        finished = 0
        rounds = iters = 0
        statuses: dict[str, int] = {}
        results = {}
        device = requests[0].problem.b.device if n else None
        self._sync(device)
        t0 = time.perf_counter()
        while finished < n:
            now = time.perf_counter() - t0
            while nxt < n and arrivals[nxt] <= now:
                queue.append(nxt)
                nxt += 1
            # admission: oldest first, while a slot is free and the workspace fits
            while queue and used + need[queue[0]] <= self.budget:
                i = queue[0]
                p = requests[i].problem
                ws, x = self._alloc(p, need[i])
                tag = eng.submit(p, x=x, workspace=ws)
                if tag is None:
                    break                       # every slot busy
                queue.popleft()
                held[tag] = (i, ws, x)
                used += need[i]
                peak = max(peak, used)
                peak_active = max(peak_active, len(held))
                admit_t[i] = time.perf_counter() - t0
            if held:
                eng.step()
                rounds += 1
                for tag, res in eng.poll():
                    i, ws, x = held.pop(tag)
                    done_t[i] = time.perf_counter() - t0
                    used -= need[i]
                    finished += 1
                    iters += res.k_done
                    statuses[res.status] = statuses.get(res.status, 0) + 1
                    if requests[i].keep_result:
                        results[i] = res
                    del ws
            elif nxt < n:
                # idle until the next arrival
                wait = arrivals[nxt] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.01))
        self._sync(device)
        lat = done_t - arrivals
        wait = admit_t - arrivals
        span = float(done_t.max() - arrivals.min()) if n else 0.0
        window = float(arrivals.max() - arrivals.min()) if n > 1 else 0.0
        return ServeReport(
            n=n, duration_s=span, offered_per_s=(n - 1) / window if window > 0 else float("inf"),
            completed_per_s=n / span if span > 0 else float("inf"),
            latency_p50_s=float(np.percentile(lat, 50)) if n else 0.0,
            latency_p99_s=float(np.percentile(lat, 99)) if n else 0.0,
            latency_max_s=float(lat.max()) if n else 0.0,
            wait_p50_s=float(np.percentile(wait, 50)) if n else 0.0,
            peak_bytes=peak, peak_active=peak_active, rounds=rounds, iterations=iters,
            statuses=statuses, latencies=lat, results=results, tiles=eng.get_tiles())


def solve_alone(p: Problem, proj: str = "f32", basis: str = "f32",
                tiles: tuple | None = None) -> SolveResult:
    """The same problem on an engine of its own (the reference for 'alone vs in a mix')."""
    e = Engine(proj=proj, basis=basis, max_slots=1)
    try:
        if tiles:
            e.set_tiles(*tiles)
        return e.run([p])[0]
    finally:
        e.close()
