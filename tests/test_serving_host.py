"""Host logic of the request loop (admission by memory, slots, FIFO order, latency
bookkeeping) with a stand-in engine that finishes each problem after k_max rounds.
Runs on the CPU."""
from dataclasses import dataclass

import numpy as np
import torch

from paper_2110_01481_amd.serving import Request, Server


@dataclass
class _G:
    n: int


@dataclass
class _P:
    g: _G
    b: torch.Tensor
    method: str
    k_max: int
    stop: str = "dp"
    nbytes: int = 0


@dataclass
class _R:
    status: str
    k_done: int


class _FakeEngine:
    def __init__(self, slots):
        self.slots = slots
        self.active = {}
        self.done = []
        self.next = 1
        self.submitted = []
        self.max_active = 0

    def submit(self, p, x=None, workspace=None):
        if len(self.active) >= self.slots:
            return None
        assert workspace.numel() == p.nbytes and x.numel() == p.g.n
        t = self.next
        self.next += 1
        self.active[t] = [p.k_max, p]
        self.submitted.append(p)
        self.max_active = max(self.max_active, len(self.active))
        return t

    def step(self):
        for t in list(self.active):
            self.active[t][0] -= 1
            if self.active[t][0] == 0:
                self.done.append((t, _R("ok", self.active[t][1].k_max)))
                del self.active[t]

    def poll(self):
        out, self.done = self.done, []
        return out

    def get_tiles(self):
        return (256, 128, 0)

    def set_tiles(self, *a):
        pass

    def close(self):
        pass


class _Server(Server):
    def request_bytes(self, p):
        return p.nbytes


def _stream(n, rate, seed=0):
    g = np.random.default_rng(seed)
    t = np.cumsum(g.exponential(1.0 / rate, n))
    reqs = []
    for i in range(n):
        nb = int(g.integers(1000, 5000))
        p = _P(_G(16), torch.zeros(4), "ab" if i % 2 else "ba", int(g.integers(2, 6)), nbytes=nb)
        reqs.append(Request(float(t[i]), p))
    return reqs


def test_budget_slots_and_fifo():
    reqs = _stream(40, rate=2000.0)
    eng = _FakeEngine(slots=5)
    srv = _Server(engine=eng, budget_bytes=12000)
    rep = srv.run(reqs)
    assert rep.n == 40 and rep.statuses == {"ok": 40}
    assert rep.peak_bytes <= 12000 and eng.max_active <= 5 and rep.peak_active <= 5
    # first come, first served
    assert [id(p) for p in eng.submitted] == [id(r.problem) for r in reqs]
    assert np.all(rep.latencies >= 0) and rep.latency_p99_s >= rep.latency_p50_s
    assert rep.iterations == sum(r.problem.k_max for r in reqs)


def test_closed_batch_and_oversized_request():
    reqs = _stream(10, rate=10.0)
    rep = _Server(engine=_FakeEngine(slots=64), budget_bytes=10 ** 9).run(reqs, realtime=False)
    assert rep.n == 10 and rep.rounds == max(r.problem.k_max for r in reqs)
    big = _stream(1, rate=1.0)
    big[0].problem.nbytes = 10 ** 6
    try:
        _Server(engine=_FakeEngine(slots=1), budget_bytes=1000).run(big)
    except ValueError:
        pass
    else:
        raise AssertionError("a request larger than the budget must be refused")
