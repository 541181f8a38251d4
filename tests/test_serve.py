"""Scheduling logic of the serving loop (paper_1703_00879_amd/serve.py) on a simulated
device: admission by footprint in arrival order, interleaving across streams, latency
bookkeeping.  The GPU test of the same loop (results identical alone and in the mix) is
in test_gpu_serve.py."""

import numpy as np
import pytest

from paper_1703_00879_amd import cola as C
from paper_1703_00879_amd.serve import Request, Server, percentile, summarize


class _Ev:
    def __init__(self, t):
        self.t = t


class FakeEngine:
    """A device with `n_streams` in-order queues; a step of a run with np1d = n takes
    n**3 * 1e-9 s of simulated time, its IC as long as one step.  Simulated time advances
    when the loop idles and by a small tick per call of now()."""

    def __init__(self, n_streams=2, tick=1e-6):
        self.n = n_streams
        self.tick = tick
        self.clock = 0.0
        self.free_at = [0.0] * n_streams
        self.load = [0] * n_streams
        self.resident = 0
        self.max_resident = 0
        self.log = []

    def footprint(self, p):
        return p.np1d ** 3 * 100

    def begin(self):
        self.clock = 0.0

    def now(self):
        self.clock += self.tick
        return self.clock

    def _enqueue(self, si, dur):
        t = max(self.free_at[si], self.clock) + dur
        self.free_at[si] = t
        return _Ev(t)

    def start(self, p):
        si = min(range(self.n), key=lambda i: self.load[i])
        self.load[si] += 1
        self.resident += self.footprint(p)
        self.max_resident = max(self.max_resident, self.resident)
        self.log.append(("start", p.seed, self.clock))
        self._enqueue(si, p.np1d ** 3 * 1e-9)
        return {"p": p, "si": si}

    def step(self, h, i):
        return self._enqueue(h["si"], h["p"].np1d ** 3 * 1e-9)

    def done(self, ev):
        return ev.t <= self.clock

    def idle(self, s):
        self.clock += max(s, 1e-5)

    def finish_time(self, ev):
        return ev.t

    def release(self, h, keep):
        self.load[h["si"]] -= 1
        self.resident -= self.footprint(h["p"])
        self.log.append(("end", h["p"].seed, self.clock))
        return None


def _req(n, steps, seed, arrival):
    return Request(C.Params(np1d=n, nmesh1d=2 * n, n_steps=steps, seed=seed), arrival=arrival, rid=seed)


def test_budget_is_never_exceeded_and_every_request_completes():
    rng = np.random.default_rng(3)
    reqs = [_req(int(rng.choice([64, 128, 192])), int(rng.integers(3, 8)), s, float(rng.uniform(0, 0.01)))
            for s in range(40)]
    eng = FakeEngine(n_streams=3)
    budget = 2 * 192 ** 3 * 100
    res = Server(eng, budget, max_active=8).run(reqs)
    assert eng.max_resident <= budget
    assert [r.rid for r in res] == [q.rid for q in reqs]
    for q, r in zip(reqs, res):
        work = (q.params.n_steps + 1) * q.params.np1d ** 3 * 1e-9
        assert r.admitted >= q.arrival
        assert r.finished >= r.admitted + work - 1e-12
        assert r.latency >= work - 1e-12


def test_admission_is_in_arrival_order():
    reqs = [_req(128, 4, s, 0.001 * (9 - s)) for s in range(10)]   # arrive in reverse seed order
    eng = FakeEngine(n_streams=2)
    res = Server(eng, 3 * 128 ** 3 * 100, max_active=3).run(reqs)
    starts = [seed for kind, seed, _ in eng.log if kind == "start"]
    assert starts == sorted(starts, key=lambda s: reqs[s].arrival)
    order = sorted(range(10), key=lambda j: reqs[j].arrival)
    adm = [res[j].admitted for j in order]
    assert adm == sorted(adm)


def test_runs_overlap_when_slots_and_memory_allow():
    reqs = [_req(128, 10, s, 0.0) for s in range(4)]
    eng = FakeEngine(n_streams=4)
    res = Server(eng, 10 ** 12, max_active=4).run(reqs)
    one = 11 * 128 ** 3 * 1e-9
    # four runs on four streams finish together, not one after the other
    assert max(r.finished for r in res) < 1.5 * one
    eng1 = FakeEngine(n_streams=1)
    res1 = Server(eng1, 10 ** 12, max_active=1).run(reqs)
    assert max(r.finished for r in res1) > 3.5 * one


def test_memory_limits_concurrency():
    reqs = [_req(128, 5, s, 0.0) for s in range(6)]
    eng = FakeEngine(n_streams=6)
    Server(eng, 2 * 128 ** 3 * 100, max_active=6).run(reqs)
    assert eng.max_resident == 2 * 128 ** 3 * 100


def test_request_larger_than_budget_is_rejected_before_any_work():
    eng = FakeEngine()
    with pytest.raises(ValueError):
        Server(eng, 64 ** 3 * 100).run([_req(64, 2, 0, 0.0), _req(128, 2, 1, 0.0)])
    assert eng.log == []


def test_percentile_and_summary():
    xs = list(np.random.default_rng(0).exponential(size=101))
    for q in (0, 50, 99, 100):
        assert percentile(xs, q) == pytest.approx(np.percentile(xs, q))
    reqs = [_req(64, 3, s, 0.0) for s in range(5)]
    res = Server(FakeEngine(n_streams=1), 10 ** 12, max_active=1).run(reqs)
    s = summarize(res)
    assert s["runs"] == 5
    assert s["runs_per_hour"] == pytest.approx(3600 * 5 / s["span_s"])
    assert s["p99_s"] >= s["p50_s"] > 0


def test_kept_states_hold_their_footprint():
    # a finished run whose state is kept stays resident: its footprint counts against the
    # budget, so admission never overcommits, and a request that can never fit is an error
    reqs = [_req(64, 2, s, 0.0) for s in range(3)]
    eng = FakeEngine(n_streams=2)
    fp = 64 ** 3 * 100
    res = Server(eng, 3 * fp, max_active=3, keep_states=True).run(reqs)
    assert len(res) == 3
    with pytest.raises(RuntimeError):
        Server(FakeEngine(n_streams=2), 2 * fp, max_active=3, keep_states=True).run(reqs)
