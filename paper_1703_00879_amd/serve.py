"""Continuous batching of mock runs on one GPU: a serving loop and ensemble runs.

The method exists to make large ensembles of mock catalogues (Sec. 1), so runs of
different sizes, models and seeds arrive as requests.  The loop keeps each admitted run's
whole state (particles, LPT fields, tables, meshes) resident in HBM until its last step
and interleaves the steps of all admitted runs:

- **admission**: requests are taken in arrival order once they have arrived, while the
  device footprint of the admitted runs (the ``cola_query_sizes`` total of each) stays
  within the HBM budget and a slot is free.  A request whose footprint exceeds the whole
  budget is rejected;
- **interleaving**: each pass over the admitted runs enqueues one ``cola_step`` of every
  run with fewer than ``depth`` steps in flight.  Runs are spread over a few streams
  (default priority), so the kernels of small runs overlap on the device, and a run
  admitted while others are running starts at once;
- **completion**: a run is retired when the event after its last step has completed; its
  time to z = 0 is that event's device time minus the request's arrival time, both on
  the loop's clock (device time is taken from an event recorded when the loop starts).

Every step is the library's own ``cola_step``: a run's result does not depend on what
else is in the mix (the deposit accumulates in integers and no kernel keeps state
between calls).  The engine is replaceable: the scheduling logic runs on the CPU with a
simulated engine in the tests.
"""

import time
from dataclasses import dataclass, field

from . import cola as C


@dataclass
class Request:
    params: "C.Params"
    arrival: float = 0.0   # seconds after the loop starts
    rid: int = 0


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    particle_steps: int
    state: object = None   # the final State when the loop keeps states

    @property
    def latency(self):
        return self.finished - self.arrival


@dataclass
class _Run:
    req: Request
    index: int
    handle: object
    admitted: float
    footprint: int
    next_step: int = 0
    last: object = None                            # event after the latest enqueued step
    inflight: list = field(default_factory=list)   # events of steps not known complete


class GpuEngine:
    """Runs requests through the library on one device, one stream per slot group."""

    def __init__(self, device="cuda:0", n_streams=4):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self.load = [0] * n_streams
        self.t0_host = None
        self.t0_event = None

    def footprint(self, p):
        return C.cola_query_sizes(p)["total_bytes"] + 5 * 256

    def begin(self):
        torch = self.torch
        torch.cuda.synchronize(self.device)
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_event.record(torch.cuda.current_stream(self.device))
        self.t0_host = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0_host

    def start(self, p):
        si = min(range(len(self.streams)), key=lambda i: self.load[i])
        self.load[si] += 1
        st = C.State(p, device=self.device)
        C.cola_make_ic(p, st, stream=self.streams[si].cuda_stream)
        return {"p": p, "state": st, "stream": si}

    def step(self, h, i):
        torch = self.torch
        s = self.streams[h["stream"]]
        C.cola_step(h["p"], h["state"], i, stream=s.cuda_stream)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(s)
        return ev

    def done(self, ev):
        return ev.query()

    def idle(self, seconds):
        time.sleep(seconds)

    def finish_time(self, ev):
        return self.t0_event.elapsed_time(ev) / 1e3

    def release(self, h, keep):
        self.load[h["stream"]] -= 1
        return h["state"] if keep else None


class Server:
    """The request loop.  ``run(requests)`` returns one Result per request (in request
    order); requests that can never fit the budget raise ValueError before any work."""

    def __init__(self, engine, hbm_budget, max_active=16, depth=2, keep_states=False):
        if depth < 1 or max_active < 1:
            raise ValueError("depth and max_active must be >= 1")
        self.engine = engine
        self.budget = int(hbm_budget)
        self.max_active = max_active
        self.depth = depth
        self.keep = keep_states

    def run(self, requests, on_result=None):
        eng = self.engine
        order = sorted(range(len(requests)), key=lambda j: (requests[j].arrival, j))
        fps = {j: eng.footprint(requests[j].params) for j in order}
        for j, fp in fps.items():
            if fp > self.budget:
                raise ValueError(f"request {requests[j].rid}: footprint {fp} B exceeds the budget")
        pending = list(order)
        active, used, results = [], 0, {}
        eng.begin()
        while pending or active:
            now = eng.now()
            # admission in arrival order: the head of the queue waits for room
            while (pending and requests[pending[0]].arrival <= now and len(active) < self.max_active
                   and used + fps[pending[0]] <= self.budget):
                j = pending.pop(0)
                active.append(_Run(req=requests[j], index=j, handle=eng.start(requests[j].params),
                                   admitted=now, footprint=fps[j]))
                used += fps[j]
            progressed = False
            for run in active:
                run.inflight = [ev for ev in run.inflight if not eng.done(ev)]
                if run.next_step < run.req.params.n_steps and len(run.inflight) < self.depth:
                    run.last = eng.step(run.handle, run.next_step)
                    run.inflight.append(run.last)
                    run.next_step += 1
                    progressed = True
            still = []
            for run in active:
                if run.next_step == run.req.params.n_steps and eng.done(run.last):
                    p = run.req.params
                    results[run.index] = Result(
                        rid=run.req.rid, arrival=run.req.arrival, admitted=run.admitted,
                        finished=eng.finish_time(run.last), particle_steps=p.np1d ** 3 * p.n_steps,
                        state=eng.release(run.handle, self.keep))
                    if not self.keep:   # a kept state stays resident and keeps its footprint
                        used -= run.footprint
                    if on_result:
                        on_result(len(results), len(requests))
                    progressed = True
                else:
                    still.append(run)
            active = still
            if not progressed:
                if not active and pending and used + fps[pending[0]] > self.budget:
                    raise RuntimeError("the HBM budget is held by kept states: request "
                                       f"{requests[pending[0]].rid} can never be admitted")
                if active:
                    eng.idle(50e-6)   # every admitted run has `depth` steps in flight
                elif pending:
                    eng.idle(min(max(requests[pending[0]].arrival - eng.now(), 0.0), 0.05))
        return [results[j] for j in range(len(requests))]


def percentile(xs, q):
    """q-th percentile (0-100) by linear interpolation between order statistics."""
    s = sorted(xs)
    if not s:
        return float("nan")
    pos = (len(s) - 1) * q / 100.0
    lo = int(pos)
    hi = min(lo + 1, len(s) - 1)
    return s[lo] + (s[hi] - s[lo]) * (pos - lo)


def summarize(results):
    """Throughput and latency of a finished request stream."""
    span = max(r.finished for r in results) - min(r.arrival for r in results)
    lat = [r.latency for r in results]
    ps = sum(r.particle_steps for r in results)
    return {"runs": len(results), "span_s": span, "runs_per_hour": 3600.0 * len(results) / span,
            "particle_steps_per_s": ps / span, "p50_s": percentile(lat, 50),
            "p99_s": percentile(lat, 99)}
