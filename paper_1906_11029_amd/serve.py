"""Serving a stream of independent solves (section 2: tents of independent problems are
independent, so the solves in flight share every launch).

Requests arrive at given times.  A FIFO queue admits the head request while the estimated
device memory of the solves in flight plus its own fits the budget; admitting a request sets
it up (mesh, pitching, solver).  In batched mode every solve in flight advances one slab per
step, all of them in one batch (rebuilt when the set changes); a solve that reaches its final
time is read out and leaves.  In sequential mode the head solve runs to its final time alone
before the next one starts.  Every request records its arrival, admission, set-up and
completion times; the latency of a request is completion minus arrival.

The executor does the work (a GPU one in bench.py, a simulated one in the tests):
  footprint(req) -> bytes        estimated device memory of the solve
  setup(req) -> handle           mesh, tents and solver (times itself via the clock)
  slabs(handle) -> int           slabs to reach the request's final time
  step(handles)                  one slab of every handle (batched mode)
  run(handle)                    every remaining slab of one handle (sequential mode)
  finish(handle) -> dict         read-out and release; may return per-request results
"""
import math
from dataclasses import dataclass, field


@dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the stream
    spec: dict              # what the executor needs to set the solve up


@dataclass
class Record:
    rid: int
    arrival: float
    admitted: float = math.nan
    setup_s: float = math.nan
    done: float = math.nan
    result: dict = field(default_factory=dict)

    @property
    def latency(self):
        return self.done - self.arrival


def percentile(values, q):
    """Nearest-rank percentile (q in [0, 100]) of a non-empty sequence."""
    v = sorted(values)
    if not v:
        raise ValueError("no values")
    k = max(1, math.ceil(q / 100.0 * len(v)))
    return v[k - 1]


class StreamServer:
    def __init__(self, executor, budget_bytes, batched=True, clock=None, sleep=None):
        import time
        self.ex = executor
        self.budget = budget_bytes
        self.batched = batched
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep

    def run(self, requests):
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in reqs:
            if self.ex.footprint(r) > self.budget:
                raise ValueError(f"request {r.rid} alone exceeds the memory budget")
        recs = {r.rid: Record(r.rid, r.arrival) for r in reqs}
        t0 = self.clock()
        now = lambda: self.clock() - t0  # noqa: E731
        queue, active = [], []          # active: (request, handle, slabs left, footprint)
        nxt = 0
        while nxt < len(reqs) or queue or active:
            while nxt < len(reqs) and reqs[nxt].arrival <= now():
                queue.append(reqs[nxt])
                nxt += 1
            # FIFO admission while the head fits (batched: beside the solves in flight)
            used = sum(a[3] for a in active)
            while queue and (not active or (self.batched and used + self.ex.footprint(queue[0]) <= self.budget)):
                r = queue.pop(0)
                rec = recs[r.rid]
                rec.admitted = now()
                h = self.ex.setup(r)
                rec.setup_s = now() - rec.admitted
                fp = self.ex.footprint(r)
                active.append((r, h, self.ex.slabs(h), fp))
                used += fp
                if not self.batched:
                    break
            if not active:
                if nxt < len(reqs):   # idle until the next arrival
                    self.sleep(max(0.0, reqs[nxt].arrival - now()))
                continue
            if self.batched:
                self.ex.step([a[1] for a in active])
                active = [(r, h, n - 1, fp) for (r, h, n, fp) in active]
            else:
                r, h, n, fp = active[0]
                self.ex.run(h)
                active = [(r, h, 0, fp)]
            left = []
            for r, h, n, fp in active:
                if n <= 0:
                    recs[r.rid].result = self.ex.finish(h) or {}
                    recs[r.rid].done = now()
                else:
                    left.append((r, h, n, fp))
            active = left
        return [recs[r.rid] for r in reqs]


def summarize(records, dof_updates):
    """Throughput and latency of a served stream: dof_updates is the total over requests."""
    span = max(r.done for r in records) - min(r.arrival for r in records)
    lat = [r.latency for r in records]
    return {"requests": len(records), "makespan_s": span, "requests_per_s": len(records) / span,
            "dof_updates_per_s": dof_updates / span, "latency_p50_s": percentile(lat, 50),
            "latency_p99_s": percentile(lat, 99), "setup_mean_s": sum(r.setup_s for r in records) / len(records)}


def poisson_arrivals(n, rate, rng):
    """n arrival times of a Poisson process of the given rate (per second), from 0."""
    gaps = rng.exponential(1.0 / rate, size=n)
    t = 0.0
    out = []
    for g in gaps:
        t += float(g)
        out.append(t)
    return out
