"""Host checks of the stream server (no GPU): FIFO admission under a memory budget,
continuous batching versus one solve at a time, and the latency statistics, on a simulated
clock with hand-computed timelines."""
import numpy as np
import pytest

from paper_1906_11029_amd.serve import Request, StreamServer, percentile, poisson_arrivals, summarize


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, s):
        self.t += s


class FakeExecutor:
    """Set-up costs SETUP seconds, a step (one slab of every solve in flight) STEP seconds
    whatever the number of solves, a sequential run STEP per slab."""
    SETUP, STEP = 0.5, 1.0

    def __init__(self, clock, fp=1):
        self.clock, self.fp, self.log = clock, fp, []

    def footprint(self, req):
        return self.fp

    def setup(self, req):
        self.clock.t += self.SETUP
        return {"rid": req.rid, "left": req.spec["slabs"]}

    def slabs(self, h):
        return h["left"]

    def step(self, hs):
        self.log.append(sorted(h["rid"] for h in hs))
        self.clock.t += self.STEP

    def run(self, h):
        self.log.append([h["rid"]])
        self.clock.t += self.STEP * h["left"]

    def finish(self, h):
        return {"rid": h["rid"]}


def reqs(*items):
    return [Request(i, t, {"slabs": n}) for i, (t, n) in enumerate(items)]


def test_batched_stream_by_hand():
    """A (t=0, 2 slabs) is set up by 0.5 and steps to 1.5; B (t=0.1) joins at 1.5 (set up by
    2.0); one step takes both to their end at 3.0; C (t=5, 1 slab) waits idle, joins at 5.0
    and ends at 6.5."""
    clk = Clock()
    ex = FakeExecutor(clk)
    out = StreamServer(ex, budget_bytes=10, batched=True, clock=clk, sleep=clk.sleep).run(
        reqs((0.0, 2), (0.1, 1), (5.0, 1)))
    assert [r.done for r in out] == [3.0, 3.0, 6.5]
    assert [r.admitted for r in out] == [0.0, 1.5, 5.0]
    assert [r.setup_s for r in out] == [0.5, 0.5, 0.5]
    assert out[1].latency == pytest.approx(2.9)
    assert ex.log == [[0], [0, 1], [2]]


def test_memory_budget_holds_the_queue():
    """Budget for two solves: A and B run together; C (same arrival) is admitted only when
    they leave."""
    clk = Clock()
    ex = FakeExecutor(clk)
    out = StreamServer(ex, budget_bytes=2, batched=True, clock=clk, sleep=clk.sleep).run(
        reqs((0.0, 3), (0.0, 3), (0.0, 3)))
    assert [r.admitted for r in out] == [0.0, 0.5, 4.0]
    assert [r.done for r in out] == [4.0, 4.0, 7.5]
    assert ex.log == [[0, 1]] * 3 + [[2]] * 3


def test_sequential_serves_one_at_a_time_fifo():
    clk = Clock()
    ex = FakeExecutor(clk)
    out = StreamServer(ex, budget_bytes=10, batched=False, clock=clk, sleep=clk.sleep).run(
        reqs((0.0, 2), (0.0, 1)))
    assert [r.done for r in out] == [2.5, 4.0]
    assert ex.log == [[0], [1]]


def test_request_above_the_budget_is_refused():
    clk = Clock()
    with pytest.raises(ValueError):
        StreamServer(FakeExecutor(clk, fp=5), budget_bytes=4, clock=clk, sleep=clk.sleep).run(reqs((0.0, 1)))


def test_percentiles_and_summary():
    assert percentile(range(1, 101), 50) == 50
    assert percentile(range(1, 101), 99) == 99
    assert percentile([3.0], 99) == 3.0
    clk = Clock()
    out = StreamServer(FakeExecutor(clk), budget_bytes=10, clock=clk, sleep=clk.sleep).run(
        reqs((0.0, 2), (0.1, 1), (5.0, 1)))
    s = summarize(out, dof_updates=6.5e6)
    assert s["makespan_s"] == 6.5 and s["dof_updates_per_s"] == pytest.approx(1e6)
    assert s["latency_p50_s"] == pytest.approx(2.9) and s["latency_p99_s"] == pytest.approx(3.0)


def test_poisson_arrivals():
    rng = np.random.default_rng(5)
    t = poisson_arrivals(20000, rate=4.0, rng=rng)
    gaps = np.diff([0.0] + t)
    assert np.all(gaps > 0)
    assert gaps.mean() == pytest.approx(0.25, rel=0.03)       # mean gap 1 / rate
    assert gaps.std() == pytest.approx(0.25, rel=0.05)        # exponential: std = mean
