"""Scheduler of the serving loop, driven on the CPU by a simulated executor:
FIFO admission, the HBM budget, lane concurrency and latency accounting."""
import time

import numpy as np
import pytest

from paper_2608_09733_amd import inputs as I
from paper_2608_09733_amd import serving as S


class FakeExecutor:
    """Completes a request `dur(n)` seconds after it starts; the result is a
    function of the request id only."""

    def __init__(self, lanes, dur=lambda n: 1e-4 * (1 << max(0, n - 10))):
        self.lanes = lanes
        self.dur = dur
        self.started = []
        self.held = [set() for _ in range(lanes)]

    def pool_bytes(self):
        return sum(S.request_bytes(n) for h in self.held for n in h)

    def evict_idle(self, need, budget, inflight):
        return True

    def needs_new(self, lane, n):
        return n not in self.held[lane]

    def start(self, lane, req):
        self.held[lane].add(req.circuit.n)
        self.started.append((req.rid, lane, time.perf_counter()))
        return (time.perf_counter() + self.dur(req.circuit.n), req.rid)

    def poll(self, lane, token):
        t, rid = token
        if time.perf_counter() < t:
            return None
        return float(rid), np.array([rid], dtype=float)


def _trace(count=40, rate=2000.0, seed=0, n_hi=16):
    return I.serving_trace(rate, count, seed=seed, n_lo=10, n_hi=n_hi, l_lo=2, l_hi=3)


def test_every_request_completes_with_its_own_result():
    tr = _trace()
    rep = S.Server(FakeExecutor(3), 3).serve(tr)
    assert [o.rid for o in rep.outcomes] == [r.rid for r in tr]
    for o in rep.outcomes:
        assert o.energy == float(o.rid)
        assert o.arrival <= o.admitted + 1e-9 <= o.done + 1e-9


def test_admission_is_fifo():
    tr = _trace(count=60)
    ex = FakeExecutor(4)
    S.Server(ex, 4).serve(tr)
    order = [rid for rid, _, _ in ex.started]
    assert order == sorted(order)


def test_budget_bounds_inflight_bytes():
    tr = _trace(count=30, n_hi=16)
    budget = S.request_bytes(16) + S.request_bytes(12)
    rep = S.Server(FakeExecutor(4), 4, budget_bytes=budget).serve(tr)
    assert rep.peak_inflight_bytes <= budget
    assert len(rep.outcomes) == 30


def test_request_larger_than_budget_is_refused():
    tr = _trace(count=5)
    with pytest.raises(ValueError):
        S.Server(FakeExecutor(1), 1, budget_bytes=S.request_bytes(9)).serve(tr)


def test_more_lanes_overlap_requests():
    tr = _trace(count=24, rate=1e6, n_hi=14)
    one = S.Server(FakeExecutor(1), 1).serve(tr)
    four = S.Server(FakeExecutor(4), 4).serve(tr)
    assert four.makespan < 0.6 * one.makespan
    s = four.summary()
    assert s["requests"] == 24 and s["latency_p99_ms"] >= s["latency_p50_ms"]


class FakeBatchExecutor(FakeExecutor):
    """FakeExecutor with a batch path for requests of n <= 13: a submission
    completes `bdur` seconds after it starts."""

    def __init__(self, lanes, dur=lambda n: 1e-4 * (1 << max(0, n - 10)), bdur=5e-4):
        super().__init__(lanes, dur)
        self.bdur = bdur
        self.batches = []
        self.live = 0
        self.max_live = 0

    def batchable(self, req):
        return 3 <= req.circuit.n <= 13

    def start_batch(self, reqs):
        self.batches.append([r.rid for r in reqs])
        self.live += 1
        self.max_live = max(self.max_live, self.live)
        return (time.perf_counter() + self.bdur, [r.rid for r in reqs])

    def poll_batch(self, token):
        t, rids = token
        if time.perf_counter() < t:
            return None
        self.live -= 1
        return [(float(r), np.array([r], dtype=float)) for r in rids]


def test_small_requests_take_the_batch_path():
    tr = _trace(count=60, rate=5000.0, n_hi=24)
    ex = FakeBatchExecutor(4)
    rep = S.Server(ex, 4).serve(tr)
    assert [o.rid for o in rep.outcomes] == [r.rid for r in tr]
    for o in rep.outcomes:
        assert o.energy == float(o.rid)
        assert (o.lane < 0) == (o.n <= 13) == (o.klass == S.SMALL)
    on_lanes = {rid for rid, _, _ in ex.started}
    batched = [rid for b in ex.batches for rid in b]
    assert not on_lanes & set(batched)
    assert sorted(on_lanes | set(batched)) == [r.rid for r in tr]
    assert batched == sorted(batched)                  # FIFO within the class
    assert ex.max_live <= 2
    assert rep.summary()["batch_submissions"] == len(ex.batches)


def test_big_requests_only_on_big_lanes_and_fifo_per_class():
    tr = _trace(count=80, rate=1e5, n_hi=24)
    ex = FakeBatchExecutor(4, dur=lambda n: 2e-4)
    rep = S.Server(ex, 4).serve(tr)
    n_of = {r.rid: r.circuit.n for r in tr}
    for rid, lane, _ in ex.started:
        if n_of[rid] >= 21:
            assert lane == 0
    for k in (S.MID, S.BIG):
        order = [rid for rid, _, _ in ex.started if (n_of[rid] >= 21) == (k == S.BIG)]
        assert order == sorted(order)
    assert len(rep.outcomes) == 80


def test_mid_requests_do_not_wait_behind_a_big_one():
    """A long big request arrives first; the mid requests after it finish
    while it still runs (they have lanes of their own)."""
    import math
    reqs = [I.Request(0, 0.0, I.layered(24, 1), I.tfim(24))]
    for k in range(1, 9):
        reqs.append(I.Request(k, 1e-3 * k, I.layered(16, 1), I.tfim(16)))
    ex = FakeBatchExecutor(4, dur=lambda n: 0.2 if n >= 21 else 1e-3)
    rep = S.Server(ex, 4).serve(reqs)
    big = rep.outcomes[0]
    assert all(o.done < big.done for o in rep.outcomes[1:])
    assert math.isclose(big.latency, 0.2, rel_tol=0.5)


def test_one_lane_without_batch_is_serial_fifo():
    tr = _trace(count=40, rate=1e5, n_hi=24)
    ex = FakeBatchExecutor(1)
    S.Server(ex, 1, batch=False).serve(tr)
    assert not ex.batches
    order = [rid for rid, _, _ in ex.started]
    assert order == sorted(order) == [r.rid for r in tr]
