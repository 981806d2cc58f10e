"""Serving loop: variational requests (circuit, angles, Hamiltonian) arrive
over time; each returns (E, dE/dtheta) from the adjoint path.

Requests fall into three classes, each FIFO within itself:

* small -- requests of at most `small_max` qubits (14 by default; the
  serving kernel takes 3..16, ops on at most 3 qubits): they join the batch
  path as they arrive.  Whenever fewer than two
  submissions are in flight, every small request that has arrived is
  submitted as one persistent launch (sv_serve_submit) on a stream of its
  own; one workgroup runs one request whole, so these never queue behind a
  28-qubit request and take a few CUs each.  14 qubits is the measured
  balance: at 200 req/s, routing up to 13, 14 and 16 qubits gave p50 122, 36
  and 16 ms, p99 7.33, 7.37 and 7.71 s, and 49.3, 49.1 and 47.5 req/s (a
  15- or 16-qubit request holds one CU for 6-13 ms, where a lane spreads it
  over many CUs in about 1 ms).
* big (n >= 21 qubits) and mid (the rest) -- run on stream lanes through
  sv_adjoint_grad_device.  One lane takes big requests first (then mid ones
  when no big request waits); the other lanes take only mid requests, so a
  mid request never waits behind a long one.  One big lane is enough: a big
  request fills the GPU by itself, and a second one running beside it only
  time-slices the GPU with it while the short kernels of the small and mid
  requests wait longer for free CUs (measured: p50 of the small requests
  16 ms with one big lane, 32 ms with two, 495 ms with three).

A request is admitted when the HBM budget holds its three states (psi,
lambda and the backward copy of psi, 3 * 2^n * 16 bytes in FP64).  Each lane
keeps one library handle per qubit count, so after warm-up a lane request
allocates only its small output buffer; plans are cached per circuit
structure.  With one lane and no batch path the loop is serial FIFO, the
baseline the served figures are compared with.  Results come back through
an asynchronous copy into pinned host memory on the request's stream, so a
poll never blocks the scheduler behind kernels still in flight.

The executor is pluggable: `GpuExecutor` runs the HIP library; tests drive
the scheduler with a simulated executor on the CPU.

    python -m paper_2608_09733_amd.serving --rate 200 --count 500 --lanes 2
    python -m paper_2608_09733_amd.serving --sweep 50,100,200,500,1000,2000 --count 500
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field
from typing import Dict, List

import numpy as np

GB = 1e9
SMALL, MID, BIG = "small", "mid", "big"


def request_bytes(n: int, elem: int = 8) -> int:
    """HBM held by one request: three states of 2^n complex amplitudes."""
    return 3 * 2 * elem * (1 << n)


@dataclass
class Outcome:
    rid: int
    n: int
    arrival: float
    admitted: float
    done: float
    energy: float
    grad: np.ndarray
    lane: int            # stream lane, or -1 for the batch path
    klass: str = MID

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def _pct(a: np.ndarray, q: float) -> float:
    return float(np.percentile(a, q) * 1e3) if len(a) else 0.0


@dataclass
class Report:
    outcomes: List[Outcome]
    makespan: float
    peak_inflight_bytes: int
    peak_pool_bytes: int
    lanes: int
    budget_bytes: float
    batches: int = 0
    stats: Dict[str, float] = field(default_factory=dict)

    def summary(self) -> Dict[str, float]:
        lat = np.array([o.latency for o in self.outcomes])
        q = np.array([o.admitted - o.arrival for o in self.outcomes])
        sv = np.array([o.done - o.admitted for o in self.outcomes])
        out = {
            "requests": len(self.outcomes),
            "lanes": self.lanes,
            "makespan_s": self.makespan,
            "throughput_req_s": len(self.outcomes) / self.makespan if self.makespan > 0 else 0.0,
            "latency_p50_ms": _pct(lat, 50),
            "latency_p99_ms": _pct(lat, 99),
            "queue_mean_ms": float(q.mean() * 1e3) if len(q) else 0.0,
            "service_mean_ms": float(sv.mean() * 1e3) if len(sv) else 0.0,
            "peak_inflight_gb": self.peak_inflight_bytes / GB,
            "peak_pool_gb": self.peak_pool_bytes / GB,
            "budget_gb": self.budget_bytes / GB,
            "batch_submissions": self.batches,
        }
        for k in (SMALL, MID, BIG):
            lk = np.array([o.latency for o in self.outcomes if o.klass == k])
            sk = np.array([o.done - o.admitted for o in self.outcomes if o.klass == k])
            out[f"{k}_requests"] = int(len(lk))
            out[f"{k}_latency_p50_ms"] = _pct(lk, 50)
            out[f"{k}_latency_p99_ms"] = _pct(lk, 99)
            out[f"{k}_service_mean_ms"] = float(sk.mean() * 1e3) if len(sk) else 0.0
        return out


class GpuExecutor:
    """Runs requests through the HIP library: lane requests on one HIP stream
    per lane (sv_adjoint_grad_device), small requests through the serving
    kernel on a stream of its own (sv_serve_submit)."""

    def __init__(self, lanes: int, dtype: str = "c128", batch: bool = True):
        import torch
        from . import sv
        self.torch = torch
        self.sv = sv
        self.dtype = dtype
        self.elem = 8 if dtype == "c128" else 4
        self.streams = [torch.cuda.Stream() for _ in range(lanes)]
        # per lane: qubit count -> handle, in least-recently-used order
        self.handles: List[OrderedDict] = [OrderedDict() for _ in range(lanes)]
        self.busy = [False] * lanes
        self.serve = sv.Serve() if (batch and dtype == "c128") else None
        self.bstream = torch.cuda.Stream() if self.serve is not None else None
        self._takes: Dict[tuple, bool] = {}

    def pool_bytes(self) -> int:
        return sum(request_bytes(n, self.elem) for h in self.handles for n in h)

    def evict_idle(self, need: int, budget: float, inflight: int) -> bool:
        """Close idle cached handles (least recently used first, from idle
        lanes) until `need` more bytes fit; False if they cannot."""
        while self.pool_bytes() + need > budget:
            victim = None
            for lane, h in enumerate(self.handles):
                if self.busy[lane] or not h:
                    continue
                victim = (lane, next(iter(h)))
                break
            if victim is None:
                return False
            lane, n = victim
            self.handles[lane].pop(n).close()
        return True

    def needs_new(self, lane: int, n: int) -> bool:
        return n not in self.handles[lane]

    def start(self, lane: int, req):
        torch, sv = self.torch, self.sv
        h = self.handles[lane]
        s = self.streams[lane]
        st = h.pop(req.circuit.n, None)
        if st is None:
            with torch.cuda.stream(s):   # planes belong to the lane's stream
                st = sv.State(req.circuit.n, self.dtype, adjoint=True, stream=s)
        h[req.circuit.n] = st       # most recently used last
        self.busy[lane] = True
        with torch.cuda.stream(s):
            out = torch.empty(1 + len(req.circuit.params), dtype=torch.float64, device="cuda")
            st.reset()
            st.adjoint_grad_device(req.circuit.ops, req.circuit.params, req.ham, out,
                                   op_array=sv.op_array_for(req.circuit))
            host = self._to_host(out)
            ev = torch.cuda.Event()
            ev.record(s)
        return (out, host, ev)

    def _to_host(self, out):
        # results go to pinned host memory on the lane's own stream, before
        # the completion event: a poll then reads host memory and never waits
        # on the device (a synchronous copy would queue behind whatever
        # kernels fill the GPU, and block the scheduler meanwhile)
        host = self.torch.empty(out.numel(), dtype=out.dtype, pin_memory=True)
        host.copy_(out, non_blocking=True)
        return host

    def poll(self, lane: int, token):
        out, host, ev = token
        if not ev.query():
            return None
        v = host.numpy()
        self.busy[lane] = False
        return float(v[0]), v[1:].copy()

    # ---- batch path
    def batchable(self, req) -> bool:
        """True if the serving kernel takes the request (decided once per
        circuit structure key)."""
        if self.serve is None:
            return False
        c = req.circuit
        if not 3 <= c.n <= self.sv.Serve.max_qubits():
            return False
        key = getattr(c, "key", None)
        if key is not None and key in self._takes:
            return self._takes[key]
        ok = self.serve.supports(c, req.ham)
        if key is not None:
            self._takes[key] = ok
        return ok

    def start_batch(self, reqs):
        torch = self.torch
        with torch.cuda.stream(self.bstream):
            tot = sum(1 + len(r.circuit.params) for r in reqs)
            out = torch.empty(tot, dtype=torch.float64, device="cuda")
            offs = self.serve.submit([r.circuit for r in reqs], [r.ham for r in reqs], out,
                                     self.bstream)
            host = self._to_host(out)
            ev = torch.cuda.Event()
            ev.record(self.bstream)
        return (out, host, offs, ev)

    def poll_batch(self, token):
        out, host, offs, ev = token
        if not ev.query():
            return None
        v = host.numpy()
        return [(float(v[offs[k]]), v[offs[k] + 1:offs[k + 1]].copy()) for k in range(len(offs) - 1)]

    def close(self):
        for h in self.handles:
            for st in h.values():
                st.close()
            h.clear()
        if self.serve is not None:
            self.serve.close()
            self.serve = None


class Server:
    """FIFO admission per request class under an HBM budget: small requests
    through the executor's batch path (when it has one and `batch`), the rest
    over `lanes` stream lanes (lane 0 big-first, the others mid-only; a single
    lane serves every class in arrival order)."""

    def __init__(self, executor, lanes: int, budget_bytes: float = 200 * GB, elem: int = 8,
                 batch: bool = True, big_qubits: int = 21, max_batch: int = 256,
                 batch_inflight: int = 2, small_max: int = 14):
        self.ex = executor
        self.lanes = lanes
        self.budget = budget_bytes
        self.elem = elem
        self.batch = batch and hasattr(executor, "start_batch")
        self.big_qubits = big_qubits
        self.max_batch = max_batch
        self.batch_inflight = batch_inflight
        self.small_max = small_max
        # queues a lane takes from, in order of preference
        self.lane_queues = [(BIG, MID) if l == 0 else (MID,) for l in range(lanes)]
        if lanes == 1:
            self.lane_queues = [("all",)]

    def klass(self, req) -> str:
        if self.batch and req.circuit.n <= self.small_max and self.ex.batchable(req):
            return SMALL
        return BIG if req.circuit.n >= self.big_qubits else MID

    def serve(self, trace, realtime: bool = True, clock=time.perf_counter,
              idle_sleep: float = 2e-4) -> Report:
        pending = deque(sorted(trace, key=lambda r: r.arrival))
        for r in pending:
            if request_bytes(r.circuit.n, self.elem) > self.budget:
                raise ValueError(f"request {r.rid}: {r.circuit.n} qubits exceed the HBM budget")
        klass = {r.rid: self.klass(r) for r in pending}
        queues: Dict[str, deque] = {k: deque() for k in (SMALL, MID, BIG, "all")}
        running: Dict[int, tuple] = {}          # lane -> (req, token, admitted)
        batches: List[tuple] = []               # (reqs, token, admitted)
        inflight = 0
        peak_inflight = 0
        peak_pool = 0
        n_batches = 0
        outcomes: List[Outcome] = []
        t0 = clock()
        now = 0.0
        while pending or any(queues.values()) or running or batches:
            now = clock() - t0
            if (not realtime and not any(queues.values()) and not running and not batches
                    and pending):
                now = max(now, pending[0].arrival)
            while pending and (pending[0].arrival <= now or not realtime):
                r = pending.popleft()
                k = klass[r.rid]
                queues[k if (k == SMALL or self.lanes > 1) else "all"].append(r)
            progressed = False
            # ---- completions
            for lane in list(running):
                req, token, adm = running[lane]
                res = self.ex.poll(lane, token)
                if res is None:
                    continue
                done = clock() - t0
                e, g = res
                outcomes.append(Outcome(req.rid, req.circuit.n, req.arrival, adm, done, e, g, lane,
                                        klass[req.rid]))
                inflight -= request_bytes(req.circuit.n, self.elem)
                del running[lane]
                progressed = True
            for b in list(batches):
                reqs, token, adm = b
                res = self.ex.poll_batch(token)
                if res is None:
                    continue
                done = clock() - t0
                for req, (e, g) in zip(reqs, res):
                    outcomes.append(Outcome(req.rid, req.circuit.n, req.arrival, adm, done, e, g, -1,
                                            SMALL))
                    inflight -= request_bytes(req.circuit.n, self.elem)
                batches.remove(b)
                progressed = True
            # ---- small requests: one submission of all that have arrived
            q = queues[SMALL]
            if q and len(batches) < self.batch_inflight:
                take = []
                while q and len(take) < self.max_batch:
                    need = request_bytes(q[0].circuit.n, self.elem)
                    if inflight + need > self.budget:
                        break
                    take.append(q.popleft())
                    inflight += need
                if take:
                    adm = clock() - t0
                    batches.append((take, self.ex.start_batch(take), adm))
                    n_batches += 1
                    peak_inflight = max(peak_inflight, inflight)
                    progressed = True
            # ---- lanes
            for lane in range(self.lanes):
                if lane in running:
                    continue
                req = None
                for k in self.lane_queues[lane]:
                    if queues[k]:
                        cand = queues[k][0]
                        need = request_bytes(cand.circuit.n, self.elem)
                        if inflight + need > self.budget:
                            break
                        if self.ex.needs_new(lane, cand.circuit.n):
                            if not self.ex.evict_idle(need, self.budget, inflight):
                                break
                        req = queues[k].popleft()
                        break
                if req is None:
                    continue
                adm = clock() - t0
                running[lane] = (req, self.ex.start(lane, req), adm)
                inflight += request_bytes(req.circuit.n, self.elem)
                peak_inflight = max(peak_inflight, inflight)
                peak_pool = max(peak_pool, self.ex.pool_bytes())
                progressed = True
            if not progressed:
                if running or batches or not pending:
                    time.sleep(idle_sleep)
                else:
                    wait = pending[0].arrival - (clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
        makespan = clock() - t0
        outcomes.sort(key=lambda o: o.rid)
        return Report(outcomes, makespan, peak_inflight, peak_pool, self.lanes, self.budget, n_batches)


def alone_vs_mix(report: Report, trace, dtype: str = "c128") -> int:
    """Re-run every request alone -- on one lane, or as a submission of one on
    the batch path, whichever served it -- and count those whose energy or
    gradient differs from the served result in any bit."""
    ex = GpuExecutor(1, dtype)
    try:
        by_id = {r.rid: r for r in trace}
        bad = 0
        for o in report.outcomes:
            req = by_id[o.rid]
            if o.lane < 0:
                tok = ex.start_batch([req])
                res = None
                while res is None:
                    res = ex.poll_batch(tok)
                e, g = res[0]
            else:
                tok = ex.start(0, req)
                res = None
                while res is None:
                    res = ex.poll(0, tok)
                e, g = res
            if e != o.energy or not np.array_equal(g, o.grad):
                bad += 1
        return bad
    finally:
        ex.close()


def run(rate: float, count: int, lanes: int, budget_gb: float = 200.0, seed: int = 0,
        dtype: str = "c128", serial_baseline: bool = True, check_identity: bool = True,
        n_hi: int = 28, log=None, small_max: int = 14) -> Dict[str, object]:
    """Served (classes, batch path, `lanes` lanes) and serial FIFO (one lane, no
    batch path) over the same trace.  Each runs the trace twice: the first pass
    builds the handles and plans (cold), the second is reported."""
    from . import inputs as I
    trace = I.serving_trace(rate, count, seed=seed, n_hi=n_hi)
    out: Dict[str, object] = {"rate_req_s": rate, "trace_requests": count, "seed": seed,
                              "trace_span_s": float(trace[-1].arrival) if trace else 0.0}
    ex = GpuExecutor(lanes, dtype)
    try:
        cold = Server(ex, lanes, budget_gb * GB, ex.elem, small_max=small_max).serve(trace)
        rep = Server(ex, lanes, budget_gb * GB, ex.elem, small_max=small_max).serve(trace)
    finally:
        ex.close()
    out["served_cold"] = cold.summary()
    out["served"] = rep.summary()
    if log:
        log(f"served {rate:g} req/s: {out['served']['throughput_req_s']:.1f} req/s")
    if check_identity:
        out["alone_vs_mix_mismatches"] = alone_vs_mix(rep, trace, dtype)
    if serial_baseline:
        ex1 = GpuExecutor(1, dtype, batch=False)
        try:
            Server(ex1, 1, budget_gb * GB, ex1.elem, batch=False).serve(trace)
            rep1 = Server(ex1, 1, budget_gb * GB, ex1.elem, batch=False).serve(trace)
        finally:
            ex1.close()
        out["serial_fifo"] = rep1.summary()
        s, b = out["served"], out["serial_fifo"]
        out["throughput_ratio"] = s["throughput_req_s"] / b["throughput_req_s"]
        if log:
            log(f"serial {rate:g} req/s: {b['throughput_req_s']:.1f} req/s")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--sweep", type=str, default="",
                    help="comma-separated rates; one JSON line per rate")
    ap.add_argument("--count", type=int, default=500)
    ap.add_argument("--lanes", type=int, default=2)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--n-hi", type=int, default=28)
    ap.add_argument("--small-max", type=int, default=14,
                    help="largest request (qubits) routed to the serving kernel")
    ap.add_argument("--no-serial", action="store_true")
    ap.add_argument("--no-identity", action="store_true")
    a = ap.parse_args()
    rates = [float(v) for v in a.sweep.split(",")] if a.sweep else [a.rate]
    for rate in rates:
        res = run(rate, a.count, a.lanes, a.budget_gb, a.seed, serial_baseline=not a.no_serial,
                  check_identity=not a.no_identity, n_hi=a.n_hi,
                  log=lambda m: print(m, file=sys.stderr, flush=True), small_max=a.small_max)
        print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
