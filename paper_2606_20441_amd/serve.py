"""Continuous-batching request loop for noise-canceling propagations on one GPU.

A request is a whole propagation O -> O~ = D O (a circuit, an observable, a threshold, a
cap and a coefficient precision), answered with <0|O~|0>.  Requests arrive over time.

- Admission.  The scheduler admits the oldest waiting request as soon as a slot is free
  and its device-memory reservation fits in what is left of the HBM budget.  A request
  whose reservation exceeds the whole budget is rejected at arrival.
- Overlap.  Every slot owns a HIP stream and a library context, driven by its own host
  thread.  The library releases the interpreter lock inside its calls, so the propagations
  of all admitted requests run concurrently on the device.  A request that arrives while
  others are running starts as soon as a slot and memory free up.  It does not wait for a
  batch to drain.
- Residency.  A request's term arrays stay on the device from creation to its
  expectation value; only the scalar result and the term count come back to the host.
- Enforcement.  A slot's context refuses device allocations beyond the request's
  reservation, so a request that outgrows it fails alone, with PP_ERR_OOM, and its
  memory returns to the budget.

The kernels of the greedy mode are deterministic and a request's arithmetic does not
depend on what else runs, so a request's result is the same alone and in a mix.

`Scheduler` holds the admission logic and does no device work, so tests can drive it on
the CPU.  `Server` runs a request stream against the wall clock with a device executor,
or with any callable given as `executor`.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple

import numpy as np

DEFAULT_CAP = 1 << 22


def term_bytes(n_qubits: int, precision: str, mode: str) -> int:
    """Bytes of one term in HBM: x and z planes, the coefficient, the order tag."""
    w = (n_qubits + 63) // 64
    return 16 * w + (8 if precision == "f64" else 4) + (1 if mode == "error_order" else 0)


def reservation_bytes(wl, factor: float = 32.0, floor: int = 1 << 30) -> int:
    """Device bytes reserved for a request.

    The observable holds a current and an output array (each up to twice the capped size
    between the gates of a run), per-term hashes and tile tables, sort buffers and the
    first guess of a fused pass's output.  The reservation is `factor` arrays of the
    capped size, and at least `floor`.
    """
    cap = wl.max_terms if wl.max_terms > 0 else DEFAULT_CAP
    b = term_bytes(wl.circuit.n_qubits, wl.precision, wl.mode)
    return int(max(floor, factor * cap * b))


@dataclass
class RequestResult:
    rid: int
    arrival: float                       # seconds since the stream started
    status: str = "waiting"              # ok | rejected | oom | error
    admitted: float = float("nan")
    finished: float = float("nan")
    slot: int = -1
    expectation: Optional[float] = None
    n_terms: int = 0
    term_updates: int = 0
    reserved_bytes: int = 0
    peak_bytes: int = 0
    message: str = ""

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    @property
    def queue_wait(self) -> float:
        return self.admitted - self.arrival


class Scheduler:
    """FIFO admission by free slot and HBM budget (host bookkeeping only)."""

    def __init__(self, n_slots: int, budget_bytes: int, reserve: Callable = reservation_bytes):
        if n_slots <= 0:
            raise ValueError("n_slots must be positive")
        self.n_slots = n_slots
        self.budget = int(budget_bytes)
        self.reserve = reserve
        self.reserved = 0
        self.free_slots: List[int] = list(range(n_slots))[::-1]
        self.waiting: Deque[Tuple[object, int]] = collections.deque()
        self.peak_reserved = 0
        self.peak_running = 0

    def offer(self, req) -> Optional[str]:
        """Queue an arrived request; returns "rejected" if it can never fit."""
        need = int(self.reserve(req.workload))
        if need > self.budget:
            return "rejected"
        self.waiting.append((req, need))
        return None

    def admit(self) -> List[Tuple[int, object, int]]:
        """Admit waiting requests in arrival order while a slot and memory are free."""
        out = []
        while self.waiting and self.free_slots:
            req, need = self.waiting[0]
            if self.reserved + need > self.budget:
                break   # head-of-line waits for memory; later arrivals do not overtake it
            self.waiting.popleft()
            slot = self.free_slots.pop()
            self.reserved += need
            self.peak_reserved = max(self.peak_reserved, self.reserved)
            out.append((slot, req, need))
        self.peak_running = max(self.peak_running, self.n_slots - len(self.free_slots))
        return out

    def release(self, slot: int, need: int) -> None:
        self.reserved -= need
        self.free_slots.append(slot)

    @property
    def running(self) -> int:
        return self.n_slots - len(self.free_slots)


class DeviceExecutor:
    """One HIP stream and one library context per slot."""

    def __init__(self, n_slots: int, device: int = 0):
        import torch
        from . import pp
        self.pp = pp
        pp.lib()
        self.streams = [torch.cuda.Stream(device) for _ in range(n_slots)]
        self.ctxs = [pp.Context(device, stream=s) for s in self.streams]

    def __call__(self, slot: int, req, reserved: int, res: RequestResult) -> None:
        pp = self.pp
        ctx = self.ctxs[slot]
        ctx.limit_bytes = reserved
        ctx.peak_bytes = ctx.live_bytes
        upd = [0]

        def on_layer(step, phase, m, obs):
            upd[0] += obs.last_layer_stats()["n_in"]

        wl = req.workload
        obs = None
        try:
            obs = pp.run_workload(ctx, wl, on_layer=on_layer)
            res.expectation = obs.expectation()
            res.n_terms = len(obs)
            res.status = "ok"
        except pp.PPError as e:
            res.status = "oom" if e.status == pp.PP_ERR_OOM else "error"
            res.message = str(e)
        finally:
            if obs is not None:
                obs.destroy()
        res.term_updates = upd[0]
        res.peak_bytes = ctx.peak_bytes

    def close(self):
        for c in self.ctxs:
            c.close()


class Server:
    """Replays a request stream against the wall clock (arrival times in seconds)."""

    def __init__(self, n_slots: int = 8, hbm_budget_bytes: int = 200 * 10**9,
                 executor: Optional[Callable] = None, device: int = 0,
                 reserve: Callable = reservation_bytes):
        self.n_slots = n_slots
        self.sched = Scheduler(n_slots, hbm_budget_bytes, reserve)
        self.executor = executor if executor is not None else DeviceExecutor(n_slots, device)
        self._cv = threading.Condition()
        self._done: List[Tuple[int, int, RequestResult]] = []

    def _worker(self, slot: int, inbox: "collections.deque", t0: float):
        while True:
            with self._cv:
                while not inbox:
                    self._cv.wait()
                item = inbox.popleft()
            if item is None:
                return
            req, need, res = item
            try:
                self.executor(slot, req, need, res)
            except Exception as e:   # a failed request must not stall the loop
                res.status = "error"
                res.message = repr(e)
            res.finished = time.perf_counter() - t0
            with self._cv:
                self._done.append((slot, need, res))
                self._cv.notify_all()

    def run(self, requests: Sequence, time_scale: float = 1.0,
            on_done: Optional[Callable[[RequestResult], None]] = None) -> List[RequestResult]:
        """Serve `requests` (objects with `rid`, `arrival_s`, `workload`), arrivals scaled
        by `time_scale`; returns one result per request in arrival order.  `on_done` is
        called (on the dispatching thread) with each finished request."""
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        results: Dict[int, RequestResult] = {}
        inboxes = [collections.deque() for _ in range(self.n_slots)]
        t0 = time.perf_counter()
        threads = [threading.Thread(target=self._worker, args=(s, inboxes[s], t0), daemon=True)
                   for s in range(self.n_slots)]
        for t in threads:
            t.start()
        i = 0
        pending = len(reqs)
        try:
            while pending:
                now = time.perf_counter() - t0
                with self._cv:
                    while self._done:
                        slot, need, res = self._done.pop()
                        self.sched.release(slot, need)
                        pending -= 1
                        if on_done:
                            on_done(res)
                    while i < len(reqs) and reqs[i].arrival_s * time_scale <= now:
                        r = reqs[i]
                        res = RequestResult(r.rid, r.arrival_s * time_scale)
                        results[r.rid] = res
                        if self.sched.offer(r) == "rejected":
                            res.status = "rejected"
                            res.finished = now
                            pending -= 1
                        i += 1
                    for slot, r, need in self.sched.admit():
                        res = results[r.rid]
                        res.admitted = time.perf_counter() - t0
                        res.slot = slot
                        res.reserved_bytes = need
                        inboxes[slot].append((r, need, res))
                    self._cv.notify_all()
                    if not pending:
                        break
                    wait = reqs[i].arrival_s * time_scale - (time.perf_counter() - t0) if i < len(reqs) else 1.0
                    if wait > 0 and not self._done:
                        self._cv.wait(timeout=min(wait, 1.0))
        finally:
            with self._cv:
                for box in inboxes:
                    box.append(None)
                self._cv.notify_all()
            for t in threads:
                t.join()
        return [results[r.rid] for r in reqs]

    def close(self):
        if hasattr(self.executor, "close"):
            self.executor.close()


def summarize(results: Sequence[RequestResult], offered_rate: float) -> dict:
    """p50/p99 latency of answered requests, throughput and offered vs achieved load."""
    ok = [r for r in results if r.status == "ok"]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(0)
    waits = np.array([r.queue_wait for r in ok]) if ok else np.zeros(0)
    if ok:
        first = min(r.arrival for r in results)
        makespan = max(r.finished for r in ok) - first
    else:
        makespan = float("nan")
    upd = sum(r.term_updates for r in ok)
    return {
        "requests": len(results),
        "ok": len(ok),
        "rejected": sum(r.status == "rejected" for r in results),
        "oom": sum(r.status == "oom" for r in results),
        "error": sum(r.status == "error" for r in results),
        "offered_rate_per_s": offered_rate,
        "achieved_rate_per_s": len(ok) / makespan if ok and makespan > 0 else 0.0,
        "p50_latency_ms": float(np.percentile(lat, 50) * 1e3) if ok else None,
        "p99_latency_ms": float(np.percentile(lat, 99) * 1e3) if ok else None,
        "mean_queue_wait_ms": float(waits.mean() * 1e3) if ok else None,
        "term_updates_per_s": upd / makespan if ok and makespan > 0 else 0.0,
        "makespan_s": makespan,
    }
