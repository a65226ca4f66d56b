"""Continuous-batching request loop over the C ABI.

Requests (one image each) arrive over time.  The scheduler admits them in
arrival order while a slot is free and their device memory fits the budget,
launches everything admitted since the last launch as ONE batch
(``ccl_label_batch``) on one of several streams — so requests that arrive
while earlier batches are still on the GPU join the next launch and overlap
with them — and retires a batch when its completion event has passed.
Latency of a request = time its labels are known complete - its arrival.

The executor is pluggable: ``GpuExecutor`` runs the HIP path; tests drive the
same scheduler with an executor that computes on the CPU, to check admission
order, slot accounting, memory back-pressure and the latency statistics
without a GPU.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Any, Callable, Sequence


@dataclass
class Request:
    rid: int
    image: Any                 # device tensor (GPU executor) or array
    connectivity: int
    arrival: float             # seconds, scheduler clock
    H: int = 0
    W: int = 0
    admitted: float = math.nan
    launched: float = math.nan
    completed: float = math.nan
    labels: Any = None
    rejected: str = ""

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


def percentile(values: Sequence[float], q: float) -> float:
    """Linear-interpolated percentile (numpy's default method)."""
    if not values:
        return math.nan
    v = sorted(values)
    pos = (len(v) - 1) * q / 100.0
    lo = math.floor(pos)
    hi = min(lo + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (pos - lo)


@dataclass
class ServeStats:
    completed: int
    rejected: int
    pixels: int
    makespan_s: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    max_in_flight: int
    launches: int
    mean_batch: float
    gpx_per_s: float = field(init=False)

    def __post_init__(self):
        self.gpx_per_s = self.pixels / self.makespan_s / 1e9 if self.makespan_s > 0 else 0.0

    def as_dict(self):
        return {"completed": self.completed, "rejected": self.rejected,
                "Gpx/s": round(self.gpx_per_s, 2), "p50_ms": round(self.p50_ms, 4),
                "p99_ms": round(self.p99_ms, 4), "mean_ms": round(self.mean_ms, 4),
                "makespan_s": round(self.makespan_s, 4), "launches": self.launches,
                "mean_batch": round(self.mean_batch, 2), "max_in_flight": self.max_in_flight}


class Scheduler:
    """Admission, batching and retirement; the clock and the executor are
    injected so that the logic runs the same on and off the GPU."""

    def __init__(self, executor, slots: int = 4, max_batch: int = 64,
                 budget_bytes: int | None = None, clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.slots = slots
        self.max_batch = max_batch
        self.budget = executor.free_bytes() if budget_bytes is None else budget_bytes
        self.clock = clock
        self.waiting: deque[Request] = deque()   # arrived, not admitted
        self.ready: list[Request] = []            # admitted, not launched
        self.in_flight: list[tuple[Any, list[Request]]] = []
        self.used_bytes = 0
        self.done: list[Request] = []
        self.rejected: list[Request] = []
        self.launches = 0
        self.launched_reqs = 0
        self.max_in_flight = 0
        self.admission_order: list[int] = []

    # -- steps ----------------------------------------------------------------
    def arrive(self, req: Request) -> None:
        need = self.ex.footprint(req)
        if need > self.budget:
            req.rejected = f"needs {need} bytes, budget {self.budget}"
            self.rejected.append(req)
            return
        self.waiting.append(req)

    def retire(self) -> int:
        """Retire every launched batch whose work has completed."""
        n = 0
        still = []
        for handle, reqs in self.in_flight:
            if self.ex.done(handle):
                now = self.clock()
                for r, lab in zip(reqs, self.ex.results(handle)):
                    r.completed = now
                    r.labels = lab
                    self.used_bytes -= self.ex.footprint(r)
                    self.done.append(r)
                n += len(reqs)
            else:
                still.append((handle, reqs))
        self.in_flight = still
        return n

    def admit(self) -> int:
        """Admit waiting requests in arrival order while memory allows (the
        head of the queue blocks later arrivals: no overtaking)."""
        n = 0
        while self.waiting:
            r = self.waiting[0]
            need = self.ex.footprint(r)
            if self.used_bytes + need > self.budget:
                break
            self.waiting.popleft()
            self.used_bytes += need
            r.admitted = self.clock()
            self.ready.append(r)
            self.admission_order.append(r.rid)
            n += 1
        return n

    def launch(self) -> int:
        """Launch the admitted requests as one batch if a slot is free."""
        if not self.ready or len(self.in_flight) >= self.slots:
            return 0
        batch, self.ready = self.ready[:self.max_batch], self.ready[self.max_batch:]
        now = self.clock()
        for r in batch:
            r.launched = now
        handle = self.ex.launch(batch)
        self.in_flight.append((handle, batch))
        self.launches += 1
        self.launched_reqs += len(batch)
        self.max_in_flight = max(self.max_in_flight, len(self.in_flight))
        return len(batch)

    def idle(self) -> bool:
        return not (self.waiting or self.ready or self.in_flight)

    # -- a whole arrival trace -----------------------------------------------
    def run(self, requests: Sequence[Request]) -> ServeStats:
        """Feed requests at their arrival times (relative to the start) and
        serve until all are retired.  Returns latency and throughput."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock()
        for r in reqs:
            r.arrival += t0
        i = 0
        while i < len(reqs) or not self.idle():
            now = self.clock()
            while i < len(reqs) and reqs[i].arrival <= now:
                self.arrive(reqs[i])
                i += 1
            self.retire()
            self.admit()
            self.launch()
            if i < len(reqs) and self.idle():
                self.ex.wait_until(reqs[i].arrival, self.clock)
        return self.stats()

    def stats(self) -> ServeStats:
        lat = [1e3 * r.latency for r in self.done]
        first = min((r.arrival for r in self.done), default=0.0)
        last = max((r.completed for r in self.done), default=0.0)
        px = sum(r.H * r.W for r in self.done)
        return ServeStats(completed=len(self.done), rejected=len(self.rejected), pixels=px,
                          makespan_s=last - first, p50_ms=percentile(lat, 50),
                          p99_ms=percentile(lat, 99),
                          mean_ms=sum(lat) / len(lat) if lat else math.nan,
                          max_in_flight=self.max_in_flight, launches=self.launches,
                          mean_batch=self.launched_reqs / max(self.launches, 1))


class GpuExecutor:
    """HIP path: one ccl_label_batch per launch on one of `streams` streams,
    a completion event per launch, label buffers kept resident per shape."""

    def __init__(self, streams: int = 4, device: int = 0):
        import torch
        from . import ccl
        self.torch = torch
        self.ccl = ccl
        self.dev = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(streams)]
        self.next_stream = 0
        self.pool: dict[tuple[int, int], list] = {}

    def footprint(self, req: Request) -> int:
        # input + labels + the library's workspace for this frame
        return req.H * req.W * 5 + self.ccl.workspace_bytes(req.H, req.W)

    def free_bytes(self) -> int:
        free, _ = self.torch.cuda.mem_get_info(self.dev)
        return int(free * 0.8)

    def _labels(self, H, W):
        lst = self.pool.get((H, W))
        if lst:
            return lst.pop()
        return self.torch.empty((H, W), dtype=self.torch.int32, device=self.dev)

    def release(self, labels) -> None:
        """Return a label buffer to the resident pool."""
        self.pool.setdefault(tuple(labels.shape), []).append(labels)

    def launch(self, reqs):
        st = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        outs = [self._labels(r.H, r.W) for r in reqs]
        # the inputs were written on the current stream: order this stream after it
        st.wait_stream(self.torch.cuda.current_stream(self.dev))
        self.ccl.label_batch([r.image for r in reqs], [r.connectivity for r in reqs],
                             outs=outs, stream=st)
        ev = self.torch.cuda.Event()
        ev.record(st)
        return (ev, outs)

    def done(self, handle) -> bool:
        return handle[0].query()

    def results(self, handle):
        return handle[1]

    def wait_until(self, t: float, clock) -> None:
        while clock() < t:
            pass
