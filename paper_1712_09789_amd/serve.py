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

import gc
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
    deadline: float | None = None   # seconds after arrival to be launched by
    status: str = "new"             # admitted / launched / done / timed_out / cancelled
    cost: int = 0                   # bytes reserved at admission
    pooled: bool = False            # admitted against a pooled label buffer

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
    timed_out: int = 0
    cancelled: int = 0
    gpx_per_s: float = field(init=False)

    def __post_init__(self):
        self.gpx_per_s = self.pixels / self.makespan_s / 1e9 if self.makespan_s > 0 else 0.0

    def as_dict(self):
        return {"completed": self.completed, "rejected": self.rejected,
                "Gpx/s": round(self.gpx_per_s, 2), "p50_ms": round(self.p50_ms, 4),
                "p99_ms": round(self.p99_ms, 4), "mean_ms": round(self.mean_ms, 4),
                "makespan_s": round(self.makespan_s, 4), "launches": self.launches,
                "mean_batch": round(self.mean_batch, 2), "max_in_flight": self.max_in_flight,
                "timed_out": self.timed_out, "cancelled": self.cancelled}


class Scheduler:
    """Admission, batching and retirement; the clock and the executor are
    injected so that the logic runs the same on and off the GPU.

    Device memory: the executor holds every byte the loop allocates — label
    buffers (handed to requests, or kept in a per-shape pool once released)
    and the library's per-stream workspaces, which only grow.  A request's
    cost is what admitting it may add: its label buffer (nothing when a
    pooled buffer of its shape is free and not promised to an earlier
    admission) plus the workspace growth its share of a batch can cause.
    Costs of admitted, not yet launched requests are pending; admission
    requires held + pending + cost <= budget and pending + cost <= the
    device's free memory, queried again at every admission.  Labels stay
    held until the caller returns them (``release``), or at retirement when
    ``keep_labels`` is False.

    Requests may carry a deadline (seconds after arrival): one still waiting
    for admission or launch at its deadline is dropped as timed out.
    ``cancel(rid)`` drops a request that has not been launched; a launched
    one finishes on the device, is marked cancelled, and its labels go back
    to the pool at retirement."""

    # free device memory is re-queried at most this often while it admits
    # (the query is a driver call); a request that the last reading would
    # refuse always gets a fresh one
    FREE_MAX_AGE_S = 0.002

    def __init__(self, executor, slots: int = 4, max_batch: int = 64,
                 budget_bytes: int | None = None, clock: Callable[[], float] = time.perf_counter,
                 keep_labels: bool = True):
        self.ex = executor
        self.slots = slots
        self.max_batch = max_batch
        self.budget = executor.free_bytes() if budget_bytes is None else budget_bytes
        self.clock = clock
        self.keep_labels = keep_labels
        self.waiting: deque[Request] = deque()   # arrived, not admitted
        self.ready: list[Request] = []            # admitted, not launched
        self.in_flight: list[tuple[Any, list[Request]]] = []
        self.pending_bytes = 0                    # costs of admitted, unlaunched requests
        self.promised: dict[tuple[int, int], int] = {}  # pooled buffers promised, by shape
        self.done: list[Request] = []
        self.rejected: list[Request] = []
        self.timed_out: list[Request] = []
        self.cancelled: list[Request] = []
        self.with_deadline = 0                    # waiting or admitted requests with a deadline
        self.launches = 0
        self.launched_reqs = 0
        self.max_in_flight = 0
        self.peak_used = 0
        self.admission_order: list[int] = []

    @property
    def used_bytes(self) -> int:
        """Device bytes held by the executor plus those promised to admitted
        requests not yet launched."""
        return self.ex.held_bytes() + self.pending_bytes

    def _cost(self, req: Request) -> tuple[int, bool]:
        """(bytes admitting req may add, whether it takes a pooled buffer)."""
        shape = (req.H, req.W)
        pooled = self.ex.pooled(shape) - self.promised.get(shape, 0) > 0
        label = 0 if pooled else self.ex.label_bytes(req)
        return label + self.ex.workspace_cost(req), pooled

    # -- steps ----------------------------------------------------------------
    def arrive(self, req: Request) -> None:
        need = self.ex.label_bytes(req) + self.ex.workspace_cost(req)
        if need > self.budget:
            req.rejected = f"needs {need} bytes, budget {self.budget}"
            self.rejected.append(req)
            return
        if req.deadline is not None:
            self.with_deadline += 1
        self.waiting.append(req)

    def _drop_labels(self, r: Request) -> None:
        if r.labels is not None:
            self.ex.release(r.labels)
            r.labels = None

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
                    if r.status == "cancelled" or not self.keep_labels:
                        self._drop_labels(r)
                    if r.status == "cancelled":
                        continue
                    r.status = "done"
                    self.done.append(r)
                n += len(reqs)
            else:
                still.append((handle, reqs))
        self.in_flight = still
        return n

    def release(self, req: Request) -> None:
        """Return a completed request's label buffer to the pool."""
        self._drop_labels(req)

    def expire(self) -> int:
        """Drop waiting or admitted requests whose deadline has passed."""
        if not self.with_deadline:
            return 0
        now = self.clock()
        late = [r for r in list(self.waiting) + self.ready
                if r.deadline is not None and now - r.arrival > r.deadline]
        for r in late:
            self._unqueue(r, "timed_out")
            self.timed_out.append(r)
        return len(late)

    def cancel(self, rid: int) -> bool:
        """Cancel a request: dropped if not yet launched, else marked so that
        its result is discarded at retirement.  False if it is unknown or
        already complete."""
        for r in list(self.waiting) + self.ready:
            if r.rid == rid:
                self._unqueue(r, "cancelled")
                self.cancelled.append(r)
                return True
        for _, reqs in self.in_flight:
            for r in reqs:
                if r.rid == rid and r.status != "cancelled":
                    r.status = "cancelled"
                    self.cancelled.append(r)
                    return True
        return False

    def _unqueue(self, r: Request, status: str) -> None:
        r.status = status
        if r.deadline is not None:
            self.with_deadline -= 1
        if r in self.waiting:
            self.waiting.remove(r)
            return
        self.ready.remove(r)
        self.pending_bytes -= r.cost
        if r.pooled:
            self.promised[(r.H, r.W)] -= 1

    def admit(self) -> int:
        """Admit waiting requests in arrival order while memory allows (the
        head of the queue blocks later arrivals: no overtaking)."""
        n = 0
        free = None
        while self.waiting:
            r = self.waiting[0]
            cost, pooled = self._cost(r)
            over = self.used_bytes + cost - self.budget
            if over > 0:
                # pooled buffers of other shapes would otherwise block the
                # queue for good: free unpromised ones to make room
                if self.ex.trim(over, self.promised) < over:
                    break
                free = None
                cost, pooled = self._cost(r)
                if self.used_bytes + cost > self.budget:
                    break
            if free is None:
                free = self.ex.free_bytes(max_age_s=self.FREE_MAX_AGE_S)
            if self.pending_bytes + cost > free:
                free = self.ex.free_bytes()
                if self.pending_bytes + cost > free:
                    break
            self.waiting.popleft()
            r.cost, r.pooled = cost, pooled
            self.pending_bytes += cost
            if pooled:
                self.promised[(r.H, r.W)] = self.promised.get((r.H, r.W), 0) + 1
            r.admitted = self.clock()
            r.status = "admitted"
            self.ready.append(r)
            self.admission_order.append(r.rid)
            n += 1
        self.peak_used = max(self.peak_used, self.used_bytes)
        return n

    def launch(self) -> int:
        """Launch the admitted requests as one batch if a slot is free."""
        if not self.ready or len(self.in_flight) >= self.slots:
            return 0
        batch, self.ready = self.ready[:self.max_batch], self.ready[self.max_batch:]
        now = self.clock()
        for r in batch:
            r.launched = now
            r.status = "launched"
            if r.deadline is not None:
                self.with_deadline -= 1
            self.pending_bytes -= r.cost
            if r.pooled:
                self.promised[(r.H, r.W)] -= 1
        handle = self.ex.launch(batch)
        self.in_flight.append((handle, batch))
        self.launches += 1
        self.launched_reqs += len(batch)
        self.max_in_flight = max(self.max_in_flight, len(self.in_flight))
        self.peak_used = max(self.peak_used, self.used_bytes)
        return len(batch)

    def idle(self) -> bool:
        return not (self.waiting or self.ready or self.in_flight)

    # -- a whole arrival trace -----------------------------------------------
    def run(self, requests: Sequence[Request],
            on_step: Callable[["Scheduler"], None] | None = None) -> ServeStats:
        """Feed requests at their arrival times (relative to the start) and
        serve until all are retired.  Returns latency and throughput.
        `on_step` (tests) is called after every scheduling step."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        # The cyclic garbage collector is paused while requests are served:
        # its full passes stopped the loop for tens of milliseconds (about 50
        # ms with a few thousand requests live), and the loop's objects are
        # freed by reference counting.
        collecting = gc.isenabled()
        gc.disable()
        try:
            return self._run(reqs, on_step)
        finally:
            if collecting:
                gc.enable()

    def _run(self, reqs: list, on_step) -> ServeStats:
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
            self.expire()
            self.admit()
            self.launch()
            if on_step is not None:
                on_step(self)
            if self.waiting and not self.ready and not self.in_flight and not self.admit():
                # nothing on the device will free memory: only the caller can
                raise RuntimeError(
                    f"admission stalled: request {self.waiting[0].rid} needs "
                    f"{self._cost(self.waiting[0])[0]} bytes, {self.used_bytes} of "
                    f"{self.budget} are held (completed requests keep their labels until "
                    "release(); use keep_labels=False to recycle them at retirement)")
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
                          mean_batch=self.launched_reqs / max(self.launches, 1),
                          timed_out=len(self.timed_out), cancelled=len(self.cancelled))


class GpuExecutor:
    """HIP path: one ccl_label_batch per launch on one of `streams` streams,
    a completion event per launch, label buffers kept resident per shape.

    Every label buffer it allocates stays allocated (handed to a request or
    pooled for the next request of that shape), so the bytes it holds are
    those buffers plus the library's workspace on each of its streams (grow
    only; read back from the library)."""

    # the library's workspace grows to 1.25 x a batch's need; a few KiB per
    # image cover the batch's image tables
    WS_GROWTH = 1.25
    WS_TABLE_SLACK = 4096

    def __init__(self, streams: int = 4, device: int = 0, reserve_frac: float = 0.05):
        import torch
        from . import ccl
        self.torch = torch
        self.ccl = ccl
        self.dev = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(streams)]
        self.next_stream = 0
        self.pool: dict[tuple[int, int], list] = {}
        self.label_bytes_held = 0
        _, total = torch.cuda.mem_get_info(self.dev)
        self.reserve = int(total * reserve_frac)
        # host-side caches: the workspace cost of each frame shape, the
        # library's workspace bytes on the streams (they change only when a
        # batch is launched), and the last free-memory reading
        self._ws_cost: dict[tuple[int, int], int] = {}
        self._ws_held = 0
        self._free = (-1.0, 0)

    def label_bytes(self, req: Request) -> int:
        return 4 * req.H * req.W

    def workspace_cost(self, req: Request) -> int:
        shape = (req.H, req.W)
        c = self._ws_cost.get(shape)
        if c is None:
            c = int(self.WS_GROWTH * self.ccl.workspace_bytes(req.H, req.W)) + self.WS_TABLE_SLACK
            self._ws_cost[shape] = c
        return c

    def pooled(self, shape) -> int:
        return len(self.pool.get(tuple(shape), ()))

    def held_bytes(self) -> int:
        return self.label_bytes_held + self._ws_held

    def free_bytes(self, max_age_s: float = 0.0) -> int:
        """Free device memory, less a reserve kept for everything else: a
        reading at most max_age_s old (0 = query now)."""
        now = time.perf_counter()
        t, val = self._free
        if max_age_s > 0 and now - t <= max_age_s:
            return val
        free, _ = self.torch.cuda.mem_get_info(self.dev)
        cached = (self.torch.cuda.memory_reserved(self.dev) -
                  self.torch.cuda.memory_allocated(self.dev))
        val = max(0, int(free) + int(cached) - self.reserve)
        self._free = (now, val)
        return val

    def _labels(self, H, W):
        lst = self.pool.get((H, W))
        if lst:
            return lst.pop()
        self.label_bytes_held += 4 * H * W
        return self.torch.empty((H, W), dtype=self.torch.int32, device=self.dev)

    def release(self, labels) -> None:
        """Return a label buffer to the resident pool."""
        self.pool.setdefault(tuple(labels.shape), []).append(labels)

    def trim(self, nbytes: int, keep: dict) -> int:
        """Drop pooled buffers (beyond keep[shape] of each shape), largest
        first, until at least nbytes are freed; returns the bytes freed.
        The memory goes back to torch's caching allocator, which the next
        label buffer can reuse (free_bytes counts it)."""
        freed = 0
        for shape in sorted(self.pool, key=lambda s: -s[0] * s[1]):
            lst = self.pool[shape]
            while freed < nbytes and len(lst) > keep.get(shape, 0):
                lst.pop()
                freed += 4 * shape[0] * shape[1]
                self.label_bytes_held -= 4 * shape[0] * shape[1]
            if freed >= nbytes:
                break
        return freed

    def launch(self, reqs):
        st = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        outs = [self._labels(r.H, r.W) for r in reqs]
        # the inputs were written on the current stream: order this stream after it
        st.wait_stream(self.torch.cuda.current_stream(self.dev))
        # one descriptor per frame: the image's pointer, size and pitch are
        # checked and read once per request, not at every launch
        descs = (self.ccl.ImageDesc * len(reqs))()
        for i, (r, o) in enumerate(zip(reqs, outs)):
            d = r.__dict__.get("_desc")
            if d is None:
                H, W, pitch = self.ccl._image_args(r.image)
                d = r.__dict__["_desc"] = (r.image.data_ptr(), H, W, pitch, int(r.connectivity))
            descs[i] = self.ccl.ImageDesc(d[0], d[1], d[2], d[3], d[4], o.data_ptr())
        self.ccl._check(self.ccl.lib().ccl_label_batch(descs, len(reqs), int(st.cuda_stream)))
        ev = self.torch.cuda.Event()
        ev.record(st)
        # the call may have grown this stream's workspace: the growth comes off
        # the cached free-memory reading (which still expires by age)
        held = sum(self.ccl.workspace_cached(s) for s in self.streams)
        t, free = self._free
        self._free = (t, max(0, free - max(0, held - self._ws_held)))
        self._ws_held = held
        return (ev, outs)

    def done(self, handle) -> bool:
        return handle[0].query()

    def results(self, handle):
        return handle[1]

    def wait_until(self, t: float, clock) -> None:
        while clock() < t:
            pass
