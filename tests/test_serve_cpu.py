"""The serving scheduler on the CPU: a fake executor (labels from the oracle,
completion after a simulated duration on a virtual clock) checks admission
order, slot accounting, memory back-pressure, rejection and the latency
statistics without a GPU."""
import numpy as np
import pytest

from oracle import oracle_label
from paper_1712_09789_amd import workloads as wl
from paper_1712_09789_amd.serve import Request, Scheduler, percentile


class VirtualClock:
    """Advances a little on every read, like a polling loop burning time."""

    def __init__(self, step=1e-6):
        self.t = 0.0
        self.step = step

    def __call__(self):
        self.t += self.step
        return self.t


class FakeExecutor:
    """One simulated device: launches run back to back, each taking
    overhead + pixels * per_px seconds; labels come from the oracle.

    Memory is modelled like the GPU executor's: label buffers are allocated
    once and then pooled per shape, and each of `streams` streams keeps a
    grow-only workspace of 1.25 x the largest batch need it has seen
    (`ws_per_px` bytes per pixel).  `allocated` is the exact byte count of
    both, and `device_total` bounds it like a device would."""

    def __init__(self, clock, budget, per_px=1e-9, overhead=20e-6, streams=2, ws_per_px=0.0,
                 device_total=None):
        self.clock = clock
        self.budget = budget
        self.per_px = per_px
        self.overhead = overhead
        self.device_free = 0.0
        self.streams = streams
        self.next_stream = 0
        self.ws_per_px = ws_per_px
        self.ws = [0] * streams
        self.pool = {}
        self.label_alloc = 0
        self.device_total = device_total if device_total is not None else budget
        self.peak_alloc = 0

    # memory model ------------------------------------------------------------
    def label_bytes(self, req):
        return 4 * req.H * req.W

    def workspace_cost(self, req):
        return int(1.25 * self.ws_per_px * req.H * req.W)

    def pooled(self, shape):
        return len(self.pool.get(tuple(shape), ()))

    @property
    def allocated(self):
        return self.label_alloc + sum(self.ws)

    def held_bytes(self):
        return self.allocated

    def free_bytes(self, max_age_s=0.0):
        return self.device_total - self.allocated

    def release(self, labels):
        self.pool.setdefault(labels.shape, []).append(labels)

    def trim(self, nbytes, keep):
        freed = 0
        for shape in sorted(self.pool, key=lambda s: -s[0] * s[1]):
            lst = self.pool[shape]
            while freed < nbytes and len(lst) > keep.get(shape, 0):
                lst.pop()
                freed += 4 * shape[0] * shape[1]
                self.label_alloc -= 4 * shape[0] * shape[1]
        return freed

    def _labels(self, H, W):
        lst = self.pool.get((H, W))
        if lst:
            return lst.pop()
        self.label_alloc += 4 * H * W
        return np.empty((H, W), np.int32)

    # execution ---------------------------------------------------------------
    def launch(self, reqs):
        now = self.clock()
        start = max(now, self.device_free)
        finish = start + self.overhead + sum(r.H * r.W for r in reqs) * self.per_px
        self.device_free = finish
        st = self.next_stream
        self.next_stream = (st + 1) % self.streams
        need = int(self.ws_per_px * sum(r.H * r.W for r in reqs))
        if need > self.ws[st]:
            self.ws[st] = int(1.25 * need)
        outs = []
        for r in reqs:
            buf = self._labels(r.H, r.W)
            buf[...] = oracle_label(r.image, r.connectivity)
            outs.append(buf)
        self.peak_alloc = max(self.peak_alloc, self.allocated)
        assert self.allocated <= self.device_total, "device memory exceeded"
        return {"finish": finish, "labels": outs}

    def done(self, h):
        return self.clock() >= h["finish"]

    def results(self, h):
        return h["labels"]

    def wait_until(self, t, clock):
        clock.t = max(clock.t, t)

def make_requests(n, seed=0, rate=2000.0, sizes=((20, 30), (40, 50), (64, 70))):
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        H, W = sizes[int(rng.integers(len(sizes)))]
        img = wl.bernoulli(H, W, float(rng.uniform(0.3, 0.7)), seed=seed * 1000 + i)
        reqs.append(Request(rid=i, image=img, connectivity=int(rng.choice([4, 8])),
                            arrival=t, H=H, W=W))
    return reqs


def test_all_served_fifo_and_correct():
    clock = VirtualClock()
    ex = FakeExecutor(clock, budget=10**9)
    sched = Scheduler(ex, slots=3, max_batch=8, clock=clock)
    reqs = make_requests(80)
    stats = sched.run(reqs)
    assert stats.completed == 80 and stats.rejected == 0
    assert sched.admission_order == sorted(sched.admission_order)  # arrival order
    assert sched.max_in_flight <= 3
    for r in sched.done:
        assert r.completed >= r.launched >= r.admitted >= r.arrival
        # each request gets the labels of its own image
        assert np.array_equal(r.labels, oracle_label(r.image, r.connectivity))


def test_memory_back_pressure():
    clock = VirtualClock()
    sizes = ((64, 64),)
    per_req = 64 * 64 * 4
    ex = FakeExecutor(clock, budget=2 * per_req, per_px=1e-6)
    sched = Scheduler(ex, slots=4, max_batch=8, clock=clock, keep_labels=False)
    reqs = make_requests(30, seed=1, rate=1e6, sizes=sizes)  # a burst
    stats = sched.run(reqs)
    assert stats.completed == 30
    # never more than two label buffers: the budget holds two, and retired
    # buffers are reused from the pool
    assert ex.peak_alloc <= 2 * per_req
    assert sched.peak_used <= 2 * per_req
    assert sched.pending_bytes == 0 and sched.used_bytes == ex.allocated


def test_ledger_matches_allocations_over_a_long_trace():
    """A long mixed-resolution trace with per-stream workspaces, releases of
    completed labels at random times and a tight budget: after every
    scheduling step the scheduler's account (held + pending) is the
    executor's real allocation plus what admitted requests may still add,
    it never exceeds the budget, and the device never runs out."""
    clock = VirtualClock()
    sizes = ((20, 30), (40, 50), (64, 70), (96, 128))
    budget = 300_000
    ex = FakeExecutor(clock, budget=budget, per_px=2e-7, streams=3, ws_per_px=1.5,
                      device_total=budget + 50_000)
    sched = Scheduler(ex, slots=3, max_batch=6, clock=clock, budget_bytes=budget)
    rng = np.random.default_rng(7)
    held_by_requests = []
    checks = [0]

    def on_step(s):
        # the caller returns some completed labels late, some never
        for r in s.done[len(held_by_requests):]:
            held_by_requests.append(r)
        for r in held_by_requests:
            if r.labels is not None and rng.random() < 0.2:
                s.release(r)
        launched_cost = sum(r.cost for r in s.ready)
        assert s.pending_bytes == launched_cost
        assert s.used_bytes == ex.allocated + s.pending_bytes
        assert s.used_bytes <= budget
        checks[0] += 1

    stats = sched.run(make_requests(400, seed=5, rate=3e4, sizes=sizes), on_step=on_step)
    assert stats.completed == 400 and stats.rejected == 0
    assert checks[0] > 400
    assert ex.peak_alloc <= budget
    assert sched.pending_bytes == 0 and sched.used_bytes == ex.allocated
    for r in sched.done:
        if r.labels is not None:
            assert np.array_equal(r.labels, oracle_label(r.image, r.connectivity))


def test_deadline_drops_requests_that_wait_too_long():
    clock = VirtualClock()
    ex = FakeExecutor(clock, budget=10**9, per_px=1e-5)  # a slow device
    sched = Scheduler(ex, slots=1, max_batch=2, clock=clock)
    reqs = make_requests(40, seed=8, rate=1e6, sizes=((64, 64),))
    for r in reqs:
        r.deadline = 2e-3
    stats = sched.run(reqs)
    assert stats.timed_out > 0
    assert stats.completed + stats.timed_out == 40
    for r in sched.timed_out:
        assert r.status == "timed_out" and r.labels is None
        assert r.launched != r.launched  # never launched (NaN)
    for r in sched.done:
        assert r.launched - r.arrival <= 2e-3 + 1e-4


def test_cancel_waiting_and_launched_requests():
    clock = VirtualClock()
    ex = FakeExecutor(clock, budget=10**9, per_px=1e-6)
    sched = Scheduler(ex, slots=1, max_batch=4, clock=clock)
    reqs = make_requests(12, seed=9, rate=1e6, sizes=((32, 32),))
    t0 = clock()
    for r in reqs:
        r.arrival += t0
        sched.arrive(r)
    sched.admit()
    sched.launch()                      # first four on the device
    assert sched.cancel(reqs[1].rid)    # launched: finishes, result discarded
    assert sched.cancel(reqs[6].rid)    # admitted, not launched
    assert sched.cancel(reqs[11].rid)   # admitted, not launched
    assert not sched.cancel(999)
    while not sched.idle():
        sched.retire()
        sched.admit()
        sched.launch()
    done = {r.rid for r in sched.done}
    assert done == set(range(12)) - {1, 6, 11}
    assert all(r.status == "cancelled" for r in sched.cancelled)
    # the cancelled request's buffer went back to the pool and was reused:
    # nine results held by their requests, nine buffers ever allocated
    assert reqs[1].labels is None
    assert ex.label_alloc == 9 * 32 * 32 * 4
    assert sched.pending_bytes == 0


def test_oversize_request_is_rejected():
    clock = VirtualClock()
    ex = FakeExecutor(clock, budget=40 * 40 * 4)
    sched = Scheduler(ex, slots=2, clock=clock, keep_labels=False)
    reqs = make_requests(20, seed=2, sizes=((20, 30), (64, 70)))
    stats = sched.run(reqs)
    big = [r for r in reqs if r.H * r.W > 1600]
    assert stats.rejected == len(big) > 0
    assert stats.completed == 20 - len(big)
    assert all(r.rejected for r in sched.rejected)


def test_batches_form_while_busy():
    # a slow device and a single slot: later arrivals accumulate and ride
    # together in the next launch (continuous batching)
    clock = VirtualClock()
    ex = FakeExecutor(clock, budget=10**9, per_px=1e-6)
    sched = Scheduler(ex, slots=1, max_batch=64, clock=clock)
    stats = sched.run(make_requests(60, seed=3, rate=5e4))
    assert stats.completed == 60
    assert stats.mean_batch > 2.0
    assert stats.launches < 60


@pytest.mark.parametrize("q", [0, 1, 37.5, 50, 99, 100])
def test_percentile_matches_numpy(q):
    rng = np.random.default_rng(int(q * 10))
    v = list(rng.exponential(size=101))
    assert percentile(v, q) == pytest.approx(float(np.percentile(v, q)))
    assert np.isnan(percentile([], 50))


def test_stats_arithmetic():
    clock = VirtualClock()
    ex = FakeExecutor(clock, budget=10**9)
    sched = Scheduler(ex, slots=2, clock=clock)
    stats = sched.run(make_requests(25, seed=4))
    lat = [1e3 * r.latency for r in sched.done]
    assert stats.p50_ms == pytest.approx(float(np.percentile(lat, 50)))
    assert stats.p99_ms == pytest.approx(float(np.percentile(lat, 99)))
    assert stats.pixels == sum(r.H * r.W for r in sched.done)
    assert stats.gpx_per_s == pytest.approx(stats.pixels / stats.makespan_s / 1e9)


def test_stall_is_reported_not_spun():
    """Completed requests keep their labels until released; when they fill
    the budget and the caller never releases them, run() raises instead of
    waiting forever."""
    clock = VirtualClock()
    ex = FakeExecutor(clock, budget=3 * 32 * 32 * 4)
    sched = Scheduler(ex, slots=2, clock=clock)
    with pytest.raises(RuntimeError, match="admission stalled"):
        sched.run(make_requests(10, seed=10, sizes=((32, 32),)))
    assert len(sched.done) == 3


def test_collector_paused_while_serving_and_restored():
    """The cyclic garbage collector is off while run() serves (its full
    passes stalled the loop) and back on afterwards, also when run() raises."""
    import gc
    assert gc.isenabled()
    clock = VirtualClock()
    ex = FakeExecutor(clock, budget=10**9)
    sched = Scheduler(ex, slots=2, max_batch=4, clock=clock)
    seen = []
    sched.run(make_requests(12, seed=3), on_step=lambda s: seen.append(gc.isenabled()))
    assert seen and not any(seen)
    assert gc.isenabled()
    ex = FakeExecutor(clock, budget=3 * 32 * 32 * 4)
    sched = Scheduler(ex, slots=2, clock=clock)
    with pytest.raises(RuntimeError, match="admission stalled"):
        sched.run(make_requests(10, seed=10, sizes=((32, 32),)))
    assert gc.isenabled()
