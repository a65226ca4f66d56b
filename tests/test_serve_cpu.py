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
    overhead + pixels * per_px seconds; labels come from the oracle."""

    def __init__(self, clock, budget, per_px=1e-9, overhead=20e-6):
        self.clock = clock
        self.budget = budget
        self.per_px = per_px
        self.overhead = overhead
        self.device_free = 0.0
        self.in_use = 0
        self.peak_in_use = 0

    def footprint(self, req):
        return req.H * req.W * 5

    def free_bytes(self):
        return self.budget

    def launch(self, reqs):
        now = self.clock()
        start = max(now, self.device_free)
        finish = start + self.overhead + sum(r.H * r.W for r in reqs) * self.per_px
        self.device_free = finish
        self.in_use += sum(self.footprint(r) for r in reqs)
        self.peak_in_use = max(self.peak_in_use, self.in_use)
        labels = [oracle_label(r.image, r.connectivity) for r in reqs]
        return {"finish": finish, "labels": labels, "bytes": sum(self.footprint(r) for r in reqs),
                "retired": False}

    def done(self, h):
        ok = self.clock() >= h["finish"]
        if ok and not h["retired"]:
            h["retired"] = True
            self.in_use -= h["bytes"]
        return ok

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
    per_req = 64 * 64 * 5
    ex = FakeExecutor(clock, budget=2 * per_req, per_px=1e-6)
    sched = Scheduler(ex, slots=4, max_batch=8, clock=clock)
    reqs = make_requests(30, seed=1, rate=1e6, sizes=sizes)  # a burst
    stats = sched.run(reqs)
    assert stats.completed == 30
    # never more than the budget admitted at once, so never more than 2 in flight
    assert ex.peak_in_use <= 2 * per_req
    assert sched.used_bytes == 0


def test_oversize_request_is_rejected():
    clock = VirtualClock()
    ex = FakeExecutor(clock, budget=40 * 40 * 5)
    sched = Scheduler(ex, slots=2, clock=clock)
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
