"""Serving on the GPU: a Poisson stream of mixed-resolution frames through the
continuous-batching scheduler; every frame's labels in the mix equal the
frame labelled alone (tolerance 0), which equals the oracle for every frame
size at both connectivities."""
import numpy as np
import pytest

from oracle import oracle_label
from paper_1712_09789_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_serving_mix_equals_alone():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1712_09789_amd.ccl as ccl
    from paper_1712_09789_amd.serve import GpuExecutor, Request, Scheduler

    rng = np.random.default_rng(0)
    frames = []
    for H, W, _ in wl.SERVING_MIX:
        for k in range(2):
            frames.append(wl.blobs(H, W, 8, seed=100 * H + k))
    dev = [torch.from_numpy(f).cuda() for f in frames]
    alone = {}
    for i, d in enumerate(dev):
        for c in (4, 8):
            alone[(i, c)] = ccl.label(d, c).cpu().numpy()
    torch.cuda.synchronize()
    for i, f in enumerate(frames):
        for c in (4, 8):
            assert np.array_equal(alone[(i, c)], oracle_label(f, c)), (f.shape, c)

    reqs, t = [], 0.0
    for rid in range(60):
        t += rng.exponential(1.0 / 4000.0)
        i = int(rng.integers(len(frames)))
        c = int(rng.choice([4, 8]))
        H, W = frames[i].shape
        reqs.append(Request(rid=rid, image=dev[i], connectivity=c, arrival=t, H=H, W=W))
    which = {}
    for r in reqs:
        which[r.rid] = next(j for j, d in enumerate(dev) if d is r.image)
    ex = GpuExecutor(streams=3)
    sched = Scheduler(ex, slots=3, max_batch=16)
    stats = sched.run(reqs)
    torch.cuda.synchronize()
    assert stats.completed == 60 and stats.rejected == 0
    assert stats.launches >= 2
    for r in sched.done:
        got = r.labels.cpu().numpy()
        assert np.array_equal(got, alone[(which[r.rid], r.connectivity)]), r.rid
        ex.release(r.labels)
