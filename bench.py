"""Benchmark: connected-components labelling throughput on one MI355X.

Headline workload: single 4096 x 4096 uint8 images, the 7 contents of the
single-image sweep (Bernoulli foreground at p = 0.1/0.3/0.5/0.7/0.9, blobs =
smoothed uniform noise thresholded at the median with sigma 4/16) under 4- and
8-connectivity: 14 images, each with its own input and label buffers, visited
in rotation so that successive steps do not find their data in the 256 MB
Infinity Cache.  A step labels one image (all four kernels).  Inputs are
resident in HBM before timing starts; host<->device copies are not timed.
Besides the aggregate rate over the timed steps, the per-step median, minimum
and 99th percentile (events between steps) and the rate of the library's copy
kernel (the achievable HBM bandwidth of the device) are reported.

The result is only reported as exact if every image's labels equal the CPU
oracle's (element-by-element, after a warm-up run), which is also timed on
one host core as the CPU baseline.

Also reported (secondary): the 8192 x 8192 images (Bernoulli p = 0.5 and the
adversarial spiral / serpentine / checkerboard / full set), as path
throughput and fraction of the 8 TB/s HBM peak; a batch of 256 mixed-size
images (one batched call against per-image calls, and the oracle on every
host core); the serving loop at saturation and at half and 0.8 of it.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
PATH_BYTES_PER_PX = 5.0        # 1 B read + 4 B written: the minimum for the path
# algorithmic HBM bytes per pixel of each kernel: what it must move at least
KERNEL_BYTES_PER_PX = {
    "local": 1.0 + 1.0 / 8.0,   # image read + foreground bitmask write
    "final": 4.0 + 1.0 / 8.0,   # label write + bitmask read
}
KERNEL_NAMES = {"local": "k_local", "block": "k_block", "seam": "k_seam", "final": "k_final"}
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_bench_4096.md")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("ccl_kernels.hip", "ccl_kernels.h"):
        with open(os.path.join(ROOT, "paper_1712_09789_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def headline_cases(size):
    from paper_1712_09789_amd import workloads as wl
    cases = []
    for kind, kw in wl.single_image_contents():
        img = wl.make(kind, size, size, seed=0, **kw)
        for conn in (4, 8):
            cases.append((f"{kind}{kw}", img, conn))
    return cases


def time_rotation(ccl, torch, devs, steps, warmup, timing=None):
    """Label devs[i % n] for `steps` steps; returns (seconds, per-kernel dict).
    `timing` lists the kernel kinds to bracket with HIP events (None: none)."""
    st = torch.cuda.current_stream()
    n = len(devs)
    for i in range(warmup):
        img, out, conn = devs[i % n]
        ccl.label(img, conn, out=out)
    torch.cuda.synchronize()
    if timing:
        ccl.timing_enable(True, kinds=timing)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for i in range(steps):
        img, out, conn = devs[i % n]
        ccl.label(img, conn, out=out)
    e1.record(st)
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1e3
    kern = None
    if timing:
        kern = ccl.timing_read()
        ccl.timing_enable(False)
    return secs, kern


def read_profile_fields(path):
    """`key: value` lines of a profile summary."""
    out = {}
    try:
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith(("#", "|", " ", "`")):
                    k, v = line.split(":", 1)
                    out[k.strip()] = v.strip()
    except OSError:
        pass
    return out


def load_traffic(src_hash, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    runs, only if they were taken on the current kernel source."""
    rec = read_profile_fields(PROFILE_TRAFFIC)
    key = f"{kernel}_bytes_per_launch"
    if rec.get("kernel_source_hash") != src_hash or key not in rec:
        return None
    return float(rec[key])


def _short_kernel(name):
    import re
    m = re.search(r"ccl::(?:(r\d+)::)?(k_\w+)(<[^>(]*>)?", name)
    if not m:
        return name[:48]
    shape = f" ({m.group(1)})" if m.group(1) else ""  # tile-height build of the kernel
    return m.group(2) + (m.group(3) or "") + shape


def summarize_trace(db, out, cmd):
    """Kernel-trace database -> markdown table of per-kernel durations."""
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), avg(duration), min(duration), max(duration), "
                       "sum(duration) from kernels group by name").fetchall()
    rows = sorted(rows, key=lambda r: -r[5])
    lines = ["# Kernel trace: " + os.path.basename(out).rsplit(".", 1)[0], "",
             "Produced by:", "", "```", cmd, "```", "",
             f"kernel_source_hash: {kernel_source_hash()}", "",
             "| kernel | launches | avg us | min us | max us | total ms |",
             "|---|---|---|---|---|---|"]
    for name, n, avg, mn, mx, tot in rows:
        lines.append(f"| {_short_kernel(name)} | {n} | {avg / 1e3:.2f} | {mn / 1e3:.2f} | "
                     f"{mx / 1e3:.2f} | {tot / 1e6:.3f} |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarize_counters(db, out, cmd, px=4096 * 4096):
    """Counter database (one rocprofv3 --pmc run) -> markdown table of each
    counter's mean per dispatch, per kernel, and per pixel of a launch."""
    import collections
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, counter_name, dispatch_id, sum(value) from "
                       "counters_collection group by dispatch_id, counter_name").fetchall()
    agg = collections.defaultdict(list)
    for name, counter, _, v in rows:
        agg[(_short_kernel(name), counter)].append(v)
    counters = sorted({c for _, c in agg})
    kernels = sorted({k for k, _ in agg if k.startswith("k_") and not k.startswith("k_copy")})
    lines = ["# Counters per launch: " + os.path.basename(out).rsplit(".", 1)[0], "",
             "Produced by:", "", "```", cmd, "```", "",
             f"kernel_source_hash: {kernel_source_hash()}", "",
             "Mean per launch (per pixel of a 4096x4096 launch in brackets).", "",
             "| kernel | launches | " + " | ".join(counters) + " |",
             "|---|---|" + "---|" * len(counters)]
    for k in kernels:
        n = max(len(agg[(k, c)]) for c in counters)
        cells = []
        for c in counters:
            vs = agg.get((k, c), [])
            m = sum(vs) / len(vs) if vs else float("nan")
            cells.append(f"{m:.4g} ({m / px:.3g})" if c != "SQ_WAVES" else f"{m:.0f}")
        lines.append(f"| {k} | {n} | " + " | ".join(cells) + " |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def _counter_mean(db, kernel_sub, counter):
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, dispatch_id, sum(value) from counters_collection "
                       "where counter_name = ? group by dispatch_id", (counter,)).fetchall()
    vals = [v for k, d, v in rows if kernel_sub in k]
    return sum(vals) / len(vals), len(vals)


# Read request size of each kernel's bulk reads, for the FETCH_SIZE factor:
# k_local reads each tile row's 64 bytes as one request; the others read
# whole contiguous blocks (slots, forest entries, bitmasks, run tables).
KERNEL_READ_REQUEST = {"local": 64, "block": 128, "seam": 128, "final": 128}


def summarize_traffic(fetch_db, write_db, copy_fetch_db, copy_write_db, copy_bytes,
                      seg_fetch_db, seg_bytes, out, cmd, px=4096 * 4096):
    """FETCH_SIZE / WRITE_SIZE runs of the labelling kernels, scaled by what the
    same counters read for a copy of a known number of bytes: the contiguous
    copy kernel (128-byte requests) and the gathering copy of 64-byte
    segments; each kernel's reads take the factor of its request size."""
    cf_kib, _ = _counter_mean(copy_fetch_db, "k_copy", "FETCH_SIZE")
    cw_kib, _ = _counter_mean(copy_write_db, "k_copy", "WRITE_SIZE")
    sf_kib, _ = _counter_mean(seg_fetch_db, "k_copy_seg", "FETCH_SIZE")
    ff = copy_bytes / (cf_kib * 1024.0)
    wf = copy_bytes / (cw_kib * 1024.0)
    sf = seg_bytes / (sf_kib * 1024.0)
    read_factor = {128: ff, 64: sf}
    lines = ["# HBM traffic per launch on the 4096x4096 headline workload", "",
             "Produced by (each counter in its own run):", "", "```", cmd, "```", "",
             f"kernel_source_hash: {kernel_source_hash()}",
             f"copy_bytes: {copy_bytes}",
             f"copy_fetch_kib: {cf_kib:.1f}",
             f"copy_write_kib: {cw_kib:.1f}",
             f"segment_copy_bytes: {seg_bytes}",
             f"segment_copy_fetch_kib: {sf_kib:.1f}",
             f"fetch_factor: {ff:.4f}",
             f"fetch_factor_64B_requests: {sf:.4f}",
             f"write_factor: {wf:.4f}", "",
             "| kernel | launches | FETCH_SIZE KiB | read request | WRITE_SIZE KiB | scaled bytes | "
             "algorithmic bytes |",
             "|---|---|---|---|---|---|---|"]
    fields = []
    path_total = 0.0
    for kind, kname in KERNEL_NAMES.items():
        f_kib, nf = _counter_mean(fetch_db, kname, "FETCH_SIZE")
        w_kib, nw = _counter_mean(write_db, kname, "WRITE_SIZE")
        req = KERNEL_READ_REQUEST[kind]
        total = f_kib * 1024.0 * read_factor[req] + w_kib * 1024.0 * wf
        path_total += total
        algo = KERNEL_BYTES_PER_PX.get(kind, 0.0) * px
        lines.append(f"| {kname} | {nf} | {f_kib:.1f} | {req} B | {w_kib:.1f} | {total:.0f} | "
                     f"{algo:.0f} |")
        fields.append(f"{kind}_bytes_per_launch: {total:.0f}")
    fields.append(f"path_bytes_per_px: {path_total / px:.3f}")
    lines += [""] + fields + [""]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def replay_durations(ccl, torch, devs, reps=10):
    """Average duration (microseconds) of one launch of k_local and of
    k_final over the rotation: each image is labelled, one of its kernels
    is launched `reps` more times back to back between two events
    (ccl_replay_last, on the current stream), and the image is labelled
    again (replaying the local step resets the merge state)."""
    st = torch.cuda.current_stream()
    out_us = {}
    for kind in ("local", "final"):
        tot = 0.0
        for img, out, conn in devs:
            ccl.label(img, conn, out=out)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            ccl.replay_last(kind, reps)
            e1.record(st)
            ccl.label(img, conn, out=out)
            torch.cuda.synchronize()
            tot += 1e3 * e0.elapsed_time(e1) / reps
        out_us[kind] = round(tot / len(devs), 2)
    return out_us


def step_distribution(ccl, torch, devs, steps):
    """Duration of each of `steps` steps from an event recorded between
    consecutive steps: median, min and 99th percentile in microseconds."""
    st = torch.cuda.current_stream()
    n = len(devs)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(st)
    for i in range(steps):
        img, out, conn = devs[i % n]
        ccl.label(img, conn, out=out)
        ev[i + 1].record(st)
    torch.cuda.synchronize()
    us = np.array([1e3 * ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    return {"median": round(float(np.median(us)), 2), "min": round(float(us.min()), 2),
            "p99": round(float(np.percentile(us, 99)), 2), "reps": steps}


def multi_stream_rate(ccl, torch, devs, steps, nstreams=4):
    """Gpixel/s when the rotation's independent images are issued round-robin
    on `nstreams` streams (each with its own workspace), so that the merge
    and final kernels of one image overlap the local step of the next.  A
    throughput figure beside the one-stream headline, not a replacement."""
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    cur = torch.cuda.current_stream()
    for i in range(2 * nstreams):
        img, out, conn = devs[i % len(devs)]
        ccl.label(img, conn, out=out, stream=streams[i % nstreams])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(cur)
    for st in streams:
        st.wait_stream(cur)
    for i in range(steps):
        img, out, conn = devs[i % len(devs)]
        ccl.label(img, conn, out=out, stream=streams[i % nstreams])
    for st in streams:
        cur.wait_stream(st)
    e1.record(cur)
    torch.cuda.synchronize()
    px = devs[0][0].shape[0] * devs[0][0].shape[1]
    return steps * px / (e0.elapsed_time(e1) / 1e3) / 1e9


def copy_bandwidth(ccl, torch, dev, mib=256, reps=10):
    """Read + write GB/s of the library's copy kernel over `mib` MiB: the
    achievable HBM rate on this machine, next to the 8 TB/s peak."""
    nbytes = mib << 20
    src = torch.ones(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    ccl.copy_bytes(src, dst)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        ccl.copy_bytes(src, dst)
    e1.record(st)
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / reps / 1e3
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / secs / 1e9


def host_cpu():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_count": os.cpu_count(), "usable": len(os.sched_getaffinity(0)), "model": model}


def oracle_all_cores(imgs, conn):
    """The oracle over a list of images, one image per worker thread on every
    usable core (the C routine releases the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as pool:
        outs = list(pool.map(lambda im: oracle.oracle_label(im, conn), imgs))
    return outs, time.perf_counter() - t0, cores


def bench_stats(ccl, torch, dev, cases, devs, label_us, steps, check=True):
    """ccl_label_stats (labels plus per-component statistics) over the
    headline rotation, next to the plain labelling rate; the statistics of
    the Bernoulli p = 0.5 images are compared with the oracle's, which is
    timed on one core."""
    size = devs[0][0].shape[0]
    cap = ccl.max_components(size, size, 4)
    comps = torch.empty(cap * ccl.COMPONENT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    count = torch.empty(1, dtype=torch.int64, device=dev)
    lib = ccl.lib()
    st = torch.cuda.current_stream()
    sh = int(st.cuda_stream)
    calls = [(img.data_ptr(), size, size, size, conn, out.data_ptr(), comps.data_ptr(), cap,
              count.data_ptr(), sh) for img, out, conn in devs]

    def run(k):
        for i in range(k):
            assert lib.ccl_label_stats(*calls[i % len(calls)]) == 0

    run(len(calls))
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    run(steps)
    e1.record(st)
    torch.cuda.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / steps
    ccl.timing_enable(True, kinds=["stats"])
    run(steps)
    kern = ccl.timing_read()
    ccl.timing_enable(False)
    ms, n = kern["stats"]
    out = {"Gpx/s": round(size * size / us / 1e3, 1), "us_per_step": round(us, 2),
           "stats_kernels_us": round(1e3 * ms / max(n, 1), 2),
           "label_only_us": round(label_us, 2), "overhead": round(us / label_us, 3)}
    if check:
        import oracle
        exact, cpu_secs, px = True, 0.0, 0
        for i, (name, img, conn) in enumerate(cases):
            if not name.startswith("bernoulli{'p': 0.5}"):
                continue
            assert lib.ccl_label_stats(*calls[i]) == 0
            got = ccl.components_to_numpy(comps, count)
            c0 = time.perf_counter()
            want = oracle.oracle_stats(img, conn)
            cpu_secs += time.perf_counter() - c0
            px += img.size
            exact &= len(got) == len(want) and all(np.array_equal(got[f], want[f])
                                                   for f in want.dtype.names)
        out["exact_sampled"] = bool(exact)
        out["cpu_baseline"] = {"value": round(px / cpu_secs / 1e9, 5), "unit": "Gpixel/s",
                               "cores": 1, "kind": "oracle",
                               "sample": "the two Bernoulli p = 0.5 images (4- and 8-connected) once"}
    del comps
    torch.cuda.empty_cache()
    return out


def bench_ablation(ccl, torch, dev, check=True):
    """The paper's study of its coarse step (4-connectivity): per-tile find
    iterations and atomic merge attempts of C2FL / RC2FL / CC2FL / NC2FL
    (means over tiles, and the largest tile) for Bernoulli p = 0.5 images of
    32^2 .. 4096^2 and for densities 0.1 .. 0.9 at 2048^2, plus the time of
    each variant's full labelling at 4096^2, p = 0.5."""
    from paper_1712_09789_amd import workloads as wl
    out = {"by_size_p0.5": {}, "by_density_2048": {}, "time_4096_us": {}, "exact": None}
    exact = True

    def counts(img, v):
        d = torch.from_numpy(img).to(dev)
        lab, cnt = ccl.label_ablation(d, v, counters=True)
        c = cnt.cpu().numpy().astype(np.int64)
        return lab, [round(float(c[:, 0].mean()), 1), round(float(c[:, 1].mean()), 1),
                     int(c[:, 0].max()), int(c[:, 1].max())]

    for v in ccl.ABLATIONS:
        out["by_size_p0.5"][v] = {}
        for n in (32, 64, 128, 256, 512, 1024, 2048, 4096):
            img = wl.bernoulli(n, n, 0.5, seed=n)
            lab, c = counts(img, v)
            out["by_size_p0.5"][v][n] = c
            if check and n == 512:
                import oracle
                exact &= bool(np.array_equal(lab.cpu().numpy(), oracle.oracle_label(img, 4)))
        out["by_density_2048"][v] = {}
        for p10 in range(1, 10):
            img = wl.bernoulli(2048, 2048, p10 / 10, seed=p10)
            out["by_density_2048"][v][p10 / 10] = counts(img, v)[1]
    img = torch.from_numpy(wl.bernoulli(4096, 4096, 0.5, seed=0)).to(dev)
    lab = torch.empty((4096, 4096), dtype=torch.int32, device=dev)
    st = torch.cuda.current_stream()
    for v in ccl.ABLATIONS:
        for _ in range(3):
            ccl.label_ablation(img, v, out=lab)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(20):
            ccl.label_ablation(img, v, out=lab)
        e1.record(st)
        torch.cuda.synchronize()
        out["time_4096_us"][v] = round(1e3 * e0.elapsed_time(e1) / 20, 1)
    out["exact"] = exact if check else None
    out["columns"] = "[mean iterations per tile, mean atomics per tile, max iterations, max atomics]"
    return out


def bench_volume(ccl, torch, dev, check=True, n=512, reps=10):
    """ccl_label_3d on n^3 volumes (Bernoulli p = 0.3 / 0.5, 3-D blobs sigma
    2 thresholded at the median) under 6- and 26-connectivity, in
    Gvoxel/s; exactness against the 3-D oracle on 192^3 volumes of the same
    kinds, whose one-core rate is the CPU baseline."""
    from paper_1712_09789_amd import workloads as wl
    kinds = (("bernoulli", {"p": 0.3}), ("bernoulli", {"p": 0.5}), ("blobs", {"sigma": 2.0}))
    out = {"size": n}
    st = torch.cuda.current_stream()
    lab = torch.empty((n, n, n), dtype=torch.int32, device=dev)
    for kind, kw in kinds:
        vol = torch.from_numpy(wl.make3d(kind, n, n, n, seed=0, **kw)).to(dev)
        for conn in (6, 26):
            ccl.label_3d(vol, conn, out=lab)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(reps):
                ccl.label_3d(vol, conn, out=lab)
            e1.record(st)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            ccl.timing_enable(True, ("vlocal", "vmerge", "vfinal"))
            for _ in range(reps):
                ccl.label_3d(vol, conn, out=lab)
            t = ccl.timing_read()
            ccl.timing_enable(False)
            out[f"{kind}{kw} conn={conn}"] = {
                "Gvox/s": round(n ** 3 / ms / 1e6, 1), "us": round(1e3 * ms, 1),
                "kernel_avg_us": {k: round(1e3 * t[k][0] / t[k][1], 1)
                                  for k in ("vlocal", "vmerge", "vfinal") if t[k][1]}}
        del vol
    del lab
    torch.cuda.empty_cache()
    if check:
        import oracle
        m = 192
        exact, cpu_secs = True, 0.0
        for kind, kw in kinds:
            vol = wl.make3d(kind, m, m, m, seed=1, **kw)
            d = torch.from_numpy(vol).to(dev)
            for conn in (6, 26):
                got = ccl.label_3d(d, conn).cpu().numpy()
                c0 = time.perf_counter()
                want = oracle.oracle_label3d(vol, conn)
                cpu_secs += time.perf_counter() - c0
                exact &= bool(np.array_equal(got, want))
        out["exact_sampled"] = exact
        out["cpu_baseline"] = {"value": round(6 * m ** 3 / cpu_secs / 1e9, 5),
                               "unit": "Gvoxel/s", "cores": 1, "kind": "oracle",
                               "sample": f"the three kinds at {m}^3, both connectivities, once"}
    return out


def bench_batch(ccl, torch, dev, check=True, n=256, reps=5):
    """256 uint8 images, sides log-uniform in [64, 2048], half Bernoulli and
    half blobs at random density, 8-connectivity: one ccl_label_batch call
    against 256 ccl_label calls on the same stream (both issued through
    precomputed ctypes arguments)."""
    import ctypes
    from paper_1712_09789_amd import workloads as wl
    specs = wl.batch_specs(n, seed=0)
    imgs = [wl.make(k, H, W, seed=sd, **kw) for (H, W, k, kw, sd) in specs]
    px = sum(im.size for im in imgs)
    dimgs = [torch.from_numpy(im).to(dev) for im in imgs]
    outs = [torch.empty(im.shape, dtype=torch.int32, device=dev) for im in imgs]
    lib = ccl.lib()
    st = torch.cuda.current_stream()
    sh = int(st.cuda_stream)
    descs = ccl.make_descs(dimgs, outs, 8)
    singles = [(d.data_ptr(), d.shape[0], d.shape[1], d.shape[1], 8, o.data_ptr(), sh)
               for d, o in zip(dimgs, outs)]

    def batch():
        assert lib.ccl_label_batch(descs, n, sh) == 0

    def per_image():
        for a in singles:
            lib.ccl_label(*a)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3

    t_single = timed(per_image)
    t_batch = timed(batch)
    # the same batch prepared once and replayed from a captured graph
    plan = ccl.Plan(dimgs, 8, outs=outs)
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(st)
    with torch.cuda.stream(cs):
        plan.run(stream=cs)
    st.wait_stream(cs)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        plan.run()
    t_graph = timed(g.replay)
    exact = None
    cpu = None
    if check:
        batch()
        torch.cuda.synchronize()
        wants, cpu_secs, cores = oracle_all_cores(imgs, 8)
        exact = all(np.array_equal(outs[i].cpu().numpy(), wants[i]) for i in range(n))
        cpu = {"Gpx/s": round(px / cpu_secs / 1e9, 4), "cores": cores, "kind": "oracle",
               "sample": "the whole batch once, one image per worker thread"}
    return {"images": n, "Mpx": round(px / 1e6, 2),
            "batch_ms": round(1e3 * t_batch, 3), "per_image_ms": round(1e3 * t_single, 3),
            "batch_Gpx/s": round(px / t_batch / 1e9, 1),
            "per_image_Gpx/s": round(px / t_single / 1e9, 1),
            "graph_ms": round(1e3 * t_graph, 3),
            "graph_Gpx/s": round(px / t_graph / 1e9, 1),
            "speedup": round(t_single / t_batch, 3),
            "speedup_graph": round(t_single / t_graph, 3),
            "exact": exact,
            "oracle_all_cores": cpu}


def bench_serving(torch, dev, n=5000, seed=0):
    """Poisson stream of frames 640x480 / 1920x1080 / 3840x2160 (weights
    .5/.35/.15), blobs with sigma 8 thresholded at the median, 8-connectivity,
    frames resident on the device.  The saturation rate S is the throughput
    with every frame arriving at once; the stream then runs at 0.5 S and 0.8 S."""
    from paper_1712_09789_amd import workloads as wl
    from paper_1712_09789_amd.serve import GpuExecutor, Request, Scheduler
    pool = {}
    for H, W, _ in wl.SERVING_MIX:
        pool[(H, W)] = [torch.from_numpy(wl.blobs(H, W, 8, seed=7 * H + k)).to(dev)
                        for k in range(3)]
    sizes = wl.serving_frames(n, seed)
    rng = np.random.default_rng(seed)

    def trace(rate):
        t, reqs = 0.0, []
        for i, (H, W, s) in enumerate(sizes):
            if rate:
                t += rng.exponential(1.0 / rate)
            reqs.append(Request(rid=i, image=pool[(H, W)][s % 3], connectivity=8,
                                arrival=t, H=H, W=W))
        return reqs

    ex = GpuExecutor(streams=4)

    def serve(rate):
        # results are not kept: each label buffer returns to the pool when its
        # request retires, as in a loop that hands labels on and forgets them
        sched = Scheduler(ex, slots=4, max_batch=64, keep_labels=False)
        stats = sched.run(trace(rate))
        torch.cuda.synchronize()
        return stats

    serve(0.0)  # warm-up: buffers and workspaces
    sat = serve(0.0)
    s_rate = sat.completed / sat.makespan_s
    out = {"frames": n, "saturation_frames_per_s": round(s_rate, 1),
           "saturation": sat.as_dict()}
    for frac in (0.5, 0.8):
        out[f"rate_{frac}S"] = serve(frac * s_rate).as_dict()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=280)
    ap.add_argument("--warmup", type=int, default=28)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--profile-stats", type=int, default=0, metavar="ROUNDS",
                    help="only run ccl_label_stats over the headline images ROUNDS times "
                         "(for a kernel trace of the statistics path) and exit")
    ap.add_argument("--profile-volume", type=int, default=0, metavar="ROUNDS",
                    help="only run ccl_label_3d on the 512^3 Bernoulli p = 0.3 volume, both "
                         "connectivities, ROUNDS times (for a kernel trace) and exit")
    ap.add_argument("--profile-large", type=int, default=0, metavar="ROUNDS",
                    help="only label the six 8192^2 8-connected images (Bernoulli 0.5 and the "
                         "adversarial geometries) ROUNDS times (for a kernel trace) and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run the copy kernel over MIB MiB (counter calibration)")
    ap.add_argument("--calibrate-segments", type=int, default=0, metavar="MIB",
                    help="only run the gathering copy of 64-byte segments (one every 256 "
                         "bytes) into MIB MiB (counter calibration)")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("DB", "OUT", "CMD"),
                    help="write a markdown table of a --pmc run's counters per kernel and exit")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("DB", "OUT", "CMD"),
                    help="write a rocprofv3 kernel-trace summary (no GPU needed)")
    ap.add_argument("--summarize-traffic", nargs=9,
                    metavar=("FETCH_DB", "WRITE_DB", "COPY_FETCH_DB", "COPY_WRITE_DB",
                             "COPY_BYTES", "SEG_FETCH_DB", "SEG_BYTES", "OUT", "CMD"),
                    help="write the per-kernel HBM traffic summary (no GPU needed)")
    args = ap.parse_args()

    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_traffic:
        a = args.summarize_traffic
        summarize_traffic(a[0], a[1], a[2], a[3], int(a[4]), a[5], int(a[6]), a[7], a[8])
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(images are independent, so batches shard by whole images). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1712_09789_amd.ccl as ccl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            ccl.copy_bytes(src, dst)
        torch.cuda.synchronize()
        ccl.timing_enable(True)
        for _ in range(10):
            ccl.copy_bytes(src, dst)
        k = ccl.timing_read()
        ccl.timing_enable(False)
        ms, n = k["copy"]
        print(json.dumps({"copy_bytes": nbytes, "launches": n,
                          "avg_us": 1e3 * ms / n,
                          "read_plus_write_GBs": 2 * nbytes / (ms / n / 1e3) / 1e9}))
        return

    if args.calibrate_segments:
        nbytes = args.calibrate_segments << 20
        src = torch.ones(nbytes * 4, dtype=torch.uint8, device=dev)
        dst = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        for _ in range(3):
            ccl.copy_segments(src, dst, 64, 256)
        torch.cuda.synchronize()
        ccl.timing_enable(True)
        for _ in range(10):
            ccl.copy_segments(src, dst, 64, 256)
        k = ccl.timing_read()
        ccl.timing_enable(False)
        ms, n = k["copy"]
        print(json.dumps({"segment_copy_bytes": nbytes, "launches": n,
                          "avg_us": 1e3 * ms / n}))
        return

    if args.profile_volume:
        from paper_1712_09789_amd import workloads as wl
        n = 512
        vol = torch.from_numpy(wl.make3d("bernoulli", n, n, n, seed=0, p=0.3)).to(dev)
        lab = torch.empty((n, n, n), dtype=torch.int32, device=dev)
        for _ in range(args.profile_volume):
            for conn in (6, 26):
                ccl.label_3d(vol, conn, out=lab)
        torch.cuda.synchronize()
        log(f"[bench] profile-volume: {args.profile_volume} rounds")
        return

    if args.profile_large:
        from paper_1712_09789_amd import workloads as wl
        big = 8192
        imgs = [torch.from_numpy(wl.make(kind, big, big, seed=0, **kw)).to(dev)
                for kind, kw in (("bernoulli", {"p": 0.5}),) + wl.ADVERSARIAL]
        lab = torch.empty((big, big), dtype=torch.int32, device=dev)
        for _ in range(args.profile_large):
            for img in imgs:
                ccl.label(img, 8, out=lab)
        torch.cuda.synchronize()
        log(f"[bench] profile-large: {args.profile_large} rounds of {len(imgs)} images")
        return

    size = args.size
    t0 = time.time()
    cases = headline_cases(size)
    log(f"[bench] generated {len(cases)} {size}x{size} cases in {time.time() - t0:.1f}s")
    devs = []
    for name, img, conn in cases:
        devs.append((torch.from_numpy(img).to(dev), torch.empty((size, size), dtype=torch.int32,
                                                              device=dev), conn))
    torch.cuda.synchronize()

    if args.profile_stats:
        cap = ccl.max_components(size, size, 4)
        comps = torch.empty(cap * ccl.COMPONENT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        count = torch.empty(1, dtype=torch.int64, device=dev)
        sh = int(torch.cuda.current_stream().cuda_stream)
        for _ in range(args.profile_stats):
            for img, out, conn in devs:
                assert ccl.lib().ccl_label_stats(img.data_ptr(), size, size, size, conn,
                                                 out.data_ptr(), comps.data_ptr(), cap,
                                                 count.data_ptr(), sh) == 0
        torch.cuda.synchronize()
        log(f"[bench] profile-stats: {args.profile_stats} rounds of {len(devs)} images")
        return

    # exactness: one labelling of every case, compared with the CPU oracle,
    # which is timed on this host's core as the baseline
    exact = True
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        os.sched_setaffinity(0, {sorted(os.sched_getaffinity(0))[0]})
        cpu_secs = 0.0
        for (name, img, conn), (dimg, dout, _) in zip(cases, devs):
            ccl.label(dimg, conn, out=dout)
            torch.cuda.synchronize()
            got = dout.cpu().numpy()
            c0 = time.perf_counter()
            want = oracle.oracle_label(img, conn)
            cpu_secs += time.perf_counter() - c0
            ok = np.array_equal(got, want)
            exact &= ok
            log(f"[bench] exact vs oracle: {name} conn={conn}: {ok}")
        os.sched_setaffinity(0, set(range(os.cpu_count() or 1)))
        cpu_px = len(cases) * size * size
        cpu = {"value": round(cpu_px / cpu_secs / 1e9, 5), "unit": "Gpixel/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{len(cases)} images of {size}x{size} (every headline case once), "
                         f"single thread pinned to one core, {cpu_secs:.1f} s total",
               "host": host_cpu()}

    # timed region (headline value); then a region with events around every
    # kernel (per-kernel breakdown), and back-to-back launches of k_local and
    # of k_final alone (their launch durations, for the roofline figure)
    secs, _ = time_rotation(ccl, torch, devs, args.steps, args.warmup)
    secs_all, kern = time_rotation(ccl, torch, devs, args.steps, args.warmup,
                                   timing=["local", "block", "seam", "final"])
    kavg = {k: round(1e3 * v[0] / v[1], 2) for k, v in kern.items() if v[1]}
    replay_us = replay_durations(ccl, torch, devs)
    dom = max(("local", "final"), key=lambda k: replay_us[k])
    dist = step_distribution(ccl, torch, devs, max(args.steps, 20))
    # (after the timed regions, and left out of profiled runs: concurrent
    # kernels would blur per-kernel durations)
    streams4 = None if args.no_extra else multi_stream_rate(ccl, torch, devs, args.steps)
    copy_gbs = copy_bandwidth(ccl, torch, dev)
    px = size * size
    value = args.steps * px / secs / 1e9
    ms_step = 1e3 * secs / args.steps
    log(f"[bench] {size}^2: {value:.1f} Gpx/s, {ms_step * 1e3:.1f} us/step "
        f"(events around every kernel: {1e6 * secs_all / args.steps:.1f} us/step); "
        f"kernel avg us {kavg}")

    # the roofline rule: the path's algorithmic bytes per pixel (5: 1 read,
    # 4 written) times the pixels one launch processes, over the dominant
    # kernel's launch duration
    dom_avg_s = replay_us[dom] * 1e-6
    algo_bytes = PATH_BYTES_PER_PX * px
    achieved = algo_bytes / dom_avg_s / 1e9
    src_hash = kernel_source_hash()
    traffic = load_traffic(src_hash, dom)

    result = {
        "metric": "Gpixel/s at 4096^2 (exact vs oracle)",
        "value": round(value, 3),
        "unit": "Gpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "exact": bool(exact) if cpu is not None else None,
        "config": {"workload": f"{size}x{size} uint8 single image; Bernoulli p in "
                               "{.1,.3,.5,.7,.9} and median-thresholded blobs sigma {4,16}; "
                               "connectivity 4 and 8; 14 resident buffer sets in rotation",
                   # tile (rows, cols) the launch policy picks for one image
                   # of this size, per connectivity
                   "tile": {f"conn{c}": [ccl.policy_tile_rows(0, size * size, c),
                                         ccl.tile_shape()[1]] for c in (4, 8)}},
        "step_us": dist,
        "streams_4_Gpx/s": round(streams4, 1) if streams4 else None,
        "path_hbm_frac": round(PATH_BYTES_PER_PX * value / HBM_PEAK_GBS, 4),
        "copy_GBs": round(copy_gbs, 1),
        "path_copy_frac": round(PATH_BYTES_PER_PX * value / copy_gbs, 4),
        "kernel_avg_us": kavg,
        # one launch of k_local / k_final alone, back to back (ccl_replay_last)
        "kernel_launch_us": {KERNEL_NAMES[k]: v for k, v in replay_us.items()},
        # launch-shape cache the binding applied (tune.py); None = built-in rule
        "launch_policy": (os.path.basename(ccl.launch_policy_applied)
                          if ccl.launch_policy_applied else None),
        # every kernel with algorithmic bytes, on its own bytes (k_local:
        # image read + bitmask write; k_final: label write + bitmask read),
        # against HBM peak, over its back-to-back launch duration
        "kernel_hbm": {KERNEL_NAMES[k]: {
            "bytes_per_px": KERNEL_BYTES_PER_PX[k],
            "GBs": round(KERNEL_BYTES_PER_PX[k] * px / (replay_us[k] * 1e-6) / 1e9, 1),
            "frac": round(KERNEL_BYTES_PER_PX[k] * px / (replay_us[k] * 1e-6) / 1e9 /
                          HBM_PEAK_GBS, 4)}
            for k in KERNEL_BYTES_PER_PX},
        "roofline": {"bound": "hbm", "kernel": KERNEL_NAMES[dom],
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": algo_bytes,
                     "algorithmic_bytes_per_px": PATH_BYTES_PER_PX,
                     "avg_launch_us": round(dom_avg_s * 1e6, 2),
                     # the whole path on the same basis: 5 B/px (1 B read, 4 B
                     # written) per step over the measured step time
                     "path_bytes_per_px": PATH_BYTES_PER_PX,
                     "path_achieved": round(PATH_BYTES_PER_PX * px / (ms_step * 1e-3) / 1e9, 1),
                     "path_frac": round(PATH_BYTES_PER_PX * value / HBM_PEAK_GBS, 4)},
        "cpu_baseline": cpu,
    }

    if not args.no_extra:
        from paper_1712_09789_amd import workloads as wl
        extra = {}
        big = 8192
        for kind, kw in (("bernoulli", {"p": 0.5}),) + wl.ADVERSARIAL:
            img = wl.make(kind, big, big, seed=0, **kw)
            d = [(torch.from_numpy(img).to(dev),
                  torch.empty((big, big), dtype=torch.int32, device=dev), 8)]
            s, _ = time_rotation(ccl, torch, d, 20, 3)
            # per-kernel averages from a second region with events around every kernel
            _, kern = time_rotation(ccl, torch, d, 10, 1, timing=list(KERNEL_NAMES))
            gpx = 20 * big * big / s / 1e9
            extra[f"{kind}{kw}"] = {"Gpx/s": round(gpx, 1),
                                    "us": round(1e6 * s / 20, 1),
                                    "path_hbm_frac": round(PATH_BYTES_PER_PX * gpx / HBM_PEAK_GBS, 4),
                                    "kernel_avg_us": {k: round(1e3 * v[0] / v[1], 1)
                                                      for k, v in kern.items() if v[1]}}
            del d
            torch.cuda.empty_cache()
        result["extra_8192_conn8"] = extra
        log(f"[bench] 8192^2: {extra}")

    if not args.no_extra:
        result["stats_4096"] = bench_stats(ccl, torch, dev, cases, devs, 1e3 * ms_step,
                                           min(args.steps, 140), check=cpu is not None)
        log(f"[bench] stats: {result['stats_4096']}")
        result["volume_512"] = bench_volume(ccl, torch, dev, check=cpu is not None)
        log(f"[bench] volume: {result['volume_512']}")
        result["ablation"] = bench_ablation(ccl, torch, dev, check=cpu is not None)
        log(f"[bench] ablation: {result['ablation']['time_4096_us']} exact {result['ablation']['exact']}")
        result["batch_256"] = bench_batch(ccl, torch, dev, check=cpu is not None)
        log(f"[bench] batch: {result['batch_256']}")
        result["serving"] = bench_serving(torch, dev)
        log(f"[bench] serving: {result['serving']}")

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
