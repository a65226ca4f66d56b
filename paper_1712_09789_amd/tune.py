"""Launch-policy autotuner: tile height and launch grids.

The paper's one tuning knob is the block shape (Section 4.1, effectiveness
of coarse labelling).  The library is built for tiles 64 pixels wide and
32, 64 or 128 rows high, and each of its two per-tile kernels (the local
step and the final relabel) runs either on a persistent grid or with one
workgroup per tile (``ccl_set_launch_policy`` in include/ccl.h).  Which is
fastest depends on the image size, on whether a launch holds one image or
many, and on the connectivity, so for every launch class (one image /
several), pixel bucket and connectivity this module

1. times every tile height with the built-in grids, on two synthetic
   contents of the bucket's size (Bernoulli(0.5) noise, the paper's worst
   density, and box-smoothed thresholded noise for large regions); a
   batch class uses images with sides log-uniform in [64, 2048], the
   batched workload's size mix;
2. times the four grid combinations with the fastest height;
3. keeps a non-built-in choice only if it beats the built-in one (64 rows,
   built-in grids) by at least MARGIN, so that noise does not decide,

applies the choices and returns them; ``--out`` writes them to a JSON cache
keyed by the GPU architecture, which ``ccl.apply_launch_policy`` loads.
Labels never depend on the choice.

    python -m paper_1712_09789_amd.tune --out launch_policy.json
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np
import torch

import paper_1712_09789_amd.ccl as ccl

GRIDS = ((0, 0), (0, 1), (1, 0), (1, 1))  # (local, final): 0 = persistent, 1 = per tile
MARGIN = 0.02  # a choice must beat the built-in one by this fraction
BATCH_SIDES = (64, 2048)  # side range of a batch class's images (log-uniform)
MAX_BATCH_IMAGES = 4096


def _pixels_of(bound: int, prev: int) -> int:
    """Pixel count representing a bucket: its bound, or twice the previous
    bound for the open-ended last bucket."""
    return bound if bound < (1 << 62) else 2 * prev


def _shapes(batch: int, px: int, seed: int) -> list[tuple[int, int]]:
    """Image sizes totalling about px pixels: one square image, or images
    with independent log-uniform sides."""
    if batch == 0:
        side = max(64, int(math.isqrt(px)))
        return [(side, side)]
    rng = np.random.default_rng(seed)
    lo, hi = math.log(BATCH_SIDES[0]), math.log(BATCH_SIDES[1])
    shapes, total = [], 0
    while total < px and len(shapes) < MAX_BATCH_IMAGES:
        H, W = (int(round(math.exp(v))) for v in rng.uniform(lo, hi, 2))
        shapes.append((H, W))
        total += H * W
    if len(shapes) < 2:
        shapes.append((64, 64))
    return shapes


def _content(shape, kind: str, gen: torch.Generator) -> torch.Tensor:
    u = torch.rand(shape, device="cuda", generator=gen)
    if kind == "bernoulli":
        return (u < 0.5).to(torch.uint8)
    s = torch.nn.functional.avg_pool2d(u[None, None], 9, stride=1, padding=4)[0, 0]
    return (s > 0.5).to(torch.uint8)


def _time(run, reps: int) -> float:
    run()
    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        run()
    e1.record()
    torch.cuda.synchronize()
    return 1e3 * e0.elapsed_time(e1) / reps  # microseconds


def tune(reps: int = 5, buckets: list[int] | None = None, seed: int = 0) -> dict:
    """Time the tile heights and grids per (launch class, bucket,
    connectivity), apply the choices and return {"arch", "buckets",
    "shapes", "choices": [{batch, bucket, connectivity, pixels, tile_rows,
    local, final, us: {config: microseconds}}]} (tile_rows 0 and local =
    final = -1: the built-in choice).  `buckets` limits the buckets tuned
    (the others keep their current setting)."""
    bounds = ccl.launch_buckets()
    shapes_built = ccl.tile_shapes()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    choices = []
    for batch in (0, 1):
        for b, bound in enumerate(bounds):
            if buckets is not None and b not in buckets:
                continue
            px = _pixels_of(bound, bounds[b - 1] if b else 1)
            sizes = _shapes(batch, px, seed + b)
            for conn in (4, 8):
                sets = []
                for kind in ("bernoulli", "smooth"):
                    imgs = [_content(s, kind, gen) for s in sizes]
                    outs = [torch.empty(s, dtype=torch.int32, device="cuda") for s in sizes]
                    sets.append((imgs, outs, ccl.make_descs(imgs, outs, conn)))
                stream = torch.cuda.current_stream()
                sh = int(stream.cuda_stream)

                def run():
                    for imgs, outs, descs in sets:
                        if batch == 0:
                            ccl.label(imgs[0], conn, out=outs[0], stream=stream)
                        else:
                            ccl._check(ccl.lib().ccl_label_batch(descs, len(imgs), sh))

                us = {}

                def measure(rows, local, final):
                    ccl.set_launch_policy(batch, b, conn, rows, local, final)
                    key = "builtin" if (rows, local, final) == (0, -1, -1) else \
                        f"r{rows or 64},{local},{final}"
                    t = round(_time(run, reps), 2)
                    us[key] = min(t, us.get(key, t))
                    return us[key]

                # the built-in choice is timed first and last (the faster
                # counts), so that clocks still settling do not count against it
                measure(0, -1, -1)
                best_rows = min(shapes_built, key=lambda r: measure(r, -1, -1))
                for local, final in GRIDS:
                    measure(best_rows, local, final)
                measure(0, -1, -1)
                best = min((k for k in us if k != "builtin"), key=us.get)
                rows, local, final = 0, -1, -1
                if us[best] < (1.0 - MARGIN) * us["builtin"]:
                    r, lo, fi = best.split(",")
                    rows, local, final = int(r[1:]), int(lo), int(fi)
                ccl.set_launch_policy(batch, b, conn, rows, local, final)
                choices.append({"batch": batch, "bucket": b, "connectivity": conn,
                                "pixels": sum(h * w for h, w in sizes),
                                "images": len(sizes), "tile_rows": rows, "local": local,
                                "final": final, "us": us})
                del sets
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return {"arch": arch, "buckets": bounds, "shapes": shapes_built, "choices": choices}


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", help="write the choices to this JSON file")
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    result = tune(reps=args.reps)
    text = json.dumps(result, indent=1)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text + "\n")
    print(text)


if __name__ == "__main__":
    main()
