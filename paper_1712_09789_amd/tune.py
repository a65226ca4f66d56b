"""Launch-shape autotuner.

The local step and the final relabel each run either on a persistent grid
(one workgroup per resident slot) or with one workgroup per tile
(``ccl_set_launch_policy`` in include/ccl.h).  Which is faster depends on the
tile count and on whether a launch holds one image or many, so for every
launch class and tile-count bucket this module times the four combinations
and the library's built-in rule on synthetic Bernoulli(0.5) inputs of that
size (4- and 8-connectivity), keeps the fastest combination if it beats the
built-in rule by at least MARGIN (else the built-in rule, so that noise does
not decide), applies it, and returns the choices; ``--out`` writes
them to a JSON cache keyed by the GPU architecture, which
``ccl.apply_launch_policy`` loads.  Labels never depend on the choice.

    python -m paper_1712_09789_amd.tune --out launch_policy.json
"""
from __future__ import annotations

import argparse
import json
import math

import torch

import paper_1712_09789_amd.ccl as ccl

COMBOS = ((0, 0), (0, 1), (1, 0), (1, 1))  # (local, final): 0 = persistent, 1 = per tile
MARGIN = 0.02  # a combination must beat the built-in rule by this fraction
BATCH_SIDE = 512  # images of a batch representative: 512 x 512, 64 tiles each


def _tiles_of(bound: int, prev: int) -> int:
    """Tile count representing a bucket: its bound, or twice the previous
    bound for the open-ended last bucket."""
    return bound if bound < (1 << 62) else 2 * prev


def _inputs(batch: int, tiles: int, gen: torch.Generator):
    """Device images totalling about `tiles` tiles: one square image, or a
    batch of 512 x 512 images."""
    tc, tr = ccl.tile_shape()[1], ccl.tile_shape()[0]
    if batch == 0:
        side_tiles = max(1, int(math.isqrt(tiles)))
        shapes = [(side_tiles * tr, side_tiles * tc)]
    else:
        per = (BATCH_SIDE // tr) * (BATCH_SIDE // tc)
        shapes = [(BATCH_SIDE, BATCH_SIDE)] * max(2, tiles // per)
    imgs = [(torch.rand(shape, device="cuda", generator=gen) < 0.5).to(torch.uint8)
            for shape in shapes]
    outs = [torch.empty(shape, dtype=torch.int32, device="cuda") for shape in shapes]
    return imgs, outs


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


def tune(reps: int = 10, buckets: list[int] | None = None, seed: int = 0) -> dict:
    """Time every combination per (launch class, bucket), apply the choice
    and return {"arch", "buckets", "choices": [{batch, bucket, local, final,
    us: {"local,final": microseconds, "builtin": microseconds}}]} (local =
    final = -1: the built-in rule).  `buckets` limits the buckets tuned (the
    others keep their current setting)."""
    bounds = ccl.launch_buckets()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    choices = []
    for batch in (0, 1):
        for b, bound in enumerate(bounds):
            if buckets is not None and b not in buckets:
                continue
            tiles = _tiles_of(bound, bounds[b - 1] if b else 1)
            imgs, outs = _inputs(batch, tiles, gen)
            stream = torch.cuda.current_stream()
            descs = {conn: ccl.make_descs(imgs, outs, conn) for conn in (4, 8)}
            sh = int(stream.cuda_stream)

            def run():
                for conn in (4, 8):
                    if batch == 0:
                        ccl.label(imgs[0], conn, out=outs[0], stream=stream)
                    else:
                        ccl._check(ccl.lib().ccl_label_batch(descs[conn], len(imgs), sh))

            # the built-in rule is timed first and last (the faster counts),
            # so that clocks still settling do not count against it
            us = {}
            for local, final in ((-1, -1),) + COMBOS + ((-1, -1),):
                ccl.set_launch_policy(batch, b, local, final)
                key = "builtin" if local < 0 else f"{local},{final}"
                t = round(_time(run, reps), 2)
                us[key] = min(t, us.get(key, t))
            best = min((k for k in us if k != "builtin"), key=us.get)
            local, final = -1, -1
            if us[best] < (1.0 - MARGIN) * us["builtin"]:
                local, final = (int(v) for v in best.split(","))
            ccl.set_launch_policy(batch, b, local, final)
            choices.append({"batch": batch, "bucket": b, "tiles": tiles, "local": local,
                            "final": final, "us": us})
            del imgs, outs, descs
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return {"arch": arch, "buckets": bounds, "choices": choices}


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
