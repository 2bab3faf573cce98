"""Autotuner of the batched form's launch schedule.

The schedule has three knobs (hr_schedule): the pixels of one histogram work
item (tile_steps x one workgroup step of pixels), the number of persistent
workgroups per compute unit, and the pixels of one remap work item
(remap_steps x one step).  tune() times every candidate on the caller's
batch with device events and stores the fastest in a JSON cache keyed by
(bins, element size, mean image size bucket); lookup() reads it back.

    python -m paper_2510_21100_amd.tune --workload ragged64
"""

from __future__ import annotations

import json
import math
import os
from typing import Sequence

TILE_STEPS = (8, 16, 24, 32, 48, 64, 128)
# one batched workgroup per CU: its LDS (about 150 KB) and registers leave room
# for no second one, and the library caps the grid at what the CUs hold
WG_PER_CU = (1,)
REMAP_STEPS = (4, 8, 16, 24, 32, 48, 64)


def key(bins: int, esz: int, npix: int, n: int) -> str:
    mean = max(1, npix // max(1, n))
    return f"bins{bins}/e{esz}/px2^{round(math.log2(mean))}"


def lookup(path: str, bins: int, esz: int, npix: int, n: int):
    try:
        with open(path) as f:
            table = json.load(f)
    except (OSError, ValueError):
        return None
    e = table.get(key(bins, esz, npix, n))
    if not e:
        return None
    return int(e["tile_steps"]), int(e["wg_per_cu"]), int(e.get("remap_steps", 0))


def tune(imgs: Sequence, params, path: str | None = None, reps: int = 5,
         tile_steps=TILE_STEPS, wg_per_cu=WG_PER_CU, remap_steps=REMAP_STEPS, verbose: bool = True):
    """Times every (tile_steps, wg_per_cu, remap_steps) on the batch ``imgs`` (device
    tensors) and returns (best, timings_us).  Writes the cache if ``path``."""
    import torch

    from . import api as H

    n = len(imgs)
    esz = imgs[0].element_size()
    npix = sum(int(x.shape[0]) * int(x.shape[1]) for x in imgs)
    outs = [torch.empty_like(x) for x in imgs]
    ws = H.Workspace(max_images=n, max_bins=params.bins)
    stream = torch.cuda.current_stream()
    times = {}
    import itertools
    for ts, wg, rs in itertools.product(tile_steps, wg_per_cu, remap_steps):
        ws.set_schedule(ts, wg, rs)
        for _ in range(2):
            H.enhance_batch(imgs, params, outs=outs, ws=ws)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            H.enhance_batch(imgs, params, outs=outs, ws=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        times[(ts, wg, rs)] = us
        if verbose:
            print(f"tile_steps={ts:3d} wg_per_cu={wg} remap_steps={rs:3d}: {us:9.1f} us  "
                  f"{npix / us:9.0f} Mpix/s", flush=True)
    ws.close()
    best = min(times, key=times.get)
    if path:
        table = {}
        if os.path.exists(path):
            try:
                with open(path) as f:
                    table = json.load(f)
            except ValueError:
                table = {}
        table[key(params.bins, esz, npix, n)] = {"tile_steps": best[0], "wg_per_cu": best[1],
                                                  "remap_steps": best[2], "us": round(times[best], 1)}
        with open(path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return best, times


def _main():
    import argparse
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import bench  # the benchmark's workload definitions
    import torch

    from . import api as H

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="ragged64")
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "schedule.json"))
    args = ap.parse_args()
    _, bits, jobs = bench.workload(args.workload)
    imgs = bench.generate(jobs, min(16, os.cpu_count() or 1))
    dev = torch.device("cuda", 0)
    g = []
    for x in imgs:
        t = torch.from_numpy(x)
        if t.dtype == torch.uint16:
            t = t.view(torch.int16)
        g.append(t.to(dev))
    best, _ = tune(g, H.Params(bins=1 << bits), path=args.out)
    print("best", best)


if __name__ == "__main__":
    _main()
