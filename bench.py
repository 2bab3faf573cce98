"""Benchmark of the HistRetinex histogram pipeline on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ragged64|uhd16]

A step is one pass of the whole pipeline (histograms, solver, target, LUT,
remap) over one batch of synthetic low-light images that are already resident
in HBM.  The timed form is the batched persistent launch; the one-image form
(one launch sequence per image) is timed on the same batch for the
batched-vs-plain ratio.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from synthetic import config_seed, make_batch_shapes, make_image  # noqa: E402

PEAK_HBM_GBS = 8000.0
METRIC = "Mpix/s end-to-end enhancement (batched vs plain, 1 GPU) + % HBM roofline"
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ("paper_2510_21100_amd/csrc/hr_kernels.hip", "paper_2510_21100_amd/csrc/hr_device.hpp",
                  "paper_2510_21100_amd/csrc/hr_launch.hpp")


def sources_digest() -> str:
    """sha256 over the kernel sources: a traffic figure measured on other
    sources no longer describes the kernel."""
    import hashlib

    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload_name: str, bits: int):
    """HBM bytes per launch of the batched kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known size), or
    None when there is none for the current kernel sources."""
    path = os.path.join(PROFILES, f"k_batch{bits}_{workload_name}.md")
    try:
        with open(path) as f:
            text = f.read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("bench-traffic:"):
            for tok in line.split()[1:]:
                k, _, v = tok.partition("=")
                vals[k] = v
    if vals.get("sources_sha256") != sources_digest() or "bytes_per_launch" not in vals:
        return None
    return int(vals["bytes_per_launch"])


def _gen(args):
    cfg, n, i, h, w, bits, ceil = args
    return make_image(config_seed(cfg, n, i), h, w, bits=bits, ceil=ceil)


def workload(name: str):
    """(description, bits, list of generator jobs)."""
    if name == "ragged64":
        n = 64
        shapes = make_batch_shapes(config_seed(3, 1, 0), n)
        rng = np.random.default_rng(2510211003)
        ceils = rng.uniform(0.03, 0.4, size=n)
        jobs = [(3, n, i, h, w, 8, float(ceils[i])) for i, (h, w) in enumerate(shapes)]
        desc = ("64 RGB uint8 images, W~U{640..4000}, H~U{480..3000}, illumination ceiling U[0.03,0.4], "
                "256 bins, 50 iterations")
        return desc, 8, jobs
    if name == "uhd16":
        n = 16
        shapes = [(2160, 3840) if i % 2 == 0 else (4320, 7680) for i in range(n)]
        jobs = [(4, n, i, h, w, 10, 0.3) for i, (h, w) in enumerate(shapes)]
        desc = "8 x 3840x2160 + 8 x 7680x4320 RGB uint16 10-bit images, 1024 bins, 50 iterations"
        return desc, 10, jobs
    if name == "single":
        jobs = [(2, 1, 0, 664, 1000, 8, 0.3)]
        return "one 1000x664 RGB uint8 image, 256 bins, 50 iterations", 8, jobs
    raise SystemExit(f"unknown workload {name}")


def _gen_truth(args):
    cfg, n, i, h, w = args
    img, rho = make_image(config_seed(cfg, n, i), h, w, return_truth=True)
    return img, (0.8 * rho).astype(np.float32)


DIFF_DESC = ("32 RGB uint8 1000x664 images against 0.8 x their reflectance (FP32 HWC), 256 bins, "
             "K = 30 unrolled iterations, checkpoints every 5")


def time_diff(dev, steps: int, workers: int):
    """Forward and forward+backward of the differentiated form on 32 images of
    1000x664 (gradients with respect to alpha, beta and the target histogram)."""
    import torch

    from paper_2510_21100_amd import api, diff

    n, (h, w) = 32, (664, 1000)
    jobs = [(5, n, i, h, w) for i in range(n)]
    if workers > 1:
        with ProcessPoolExecutor(max_workers=workers) as ex:
            pairs = list(ex.map(_gen_truth, jobs))
    else:
        pairs = [_gen_truth(j) for j in jobs]
    imgs = [torch.from_numpy(a).to(dev) for a, _ in pairs]
    tims = [torch.from_numpy(t).to(dev) for _, t in pairs]
    ws = api.Workspace(max_images=n, max_bins=256)

    def run(backward: bool):
        alpha = torch.tensor(0.01, dtype=torch.float64, requires_grad=True)
        beta = torch.tensor(0.01, dtype=torch.float64, requires_grad=True)
        loss, target = diff.enhancement_loss(imgs, tims, alpha, beta, iters=30, ckpt_every=5, ws=ws)
        if backward:
            loss.backward()
        return loss

    out = {}
    for name, bw in (("forward", False), ("forward_backward", True)):
        run(bw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            run(bw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        out[name + "_ms"] = round(ms, 3)
    npix = n * h * w
    out.update({"workload": DIFF_DESC, "pixels": npix,
                "Mpix_per_s_forward_backward": round(npix / (out["forward_backward_ms"] * 1e-3) / 1e6, 1)})
    ws.close()
    return out


def generate(jobs, workers: int):
    if len(jobs) == 1 or workers <= 1:
        return [_gen(j) for j in jobs]
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_gen, jobs))


def cpu_baseline(imgs, bits, budget_s: float):
    """The FP64 oracle, as it is, on whole images of the workload until about
    budget_s seconds of CPU time have been spent (at least one image)."""
    import oracle as O

    params = O.Params(bins=1 << bits, iters=50)
    O.classify(params.bins)  # one-time table, not timed
    O.classify_enhanced(params.bins, params.gamma)
    order = sorted(range(len(imgs)), key=lambda i: imgs[i].shape[0] * imgs[i].shape[1])
    done_px, spent, used = 0, 0.0, []
    for i in order:
        t0 = time.perf_counter()
        O.enhance(imgs[i], params)
        spent += time.perf_counter() - t0
        done_px += imgs[i].shape[0] * imgs[i].shape[1]
        used.append(i)
        if spent >= budget_s:
            break
    return {
        "value": done_px / spent / 1e6,
        "unit": "Mpix/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{len(used)} whole image(s) of the workload, smallest first, {done_px} pixels, "
                  f"{spent:.1f} s, single-threaded numpy FP64",
    }


def time_plain(H, gimgs, outs, params, bins, stream, steps):
    """The one-image form (three calls per image) on the same batch, and the
    solver alone on the first image's histograms."""
    import torch

    pl_ws = H.Workspace(max_images=1, max_bins=bins)

    def one_pass():
        for g, o in zip(gimgs, outs):
            hv, hg, _ = H.build_hist(g, pl_ws)
            _, _, tg = H.solve(hv, hg, g.shape[0] * g.shape[1], params, pl_ws)
            H.match(g, hv, tg, out=o, ws=pl_ws)

    one_pass()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        one_pass()
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t1) * 1e3 / steps
    npix = sum(g.shape[0] * g.shape[1] for g in gimgs)
    plain_value = npix / (plain_ms * 1e-3) / 1e6

    hv, hg, _ = H.build_hist(gimgs[0], pl_ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record(stream)
    for _ in range(reps):
        H.solve(hv, hg, gimgs[0].shape[0] * gimgs[0].shape[1], params, pl_ws)
    e1.record(stream)
    torch.cuda.synchronize()
    solve_us = e0.elapsed_time(e1) * 1e3 / reps
    pl_ws.close()
    return plain_ms, plain_value, solve_us


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--workload", default="ragged64", choices=["ragged64", "uhd16", "single"])
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time (0 = skip)")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--tile-steps", type=int, default=0)
    ap.add_argument("--wg-per-cu", type=int, default=0)
    ap.add_argument("--remap-steps", type=int, default=0)
    ap.add_argument("--schedule", default=os.path.join(ROOT, "paper_2510_21100_amd", "schedule.json"))
    ap.add_argument("--no-plain", action="store_true", help="skip the one-image form and the solver timing")
    ap.add_argument("--no-diff", action="store_true", help="skip the differentiated-form timing")
    ap.add_argument("--device-warmup-s", type=float, default=0.3,
                    help="seconds of untimed batched calls before the warmup steps")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="after the batched steps, one device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the images of a batch are independent and the bench "
              "measures one GPU's share; use --gpus 1", file=sys.stderr)
        raise SystemExit(2)

    desc, bits, jobs = workload(args.workload)
    t0 = time.perf_counter()
    imgs = generate(jobs, args.workers)
    gen_s = time.perf_counter() - t0

    import torch

    import paper_2510_21100_amd as H
    from paper_2510_21100_amd import tune

    bins = 1 << bits
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    def to_dev(x):
        t = torch.from_numpy(x)
        if t.dtype == torch.uint16:
            t = t.view(torch.int16)
        return t.to(dev)

    gimgs = [to_dev(x) for x in imgs]
    outs = [torch.empty_like(g) for g in gimgs]
    npix = sum(g.shape[0] * g.shape[1] for g in gimgs)
    esz = 1 if bits == 8 else 2
    alg_bytes = 9 * esz * npix  # read + re-read + write of 3 channels
    params = H.Params(bins=bins, iters=50)
    ws = H.Workspace(max_images=len(gimgs), max_bins=bins)
    sched = (args.tile_steps, args.wg_per_cu, args.remap_steps)
    if sched == (0, 0, 0):
        sched = tune.lookup(args.schedule, bins, esz, npix, len(gimgs)) or (0, 0, 0)
    ws.set_schedule(*sched)
    stream = torch.cuda.current_stream()

    # ---- batched form --------------------------------------------------------
    # device warm-up before the warmup steps: a first process on an idle GPU
    # has been seen running several times slower for its first tens of ms
    t_w = time.perf_counter()
    n_w = 0
    while time.perf_counter() - t_w < args.device_warmup_s or n_w < 2:
        H.enhance_batch(gimgs, params, outs=outs, ws=ws)
        torch.cuda.synchronize()
        n_w += 1
    for _ in range(args.warmup):
        H.enhance_batch(gimgs, params, outs=outs, ws=ws)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        H.enhance_batch(gimgs, params, outs=outs, ws=ws)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    launch_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    ms_step = wall * 1e3 / args.steps
    value = npix / (ms_step * 1e-3) / 1e6
    avg_launch_s = float(np.mean(launch_ms)) * 1e-3
    achieved = alg_bytes / avg_launch_s / 1e9

    if args.calibrate_copy_mb > 0:
        nbytes = args.calibrate_copy_mb << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    plain_ms = plain_value = solve_us = None
    if not args.no_plain:
        plain_ms, plain_value, solve_us = time_plain(H, gimgs, outs, params, bins, stream, args.plain_steps)
    diff_line = None
    if not args.no_plain and not args.no_diff:
        diff_line = time_diff(dev, 3, args.workers)

    cpu = None
    if args.cpu_budget > 0:
        cpu = cpu_baseline(imgs, bits, args.cpu_budget)

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8" if bits == 8 else "u16",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "form": "batched: one persistent launch per step, replayed from a captured HIP graph",
            "images": len(gimgs),
            "pixels": npix,
            "bins": bins,
            "iters": 50,
            "schedule": {"tile_steps": sched[0], "wg_per_cu": sched[1], "remap_steps": sched[2]},
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": measured_traffic(args.workload, bits),
            "kernel": f"k_batch<{bits}> (graph: descriptor copy + persistent kernel)",
            "alg_bytes_per_launch": alg_bytes,
            "avg_launch_us": round(avg_launch_s * 1e6, 2),
        },
        "plain": None if plain_ms is None else {
            "value": round(plain_value, 1), "unit": "Mpix/s", "ms_per_step": round(plain_ms, 3),
            "batched_over_plain": round(value / plain_value, 3),
            "form": "one image per call: hr_build_hist, hr_solve, hr_match launched per image"},
        "solve_us_per_image": None if solve_us is None else round(solve_us, 1),
        "differentiated": diff_line,
        "gen_seconds": round(gen_s, 1),
        "device_warmup_calls": n_w,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ws.close()


if __name__ == "__main__":
    main()
