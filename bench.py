"""Benchmark of the HistRetinex histogram pipeline on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ragged64|uhd16|single]

A step is one pass of the whole pipeline (histograms, solver, target, LUT,
remap) over one batch of synthetic low-light images that are already resident
in HBM.  The timed form is the batched persistent launch; the one-image form
(one launch sequence per image) is timed on the same batch for the
batched-vs-plain ratio.  Prints one JSON line: the headline workload
(ragged64 by default), and beside it the 10-bit workload (uhd16), the paper's
1000x664 single image, a gamma sweep with quality against the synthetic
ground truth, a resolution sweep, the differentiated form and the oracle on
the host cores.
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
        import multiprocessing as mp

        # spawn: the GPU is in use in this process by now
        with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
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
    import multiprocessing as mp

    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_gen, jobs))


def _oracle_init(bins: int, gamma: float):
    import oracle as O

    O.classify(bins)  # one-time tables, not timed
    O.classify_enhanced(bins, gamma)


def _oracle_enhance(args):
    import oracle as O

    img, bits = args
    t0 = time.perf_counter()
    O.enhance(img, O.Params(bins=1 << bits, iters=50))
    return time.perf_counter() - t0


def host_cpu() -> dict:
    """Host cores this process may use (at most 16, a one-GPU share), the CPU
    model and the numpy version."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cores": min(16, avail), "cpu_model": model, "numpy": np.__version__}


def cpu_baseline(imgs, bits, budget_s: float):
    """The FP64 oracle, as it is, on whole images of the workload: one core
    until about budget_s seconds of CPU time have been spent (smallest images
    first, at least one), then every image of the workload over a pool of P
    worker processes (one image per task; P = the host cores this process may
    use, at most 16)."""
    import multiprocessing as mp

    import oracle as O

    params = O.Params(bins=1 << bits, iters=50)
    _oracle_init(params.bins, params.gamma)
    order = sorted(range(len(imgs)), key=lambda i: imgs[i].shape[0] * imgs[i].shape[1])
    done_px, spent, used = 0, 0.0, []
    for i in order:
        spent += _oracle_enhance((imgs[i], bits))
        done_px += imgs[i].shape[0] * imgs[i].shape[1]
        used.append(i)
        if spent >= budget_s:
            break
    single = done_px / spent / 1e6
    host = host_cpu()
    P = host["cores"]
    pool_px = sum(x.shape[0] * x.shape[1] for x in imgs)
    # spawn: fresh interpreters, nothing of this process's GPU state
    with ProcessPoolExecutor(max_workers=P, mp_context=mp.get_context("spawn"), initializer=_oracle_init,
                             initargs=(params.bins, params.gamma)) as ex:
        list(ex.map(_oracle_enhance, [(imgs[order[0]], bits)] * P))  # workers up and warm
        t0 = time.perf_counter()
        list(ex.map(_oracle_enhance, [(imgs[i], bits) for i in sorted(order, key=lambda i: -imgs[i].size)]))
        pool_s = time.perf_counter() - t0
    pooled = pool_px / pool_s / 1e6
    return {
        "value": round(pooled, 2),
        "unit": "Mpix/s",
        "cores": P,
        "kind": "oracle",
        "sample": f"all {len(imgs)} images of the workload ({pool_px} pixels) over {P} worker processes, one "
                  f"image per task, {pool_s:.1f} s wall; numpy FP64, one thread per process",
        "single_core": {"value": round(single, 2), "unit": "Mpix/s", "cores": 1,
                        "sample": f"{len(used)} whole image(s), smallest first, {done_px} pixels, {spent:.1f} s"},
        "cpu_model": host["cpu_model"],
        "numpy": host["numpy"],
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


def to_dev(x, dev):
    import torch

    t = torch.from_numpy(x)
    if t.dtype == torch.uint16:
        t = t.view(torch.int16)
    return t.to(dev)


def time_batched(H, gimgs, outs, params, ws, steps: int, warmup: int, device_warmup_s: float):
    """Untimed device warm-up and `warmup` steps, then `steps` timed graph
    launches with HIP events on the launch stream.  Returns (wall ms per step,
    per-launch ms list, warm-up calls)."""
    import torch

    stream = torch.cuda.current_stream()
    # device warm-up before the warmup steps: a first process on an idle GPU
    # has been seen running several times slower for its first tens of ms
    t_w = time.perf_counter()
    n_w = 0
    while time.perf_counter() - t_w < device_warmup_s or n_w < 2:
        H.enhance_batch(gimgs, params, outs=outs, ws=ws)
        torch.cuda.synchronize()
        n_w += 1
    for _ in range(warmup):
        H.enhance_batch(gimgs, params, outs=outs, ws=ws)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(steps):
        starts[k].record(stream)
        H.enhance_batch(gimgs, params, outs=outs, ws=ws)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    launch_ms = [a.elapsed_time(b) for a, b in zip(starts, ends)]
    return wall * 1e3 / steps, launch_ms, n_w


def time_in_flight(H, gimgs, params, sched, bins, streams: int, steps: int):
    """Consecutive batches on `streams` streams, each with its own workspace
    and outputs (batch k on stream k mod streams): the tail of one launch
    (the last solves, while most CUs are idle) overlaps the next launch's
    histogram pass.  Returns (wall ms per batch, outputs of every stream equal)."""
    import torch

    wss = [H.Workspace(max_images=len(gimgs), max_bins=bins) for _ in range(streams)]
    for w in wss:
        w.set_schedule(*sched)
    outs = [[torch.empty_like(g) for g in gimgs] for _ in range(streams)]
    strs = [torch.cuda.Stream() for _ in range(streams)]
    torch.cuda.synchronize()
    for k in range(2 * streams):
        with torch.cuda.stream(strs[k % streams]):
            H.enhance_batch(gimgs, params, outs=outs[k % streams], ws=wss[k % streams])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        with torch.cuda.stream(strs[k % streams]):
            H.enhance_batch(gimgs, params, outs=outs[k % streams], ws=wss[k % streams])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    equal = all(torch.equal(a, b) for o in outs[1:] for a, b in zip(outs[0], o))
    for w in wss:
        w.close()
    del outs
    torch.cuda.empty_cache()
    return ms, equal


def batched_line(H, tune, name, imgs, bits, args, dev, with_plain: bool):
    """The batched form on one workload: Mpix/s, roofline of the persistent
    kernel, schedule; with_plain adds the one-image form and the solver alone."""
    import torch

    gimgs = [to_dev(x, dev) for x in imgs]
    outs = [torch.empty_like(g) for g in gimgs]
    npix = sum(g.shape[0] * g.shape[1] for g in gimgs)
    bins = 1 << bits
    esz = 1 if bits == 8 else 2
    alg_bytes = 9 * esz * npix  # read + re-read + write of 3 channels
    params = H.Params(bins=bins, iters=50)
    ws = H.Workspace(max_images=len(gimgs), max_bins=bins)
    sched = (args.tile_steps, args.wg_per_cu, args.remap_steps) if name == args.workload else (0, 0, 0)
    if sched == (0, 0, 0):
        sched = tune.lookup(args.schedule, bins, esz, npix, len(gimgs)) or (0, 0, 0)
    ws.set_schedule(*sched)
    ms_step, launch_ms, n_w = time_batched(H, gimgs, outs, params, ws, args.steps, args.warmup,
                                           args.device_warmup_s)
    avg_launch_s = float(np.mean(launch_ms)) * 1e-3
    achieved = alg_bytes / avg_launch_s / 1e9
    res = {
        "value": round(npix / (ms_step * 1e-3) / 1e6, 1),
        "unit": "Mpix/s",
        "ms_per_step": round(ms_step, 4),
        "images": len(gimgs),
        "pixels": npix,
        "bins": bins,
        "schedule": {"tile_steps": sched[0], "wg_per_cu": sched[1], "remap_steps": sched[2]},
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": measured_traffic(name, bits),
            "kernel": f"k_batch<{bits}> (persistent kernel; the descriptor copy only when the table changes)",
            "alg_bytes_per_launch": alg_bytes,
            "avg_launch_us": round(avg_launch_s * 1e6, 2),
        },
        "device_warmup_calls": n_w,
    }
    if args.in_flight > 1:
        fl_ms, fl_equal = time_in_flight(H, gimgs, params, sched, bins, args.in_flight, args.steps)
        res["in_flight"] = {"streams": args.in_flight, "ms_per_batch": round(fl_ms, 4),
                            "value": round(npix / (fl_ms * 1e-3) / 1e6, 1), "unit": "Mpix/s",
                            "over_one_stream": round(ms_step / fl_ms, 3), "outputs_equal": fl_equal,
                            "form": "consecutive batches on separate streams, workspaces and outputs"}
    if args.calibrate_copy_mb > 0 and name == args.workload:
        nbytes = args.calibrate_copy_mb << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if with_plain:
        stream = torch.cuda.current_stream()
        plain_ms, plain_value, solve_us = time_plain(H, gimgs, outs, params, bins, stream, args.plain_steps)
        res["plain"] = {"value": round(plain_value, 1), "unit": "Mpix/s", "ms_per_step": round(plain_ms, 3),
                        "batched_over_plain": round(res["value"] / plain_value, 3),
                        "form": "one image per call: hr_build_hist, hr_solve, hr_match launched per image"}
        res["solve_us_per_image"] = round(solve_us, 1)
    ws.close()
    del gimgs, outs
    torch.cuda.empty_cache()
    return res


PAPER_1000x664_S = 1.8645  # Table IV: the paper's time for one 1000x664 image (MATLAB, laptop CPU)
# Table V: the paper's time for one image resized to n x n, n = 100 .. 1000
PAPER_TABLE_V_S = {100: 1.6990, 200: 2.0995, 300: 1.6570, 400: 1.6803, 500: 1.6733, 600: 1.7376, 700: 1.7012,
                   800: 1.7344, 900: 1.7486, 1000: 1.6960}


def time_one_image(H, g, params, ws, reps: int):
    """The one-image form (three calls) and the batched form with n = 1 on
    one device image: ms per image each (HIP events, after a warm-up)."""
    import torch

    stream = torch.cuda.current_stream()
    out = torch.empty_like(g)
    npix = g.shape[0] * g.shape[1]

    def plain():
        hv, hg, _ = H.build_hist(g, ws)
        _, _, tg = H.solve(hv, hg, npix, params, ws)
        H.match(g, hv, tg, out=out, ws=ws)

    def batched():
        H.enhance_batch([g], params, outs=[out], ws=ws)

    res = {}
    for name, fn in (("plain_ms", plain), ("batched_ms", batched)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / reps
    return res


def single_line(H, img, dev):
    """The paper's quoted resolution: one 1000x664 8-bit image."""
    g = to_dev(img, dev)
    ws = H.Workspace(max_images=1, max_bins=256)
    t = time_one_image(H, g, H.Params(bins=256, iters=50), ws, 20)
    ws.close()
    npix = img.shape[0] * img.shape[1]
    return {
        "workload": "one 1000x664 RGB uint8 image, 256 bins, 50 iterations",
        "plain_ms": round(t["plain_ms"], 4),
        "plain_Mpix_per_s": round(npix / (t["plain_ms"] * 1e-3) / 1e6, 1),
        "batched_ms": round(t["batched_ms"], 4),
        "batched_Mpix_per_s": round(npix / (t["batched_ms"] * 1e-3) / 1e6, 1),
        "paper_s": PAPER_1000x664_S,
        "paper_Mpix_per_s": round(npix / PAPER_1000x664_S / 1e6, 3),
        "paper_context": "Table IV, MATLAB on an Intel i5-7300HQ laptop, at most 10 iterations: context only",
    }


def resolution_jobs():
    sizes = [(n, n) for n in range(100, 1001, 100)] + [(2160, 3840), (4320, 7680)]
    return sizes, [(2, len(sizes), i, h, w, 8, 0.3) for i, (h, w) in enumerate(sizes)]


def resolution_line(H, imgs, sizes, dev):
    """Table V analogue: the one-image form and the batched form (n = 1)
    against resolution, 100x100 .. 1000x1000 and 4K / 8K, 8-bit, 256 bins."""
    import torch

    ws = H.Workspace(max_images=1, max_bins=256)
    params = H.Params(bins=256, iters=50)
    rows = []
    for (h, w), img in zip(sizes, imgs):
        g = to_dev(img, dev)
        t = time_one_image(H, g, params, ws, 5)
        hv, hg, _ = H.build_hist(g, ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        stream = torch.cuda.current_stream()
        e0.record(stream)
        for _ in range(5):
            H.solve(hv, hg, h * w, params, ws)
        e1.record(stream)
        torch.cuda.synchronize()
        row = {"h": h, "w": w, "plain_ms": round(t["plain_ms"], 4), "batched_ms": round(t["batched_ms"], 4),
               "solve_us": round(e0.elapsed_time(e1) * 1e3 / 5, 1),
               "batched_Mpix_per_s": round(h * w / (t["batched_ms"] * 1e-3) / 1e6, 1)}
        if h == w and h in PAPER_TABLE_V_S:
            row["paper_s"] = PAPER_TABLE_V_S[h]
        rows.append(row)
        del g
    ws.close()
    return {"workload": "one RGB uint8 image per size from the single-image generator, 256 bins, 50 iterations",
            "rows": rows,
            "paper_context": "Table V: MATLAB on an Intel i5-7300HQ laptop, one image resized; context only"}


GAMMAS = (1.0, 1.5, 2.2, 5.0, 10.0)


def gamma_line(H, pairs, dev):
    """Table III analogue on synthetic ground truth: the batched form over 32
    images of 1000x664 at each gamma of Eq. (17); PSNR of the output against
    0.8 x the generator's reflectance (the pre-darkening image) and, for
    gamma = 1, against the input (the method then keeps the image nearly as
    it is)."""
    import torch

    imgs = [to_dev(a, dev) for a, _ in pairs]
    truth = [torch.from_numpy(t).to(dev) for _, t in pairs]
    outs = [torch.empty_like(g) for g in imgs]
    ws = H.Workspace(max_images=len(imgs), max_bins=256)
    stream = torch.cuda.current_stream()
    rows = []
    for gm in GAMMAS:
        params = H.Params(bins=256, iters=50, gamma=gm)
        for _ in range(2):
            H.enhance_batch(imgs, params, outs=outs, ws=ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            H.enhance_batch(imgs, params, outs=outs, ws=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        psnr_t, psnr_in = [], []
        for g, o, t in zip(imgs, outs, truth):
            of = o.float()
            mse_t = ((of - t * 255.0) ** 2).mean().item()
            mse_in = ((of - g.float()) ** 2).mean().item()
            psnr_t.append(10 * np.log10(255.0 ** 2 / mse_t))
            psnr_in.append(10 * np.log10(255.0 ** 2 / mse_in) if mse_in > 0 else float("inf"))
        rows.append({"gamma": gm, "ms_per_batch": round(ms, 4), "psnr_vs_truth_db": round(float(np.mean(psnr_t)), 3),
                     "psnr_vs_input_db": round(float(np.mean(psnr_in)), 3)})
    ws.close()
    return {"workload": "32 RGB uint8 1000x664 images of the differentiated-form generator, batched form, "
                        "256 bins, 50 iterations; truth = 0.8 x reflectance",
            "rows": rows,
            "paper_context": "Table III (one MEF image): PSNR falls as gamma grows, gamma = 1 nearly the input"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--workload", default="ragged64", choices=["ragged64", "uhd16", "single"])
    ap.add_argument("--cpu-budget", type=float, default=10.0, help="seconds of one-core oracle time (0 = skip)")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--tile-steps", type=int, default=0)
    ap.add_argument("--wg-per-cu", type=int, default=0)
    ap.add_argument("--remap-steps", type=int, default=0)
    ap.add_argument("--schedule", default=os.path.join(ROOT, "paper_2510_21100_amd", "schedule.json"))
    ap.add_argument("--in-flight", type=int, default=3,
                    help="also time consecutive batches on this many streams (0 or 1: skip)")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-image form and the solver timing")
    ap.add_argument("--no-diff", action="store_true", help="skip the differentiated-form timing")
    ap.add_argument("--no-extra", action="store_true",
                    help="time the headline workload only (no uhd16/single/sweep sub-objects)")
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

    extra = not args.no_extra
    desc, bits, jobs = workload(args.workload)
    t0 = time.perf_counter()
    imgs = generate(jobs, args.workers)
    gen_s = time.perf_counter() - t0

    import torch

    import paper_2510_21100_amd as H
    from paper_2510_21100_amd import tune

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    head = batched_line(H, tune, args.workload, imgs, bits, args, dev, with_plain=not args.no_plain)
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8" if bits == 8 else "u16",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "form": "batched: one persistent launch per step (a captured HIP graph with the descriptor copy when the table changes, the kernel alone when it repeats)",
            "images": head["images"],
            "pixels": head["pixels"],
            "bins": head["bins"],
            "iters": 50,
            "schedule": head["schedule"],
        },
        "roofline": head["roofline"],
        "plain": head.get("plain"),
        "solve_us_per_image": head.get("solve_us_per_image"),
    }
    if "in_flight" in head:
        line["in_flight"] = head["in_flight"]
    if extra and args.workload != "uhd16":
        d10, b10, j10 = workload("uhd16")
        u = batched_line(H, tune, "uhd16", generate(j10, args.workers), b10, args, dev, with_plain=not args.no_plain)
        u["workload"] = d10
        line["uhd16"] = u
    if extra:
        _, _, js = workload("single")
        line["single"] = single_line(H, generate(js, 1)[0], dev)
        sizes, jr = resolution_jobs()
        line["resolution_sweep"] = resolution_line(H, generate(jr, args.workers), sizes, dev)
        import multiprocessing as mp

        with ProcessPoolExecutor(max_workers=args.workers, mp_context=mp.get_context("spawn")) as ex:
            pairs = list(ex.map(_gen_truth, [(5, 32, i, 664, 1000) for i in range(32)]))
        line["gamma_sweep"] = gamma_line(H, pairs, dev)
        del pairs
    if not args.no_plain and not args.no_diff:
        line["differentiated"] = time_diff(dev, 3, args.workers)
    line["gen_seconds"] = round(gen_s, 1)
    line["device_warmup_calls"] = head["device_warmup_calls"]
    if args.cpu_budget > 0:
        line["cpu_baseline"] = cpu_baseline(imgs, bits, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
