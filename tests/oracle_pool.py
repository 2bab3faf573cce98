"""Oracle checks of whole images in worker processes (not a test module).

The GPU tests of the full-size workloads hand each image and its GPU results
to a spawn-context process pool; a worker runs the FP64 oracle on the image
and applies the parity contract.  Fresh
interpreters inherit nothing of the parent's GPU state.
"""

from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

import oracle as O
from gpu_cases import REL_TOL, lut_contract, pixel_contract, rel_err


def check_image(task):
    """task = (index, image, bits, out, lut, illum, refl, target); returns
    the parity figures of the image (raises on a contract failure)."""
    i, img, bits, out, lut, illum, refl, target = task
    ref = O.enhance(img, O.Params(bins=1 << bits))
    res = {"i": i, "npix": int(ref["npix"])}
    res["illum_err"] = rel_err(illum, ref["illum"])
    res["refl_err"] = rel_err(refl, ref["refl"])
    res["target_err"] = rel_err(target, ref["target"])
    assert res["illum_err"] <= REL_TOL, (i, res["illum_err"])
    assert res["refl_err"] <= REL_TOL, (i, res["refl_err"])
    res["near_ties"] = lut_contract(lut, ref)
    res["off_frac"] = pixel_contract(out, ref["out"])
    return res


def pool_size(bytes_per_worker: int) -> int:
    """Workers for the host: at most 16 (the CPU share of a one-GPU machine) and
    what the host memory holds at bytes_per_worker each."""
    n = min(16, os.cpu_count() or 1)
    try:
        avail = os.sysconf("SC_AVPHYS_PAGES") * os.sysconf("SC_PAGE_SIZE")
        n = max(1, min(n, int(avail * 0.6) // max(1, bytes_per_worker)))
    except (ValueError, OSError):
        pass
    return n


def check_all(tasks, bytes_per_worker: int):
    """Runs check_image over tasks in a spawn pool; returns the results in
    image order and prints one line per image as it ends."""
    res = []
    with mp.get_context("spawn").Pool(pool_size(bytes_per_worker), maxtasksperchild=4) as pool:
        for r in pool.imap_unordered(check_image, tasks):
            print(f"image {r['i']:3d}: {r['npix']:9d} px  illum {r['illum_err']:.2e}  refl {r['refl_err']:.2e}  "
                  f"target {r['target_err']:.2e}  near-tie levels {r['near_ties']}  pixels off {r['off_frac']:.2e}",
                  flush=True)
            res.append(r)
    return sorted(res, key=lambda r: r["i"])
