"""Shared helpers of the GPU parity tests (not a test module)."""

from __future__ import annotations

import numpy as np
import torch

import oracle as O
from synthetic import config_seed, make_image

# Tolerances.  Histograms, counts and index maps are integers and must match
# exactly.  The FP32 solver must stay within 1e-5 (infinity-norm relative) of
# the FP64 oracle.  LUT entries must match wherever the oracle's decision is
# at least TAU away from a flip; pixels may differ by one level on at most
# 0.1 % of an image and never by more.
REL_TOL = 1e-5
TAU = 1e-5
PIX_FRAC = 1e-3


def to_gpu(img: np.ndarray) -> torch.Tensor:
    t = torch.from_numpy(np.ascontiguousarray(img))
    if t.dtype == torch.uint16:
        t = t.view(torch.int16)
    return t.cuda()


def to_np(t: torch.Tensor) -> np.ndarray:
    a = t.cpu()
    if a.dtype == torch.int16:
        a = a.view(torch.uint16)
    return a.numpy()


def padded_gpu(img: np.ndarray, pad_elems: int, offset_bytes: int = 0) -> torch.Tensor:
    """The image with rows pad_elems elements longer than 3W and, optionally,
    a base offset in bytes from a 16-byte aligned allocation: exercises the
    strided (non-vector) path."""
    H, W, _ = img.shape
    es = img.dtype.itemsize
    row = 3 * W + pad_elems
    assert offset_bytes % es == 0
    off = offset_bytes // es
    buf = np.zeros(off + H * row + 16, dtype=img.dtype)
    view = np.lib.stride_tricks.as_strided(buf[off:], shape=(H, W, 3), strides=(row * es, 3 * es, es))
    view[...] = img
    tb = torch.from_numpy(buf)
    if tb.dtype == torch.uint16:
        tb = tb.view(torch.int16)
    tb = tb.cuda()
    return torch.as_strided(tb, (H, W, 3), (row, 3, 1), storage_offset=off)


def rel_err(x, ref) -> float:
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.abs(x - ref).max() / np.abs(ref).max())


def lut_contract(lut_gpu, ref):
    """LUT equal wherever the oracle's margin >= TAU, off by <= 1 elsewhere
    (occupied levels only).  Returns the number of near-tie levels."""
    occ = ref["hS"] > 0
    lut_gpu = np.asarray(lut_gpu, np.int64)
    diff = np.abs(lut_gpu - ref["lut"])
    sure = occ & (ref["margin"] >= TAU)
    assert np.array_equal(lut_gpu[sure], ref["lut"][sure]), np.nonzero(sure & (diff > 0))[0]
    assert diff[occ].max(initial=0) <= 1
    return int((occ & ~sure).sum())


def pixel_contract(out_gpu: np.ndarray, out_ref: np.ndarray):
    d = np.abs(out_gpu.astype(np.int64) - out_ref.astype(np.int64))
    off = (d.max(axis=2) > 0).mean()
    assert d.max(initial=0) <= 1, d.max()
    assert off <= PIX_FRAC, off
    return float(off)


def cfg_image(cfg: int, H: int, W: int, i: int = 0, n: int = 1, bits: int = 8, ceil: float = 0.3):
    return make_image(config_seed(cfg, n, i), H, W, bits=bits, ceil=ceil)


def oracle_hists(img: np.ndarray, bins: int):
    V = O.value_channel(img)
    hS = O.count_histogram(V, bins)
    graw, gmax, hG = O.gradient_histogram(V, bins)
    return hS, graw, gmax, hG


def gpu_params(H, p: "O.Params"):
    """The library's Params for the oracle's: the same numbers, the readings
    as HR_VARIANT_* bits."""
    from paper_2510_21100_amd import _lib as L

    variant = 0
    variant |= {"fwd_l1": 0, "fwd_l2": L.HR_VARIANT_GRAD_L2, "sobel_l1": L.HR_VARIANT_GRAD_SOBEL}[p.grad_op]
    variant |= L.HR_VARIANT_GRAD_CLIP if p.grad_rescale == "clip" else 0
    variant |= L.HR_VARIANT_UPDATE_DIV if p.update == "div" else 0
    variant |= L.HR_VARIANT_INIT_UNIFORM if p.init_l == "uniform" else 0
    return H.Params(bins=p.bins, iters=p.iters, alpha=p.alpha, beta=p.beta, gamma=p.gamma, eps=p.eps,
                    variant=variant)
