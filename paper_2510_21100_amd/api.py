"""Torch-facing API of the HistRetinex library.

Tensors live on the ROCm device; torch provides the memory and the current
stream, the HIP library does all the work.  Images are (H, W, 3) tensors:
uint8 for 8-bit (256 levels), uint16 or int16 holding 0..1023 for 10-bit
(1024 levels).
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Sequence

import torch

from . import _lib
from ._lib import HrImage, HrParams, HrSchedule, check, lib


@dataclass(frozen=True)
class Params:
    """bins l, the maximum number of passes T, prior weights alpha, beta
    (Eq. 10), gamma (Eq. 17), the stopping threshold eps of Alg. 1 (the
    squared change of both normalised histograms in a pass; <= 0: exactly T
    passes) and the HR_VARIANT_* bits of other readings (0: the main path)."""

    bins: int = 256
    iters: int = 50
    alpha: float = 0.01
    beta: float = 0.01
    gamma: float = 2.2
    eps: float = 0.0
    variant: int = 0

    def c(self, variant: int | None = None) -> HrParams:
        v = self.variant if variant is None else variant
        return HrParams(self.bins, self.iters, self.alpha, self.beta, self.gamma, self.eps, v, 0)


def _bits_of(img: torch.Tensor) -> int:
    if img.dtype == torch.uint8:
        return 8
    if img.dtype in (torch.uint16, torch.int16):
        return 10
    raise TypeError("image dtype must be uint8 (8-bit) or uint16/int16 (10-bit)")


def _image(img: torch.Tensor) -> HrImage:
    if img.dim() != 3 or img.shape[2] != 3:
        raise ValueError("expected an (H, W, 3) image")
    if not img.is_cuda:
        raise ValueError("image must be on the GPU")
    if img.stride(2) != 1 or img.stride(1) != 3:
        raise ValueError("image pixels must be interleaved RGB (stride (row, 3, 1))")
    return HrImage(img.data_ptr(), img.shape[1], img.shape[0], img.stride(0) * img.element_size())


def _on_gpu(t: torch.Tensor, what: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{what} must be on the GPU")
    return t


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Workspace:
    """Device scratch, counters and cached launch graphs (one per stream)."""

    def __init__(self, max_images: int = 1, max_bins: int = 1024):
        h = C.c_void_p()
        check(lib.hr_workspace_create(max_images, max_bins, C.byref(h)))
        self.handle = h
        self.max_images = max_images
        self.max_bins = max_bins

    def set_schedule(self, tile_steps: int = 0, wg_per_cu: int = 0, remap_steps: int = 0) -> None:
        check(lib.hr_workspace_set_schedule(self.handle,
                                            C.byref(HrSchedule(tile_steps, wg_per_cu, remap_steps))))

    def flags(self, clear: bool = False) -> int:
        f = C.c_uint32()
        check(lib.hr_get_flags(self.handle, C.byref(f), int(clear)))
        return f.value

    def close(self) -> None:
        if self.handle:
            lib.hr_workspace_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ws: dict = {}


def workspace(max_images: int = 1, max_bins: int = 1024) -> Workspace:
    """A process-wide workspace for the current device with room for at least
    ``max_images`` images.  A smaller one it replaces is only dropped from the
    cache: whoever still holds it (a pending backward, say) keeps it alive, and
    it is freed with its last reference."""
    dev = torch.cuda.current_device()
    ws = _default_ws.get(dev)
    if ws is None or ws.max_images < max_images or ws.max_bins < max_bins:
        ws = Workspace(max(max_images, 1), max(max_bins, 1024))
        _default_ws[dev] = ws
    return ws


def build_hist(img: torch.Tensor, ws: Workspace | None = None, variant: int = 0):
    """Returns (hist_v, hist_grad, hist_grad_raw) as int32 tensors (counts).
    ``variant``: HR_VARIANT_GRAD_* bits (another gradient operator or
    rescaling, through hr_build_hist_variant)."""
    bits = _bits_of(img)
    bins = 1 << bits
    ws = ws or workspace()
    dev = img.device
    hv = torch.empty(bins, dtype=torch.int32, device=dev)
    hg = torch.empty(bins, dtype=torch.int32, device=dev)
    hraw = torch.empty(2 * bins - 1, dtype=torch.int32, device=dev)
    d = _image(img)
    if variant:
        check(lib.hr_build_hist_variant(C.byref(d), bits, variant, hv.data_ptr(), hg.data_ptr(), hraw.data_ptr(),
                                        ws.handle, _stream()))
    else:
        check(lib.hr_build_hist(C.byref(d), bits, hv.data_ptr(), hg.data_ptr(), hraw.data_ptr(), ws.handle,
                                _stream()))
    return hv, hg, hraw


def build_hist_batch(imgs: Sequence[torch.Tensor], ws: Workspace | None = None):
    """Histograms of n images (same bit depth) in one launch.  Returns
    (hist_v, hist_grad) as (n, bins) int32 tensors (counts)."""
    n = len(imgs)
    if n == 0:
        raise ValueError("empty batch")
    bits = _bits_of(imgs[0])
    if any(_bits_of(x) != bits for x in imgs):
        raise ValueError("all images of a batch must have the same bit depth")
    bins = 1 << bits
    ws = ws or workspace(max_images=n)
    dev = imgs[0].device
    hv = torch.empty((n, bins), dtype=torch.int32, device=dev)
    hg = torch.empty((n, bins), dtype=torch.int32, device=dev)
    arr = (HrImage * n)(*[_image(x) for x in imgs])
    check(lib.hr_build_hist_batch(arr, n, bits, hv.data_ptr(), hg.data_ptr(), ws.handle, _stream()))
    return hv, hg


def solve(hist_v: torch.Tensor, hist_grad: torch.Tensor, npix: int, params: Params = Params(),
          ws: Workspace | None = None, passes: torch.Tensor | None = None):
    """Returns (illum, refl, target) float32 histograms in counts.  ``passes``
    (a one-element int32 GPU tensor) receives the number of passes run."""
    ws = ws or workspace()
    bins = params.bins
    if hist_v.numel() != bins or hist_grad.numel() != bins:
        raise ValueError("histograms must have params.bins entries")
    if hist_v.dtype != torch.int32 or hist_grad.dtype != torch.int32:
        raise TypeError("histograms must be int32 tensors")
    _on_gpu(hist_v, "hist_v")
    _on_gpu(hist_grad, "hist_grad")
    dev = hist_v.device
    illum = torch.empty(bins, dtype=torch.float32, device=dev)
    refl = torch.empty(bins, dtype=torch.float32, device=dev)
    target = torch.empty(bins, dtype=torch.float32, device=dev)
    pp = None
    if passes is not None:
        if passes.dtype != torch.int32 or passes.numel() < 1:
            raise ValueError("passes must be an int32 tensor with at least one element")
        pp = _on_gpu(passes, "passes").data_ptr()
    p = params.c(params.variant & _lib.HR_VARIANT_SOLVE_BITS)
    check(lib.hr_solve(hist_v.contiguous().data_ptr(), hist_grad.contiguous().data_ptr(), int(npix), C.byref(p),
                       illum.data_ptr(), refl.data_ptr(), target.data_ptr(), pp, ws.handle, _stream()))
    return illum, refl, target


def match(img: torch.Tensor, hist_v: torch.Tensor, target: torch.Tensor, out: torch.Tensor | None = None,
          ws: Workspace | None = None):
    """Histogram-match ``img`` to ``target``; returns (out, lut)."""
    bits = _bits_of(img)
    bins = 1 << bits
    ws = ws or workspace()
    if hist_v.numel() != bins or target.numel() != bins:
        raise ValueError("histograms must have 2^bits entries")
    if target.dtype != torch.float32:
        raise TypeError("target must be float32")
    _on_gpu(hist_v, "hist_v")
    _on_gpu(target, "target")
    if out is None:
        out = torch.empty_like(img)
    if out.shape != img.shape or out.dtype != img.dtype:
        raise ValueError("out must match the image's shape and dtype")
    lut = torch.empty(bins, dtype=torch.int16, device=img.device)
    d = _image(img)
    od = _image(out)
    check(lib.hr_match(C.byref(d), bits, hist_v.contiguous().data_ptr(), target.contiguous().data_ptr(),
                       C.c_void_p(od.data), od.row_stride_bytes, lut.data_ptr(), ws.handle, _stream()))
    return out, lut


def equalize(img: torch.Tensor, hist_v: torch.Tensor | None = None, out: torch.Tensor | None = None,
             ws: Workspace | None = None):
    """Classical histogram equalisation of Eq. (5) through the same remap as
    match(); returns (out, lut)."""
    bits = _bits_of(img)
    bins = 1 << bits
    ws = ws or workspace()
    if hist_v is None:
        hist_v, _, _ = build_hist(img, ws)
    if hist_v.numel() != bins or hist_v.dtype != torch.int32:
        raise ValueError("hist_v must be an int32 histogram of 2^bits entries")
    _on_gpu(hist_v, "hist_v")
    if out is None:
        out = torch.empty_like(img)
    if out.shape != img.shape or out.dtype != img.dtype:
        raise ValueError("out must match the image's shape and dtype")
    lut = torch.empty(bins, dtype=torch.int16, device=img.device)
    d = _image(img)
    od = _image(out)
    check(lib.hr_equalize(C.byref(d), bits, hist_v.contiguous().data_ptr(), C.c_void_p(od.data), od.row_stride_bytes,
                          lut.data_ptr(), ws.handle, _stream()))
    return out, lut


def enhance(img: torch.Tensor, params: Params | None = None, ws: Workspace | None = None):
    """One image through the whole pipeline, one launch per stage.
    Returns (out, extras) with extras = dict of the intermediate histograms."""
    bits = _bits_of(img)
    params = params or Params(bins=1 << bits)
    if params.bins != 1 << bits:
        raise ValueError("params.bins must equal 2^bits of the image")
    hv, hg, hraw = build_hist(img, ws, params.variant & _lib.HR_VARIANT_GRAD_BITS)
    npix = img.shape[0] * img.shape[1]
    passes = torch.empty(1, dtype=torch.int32, device=img.device)
    illum, refl, target = solve(hv, hg, npix, params, ws, passes=passes)
    out, lut = match(img, hv, target, ws=ws)
    return out, {"hist_v": hv, "hist_grad": hg, "hist_grad_raw": hraw, "illum": illum, "refl": refl,
                 "target": target, "lut": lut, "passes": passes}


def enhance_batch(imgs: Sequence[torch.Tensor], params: Params | None = None,
                  outs: Sequence[torch.Tensor] | None = None, ws: Workspace | None = None,
                  extras: bool = False):
    """Many images of any sizes (same bit depth) in one persistent launch.
    Returns (outs, extras) where extras holds per-image LUTs and solver outputs
    (stacked (n, bins)) when ``extras`` is set, else None."""
    n = len(imgs)
    if n == 0:
        raise ValueError("empty batch")
    bits = _bits_of(imgs[0])
    if any(_bits_of(x) != bits for x in imgs):
        raise ValueError("all images of a batch must have the same bit depth")
    bins = 1 << bits
    params = params or Params(bins=bins)
    ws = ws or workspace(max_images=n)
    arr_in = (HrImage * n)(*[_image(x) for x in imgs])
    if outs is None:
        outs = [torch.empty_like(x) for x in imgs]
    if len(outs) != n:
        raise ValueError("one output per image")
    for x, o in zip(imgs, outs):
        _image(o)  # on the GPU, interleaved RGB rows
        if o.shape != x.shape or o.dtype != x.dtype:
            raise ValueError("each output must match its image's shape and dtype")
    arr_out = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
    arr_stride = (C.c_int64 * n)(*[o.stride(0) * o.element_size() for o in outs])
    ex = None
    ptrs = [None, None, None, None, None]
    if extras:
        dev = imgs[0].device
        ex = {"lut": torch.empty((n, bins), dtype=torch.int16, device=dev),
              "illum": torch.empty((n, bins), dtype=torch.float32, device=dev),
              "refl": torch.empty((n, bins), dtype=torch.float32, device=dev),
              "target": torch.empty((n, bins), dtype=torch.float32, device=dev),
              "passes": torch.empty(n, dtype=torch.int32, device=dev)}
        ptrs = [ex[k].data_ptr() for k in ("lut", "illum", "refl", "target", "passes")]
    p = params.c()
    check(lib.hr_enhance_batch(arr_in, arr_out, arr_stride, n, bits, C.byref(p), *ptrs, ws.handle, _stream()))
    return list(outs), ex


def enhance_batch_noalloc(imgs: Sequence[torch.Tensor], outs: Sequence[torch.Tensor], params: Params | None = None,
                          extras: dict | None = None, flags: torch.Tensor | None = None) -> None:
    """hr_enhance_batch_noalloc: up to HR_NOALLOC_MAX_IMAGES images through the
    batched pipeline without any device allocation by the library (its scratch
    is a fixed device array shared by every call on the GPU).  The caller
    provides the outputs: ``outs`` (one per image), optionally ``extras`` with
    any of the keys lut, illum, refl, target (n, bins) and passes (n), and
    ``flags`` (one int32/uint32 element that receives the sticky flags)."""
    n = len(imgs)
    if n == 0:
        raise ValueError("empty batch")
    bits = _bits_of(imgs[0])
    if any(_bits_of(x) != bits for x in imgs):
        raise ValueError("all images of a batch must have the same bit depth")
    bins = 1 << bits
    params = params or Params(bins=bins)
    if len(outs) != n:
        raise ValueError("one output per image")
    arr_in = (HrImage * n)(*[_image(x) for x in imgs])
    for x, o in zip(imgs, outs):
        _image(o)
        if o.shape != x.shape or o.dtype != x.dtype:
            raise ValueError("each output must match its image's shape and dtype")
    arr_out = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
    arr_stride = (C.c_int64 * n)(*[o.stride(0) * o.element_size() for o in outs])
    extras = extras or {}
    want = {"lut": ((n, bins), (torch.int16, torch.uint16)), "illum": ((n, bins), (torch.float32,)),
            "refl": ((n, bins), (torch.float32,)), "target": ((n, bins), (torch.float32,)),
            "passes": ((n,), (torch.int32,))}
    ptrs = []
    for k in ("lut", "illum", "refl", "target", "passes"):
        t = extras.get(k)
        if t is None:
            ptrs.append(None)
            continue
        shape, dtypes = want[k]
        if tuple(t.shape) != shape or t.dtype not in dtypes or not t.is_contiguous():
            raise ValueError(f"extras[{k!r}] must be a contiguous {shape} tensor of {dtypes[0]}")
        ptrs.append(_on_gpu(t, k).data_ptr())
    fp = None
    if flags is not None:
        if flags.numel() < 1 or flags.dtype not in (torch.int32, torch.uint32):
            raise ValueError("flags must be an int32 tensor with at least one element")
        fp = _on_gpu(flags, "flags").data_ptr()
    p = params.c()
    check(lib.hr_enhance_batch_noalloc(arr_in, arr_out, arr_stride, n, bits, C.byref(p), *ptrs, fp, _stream()))
