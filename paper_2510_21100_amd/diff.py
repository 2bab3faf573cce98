"""Differentiated form: gradients of a soft-matching enhancement loss with
respect to the prior weights alpha, beta and the target histogram h~.

Two autograd functions chain the HIP calls (argument marshalling only):

- ``TargetFn``: (alpha, beta) -> h~ per image.  Forward runs hr_solve_ckpt
  (K passes of Alg. 1 with the (L, R) checkpoints); backward runs
  hr_solve_vjp (Eq. 20 adjoint, then the passes in reverse, each checkpoint
  segment recomputed).
- ``SoftMatchLossFn``: h~ -> mean loss over the images.  Forward runs
  hr_softmatch_loss_grad, which also returns dLoss/dh~; backward scales it.

The histograms H_C(S), H_C(grad S) and the pixel data are constants.
"""

from __future__ import annotations

import ctypes as C
from typing import Sequence

import torch

from . import api
from ._lib import HrImage, check, lib

BINS = 256


def _ptr(t: torch.Tensor) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _params(alpha: float, beta: float, iters: int, gamma: float):
    return api.Params(bins=BINS, iters=iters, alpha=alpha, beta=beta, gamma=gamma, eps=0.0).c()


class TargetFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alpha, beta, hv, hg, iters: int, gamma: float, every: int, ws):
        n = hv.shape[0]
        ncp = iters // every + 1
        ckpt = torch.empty((n, ncp, 2, BINS), dtype=torch.float32, device=hv.device)
        target = torch.empty((n, BINS), dtype=torch.float32, device=hv.device)
        p = _params(float(alpha), float(beta), iters, gamma)
        check(lib.hr_solve_ckpt(_ptr(hv), _ptr(hg), n, C.byref(p), every, _ptr(ckpt), _ptr(target), ws.handle,
                                api._stream()))
        ctx.save_for_backward(hv, hg, ckpt)
        ctx.cfg = (float(alpha), float(beta), iters, gamma, every, ws)
        ctx.dtypes = (alpha.dtype, beta.dtype)
        return target

    @staticmethod
    def backward(ctx, g_target):
        hv, hg, ckpt = ctx.saved_tensors
        alpha, beta, iters, gamma, every, ws = ctx.cfg
        n = hv.shape[0]
        da = torch.empty(n, dtype=torch.float64, device=hv.device)
        db = torch.empty(n, dtype=torch.float64, device=hv.device)
        g = g_target.to(torch.float32).contiguous()
        p = _params(alpha, beta, iters, gamma)
        check(lib.hr_solve_vjp(_ptr(hv), _ptr(hg), n, C.byref(p), every, _ptr(ckpt), _ptr(g), _ptr(da), _ptr(db),
                               ws.handle, api._stream()))
        return da.sum().to(ctx.dtypes[0]), db.sum().to(ctx.dtypes[1]), None, None, None, None, None, None


class SoftMatchLossFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, target, hv, images, target_imgs, ws):
        n = len(images)
        arr_in = (HrImage * n)(*[api._image(x) for x in images])
        arr_t = (C.c_void_p * n)(*[t.data_ptr() for t in target_imgs])
        loss = torch.empty(n, dtype=torch.float64, device=target.device)
        dtarget = torch.empty((n, BINS), dtype=torch.float32, device=target.device)
        tg = target.to(torch.float32).contiguous()
        check(lib.hr_softmatch_loss_grad(arr_in, arr_t, n, _ptr(hv), _ptr(tg), _ptr(loss), _ptr(dtarget),
                                         ws.handle, api._stream()))
        ctx.save_for_backward(dtarget)
        ctx.n = n
        ctx.per_image = loss
        return loss.mean()

    @staticmethod
    def backward(ctx, g):
        (dtarget,) = ctx.saved_tensors
        return (dtarget * (g.to(torch.float32) / ctx.n)), None, None, None, None


def histograms(images: Sequence[torch.Tensor], ws: api.Workspace):
    """Stacked (n, 256) int32 H_C(S) and H_C(grad S) of 8-bit images (one launch)."""
    return api.build_hist_batch(list(images), ws)


def enhancement_loss(images: Sequence[torch.Tensor], target_imgs: Sequence[torch.Tensor], alpha: torch.Tensor,
                     beta: torch.Tensor, iters: int = 30, gamma: float = 2.2, ckpt_every: int = 5,
                     ws: api.Workspace | None = None):
    """Mean soft-matching loss of a batch of 8-bit images against FP32 HWC
    targets, differentiable in the scalar tensors alpha and beta.  Returns
    (loss, target): target is h~ (n, 256); call target.retain_grad() before
    backward to read dLoss/dh~."""
    if any(x.dtype != torch.uint8 for x in images):
        raise TypeError("the differentiated form takes 8-bit images")
    if len(images) != len(target_imgs):
        raise ValueError("one target image per image")
    for x, t in zip(images, target_imgs):
        if t.dtype != torch.float32 or tuple(t.shape) != tuple(x.shape) or not t.is_contiguous():
            raise ValueError("target images must be contiguous float32 tensors of the image's shape")
        if not (x.is_cuda and t.is_cuda):
            raise ValueError("images and target images must be on the GPU")
    ws = ws or api.workspace(max_images=len(images))
    hv, hg = histograms(images, ws)
    target = TargetFn.apply(alpha, beta, hv, hg, iters, gamma, ckpt_every, ws)
    loss = SoftMatchLossFn.apply(target, hv, list(images), list(target_imgs), ws)
    return loss, target
