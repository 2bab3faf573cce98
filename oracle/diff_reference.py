"""Reference gradient of the differentiated form (FP64, torch autograd on CPU).

TEST INFRASTRUCTURE ONLY.  An independent, literal transcription of the
forward pass (it shares nothing with oracle.histretinex or oracle.diff, so
that they check each other): dense l x l count and weight matrices, the
arg-min classifications computed from the location products of Eqs. (7) and
(18), the updates of Eqs. (11)-(15) in Alg. 1 order, the scatter of Eq. (20),
then the soft matching map and the loss as defined in oracle.diff.  Autograd
through all of it gives dLoss/dalpha, dLoss/dbeta and dLoss/dh~.
"""

from __future__ import annotations

import functools

import numpy as np
import torch

F64 = torch.float64


@functools.lru_cache(maxsize=8)
def _argmin_classes(levels: int, gamma: float | None) -> torch.Tensor:
    """index(a, b) (gamma None) or index_1(a, b): nearest grid level k/(l-1)
    to the location product, ties to the smaller k (torch.argmin returns the
    first minimum).  Row blocks keep the l^3 comparison small."""
    k = torch.arange(levels, dtype=F64)
    grid = k / (levels - 1)
    rows = grid if gamma is None else grid ** (1.0 / gamma)
    out = torch.empty((levels, levels), dtype=torch.long)
    for a0 in range(0, levels, 64):
        loc = rows[a0:a0 + 64, None] * grid[None, :]
        out[a0:a0 + 64] = torch.argmin((loc[..., None] - grid).abs(), dim=-1)
    return out


def target_of(hS, hG, alpha, beta, gamma: float, iters: int) -> torch.Tensor:
    """h~ of Eq. (20) after `iters` passes of Alg. 1, as a differentiable
    function of the tensors alpha and beta."""
    hS = torch.as_tensor(np.asarray(hS), dtype=F64)
    hG = torch.as_tensor(np.asarray(hG), dtype=F64)
    levels = hS.numel()
    N = hS.sum()
    s, g = hS / N, hG / N
    L, R = s.clone(), g.clone()
    idx = _argmin_classes(levels, None)
    s_idx = s[idx]
    for _ in range(iters):
        C = L[:, None] * R[None, :]
        d = torch.zeros(levels, dtype=F64).index_add(0, idx.reshape(-1), C.reshape(-1))
        dcell = d[idx]
        K = torch.where(dcell > 0, C / torch.where(dcell > 0, dcell, torch.ones_like(dcell)),
                        torch.zeros_like(C))
        R1 = ((L[:, None] * K * s_idx).sum(0) + beta * g) / ((L * L).sum() + beta)
        L1 = ((R1[None, :] * K * s_idx).sum(1) + alpha * s) / ((R1 * R1).sum() + alpha)
        L, R = L1 / L1.sum(), R1 / R1.sum()
    idx1 = _argmin_classes(levels, float(gamma))
    CN = N * L[:, None] * R[None, :]
    return torch.zeros(levels, dtype=F64).index_add(0, idx1.reshape(-1), CN.reshape(-1))


def loss_of_target(target: torch.Tensor, hS, img: np.ndarray, target_img: np.ndarray) -> torch.Tensor:
    """Soft matching loss as a differentiable function of h~."""
    levels = target.numel()
    hS = torch.as_tensor(np.asarray(hS), dtype=F64)
    cS = torch.cumsum(hS, 0)
    u = (2 * cS - hS) / (2 * hS.sum())
    Ft = torch.cumsum(target, 0)
    Ft = Ft / Ft[-1]
    k = torch.searchsorted(Ft.detach(), u)  # first k with Ft[k] >= u
    k = k.clamp(max=levels - 1)
    lo = torch.where(k > 0, Ft[(k - 1).clamp(min=0)], torch.zeros_like(u))
    hi = Ft[k]
    m = (k.to(F64) - 0.5 + (u - lo) / (hi - lo)).clamp(0.0, levels - 1)
    X = torch.as_tensor(img.astype(np.float64))
    V = torch.as_tensor(img.max(axis=2).astype(np.int64))
    mv = m[V]
    Vf = V.to(F64)
    scale = torch.where(V > 0, mv / (torch.where(V > 0, Vf, torch.ones_like(Vf)) * (levels - 1)),
                        torch.zeros_like(mv))
    out = torch.where((V > 0)[..., None], X * scale[..., None], (mv / (levels - 1))[..., None].expand_as(X))
    t = torch.as_tensor(np.asarray(target_img, dtype=np.float64))
    return ((out - t) ** 2).mean()


def reference_gradients(img: np.ndarray, target_img: np.ndarray, hS, hG, alpha: float, beta: float,
                        gamma: float, iters: int):
    """loss, dloss/dalpha, dloss/dbeta, dloss/dh~ and h~ itself (FP64)."""
    a = torch.tensor(float(alpha), dtype=F64, requires_grad=True)
    b = torch.tensor(float(beta), dtype=F64, requires_grad=True)
    tgt = target_of(hS, hG, a, b, gamma, iters)
    tgt.retain_grad()
    loss = loss_of_target(tgt, hS, img, target_img)
    loss.backward()
    return {"loss": float(loss.detach()), "dalpha": float(a.grad), "dbeta": float(b.grad),
            "dtarget": tgt.grad.numpy().copy(), "target": tgt.detach().numpy().copy()}


def target_vjp(hS, hG, alpha: float, beta: float, gamma: float, iters: int, cotangent):
    """(d/dalpha, d/dbeta) of sum_k cotangent_k h~_k: the reverse pass of the
    solve alone for a given dLoss/dh~."""
    a = torch.tensor(float(alpha), dtype=F64, requires_grad=True)
    b = torch.tensor(float(beta), dtype=F64, requires_grad=True)
    tgt = target_of(hS, hG, a, b, gamma, iters)
    (tgt * torch.as_tensor(np.asarray(cotangent, dtype=np.float64))).sum().backward()
    return float(a.grad), float(b.grad)
