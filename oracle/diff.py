"""FP64 reference of the differentiated form (not part of the paper).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

The exact pipeline is piecewise constant in the target histogram (the LUT is
an integer search), so the differentiated form replaces the LUT by a soft
matching map m(v): the piecewise-linear inverse of the normalised target CDF
F~ through the knots (k + 1/2, F~(k)), with F~(-1) = 0 at -1/2, evaluated at
the same mid-rank source CDF u(v) that the exact LUT uses.  For
F~(k-1) < u(v) <= F~(k), i.e. exactly where LUT[v] = k,

    m(v) = k - 1/2 + (u(v) - F~(k-1)) / (F~(k) - F~(k-1)),

so m(v) lies in (k - 1/2, k + 1/2] and rounds to LUT[v].  It is clamped to
[0, l-1].  The soft output keeps hue and saturation as the exact remap does,
out_c = c m(V) / (V (l-1)) in [0, 1] units (m(0) / (l-1) for black pixels),
and the loss is the mean over pixels and channels of (out_c - t_c)^2 against
a target image t.  The histograms H_C(S), H_C(grad S) and the classes are
integer constants; the gradient flows through the target histogram (Eq. 20)
into the K iterations of Eqs. (11)-(15) and their prior weights alpha, beta.
"""

from __future__ import annotations

import numpy as np

from .histretinex import (Params, classify, count_histogram, gradient_histogram, init_state, solve,
                          target_histogram, update_step, value_channel)


def source_cdf_midrank(hS) -> np.ndarray:
    """u(v) = (F_S(v-1) + F_S(v)) / 2, the mid-rank image CDF."""
    hS = np.asarray(hS, dtype=np.int64)
    cS = np.cumsum(hS)
    return (2 * cS - hS).astype(np.float64) / (2.0 * hS.sum())


def soft_map(hS, target):
    """m(v) for every level and the exact LUT it rounds to.

    Returns (m, lut, clamped): clamped marks levels whose m was cut to the
    range [0, l-1] (their derivative is 0)."""
    target = np.asarray(target, dtype=np.float64)
    levels = target.size
    u = source_cdf_midrank(hS)
    C = np.cumsum(target)
    Ft = C / C[-1]
    m = np.empty(levels)
    lut = np.empty(levels, dtype=np.int64)
    for v in range(levels):
        k = int(np.argmax(Ft >= u[v]))
        lo = Ft[k - 1] if k > 0 else 0.0
        lut[v] = k
        m[v] = k - 0.5 + (u[v] - lo) / (Ft[k] - lo)
    clamped = (m < 0.0) | (m > levels - 1)
    return np.clip(m, 0.0, levels - 1), lut, clamped


def soft_output(img: np.ndarray, m: np.ndarray) -> np.ndarray:
    """Continuous output in [0, 1] units: c m(V) / (V (l-1)), black -> m(0)/(l-1)."""
    levels = m.size
    X = img.astype(np.float64)
    V = img.max(axis=2).astype(np.int64)
    mv = m[V]
    out = np.empty_like(X)
    pos = V > 0
    out[pos] = X[pos] * (mv[pos] / (V[pos] * (levels - 1)))[:, None]
    out[~pos] = (mv[~pos] / (levels - 1))[:, None]
    return out


def soft_loss(img: np.ndarray, target_img: np.ndarray, m: np.ndarray) -> float:
    """Mean over pixels and channels of (out - t)^2."""
    d = soft_output(img, m) - np.asarray(target_img, dtype=np.float64)
    return float((d * d).mean())


def solve_with_checkpoints(hS, hG, params: Params, every: int):
    """Alg. 1 for params.iters passes; returns (l, r, checkpoints) where the
    checkpoints are the (l, r) pairs at t = 0, every, 2 every, ... and at the
    end when params.iters is a multiple of every."""
    idx = classify(int(params.bins))
    s, g, lv, rv = init_state(hS, hG)
    ckpt = []
    for t in range(int(params.iters)):
        if t % every == 0:
            ckpt.append((lv.copy(), rv.copy()))
        step = update_step(lv, rv, s, g, idx, params.alpha, params.beta)
        lv, rv = step["l"], step["r"]
    if int(params.iters) % every == 0:
        ckpt.append((lv.copy(), rv.copy()))
    return lv, rv, ckpt


def forward(img: np.ndarray, target_img: np.ndarray, params: Params, target_override=None):
    """The differentiated form's forward pass for one image (FP64).

    target_override replaces the target histogram of Eq. (20) (to probe the
    matching part on its own).  Returns a dict with the loss and every
    intermediate."""
    levels = int(params.bins)
    V = value_channel(img)
    npix = V.size
    hS = count_histogram(V, levels)
    _, _, hG = gradient_histogram(V, levels)
    lv, rv, _ = solve(hS, hG, params)
    target = target_histogram(lv, rv, npix, params.gamma) if target_override is None else \
        np.asarray(target_override, dtype=np.float64)
    m, lut, clamped = soft_map(hS, target)
    return {"loss": soft_loss(img, target_img, m), "hS": hS, "hG": hG, "l": lv, "r": rv,
            "target": target, "m": m, "lut": lut, "clamped": clamped}


def near_kink(hS, target, tol: float = 1e-9) -> np.ndarray:
    """Levels k whose CDF knot F~(k) lies within tol of some u(v): moving h~
    there can change the piecewise-linear branch, so finite differences
    across it are not derivatives."""
    u = source_cdf_midrank(hS)[np.asarray(hS) > 0]
    C = np.cumsum(np.asarray(target, dtype=np.float64))
    Ft = C / C[-1]
    return np.array([np.abs(u - f).min() < tol for f in Ft])
