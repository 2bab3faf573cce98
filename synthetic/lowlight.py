"""Seeded synthetic low-light images standing in for the paper's datasets.

The paper evaluates on MEF, NPE, LOL, LSRW and ExDark photographs (Sec. IV),
none of which is available here.  These images mimic their structure instead:
a colour reflectance made of flat 16x16 patches with fine texture, a smooth
dim illumination built from Gaussian blobs, and Poisson-Gaussian sensor noise,
quantised to 8-bit or 10-bit HWC RGB.

Recipe (one image, all randomness from one numpy PCG64 stream):
  reflectance  rho = clip(P + N(0, 0.02^2), 0, 1), P constant per 16x16 patch
               and channel, P ~ U[0.2, 1]
  illumination L = affine rescale of sum_{k<4} A_k exp(-|x - c_k|^2 / (2 s_k^2))
               to [floor, ceil]; c_k ~ U(image), s_k ~ U[0.15, 0.5] * min(H, W),
               A_k ~ U[0.5, 1]
  signal       x = rho * L (L broadcast over channels)
  noise        y = a * Poisson(x / a) + N(0, sigma^2), a = 1/255, sigma = 2/255
  quantise     q = clip(rint(y * (2^bits - 1)), 0, 2^bits - 1)
"""

from __future__ import annotations

import numpy as np

BASE_SEED = 2510211000
PATCH = 16
POISSON_GAIN = 1.0 / 255.0
READ_SIGMA = 2.0 / 255.0


def config_seed(config_index: int, n: int, i: int) -> np.random.SeedSequence:
    """Seed of image ``i`` of ``n`` in workload ``config_index``."""
    return np.random.SeedSequence(BASE_SEED + config_index).spawn(n)[i]


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.Generator):
        return seed
    if isinstance(seed, np.random.SeedSequence):
        return np.random.Generator(np.random.PCG64(seed))
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(int(seed))))


def make_image(seed, height: int, width: int, bits: int = 8, ceil: float = 0.3,
               floor: float | None = None, return_truth: bool = False):
    """Return an (H, W, 3) uint8 (bits=8) or uint16 (bits=10) low-light image.

    With ``return_truth`` also returns the float32 reflectance (H, W, 3) in [0, 1].
    ``floor`` defaults to 0.05 when ceil >= 0.3 and to ceil / 6 otherwise, so the
    ratio between the darkest and brightest illumination stays that of the
    0.05..0.3 default.
    """
    if bits not in (8, 10):
        raise ValueError("bits must be 8 or 10")
    if height <= 0 or width <= 0:
        raise ValueError("image must be non-empty")
    if floor is None:
        floor = 0.05 if ceil >= 0.3 else ceil / 6.0
    rng = _rng(seed)
    H, W = int(height), int(width)

    # reflectance: flat patches + texture
    ph, pw = -(-H // PATCH), -(-W // PATCH)
    patches = rng.uniform(0.2, 1.0, size=(ph, pw, 3)).astype(np.float32)
    rho = np.repeat(np.repeat(patches, PATCH, axis=0), PATCH, axis=1)[:H, :W, :]
    rho = rho + rng.standard_normal(size=(H, W, 3), dtype=np.float32) * np.float32(0.02)
    np.clip(rho, 0.0, 1.0, out=rho)

    # illumination: 4 separable Gaussian blobs, rescaled to [floor, ceil]
    ys = np.arange(H, dtype=np.float64)
    xs = np.arange(W, dtype=np.float64)
    illum = np.zeros((H, W), dtype=np.float64)
    m = min(H, W)
    for _ in range(4):
        cy = rng.uniform(0, H)
        cx = rng.uniform(0, W)
        s = rng.uniform(0.15, 0.5) * m
        amp = rng.uniform(0.5, 1.0)
        gy = np.exp(-((ys - cy) ** 2) / (2 * s * s))
        gx = np.exp(-((xs - cx) ** 2) / (2 * s * s))
        illum += amp * np.outer(gy, gx)
    lo, hi = illum.min(), illum.max()
    if hi > lo:
        illum = floor + (ceil - floor) * (illum - lo) / (hi - lo)
    else:
        illum = np.full_like(illum, 0.5 * (floor + ceil))
    illum = illum.astype(np.float32)

    x = rho * illum[:, :, None]
    lam = x.astype(np.float64) * (1.0 / POISSON_GAIN)
    y = rng.poisson(lam).astype(np.float32) * np.float32(POISSON_GAIN)
    del lam
    y += rng.standard_normal(size=y.shape, dtype=np.float32) * np.float32(READ_SIGMA)
    top = (1 << bits) - 1
    q = np.rint(y * np.float32(top))
    np.clip(q, 0, top, out=q)
    img = q.astype(np.uint8 if bits == 8 else np.uint16)
    if return_truth:
        return img, rho
    return img


def make_batch_shapes(seed, n: int, wmin: int = 640, wmax: int = 4000,
                      hmin: int = 480, hmax: int = 3000):
    """Independent uniform integer widths and heights (uneven aspect ratios)."""
    rng = _rng(seed)
    ws = rng.integers(wmin, wmax + 1, size=n)
    hs = rng.integers(hmin, hmax + 1, size=n)
    return [(int(h), int(w)) for h, w in zip(hs, ws)]


def edge_images(bits: int = 8):
    """Hand-built degenerate images: name -> (H, W, 3) array."""
    top = (1 << bits) - 1
    dt = np.uint8 if bits == 8 else np.uint16
    out = {}
    out["black"] = np.zeros((7, 9, 3), dt)
    out["white"] = np.full((5, 6, 3), top, dt)
    out["constant"] = np.full((4, 11, 3), top // 3, dt)
    two = np.zeros((6, 6, 3), dt)
    two[:, 3:, :] = top // 2
    out["two_level"] = two
    cb = np.zeros((8, 8, 3), dt)
    cb[(np.add.outer(np.arange(8), np.arange(8)) % 2) == 1] = top
    out["checkerboard"] = cb
    sp = np.zeros((9, 13, 3), dt)
    sp[4, 6, :] = (top, top // 2, 1)
    out["single_bright"] = sp
    out["one_pixel"] = np.array([[[3, 1, 2]]], dt)
    rng = np.random.default_rng(7)
    out["one_row"] = rng.integers(0, top + 1, size=(1, 37, 3)).astype(dt)
    out["one_col"] = rng.integers(0, top + 1, size=(29, 1, 3)).astype(dt)
    out["odd_width"] = rng.integers(0, top // 4, size=(13, 31, 3)).astype(dt)
    return out
