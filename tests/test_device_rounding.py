"""The GPU solver never evaluates index(a, b) of Eq. (10) with integer
division in its hot loops: it uses FP32 shortcuts.  These tests emulate those
shortcuts bit for bit in numpy and compare them, for every level pair, with
the exact integer forms:

  * class of a cell in the dense sweeps: the product a * float32(b / (l-1)),
    plus 2^23, rounded once to FP32 (one fused multiply-add), whose low
    mantissa bits are then the class;
  * the run of reflectance levels of class m on illumination row a (class
    list, 1024-level class totals, reverse pass): the FP32 fused multiply-add
    float32((2m-1)(l-1)) * float32(1 / (2a)) + 1, rounded once and truncated,
    gives the lower bound E(m) = floor((2m-1)(l-1) / 2a) + 1 (capped at l);
    the FP32 product float32((2m+1)(l-1)) * float32(1 / (2a)), truncated,
    gives the upper bound floor((2m+1)(l-1) / 2a) (capped at l-1).

The exact references are integer arithmetic only (no oracle code).
"""

import numpy as np
import pytest


def _round_half_even_exact(x: np.ndarray) -> np.ndarray:
    # x holds exact values (products of small integers and float32 values,
    # at most 34 significant bits, exact in float64)
    return np.rint(x).astype(np.int64)


@pytest.mark.parametrize("levels", [256, 1024])
def test_dense_sweep_class_rounding_is_exact(levels):
    D = levels - 1
    a = np.arange(levels, dtype=np.float32)
    bq = np.arange(levels, dtype=np.float32) / np.float32(D)  # IEEE FP32 division
    assert bq.dtype == np.float32
    # fmaf(a, bq, 2^23): the exact product plus 2^23, rounded once to FP32.
    # Sums in [2^23, 2^24) are spaced 1 apart in FP32, so that rounding is
    # round-half-even of the exact product.  The product of a 10-bit integer
    # and a float32 is exact in float64.
    prod = np.multiply.outer(a.astype(np.float64), bq.astype(np.float64))
    assert np.all(prod < 2.0 ** 23)
    cls = _round_half_even_exact(prod)
    A = np.arange(levels, dtype=np.int64)[:, None]
    B = np.arange(levels, dtype=np.int64)[None, :]
    exact = (2 * A * B + D) // (2 * D)
    assert np.array_equal(cls, exact)
    # the FP32 product is never within 1e-4 of a rounding boundary (the
    # exact a b / (l-1) lies at least 1 / (2 (l-1)) from one)
    dist = np.abs(prod - np.floor(prod) - 0.5)
    assert dist.min() > 1e-4


def _fp32_run_bounds(levels: int, a: int, m: np.ndarray):
    """(E(m), upper(m)) as the device computes them for row a >= 1."""
    D = levels - 1
    inv = np.float32(1.0) / np.float32(2 * a)  # IEEE FP32 division
    lo_num = ((2 * m - 1) * D).astype(np.float32)  # exact: below 2^24
    hi_num = ((2 * m + 1) * D).astype(np.float32)
    # fmaf(lo_num, inv, 1): the exact product plus 1 (exact in float64: at most
    # 46 significant bits below 2^22), rounded once to FP32, then truncated
    lo_fma = (lo_num.astype(np.float64) * np.float64(inv) + 1.0).astype(np.float32)
    lo1 = np.floor(lo_fma.astype(np.float64)).astype(np.int64)  # truncation of a positive float
    hi = np.floor((hi_num * inv).astype(np.float64)).astype(np.int64)
    E = np.where(m == 0, 0, np.minimum(lo1, levels))
    upper = np.minimum(hi, levels - 1)
    return E, upper


@pytest.mark.parametrize("levels", [256, 1024])
def test_class_run_bounds_are_exact(levels):
    D = levels - 1
    for a in range(1, levels):
        m = np.arange(0, min(a + 6, levels + 1), dtype=np.int64)
        E, upper = _fp32_run_bounds(levels, a, m)
        E_exact = np.where(m == 0, 0, np.minimum(((2 * m - 1) * D) // (2 * a) + 1, levels))
        up_exact = np.minimum(((2 * m + 1) * D) // (2 * a), levels - 1)
        assert np.array_equal(E, E_exact), a
        mm = m[m <= a]
        assert np.array_equal(upper[: mm.size], up_exact[: mm.size]), a
        # classes above a: the run is empty at both ends (E = l)
        assert np.all(E[m > a] == levels), a


@pytest.mark.parametrize("levels", [256, 1024])
def test_run_bounds_reproduce_the_class_map(levels):
    """Rows cut into class runs by E(m) give back index(a, b) for every b."""
    D = levels - 1
    b = np.arange(levels, dtype=np.int64)
    for a in range(1, levels, 7 if levels == 1024 else 1):
        m = np.arange(0, a + 2, dtype=np.int64)
        E, _ = _fp32_run_bounds(levels, a, m)
        cls = np.searchsorted(E, b, side="right") - 1
        assert np.array_equal(cls, (2 * a * b + D) // (2 * D)), a


def test_uncapped_run_bounds_stay_in_the_padded_sums():
    """At 1024 levels the class totals read the running sums of R at E(m)
    without clamping to l: the sums repeat their total up to index
    7 (l-1) / 2 + 1.  Every bound a class group evaluates (classes
    4q .. 4q + 4 on the rows a >= max(4q, 1)) lies inside that range."""
    levels = 1024
    D = levels - 1
    rcum_len = 7 * D // 2 + 2
    worst = 0
    for a in range(1, levels):
        inv = np.float32(1.0) / np.float32(2 * a)
        q = np.arange(0, a // 4 + 1, dtype=np.int64)
        m = (4 * q[:, None] + np.arange(5, dtype=np.int64)[None, :]).ravel()
        m = m[m > 0]
        num = ((2 * m - 1) * D).astype(np.float32)
        e = np.floor((num.astype(np.float64) * np.float64(inv) + 1.0).astype(np.float32).astype(np.float64))
        worst = max(worst, int(e.max()))
    assert worst < rcum_len, worst
    assert worst == rcum_len - 1  # the padding is as long as it needs to be
