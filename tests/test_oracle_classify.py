"""Pins of the classification maps index(a,b) (Eqs. 7, 10) and index_1(a,b)
(Eqs. 17-19) against exact arithmetic."""

from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def exact_nearest(x: Fraction, levels: int) -> int:
    """argmin_k |x - k/(l-1)| in exact rationals, ties to the smaller k."""
    best, bestd = None, None
    for k in range(levels):
        d = abs(x - Fraction(k, levels - 1))
        if bestd is None or d < bestd:
            best, bestd = k, d
    return best


@pytest.mark.parametrize("levels", [2, 4, 8, 16])
def test_index_exact_rationals(levels):
    idx = O.classify(levels)
    for a in range(levels):
        for b in range(levels):
            x = Fraction(a, levels - 1) * Fraction(b, levels - 1)
            assert idx[a, b] == exact_nearest(x, levels)


@pytest.mark.parametrize("levels", [2, 4, 8, 16, 256, 1024])
def test_index_integer_form(levels):
    # nearest level of ab/(l-1)^2 on the grid k/(l-1) is round(ab/(l-1)); for odd
    # l-1 the quantity 2ab - (l-1)(2m+1) is odd, so there are no ties
    D = levels - 1
    a = np.arange(levels)[:, None]
    b = np.arange(levels)[None, :]
    expect = (2 * a * b + D) // (2 * D)
    assert np.array_equal(O.classify(levels), expect)
    assert np.all(np.abs(2 * a * b - D * (2 * expect + 1)) >= 1)


@pytest.mark.parametrize("levels", [4, 256])
def test_index_symmetric_and_bounded(levels):
    idx = O.classify(levels)
    assert np.array_equal(idx, idx.T)
    a = np.arange(levels)
    assert np.all(idx <= np.minimum.outer(a, a))
    assert np.array_equal(idx[-1], a)  # the top illumination level is the identity


def test_index1_gamma_one_equals_index():
    for levels in (16, 256):
        assert np.array_equal(O.classify_enhanced(levels, 1.0), O.classify(levels))


@pytest.mark.parametrize("levels,gamma", [(16, 2.2), (64, 1.5), (64, 5.0)])
def test_index1_high_precision(levels, gamma):
    getcontext().prec = 50
    idx1 = O.classify_enhanced(levels, gamma)
    D = Decimal(levels - 1)
    inv = Decimal(1) / Decimal(str(gamma))
    for a in range(levels):
        theta = (Decimal(a) / D) ** inv if a else Decimal(0)
        for b in range(levels):
            x = theta * Decimal(b)  # position in level units
            k = int((x + Decimal("0.5")).to_integral_value(rounding="ROUND_FLOOR"))
            assert idx1[a, b] == k, (a, b)


@pytest.mark.parametrize("levels", [256, 1024])
@pytest.mark.parametrize("gamma", [1.5, 2.2, 5.0, 10.0])
def test_index1_far_from_ties(levels, gamma):
    """The gamma-brightened products of the workloads never sit within 1e-9 of
    a rounding boundary, so an FP64 evaluation in any order decides every cell
    the same way."""
    D = levels - 1
    theta = (np.arange(levels) / D) ** (1.0 / gamma)
    x = np.outer(theta, np.arange(levels))
    frac = x - np.floor(x)
    inner = (np.arange(levels) > 0) & (np.arange(levels) < D)
    dist = np.abs(frac[inner][:, 1:] - 0.5)
    assert dist.min() > 1e-9
    idx1 = O.classify_enhanced(levels, gamma)
    assert np.array_equal(idx1, np.floor(x + 0.5).astype(np.int64))
