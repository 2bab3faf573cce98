"""Pins of the histogram-matching LUT and the pixel remap (end of Sec. III-C)
against closed forms and exact integer arithmetic."""

from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from synthetic import make_image, config_seed


def _hist(seed, bits=8, H=40, W=52):
    img = make_image(config_seed(1, 8, seed), H, W, bits=bits)
    return img, O.count_histogram(O.value_channel(img), 1 << bits)


@pytest.mark.parametrize("bits", [8, 10])
def test_self_match_is_identity(bits):
    img, hS = _hist(0, bits)
    lut, margin = O.matching_lut(hS, hS.astype(np.float64))
    occ = hS > 0
    assert np.array_equal(lut[occ], np.nonzero(occ)[0])


@pytest.mark.parametrize("bits", [8, 10])
def test_uniform_target_closed_form(bits):
    """Uniform target: F~(k) = (k+1)/l, so LUT[v] = ceil(l u(v)) - 1 with the
    mid-rank u(v) = (F_S(v-1) + F_S(v))/2 -- an equalisation map (cf. Eq. 5)."""
    img, hS = _hist(1, bits)
    levels = 1 << bits
    N = int(hS.sum())
    lut, margin = O.matching_lut(hS, np.ones(levels))
    cS = np.cumsum(hS)
    for v in np.nonzero(hS)[0]:
        u = Fraction(int(cS[v] - hS[v] + cS[v]), 2 * N)
        x = levels * u
        k = max(0, -(-x.numerator // x.denominator) - 1)
        if x.denominator == 1:
            continue  # exact tie between two levels: either side is a valid reading
        assert lut[v] == k, v


def test_lut_monotone_and_in_range():
    for seed in range(4):
        img, hS = _hist(seed)
        rng = np.random.default_rng(seed)
        target = rng.random(256) * (rng.random(256) < 0.5)
        target[10] += 1.0
        lut, _ = O.matching_lut(hS, target)
        assert np.all(np.diff(lut) >= 0) and lut.min() >= 0 and lut.max() <= 255
        # only levels carrying target mass are ever produced for occupied levels
        assert np.all(target[lut[hS > 0]] > 0)


def test_margin_certifies_decisions():
    img, hS = _hist(2)
    rng = np.random.default_rng(9)
    target = rng.random(256)
    lut, margin = O.matching_lut(hS, target)
    N = hS.sum()
    cS = np.cumsum(hS)
    Ft = np.cumsum(target) / np.cumsum(target)[-1]
    for v in np.nonzero(hS)[0]:
        u = (cS[v] - hS[v] + cS[v]) / (2 * N)
        k = lut[v]
        assert Ft[k] - u >= margin[v] - 1e-15
        if k > 0:
            assert u - Ft[k - 1] >= margin[v] - 1e-15 and u > Ft[k - 1]


@pytest.mark.parametrize("bits", [8, 10])
def test_remap_value_channel_is_lut(bits):
    levels = 1 << bits
    img, hS = _hist(3, bits)
    rng = np.random.default_rng(bits)
    lut = np.sort(rng.integers(0, levels, size=levels))
    out = O.remap(img, lut)
    V = img.max(axis=2).astype(np.int64)
    Vo = out.max(axis=2).astype(np.int64)
    assert np.array_equal(Vo, lut[V])
    X = img.astype(np.int64)
    Y = out.astype(np.int64)
    assert np.all(Y <= lut[V][..., None])
    # channel order is preserved
    for c0, c1 in ((0, 1), (1, 2), (0, 2)):
        assert np.all((X[..., c0] <= X[..., c1]) <= (Y[..., c0] <= Y[..., c1]))


def test_remap_exact_rounding_and_black():
    img = np.array([[[0, 0, 0], [10, 5, 3], [7, 7, 1]]], np.uint8)
    lut = np.arange(256)
    lut[0] = 4
    lut[10] = 25
    lut[7] = 9
    out = O.remap(img, lut)
    # 5 * 25 / 10 = 12.5 -> 13 ; 3 * 25 / 10 = 7.5 -> 8 ; 1 * 9 / 7 = 1.29 -> 1
    assert out.tolist() == [[[4, 4, 4], [25, 13, 8], [9, 9, 1]]]


def test_enhance_end_to_end_brightens():
    img = make_image(config_seed(1, 1, 0), 96, 80)
    res = O.enhance(img, O.Params(iters=10))
    assert res["out"].mean() > 1.5 * img.mean()
    assert res["out"].shape == img.shape and res["out"].dtype == img.dtype
