"""Pins of the oracle's pixel front end and histograms (Sec. II, Eq. 3,
Alg. 1 initialisation) against brute-force loops on tiny images."""

from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle as O
from synthetic import edge_images, make_image, config_seed


def brute_histograms(img, levels):
    H, W, _ = img.shape
    V = [[max(int(img[y, x, c]) for c in range(3)) for x in range(W)] for y in range(H)]
    hS = [0] * levels
    raw = [0] * (2 * levels - 1)
    for y in range(H):
        for x in range(W):
            hS[V[y][x]] += 1
            right = V[y][x + 1] if x + 1 < W else V[y][x]
            down = V[y + 1][x] if y + 1 < H else V[y][x]
            raw[abs(right - V[y][x]) + abs(down - V[y][x])] += 1
    gmax = max(j for j in range(len(raw)) if raw[j])
    hG = [0] * levels
    for j, n in enumerate(raw):
        if not n:
            continue
        if gmax == 0:
            hG[0] += n
            continue
        q = Fraction(j * (levels - 1), gmax) + Fraction(1, 2)
        hG[q.numerator // q.denominator] += n  # round half up, exact
    return V, hS, raw, gmax, hG


@settings(max_examples=60, deadline=None)
@given(st.integers(1, 8), st.integers(1, 8), st.sampled_from([4, 8, 16]), st.integers(0, 2**31 - 1))
def test_histograms_brute_force(H, W, levels, seed):
    rng = np.random.default_rng(seed)
    img = rng.integers(0, levels, size=(H, W, 3)).astype(np.uint8)
    V, hS, raw, gmax, hG = brute_histograms(img, levels)
    Vo = O.value_channel(img)
    assert Vo.tolist() == V
    assert O.count_histogram(Vo, levels).tolist() == hS
    r, gm, hg = O.gradient_histogram(Vo, levels)
    assert r.tolist() == raw and gm == gmax and hg.tolist() == hG
    assert sum(hS) == sum(hG) == H * W


@pytest.mark.parametrize("bits", [8, 10])
def test_edge_images(bits):
    levels = 1 << bits
    for name, img in edge_images(bits).items():
        V, hS, raw, gmax, hG = brute_histograms(img, levels)
        Vo = O.value_channel(img)
        assert O.count_histogram(Vo, levels).tolist() == hS, name
        r, gm, hg = O.gradient_histogram(Vo, levels)
        assert r.tolist() == raw and gm == gmax and hg.tolist() == hG, name


def test_constant_image_gradient_is_all_zero():
    img = np.full((5, 7, 3), 9, np.uint8)
    r, gm, hg = O.gradient_histogram(O.value_channel(img), 256)
    assert gm == 0 and hg[0] == 35 and hg[1:].sum() == 0


def test_gradient_rebin_puts_max_on_top_level():
    rng = np.random.default_rng(3)
    img = rng.integers(0, 40, size=(20, 30, 3)).astype(np.uint8)
    raw, gmax, hG = O.gradient_histogram(O.value_channel(img), 256)
    assert gmax > 0 and hG[255] == raw[gmax]


def test_generator_is_deterministic_and_low_light():
    a = make_image(config_seed(1, 1, 0), 64, 48)
    b = make_image(config_seed(1, 1, 0), 64, 48)
    c = make_image(config_seed(1, 2, 1), 64, 48)
    assert a.dtype == np.uint8 and a.shape == (64, 48, 3)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.max() < 160  # dim: illumination ceiling 0.3
    t = make_image(config_seed(4, 1, 0), 40, 50, bits=10)
    assert t.dtype == np.uint16 and t.max() <= 1023 and t.max() > 255
