"""Pins of the oracle's stopping rule of Alg. 1 (at most T passes; earlier
once both normalised histograms change by at most eps in squared norm) and of
the classical equalisation map of Eq. (5)."""

from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from synthetic import config_seed, make_image

from test_oracle_bruteforce import _weights


def _hists(seed=0, H=64, W=48, bits=8, ceil=0.3):
    img = make_image(config_seed(1, 8, seed), H, W, bits=bits, ceil=ceil)
    V = O.value_channel(img)
    hS = O.count_histogram(V, 1 << bits)
    _, _, hG = O.gradient_histogram(V, 1 << bits)
    return hS, hG


def test_eps_zero_runs_exactly_T_passes():
    hS, hG = _hists(1)
    for T in (0, 1, 7, 40):
        lv, rv, info = O.solve(hS, hG, O.Params(iters=T, eps=0.0))
        assert info["passes"] == T and len(info["change_l"]) == T
        assert info["stop_margin"] == np.inf


def test_large_eps_stops_after_one_pass():
    # changes of unit-mass non-negative vectors are at most 2 in squared norm
    hS, hG = _hists(2)
    lv, rv, info = O.solve(hS, hG, O.Params(iters=50, eps=2.0))
    assert info["passes"] == 1
    l1, r1, _ = O.solve(hS, hG, O.Params(iters=1))
    assert np.array_equal(lv, l1) and np.array_equal(rv, r1)


@pytest.mark.parametrize("eps", [1e-4, 1e-5, 3e-6])
def test_stop_pass_is_the_first_pass_with_both_changes_small(eps):
    hS, hG = _hists(3)
    T = 60
    _, _, full = O.solve(hS, hG, O.Params(iters=T))
    cl, cr = np.array(full["change_l"]), np.array(full["change_r"])
    ok = np.nonzero((cl <= eps) & (cr <= eps))[0]
    expect = int(ok[0]) + 1 if ok.size and ok[0] + 1 < T else T
    lv, rv, info = O.solve(hS, hG, O.Params(iters=T, eps=eps))
    assert info["passes"] == expect
    # the early-exit state is the state after that many plain passes
    lp, rp, _ = O.solve(hS, hG, O.Params(iters=expect))
    assert np.array_equal(lv, lp) and np.array_equal(rv, rp)
    # the certified margin is the closest decision to eps among those taken
    q = np.maximum(cl, cr)[: min(expect, T - 1)]
    assert info["stop_margin"] == pytest.approx(np.min(np.abs(q - eps) / eps), rel=1e-12)


def _bruteforce_stop(hS, hG, T, alpha, beta, eps):
    n = len(hS)
    cls = [[(2 * a * b + (n - 1)) // (2 * (n - 1)) for b in range(n)] for a in range(n)]
    N = float(sum(hS))
    s = [x / N for x in hS]
    g = [x / N for x in hG]
    lv, rv = list(s), list(g)
    _, _, K = _weights(lv, rv, cls)
    passes = 0
    while passes < T:
        Sidx = [[s[cls[a][b]] for b in range(n)] for a in range(n)]
        den_r = sum(x * x for x in lv) + beta
        r_new = [(sum(lv[a] * K[a][b] * Sidx[a][b] for a in range(n)) + beta * g[b]) / den_r for b in range(n)]
        den_l = sum(x * x for x in r_new) + alpha
        l_new = [(sum(r_new[b] * K[a][b] * Sidx[a][b] for b in range(n)) + alpha * s[a]) / den_l for a in range(n)]
        r_n = [x / sum(r_new) for x in r_new]
        l_n = [x / sum(l_new) for x in l_new]
        dl = sum((x - y) ** 2 for x, y in zip(l_n, lv))
        dr = sum((x - y) ** 2 for x, y in zip(r_n, rv))
        lv, rv = l_n, r_n
        passes += 1
        _, _, K = _weights(lv, rv, cls)
        if dl <= eps and dr <= eps:
            break
    return passes, np.array(lv), np.array(rv)


@pytest.mark.parametrize("levels", [4, 8, 16])
def test_stop_matches_materialised_loops(levels):
    rng = np.random.default_rng(7 + levels)
    hS = rng.integers(0, 40, size=levels)
    hS[0] += 1
    N = int(hS.sum())
    hG = np.floor(rng.dirichlet(np.ones(levels)) * N).astype(np.int64)
    hG[0] += N - hG.sum()
    for eps in (1e-3, 1e-5, 1e-7):
        p_b, l_b, r_b = _bruteforce_stop(list(hS), list(hG), 80, 0.05, 0.02, eps)
        lv, rv, info = O.solve(hS, hG, O.Params(bins=levels, iters=80, alpha=0.05, beta=0.02, eps=eps))
        assert info["passes"] == p_b, eps
        assert np.abs(lv - l_b).max() <= 1e-13 and np.abs(rv - r_b).max() <= 1e-13


# --------------------------------------------------------------------------
# Eq. (5): classical equalisation
# --------------------------------------------------------------------------

def _he_exact(hS):
    """t_i = (l-1) sum_{j<=i} n_j / N rounded to the nearest integer (ties
    up), in exact rationals."""
    levels = len(hS)
    N = sum(hS)
    out, c = [], 0
    for i in range(levels):
        c += hS[i]
        t = Fraction((levels - 1) * c, N)
        out.append(int(t + Fraction(1, 2)))  # floor of a non-negative rational
    return out


@pytest.mark.parametrize("levels", [2, 4, 16, 256, 1024])
def test_equalization_lut_exact(levels):
    rng = np.random.default_rng(levels)
    for _ in range(5):
        hS = rng.integers(0, 9, size=levels)
        hS[rng.integers(0, levels)] += 1
        t = O.equalization_lut(hS)
        assert t.tolist() == _he_exact(hS.tolist())
        assert np.all(np.diff(t) >= 0) and t[-1] == levels - 1 and t.min() >= 0


def test_equalization_of_a_flat_histogram_and_a_two_level_image():
    # every level equally often: t_i = round((l-1)(i+1)/l)
    levels = 256
    t = O.equalization_lut(np.full(levels, 3))
    assert t.tolist() == [((2 * (levels - 1) * (i + 1) + levels) // (2 * levels)) for i in range(levels)]
    # two occupied levels holding a and b pixels: the lower one goes to
    # round((l-1) a / (a + b)), the upper one (and everything above) to l-1
    hS = np.zeros(levels, dtype=np.int64)
    hS[10], hS[40] = 3, 1
    t = O.equalization_lut(hS)
    assert t[10] == round(255 * 3 / 4) and t[40] == 255 and t[9] == 0 and t[255] == 255
