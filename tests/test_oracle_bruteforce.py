"""Brute-force pins of the oracle's objective and iteration, written with
plain Python loops over the cells of the l x l matrices (no numpy
vectorisation, no oracle helpers), for small level counts.

  * objective(): Eq. (10) with the weights of Eq. (11), in exact rational
    arithmetic, compared with the oracle's FP64 value;
  * solve(): Alg. 1 (Eq. 13, then Eq. 12 with the new unnormalised R, then
    Eqs. 15 and 14, then Eq. 11) with materialised count, class and K
    matrices held in nested lists, compared with the vectorised oracle.
"""

from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def _nearest(x, levels):
    """argmin_k |x - k/(l-1)| in exact rationals, ties to the smaller k."""
    best, bestd = 0, None
    for k in range(levels):
        d = abs(x - Fraction(k, levels - 1))
        if bestd is None or d < bestd:
            best, bestd = k, d
    return best


def _classes(levels):
    return [[_nearest(Fraction(a, levels - 1) * Fraction(b, levels - 1), levels) for b in range(levels)]
            for a in range(levels)]


def _weights(lv, rv, cls):
    n = len(lv)
    C = [[lv[a] * rv[b] for b in range(n)] for a in range(n)]
    d = [0 * lv[0]] * n
    for a in range(n):
        for b in range(n):
            d[cls[a][b]] = d[cls[a][b]] + C[a][b]
    K = [[(C[a][b] / d[cls[a][b]]) if d[cls[a][b]] != 0 else 0 * C[a][b] for b in range(n)] for a in range(n)]
    return C, d, K


def _J(lv, rv, K, s, g, cls, alpha, beta):
    n = len(lv)
    J = 0 * lv[0]
    for a in range(n):
        for b in range(n):
            J += (lv[a] * rv[b] - K[a][b] * s[cls[a][b]]) ** 2
    for a in range(n):
        J += alpha * (lv[a] - s[a]) ** 2
    for b in range(n):
        J += beta * (rv[b] - g[b]) ** 2
    return J


def _rational_hist(rng, levels, zeros):
    h = [int(x) for x in rng.integers(1, 50, size=levels)]
    for z in zeros:
        h[z] = 0
    tot = sum(h)
    return [Fraction(x, tot) for x in h], h


@pytest.mark.parametrize("levels", [2, 4, 8])
def test_objective_exact_rationals(levels):
    rng = np.random.default_rng(levels)
    cls = _classes(levels)
    s, _ = _rational_hist(rng, levels, [levels - 1])
    g, _ = _rational_hist(rng, levels, [1] if levels > 2 else [])
    lv, _ = _rational_hist(rng, levels, [0])
    rv, _ = _rational_hist(rng, levels, [])
    for K_from in ("own", "other"):
        # K from the same iterate, and K frozen from a different one
        src_l, src_r = (lv, rv) if K_from == "own" else (s, g)
        _, _, K = _weights(src_l, src_r, cls)
        alpha, beta = Fraction(3, 100), Fraction(7, 10)
        J_exact = _J(lv, rv, K, s, g, cls, alpha, beta)
        f = lambda v: np.array([float(x) for x in v])
        Kf = np.array([[float(x) for x in row] for row in K])
        J = O.objective(f(lv), f(rv), Kf, f(s), f(g), O.classify(levels), float(alpha), float(beta))
        assert J == pytest.approx(float(J_exact), rel=1e-13, abs=1e-16)


def _bruteforce_solve(hS, hG, iters, alpha, beta):
    n = len(hS)
    cls = [[(2 * a * b + (n - 1)) // (2 * (n - 1)) for b in range(n)] for a in range(n)]
    N = float(sum(hS))
    s = [x / N for x in hS]
    g = [x / N for x in hG]
    lv, rv = list(s), list(g)
    _, _, K = _weights(lv, rv, cls)
    for _ in range(iters):
        Sidx = [[s[cls[a][b]] for b in range(n)] for a in range(n)]
        den_r = sum(x * x for x in lv) + beta
        r_new = [(sum(lv[a] * K[a][b] * Sidx[a][b] for a in range(n)) + beta * g[b]) / den_r for b in range(n)]
        den_l = sum(x * x for x in r_new) + alpha
        l_new = [(sum(r_new[b] * K[a][b] * Sidx[a][b] for b in range(n)) + alpha * s[a]) / den_l for a in range(n)]
        sr, sl = sum(r_new), sum(l_new)
        rv = [x / sr for x in r_new]
        lv = [x / sl for x in l_new]
        _, _, K = _weights(lv, rv, cls)
    return np.array(lv), np.array(rv)


@pytest.mark.parametrize("levels", [2, 4, 8, 16])
@pytest.mark.parametrize("alpha,beta", [(0.01, 0.01), (1.0, 0.1)])
def test_solve_matches_materialised_loops(levels, alpha, beta):
    rng = np.random.default_rng(100 + levels)
    hS = rng.integers(0, 30, size=levels)
    hS[levels // 2] = 0
    hS[0] += 1
    N = int(hS.sum())
    # gradient histogram of the same mass with its own zero pattern
    hG = np.zeros(levels, dtype=np.int64)
    p = rng.dirichlet(np.ones(levels))
    hG += np.floor(p * N).astype(np.int64)
    hG[0] += N - hG.sum()
    hG[-1] = 0 if levels > 2 else hG[-1]
    hG[0] += N - hG.sum()
    lv_b, rv_b = _bruteforce_solve(list(hS), list(hG), 25, alpha, beta)
    lv, rv, _ = O.solve(hS, hG, O.Params(bins=levels, iters=25, alpha=alpha, beta=beta))
    assert np.abs(lv - lv_b).max() <= 1e-13
    assert np.abs(rv - rv_b).max() <= 1e-13
