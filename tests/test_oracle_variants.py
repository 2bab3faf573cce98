"""Pins of the oracle's alternative readings (the variant switches), each
against an independent route: exact integer / decimal arithmetic, explicit
loops over the pixels and the l x l cells, and a two-level step worked by
hand.

  * gradient operators: fwd_l2 (rounded Euclidean magnitude of the forward
    differences) and sobel_l1 (3x3 Sobel, |gx| + |gy| over 4, rounded);
  * rescale "clip" of the gradient histogram;
  * the printed form of Eqs. (12)-(13) that divides by K ("div");
  * a uniform initial illumination histogram.
"""

from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

getcontext().prec = 50


def _round_sqrt_decimal(q: int) -> int:
    """The integer nearest to sqrt(q) (no ties: sqrt(q) = k + 1/2 needs
    q = k^2 + k + 1/4), by 50-digit decimal square roots."""
    r = Decimal(q).sqrt()
    k = int(r)
    return k + 1 if (r - k) > Decimal("0.5") else k


def _fwd_l2_loops(V):
    H, W = len(V), len(V[0])
    out = [[0] * W for _ in range(H)]
    for y in range(H):
        for x in range(W):
            dx = V[y][x + 1] - V[y][x] if x + 1 < W else 0
            dy = V[y + 1][x] - V[y][x] if y + 1 < H else 0
            out[y][x] = _round_sqrt_decimal(dx * dx + dy * dy)
    return out


SOBEL_X = ((-1, 0, 1), (-2, 0, 2), (-1, 0, 1))
SOBEL_Y = ((-1, -2, -1), (0, 0, 0), (1, 2, 1))


def _sobel_loops(V):
    H, W = len(V), len(V[0])
    out = [[0] * W for _ in range(H)]
    for y in range(H):
        for x in range(W):
            gx = gy = 0
            for i in range(3):
                for j in range(3):
                    yy = min(max(y + i - 1, 0), H - 1)
                    xx = min(max(x + j - 1, 0), W - 1)
                    gx += SOBEL_X[i][j] * V[yy][xx]
                    gy += SOBEL_Y[i][j] * V[yy][xx]
            m = Fraction(abs(gx) + abs(gy), 4)
            out[y][x] = int(m + Fraction(1, 2))  # floor(m + 1/2), m >= 0
    return out


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("levels", [16, 256, 1024])
def test_gradient_operators_match_loops(seed, levels):
    rng = np.random.default_rng(seed + levels)
    H, W = int(rng.integers(1, 9)), int(rng.integers(1, 9))
    V = rng.integers(0, levels, size=(H, W))
    Vl = V.tolist()
    assert O.gradient_magnitude(V, "fwd_l2").tolist() == _fwd_l2_loops(Vl)
    assert O.gradient_magnitude(V, "sobel_l1").tolist() == _sobel_loops(Vl)


def test_gradient_operator_special_values():
    # 3-4-5: a forward step of 3 along x and 4 along y
    V = np.array([[0, 3], [4, 4]])
    assert O.gradient_magnitude(V, "fwd_l2")[0, 0] == 5
    # |(1, 1)| = 1.41 -> 1, |(1, 2)| = 2.24 -> 2, |(2, 2)| = 2.83 -> 3
    for dx, dy, want in [(1, 1, 1), (1, 2, 2), (2, 2, 3), (0, 0, 0), (7, 0, 7)]:
        V = np.array([[0, dx], [dy, 0]])
        assert O.gradient_magnitude(V, "fwd_l2")[0, 0] == want
    # a vertical step edge of height h: Sobel gives h on both sides of the
    # edge and 0 elsewhere; a constant image gives 0 everywhere
    for h in (1, 5, 255, 1023):
        V = np.zeros((5, 8), dtype=np.int64)
        V[:, 4:] = h
        g = O.gradient_magnitude(V, "sobel_l1")
        assert (g[:, 3] == h).all() and (g[:, 4] == h).all()
        assert (g[:, [0, 1, 2, 5, 6, 7]] == 0).all()
    assert (O.gradient_magnitude(np.full((4, 4), 9), "sobel_l1") == 0).all()
    # the largest magnitudes stay within the 2l-1 raw levels
    for levels in (256, 1024):
        top = levels - 1
        V = np.array([[0, top], [top, 0]])
        assert O.gradient_magnitude(V, "fwd_l2").max() <= 2 * top
        V = np.zeros((3, 3), dtype=np.int64)
        V[0, 2] = V[1, 2] = V[2, 2] = top
        V[2, 0] = V[2, 1] = top
        assert O.gradient_magnitude(V, "sobel_l1").max() <= 2 * top


@pytest.mark.parametrize("op", ["fwd_l1", "fwd_l2", "sobel_l1"])
def test_clip_rescale_closed_form(op):
    rng = np.random.default_rng(3)
    levels = 16
    V = rng.integers(0, levels, size=(9, 7))
    raw, gmax, hist = O.gradient_histogram(V, levels, op, "clip")
    want = np.concatenate([raw[:levels - 1], [raw[levels - 1:].sum()]])
    assert np.array_equal(hist, want)
    assert hist.sum() == V.size
    # the max rescale of the same raw histogram keeps the mass too
    assert O.gradient_histogram(V, levels, op, "max")[2].sum() == V.size


def _classes(levels):
    return [[(2 * a * b + (levels - 1)) // (2 * (levels - 1)) for b in range(levels)] for a in range(levels)]


def _bruteforce_div_solve(s, g, lv, rv, iters, alpha, beta):
    """Alg. 1 with the printed division by K (cells with K = 0 skipped), in
    exact rationals over explicit loops."""
    n = len(s)
    cls = _classes(n)
    for _ in range(iters):
        d = [Fraction(0)] * n
        for a in range(n):
            for b in range(n):
                d[cls[a][b]] += lv[a] * rv[b]
        K = [[(lv[a] * rv[b] / d[cls[a][b]]) if d[cls[a][b]] else Fraction(0) for b in range(n)] for a in range(n)]
        den_r = sum(x * x for x in lv) + beta
        r_new = []
        for b in range(n):
            acc = Fraction(0)
            for a in range(n):
                if K[a][b]:
                    acc += lv[a] * s[cls[a][b]] / K[a][b]
            r_new.append((acc + beta * g[b]) / den_r)
        den_l = sum(x * x for x in r_new) + alpha
        l_new = []
        for a in range(n):
            acc = Fraction(0)
            for b in range(n):
                if K[a][b]:
                    acc += r_new[b] * s[cls[a][b]] / K[a][b]
            l_new.append((acc + alpha * s[a]) / den_l)
        sr, sl = sum(r_new), sum(l_new)
        rv = [x / sr for x in r_new]
        lv = [x / sl for x in l_new]
    return lv, rv


def _fr_hist(rng, levels, zeros=()):
    h = [int(x) for x in rng.integers(1, 40, size=levels)]
    for z in zeros:
        h[z] = 0
    return h


@pytest.mark.parametrize("levels", [2, 4, 8])
@pytest.mark.parametrize("init_l", ["image", "uniform"])
def test_div_update_matches_exact_loops(levels, init_l):
    rng = np.random.default_rng(40 + levels)
    hS = _fr_hist(rng, levels, [levels - 1] if levels > 2 else [])
    N = sum(hS)
    hG = _fr_hist(rng, levels)
    hG[0] += N - sum(hG) if N > sum(hG) else 0
    while sum(hG) > N:
        k = int(np.argmax(hG))
        hG[k] -= 1
    hG[0] += N - sum(hG)
    s = [Fraction(x, N) for x in hS]
    g = [Fraction(x, N) for x in hG]
    l0 = [Fraction(1, levels)] * levels if init_l == "uniform" else list(s)
    alpha, beta = Fraction(1, 10), Fraction(1, 20)
    lb, rb = _bruteforce_div_solve(s, g, l0, list(g), 3, alpha, beta)
    lv, rv, _ = O.solve(np.array(hS), np.array(hG),
                        O.Params(bins=levels, iters=3, alpha=0.1, beta=0.05, update="div", init_l=init_l))
    assert np.abs(lv - np.array([float(x) for x in lb])).max() <= 1e-12
    assert np.abs(rv - np.array([float(x) for x in rb])).max() <= 1e-12


def test_div_update_two_levels_by_hand():
    """l = 2: index(a, b) = a b, so class 1 is the cell (1, 1) and class 0
    the other three.  With d_0 = 1 - l_1 r_1, d_1 = l_1 r_1 and
    1/K_ab = d_m / (l_a r_b), Eq. (13) as printed gives
      r'_0 = (2 s_0 d_0 / r_0 + beta g_0) / (|l|^2 + beta)
      r'_1 = ((s_0 d_0 + s_1 d_1) / r_1 + beta g_1) / (|l|^2 + beta)
    and Eq. (12) as printed
      l'_0 = (s_0 d_0 (r'_0 / r_0 + r'_1 / r_1) / l_0 + alpha s_0) / (|r'|^2 + alpha)
      l'_1 = ((s_0 d_0 r'_0 / r_0 + s_1 d_1 r'_1 / r_1) / l_1 + alpha s_1) / (|r'|^2 + alpha)."""
    s0, s1 = Fraction(3, 5), Fraction(2, 5)
    g0, g1 = Fraction(1, 4), Fraction(3, 4)
    l0, l1 = s0, s1
    r0, r1 = g0, g1
    alpha, beta = Fraction(1, 10), Fraction(1, 5)
    d1 = l1 * r1
    d0 = 1 - d1
    nl = l0 * l0 + l1 * l1 + beta
    rp0 = (2 * s0 * d0 / r0 + beta * g0) / nl
    rp1 = ((s0 * d0 + s1 * d1) / r1 + beta * g1) / nl
    nr = rp0 * rp0 + rp1 * rp1 + alpha
    lp0 = (s0 * d0 * (rp0 / r0 + rp1 / r1) / l0 + alpha * s0) / nr
    lp1 = ((s0 * d0 * rp0 / r0 + s1 * d1 * rp1 / r1) / l1 + alpha * s1) / nr
    step = O.update_step(np.array([0.6, 0.4]), np.array([0.25, 0.75]), np.array([0.6, 0.4]),
                         np.array([0.25, 0.75]), O.classify(2), 0.1, 0.2, update="div")
    assert step["r_unnorm"] == pytest.approx([float(rp0), float(rp1)], rel=1e-14)
    assert step["l_unnorm"] == pytest.approx([float(lp0), float(lp1)], rel=1e-14)


@pytest.mark.parametrize("levels", [4, 8, 16])
def test_uniform_start_matches_materialised_loops(levels):
    """The multiplying reading from L(0) = 1/l: pure-Python loops over the
    materialised class and K matrices (no oracle helpers)."""
    rng = np.random.default_rng(70 + levels)
    hS = rng.integers(0, 30, size=levels)
    hS[1] = 0
    hS[0] += 1
    N = int(hS.sum())
    hG = np.bincount(rng.integers(0, levels, size=N), minlength=levels)
    n = levels
    cls = _classes(n)
    s = [x / N for x in hS.tolist()]
    g = [x / N for x in hG.tolist()]
    lv, rv = [1.0 / n] * n, list(g)
    alpha, beta = 0.05, 0.02
    for _ in range(20):
        d = [0.0] * n
        for a in range(n):
            for b in range(n):
                d[cls[a][b]] += lv[a] * rv[b]
        K = [[(lv[a] * rv[b] / d[cls[a][b]]) if d[cls[a][b]] > 0 else 0.0 for b in range(n)] for a in range(n)]
        den_r = sum(x * x for x in lv) + beta
        r_new = [(sum(lv[a] * K[a][b] * s[cls[a][b]] for a in range(n)) + beta * g[b]) / den_r for b in range(n)]
        den_l = sum(x * x for x in r_new) + alpha
        l_new = [(sum(r_new[b] * K[a][b] * s[cls[a][b]] for b in range(n)) + alpha * s[a]) / den_l
                 for a in range(n)]
        rv = [x / sum(r_new) for x in r_new]
        lv = [x / sum(l_new) for x in l_new]
    lo, ro, _ = O.solve(hS, hG, O.Params(bins=levels, iters=20, alpha=alpha, beta=beta, init_l="uniform"))
    assert np.abs(lo - np.array(lv)).max() <= 1e-13
    assert np.abs(ro - np.array(rv)).max() <= 1e-13
    # the unoccupied level 1 of s keeps illumination mass from the uniform start
    assert lo[1] > 0


def test_params_reject_unknown_readings():
    for kw in ({"grad_op": "sobel"}, {"grad_rescale": "cut"}, {"update": "/K"}, {"init_l": "flat"}):
        with pytest.raises(ValueError):
            O.Params(**kw)
