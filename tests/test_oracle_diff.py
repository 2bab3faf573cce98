"""Pins of the differentiated form's FP64 references: the soft map agrees with
the exact matching LUT, the two independent forward transcriptions agree, and
the autograd gradients agree with central finite differences."""

import numpy as np
import pytest

import oracle as O
from oracle import diff as D
from oracle import diff_reference as REF
from synthetic import config_seed, make_image

K = 30
PARAMS = O.Params(bins=256, iters=K)


def _case(i=0, shape=(40, 56)):
    img, rho = make_image(config_seed(5, 4, i), *shape, return_truth=True)
    return img, 0.8 * rho.astype(np.float64)


@pytest.fixture(scope="module")
def case():
    img, t = _case()
    fw = D.forward(img, t, PARAMS)
    ref = REF.reference_gradients(img, t, fw["hS"], fw["hG"], PARAMS.alpha, PARAMS.beta, PARAMS.gamma, K)
    return img, t, fw, ref


def test_soft_map_rounds_to_the_exact_lut(case):
    img, t, fw, _ = case
    lut, margin = O.matching_lut(fw["hS"], fw["target"])
    occ = fw["hS"] > 0
    assert np.array_equal(fw["lut"][occ], lut[occ])
    k = fw["lut"][occ]
    m = fw["m"][occ]
    inside = ~fw["clamped"][occ]
    assert np.all(m[inside] > k[inside] - 0.5) and np.all(m[inside] <= k[inside] + 0.5)
    sure = margin[occ] > 1e-9
    assert np.array_equal(np.floor(m[sure & inside] + 0.5).astype(int), k[sure & inside])


def test_soft_map_of_a_uniform_target_is_linear_in_u():
    # F~(k) = (k+1)/l: the inverse through (k+1/2, (k+1)/l) is m = l u - 1/2
    hS = np.zeros(16, np.int64)
    hS[[2, 5, 9, 12]] = [3, 7, 1, 5]
    m, lut, clamped = D.soft_map(hS, np.ones(16))
    u = D.source_cdf_midrank(hS)
    occ = hS > 0
    assert np.allclose(m[occ], np.clip(16 * u[occ] - 0.5, 0, 15), rtol=0, atol=1e-12)


def test_independent_forwards_agree(case):
    img, t, fw, ref = case
    assert abs(ref["loss"] - fw["loss"]) <= 1e-12 * fw["loss"]
    assert np.allclose(ref["target"], fw["target"], rtol=1e-10, atol=1e-9)


def _loss_at(img, t, alpha=PARAMS.alpha, beta=PARAMS.beta):
    p = O.Params(bins=256, iters=K, alpha=alpha, beta=beta, gamma=PARAMS.gamma)
    return D.forward(img, t, p)["loss"]


@pytest.mark.parametrize("which", ["alpha", "beta"])
def test_prior_weight_gradient_matches_central_differences(case, which):
    img, t, fw, ref = case
    x0 = getattr(PARAMS, which)
    h = 1e-4 * x0
    fp = _loss_at(img, t, **{which: x0 + h})
    fm = _loss_at(img, t, **{which: x0 - h})
    fd = (fp - fm) / (2 * h)
    g = ref["d" + which]
    assert abs(fd - g) <= 1e-6 * abs(g) + 1e-12, (fd, g)


def test_target_gradient_matches_central_differences(case):
    img, t, fw, ref = case
    target = fw["target"]
    skip = D.near_kink(fw["hS"], target, tol=1e-7)
    rng = np.random.default_rng(0)
    bins = [k for k in rng.permutation(np.nonzero(target > 0)[0]) if not skip[k]][:12]
    assert len(bins) >= 6
    for k in bins:
        h = 1e-6 * target.sum()
        tp, tm = target.copy(), target.copy()
        tp[k] += h
        tm[k] -= h
        fd = (D.soft_loss(img, t, D.soft_map(fw["hS"], tp)[0]) -
              D.soft_loss(img, t, D.soft_map(fw["hS"], tm)[0])) / (2 * h)
        g = ref["dtarget"][k]
        assert abs(fd - g) <= 1e-5 * np.abs(ref["dtarget"]).max() + 1e-12 * abs(g), (k, fd, g)


def test_solve_vjp_matches_central_differences(case):
    img, t, fw, ref = case
    cot = np.random.default_rng(1).standard_normal(256)
    da, db = REF.target_vjp(fw["hS"], fw["hG"], PARAMS.alpha, PARAMS.beta, PARAMS.gamma, K, cot)
    for name, g in (("alpha", da), ("beta", db)):
        x0 = getattr(PARAMS, name)
        h = 1e-4 * x0
        vals = []
        for x in (x0 + h, x0 - h):
            p = O.Params(bins=256, iters=K, **{"alpha": PARAMS.alpha, "beta": PARAMS.beta, name: x})
            lv, rv, _ = O.solve(fw["hS"], fw["hG"], p)
            vals.append(float(cot @ O.target_histogram(lv, rv, int(fw["hS"].sum()), PARAMS.gamma)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g) <= 1e-6 * abs(g) + 1e-9, (name, fd, g)


def test_checkpoints_are_the_iterates():
    img, t = _case(1, (24, 32))
    V = O.value_channel(img)
    hS = O.count_histogram(V, 256)
    hG = O.gradient_histogram(V, 256)[2]
    lv, rv, ck = D.solve_with_checkpoints(hS, hG, PARAMS, 5)
    assert len(ck) == K // 5 + 1
    l_ref, r_ref, _ = O.solve(hS, hG, PARAMS)
    assert np.array_equal(ck[-1][0], lv) and np.allclose(lv, l_ref, rtol=0, atol=0)
    p10 = O.Params(bins=256, iters=10)
    l10, r10, _ = O.solve(hS, hG, p10)
    assert np.array_equal(ck[2][0], l10) and np.array_equal(ck[2][1], r10)
