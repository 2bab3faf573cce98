"""Pins of the oracle's optimisation (Eqs. 8, 10-15, Alg. 1) and reprocessing
(Eqs. 17-20) against a hand-worked example, the objective of Eq. (10) and
invariants of the iteration."""

import json
import os
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle as O
from synthetic import make_image, config_seed

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _case(seed=0, H=48, W=40, ceil=0.3):
    img = make_image(config_seed(1, 8, seed), H, W, ceil=ceil)
    V = O.value_channel(img)
    hS = O.count_histogram(V, 256)
    _, _, hG = O.gradient_histogram(V, 256)
    return hS, hG


def test_two_level_worked_example():
    with open(os.path.join(GOLDEN, "two_level_step.json")) as f:
        gold = json.load(f)
    s, g, lv, rv = O.init_state(np.array(gold["inputs"]["hS"]), np.array(gold["inputs"]["hG"]))
    idx = O.classify(2)
    step = O.update_step(lv, rv, s, g, idx, float(Fraction(gold["inputs"]["alpha"])),
                         float(Fraction(gold["inputs"]["beta"])))
    for key, vals in gold["expected"].items():
        np.testing.assert_allclose(step[key], [float(Fraction(v)) for v in vals], rtol=1e-14)


def _grad_J(lv, rv, K, s, g, idx, alpha, beta):
    """Gradient of Eq. (10) (K frozen) by float64 autograd of the objective
    written out cell by cell."""
    L = torch.tensor(lv, dtype=torch.float64, requires_grad=True)
    R = torch.tensor(rv, dtype=torch.float64, requires_grad=True)
    Kt = torch.tensor(K, dtype=torch.float64)
    Sidx = torch.tensor(s[idx], dtype=torch.float64)
    st_ = torch.tensor(s, dtype=torch.float64)
    gt = torch.tensor(g, dtype=torch.float64)
    J = ((L[:, None] * R[None, :] - Kt * Sidx) ** 2).sum() \
        + alpha * ((L - st_) ** 2).sum() + beta * ((R - gt) ** 2).sum()
    J.backward()
    return L.grad.numpy(), R.grad.numpy()


@pytest.mark.parametrize("alpha,beta", [(0.01, 0.01), (0.1, 0.1), (1.0, 1.0), (0.3, 0.02)])
def test_updates_are_block_minimisers_of_eq10(alpha, beta):
    hS, hG = _case(1)
    idx = O.classify(256)
    s, g, lv, rv = O.init_state(hS, hG)
    for _ in range(3):
        _, _, K = O.weights(lv, rv, idx)
        step = O.update_step(lv, rv, s, g, idx, alpha, beta, K=K)
        # after the R update the R-gradient vanishes at (L^t, R')
        _, gR = _grad_J(lv, step["r_unnorm"], K, s, g, idx, alpha, beta)
        scale = np.abs(step["r_unnorm"]).max() * ((lv ** 2).sum() + beta)
        assert np.abs(gR).max() <= 1e-12 * scale
        # after the L update the L-gradient vanishes at (L', R')
        gL, _ = _grad_J(step["l_unnorm"], step["r_unnorm"], K, s, g, idx, alpha, beta)
        scale = np.abs(step["l_unnorm"]).max() * ((step["r_unnorm"] ** 2).sum() + alpha)
        assert np.abs(gL).max() <= 1e-12 * scale
        lv, rv = step["l"], step["r"]


def test_objective_decreases_within_each_pass():
    hS, hG = _case(2)
    _, _, info = O.solve(hS, hG, O.Params(iters=12), record=True)
    for jb, jr, jl in zip(info["J_before"], info["J_after_r"], info["J_after_l"]):
        assert jr <= jb * (1 + 1e-12) and jl <= jr * (1 + 1e-12)


def test_invariants_mass_support_sign():
    for seed in range(3):
        hS, hG = _case(seed)
        lv, rv, info = O.solve(hS, hG, O.Params(iters=20))
        assert np.all(lv >= 0) and np.all(rv >= 0)
        assert abs(lv.sum() - 1) < 1e-14 and abs(rv.sum() - 1) < 1e-14
        assert np.array_equal(lv > 0, hS > 0)
        assert np.array_equal(rv > 0, hG > 0)
        assert info["d"].sum() == pytest.approx(1.0, abs=1e-14)


def test_strong_priors_pin_to_data():
    hS, hG = _case(3)
    s, g = hS / hS.sum(), hG / hG.sum()
    lv, rv, _ = O.solve(hS, hG, O.Params(iters=5, alpha=1e12, beta=1e12))
    assert np.abs(lv - s).max() < 1e-10 and np.abs(rv - g).max() < 1e-10


def test_zero_iterations_returns_initialisation():
    hS, hG = _case(4)
    lv, rv, _ = O.solve(hS, hG, O.Params(iters=0))
    assert np.array_equal(lv, hS / hS.sum()) and np.array_equal(rv, hG / hG.sum())


def test_target_histogram_mass_and_gamma_one():
    hS, hG = _case(5)
    N = int(hS.sum())
    lv, rv, info = O.solve(hS, hG, O.Params(iters=10))
    t = O.target_histogram(lv, rv, N, 2.2)
    assert t.sum() == pytest.approx(N, rel=1e-13) and np.all(t >= 0)
    # with gamma = 1 the enhanced classes are the original ones: target = N * d
    t1 = O.target_histogram(lv, rv, N, 1.0)
    np.testing.assert_allclose(t1, N * info["d"], rtol=1e-12, atol=1e-9)


def test_gamma_brightens():
    hS, hG = _case(6)
    N = int(hS.sum())
    lv, rv, _ = O.solve(hS, hG, O.Params(iters=10))
    lev = np.arange(256)
    means = [(O.target_histogram(lv, rv, N, gm) * lev).sum() / N for gm in (1.0, 1.5, 2.2, 5.0)]
    assert all(a < b for a, b in zip(means, means[1:]))
