"""Alg. 1's stopping rule on the GPU (at most T passes, earlier once both
normalised histograms change by at most eps in squared norm) and the
classical equalisation comparator of Eq. (5), against the oracle."""

import numpy as np
import pytest
import torch

import oracle as O
from synthetic import config_seed, edge_images, make_batch_shapes, make_image
from gpu_cases import REL_TOL, gpu_params, lut_contract, oracle_hists, padded_gpu, rel_err, to_gpu, to_np

pytestmark = pytest.mark.gpu

# a stopping decision of the oracle closer than this (relative) to eps may
# flip in FP32: there the pass count may differ by one
STOP_TAU = 1e-3


@pytest.fixture(scope="module")
def H():
    import paper_2510_21100_amd as H
    assert torch.cuda.is_available()
    return H


def _solve_gpu(H, hS, hG, params):
    hv = torch.from_numpy(hS.astype(np.int32)).cuda()
    hg = torch.from_numpy(hG.astype(np.int32)).cuda()
    passes = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    illum, refl, target = H.solve(hv, hg, int(hS.sum()), gpu_params(H, params), passes=passes)
    torch.cuda.synchronize()
    return to_np(illum), to_np(refl), to_np(target), int(passes.item())


CASES = [(2, (664, 1000), 8, 0.3), (1, (256, 256), 8, 0.3), (3, (480, 640), 8, 0.05), (3, (300, 977), 8, 0.4),
         (4, (360, 640), 10, 0.3), (4, (217, 383), 10, 0.1)]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("eps", [1e-4, 1e-5, 2e-6])
def test_pass_count_and_histograms_match_the_oracle(H, case, eps):
    cfg, (h, w), bits, ceil = case
    img = make_image(config_seed(cfg, 9, 1), h, w, bits=bits, ceil=ceil)
    hS, _, _, hG = oracle_hists(img, 1 << bits)
    params = O.Params(bins=1 << bits, iters=60, eps=eps)
    lv, rv, info = O.solve(hS, hG, params)
    illum, refl, target, passes = _solve_gpu(H, hS, hG, params)
    print(f"eps {eps:g}: oracle {info['passes']} passes (margin {info['stop_margin']:.2e}), GPU {passes}")
    if info["stop_margin"] >= STOP_TAU:
        assert passes == info["passes"]
    else:
        assert abs(passes - info["passes"]) <= 1
    if passes == info["passes"]:
        N = int(hS.sum())
        assert rel_err(illum, N * lv) <= REL_TOL and rel_err(refl, N * rv) <= REL_TOL


def test_eps_zero_and_negative_run_exactly_T(H):
    img = make_image(config_seed(2, 1, 0), 200, 300)
    hS, _, _, hG = oracle_hists(img, 256)
    ref = _solve_gpu(H, hS, hG, O.Params(iters=17))
    for eps in (0.0, -1.0):
        got = _solve_gpu(H, hS, hG, O.Params(iters=17, eps=eps))
        assert got[3] == 17
        for a, b in zip(got[:3], ref[:3]):
            assert np.array_equal(a, b)


def test_huge_eps_stops_after_one_pass(H):
    img = make_image(config_seed(2, 1, 0), 120, 90)
    hS, _, _, hG = oracle_hists(img, 256)
    one = _solve_gpu(H, hS, hG, O.Params(iters=1))
    got = _solve_gpu(H, hS, hG, O.Params(iters=50, eps=4.0))
    assert got[3] == 1
    for a, b in zip(got[:3], one[:3]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("name", sorted(edge_images(8)))
def test_edge_images_with_early_exit(H, name):
    img = edge_images(8)[name]
    hS, _, _, hG = oracle_hists(img, 256)
    params = O.Params(iters=40, eps=1e-6)
    lv, rv, info = O.solve(hS, hG, params)
    illum, refl, _, passes = _solve_gpu(H, hS, hG, params)
    if info["stop_margin"] >= STOP_TAU:
        assert passes == info["passes"], name
    N = int(hS.sum())
    if passes == info["passes"]:
        assert rel_err(illum, N * lv) <= 10 * REL_TOL and rel_err(refl, N * rv) <= 10 * REL_TOL


@pytest.mark.parametrize("bits", [8, 10])
def test_batched_early_exit_equals_plain(H, bits):
    """Per-image pass counts and every output of the batched form equal the
    one-image form with the same eps (same solver code)."""
    shapes = make_batch_shapes(config_seed(3, 8, 5), 6, 64, 900, 48, 700)
    rng = np.random.default_rng(3)
    imgs = [make_image(config_seed(3 if bits == 8 else 4, 6, i), hh, ww, bits=bits,
                       ceil=float(rng.uniform(0.03, 0.4))) for i, (hh, ww) in enumerate(shapes)]
    g = [to_gpu(x) for x in imgs]
    params = H.Params(bins=1 << bits, iters=60, eps=1e-5)
    outs, ex = H.enhance_batch(g, params, extras=True)
    torch.cuda.synchronize()
    counts = to_np(ex["passes"]).tolist()
    print("passes", counts)
    assert all(1 <= c <= 60 for c in counts)
    for i, x in enumerate(g):
        out_p, exp = H.enhance(x, params)
        torch.cuda.synchronize()
        assert int(exp["passes"].item()) == counts[i], i
        assert torch.equal(outs[i], out_p), i
        assert torch.equal(ex["illum"][i], exp["illum"]) and torch.equal(ex["target"][i], exp["target"]), i


# --------------------------------------------------------------------------
# Eq. (5) through the remap of the matching step
# --------------------------------------------------------------------------

@pytest.mark.parametrize("bits,shape,strided", [(8, (256, 256), False), (8, (97, 1201), True),
                                                (10, (216, 384), False), (10, (61, 700), True)])
def test_equalize_bit_exact(H, bits, shape, strided):
    img = make_image(config_seed(1, 2, 1), *shape, bits=bits, ceil=0.2)
    g = padded_gpu(img, 5, 1 if bits == 8 else 2) if strided else to_gpu(img)
    out, lut = H.equalize(g)
    torch.cuda.synchronize()
    hS = O.count_histogram(O.value_channel(img), 1 << bits)
    ref = O.equalization_lut(hS)
    assert np.array_equal(to_np(lut).astype(np.int64), ref)
    assert np.array_equal(to_np(out), O.remap(img, ref))


def test_equalize_edge_images(H):
    for name, img in edge_images(8).items():
        out, lut = H.equalize(to_gpu(img))
        torch.cuda.synchronize()
        ref = O.equalization_lut(O.count_histogram(O.value_channel(img), 256))
        assert np.array_equal(to_np(lut).astype(np.int64), ref), name
        assert np.array_equal(to_np(out), O.remap(img, ref)), name


@pytest.mark.parametrize("bits", [8, 10])
def test_match_to_a_uniform_target(H, bits):
    """Histogram matching to a flat target: the LUT contract against the
    oracle's matching rule on a uniform histogram."""
    img = make_image(config_seed(1, 2, 0), 300, 200, bits=bits, ceil=0.25)
    bins = 1 << bits
    g = to_gpu(img)
    hv, _, _ = H.build_hist(g)
    flat = torch.ones(bins, dtype=torch.float32, device="cuda")
    out, lut = H.match(g, hv, flat)
    torch.cuda.synchronize()
    hS = O.count_histogram(O.value_channel(img), bins)
    lut_ref, margin = O.matching_lut(hS, np.ones(bins))
    lut_contract(to_np(lut), {"hS": hS, "lut": lut_ref, "margin": margin})
