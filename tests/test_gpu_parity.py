"""Parity of the HIP path (through the C ABI) with the FP64 oracle."""

import numpy as np
import pytest
import torch

import oracle as O
from synthetic import edge_images
from gpu_cases import (REL_TOL, cfg_image, gpu_params, lut_contract, oracle_hists, padded_gpu,
                       pixel_contract, rel_err, to_gpu, to_np)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import paper_2510_21100_amd as H
    assert torch.cuda.is_available()
    return H


def _hist_case(H, img, gpu_img=None):
    bins = 256 if img.dtype == np.uint8 else 1024
    g = gpu_img if gpu_img is not None else to_gpu(img)
    hv, hg, hraw = H.build_hist(g)
    torch.cuda.synchronize()
    hS, graw, gmax, hG = oracle_hists(img, bins)
    assert np.array_equal(to_np(hv).astype(np.int64), hS)
    assert np.array_equal(to_np(hraw).astype(np.int64), graw)
    assert np.array_equal(to_np(hg).astype(np.int64), hG)


HIST_SHAPES = [(256, 256), (664, 1000), (13, 31), (1, 37), (29, 1), (3, 5000), (2, 16384), (97, 4001)]


@pytest.mark.parametrize("shape", HIST_SHAPES)
def test_hist_bit_exact_8bit(H, shape):
    img = cfg_image(1, *shape)
    _hist_case(H, img)


@pytest.mark.parametrize("name", sorted(edge_images(8)))
def test_hist_edge_images(H, name):
    _hist_case(H, edge_images(8)[name])


@pytest.mark.parametrize("name", sorted(edge_images(10)))
def test_hist_edge_images_10bit(H, name):
    _hist_case(H, edge_images(10)[name])


@pytest.mark.parametrize("shape", [(300, 500), (17, 8192), (64, 2049)])
def test_hist_bit_exact_10bit(H, shape):
    img = cfg_image(4, *shape, bits=10)
    _hist_case(H, img)


@pytest.mark.parametrize("pad,offset", [(1, 0), (5, 1), (0, 3), (16, 16)])
def test_hist_strided_and_unaligned(H, pad, offset):
    img = cfg_image(1, 123, 77)
    _hist_case(H, img, padded_gpu(img, pad, offset))


def test_hist_strided_10bit(H):
    img = cfg_image(4, 45, 91, bits=10)
    _hist_case(H, img, padded_gpu(img, 3, 2))


@pytest.mark.parametrize("bits", [8, 10])
def test_hist_batch_bit_exact(H, bits):
    # ragged sizes (ragged tails, width 1, height 1, wide rows) plus a strided
    # member: every image's histograms equal the oracle's, in one launch
    shapes = [(256, 256), (13, 31), (1, 37), (29, 1), (3, 5000), (97, 4001)] if bits == 8 else \
             [(300, 500), (17, 8192), (1, 3), (45, 91)]
    imgs = [cfg_image(1 if bits == 8 else 4, *sh, bits=bits) for sh in shapes]
    gpu = [to_gpu(x) for x in imgs]
    gpu[-1] = padded_gpu(imgs[-1], 5, 1 if bits == 8 else 2)
    ws = H.Workspace(max_images=len(imgs), max_bins=1 << bits)
    for rep in range(2):  # a second call reuses the state left by the first
        hv, hg = H.build_hist_batch(gpu, ws)
        torch.cuda.synchronize()
        for i, img in enumerate(imgs):
            hS, graw, gmax, hG = oracle_hists(img, 1 << bits)
            assert np.array_equal(to_np(hv[i]).astype(np.int64), hS), (rep, i)
            assert np.array_equal(to_np(hg[i]).astype(np.int64), hG), (rep, i)
    ws.close()


def _solve_case(H, img, params):
    bins = params.bins
    hS, graw, gmax, hG = oracle_hists(img, bins)
    N = int(hS.sum())
    hv = torch.from_numpy(hS.astype(np.int32)).cuda()
    hg = torch.from_numpy(hG.astype(np.int32)).cuda()
    illum, refl, target = H.solve(hv, hg, N, gpu_params(H, params))
    torch.cuda.synchronize()
    lv, rv, _ = O.solve(hS, hG, params)
    tref = O.target_histogram(lv, rv, N, params.gamma)
    e = (rel_err(to_np(illum), N * lv), rel_err(to_np(refl), N * rv), rel_err(to_np(target), tref))
    return e


@pytest.mark.parametrize("shape,alpha,beta", [((256, 256), 0.01, 0.01), ((664, 1000), 0.01, 0.01),
                                              ((256, 256), 0.1, 0.1), ((256, 256), 1.0, 1.0),
                                              ((120, 90), 0.3, 0.02)])
def test_solve_parity_8bit(H, shape, alpha, beta):
    img = cfg_image(2, *shape)
    e = _solve_case(H, img, O.Params(bins=256, iters=50, alpha=alpha, beta=beta))
    print("rel err illum %.2e refl %.2e target %.2e" % e)
    assert e[0] <= REL_TOL and e[1] <= REL_TOL and e[2] <= 10 * REL_TOL


def test_solve_parity_10bit(H):
    img = cfg_image(4, 360, 640, bits=10)
    e = _solve_case(H, img, O.Params(bins=1024, iters=50))
    print("rel err illum %.2e refl %.2e target %.2e" % e)
    assert e[0] <= REL_TOL and e[1] <= REL_TOL and e[2] <= 10 * REL_TOL


@pytest.mark.parametrize("iters", [0, 1, 3])
def test_solve_few_iterations(H, iters):
    img = cfg_image(2, 64, 80)
    e = _solve_case(H, img, O.Params(bins=256, iters=iters))
    assert max(e[:2]) <= REL_TOL


@pytest.mark.parametrize("name", ["constant", "two_level", "checkerboard", "single_bright", "one_pixel"])
def test_solve_degenerate(H, name):
    img = edge_images(8)[name]
    e = _solve_case(H, img, O.Params(bins=256, iters=10))
    assert max(e) <= 10 * REL_TOL


@pytest.mark.parametrize("bits", [8, 10])
@pytest.mark.parametrize("name", sorted(edge_images(10)))
def test_solve_edge_images(H, bits, name):
    # every edge image at both level counts, 50 passes: one occupied level
    # (black, white, constant), two levels, single rows and columns
    img = edge_images(bits)[name]
    e = _solve_case(H, img, O.Params(bins=1 << bits, iters=50))
    assert max(e) <= 10 * REL_TOL


def test_solve_parity_10bit_all_levels(H):
    # uniform random 10-bit pixels: V on ~950 levels and ~850 gradient levels,
    # the most classes and the widest sweeps at 1024 levels
    img = np.random.default_rng(11).integers(0, 1024, size=(192, 256, 3), dtype=np.uint16)
    e = _solve_case(H, img, O.Params(bins=1024, iters=50))
    print("rel err illum %.2e refl %.2e target %.2e" % e)
    assert e[0] <= REL_TOL and e[1] <= REL_TOL and e[2] <= 10 * REL_TOL


@pytest.mark.parametrize("ceil,form", [(0.9, "class list, classes computed in the sweeps"),
                                       (1.0, "running sums (more than 40 000 occupied cells)"),
                                       (None, "running sums, every level occupied")])
def test_solve_parity_8bit_many_cells(H, ceil, form):
    # bright 8-bit images: the forms the solver takes past the low-light range
    if ceil is None:
        img = np.random.default_rng(12).integers(0, 256, size=(192, 256, 3), dtype=np.uint8)
    else:
        img = cfg_image(2, 300, 400, ceil=ceil)
    hS, _, _, hG = oracle_hists(img, 256)
    print(form, "occupied cells", int((hS > 0).sum()) * int((hG > 0).sum()))
    e = _solve_case(H, img, O.Params(bins=256, iters=50))
    print("rel err illum %.2e refl %.2e target %.2e" % e)
    assert e[0] <= REL_TOL and e[1] <= REL_TOL and e[2] <= 10 * REL_TOL


@pytest.mark.parametrize("iters", [0, 1, 3])
def test_solve_few_iterations_10bit(H, iters):
    img = cfg_image(4, 90, 120, bits=10)
    e = _solve_case(H, img, O.Params(bins=1024, iters=iters))
    assert max(e[:2]) <= REL_TOL


@pytest.mark.parametrize("bits,shape", [(8, (256, 256)), (8, (664, 1000)), (10, (200, 300))])
def test_match_given_target(H, bits, shape):
    """LUT and remap from the same FP32 target as the oracle: the LUT must be
    identical wherever the oracle's decision margin exceeds FP64 rounding, and
    the pixels identical to the oracle's remap with that LUT."""
    img = cfg_image(2, *shape, bits=bits)
    bins = 1 << bits
    hS, _, _, hG = oracle_hists(img, bins)
    rng = np.random.default_rng(5)
    target = (rng.random(bins) * (rng.random(bins) < 0.7)).astype(np.float32) * 1000
    g = to_gpu(img)
    hv = torch.from_numpy(hS.astype(np.int32)).cuda()
    out, lut = H.match(g, hv, torch.from_numpy(target).cuda())
    torch.cuda.synchronize()
    lut_ref, margin = O.matching_lut(hS, target.astype(np.float64))
    lut_g = to_np(lut).astype(np.int64)
    occ = hS > 0
    sure = occ & (margin > 1e-12)
    assert np.array_equal(lut_g[sure], lut_ref[sure])
    assert np.array_equal(to_np(out), O.remap(img, lut_g))


def test_match_in_place_and_strided_output(H):
    img = cfg_image(2, 77, 131)
    hS, _, _, _ = oracle_hists(img, 256)
    target = np.ones(256, np.float32)
    g = to_gpu(img)
    hv = torch.from_numpy(hS.astype(np.int32)).cuda()
    out_strided = padded_gpu(np.zeros_like(img), 7, 5)
    out, lut = H.match(g, hv, torch.from_numpy(target).cuda(), out=out_strided)
    ref = O.remap(img, to_np(lut).astype(np.int64))
    assert np.array_equal(to_np(out.contiguous()), ref)
    out2, _ = H.match(g, hv, torch.from_numpy(target).cuda(), out=g)  # in place
    torch.cuda.synchronize()
    assert np.array_equal(to_np(g), ref)


@pytest.mark.parametrize("cfg,shape,bits", [(1, (256, 256), 8), (2, (664, 1000), 8), (4, (270, 480), 10)])
def test_end_to_end_plain(H, cfg, shape, bits):
    img = cfg_image(cfg, *shape, bits=bits)
    params = O.Params(bins=1 << bits, iters=50)
    out, ex = H.enhance(to_gpu(img), gpu_params(H, params))
    torch.cuda.synchronize()
    ref = O.enhance(img, params)
    assert np.array_equal(to_np(ex["hist_v"]).astype(np.int64), ref["hS"])
    assert np.array_equal(to_np(ex["hist_grad"]).astype(np.int64), ref["hG"])
    assert rel_err(to_np(ex["illum"]), ref["illum"]) <= REL_TOL
    assert rel_err(to_np(ex["refl"]), ref["refl"]) <= REL_TOL
    ties = lut_contract(to_np(ex["lut"]), ref)
    frac = pixel_contract(to_np(out), ref["out"])
    print(f"near-tie levels {ties}, pixels off by one {frac:.2e}")


@pytest.mark.parametrize("bits", [8, 10])
def test_solve_empty_histograms_flagged(H, bits):
    # histograms without mass (a caller error the host cannot see): the mass
    # flag is set and every output is zero
    from paper_2510_21100_amd import _lib
    bins = 1 << bits
    ws = H.Workspace(max_images=1, max_bins=bins)
    ws.flags(clear=True)
    z = torch.zeros(bins, dtype=torch.int32, device="cuda")
    illum, refl, target = H.solve(z, z.clone(), 100, H.Params(bins=bins, iters=50), ws)
    torch.cuda.synchronize()
    assert ws.flags(clear=True) & _lib.HR_FLAG_HIST_MASS
    for x in (illum, refl, target):
        assert not torch.any(x != 0)
    ws.close()


def test_solve_mass_mismatch_flagged(H):
    # npix different from the histogram mass: flagged; the solve itself uses
    # the histograms as given
    from paper_2510_21100_amd import _lib
    img = cfg_image(2, 64, 80)
    hS, graw, gmax, hG = oracle_hists(img, 256)
    N = int(hS.sum())
    hv = torch.from_numpy(hS.astype(np.int32)).cuda()
    hg = torch.from_numpy(hG.astype(np.int32)).cuda()
    ws = H.Workspace(max_images=1, max_bins=256)
    ws.flags(clear=True)
    ref = H.solve(hv, hg, N, H.Params(bins=256), ws)
    torch.cuda.synchronize()
    assert not ws.flags(clear=True) & _lib.HR_FLAG_HIST_MASS
    got = H.solve(hv, hg, N + 1, H.Params(bins=256), ws)
    torch.cuda.synchronize()
    assert ws.flags(clear=True) & _lib.HR_FLAG_HIST_MASS
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    ws.close()
