"""The allocation-free batched call (hr_enhance_batch_noalloc) against
hr_enhance_batch on the same images: outputs, LUTs, solver histograms and
pass counts bit for bit, on consecutive calls that share the library's fixed
scratch (the second call smaller than the first, and a change of bit depth
between calls)."""

import numpy as np
import pytest
import torch

from synthetic import config_seed, make_image
from gpu_cases import to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import paper_2510_21100_amd as H
    assert torch.cuda.is_available()
    return H


def _imgs(shapes, bits, cfg):
    n = len(shapes)
    rng = np.random.default_rng(5 + bits)
    return [to_gpu(make_image(config_seed(cfg, n, i), h, w, bits=bits, ceil=float(rng.uniform(0.05, 0.4))))
            for i, (h, w) in enumerate(shapes)]


def _extras(n, bins, dev):
    return {"lut": torch.full((n, bins), -1, dtype=torch.int16, device=dev),
            "illum": torch.full((n, bins), -1.0, dtype=torch.float32, device=dev),
            "refl": torch.full((n, bins), -1.0, dtype=torch.float32, device=dev),
            "target": torch.full((n, bins), -1.0, dtype=torch.float32, device=dev),
            "passes": torch.full((n,), -1, dtype=torch.int32, device=dev)}


def _noalloc(H, gimgs, params):
    n = len(gimgs)
    outs = [torch.full_like(g, 7) for g in gimgs]
    ex = _extras(n, params.bins, gimgs[0].device)
    flags = torch.zeros(1, dtype=torch.int32, device=gimgs[0].device)
    H.enhance_batch_noalloc(gimgs, outs, params, extras=ex, flags=flags)
    return outs, ex, flags


def _check_equal(H, gimgs, params, got):
    outs, ex, flags = got
    ws = H.Workspace(max_images=len(gimgs), max_bins=params.bins)
    ref_outs, ref = H.enhance_batch(gimgs, params, ws=ws, extras=True)
    torch.cuda.synchronize()
    for i in range(len(gimgs)):
        assert torch.equal(outs[i], ref_outs[i]), i
        for k in ("lut", "illum", "refl", "target"):
            assert torch.equal(ex[k][i], ref[k][i]), (k, i)
    assert torch.equal(ex["passes"], ref["passes"])
    assert int(flags.item()) == ws.flags()
    ws.close()


@pytest.mark.parametrize("eps", [0.0, 1e-5])
def test_noalloc_equals_batched_two_calls(H, eps):
    big = _imgs([(480, 640), (97, 1201), (300, 77)], 8, 3)
    small = _imgs([(64, 80), (13, 13)], 8, 3)
    p8 = H.Params(bins=256, eps=eps)
    first = _noalloc(H, big, p8)
    second = _noalloc(H, small, p8)  # same scratch, fewer and smaller images
    torch.cuda.synchronize()
    _check_equal(H, big, p8, first)
    _check_equal(H, small, p8, second)


def test_noalloc_bit_depth_change_and_flags(H):
    p10 = H.Params(bins=1024)
    p8 = H.Params(bins=256)
    ten = _imgs([(216, 384), (61, 700)], 10, 4)
    bad = ten[1].clone()
    bad[3, 5, 1] = 2000  # a value above 1023: clamped, flagged
    r10 = _noalloc(H, [ten[0], bad], p10)
    r8 = _noalloc(H, _imgs([(100, 90)], 8, 3), p8)  # 8-bit layout after a 10-bit call
    r10b = _noalloc(H, ten[:1], p10)
    torch.cuda.synchronize()
    assert int(r10[2].item()) & 0x1
    assert int(r8[2].item()) == 0 and int(r10b[2].item()) == 0
    _check_equal(H, [ten[0], bad], p10, r10)
    _check_equal(H, _imgs([(100, 90)], 8, 3), p8, r8)
    _check_equal(H, ten[:1], p10, r10b)


def test_noalloc_refuses_more_images(H):
    imgs = _imgs([(8, 8)] * 5, 8, 3)
    outs = [torch.empty_like(g) for g in imgs]
    with pytest.raises(Exception) as e:
        H.enhance_batch_noalloc(imgs, outs, H.Params(bins=256))
    assert "HR_NOALLOC_MAX_IMAGES" in str(e.value)
