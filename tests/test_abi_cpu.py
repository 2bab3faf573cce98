"""The C ABI without a GPU: the library loads, exports what the header
declares, and rejects bad arguments before anything touches the device."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "histretinex.h")


@pytest.fixture(scope="module")
def L():
    from paper_2510_21100_amd import build

    if not os.path.exists(build.LIB):
        build.build()
    from paper_2510_21100_amd import _lib

    return _lib


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hr_[a-z_]+)\s*\(", text)))


def test_exports_match_header(L):
    declared = header_functions()
    assert declared == sorted(L.EXPORTS)
    for name in declared:
        assert hasattr(L.lib, name), name


def test_abi_version_and_status_strings(L):
    text = open(HEADER).read()
    version = int(re.search(r"#define HR_ABI_VERSION (\d+)", text).group(1))
    assert L.lib.hr_abi_version() == version
    for st in range(5):
        assert L.lib.hr_status_string(st)
    assert L.lib.hr_status_string(99)


def _img(data=0x1000, w=64, h=32, stride=None, esz=1):
    return L_.HrImage(data, w, h, stride if stride is not None else 3 * w * esz)


L_ = None


@pytest.fixture(autouse=True)
def _bind(L):
    global L_
    L_ = L


def _err(L):
    return L.lib.hr_last_error().decode()


def _hist(L, img, bits=8, ws=None):
    return L.lib.hr_build_hist(C.byref(img) if img is not None else None, bits, 0x2000, 0x3000, None, ws, None)


def test_build_hist_validation(L):
    assert _hist(L, None) == L.HR_ERR_INVALID_ARG
    assert _hist(L, _img(data=0)) == L.HR_ERR_INVALID_ARG
    assert _hist(L, _img(w=0)) == L.HR_ERR_INVALID_ARG
    assert _hist(L, _img(h=-1)) == L.HR_ERR_INVALID_ARG
    assert _hist(L, _img(stride=3 * 64 - 1)) == L.HR_ERR_INVALID_ARG
    assert "stride" in _err(L)
    assert _hist(L, _img(), bits=9) == L.HR_ERR_UNSUPPORTED
    assert _hist(L, _img(w=16385)) == L.HR_ERR_UNSUPPORTED
    assert _hist(L, _img(w=8193, esz=2), bits=10) == L.HR_ERR_UNSUPPORTED
    assert _hist(L, _img(data=0x1001, esz=2), bits=10) == L.HR_ERR_INVALID_ARG  # odd 16-bit base
    assert _hist(L, _img(stride=3 * 64 * 2 + 1, esz=2), bits=10) == L.HR_ERR_INVALID_ARG
    # valid arguments, no workspace: refused before any device call
    assert _hist(L, _img()) == L.HR_ERR_INVALID_ARG
    assert "workspace" in _err(L)
    assert L.lib.hr_build_hist(C.byref(_img()), 8, None, 0x3000, None, None, None) == L.HR_ERR_INVALID_ARG


def test_build_hist_batch_validation(L):
    arr = (L.HrImage * 2)(_img(), _img(w=0))
    f = L.lib.hr_build_hist_batch
    assert f(None, 1, 8, 0x2000, 0x3000, None, None) == L.HR_ERR_INVALID_ARG
    assert f(arr, 0, 8, 0x2000, 0x3000, None, None) == L.HR_ERR_INVALID_ARG
    assert f(arr, 1, 8, None, 0x3000, None, None) == L.HR_ERR_INVALID_ARG
    assert f(arr, 1, 9, 0x2000, 0x3000, None, None) == L.HR_ERR_UNSUPPORTED
    assert f(arr, 2, 8, 0x2000, 0x3000, None, None) == L.HR_ERR_INVALID_ARG  # second image has width 0
    assert "width" in _err(L)
    assert f(arr, 1, 8, 0x2000, 0x3000, None, None) == L.HR_ERR_INVALID_ARG  # no workspace
    assert "workspace" in _err(L)


def _params(L, bins=256, iters=50, alpha=0.01, beta=0.01, gamma=2.2, eps=0.0, variant=0, reserved=0):
    return L.HrParams(bins, iters, alpha, beta, gamma, eps, variant, reserved)


def _solve(L, p):
    return L.lib.hr_solve(0x2000, 0x3000, 100, C.byref(p), 0x4000, 0x5000, 0x6000, None, None, None)


def test_solve_validation(L):
    assert _solve(L, _params(L, bins=300)) == L.HR_ERR_UNSUPPORTED
    assert _solve(L, _params(L, iters=-1)) == L.HR_ERR_INVALID_ARG
    assert _solve(L, _params(L, alpha=0.0)) == L.HR_ERR_INVALID_ARG
    assert _solve(L, _params(L, beta=-1.0)) == L.HR_ERR_INVALID_ARG
    assert _solve(L, _params(L, gamma=float("nan"))) == L.HR_ERR_INVALID_ARG
    assert _solve(L, _params(L, alpha=float("inf"))) == L.HR_ERR_INVALID_ARG
    assert _solve(L, _params(L, eps=float("nan"))) == L.HR_ERR_INVALID_ARG
    assert _solve(L, _params(L, variant=0x20)) == L.HR_ERR_UNSUPPORTED  # unknown bit
    assert _solve(L, _params(L, variant=L.HR_VARIANT_GRAD_L2)) == L.HR_ERR_INVALID_ARG
    assert "gradient" in _err(L)
    assert _solve(L, _params(L, variant=L.HR_VARIANT_GRAD_L2 | L.HR_VARIANT_GRAD_SOBEL)) == L.HR_ERR_INVALID_ARG
    for v in (L.HR_VARIANT_UPDATE_DIV, L.HR_VARIANT_INIT_UNIFORM, L.HR_VARIANT_SOLVE_BITS):
        assert _solve(L, _params(L, variant=v)) == L.HR_ERR_INVALID_ARG  # valid: stops at the missing workspace
        assert "workspace" in _err(L)
    assert _solve(L, _params(L, reserved=3)) == L.HR_ERR_INVALID_ARG
    assert L.lib.hr_solve(0x2000, 0x3000, 100, None, 0x4000, 0x5000, 0x6000, None, None, None) == L.HR_ERR_INVALID_ARG
    p = _params(L)
    assert L.lib.hr_solve(None, 0x3000, 100, C.byref(p), 0x4000, 0x5000, 0x6000, None, None, None) \
        == L.HR_ERR_INVALID_ARG
    assert L.lib.hr_solve(0x2000, 0x3000, 100, C.byref(p), None, 0x5000, 0x6000, None, None, None) \
        == L.HR_ERR_INVALID_ARG
    # eps > 0 and negative eps are both valid (negative: exactly iters passes)
    for eps in (1e-5, -1.0):
        assert _solve(L, _params(L, eps=eps)) == L.HR_ERR_INVALID_ARG
        assert "workspace" in _err(L)
    assert _solve(L, p) == L.HR_ERR_INVALID_ARG  # no workspace
    assert "workspace" in _err(L)


def test_match_validation(L):
    img = _img()
    assert L.lib.hr_match(C.byref(img), 8, 0x2000, None, 0x7000, 192, None, None, None) == L.HR_ERR_INVALID_ARG
    assert L.lib.hr_match(C.byref(img), 8, 0x2000, 0x3000, None, 192, None, None, None) == L.HR_ERR_INVALID_ARG
    assert L.lib.hr_match(C.byref(img), 8, 0x2000, 0x3000, 0x7000, 191, None, None, None) == L.HR_ERR_INVALID_ARG
    assert L.lib.hr_match(C.byref(img), 8, 0x2000, 0x3000, 0x7000, 192, None, None, None) == L.HR_ERR_INVALID_ARG
    assert "workspace" in _err(L)


def test_equalize_validation(L):
    img = _img()
    f = L.lib.hr_equalize
    assert f(None, 8, 0x2000, 0x7000, 192, None, None, None) == L.HR_ERR_INVALID_ARG
    assert f(C.byref(img), 9, 0x2000, 0x7000, 192, None, None, None) == L.HR_ERR_UNSUPPORTED
    assert f(C.byref(img), 8, None, 0x7000, 192, None, None, None) == L.HR_ERR_INVALID_ARG
    assert f(C.byref(img), 8, 0x2000, None, 192, None, None, None) == L.HR_ERR_INVALID_ARG
    assert f(C.byref(img), 8, 0x2000, 0x7000, 191, None, None, None) == L.HR_ERR_INVALID_ARG
    assert f(C.byref(img), 8, 0x2000, 0x7000, 192, None, None, None) == L.HR_ERR_INVALID_ARG
    assert "workspace" in _err(L)


def test_enhance_batch_validation(L):
    n = 2
    imgs = (L.HrImage * n)(_img(), _img(w=100, h=50))
    outs = (C.c_void_p * n)(0x8000, 0x9000)
    strides = (C.c_int64 * n)(3 * 64, 3 * 100)
    p = _params(L)
    f = L.lib.hr_enhance_batch
    assert f(imgs, outs, strides, 0, 8, C.byref(p), None, None, None, None, None, None, None) == L.HR_ERR_INVALID_ARG
    assert f(None, outs, strides, n, 8, C.byref(p), None, None, None, None, None, None, None) == L.HR_ERR_INVALID_ARG
    assert f(imgs, outs, strides, n, 10, C.byref(p), None, None, None, None, None, None, None) == L.HR_ERR_INVALID_ARG
    bad = (C.c_int64 * n)(3 * 64, 3 * 100 - 3)
    assert f(imgs, outs, bad, n, 8, C.byref(p), None, None, None, None, None, None, None) == L.HR_ERR_INVALID_ARG
    assert f(imgs, outs, strides, n, 8, C.byref(p), None, None, None, None, None, None, None) == L.HR_ERR_INVALID_ARG
    assert "workspace" in _err(L)


def test_variant_calls_validation(L):
    """hr_build_hist_variant takes gradient bits only; the batched and
    differentiated calls take no variant bits."""
    f = L.lib.hr_build_hist_variant
    img = _img()
    assert f(C.byref(img), 8, L.HR_VARIANT_UPDATE_DIV, 0x2000, 0x3000, None, None, None) == L.HR_ERR_INVALID_ARG
    assert f(C.byref(img), 8, L.HR_VARIANT_GRAD_L2 | L.HR_VARIANT_GRAD_SOBEL, 0x2000, 0x3000, None, None, None) \
        == L.HR_ERR_INVALID_ARG
    assert f(None, 8, L.HR_VARIANT_GRAD_SOBEL, 0x2000, 0x3000, None, None, None) == L.HR_ERR_INVALID_ARG
    assert f(C.byref(img), 9, L.HR_VARIANT_GRAD_SOBEL, 0x2000, 0x3000, None, None, None) == L.HR_ERR_UNSUPPORTED
    for v in (L.HR_VARIANT_GRAD_L2, L.HR_VARIANT_GRAD_SOBEL | L.HR_VARIANT_GRAD_CLIP, 0):
        assert f(C.byref(img), 8, v, 0x2000, 0x3000, None, None, None) == L.HR_ERR_INVALID_ARG
        assert "workspace" in _err(L)
    n = 1
    imgs = (L.HrImage * n)(_img())
    outs = (C.c_void_p * n)(0x8000)
    strides = (C.c_int64 * n)(3 * 64)
    p = _params(L, variant=L.HR_VARIANT_UPDATE_DIV)
    args = (None, None, None, None, None, None, None)
    assert L.lib.hr_enhance_batch(imgs, outs, strides, n, 8, C.byref(p), *args) == L.HR_ERR_UNSUPPORTED
    assert L.lib.hr_enhance_batch_noalloc(imgs, outs, strides, n, 8, C.byref(p), *args) == L.HR_ERR_UNSUPPORTED
    assert L.lib.hr_solve_ckpt(0x2000, 0x3000, 1, C.byref(p), 5, 0x4000, 0x5000, None, None) == L.HR_ERR_UNSUPPORTED


def test_enhance_batch_noalloc_validation(L):
    """Refusals of the allocation-free call happen on the host, before any
    device call: more images than HR_NOALLOC_MAX_IMAGES, bad descriptors."""
    f = L.lib.hr_enhance_batch_noalloc
    p = _params(L)
    n = L.HR_NOALLOC_MAX_IMAGES + 1
    imgs = (L.HrImage * n)(*[_img() for _ in range(n)])
    outs = (C.c_void_p * n)(*[0x8000 + 0x1000 * i for i in range(n)])
    strides = (C.c_int64 * n)(*[3 * 64] * n)
    args = (None, None, None, None, None, None, None)
    assert f(imgs, outs, strides, n, 8, C.byref(p), *args) == L.HR_ERR_UNSUPPORTED
    assert "HR_NOALLOC_MAX_IMAGES" in _err(L)
    assert f(imgs, outs, strides, 0, 8, C.byref(p), *args) == L.HR_ERR_INVALID_ARG
    assert f(None, outs, strides, 2, 8, C.byref(p), *args) == L.HR_ERR_INVALID_ARG
    assert f(imgs, outs, strides, 2, 10, C.byref(p), *args) == L.HR_ERR_INVALID_ARG  # bins != 2^bits
    bad = (C.c_int64 * n)(3 * 64, 3 * 64 - 3, 3 * 64, 3 * 64, 3 * 64)
    assert f(imgs, outs, bad, 2, 8, C.byref(p), *args) == L.HR_ERR_INVALID_ARG
    assert "stride" in _err(L)
    header = open(HEADER).read()
    assert int(re.search(r"#define HR_NOALLOC_MAX_IMAGES (\d+)", header).group(1)) == L.HR_NOALLOC_MAX_IMAGES


def test_workspace_calls_reject_null(L):
    s = L.HrSchedule(4, 1, 8)
    assert L.lib.hr_workspace_set_schedule(None, C.byref(s)) == L.HR_ERR_INVALID_ARG
    f = C.c_uint32()
    assert L.lib.hr_get_flags(None, C.byref(f), 0) == L.HR_ERR_INVALID_ARG
    L.lib.hr_workspace_destroy(None)  # ignored
    out = C.c_void_p()
    assert L.lib.hr_workspace_create(0, 256, C.byref(out)) == L.HR_ERR_INVALID_ARG
    assert L.lib.hr_workspace_create(4, 512, C.byref(out)) == L.HR_ERR_UNSUPPORTED


def test_default_workspace_replacement_keeps_the_old_one_alive(L, monkeypatch):
    """workspace() grows the cached default workspace by replacing it; a
    holder of the old one (a pending backward) must still find it open."""
    from paper_2510_21100_amd import api

    closed = []

    class FakeWorkspace:
        def __init__(self, max_images=1, max_bins=1024):
            self.max_images, self.max_bins, self.handle = max_images, max_bins, object()

        def close(self):
            closed.append(self)
            self.handle = None

    monkeypatch.setattr(api, "Workspace", FakeWorkspace)
    monkeypatch.setattr(api, "_default_ws", {})
    monkeypatch.setattr(api.torch.cuda, "current_device", lambda: 0)
    small = api.workspace(max_images=2)
    assert api.workspace(max_images=1) is small
    big = api.workspace(max_images=8)
    assert big is not small and big.max_images == 8
    assert small.handle is not None and not closed
    assert api.workspace(max_images=3) is big
