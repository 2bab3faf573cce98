"""The batched persistent form against the one-image form and the oracle."""

import numpy as np
import pytest
import torch

import oracle as O
from synthetic import config_seed, make_batch_shapes, make_image
from gpu_cases import lut_contract, padded_gpu, pixel_contract, rel_err, to_gpu, to_np, REL_TOL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import paper_2510_21100_amd as H
    assert torch.cuda.is_available()
    return H


def _batch_imgs(shapes, bits=8, cfg=3):
    n = len(shapes)
    rng = np.random.default_rng(11)
    return [make_image(config_seed(cfg, n, i), h, w, bits=bits, ceil=float(rng.uniform(0.03, 0.4)))
            for i, (h, w) in enumerate(shapes)]


def _compare_to_plain(H, imgs, gimgs, params, ws=None):
    outs, ex = H.enhance_batch(gimgs, params, extras=True, ws=ws)
    torch.cuda.synchronize()
    for i, g in enumerate(gimgs):
        out_p, exp = H.enhance(g, params)
        torch.cuda.synchronize()
        assert torch.equal(outs[i], out_p), i
        assert torch.equal(ex["lut"][i], exp["lut"]), i
        assert torch.equal(ex["illum"][i], exp["illum"]), i
        assert torch.equal(ex["refl"][i], exp["refl"]), i
        assert torch.equal(ex["target"][i], exp["target"]), i
    return outs, ex


SHAPES = [(480, 640), (97, 1201), (1, 333), (300, 77), (13, 13), (664, 1000), (2000, 37)]


def test_batch_equals_plain_8bit(H):
    imgs = _batch_imgs(SHAPES)
    _compare_to_plain(H, imgs, [to_gpu(x) for x in imgs], H.Params(bins=256))


def test_batch_repeated_unchanged_table(H):
    """Calls with an unchanged descriptor table skip its upload: the previous
    launch's last workgroup has put the cursors and counters back to zero.
    Repeats, changes and returns, with the outputs cleared before each call."""
    ws = H.Workspace(max_images=8, max_bins=1024)
    params = H.Params(bins=256)
    a = [to_gpu(x) for x in _batch_imgs(SHAPES[:5])]
    b = [to_gpu(x) for x in _batch_imgs(SHAPES[2:7])]
    refs = {}
    for name, g in (("a", a), ("b", b)):
        refs[name] = [H.enhance(x, params)[0] for x in g]
    torch.cuda.synchronize()
    outs = {"a": [torch.empty_like(x) for x in a], "b": [torch.empty_like(x) for x in b]}
    for k, name in enumerate("aaabbaab"):
        g = a if name == "a" else b
        for o in outs[name]:
            o.zero_()
        H.enhance_batch(g, params, outs=outs[name], ws=ws)
        torch.cuda.synchronize()
        for i, (x, y) in enumerate(zip(outs[name], refs[name])):
            assert torch.equal(x, y), (k, name, i)
    ws.close()


def test_batch_fresh_workspaces(H):
    """Batches on freshly created workspaces (their LUT memory never written):
    a remap that read an image's LUT before the finishing workgroup's stores
    reached memory would produce zeros.  Every call equals the one-image path."""
    params = H.Params(bins=256)
    for shapes in (SHAPES[:5], SHAPES):
        imgs = _batch_imgs(shapes)
        gimgs = [to_gpu(x) for x in imgs]
        ref = []
        for g in gimgs:
            o, _ = H.enhance(g, params)
            ref.append(o)
        torch.cuda.synchronize()
        for rep in range(16):
            ws = H.Workspace(max_images=8, max_bins=1024)
            outs, _ = H.enhance_batch(gimgs, params, ws=ws)
            torch.cuda.synchronize()
            for i, (a, b) in enumerate(zip(outs, ref)):
                assert torch.equal(a, b), (len(shapes), rep, i)
            ws.close()


def test_batch_equals_plain_bright_8bit(H):
    """Bright images take the solver's other forms (no class tables, running
    sums past 40 000 occupied cells): batched still equals one-image."""
    rng = np.random.default_rng(13)
    imgs = [make_image(config_seed(3, 3, i), h, w, bits=8, ceil=c)
            for i, (h, w, c) in enumerate([(300, 400, 0.9), (240, 320, 1.0), (100, 700, 0.8)])]
    imgs.append(rng.integers(0, 256, size=(150, 200, 3), dtype=np.uint8))
    _compare_to_plain(H, imgs, [to_gpu(x) for x in imgs], H.Params(bins=256))


def test_batch_equals_plain_10bit(H):
    shapes = [(216, 384), (61, 700), (400, 33)]
    imgs = _batch_imgs(shapes, bits=10, cfg=4)
    _compare_to_plain(H, imgs, [to_gpu(x) for x in imgs], H.Params(bins=1024))


def test_batch_graph_replay_changing_batches(H):
    """Consecutive calls replay the captured graph with new descriptors;
    every replay must equal the one-image path."""
    ws = H.Workspace(max_images=8, max_bins=256)
    for rep, shapes in enumerate([SHAPES[:3], SHAPES[2:7], SHAPES[:3], [(50, 60)]]):
        imgs = _batch_imgs(shapes)
        gimgs = [to_gpu(x) for x in imgs]
        if rep == 1:
            gimgs[1] = padded_gpu(imgs[1], 3, 1)  # strided member
        _compare_to_plain(H, imgs, gimgs, H.Params(bins=256), ws=ws)
    ws.close()


def test_batch_state_across_bit_depths_and_calls(H):
    """One workspace: 8-bit and 10-bit batches of changing sizes, with the
    histogram-only batch call in between.  The per-image partial histograms
    are cleared by the workgroup that sums them (and fully when the bit depth
    changes), so every call must equal the one-image path."""
    ws = H.Workspace(max_images=6, max_bins=1024)
    b8 = _batch_imgs(SHAPES[:5])
    b10 = _batch_imgs([(216, 384), (61, 700), (400, 33), (7, 9)], bits=10, cfg=4)
    g8 = [to_gpu(x) for x in b8]
    g10 = [to_gpu(x) for x in b10]
    steps = [("8", g8), ("10", g10[:2]), ("8", g8[:2]), ("8", g8), ("hist", g8[:3]), ("8", g8),
             ("10", g10), ("hist", g10[:1]), ("10", g10), ("8", g8[1:4])]
    for k, (what, gimgs) in enumerate(steps):
        if what == "hist":
            hv, hg = H.build_hist_batch(gimgs, ws)
            torch.cuda.synchronize()
            for i, g in enumerate(gimgs):
                a, b, _ = H.build_hist(g)
                torch.cuda.synchronize()
                assert torch.equal(hv[i], a) and torch.equal(hg[i], b), (k, i)
        else:
            _compare_to_plain(H, None, gimgs, H.Params(bins=256 if what == "8" else 1024), ws=ws)
    ws.close()


def test_batch_schedules_agree(H):
    imgs = _batch_imgs(SHAPES[:5])
    gimgs = [to_gpu(x) for x in imgs]
    ref, _ = H.enhance_batch(gimgs, H.Params(bins=256))
    torch.cuda.synchronize()
    ws = H.Workspace(max_images=8, max_bins=256)
    for ts, wg, rs in [(1, 1, 1), (4, 3, 64), (64, 2, 3), (16, 4, 8), (200, 1, 1)]:
        ws.set_schedule(ts, wg, rs)
        outs, _ = H.enhance_batch(gimgs, H.Params(bins=256), ws=ws)
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert torch.equal(a, b), (ts, wg, rs)
    ws.close()


def test_batches_in_flight_on_streams(H):
    """Consecutive batches on three streams, each with its own workspace and
    outputs (launches overlap on the device): every batch equals the batch
    run alone, for both bit depths."""
    for bits, shapes in ((8, SHAPES[:5]), (10, [(216, 384), (61, 700), (400, 33)])):
        imgs = _batch_imgs(shapes, bits=bits, cfg=3 if bits == 8 else 4)
        gimgs = [to_gpu(x) for x in imgs]
        params = H.Params(bins=1 << bits)
        ref, _ = H.enhance_batch(gimgs, params)
        torch.cuda.synchronize()
        wss = [H.Workspace(max_images=len(gimgs), max_bins=1 << bits) for _ in range(3)]
        streams = [torch.cuda.Stream() for _ in range(3)]
        outs = [[torch.empty_like(g) for g in gimgs] for _ in range(3)]
        for rnd in range(3):
            for k in range(3):
                for o in outs[k]:
                    o.zero_()
            torch.cuda.synchronize()
            for k in range(3):
                with torch.cuda.stream(streams[k]):
                    H.enhance_batch(gimgs, params, outs=outs[k], ws=wss[k])
            torch.cuda.synchronize()
            for k in range(3):
                for i, (a, b) in enumerate(zip(outs[k], ref)):
                    assert torch.equal(a, b), (bits, rnd, k, i)
        for w in wss:
            w.close()


def test_batch_vs_oracle(H):
    imgs = _batch_imgs([(300, 400), (128, 999)])
    outs, ex = H.enhance_batch([to_gpu(x) for x in imgs], H.Params(bins=256), extras=True)
    torch.cuda.synchronize()
    for i, img in enumerate(imgs):
        ref = O.enhance(img, O.Params(bins=256))
        assert rel_err(to_np(ex["illum"][i]), ref["illum"]) <= REL_TOL
        lut_contract(to_np(ex["lut"][i]), ref)
        pixel_contract(to_np(outs[i]), ref["out"])


def test_clamped_10bit_values_flag(H):
    img = make_image(config_seed(4, 1, 0), 40, 64, bits=10)
    bad = img.copy()
    bad[3, 5, 1] = 1500
    bad[10, 60, 2] = 65535
    ws = H.Workspace(max_images=2, max_bins=1024)
    ws.flags(clear=True)
    out, ex = H.enhance(to_gpu(bad), H.Params(bins=1024), ws=ws)
    torch.cuda.synchronize()
    assert ws.flags(clear=True) & 1
    ref = O.enhance(np.minimum(bad, 1023), O.Params(bins=1024))
    assert np.array_equal(to_np(ex["hist_v"]).astype(np.int64), ref["hS"])
    outs, _ = H.enhance_batch([to_gpu(bad)], H.Params(bins=1024), ws=ws)
    torch.cuda.synchronize()
    assert ws.flags(clear=True) & 1
    assert torch.equal(outs[0], out)
    ws.close()


def test_batch_rejects_bad_outputs_before_launch(H):
    """Outputs of the wrong shape, dtype, device or layout raise before
    anything is enqueued."""
    imgs = _batch_imgs([(40, 50), (30, 20)])
    gimgs = [to_gpu(x) for x in imgs]
    good = [torch.empty_like(g) for g in gimgs]
    bad_cases = [
        [good[0]],                                                        # too few
        [good[0], torch.empty((29, 20, 3), dtype=torch.uint8, device="cuda")],   # fewer rows
        [good[0], torch.empty((30, 20, 3), dtype=torch.int16, device="cuda")],   # wrong dtype
        [good[0], torch.empty((30, 20, 3), dtype=torch.uint8)],                  # host memory
        [good[0], torch.empty((3, 30, 20), dtype=torch.uint8, device="cuda").permute(1, 2, 0)],  # planar
    ]
    for outs in bad_cases:
        with pytest.raises(ValueError):
            H.enhance_batch(gimgs, H.Params(bins=256), outs=outs)
    hv, hg, _ = H.build_hist(gimgs[0])
    with pytest.raises(ValueError):
        H.solve(hv.cpu(), hg, 40 * 50)
    with pytest.raises(ValueError):
        H.match(gimgs[0], hv, torch.ones(256))
    torch.cuda.synchronize()
