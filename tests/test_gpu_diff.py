"""Differentiated form on the GPU (through the C ABI) against the FP64
references: checkpointed forward, soft-matching loss and dLoss/dh~, the
reverse pass of the solve, and the chained autograd functions."""

import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
from oracle import diff as D
from oracle import diff_reference as REF
from synthetic import config_seed, make_image
from gpu_cases import to_gpu

pytestmark = pytest.mark.gpu

K, EVERY = 30, 5
PARAMS = O.Params(bins=256, iters=K)
SHAPES = [(64, 80), (120, 90), (33, 157)]
GRAD_REL = 1e-3


@pytest.fixture(scope="module")
def H():
    import paper_2510_21100_amd as H
    from paper_2510_21100_amd import diff

    assert torch.cuda.is_available()
    return H, diff


def _images(shapes, cfg=5):
    out = []
    for i, (h, w) in enumerate(shapes):
        img, rho = make_image(config_seed(cfg, len(shapes), i), h, w, return_truth=True)
        out.append((img, (0.8 * rho).astype(np.float32)))
    return out


def _hists(img):
    V = O.value_channel(img)
    return O.count_histogram(V, 256), O.gradient_histogram(V, 256)[2]


def _rel_inf(x, ref):
    return float(np.abs(np.asarray(x, np.float64) - ref).max() / max(np.abs(ref).max(), 1e-300))


def test_solve_ckpt_matches_the_oracle(H):
    H, diff = H
    cases = _images(SHAPES)
    hs = [_hists(img) for img, _ in cases]
    hv = torch.from_numpy(np.stack([a for a, _ in hs]).astype(np.int32)).cuda()
    hg = torch.from_numpy(np.stack([b for _, b in hs]).astype(np.int32)).cuda()
    ws = H.Workspace(max_images=len(cases), max_bins=256)
    alpha = torch.tensor(PARAMS.alpha, dtype=torch.float64)
    beta = torch.tensor(PARAMS.beta, dtype=torch.float64)
    target = diff.TargetFn.apply(alpha, beta, hv, hg, K, PARAMS.gamma, EVERY, ws)
    torch.cuda.synchronize()
    for i, (hS, hG) in enumerate(hs):
        lv, rv, ck = D.solve_with_checkpoints(hS, hG, PARAMS, EVERY)
        tref = O.target_histogram(lv, rv, int(hS.sum()), PARAMS.gamma)
        assert _rel_inf(target[i].cpu().numpy(), tref) <= 1e-4
    ws.close()


def test_checkpoints_are_the_oracle_iterates(H):
    H, _ = H
    from paper_2510_21100_amd import _lib

    (img, _), = _images(SHAPES[:1])
    hS, hG = _hists(img)
    hv = torch.from_numpy(hS.astype(np.int32)).cuda()[None]
    hg = torch.from_numpy(hG.astype(np.int32)).cuda()[None]
    ws = H.Workspace(max_images=1, max_bins=256)
    ncp = K // EVERY + 1
    ckpt = torch.empty((1, ncp, 2, 256), dtype=torch.float32, device="cuda")
    target = torch.empty((1, 256), dtype=torch.float32, device="cuda")
    p = H.Params(bins=256, iters=K).c()
    _lib.check(_lib.lib.hr_solve_ckpt(C.c_void_p(hv.data_ptr()), C.c_void_p(hg.data_ptr()), 1, C.byref(p), EVERY,
                                      C.c_void_p(ckpt.data_ptr()), C.c_void_p(target.data_ptr()), ws.handle, None))
    torch.cuda.synchronize()
    _, _, ck = D.solve_with_checkpoints(hS, hG, PARAMS, EVERY)
    assert len(ck) == ncp
    got = ckpt.cpu().numpy()[0]
    for k, (lv, rv) in enumerate(ck):
        assert _rel_inf(got[k, 0], lv) <= 1e-5, k
        assert _rel_inf(got[k, 1], rv) <= 1e-5, k
    ws.close()


def test_softmatch_loss_and_target_gradient(H):
    H, diff = H
    cases = _images(SHAPES)
    n = len(cases)
    hs = [_hists(img) for img, _ in cases]
    targets = []
    for (hS, hG) in hs:
        lv, rv, _ = O.solve(hS, hG, PARAMS)
        targets.append(O.target_histogram(lv, rv, int(hS.sum()), PARAMS.gamma).astype(np.float32))
    hv = torch.from_numpy(np.stack([a for a, _ in hs]).astype(np.int32)).cuda()
    tg = torch.from_numpy(np.stack(targets)).cuda().requires_grad_(True)
    imgs = [to_gpu(img) for img, _ in cases]
    tims = [torch.from_numpy(t).cuda() for _, t in cases]
    ws = H.Workspace(max_images=n, max_bins=256)
    loss = diff.SoftMatchLossFn.apply(tg, hv, imgs, tims, ws)
    loss.backward()
    torch.cuda.synchronize()
    grads = tg.grad.cpu().numpy()
    ref_losses = []
    for i, (img, t) in enumerate(cases):
        tt = torch.tensor(targets[i].astype(np.float64), requires_grad=True)
        lref = REF.loss_of_target(tt, hs[i][0], img, t.astype(np.float64))
        lref.backward()
        ref_losses.append(float(lref.detach()))
        ref = tt.grad.numpy() / n
        got = grads[i]
        cos = float(got @ ref / (np.linalg.norm(got) * np.linalg.norm(ref)))
        assert cos >= 0.9999, (i, cos)
        assert _rel_inf(got, ref) <= GRAD_REL, i
    assert abs(float(loss.detach()) - np.mean(ref_losses)) <= 1e-5 * np.mean(ref_losses)
    ws.close()


# checkpoint intervals: the default; one pass per segment; the longest
# segments whose forward quantities the reverse keeps (10 passes after the
# checkpoint) and the shortest it recomputes; the longest allowed
@pytest.mark.parametrize("iters,every", [(K, EVERY), (30, 1), (33, 11), (24, 12), (32, 16)])
def test_solve_vjp_matches_the_reference(H, iters, every):
    H, diff = H
    cases = _images(SHAPES if every == EVERY else SHAPES[:2])
    hs = [_hists(img) for img, _ in cases]
    hv = torch.from_numpy(np.stack([a for a, _ in hs]).astype(np.int32)).cuda()
    hg = torch.from_numpy(np.stack([b for _, b in hs]).astype(np.int32)).cuda()
    ws = H.Workspace(max_images=len(cases), max_bins=256)
    rng = np.random.default_rng(7)
    cot = rng.standard_normal((len(cases), 256)) * 1e-6
    for i, (hS, hG) in enumerate(hs):
        a = torch.tensor(PARAMS.alpha, dtype=torch.float64, requires_grad=True)
        b = torch.tensor(PARAMS.beta, dtype=torch.float64, requires_grad=True)
        target = diff.TargetFn.apply(a, b, hv[i:i + 1], hg[i:i + 1], iters, PARAMS.gamma, every, ws)
        (target * torch.from_numpy(cot[i:i + 1].astype(np.float32)).cuda()).sum().backward()
        torch.cuda.synchronize()
        da, db = REF.target_vjp(hS, hG, PARAMS.alpha, PARAMS.beta, PARAMS.gamma, iters, cot[i])
        assert abs(float(a.grad) - da) <= GRAD_REL * abs(da), (i, float(a.grad), da)
        assert abs(float(b.grad) - db) <= GRAD_REL * abs(db), (i, float(b.grad), db)
    ws.close()


def _loss_case(H, cases):
    H, diff = H
    n = len(cases)
    imgs = [to_gpu(img) for img, _ in cases]
    tims = [torch.from_numpy(t).cuda() for _, t in cases]
    alpha = torch.tensor(PARAMS.alpha, dtype=torch.float64, requires_grad=True)
    beta = torch.tensor(PARAMS.beta, dtype=torch.float64, requires_grad=True)
    loss, target = diff.enhancement_loss(imgs, tims, alpha, beta, iters=K, gamma=PARAMS.gamma, ckpt_every=EVERY)
    target.retain_grad()
    loss.backward()
    torch.cuda.synchronize()
    ref_da = ref_db = ref_loss = 0.0
    for i, (img, t) in enumerate(cases):
        hS, hG = _hists(img)
        r = REF.reference_gradients(img, t.astype(np.float64), hS, hG, PARAMS.alpha, PARAMS.beta, PARAMS.gamma, K)
        ref_da += r["dalpha"] / n
        ref_db += r["dbeta"] / n
        ref_loss += r["loss"] / n
        got = target.grad[i].cpu().numpy()
        ref = r["dtarget"] / n
        cos = float(got @ ref / (np.linalg.norm(got) * np.linalg.norm(ref)))
        assert cos >= 0.9999, (i, cos)
    assert abs(float(loss.detach()) - ref_loss) <= 1e-4 * ref_loss
    assert abs(float(alpha.grad) - ref_da) <= GRAD_REL * abs(ref_da), (float(alpha.grad), ref_da)
    assert abs(float(beta.grad) - ref_db) <= GRAD_REL * abs(ref_db), (float(beta.grad), ref_db)


def test_enhancement_loss_end_to_end(H):
    _loss_case(H, _images(SHAPES[:2]))


def test_enhancement_loss_full_size(H):
    # the bench's differentiated workload: 32 images of 1000x664, K = 30,
    # checkpoints every 5; every image against the FP64 reference
    _loss_case(H, _images([(664, 1000)] * 32))


def test_diff_calls_validate(H):
    H, _ = H
    from paper_2510_21100_amd import _lib

    ws = H.Workspace(max_images=2, max_bins=256)
    p = H.Params(bins=256, iters=30).c()
    d = C.c_void_p(0x1000)
    L = _lib.lib
    assert L.hr_solve_ckpt(d, d, 1, C.byref(p), 7, d, d, ws.handle, None) == _lib.HR_ERR_INVALID_ARG
    assert L.hr_solve_ckpt(d, d, 1, C.byref(p), 0, d, d, ws.handle, None) == _lib.HR_ERR_INVALID_ARG
    assert L.hr_solve_ckpt(d, d, 3, C.byref(p), 5, d, d, ws.handle, None) == _lib.HR_ERR_WORKSPACE
    p10 = H.Params(bins=1024, iters=30).c()
    assert L.hr_solve_ckpt(d, d, 1, C.byref(p10), 5, d, d, ws.handle, None) != _lib.HR_OK
    ws.close()
