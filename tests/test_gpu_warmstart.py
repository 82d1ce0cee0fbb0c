"""The temporal-weight fit and its learned warm start on the GPU.

Kernels are checked against FP64 NumPy: the BF16 matrix-core product (against the product of the
same BF16-rounded operands, and within BF16 error of the unrounded one), the MLP's gradient
(against an FP64 NumPy backward of the same network), the LM normal equations and the
downsampling. The plain fit must recover the weights a view was rendered with; the trained warm
start must reach the same residual tolerance in fewer renders than the plain fit on views of
phantoms it never saw (parity unpinned for the predicted weights themselves: the fit's residual
judges them).
"""
import time

import numpy as np
import pytest
import torch

from paper_2506_22280_amd import _lib, synth, warmstart
from gpu_helpers import dev

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _bf16(x):
    """Round to bfloat16 (nearest even), returned as float64."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("M,N,K", [(64, 64, 32), (100, 37, 50), (256, 256, 4098), (7, 3, 300)])
def test_gemm_bf16_matches_fp64(M, N, K):
    _print("case: gemm_bf16 M=%d N=%d K=%d, all transposes and epilogues" % (M, N, K))
    rng = np.random.default_rng(M * 7 + N)
    A = rng.normal(0, 1, (M, K)).astype(np.float32)
    B = rng.normal(0, 1, (K, N)).astype(np.float32)
    bias = rng.normal(0, 1, N).astype(np.float32)
    C0 = rng.normal(0, 1, (M, N)).astype(np.float32)
    gate = rng.normal(0, 1, (M, N)).astype(np.float32)
    exact = _bf16(A) @ _bf16(B)
    for ta in (False, True):
        for tb in (False, True):
            dA = dev(A.T.copy() if ta else A)
            dB = dev(B.T.copy() if tb else B)
            C = dev(C0)
            _lib.gemm_bf16(dA, dB, C, transA=ta, transB=tb, bias=dev(bias), accumulate=True,
                           relu=True, gate=dev(gate))
            ref = np.maximum(exact + C0 + bias[None, :], 0.0) * (gate > 0)
            got = C.cpu().numpy()
            scale = np.abs(exact).max() + 1.0
            assert np.abs(got - ref).max() <= 2e-6 * scale * np.sqrt(K), (ta, tb)
    # against the unrounded FP64 product: BF16 operand rounding only
    C = torch.zeros((M, N), device="cuda")
    _lib.gemm_bf16(dev(A), dev(B), C)
    full = A.astype(np.float64) @ B.astype(np.float64)
    err = np.linalg.norm(C.cpu().numpy() - full) / np.linalg.norm(full)
    assert err <= 1e-2, err


def _np_mlp_grad(w, X, T, mean, std, nin, hid, R):
    """FP64 NumPy forward and backward of the network with BF16-rounded product operands."""
    o = np.cumsum([0, nin * hid, hid, hid * hid, hid, hid * R, R])
    W1 = w[o[0]:o[1]].reshape(nin, hid); b1 = w[o[1]:o[2]]
    W2 = w[o[2]:o[3]].reshape(hid, hid); b2 = w[o[3]:o[4]]
    W3 = w[o[4]:o[5]].reshape(hid, R); b3 = w[o[5]:o[6]]
    q = _bf16
    H1 = np.maximum(q(X) @ q(W1) + b1, 0)
    H2 = np.maximum(q(H1) @ q(W2) + b2, 0)
    Y = q(H2) @ q(W3) + b3
    D = Y - (T - mean) / std
    dY = 2 * D / D.size
    gW3 = q(H2).T @ q(dY); gb3 = dY.sum(0)
    dH2 = (q(dY) @ q(W3).T) * (H2 > 0)
    gW2 = q(H1).T @ q(dH2); gb2 = dH2.sum(0)
    dH1 = (q(dH2) @ q(W2).T) * (H1 > 0)
    gW1 = q(X).T @ q(dH1); gb1 = dH1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3]), (D ** 2).mean()


def test_mlp_gradient_matches_fp64():
    _print("case: warm-start MLP gradient (4098-256-256-3, batch 128) against FP64 NumPy")
    nin, hid, R, B = 4098, 256, 3, 128
    net = warmstart.WarmStartNet(nin, R, hid, seed=3)
    rng = np.random.default_rng(4)
    X = rng.normal(0, 1, (B, nin)).astype(np.float32)
    T = rng.normal(5, 3, (B, R)).astype(np.float32)
    net.mean_h = np.array([5.0, 4.0, 6.0]); net.std_h = np.array([3.0, 2.0, 1.0])
    net.mean = dev(net.mean_h); net.std = dev(net.std_h)
    w0 = net.w.cpu().numpy().astype(np.float64)
    loss = torch.zeros(1, device="cuda")
    net.train_step(dev(X), dev(T), lr=0.0, loss=loss)
    torch.cuda.synchronize()
    g = net.g.cpu().numpy().astype(np.float64)
    gref, lref = _np_mlp_grad(w0, X.astype(np.float64), T.astype(np.float64), net.mean_h,
                              net.std_h, nin, hid, R)
    err = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    _print("gradient norm-wise error", err, "loss", float(loss.item()), lref)
    assert err <= 1e-3
    assert abs(float(loss.item()) - lref) <= 1e-4 * lref
    assert np.array_equal(net.w.cpu().numpy(), w0.astype(np.float32))   # lr = 0: no change


def test_lm_normal_eq_and_downsample():
    _print("case: LM normal equations (R=3, 5 views) and 8x6 block-mean downsampling")
    rng = np.random.default_rng(8)
    T, R, nv, nu = 5, 3, 384, 512
    imgs = rng.normal(0, 1, (T, R + 1, nv, nu)).astype(np.float32)
    meas = rng.normal(0, 1, (T, nv, nu)).astype(np.float32)
    h = np.array([0.1, 0.2, 0.05], dtype=np.float32)
    out = _lib.lm_normal_eq(dev(imgs), dev(meas), dev(h), R).cpu().numpy()
    I = imgs.astype(np.float64).reshape(T, R + 1, -1)
    J = (I[:, 1:] - I[:, :1]) / h.astype(np.float64)[None, :, None]
    res = I[:, 0] - meas.astype(np.float64).reshape(T, -1)
    for t in range(T):
        G = J[t] @ J[t].T
        ref = np.concatenate([G[np.triu_indices(R)], J[t] @ res[t], [res[t] @ res[t]]])
        np.testing.assert_allclose(out[t], ref, rtol=2e-5, atol=2e-5 * np.abs(ref).max())
    ang = rng.uniform(0, 6.28, T).astype(np.float32)
    f = _lib.downsample(dev(meas), 6, 8, angles=dev(ang), scale=2.0).cpu().numpy()
    ref = 2.0 * meas.astype(np.float64).reshape(T, 64, 6, 64, 8).mean((2, 4)).reshape(T, -1)
    np.testing.assert_allclose(f[:, :4096], ref, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(f[:, 4096], np.sin(ang), atol=1e-6)
    np.testing.assert_allclose(f[:, 4097], np.cos(ang), atol=1e-6)


def _phantom_scene(seed, nviews):
    p = synth.lung_phantom("warm_%d" % seed, 4096, 128, 128, 2.5, nviews, 3, 20.0, seed)
    return p, warmstart.Scene(p.geom, p.grid, p.coef, p.mu, p.scale, p.quat, p.rho)


def _views(p, scene, idx):
    ang = dev(p.angles[idx])
    meas = scene.render(ang, dev(p.w[idx])).clone()
    return ang, meas


def test_plain_fit_recovers_rendered_weights():
    _print("case: LM fit of 64 views rendered at known weights (4096-Gaussian phantom, 128x128)")
    p, scene = _phantom_scene(0, 64)
    idx = np.arange(64)
    ang, meas = _views(p, scene, idx)
    w0 = np.tile(p.w.mean(0, dtype=np.float64), (64, 1))
    w, images, rel = warmstart.lm_fit(scene, ang, meas, w0, tol=1e-3, max_steps=30)
    _print("images per view: mean %.2f max %d; rel residual max %.2e" % (images.mean(),
                                                                        images.max(), rel.max()))
    # each iteration renders the trial (1 image) and, after an accepted trial, the R = 3 raised
    # copies: at most 4 images per iteration
    assert (images <= 4 * 30).all() and (rel <= 1e-3).all()
    assert np.abs(w - p.w[idx]).max() <= 0.05 * np.abs(p.w).max()


def test_warm_start_beats_plain_fit_on_unseen_phantoms():
    _print("case: warm start trained on plain fits of 8 phantoms x 256 views (50k Gaussians, "
           "256x192 at 1.6 mm), judged on 2 unseen phantoms x 256 views")
    out = warmstart.experiment(50_000, 256, 192, 1.6, 680, 10.0, list(range(8)), [100, 101],
                               3, 4, views_per_seed=256, epochs=100,
                               log=lambda m: _print("  " + m))
    _print(out)
    assert out["train_pairs"] >= 0.95 * 8 * 256          # the plain fits that label the data
    assert out["loss_first_last"][1] < 0.1 * out["loss_first_last"][0]
    n = out["test_views"]
    assert out["plain"]["converged"] == n and out["warm"]["converged"] == n
    # images rendered per view until the residual tolerance, the warm fit's evaluation of the
    # plain start included
    assert out["warm"]["mean_images_per_view"] < out["plain"]["mean_images_per_view"]
