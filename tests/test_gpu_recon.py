"""The reconstruction loop (Sec. 4.2) on the GPU.

Its two kernels against FP64 NumPy: the L2 residual and loss, and the Adam step in each
parameterisation (identity, exp for scales, softplus for densities). The loop itself (parity
unpinned: a trajectory has no oracle) is judged by what it must do: on a small lung phantom with
the paper's noise model and the true motion lattice as the start, the mean loss per view falls by
an order of magnitude and the dynamic volume gets closer to the ground truth (PSNR); two runs from
the same seed end in the same bits.
"""
import numpy as np
import pytest
import torch

from paper_2506_22280_amd import _lib, recon, synth
from gpu_helpers import dev

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def test_l2_residual_matches_fp64():
    _print("case: l2_residual on 3 x 75 x 90 and 64 x 384 x 512 values")
    rng = np.random.default_rng(1)
    a, b = rng.normal(0, 1, (3, 75, 90)), rng.normal(0, 1, (3, 75, 90))
    grad = torch.empty((3, 75, 90), device="cuda")
    loss = torch.zeros(1 + _lib.L2_PARTS, device="cuda")
    _lib.l2_residual(dev(a), dev(b), grad, loss)
    d = a.astype(np.float32).astype(np.float64) - b.astype(np.float32).astype(np.float64)
    np.testing.assert_allclose(grad.cpu().numpy(), d, rtol=0, atol=1e-6)
    assert abs(float(loss[0].item()) - 0.5 * (d * d).sum()) <= 1e-5 * 0.5 * (d * d).sum()
    # many workgroups: the same value on a second call
    big_a, big_b = dev(rng.normal(0, 1, (64, 384, 512))), dev(rng.normal(0, 1, (64, 384, 512)))
    g2 = torch.empty_like(big_a)
    _lib.l2_residual(big_a, big_b, g2, loss)
    first = loss[0].clone()
    _lib.l2_residual(big_a, big_b, g2, loss)
    ref = 0.5 * ((big_a.double() - big_b.double()) ** 2).sum()
    assert torch.equal(loss[0], first)
    assert abs(float(first) - float(ref)) <= 1e-5 * float(ref)
    # no values: L = 0
    loss.fill_(7.0)
    e = torch.empty(0, device="cuda")
    _lib.l2_residual(e, e, e, loss)
    assert float(loss[0].item()) == 0.0


@pytest.mark.parametrize("mapping", ["identity", "exp", "softplus"])
def test_adam_mapped_matches_fp64(mapping):
    _print("case: adam_mapped (%s), two steps on 1000 parameters" % mapping)
    rng = np.random.default_rng(2)
    raw0 = rng.normal(0, 1, 1000)
    fmap = {"identity": lambda x: x, "exp": np.exp,
            "softplus": lambda x: np.logaddexp(0.0, x)}[mapping]
    dmap = {"identity": lambda x: np.ones_like(x), "exp": np.exp,
            "softplus": lambda x: 1.0 / (1.0 + np.exp(-x))}[mapping]
    raw = dev(raw0)
    value = raw if mapping == "identity" else dev(fmap(raw0.astype(np.float32)))
    m, v = torch.zeros_like(raw), torch.zeros_like(raw)
    x, mm, vv = raw0.astype(np.float32).astype(np.float64), np.zeros(1000), np.zeros(1000)
    b1, b2, eps, lr = 0.9, 0.999, 1e-8, 1e-2
    for step in (1, 2):
        gv = rng.normal(0, 1, 1000)
        _lib.adam_mapped(raw, value, dev(gv), m, v, lr, step, mapping)
        g = gv.astype(np.float32).astype(np.float64) * dmap(x)
        mm = b1 * mm + (1 - b1) * g
        vv = b2 * vv + (1 - b2) * g * g
        x = x - lr * (mm / (1 - b1 ** step)) / (np.sqrt(vv / (1 - b2 ** step)) + eps)
    np.testing.assert_allclose(raw.cpu().numpy(), x, rtol=0, atol=2e-6)
    np.testing.assert_allclose(value.cpu().numpy(), fmap(x), rtol=2e-6, atol=1e-7)


def _problem():
    # 64 views over 16 s: about 16 views per breathing cycle, like the paper's sampling
    return synth.lung_phantom("recon_small", 2048, 90, 75, 2.0, 64, 3, 20.0, 3, scan_s=16.0)


def test_loop_reduces_loss_and_improves_the_volume():
    _print("case: 1500 iterations on a 2048-Gaussian phantom, 90x75, 64 noisy views")
    out = recon.experiment(_problem(), 1500, motion="true", noise=True,
                           log=lambda m: _print("  " + m))
    _print(out)
    first, last = out["loss_first_last"]
    assert last < 0.1 * first
    assert out["after"]["psnr_db"] > out["before"]["psnr_db"] + 0.5
    assert out["after"]["rmse"] < out["before"]["rmse"]


def test_loop_is_deterministic():
    _print("case: two 200-iteration runs from the same seed give the same bits")
    p = _problem()
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    ws = _lib.Workspace()
    meas = _lib.project_fwd(p.geom, p.grid, d(p.coef), d(p.mu), d(p.scale), d(p.quat),
                            d(p.rho), d(p.angles), d(p.w), ws).clone()
    outs = []
    for _ in range(2):
        rec = recon.Reconstruction(p, meas, recon.perturbed_init(p, np.random.default_rng(5)),
                                   iters=200, seed=7)
        rec.run(200)
        torch.cuda.synchronize()
        outs.append([t.clone() for t in (rec.mu, rec.scale, rec.quat, rec.rho, rec.coef,
                                         rec.ctrl)])
        rec.close()
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_loop_repeats_a_window_whose_renders_overflowed():
    _print("case: a loop whose plan starts with a far too small instance capacity: the first "
           "window is rolled back and repeated; the result equals a run that never overflowed")
    p = _problem()
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    ws = _lib.Workspace()
    meas = _lib.project_fwd(p.geom, p.grid, d(p.coef), d(p.mu), d(p.scale), d(p.quat),
                            d(p.rho), d(p.angles), d(p.w), ws).clone()
    outs, resized = [], []
    # the same tile shape in both runs (the autotuner may pick another, which sums in another
    # order); the second run's capacity is ample
    for tuning in (dict(capacity=64), dict(capacity=64 * p.n)):
        rec = recon.Reconstruction(p, meas, recon.perturbed_init(p, np.random.default_rng(5)),
                                   iters=60, seed=7, tuning=tuning)
        losses = rec.run(60, log_every=20, check_every=20)
        torch.cuda.synchronize()
        outs.append([t.clone() for t in (rec.mu, rec.scale, rec.quat, rec.rho, rec.coef,
                                         rec.ctrl)] + [losses])
        resized.append(rec.resized)
        rec.close()
    assert resized == [1, 0]
    for a, b in zip(outs[0][:-1], outs[1][:-1]):
        assert torch.equal(a, b)
    assert outs[0][-1] == outs[1][-1]
