"""Host-side parts of the reconstruction loop and of the paper-geometry inputs (no GPU): the
learning-rate schedule, the noise model's statistics and the acquisition parameters."""
import math

import numpy as np

from paper_2506_22280_amd import recon, synth


def test_linear_rates_endpoints_and_midpoint():
    lr = {"a": (1e-2, 1e-3), "b": (1e-4, 1e-5)}
    r0, r1, rm = (recon.linear_rates(k, 101, lr) for k in (0, 100, 50))
    assert r0 == {"a": 1e-2, "b": 1e-4}
    assert abs(r1["a"] - 1e-3) < 1e-15 and abs(r1["b"] - 1e-5) < 1e-18
    assert abs(rm["a"] - 5.5e-3) < 1e-15
    assert recon.linear_rates(500, 101, lr) == r1        # held at the final value
    # the space and time grids follow the paper's Sec. 4.2 schedule
    assert recon.LR["coef"] == (1e-4, 1e-5) and recon.LR["ctrl"] == (1e-2, 1e-3)


def test_noise_model_statistics():
    # counts ~ Poisson(lam e^-p) + N(0, sigma^2); p' = -log(counts / lam): unbiased to first order
    # with variance 1/(lam e^-p) + sigma^2/(lam e^-p)^2 (delta method)
    for p, lam, sigma in ((2.0, 1e8, 4.0), (4.0, 1e5, 4.0), (1.0, 1e4, 20.0)):
        x = np.full(400_000, p)
        y = synth.add_noise(x, lam=lam, sigma=sigma, seed=1).astype(np.float64)
        n = lam * math.exp(-p)
        sd = math.sqrt(1.0 / n + sigma ** 2 / n ** 2)
        assert abs(y.mean() - p) < 5 * sd / math.sqrt(x.size) + 1.0 / n
        assert abs(y.std() / sd - 1.0) < 0.01
    # deterministic per seed
    a = synth.add_noise(np.ones((4, 5)), seed=3)
    assert np.array_equal(a, synth.add_noise(np.ones((4, 5)), seed=3))


def test_paper_case_acquisition():
    p = synth.paper_case(n=500)
    g = p.geom
    assert (g["nu"], g["nv"], g["pitch_u"], g["sid"], g["sdd"], g["off_u"]) == \
        (512, 512, 0.8, 1000.0, 1536.0, 116.0)
    assert len(p.angles) == 310 and p.grid["R"] == 2 and p.grid["spacing"] == [8.0] * 3
    assert abs(p.angles[1] - 2 * math.pi / 310) < 1e-6
    # about 20 breathing cycles: the SI weight returns to ~0 about 20 times
    w = p.w[:, 0]
    minima = np.sum((w[1:-1] < w[:-2]) & (w[1:-1] <= w[2:]))
    assert 15 <= minima <= 25
