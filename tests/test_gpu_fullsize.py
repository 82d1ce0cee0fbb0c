"""GPU parity at full problem sizes, through the batched plan path (C ABI), on sampled outputs
that the FP64 oracle computes one by one.

* The paper's acquisition (Sec. 4.1): 80k Gaussians of the lung phantom, 512x512 detector at
  0.8 mm offset by 116 mm along e_u (half fan), SID 1000 mm, SDD 1536 mm, rank-2 motion on an
  8 mm lattice; a launch of 8 views spread over the scan. Exact model: the forward on sampled
  pixels against the oracle, the backward with dL/dI nonzero on sampled pixels of two views (so
  that the oracle's adjoint over those pixels is the whole gradient). EWA model (Eq. 4): the
  forward the same way; the backward against FP64 central differences of the oracle's EWA
  forward. Each difference is taken on the part of the problem the perturbed parameter reaches,
  which is exact because a projection is a sum over Gaussians: one Gaussian's own parameters, the
  Gaussians whose B-spline stencil holds the perturbed control point, or every Gaussian for w.
* The large volume: 500k Gaussians, 1024x768 detector at 0.4 mm, rank-4 motion on a 55^3
  lattice (5 mm), a batch of 64 uneven-time views through an autotuned plan and through a plan
  whose splats are the persistent kernels (bitwise equal), with forward and backward parity on
  sampled pixels.

Bars: forward |GPU - oracle| <= 1e-4 x the view's maximum per sampled pixel; gradients per group
norm-wise <= 1e-4 and element-wise <= 1e-3 of the group's maximum.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2506_22280_amd import _lib, synth
from gpu_helpers import check_grads, dev, problem_tensors

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


GRADS = ("g_mu", "g_scale", "g_quat", "g_rho", "g_coef", "g_w")


def _buffers(p, idx, geom):
    T, n = len(idx), p.n
    nv, nu = geom["nv"], geom["nu"]
    t = problem_tensors(p, idx)
    return dict(t, proj=torch.empty((T, nv, nu), device="cuda"),
                grad_proj=torch.zeros((T, nv, nu), device="cuda"),
                g_mu=torch.empty((3, n), device="cuda"), g_scale=torch.empty((3, n), device="cuda"),
                g_quat=torch.empty((4, n), device="cuda"), g_rho=torch.empty((n,), device="cuda"),
                g_coef=torch.empty_like(t["coef"]),
                g_w=torch.empty((T, p.grid["R"]), device="cuda"))


def _run_plan(p, idx, geom, G, tuning=None):
    """One plan over the views idx: forward, then backward with dL/dproj = G (host array);
    returns the projection, the gradients (host, float64) and the plan's tuning."""
    b = _buffers(p, idx, geom)
    with _lib.Plan(geom, p.grid, p.n, len(idx), b, tuning=tuning) as plan:
        tun = plan.tuning()[0]
        _print("plan tuning", tun)
        plan.fwd()
        b["grad_proj"].copy_(dev(G))
        plan.bwd()
        diag, resized = plan.check()
        assert not resized and diag["overflow"] == 0 and diag["nonfinite"] == 0, diag
        proj = b["proj"].cpu().numpy()
        grads = {k: b[k].double().cpu().numpy() for k in GRADS}
    return proj, grads, tun


def _sample(rng, views, m, nv, nu):
    pt = np.repeat(np.asarray(views), m)
    return pt, rng.integers(0, nv, pt.size), rng.integers(0, nu, pt.size)


def _check_fwd(p, geom, idx, proj, views, m, seed):
    """Sampled pixels of the given launch views against the oracle (only those views' angles
    and weights go to the oracle)."""
    rng = np.random.default_rng(seed)
    pt, pj, pi = _sample(rng, views, m, geom["nv"], geom["nu"])
    angles, w = p.views(np.asarray(idx)[views])
    local = np.searchsorted(np.asarray(views), pt)
    ref = oracle.project_pixels(geom, p.grid, p.coef, p.mu, p.scale, p.quat, p.rho, angles, w,
                                local, pj, pi)
    got = proj[pt, pj, pi]
    pmax = proj[np.asarray(views)].reshape(len(views), -1).max(1)
    err = np.abs(got - ref) / pmax[local]
    _print("forward: max |GPU - oracle| / view max = %.3e over %d pixels" % (err.max(), pt.size))
    assert err.max() <= 1e-4


def _sparse_dldi(rng, T, views, m, nv, nu):
    pt, pj, pi = _sample(rng, views, m, nv, nu)
    pg = rng.normal(0.0, 1.0, pt.size)
    G = np.zeros((T, nv, nu), np.float32)
    np.add.at(G, (pt, pj, pi), pg.astype(np.float32))
    # the oracle sees each pixel once, with the float32 value the GPU reads
    key = np.unique(np.stack([pt, pj, pi]), axis=1)
    return G, (key[0], key[1], key[2], G[key[0], key[1], key[2]].astype(np.float64))


def _check_bwd_exact(p, geom, idx, grads, pix, views):
    """Gradients of a launch whose dL/dI is nonzero only at pix (views `views`) against the
    oracle's reverse mode over those views; the other views' dL/dw are exactly zero."""
    pt, pj, pi, pg = pix
    angles, w = p.views(np.asarray(idx)[views])
    local = np.searchsorted(np.asarray(views), pt)
    ref = oracle.project_bwd(geom, p.grid, p.coef, p.mu, p.scale, p.quat, p.rho, angles, w,
                             pixels=(local, pj, pi, pg))
    got = dict(grads)
    others = np.setdiff1d(np.arange(len(idx)), views)
    assert np.all(got["g_w"][others] == 0.0)
    got["g_w"] = got["g_w"][np.asarray(views)]
    check_grads(got, ref)


def _paper_problem():
    p = synth.paper_case(seed=0)
    idx = np.linspace(0, len(p.angles) - 1, 8).round().astype(int)
    return p, idx


def test_paper_acquisition_exact_matches_oracle():
    _print("case: paper acquisition (80k Gaussians, 512x512 at 0.8 mm, offset 116 mm, SDD 1536, "
           "rank 2 / 8 mm), exact model, 8 views through an autotuned plan")
    p, idx = _paper_problem()
    geom = p.geom
    assert geom["off_u"] == 116.0 and geom["sdd"] == 1536.0 and geom["nu"] == 512
    rng = np.random.default_rng(301)
    G, pix = _sparse_dldi(rng, len(idx), [1, 6], 96, geom["nv"], geom["nu"])
    proj, grads, _ = _run_plan(p, idx, geom, G)
    _check_fwd(p, geom, idx, proj, [0, 3, 7], 1024, 302)
    _check_bwd_exact(p, geom, idx, grads, pix, [1, 6])


def _stencil_members(grid, mu, cp):
    """Gaussians whose cubic B-spline stencil holds control point cp = (i, j, k)."""
    dims = (grid["nx"], grid["ny"], grid["nz"])
    keep = np.ones(mu.shape[1], bool)
    for a in range(3):
        f = np.floor((mu[a].astype(np.float64) - grid["origin"][a]) / grid["spacing"][a])
        hit = np.zeros_like(keep)
        for l in range(4):
            hit |= np.clip(f - 1 + l, 0, dims[a] - 1) == cp[a]
        keep &= hit
    return np.flatnonzero(keep)


def test_paper_acquisition_ewa_matches_oracle():
    _print("case: paper acquisition, EWA model (Eq. 4), 8 views through an autotuned plan: "
           "forward against the oracle, backward against its central differences")
    p, idx = _paper_problem()
    geom = dict(p.geom, model="ewa")
    views = [2, 5]
    rng = np.random.default_rng(311)
    G, (pt, pj, pi, pg) = _sparse_dldi(rng, len(idx), views, 96, geom["nv"], geom["nu"])
    proj, grads, _ = _run_plan(p, idx, geom, G)
    _check_fwd(p, geom, idx, proj, [1, 4, 6], 1024, 312)
    others = np.setdiff1d(np.arange(len(idx)), views)
    assert np.all(grads["g_w"][others] == 0.0)
    angles, w = p.views(idx[views])
    local = np.searchsorted(np.asarray(views), pt)
    base = dict(coef=p.coef.astype(np.float64), mu=p.mu.astype(np.float64),
                scale=p.scale.astype(np.float64), quat=p.quat.astype(np.float64),
                rho=p.rho.astype(np.float64), w=w.astype(np.float64))

    def loss(Q, sub=None):
        s = slice(None) if sub is None else sub
        val = oracle.project_pixels(geom, p.grid, Q["coef"], Q["mu"][:, s], Q["scale"][:, s],
                                    Q["quat"][:, s], Q["rho"][s], angles, Q["w"], local, pj, pi)
        return float(val @ pg)

    def central(k, flat_index, h, sub=None):
        vals = []
        for sgn in (1.0, -1.0):
            arr = base[k].copy()
            arr.reshape(-1)[flat_index] += sgn * h
            vals.append(loss(dict(base, **{k: arr}), sub))
        return (vals[0] - vals[1]) / (2.0 * h)

    got, ref = {}, {}
    # the Gaussians' own parameters: the 24 with the largest density gradient, each on its own
    top = np.argsort(-np.abs(grads["g_rho"]))[:24]
    steps = dict(mu=1e-4, scale=1e-5, quat=1e-6, rho=1e-4)
    for k, h in steps.items():
        rows = base[k].shape[0] if base[k].ndim == 2 else 1
        gk, fd = [], []
        for n in top:
            sub = np.array([n])
            for a in range(rows):
                e = a * p.n + n if rows > 1 else n
                fd.append(central(k, e, h, sub))
                gk.append(grads["g_" + k].reshape(-1)[e])
        got[k], ref[k] = np.array(gk), np.array(fd)
    # temporal weights of the views with pixels: every Gaussian
    gw, fw = [], []
    for v in range(len(views)):
        for r in range(p.grid["R"]):
            fw.append(central("w", v * p.grid["R"] + r, 1e-5))
            gw.append(grads["g_w"][views[v], r])
    got["w"], ref["w"] = np.array(gw), np.array(fw)
    # control points with the largest gradients: the Gaussians of their stencil
    gc = grads["g_coef"].reshape(-1)
    order = np.argsort(-np.abs(gc))[:16]
    gcs, fcs = [], []
    for e in order:
        r, k_, j_, i_, a = np.unravel_index(e, p.coef.shape)
        sub = _stencil_members(p.grid, p.mu, (i_, j_, k_))
        fcs.append(central("coef", e, 1e-4, sub))
        gcs.append(gc[e])
    got["coef"], ref["coef"] = np.array(gcs), np.array(fcs)
    check_grads(got, ref)


def test_large_500k_persistent_plan_matches_oracle():
    _print("case: 500k Gaussians, 1024x768 at 0.4 mm, rank 4 on 55^3 (5 mm), batch of 64 "
           "uneven-time views: autotuned plan and persistent-splat plan, sampled pixels")
    p = synth.large(seed=0)
    assert p.n == 500_000 and p.grid["R"] == 4 and p.grid["nx"] == 55
    idx = synth.batch_schedule(len(p.angles), 64, 0)[0]
    geom = p.geom
    rng = np.random.default_rng(401)
    bviews = [0, 63]
    G, pix = _sparse_dldi(rng, len(idx), bviews, 64, geom["nv"], geom["nu"])
    proj, grads, tun = _run_plan(p, idx, geom, G)
    if tun["persistent"] != 1:
        forced = dict(splat_waves=tun["splat_waves"], persistent=1, capacity=tun["capacity"])
        proj_p, grads_p, _ = _run_plan(p, idx, geom, G, tuning=forced)
        assert np.array_equal(proj_p, proj)
        for k in GRADS:
            assert np.array_equal(grads_p[k], grads[k]), k
    _check_fwd(p, geom, idx, proj, [0, 31, 63], 1024, 402)
    _check_bwd_exact(p, geom, idx, grads, pix, bviews)
