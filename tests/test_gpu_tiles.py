"""GPU parity of every detector tile shape (one, two or four 8x8 blocks per tile) against the FP64
oracle, and the autotuner's tile-shape axis.

Tolerances as in test_gpu_parity: forward per pixel |GPU - oracle| <= 1e-4 * max|oracle| of the
projection; gradients per group norm-wise <= 1e-4 and element-wise <= 1e-3 of the group's maximum.
Launch shapes of one tile shape must agree bit for bit; list slices and tile shapes add the same
terms in other orders, so they are held to the oracle's bars (and to each other at rounding level).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2506_22280_amd import _lib, synth
from gpu_helpers import check_grads, dev, max_rel_to_max, oracle_inputs, problem_tensors

pytestmark = pytest.mark.gpu

SHAPES = [(16, 16), (32, 8), (8, 32), (16, 8), (8, 16), (8, 8)]


def _print(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def offset_case():
    """Exact model, 90x75 detector (ragged tiles in every shape), pitches 0.9 x 1.3 mm, offsets
    (5, -2) mm, 1024 Gaussians, 4 views; the oracle's projections and adjoint."""
    p = synth.tiny(seed=41, n=1024, nviews=4, det=64)
    p.geom = dict(p.geom, nu=90, nv=75, pitch_u=0.9, pitch_v=1.3, off_u=5.0, off_v=-2.0)
    ref = oracle.project(p.geom, p.grid, *oracle_inputs(p))
    G = np.random.default_rng(42).normal(0, 1, ref.shape).astype(np.float32)
    gref = oracle.project_bwd(p.geom, p.grid, *oracle_inputs(p), grad_proj=G)
    return p, ref, G, gref


def _fwd(p, t, tuning, ws=None):
    ws = ws or _lib.Workspace()
    proj = _lib.project_fwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                            t["angles"], t["w"], ws, tuning=tuning)
    torch.cuda.synchronize()
    return proj, ws


def _check_fwd(proj, ref, label):
    for k in range(ref.shape[0]):
        err = max_rel_to_max(proj[k].cpu().numpy(), ref[k])
        assert err <= 1e-4, (label, k, err)


@pytest.mark.parametrize("shape", SHAPES, ids=["%dx%d" % s for s in SHAPES])
def test_tile_shape_matches_oracle(offset_case, shape):
    p, ref, G, gref = offset_case
    tw, th = shape
    _print("case: tile %dx%d, 90x75 offset detector, 1024 Gaussians, 4 views: forward for waves "
           "4/1 x persistent 0/1 x slices 1/3, backward; against the oracle" % shape)
    t = problem_tensors(p)
    base = dict(tile_w=tw, tile_h=th)
    first = None
    for waves in (4, 1):
        for persistent in (0, 1):
            tun = dict(base, splat_waves=waves, persistent=persistent, slices=1)
            proj, ws = _fwd(p, t, tun)
            d = ws.diagnostics()
            assert d["overflow"] == 0 and d["nonfinite"] == 0
            _check_fwd(proj, ref, (shape, waves, persistent))
            if first is None:
                first = proj.clone()
            else:   # launch shapes of one tile shape: the same bits
                assert torch.equal(proj, first), (shape, waves, persistent)
    proj3, _ = _fwd(p, t, dict(base, slices=3))
    _check_fwd(proj3, ref, (shape, "slices 3"))
    tun = dict(base, slices=1)
    proj, ws = _fwd(p, t, tun)
    out = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                           t["angles"], t["w"], dev(G), ws, tuning=tun, reuse_fwd=True)
    torch.cuda.synchronize()
    check_grads({k: out[k] for k in gref}, gref)
    # the backward that recomputes the forward gives the same bits
    out2 = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                            t["angles"], t["w"], dev(G), _lib.Workspace(), tuning=tun)
    for k in out:
        assert torch.equal(out[k], out2[k]), (shape, k)


@pytest.mark.parametrize("shape", [(32, 8), (8, 8)], ids=["32x8", "8x8"])
def test_tile_shape_large_footprints(shape):
    """Footprint rectangles of more than 32 tiles (every tile an instance) in small tiles."""
    tw, th = shape
    _print("case: tile %dx%d, 48 large Gaussians (scales 8-16 mm), 128x128, 4 views: fwd and bwd "
           "against the oracle" % shape)
    p = synth.tiny(seed=31, n=48, nviews=4, det=128)
    rng = np.random.default_rng(32)
    p.scale = np.exp(rng.uniform(np.log(8.0), np.log(16.0), (3, p.n))).astype(np.float32)
    t = problem_tensors(p)
    T = len(p.angles)
    ntiles = (128 // tw) * (128 // th)
    tun = dict(tile_w=tw, tile_h=th, capacity=ntiles * p.n * T)
    proj, ws = _fwd(p, t, tun)
    d = ws.diagnostics()
    assert d["overflow"] == 0 and d["nonfinite"] == 0
    assert d["instances"] > 32 * p.n * T
    ref = oracle.project(p.geom, p.grid, *oracle_inputs(p))
    _check_fwd(proj, ref, shape)
    G = rng.normal(0, 1, ref.shape).astype(np.float32)
    out = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                           t["angles"], t["w"], dev(G), ws, reuse_fwd=True, tuning=tun)
    torch.cuda.synchronize()
    gref = oracle.project_bwd(p.geom, p.grid, *oracle_inputs(p), grad_proj=G)
    check_grads({k: out[k] for k in gref}, gref)


@pytest.mark.parametrize("shape", [(32, 8), (8, 8)], ids=["32x8", "8x8"])
def test_tile_shape_ewa(shape):
    """EWA model: the forward against the oracle's EWA model at every pixel; the backward against
    the 16x16 EWA backward (which test_gpu_ewa checks against differences of the oracle's EWA
    forward; the oracle has no EWA reverse mode) at rounding level."""
    tw, th = shape
    _print("case: EWA model, tile %dx%d, tiny (2000 Gaussians, 48x48, 4 views): fwd against the "
           "oracle, bwd against the 16x16 tiles" % shape)
    p = synth.tiny(seed=51, n=2000, nviews=4, det=48)
    p.geom = dict(p.geom, model="ewa")
    t = problem_tensors(p)
    tun = dict(tile_w=tw, tile_h=th)
    proj, ws = _fwd(p, t, tun)
    ref = oracle.project(p.geom, p.grid, *oracle_inputs(p))
    _check_fwd(proj, ref, shape)
    G = dev(np.random.default_rng(52).normal(0, 1, ref.shape))
    out = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                           t["angles"], t["w"], G, ws, reuse_fwd=True, tuning=tun)
    base = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                            t["angles"], t["w"], G, _lib.Workspace())
    torch.cuda.synchronize()
    check_grads(out, base, norm_bar=1e-5, elem_bar=1e-4)


def test_tile_shapes_agree_at_rounding_level(offset_case):
    p, ref, G, gref = offset_case
    _print("case: every tile shape against 16x16 (forward <= 1e-6 of the maximum, gradients "
           "<= 1e-5 norm-wise)")
    t = problem_tensors(p)
    base, ws = _fwd(p, t, dict(tile_w=16, tile_h=16))
    gbase = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"],
                             t["rho"], t["angles"], t["w"], dev(G), ws, reuse_fwd=True)
    torch.cuda.synchronize()
    for tw, th in SHAPES[1:]:
        tun = dict(tile_w=tw, tile_h=th)
        proj, ws = _fwd(p, t, tun)
        e = (proj - base).abs().max().item() / base.abs().max().item()
        out = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"],
                               t["rho"], t["angles"], t["w"], dev(G), ws, reuse_fwd=True,
                               tuning=tun)
        torch.cuda.synchronize()
        ge = {k: ((out[k] - gbase[k]).norm() / gbase[k].norm()).item() for k in gbase}
        _print((tw, th), "fwd %.2e" % e, {k: "%.1e" % v for k, v in ge.items()})
        assert e <= 1e-6
        assert max(ge.values()) <= 1e-5


def test_autotuner_tries_the_tile_shapes():
    _print("case: plan autotuner on the small phantom (90x75, 8 views): 3 tile shapes x 4 launch "
           "shapes timed; the chosen tuning replays to the eager result")
    p = synth.small_phantom(seed=5)
    t = problem_tensors(p)
    T = len(p.angles)
    bufs = dict(t, proj=torch.empty((T, p.geom["nv"], p.geom["nu"]), device="cuda"))
    G = torch.randn((T, p.geom["nv"], p.geom["nu"]), device="cuda")
    bufs["grad_proj"] = G
    for k, shp in (("g_mu", (3, p.n)), ("g_scale", (3, p.n)), ("g_quat", (4, p.n)),
                   ("g_rho", (p.n,)), ("g_coef", tuple(t["coef"].shape)), ("g_w", (T, p.grid["R"]))):
        bufs[k] = torch.empty(shp, device="cuda")
    plan = _lib.Plan(p.geom, p.grid, p.n, T, bufs)
    try:
        tun, ms = plan.tuning()
        _print("chosen", tun, "candidates", [[round(a, 3), round(b, 3)] for a, b in ms])
        assert len(ms) == _lib.TUNE_CANDIDATES == 12
        # every shape fits this detector, so every candidate was timed
        assert all(a > 0 and b > 0 for a, b in ms)
        assert (tun["tile_w"], tun["tile_h"]) in ((16, 16), (32, 8), (8, 8))
        assert tun["capacity"] > 0
        plan.fwd()
        torch.cuda.synchronize()
        eager, _ = _fwd(p, t, tun)
        assert torch.equal(bufs["proj"], eager)
    finally:
        plan.close()

