"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: forward per pixel |GPU - oracle| <= 1e-4 * max|oracle| of the projection; FFD and
warp outputs <= 2e-5 of their maximum magnitude (FP32 arithmetic on mm-sized values);
gradients per parameter group (dL/dw included) norm-wise <= 1e-4 and element-wise
max |GPU - oracle| <= 1e-3 * max |oracle| against the oracle's adjoint.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2506_22280_amd import _lib, synth
from gpu_helpers import check_grads, dev, max_rel_to_max, oracle_inputs, problem_tensors

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _grid_small(R=2):
    return dict(R=R, nx=7, ny=6, nz=5, origin=[-30.0, -25.0, -28.0], spacing=[9.0, 11.0, 13.0])


def test_ffd_eval_matches_oracle():
    _print("case: ffd_eval R=2 lattice 7x6x5, 3000 points (some outside the lattice)")
    rng = np.random.default_rng(100)
    g = _grid_small()
    coef = rng.normal(0, 2.0, (2, 5, 6, 7, 3)).astype(np.float32)
    x = rng.uniform(-45, 55, (3, 3000)).astype(np.float32)
    U, V = oracle.ffd_eval(g, coef, x)
    d, J = _lib.ffd_eval(g, dev(coef), dev(x))
    torch.cuda.synchronize()
    assert max_rel_to_max(d.cpu().numpy(), U) < 2e-5
    assert max_rel_to_max(J.cpu().numpy(), V) < 2e-5
    w = rng.normal(0, 1, (3, 2)).astype(np.float32)
    dw, Jw = _lib.ffd_eval(g, dev(coef), dev(x), w=dev(w))
    refd = np.einsum("tr,ran->tan", w.astype(np.float64), U)
    refJ = np.einsum("tr,ran->tan", w.astype(np.float64), V)
    assert max_rel_to_max(dw.cpu().numpy(), refd) < 2e-5
    assert max_rel_to_max(Jw.cpu().numpy(), refJ) < 2e-5


def test_deform_matches_oracle():
    _print("case: deform_gaussians tiny problem, 16 views")
    p = synth.tiny(seed=5, n=2000)
    t = problem_tensors(p)
    mu_t, cov_t = _lib.deform_gaussians(p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["w"])
    rm, rc = oracle.deform(p.grid, p.coef, p.mu, p.scale, p.quat, p.w)
    torch.cuda.synchronize()
    assert max_rel_to_max(mu_t.cpu().numpy(), rm) < 2e-6
    assert max_rel_to_max(cov_t.cpu().numpy(), rc) < 2e-5


def _fwd(p, t, tuning=None, ws=None):
    ws = ws or _lib.Workspace()
    proj = _lib.project_fwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                            t["angles"], t["w"], ws, tuning=tuning)
    torch.cuda.synchronize()
    return proj, ws


def test_project_fwd_tiny_all_pixels():
    _print("case: project_fwd tiny (4096 Gaussians, 64x64, 16 views), every pixel")
    p = synth.tiny()
    t = problem_tensors(p)
    proj, ws = _fwd(p, t)
    ref = oracle.project(p.geom, p.grid, *oracle_inputs(p))
    d = ws.diagnostics()
    assert d["overflow"] == 0 and d["nonfinite"] == 0 and d["behind_source"] == 0
    for k in range(ref.shape[0]):
        err = max_rel_to_max(proj[k].cpu().numpy(), ref[k])
        assert err <= 1e-4, (k, err)


def test_project_fwd_ragged_tiles_and_single_wave():
    _print("case: project_fwd small phantom 90x75 (ragged tiles), 8 views, both splat shapes, "
           "1, 3 and (by shape) 8 list slices")
    p = synth.small_phantom()
    t = problem_tensors(p)
    ref = oracle.project(p.geom, p.grid, *oracle_inputs(p))
    for waves in (4, 1):
        for slices in (1, 3, 0):
            proj, _ = _fwd(p, t, tuning=dict(splat_waves=waves, slices=slices))
            for k in range(ref.shape[0]):
                err = max_rel_to_max(proj[k].cpu().numpy(), ref[k])
                assert err <= 1e-4, (waves, slices, k, err)


def test_project_fwd_full_size_sampled():
    """The benchmark's launch: 200k Gaussians, 512x384, a batch of 64 uneven-time views;
    2048 sampled pixels in each of 3 views of the batch against the uncut oracle."""
    _print("case: project_fwd 200k Gaussians 512x384, batch of 64 views, sampled pixels")
    p = synth.batched(seed=0)
    batch = synth.batch_schedule(len(p.angles), 64, seed=0)[0]
    t = problem_tensors(p, batch)
    proj, ws = _fwd(p, t)
    d = ws.diagnostics()
    assert d["overflow"] == 0 and d["nonfinite"] == 0
    rng = np.random.default_rng(7)
    sel = [0, 31, 63]
    m = 2048
    pt = np.repeat(np.arange(len(sel)), m)
    pj = rng.integers(0, p.geom["nv"], pt.size)
    pi = rng.integers(0, p.geom["nu"], pt.size)
    angles, w = p.views(batch[sel])
    ref = oracle.project_pixels(p.geom, p.grid, p.coef, p.mu, p.scale, p.quat, p.rho, angles, w,
                                pt, pj, pi)
    got = proj.cpu().numpy()[np.asarray(sel)[pt], pj, pi]
    pmax = proj.cpu().numpy()[sel].reshape(len(sel), -1).max(1)
    err = np.abs(got - ref) / pmax[pt]
    _print("max err / max", err.max())
    assert err.max() <= 1e-4


def test_project_many_gaussians_small_detector():
    """70,000 Gaussians (above the count from which the canonical FFD stages each workgroup's
    control points in LDS) on a 32x32 detector, 2 views: every pixel, and the adjoint, against the
    oracle."""
    _print("case: 70k Gaussians, 32x32, 2 views: fwd every pixel and bwd against the oracle")
    p = synth.tiny(seed=61, n=70000, nviews=2, det=32)
    t = problem_tensors(p)
    proj, ws = _fwd(p, t)
    d = ws.diagnostics()
    assert d["overflow"] == 0 and d["nonfinite"] == 0
    ref = oracle.project(p.geom, p.grid, *oracle_inputs(p))
    for k in range(ref.shape[0]):
        err = max_rel_to_max(proj[k].cpu().numpy(), ref[k])
        assert err <= 1e-4, (k, err)
    G = np.random.default_rng(62).normal(0, 1, ref.shape).astype(np.float32)
    out = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                           t["angles"], t["w"], dev(G), ws, reuse_fwd=True)
    torch.cuda.synchronize()
    gref = oracle.project_bwd(p.geom, p.grid, *oracle_inputs(p), grad_proj=G)
    check_grads({k: out[k] for k in gref}, gref)


def test_backward_twice_after_one_forward():
    """Backward calls that reuse one forward leave its intermediates intact: a second and a third
    backward on the same workspace equal the first, and a backward that recomputes the forward,
    bit for bit."""
    _print("case: small phantom, one forward, three reusing backward calls")
    p = synth.small_phantom(seed=8)
    t = problem_tensors(p)
    _, ws = _fwd(p, t)
    shape = (len(p.angles), p.geom["nv"], p.geom["nu"])
    rng = np.random.default_rng(81)
    G1, G2 = dev(rng.normal(0, 1, shape)), dev(rng.normal(0, 1, shape))
    args = (p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"], t["angles"],
            t["w"])
    o1 = _lib.project_bwd(*args, G1, ws, reuse_fwd=True)
    o2 = _lib.project_bwd(*args, G2, ws, reuse_fwd=True)
    o3 = _lib.project_bwd(*args, G1, ws, reuse_fwd=True)
    f2 = _lib.project_bwd(*args, G2, _lib.Workspace())
    torch.cuda.synchronize()
    for k in o1:
        assert torch.equal(o1[k], o3[k]), k
        assert torch.equal(o2[k], f2[k]), k


def test_project_deterministic_and_batch_invariant():
    _print("case: bitwise repeatability; batched equals one view per launch")
    p = synth.small_phantom(seed=3)
    t = problem_tensors(p)
    a, _ = _fwd(p, t)
    b, _ = _fwd(p, t)
    assert torch.equal(a, b)
    for k in range(len(p.angles)):
        tk = problem_tensors(p, [k])
        s, _ = _fwd(p, tk)
        assert torch.equal(s[0], a[k])


def test_edge_cases():
    _print("case: edge cases (no Gaussians, off-detector, behind the source, tiny capacity)")
    p = synth.tiny(n=64, nviews=2, det=32)
    t = problem_tensors(p)
    ws = _lib.Workspace()
    # no Gaussians: zeros
    z = _lib.project_fwd(p.geom, p.grid, t["coef"], t["mu"][:, :0].contiguous(),
                         t["scale"][:, :0].contiguous(), t["quat"][:, :0].contiguous(),
                         t["rho"][:0].contiguous(), t["angles"], t["w"], ws)
    torch.cuda.synchronize()
    assert z.abs().max().item() == 0.0
    # a Gaussian far off the detector contributes nothing; one behind the source is counted
    mu = p.mu.copy()
    mu[:, 0] = [0.0, 0.0, 900.0]
    mu[:, 1] = [1500.0, 0.0, 0.0]
    q = dict(t, mu=dev(mu))
    ws2 = _lib.Workspace()
    proj = _lib.project_fwd(p.geom, p.grid, q["coef"], q["mu"], q["scale"], q["quat"], q["rho"],
                            q["angles"], q["w"], ws2)
    d = ws2.diagnostics()
    assert d["behind_source"] >= 1 and d["overflow"] == 0
    assert torch.isfinite(proj).all()
    # a capacity that is too small is reported, never silent
    ws3 = _lib.Workspace()
    _lib.project_fwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                     t["angles"], t["w"], ws3, tuning=dict(capacity=8))
    d = ws3.diagnostics()
    assert d["overflow"] == 1 and d["instances"] > 8


def test_invalid_gaussians_are_skipped():
    _print("case: Gaussians with a NaN or infinite mean, a zero scale, a zero quaternion or a NaN "
           "density among 300 valid ones (3 views 40x40): skipped, counted, zero gradients")
    p = synth.tiny(seed=51, n=305, nviews=3, det=40)
    T = len(p.angles)
    bad = p.n - 5 + np.arange(5)
    p.mu[:, bad[0]] = np.nan
    p.mu[1, bad[1]] = np.inf
    p.scale[0, bad[2]] = 0.0
    p.quat[:, bad[3]] = 0.0
    p.rho[bad[4]] = np.nan
    good = np.arange(p.n - 5)
    t = problem_tensors(p)
    proj, ws = _fwd(p, t)
    d = ws.diagnostics()
    assert d["nonfinite"] == 5 * T and d["overflow"] == 0, d
    keep = (p.coef, p.mu[:, good], p.scale[:, good], p.quat[:, good], p.rho[good], p.angles, p.w)
    ref = oracle.project(p.geom, p.grid, *keep)
    for k in range(T):
        err = max_rel_to_max(proj[k].cpu().numpy(), ref[k])
        assert err <= 1e-4, (k, err)
    G = np.random.default_rng(52).normal(0, 1, ref.shape).astype(np.float32)
    out = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                           t["angles"], t["w"], dev(G), ws, reuse_fwd=True)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    for k in ("g_mu", "g_scale", "g_quat", "g_rho"):
        assert np.all(got[k][..., bad] == 0.0), k
    gref = oracle.project_bwd(p.geom, p.grid, *keep, grad_proj=G)
    sel = {k: got[k][..., good] for k in ("g_mu", "g_scale", "g_quat", "g_rho")}
    check_grads(dict(sel, g_coef=got["g_coef"], g_w=got["g_w"]), gref)


def test_folded_deformation_matches_oracle():
    _print("case: a deformation with det K < 0 (u_x = -2.5 x on the lattice, the means inside its "
           "exact region), 400 Gaussians, 3 views 40x40: rendered, counted, fwd and bwd parity")
    p = synth.tiny(seed=61, n=400, nviews=3, det=40)
    g = p.grid
    x_cp = g["origin"][0] + g["spacing"][0] * np.arange(g["nx"])
    coef = np.zeros_like(p.coef)
    coef[0, :, :, :, 0] = -2.5 * x_cp[None, None, :]    # cubic B-splines reproduce it exactly
    p.coef = coef.astype(np.float32)
    p.w = np.tile(np.array([[1.0, 0.0, 0.0]], np.float32), (len(p.angles), 1))
    T = len(p.angles)
    t = problem_tensors(p)
    proj, ws = _fwd(p, t)
    d = ws.diagnostics()
    assert d["folded"] == p.n * T and d["nonfinite"] == 0, d
    ref = oracle.project(p.geom, p.grid, *oracle_inputs(p))
    for k in range(T):
        err = max_rel_to_max(proj[k].cpu().numpy(), ref[k])
        assert err <= 1e-4, (k, err)
    G = np.random.default_rng(62).normal(0, 1, ref.shape).astype(np.float32)
    out = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                           t["angles"], t["w"], dev(G), ws, reuse_fwd=True)
    torch.cuda.synchronize()
    gref = oracle.project_bwd(p.geom, p.grid, *oracle_inputs(p), grad_proj=G)
    check_grads({k: out[k] for k in gref}, gref)


# ------------------------------------------------------------------------------------------------
# Backward
def _bwd_problem():
    p = synth.tiny(seed=9, n=600, nviews=4, det=40)
    G = np.random.default_rng(10).normal(0, 1, (4, 40, 40)).astype(np.float32)
    return p, G


def test_project_bwd_matches_oracle():
    _print("case: project_bwd tiny (600 Gaussians, 4 views, 40x40) against the oracle adjoint")
    p, G = _bwd_problem()
    t = problem_tensors(p)
    ws = _lib.Workspace()
    _lib.project_fwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                     t["angles"], t["w"], ws)
    out = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                           t["angles"], t["w"], dev(G), ws, reuse_fwd=True)
    torch.cuda.synchronize()
    ref = oracle.project_bwd(p.geom, p.grid, *oracle_inputs(p), grad_proj=G)
    check_grads({k: out[k] for k in ref}, ref)
    # recomputing the forward inside the backward gives the same bits
    out2 = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                            t["angles"], t["w"], dev(G), _lib.Workspace(), reuse_fwd=False)
    for k in out:
        assert torch.equal(out[k], out2[k]), k


def test_signed_densities_match_oracle():
    _print("case: densities of both signs (tiny, 2000 Gaussians, 8 views 48x48): fwd and bwd "
           "against the oracle")
    p = synth.tiny(seed=21, n=2000, nviews=8, det=48)
    flip = np.random.default_rng(22).random(p.n) < 0.3
    p.rho = np.where(flip, -p.rho, p.rho).astype(np.float32)
    t = problem_tensors(p)
    proj, ws = _fwd(p, t)
    ref = oracle.project(p.geom, p.grid, *oracle_inputs(p))
    for k in range(ref.shape[0]):
        err = max_rel_to_max(proj[k].cpu().numpy(), ref[k])
        assert err <= 1e-4, (k, err)
    G = np.random.default_rng(23).normal(0, 1, ref.shape).astype(np.float32)
    out = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                           t["angles"], t["w"], dev(G), ws, reuse_fwd=True)
    torch.cuda.synchronize()
    gref = oracle.project_bwd(p.geom, p.grid, *oracle_inputs(p), grad_proj=G)
    check_grads({k: out[k] for k in gref}, gref)


def test_offset_anisotropic_detector_matches_oracle():
    _print("case: exact model, 90x75 detector with pitches 0.9 x 1.3 mm and offsets (5, -2) mm, "
           "1024 Gaussians, 4 views: fwd and bwd against the oracle")
    p = synth.tiny(seed=41, n=1024, nviews=4, det=64)
    p.geom = dict(p.geom, nu=90, nv=75, pitch_u=0.9, pitch_v=1.3, off_u=5.0, off_v=-2.0)
    t = problem_tensors(p)
    proj, ws = _fwd(p, t)
    d = ws.diagnostics()
    assert d["overflow"] == 0 and d["nonfinite"] == 0
    ref = oracle.project(p.geom, p.grid, *oracle_inputs(p))
    for k in range(ref.shape[0]):
        err = max_rel_to_max(proj[k].cpu().numpy(), ref[k])
        assert err <= 1e-4, (k, err)
    G = np.random.default_rng(42).normal(0, 1, ref.shape).astype(np.float32)
    out = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                           t["angles"], t["w"], dev(G), ws, reuse_fwd=True)
    torch.cuda.synchronize()
    gref = oracle.project_bwd(p.geom, p.grid, *oracle_inputs(p), grad_proj=G)
    check_grads({k: out[k] for k in gref}, gref)


def test_large_footprints_match_oracle():
    _print("case: 48 large Gaussians (scales 8-16 mm) on a 128x128 detector, 4 views: footprint "
           "rectangles of more than 32 tiles (every tile an instance); fwd and bwd against the oracle")
    p = synth.tiny(seed=31, n=48, nviews=4, det=128)
    rng = np.random.default_rng(32)
    p.scale = np.exp(rng.uniform(np.log(8.0), np.log(16.0), (3, p.n))).astype(np.float32)
    t = problem_tensors(p)
    T = len(p.angles)
    # capacity for every tile of the 8x8-tile detector (the default, 16 per (view, Gaussian),
    # would overflow, which the diagnostics report)
    proj, ws = _fwd(p, t, tuning=dict(capacity=64 * p.n * T))
    d = ws.diagnostics()
    assert d["overflow"] == 0 and d["nonfinite"] == 0
    # on average more than 32 instances per (view, Gaussian): rectangles above 32 tiles
    assert d["instances"] > 32 * p.n * T
    ref = oracle.project(p.geom, p.grid, *oracle_inputs(p))
    for k in range(ref.shape[0]):
        err = max_rel_to_max(proj[k].cpu().numpy(), ref[k])
        assert err <= 1e-4, (k, err)
    G = rng.normal(0, 1, ref.shape).astype(np.float32)
    out = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                           t["angles"], t["w"], dev(G), ws, reuse_fwd=True,
                           tuning=dict(capacity=64 * p.n * T))
    torch.cuda.synchronize()
    gref = oracle.project_bwd(p.geom, p.grid, *oracle_inputs(p), grad_proj=G)
    check_grads({k: out[k] for k in gref}, gref)


def test_project_bwd_identities():
    _print("case: gradient identities on the GPU (rho-linearity, quaternion, homogeneity)")
    p, G = _bwd_problem()
    t = problem_tensors(p)
    ws = _lib.Workspace()
    proj = _lib.project_fwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                            t["angles"], t["w"], ws)
    out = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                           t["angles"], t["w"], dev(G), ws, reuse_fwd=True)
    torch.cuda.synchronize()
    L = float((proj.double().cpu().numpy() * G).sum())
    lhs = float((out["g_rho"].double().cpu().numpy() * p.rho).sum())
    assert abs(lhs - L) <= 1e-5 * abs(L)
    qg = (out["g_quat"].cpu().numpy().astype(np.float64) * p.quat).sum(0)
    scale = np.abs(out["g_quat"].cpu().numpy()).max()
    assert np.abs(qg).max() <= 1e-5 * scale
    t1 = problem_tensors(p, [1])
    ws1 = _lib.Workspace()
    o1 = _lib.project_bwd(p.geom, p.grid, t1["coef"], t1["mu"], t1["scale"], t1["quat"],
                          t1["rho"], t1["angles"], t1["w"], dev(G[1:2]), ws1)
    torch.cuda.synchronize()
    for r in range(p.grid["R"]):
        lhs = float(p.w[1, r]) * float(o1["g_w"][0, r])
        rhs = float((p.coef[r].astype(np.float64) * o1["g_coef"][r].double().cpu().numpy()).sum())
        assert abs(lhs - rhs) <= 2e-4 * max(abs(lhs), 1e-12), (r, lhs, rhs)


def test_project_bwd_full_size_sampled():
    """The benchmark's launch: 200k Gaussians, 512x384, a batch of 64 uneven-time views, through
    an autotuned plan. dL/dI is nonzero on 2 x 96 sampled pixels (views 0 and 63), so that the
    oracle's adjoint over those pixels alone is the whole gradient; then with a dense dL/dI the
    rho-linearity identity sum_n rho_n dL/drho_n = L at full size."""
    _print("case: project_bwd 200k Gaussians 512x384, batch of 64 views (plan), sampled pixels")
    p = synth.batched(seed=0)
    batch = synth.batch_schedule(len(p.angles), 64, seed=0)[0]
    angles, w = p.views(batch)
    T, n, nv, nu = len(batch), p.n, p.geom["nv"], p.geom["nu"]
    rng = np.random.default_rng(11)
    sel, m = np.array([0, 63]), 96
    pt = np.repeat(sel, m)
    pj = rng.integers(0, nv, pt.size)
    pi = rng.integers(0, nu, pt.size)
    pg = rng.normal(0, 1, pt.size).astype(np.float32)
    G = np.zeros((T, nv, nu), np.float32)
    np.add.at(G, (pt, pj, pi), pg)
    b = dict(problem_tensors(p, batch), proj=torch.empty((T, nv, nu), device="cuda"),
             grad_proj=dev(G), g_mu=torch.empty((3, n), device="cuda"),
             g_scale=torch.empty((3, n), device="cuda"), g_quat=torch.empty((4, n), device="cuda"),
             g_rho=torch.empty((n,), device="cuda"), g_coef=torch.empty_like(dev(p.coef)),
             g_w=torch.empty((T, p.grid["R"]), device="cuda"))
    with _lib.Plan(p.geom, p.grid, n, T, b) as plan:
        _print("tuning", plan.tuning()[0])
        plan.fwd()
        plan.bwd()
        diag, resized = plan.check()
        assert not resized and diag["overflow"] == 0 and diag["nonfinite"] == 0
        got = {k: b[k].double().cpu().numpy() for k in
               ("g_mu", "g_scale", "g_quat", "g_rho", "g_coef", "g_w")}
        # a dense dL/dI through the same plan: rho-linearity of the whole projection
        Gd = rng.normal(0, 1, (T, nv, nu)).astype(np.float32)
        b["grad_proj"].copy_(dev(Gd))
        plan.bwd()
        torch.cuda.synchronize()
        L = float((b["proj"].double().cpu().numpy() * Gd).sum())
        lhs = float((b["g_rho"].double().cpu().numpy() * p.rho).sum())
        _print("rho-linearity", lhs, L)
        assert abs(lhs - L) <= 1e-5 * abs(L)
    ref = oracle.project_bwd(p.geom, p.grid, p.coef, p.mu, p.scale, p.quat, p.rho, angles, w,
                             pixels=(pt, pj, pi, pg))
    check_grads({k: got[k] for k in ref}, ref)


@pytest.mark.parametrize("R", [1, 2, 4, 5, 8])
def test_every_rank_matches_oracle(R):
    """Motion ranks 1 to 8 (each compiled separately in the set-up, the per-Gaussian adjoint and
    the coefficient gather): fwd and bwd of a small problem against the oracle."""
    _print("case: rank %d FFD on 8^3, 500 Gaussians, 3 views 40x40: fwd and bwd" % R)
    p = synth.tiny(seed=70 + R, n=500, nviews=3, det=40)
    rng = np.random.default_rng(80 + R)
    p.grid = dict(p.grid, R=R)
    p.coef = rng.normal(0.0, 2.0, (R, 8, 8, 8, 3)).astype(np.float32)
    p.w = rng.uniform(-0.6, 0.6, (len(p.angles), R)).astype(np.float32)
    t = problem_tensors(p)
    proj, ws = _fwd(p, t)
    ref = oracle.project(p.geom, p.grid, *oracle_inputs(p))
    for k in range(ref.shape[0]):
        err = max_rel_to_max(proj[k].cpu().numpy(), ref[k])
        assert err <= 1e-4, (k, err)
    G = rng.normal(0, 1, ref.shape).astype(np.float32)
    out = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                           t["angles"], t["w"], dev(G), ws, reuse_fwd=True)
    torch.cuda.synchronize()
    gref = oracle.project_bwd(p.geom, p.grid, *oracle_inputs(p), grad_proj=G)
    check_grads({k: out[k] for k in gref}, gref)


@pytest.mark.parametrize("seed", range(6))
def test_random_configurations_match_oracle(seed):
    """Seeded random combinations of what the other cases vary one at a time: detector size
    (ragged tiles), unequal pitches, offsets, source and detector distances, motion rank, number
    of views and Gaussians, Gaussian sizes and density signs; fwd and bwd against the oracle."""
    rng = np.random.default_rng(1000 + seed)
    R = int(rng.integers(1, 6))
    nviews = int(rng.integers(1, 5))
    n = int(rng.integers(50, 900))
    nu, nv = int(rng.integers(17, 80)), int(rng.integers(17, 80))
    _print("case: random configuration seed %d: R=%d, %d views, %d Gaussians, %dx%d detector"
           % (seed, R, nviews, n, nu, nv))
    p = synth.tiny(seed=2000 + seed, n=n, nviews=nviews, det=32)
    p.geom = dict(p.geom, nu=nu, nv=nv, pitch_u=float(rng.uniform(0.6, 1.6)),
                  pitch_v=float(rng.uniform(0.6, 1.6)), off_u=float(rng.uniform(-6, 6)),
                  off_v=float(rng.uniform(-6, 6)), sid=float(rng.uniform(600, 1100)))
    p.geom["sdd"] = p.geom["sid"] * float(rng.uniform(1.2, 1.8))
    p.scale = np.exp(rng.uniform(np.log(0.6), np.log(6.0), (3, n))).astype(np.float32)
    p.rho = np.where(rng.random(n) < 0.2, -p.rho, p.rho).astype(np.float32)
    p.grid = dict(p.grid, R=R)
    p.coef = rng.normal(0.0, 1.5, (R, 8, 8, 8, 3)).astype(np.float32)
    p.angles = rng.uniform(0, 2 * np.pi, nviews).astype(np.float32)
    p.w = rng.uniform(-0.5, 0.5, (nviews, R)).astype(np.float32)
    t = problem_tensors(p)
    proj, ws = _fwd(p, t, tuning=dict(capacity=64 * n * nviews))
    d = ws.diagnostics()
    assert d["overflow"] == 0 and d["nonfinite"] == 0, d
    ref = oracle.project(p.geom, p.grid, *oracle_inputs(p))
    for k in range(nviews):
        err = max_rel_to_max(proj[k].cpu().numpy(), ref[k])
        assert err <= 1e-4, (k, err)
    G = rng.normal(0, 1, ref.shape).astype(np.float32)
    out = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                           t["angles"], t["w"], dev(G), ws, reuse_fwd=True,
                           tuning=dict(capacity=64 * n * nviews))
    torch.cuda.synchronize()
    gref = oracle.project_bwd(p.geom, p.grid, *oracle_inputs(p), grad_proj=G)
    check_grads({k: out[k] for k in gref}, gref)


def test_temporal_weights_matches_oracle():
    _print("case: temporal weights, 40 control values x rank 3, 1320 time points (some outside)")
    rng = np.random.default_rng(61)
    Ct, R, t0, dt = 40, 3, 0.0, 4.0
    ctrl = rng.normal(0, 5.0, (Ct, R)).astype(np.float32)
    times = rng.uniform(-8.0, dt * Ct + 8.0, 1320).astype(np.float32)
    w = _lib.temporal_weights(dev(ctrl), t0, dt, dev(times))
    ref = oracle.temporal_weights(ctrl, t0, dt, times)
    gw = rng.normal(0, 1, (1320, R)).astype(np.float32)
    gc = _lib.temporal_weights_bwd(Ct, t0, dt, dev(times), dev(gw))
    gref = oracle.temporal_weights_bwd(Ct, t0, dt, times, gw)
    torch.cuda.synchronize()
    assert max_rel_to_max(w.cpu().numpy(), ref) < 2e-6
    assert max_rel_to_max(gc.cpu().numpy(), gref) < 2e-6
