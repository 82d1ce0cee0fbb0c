"""The 2D-Gaussian (EWA) projection model of Eq. 4 on the GPU, through the C ABI.

Forward: every pixel against the FP64 oracle's EWA model (<= 1e-4 of the image maximum, as for
the exact model), on the 64x64 tiny problem and on a ragged detector with offsets; the GPU's
EWA-minus-exact difference against the oracle's. Backward: the gradients of a linear functional
L = sum_p c_p I_p against central differences of the FP64 oracle's EWA forward (the oracle has
no EWA reverse mode), per parameter group norm-wise and element-wise. Plan replays equal the eager call.
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


def _ewa(p, **kw):
    p.geom = dict(p.geom, model="ewa", **kw)
    return p


def _fwd(p, t, ws=None, tuning=None):
    ws = ws or _lib.Workspace()
    proj = _lib.project_fwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                            t["angles"], t["w"], ws, tuning=tuning)
    torch.cuda.synchronize()
    return proj, ws


def test_ewa_fwd_tiny_all_pixels():
    _print("case: EWA project_fwd tiny (4096 Gaussians, 64x64, 16 views), every pixel")
    p = _ewa(synth.tiny())
    t = problem_tensors(p)
    proj, ws = _fwd(p, t)
    ref = oracle.project(p.geom, p.grid, *oracle_inputs(p))
    d = ws.diagnostics()
    assert d["overflow"] == 0 and d["nonfinite"] == 0
    for k in range(ref.shape[0]):
        err = max_rel_to_max(proj[k].cpu().numpy(), ref[k])
        assert err <= 1e-4, (k, err)


def test_ewa_fwd_signed_densities():
    _print("case: EWA project_fwd with densities of both signs (tiny, 2000 Gaussians, 8 views)")
    p = _ewa(synth.tiny(seed=24, n=2000, nviews=8, det=48))
    flip = np.random.default_rng(25).random(p.n) < 0.3
    p.rho = np.where(flip, -p.rho, p.rho).astype(np.float32)
    t = problem_tensors(p)
    proj, _ = _fwd(p, t)
    ref = oracle.project(p.geom, p.grid, *oracle_inputs(p))
    for k in range(ref.shape[0]):
        err = max_rel_to_max(proj[k].cpu().numpy(), ref[k])
        assert err <= 1e-4, (k, err)


def test_ewa_fwd_ragged_detector_with_offsets():
    _print("case: EWA project_fwd small phantom, 90x75 detector, offsets (7.5, -3) mm, 4 views")
    p = _ewa(synth.small_phantom(n=2048, nviews=4), off_u=7.5, off_v=-3.0)
    t = problem_tensors(p)
    proj, _ = _fwd(p, t)
    ref = oracle.project(p.geom, p.grid, *oracle_inputs(p))
    for k in range(ref.shape[0]):
        err = max_rel_to_max(proj[k].cpu().numpy(), ref[k])
        assert err <= 1e-4, (k, err)


@pytest.mark.parametrize("seed", range(4))
def test_ewa_random_configurations_match_oracle(seed):
    """Seeded random geometry (detector size, pitches, offsets, distances), rank, views and
    Gaussian sizes and signs: the EWA forward at every pixel against the oracle's EWA model."""
    rng = np.random.default_rng(3000 + seed)
    R, nviews, n = int(rng.integers(1, 6)), int(rng.integers(1, 5)), int(rng.integers(50, 900))
    nu, nv = int(rng.integers(17, 80)), int(rng.integers(17, 80))
    _print("case: EWA random configuration seed %d: R=%d, %d views, %d Gaussians, %dx%d"
           % (seed, R, nviews, n, nu, nv))
    p = synth.tiny(seed=4000 + seed, n=n, nviews=nviews, det=32)
    sid = float(rng.uniform(600, 1100))
    p = _ewa(p, nu=nu, nv=nv, pitch_u=float(rng.uniform(0.6, 1.6)),
             pitch_v=float(rng.uniform(0.6, 1.6)), off_u=float(rng.uniform(-6, 6)),
             off_v=float(rng.uniform(-6, 6)), sid=sid, sdd=sid * float(rng.uniform(1.2, 1.8)))
    p.scale = np.exp(rng.uniform(np.log(0.6), np.log(6.0), (3, n))).astype(np.float32)
    p.rho = np.where(rng.random(n) < 0.2, -p.rho, p.rho).astype(np.float32)
    p.grid = dict(p.grid, R=R)
    p.coef = rng.normal(0.0, 1.5, (R, 8, 8, 8, 3)).astype(np.float32)
    p.angles = rng.uniform(0, 2 * np.pi, nviews).astype(np.float32)
    p.w = rng.uniform(-0.5, 0.5, (nviews, R)).astype(np.float32)
    t = problem_tensors(p)
    ws = _lib.Workspace()
    proj = _lib.project_fwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                            t["angles"], t["w"], ws, tuning=dict(capacity=64 * n * nviews))
    torch.cuda.synchronize()
    d = ws.diagnostics()
    assert d["overflow"] == 0 and d["nonfinite"] == 0, d
    ref = oracle.project(p.geom, p.grid, *oracle_inputs(p))
    for k in range(nviews):
        err = max_rel_to_max(proj[k].cpu().numpy(), ref[k])
        assert err <= 1e-4, (k, err)


def test_ewa_minus_exact_matches_oracle():
    _print("case: EWA - exact on the GPU against the oracle's difference (tiny, 4 views)")
    p = synth.tiny(seed=3, nviews=4)
    t = problem_tensors(p)
    exact, _ = _fwd(p, t)
    ref_exact = oracle.project(p.geom, p.grid, *oracle_inputs(p))
    q = _ewa(synth.tiny(seed=3, nviews=4))
    ewa, _ = _fwd(q, t)
    ref_ewa = oracle.project(q.geom, q.grid, *oracle_inputs(q))
    got = (ewa - exact).double().cpu().numpy()
    ref = ref_ewa - ref_exact
    scale = np.abs(ref_exact).max()
    dev_ = np.abs(ref).max() / scale
    _print("oracle max |EWA - exact| / max = %.3e" % dev_)
    assert dev_ > 1e-5          # the models differ measurably
    assert np.abs(got - ref).max() <= 2e-4 * scale


def _fd_problem():
    p = _ewa(synth.tiny(seed=21, n=40, nviews=2, det=40))
    p.geom = dict(p.geom, pitch_u=1.6, pitch_v=1.6)
    return p


def test_ewa_bwd_against_oracle_differences():
    _print("case: EWA project_bwd against central differences of the FP64 oracle (40 Gaussians)")
    p = _fd_problem()
    t = problem_tensors(p)
    T = len(p.angles)
    rng = np.random.default_rng(22)
    c = rng.normal(0.0, 1.0, (T, p.geom["nv"], p.geom["nu"]))
    g = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                         t["angles"], t["w"], dev(c), _lib.Workspace())
    torch.cuda.synchronize()
    base = dict(coef=p.coef.astype(np.float64), mu=p.mu.astype(np.float64),
                scale=p.scale.astype(np.float64), quat=p.quat.astype(np.float64),
                rho=p.rho.astype(np.float64), w=p.w.astype(np.float64))
    ang = p.angles.astype(np.float64)

    def loss(Q):
        img = oracle.project(p.geom, p.grid, Q["coef"], Q["mu"], Q["scale"], Q["quat"], Q["rho"],
                             ang, Q["w"])
        return float((img * c).sum())

    steps = dict(mu=1e-4, scale=1e-5, quat=1e-6, rho=1e-4, coef=1e-4, w=1e-5)
    got, ref = {}, {}
    for k, h in steps.items():
        gk = g["g_" + k].double().cpu().numpy().ravel()
        flat = base[k].ravel()
        if k == "coef":   # the entries near the Gaussians (largest gradients) and a few others
            order = np.argsort(-np.abs(gk))
            idx = np.concatenate([order[:40], rng.choice(order[40:], 10, replace=False)])
        else:
            idx = np.arange(flat.size)
        fd = np.zeros(idx.size)
        for j, e in enumerate(idx):
            vals = []
            for sgn in (1.0, -1.0):
                pert = flat.copy()
                pert[e] += sgn * h
                vals.append(loss(dict(base, **{k: pert.reshape(base[k].shape)})))
            fd[j] = (vals[0] - vals[1]) / (2 * h)
        got[k], ref[k] = gk[idx], fd
    check_grads(got, ref)


def test_ewa_plan_replays_equal_eager():
    _print("case: EWA plan (graph) forward and backward equal the eager calls, 3 replays")
    p = _ewa(synth.tiny(seed=4, n=3000, nviews=8))
    t = problem_tensors(p)
    T = len(p.angles)
    c = torch.randn((T, p.geom["nv"], p.geom["nu"]), device="cuda",
                    generator=torch.Generator("cuda").manual_seed(5))
    bufs = dict(t, proj=torch.empty((T, p.geom["nv"], p.geom["nu"]), device="cuda"), grad_proj=c,
                g_mu=torch.empty_like(t["mu"]), g_scale=torch.empty_like(t["scale"]),
                g_quat=torch.empty_like(t["quat"]), g_rho=torch.empty_like(t["rho"]),
                g_coef=torch.empty_like(t["coef"]), g_w=torch.empty_like(t["w"]))
    with _lib.Plan(p.geom, p.grid, p.n, T, bufs) as plan:
        # the eager calls with the tile shape and list slices the autotuner chose
        tun = plan.tuning()[0]
        shape = {k: tun[k] for k in ("tile_w", "tile_h", "slices")}
        eager, _ = _fwd(p, t, tuning=shape)
        g_eager = _lib.project_bwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"],
                                   t["rho"], t["angles"], t["w"], c, _lib.Workspace(),
                                   tuning=shape)
        for _ in range(3):
            plan.fwd()
            plan.bwd()
            torch.cuda.synchronize()
            assert torch.equal(bufs["proj"], eager)
            for k in ("g_mu", "g_scale", "g_quat", "g_rho", "g_coef", "g_w"):
                assert torch.equal(bufs[k], g_eager[k]), k
