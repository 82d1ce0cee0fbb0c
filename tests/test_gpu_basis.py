"""The second ablation's motion model (Sec. 4.3: a spatial basis stored per Gaussian instead of
the lattice) on the GPU, through the C ABI, against the FP64 oracle's basis model: the forward at
every pixel (<= 1e-4 of the image maximum), the gradients per group norm-wise (<= 1e-4) and
element-wise (<= 1e-3 of the group's maximum), and a basis sampled from the FFD at the means reproduces the lattice model's forward.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2506_22280_amd import _lib, synth
from gpu_helpers import check_grads, dev, max_rel_to_max, problem_tensors

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _basis(p, rng):
    """A basis like the lattice's at the means plus independent per-Gaussian variation."""
    U, V = oracle.ffd_eval(p.grid, p.coef, p.mu)
    b = np.concatenate([U, V], axis=1)
    return b + rng.normal(0.0, 0.3, b.shape) * np.abs(b).mean(axis=2, keepdims=True)


def test_basis_fwd_matches_oracle_and_reduces_to_the_lattice():
    _print("case: basis-model project_fwd tiny (4096 Gaussians, 64x64, 8 views), every pixel")
    p = synth.tiny(seed=8, nviews=8)
    t = problem_tensors(p)
    rng = np.random.default_rng(9)
    basis = _basis(p, rng)
    ws = _lib.Workspace()
    got = _lib.project_basis_fwd(p.geom, p.grid, dev(basis), t["mu"], t["scale"], t["quat"],
                                 t["rho"], t["angles"], t["w"], ws)
    torch.cuda.synchronize()
    ref = oracle.project(p.geom, p.grid, None, p.mu, p.scale, p.quat, p.rho, p.angles, p.w,
                         basis=basis)
    for k in range(ref.shape[0]):
        assert max_rel_to_max(got[k].cpu().numpy(), ref[k]) <= 1e-4, k
    # the lattice's own basis at the means gives the lattice model's image
    U, V = oracle.ffd_eval(p.grid, p.coef, p.mu)
    same = _lib.project_basis_fwd(p.geom, p.grid, dev(np.concatenate([U, V], axis=1)), t["mu"],
                                  t["scale"], t["quat"], t["rho"], t["angles"], t["w"], ws)
    lat = _lib.project_fwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                           t["angles"], t["w"], _lib.Workspace())
    torch.cuda.synchronize()
    assert max_rel_to_max(same.cpu().numpy(), lat.cpu().numpy()) <= 2e-5


@pytest.mark.parametrize("tile", [None, (32, 8), (8, 8)], ids=["16x16", "32x8", "8x8"])
def test_basis_bwd_matches_oracle(tile):
    _print("case: basis-model project_bwd small phantom (2048 Gaussians, 90x75, 4 views), tile %s"
           % (tile or "16x16",))
    p = synth.small_phantom(n=2048, nviews=4, seed=2)
    t = problem_tensors(p)
    rng = np.random.default_rng(10)
    basis = _basis(p, rng)
    c = rng.normal(0.0, 1.0, (4, p.geom["nv"], p.geom["nu"]))
    tun = dict(tile_w=tile[0], tile_h=tile[1]) if tile else None
    ws = _lib.Workspace()
    g = _lib.project_basis_bwd(p.geom, p.grid, dev(basis), t["mu"], t["scale"], t["quat"],
                               t["rho"], t["angles"], t["w"], dev(c), ws, tuning=tun)
    torch.cuda.synchronize()
    d = ws.diagnostics()
    assert d["overflow"] == 0 and d["nonfinite"] == 0, d
    ref = oracle.project_bwd(p.geom, p.grid, None, p.mu, p.scale, p.quat, p.rho, p.angles, p.w,
                             grad_proj=c.astype(np.float32).astype(np.float64), basis=basis)
    check_grads({k: g[k] for k in ref}, ref)
