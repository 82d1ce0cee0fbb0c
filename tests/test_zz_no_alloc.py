"""The allocation-free forward (digs_project_fwd_noalloc, through the C ABI) against the
workspace forward (digs_project_fwd) on the same inputs: two calls in a row, the second with a
smaller problem, each equal to the workspace call bit for bit (the same kernels on the same data;
this exceeds the forward's parity bar of 1e-4 of the image maximum), with the diagnostics the call
writes to its device buffer; an overflow reported there; a problem larger than the fixed array
rejected before any device work."""
import ctypes

import pytest
import torch

from paper_2506_22280_amd import _lib, synth
from gpu_helpers import problem_tensors

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _both(p, tuning=None):
    t = problem_tensors(p)
    ws = _lib.Workspace()
    ref = _lib.project_fwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"],
                           t["angles"], t["w"], ws, tuning=tuning)
    ref_diag = ws.diagnostics()
    diag = torch.zeros(ctypes.sizeof(_lib.Diag), dtype=torch.uint8, device="cuda")
    got = _lib.project_fwd_noalloc(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"],
                                   t["rho"], t["angles"], t["w"], tuning=tuning, diag=diag)
    torch.cuda.synchronize()
    return got, ref, _lib.diag_from_device(diag), ref_diag


def test_noalloc_forward_equals_workspace_forward_twice():
    _print("case: no-allocation forward, tiny problem (4096 Gaussians, 16 views, 64x64), then a "
           "smaller one (512 Gaussians, 4 views, 48x48)")
    for p in (synth.tiny(seed=1), synth.tiny(seed=2, n=512, nviews=4, det=48)):
        got, ref, d, rd = _both(p)
        _print("diagnostics", d)
        assert torch.equal(got, ref)
        assert d["overflow"] == 0 and d["nonfinite"] == 0
        assert d["instances"] == rd["instances"] > 0


def test_noalloc_forward_with_other_tile_shapes():
    _print("case: no-allocation forward with 32x8 and 8x8 tiles and 3 list slices (tiny problem)")
    p = synth.tiny(seed=5, n=2048, nviews=4, det=64)
    for tun in (dict(tile_w=32, tile_h=8), dict(tile_w=8, tile_h=8, slices=3)):
        got, ref, d, rd = _both(p, tuning=tun)
        assert torch.equal(got, ref), tun
        assert d["overflow"] == 0 and d["instances"] == rd["instances"] > 0


def test_noalloc_forward_reports_overflow():
    _print("case: no-allocation forward with an instance capacity of 8: overflow reported")
    p = synth.tiny(seed=3, n=256, nviews=2, det=32)
    got, ref, d, rd = _both(p, tuning=dict(capacity=8))
    assert d["overflow"] == 1 and rd["overflow"] == 1
    assert d["instances"] == rd["instances"] > 8


def test_noalloc_forward_rejects_problems_beyond_the_array():
    _print("case: a problem whose forward needs more than the fixed array: DIGS_ESCRATCH")
    p = synth.tiny(seed=4, n=4096, nviews=16, det=64)
    t = problem_tensors(p)
    with pytest.raises(_lib.DigsError) as e:
        _lib.project_fwd_noalloc(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"],
                                 t["rho"], t["angles"], t["w"],
                                 tuning=dict(capacity=_lib.NOALLOC_SCRATCH_BYTES // 4))
    assert e.value.code == -6
