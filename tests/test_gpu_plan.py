"""The batched path (digs_plan_*): replays (HIP graphs, direct launches, or the faster of the
two) equal the eager calls bit for bit, also after eager work and synchronisations between
replays and after new inputs are written into the plan's buffers; every autotuner candidate gives the same bits; an instance-capacity overflow is
detected, the plan grows and the repeated call is complete."""
import numpy as np
import pytest
import torch

from paper_2506_22280_amd import _lib, synth
from gpu_helpers import dev

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _buffers(p, idx):
    angles, w = p.views(idx)
    T, n = len(idx), p.n
    nv, nu = p.geom["nv"], p.geom["nu"]
    rng = np.random.default_rng(5)
    b = dict(coef=dev(p.coef), mu=dev(p.mu), scale=dev(p.scale), quat=dev(p.quat),
             rho=dev(p.rho), angles=dev(angles), w=dev(w),
             proj=torch.empty((T, nv, nu), device="cuda"),
             grad_proj=dev(rng.normal(0, 1, (T, nv, nu))),
             g_mu=torch.empty((3, n), device="cuda"), g_scale=torch.empty((3, n), device="cuda"),
             g_quat=torch.empty((4, n), device="cuda"), g_rho=torch.empty((n,), device="cuda"),
             g_coef=torch.empty_like(dev(p.coef)), g_w=torch.empty((T, p.grid["R"]), device="cuda"))
    return b


def _eager(p, b, tuning=None):
    ws = _lib.Workspace()
    proj = _lib.project_fwd(p.geom, p.grid, b["coef"], b["mu"], b["scale"], b["quat"], b["rho"],
                            b["angles"], b["w"], ws, tuning=tuning)
    g = _lib.project_bwd(p.geom, p.grid, b["coef"], b["mu"], b["scale"], b["quat"], b["rho"],
                         b["angles"], b["w"], b["grad_proj"], ws, tuning=tuning, reuse_fwd=True)
    torch.cuda.synchronize()
    return proj, g


_GRADS = ("g_mu", "g_scale", "g_quat", "g_rho", "g_coef", "g_w")


@pytest.mark.parametrize("nviews,replay", [(8, "timed"), (6, "timed"), (8, "graph"),
                                           (8, "direct")])
def test_plan_replays_equal_eager(nviews, replay):
    _print("case: plan (autotuned) replays (%s) vs eager, small phantom, %d views"
           % (replay, nviews))
    p = synth.small_phantom(n=2048, nviews=nviews, seed=4)
    idx = np.arange(nviews)
    b = _buffers(p, idx)
    with _lib.Plan(p.geom, p.grid, p.n, nviews, b, replay=replay) as plan:
        tuning, ms = plan.tuning()
        _print("chosen", tuning, "timings", ms)
        assert tuning["capacity"] > 0
        # eager calls with the tile shape and list slices the autotuner chose
        shape = {k: tuning[k] for k in ("tile_w", "tile_h", "slices")}
        ref_proj, ref_g = _eager(p, b, tuning=shape)
        for rep in range(3):
            b["proj"].fill_(-1.0)
            for k in _GRADS:
                b[k].fill_(-1.0)
            plan.fwd()
            plan.bwd()
            torch.cuda.synchronize()
            assert torch.equal(b["proj"], ref_proj), rep
            for k in _GRADS:
                assert torch.equal(b[k], ref_g[k]), (rep, k)
            # eager work of the program itself between replays
            _eager(p, b, tuning=shape)
        # a new batch: other views written into the same buffers
        p2 = synth.small_phantom(n=2048, nviews=2 * nviews, seed=4)
        a2, w2 = p2.views(np.arange(nviews, 2 * nviews))
        b["angles"].copy_(dev(a2))
        b["w"].copy_(dev(w2))
        plan.fwd()
        plan.bwd()
        diag, resized = plan.check()
        assert not resized and diag["overflow"] == 0
        got = b["proj"].clone()
        gg = {k: b[k].clone() for k in _GRADS}
        ref2_proj, ref2_g = _eager(p, b, tuning=shape)
        assert torch.equal(got, ref2_proj)
        for k in _GRADS:
            assert torch.equal(gg[k], ref2_g[k]), k
        modes = plan.replay_modes()
        _print("replay", modes)
        assert modes["fwd_views"] is None
        if replay == "timed":
            assert modes["fwd"] in ("graph", "direct") and modes["bwd"] in ("graph", "direct")
        else:
            assert modes["fwd"] == replay and modes["bwd"] == replay


def test_every_tuning_candidate_gives_the_same_bits():
    _print("case: forward/backward under every launch shape the autotuner chooses from, and "
           "under list slices")
    p = synth.small_phantom(n=2048, nviews=8, seed=6)
    b = _buffers(p, np.arange(8))
    ref_proj, ref_g = _eager(p, b, tuning=dict(slices=1))
    for waves in (4, 1):
        for persistent in (0, 1):
            proj, g = _eager(p, b, tuning=dict(splat_waves=waves, persistent=persistent,
                                               slices=1))
            assert torch.equal(proj, ref_proj), (waves, persistent)
            for k in _GRADS:
                assert torch.equal(g[k], ref_g[k]), (waves, persistent, k)
    # list slices: the same terms added in another order (rounding only), and the same bits on
    # a repeated call
    for slices in (2, 3, 8, 16):
        for waves in (4, 1):
            proj, g = _eager(p, b, tuning=dict(splat_waves=waves, slices=slices))
            err = float((proj - ref_proj).abs().max() / ref_proj.abs().max())
            assert err <= 1e-6, (slices, waves, err)
            for k in _GRADS:
                gerr = float((g[k] - ref_g[k]).abs().max() / ref_g[k].abs().max())
                assert gerr <= 1e-5, (slices, waves, k, gerr)
            proj2, g2 = _eager(p, b, tuning=dict(splat_waves=waves, slices=slices))
            assert torch.equal(proj2, proj)
            for k in _GRADS:
                assert torch.equal(g2[k], g[k]), (slices, waves, k)


def test_plan_overflow_is_detected_and_recovered():
    _print("case: plan with a far too small instance capacity; check, grow, repeat")
    p = synth.small_phantom(n=2048, nviews=8, seed=7)
    b = _buffers(p, np.arange(8))
    ref_proj, ref_g = _eager(p, b)
    with _lib.Plan(p.geom, p.grid, p.n, 8, b, tuning=dict(capacity=64, persistent=1)) as plan:
        plan.fwd()
        diag, resized = plan.check()
        assert diag["overflow"] == 1 and resized and diag["instances"] > 64
        plan.fwd()
        plan.bwd()
        diag, resized = plan.check()
        assert diag["overflow"] == 0 and not resized
        assert torch.equal(b["proj"], ref_proj)
        for k in _GRADS:
            assert torch.equal(b[k], ref_g[k]), k


def test_plan_check_grows_to_the_largest_need_since_the_last_check():
    _print("case: a call that overflows, then one that fits, then check: the plan grows to the "
           "first call's need")
    p = synth.small_phantom(n=2048, nviews=8, seed=8)
    b = _buffers(p, np.arange(8))
    big, small = dev(p.scale * 2.0), dev(p.scale)
    need = {}
    roomy = dict(capacity=64 * p.n * 8)
    for name, sc in (("big", big), ("small", small)):
        ws = _lib.Workspace()
        _lib.project_fwd(p.geom, p.grid, b["coef"], b["mu"], sc, b["quat"], b["rho"],
                         b["angles"], b["w"], ws, tuning=roomy)
        need[name] = ws.diagnostics()["instances"]
    _print("instances", need)
    assert need["big"] > 1.5 * need["small"]
    cap = int(need["small"] * 1.1)
    with _lib.Plan(p.geom, p.grid, p.n, 8, b, tuning=dict(capacity=cap)) as plan:
        b["scale"].copy_(big)
        plan.fwd()            # overflows
        b["scale"].copy_(small)
        plan.fwd()            # fits
        diag, resized = plan.check()
        assert resized and diag["overflow"] == 1
        assert diag["instances"] == need["small"] and diag["max_instances"] == need["big"]
        assert plan.tuning()[0]["capacity"] >= need["big"]
        b["scale"].copy_(big)
        plan.fwd()
        plan.bwd()
        diag, resized = plan.check()
        assert diag["overflow"] == 0 and not resized
        ref_proj, ref_g = _eager(p, b, tuning=roomy)
        assert torch.equal(b["proj"], ref_proj)
        for k in _GRADS:
            assert torch.equal(b[k], ref_g[k]), k


def test_new_workspace_diagnostics_start_clear():
    _print("case: a workspace filled with garbage reports clean diagnostics after its first call")
    p = synth.small_phantom(n=2048, nviews=4, seed=9)
    b = _buffers(p, np.arange(4))
    ws = _lib.Workspace()
    nbytes = _lib.workspace_size(p.geom, p.grid, p.n, 4)
    ws.buf = torch.full((nbytes,), 0xA5, dtype=torch.uint8, device="cuda")
    _lib.project_fwd(p.geom, p.grid, b["coef"], b["mu"], b["scale"], b["quat"], b["rho"],
                     b["angles"], b["w"], ws)
    d = ws.diagnostics()
    assert d["overflow"] == 0 and d["nonfinite"] == 0 and d["folded"] == 0, d
    assert d["behind_source"] == 0 and d["wide"] == 0 and d["max_instances"] == d["instances"]


@pytest.mark.parametrize("replay", ["timed", "graph", "direct"])
def test_plan_views_only_forward_equals_full_forward(replay):
    _print("case: plan forward of the per-view stages only (%s), after new views are written; "
           "the backward after it; equal to eager calls with the plan's tuning" % replay)
    p = synth.small_phantom(n=2048, nviews=8, seed=10)
    b = _buffers(p, np.arange(4))
    with _lib.Plan(p.geom, p.grid, p.n, 4, b, replay=replay) as plan:
        with pytest.raises(_lib.DigsError):
            plan.fwd_views()          # no per-Gaussian stage yet
        plan.fwd()
        tun = {k: v for k, v in plan.tuning()[0].items() if k != "cull_radius"}
        for first in (4, 2):
            a2, w2 = p.views(np.arange(first, first + 4))
            b["angles"].copy_(dev(a2))
            b["w"].copy_(dev(w2))
            plan.fwd_views()
            plan.bwd()
            diag, resized = plan.check()
            assert not resized and diag["overflow"] == 0
            got = b["proj"].clone()
            gg = {k: b[k].clone() for k in _GRADS}
            ref_proj, ref_g = _eager(p, b, tuning=tun)
            assert torch.equal(got, ref_proj), first
            for k in _GRADS:
                assert torch.equal(gg[k], ref_g[k]), (first, k)
        modes = plan.replay_modes()
        _print("replay", modes)
        if replay != "timed":
            assert modes["fwd_views"] == replay
        # another replay mode keeps the per-Gaussian stage: the per-view forward stays valid
        other = "direct" if modes["fwd_views"] == "graph" else "graph"
        plan.set_replay(other)
        b["proj"].fill_(-1.0)
        plan.fwd_views()
        torch.cuda.synchronize()
        assert torch.equal(b["proj"], ref_proj)
        assert plan.replay_modes()["fwd_views"] == other


def test_plan_first_calls_on_a_side_stream_are_ordered():
    _print("case: first (timed) plan calls on a side stream, inputs written on that stream just "
           "before; equal to the eager calls")
    p = synth.small_phantom(n=2048, nviews=8, seed=12)
    b = _buffers(p, np.arange(4))
    with _lib.Plan(p.geom, p.grid, p.n, 4, b) as plan:
        shape = {k: v for k, v in plan.tuning()[0].items() if k != "cull_radius"}
        a2, w2 = p.views(np.arange(4, 8))
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            # the new views reach the buffers on the side stream only; the plan's first calls
            # (which time both replay modes on the plan's own stream) must see them
            b["angles"].copy_(dev(a2), non_blocking=True)
            b["w"].copy_(dev(w2), non_blocking=True)
            b["proj"].fill_(-1.0)
            plan.fwd(stream=side)
            plan.bwd(stream=side)
            got = b["proj"].clone()
            gg = {k: b[k].clone() for k in _GRADS}
        side.synchronize()
        ref_proj, ref_g = _eager(p, b, tuning=shape)
        assert torch.equal(got, ref_proj)
        for k in _GRADS:
            assert torch.equal(gg[k], ref_g[k]), k
