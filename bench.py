#!/usr/bin/env python3
"""Benchmark: fwd+bwd projections/s of the deformation-informed Gaussian X-ray renderer.

Workload (the batched differentiable path): 200,000 Gaussians of the lung-like phantom, a
512x384 detector at 0.8 mm (source-isocentre 1000 mm, source-detector 1500 mm), 1,320 views over
a 60 s scan with irregular breathing, rank-3 FFD on a 29^3 lattice (10 mm). A step is one batch
of 64 uneven-time views (a seeded permutation of the scan cut into 64s): the forward of every
view (FFD at the canonical means, the warp, the projected records, tile binning, the splat), the
gradient of the L2 projection loss against synthetic measured projections, and the hand-written
backward to mu, scale, quaternion, density, FFD coefficients and the temporal weights.

The timed steps run the batched path: a plan (digs_plan_*) over fixed device buffers, its launch
shape and instance capacity chosen by the library's autotuner on the first batch, replayed as HIP
graphs or as direct launches (the plan times both once and keeps the faster). Per-kernel durations come from a second pass over the same steps launched eagerly with the
same tuning, each kernel stage bracketed by HIP events on its launch stream.

Inputs (Gaussians, lattice, per-batch angles and weights, measured projections) are resident in
HBM before the timed region. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd projections/s @200k Gaussians 512×384 det; % HBM roofline; speedup vs plain"

# Algorithmic FP32 work per (Gaussian, pixel) pair inside a cut-off footprint, in the splats'
# forward-difference formulation (FMA = 2 FLOP, add/mul = 1, rsqrt/exp2 = 1), and the VALU issue
# slots it needs: forward 4 adds (q, dq, E, dE), r^2, x = E r^2 + log2 amp (FMA), the sum (FMA),
# rsqrt and exp2 (7 VALU ops, 2 transcendentals); backward the same evaluation (r^2, x, g r 2^x:
# 3 muls; a = . r^2, a x: 2 muls) plus its moment sums (3 adds and 4 FMAs per pixel: 17 VALU ops,
# 2 transcendentals). A transcendental issues at half the FMA rate on gfx950 (measured), i.e.
# TRANS_SLOTS = 2 slots.
FWD_FLOP, FWD_VALU, FWD_TRANS = 11, 7, 2
BWD_FLOP, BWD_VALU, BWD_TRANS = 23, 17, 2
TRANS_SLOTS = 2
LANE_OPS_PER_S = 256 * 4 * 16 * 2.4e9      # CUs x SIMDs x lanes per cycle x clock
# MI355X's published dense FP32 vector peak (the roofline's peak); it counts packed FP32 FMAs
# (two per lane per cycle), which the library's kernels do not use (packed FP32 is switched off
# when they are compiled), so their unpacked FMA rate is half of it
FP32_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per projection of one fwd+bwd step (see the design notes): Gaussians read
# twice, lattice read twice and its gradient written, projection written, dL/dI read, Gaussian
# gradients written, per batch of 64
ALGO_BYTES_PER_PROJ = (2 * 200_000 * 44 + 3 * 29 ** 3 * 9 * 4 + 64 * 512 * 384 * 4 * 2 +
                       200_000 * 44) / 64.0
ALGO_BYTES_PER_STEP = ALGO_BYTES_PER_PROJ * 64   # 129.7 MB per 64-view fwd+bwd step


# HBM bytes per launch of k_splat_bwd (the roofline kernel) from two rocprofv3 --pmc runs of this
# bench (FETCH_SIZE, then WRITE_SIZE, mean KiB per dispatch, scaled by what the same counters read
# for a 512 MiB device copy: x2.0 and x1.0; profiles/batched_200k_hbm_counters.md), taken on the
# library sources whose digest is given; reported only while their code (comments aside) is unchanged
TRAFFIC = {"kernel": "k_splat_bwd", "read_bytes": 2219897.6 * (524288.0 / 262166.5625) * 1024,
           "write_bytes": 6624472.5 * 1.000 * 1024,
           "sources_sha256": "cae9094998698b08728fd85aeb2bfaded4df50dc64d9a9cf70e53e5c95fb4d58"}


def sources_digest() -> str:
    """sha256 over the library's HIP sources and headers in name order, each with its comments and
    blank lines removed (a comment edit does not change the kernels the figures were taken on)."""
    import hashlib
    import re
    d = os.path.join(ROOT, "paper_2506_22280_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h")):
            text = open(os.path.join(d, name), encoding="utf-8").read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)      # block comments
            text = re.sub(r"//[^\n]*", "", text)                     # line comments
            code = "\n".join(l.rstrip() for l in text.splitlines() if l.strip())
            h.update(name.encode())
            h.update(code.encode())
    return h.hexdigest()


def traffic_bytes():
    if TRAFFIC["sources_sha256"] is None or TRAFFIC["sources_sha256"] != sources_digest():
        return None
    return int(TRAFFIC["read_bytes"] + TRAFFIC["write_bytes"])


def tuning_candidates(tune_ms):
    """The autotuner's timings by name: tile shape, forward waves per tile, persistent splats
    (candidate c: tile shape c // 4, launch shape c % 4); shapes it did not try are left out."""
    names = {}
    for c, ms in enumerate(tune_ms):
        tw, th = ((16, 16), (32, 8), (8, 8))[c // 4]
        w_, p_ = ((4, 0), (4, 1), (1, 0), (1, 1))[c % 4]
        if ms[0] > 0:
            names["t%dx%d_w%d_p%d" % (tw, th, w_, p_)] = [round(x, 3) for x in ms]
    return names


def op_mix_peak_tflops(flop, valu, trans):
    """FLOP/s at full unpacked VALU issue for the kernel's per-pair operation mix (each
    transcendental issues at half rate, two slots): a secondary reference, not the roofline's."""
    return LANE_OPS_PER_S * flop / (valu + TRANS_SLOTS * trans) / 1e12


def cpu_baseline(p, params, batch_views, rows_every: int = 16):
    """The FP64 oracle (uncut, as it stands) on one view of the batch, every `rows_every`-th
    detector row: forward at those pixels and the adjoint of the L2 loss there."""
    import oracle
    oracle.build(force=False)
    v = batch_views[0]
    angles, w = p.views([v])
    mu, scale, quat, rho, coef = params
    nv, nu = p.geom["nv"], p.geom["nu"]
    rows = np.arange(0, nv, rows_every)
    pj = np.repeat(rows, nu)
    pi = np.tile(np.arange(nu), rows.size)
    pt = np.zeros_like(pj)
    t0 = time.perf_counter()
    val = oracle.project_pixels(p.geom, p.grid, coef, mu, scale, quat, rho, angles, w, pt, pj, pi)
    g = val - 0.9 * val
    oracle.project_bwd(p.geom, p.grid, coef, mu, scale, quat, rho, angles, w,
                       pixels=(pt, pj, pi, g))
    dt = time.perf_counter() - t0
    frac = pj.size / float(nu * nv)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": frac / dt, "unit": "projections/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 oracle, no cut-off: forward + L2 adjoint of one 512x384 view at "
                      "every %dth detector row (%d pixels, 200k Gaussians) took %.2f s; value "
                      "scales that to a whole view" % (rows_every, pj.size, dt)}


def _time_ms(fn, reps: int):
    """Average milliseconds per call of fn, HIP events on torch's current stream (the stream the
    library launches on), after one untimed call."""
    import torch
    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def single_view_leg(dev):
    """The single-projection forward path: 50k Gaussians, 256x256 at 1.6 mm, one view per call,
    eagerly and as a plan replay (HIP graph or direct launches, whichever the plan timed faster)."""
    import torch
    from paper_2506_22280_amd import _lib, synth
    p = synth.single_view(seed=0)

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    t = dict(coef=d(p.coef), mu=d(p.mu), scale=d(p.scale), quat=d(p.quat), rho=d(p.rho))
    ang, w = d(p.angles[:1]), d(p.w[:1])
    ws = _lib.Workspace(dev)
    proj = torch.empty((1, p.geom["nv"], p.geom["nu"]), device=dev)
    def fwd():
        _lib.project_fwd(p.geom, p.grid, t["coef"], t["mu"], t["scale"], t["quat"], t["rho"], ang,
                         w, ws, proj=proj)
    eager = _time_ms(fwd, 200)
    # per-stage HIP-event timing of the same eager call (stage events add their own overhead)
    _lib.profile_enable(True)
    _lib.profile_read(reset=True)
    for _ in range(50):
        fwd()
    torch.cuda.synchronize()
    prof = _lib.profile_read(reset=True)
    _lib.profile_enable(False)
    stages = {k: round(v[1] / 50, 4) for k, v in prof.items() if v[0]}
    grads = dict(g_mu=torch.empty((3, p.n), device=dev), g_scale=torch.empty((3, p.n), device=dev),
                 g_quat=torch.empty((4, p.n), device=dev), g_rho=torch.empty((p.n,), device=dev),
                 g_coef=torch.empty_like(t["coef"]), g_w=torch.empty((1, 3), device=dev))
    plan = _lib.Plan(p.geom, p.grid, p.n, 1, dict(t, angles=ang, w=w, proj=proj, **grads))
    replayed = _time_ms(plan.fwd, 200)
    # the scan's 680 views of the same model, one per launch: each writes its angle and weights
    # into the plan's buffers and replays the per-view stages (the per-Gaussian stage, shared by
    # every view, ran once in the plan's first fwd above)
    ang_all, w_all = d(p.angles), d(p.w)
    state = {"k": 0}

    def view():
        k = state["k"] % ang_all.shape[0]
        state["k"] += 1
        ang.copy_(ang_all[k:k + 1])
        w.copy_(w_all[k:k + 1])
        plan.fwd_views()
    views = _time_ms(view, ang_all.shape[0])
    tuning, _ = plan.tuning()
    replay = plan.replay_modes()
    plan.close()
    return {"ms_per_view_eager": round(eager, 4), "ms_per_view_plan": round(replayed, 4),
            "views_per_s_plan": round(1e3 / replayed, 1),
            "plan_replay": {k: replay[k] for k in ("fwd", "fwd_views")},
            "ms_per_view_scan_views_only": round(views, 4),
            "views_per_s_scan_views_only": round(1e3 / views, 1),
            "stage_ms_per_view_eager": stages,
            "tuning": {k: tuning[k] for k in ("tile_w", "tile_h", "splat_waves", "persistent",
                                              "slices")}}


def volume_leg(dev):
    """The volume query at one time point: 500k-Gaussian phantom, rank-4 FFD at 5 mm, a 256^3
    grid of 1 mm voxels: the displacement field (HBM-write-bound: 12 bytes per voxel) and phi."""
    import torch
    from paper_2506_22280_amd import _lib, synth
    p = synth.large(seed=0)

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    v = dict(nx=256, ny=256, nz=256, origin=[-127.5] * 3, spacing=[1.0] * 3)
    coef, w = d(p.coef), d(p.w[1000])
    mu, scale, quat, rho = d(p.mu), d(p.scale), d(p.quat), d(p.rho)
    dvf = torch.empty((3, 256, 256, 256), device=dev)
    import ctypes
    G, V = _lib.make_grid(p.grid), _lib.make_vgrid(v)

    def run_dvf():
        _lib._check("digs_dvf_grid", _lib.load().digs_dvf_grid(
            ctypes.byref(G), _lib._ptr(coef), _lib._ptr(w), ctypes.byref(V), _lib._ptr(dvf),
            _lib._stream()))
    dvf_ms = _time_ms(run_dvf, 20)
    ws = _lib.Workspace(dev)
    phi = _lib.phi_grid(p.grid, coef, mu, scale, quat, rho, w, v, ws)     # sizes the capacity
    cap = int(ws.diagnostics()["instances"] * 1.25) + 4096
    phi_ms = _time_ms(lambda: _lib.phi_grid(p.grid, coef, mu, scale, quat, rho, w, v, ws,
                                            capacity=cap, out=phi, grow=False), 10)
    dvf_bytes = 12 * 256 ** 3 + coef.numel() * 4
    return {"dvf_ms": round(dvf_ms, 4),
            "dvf_roofline": {"bound": "hbm", "achieved": round(dvf_bytes / dvf_ms / 1e6, 1),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(dvf_bytes / dvf_ms / 1e6 / HBM_PEAK_GBS, 4)},
            "phi_ms": round(phi_ms, 4), "phi_brick_pairs": int(ws.diagnostics()["instances"])}


def _plan_steps(G, Gd, n, est, ang, wts, meas, steps: int, warmup: int):
    """Seconds per fwd+bwd step of an autotuned plan over the batches (ang, wts, meas), graph
    replays between two synchronisations, and the plan's tuning."""
    import torch
    from paper_2506_22280_amd import _lib
    dev, B = ang[0].device, ang[0].shape[0]
    proj = torch.empty((B, G["nv"], G["nu"]), device=dev)
    gradp = torch.zeros_like(proj)
    ang_buf, w_buf = ang[0].clone(), wts[0].clone()
    grads = dict(g_mu=torch.empty((3, n), device=dev), g_scale=torch.empty((3, n), device=dev),
                 g_quat=torch.empty((4, n), device=dev), g_rho=torch.empty((n,), device=dev),
                 g_coef=torch.empty_like(est["coef"]), g_w=torch.empty((B, Gd["R"]), device=dev))
    plan = _lib.Plan(G, Gd, n, B, dict(est, angles=ang_buf, w=w_buf, proj=proj, grad_proj=gradp,
                                       **grads))
    tuning, _ = plan.tuning()

    def step(k):
        kb = k % len(ang)
        ang_buf.copy_(ang[kb])
        w_buf.copy_(wts[kb])
        plan.fwd()
        torch.sub(proj, meas[kb], out=gradp)
        plan.bwd()

    for k in range(warmup):
        step(k)
    _, resized = plan.check()
    if resized:
        for k in range(warmup):
            step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(warmup + k)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    diag, resized = plan.check()
    plan.close()
    if resized or diag["overflow"] or diag["nonfinite"]:
        raise SystemExit("diagnostics report a problem in a timed leg: %s" % diag)
    return dt, tuning


def _estimate(p, rng, d):
    """The estimate being fitted: a perturbed copy of the reference phantom."""
    return dict(mu=d(p.mu + rng.normal(0, 0.3, p.mu.shape)),
                scale=d(p.scale * np.exp(rng.normal(0, 0.05, p.scale.shape))),
                quat=d(p.quat + rng.normal(0, 0.05, p.quat.shape)),
                rho=d(p.rho * (1 + rng.normal(0, 0.05, p.rho.shape))), coef=d(p.coef * 0.9))


def large_leg(dev, steps: int, warmup: int):
    """The large-volume configuration: 500k Gaussians, 1024x768 detector at 0.4 mm, rank-4 FFD at
    5 mm, batches of 64 uneven-time views, fwd+bwd through an autotuned plan; with the volume
    query (DVF and phi of a 256^3 grid) at every 10th projection, amortised per projection."""
    from paper_2506_22280_amd import _lib, synth
    p = synth.large(seed=0)
    B = p.extra["batch"]
    batches = [b for b in synth.batch_schedule(len(p.angles), B, 0) if len(b) == B][:4]

    def d(a):
        import torch
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)

    ref = dict(coef=d(p.coef), mu=d(p.mu), scale=d(p.scale), quat=d(p.quat), rho=d(p.rho))
    est = _estimate(p, np.random.default_rng(2), d)
    ang = [d(p.angles[b]) for b in batches]
    wts = [d(p.w[b]) for b in batches]
    ws = _lib.Workspace(dev)
    meas, tun, inst = [], None, 0
    for k in range(len(batches)):
        for _ in range(2):   # a second pass with the capacity the first one measured
            img = _lib.project_fwd(p.geom, p.grid, ref["coef"], ref["mu"], ref["scale"],
                                   ref["quat"], ref["rho"], ang[k], wts[k], ws, tuning=tun)
            dg = ws.diagnostics()
            if not dg["overflow"]:
                break
            tun = dict(capacity=int(dg["instances"] * 1.25) + 4096)
            ws.reset()
        if dg["overflow"]:
            raise SystemExit("large leg: instance capacity exceeded")
        meas.append(img.clone())
        inst = max(inst, dg["instances"])
    del ws
    dt, tuning = _plan_steps(p.geom, p.grid, p.n, est, ang, wts, meas, steps, warmup)
    return {"gaussians": p.n, "detector": [p.geom["nu"], p.geom["nv"]], "batch": B,
            "ms_per_step": round(dt * 1e3, 3), "projections_per_s": round(B / dt, 2),
            "instances_per_view": int(inst / B),
            "tuning": {k: tuning[k] for k in ("tile_w", "tile_h", "splat_waves", "persistent",
                                              "capacity")}}


def recon_leg(iters: int = 50_000):
    """The reconstruction loop (Sec. 4.2) at the paper's acquisition (Sec. 4.1): 80k Gaussians,
    310 noisy views of 512x512 at 0.8 mm, detector offset 116 mm, SDD 1536 mm, rank 2 on an 8 mm
    lattice, one view per iteration, from a perturbed start without motion; time per iteration,
    the projected time of the paper's 50K iterations, and the dynamic volume's PSNR/RMSE against
    the ground truth before, after 3,000 and after `iters` iterations (the paper runs 50K)."""
    from paper_2506_22280_amd import recon, synth
    p = synth.paper_case(seed=0)
    out = recon.experiment(p, iters, motion="zero", noise=True, seed=0,
                           eval_at=[3000] if iters > 3000 else [])
    out["workload"] = ("80k Gaussians, 310 views 512x512 at 0.8 mm, offset 116 mm, SDD 1536, "
                       "rank 2 / 8 mm, 1 view per iteration, Poisson 1e8 + Gaussian 4 noise")
    return out


def basis_leg(p, est, ang, wts, meas, steps: int, tuning: dict):
    """The second ablation's motion model (Sec. 4.3: the spatial basis stored per Gaussian, no
    lattice) against the lattice model, both as eager fwd+bwd calls on the same batches (the plan
    path covers the lattice model only), HIP events around `steps` steps each."""
    import torch
    from paper_2506_22280_amd import _lib
    dev = ang[0].device
    G, Gd, n, B = p.geom, p.grid, p.n, ang[0].shape[0]
    ws = _lib.Workspace(dev)
    U, J = _lib.ffd_eval(Gd, est["coef"], est["mu"])          # per-rank u and grad u at the means
    basis = torch.cat([U, J], dim=1).contiguous()             # [R][12][n]
    proj = torch.empty((B, G["nv"], G["nu"]), device=dev)
    gradp = torch.empty_like(proj)
    g_l = dict(g_mu=torch.empty((3, n), device=dev), g_scale=torch.empty((3, n), device=dev),
               g_quat=torch.empty((4, n), device=dev), g_rho=torch.empty((n,), device=dev),
               g_coef=torch.empty_like(est["coef"]), g_w=torch.empty((B, Gd["R"]), device=dev))
    g_b = dict(g_l, g_basis=torch.empty_like(basis))
    del g_b["g_coef"]
    state = {"k": 0}

    def lattice_step():
        kb = state["k"] % len(ang)
        state["k"] += 1
        _lib.project_fwd(G, Gd, est["coef"], est["mu"], est["scale"], est["quat"], est["rho"],
                         ang[kb], wts[kb], ws, tuning=tuning, proj=proj)
        torch.sub(proj, meas[kb], out=gradp)
        _lib.project_bwd(G, Gd, est["coef"], est["mu"], est["scale"], est["quat"], est["rho"],
                         ang[kb], wts[kb], gradp, ws, tuning=tuning, reuse_fwd=True, out=g_l)

    def basis_step():
        kb = state["k"] % len(ang)
        state["k"] += 1
        _lib.project_basis_fwd(G, Gd, basis, est["mu"], est["scale"], est["quat"], est["rho"],
                               ang[kb], wts[kb], ws, tuning=tuning, proj=proj)
        torch.sub(proj, meas[kb], out=gradp)
        _lib.project_basis_bwd(G, Gd, basis, est["mu"], est["scale"], est["quat"], est["rho"],
                               ang[kb], wts[kb], gradp, ws, tuning=tuning, reuse_fwd=True,
                               out=g_b)

    lat_ms = _time_ms(lattice_step, steps)
    bas_ms = _time_ms(basis_step, steps)
    return {"eager_ms_per_step_lattice": round(lat_ms, 3),
            "eager_ms_per_step_basis": round(bas_ms, 3),
            "projections_per_s_basis": round(B / bas_ms * 1e3, 2),
            "basis_floats_per_gaussian": 12 * Gd["R"]}


def ewa_leg(p, est, ang, wts, meas, steps: int, warmup: int, ref, exact_ms: float):
    """The batched fwd+bwd step under the EWA model of Eq. 4 (same phantom, batches and plan
    machinery, its own autotuned plan), and the model's deviation from the exact line integral:
    max |I_EWA - I_exact| / max I_exact over the first batch of the reference phantom's views."""
    import torch
    from paper_2506_22280_amd import _lib
    dev = ang[0].device
    G, Gd, n, B = dict(p.geom, model="ewa"), p.grid, p.n, ang[0].shape[0]
    ws = _lib.Workspace(dev)
    exact = _lib.project_fwd(p.geom, Gd, ref["coef"], ref["mu"], ref["scale"], ref["quat"],
                             ref["rho"], ang[0], wts[0], ws).clone()
    ewa = _lib.project_fwd(G, Gd, ref["coef"], ref["mu"], ref["scale"], ref["quat"], ref["rho"],
                           ang[0], wts[0], ws)
    dev_max = float((ewa - exact).abs().max() / exact.abs().max())
    del ws, ewa, exact
    dt, tuning = _plan_steps(G, Gd, n, est, ang, wts, meas, steps, warmup)
    return {"ms_per_step": round(dt * 1e3, 3), "projections_per_s": round(B / dt, 2),
            "speedup_vs_exact": round(exact_ms / (dt * 1e3), 3),
            "max_dev_vs_exact_rel_to_max": round(dev_max, 6),
            "tuning": {k: tuning[k] for k in ("tile_w", "tile_h", "splat_waves", "persistent")}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the HIP-event stage timing (plain timed loop only)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the single-view and volume-query legs")
    ap.add_argument("--no-warmstart", action="store_true",
                    help="skip the learned-warm-start leg (speedup vs the plain fit)")
    ap.add_argument("--recon-iters", type=int, default=50_000,
                    help="iterations of the reconstruction leg (the paper runs 50K)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="before the timed region, run a plain device-to-device copy of this many "
                         "MiB three times (the reference kernel for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the renderer has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2506_22280_amd import _lib, synth

    dev = torch.device("cuda:0")
    p = synth.batched(seed=args.seed)
    B = p.extra["batch"]
    batches = [b for b in synth.batch_schedule(len(p.angles), B, args.seed) if len(b) == B]

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)

    # reference phantom -> measured projections; the estimate being fitted is a perturbed copy
    rng = np.random.default_rng(args.seed + 1)
    ref = dict(coef=d(p.coef), mu=d(p.mu), scale=d(p.scale), quat=d(p.quat), rho=d(p.rho))
    est = _estimate(p, rng, d)
    ang = [d(p.angles[b]) for b in batches]
    wts = [d(p.w[b]) for b in batches]
    ws = _lib.Workspace(dev)
    meas = []
    for k in range(len(batches)):
        meas.append(_lib.project_fwd(p.geom, p.grid, ref["coef"], ref["mu"], ref["scale"],
                                     ref["quat"], ref["rho"], ang[k], wts[k], ws).clone())
    diag = ws.diagnostics()
    if diag["overflow"]:
        raise SystemExit("instance capacity exceeded while rendering the measured projections")
    n, G, Gd = p.n, p.geom, p.grid
    proj = torch.empty((B, G["nv"], G["nu"]), device=dev)
    gradp = torch.empty_like(proj)
    ang_buf, w_buf = ang[0].clone(), wts[0].clone()
    grads = dict(g_mu=torch.empty((3, n), device=dev), g_scale=torch.empty((3, n), device=dev),
                 g_quat=torch.empty((4, n), device=dev), g_rho=torch.empty((n,), device=dev),
                 g_coef=torch.empty_like(est["coef"]), g_w=torch.empty((B, Gd["R"]), device=dev))
    if args.calib_copy_mb > 0:
        src = torch.ones(args.calib_copy_mb << 18, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # the batched path: a plan over fixed buffers, autotuned on the first batch, replayed as HIP
    # graphs or direct launches (whichever it timed faster); a step writes the batch's angles and weights into the plan's buffers, replays the
    # forward, forms dL/dI = I - P of the L2 loss, and replays the backward
    torch.sub(meas[0], meas[0], out=gradp)
    plan = _lib.Plan(G, Gd, n, B, dict(est, angles=ang_buf, w=w_buf, proj=proj, grad_proj=gradp,
                                       **grads))
    tuning, tune_ms = plan.tuning()

    def step(k):
        kb = k % len(batches)
        ang_buf.copy_(ang[kb])
        w_buf.copy_(wts[kb])
        plan.fwd()
        torch.sub(proj, meas[kb], out=gradp)
        plan.bwd()

    for k in range(args.warmup):
        step(k)
    diag, resized = plan.check()
    if resized:                      # the capacity grew: warm the re-captured graphs up again
        for k in range(args.warmup):
            step(k)
    # HIP events between the steps (on the stream the plan replays on) give the per-step spread
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for k in range(args.steps):
        step(args.warmup + k)
        evs[k + 1].record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    per_step_ms = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])
    diag, resized = plan.check()
    if resized or diag["overflow"] or diag["nonfinite"]:
        raise SystemExit("diagnostics report a problem in the timed steps: %s" % diag)
    replay = plan.replay_modes()
    plan.close()

    # per-kernel timing: the same steps, launched eagerly with the plan's tuning, every kernel
    # stage bracketed by HIP events on its launch stream
    eager_tuning = dict(splat_waves=tuning["splat_waves"], persistent=tuning["persistent"],
                        capacity=tuning["capacity"], slices=tuning["slices"],
                        tile_w=tuning["tile_w"], tile_h=tuning["tile_h"])

    def eager_step(k):
        kb = k % len(batches)
        _lib.project_fwd(G, Gd, est["coef"], est["mu"], est["scale"], est["quat"], est["rho"],
                         ang[kb], wts[kb], ws, tuning=eager_tuning, proj=proj)
        torch.sub(proj, meas[kb], out=gradp)
        _lib.project_bwd(G, Gd, est["coef"], est["mu"], est["scale"], est["quat"], est["rho"],
                         ang[kb], wts[kb], gradp, ws, tuning=eager_tuning, reuse_fwd=True,
                         out=grads)

    ws.reset()
    eager_step(0)
    torch.cuda.synchronize()
    prof = {}
    if not args.no_profile:
        _lib.profile_enable(True)
        _lib.profile_read(reset=True)
        t1 = time.perf_counter()
        for k in range(args.steps):
            eager_step(args.warmup + k)
        torch.cuda.synchronize()
        dt_eager = time.perf_counter() - t1
        prof = _lib.profile_read(reset=True)
        _lib.profile_enable(False)
    # algorithmic pair counts of the batches the timed steps use
    pairs = []
    for k in range(args.steps):
        kb = (args.warmup + k) % len(batches)
        _lib.project_fwd(G, Gd, est["coef"], est["mu"], est["scale"], est["quat"], est["rho"],
                         ang[kb], wts[kb], ws, tuning=eager_tuning, proj=proj)
        pairs.append(_lib.count_pairs(G, Gd, n, B, ws, tuning=eager_tuning))
    torch.cuda.synchronize()
    diag = ws.diagnostics()
    if diag["overflow"] or diag["nonfinite"]:
        raise SystemExit("diagnostics report a problem: %s" % diag)

    value = B * args.steps / dt
    in_fp = sum(x[0] for x in pairs)
    out = {"metric": METRIC, "value": round(value, 2), "unit": "projections/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(dt / args.steps * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "batched_200k: 200k Gaussians (lung phantom), 512x384 detector "
                                  "at 0.8 mm, 1320 views / 60 s, batches of 64 uneven-time "
                                  "views, rank-3 FFD on 29^3 (10 mm)",
                      "global_batch": B, "gaussians": n, "detector": [G["nu"], G["nv"]],
                      "parallelism": "single GPU"}}
    out["ms_per_step_events"] = {
        "median": round(float(np.median(per_step_ms)), 3),
        "p10": round(float(np.percentile(per_step_ms, 10)), 3),
        "p90": round(float(np.percentile(per_step_ms, 90)), 3),
        "meaning": "HIP events between the timed steps on the plan's stream"}
    out["sources_sha256"] = sources_digest()
    out["tuning"] = {"chosen": {k: tuning[k] for k in ("tile_w", "tile_h", "splat_waves",
                                                       "persistent", "capacity", "slices")},
                     "candidates_fwd_bwd_ms": tuning_candidates(tune_ms),
                     "replay": {k: replay[k] for k in ("fwd", "bwd")}}
    out["hbm_roofline_end_to_end"] = {
        "algorithmic_bytes_per_projection": int(ALGO_BYTES_PER_PROJ),
        "achieved_GBs": round(value * ALGO_BYTES_PER_PROJ / 1e9, 3),
        "frac": round(value * ALGO_BYTES_PER_PROJ / 1e9 / HBM_PEAK_GBS, 6)}
    if prof:
        out["eager_profiled_ms_per_step"] = round(dt_eager / args.steps * 1e3, 3)
        stages = {k: round(v[1] / max(v[0], 1), 4) for k, v in prof.items() if v[0]}
        totals = {k: v[1] for k, v in prof.items() if v[0]}
        out["stage_ms_per_step"] = {k: round(v / args.steps, 4) for k, v in totals.items()}
        out["stage_avg_ms_per_launch"] = stages
        out["stage_share"] = {k: round(v / sum(totals.values()), 4) for k, v in totals.items()}
        dom = max(("splat_fwd", "splat_bwd"), key=lambda k: totals.get(k, 0.0))
        avg_s = prof[dom][1] / prof[dom][0] / 1e3
        per_launch_pairs = in_fp / len(pairs)
        flop, valu, trans = ((FWD_FLOP, FWD_VALU, FWD_TRANS) if dom == "splat_fwd" else
                             (BWD_FLOP, BWD_VALU, BWD_TRANS))
        achieved = per_launch_pairs * flop / avg_s / 1e12
        mix = op_mix_peak_tflops(flop, valu, trans)
        traffic = traffic_bytes() if dom == "splat_bwd" else None
        out["roofline"] = {"kernel": "k_" + dom, "bound": "alu", "achieved": round(achieved, 3),
                           "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                           "traffic": traffic,
                           "avg_launch_ms": round(avg_s * 1e3, 4),
                           "pairs_per_launch": int(per_launch_pairs),
                           "flop_per_pair": flop,
                           "op_mix": {"peak": round(mix, 2), "frac": round(achieved / mix, 4),
                                      "meaning": "unpacked VALU issue rate for this kernel's "
                                                 "per-pair mix (transcendentals two slots)"},
                           "algorithmic_bytes_per_step": int(ALGO_BYTES_PER_STEP),
                           "traffic_over_algorithmic": (round(traffic / ALGO_BYTES_PER_STEP, 2)
                                                        if traffic else None)}
        ev_f = sum(x[1] for x in pairs) / len(pairs) / B
        out["pairs_per_projection"] = {
            "in_footprint": int(in_fp / len(pairs) / B),
            "evaluated_fwd": int(ev_f),
            "evaluated_bwd": int(sum(x[2] for x in pairs) / len(pairs) / B),
            "evaluated_over_in_footprint": round(ev_f / (in_fp / len(pairs) / B), 4)}
    if not args.no_extra:
        out["ewa_model"] = ewa_leg(p, est, ang, wts, meas, max(5, args.steps // 2), args.warmup,
                                   ref, dt / args.steps * 1e3)
        out["basis_model"] = basis_leg(p, est, ang, wts, meas, max(5, args.steps // 2),
                                       eager_tuning)
        out["single_view_50k"] = single_view_leg(dev)
        out["volume_query_500k_256cubed"] = volume_leg(dev)
        lg = large_leg(dev, 5, 2)
        vq = out["volume_query_500k_256cubed"]
        lg["ms_per_projection_with_volume_query_every_10th"] = round(
            lg["ms_per_step"] / lg["batch"] + (vq["dvf_ms"] + vq["phi_ms"]) / 10.0, 4)
        out["large_500k_1024x768"] = lg
        out["reconstruction_paper_case"] = recon_leg(args.recon_iters)
    if not args.no_warmstart:
        # "speedup vs plain": the learned warm start against the plain per-projection fit, time
        # to the same residual tolerance on views of unseen phantoms of the same family and size:
        # plain fits of all 1,320 views of 15 training phantoms (19.8k pairs) label the training
        # set; every view of 3 held-out phantoms is fitted both ways
        from paper_2506_22280_amd import warmstart
        ws_out = warmstart.experiment(n, G["nu"], G["nv"], G["pitch_u"], len(p.angles),
                                      Gd["spacing"][0], list(range(15)), [100, 101, 102],
                                      G["nv"] // 64, G["nu"] // 64, views_per_seed=None,
                                      log=lambda m: print(m, file=sys.stderr, flush=True))
        out["speedup_vs_plain"] = {
            "value": ws_out["wall_clock_speedup"],
            "meaning": "plain-fit seconds / warm-started-fit seconds to RMS residual <= 1e-3 of "
                       "the view, same GPU, every view of 3 unseen phantoms",
            "plain_s": ws_out["plain"]["seconds"], "warm_s": ws_out["warm"]["seconds"],
            "images_per_view": [ws_out["plain"]["mean_images_per_view"],
                                ws_out["warm"]["mean_images_per_view"]],
            "test_views": ws_out["test_views"], "train_pairs": ws_out["train_pairs"],
            "fallbacks": ws_out["warm"]["fallbacks"],
            "fallback_share": round(ws_out["warm"]["fallbacks"] / max(ws_out["test_views"], 1), 4),
            "plain_start_checked_above_rel_residual": round(ws_out["warm"]["alt_above"], 5),
            "label_fit_s": ws_out["label_fit_s"], "train_s": ws_out["train_s"]}
    if not args.no_cpu_baseline:
        params = tuple(est[k].double().cpu().numpy() for k in ("mu", "scale", "quat", "rho")) + (
            est["coef"].double().cpu().numpy(),)
        out["cpu_baseline"] = cpu_baseline(p, params, batches[0])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
