"""The DIGS reconstruction loop (Sec. 4.2) on the library's kernels.

The reference Gaussians (means, scales, rotations, densities), the spatial B-spline lattice of the
low-rank motion model (Eq. 9-10) and its temporal B-spline control values (a control value every
4 time points) are updated jointly by Adam on the L2 projection loss, one (or a few) measured
views per iteration, with learning rates that decay linearly from their initial to their final
values over the run. Per iteration, all on the GPU:

  digs_temporal_weights       w_r(t) of the iteration's views from the control values
  digs_plan_fwd (HIP graph)   the renderer's forward (FFD, warp, records, binning, splat)
  digs_l2_residual            dL/dI = I - P and the loss
  digs_plan_bwd (HIP graph)   the hand-written adjoint to every parameter and to w
  digs_temporal_weights_bwd   dL/d(control values)
  digs_adam_mapped            one Adam step per parameter group (scales through exp, densities
                              through softplus, so both stay positive)

The host picks the views, computes the learning rates and launches; nothing is read back except
the loss when asked for. Scoring (`evaluate`) renders the dynamic volume phi(x, t) of the
estimate and of the ground truth on a voxel grid with digs_phi_grid and reports RMSE and PSNR
(the paper's Sec. 4.3 metrics, here against the known synthetic phantom).
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import _lib

# Initial and final learning rates. The two B-spline grids follow Sec. 4.2; the Gaussians' rates
# are a reading of the paper (which defers them to R2-Gaussian): means in mm, log-scales,
# quaternions and softplus-densities in their own units.
LR = {"mu": (0.05, 0.0005), "log_scale": (5e-3, 5e-4), "quat": (1e-3, 1e-4),
      "rho_raw": (1e-2, 1e-3), "coef": (1e-4, 1e-5), "ctrl": (1e-2, 1e-3)}


def linear_rates(k: int, iters: int, lr: dict) -> dict:
    """Learning rates at iteration k (0-based) of a run of `iters`: linear from each group's
    initial value at k = 0 to its final value at k = iters - 1."""
    f = min(k / max(iters - 1, 1), 1.0)
    return {g: a + (b - a) * f for g, (a, b) in lr.items()}


def _softplus_inv(y):
    y = np.asarray(y, dtype=np.float64)
    return np.where(y > 20.0, y, np.log(np.expm1(np.maximum(y, 1e-30))))


class Reconstruction:
    """State and iteration of the loop on one problem (synth.Problem-like: geom, grid, angles,
    times) with measured projections `meas` [V][nv][nu] (device) and an initial estimate."""

    def __init__(self, prob, meas, init: dict, views_per_iter: int = 1, lr: dict | None = None,
                 iters: int = 50_000, seed: int = 0, device="cuda", tuning: dict | None = None):
        self.geom, self.grid = prob.geom, prob.grid
        self.meas = meas
        self.V = meas.shape[0]
        self.B = views_per_iter
        self.iters = iters
        self.lr = dict(LR, **(lr or {}))
        self.rng = np.random.default_rng(seed + 4242)
        dev = torch.device(device)

        def d(a):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)

        self.angles_all = d(prob.angles)
        self.times_all = d(prob.times)
        # temporal control values: one every 4 views' time step, padded by one on each side
        tstep = float(prob.times[1] - prob.times[0]) if self.V > 1 else 1.0
        self.dt = 4.0 * tstep
        self.t0 = float(prob.times[0]) - self.dt
        self.Ct = int(math.ceil((float(prob.times[-1]) - self.t0) / self.dt)) + 3
        R = self.grid["R"]
        n = init["mu"].shape[1]
        self.n = n
        # parameters: the renderer's values and, where mapped, the unconstrained raw values
        self.mu = d(init["mu"])
        self.quat = d(init["quat"])
        self.log_scale = d(np.log(init["scale"]))
        self.scale = d(init["scale"])
        self.rho_raw = d(_softplus_inv(init["rho"]))
        self.rho = d(init["rho"])
        self.coef = d(init["coef"])
        self.ctrl = d(init.get("ctrl", np.zeros((self.Ct, R))))
        assert self.ctrl.shape == (self.Ct, R)
        self.groups = [("mu", self.mu, self.mu, "identity"),
                       ("log_scale", self.log_scale, self.scale, "exp"),
                       ("quat", self.quat, self.quat, "identity"),
                       ("rho_raw", self.rho_raw, self.rho, "softplus"),
                       ("coef", self.coef, self.coef, "identity"),
                       ("ctrl", self.ctrl, self.ctrl, "identity")]
        self.m = {k: torch.zeros_like(raw) for k, raw, _, _ in self.groups}
        self.v = {k: torch.zeros_like(raw) for k, raw, _, _ in self.groups}
        # the plan: fixed buffers for B views per iteration
        B, nv, nu = self.B, self.geom["nv"], self.geom["nu"]
        self.ang_buf = torch.empty(B, device=dev)
        self.time_buf = torch.empty(B, device=dev)
        self.w_buf = torch.zeros((B, R), device=dev)
        self.proj = torch.zeros((B, nv, nu), device=dev)
        self.grad = torch.zeros_like(self.proj)
        self.meas_buf = torch.empty_like(self.proj)
        self.loss = torch.zeros(1 + _lib.L2_PARTS, device=dev)   # loss[0] and its parts
        self.g = dict(g_mu=torch.empty_like(self.mu), g_scale=torch.empty_like(self.scale),
                      g_quat=torch.empty_like(self.quat), g_rho=torch.empty_like(self.rho),
                      g_coef=torch.empty_like(self.coef), g_w=torch.empty((B, R), device=dev))
        self.g_ctrl = torch.empty_like(self.ctrl)
        idx0 = torch.arange(B, device=dev)
        self._select(idx0)
        self.plan = _lib.Plan(self.geom, self.grid, n, B, dict(
            coef=self.coef, mu=self.mu, scale=self.scale, quat=self.quat, rho=self.rho,
            angles=self.ang_buf, w=self.w_buf, proj=self.proj, grad_proj=self.grad, **self.g),
            tuning=tuning)
        self.step_no = 0
        self.order = None      # this pass's view order (device) and the position in it
        self.pos = 0
        self.resized = 0

    def _select(self, idx):
        torch.index_select(self.angles_all, 0, idx, out=self.ang_buf)
        torch.index_select(self.times_all, 0, idx, out=self.time_buf)
        torch.index_select(self.meas, 0, idx, out=self.meas_buf)

    def _next_views(self):
        """Views in seeded random order, every view once per pass (a pass's order is copied to
        the device once; a pass ends early if fewer than B views remain)."""
        if self.order is None or self.pos + self.B > self.V:
            perm = self.rng.permutation(self.V)
            self.order = torch.from_numpy(perm).to(self.ang_buf.device)
            self.pos = 0
        idx = self.order[self.pos:self.pos + self.B]
        self.pos += self.B
        return idx

    def rates(self, k: int) -> dict:
        return linear_rates(k, self.iters, self.lr)

    def step(self):
        """One iteration; returns nothing (the loss stays on the device, in self.loss)."""
        self._select(self._next_views())
        _lib._check("digs_temporal_weights", _lib.load().digs_temporal_weights(
            self.Ct, self.grid["R"], _lib._ptr(self.ctrl), float(self.t0), float(self.dt), self.B,
            _lib._ptr(self.time_buf), _lib._ptr(self.w_buf), _lib._stream()))
        self.plan.fwd()
        _lib.l2_residual(self.proj, self.meas_buf, self.grad, self.loss)
        self.plan.bwd()
        _lib._check("digs_temporal_weights_bwd", _lib.load().digs_temporal_weights_bwd(
            self.Ct, self.grid["R"], float(self.t0), float(self.dt), self.B,
            _lib._ptr(self.time_buf), _lib._ptr(self.g["g_w"]), _lib._ptr(self.g_ctrl),
            _lib._stream()))
        rates = self.rates(self.step_no)
        self.step_no += 1
        grads = {"mu": self.g["g_mu"], "log_scale": self.g["g_scale"], "quat": self.g["g_quat"],
                 "rho_raw": self.g["g_rho"], "coef": self.g["g_coef"], "ctrl": self.g_ctrl}
        for name, raw, value, mapping in self.groups:
            _lib.adam_mapped(raw, value, grads[name], self.m[name], self.v[name], rates[name],
                             self.step_no, mapping)

    def _snapshot(self):
        """The loop's state at a clean check: every parameter group's raw values, mapped values
        and Adam moments (device copies), the iteration count and the view order."""
        return dict(t={k: (raw.clone(), None if value is raw else value.clone(),
                           self.m[k].clone(), self.v[k].clone())
                       for k, raw, value, _ in self.groups},
                    step_no=self.step_no, rng=self.rng.bit_generator.state,
                    order=self.order, pos=self.pos)

    def _restore(self, snap):
        for k, raw, value, _ in self.groups:
            r, val, m, v = snap["t"][k]
            raw.copy_(r)
            if val is not None:
                value.copy_(val)
            self.m[k].copy_(m)
            self.v[k].copy_(v)
        self.step_no = snap["step_no"]
        self.rng.bit_generator.state = snap["rng"]
        self.order, self.pos = snap["order"], snap["pos"]

    def run(self, iters: int, log_every: int = 0, log=None, check_every: int = 100):
        """iters iterations; returns (iteration, mean loss per view over the last log_every
        iterations) every log_every iterations.

        The iterations run in windows of check_every; after each window the plan's diagnostics
        are read (a synchronisation). If any view of the window needed more (Gaussian, tile)
        instances than the plan holds, its renders were incomplete: the plan grows (counted in
        self.resized), the parameters, Adam moments and view order go back to their state at the
        previous check, and the window is run again, so no update from an incomplete render
        survives. check_every = 0 runs without checks."""
        losses = []
        acc = torch.zeros(1, device=self.loss.device)
        cnt = 0
        window = check_every if check_every else iters
        k = 0
        snap = self._snapshot() if check_every else None
        while k < iters:
            end = min(k + window, iters)
            w_losses, w_acc, w_cnt = [], acc.clone(), cnt
            for kk in range(k, end):
                self.step()
                w_acc += self.loss[:1]
                w_cnt += 1
                if log_every and ((kk + 1) % log_every == 0 or kk == iters - 1):
                    w_losses.append((self.step_no, w_acc, w_cnt))
                    w_acc = torch.zeros(1, device=self.loss.device)
                    w_cnt = 0
            if check_every:
                diag, resized = self.plan.check()
                if resized:
                    self.resized += 1
                    self._restore(snap)
                    continue
                if diag["nonfinite"]:
                    raise FloatingPointError("non-finite Gaussians at iteration %d" % self.step_no)
                snap = self._snapshot()
            for step_no, a, c in w_losses:
                losses.append((step_no, float(a[0].item()) / (c * self.B)))
                if log:
                    log("iteration %d: mean loss per view %.4e" % losses[-1])
            acc, cnt = w_acc, w_cnt
            k = end
        return losses

    def fit_ctrl(self, w_views):
        """Set the temporal control values to the least-squares fit of per-view weights
        w_views [V][R] (host array) at the views' times: the B-spline basis is evaluated by the
        library's kernel on unit control vectors."""
        dev = self.ctrl.device
        basis = np.zeros((self.V, self.Ct))
        for j in range(self.Ct):
            e = torch.zeros((self.Ct, 1), device=dev)
            e[j, 0] = 1.0
            basis[:, j] = _lib.temporal_weights(e, self.t0, self.dt,
                                                self.times_all)[:, 0].cpu().numpy()
        sol = np.linalg.lstsq(basis, np.asarray(w_views, dtype=np.float64), rcond=None)[0]
        self.ctrl.copy_(torch.from_numpy(sol.astype(np.float32)).to(dev))

    def weights_at(self, times) -> torch.Tensor:
        """w [T][R] of the estimated temporal B-spline at the given times (device)."""
        return _lib.temporal_weights(self.ctrl, self.t0, self.dt, times)

    def close(self):
        self.plan.close()


def phi_volume(grid, coef, mu, scale, quat, rho, w, vgrid, ws):
    return _lib.phi_grid(grid, coef, mu, scale, quat, rho, w, vgrid, ws)


def evaluate(rec: Reconstruction, truth: dict, views, vgrid: dict, ws=None) -> dict:
    """RMSE and PSNR of the estimated dynamic volume against the ground truth at the times of the
    given views (means over the views): PSNR = 20 log10(max phi_true / RMSE) on the voxel grid."""
    ws = ws or _lib.Workspace(rec.mu.device)
    times = rec.times_all[torch.as_tensor(views, device=rec.mu.device)]
    w_est = rec.weights_at(times.contiguous())
    rmse, psnr = [], []
    for j, v in enumerate(views):
        gt = phi_volume(rec.grid, truth["coef"], truth["mu"], truth["scale"], truth["quat"],
                        truth["rho"], truth["w"][v].contiguous(), vgrid, ws).clone()
        est = phi_volume(rec.grid, rec.coef, rec.mu, rec.scale, rec.quat, rec.rho,
                         w_est[j].contiguous(), vgrid, ws)
        e = float(torch.sqrt(torch.mean((est - gt).double() ** 2)))
        rmse.append(e)
        psnr.append(20.0 * math.log10(float(gt.max()) / max(e, 1e-30)))
    return {"rmse": float(np.mean(rmse)), "psnr_db": float(np.mean(psnr))}


def perturbed_init(prob, rng, pos_mm=0.5, rho_frac=0.3, coef_mm=0.05, motion="zero"):
    """The estimate the loop starts from: the phantom's Gaussians with jittered means and
    densities, scales and rotations as they are. motion "zero": no motion (a small random lattice
    breaks the symmetry of w = 0, coef = 0); "true": the true lattice (the caller then fits the
    temporal control values to the true weights). Stands in for the paper's cloud sampled from a
    CGLS image."""
    coef = (rng.normal(0.0, coef_mm, prob.coef.shape) if motion == "zero" else
            prob.coef.astype(np.float64))
    return dict(mu=prob.mu + rng.normal(0, pos_mm, prob.mu.shape),
                scale=prob.scale.astype(np.float64),
                quat=prob.quat.astype(np.float64),
                rho=prob.rho * rng.uniform(1.0 - rho_frac, 1.0 + rho_frac, prob.rho.shape),
                coef=coef)


def experiment(prob, iters: int, views_per_iter: int = 1, eval_views=None, vgrid=None,
               noise: bool = True, seed: int = 0, motion: str = "zero", lr: dict | None = None,
               log=None, eval_at=()) -> dict:
    """Render the measured views of `prob` (ground-truth motion), optionally with the paper's
    noise model, run the loop from a perturbed start and score it before and after. eval_at:
    iteration counts inside the run at which the volume is also scored (the learning rates decay
    over the whole run of `iters`); time per iteration excludes the scoring."""
    from . import synth
    dev = torch.device("cuda")

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)

    truth = dict(coef=d(prob.coef), mu=d(prob.mu), scale=d(prob.scale), quat=d(prob.quat),
                 rho=d(prob.rho), w=d(prob.w))
    ws = _lib.Workspace(dev)
    meas = []
    for b in range(0, len(prob.angles), 32):
        sl = slice(b, min(b + 32, len(prob.angles)))
        meas.append(_lib.project_fwd(prob.geom, prob.grid, truth["coef"], truth["mu"],
                                     truth["scale"], truth["quat"], truth["rho"],
                                     d(prob.angles[sl]), d(prob.w[sl]), ws).clone())
    meas = torch.cat(meas)
    if noise:
        meas = d(synth.add_noise(meas.cpu().numpy(), seed=seed))
    rng = np.random.default_rng(seed + 17)
    rec = Reconstruction(prob, meas, perturbed_init(prob, rng, motion=motion), views_per_iter,
                         iters=iters, seed=seed, lr=lr)
    if motion == "true":
        rec.fit_ctrl(prob.w)
    if eval_views is None:
        eval_views = list(np.linspace(0, len(prob.angles) - 1, 6).astype(int))
    if vgrid is None:
        vgrid = dict(nx=96, ny=96, nz=96, origin=[-126.0] * 3, spacing=[2.65] * 3)
    before = evaluate(rec, truth, eval_views, vgrid)
    marks = sorted({int(k) for k in eval_at if 0 < int(k) < iters}) + [iters]
    sec, done, losses, scores = 0.0, 0, [], {}
    for mark in marks:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses += rec.run(mark - done, log_every=max(iters // 10, 1), log=log)
        torch.cuda.synchronize()
        sec += time.perf_counter() - t0
        done = mark
        if mark != iters:
            scores[str(mark)] = evaluate(rec, truth, eval_views, vgrid)
    after = evaluate(rec, truth, eval_views, vgrid)
    rec.close()
    out = {"iters": iters, "views_per_iter": views_per_iter, "seconds": round(sec, 3),
           "ms_per_iter": round(sec / iters * 1e3, 4), "loss_first_last": [losses[0][1],
                                                                          losses[-1][1]],
           "plan_resized": rec.resized, "before": before, "after": after}
    if scores:
        out["during"] = scores
    return out
