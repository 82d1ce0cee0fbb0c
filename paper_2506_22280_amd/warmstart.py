"""Per-projection temporal-weight fit and its learned warm start (host loops over library kernels).

Plain fit. For views t with measured projections P_t, find the rank-R weights w_t of the low-rank
motion model (Sec. 3.3, Eq. 9) that minimise 1/2 ||I(w_t) - P_t||^2, with the Gaussians and the
lattice fixed, by Levenberg-Marquardt. Each iteration renders, in one digs_project_fwd launch,
every active view at its trial weights; the views whose trial lowered the residual (and did not
yet meet the tolerance) are then rendered at R copies with one weight raised by h, and
digs_lm_normal_eq reduces those images to J^T J, J^T res and res.res per view; the 3x3 (R x R)
damped solve and the accept/reject logic run on the host in FP64. A view is done when its RMS
residual falls to `tol` times the RMS of its measured projection.

Warm start. A small MLP maps the view downsampled to 64x64 (block means) plus sin and cos of the
gantry angle to w_t: 4098 -> 256 -> 256 -> R with ReLU, FP32 master weights, every product on the
matrix cores in BF16 with FP32 accumulation (digs_gemm_bf16), trained with Adam (digs_adam) on
weights that plain fits produced. Its prediction starts the same LM fit; if the predicted weights
leave a larger residual than the plain start, the fit starts from the plain start instead (the
plain fit is both fallback and judge).
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import _lib


# ------------------------------------------------------------------------------------------------
class Scene:
    """Fixed Gaussians and lattice on the device, with the geometry: what the fit holds fixed."""

    def __init__(self, geom: dict, grid: dict, coef, mu, scale, quat, rho, device="cuda"):
        def d(a):
            return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=device)
        self.geom, self.grid = geom, grid
        self.coef, self.mu, self.scale, self.quat, self.rho = (d(x) for x in
                                                               (coef, mu, scale, quat, rho))
        self.ws = _lib.Workspace(device)
        self.device = device
        self.capacity = 0

    @property
    def R(self) -> int:
        return int(self.grid["R"])

    def render(self, angles, w):
        """proj [T][nv][nu] at device angles [T] and weights w [T][R]. The instance capacity
        starts at the library default and grows (and the call repeats) if the diagnostics report
        an overflow: an incomplete render never reaches the fit."""
        while True:
            tuning = {"capacity": self.capacity} if self.capacity else None
            proj = _lib.project_fwd(self.geom, self.grid, self.coef, self.mu, self.scale,
                                    self.quat, self.rho, angles, w, self.ws, tuning=tuning)
            d = self.ws.diagnostics()
            if not d["overflow"]:
                return proj
            self.ws.reset()
            self.capacity = int(d["instances"] * 1.25) + 4096


def meas_norm2(meas):
    """sum over pixels of P_t^2 per view (host FP64), by the normal-equation kernel with zero
    rendered images (res = -P)."""
    T = meas.shape[0]
    zeros = torch.zeros((T, 2) + tuple(meas.shape[1:]), device=meas.device)
    h = torch.ones(1, device=meas.device)
    return _lib.lm_normal_eq(zeros, meas, h, 1)[:, 2].double().cpu().numpy()


def lm_fit(scene: Scene, angles, meas, start, alt=None, alt_above: float | None = None,
           tol: float = 1e-3, max_steps: int = 30, h: float = 0.05, lam0: float = 1e-3,
           info: dict | None = None):
    """Fit w for every view. angles [T] and meas [T][nv][nu] on the device; start [T][R] (host).
    alt [T][R] (host, optional): a second start, rendered once the start's residual is known for
    the views whose relative residual at the start is at least alt_above (every view if None;
    one more image per such view); a view whose alt start leaves the smaller residual continues
    from it instead.
    Each iteration first renders every active view at its trial weights only; a view whose trial
    meets the tolerance stops there, a trial that lowers the residual is accepted, and only then
    are the R raised copies rendered for the Jacobian at the new point (forward differences of
    step h); a rejected trial keeps the Jacobian and raises the damping.
    Returns (w [T][R] host FP64, images [T]: images rendered per view until the view met the
    tolerance (the alt image included), or those of max_steps + 1 iterations if it never did,
    rel [T]: final RMS residual / RMS of the measurement). info, if given, receives "used_alt"
    [T] (bool) and "rel_start" [T] (the relative residual at the start)."""
    T, R = meas.shape[0], scene.R
    npix = meas[0].numel()
    dev = meas.device
    w = np.array(start, dtype=np.float64).reshape(T, R)
    used_alt = np.zeros(T, dtype=bool)
    lam = np.full(T, lam0)
    pn = np.sqrt(meas_norm2(meas) / npix)
    target = tol * pn
    hvec = torch.full((R,), h, device=dev)
    ones = torch.ones(1, device=dev)
    images = np.zeros(T, dtype=np.int64)
    done = np.zeros(T, dtype=bool)
    JtJ = np.zeros((T, R, R)); Jtr = np.zeros((T, R)); rr = np.full(T, np.inf)
    tri = np.triu_indices(R)
    nt = R * (R + 1) // 2
    active = np.arange(T)
    trial = w.copy()
    rel_start = np.full(T, np.inf)

    def sq_residual(imgs, m):   # sum of squared residuals per image (images [A][nv][nu])
        return _lib.lm_normal_eq(torch.stack([imgs, imgs], 1), m, ones, 1)[:, 2].double().cpu().numpy()

    for it in range(max_steps + 1):
        if active.size == 0:
            break
        A = active.size
        idx = torch.as_tensor(active, device=dev)
        m_act = meas[idx].contiguous()
        # 1. the trial weights of every active view (at the first iteration, then the alt start
        # of the views whose start left a relative residual of at least alt_above)
        imgs = scene.render(angles[idx], torch.as_tensor(trial[active], dtype=torch.float32,
                                                         device=dev))
        r2 = sq_residual(imgs, m_act)
        images[active] += 1
        base = imgs.clone()              # the image at each view's accepted point
        r2_alt = {}
        if it == 0:
            rel_start = np.sqrt(np.maximum(r2, 0.0) / npix) / np.maximum(pn, 1e-300)
            if alt is not None:
                sel = [j for j in range(A) if alt_above is None or rel_start[j] >= alt_above]
                if sel:
                    ta = active[sel]
                    aimg = scene.render(angles[torch.as_tensor(ta, device=dev)],
                                        torch.as_tensor(np.asarray(alt, dtype=np.float64)[ta],
                                                        dtype=torch.float32, device=dev))
                    ra = sq_residual(aimg, meas[torch.as_tensor(ta, device=dev)].contiguous())
                    images[ta] += 1
                    r2_alt = {j: (k, ra[k]) for k, j in enumerate(sel)}
        accepted = np.zeros(A, dtype=bool)
        for j, t in enumerate(active):
            if j in r2_alt and r2_alt[j][1] < r2[j]:
                used_alt[t] = True
                w[t] = np.asarray(alt, dtype=np.float64)[t]
                rr[t] = r2_alt[j][1]
                base[j] = aimg[r2_alt[j][0]]
                accepted[j] = True
            elif r2[j] < rr[t]:
                w[t] = trial[t]
                rr[t] = r2[j]
                accepted[j] = True
                if it:
                    lam[t] = max(lam[t] / 3.0, 1e-9)
            else:
                lam[t] *= 4.0
            if np.sqrt(max(rr[t], 0.0) / npix) <= target[t]:
                done[t] = True
        # 2. the Jacobian at the newly accepted points of the views still open
        need = [j for j in range(A) if accepted[j] and not done[active[j]]]
        if need and it < max_steps:
            nsel = torch.as_tensor(need, device=dev)
            tj = active[need]
            Wr = np.repeat(w[tj][:, None, :], R, axis=1) + h * np.eye(R)[None]
            raised = scene.render(angles[torch.as_tensor(tj, device=dev)].repeat_interleave(R),
                                  torch.as_tensor(Wr.reshape(-1, R), dtype=torch.float32,
                                                  device=dev))
            images[tj] += R
            stack = torch.cat([base[nsel][:, None], raised.view(len(need), R, *raised.shape[1:])],
                              1).reshape(-1, *raised.shape[1:])
            ne = _lib.lm_normal_eq(stack, meas[torch.as_tensor(tj, device=dev)].contiguous(), hvec,
                                   R).double().cpu().numpy()
            for k, t in enumerate(tj):
                Am = np.zeros((R, R)); Am[tri] = ne[k, :nt]; Am = Am + np.triu(Am, 1).T
                JtJ[t] = Am
                Jtr[t] = ne[k, nt:nt + R]
        # 3. the next trial of every view still open (a rejected one: the same point, more damping)
        still = []
        for t in active:
            if done[t]:
                continue
            M = JtJ[t] + lam[t] * np.diag(np.maximum(np.diag(JtJ[t]), 1e-12))
            try:
                trial[t] = w[t] + np.linalg.solve(M, -Jtr[t])
            except np.linalg.LinAlgError:
                trial[t] = w[t]
            still.append(t)
        active = np.asarray(still, dtype=np.int64)
    if info is not None:
        info["used_alt"] = used_alt
        info["rel_start"] = rel_start
    rms = np.sqrt(np.maximum(rr, 0.0) / npix)
    return w, images, rms / np.maximum(pn, 1e-300)


# ------------------------------------------------------------------------------------------------
class WarmStartNet:
    """MLP nin -> hidden -> hidden -> R (ReLU). FP32 master weights in one flat device buffer;
    products on the matrix cores in BF16 with FP32 accumulation."""

    def __init__(self, nin: int, R: int, hidden: int = 256, seed: int = 0, device="cuda"):
        self.nin, self.R, self.hidden, self.device = nin, R, hidden, device
        shapes = [(nin, hidden), (hidden,), (hidden, hidden), (hidden,), (hidden, R), (R,)]
        sizes = [int(np.prod(s)) for s in shapes]
        self.P = sum(sizes)
        rng = np.random.default_rng(seed)
        init = []
        for s in shapes:                     # He-normal weights, zero biases
            init.append(rng.normal(0, np.sqrt(2.0 / s[0]), s) if len(s) == 2 else np.zeros(s))
        flat = np.concatenate([x.ravel() for x in init]).astype(np.float32)
        self.w = torch.as_tensor(flat, device=device)
        self.g = torch.zeros_like(self.w)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.step = 0
        offs = np.cumsum([0] + sizes)
        self._views = lambda buf: [buf[offs[i]:offs[i + 1]].view(shapes[i]) for i in range(6)]
        self.W1, self.b1, self.W2, self.b2, self.W3, self.b3 = self._views(self.w)
        self.gW1, self.gb1, self.gW2, self.gb2, self.gW3, self.gb3 = self._views(self.g)
        self.fmean = None
        self.fistd = None
        self.std_floor = 1.0
        self.mean_h = np.zeros(R)
        self.std_h = np.ones(R)
        self.mean = torch.zeros(R, device=device)
        self.std = torch.ones(R, device=device)

    def _forward(self, X):
        B = X.shape[0]
        H1 = torch.empty((B, self.hidden), device=self.device)
        H2 = torch.empty_like(H1)
        Y = torch.empty((B, self.R), device=self.device)
        _lib.gemm_bf16(X, self.W1, H1, bias=self.b1, relu=True)
        _lib.gemm_bf16(H1, self.W2, H2, bias=self.b2, relu=True)
        _lib.gemm_bf16(H2, self.W3, Y, bias=self.b3)
        return H1, H2, Y

    def features(self, proj, angles, fy: int, fx: int):
        """Standardised network inputs of views proj [T][nv][nu] (device)."""
        return _lib.downsample(proj, fy, fx, angles=angles, fmean=self.fmean, fistd=self.fistd)

    def predict(self, X):
        """w [B][R] (host FP64) from network inputs X [B][nin] (device): the network predicts
        standardised weights; the affine map back runs on the host."""
        Y = self._forward(X)[2].double().cpu().numpy()
        return Y * self.std_h + self.mean_h

    def train_step(self, X, target, lr: float, loss=None):
        """One Adam step on a batch: X [B][nin], target w [B][R] (device)."""
        H1, H2, Y = self._forward(X)
        dY = torch.empty_like(Y)
        _lib.mse(Y, target, self.mean, self.std, dY, loss)
        dH2 = torch.empty_like(H2)
        dH1 = torch.empty_like(H1)
        _lib.gemm_bf16(H2, dY, self.gW3, transA=True)
        _lib.colsum(dY, self.gb3)
        _lib.gemm_bf16(dY, self.W3, dH2, transB=True, gate=H2)
        _lib.gemm_bf16(H1, dH2, self.gW2, transA=True)
        _lib.colsum(dH2, self.gb2)
        _lib.gemm_bf16(dH2, self.W2, dH1, transB=True, gate=H1)
        _lib.gemm_bf16(X, dH1, self.gW1, transA=True)
        _lib.colsum(dH1, self.gb1)
        self.step += 1
        _lib.adam(self.w, self.g, self.m, self.v, lr, self.step)

    def fit(self, X, W, epochs: int = 60, batch: int = 128, lr: float = 1e-3, seed: int = 0):
        """Train on raw inputs X [S][nin] (device; block means and sin, cos of the angle, as
        `features` gives them before standardisation; standardised here in place) and target
        weights W [S][R] (host array)."""
        nimg = X.shape[1] - 2
        Xh = X[:, :nimg].double().cpu().numpy()
        self.fmean = torch.as_tensor(Xh.mean(0), dtype=torch.float32, device=self.device)
        # floor the per-feature spread at a fraction of the typical spread, so that pixels that
        # hardly vary over the training set (background, detector edges) are not amplified
        sd = Xh.std(0)
        self.fistd = torch.as_tensor(1.0 / np.maximum(sd, self.std_floor * np.median(sd) + 1e-12),
                                     dtype=torch.float32, device=self.device)
        del Xh
        _lib.standardize(X, self.fmean, self.fistd, ncols=nimg)
        Wh = np.asarray(W, dtype=np.float64)
        self.mean_h = Wh.mean(0)
        self.std_h = Wh.std(0) + 1e-6
        self.mean = torch.as_tensor(self.mean_h, dtype=torch.float32, device=self.device)
        self.std = torch.as_tensor(self.std_h, dtype=torch.float32, device=self.device)
        W = torch.as_tensor(Wh, dtype=torch.float32, device=self.device)
        rng = np.random.default_rng(seed)
        S = X.shape[0]
        loss = torch.zeros(1, device=self.device)
        hist = []
        for ep in range(epochs):
            perm = torch.as_tensor(rng.permutation(S), device=self.device)
            lr_ep = lr * (1.0 - 0.9 * ep / max(epochs - 1, 1))      # linear decay to lr / 10
            for i in range(0, S - batch + 1, batch):
                sel = perm[i:i + batch]
                self.train_step(X[sel].contiguous(), W[sel].contiguous(), lr_ep, loss)
            hist.append(float(loss.item()))
        return hist


def raw_features(proj, angles, fy: int, fx: int):
    """Unstandardised network inputs of views proj [T][nv][nu]: block means + sin, cos."""
    return _lib.downsample(proj, fy, fx, angles=angles)


def warm_fit(scene: Scene, net: WarmStartNet, angles, meas, w_plain0, fy: int, fx: int,
             alt_above: float | None = None, **kw):
    """The warm-started fit: the network's prediction starts the LM fit; the views whose predicted
    start leaves a relative residual of at least alt_above (every view if None) also render the
    plain start (one more image per such view), and a view whose plain start leaves the smaller
    residual continues from it (the plain fit is the fallback). Returns (w, images, rel, seconds,
    fallbacks) with feature extraction, inference and the whole fit inside the timed span."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X = net.features(meas, angles, fy, fx)
    w_pred = net.predict(X)
    w_plain = np.broadcast_to(np.asarray(w_plain0, dtype=np.float64), w_pred.shape)
    info = {}
    w, images, rel = lm_fit(scene, angles, meas, w_pred, alt=w_plain, alt_above=alt_above,
                            info=info, **kw)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    return w, images, rel, sec, int(info["used_alt"].sum())


# ------------------------------------------------------------------------------------------------
def experiment(n: int, det_u: int, det_v: int, pitch: float, nviews: int, h_lattice: float,
               train_seeds, test_seeds, fy: int, fx: int, views_per_seed: int | None = None,
               batch: int = 64, tol: float = 1e-3, max_steps: int = 30, epochs: int = 40,
               lr: float = 1e-3, std_floor: float = 3.0, train_batch: int = 32, log=print):
    """The learned-warm-start experiment on the lung-phantom family: plain fits (started at the
    mean weights of the first training phantom's scan) label views of the training phantoms; the
    network is trained on those labels; on views of unseen phantoms, plain and warm-started fits
    race to the same residual tolerance. The training defaults (40 epochs of minibatches of 32,
    input spread floored at 3x the median) gave the fewest rendered images per view among the
    settings tried on an unseen phantom of the 200k / 512x384 family (9.5 against 10.4 for 60
    epochs of 128 with the floor at 1x). Returns a summary dict."""
    from . import synth
    rng = np.random.default_rng(12345)
    Xs, Ws, wmean, rel_plain = [], [], None, []
    t_label = 0.0
    for seed in train_seeds:
        p = synth.lung_phantom("warm_%d" % seed, n, det_u, det_v, pitch, nviews, 3, h_lattice,
                               seed)
        scene = Scene(p.geom, p.grid, p.coef, p.mu, p.scale, p.quat, p.rho)
        if wmean is None:
            wmean = p.w.mean(0, dtype=np.float64)
        views = np.arange(nviews) if views_per_seed is None else np.sort(
            rng.choice(nviews, views_per_seed, replace=False))
        conv = 0
        for b in range(0, len(views), batch):
            idx = views[b:b + batch]
            ang = torch.as_tensor(p.angles[idx], device="cuda")
            meas = scene.render(ang, torch.as_tensor(p.w[idx], device="cuda")).clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = {}
            w, steps, rel = lm_fit(scene, ang, meas, np.tile(wmean, (len(idx), 1)), tol=tol,
                                   max_steps=max_steps, info=info)
            torch.cuda.synchronize()
            t_label += time.perf_counter() - t0
            rel_plain.append(info["rel_start"])
            ok = rel <= tol
            conv += int(ok.sum())
            Xs.append(raw_features(meas, ang, fy, fx)[torch.as_tensor(ok, device="cuda")])
            Ws.append(w[ok])
        log("train phantom %d: %d/%d plain fits converged" % (seed, conv, len(views)))
        del scene
    X = torch.cat(Xs).contiguous()
    # a warm-started view also renders the plain start only if its predicted start leaves a
    # relative residual above the plain start's 5th percentile over the training views (below
    # it the plain start is very unlikely to be the better one)
    alt_above = float(np.percentile(np.concatenate(rel_plain), 5.0))
    W = np.concatenate(Ws)
    net = WarmStartNet(X.shape[1], 3, 256, seed=0)
    net.std_floor = std_floor
    t0 = time.perf_counter()
    hist = net.fit(X, W, epochs=epochs, batch=train_batch, lr=lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log("trained on %d pairs in %.1f s; loss %.4f -> %.4f" % (len(W), t_train, hist[0], hist[-1]))
    res = dict(plain_images=[], warm_images=[], plain_s=0.0, warm_s=0.0, plain_conv=0, warm_conv=0,
               fallbacks=0, views=0)
    for seed in test_seeds:
        p = synth.lung_phantom("warm_%d" % seed, n, det_u, det_v, pitch, nviews, 3, h_lattice,
                               seed)
        scene = Scene(p.geom, p.grid, p.coef, p.mu, p.scale, p.quat, p.rho)
        views = np.arange(nviews) if views_per_seed is None else np.sort(
            rng.choice(nviews, views_per_seed, replace=False))
        for b in range(0, len(views), batch):
            idx = views[b:b + batch]
            ang = torch.as_tensor(p.angles[idx], device="cuda")
            meas = scene.render(ang, torch.as_tensor(p.w[idx], device="cuda")).clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, sp, rp = lm_fit(scene, ang, meas, np.tile(wmean, (len(idx), 1)), tol=tol,
                               max_steps=max_steps)
            torch.cuda.synchronize()
            res["plain_s"] += time.perf_counter() - t0
            _, sw, rw, sec, fb = warm_fit(scene, net, ang, meas, wmean, fy, fx,
                                          alt_above=alt_above, tol=tol, max_steps=max_steps)
            res["warm_s"] += sec
            res["plain_images"].append(sp)
            res["warm_images"].append(sw)
            res["plain_conv"] += int((rp <= tol).sum())
            res["warm_conv"] += int((rw <= tol).sum())
            res["fallbacks"] += fb
            res["views"] += len(idx)
        log("test phantom %d done" % seed)
        del scene
    ps, ws_ = np.concatenate(res["plain_images"]), np.concatenate(res["warm_images"])
    return {"gaussians": n, "detector": [det_u, det_v], "tolerance": tol,
            "train_pairs": int(len(W)), "label_fit_s": round(t_label, 2),
            "train_s": round(t_train, 2), "loss_first_last": [hist[0], hist[-1]],
            "test_views": res["views"],
            "plain": {"mean_images_per_view": float(ps.mean()),
                      "converged": res["plain_conv"], "seconds": round(res["plain_s"], 3)},
            "warm": {"mean_images_per_view": float(ws_.mean()), "alt_above": alt_above,
                     "converged": res["warm_conv"], "seconds": round(res["warm_s"], 3),
                     "fallbacks": res["fallbacks"]},
            "wall_clock_speedup": round(res["plain_s"] / max(res["warm_s"], 1e-9), 3)}


def main(argv=None):
    """Run the learned-warm-start experiment. Default: the full-scale configuration (200k
    Gaussians, 512x384 at 0.8 mm, 1,320 views, training phantoms 0-14, held-out 100-102, 64x64
    network input from 8x6 block means)."""
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=200_000)
    ap.add_argument("--det", type=int, nargs=2, default=[512, 384])
    ap.add_argument("--pitch", type=float, default=0.8)
    ap.add_argument("--views", type=int, default=1320)
    ap.add_argument("--views-per-seed", type=int, default=None)
    ap.add_argument("--lattice", type=float, default=10.0)
    ap.add_argument("--train-seeds", type=int, default=15)
    ap.add_argument("--test-seeds", type=int, nargs="*", default=[100, 101, 102])
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--epochs", type=int, default=40)
    args = ap.parse_args(argv)
    fx, fy = args.det[0] // 64, args.det[1] // 64
    out = experiment(args.n, args.det[0], args.det[1], args.pitch, args.views, args.lattice,
                     list(range(args.train_seeds)), args.test_seeds, fy, fx,
                     views_per_seed=args.views_per_seed, tol=args.tol, epochs=args.epochs,
                     log=lambda m: print(m, flush=True))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
