"""torch.autograd wrapper of the renderer: forward = digs_project_fwd, backward = the library's
hand-written adjoint digs_project_bwd (no autograd tape through the renderer's arithmetic).

    proj = project(geom, grid, mu, scale, quat, rho, coef, w, angles, ws)

Differentiable inputs: mu [3][N], scale [3][N], quat [4][N], rho [N], coef [R][nz][ny][nx][3],
w [T][R] (all float32 on the GPU). angles [T] and the geometry are constants. The loss's gradient
dL/dproj arrives in backward; the adjoint turns it into the six input gradients (Sec. 3.1-3.3:
through the splat, the projected record, the covariance warp K Sigma K^T, the quaternion
normalisation and the B-spline FFD including its second derivatives).

An instance-capacity overflow is never silent here: the forward reads the workspace's diagnostics
after its call (a synchronisation) and, if the capacity was exceeded, repeats the call with room
for what it needed; the backward uses the capacity the forward ended with.
"""
from __future__ import annotations

import torch

from . import _lib


def project_checked(geom, grid, coef, mu, scale, quat, rho, angles, w, ws, tuning=None):
    """project_fwd whose result is complete: after the call the diagnostics are read, and an
    instance-capacity overflow repeats the call with the capacity it needed (1.25 x + 4096).
    Returns the projections and the tuning the complete call used."""
    if ws.buf is not None:
        ws.reset()   # counts from earlier calls on this workspace do not concern this one
    while True:
        proj = _lib.project_fwd(geom, grid, coef, mu, scale, quat, rho, angles, w, ws,
                                tuning=tuning)
        d = ws.diagnostics()
        if not d["overflow"]:
            return proj, tuning
        need = max(d["instances"], d["max_instances"])
        tuning = dict(tuning or {}, capacity=int(need * 1.25) + 4096)
        ws.reset()


class DigsProject(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mu, scale, quat, rho, coef, w, angles, geom, grid, ws, tuning):
        mu, scale, quat, rho, coef, w, angles = (
            x.detach().contiguous() for x in (mu, scale, quat, rho, coef, w, angles))
        proj, tuning = project_checked(geom, grid, coef, mu, scale, quat, rho, angles, w, ws,
                                       tuning)
        ctx.save_for_backward(mu, scale, quat, rho, coef, w, angles)
        ctx.geom, ctx.grid, ctx.ws, ctx.tuning = geom, grid, ws, tuning
        ctx.stamp = ws.stamp()
        return proj

    @staticmethod
    def backward(ctx, grad_proj):
        mu, scale, quat, rho, coef, w, angles = ctx.saved_tensors
        ws = ctx.ws
        # the forward's binning is still in the workspace unless another call used it since
        reuse = ws.stamp() == ctx.stamp
        g = _lib.project_bwd(ctx.geom, ctx.grid, coef, mu, scale, quat, rho, angles, w,
                             grad_proj.contiguous(), ws, tuning=ctx.tuning, reuse_fwd=reuse)
        return (g["g_mu"], g["g_scale"], g["g_quat"], g["g_rho"], g["g_coef"], g["g_w"],
                None, None, None, None, None)


def project(geom: dict, grid: dict, mu, scale, quat, rho, coef, w, angles,
            ws: _lib.Workspace | None = None, tuning: dict | None = None):
    """Differentiable projections proj [T][nv][nu] of the deformed Gaussians."""
    if ws is None:
        ws = _lib.Workspace(mu.device)
    return DigsProject.apply(mu, scale, quat, rho, coef, w, angles, geom, grid, ws, tuning)
