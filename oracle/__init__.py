"""FP64 CPU oracle of the DIGS deformation-informed Gaussian X-ray renderer.

TEST INFRASTRUCTURE, NOT PRODUCT CODE. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package. It shares no code with the HIP library in
``paper_2506_22280_amd``: the arithmetic lives in ``digs_oracle.c`` (plain C, double precision,
written from the paper's Eq. 1-11), and this module only marshals numpy arrays into it.

Functions mirror the product's entry points in argument meaning (not in precision):
  ffd_eval        Eq. 10-11   per-rank u_r(x) and grad u_r(x)
  deform          Eq. 7-9     mu' and Sigma' for every (t, n)
  project         Eq. 1,3,6   the closed-form line-integral sum at every pixel, no cut-off
                  Eq. 4       or, with geom["model"] == "ewa", the sum of the 2D Gaussians of Eq. 4
  ewa_gaussian    Eq. 4       one Gaussian's 2D mean, covariance and scaled density
  project_pixels              the same at a list of sampled pixels
  project_bwd                 reverse mode of ``project`` for a sparse dL/dI
                  Sec. 4.3    with ``basis`` (project, project_pixels, project_bwd): the second
                              ablation's motion model, a basis stored per Gaussian
  line_integral               one Gaussian along one line
  dvf, phi        Eq. 9, 6    displacement field and dynamic attenuation at query points
  temporal_weights            the 1-D cubic B-spline w_r(t) of the temporal control values, and
  temporal_weights_bwd        its adjoint
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "digs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
            "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Grid(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("nz", ctypes.c_int), ("origin", ctypes.c_double * 3),
                ("spacing", ctypes.c_double * 3), ("basis", ctypes.POINTER(ctypes.c_double))]


class Geom(ctypes.Structure):
    _fields_ = [("sid", ctypes.c_double), ("sdd", ctypes.c_double), ("nu", ctypes.c_int),
                ("nv", ctypes.c_int), ("pitch_u", ctypes.c_double),
                ("pitch_v", ctypes.c_double), ("off_u", ctypes.c_double),
                ("off_v", ctypes.c_double), ("model", ctypes.c_int)]


_lib = None
_P = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_bspline.argtypes = [ctypes.c_double, _P, _P, _P]
        lib.oracle_ffd_eval.argtypes = [ctypes.POINTER(Grid), _P, ctypes.c_int, _P, _P, _P]
        lib.oracle_deform.argtypes = [ctypes.POINTER(Grid), _P, ctypes.c_int, _P, _P, _P,
                                      ctypes.c_int, _P, _P, _P]
        lib.oracle_project.argtypes = [ctypes.POINTER(Geom), ctypes.POINTER(Grid), _P,
                                       ctypes.c_int, _P, _P, _P, _P, ctypes.c_int, _P, _P, _P]
        lib.oracle_project.restype = ctypes.c_int
        lib.oracle_project_pixels.argtypes = [ctypes.POINTER(Geom), ctypes.POINTER(Grid), _P,
                                              ctypes.c_int, _P, _P, _P, _P, ctypes.c_int, _P, _P,
                                              ctypes.c_int, _IP, _IP, _IP, _P]
        lib.oracle_project_pixels.restype = ctypes.c_int
        lib.oracle_project_bwd.argtypes = [ctypes.POINTER(Geom), ctypes.POINTER(Grid), _P,
                                           ctypes.c_int, _P, _P, _P, _P, ctypes.c_int, _P, _P,
                                           ctypes.c_int, _IP, _IP, _IP, _P,
                                           _P, _P, _P, _P, _P, _P]
        lib.oracle_project_bwd.restype = ctypes.c_int
        lib.oracle_ewa_gaussian.argtypes = [ctypes.POINTER(Geom), ctypes.c_double, _P, _P,
                                            ctypes.c_double, _P]
        lib.oracle_line_integral.argtypes = [_P, _P, ctypes.c_double, _P, _P]
        lib.oracle_line_integral.restype = ctypes.c_double
        lib.oracle_dvf.argtypes = [ctypes.POINTER(Grid), _P, _P, ctypes.c_int, _P, _P]
        lib.oracle_phi.argtypes = [ctypes.c_int, _P, _P, _P, ctypes.c_int, _P, _P]
        lib.oracle_temporal_weights.argtypes = [ctypes.c_int, ctypes.c_int, _P, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_int, _P, _P]
        lib.oracle_temporal_weights_bwd.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                    ctypes.c_double, ctypes.c_int, _P, _P, _P]
        _lib = lib
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_P)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_IP)


def make_grid(grid: dict) -> Grid:
    g = Grid()
    g.R, g.nx, g.ny, g.nz = int(grid["R"]), int(grid["nx"]), int(grid["ny"]), int(grid["nz"])
    for a in range(3):
        g.origin[a] = float(grid["origin"][a])
        g.spacing[a] = float(grid["spacing"][a])
    return g


def make_geom(geom: dict) -> Geom:
    G = Geom()
    G.sid, G.sdd = float(geom["sid"]), float(geom["sdd"])
    G.nu, G.nv = int(geom["nu"]), int(geom["nv"])
    G.pitch_u, G.pitch_v = float(geom["pitch_u"]), float(geom["pitch_v"])
    G.off_u, G.off_v = float(geom.get("off_u", 0.0)), float(geom.get("off_v", 0.0))
    G.model = {"exact": 0, "ewa": 1}[geom.get("model", "exact")]
    return G


def bspline(u: float):
    """B_l(u), B_l'(u), B_l''(u) for l = 0..3 (Eq. 10)."""
    B = np.zeros(4); dB = np.zeros(4); d2B = np.zeros(4)
    _load().oracle_bspline(float(u), B.ctypes.data_as(_P), dB.ctypes.data_as(_P),
                           d2B.ctypes.data_as(_P))
    return B, dB, d2B


def ffd_eval(grid: dict, coef, x):
    """Per-rank U[R][3][n] = u_r(x) and V[R][9][n] = grad u_r(x) (Eq. 10-11). x is [3][n]."""
    g = make_grid(grid)
    coef, pc = _d(coef)
    x, px = _d(x)
    n = x.shape[1]
    U = np.zeros((g.R, 3, n)); V = np.zeros((g.R, 9, n))
    _load().oracle_ffd_eval(ctypes.byref(g), pc, n, px, U.ctypes.data_as(_P),
                            V.ctypes.data_as(_P))
    return U, V


def deform(grid: dict, coef, mu, scale, quat, w):
    """mu_t[T][3][n], cov_t[T][6][n] (xx,xy,xz,yy,yz,zz) after Eq. 7-9; w is [T][R]."""
    g = make_grid(grid)
    coef, pc = _d(coef); mu, pm = _d(mu); scale, ps = _d(scale); quat, pq = _d(quat)
    w, pw = _d(np.atleast_2d(w))
    n, T = mu.shape[1], w.shape[0]
    mu_t = np.zeros((T, 3, n)); cov_t = np.zeros((T, 6, n))
    _load().oracle_deform(ctypes.byref(g), pc, n, pm, ps, pq, T, pw, mu_t.ctypes.data_as(_P),
                          cov_t.ctypes.data_as(_P))
    return mu_t, cov_t


def _with_basis(g: Grid, basis, n):
    """Point g at a per-Gaussian basis [R][12][n] (returns the array to keep alive)."""
    if basis is None:
        return None
    b = np.ascontiguousarray(basis, dtype=np.float64)
    assert b.shape == (g.R, 12, n), b.shape
    g.basis = b.ctypes.data_as(_P)
    return b


def project(geom: dict, grid: dict, coef, mu, scale, quat, rho, angles, w, basis=None):
    """proj[T][nv][nu]: the sum of every Gaussian's closed-form line integral (no cut-off).
    basis [R][12][n]: the per-Gaussian motion basis of the second ablation instead of the FFD
    (coef is then ignored and may be None)."""
    G, g = make_geom(geom), make_grid(grid)
    keep = _with_basis(g, basis, np.shape(mu)[1])
    if coef is None:
        coef = np.zeros(1)
    coef, pc = _d(coef); mu, pm = _d(mu); scale, ps = _d(scale); quat, pq = _d(quat)
    rho, pr = _d(rho); angles, pa = _d(np.atleast_1d(angles)); w, pw = _d(np.atleast_2d(w))
    n, T = mu.shape[1], angles.shape[0]
    assert w.shape == (T, g.R)
    out = np.zeros((T, G.nv, G.nu))
    rc = _load().oracle_project(ctypes.byref(G), ctypes.byref(g), pc, n, pm, ps, pq, pr, T, pa,
                                pw, out.ctypes.data_as(_P))
    del keep
    if rc != 0:
        raise MemoryError("oracle_project failed")
    return out


def project_pixels(geom: dict, grid: dict, coef, mu, scale, quat, rho, angles, w, pt, pj, pi):
    """The projection value at sampled pixels (pt[k], pj[k], pi[k])."""
    G, g = make_geom(geom), make_grid(grid)
    coef, pc = _d(coef); mu, pm = _d(mu); scale, ps = _d(scale); quat, pq = _d(quat)
    rho, pr = _d(rho); angles, pa = _d(np.atleast_1d(angles)); w, pw = _d(np.atleast_2d(w))
    pt, ppt = _i(pt); pj, ppj = _i(pj); pi, ppi = _i(pi)
    n, T = mu.shape[1], angles.shape[0]
    out = np.zeros(pt.shape[0])
    rc = _load().oracle_project_pixels(ctypes.byref(G), ctypes.byref(g), pc, n, pm, ps, pq, pr,
                                       T, pa, pw, pt.shape[0], ppt, ppj, ppi,
                                       out.ctypes.data_as(_P))
    if rc != 0:
        raise MemoryError("oracle_project_pixels failed")
    return out


def project_bwd(geom: dict, grid: dict, coef, mu, scale, quat, rho, angles, w, grad_proj=None,
                pixels=None, basis=None):
    """Gradients of L with dL/dI given densely (grad_proj[T][nv][nu]) or sparsely
    (pixels = (pt, pj, pi, g)). Returns dict g_mu, g_scale, g_quat, g_rho, g_coef, g_w; with a
    per-Gaussian basis [R][12][n], g_basis replaces g_coef."""
    G, g = make_geom(geom), make_grid(grid)
    keep = _with_basis(g, basis, np.shape(mu)[1])
    if coef is None:
        coef = np.zeros(1)
    coef, pc = _d(coef); mu, pm = _d(mu); scale, ps = _d(scale); quat, pq = _d(quat)
    rho, pr = _d(rho); angles, pa = _d(np.atleast_1d(angles)); w, pw = _d(np.atleast_2d(w))
    n, T = mu.shape[1], angles.shape[0]
    if pixels is None:
        gp = np.asarray(grad_proj, dtype=np.float64).reshape(T, G.nv, G.nu)
        pt, pj, pi = np.nonzero(gp)
        pg = gp[pt, pj, pi]
    else:
        pt, pj, pi, pg = pixels
    pt, ppt = _i(pt); pj, ppj = _i(pj); pi, ppi = _i(pi); pg, ppg = _d(pg)
    out = dict(g_mu=np.zeros((3, n)), g_scale=np.zeros((3, n)), g_quat=np.zeros((4, n)),
               g_rho=np.zeros(n), g_coef=np.zeros_like(coef) if keep is None else
               np.zeros((g.R, 12, n)), g_w=np.zeros((T, g.R)))
    if G.model != 0:
        raise ValueError("the oracle's reverse mode covers the exact model only")
    rc = _load().oracle_project_bwd(
        ctypes.byref(G), ctypes.byref(g), pc, n, pm, ps, pq, pr, T, pa, pw, pt.shape[0], ppt,
        ppj, ppi, ppg, *[out[k].ctypes.data_as(_P) for k in
                         ("g_mu", "g_scale", "g_quat", "g_rho", "g_coef", "g_w")])
    del keep
    if rc != 0:
        raise MemoryError("oracle_project_bwd failed")
    if basis is not None:
        out["g_basis"] = out.pop("g_coef")
    return out


def line_integral(mu, cov6, rho, src, direction) -> float:
    """One Gaussian's integral along the whole line src + lambda * direction."""
    mu, pm = _d(mu); cov6, pc = _d(cov6); src, ps = _d(src); direction, pd = _d(direction)
    return float(_load().oracle_line_integral(pm, pc, float(rho), ps, pd))


def ewa_gaussian(geom: dict, theta: float, mu, cov6, rho):
    """Eq. 4's 2D Gaussian of one 3D Gaussian at view angle theta: (mean[2] in detector mm from
    the detector centre, covariance [[uu, uv], [uv, vv]] in mm^2, scaled density rho~)."""
    G = make_geom(geom)
    mu, pm = _d(mu); cov6, pc = _d(cov6)
    out = np.zeros(6)
    _load().oracle_ewa_gaussian(ctypes.byref(G), float(theta), pm, pc, float(rho),
                                out.ctypes.data_as(_P))
    return out[:2].copy(), np.array([[out[2], out[3]], [out[3], out[4]]]), float(out[5])


def dvf(grid: dict, coef, w_t, x):
    """Displacement sum_r w_r u_r(x) at points x[3][m] (Eq. 9), returned as [3][m]."""
    g = make_grid(grid)
    coef, pc = _d(coef); w_t, pw = _d(w_t); x, px = _d(x)
    out = np.zeros((3, x.shape[1]))
    _load().oracle_dvf(ctypes.byref(g), pc, pw, x.shape[1], px, out.ctypes.data_as(_P))
    return out


def phi(mu_t, cov_t, rho, x):
    """phi(x) = sum_n rho_n exp(-(x-mu_n)^T Sigma_n^-1 (x-mu_n)/2) (Eq. 2-3, 6) at x[3][m];
    mu_t [3][n], cov_t [6][n] of one time point."""
    mu_t, pm = _d(mu_t); cov_t, pc = _d(cov_t); rho, pr = _d(rho); x, px = _d(x)
    out = np.zeros(x.shape[1])
    _load().oracle_phi(mu_t.shape[1], pm, pc, pr, x.shape[1], px, out.ctypes.data_as(_P))
    return out


def temporal_weights(ctrl, t0: float, dt: float, times):
    """w[T][R] of the temporal cubic B-spline over control values ctrl[Ct][R] every dt from t0."""
    ctrl, pc = _d(ctrl); times, pt = _d(np.atleast_1d(times))
    Ct, R = ctrl.shape
    w = np.zeros((times.shape[0], R))
    _load().oracle_temporal_weights(Ct, R, pc, float(t0), float(dt), times.shape[0], pt,
                                    w.ctypes.data_as(_P))
    return w


def temporal_weights_bwd(Ct: int, t0: float, dt: float, times, g_w):
    """dL/dctrl[Ct][R] given dL/dw[T][R]."""
    times, pt = _d(np.atleast_1d(times)); g_w, pg = _d(g_w)
    R = g_w.shape[1]
    g = np.zeros((Ct, R))
    _load().oracle_temporal_weights_bwd(Ct, R, float(t0), float(dt), times.shape[0], pt, pg,
                                        g.ctypes.data_as(_P))
    return g
