"""ctypes binding of libdigs (include/digs.h): argument marshalling only.

Every step of the renderer runs in the HIP library; this module converts torch tensors to device
pointers, geometry/lattice dicts to the C structs, and raises on error codes. If the library is
missing the import fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdigs.so")

DIGS_BWD_REUSE_FWD = 1
_ERRORS = {-1: "DIGS_EINVAL", -2: "DIGS_ENOWS", -3: "DIGS_EHIP", -4: "DIGS_ECAPACITY",
           -5: "DIGS_ENOMEM", -6: "DIGS_ESCRATCH"}
NOALLOC_SCRATCH_BYTES = 64 << 20   # DIGS_NOALLOC_SCRATCH_BYTES


class DigsError(RuntimeError):
    def __init__(self, fn, code, hip=0):
        self.code = code
        super().__init__("%s failed: %s (%d)%s" % (fn, _ERRORS.get(code, "?"), code,
                                                    (", hip error %d" % hip) if hip else ""))


class Geom(ctypes.Structure):
    _fields_ = [("sid", ctypes.c_float), ("sdd", ctypes.c_float), ("nu", ctypes.c_int),
                ("nv", ctypes.c_int), ("pitch_u", ctypes.c_float), ("pitch_v", ctypes.c_float),
                ("off_u", ctypes.c_float), ("off_v", ctypes.c_float), ("model", ctypes.c_int)]


MODELS = {"exact": 0, "ewa": 1}   # DIGS_MODEL_EXACT, DIGS_MODEL_EWA


class Grid(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("nz", ctypes.c_int), ("origin", ctypes.c_float * 3),
                ("spacing", ctypes.c_float * 3)]


class Tuning(ctypes.Structure):
    _fields_ = [("cull_radius", ctypes.c_float), ("capacity", ctypes.c_int64),
                ("splat_waves", ctypes.c_int), ("slices", ctypes.c_int),
                ("persistent", ctypes.c_int), ("tile_w", ctypes.c_int), ("tile_h", ctypes.c_int)]


class Diag(ctypes.Structure):
    _fields_ = [("instances", ctypes.c_uint64), ("capacity", ctypes.c_uint64),
                ("overflow", ctypes.c_uint32), ("nonfinite", ctypes.c_uint32),
                ("folded", ctypes.c_uint32), ("behind_source", ctypes.c_uint32),
                ("wide", ctypes.c_uint32), ("reserved0", ctypes.c_uint32),
                ("max_instances", ctypes.c_uint64), ("reserved", ctypes.c_uint32 * 4)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_
                if not k.startswith("reserved")}


class VGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("origin", ctypes.c_float * 3), ("spacing", ctypes.c_float * 3)]


def make_vgrid(v: dict) -> VGrid:
    V = VGrid()
    V.nx, V.ny, V.nz = int(v["nx"]), int(v["ny"]), int(v["nz"])
    for a in range(3):
        V.origin[a] = float(v["origin"][a])
        V.spacing[a] = float(v["spacing"][a])
    return V


class PlanBuffers(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in (
        "coef", "mu", "scale", "quat", "rho", "angles", "w", "proj", "grad_proj", "g_mu",
        "g_scale", "g_quat", "g_rho", "g_coef", "g_w")]


TUNE_CANDIDATES = 12   # 3 tile shapes x 4 launch shapes
REPLAY_MODES = {"timed": 0, "graph": 1, "direct": 2}   # digs_plan_set_replay
_VP = ctypes.c_void_p
_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "digs_ffd_eval": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, ctypes.c_int, _VP, ctypes.c_int,
                                     _VP, _VP, _VP, _VP]),
    "digs_deform_gaussians": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, ctypes.c_int, _VP, _VP,
                                             _VP, ctypes.c_int, _VP, _VP, _VP, _VP]),
    "digs_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(Geom), ctypes.POINTER(Grid),
                                              ctypes.c_int, ctypes.c_int,
                                              ctypes.POINTER(Tuning)]),
    "digs_project_fwd": (ctypes.c_int, [ctypes.POINTER(Geom), ctypes.POINTER(Grid), _VP,
                                        ctypes.c_int, _VP, _VP, _VP, _VP, ctypes.c_int, _VP, _VP,
                                        _VP, _VP, ctypes.c_size_t, ctypes.POINTER(Tuning), _VP]),
    "digs_project_bwd": (ctypes.c_int, [ctypes.POINTER(Geom), ctypes.POINTER(Grid), _VP,
                                        ctypes.c_int, _VP, _VP, _VP, _VP, ctypes.c_int, _VP, _VP,
                                        _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t,
                                        ctypes.POINTER(Tuning), ctypes.c_int, _VP]),
    "digs_project_fwd_noalloc": (ctypes.c_int, [ctypes.POINTER(Geom), ctypes.POINTER(Grid), _VP,
                                                ctypes.c_int, _VP, _VP, _VP, _VP, ctypes.c_int,
                                                _VP, _VP, _VP, _VP, ctypes.POINTER(Tuning), _VP]),
    "digs_project_basis_fwd": (ctypes.c_int, [ctypes.POINTER(Geom), ctypes.POINTER(Grid), _VP,
                                              ctypes.c_int, _VP, _VP, _VP, _VP, ctypes.c_int,
                                              _VP, _VP, _VP, _VP, ctypes.c_size_t,
                                              ctypes.POINTER(Tuning), _VP]),
    "digs_project_basis_bwd": (ctypes.c_int, [ctypes.POINTER(Geom), ctypes.POINTER(Grid), _VP,
                                              ctypes.c_int, _VP, _VP, _VP, _VP, ctypes.c_int,
                                              _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                              ctypes.c_size_t, ctypes.POINTER(Tuning),
                                              ctypes.c_int, _VP]),
    "digs_read_diagnostics": (ctypes.c_int, [_VP, ctypes.POINTER(Diag), _VP]),
    "digs_reset_diagnostics": (ctypes.c_int, [_VP, _VP]),
    "digs_count_pairs": (ctypes.c_int, [ctypes.POINTER(Geom), ctypes.POINTER(Grid), ctypes.c_int,
                                        ctypes.c_int, _VP, ctypes.c_size_t,
                                        ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_uint64),
                                        _VP]),
    "digs_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "digs_profile_read": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int]),
    "digs_temporal_weights": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _VP, ctypes.c_float,
                                             ctypes.c_float, ctypes.c_int, _VP, _VP, _VP]),
    "digs_temporal_weights_bwd": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_float,
                                                 ctypes.c_float, ctypes.c_int, _VP, _VP, _VP,
                                                 _VP]),
    "digs_plan_create": (ctypes.c_int, [ctypes.POINTER(Geom), ctypes.POINTER(Grid), ctypes.c_int,
                                        ctypes.c_int, ctypes.POINTER(Tuning),
                                        ctypes.POINTER(PlanBuffers), ctypes.POINTER(_VP)]),
    "digs_plan_fwd": (ctypes.c_int, [_VP, _VP]),
    "digs_plan_fwd_views": (ctypes.c_int, [_VP, _VP]),
    "digs_plan_bwd": (ctypes.c_int, [_VP, _VP]),
    "digs_plan_check": (ctypes.c_int, [_VP, ctypes.POINTER(Diag), ctypes.POINTER(ctypes.c_int),
                                       _VP]),
    "digs_plan_get_tuning": (ctypes.c_int, [_VP, ctypes.POINTER(Tuning), _VP]),
    "digs_plan_set_replay": (ctypes.c_int, [_VP, ctypes.c_int]),
    "digs_plan_get_replay": (ctypes.c_int, [_VP, _VP]),
    "digs_plan_destroy": (ctypes.c_int, [_VP]),
    "digs_dvf_grid": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, _VP, ctypes.POINTER(VGrid), _VP,
                                     _VP]),
    "digs_phi_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(VGrid), ctypes.c_int,
                                                  ctypes.c_int64]),
    "digs_phi_grid": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, ctypes.c_int, _VP, _VP, _VP, _VP,
                                     _VP, ctypes.POINTER(VGrid), ctypes.c_float, ctypes.c_int64,
                                     _VP, _VP, ctypes.c_size_t, _VP]),
    "digs_lm_normal_eq": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, _VP, _VP,
                                         _VP, _VP]),
    "digs_gemm_bf16": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int,
                                      ctypes.c_int, _VP, ctypes.c_int, ctypes.c_int, _VP,
                                      ctypes.c_int, _VP, _VP, ctypes.c_int, ctypes.c_int, _VP]),
    "digs_colsum": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, _VP, _VP]),
    "digs_mse": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "digs_l2_residual": (ctypes.c_int, [ctypes.c_int64, _VP, _VP, _VP, _VP, _VP]),
    "digs_adam_mapped": (ctypes.c_int, [ctypes.c_int, _VP, _VP, _VP, _VP, _VP, ctypes.c_float,
                                        ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_int, ctypes.c_int, _VP]),
    "digs_adam": (ctypes.c_int, [ctypes.c_int, _VP, _VP, _VP, _VP, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_float, ctypes.c_int, _VP]),
    "digs_downsample": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, _VP, _VP, ctypes.c_float, _VP, _VP, _VP,
                                       ctypes.c_int, _VP]),
    "digs_standardize": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int, _VP, _VP,
                                        _VP]),
    "digs_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "digs_last_hip_error": (ctypes.c_int, []),
}


def load():
    """Load libdigs.so (built in-tree by paper_2506_22280_amd.build); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libdigs.so not found at %s: build it with "
                              "`python -m paper_2506_22280_amd.build` (no CPU fallback exists)"
                              % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(fn, rc):
    if rc != 0:
        raise DigsError(fn, rc, load().digs_last_hip_error() if rc == -3 else 0)


def make_geom(g: dict) -> Geom:
    G = Geom()
    G.sid, G.sdd = float(g["sid"]), float(g["sdd"])
    G.nu, G.nv = int(g["nu"]), int(g["nv"])
    G.pitch_u, G.pitch_v = float(g["pitch_u"]), float(g["pitch_v"])
    G.off_u, G.off_v = float(g.get("off_u", 0.0)), float(g.get("off_v", 0.0))
    G.model = MODELS[g.get("model", "exact")]
    return G


def make_grid(g: dict) -> Grid:
    G = Grid()
    G.R, G.nx, G.ny, G.nz = int(g["R"]), int(g["nx"]), int(g["ny"]), int(g["nz"])
    for a in range(3):
        G.origin[a] = float(g["origin"][a])
        G.spacing[a] = float(g["spacing"][a])
    return G


def make_tuning(t: dict | None):
    if not t:
        return None
    T = Tuning()
    T.cull_radius = float(t.get("cull_radius", 0.0))
    T.capacity = int(t.get("capacity", 0))
    T.splat_waves = int(t.get("splat_waves", 0))
    T.slices = int(t.get("slices", 0))
    T.persistent = int(t.get("persistent", 0))
    T.tile_w = int(t.get("tile_w", 0))
    T.tile_h = int(t.get("tile_h", 0))
    return T


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libdigs takes device tensors")
    if t.dtype != torch.float32 and t.dtype != torch.uint8:
        raise ValueError("libdigs takes float32 tensors, got %s" % t.dtype)
    if not t.is_contiguous():
        raise ValueError("libdigs takes contiguous tensors")
    return ctypes.c_void_p(t.data_ptr())


def _shape(name, t, shape):
    """Raise unless tensor t (or None, if allowed by the caller) has exactly this shape: the
    library indexes every buffer by the sizes passed beside it, so a smaller tensor would be read
    or written past its end."""
    if t is None:
        raise ValueError("%s is required" % name)
    if tuple(t.shape) != tuple(int(x) for x in shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))


def _lattice(grid: dict):
    return (grid["R"], grid["nz"], grid["ny"], grid["nx"], 3)


def _gaussians(n, mu, scale, quat, rho):
    _shape("mu", mu, (3, n))
    _shape("scale", scale, (3, n))
    _shape("quat", quat, (4, n))
    _shape("rho", rho, (n,))


def _views(T, R, angles, w):
    _shape("angles", angles, (T,))
    _shape("w", w, (T, R))


def _same_numel(name, t, numel):
    if t is not None and t.numel() != numel:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), numel))


def _grad_shapes(out: dict, motion: str, motion_shape, n, T, R):
    for k, shp in (("g_mu", (3, n)), ("g_scale", (3, n)), ("g_quat", (4, n)), ("g_rho", (n,)),
                   (motion, motion_shape), ("g_w", (T, R))):
        _shape(k, out.get(k), shp)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _byref(x):
    return ctypes.byref(x) if x is not None else None


# ------------------------------------------------------------------------------------------------
def ffd_eval(grid: dict, coef, x, w=None, jac=True, stream=None):
    """Per-rank (w None) or weighted (w [T][R]) FFD displacement and Jacobian (Eq. 9-11)."""
    n = x.shape[1]
    R = grid["R"]
    lead = R if w is None else w.shape[0]
    _shape("coef", coef, _lattice(grid))
    _shape("x", x, (3, n))
    if w is not None:
        _shape("w", w, (lead, R))
    disp = torch.empty((lead, 3, n), device=x.device, dtype=torch.float32)
    J = torch.empty((lead, 9, n), device=x.device, dtype=torch.float32) if jac else None
    G = make_grid(grid)
    _check("digs_ffd_eval", load().digs_ffd_eval(
        ctypes.byref(G), _ptr(coef), n, _ptr(x), 0 if w is None else w.shape[0], _ptr(w),
        _ptr(disp), _ptr(J), _stream(stream)))
    return disp, J


def deform_gaussians(grid: dict, coef, mu, scale, quat, w, stream=None):
    """mu_t [T][3][n], cov_t [T][6][n] of the deformation-informed warp (Eq. 7-8)."""
    n, T = mu.shape[1], w.shape[0]
    _shape("coef", coef, _lattice(grid))
    _shape("mu", mu, (3, n))
    _shape("scale", scale, (3, n))
    _shape("quat", quat, (4, n))
    _shape("w", w, (T, grid["R"]))
    mu_t = torch.empty((T, 3, n), device=mu.device, dtype=torch.float32)
    cov_t = torch.empty((T, 6, n), device=mu.device, dtype=torch.float32)
    G = make_grid(grid)
    _check("digs_deform_gaussians", load().digs_deform_gaussians(
        ctypes.byref(G), _ptr(coef), n, _ptr(mu), _ptr(scale), _ptr(quat), T, _ptr(w),
        _ptr(mu_t), _ptr(cov_t), _stream(stream)))
    return mu_t, cov_t


def temporal_weights(ctrl, t0: float, dt: float, times, stream=None):
    """w [T][R] of the temporal cubic B-spline over control values ctrl [Ct][R]."""
    Ct, R = ctrl.shape
    T = times.shape[0]
    w = torch.empty((T, R), device=ctrl.device, dtype=torch.float32)
    _check("digs_temporal_weights", load().digs_temporal_weights(
        Ct, R, _ptr(ctrl), float(t0), float(dt), T, _ptr(times), _ptr(w), _stream(stream)))
    return w


def temporal_weights_bwd(Ct: int, t0: float, dt: float, times, g_w, stream=None):
    """dL/dctrl [Ct][R] given dL/dw [T][R]."""
    T, R = g_w.shape
    _shape("times", times, (T,))
    g = torch.empty((Ct, R), device=g_w.device, dtype=torch.float32)
    _check("digs_temporal_weights_bwd", load().digs_temporal_weights_bwd(
        Ct, R, float(t0), float(dt), T, _ptr(times), _ptr(g_w), _ptr(g), _stream(stream)))
    return g


def workspace_size(geom: dict, grid: dict, n: int, T: int, tuning: dict | None = None) -> int:
    G, R, Tu = make_geom(geom), make_grid(grid), make_tuning(tuning)
    return int(load().digs_workspace_size(ctypes.byref(G), ctypes.byref(R), n, T, _byref(Tu)))


class Workspace:
    """A device workspace for project_fwd/project_bwd that grows when a call needs more."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None
        self._gen = 0

    def get(self, nbytes: int, stream=None):
        """The buffer, of at least nbytes; a new buffer's diagnostics block is cleared (on
        `stream`, before the call that uses it)."""
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
            self._gen += 1
            _check("digs_reset_diagnostics",
                   load().digs_reset_diagnostics(_ptr(self.buf), _stream(stream)))
        return self.buf

    def stamp(self):
        """Changes whenever a call re-bins into this workspace (or it is reallocated): a
        backward may reuse the forward's binning only while the stamp is unchanged."""
        return self._gen

    def touched(self):
        self._gen += 1

    def diagnostics(self, stream=None) -> dict:
        d = Diag()
        _check("digs_read_diagnostics",
               load().digs_read_diagnostics(_ptr(self.buf), ctypes.byref(d), _stream(stream)))
        return d.as_dict()

    def reset(self, stream=None):
        _check("digs_reset_diagnostics",
               load().digs_reset_diagnostics(_ptr(self.buf), _stream(stream)))


def project_fwd(geom: dict, grid: dict, coef, mu, scale, quat, rho, angles, w, ws: Workspace,
                tuning: dict | None = None, proj=None, stream=None):
    """proj [T][nv][nu] of the deformed Gaussians (Eq. 1, 3, 4, 6)."""
    n, T = mu.shape[1], angles.shape[0]
    _shape("coef", coef, _lattice(grid))
    _gaussians(n, mu, scale, quat, rho)
    _views(T, grid["R"], angles, w)
    if proj is not None:
        _shape("proj", proj, (T, geom["nv"], geom["nu"]))
    G, R, Tu = make_geom(geom), make_grid(grid), make_tuning(tuning)
    nbytes = int(load().digs_workspace_size(ctypes.byref(G), ctypes.byref(R), n, T, _byref(Tu)))
    if nbytes == 0:
        raise DigsError("digs_workspace_size", -1)
    buf = ws.get(nbytes, stream)
    if proj is None:
        proj = torch.empty((T, geom["nv"], geom["nu"]), device=mu.device, dtype=torch.float32)
    _check("digs_project_fwd", load().digs_project_fwd(
        ctypes.byref(G), ctypes.byref(R), _ptr(coef), n, _ptr(mu), _ptr(scale), _ptr(quat),
        _ptr(rho), T, _ptr(angles), _ptr(w), _ptr(proj), _ptr(buf), buf.numel(), _byref(Tu),
        _stream(stream)))
    ws.touched()
    return proj


def project_bwd(geom: dict, grid: dict, coef, mu, scale, quat, rho, angles, w, grad_proj,
                ws: Workspace, tuning: dict | None = None, reuse_fwd: bool = False, out=None,
                stream=None):
    """dL/d(mu, scale, quat, rho, coef, w) given dL/dproj (hand-written adjoint)."""
    n, T = mu.shape[1], angles.shape[0]
    _shape("coef", coef, _lattice(grid))
    _gaussians(n, mu, scale, quat, rho)
    _views(T, grid["R"], angles, w)
    _shape("grad_proj", grad_proj, (T, geom["nv"], geom["nu"]))
    if out is not None:
        _grad_shapes(out, "g_coef", _lattice(grid), n, T, grid["R"])
    G, R, Tu = make_geom(geom), make_grid(grid), make_tuning(tuning)
    nbytes = int(load().digs_workspace_size(ctypes.byref(G), ctypes.byref(R), n, T, _byref(Tu)))
    if nbytes == 0:
        raise DigsError("digs_workspace_size", -1)
    if reuse_fwd and (ws.buf is None or ws.buf.numel() < nbytes):
        reuse_fwd = False
    buf = ws.get(nbytes, stream)
    if out is None:
        dev = mu.device
        out = dict(g_mu=torch.empty((3, n), device=dev), g_scale=torch.empty((3, n), device=dev),
                   g_quat=torch.empty((4, n), device=dev), g_rho=torch.empty((n,), device=dev),
                   g_coef=torch.empty_like(coef), g_w=torch.empty((T, grid["R"]), device=dev))
    _check("digs_project_bwd", load().digs_project_bwd(
        ctypes.byref(G), ctypes.byref(R), _ptr(coef), n, _ptr(mu), _ptr(scale), _ptr(quat),
        _ptr(rho), T, _ptr(angles), _ptr(w), _ptr(grad_proj), _ptr(out["g_mu"]),
        _ptr(out["g_scale"]), _ptr(out["g_quat"]), _ptr(out["g_rho"]), _ptr(out["g_coef"]),
        _ptr(out["g_w"]), _ptr(buf), buf.numel(), _byref(Tu),
        DIGS_BWD_REUSE_FWD if reuse_fwd else 0, _stream(stream)))
    if not reuse_fwd:
        ws.touched()
    return out


def project_fwd_noalloc(geom: dict, grid: dict, coef, mu, scale, quat, rho, angles, w,
                        tuning: dict | None = None, proj=None, diag=None, stream=None):
    """project_fwd without a workspace (digs_project_fwd_noalloc: the library's fixed device
    array holds the intermediate buffers; nothing is allocated by the library). diag: a device
    uint8 tensor of at least ctypes.sizeof(Diag) bytes that receives the call's diagnostics
    (read it with diag_from_device), or None."""
    n, T = mu.shape[1], angles.shape[0]
    _shape("coef", coef, _lattice(grid))
    _gaussians(n, mu, scale, quat, rho)
    _views(T, grid["R"], angles, w)
    if proj is None:
        proj = torch.empty((T, geom["nv"], geom["nu"]), device=mu.device, dtype=torch.float32)
    _shape("proj", proj, (T, geom["nv"], geom["nu"]))
    if diag is not None and (diag.dtype != torch.uint8 or diag.numel() < ctypes.sizeof(Diag)):
        raise ValueError("diag must be a device uint8 tensor of at least %d bytes"
                         % ctypes.sizeof(Diag))
    G, R, Tu = make_geom(geom), make_grid(grid), make_tuning(tuning)
    _check("digs_project_fwd_noalloc", load().digs_project_fwd_noalloc(
        ctypes.byref(G), ctypes.byref(R), _ptr(coef), n, _ptr(mu), _ptr(scale), _ptr(quat),
        _ptr(rho), T, _ptr(angles), _ptr(w), _ptr(proj), _ptr(diag), _byref(Tu),
        _stream(stream)))
    return proj


def diag_from_device(diag) -> dict:
    """The digs_diag a no-allocation call wrote into the device buffer `diag` (synchronises
    with the copy)."""
    raw = bytes(diag[:ctypes.sizeof(Diag)].cpu().numpy().tobytes())
    return Diag.from_buffer_copy(raw).as_dict()


def project_basis_fwd(geom: dict, grid: dict, basis, mu, scale, quat, rho, angles, w,
                      ws: Workspace, tuning: dict | None = None, proj=None, stream=None):
    """The forward with the second ablation's motion model: basis [R][12][n] per Gaussian
    instead of the lattice (grid gives R and the lattice geometry that orders the Gaussians)."""
    n, T = mu.shape[1], angles.shape[0]
    _shape("basis", basis, (grid["R"], 12, n))
    _gaussians(n, mu, scale, quat, rho)
    _views(T, grid["R"], angles, w)
    if proj is not None:
        _shape("proj", proj, (T, geom["nv"], geom["nu"]))
    G, R, Tu = make_geom(geom), make_grid(grid), make_tuning(tuning)
    nbytes = int(load().digs_workspace_size(ctypes.byref(G), ctypes.byref(R), n, T, _byref(Tu)))
    if nbytes == 0:
        raise DigsError("digs_workspace_size", -1)
    buf = ws.get(nbytes, stream)
    if proj is None:
        proj = torch.empty((T, geom["nv"], geom["nu"]), device=mu.device, dtype=torch.float32)
    _check("digs_project_basis_fwd", load().digs_project_basis_fwd(
        ctypes.byref(G), ctypes.byref(R), _ptr(basis), n, _ptr(mu), _ptr(scale), _ptr(quat),
        _ptr(rho), T, _ptr(angles), _ptr(w), _ptr(proj), _ptr(buf), buf.numel(), _byref(Tu),
        _stream(stream)))
    ws.touched()
    return proj


def project_basis_bwd(geom: dict, grid: dict, basis, mu, scale, quat, rho, angles, w, grad_proj,
                      ws: Workspace, tuning: dict | None = None, reuse_fwd: bool = False,
                      out=None, stream=None):
    """dL/d(mu, scale, quat, rho, basis, w) of the basis model (reuse_fwd: ws holds the state
    of a project_basis_fwd with the same inputs)."""
    n, T = mu.shape[1], angles.shape[0]
    _shape("basis", basis, (grid["R"], 12, n))
    _gaussians(n, mu, scale, quat, rho)
    _views(T, grid["R"], angles, w)
    _shape("grad_proj", grad_proj, (T, geom["nv"], geom["nu"]))
    if out is not None:
        _grad_shapes(out, "g_basis", (grid["R"], 12, n), n, T, grid["R"])
    G, R, Tu = make_geom(geom), make_grid(grid), make_tuning(tuning)
    nbytes = int(load().digs_workspace_size(ctypes.byref(G), ctypes.byref(R), n, T, _byref(Tu)))
    if nbytes == 0:
        raise DigsError("digs_workspace_size", -1)
    if reuse_fwd and (ws.buf is None or ws.buf.numel() < nbytes):
        reuse_fwd = False
    buf = ws.get(nbytes, stream)
    dev = mu.device
    if out is None:
        out = dict(g_mu=torch.empty((3, n), device=dev), g_scale=torch.empty((3, n), device=dev),
                   g_quat=torch.empty((4, n), device=dev), g_rho=torch.empty((n,), device=dev),
                   g_basis=torch.empty_like(basis), g_w=torch.empty((T, grid["R"]), device=dev))
    _check("digs_project_basis_bwd", load().digs_project_basis_bwd(
        ctypes.byref(G), ctypes.byref(R), _ptr(basis), n, _ptr(mu), _ptr(scale), _ptr(quat),
        _ptr(rho), T, _ptr(angles), _ptr(w), _ptr(grad_proj), _ptr(out["g_mu"]),
        _ptr(out["g_scale"]), _ptr(out["g_quat"]), _ptr(out["g_rho"]), _ptr(out["g_basis"]),
        _ptr(out["g_w"]), _ptr(buf), buf.numel(), _byref(Tu),
        DIGS_BWD_REUSE_FWD if reuse_fwd else 0, _stream(stream)))
    if not reuse_fwd:
        ws.touched()
    return out


class ProfileEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


def profile_enable(on: bool = True):
    load().digs_profile_enable(1 if on else 0)


def profile_read(reset: bool = True) -> dict:
    """{stage: (launches, total_ms)} from the HIP events recorded around each stage launch."""
    buf = (ProfileEntry * 32)()
    k = load().digs_profile_read(ctypes.cast(buf, ctypes.c_void_p), 32, 1 if reset else 0)
    if k < 0:
        raise DigsError("digs_profile_read", k)
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms))
            for i in range(k)}


def count_pairs(geom: dict, grid: dict, n: int, T: int, ws: Workspace,
                tuning: dict | None = None, stream=None):
    """(pairs inside the cut-off footprints, forward-evaluated pairs, backward-evaluated pairs)
    of the last project_fwd on ws."""
    G, R, Tu = make_geom(geom), make_grid(grid), make_tuning(tuning)
    out = (ctypes.c_uint64 * 3)()
    _check("digs_count_pairs", load().digs_count_pairs(
        ctypes.byref(G), ctypes.byref(R), n, T, _ptr(ws.buf), ws.buf.numel(), _byref(Tu), out,
        _stream(stream)))
    return int(out[0]), int(out[1]), int(out[2])


class Plan:
    """The batched path (digs_plan_*): fixed shapes and buffers, its own workspace, the forward
    and backward replayed as HIP graphs or direct launches (``replay``: "timed", the faster of the
    two per sequence, or "graph" or "direct"). ``buffers`` maps the digs_plan_buffers names to
    device tensors; the plan keeps references to them, and a new batch is given by writing into
    them. tuning=None runs the library's autotuner on the buffers' current contents."""

    def __init__(self, geom: dict, grid: dict, n: int, T: int, buffers: dict,
                 tuning: dict | None = None, replay: str = "timed"):
        self.buffers = dict(buffers)
        R, nv, nu = grid["R"], geom["nv"], geom["nu"]
        expect = dict(coef=_lattice(grid), mu=(3, n), scale=(3, n), quat=(4, n), rho=(n,),
                      angles=(T,), w=(T, R), proj=(T, nv, nu), grad_proj=(T, nv, nu),
                      g_mu=(3, n), g_scale=(3, n), g_quat=(4, n), g_rho=(n,),
                      g_coef=_lattice(grid), g_w=(T, R))
        for k, shp in expect.items():
            if self.buffers.get(k) is not None:
                _shape(k, self.buffers[k], shp)
        B = PlanBuffers()
        for k, _ in PlanBuffers._fields_:
            t = self.buffers.get(k)
            setattr(B, k, _ptr(t).value if t is not None else None)
        G, R, Tu = make_geom(geom), make_grid(grid), make_tuning(tuning)
        h = ctypes.c_void_p()
        _check("digs_plan_create", load().digs_plan_create(
            ctypes.byref(G), ctypes.byref(R), n, T, _byref(Tu), ctypes.byref(B), ctypes.byref(h)))
        self._h = h
        if replay != "timed":
            self.set_replay(replay)

    def fwd(self, stream=None):
        _check("digs_plan_fwd", load().digs_plan_fwd(self._h, _stream(stream)))

    def fwd_views(self, stream=None):
        """The forward of new views of the same model: the per-Gaussian stage is taken from the
        last fwd() (valid while the Gaussian and lattice buffers are unchanged since it)."""
        _check("digs_plan_fwd_views", load().digs_plan_fwd_views(self._h, _stream(stream)))

    def bwd(self, stream=None):
        _check("digs_plan_bwd", load().digs_plan_bwd(self._h, _stream(stream)))

    def check(self, stream=None):
        """(diagnostics dict, resized): after resized, repeat the calls since the last check."""
        d = Diag()
        r = ctypes.c_int(0)
        _check("digs_plan_check", load().digs_plan_check(self._h, ctypes.byref(d),
                                                         ctypes.byref(r), _stream(stream)))
        return d.as_dict(), bool(r.value)

    def set_replay(self, mode: str):
        """"timed", "graph" or "direct" (digs_plan_set_replay)."""
        if mode not in REPLAY_MODES:
            raise ValueError("replay mode %r: one of %s" % (mode, sorted(REPLAY_MODES)))
        _check("digs_plan_set_replay", load().digs_plan_set_replay(self._h, REPLAY_MODES[mode]))

    def replay_modes(self):
        """{"fwd", "fwd_views", "bwd"} -> "graph", "direct" or None (not called yet)."""
        m = (ctypes.c_int * 3)()
        _check("digs_plan_get_replay", load().digs_plan_get_replay(
            self._h, ctypes.cast(m, ctypes.c_void_p)))
        names = {0: None, 1: "graph", 2: "direct"}
        return {k: names[m[i]] for i, k in enumerate(("fwd", "fwd_views", "bwd"))}

    def tuning(self):
        """(tuning dict, autotuner timings [candidate][fwd ms, bwd ms])."""
        t = Tuning()
        ms = (ctypes.c_float * (2 * TUNE_CANDIDATES))()
        _check("digs_plan_get_tuning", load().digs_plan_get_tuning(
            self._h, ctypes.byref(t), ctypes.cast(ms, ctypes.c_void_p)))
        d = {k: getattr(t, k) for k, _ in Tuning._fields_}
        return d, [[ms[2 * c], ms[2 * c + 1]] for c in range(TUNE_CANDIDATES)]

    def close(self):
        """Free the plan (its workspace and graphs); call before the process ends."""
        if getattr(self, "_h", None):
            load().digs_plan_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ------------------------------------------------------------------------------------------------
# Temporal-weight fit and learned warm start (kernels; the loops live in warmstart.py)
def lm_normal_eq(imgs, meas, h, R: int, stream=None):
    """[T][R(R+1)/2 + R + 1] normal-equation terms from imgs [T][R+1][npix], meas [T][npix]."""
    T = meas.shape[0]
    npix = meas[0].numel() if T else 0
    out = torch.empty((T, R * (R + 1) // 2 + R + 1), device=meas.device)
    _check("digs_lm_normal_eq", load().digs_lm_normal_eq(T, R, npix, _ptr(imgs), _ptr(meas),
                                                         _ptr(h), _ptr(out), _stream(stream)))
    return out


def gemm_bf16(A, B, C, transA=False, transB=False, bias=None, gate=None, relu=False,
              accumulate=False, stream=None):
    """C = epilogue(op(A) . op(B)) on the matrix cores (BF16 operands, FP32 accumulate)."""
    M = A.shape[1] if transA else A.shape[0]
    K = A.shape[0] if transA else A.shape[1]
    N = B.shape[0] if transB else B.shape[1]
    _check("digs_gemm_bf16", load().digs_gemm_bf16(
        M, N, K, _ptr(A), A.stride(0), int(transA), _ptr(B), B.stride(0), int(transB), _ptr(C),
        C.stride(0), _ptr(bias), _ptr(gate), int(relu), int(accumulate), _stream(stream)))
    return C


def colsum(X, out, stream=None):
    _check("digs_colsum", load().digs_colsum(X.shape[0], X.shape[1], _ptr(X), X.stride(0),
                                             _ptr(out), _stream(stream)))
    return out


def mse(pred, target, mean, std, dpred, loss=None, stream=None):
    _check("digs_mse", load().digs_mse(pred.shape[0], pred.shape[1], _ptr(pred), _ptr(target),
                                       _ptr(mean), _ptr(std), _ptr(dpred), _ptr(loss),
                                       _stream(stream)))


def adam(w, g, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    for k, t in (("g", g), ("m", m), ("v", v)):
        _same_numel(k, t, w.numel())
    _check("digs_adam", load().digs_adam(w.numel(), _ptr(w), _ptr(g), _ptr(m), _ptr(v),
                                         float(lr), float(b1), float(b2), float(eps), int(step),
                                         _stream(stream)))


MAPS = {"identity": 0, "exp": 1, "softplus": 2}


L2_PARTS = 256   # DIGS_L2_PARTS


def l2_residual(proj, meas, grad, loss=None, stream=None):
    """grad = proj - meas and (if loss, a device tensor of 1 + L2_PARTS floats)
    loss[0] = 1/2 ||proj - meas||^2."""
    _same_numel("meas", meas, proj.numel())
    _same_numel("grad", grad, proj.numel())
    _same_numel("loss", loss, 1 + L2_PARTS)
    _check("digs_l2_residual", load().digs_l2_residual(proj.numel(), _ptr(proj), _ptr(meas),
                                                       _ptr(grad), _ptr(loss), _stream(stream)))


def adam_mapped(raw, value, g_value, m, v, lr, step, mapping="identity", b1=0.9, b2=0.999,
                eps=1e-8, stream=None):
    """One Adam step on raw given dL/dvalue, value = mapping(raw) (rewritten)."""
    for k, t in (("value", value), ("g_value", g_value), ("m", m), ("v", v)):
        _same_numel(k, t, raw.numel())
    _check("digs_adam_mapped", load().digs_adam_mapped(
        raw.numel(), _ptr(raw), _ptr(value), _ptr(g_value), _ptr(m), _ptr(v), float(lr),
        float(b1), float(b2), float(eps), int(step), MAPS[mapping], _stream(stream)))


def downsample(proj, fy: int, fx: int, angles=None, scale=1.0, fmean=None, fistd=None, out=None,
               stream=None):
    """[T][(nv/fy)(nu/fx) (+2)] block means (x scale, standardised per feature if fmean/fistd are
    given, + sin, cos of the angle) of proj [T][nv][nu]."""
    T, nv, nu = proj.shape
    nfeat = (nv // fy) * (nu // fx) + (2 if angles is not None else 0)
    if out is None:
        out = torch.empty((T, nfeat), device=proj.device)
    _check("digs_downsample", load().digs_downsample(T, nv, nu, fy, fx, _ptr(proj), _ptr(angles),
                                                     float(scale), _ptr(fmean), _ptr(fistd),
                                                     _ptr(out), out.stride(0), _stream(stream)))
    return out


def standardize(X, mean, istd, ncols: int | None = None, stream=None):
    """In place: X[:, :ncols] = (X - mean) * istd per column."""
    N = X.shape[1] if ncols is None else ncols
    _check("digs_standardize", load().digs_standardize(X.shape[0], N, _ptr(X), X.stride(0),
                                                       _ptr(mean), _ptr(istd), _stream(stream)))
    return X


# ------------------------------------------------------------------------------------------------
# The dynamic volume at one time point on a voxel grid
def dvf_grid(grid: dict, coef, w, vgrid: dict, stream=None):
    """dvf [3][nz][ny][nx] = sum_r w_r u_r(x) at the voxel centres (w: device [R])."""
    V = make_vgrid(vgrid)
    _shape("coef", coef, _lattice(grid))
    _shape("w", w, (grid["R"],))
    out = torch.empty((3, V.nz, V.ny, V.nx), device=coef.device)
    G = make_grid(grid)
    _check("digs_dvf_grid", load().digs_dvf_grid(ctypes.byref(G), _ptr(coef), _ptr(w),
                                                 ctypes.byref(V), _ptr(out), _stream(stream)))
    return out


def phi_grid(grid: dict, coef, mu, scale, quat, rho, w, vgrid: dict, ws: "Workspace",
             cull: float = 0.0, capacity: int = 0, out=None, grow: bool = True, stream=None):
    """phi [nz][ny][nx]: the warped Gaussians (weights w, device [R]) summed at voxel centres.
    With grow, an overflow of the (brick, Gaussian) capacity reported by the diagnostics makes
    the call repeat with the capacity the diagnostics say is needed (this synchronises)."""
    V, G = make_vgrid(vgrid), make_grid(grid)
    n = mu.shape[1]
    _shape("coef", coef, _lattice(grid))
    _gaussians(n, mu, scale, quat, rho)
    _shape("w", w, (grid["R"],))
    if out is None:
        out = torch.empty((V.nz, V.ny, V.nx), device=mu.device)
    else:
        _shape("out", out, (V.nz, V.ny, V.nx))
    while True:
        nbytes = int(load().digs_phi_workspace_size(ctypes.byref(V), n, int(capacity)))
        if nbytes == 0:
            raise DigsError("digs_phi_workspace_size", -1)
        buf = ws.get(nbytes, stream)
        _check("digs_phi_grid", load().digs_phi_grid(
            ctypes.byref(G), _ptr(coef), n, _ptr(mu), _ptr(scale), _ptr(quat), _ptr(rho), _ptr(w),
            ctypes.byref(V), float(cull), int(capacity), _ptr(out), _ptr(buf), buf.numel(),
            _stream(stream)))
        ws.touched()
        if not grow:
            return out
        d = ws.diagnostics(stream)
        if not d["overflow"]:
            return out
        capacity = int(d["instances"] * 1.25) + 4096
