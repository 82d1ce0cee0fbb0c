"""Seeded synthetic inputs: Gaussian phantoms, low-rank breathing motion and CBCT geometry.

This module only draws inputs. It holds none of the renderer's arithmetic (no B-spline, no
deformation, no projection): tests, the benchmark and the oracle-based checks all take their
inputs from here, so the HIP path and the oracle always see the same float32 values.

The paper's own data (the XCAT phantom with processed DVFs, and 4D-Lung patient 4DCT with PCA
motion; Sec. 4.1) are not available. These phantoms stand in for them with the same geometry
class (source-isocentre 1000 mm, circular orbit, 0.4-1.6 mm detector pitch) and the same kind of
motion: a few spatial modes whose weights follow irregular breathing with cycle-to-cycle
amplitude variation and slow drift (the recipe of Sec. 4.1's 4DCT simulation).

Every array is float32 and C-contiguous, in the layouts of the C ABI:
  mu[3][N], scale[3][N] (linear mm), quat[4][N] (w,x,y,z), rho[N] (mm^-1),
  coef[R][nz][ny][nx][3] (mm per unit weight), w[T][R], angles[T] (rad).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SID_MM = 1000.0
SDD_MM = 1500.0


@dataclass
class Problem:
    name: str
    geom: dict
    grid: dict
    coef: np.ndarray
    mu: np.ndarray
    scale: np.ndarray
    quat: np.ndarray
    rho: np.ndarray
    angles: np.ndarray      # all views of the scan
    times: np.ndarray       # acquisition time of each view (s)
    w: np.ndarray           # temporal weights of each view [T][R]
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.mu.shape[1])

    def gaussians(self):
        return self.mu, self.scale, self.quat, self.rho

    def views(self, idx):
        idx = np.asarray(idx)
        return (np.ascontiguousarray(self.angles[idx]), np.ascontiguousarray(self.w[idx]))


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _random_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def geometry(nu, nv, pitch, sid=SID_MM, sdd=SDD_MM, off_u=0.0, off_v=0.0) -> dict:
    return dict(sid=float(sid), sdd=float(sdd), nu=int(nu), nv=int(nv), pitch_u=float(pitch),
                pitch_v=float(pitch), off_u=float(off_u), off_v=float(off_v))


# ------------------------------------------------------------------------------------------------
# Tiny problem: 4,096 Gaussians in a 64 mm cube, 64x64 detector, 16 views, rank-3 FFD on 8^3.
def tiny(seed: int = 0, n: int = 4096, nviews: int = 16, det: int = 64) -> Problem:
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-32.0, 32.0, (3, n))
    scale = np.exp(rng.uniform(math.log(1.0), math.log(4.0), (3, n)))
    quat = _random_quats(rng, n)
    rho = rng.uniform(0.0, 1.0, n)
    R = 3
    h = 12.8
    grid = dict(R=R, nx=8, ny=8, nz=8, origin=[-44.8] * 3, spacing=[h] * 3)
    coef = rng.normal(0.0, 2.0, (R, 8, 8, 8, 3))
    k = np.arange(nviews)
    angles = 2.0 * math.pi * k / nviews
    times = 0.25 * k
    amp = np.array([1.0, 0.5, 0.25])
    eps = rng.uniform(-0.1, 0.1, (nviews, R))
    w = np.stack([amp[r] * (1.0 + eps[:, r]) *
                  np.sin(2.0 * math.pi * times / 4.0 + 2.0 * math.pi * r / 3.0)
                  for r in range(R)], axis=1)
    return Problem("tiny", geometry(det, det, 1.0), grid, _f32(coef), _f32(mu), _f32(scale),
                   _f32(quat), _f32(rho), _f32(angles), _f32(times), _f32(w))


# ------------------------------------------------------------------------------------------------
# Lung-like phantom family (body shell, two lungs, a dense lesion) with breathing motion.
BODY_AXES = np.array([125.0, 95.0, 128.0])
SHELL_MM = 8.0
LUNG_CENTRES = np.array([[55.0, 0.0, 20.0], [-55.0, 0.0, 20.0]])
LUNG_AXES = np.array([45.0, 60.0, 90.0])
LESION_CENTRE = np.array([50.0, 10.0, 0.0])
LESION_RADIUS = 10.0
F_BODY, F_SHELL, F_LUNG, F_LESION = 0.019, 0.025, 0.004, 0.022


def _ell_r(x, c, axes):
    return np.sqrt((((x - c[:, None]) / axes[:, None]) ** 2).sum(0))


def attenuation(x):
    """Piecewise-constant attenuation (mm^-1) of the phantom at points x[3][m]."""
    f = np.zeros(x.shape[1])
    rb = _ell_r(x, np.zeros(3), BODY_AXES)
    inner = _ell_r(x, np.zeros(3), BODY_AXES - SHELL_MM)
    f[rb <= 1.0] = F_BODY
    f[(rb <= 1.0) & (inner > 1.0)] = F_SHELL
    for c in LUNG_CENTRES:
        f[_ell_r(x, c, LUNG_AXES) <= 1.0] = F_LUNG
    f[np.linalg.norm(x - LESION_CENTRE[:, None], axis=0) <= LESION_RADIUS] = F_LESION
    return f


def _uniform_in_ellipsoid(rng, m, centre, axes):
    out = np.empty((3, 0))
    while out.shape[1] < m:
        p = rng.uniform(-1.0, 1.0, (3, 2 * m + 16))
        p = p[:, (p ** 2).sum(0) <= 1.0]
        out = np.concatenate([out, centre[:, None] + axes[:, None] * p], axis=1)
    return out[:, :m]


def phantom_gaussians(n: int, seed: int):
    """Gaussians whose sum approximates the phantom: centres uniform in the body, 2% of them in
    the lesion; scales log-uniform in [0.3, 0.9] of the mean spacing; densities set so that the
    local sum of Gaussians is about the phantom's attenuation."""
    rng = np.random.default_rng(seed)
    n_les = max(1, int(round(0.02 * n)))
    n_body = n - n_les
    v_body = 4.0 / 3.0 * math.pi * BODY_AXES.prod()
    v_les = 4.0 / 3.0 * math.pi * LESION_RADIUS ** 3
    mu_b = _uniform_in_ellipsoid(rng, n_body, np.zeros(3), BODY_AXES)
    mu_l = _uniform_in_ellipsoid(rng, n_les, LESION_CENTRE, np.full(3, LESION_RADIUS))
    h_b = (v_body / n_body) ** (1.0 / 3.0)
    h_l = (v_les / n_les) ** (1.0 / 3.0)
    s_b = h_b * np.exp(rng.uniform(math.log(0.3), math.log(0.9), (3, n_body)))
    s_l = h_l * np.exp(rng.uniform(math.log(0.3), math.log(0.9), (3, n_les)))
    # body Gaussians carry the background (the lesion counts as lung there); the lesion
    # Gaussians add the lesion's excess over lung
    f_b = attenuation(mu_b)
    in_les = np.linalg.norm(mu_b - LESION_CENTRE[:, None], axis=0) <= LESION_RADIUS
    f_b[in_les] = F_LUNG
    norm = (2.0 * math.pi) ** 1.5
    rho_b = f_b * h_b ** 3 / (norm * s_b.prod(0))
    rho_l = np.full(n_les, F_LESION - F_LUNG) * h_l ** 3 / (norm * s_l.prod(0))
    mu = np.concatenate([mu_b, mu_l], axis=1)
    scale = np.concatenate([s_b, s_l], axis=1)
    rho = np.concatenate([rho_b, rho_l])
    quat = _random_quats(rng, n)
    perm = rng.permutation(n)
    return mu[:, perm], scale[:, perm], quat[:, perm], rho[perm]


def _bump(x, shift=(0.0, 0.0, 0.0)):
    """Smooth motion envelope: 1 deep in the chest (including the lungs), falling to 0 with a
    cosine taper at the body's edge."""
    rb = _ell_r(x - np.asarray(shift)[:, None], np.zeros(3), BODY_AXES)
    t = np.clip((rb - 0.55) / (1.1 - 0.55), 0.0, 1.0)
    return 0.5 * (1.0 + np.cos(math.pi * t))


# spatial modes: (direction, envelope shift in mm); the weights carry the amplitude in mm
MODES = [
    ((0.0, 0.0, 1.0), (0.0, 0.0, 0.0)),      # superior-inferior
    ((0.0, 0.3, 0.0), (0.0, 0.0, 0.0)),      # anterior-posterior
    ((0.1, 0.0, 0.2), (0.0, 0.0, -30.0)),    # hysteresis, centred 30 mm inferior
    ((0.2, 0.1, 0.0), (0.0, 20.0, 0.0)),     # lateral (rank 4 only)
]


def motion_lattice(R: int, h: float, fov: float = 256.0):
    """Control lattice covering the field of view plus one cell and the B-spline support, with
    coefficients sampled from the spatial modes at the control points."""
    n = int(math.ceil(fov / h)) + 3
    o = -fov / 2.0 - h
    grid = dict(R=R, nx=n, ny=n, nz=n, origin=[o] * 3, spacing=[h] * 3)
    ax = o + h * np.arange(n)
    zz, yy, xx = np.meshgrid(ax, ax, ax, indexing="ij")
    pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()])
    coef = np.zeros((R, n, n, n, 3))
    for r in range(R):
        d, shift = MODES[r]
        env = _bump(pts, shift).reshape(n, n, n)
        for a in range(3):
            coef[r, ..., a] = d[a] * env
    return grid, coef


def breathing_weights(times, R: int, seed: int):
    """Irregular breathing: per-cycle period U(3,5) s and amplitude U(5,15) mm for the SI mode,
    a phase-lagged AP mode, and a slow 2 mm/min drift on the third mode."""
    rng = np.random.default_rng(seed + 7919)
    tmax = float(np.max(times)) + 5.0
    starts, periods, amps = [0.0], [], []
    while starts[-1] < tmax:
        periods.append(rng.uniform(3.0, 5.0))
        amps.append(rng.uniform(5.0, 15.0))
        starts.append(starts[-1] + periods[-1])
    starts = np.array(starts[:-1]); periods = np.array(periods); amps = np.array(amps)
    c = np.searchsorted(starts, times, side="right") - 1
    phase = (times - starts[c]) / periods[c]
    A = amps[c]
    w = np.zeros((len(times), R))
    w[:, 0] = A * 0.5 * (1.0 - np.cos(2.0 * math.pi * phase))
    if R > 1:
        w[:, 1] = A * 0.5 * (1.0 - np.cos(2.0 * math.pi * phase - 0.3))
    if R > 2:
        w[:, 2] = 2.0 * times / 60.0
    if R > 3:
        w[:, 3] = 0.5 * A * np.sin(2.0 * math.pi * phase)
    return w


def lung_phantom(name: str, n: int, det_u: int, det_v: int, pitch: float, nviews: int,
                 R: int, h: float, seed: int, scan_s: float = 60.0) -> Problem:
    mu, scale, quat, rho = phantom_gaussians(n, seed)
    grid, coef = motion_lattice(R, h)
    k = np.arange(nviews)
    angles = 2.0 * math.pi * k / nviews
    times = scan_s * k / nviews
    w = breathing_weights(times, R, seed)
    return Problem(name, geometry(det_u, det_v, pitch), grid, _f32(coef), _f32(mu), _f32(scale),
                   _f32(quat), _f32(rho), _f32(angles), _f32(times), _f32(w))


def single_view(seed: int = 0) -> Problem:
    """50k Gaussians, 256x256 detector at 1.6 mm, 680 views over 60 s, rank-3 FFD at 10 mm."""
    return lung_phantom("single_view_50k", 50_000, 256, 256, 1.6, 680, 3, 10.0, seed)


def batched(seed: int = 0) -> Problem:
    """200k Gaussians, 512x384 detector at 0.8 mm, 1,320 views, rank-3 FFD at 10 mm."""
    p = lung_phantom("batched_200k", 200_000, 512, 384, 0.8, 1320, 3, 10.0, seed)
    p.extra["batch"] = 64
    return p


def large(seed: int = 0) -> Problem:
    """500k Gaussians, 1024x768 detector at 0.4 mm, 2,000 views, rank-4 FFD at 5 mm."""
    p = lung_phantom("large_500k", 500_000, 1024, 768, 0.4, 2000, 4, 5.0, seed)
    p.extra["batch"] = 64
    return p


def paper_case(seed: int = 0, n: int = 80_000, nviews: int = 310, R: int = 2, h: float = 8.0,
               det: int = 512, pitch: float = 0.8, scan_s: float = 80.0) -> Problem:
    """The paper's acquisition (Sec. 4.1) on the lung phantom family: views over a full circle at
    times sampled uniformly over about 20 breathing cycles (80 s at a mean period of 4 s), a
    512x512 detector at 0.8 mm offset by 116 mm along e_u (half fan), SID 1000 mm and SDD 1536 mm;
    rank-2 motion on a lattice of 8 mm spacing (Sec. 4.2); 80k Gaussians (the initial cloud's
    size)."""
    mu, scale, quat, rho = phantom_gaussians(n, seed)
    grid, coef = motion_lattice(R, h)
    k = np.arange(nviews)
    angles = 2.0 * math.pi * k / nviews
    times = scan_s * k / nviews
    w = breathing_weights(times, R, seed)
    geom = geometry(det, det, pitch, sid=1000.0, sdd=1536.0, off_u=116.0 * det / 512.0)
    p = Problem("paper_case", geom, grid, _f32(coef), _f32(mu), _f32(scale), _f32(quat),
                _f32(rho), _f32(angles), _f32(times), _f32(w))
    p.extra["scan_s"] = scan_s
    return p


def add_noise(proj, lam: float = 1e8, sigma: float = 4.0, seed: int = 0):
    """Quantum and electronic noise on line-integral projections (Sec. 4.1): detected counts
    Poisson(lam e^-p) plus N(0, sigma^2), converted back to p = -log(max(counts, 1) / lam)."""
    rng = np.random.default_rng(seed + 31337)
    p = np.asarray(proj, dtype=np.float64)
    counts = rng.poisson(lam * np.exp(-p)).astype(np.float64) + rng.normal(0.0, sigma, p.shape)
    return _f32(-np.log(np.maximum(counts, 1.0) / lam))


def batch_schedule(nviews: int, batch: int, seed: int):
    """Uneven-time batches: a seeded permutation of all views cut into chunks of ``batch``."""
    perm = np.random.default_rng(seed + 104729).permutation(nviews)
    return [perm[i:i + batch] for i in range(0, nviews, batch)]


def small_phantom(n: int = 2048, det_u: int = 90, det_v: int = 75, pitch: float = 2.0,
                  nviews: int = 8, R: int = 3, h: float = 20.0, seed: int = 0) -> Problem:
    """A scaled-down member of the lung family that the oracle finishes in seconds; its detector
    is not a multiple of the tile size, so it also exercises ragged tiles."""
    return lung_phantom("small_phantom", n, det_u, det_v, pitch, nviews, R, h, seed)
