"""Seeded synthetic scenes, cameras and gaze points.

This module builds inputs only.  It holds none of the renderer's arithmetic
(no projection, colour, binning or compositing): both the HIP path and the
FP64 oracle consume what it returns, and neither is imported here.

The scenes stand in for the trained models and datasets the paper measures
on (Mip-NeRF 360, Tanks & Temples, DeepBlending; Section 6), which are not
available.  What they take from the paper: 16x16 tiles (Section 5.2), about
sixty parameters per point with degree-3 spherical harmonics (Section 7.4),
uneven per-tile load from clustered geometry (Section 5.2), nested quality
subsets with per-level opacity and DC colour (Section 4.2) and four
eccentricity rings (Section 6).

Random draws are made with numpy's PCG64 ``default_rng(seed)`` in a fixed
order: means, log-scales, quaternions, opacity logits, DC, higher-order SH,
importance, level perturbations, cameras.  Arrays are cast to float32 last.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

SH_DC_BASIS = 0.28209479177387814  # value of the l=0 real SH basis, 1/(2 sqrt(pi))

CAMERA_FIELDS = 19  # width, height, fx, fy, cx, cy, R[9], t[3], near_z


@dataclass
class Camera:
    """Pinhole camera in the OpenCV frame (x right, y down, z forward).

    A world point x maps to camera space as ``R @ x + t``; pixel (i, j) is
    sampled at its integer coordinates.
    """

    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # (3, 3) world -> camera rotation
    t: np.ndarray  # (3,)
    near_z: float = 0.2

    @property
    def center(self) -> np.ndarray:
        return -self.R.T @ self.t

    def as_row(self) -> np.ndarray:
        """Flat float64 row in the field order of the C ``gs_camera`` struct."""
        return np.concatenate([
            [self.width, self.height, self.fx, self.fy, self.cx, self.cy],
            np.asarray(self.R, np.float64).reshape(9),
            np.asarray(self.t, np.float64).reshape(3),
            [self.near_z],
        ]).astype(np.float64)


def pinhole(width: int, height: int, fov_x_deg: float, R=None, t=None,
            near_z: float = 0.2) -> Camera:
    """Camera with a horizontal field of view, square pixels and the principal
    point at the image centre ((W-1)/2, (H-1)/2)."""
    f = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    R = np.eye(3) if R is None else np.asarray(R, np.float64)
    t = np.zeros(3) if t is None else np.asarray(t, np.float64)
    return Camera(width, height, f, f, (width - 1) / 2.0, (height - 1) / 2.0,
                  R, t, near_z)


def look_at(eye, target, width, height, fov_x_deg, up=(0.0, -1.0, 0.0)) -> Camera:
    """Camera at ``eye`` whose +z axis points at ``target``; ``up`` is the
    world direction that maps to image -y (y points down in the image)."""
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    upv = np.asarray(up, np.float64)
    x = np.cross(-upv, z)  # image right
    if np.linalg.norm(x) < 1e-9:
        x = np.cross(np.array([1.0, 0.0, 0.0]), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)  # image down
    R = np.stack([x, y, z])  # rows: camera axes in world coordinates
    return pinhole(width, height, fov_x_deg, R, -R @ eye)


def cameras_to_array(cams) -> np.ndarray:
    return np.stack([c.as_row() for c in cams])


@dataclass
class Scene:
    means: np.ndarray            # (N, 3) f32
    log_scales: np.ndarray       # (N, 3) f32
    quats: np.ndarray            # (N, 4) f32, (w, x, y, z), unit-norm draw
    opacity_logits: np.ndarray   # (N,) f32
    sh: np.ndarray               # (N, K, 3) f32, K = (d+1)^2
    sh_degree: int
    qbound: np.ndarray | None = None             # (N,) u8 in 1..4
    lvl_opacity_logits: np.ndarray | None = None  # (L, N) f32
    lvl_sh_dc: np.ndarray | None = None           # (L, N, 3) f32
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.means, self.log_scales, self.quats, self.opacity_logits,
                  self.sh, self.qbound, self.lvl_opacity_logits, self.lvl_sh_dc):
            if a is not None:
                h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(
            self.means[idx], self.log_scales[idx], self.quats[idx],
            self.opacity_logits[idx], self.sh[idx], self.sh_degree,
            None if self.qbound is None else self.qbound[idx],
            None if self.lvl_opacity_logits is None else self.lvl_opacity_logits[:, idx],
            None if self.lvl_sh_dc is None else self.lvl_sh_dc[:, idx],
            dict(self.meta))


def _random_rotations(rng, k):
    q = rng.standard_normal((k, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], 1)


def make_scene(n: int, sh_degree: int, seed: int, *, clustered: bool,
               log_scale_mu: float, log_scale_sigma: float,
               n_clusters: int = 64, fr_levels: int = 0,
               subset_fracs=(0.40, 0.15, 0.05)) -> Scene:
    """Draw a seeded scene (means, scales, rotations, opacity, SH, and for
    ``fr_levels`` > 0 the nested quality bounds and per-level versions)."""
    rng = np.random.default_rng(seed)
    # 1. means
    if clustered:
        centres = rng.uniform(-1.0, 1.0, (n_clusters, 3))
        weights = rng.dirichlet(np.ones(n_clusters))
        stds = np.exp(rng.uniform(math.log(0.05), math.log(0.4), (n_clusters, 3)))
        rots = _random_rotations(rng, n_clusters)
        assign = rng.choice(n_clusters, size=n, p=weights)
        local = rng.standard_normal((n, 3)) * stds[assign]
        means = centres[assign] + np.einsum("nij,nj->ni", rots[assign], local)
    else:
        means = rng.uniform(-1.0, 1.0, (n, 3))
    # 2. log-scales
    log_scales = rng.normal(log_scale_mu, log_scale_sigma, (n, 3))
    # 3. quaternions, uniform on S^3
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    # 4. opacity logits
    logits = rng.standard_normal(n)
    # 5. DC: base colour uniform in [0, 1]
    K = (sh_degree + 1) ** 2
    sh = np.zeros((n, K, 3))
    sh[:, 0, :] = (rng.uniform(0.0, 1.0, (n, 3)) - 0.5) / SH_DC_BASIS
    # 6. higher-order SH
    if K > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.2, (n, K - 1, 3))
    scene = Scene(means.astype(np.float32), log_scales.astype(np.float32),
                  q.astype(np.float32), logits.astype(np.float32),
                  sh.astype(np.float32), sh_degree)
    if fr_levels:
        # 7. importance -> nested quality bounds m in 1..L (Section 4.2)
        u = rng.uniform(0.0, 1.0, n)
        m = np.ones(n, np.int64)
        for frac in subset_fracs[: fr_levels - 1]:
            m += (u < frac)
        # 8. per-level versions of opacity and DC (selective multi-versioning)
        lvl_logits = np.empty((fr_levels, n))
        lvl_dc = np.empty((fr_levels, n, 3))
        lvl_logits[0] = logits
        lvl_dc[0] = sh[:, 0, :]
        for t in range(1, fr_levels):
            lvl_logits[t] = logits + rng.normal(0.0, 0.3, n)
            lvl_dc[t] = sh[:, 0, :] + rng.normal(0.0, 0.1, (n, 3))
        scene.qbound = m.astype(np.uint8)
        scene.lvl_opacity_logits = lvl_logits.astype(np.float32)
        scene.lvl_sh_dc = lvl_dc.astype(np.float32)
    scene.meta = dict(seed=seed, numpy=np.__version__, n=n, sh_degree=sh_degree,
                      clustered=clustered)
    scene.meta["sha256"] = scene.digest()
    return scene


@dataclass
class Fovea:
    """Gaze pixel, ring start eccentricities (degrees) and blend band width."""

    gaze_x: float
    gaze_y: float
    rings_deg: tuple = (18.0, 27.0, 33.0)
    band_deg: float = 3.5

    def as_row(self) -> np.ndarray:
        return np.array([self.gaze_x, self.gaze_y, *self.rings_deg, self.band_deg],
                        np.float64)


@dataclass
class Workload:
    name: str
    scene: Scene
    cams: list
    foveae: list | None = None
    tile: int = 16
    extra: dict = field(default_factory=dict)


FR_FOV_DEG = 94.0
PLAIN_FOV_DEG = 60.0


def config1(seed: int = 1001) -> Workload:
    """4,096 uniform Gaussians, SH0, 128x128, camera at distance 4."""
    sc = make_scene(4096, 0, seed, clustered=False, log_scale_mu=-3.5, log_scale_sigma=0.5)
    cam = pinhole(128, 128, PLAIN_FOV_DEG, t=(0.0, 0.0, 4.0))
    return Workload("cfg1_plain_4k_128", sc, [cam])


def config2(seed: int = 1002, n: int = 500_000) -> Workload:
    """500k clustered Gaussians, SH3, 1280x720."""
    sc = make_scene(n, 3, seed, clustered=True, log_scale_mu=-4.5, log_scale_sigma=0.7)
    cam = pinhole(1280, 720, PLAIN_FOV_DEG, t=(0.0, 0.0, 4.0))
    return Workload("cfg2_plain_500k_720p", sc, [cam])


def _eyes(rng, width=1920, height=1080, ipd=0.06, dist=2.0):
    gx = rng.uniform(width * 0.25, width * 0.75)
    gy = rng.uniform(height * 0.25, height * 0.75)
    cams, fov = [], []
    for sx in (-1.0, 1.0):
        eye = np.array([sx * ipd / 2, 0.0, -dist])
        cams.append(pinhole(width, height, FR_FOV_DEG, t=-eye))
        fov.append(Fovea(gx, gy))
    return cams, fov


def config3(seed: int = 1003, n: int = 1_500_000, width=1920, height=1080) -> Workload:
    """1.5M clustered Gaussians, SH3, nested 100/40/15/5 % subsets with
    per-level opacity and DC; two eyes at 1920x1080 with a shared gaze."""
    sc = make_scene(n, 3, seed, clustered=True, log_scale_mu=-4.5, log_scale_sigma=0.7,
                    fr_levels=4)
    rng = np.random.default_rng(seed + 7919)  # 9. cameras and gaze
    cams, fov = _eyes(rng, width, height)
    return Workload("cfg3_foveated_stereo_1p5M_1080p", sc, cams, fov)


def config4(seed: int = 1004, n: int = 1_000_000) -> Workload:
    """1M clustered Gaussians, SH3, 1280x720; the L1 target comes from a
    perturbed copy (means + N(0, 0.01), logits + N(0, 0.3), seed + 1)."""
    sc = make_scene(n, 3, seed, clustered=True, log_scale_mu=-4.5, log_scale_sigma=0.7)
    cam = pinhole(1280, 720, PLAIN_FOV_DEG, t=(0.0, 0.0, 4.0))
    return Workload("cfg4_fwd_bwd_1M_720p", sc, [cam], extra=dict(target_scene=perturbed(sc, seed + 1)))


def perturbed(sc: Scene, seed: int) -> Scene:
    rng = np.random.default_rng(seed)
    out = sc.subset(np.arange(sc.n))
    out.means = (sc.means + rng.normal(0.0, 0.01, sc.means.shape)).astype(np.float32)
    out.opacity_logits = (sc.opacity_logits + rng.normal(0.0, 0.3, sc.n)).astype(np.float32)
    return out


def fd_subcase(seed: int = 1004) -> Workload:
    """256 Gaussians of a config-1-style draw with SH3, 32x32, FOV 60."""
    sc = make_scene(256, 3, seed, clustered=False, log_scale_mu=-2.5, log_scale_sigma=0.4)
    cam = pinhole(32, 32, PLAIN_FOV_DEG, t=(0.0, 0.0, 4.0))
    return Workload("fd_256_32x32", sc, [cam])


ORBIT_RES = ((640, 360), (960, 540), (1280, 720), (1920, 1080))


def config5(seed: int = 1005, n: int = 3_000_000, n_orbit: int = 32) -> Workload:
    """3M clustered Gaussians, SH3, FR subsets; 32 orbit views at mixed
    resolutions plus two foveated eyes."""
    sc = make_scene(n, 3, seed, clustered=True, log_scale_mu=-4.5, log_scale_sigma=0.7,
                    fr_levels=4)
    rng = np.random.default_rng(seed + 7919)
    cams = []
    for _ in range(n_orbit):
        az = rng.uniform(0.0, 2 * math.pi)
        el = math.radians(rng.uniform(-30.0, 30.0))
        w, h = ORBIT_RES[rng.integers(0, len(ORBIT_RES))]
        eye = 4.0 * np.array([math.cos(el) * math.sin(az), -math.sin(el), -math.cos(el) * math.cos(az)])
        cams.append(look_at(eye, (0.0, 0.0, 0.0), w, h, PLAIN_FOV_DEG))
    eyes, fov = _eyes(rng)
    return Workload("cfg5_batched_3M_32views_2eyes", sc, cams, extra=dict(eyes=eyes, eye_foveae=fov))


def small_scene(n: int, seed: int, sh_degree: int = 3, clustered: bool = True,
                fr_levels: int = 0, log_scale_mu: float = -3.0,
                log_scale_sigma: float = 0.6) -> Scene:
    """Scaled-down draw used by the parity tests."""
    return make_scene(n, sh_degree, seed, clustered=clustered, log_scale_mu=log_scale_mu,
                      log_scale_sigma=log_scale_sigma, fr_levels=fr_levels)
