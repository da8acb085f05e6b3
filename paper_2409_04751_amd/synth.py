"""Seeded synthetic scenes, cameras and poses.

This module only draws random inputs; it holds none of the rasterizer's
arithmetic.  Both the HIP path and the CPU oracle consume its arrays, so a
parity test feeds the two exactly the same numbers.

Parameter layout (structure of arrays, float32, C-contiguous):
  means   [3, N]   world positions
  scales  [3, N]   activated scales  (exp of the drawn log-scales)
  quats   [4, N]   unit quaternions (w, x, y, z)
  opacity [N]      activated opacity (sigmoid of the drawn logits)
  sh      [S, N]   spherical-harmonic coefficients, plane k*3 + c holds
                   basis function k for colour channel c; S = 3 (deg+1)^2

The draw order inside each generator is fixed and listed in its docstring, so
a scene is reproducible from (recipe, N, seed) alone.

The paper trains on ScanNet++ fisheye rooms at 1752x1168 (Sec. 5.1) and
reports scenes of 0.59-2.6 M Gaussians (Table 1).  Those scenes are not
available; the box scenes here stand in for them with the same image size and
Gaussian counts of the same order.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

TILE = 16


@dataclasses.dataclass(frozen=True)
class Camera:
    """Intrinsics of one view.  model: 0 equidistant fisheye (Sec. 3.2),
    1 pinhole, 2 panorama (Sec. 5.3), 3 equisolid-angle, 4 orthographic,
    5 stereographic fisheye."""

    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    model: int = 0
    near: float = 0.2
    theta_max: float = 0.95 * math.pi

    @property
    def tiles_x(self) -> int:
        return (self.width + TILE - 1) // TILE

    @property
    def tiles_y(self) -> int:
        return (self.height + TILE - 1) // TILE


@dataclasses.dataclass(frozen=True)
class Pose:
    """World-to-camera transform x_c = R x + t (R row-major 3x3)."""

    R: np.ndarray
    t: np.ndarray


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opacity: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    def subset(self, ids: np.ndarray) -> "Scene":
        ids = np.asarray(ids)
        return Scene(
            np.ascontiguousarray(self.means[:, ids]),
            np.ascontiguousarray(self.scales[:, ids]),
            np.ascontiguousarray(self.quats[:, ids]),
            np.ascontiguousarray(self.opacity[ids]),
            np.ascontiguousarray(self.sh[:, ids]),
            self.sh_degree,
        )


MODEL_EQUIDISTANT, MODEL_PINHOLE, MODEL_PANORAMA, MODEL_EQUISOLID, MODEL_ORTHOGRAPHIC, MODEL_STEREOGRAPHIC = range(6)
RADIAL_MODELS = (MODEL_EQUIDISTANT, MODEL_PINHOLE, MODEL_EQUISOLID, MODEL_ORTHOGRAPHIC, MODEL_STEREOGRAPHIC)

# r(theta) and its inverse for the radial models, and the largest theta_max
# the camera builder hands out for each (where r' or the splat degenerates)
_RADIAL = {
    MODEL_PINHOLE: (math.tan, math.atan, 0.45 * math.pi),
    MODEL_EQUISOLID: (lambda t: 2.0 * math.sin(t / 2.0), lambda r: 2.0 * math.asin(min(1.0, r / 2.0)), 0.95 * math.pi),
    MODEL_ORTHOGRAPHIC: (math.sin, lambda r: math.asin(min(1.0, r)), 0.45 * math.pi),
    MODEL_STEREOGRAPHIC: (lambda t: 2.0 * math.tan(t / 2.0), lambda r: 2.0 * math.atan(r / 2.0), 0.95 * math.pi),
}


def fisheye_camera(width: int, height: int, fov_deg: float, near: float = 0.2, model: int = MODEL_EQUIDISTANT) -> Camera:
    """Radial camera whose horizontal field of view spans the image width.

    Equidistant (the default): f = width / FOV (radians).  Other radial
    models: f r(FOV / 2) = width / 2.  Principal point at (width/2, height/2).
    theta_max (the rear-axis cull) = min(theta_corner + 0.25, cap), where
    theta_corner is the incidence angle of the image corner farthest from the
    principal point and cap is 0.95 pi (0.45 pi for the pinhole and
    orthographic models).  These are workload parameters handed unchanged to
    both implementations.
    """
    cx, cy = width / 2.0, height / 2.0
    corner = max(math.hypot(ax - cx, ay - cy) for ax in (0.0, float(width)) for ay in (0.0, float(height)))
    if model == MODEL_EQUIDISTANT:
        f = width / math.radians(fov_deg)
        theta_max = min(corner / f + 0.25, 0.95 * math.pi)
        return Camera(width, height, f, f, cx, cy, 0, near, theta_max)
    r, r_inv, cap = _RADIAL[model]
    f = (width / 2.0) / r(math.radians(fov_deg) / 2.0)
    theta_max = min(r_inv(corner / f) + 0.25, cap)
    return Camera(width, height, f, f, cx, cy, model, near, theta_max)


def panorama_camera(width: int, height: int, near: float = 0.2, lat_max: float = 0.45 * math.pi) -> Camera:
    """Equirectangular panorama (Sec. 5.3): longitude over the full width,
    latitude over the full height: f_x = width / (2 pi), f_y = height / pi,
    c = (width/2, height/2).  Gaussians above |latitude| lat_max are culled
    (theta_max carries it)."""
    return Camera(width, height, width / (2.0 * math.pi), height / math.pi, width / 2.0, height / 2.0,
                  MODEL_PANORAMA, near, lat_max)


def identity_pose(position=(0.0, 0.0, 0.0)) -> Pose:
    p = np.asarray(position, dtype=np.float64)
    return Pose(np.eye(3, dtype=np.float32), (-p).astype(np.float32))


def _haar_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation: QR of a Gaussian matrix with the sign fix."""
    a = rng.normal(size=(3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def random_poses(count: int, seed: int, lo, hi) -> list[Pose]:
    """Draw order: per pose, a position uniform in [lo, hi]^3 (3 draws), then
    a 3x3 Gaussian matrix for the rotation."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    poses = []
    for _ in range(count):
        pos = lo + (hi - lo) * rng.random(3)
        Rm = _haar_rotation(rng)
        R32 = Rm.astype(np.float32)
        t = -(R32.astype(np.float64) @ pos)
        poses.append(Pose(R32, t.astype(np.float32)))
    return poses


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _finish(means, log_scales, quats, logits, sh, degree) -> Scene:
    q = quats / np.linalg.norm(quats, axis=0, keepdims=True)
    return Scene(
        np.ascontiguousarray(means, dtype=np.float32),
        np.ascontiguousarray(np.exp(log_scales), dtype=np.float32),
        np.ascontiguousarray(q, dtype=np.float32),
        np.ascontiguousarray(_sigmoid(logits), dtype=np.float32),
        np.ascontiguousarray(sh, dtype=np.float32),
        degree,
    )


def shell_scene(n: int = 1000, seed: int = 0) -> Scene:
    """Small fisheye test scene in front of a camera at the origin.

    Draw order: directions as 3 normals per Gaussian ([3, N]) with z folded
    to be positive, radius as U(1, 125)^(1/3), log-scales N(-3, 0.5) [3, N],
    quaternions N(0, 1) [4, N] normalised, opacity logits N(0, 1) [N],
    degree-0 SH (DC) U(0, 1) [3, N].
    """
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(3, n))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    d[2] = np.abs(d[2])
    r = rng.uniform(1.0, 125.0, size=n) ** (1.0 / 3.0)
    means = d * r
    log_scales = rng.normal(-3.0, 0.5, size=(3, n))
    quats = rng.normal(size=(4, n))
    logits = rng.normal(size=n)
    sh = rng.random(size=(3, n))
    return _finish(means, log_scales, quats, logits, sh, 0)


ROOM_LO = (-5.0, -2.0, -5.0)
ROOM_HI = (5.0, 2.0, 5.0)


def room_scene(n: int, seed: int = 0, large_frac: float = 0.0, sh_degree: int = 3) -> Scene:
    """Room-shaped scene: means uniform in a 10 x 4 x 10 m box (y is height).

    Draw order: means U(0,1) [3, N] mapped to the box, log-scales
    N(-4, 0.7) [3, N], a U(0,1) [N] draw that marks `large_frac` of the
    Gaussians as large, N(-1, 0.5) [3, n_large] log-scales for those,
    quaternions N(0,1) [4, N] normalised, opacity logits N(0,1) [N],
    DC coefficients U(0,1) [3, N], higher-order coefficients N(0, 0.2)
    [S-3, N].
    """
    rng = np.random.default_rng(seed)
    lo = np.asarray(ROOM_LO)[:, None]
    hi = np.asarray(ROOM_HI)[:, None]
    means = lo + (hi - lo) * rng.random(size=(3, n))
    log_scales = rng.normal(-4.0, 0.7, size=(3, n)).astype(np.float32)
    big = rng.random(size=n) < large_frac
    nb = int(big.sum())
    if nb:
        log_scales[:, big] = rng.normal(-1.0, 0.5, size=(3, nb))
    quats = rng.normal(size=(4, n)).astype(np.float32)
    logits = rng.normal(size=n)
    S = 3 * (sh_degree + 1) ** 2
    sh = np.empty((S, n), dtype=np.float32)
    sh[:3] = rng.random(size=(3, n))
    if S > 3:
        sh[3:] = rng.normal(0.0, 0.2, size=(S - 3, n))
    return _finish(means, log_scales, quats, logits, sh, sh_degree)


def target_image(width: int, height: int, seed: int = 1) -> np.ndarray:
    """Random L1 target, U(0,1) [3, H, W]."""
    rng = np.random.default_rng(seed)
    return rng.random(size=(3, height, width)).astype(np.float32)


# Named workloads ----------------------------------------------------------

def workload(name: str):
    """Return (scene_fn, camera, poses) for a named workload.

    shell1k      1,000 Gaussians, 256x256 fisheye at 180 deg, forward only
    room500k     500k Gaussians SH3, 1752x1168 at 180 deg, camera at centre
    room3m       3M Gaussians SH3 (1% large), 1752x1168 at 180 deg
    room3m_2k    3M Gaussians SH3 (1% large), 2048x2048 at 200 deg, 4 poses
    """
    if name == "shell1k":
        return (lambda: shell_scene(1000, 0)), fisheye_camera(256, 256, 180.0), [identity_pose()]
    if name == "room500k":
        return (lambda: room_scene(500_000, 0, 0.0, 3)), fisheye_camera(1752, 1168, 180.0), [identity_pose()]
    if name == "room3m":
        return (lambda: room_scene(3_000_000, 0, 0.01, 3)), fisheye_camera(1752, 1168, 180.0), [identity_pose()]
    if name == "room3m_2k":
        lo = [a + 1.0 for a in ROOM_LO]
        hi = [a - 1.0 for a in ROOM_HI]
        return (lambda: room_scene(3_000_000, 0, 0.01, 3)), fisheye_camera(2048, 2048, 200.0), random_poses(4, 2, lo, hi)
    raise KeyError(name)
