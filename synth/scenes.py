"""Seeded generators for Gaussian scenes, cameras, foveae and renderer knobs.

Conventions (fixed here, used identically by the oracle and the GPU path):

* Gaussians are stored structure-of-arrays in float32: ``means[3][N]``,
  ``log_scales[3][N]`` (natural log of the per-axis standard deviation),
  ``quats[4][N]`` as (w, x, y, z), not necessarily unit length,
  ``opacity_logits[N]`` and ``sh[K][3][N]`` with ``K = (degree+1)^2``.
* Cameras follow the usual computer-vision axes: x right, y down, z forward.
  ``world_to_cam`` is the row-major 3x4 matrix [R | t] with x_cam = R x + t.
  ``fov_x_deg`` is the horizontal field of view; pixels are square, so the
  focal length in pixels is (width/2) / tan(fov_x/2) on both axes.
* The world is y-down as well: a ground slab sits at y ~ +1 below a head at
  y = 0.

Only random draws and array layout live here (see the package docstring).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

F32 = np.float32


def _f32(x):
    return np.asarray(x, dtype=np.float32)


@dataclasses.dataclass
class Params:
    """Renderer knobs.  ``tile`` is 16 (plain) or 32 (foveated, split into 16^2
    subtiles near the fovea); ``window`` is the per-sample resort window length;
    ``blend_batch`` is the number of list entries staged per wave and batch
    and ``schedule`` selects the blend launch (0 one block per work item,
    1 persistent waves); both are performance knobs that never change the
    output.  ``depth`` is the key depth of the sort: 0 the per-tile depth at
    the splat's maximum point (the method), 1 view-space z, 2 distance to the
    eye (the global-sort orders of the comparison systems); ``window`` 0
    blends in key order without per-sample resorting."""
    tile: int = 16
    window: int = 16
    depth: int = 0
    blend_batch: int = 64
    schedule: int = 0
    z_near: float = float(F32(0.2))
    alpha_min: float = float(F32(1.0 / 255.0))
    alpha_max: float = float(F32(0.99))
    t_min: float = float(F32(1e-4))
    dilation: float = float(F32(0.3))
    background: Tuple[float, float, float] = (0.0, 0.0, 0.0)

    def replace(self, **kw) -> "Params":
        p = dataclasses.replace(self, **kw)
        for k in ("z_near", "alpha_min", "alpha_max", "t_min", "dilation"):
            setattr(p, k, float(F32(getattr(p, k))))
        p.background = tuple(float(F32(b)) for b in p.background)
        return p


def default_params(**kw) -> Params:
    return Params().replace(**kw)


@dataclasses.dataclass
class Camera:
    world_to_cam: np.ndarray  # (3, 4) float32
    fov_x_deg: float
    cx: float
    cy: float
    width: int
    height: int


@dataclasses.dataclass
class Fovea:
    """Full-resolution centre region.  shape 0: a disc of radius_deg (angle
    around the ray through center_px); shape 1: a rectangle of half-extents
    half_px (pixels) around center_px.  band_frac: the blending band's width
    as a fraction of the radius or half-extent."""
    enabled: bool
    center_px: Tuple[float, float] = (0.0, 0.0)
    radius_deg: float = 15.0
    band_frac: float = 0.10
    shape: int = 0
    half_px: Tuple[float, float] = (0.0, 0.0)


@dataclasses.dataclass
class Scene:
    means: np.ndarray           # (3, N) float32
    log_scales: np.ndarray      # (3, N)
    quats: np.ndarray           # (4, N)  (w, x, y, z)
    opacity_logits: np.ndarray  # (N,)
    sh: np.ndarray              # (K, 3, N)
    sh_degree: int = 3

    @property
    def n(self) -> int:
        return int(self.means.shape[1])


def _camera(R: np.ndarray, eye: np.ndarray, fov_x_deg: float, width: int,
            height: int, cx: Optional[float] = None,
            cy: Optional[float] = None) -> Camera:
    t = -R @ eye
    m = np.concatenate([R, t[:, None]], axis=1)
    return Camera(world_to_cam=_f32(m), fov_x_deg=float(F32(fov_x_deg)),
                  cx=float(F32(width / 2.0 if cx is None else cx)),
                  cy=float(F32(height / 2.0 if cy is None else cy)),
                  width=int(width), height=int(height))


def camera_translate(eye, fov_x_deg, width, height, cx=None, cy=None) -> Camera:
    """Camera at ``eye`` with identity orientation (looking along +z)."""
    return _camera(np.eye(3), np.asarray(eye, np.float64), fov_x_deg, width,
                   height, cx, cy)


def camera_lookat(eye, target, fov_x_deg, width, height, yaw_deg=0.0) -> Camera:
    """Camera at ``eye`` looking at ``target``; world up is -y (y-down world)."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    up = np.array([0.0, -1.0, 0.0])
    right = np.cross(fwd, up)
    if np.linalg.norm(right) < 1e-9:
        right = np.array([1.0, 0.0, 0.0])
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    return _camera(R, eye, fov_x_deg, width, height)


def stereo_head(head=(0.0, 0.0, -3.0), baseline=0.064, yaw_deg=0.0,
                fov_x_deg=110.0, width=2064, height=2208) -> List[Camera]:
    """Two parallel-axis eyes at +-baseline/2 along the head's x axis.  The
    head yaws about the world vertical (y) axis through its own centre."""
    a = math.radians(yaw_deg)
    # Rotation of the head frame about world y; columns are head axes in world.
    Ry = np.array([[math.cos(a), 0.0, math.sin(a)],
                   [0.0, 1.0, 0.0],
                   [-math.sin(a), 0.0, math.cos(a)]])
    R = Ry.T  # world -> head/camera
    head = np.asarray(head, np.float64)
    cams = []
    for sx in (-0.5, 0.5):
        eye = head + Ry @ np.array([sx * baseline, 0.0, 0.0])
        cams.append(_camera(R, eye, fov_x_deg, width, height))
    return cams


def ring_cameras(rng: np.random.Generator, n: int, radius: float,
                 sizes: List[Tuple[int, int]], fov_range=(60.0, 120.0),
                 fixed_fov: Optional[float] = None) -> List[Camera]:
    """Eyes on a horizontal ring around the origin at seeded angles, each
    looking at the origin, with a seeded height jitter."""
    cams = []
    for i in range(n):
        ang = rng.uniform(0.0, 2.0 * math.pi)
        h = rng.uniform(-0.6, 0.3)
        eye = np.array([radius * math.sin(ang), h, -radius * math.cos(ang)])
        fov = fixed_fov if fixed_fov is not None else rng.uniform(*fov_range)
        w, hgt = sizes[i % len(sizes)]
        cams.append(camera_lookat(eye, (0.0, 0.0, 0.0), fov, w, hgt))
    return cams


def fovea_off() -> Fovea:
    return Fovea(enabled=False)


def fovea_at_center(cam: Camera, radius_deg=15.0, band_frac=0.10) -> Fovea:
    return Fovea(enabled=True, center_px=(cam.cx, cam.cy),
                 radius_deg=float(F32(radius_deg)),
                 band_frac=float(F32(band_frac)))


def fovea_rect(cam: Camera, frac=0.5, band_frac=0.10) -> Fovea:
    """The paper's layout (Sec. 5): a centre region of ``frac`` of the image
    size in each dimension around the principal point, with a band of
    band_frac of it."""
    return Fovea(enabled=True, center_px=(cam.cx, cam.cy), radius_deg=0.0,
                 band_frac=float(F32(band_frac)), shape=1,
                 half_px=(float(F32(frac * cam.width / 2.0)), float(F32(frac * cam.height / 2.0))))


# Semi-axes of the synthetic lens mask as fractions of the half image size:
# chosen so that 508 of the 4615 32x32 tiles of a 2064x2272 eye are
# invisible, next to the 507 the paper reports for its headset (Sec. 5.4;
# the symmetric ellipse moves the count in steps of four).
LENS_AXES = (1.087, 1.087)


def lens_mask(width: int, height: int, axes=LENS_AXES) -> np.ndarray:
    """Synthetic head-mounted-display visibility mask (uint8 [height][width],
    1 = visible): the pixels whose centres lie inside an ellipse around the
    image centre with semi-axes axes * (width/2, height/2).  A stand-in for
    the mask a headset runtime provides."""
    ys, xs = np.mgrid[0:height, 0:width]
    u = (xs + 0.5 - width / 2.0) / (axes[0] * width / 2.0)
    v = (ys + 0.5 - height / 2.0) / (axes[1] * height / 2.0)
    return (u * u + v * v <= 1.0).astype(np.uint8)


def _random_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _sh(rng, n, degree, std=0.3):
    k = (degree + 1) ** 2
    return rng.normal(0.0, std, size=(k, 3, n))


def uniform_scene(seed: int, n: int, lo=-1.0, hi=1.0, log_scale=(-4.0, 0.5),
                  opacity=(0.0, 1.0), sh_degree=3, sh_std=0.3) -> Scene:
    """Means uniform in a cube, log-scales N(m, s) per axis, opacity logits
    N(m, s), random rotations, SH coefficients N(0, sh_std)."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(lo, hi, size=(3, n))
    ls = rng.normal(log_scale[0], log_scale[1], size=(3, n))
    q = _random_quats(rng, n)
    o = rng.normal(opacity[0], opacity[1], size=n)
    sh = _sh(rng, n, sh_degree, sh_std)
    return Scene(_f32(means), _f32(ls), _f32(q), _f32(o), _f32(sh), sh_degree)


def _random_rotation(rng):
    # Haar-random orthogonal matrix via QR of a Gaussian matrix, det fixed to +1.
    a = rng.standard_normal((3, 3))
    qm, r = np.linalg.qr(a)
    qm = qm * np.sign(np.diag(r))[None, :]
    if np.linalg.det(qm) < 0:
        qm[:, 0] = -qm[:, 0]
    return qm


def cluster_scene(seed: int, n: int, log_scale=(-5.0, 0.7), opacity=(0.0, 1.0),
                  n_clusters=64, cluster_frac=0.85, sh_degree=3,
                  sh_std=0.3) -> Scene:
    """Mixture of anisotropic Gaussian clusters plus a ground slab.

    Cluster centres are uniform in [-1.5,1.5]x[-1,0.8]x[-1.5,1.5], per-axis
    standard deviations uniform in [0.05, 0.35] under a random rotation, equal
    weights.  The slab is uniform in x, z in [-4, 4] and y in [0.95, 1.05]."""
    rng = np.random.default_rng(seed)
    n_cl = int(round(n * cluster_frac))
    n_slab = n - n_cl
    centres = np.stack([rng.uniform(-1.5, 1.5, n_clusters),
                        rng.uniform(-1.0, 0.8, n_clusters),
                        rng.uniform(-1.5, 1.5, n_clusters)], axis=1)
    stds = rng.uniform(0.05, 0.35, size=(n_clusters, 3))
    rots = np.stack([_random_rotation(rng) for _ in range(n_clusters)])
    which = rng.integers(0, n_clusters, size=n_cl)
    local = rng.standard_normal((n_cl, 3)) * stds[which]
    pts = centres[which] + np.einsum("nij,nj->ni", rots[which], local)
    slab = np.stack([rng.uniform(-4.0, 4.0, n_slab),
                     rng.uniform(0.95, 1.05, n_slab),
                     rng.uniform(-4.0, 4.0, n_slab)], axis=1)
    means = np.concatenate([pts, slab], axis=0).T
    ls = rng.normal(log_scale[0], log_scale[1], size=(3, n))
    q = _random_quats(rng, n)
    o = rng.normal(opacity[0], opacity[1], size=n)
    sh = _sh(rng, n, sh_degree, sh_std)
    return Scene(_f32(means), _f32(ls), _f32(q), _f32(o), _f32(sh), sh_degree)


def make_scene(kind: str, seed: int, n: int, **kw) -> Scene:
    if kind == "uniform":
        return uniform_scene(seed, n, **kw)
    if kind == "cluster":
        return cluster_scene(seed, n, **kw)
    raise ValueError(kind)


def subset_scene(s: Scene, idx) -> Scene:
    idx = np.asarray(idx)
    return Scene(s.means[:, idx].copy(), s.log_scales[:, idx].copy(),
                 s.quats[:, idx].copy(), s.opacity_logits[idx].copy(),
                 s.sh[:, :, idx].copy(), s.sh_degree)


def permute_scene(s: Scene, seed: int) -> Tuple[Scene, np.ndarray]:
    perm = np.random.default_rng(seed).permutation(s.n)
    return subset_scene(s, perm), perm


# ---------------------------------------------------------------------------
# Workload configurations.  Sizes are parameters so that tests can shrink them
# while keeping the same distributions.
# ---------------------------------------------------------------------------

def config_tiny(seed=0, n=10_000, size=256, window=16):
    """10k Gaussians in [-1,1]^3, one 256x256 90-degree view from (0,0,-3),
    plain 16x16 tiles."""
    scene = uniform_scene(seed, n, log_scale=(-4.0, 0.5))
    cam = camera_translate((0.0, 0.0, -3.0), 90.0, size, size)
    return scene, [cam], fovea_off(), default_params(tile=16, window=window)


def config_stereo(seed=0, n=500_000, width=2064, height=2208, radius_deg=15.0,
                  window=16, fov_x_deg=110.0):
    """500k-Gaussian cluster+slab scene, two eyes (64 mm baseline) at
    2064x2208, 110-degree horizontal FoV, 15-degree fovea at the principal
    point, 32x32 tiles split to 16x16 near the fovea."""
    scene = cluster_scene(seed, n, log_scale=(-5.0, 0.7))
    cams = stereo_head(fov_x_deg=fov_x_deg, width=width, height=height)
    foveas = [fovea_at_center(c, radius_deg) for c in cams]
    return scene, cams, foveas, default_params(tile=32, window=window)


def config_unpruned(seed=0, n=3_000_000, frame=0, n_frames=30, width=2064,
                    height=2208, window=16):
    """3M Gaussians, smaller and fainter, stereo cameras yawing over a +-20
    degree arc (frame k of n_frames)."""
    scene = cluster_scene(seed, n, log_scale=(-5.5, 0.8), opacity=(-1.0, 1.5))
    yaw = -20.0 + 40.0 * frame / max(1, n_frames - 1)
    cams = stereo_head(yaw_deg=yaw, width=width, height=height)
    foveas = [fovea_at_center(c) for c in cams]
    return scene, cams, foveas, default_params(tile=32, window=window)


def config_batch(seed=0, n=1_000_000, sizes=None):
    """1M cluster Gaussians, 16 ring views of mixed resolution and FoV, a
    random half foveated around a centre drawn from the middle of the image."""
    scene = cluster_scene(seed, n, log_scale=(-5.0, 0.7))
    rng = np.random.default_rng(seed + 1000)
    sizes = sizes or [(512, 512), (1024, 1024), (1920, 1080), (2064, 2208)]
    order = [sizes[i // 4 % len(sizes)] for i in range(16)]
    cams = ring_cameras(rng, 16, 3.0, order)
    fov_idx = set(rng.permutation(16)[:8].tolist())
    foveas = []
    for i, c in enumerate(cams):
        if i in fov_idx:
            cxp = rng.uniform(0.25, 0.75) * c.width
            cyp = rng.uniform(0.25, 0.75) * c.height
            foveas.append(Fovea(True, (float(F32(cxp)), float(F32(cyp))),
                                float(F32(15.0)), float(F32(0.10))))
        else:
            foveas.append(fovea_off())
    return scene, cams, foveas, default_params(tile=32, window=16)


def config_diff(seed=0, n=1_000_000, size=1024, n_views=4):
    """1M cluster Gaussians, 4 ring views at 1024^2 and 90-degree FoV, plain
    16x16 tiles, plus a perturbed copy used to render targets."""
    scene = cluster_scene(seed, n, log_scale=(-5.0, 0.7))
    rng = np.random.default_rng(seed + 2000)
    cams = ring_cameras(rng, n_views, 3.0, [(size, size)], fixed_fov=90.0)
    pert = Scene(_f32(scene.means + rng.normal(0, 0.01, scene.means.shape)),
                 scene.log_scales.copy(), scene.quats.copy(),
                 _f32(scene.opacity_logits
                      + rng.normal(0, 0.2, scene.opacity_logits.shape)),
                 scene.sh.copy(), scene.sh_degree)
    return scene, pert, cams, default_params(tile=16, window=16)
