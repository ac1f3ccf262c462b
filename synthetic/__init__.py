"""Seeded synthetic inputs for 3D Gaussian Splatting training steps.

This module draws scenes (Gaussian parameters), cameras and target images'
source scenes from fixed seeds.  It holds no part of the method's arithmetic:
no projection, compositing, gradient or optimiser step.  Both the CPU oracle
and the GPU path take their inputs from here.

Scene parameterisation (3DGS, paper Sec. 2): per Gaussian a mean (3), per-axis
log-scales (3), a rotation quaternion stored (w, x, y, z) (4), an opacity logit
(1) and degree-3 spherical-harmonic colour coefficients (16 x 3, coefficient
index major, channel minor).  All arrays are float32, array-of-structures:

    means [N,3], log_scales [N,3], quats [N,4], opacity_logits [N], sh [N,16,3]

Cameras use the OpenCV convention (x right, y down, z forward).  A view is one
128-byte record (``VIEW_DTYPE``): world-to-camera rotation R (row-major) and
translation t, the camera centre, pinhole intrinsics, the clamp bounds
1.3 * tan(half-fov) used by the EWA Jacobian, near/far planes, background
colour and the image size.  Camera values are computed in float64 and rounded
once to float32, so both implementations read identical numbers.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

VIEW_DTYPE = np.dtype([
    ("R", "<f4", (9,)),
    ("t", "<f4", (3,)),
    ("campos", "<f4", (3,)),
    ("fx", "<f4"), ("fy", "<f4"), ("cx", "<f4"), ("cy", "<f4"),
    ("lim_x", "<f4"), ("lim_y", "<f4"),
    ("znear", "<f4"), ("zfar", "<f4"),
    ("bg", "<f4", (3,)),
    ("width", "<i4"), ("height", "<i4"),
    ("pad", "<i4", (4,)),
])
assert VIEW_DTYPE.itemsize == 128

N_PARAMS = 59          # floats per Gaussian: 3 + 3 + 4 + 1 + 48
SH_COEFFS = 16         # degree 3


@dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def arrays(self):
        return self.means, self.log_scales, self.quats, self.opacity_logits, self.sh

    def copy(self) -> "Scene":
        return Scene(*(a.copy() for a in self.arrays()))

    def flat(self) -> np.ndarray:
        """[N, 59] float32 in the canonical parameter order
        (means, log-scales, quaternion, opacity logit, SH m*3+k)."""
        n = self.n
        return np.concatenate([self.means, self.log_scales, self.quats,
                               self.opacity_logits[:, None],
                               self.sh.reshape(n, 48)], axis=1).astype(np.float32)

    @staticmethod
    def from_flat(flat: np.ndarray) -> "Scene":
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        n = flat.shape[0]
        return Scene(flat[:, 0:3].copy(), flat[:, 3:6].copy(), flat[:, 6:10].copy(),
                     flat[:, 10].copy(), flat[:, 11:59].reshape(n, 16, 3).copy())


def _finish(means, log_scales, q, logits, dc, rest) -> Scene:
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    n = means.shape[0]
    sh = np.concatenate([dc[:, None, :], rest.reshape(n, 15, 3)], axis=1)
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(f(means), f(log_scales), f(q), f(logits), f(sh))


def scene_uniform_cube(n: int, seed: int, log_scale_mean=-3.0, log_scale_std=0.5,
                       logit_mean=0.0, logit_std=1.0, half_extent=1.0) -> Scene:
    """Means uniform in [-e, e]^3 (the 2k-Gaussian plain-method workload)."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-half_extent, half_extent, size=(n, 3))
    ls = rng.normal(log_scale_mean, log_scale_std, size=(n, 3))
    q = rng.normal(0.0, 1.0, size=(n, 4))
    logits = rng.normal(logit_mean, logit_std, size=n)
    dc = rng.normal(0.0, 0.5, size=(n, 3))
    rest = rng.normal(0.0, 0.2, size=(n, 45))
    return _finish(means, ls, q, logits, dc, rest)


def scene_normal(n: int, seed: int, log_scale_mean=-4.0, log_scale_std=0.7,
                 logit_mean=0.0, logit_std=1.0) -> Scene:
    """Means ~ N(0,1)^3, isotropic log-scale spread (the 300k/3M/6M workloads)."""
    rng = np.random.default_rng(seed)
    means = rng.normal(0.0, 1.0, size=(n, 3))
    ls = rng.normal(log_scale_mean, log_scale_std, size=(n, 3))
    q = rng.normal(0.0, 1.0, size=(n, 4))
    logits = rng.normal(logit_mean, logit_std, size=n)
    dc = rng.normal(0.0, 0.5, size=(n, 3))
    rest = rng.normal(0.0, 0.2, size=(n, 45))
    return _finish(means, ls, q, logits, dc, rest)


def scene_anisotropic(n: int, seed: int) -> Scene:
    """Anisotropic scales (per-Gaussian N(-4.5,0.5) plus per-axis N(0,1)) and a
    long-tailed opacity (logit ~ N(-1,1.5)): the differentiation-check workload."""
    rng = np.random.default_rng(seed)
    means = rng.normal(0.0, 1.0, size=(n, 3))
    base = rng.normal(-4.5, 0.5, size=(n, 1))
    spread = rng.normal(0.0, 1.0, size=(n, 3))
    q = rng.normal(0.0, 1.0, size=(n, 4))
    logits = rng.normal(-1.0, 1.5, size=n)
    dc = rng.normal(0.0, 0.5, size=(n, 3))
    rest = rng.normal(0.0, 0.2, size=(n, 45))
    return _finish(means, base + spread, q, logits, dc, rest)


# ----------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------

def look_at(campos, target=(0.0, 0.0, 0.0)):
    """World-to-camera (R, t) for an OpenCV camera at ``campos`` looking at
    ``target`` with world up +y (float64)."""
    c = np.asarray(campos, dtype=np.float64)
    z = np.asarray(target, dtype=np.float64) - c
    z /= np.linalg.norm(z)
    x = np.cross(z, np.array([0.0, 1.0, 0.0]))
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    t = -R @ c
    return R, t


def make_view(width: int, height: int, campos, target=(0.0, 0.0, 0.0),
              fov_x_deg: float = 60.0, znear: float = 0.01, zfar: float = 1000.0,
              bg=(0.0, 0.0, 0.0)) -> np.ndarray:
    """One view record: pinhole camera, horizontal field of view, fy = fx,
    principal point at the image centre."""
    R, t = look_at(campos, target)
    tan_x = math.tan(math.radians(fov_x_deg) * 0.5)
    fx = (width * 0.5) / tan_x
    fy = fx
    tan_y = (height * 0.5) / fy
    v = np.zeros((), dtype=VIEW_DTYPE)
    v["R"] = R.reshape(9)
    v["t"] = t
    v["campos"] = np.asarray(campos, dtype=np.float64)
    v["fx"], v["fy"] = fx, fy
    v["cx"], v["cy"] = width * 0.5, height * 0.5
    v["lim_x"], v["lim_y"] = 1.3 * tan_x, 1.3 * tan_y
    v["znear"], v["zfar"] = znear, zfar
    v["bg"] = bg
    v["width"], v["height"] = width, height
    return v


def views_array(views) -> np.ndarray:
    out = np.zeros(len(views), dtype=VIEW_DTYPE)
    for i, v in enumerate(views):
        out[i] = v
    return out


def fibonacci_sphere(n: int, radius: float):
    """n camera centres on a sphere: y_i = 1 - 2(i+0.5)/n, azimuth i*pi*(3-sqrt 5)."""
    pts = []
    for i in range(n):
        y = 1.0 - 2.0 * (i + 0.5) / n
        r = math.sqrt(max(0.0, 1.0 - y * y))
        phi = i * math.pi * (3.0 - math.sqrt(5.0))
        pts.append((radius * r * math.cos(phi), radius * y, radius * r * math.sin(phi)))
    return pts


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    scene: Scene
    target_scene: Scene
    views: np.ndarray                 # VIEW_DTYPE[n_cameras]
    tile: int = 16
    lr: float = 1e-3
    steps: int = 1
    view_order: np.ndarray = field(default_factory=lambda: np.zeros(1, np.int64))
    extra: dict = field(default_factory=dict)


def workload_plain_small(n: int = 2000, width: int = 256, height: int = 256,
                         tile: int = 16, seed_base: int = 1000) -> Workload:
    """2k Gaussians uniform in [-1,1]^3, one 256x256 view from (0,0,-4)."""
    scene = scene_uniform_cube(n, seed_base)
    target = scene_uniform_cube(n, seed_base + 1)
    views = views_array([make_view(width, height, (0.0, 0.0, -4.0))])
    return Workload("plain-2k-256x256", scene, target, views, tile=tile, lr=1e-3,
                    steps=1, view_order=np.zeros(1, np.int64))


def workload_plain_300k(n: int = 300_000, width: int = 1280, height: int = 720,
                        n_cameras: int = 50, steps: int = 100, seed_base: int = 2000,
                        log_scale_mean: float = -4.0, log_scale_std: float = 0.7) -> Workload:
    """300k Gaussians ~N(0,1)^3, log-scales N(-4,0.7), 50 cameras on a radius-5
    sphere, 1280x720, one view per step.  Other log-scale distributions give
    the sparse-footprint form (N(-6, 0.3): footprints of about one pixel)."""
    scene = scene_normal(n, seed_base, log_scale_mean, log_scale_std)
    target = scene_normal(n, seed_base + 1, log_scale_mean, log_scale_std)
    cams = fibonacci_sphere(n_cameras, 5.0)
    views = views_array([make_view(width, height, c) for c in cams])
    order = np.random.default_rng(seed_base + 2).permutation(n_cameras)
    sparse = "" if (log_scale_mean, log_scale_std) == (-4.0, 0.7) else f"-ls{log_scale_mean:g}"
    return Workload(f"plain-{n // 1000}k-{width}x{height}{sparse}", scene, target, views, tile=16,
                    lr=1e-3, steps=steps, view_order=order)


def workload_diffcheck(n: int = 1_000_000, width: int = 1600, height: int = 1060,
                       seed_base: int = 3000) -> Workload:
    """1M anisotropic Gaussians, long-tailed opacity, one 1600x1060 view."""
    scene = scene_anisotropic(n, seed_base)
    target = scene_anisotropic(n, seed_base + 1)
    cams = fibonacci_sphere(50, 5.0)
    views = views_array([make_view(width, height, cams[0])])
    return Workload(f"diffcheck-{n // 1000}k-{width}x{height}", scene, target, views,
                    tile=16, steps=1, view_order=np.zeros(1, np.int64),
                    extra={"crop": (544, 272, 512, 512)})


BATCH_RESOLUTIONS = [(640, 480), (800, 600), (1024, 768), (1280, 720), (1280, 720),
                     (1600, 900), (1920, 1080), (1920, 1080)]


def workload_batched(n: int = 3_000_000, resolutions=None, steps: int = 200,
                     seed_base: int = 4000) -> Workload:
    """300k-workload distributions at 3M Gaussians; 8 views of uneven
    resolution per step; slot k of step i holds camera (8i + k) mod 50 at the
    slot's resolution (`batched_views`)."""
    res = resolutions or BATCH_RESOLUTIONS
    scene = scene_normal(n, seed_base)
    target = scene_normal(n, seed_base + 1)
    cams = fibonacci_sphere(50, 5.0)
    return Workload(f"batched-{n // 1000}k-{len(res)}views", scene, target,
                    views_array([make_view(w, h, cams[k]) for k, (w, h) in enumerate(res)]),
                    tile=16, steps=steps, extra={"resolutions": res, "cameras": cams})


def batched_views(cams, resolutions, step: int) -> np.ndarray:
    """Views of one step: camera (k*step + s) mod len(cams) in slot s."""
    k = len(resolutions)
    return views_array([make_view(w, h, cams[(k * step + s) % len(cams)])
                        for s, (w, h) in enumerate(resolutions)])


def workload_learned(n: int = 6_000_000, n_views: int = 4, width: int = 1920,
                     height: int = 1080, seed_base: int = 5000) -> Workload:
    """300k-workload distributions at 6M Gaussians, 4 x 1080p views per launch."""
    scene = scene_normal(n, seed_base)
    target = scene_normal(n, seed_base + 1)
    cams = fibonacci_sphere(50, 5.0)
    return Workload(f"learned-{n // 1000}k-{n_views}x{width}x{height}", scene, target,
                    views_array([make_view(width, height, c) for c in cams[:n_views]]), tile=16,
                    extra={"views_per_launch": n_views, "cameras": cams,
                           "resolutions": [(width, height)] * n_views})


def random_image(height: int, width: int, seed: int) -> np.ndarray:
    """A seeded target image in [0,1], [H,W,3] float32."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(height, width, 3)).astype(np.float32)
