"""Seeded synthetic inputs for the splatting hot path.

This module only draws inputs: Gaussian parameters, cameras and targets.  It
holds none of the rasteriser's arithmetic (no projection, compositing or loss),
so that the HIP path and the CPU oracle can both be fed from it without
sharing any computation.

The scenes stand in for the paper's LiDAR-visual-inertial sequences (Section
IV-A), which are not available: Gaussians are initialised from a synthetic
colourised LiDAR scan as the mapping thread does (Section III-E: centres from
LiDAR points, scale from nearest-neighbour spacing, inverse-sigmoid opacity,
SH DC coefficient from the point colour), images are 640x512 to 1280x1024
(Section IV-A), and each keyframe is rendered as a 3-level image pyramid
(Section III-D).  Seeds are ``numpy.random.default_rng(1000 * cfg + stream)``.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# Constant term of the degree-0 real spherical harmonic, 1 / (2 sqrt(pi)); used
# only to turn a drawn RGB colour into the DC coefficient that reproduces it.
_SH_DC = 0.28209479177387814


@dataclasses.dataclass
class Camera:
    """Pinhole camera.  World->camera: t = R @ mu + T (x right, y down, z forward).

    Pixel (u, v) has its centre at (u + 0.5, v + 0.5).
    """

    R: np.ndarray  # (3, 3) float64
    T: np.ndarray  # (3,) float64
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    weight: float = 1.0  # loss weight w_v of this view

    @property
    def campos(self) -> np.ndarray:
        """Camera centre in world coordinates, -R^T T."""
        return -self.R.T @ self.T

    def scaled(self, level: int) -> "Camera":
        """The same pose at pyramid level `level` (intrinsics and size divided by 2**level)."""
        s = 2 ** level
        return Camera(self.R.copy(), self.T.copy(), self.fx / s, self.fy / s, self.cx / s, self.cy / s,
                      self.width // s, self.height // s, self.weight)

    def cropped(self, x0: int, y0: int, w: int, h: int) -> "Camera":
        """A w x h window of this view whose top-left pixel is (x0, y0)."""
        return Camera(self.R.copy(), self.T.copy(), self.fx, self.fy, self.cx - x0, self.cy - y0, w, h,
                      self.weight)


@dataclasses.dataclass
class Scene:
    """Gaussian parameters (float32, torch-natural shapes) plus views and targets."""

    means: np.ndarray        # (N, 3)
    log_scales: np.ndarray   # (N, 3)
    quats: np.ndarray        # (N, 4) w, x, y, z (not normalised)
    opacity: np.ndarray      # (N,) logits
    sh: np.ndarray           # (N, K, 3)
    sh_degree: int
    cams: List[Camera]
    tgt_rgb: Optional[np.ndarray] = None    # concatenated over views, planar (3, H, W) per view
    tgt_depth: Optional[np.ndarray] = None  # concatenated over views, (H, W) per view, 0 = no LiDAR depth

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def params(self) -> Dict[str, np.ndarray]:
        return dict(means=self.means, log_scales=self.log_scales, quats=self.quats, opacity=self.opacity,
                    sh=self.sh)

    @property
    def total_pixels(self) -> int:
        return int(sum(c.width * c.height for c in self.cams))


def pixel_offsets(cams: Sequence[Camera]) -> List[int]:
    off, out = 0, []
    for c in cams:
        out.append(off)
        off += c.width * c.height
    return out


# --------------------------------------------------------------------------- cameras
def look_camera(pos: Sequence[float], yaw: float, pitch: float, fx: float, fy: float, W: int, H: int,
                weight: float = 1.0) -> Camera:
    """Camera at `pos` (world, z up) looking along heading `yaw` and elevation `pitch` (radians), roll 0."""
    f = np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch), math.sin(pitch)])
    r = np.cross(f, [0.0, 0.0, 1.0])
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    c2w = np.stack([r, d, f], axis=1)
    R = c2w.T.copy()
    T = -R @ np.asarray(pos, dtype=np.float64)
    return Camera(R, T, fx, fy, W / 2.0, H / 2.0, W, H, weight)


def identity_camera(fx: float, fy: float, cx: float, cy: float, W: int, H: int) -> Camera:
    return Camera(np.eye(3), np.zeros(3), fx, fy, cx, cy, W, H, 1.0)


# --------------------------------------------------------------------------- random Gaussians
def random_quats(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.standard_normal((n, 4)).astype(np.float32)  # direction uniform on S^3


def dc_from_rgb(rgb: np.ndarray) -> np.ndarray:
    return (rgb - 0.5) / _SH_DC


def frustum_scene(seed: int, n: int, cam: Camera, sh_degree: int = 0, zrange=(2.0, 20.0),
                  log_scale_mu: float = -3.0, log_scale_sigma: float = 0.5, widen: float = 0.1,
                  opacity_sigma: float = 1.0, sh_rest_sigma: float = 0.05) -> Scene:
    """Gaussians uniform in a camera-frustum box: depth U[zrange], pixel position uniform over the
    image widened by `widen` per side, back-projected through `cam` (which must be the identity pose)."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(zrange[0], zrange[1], n)
    u = rng.uniform(-widen * cam.width, (1 + widen) * cam.width, n)
    v = rng.uniform(-widen * cam.height, (1 + widen) * cam.height, n)
    x = (u - cam.cx) * z / cam.fx
    y = (v - cam.cy) * z / cam.fy
    cam_pts = np.stack([x, y, z], axis=1)
    means = (cam.R.T @ (cam_pts - cam.T).T).T
    log_scales = rng.normal(log_scale_mu, log_scale_sigma, (n, 3))
    quats = random_quats(rng, n)
    opacity = rng.normal(0.0, opacity_sigma, n)
    K = (sh_degree + 1) ** 2
    sh = np.zeros((n, K, 3))
    sh[:, 0, :] = dc_from_rgb(rng.uniform(0, 1, (n, 3)))
    if K > 1:
        sh[:, 1:, :] = rng.normal(0.0, sh_rest_sigma, (n, K - 1, 3))
    return Scene(means.astype(np.float32), log_scales.astype(np.float32), quats, opacity.astype(np.float32),
                 sh.astype(np.float32), sh_degree, [cam])


def uniform_targets(seed: int, cams: Sequence[Camera], depth_range=(2.0, 20.0),
                    depth_fraction: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """RGB U[0,1] and depth U[depth_range] with a fraction `depth_fraction` of valid pixels (0 = none)."""
    rng = np.random.default_rng(seed)
    rgbs, depths = [], []
    for c in cams:
        P = c.width * c.height
        rgbs.append(rng.uniform(0, 1, 3 * P))
        d = rng.uniform(depth_range[0], depth_range[1], P)
        if depth_fraction < 1.0:
            d[rng.uniform(0, 1, P) >= depth_fraction] = 0.0
        depths.append(d)
    return np.concatenate(rgbs).astype(np.float32), np.concatenate(depths).astype(np.float32)


# --------------------------------------------------------------------------- LiDAR scene
@dataclasses.dataclass
class Boxes:
    lo: np.ndarray  # (B, 3)
    hi: np.ndarray  # (B, 3)


def random_boxes(rng: np.random.Generator, count: int, keep_clear: np.ndarray, extent: str,
                 r_in: float = 5.0, r_out: float = 55.0, half: float = 100.0) -> Boxes:
    """Axis-aligned boxes standing on the ground z = 0: footprint U[1,8] m, height U[1,10] m.

    extent "annulus": centres 5-55 m from the nearest trajectory point; "square": a 200 m x 200 m area.
    No box covers a trajectory point (keep_clear, (P, 2) xy)."""
    lo, hi = [], []
    while len(lo) < count:
        fx, fy = rng.uniform(1, 8, 2)
        h = rng.uniform(1, 10)
        if extent == "annulus":
            anchor = keep_clear[rng.integers(len(keep_clear))]
            ang = rng.uniform(0, 2 * math.pi)
            rad = math.sqrt(rng.uniform(r_in ** 2, r_out ** 2))
            c = anchor + rad * np.array([math.cos(ang), math.sin(ang)])
        else:
            c = rng.uniform(-half, half, 2)
        d = np.abs(keep_clear - c)
        if np.any((d[:, 0] < fx / 2 + 1.0) & (d[:, 1] < fy / 2 + 1.0)):
            continue
        lo.append([c[0] - fx / 2, c[1] - fy / 2, 0.0])
        hi.append([c[0] + fx / 2, c[1] + fy / 2, h])
    return Boxes(np.array(lo), np.array(hi))


def _raycast(origin: np.ndarray, dirs: np.ndarray, boxes: Boxes) -> np.ndarray:
    """Distance along each unit ray to the first hit of the ground plane or a box (inf if none)."""
    best = np.full(dirs.shape[0], np.inf)
    dz = dirs[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        tg = np.where(dz < 0, -origin[2] / dz, np.inf)
        best = np.minimum(best, tg)
        inv = 1.0 / dirs
        for b in range(boxes.lo.shape[0]):
            t1 = (boxes.lo[b] - origin) * inv
            t2 = (boxes.hi[b] - origin) * inv
            tmin = np.nanmax(np.minimum(t1, t2), axis=1)
            tmax = np.nanmin(np.maximum(t1, t2), axis=1)
            hit = (tmax >= np.maximum(tmin, 0.0)) & (tmin > 0)
            best = np.where(hit & (tmin < best), tmin, best)
    return best


def lidar_points(rng: np.random.Generator, n: int, origins: np.ndarray, boxes: Boxes,
                 rmax: float = 60.0, rmin: float = 1.0, noise: float = 0.02,
                 elev=(-30.0, 15.0)) -> np.ndarray:
    """n LiDAR returns from scan poses `origins`: azimuth U[0,2pi), elevation U[elev] degrees,
    ranges in [rmin, rmax], Gaussian range noise along the ray."""
    pts = []
    have = 0
    batch = max(200_000, n // 2)
    while have < n:
        o = origins[rng.integers(len(origins), size=batch)]
        az = rng.uniform(0, 2 * math.pi, batch)
        el = np.radians(rng.uniform(elev[0], elev[1], batch))
        d = np.stack([np.cos(az) * np.cos(el), np.sin(az) * np.cos(el), np.sin(el)], axis=1)
        rng_out = np.empty(batch)
        for oi in np.unique(o, axis=0):
            sel = np.all(o == oi, axis=1)
            rng_out[sel] = _raycast(oi, d[sel], boxes)
        ok = (rng_out >= rmin) & (rng_out <= rmax)
        r = rng_out[ok] + rng.normal(0.0, noise, int(ok.sum()))
        p = o[ok] + d[ok] * r[:, None]
        pts.append(p)
        have += p.shape[0]
    return np.concatenate(pts)[:n]


def init_from_points(rng: np.random.Generator, pts: np.ndarray, sh_degree: int, opacity0: float = 0.1,
                     scale_jitter: float = 0.3, opacity_jitter: float = 0.5,
                     sh_rest_sigma: float = 0.05) -> Dict[str, np.ndarray]:
    """Gaussians on LiDAR points: log-scale from the mean squared distance to the 3 nearest neighbours
    (clamped at 1e-7), random rotation, opacity logit(opacity0) + noise, SH DC from a U[0,1] colour."""
    from scipy.spatial import cKDTree

    n = pts.shape[0]
    tree = cKDTree(pts)
    dist, _ = tree.query(pts, k=4, workers=-1)
    d2 = np.maximum((dist[:, 1:] ** 2).mean(axis=1), 1e-7)
    log_s = np.log(np.sqrt(d2))[:, None].repeat(3, axis=1)
    log_s = log_s + rng.normal(0.0, scale_jitter, (n, 3))
    quats = random_quats(rng, n)
    logit0 = math.log(opacity0 / (1 - opacity0))
    opacity = logit0 + rng.normal(0.0, opacity_jitter, n)
    K = (sh_degree + 1) ** 2
    sh = np.zeros((n, K, 3), dtype=np.float32)
    sh[:, 0, :] = dc_from_rgb(rng.uniform(0, 1, (n, 3)))
    if K > 1:
        sh[:, 1:, :] = rng.normal(0.0, sh_rest_sigma, (n, K - 1, 3))
    return dict(means=pts.astype(np.float32), log_scales=log_s.astype(np.float32), quats=quats,
                opacity=opacity.astype(np.float32), sh=sh)


def pyramid_targets(rng: np.random.Generator, cam0: Camera, levels: int, depth_fraction: float = 0.05,
                    depth_range=(1.0, 60.0)) -> Tuple[List[np.ndarray], List[np.ndarray]]:
    """Targets of one keyframe: RGB U[0,1] and a sparse depth map (a fraction of valid level-0 pixels),
    then repeated 2x2 reductions: box average for RGB, mean of the valid children for depth."""
    H, W = cam0.height, cam0.width
    rgb = rng.uniform(0, 1, (3, H, W))
    depth = rng.uniform(depth_range[0], depth_range[1], (H, W))
    depth[rng.uniform(0, 1, (H, W)) >= depth_fraction] = 0.0
    rgbs, depths = [rgb], [depth]
    for _ in range(1, levels):
        r = rgbs[-1]
        c, h, w = r.shape
        rgbs.append(r.reshape(c, h // 2, 2, w // 2, 2).mean(axis=(2, 4)))
        d = depths[-1].reshape(h // 2, 2, w // 2, 2)
        cnt = (d > 0).sum(axis=(1, 3))
        s = d.sum(axis=(1, 3))
        depths.append(np.where(cnt > 0, s / np.maximum(cnt, 1), 0.0))
    return rgbs, depths


# --------------------------------------------------------------------------- workload configurations
RESOLUTIONS = [(640, 512), (800, 640), (960, 768), (1120, 896), (1280, 1024)]


def _cache_path(name: str) -> Optional[str]:
    root = os.environ.get("GS_SCENE_CACHE")
    if root is None:
        root = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), ".scene_cache")
    try:
        os.makedirs(root, exist_ok=True)
    except OSError:
        return None
    return os.path.join(root, name + ".npz")


def _lidar_gaussians(cfg: int, n: int, sh_degree: int, origins: np.ndarray, extent: str,
                     rmax: float) -> Dict[str, np.ndarray]:
    path = _cache_path(f"lidar_cfg{cfg}_n{n}_d{sh_degree}_v2")
    if path and os.path.exists(path):
        with np.load(path) as z:
            return {k: z[k] for k in z.files}
    rng = np.random.default_rng(1000 * cfg + 0)
    boxes = random_boxes(rng, 50, origins[:, :2], extent)
    pts = lidar_points(rng, n, origins, boxes, rmax=rmax)
    prm = init_from_points(np.random.default_rng(1000 * cfg + 1), pts, sh_degree)
    if path:
        tmp = path + ".tmp.npz"
        np.savez(tmp, **prm)
        os.replace(tmp, path)
    return prm


def _trajectory(length: float, count: int, height: float = 1.8) -> np.ndarray:
    x = np.linspace(-length / 2, length / 2, count)
    return np.stack([x, np.zeros(count), np.full(count, height)], axis=1)


def _loop(radius: float, count: int, height: float = 1.8) -> np.ndarray:
    a = np.linspace(0, 2 * math.pi, count, endpoint=False)
    return np.stack([radius * np.cos(a), radius * np.sin(a), np.full(count, height)], axis=1)


def _keyframe_cams(rng: np.random.Generator, traj_len: float, n_kf: int, res_choices: List[Tuple[int, int]],
                   levels: int, loop_radius: Optional[float] = None) -> List[Camera]:
    cams = []
    for k in range(n_kf):
        W, H = res_choices[k]
        if loop_radius is None:
            s = rng.uniform(-traj_len / 2, traj_len / 2)
            pos = [s, 0.0, rng.uniform(1.5, 2.0)]
            heading = 0.0 if rng.uniform() < 0.5 else math.pi
        else:
            a = rng.uniform(0, 2 * math.pi)
            pos = [loop_radius * math.cos(a), loop_radius * math.sin(a), rng.uniform(1.5, 2.0)]
            heading = a + math.pi / 2
        yaw = heading + math.radians(rng.uniform(-30, 30))
        pitch = math.radians(rng.uniform(-5, 5))
        fx = 900.0 * W / 1280.0
        base = look_camera(pos, yaw, pitch, fx, fx, W, H, 1.0 / levels)
        for l in range(levels):
            cams.append(base.scaled(l))
    return cams


def _pyramid_target_set(rng: np.random.Generator, cams: List[Camera], levels: int) -> Tuple[np.ndarray, np.ndarray]:
    rgbs, depths = [], []
    for k in range(0, len(cams), levels):
        r, d = pyramid_targets(rng, cams[k], levels)
        for l in range(levels):
            rgbs.append(r[l].reshape(-1))
            depths.append(d[l].reshape(-1))
    return np.concatenate(rgbs).astype(np.float32), np.concatenate(depths).astype(np.float32)


def config(cfg: int, n: Optional[int] = None) -> Scene:
    """The five workloads.  `n` overrides the Gaussian count (smaller variants for tests)."""
    if cfg == 1:
        cam = identity_camera(100.0, 100.0, 64.0, 48.0, 128, 96)
        sc = frustum_scene(1000 * 1 + 0, n or 2000, cam, sh_degree=0)
        sc.tgt_rgb, sc.tgt_depth = uniform_targets(1000 * 1 + 1, sc.cams, (2.0, 20.0), 1.0)
        return sc
    if cfg == 2:
        origins = np.array([[0.0, 0.0, 1.8]])
        prm = _lidar_gaussians(2, n or 300_000, 3, origins, "annulus", 60.0)
        cam = look_camera([0.0, 0.0, 1.8], 0.0, 0.0, 900.0, 900.0, 1280, 1024, 1.0)
        sc = Scene(**prm, sh_degree=3, cams=[cam])
        rng = np.random.default_rng(1000 * 2 + 2)
        r, d = pyramid_targets(rng, cam, 1)
        sc.tgt_rgb, sc.tgt_depth = r[0].reshape(-1).astype(np.float32), d[0].reshape(-1).astype(np.float32)
        return sc
    if cfg in (3, 4):
        origins = _trajectory(30.0, 20)
        prm = _lidar_gaussians(3, n or 1_000_000, 3, origins, "annulus", 60.0)
        rng = np.random.default_rng(1000 * cfg + 2)
        if cfg == 3:
            cams = _keyframe_cams(rng, 30.0, 1, [(1280, 1024)], 3)
        else:
            res = [RESOLUTIONS[0], RESOLUTIONS[-1]] + [RESOLUTIONS[i] for i in rng.integers(0, 5, 6)]
            cams = _keyframe_cams(rng, 30.0, 8, res, 3)
        sc = Scene(**prm, sh_degree=3, cams=cams)
        sc.tgt_rgb, sc.tgt_depth = _pyramid_target_set(np.random.default_rng(1000 * cfg + 3), cams, 3)
        return sc
    if cfg == 5:
        origins = _loop(60.0, 100)
        prm = _lidar_gaussians(5, n or 4_000_000, 3, origins, "square", 80.0)
        rng = np.random.default_rng(1000 * 5 + 2)
        res = [RESOLUTIONS[0], RESOLUTIONS[-1]] + [RESOLUTIONS[i] for i in rng.integers(0, 5, 14)]
        cams = _keyframe_cams(rng, 0.0, 16, res, 3, loop_radius=60.0)
        sc = Scene(**prm, sh_degree=3, cams=cams)
        sc.tgt_rgb, sc.tgt_depth = _pyramid_target_set(np.random.default_rng(1000 * 5 + 3), cams, 3)
        return sc
    raise ValueError(f"unknown configuration {cfg}")


def random_scene(seed: int, n: int, W: int, H: int, sh_degree: int = 0, views: int = 1, fx: float = None,
                 log_scale_mu: float = -3.0, log_scale_sigma: float = 0.5, zrange=(2.0, 20.0),
                 opacity_sigma: float = 1.0, depth_fraction: float = 1.0) -> Scene:
    """Small test scene: Gaussians in the frustum of an identity camera, plus `views - 1` further
    views from nearby rotated poses with different sizes, and random targets."""
    fx = fx or 0.8 * W
    cam0 = identity_camera(fx, fx, W / 2.0, H / 2.0, W, H)
    sc = frustum_scene(seed, n, cam0, sh_degree, zrange=zrange, log_scale_mu=log_scale_mu,
                       log_scale_sigma=log_scale_sigma, opacity_sigma=opacity_sigma)
    rng = np.random.default_rng(seed + 7)
    cams = [cam0]
    for k in range(1, views):
        Wk = max(8, int(W * rng.uniform(0.6, 1.2)))
        Hk = max(8, int(H * rng.uniform(0.6, 1.2)))
        yaw = math.radians(rng.uniform(-10, 10))
        pitch = math.radians(rng.uniform(-8, 8))
        f = np.array([math.sin(yaw) * math.cos(pitch), math.sin(pitch), math.cos(yaw) * math.cos(pitch)])
        # camera frame: forward f, right r, down d (world here is the first camera's frame, y down)
        r = np.cross([0.0, 1.0, 0.0], f)
        r /= np.linalg.norm(r)
        d = np.cross(f, r)
        R = np.stack([r, d, f], axis=0)
        pos = rng.uniform(-0.5, 0.5, 3)
        T = -R @ pos
        fk = fx * Wk / W
        cams.append(Camera(R, T, fk, fk, Wk / 2.0 + rng.uniform(-2, 2), Hk / 2.0 + rng.uniform(-2, 2), Wk, Hk,
                           1.0 / views))
    if views > 1:
        cams[0].weight = 1.0 / views
    sc.cams = cams
    sc.tgt_rgb, sc.tgt_depth = uniform_targets(seed + 11, cams, zrange, depth_fraction)
    return sc
