"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP path: inputs come from the
seeded generator as numpy arrays and are passed here as float64.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np

from . import build as _build

# Readings of the constants the paper leaves open (Section III-B): near plane 0.2 m,
# guard band 1.3, EWA low-pass 0.3 px^2, skip below alpha 1/255, clamp at 0.99, stop
# before T < 1e-4, black background, 16x16 tiles, lambda_d = 0.1; the SSIM weight of eq. Lc is 0 unless
# given (lambda_ssim; SSIM_LAMBDA = 0.2 is the usual 3DGS value).
DEFAULT_OPTS = dict(near=0.2, guard=1.3, lowpass=0.3, alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4,
                    bg=(0.0, 0.0, 0.0), tile_w=16, tile_h=16, lambda_d=0.1, stop_near=1e-5, lambda_ssim=0.0)

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(_build.ensure_built())
        D = ctypes.POINTER(ctypes.c_double)
        _lib.oracle_backward.restype = ctypes.c_double
        _lib.oracle_reference.restype = ctypes.c_double
        _lib.oracle_loss.restype = ctypes.c_double
        _lib.oracle_bin.restype = ctypes.c_int64
        _lib.oracle_ssim_plane.restype = ctypes.c_double
        _lib.oracle_prune.restype = ctypes.c_int64
        _lib.oracle_expand.restype = ctypes.c_int64
        _lib.oracle_ssim_loss.restype = ctypes.c_double
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def opts_array(**over) -> np.ndarray:
    o = dict(DEFAULT_OPTS)
    o.update(over)
    return _f64([o["near"], o["guard"], o["lowpass"], o["alpha_min"], o["alpha_max"], o["t_min"], *o["bg"],
                 o["tile_w"], o["tile_h"], o["lambda_d"], o["stop_near"], o["lambda_ssim"]])


def cams_array(cams: Sequence) -> np.ndarray:
    rows = []
    for c in cams:
        rows.append([*np.asarray(c.R, np.float64).reshape(-1), *np.asarray(c.T, np.float64), c.fx, c.fy, c.cx, c.cy,
                     c.width, c.height, *np.asarray(c.campos, np.float64), c.weight])
    return _f64(rows)


class _Params:
    def __init__(self, params: Dict[str, np.ndarray], sh_degree: int):
        self.means = _f64(params["means"])
        self.log_scales = _f64(params["log_scales"])
        self.quats = _f64(params["quats"])
        self.opacity = _f64(params["opacity"])
        self.sh = _f64(params["sh"])
        self.n = self.means.shape[0]
        self.deg = int(sh_degree)

    def args(self):
        return (_p(self.means), _p(self.log_scales), _p(self.quats), _p(self.opacity), _p(self.sh),
                ctypes.c_int64(self.n), ctypes.c_int(self.deg))


def tiles_of(cams, tile_w=16, tile_h=16):
    tx = [(c.width + tile_w - 1) // tile_w for c in cams]
    ty = [(c.height + tile_h - 1) // tile_h for c in cams]
    off = np.concatenate([[0], np.cumsum([a * b for a, b in zip(tx, ty)])]).astype(np.int64)
    return np.array(tx, np.int32), off[:-1].astype(np.int32), int(off[-1])


def project(prec: int, params, sh_degree: int, cams, **opt_over) -> Dict[str, np.ndarray]:
    P = _Params(params, sh_degree)
    V = len(cams)
    R = V * P.n
    out = dict(visible=np.zeros(R, np.int32), cull_reason=np.zeros(R, np.int32), mean2d=np.zeros((R, 2)),
               z=np.zeros(R), zbits=np.zeros(R, np.uint32), conic=np.zeros((R, 3)), opacity=np.zeros(R),
               rgb=np.zeros((R, 3)), pxrect=np.zeros((R, 4), np.int32), tilerect=np.zeros((R, 4), np.int32),
               rect_margin=np.zeros(R), near_margin=np.zeros(R), pass_mask=np.zeros(R, np.int32))
    lib().oracle_project(ctypes.c_int(prec), *P.args(), _p(cams_array(cams)), ctypes.c_int(V), _p(opts_array(**opt_over)),
                         _p(out["visible"]), _p(out["cull_reason"]), _p(out["mean2d"]), _p(out["z"]),
                         _p(out["zbits"]), _p(out["conic"]), _p(out["opacity"]), _p(out["rgb"]),
                         _p(out["pxrect"]), _p(out["tilerect"]), _p(out["rect_margin"]), _p(out["near_margin"]),
                         _p(out["pass_mask"]))
    return out


def bin_records(tilerect, zbits, visible, n: int, cams, tile_w=16, tile_h=16):
    """Sorted (key, value) instances and per-tile [lo, hi) ranges for given records."""
    tx, toff, total = tiles_of(cams, tile_w, tile_h)
    tilerect = np.ascontiguousarray(tilerect, np.int32)
    zbits = np.ascontiguousarray(zbits, np.uint32)
    visible = np.ascontiguousarray(visible, np.int32)
    lo = np.zeros(total, np.int64)
    hi = np.zeros(total, np.int64)
    cap = 0
    I = lib().oracle_bin(_p(tilerect), _p(zbits), _p(visible), ctypes.c_int64(n), ctypes.c_int(len(cams)), _p(tx),
                         _p(toff), ctypes.c_int(total), None, None, ctypes.c_int64(cap), _p(lo), _p(hi))
    keys = np.zeros(max(I, 1), np.uint64)
    vals = np.zeros(max(I, 1), np.int64)
    lib().oracle_bin(_p(tilerect), _p(zbits), _p(visible), ctypes.c_int64(n), ctypes.c_int(len(cams)), _p(tx),
                     _p(toff), ctypes.c_int(total), _p(keys), _p(vals), ctypes.c_int64(I), _p(lo), _p(hi))
    return keys[:I], vals[:I], lo, hi


def _image_buffers(cams):
    P = sum(c.width * c.height for c in cams)
    return dict(rgb=np.zeros(3 * P), depth=np.zeros(P), vis=np.zeros(P), final_T=np.zeros(P),
                n_contrib=np.zeros(P, np.int32), near=np.zeros(P, np.int8))


def composite(prec: int, mode: int, rec: Dict[str, np.ndarray], n: int, cams, **opt_over) -> Dict[str, np.ndarray]:
    """Composite given records (keys: mean2d, z, zbits, conic, opacity, rgb, tilerect, visible)."""
    out = _image_buffers(cams)
    lib().oracle_composite(ctypes.c_int(prec), ctypes.c_int(mode), _p(_f64(rec["mean2d"])), _p(_f64(rec["z"])),
                           _p(np.ascontiguousarray(rec["zbits"], np.uint32)), _p(_f64(rec["conic"])),
                           _p(_f64(rec["opacity"])), _p(_f64(rec["rgb"])),
                           _p(np.ascontiguousarray(rec["tilerect"], np.int32)),
                           _p(np.ascontiguousarray(rec["visible"], np.int32)), ctypes.c_int64(n),
                           _p(cams_array(cams)), ctypes.c_int(len(cams)), _p(opts_array(**opt_over)), _p(out["rgb"]),
                           _p(out["depth"]), _p(out["vis"]), _p(out["final_T"]), _p(out["n_contrib"]),
                           _p(out["near"]))
    return out


def forward(prec: int, params, sh_degree: int, cams, mode: int = 1, **opt_over) -> Dict[str, np.ndarray]:
    P = _Params(params, sh_degree)
    out = _image_buffers(cams)
    lib().oracle_forward(ctypes.c_int(prec), ctypes.c_int(mode), *P.args(), _p(cams_array(cams)),
                         ctypes.c_int(len(cams)), _p(opts_array(**opt_over)), _p(out["rgb"]), _p(out["depth"]),
                         _p(out["vis"]), _p(out["final_T"]), _p(out["n_contrib"]), _p(out["near"]))
    return out


def backward(prec: int, params, sh_degree: int, cams, g_rgb=None, g_depth=None, g_vis=None, tgt_rgb=None,
             tgt_depth=None, decisions: Optional[int] = None, **opt_over):
    """Loss and analytic gradients (+ excused Gaussians and the count of near-threshold pixels).

    prec=64 with decisions=32: every discrete choice (cull, skip, clamp, stop, colour clamp, loss sign) taken
    by the FP32 evaluation, every value computed in FP64 along those choices."""
    P = _Params(params, sh_degree)
    K = (sh_degree + 1) ** 2
    gr = dict(means=np.zeros((P.n, 3)), log_scales=np.zeros((P.n, 3)), quats=np.zeros((P.n, 4)),
              opacity=np.zeros(P.n), sh=np.zeros((P.n, K, 3)))
    exc = np.zeros(P.n, np.int8)
    nn = np.zeros(1, np.int64)
    img = _image_buffers(cams)
    conv = lambda a: None if a is None else _f64(a)
    g_rgb, g_depth, g_vis, tgt_rgb, tgt_depth = map(conv, (g_rgb, g_depth, g_vis, tgt_rgb, tgt_depth))
    code = 3264 if (prec == 64 and decisions == 32) else prec
    L = lib().oracle_backward(ctypes.c_int(code), *P.args(), _p(cams_array(cams)), ctypes.c_int(len(cams)),
                              _p(opts_array(**opt_over)), _p(g_rgb), _p(g_depth), _p(g_vis), _p(tgt_rgb),
                              _p(tgt_depth), _p(gr["means"]), _p(gr["log_scales"]), _p(gr["quats"]),
                              _p(gr["opacity"]), _p(gr["sh"]), _p(exc), _p(nn), _p(img["rgb"]), _p(img["depth"]),
                              _p(img["vis"]))
    return float(L), gr, exc.astype(bool), int(nn[0]), img


def reference(params, sh_degree: int, cams, g_rgb=None, g_depth=None, g_vis=None, tgt_rgb=None, tgt_depth=None,
              **opt_over) -> Dict[str, object]:
    """The gradient reference of the tests: loss and gradients in FP64 along the FP32 decisions, with the flip
    allowance of every gradient entry (the change the entry would see if one near-threshold decision -- a skip,
    clamp or stop at a pixel, or the sign of an L1 term -- were taken the other way, summed over such
    decisions), the Gaussians excused outright (a cull or colour-clamp decision near its threshold, or visible
    in one precision only) and the count of pixels holding a near decision."""
    P = _Params(params, sh_degree)
    K = (sh_degree + 1) ** 2
    shapes = dict(means=(P.n, 3), log_scales=(P.n, 3), quats=(P.n, 4), opacity=(P.n,), sh=(P.n, K, 3))
    gr = {k: np.zeros(v) for k, v in shapes.items()}
    al = {k: np.zeros(v) for k, v in shapes.items()}
    exc = np.zeros(P.n, np.int8)
    nn = np.zeros(1, np.int64)
    img = _image_buffers(cams)
    conv = lambda a: None if a is None else _f64(a)
    g_rgb, g_depth, g_vis, tgt_rgb, tgt_depth = map(conv, (g_rgb, g_depth, g_vis, tgt_rgb, tgt_depth))
    keys = ("means", "log_scales", "quats", "opacity", "sh")
    L = lib().oracle_reference(*P.args(), _p(cams_array(cams)), ctypes.c_int(len(cams)), _p(opts_array(**opt_over)),
                               _p(g_rgb), _p(g_depth), _p(g_vis), _p(tgt_rgb), _p(tgt_depth),
                               *[_p(gr[k]) for k in keys], *[_p(al[k]) for k in keys], _p(exc), _p(nn),
                               _p(img["rgb"]), _p(img["depth"]), _p(img["vis"]))
    return dict(loss=float(L), grads=gr, allowance=al, excused=exc.astype(bool), near_pixels=int(nn[0]), images=img)


def gradient_scale(params, sh_degree: int, cams, g_rgb=None, g_depth=None, g_vis=None, tgt_rgb=None,
                   tgt_depth=None, **opt_over) -> Dict[str, np.ndarray]:
    """Per gradient entry, the sum of the magnitudes of the terms it sums (FP64): an FP32 evaluation of the
    gradient, in any order, is within a small multiple of 2^-24 times this of the exact value."""
    P = _Params(params, sh_degree)
    K = (sh_degree + 1) ** 2
    s = dict(means=np.zeros((P.n, 3)), log_scales=np.zeros((P.n, 3)), quats=np.zeros((P.n, 4)),
             opacity=np.zeros(P.n), sh=np.zeros((P.n, K, 3)))
    conv = lambda a: None if a is None else _f64(a)
    g_rgb, g_depth, g_vis, tgt_rgb, tgt_depth = map(conv, (g_rgb, g_depth, g_vis, tgt_rgb, tgt_depth))
    lib().oracle_gradient_scale(*P.args(), _p(cams_array(cams)), ctypes.c_int(len(cams)), _p(opts_array(**opt_over)),
                                _p(g_rgb), _p(g_depth), _p(g_vis), _p(tgt_rgb), _p(tgt_depth), _p(s["means"]),
                                _p(s["log_scales"]), _p(s["quats"]), _p(s["opacity"]), _p(s["sh"]))
    return s


def loss(params, sh_degree: int, cams, tgt_rgb, tgt_depth, **opt_over) -> float:
    P = _Params(params, sh_degree)
    return float(lib().oracle_loss(*P.args(), _p(cams_array(cams)), ctypes.c_int(len(cams)),
                                   _p(opts_array(**opt_over)), _p(_f64(tgt_rgb)), _p(_f64(tgt_depth))))


def adam(p, g, m, v, lr, beta1=0.9, beta2=0.999, eps=1e-15, step=1):
    p, g, m, v = (_f64(a).copy() for a in (p, g, m, v))
    lib().oracle_adam(_p(p), _p(g), _p(m), _p(v), ctypes.c_int64(p.size), ctypes.c_double(lr),
                      ctypes.c_double(beta1), ctypes.c_double(beta2), ctypes.c_double(eps), ctypes.c_int64(step))
    return p, m, v


def sh_basis(deg: int, d):
    K = (deg + 1) ** 2
    Y = np.zeros(K)
    dY = np.zeros((K, 3))
    lib().oracle_sh_basis(ctypes.c_int(deg), _p(_f64(d)), _p(Y), _p(dY))
    return Y, dY


def quat_to_rot(q) -> np.ndarray:
    M = np.zeros(9)
    lib().oracle_quat_to_rot(_p(_f64(q)), _p(M))
    return M.reshape(3, 3)


def prune(opacity_logit, min_opacity: float) -> np.ndarray:
    """Indices (in order) of the Gaussians kept by opacity pruning at min_opacity."""
    o = _f64(np.asarray(opacity_logit).reshape(-1))
    idx = np.zeros(max(o.size, 1), np.int64)
    k = lib().oracle_prune(_p(o), ctypes.c_int64(o.size), ctypes.c_double(min_opacity), _p(idx))
    return idx[:k]


def prune(opacity_logit, min_opacity: float) -> np.ndarray:
    """Indices (in order) of the Gaussians kept by opacity pruning at min_opacity."""
    o = _f64(np.asarray(opacity_logit).reshape(-1))
    idx = np.zeros(max(o.size, 1), np.int64)
    k = lib().oracle_prune(_p(o), ctypes.c_int64(o.size), ctypes.c_double(min_opacity), _p(idx))
    return idx[:k]


def expand(points, colours, cam, vis, tau_alpha: float, map_means, voxel: float, cap: int = 1,
           init_opacity: float = 0.1, sh_degree: int = 0, near: float = 0.2):
    """Map expansion of one keyframe's points: (kept mask [M], new Gaussians' parameters in input order)."""
    pts = _f64(np.asarray(points).reshape(-1, 3))
    rgb = _f64(np.asarray(colours).reshape(-1, 3))
    M = pts.shape[0]
    camv = _f64([*np.asarray(cam.R, np.float64).reshape(-1), *np.asarray(cam.T, np.float64), cam.fx, cam.fy, cam.cx,
                 cam.cy, cam.width, cam.height])
    mm = _f64(np.asarray(map_means).reshape(-1, 3)) if map_means is not None else np.zeros((0, 3))
    K = (sh_degree + 1) ** 2
    kept = np.zeros(M, np.int32)
    out = dict(means=np.zeros((M, 3)), log_scales=np.zeros((M, 3)), quats=np.zeros((M, 4)), opacity=np.zeros(M),
               sh=np.zeros((M, K, 3)))
    A = lib().oracle_expand(_p(pts), _p(rgb), ctypes.c_int64(M), _p(camv), _p(_f64(np.asarray(vis).reshape(-1))),
                            ctypes.c_double(tau_alpha), ctypes.c_double(near), _p(mm), ctypes.c_int64(mm.shape[0]),
                            ctypes.c_double(voxel), ctypes.c_int(cap), ctypes.c_double(init_opacity),
                            ctypes.c_int(sh_degree), _p(kept), _p(out["means"]), _p(out["log_scales"]),
                            _p(out["quats"]), _p(out["opacity"]), _p(out["sh"]))
    return kept.astype(bool), {k: v[:A] for k, v in out.items()}


def spatial_order(means) -> np.ndarray:
    """The Morton-order permutation of the Gaussians (new row k = old row perm[k])."""
    mm = _f64(np.asarray(means).reshape(-1, 3))
    perm = np.zeros(max(mm.shape[0], 1), np.int32)
    lib().oracle_spatial_order(_p(mm), ctypes.c_int64(mm.shape[0]), _p(perm))
    return perm[:mm.shape[0]]


SSIM_LAMBDA = 0.2  # weight of the SSIM term in eq. Lc (the value of the 3DGS work the paper builds on)


def ssim_window() -> np.ndarray:
    w = np.zeros(121)
    lib().oracle_ssim_window(_p(w))
    return w.reshape(11, 11)


def ssim_plane(x, y, grad: bool = False):
    """(mean SSIM, per-pixel SSIM map, d mean / d x or None) of one channel plane [H, W] (FP64)."""
    x, y = _f64(x), _f64(y)
    H, W = x.shape
    m = np.zeros((H, W))
    g = np.zeros((H, W)) if grad else None
    mean = lib().oracle_ssim_plane(_p(x), _p(y), ctypes.c_int(H), ctypes.c_int(W), _p(m), _p(g))
    return float(mean), m, g


def ssim_loss(x, y, cams, lam: float = SSIM_LAMBDA, grad: bool = True):
    """The SSIM term sum_v w_v lam (1 - mean SSIM_v) of planar per-view images [3][H_v][W_v] (concatenated over
    views) and its gradient with respect to x (same layout)."""
    x, y = _f64(x), _f64(y)
    sizes = np.ascontiguousarray([[c.height, c.width] for c in cams], np.int32).reshape(-1)
    w = _f64([c.weight for c in cams])
    g = np.zeros_like(x) if grad else None
    L = lib().oracle_ssim_loss(_p(x), _p(y), ctypes.c_int(len(cams)), _p(sizes), _p(w), ctypes.c_double(lam), _p(g))
    return float(L), g


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of the following oracle calls."""
    lib().oracle_set_threads(ctypes.c_int(int(n)))
