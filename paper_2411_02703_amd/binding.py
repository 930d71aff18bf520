"""ctypes binding of libgs.so: the C-ABI calls under the same names, plus argument marshalling.

Every step of the splatting path runs in the HIP library; this module only turns torch tensors and
camera descriptions into the C structures and raises on a non-zero status.  There is no fallback:
if libgs.so is missing or fails to load, `load()` raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgs.so")

c_f = ctypes.c_float
c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_vp = ctypes.c_void_p
P = ctypes.POINTER


class gs_camera(ctypes.Structure):
    _fields_ = [("R", c_f * 9), ("T", c_f * 3), ("fx", c_f), ("fy", c_f), ("cx", c_f), ("cy", c_f),
                ("campos", c_f * 3), ("loss_weight", c_f), ("width", c_i32), ("height", c_i32),
                ("tiles_x", c_i32), ("tiles_y", c_i32), ("tile_offset", c_i32), ("pixel_offset", c_i32),
                ("guard_lo_x", c_f), ("guard_hi_x", c_f), ("guard_lo_y", c_f), ("guard_hi_y", c_f),
                ("reserved", c_i32 * 2)]


class gs_opts(ctypes.Structure):
    _fields_ = [("tile_w", c_i32), ("tile_h", c_i32), ("near_z", c_f), ("guard", c_f), ("lowpass", c_f),
                ("alpha_min", c_f), ("alpha_max", c_f), ("t_min", c_f), ("bg", c_f * 3), ("waves_per_tile", c_i32),
                ("block_w", c_i32), ("batch_depth", c_i32), ("seg_len", c_i32), ("persistent", c_i32)]


class gs_params(ctypes.Structure):
    _fields_ = [("means", c_vp), ("log_scales", c_vp), ("quats", c_vp), ("opacity", c_vp), ("sh", c_vp),
                ("n", c_i64), ("sh_degree", c_i32), ("reserved", c_i32)]


class gs_frame(ctypes.Structure):
    _fields_ = [("n", c_i64), ("n_views", c_i32), ("n_tiles", c_i32), ("n_pixels", c_i64),
                ("max_view_pixels", c_i64), ("capacity", c_i64), ("key_bits", c_i32), ("sort_passes", c_i32),
                ("tile_w", c_i32), ("tile_h", c_i32), ("seg_len", c_i32), ("seg_cap", c_i32), ("long_cap", c_i32),
                ("item_cap", c_i32), ("cams", c_vp), ("block", c_vp), ("bytes", ctypes.c_size_t),
                ("rec", c_vp), ("rect", c_vp), ("ipart", c_vp), ("inst_first", c_vp), ("vis_mask", c_vp),
                ("n_inst", c_vp), ("n_rec", c_vp), ("rec_first", c_vp), ("zbits", c_vp), ("rec_slot", c_vp), ("big_rec", c_vp), ("rec_cap", c_i64),
                ("rkeys", c_vp * 2), ("rvals", c_vp * 2), ("keys", c_vp * 2), ("vals", c_vp * 2), ("tile_range", c_vp),
                ("tile_order", c_vp), ("counters", c_vp), ("seg_count", c_vp), ("seg_first", c_vp), ("items", c_vp),
                ("seg", c_vp), ("split", c_vp), ("loss", c_vp), ("scratch", c_vp), ("scratch_ints", ctypes.c_size_t)]


class gs_images(ctypes.Structure):
    _fields_ = [("rgb", c_vp), ("depth", c_vp), ("vis", c_vp)]


class gs_loss(ctypes.Structure):
    _fields_ = [("g_rgb", c_vp), ("g_depth", c_vp), ("g_vis", c_vp), ("tgt_rgb", c_vp), ("tgt_depth", c_vp),
                ("lambda_d", c_f), ("lambda_ssim", c_f)]


class gs_expand_opts(ctypes.Structure):
    _fields_ = [("tau_alpha", c_f), ("near_z", c_f), ("voxel", c_f), ("knn_cell", c_f), ("init_opacity", c_f),
                ("cap", c_i32)]


class gs_adam(ctypes.Structure):
    _fields_ = [("lr", c_f * 6), ("beta1", c_f), ("beta2", c_f), ("eps", c_f), ("flags", c_i32),
                ("step", c_vp), ("bias", c_vp), ("skip_flags", c_vp)]


assert ctypes.sizeof(gs_camera) == 128

GS_FLAG_INSTANCE_OVERFLOW = 1
GS_FLAG_NONFINITE = 2
GS_ADAM_SPARSE = 1

EXPORTED = ["gs_default_opts", "gs_plan_cameras", "gs_frame_bytes", "gs_frame_init", "gs_project", "gs_bin_tiles",
            "gs_render_fwd", "gs_render_bwd", "gs_composite_bwd", "gs_project_bwd", "gs_adam_step",
            "gs_render_bwd_adam", "gs_ssim", "gs_prune_scratch_bytes", "gs_prune",
            "gs_expand_scratch_bytes", "gs_expand", "gs_spatial_order_scratch_bytes", "gs_spatial_order",
            "gs_count_pairs", "gs_read_counters", "gs_sort_scratch_ints", "gs_sort_pairs", "gs_sort_static_max",
            "gs_sort_pairs_static", "gs_status_string",
            "gs_last_error", "gs_version"]

_lib: Optional[ctypes.CDLL] = None


def load() -> ctypes.CDLL:
    """Load libgs.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2411_02703_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    lib.gs_default_opts.argtypes = [P(gs_opts)]
    lib.gs_default_opts.restype = None
    lib.gs_plan_cameras.argtypes = [P(gs_camera), c_i32, P(gs_opts)]
    lib.gs_frame_bytes.argtypes = [c_i64, P(gs_camera), c_i32, P(gs_opts), c_i64]
    lib.gs_frame_bytes.restype = ctypes.c_size_t
    lib.gs_frame_init.argtypes = [P(gs_frame), c_vp, ctypes.c_size_t, c_i64, P(gs_camera), c_vp, c_i32, P(gs_opts),
                                  c_i64]
    lib.gs_project.argtypes = [P(gs_params), P(gs_frame), P(gs_opts), c_vp]
    lib.gs_bin_tiles.argtypes = [P(gs_frame), P(gs_opts), c_i32, P(c_i64), c_vp]
    lib.gs_render_fwd.argtypes = [P(gs_frame), P(gs_opts), P(gs_images), c_vp]
    lib.gs_render_bwd.argtypes = [P(gs_params), P(gs_frame), P(gs_opts), P(gs_images), P(gs_loss), P(gs_params),
                                  c_vp]
    lib.gs_composite_bwd.argtypes = [P(gs_frame), P(gs_opts), P(gs_images), P(gs_loss), c_vp]
    lib.gs_project_bwd.argtypes = [P(gs_params), P(gs_frame), P(gs_opts), P(gs_params), c_vp]
    lib.gs_adam_step.argtypes = [P(gs_params), P(gs_params), P(gs_params), P(gs_params), P(gs_adam), c_vp]
    lib.gs_expand_scratch_bytes.argtypes = [c_i64, c_i64]
    lib.gs_expand_scratch_bytes.restype = ctypes.c_size_t
    lib.gs_expand.argtypes = [P(gs_params), P(gs_params), P(gs_params), c_i64, c_vp, c_vp, c_i64, P(gs_camera), c_vp,
                              P(gs_expand_opts), c_vp, c_vp, c_vp]
    lib.gs_spatial_order_scratch_bytes.argtypes = [c_i64]
    lib.gs_spatial_order_scratch_bytes.restype = ctypes.c_size_t
    lib.gs_spatial_order.argtypes = [P(gs_params), P(gs_params), P(gs_params), P(gs_params), P(gs_params),
                                     P(gs_params), c_vp, c_vp, c_vp]
    lib.gs_prune_scratch_bytes.argtypes = [c_i64]
    lib.gs_prune_scratch_bytes.restype = ctypes.c_size_t
    lib.gs_prune.argtypes = [P(gs_params), P(gs_params), P(gs_params), c_f, P(gs_params), P(gs_params), P(gs_params),
                             c_vp, c_vp, c_vp]
    lib.gs_ssim.argtypes = [P(gs_camera), c_vp, c_i32, c_vp, c_vp, c_f, c_vp, c_vp, c_vp]
    lib.gs_render_bwd_adam.argtypes = [P(gs_params), P(gs_frame), P(gs_opts), P(gs_images), P(gs_loss),
                                       P(gs_params), P(gs_params), P(gs_adam), P(gs_params), c_vp]
    lib.gs_count_pairs.argtypes = [P(gs_frame), P(gs_opts), c_vp, c_vp]
    lib.gs_read_counters.argtypes = [P(gs_frame), P(c_i64), P(c_i32), c_vp]
    lib.gs_sort_scratch_ints.argtypes = [c_i64]
    lib.gs_sort_scratch_ints.restype = ctypes.c_size_t
    lib.gs_sort_pairs.argtypes = [c_vp, c_vp, c_vp, c_vp, c_i64, c_i32, c_vp, c_vp]
    lib.gs_sort_static_max.argtypes = []
    lib.gs_sort_static_max.restype = c_i64
    lib.gs_sort_pairs_static.argtypes = [c_vp, c_vp, c_i64, c_i32, c_vp]
    lib.gs_status_string.argtypes = [ctypes.c_int]
    lib.gs_status_string.restype = ctypes.c_char_p
    lib.gs_last_error.argtypes = []
    lib.gs_last_error.restype = ctypes.c_char_p
    lib.gs_version.argtypes = []
    _lib = lib
    return lib


def _check(rc: int, what: str) -> None:
    if rc != 0:
        lib = load()
        raise RuntimeError(f"{what}: {lib.gs_status_string(rc).decode()} ({lib.gs_last_error().decode()})")


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("image arguments must be contiguous float32 CUDA tensors")
    return t.data_ptr()


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


# --------------------------------------------------------------------------- structures
def default_opts(**over) -> gs_opts:
    o = gs_opts()
    load().gs_default_opts(ctypes.byref(o))
    for k, v in over.items():
        if k == "bg":
            for i in range(3):
                o.bg[i] = v[i]
        else:
            setattr(o, k, v)
    return o


def make_cameras(cams: Sequence) -> ctypes.Array:
    """gs_camera array from scenes.Camera-like objects (R, T, fx, fy, cx, cy, width, height, weight)."""
    arr = (gs_camera * len(cams))()
    for i, c in enumerate(cams):
        R = np.asarray(c.R, np.float64)
        T = np.asarray(c.T, np.float64)
        pos = -R.T @ T
        a = arr[i]
        for k in range(9):
            a.R[k] = float(R.reshape(-1)[k])
        for k in range(3):
            a.T[k] = float(T[k])
            a.campos[k] = float(pos[k])
        a.fx, a.fy, a.cx, a.cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        a.width, a.height = int(c.width), int(c.height)
        a.loss_weight = float(c.weight)
    return arr


def params_struct(p: Dict[str, torch.Tensor], sh_degree: int) -> gs_params:
    for k in ("means", "log_scales", "quats", "opacity", "sh"):
        t = p[k]
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError(f"{k} must be a contiguous float32 CUDA tensor")
    return gs_params(p["means"].data_ptr(), p["log_scales"].data_ptr(), p["quats"].data_ptr(),
                     p["opacity"].data_ptr(), p["sh"].data_ptr(), int(p["means"].shape[0]), int(sh_degree), 0)


class Frame:
    """A frame block (device memory owned by torch) carved by gs_frame_init, with its cameras."""

    def __init__(self, n: int, cams: Sequence, opts: Optional[gs_opts] = None, capacity: Optional[int] = None,
                 device: str = "cuda"):
        lib = load()
        self.opts = opts if opts is not None else default_opts()
        self.cams_host = make_cameras(cams)
        self.n_views = len(cams)
        _check(lib.gs_plan_cameras(self.cams_host, self.n_views, ctypes.byref(self.opts)), "gs_plan_cameras")
        raw = bytes(self.cams_host)
        self.cams_dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)
        self.n = int(n)
        self.n_pixels = sum(c.width * c.height for c in self.cams_host)
        self.capacity = int(capacity) if capacity else max(1 << 16, 4 * self.n)
        nbytes = lib.gs_frame_bytes(self.n, self.cams_host, self.n_views, ctypes.byref(self.opts), self.capacity)
        if nbytes == 0:
            _check(-1, "gs_frame_bytes")
        self.block = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.block.data_ptr()
        aligned = (base + 255) & ~255
        self.f = gs_frame()
        _check(lib.gs_frame_init(ctypes.byref(self.f), aligned, nbytes, self.n, self.cams_host,
                                 self.cams_dev.data_ptr(), self.n_views, ctypes.byref(self.opts), self.capacity),
               "gs_frame_init")
        self.pixel_offsets = [c.pixel_offset for c in self.cams_host]

    @property
    def sorted_index(self) -> int:
        return self.f.sort_passes & 1

    def empty_images(self, device="cuda"):
        P = self.n_pixels
        return (torch.empty(3 * P, device=device), torch.empty(P, device=device), torch.empty(P, device=device))

    def view_slices(self, v: int):
        c = self.cams_host[v]
        P = c.width * c.height
        return c.pixel_offset, P, c.height, c.width


# --------------------------------------------------------------------------- the C-ABI calls
def gs_project(params: gs_params, frame: Frame, stream=None) -> None:
    _check(load().gs_project(ctypes.byref(params), ctypes.byref(frame.f), ctypes.byref(frame.opts),
                             _stream(stream)), "gs_project")


def gs_bin_tiles(frame: Frame, sync_count: bool = True, stream=None) -> Optional[int]:
    n = c_i64(-1)
    _check(load().gs_bin_tiles(ctypes.byref(frame.f), ctypes.byref(frame.opts), int(sync_count), ctypes.byref(n),
                               _stream(stream)), "gs_bin_tiles")
    return int(n.value) if sync_count else None


def gs_render_fwd(frame: Frame, rgb: torch.Tensor, depth: torch.Tensor, vis: torch.Tensor, stream=None) -> None:
    im = gs_images(rgb.data_ptr(), depth.data_ptr(), vis.data_ptr())
    _check(load().gs_render_fwd(ctypes.byref(frame.f), ctypes.byref(frame.opts), ctypes.byref(im), _stream(stream)),
           "gs_render_fwd")


def gs_render_bwd(params: gs_params, frame: Frame, fwd: Optional[Sequence[torch.Tensor]], grads: gs_params,
                  g_rgb=None, g_depth=None, g_vis=None, tgt_rgb=None, tgt_depth=None, lambda_d: float = 0.1,
                  lambda_ssim: float = 0.0, stream=None) -> None:
    im = None
    if fwd is not None:
        im = gs_images(fwd[0].data_ptr(), fwd[1].data_ptr(), fwd[2].data_ptr())
    l = _loss_struct(g_rgb, g_depth, g_vis, tgt_rgb, tgt_depth, lambda_d, lambda_ssim)
    _check(load().gs_render_bwd(ctypes.byref(params), ctypes.byref(frame.f), ctypes.byref(frame.opts),
                                ctypes.byref(im) if im is not None else None, ctypes.byref(l), ctypes.byref(grads),
                                _stream(stream)), "gs_render_bwd")


def _loss_struct(g_rgb, g_depth, g_vis, tgt_rgb, tgt_depth, lambda_d, lambda_ssim=0.0) -> gs_loss:
    return gs_loss(_ptr(g_rgb), _ptr(g_depth), _ptr(g_vis), _ptr(tgt_rgb), _ptr(tgt_depth), float(lambda_d),
                   float(lambda_ssim))


def gs_composite_bwd(frame: Frame, fwd: Optional[Sequence[torch.Tensor]], g_rgb=None, g_depth=None, g_vis=None,
                     tgt_rgb=None, tgt_depth=None, lambda_d: float = 0.1, lambda_ssim: float = 0.0,
                     stream=None) -> None:
    im = None
    if fwd is not None:
        im = gs_images(fwd[0].data_ptr(), fwd[1].data_ptr(), fwd[2].data_ptr())
    l = _loss_struct(g_rgb, g_depth, g_vis, tgt_rgb, tgt_depth, lambda_d, lambda_ssim)
    _check(load().gs_composite_bwd(ctypes.byref(frame.f), ctypes.byref(frame.opts),
                                   ctypes.byref(im) if im is not None else None, ctypes.byref(l), _stream(stream)),
           "gs_composite_bwd")


def gs_project_bwd(params: gs_params, frame: Frame, grads: gs_params, stream=None) -> None:
    _check(load().gs_project_bwd(ctypes.byref(params), ctypes.byref(frame.f), ctypes.byref(frame.opts),
                                 ctypes.byref(grads), _stream(stream)), "gs_project_bwd")


def gs_count_pairs(frame: Frame, stream=None):
    """(evaluated, contributing) pairs of the frame's forward compositing (synchronises)."""
    c = torch.zeros(2, dtype=torch.int64, device="cuda")
    _check(load().gs_count_pairs(ctypes.byref(frame.f), ctypes.byref(frame.opts), c.data_ptr(), _stream(stream)),
           "gs_count_pairs")
    ev, co = c.cpu().tolist()
    return int(ev), int(co)


def gs_adam_step(params: gs_params, grads: gs_params, m: gs_params, v: gs_params, adam: gs_adam,
                 stream=None) -> None:
    _check(load().gs_adam_step(ctypes.byref(params), ctypes.byref(grads), ctypes.byref(m), ctypes.byref(v),
                               ctypes.byref(adam), _stream(stream)), "gs_adam_step")


def gs_render_bwd_adam(params: gs_params, frame: Frame, fwd: Optional[Sequence[torch.Tensor]], m: gs_params,
                       v: gs_params, adam: gs_adam, grads_out: Optional[gs_params] = None, g_rgb=None, g_depth=None,
                       g_vis=None, tgt_rgb=None, tgt_depth=None, lambda_d: float = 0.1, lambda_ssim: float = 0.0,
                       stream=None) -> None:
    """Backward and Adam fused (params, m, v updated in place; the gradient written to grads_out if given)."""
    im = None
    if fwd is not None:
        im = gs_images(fwd[0].data_ptr(), fwd[1].data_ptr(), fwd[2].data_ptr())
    l = _loss_struct(g_rgb, g_depth, g_vis, tgt_rgb, tgt_depth, lambda_d, lambda_ssim)
    _check(load().gs_render_bwd_adam(ctypes.byref(params), ctypes.byref(frame.f), ctypes.byref(frame.opts),
                                     ctypes.byref(im) if im is not None else None, ctypes.byref(l), ctypes.byref(m),
                                     ctypes.byref(v), ctypes.byref(adam),
                                     ctypes.byref(grads_out) if grads_out is not None else None, _stream(stream)),
           "gs_render_bwd_adam")


def gs_ssim(frame: Frame, rgb: torch.Tensor, tgt_rgb: torch.Tensor, lambda_ssim: float, g_rgb: torch.Tensor,
            loss_out: torch.Tensor, stream=None) -> None:
    """SSIM term of the frame's views: its image gradient written to g_rgb, its value to loss_out[0] (64 floats)."""
    if loss_out.numel() < 64 or loss_out.dtype != torch.float32 or not loss_out.is_cuda:
        raise ValueError("loss_out must be a float32 CUDA tensor of at least 64 elements")
    _check(load().gs_ssim(frame.cams_host, frame.cams_dev.data_ptr(), frame.n_views, _ptr(rgb), _ptr(tgt_rgb),
                          float(lambda_ssim), _ptr(g_rgb), loss_out.data_ptr(), _stream(stream)), "gs_ssim")


def gs_prune(params: gs_params, m: gs_params, v: gs_params, min_opacity: float, out_params: gs_params,
             out_m: gs_params, out_v: gs_params, n_kept: torch.Tensor, stream=None) -> None:
    """Opacity pruning into the out_* arrays; n_kept (int64 CUDA tensor) receives the count kept."""
    scratch = torch.empty(int(load().gs_prune_scratch_bytes(params.n)) // 4 + 64, dtype=torch.int32,
                          device=n_kept.device)
    _check(load().gs_prune(ctypes.byref(params), ctypes.byref(m), ctypes.byref(v), float(min_opacity),
                           ctypes.byref(out_params), ctypes.byref(out_m), ctypes.byref(out_v), n_kept.data_ptr(),
                           scratch.data_ptr(), _stream(stream)), "gs_prune")


def gs_expand(params: gs_params, m: gs_params, v: gs_params, n_old: int, points: torch.Tensor,
              colours: torch.Tensor, cam, vis: torch.Tensor, opts: gs_expand_opts, n_added: torch.Tensor,
              stream=None) -> None:
    """Map expansion: accepted points appended as rows n_old.. of params, m, v; n_added (int64 CUDA) the count."""
    M = int(points.shape[0])
    for t in (points, colours, vis):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError("points, colours and vis must be contiguous float32 CUDA tensors")
    c = make_cameras([cam])
    scratch = torch.empty(int(load().gs_expand_scratch_bytes(n_old, M)) // 4 + 64, dtype=torch.int32,
                          device=points.device)
    _check(load().gs_expand(ctypes.byref(params), ctypes.byref(m), ctypes.byref(v), int(n_old), points.data_ptr(),
                            colours.data_ptr(), M, c, vis.data_ptr(), ctypes.byref(opts), n_added.data_ptr(),
                            scratch.data_ptr(), _stream(stream)), "gs_expand")


def gs_spatial_order(params: gs_params, m: gs_params, v: gs_params, out_params: gs_params, out_m: gs_params,
                     out_v: gs_params, perm: Optional[torch.Tensor] = None, stream=None) -> None:
    """Rows of params, m, v in Morton order of the means into the out_* arrays; perm (int32 CUDA, [n]) optional."""
    scratch = torch.empty(int(load().gs_spatial_order_scratch_bytes(params.n)) // 4 + 64, dtype=torch.int32,
                          device="cuda")
    _check(load().gs_spatial_order(ctypes.byref(params), ctypes.byref(m), ctypes.byref(v), ctypes.byref(out_params),
                                   ctypes.byref(out_m), ctypes.byref(out_v),
                                   perm.data_ptr() if perm is not None else None, scratch.data_ptr(),
                                   _stream(stream)), "gs_spatial_order")


def gs_read_counters(frame: Frame, stream=None):
    n = c_i64(0)
    fl = c_i32(0)
    _check(load().gs_read_counters(ctypes.byref(frame.f), ctypes.byref(n), ctypes.byref(fl), _stream(stream)),
           "gs_read_counters")
    return int(n.value), int(fl.value)


def gs_sort_pairs(keys: torch.Tensor, vals: torch.Tensor, key_bits: int, stream=None) -> None:
    """Sort int64 (used as uint64) keys with int32 values in place."""
    n = keys.numel()
    kt = torch.empty_like(keys)
    vt = torch.empty_like(vals)
    scratch = torch.empty(int(load().gs_sort_scratch_ints(n)) + 64, dtype=torch.int32, device=keys.device)
    _check(load().gs_sort_pairs(keys.data_ptr(), vals.data_ptr(), kt.data_ptr(), vt.data_ptr(), n, int(key_bits),
                                scratch.data_ptr(), _stream(stream)), "gs_sort_pairs")


def gs_sort_static_max() -> int:
    return int(load().gs_sort_static_max())


def gs_sort_pairs_static(keys: torch.Tensor, vals: torch.Tensor, key_bits: int, stream=None) -> None:
    """The same sort in place with the library's static scratch array (allocates nothing)."""
    if not (keys.is_cuda and keys.dtype == torch.int64 and keys.is_contiguous() and vals.dtype == torch.int32
            and vals.is_contiguous() and vals.numel() == keys.numel()):
        raise ValueError("keys must be contiguous int64 and vals contiguous int32 CUDA tensors of equal length")
    _check(load().gs_sort_pairs_static(keys.data_ptr(), vals.data_ptr(), keys.numel(), int(key_bits),
                                       _stream(stream)), "gs_sort_pairs_static")


# --------------------------------------------------------------------------- frame views (torch, zero-copy)
def frame_tensor(frame: Frame, field: str, count: int, dtype: torch.dtype) -> torch.Tensor:
    """A torch view of a carved frame array (for tests and diagnostics)."""
    if field in ("keys", "vals"):
        raise ValueError("use sorted_keys / sorted_vals")
    addr = getattr(frame.f, field)
    off = addr - frame.block.data_ptr()
    nbytes = count * torch.tensor([], dtype=dtype).element_size()
    return frame.block[off:off + nbytes].view(dtype)


def sorted_pairs(frame: Frame, count: int):
    """The binned instances: (global tile id of each, as int32; record id of each), in sorted order."""
    i = frame.sorted_index
    koff = frame.f.keys[i] - frame.block.data_ptr()
    voff = frame.f.vals[i] - frame.block.data_ptr()
    k = frame.block[koff:koff + 4 * count].view(torch.int32)
    v = frame.block[voff:voff + 4 * count].view(torch.int32)
    return k, v
