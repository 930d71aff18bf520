"""One optimisation iteration of LVI-GS mapping over a set of views (keyframes x pyramid levels).

Section III-D renders every pyramid level of a keyframe and compares it with the down-sampled targets;
Section III-E sums an L1 colour and an L1 LiDAR-depth loss and optimises the Gaussians.  An iteration
here is: every view forward and backward with that loss, then one Adam step over all parameters.

PlainStep  : the per-view launch sequence (project, bin with a host-synchronised instance count, render,
             backward with the loss against the view's targets), then Adam.
BatchedStep: all views in one frame - one projection launch that reads every Gaussian once, one binning
             over global (view, tile) keys sized by a capacity (no host synchronisation), one fused
             forward + loss + backward compositing launch group over every tile of every view, and the
             projection backward fused with Adam - captured once as a HIP graph and replayed.
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import binding as B

PARAM_KEYS = ("means", "log_scales", "quats", "opacity", "sh")

# Learning rates per group (means, log-scales, rotations, opacity, SH degree 0, SH degree >= 1).  The
# paper does not state them; these follow common 3DGS practice.
DEFAULT_LR = (1.6e-4, 5e-3, 1e-3, 2.5e-2, 2.5e-3, 1.25e-4)


class GaussianModel:
    """Gaussian parameters on the device plus their gradients and Adam moments."""

    def __init__(self, params: Dict[str, np.ndarray], sh_degree: int, device: str = "cuda",
                 lr: Sequence[float] = DEFAULT_LR, betas=(0.9, 0.999), eps: float = 1e-15):
        self.sh_degree = int(sh_degree)
        self.p = {k: torch.as_tensor(np.ascontiguousarray(params[k]), dtype=torch.float32).to(device)
                  for k in PARAM_KEYS}
        self.g = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.m = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.step_count = torch.zeros(1, dtype=torch.int64, device=device)
        self.bias = torch.zeros(4, dtype=torch.float32, device=device)
        self.ps = B.params_struct(self.p, self.sh_degree)
        self.gs = B.params_struct(self.g, self.sh_degree)
        self.ms = B.params_struct(self.m, self.sh_degree)
        self.vs = B.params_struct(self.v, self.sh_degree)
        self.adam = B.gs_adam()
        for i in range(6):
            self.adam.lr[i] = float(lr[i])
        self.adam.beta1, self.adam.beta2, self.adam.eps = float(betas[0]), float(betas[1]), float(eps)
        self.adam.step = self.step_count.data_ptr()
        self.adam.bias = self.bias.data_ptr()

    @property
    def n(self) -> int:
        return int(self.p["means"].shape[0])

    def zero_grad(self) -> None:
        for t in self.g.values():
            t.zero_()

    def adam_step(self, stream=None) -> None:
        B.gs_adam_step(self.ps, self.gs, self.ms, self.vs, self.adam, stream)

    def set_sh_degree(self, degree: int) -> None:
        """Raise (or lower) the SH degree: the coefficients and their Adam moments are re-packed to
        [n, (degree + 1)^2, 3]; coefficients of the new bands start at 0 (with zero moments), so the rendered
        colours do not change.  Frames and steps must be rebuilt (the parameter pointers change)."""
        degree = int(degree)
        if not 0 <= degree <= 3:
            raise ValueError("SH degree must be in [0, 3]")
        K = (degree + 1) ** 2
        for d in (self.p, self.m, self.v):
            old = d["sh"]
            new = torch.zeros((old.shape[0], K, 3), dtype=old.dtype, device=old.device)
            k = min(K, old.shape[1])
            new[:, :k] = old[:, :k]
            d["sh"] = new
        self.g["sh"] = torch.zeros_like(self.p["sh"])
        self.sh_degree = degree
        self.ps = B.params_struct(self.p, degree)
        self.gs = B.params_struct(self.g, degree)
        self.ms = B.params_struct(self.m, degree)
        self.vs = B.params_struct(self.v, degree)

    def expand(self, points, colours, cam, vis: torch.Tensor, tau_alpha: float = 0.5, voxel: float = 0.1,
               cap: int = 1, knn_cell: float = 0.5, init_opacity: float = 0.1, near_z: float = 0.2) -> int:
        """Append a keyframe's LiDAR points as new Gaussians (visibility filter against the keyframe's rendered
        visibility `vis` [H*W], voxel cap against the map, neighbour-spacing initialisation; gs_expand).  Returns
        the number added.  Frames and steps must be rebuilt (the count changes)."""
        dev = self.p["means"].device
        pts = torch.as_tensor(np.ascontiguousarray(points, np.float32)).to(dev)
        rgb = torch.as_tensor(np.ascontiguousarray(colours, np.float32)).to(dev)
        n_old, M = self.n, int(pts.shape[0])
        grown = []
        for d in (self.p, self.m, self.v):
            out = {}
            for k, t in d.items():
                big = torch.zeros((n_old + M,) + tuple(t.shape[1:]), dtype=t.dtype, device=dev)
                big[:n_old] = t
                out[k] = big
            grown.append(out)
        structs = [B.params_struct(d, self.sh_degree) for d in grown]
        n_added = torch.zeros(1, dtype=torch.int64, device=dev)
        o = B.gs_expand_opts(float(tau_alpha), float(near_z), float(voxel), float(knn_cell), float(init_opacity),
                             int(cap))
        B.gs_expand(structs[0], structs[1], structs[2], n_old, pts, rgb, cam, vis.contiguous(), o, n_added)
        k = int(n_added.item())
        self.p, self.m, self.v = ({key: t[:n_old + k] for key, t in d.items()} for d in grown)
        self.g = {key: torch.zeros_like(t) for key, t in self.p.items()}
        self.ps = B.params_struct(self.p, self.sh_degree)
        self.gs = B.params_struct(self.g, self.sh_degree)
        self.ms = B.params_struct(self.m, self.sh_degree)
        self.vs = B.params_struct(self.v, self.sh_degree)
        return k

    def reorder_spatially(self) -> np.ndarray:
        """Store the Gaussians (parameters and moments) in Morton order of their means (gs_spatial_order), a layout
        for locality: a wave of threads then holds neighbouring Gaussians.  Returns the permutation (new row k was
        old row perm[k]).  Frames and steps built before must be rebuilt."""
        out = [{k: torch.empty_like(t) for k, t in d.items()} for d in (self.p, self.m, self.v)]
        structs = [B.params_struct(d, self.sh_degree) for d in out]
        perm = torch.empty(self.n, dtype=torch.int32, device=self.p["means"].device)
        B.gs_spatial_order(self.ps, self.ms, self.vs, structs[0], structs[1], structs[2], perm)
        self.p, self.m, self.v = out
        self.g = {key: torch.zeros_like(t) for key, t in self.p.items()}
        self.ps = B.params_struct(self.p, self.sh_degree)
        self.gs = B.params_struct(self.g, self.sh_degree)
        self.ms = B.params_struct(self.m, self.sh_degree)
        self.vs = B.params_struct(self.v, self.sh_degree)
        return perm.cpu().numpy()

    def set_sparse_adam(self, on: bool = True) -> None:
        """Visible-only Adam in the fused backward (gs_render_bwd_adam): Gaussians seen by no view of the step keep
        their parameters and moments."""
        self.adam.flags = B.GS_ADAM_SPARSE if on else 0

    def prune(self, min_opacity: float) -> int:
        """Drop every Gaussian whose opacity is below min_opacity (parameters and Adam moments compacted on the
        device, order kept); returns the new count.  Frames and steps built for the old count must be rebuilt."""
        dev = self.p["means"].device
        out = [{k: torch.empty_like(t) for k, t in d.items()} for d in (self.p, self.m, self.v)]
        structs = [B.params_struct(d, self.sh_degree) for d in out]
        n_kept = torch.zeros(1, dtype=torch.int64, device=dev)
        B.gs_prune(self.ps, self.ms, self.vs, min_opacity, structs[0], structs[1], structs[2], n_kept)
        k = int(n_kept.item())
        self.p, self.m, self.v = ({key: t[:k] for key, t in d.items()} for d in out)
        self.g = {key: torch.zeros_like(t) for key, t in self.p.items()}
        self.ps = B.params_struct(self.p, self.sh_degree)
        self.gs = B.params_struct(self.g, self.sh_degree)
        self.ms = B.params_struct(self.m, self.sh_degree)
        self.vs = B.params_struct(self.v, self.sh_degree)
        return k

    def state(self) -> Dict[str, torch.Tensor]:
        out = {}
        for k in PARAM_KEYS:
            out[k] = self.p[k].detach().cpu()
            out["m_" + k] = self.m[k].detach().cpu()
            out["v_" + k] = self.v[k].detach().cpu()
        out["step"] = self.step_count.detach().cpu()
        return out

    def load_state(self, st: Dict[str, torch.Tensor]) -> None:
        for k in PARAM_KEYS:
            self.p[k].copy_(st[k])
            self.m[k].copy_(st["m_" + k])
            self.v[k].copy_(st["v_" + k])
        self.step_count.copy_(st["step"])


def _targets_for(cams, tgt_rgb: np.ndarray, tgt_depth: np.ndarray, device: str):
    """Per-view target tensors cut from the concatenated arrays."""
    out, off = [], 0
    for c in cams:
        P = c.width * c.height
        out.append((torch.as_tensor(tgt_rgb[3 * off:3 * off + 3 * P]).to(device).contiguous(),
                    torch.as_tensor(tgt_depth[off:off + P]).to(device).contiguous()))
        off += P
    return out


class PlainStep:
    """The per-view launch sequence of the library calls (one frame per view)."""

    def __init__(self, model: GaussianModel, cams: Sequence, tgt_rgb: np.ndarray, tgt_depth: np.ndarray,
                 lambda_d: float = 0.1, opts: Optional[B.gs_opts] = None, device: str = "cuda",
                 lambda_ssim: float = 0.0):
        self.model = model
        self.cams = list(cams)
        self.opts = opts if opts is not None else B.default_opts()
        self.lambda_d = float(lambda_d)
        self.lambda_ssim = float(lambda_ssim)
        self.frames = [B.Frame(model.n, [c], self.opts, None, device) for c in self.cams]
        self.images = [f.empty_images(device) for f in self.frames]
        self.targets = _targets_for(self.cams, tgt_rgb, tgt_depth, device)
        self.device = device
        if self.lambda_ssim > 0:
            self.g_ssim = [torch.empty(3 * c.width * c.height, device=device) for c in self.cams]
            self.ssim_loss = [torch.zeros(64, device=device) for _ in self.cams]

    def run(self) -> None:
        m = self.model
        m.zero_grad()
        for v, fr in enumerate(self.frames):
            while True:
                B.gs_project(m.ps, fr)
                n = B.gs_bin_tiles(fr, sync_count=True)
                if n <= fr.capacity:
                    break
                fr = self.frames[v] = B.Frame(m.n, [self.cams[v]], self.opts, int(n * 1.25) + 1024, self.device)
                self.images[v] = fr.empty_images(self.device)
            rgb, depth, vis = self.images[v]
            B.gs_render_fwd(fr, rgb, depth, vis)
            tr, td = self.targets[v]
            g_ssim = None
            if self.lambda_ssim > 0:
                g_ssim = self.g_ssim[v]
                B.gs_ssim(fr, rgb, tr, self.lambda_ssim, g_ssim, self.ssim_loss[v])
            B.gs_render_bwd(m.ps, fr, (rgb, depth, vis), m.gs, g_rgb=g_ssim, tgt_rgb=tr, tgt_depth=td,
                            lambda_d=self.lambda_d, lambda_ssim=self.lambda_ssim)
        m.adam_step()

    def loss(self) -> float:
        """Sum of the per-view loss values of the last run (synchronises)."""
        tot = 0.0
        for v, fr in enumerate(self.frames):
            t = B.frame_tensor(fr, "loss", 1, torch.float32)
            tot += float(t.item())
            if self.lambda_ssim > 0:
                tot += float(self.ssim_loss[v][0].item())
        return tot


class BatchedStep:
    """All views in one frame: projection, binning, the fused forward + loss + backward compositing, and the
    projection backward fused with Adam (one pass per Gaussian, no gradient buffer), captured as a HIP graph.

    Capacity: the instance count is measured once and given `headroom`.  A replay whose instances exceed the
    capacity leaves the model untouched (the library skips the Adam step of an overflowed frame).  run() reads
    each replay's counters one replay late (no stall: the next replay is already queued); on an overflow it
    re-plans the capacity at `regrow` times the largest count seen, re-captures the graph and runs the skipped
    steps again, so the sequence of parameter updates is the one a large enough frame would have produced.
    keep_grads: also write each step's gradient to model.g (for inspection; costs one extra write).
    lambda_ssim > 0 adds the SSIM term of eq. Lc: its window couples neighbouring pixels, so the step then renders
    the images (gs_render_fwd), forms the SSIM gradient image (gs_ssim) and runs the image-fed backward with it,
    instead of the fused forward + backward that needs no image."""

    def __init__(self, model: GaussianModel, cams: Sequence, tgt_rgb: np.ndarray, tgt_depth: np.ndarray,
                 lambda_d: float = 0.1, opts: Optional[B.gs_opts] = None, device: str = "cuda",
                 capacity: Optional[int] = None, headroom: float = 1.25, regrow: float = 1.5,
                 keep_grads: bool = False, lambda_ssim: float = 0.0):
        self.model = model
        self.cams = list(cams)
        self.opts = opts if opts is not None else B.default_opts()
        self.lambda_d = float(lambda_d)
        self.lambda_ssim = float(lambda_ssim)
        self.device = device
        self.headroom = headroom
        self.regrow = regrow
        self.keep_grads = keep_grads
        self.tgt_rgb = torch.as_tensor(tgt_rgb).to(device).contiguous()
        self.tgt_depth = torch.as_tensor(tgt_depth).to(device).contiguous()
        if capacity is None:
            capacity = self._measure_capacity()
        self.frame = B.Frame(model.n, self.cams, self.opts, capacity, device)
        self._ssim_buffers()
        self.graph: Optional[torch.cuda.CUDAGraph] = None
        self.replans = 0
        self.steps_redone = 0
        self._host = torch.zeros((2, 2), dtype=torch.int32, pin_memory=True)
        self._pending: List = []  # (event, slot) of replays whose counters have not been checked
        self._slot = 0

    def _measure_capacity(self) -> int:
        probe = B.Frame(self.model.n, self.cams, self.opts, max(1 << 20, 8 * self.model.n), self.device)
        B.gs_project(self.model.ps, probe)
        n = B.gs_bin_tiles(probe, sync_count=True)
        del probe
        return int(n * self.headroom) + 4096

    def _ssim_buffers(self) -> None:
        if self.lambda_ssim > 0:
            self.images = self.frame.empty_images(self.device)
            self.g_ssim = torch.empty_like(self.images[0])
            self.ssim_loss = torch.zeros(64, device=self.device)

    def _body(self, stream=None) -> None:
        m = self.model
        B.gs_project(m.ps, self.frame, stream=stream)
        B.gs_bin_tiles(self.frame, sync_count=False, stream=stream)
        grads = m.gs if self.keep_grads else None
        if self.lambda_ssim > 0:
            rgb, depth, vis = self.images
            B.gs_render_fwd(self.frame, rgb, depth, vis, stream=stream)
            B.gs_ssim(self.frame, rgb, self.tgt_rgb, self.lambda_ssim, self.g_ssim, self.ssim_loss, stream=stream)
            B.gs_render_bwd_adam(m.ps, self.frame, self.images, m.ms, m.vs, m.adam, grads, g_rgb=self.g_ssim,
                                 tgt_rgb=self.tgt_rgb, tgt_depth=self.tgt_depth, lambda_d=self.lambda_d,
                                 lambda_ssim=self.lambda_ssim, stream=stream)
        else:
            B.gs_render_bwd_adam(m.ps, self.frame, None, m.ms, m.vs, m.adam, grads, tgt_rgb=self.tgt_rgb,
                                 tgt_depth=self.tgt_depth, lambda_d=self.lambda_d, stream=stream)

    def run_eager(self) -> None:
        """One step without the graph (the same library calls); the overflow is checked at once."""
        self._body()
        n, fl = B.gs_read_counters(self.frame)
        if fl & B.GS_FLAG_INSTANCE_OVERFLOW:
            self._replan(n)
            self.steps_redone += 1
            self.run_eager()

    def capture(self) -> None:
        """Capture the step as a graph.  The warm-up run that precedes the capture is undone, so capturing does
        not advance the model."""
        m = self.model
        snap = [t.clone() for d in (m.p, m.m, m.v) for t in d.values()] + [m.step_count.clone(), m.bias.clone()]
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self._body(s)  # warm-up on the side stream (not captured)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        dst = [t for d in (m.p, m.m, m.v) for t in d.values()] + [m.step_count, m.bias]
        for a, b in zip(dst, snap):
            a.copy_(b)
        torch.cuda.synchronize()
        del snap
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._body()
        self.graph = g

    def _replay(self) -> None:
        self.graph.replay()
        slot = self._slot
        self._slot ^= 1
        self._host[slot].copy_(B.frame_tensor(self.frame, "counters", 2, torch.int32), non_blocking=True)
        ev = torch.cuda.Event()
        ev.record()
        self._pending.append((ev, slot))

    def run(self) -> None:
        """One step (a graph replay); checks the previous replay's counters."""
        if self.graph is None:
            self.capture()
        self._replay()
        if len(self._pending) > 1:
            self._check(self._pending.pop(0))

    def finish(self) -> None:
        """Wait for the queued replays and handle an overflow among them."""
        while self._pending:
            self._check(self._pending.pop(0))

    def _check(self, item) -> None:
        ev, slot = item
        ev.synchronize()
        n, fl = (int(x) for x in self._host[slot].tolist())
        if not fl & B.GS_FLAG_INSTANCE_OVERFLOW:
            return
        # this replay (and possibly the queued ones) skipped its step: re-plan, re-capture, run them again
        torch.cuda.synchronize()
        lost, n_max = 1, n
        for ev2, slot2 in self._pending:
            n2, fl2 = (int(x) for x in self._host[slot2].tolist())
            n_max = max(n_max, n2)
            lost += 1 if fl2 & B.GS_FLAG_INSTANCE_OVERFLOW else 0
        self._pending.clear()
        self._replan(n_max)
        self.steps_redone += lost
        for _ in range(lost):
            self.run()
        self.finish()

    def _replan(self, n_needed: int) -> None:
        self.replans += 1
        cap = int(n_needed * self.regrow) + 4096
        self.graph = None
        self.frame = B.Frame(self.model.n, self.cams, self.opts, cap, self.device)
        self._ssim_buffers()

    def set_weights(self, weights: Sequence[float]) -> None:
        """New loss weights w_v of the frame's views (a negative weight switches a view off: nothing is projected
        into it).  The device camera table is rewritten in stream order, so a captured graph uses the new
        weights from its next replay on; frame layout and capacity are unchanged."""
        if len(weights) != self.frame.n_views:
            raise ValueError("one weight per view")
        for c, w in zip(self.frame.cams_host, weights):
            c.loss_weight = float(w)
        raw = torch.frombuffer(bytearray(bytes(self.frame.cams_host)), dtype=torch.uint8)
        self.frame.cams_dev.copy_(raw)

    def flags(self) -> int:
        _, fl = B.gs_read_counters(self.frame)
        return fl

    def overflowed(self) -> bool:
        return bool(self.flags() & B.GS_FLAG_INSTANCE_OVERFLOW)

    def loss(self) -> float:
        L = float(B.frame_tensor(self.frame, "loss", 1, torch.float32).item())
        if self.lambda_ssim > 0:
            L += float(self.ssim_loss[0].item())
        return L

    def n_instances(self) -> int:
        n, _ = B.gs_read_counters(self.frame)
        return n


class Mapper:
    """LVI-GS mapping iterations driven by the training policies (Sections III-C, III-D, III-E) on one captured
    batched step.

    The frame holds every keyframe's pyramid levels as views.  Keyframes arrive one every `arrive_every`
    iterations (the front-end's keyframe stream); a DelayBuffer holds each one back until `delay` newer ones have
    arrived, then it joins the KeyframeQueue.  Each iteration the queue picks `batch` keyframes (a new one is
    optimised once first; afterwards random picks; capped keyframes retire), the PyramidSchedule picks each one's
    level from its own iteration count, every other view is switched off (negative weight), and the graph is
    replayed.  The SH degree follows the SHSchedule (re-pack and re-capture at each change), and every
    `prune_every` iterations Gaussians below `min_opacity` are pruned (re-capture)."""

    def __init__(self, model: GaussianModel, keyframes: Sequence[Sequence], tgt_rgb: np.ndarray,
                 tgt_depth: np.ndarray, queue=None, delay=None, pyramid=None, sh=None, arrive_every: int = 1,
                 prune_every: int = 0, min_opacity: float = 0.005, opts: Optional[B.gs_opts] = None,
                 lambda_ssim: float = 0.0, device: str = "cuda"):
        from .schedule import DelayBuffer, KeyframeQueue, PyramidSchedule, SHSchedule

        self.model = model
        self.keyframes = [list(levels) for levels in keyframes]  # per keyframe: its cameras, finest level first
        self.cams = [c for levels in self.keyframes for c in levels]
        self.view_of = []
        v = 0
        for levels in self.keyframes:
            self.view_of.append(list(range(v, v + len(levels))))
            v += len(levels)
        self.tgt_rgb, self.tgt_depth = tgt_rgb, tgt_depth
        self.queue = queue or KeyframeQueue()
        self.delay = delay or DelayBuffer()
        self.pyramid = pyramid or PyramidSchedule(levels=len(self.keyframes[0]))
        self.sh = sh
        self.arrive_every = max(1, int(arrive_every))
        self.prune_every = int(prune_every)
        self.min_opacity = float(min_opacity)
        self.opts = opts
        self.lambda_ssim = lambda_ssim
        self.device = device
        self.it = 0
        self.arrived = 0
        self.history: List[Dict] = []
        if self.sh is not None and self.model.sh_degree != self.sh.degree(0):
            self.model.set_sh_degree(self.sh.degree(0))
        self._build()

    def _build(self) -> None:
        self.step = BatchedStep(self.model, self.cams, self.tgt_rgb, self.tgt_depth, opts=self.opts,
                                device=self.device, lambda_ssim=self.lambda_ssim)

    def weights_for(self, picked: Sequence[int]) -> List[float]:
        w = [-1.0] * len(self.cams)
        for k in picked:
            for lv, wl in enumerate(self.pyramid.weights(self.queue.counts[k] - 1)):
                if wl > 0:
                    w[self.view_of[k][lv]] = wl / len(picked)
        return w

    def iterate(self) -> Dict:
        """One mapping iteration; returns what it did (keyframes, levels, loss of the previous replay)."""
        if self.it % self.arrive_every == 0 and self.arrived < len(self.keyframes):
            for k in self.delay.push(self.arrived):
                self.queue.add(k)
            self.arrived += 1
            if self.arrived == len(self.keyframes):
                for k in self.delay.flush():
                    self.queue.add(k)
        rebuild = False
        if self.sh is not None and self.sh.degree(self.it) != self.model.sh_degree:
            self.step.finish()
            self.model.set_sh_degree(self.sh.degree(self.it))
            rebuild = True
        if self.prune_every and self.it > 0 and self.it % self.prune_every == 0:
            self.step.finish()
            self.model.prune(self.min_opacity)
            rebuild = True
        if rebuild:
            self._build()
        picked = self.queue.select()
        rec = dict(it=self.it, keyframes=picked, n=self.model.n, sh_degree=self.model.sh_degree)
        if picked:
            self.step.set_weights(self.weights_for(picked))
            self.step.run()
            rec["levels"] = [self.pyramid.level(self.queue.counts[k] - 1) for k in picked]
        self.history.append(rec)
        self.it += 1
        return rec
