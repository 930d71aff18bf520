"""torch.autograd.Function around the HIP rasteriser.

forward(means, log_scales, quats, opacity, sh) -> (rgb, depth, vis) for every view of a Rasterizer,
backward(g_rgb, g_depth, g_vis) -> gradients of the five parameter groups.  All work runs in libgs; the
backward needs only the forward's output images (no per-pixel state is stored).

A Rasterizer's frame holds the binning of its latest forward.  Each forward records the frame's generation;
a backward whose forward is no longer the latest one (another forward through the same Rasterizer came in
between) projects and bins its own saved parameters again before the compositing backward, so that its
gradient never mixes two forwards' binnings.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import binding as B


class Rasterizer:
    """Owns a frame for a fixed set of views and grows its instance capacity when it overflows."""

    def __init__(self, n: int, cams: Sequence, sh_degree: int, opts: Optional[B.gs_opts] = None,
                 capacity: Optional[int] = None, device: str = "cuda"):
        self.cams = list(cams)
        self.n = int(n)
        self.sh_degree = int(sh_degree)
        self.opts = opts if opts is not None else B.default_opts()
        self.device = device
        self.frame = B.Frame(self.n, self.cams, self.opts, capacity, device)
        self.n_instances = 0
        self.generation = 0  # incremented by every projection + binning into the frame

    def project_and_bin(self, ps: B.gs_params, stream=None) -> int:
        """Project and bin with a synchronised instance count; re-plan the frame on overflow."""
        self.generation += 1
        while True:
            B.gs_project(ps, self.frame, stream=stream)
            n = B.gs_bin_tiles(self.frame, sync_count=True, stream=stream)
            if n <= self.frame.capacity:
                self.n_instances = n
                return n
            self.frame = B.Frame(self.n, self.cams, self.opts, int(n * 1.25) + 1024, self.device)

    def slices(self, rgb, depth, vis):
        """Per-view (rgb [3,H,W], depth [H,W], vis [H,W]) views of concatenated images."""
        out = []
        for v in range(len(self.cams)):
            off, P, H, W = self.frame.view_slices(v)
            out.append((rgb[3 * off:3 * off + 3 * P].view(3, H, W), depth[off:off + P].view(H, W),
                        vis[off:off + P].view(H, W)))
        return out


class GaussianRasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity, sh, rast: Rasterizer):
        params = dict(means=means.contiguous(), log_scales=log_scales.contiguous(), quats=quats.contiguous(),
                      opacity=opacity.contiguous(), sh=sh.contiguous())
        ps = B.params_struct(params, rast.sh_degree)
        rast.project_and_bin(ps)
        rgb, depth, vis = rast.frame.empty_images(rast.device)
        B.gs_render_fwd(rast.frame, rgb, depth, vis)
        ctx.rast = rast
        ctx.generation = rast.generation
        ctx.save_for_backward(params["means"], params["log_scales"], params["quats"], params["opacity"],
                              params["sh"], rgb, depth, vis)
        return rgb, depth, vis

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_vis):
        means, log_scales, quats, opacity, sh, rgb, depth, vis = ctx.saved_tensors
        rast = ctx.rast
        params = dict(means=means, log_scales=log_scales, quats=quats, opacity=opacity, sh=sh)
        ps = B.params_struct(params, rast.sh_degree)
        grads = {k: torch.zeros_like(v) for k, v in params.items()}
        gs = B.params_struct(grads, rast.sh_degree)
        if rast.generation != ctx.generation:
            # another forward re-binned the frame since ours: bin our parameters again (same records, same
            # order: projection and binning are deterministic)
            rast.project_and_bin(ps)
        ctx.generation = rast.generation
        cont = lambda t: None if t is None else t.contiguous()
        B.gs_render_bwd(ps, rast.frame, (rgb, depth, vis), gs, g_rgb=cont(g_rgb), g_depth=cont(g_depth),
                        g_vis=cont(g_vis))
        return grads["means"], grads["log_scales"], grads["quats"], grads["opacity"], grads["sh"], None


def rasterize(means, log_scales, quats, opacity, sh, rast: Rasterizer):
    return GaussianRasterize.apply(means, log_scales, quats, opacity, sh, rast)


class SSIMTerm(torch.autograd.Function):
    """The SSIM term of eq. Lc, lambda sum_v w_v (1 - mean SSIM_v), of a Rasterizer's concatenated colour images
    against targets of the same layout; gs_ssim forms its value and image gradient in one pass."""

    @staticmethod
    def forward(ctx, rgb, tgt_rgb, rast: Rasterizer, lam: float):
        rgb = rgb.contiguous()
        g = torch.empty_like(rgb)
        loss = torch.zeros(64, device=rgb.device, dtype=torch.float32)
        B.gs_ssim(rast.frame, rgb, tgt_rgb.contiguous(), lam, g, loss)
        ctx.save_for_backward(g)
        return loss[0].clone()

    @staticmethod
    def backward(ctx, g_out):
        (g,) = ctx.saved_tensors
        return g * g_out, None, None, None


def ssim_term(rgb, tgt_rgb, rast: Rasterizer, lam: float = 0.2):
    return SSIMTerm.apply(rgb, tgt_rgb, rast, lam)
