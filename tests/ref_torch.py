"""Dense float64 torch renderer, used only to pin the oracle's analytic gradient.

It evaluates every Gaussian at every pixel (no tiles, no bounding boxes, no
sort keys) in plain torch ops and lets autograd differentiate the loss.  The
discrete decisions (culls, alpha skip below 1/255, stop before T < 1e-4, the
0.99 clamp, the colour clamp) are taken on detached values, exactly as the
method defines them (LVI-GS Section III-B, eqs. Cp, Dp, Vp and alpha), so that
autograd sees the same piecewise-smooth function as the analytic backward.
Written independently of oracle/oracle.cpp; for tiny scenes only.
"""
from __future__ import annotations

import math

import torch

_C0 = 0.28209479177387814
_C1 = 0.4886025119029199
_C2 = (1.0925484305920792, 1.0925484305920792, 0.31539156525252005, 1.0925484305920792, 0.5462742152960396)
_C3 = (0.5900435899266435, 2.890611442640554, 0.4570457994644658, 0.3731763325901154, 0.4570457994644658,
       1.445305721320277, 0.5900435899266435)


def sh_cartesian(d: torch.Tensor, deg: int) -> torch.Tensor:
    """Real orthonormal SH (no Condon-Shortley phase in the real form) at unit directions d [G,3] -> [G,K]."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    Y = [torch.full_like(x, _C0)]
    if deg >= 1:
        Y += [_C1 * y, _C1 * z, _C1 * x]
    if deg >= 2:
        Y += [_C2[0] * x * y, _C2[1] * y * z, _C2[2] * (2 * z * z - x * x - y * y), _C2[3] * x * z,
              _C2[4] * (x * x - y * y)]
    if deg >= 3:
        Y += [_C3[0] * y * (3 * x * x - y * y), _C3[1] * x * y * z, _C3[2] * y * (4 * z * z - x * x - y * y),
              _C3[3] * z * (2 * z * z - 3 * x * x - 3 * y * y), _C3[4] * x * (4 * z * z - x * x - y * y),
              _C3[5] * z * (x * x - y * y), _C3[6] * x * (x * x - 3 * y * y)]
    return torch.stack(Y, dim=1)


def _rot(q: torch.Tensor) -> torch.Tensor:
    q = q / q.norm(dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1),
    ], 1)


def render(means, log_scales, quats, opacity, sh, sh_degree, cams, near=0.2, guard=1.3, lowpass=0.3,
           alpha_min=1 / 255, alpha_max=0.99, t_min=1e-4):
    """Returns per view (rgb [3,H,W], depth [H,W], vis [H,W])."""
    outs = []
    o_all = torch.sigmoid(opacity)
    S = torch.exp(log_scales)
    Rq = _rot(quats)
    M = Rq * S[:, None, :]
    Sig = M @ M.transpose(1, 2)
    for cam in cams:
        R = torch.tensor(cam.R, dtype=torch.float64)
        T = torch.tensor(cam.T, dtype=torch.float64)
        t = means @ R.T + T
        tx, ty, tz = t[:, 0], t[:, 1], t[:, 2]
        with torch.no_grad():
            u = cam.fx * tx / tz + cam.cx
            v = cam.fy * ty / tz + cam.cy
            gx, gy = (guard - 1) * 0.5 * cam.width, (guard - 1) * 0.5 * cam.height
            keep = (tz >= near) & (u >= -gx) & (u <= cam.width + gx) & (v >= -gy) & (v <= cam.height + gy)
            keep &= o_all >= alpha_min
        idx = torch.nonzero(keep).flatten()
        W_, H_ = cam.width, cam.height
        ys, xs = torch.meshgrid(torch.arange(H_, dtype=torch.float64) + 0.5,
                                torch.arange(W_, dtype=torch.float64) + 0.5, indexing="ij")
        C = torch.zeros(3, H_, W_, dtype=torch.float64)
        D = torch.zeros(H_, W_, dtype=torch.float64)
        Vv = torch.zeros(H_, W_, dtype=torch.float64)
        if idx.numel() == 0:
            outs.append((C, D, Vv))
            continue
        tx, ty, tz = tx[idx], ty[idx], tz[idx]
        mx = cam.fx * tx / tz + cam.cx
        my = cam.fy * ty / tz + cam.cy
        zeros = torch.zeros_like(tz)
        J = torch.stack([torch.stack([cam.fx / tz, zeros, -cam.fx * tx / tz ** 2], 1),
                         torch.stack([zeros, cam.fy / tz, -cam.fy * ty / tz ** 2], 1)], 1)
        T2 = J @ R
        SI = T2 @ Sig[idx] @ T2.transpose(1, 2)
        A = SI[:, 0, 0] + lowpass
        B = SI[:, 0, 1]
        Cc = SI[:, 1, 1] + lowpass
        det = A * Cc - B * B
        ca, cb, cc = Cc / det, -B / det, A / det
        d = means[idx] - torch.tensor(cam.campos, dtype=torch.float64)
        d = d / d.norm(dim=1, keepdim=True)
        Y = sh_cartesian(d, sh_degree)
        pre = torch.einsum("gk,gkc->gc", Y, sh[idx]) + 0.5
        rgb = torch.where(pre.detach() >= 0, pre, torch.zeros_like(pre))
        o = o_all[idx]
        order = torch.argsort(tz.detach().float(), stable=True)
        T = torch.ones(H_, W_, dtype=torch.float64)
        active = torch.ones(H_, W_, dtype=torch.bool)
        for j in order.tolist():
            dx = mx[j] - xs
            dy = my[j] - ys
            power = -0.5 * (ca[j] * dx * dx + cc[j] * dy * dy) - cb[j] * dx * dy
            oG = o[j] * torch.exp(power)
            alpha = torch.where(oG.detach() > alpha_max, torch.full_like(oG, alpha_max), oG)
            with torch.no_grad():
                ok = active & (power <= 0) & (alpha >= alpha_min)
                Tn = T * (1 - alpha)
                stop = ok & (Tn < t_min)
                use = ok & ~stop
                active = active & ~stop
            w = torch.where(use, alpha * T, torch.zeros_like(alpha))
            C = C + w[None] * rgb[j][:, None, None]
            D = D + w * tz[j]
            Vv = Vv + w
            T = torch.where(use, T * (1 - alpha), T)
        outs.append((C, D, Vv))
    return outs


def l1_loss(outs, cams, tgt_rgb, tgt_depth, lambda_d=0.1):
    """sum_v w_v [ mean |C - I| + lambda_d mean_valid |D - D_lidar| ] (eqs. L, Lc, Ld)."""
    L = 0.0
    off = 0
    for (C, D, _), cam in zip(outs, cams):
        P = cam.width * cam.height
        I = torch.as_tensor(tgt_rgb[3 * off:3 * off + 3 * P], dtype=torch.float64).reshape(3, cam.height, cam.width)
        Dt = torch.as_tensor(tgt_depth[off:off + P], dtype=torch.float64).reshape(cam.height, cam.width)
        L = L + cam.weight * (C - I).abs().sum() / (3 * P)
        valid = Dt > 0
        if valid.any():
            L = L + cam.weight * lambda_d * (D - Dt).abs()[valid].sum() / valid.sum()
        off += P
    return L


def ssim_loss(outs, cams, tgt_rgb, lam):
    """sum_v w_v lam (1 - mean SSIM_v): SSIM per channel with an 11 x 11 Gaussian window (sigma 1.5, summing
    to 1) applied by a zero-padded 2D convolution, C1 = 0.01^2, C2 = 0.03^2 (eq. Lc with the 3DGS readings)."""
    g = torch.exp(-torch.arange(-5, 6, dtype=torch.float64) ** 2 / (2 * 1.5 ** 2))
    g = g / g.sum()
    win = torch.outer(g, g)[None, None]
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    L = 0.0
    off = 0
    for (C, _, _), cam in zip(outs, cams):
        P = cam.width * cam.height
        I = torch.as_tensor(tgt_rgb[3 * off:3 * off + 3 * P], dtype=torch.float64).reshape(3, 1, cam.height, cam.width)
        X = C.reshape(3, 1, cam.height, cam.width)
        f = lambda z: torch.nn.functional.conv2d(z, win, padding=5)
        mx, my = f(X), f(I)
        sx = f(X * X) - mx * mx
        sy = f(I * I) - my * my
        sxy = f(X * I) - mx * my
        S = (2 * mx * my + c1) * (2 * sxy + c2) / ((mx * mx + my * my + c1) * (sx + sy + c2))
        L = L + cam.weight * lam * (1.0 - S.mean())
        off += P
    return L


def photometric_loss(outs, cams, tgt_rgb, tgt_depth, lambda_d=0.1, lambda_ssim=0.0):
    """sum_v w_v [ (1 - lambda_ssim) mean |C - I| + lambda_ssim (1 - SSIM_v) + lambda_d mean_valid |D - D_lidar| ]."""
    L = 0.0
    off = 0
    for (C, D, _), cam in zip(outs, cams):
        P = cam.width * cam.height
        I = torch.as_tensor(tgt_rgb[3 * off:3 * off + 3 * P], dtype=torch.float64).reshape(3, cam.height, cam.width)
        Dt = torch.as_tensor(tgt_depth[off:off + P], dtype=torch.float64).reshape(cam.height, cam.width)
        L = L + cam.weight * (1.0 - lambda_ssim) * (C - I).abs().sum() / (3 * P)
        valid = Dt > 0
        if valid.any():
            L = L + cam.weight * lambda_d * (D - Dt).abs()[valid].sum() / valid.sum()
        off += P
    return L + ssim_loss(outs, cams, tgt_rgb, lambda_ssim)
