"""Pins of the oracle's SSIM term (eq. Lc: the SSIM error of the rendered colour image), no GPU needed.

Readings (the paper gives no SSIM parameters): 11 x 11 Gaussian window of standard deviation 1.5 px summing
to 1, zero padding at the image borders, C1 = 0.01^2, C2 = 0.03^2, mean over channels and pixels,
L_ssim = 1 - mean.  Each pin is fixed by the definition or by closed forms, not by the oracle's own code.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2411_02703_amd import scenes

C1, C2 = 0.01 ** 2, 0.03 ** 2


def gauss1d():
    g = np.exp(-np.arange(-5, 6) ** 2 / (2 * 1.5 ** 2))
    return g / g.sum()


def test_window_is_a_normalised_separable_gaussian():
    w = oracle.ssim_window()
    assert w.shape == (11, 11)
    assert abs(w.sum() - 1.0) < 1e-14
    np.testing.assert_allclose(w, np.outer(gauss1d(), gauss1d()), rtol=1e-14)
    assert math.isclose(w[5, 6] / w[5, 5], math.exp(-1.0 / (2 * 2.25)), rel_tol=1e-14)


def test_ssim_of_an_image_with_itself_is_one_and_stationary():
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(23, 19))
    mean, m, g = oracle.ssim_plane(x, x, grad=True)
    assert mean == pytest.approx(1.0, abs=1e-14)
    np.testing.assert_allclose(m, 1.0, atol=1e-13)
    assert np.abs(g).max() < 1e-12


def test_ssim_is_symmetric():
    rng = np.random.default_rng(2)
    x, y = rng.uniform(size=(2, 17, 21))
    _, mxy, _ = oracle.ssim_plane(x, y)
    _, myx, _ = oracle.ssim_plane(y, x)
    np.testing.assert_allclose(mxy, myx, rtol=1e-12, atol=1e-14)  # (g x) y and (g y) x round differently


def test_constant_images_closed_form_inside_and_at_the_borders():
    """Constant images a and b: where the window lies inside the image the variances vanish and SSIM =
    (2ab + C1)/(a^2 + b^2 + C1); at a pixel whose window holds a weight s of in-image pixels (zero padding),
    mu = a s, var = a^2 s (1 - s), cov = a b s (1 - s)."""
    a, b = 0.7, 0.2
    H, W = 24, 30
    _, m, _ = oracle.ssim_plane(np.full((H, W), a), np.full((H, W), b))
    inner = (2 * a * b + C1) / (a * a + b * b + C1)
    np.testing.assert_allclose(m[5:H - 5, 5:W - 5], inner, rtol=1e-12)
    g = gauss1d()
    for (py, px) in [(0, 0), (0, 12), (2, W - 1), (H - 1, 3)]:
        sy = g[max(0, 5 - py):min(11, 5 + H - py)].sum()
        sx = g[max(0, 5 - px):min(11, 5 + W - px)].sum()
        s = sy * sx
        num = (2 * a * b * s * s + C1) * (2 * a * b * s * (1 - s) + C2)
        den = ((a * a + b * b) * s * s + C1) * ((a * a + b * b) * s * (1 - s) + C2)
        assert m[py, px] == pytest.approx(num / den, rel=1e-12), (py, px)


def test_single_bright_pixel_closed_form():
    """x = a at one pixel and 0 elsewhere, y = 0: at a pixel whose window gives the bright pixel weight g,
    SSIM = C1 C2 / ((a^2 g^2 + C1)(a^2 g (1 - g) + C2)); elsewhere both images are 0 in the window and SSIM = 1."""
    a = 0.9
    H, W = 21, 21
    x = np.zeros((H, W))
    x[10, 10] = a
    _, m, _ = oracle.ssim_plane(x, np.zeros((H, W)))
    g1 = gauss1d()
    for py in range(H):
        for px in range(W):
            dy, dx = 10 - py, 10 - px
            if abs(dy) > 5 or abs(dx) > 5:
                assert m[py, px] == pytest.approx(1.0, abs=1e-15)
                continue
            g = g1[dy + 5] * g1[dx + 5]
            want = C1 * C2 / ((a * a * g * g + C1) * (a * a * g * (1 - g) + C2))
            assert m[py, px] == pytest.approx(want, rel=1e-12), (py, px)


@pytest.mark.parametrize("H,W", [(16, 16), (9, 25), (30, 7)])
def test_gradient_matches_central_differences(H, W):
    rng = np.random.default_rng(H * 100 + W)
    x, y = rng.uniform(size=(2, H, W))
    _, _, g = oracle.ssim_plane(x, y, grad=True)
    picks = [(0, 0), (H - 1, W - 1), (H // 2, W // 2)] + [tuple(rng.integers(0, [H, W])) for _ in range(12)]
    h = 1e-6
    for (i, j) in picks:
        xp, xm = x.copy(), x.copy()
        xp[i, j] += h
        xm[i, j] -= h
        fd = (oracle.ssim_plane(xp, y)[0] - oracle.ssim_plane(xm, y)[0]) / (2 * h)
        assert g[i, j] == pytest.approx(fd, rel=1e-6, abs=1e-11), (i, j)


def test_gradient_points_toward_the_target():
    """Moving the rendered image a small step along the gradient raises the mean SSIM."""
    rng = np.random.default_rng(7)
    x, y = rng.uniform(size=(2, 20, 20))
    m0, _, g = oracle.ssim_plane(x, y, grad=True)
    m1, _, _ = oracle.ssim_plane(x + 1e-3 * g / np.abs(g).max(), y)
    assert m1 > m0


def test_loss_over_views_weights_and_layout():
    """L = sum_v w_v lambda (1 - mean over channels of SSIM_v), gradient in the planar per-view layout."""
    cams = [scenes.identity_camera(20.0, 20.0, 8.0, 6.0, 16, 12), scenes.identity_camera(10.0, 10.0, 4.0, 3.0, 8, 6)]
    cams[0].weight, cams[1].weight = 0.7, 0.3
    rng = np.random.default_rng(9)
    P = [c.width * c.height for c in cams]
    x = rng.uniform(size=3 * sum(P))
    y = rng.uniform(size=3 * sum(P))
    lam = 0.2
    L, g = oracle.ssim_loss(x, y, cams, lam)
    want, off = 0.0, 0
    for c, p in zip(cams, P):
        means = [oracle.ssim_plane(x[off + k * p:off + (k + 1) * p].reshape(c.height, c.width),
                                   y[off + k * p:off + (k + 1) * p].reshape(c.height, c.width))[0] for k in range(3)]
        want += c.weight * lam * (1.0 - np.mean(means))
        off += 3 * p
    assert L == pytest.approx(want, rel=1e-14)
    h = 1e-6
    for idx in rng.integers(0, x.size, 10):
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (oracle.ssim_loss(xp, y, cams, lam, grad=False)[0] - oracle.ssim_loss(xm, y, cams, lam, grad=False)[0]) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-6, abs=1e-12), idx


@pytest.mark.parametrize("deg,seed", [(0, 31), (2, 32)])
def test_loss_mode_with_ssim_matches_dense_torch_autograd(deg, seed):
    """The whole loss of eq. L with the SSIM term (lambda 0.2): the oracle's analytic FP64 gradient equals
    autograd through the dense torch renderer and a convolution-based SSIM."""
    import torch

    from tests import ref_torch

    sc = scenes.random_scene(seed, 48, 32, 24, sh_degree=deg, views=2, log_scale_mu=-2.3, depth_fraction=0.5)
    p = {k: torch.tensor(v.astype(np.float64), requires_grad=True) for k, v in sc.params().items()}
    outs = ref_torch.render(p["means"], p["log_scales"], p["quats"], p["opacity"], p["sh"], deg, sc.cams)
    Lt = ref_torch.photometric_loss(outs, sc.cams, sc.tgt_rgb, sc.tgt_depth, lambda_ssim=0.2)
    Lt.backward()
    L, g, exc, nn, _ = oracle.backward(64, sc.params(), deg, sc.cams, tgt_rgb=sc.tgt_rgb, tgt_depth=sc.tgt_depth,
                                       lambda_ssim=0.2)
    assert nn == 0
    np.testing.assert_allclose(L, Lt.item(), rtol=1e-12)
    for k in g:
        gt = p[k].grad.numpy()
        scale = np.abs(gt).max() + 1e-30
        np.testing.assert_allclose(g[k], gt, rtol=1e-7, atol=1e-9 * scale, err_msg=k)
    # the SSIM term changes the gradient (it is not silently dropped)
    _, g0, _, _, _ = oracle.backward(64, sc.params(), deg, sc.cams, tgt_rgb=sc.tgt_rgb, tgt_depth=sc.tgt_depth)
    assert np.abs(g["means"] - g0["means"]).max() > 1e-3 * np.abs(g0["means"]).max()


def test_mixed_reference_with_ssim_equals_fp64_away_from_thresholds():
    """The FP64-along-FP32-decisions reference with the SSIM term agrees with the pure FP64 backward where no
    decision is near its threshold."""
    sc = scenes.random_scene(33, 60, 40, 30, sh_degree=1, views=2, log_scale_mu=-2.3, depth_fraction=0.5)
    r = oracle.reference(sc.params(), 1, sc.cams, tgt_rgb=sc.tgt_rgb, tgt_depth=sc.tgt_depth, lambda_ssim=0.2)
    L, g, _, nn, _ = oracle.backward(64, sc.params(), 1, sc.cams, tgt_rgb=sc.tgt_rgb, tgt_depth=sc.tgt_depth,
                                     lambda_ssim=0.2)
    assert r["near_pixels"] == 0 and nn == 0
    assert r["loss"] == pytest.approx(L, rel=1e-12)
    for k in g:
        # the SSIM gradient of the mixed reference comes from the FP64 image as well
        np.testing.assert_allclose(r["grads"][k], g[k], rtol=1e-9, atol=1e-12 * (np.abs(g[k]).max() + 1e-30))
