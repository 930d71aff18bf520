"""Host-side logic: seeded inputs, camera conventions, pyramid targets, planner helpers (no GPU)."""
import math

import numpy as np
import pytest

from paper_2411_02703_amd import scenes


def test_generator_is_deterministic():
    a = scenes.random_scene(3, 100, 40, 30, sh_degree=2, views=3)
    b = scenes.random_scene(3, 100, 40, 30, sh_degree=2, views=3)
    for k in a.params():
        assert np.array_equal(a.params()[k], b.params()[k])
    assert np.array_equal(a.tgt_rgb, b.tgt_rgb) and np.array_equal(a.tgt_depth, b.tgt_depth)
    c = scenes.random_scene(4, 100, 40, 30, sh_degree=2, views=3)
    assert not np.array_equal(a.means, c.means)


def test_config1_matches_its_description():
    sc = scenes.config(1)
    assert sc.n == 2000 and sc.sh_degree == 0 and len(sc.cams) == 1
    cam = sc.cams[0]
    assert (cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy) == (128, 96, 100.0, 100.0, 64.0, 48.0)
    assert sc.means[:, 2].min() >= 2.0 and sc.means[:, 2].max() <= 20.0
    assert abs(sc.log_scales.mean() + 3.0) < 0.05 and abs(sc.log_scales.std() - 0.5) < 0.05
    rgb = sc.sh[:, 0, :] * 0.28209479177387814 + 0.5
    assert rgb.min() >= 0.0 and rgb.max() <= 1.0
    assert sc.tgt_depth.min() >= 2.0 and sc.tgt_rgb.size == 3 * 128 * 96


def test_look_camera_conventions():
    # looking along +x from (0, 0, 2): a point 5 m ahead maps to the image centre at depth 5,
    # a point above (+z world) maps to the upper half (smaller v), a point to the left (+y world) to smaller u
    cam = scenes.look_camera([0.0, 0.0, 2.0], 0.0, 0.0, 500.0, 500.0, 640, 480)
    def proj(p):
        t = cam.R @ np.asarray(p) + cam.T
        return cam.fx * t[0] / t[2] + cam.cx, cam.fy * t[1] / t[2] + cam.cy, t[2]
    u, v, z = proj([5.0, 0.0, 2.0])
    assert abs(u - 320) < 1e-9 and abs(v - 240) < 1e-9 and abs(z - 5) < 1e-12
    assert proj([5.0, 0.0, 3.0])[1] < 240
    assert proj([5.0, 1.0, 2.0])[0] < 320
    np.testing.assert_allclose(cam.R @ cam.R.T, np.eye(3), atol=1e-12)
    assert abs(np.linalg.det(cam.R) - 1) < 1e-12
    np.testing.assert_allclose(cam.campos, [0.0, 0.0, 2.0], atol=1e-12)


def test_pyramid_levels_are_consistent():
    cam = scenes.look_camera([0.0, 0.0, 2.0], 0.3, 0.05, 900.0, 900.0, 1280, 1024)
    for l in (1, 2):
        c = cam.scaled(l)
        assert (c.width, c.height) == (1280 >> l, 1024 >> l)
        # pixel centre (u + 0.5) at level l is the centre of the 2^l x 2^l block at level 0
        assert c.fx == cam.fx / 2 ** l and c.cx == cam.cx / 2 ** l
    rng = np.random.default_rng(0)
    rgbs, depths = scenes.pyramid_targets(rng, scenes.look_camera([0, 0, 2], 0, 0, 100, 100, 16, 8), 3)
    assert rgbs[1].shape == (3, 4, 8) and rgbs[2].shape == (3, 2, 4)
    np.testing.assert_allclose(rgbs[1][:, 0, 0], rgbs[0][:, 0:2, 0:2].mean(axis=(1, 2)))
    d0 = depths[0][0:2, 0:2]
    valid = d0[d0 > 0]
    assert depths[1][0, 0] == (valid.mean() if valid.size else 0.0)


def test_lidar_points_lie_on_the_scene():
    rng = np.random.default_rng(5)
    origins = np.array([[0.0, 0.0, 1.8]])
    boxes = scenes.random_boxes(rng, 10, origins[:, :2], "annulus")
    pts = scenes.lidar_points(rng, 5000, origins, boxes, rmax=60.0, noise=0.0)
    r = np.linalg.norm(pts - origins[0], axis=1)
    assert r.min() >= 1.0 - 1e-9 and r.max() <= 60.0 + 1e-9
    on_ground = np.abs(pts[:, 2]) < 1e-6
    in_box = np.zeros(len(pts), bool)
    for lo, hi in zip(boxes.lo, boxes.hi):
        in_box |= np.all((pts >= lo - 1e-6) & (pts <= hi + 1e-6), axis=1)
    assert np.all(on_ground | in_box)


def test_crop_camera_shifts_principal_point():
    cam = scenes.identity_camera(100.0, 90.0, 32.0, 24.0, 64, 48)
    c = cam.cropped(10, 5, 20, 16)
    assert (c.cx, c.cy, c.width, c.height) == (22.0, 19.0, 20, 16)


def test_autotune_cache_key_bands():
    pytest.importorskip("torch")
    from paper_2411_02703_amd import autotune

    cams = [scenes.identity_camera(100, 100, 32, 24, 64, 48)] * 3
    k1 = autotune.cache_key(1_000_000, cams, 3)
    k2 = autotune.cache_key(1_100_000, cams, 3)
    k3 = autotune.cache_key(4_000_000, cams, 3)
    assert k1 == k2 and k1 != k3 and "deg3" in k1 and "views3" in k1
