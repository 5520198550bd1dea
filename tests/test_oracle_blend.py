"""Pins for the oracle's blending (Eqs. 1-2) and contribution-aware blending
(Algorithm 1): closed forms, invariants and brute force (CPU only)."""
import math

import numpy as np
import pytest

import synthetic
from oracle import binning, blend, project

A_T = 1.0 / 255.0


def _one_tile(mean2d, conic, opacity, rgb, size=16, tile=16, mode="plain", group=(2, 2),
              bg=(0.0, 0.0, 0.0)):
    L = len(opacity)
    sp = dict(mean2d=np.asarray(mean2d, float), conic=np.asarray(conic, float),
              opacity=np.asarray(opacity, float), rgb=np.asarray(rgb, float))
    ranges = np.array([[0, L]])
    return blend.render_tiles(sp, ranges, np.arange(L), size, size, tile, mode=mode,
                              group=group, bg=bg)


def test_single_flat_layer():
    # conic 0 -> q = 0 -> alpha = o everywhere
    r = _one_tile([[8, 8]], [[0, 0, 0]], [0.3], [[0.2, 0.5, 0.9]], bg=(0.1, 0.2, 0.3))
    np.testing.assert_allclose(r["image"][:, 3, 5], 0.3 * np.array([0.2, 0.5, 0.9])
                               + 0.7 * np.array([0.1, 0.2, 0.3]), atol=1e-15)
    assert np.allclose(r["final_T"], 0.7) and (r["n_contrib"] == 1).all()


def test_gaussian_profile_closed_form():
    # isotropic conic I/s^2: alpha = o exp(-r^2 / (2 s^2)) at distance r from the mean
    s, o = 2.5, 0.8
    r = _one_tile([[7.3, 9.1]], [[1 / s ** 2, 0, 1 / s ** 2]], [o], [[1, 1, 1]])
    for (y, x) in [(9, 7), (3, 12), (15, 0), (0, 15)]:
        d2 = (x + 0.5 - 7.3) ** 2 + (y + 0.5 - 9.1) ** 2
        a = o * math.exp(-d2 / (2 * s * s))
        want = a if a >= A_T else 0.0
        assert r["image"][0, y, x] == pytest.approx(want, abs=1e-15)
        assert r["final_T"][y, x] == pytest.approx(1 - want, abs=1e-15)


def test_two_layers_and_opaque_front():
    c1, c2 = np.array([0.9, 0.1, 0.2]), np.array([0.3, 0.7, 0.4])
    r = _one_tile([[8, 8]] * 2, [[0, 0, 0]] * 2, [0.4, 0.6], [c1, c2])
    np.testing.assert_allclose(r["image"][:, 4, 4], 0.4 * c1 + 0.6 * 0.6 * c2, atol=1e-15)
    assert r["final_T"][4, 4] == pytest.approx(0.6 * 0.4, abs=1e-15)
    # opaque front layer is clamped to alpha = 0.99; T_behind = 0.5 >= 0.02
    cf = np.array([0.5, 0.25, 1.0])
    r = _one_tile([[8, 8]] * 2, [[0, 0, 0]] * 2, [1.0, 0.5], [cf, c2])
    np.testing.assert_allclose(r["image"][:, 4, 4], 0.99 * cf + 0.01 * (0.5 * c2), atol=1e-15)
    assert r["final_T"][4, 4] == pytest.approx(0.01 * 0.5, abs=1e-15)


def test_alpha_skip_and_termination():
    # o below alpha_theta is skipped; layers of 0.98 stop when T' < 1e-4
    r = _one_tile([[8, 8]] * 5, [[0, 0, 0]] * 5, [A_T * 0.999, 0.98, 0.98, 0.98, 0.5],
                  [[1, 0, 0]] * 5)
    # T: 1 -> 0.02 -> 4e-4 -> (8e-6 < 1e-4: stop, not blended)
    assert r["final_T"][0, 0] == pytest.approx(0.02 * 0.02, rel=1e-12)
    assert r["n_contrib"][0, 0] == 3  # 1-based position of the last blended entry
    assert r["image"][0, 0, 0] == pytest.approx(0.98 + 0.02 * 0.98, rel=1e-12)


def _random_view(seed, n=60, size=(48, 40), tile=8, opacity_cap=None, extent="3sigma"):
    scene = synthetic.ball_scene(seed, n, log_scale_mu=-2.6, log_scale_sigma=0.5, radius=0.8)
    if opacity_cap is not None:
        o = 1 / (1 + np.exp(-scene.opacity_logits.astype(np.float64)))
        o = np.minimum(o, opacity_cap)
        scene.opacity_logits = np.log(o / (1 - o)).astype(np.float32)
    cam = synthetic.look_at((0.1, -0.2, -3), width=size[0], height=size[1])
    return scene, cam, project.project_view(scene, cam, tile=tile, extent=extent)


def test_partition_of_unity():
    scene, cam, p = _random_view(3)
    p["rgb"][:] = np.array([0.25, 0.5, 0.75])
    r = blend.render_view(p)
    np.testing.assert_allclose(r["image"], np.array([0.25, 0.5, 0.75])[:, None, None]
                               * (1 - r["final_T"])[None], atol=1e-13)


def test_transmittance_bounds_and_prefix_monotonicity():
    scene, cam, p = _random_view(4, n=120)
    r = blend.render_view(p)
    assert (r["final_T"] >= 1e-4).all() and (r["final_T"] <= 1).all()
    b = r["binning"]
    # truncating every tile list after k entries can only raise T
    prev = np.zeros_like(r["final_T"])
    for k in (1, 2, 4, 8, 16, 10 ** 6):
        rng = b["ranges"].copy()
        rng[:, 1] = np.minimum(rng[:, 1], rng[:, 0] + k)
        rk = blend.render_tiles(blend.splats_from_projection(p), rng, b["ids"], p["width"],
                                p["height"], p["tile"])
        if k > 1:
            assert (rk["final_T"] <= prev + 1e-15).all()
        prev = rk["final_T"]
    np.testing.assert_array_equal(prev, r["final_T"])


@pytest.mark.parametrize("seed,tile", [(5, 8), (6, 16)])
def test_tiled_equals_brute_force_per_pixel(seed, tile):
    scene, cam, p = _random_view(seed, n=40, size=(40, 24), tile=tile)
    r = blend.render_view(p)
    bf = blend.brute_force_view(p)
    np.testing.assert_allclose(r["image"], bf["image"], atol=1e-14)
    np.testing.assert_allclose(r["final_T"], bf["final_T"], atol=1e-14)
    np.testing.assert_array_equal(r["n_contrib"], bf["n_contrib"])


def test_low_opacity_scene_is_tile_size_and_extent_independent():
    # with every o <= alpha_theta e^4.5 each alpha >= alpha_theta lies in the tau-ellipse, which
    # both extents cover: image and T do not depend on the extent or the tile size, and equal a
    # blend of *all* Gaussians per pixel in depth order (no tiles at all).
    scene, cam, _ = _random_view(7, n=80, opacity_cap=0.35)
    outs = []
    for tile in (8, 16):
        for ext in ("3sigma", "opacity"):
            p = project.project_view(scene, cam, tile=tile, extent=ext)
            outs.append(blend.render_view(p))
    for o in outs[1:]:
        np.testing.assert_allclose(o["image"], outs[0]["image"], atol=1e-14)
        np.testing.assert_allclose(o["final_T"], outs[0]["final_T"], atol=1e-14)
    p = project.project_view(scene, cam, tile=8)
    order = sorted(np.nonzero(p["visible"])[0], key=lambda g: (float(np.float32(p["depth"][g])), g))
    H, W = p["height"], p["width"]
    for (y, x) in [(5, 7), (12, 30), (20, 20), (0, 0), (23, 47)]:
        T, C = 1.0, np.zeros(3)
        for g in order:
            d = np.array([x + 0.5, y + 0.5]) - p["mean2d"][g]
            a, b, c = p["conic"][g]
            al = min(0.99, p["opacity"][g] * math.exp(-0.5 * (a * d[0] ** 2 + 2 * b * d[0] * d[1]
                                                               + c * d[1] ** 2)))
            if al < A_T:
                continue
            if T * (1 - al) < 1e-4:
                break
            C += T * al * p["rgb"][g]
            T *= 1 - al
        np.testing.assert_allclose(outs[0]["image"][:, y, x], C, atol=1e-14)
        assert x < W and y < H


def test_cr_group1_equals_plain():
    scene, cam, p = _random_view(8, n=80)
    a = blend.render_view(p)
    b = blend.render_view(p, mode="cr", group=(1, 1))
    for k in ("image", "final_T", "n_contrib"):
        np.testing.assert_array_equal(a[k], b[k])


def test_cr_equals_plain_when_leaders_always_pass():
    # flat layers (conic 0) give every pixel, leader included, alpha = o >= alpha_theta
    rng = np.random.default_rng(9)
    L = 12
    args = ([[8, 8]] * L, [[0, 0, 0]] * L, rng.uniform(0.05, 0.5, L), rng.uniform(0, 1, (L, 3)))
    a = _one_tile(*args)
    b = _one_tile(*args, mode="cr")
    for k in ("image", "final_T", "n_contrib"):
        np.testing.assert_array_equal(a[k], b[k])


def test_cr_leader_skip_hides_follower_contribution():
    # narrow Gaussian centred on pixel (x=1, y=0): its leader (0, 0) sees alpha < alpha_theta
    s = 0.25
    args = ([[1.5, 0.5]], [[1 / s ** 2, 0, 1 / s ** 2]], [0.9], [[1, 1, 1]])
    plain = _one_tile(*args)
    cr = _one_tile(*args, mode="cr")
    lead_alpha = 0.9 * math.exp(-1.0 / (2 * s * s))
    assert lead_alpha < A_T
    assert plain["image"][0, 0, 1] == pytest.approx(0.9, rel=1e-12)
    assert cr["image"][0, 0, 1] == 0.0 and cr["n_contrib"][0, 1] == 0
    # centred on the leader instead: the whole group evaluates it
    args2 = ([[0.5, 0.5]], [[1 / s ** 2, 0, 1 / s ** 2]], [0.9], [[1, 1, 1]])
    cr2 = _one_tile(*args2, mode="cr")
    assert cr2["image"][0, 0, 0] == pytest.approx(0.9, rel=1e-12)
    assert cr2["n_contrib"][0, 1] == 0  # follower's own alpha < alpha_theta: still skipped


def test_cr_terminated_leader_keeps_testing():
    # three 0.98 layers concentrated on the leader stop it; a later flat layer still passes the
    # stopped leader's test, so the followers blend it
    s = 0.2
    mean = [[0.5, 0.5]] * 3 + [[8, 8]]
    conic = [[1 / s ** 2, 0, 1 / s ** 2]] * 3 + [[0, 0, 0]]
    r = _one_tile(mean, conic, [0.98, 0.98, 0.98, 0.5], [[1, 0, 0]] * 3 + [[0, 1, 0]], mode="cr")
    assert r["n_contrib"][0, 0] == 2            # leader stopped at the third layer
    assert r["image"][1, 0, 1] == pytest.approx(0.5, rel=1e-12)  # follower got the flat layer
    assert r["n_contrib"][0, 1] == 4


def test_cr_counters_and_margins():
    scene, cam, p = _random_view(10, n=80)
    r = blend.render_view(p, mode="cr")
    c = r["counters"]
    assert c["leader_pass"] <= c["leader_tests"] and c["pass_evals"] <= 4 * c["leader_pass"]
    assert np.isfinite(r["margin"]).any()


def test_binning_order_matches_python_sorted():
    scene, cam, p = _random_view(11, n=200, tile=8)
    depth32 = p["depth"].astype(np.float32)
    depth32[5] = depth32[17] = depth32[40]  # force depth ties: resolved by id
    p["rect"][[5, 17, 40]] = p["rect"][40]
    p["n_tiles"][[5, 17, 40]] = p["n_tiles"][40]
    b = binning.bin_and_sort([dict(rect=p["rect"], n_tiles=p["n_tiles"], depth_f32=depth32,
                                   grid_w=p["grid_w"], grid_h=p["grid_h"])], 200)
    pairs = []
    for g in range(200):
        if p["n_tiles"][g] == 0:
            continue
        x0, y0, x1, y1 = p["rect"][g]
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                pairs.append((ty * p["grid_w"] + tx, float(depth32[g]), g))
    pairs.sort()
    assert [q[2] for q in pairs] == b["ids"].tolist()
    assert [q[0] for q in pairs] == b["tiles"].tolist()
    for t in range(p["grid_w"] * p["grid_h"]):
        s, e = b["ranges"][t]
        assert all(q[0] == t for q in pairs[s:e])
        assert sum(1 for q in pairs if q[0] == t) == e - s


def test_binning_multi_view_tile_bases():
    scene = synthetic.ball_scene(12, 50, log_scale_mu=-2.5)
    cams = [synthetic.look_at((0, 0, -3), width=32, height=16),
            synthetic.look_at((1, 0, -3), width=24, height=24)]
    views = []
    for cam in cams:
        p = project.project_view(scene, cam, tile=8)
        views.append(dict(rect=p["rect"], n_tiles=p["n_tiles"], depth_f32=p["depth"].astype(
            np.float32), grid_w=p["grid_w"], grid_h=p["grid_h"]))
    b = binning.bin_and_sort(views, 50)
    assert b["tile_bases"].tolist() == [0, 8]
    assert b["ranges"].shape == (8 + 9, 2)
    first = b["ids"][b["tiles"] < 8]
    assert (first < 50).all() and (b["ids"][b["tiles"] >= 8] >= 50).all()


def test_plain_counters_by_hand_count():
    # one 16x16 tile, five entries; the narrow entry (sigma = 0.2 px, centred on pixel (3, 4))
    # reaches alpha_theta at that pixel only: a neighbour one pixel away sees
    # 0.99 exp(-1 / (2 * 0.04)) ~ 4e-6 < 1/255
    s = 0.2
    mean = [[8, 8], [8, 8], [3.5, 4.5], [8, 8], [8, 8]]
    conic = [[0, 0, 0], [0, 0, 0], [1 / s ** 2, 0, 1 / s ** 2], [0, 0, 0], [0, 0, 0]]
    r = _one_tile(mean, conic, [0.98, 0.98, 0.995, 0.5, 0.6], [[1, 1, 1]] * 5)
    # per pixel, T: 1 -> 0.02 -> 4e-4; entry 2 stops pixel (3, 4) (4e-4 * 0.01 < 1e-4) and is
    # skipped (alpha < alpha_theta) everywhere else; entry 3 blends (T = 2e-4) at the 255 live
    # pixels; entry 4 stops them all (2e-4 * 0.4 < 1e-4)
    # evaluations are counted for live pixels only: 256 + 256 + 256 + 255 + 255
    assert r["counters"]["evals"] == 1278
    # blends: 256 + 256 + 0 + 255 + 0
    assert r["counters"]["blends"] == 767
    assert r["n_contrib"][4, 3] == 2 and r["n_contrib"][0, 0] == 4
    assert r["counters"]["leader_tests"] == 0 and r["counters"]["pass_evals"] == 0


def test_skip_and_termination_counters_by_hand_count():
    # the five flat layers of test_alpha_skip_and_termination: every pixel evaluates the
    # sub-threshold layer, blends two, evaluates the third 0.98 layer and stops there; the
    # last layer is never evaluated -> 4 evaluations and 2 blends per pixel
    r = _one_tile([[8, 8]] * 5, [[0, 0, 0]] * 5, [A_T * 0.999, 0.98, 0.98, 0.98, 0.5],
                  [[1, 0, 0]] * 5)
    assert r["counters"]["evals"] == 4 * 256
    assert r["counters"]["blends"] == 2 * 256


def test_cr_counters_by_hand_count():
    # a 4x4 image in one 4x4 tile, 2x2 groups: leaders (0,0), (2,0), (0,2), (2,2)
    s = 0.2
    mean = [[2, 2], [2.5, 2.5], [1.5, 0.5], [2, 2], [2, 2], [2, 2]]
    conic = [[0, 0, 0], [1 / s ** 2, 0, 1 / s ** 2], [1 / s ** 2, 0, 1 / s ** 2],
             [0, 0, 0], [0, 0, 0], [0, 0, 0]]
    r = _one_tile(mean, conic, [0.5, 0.9, 0.9, 0.98, 0.98, 0.6], [[1, 1, 1]] * 6, size=4,
                  tile=4, mode="cr")
    c = r["counters"]
    # entry: live groups tested / accepted, live pixels of accepted groups, blends
    #  0 flat 0.5            4 / 4, 16, 16        (T = 0.5)
    #  1 narrow on leader (2,2)   4 / 1, 4, 1     (only that pixel: T = 0.05)
    #  2 narrow on follower (1,0) 4 / 0, 0, 0     (its leader sees alpha ~ 1e-11)
    #  3 flat 0.98           4 / 4, 16, 16        (T = 0.01; pixel (2,2): 1e-3)
    #  4 flat 0.98           4 / 4, 16, 15        (T = 2e-4; pixel (2,2) stops: 2e-5 < 1e-4)
    #  5 flat 0.6            4 / 4, 15, 0         (2e-4 * 0.4 < 1e-4: every live pixel stops;
    #                                              group (2,2) still counts, its followers live)
    assert c["leader_tests"] == 24
    assert c["leader_pass"] == 17
    assert c["pass_evals"] == 67
    assert c["blends"] == 48
    assert r["n_contrib"][2, 2] == 4 and r["n_contrib"][0, 1] == 5
    assert c["evals"] == 0


def test_tile_aligned_crop_renders_the_same_pixels():
    # a camera restricted to a window whose origin is a multiple of the tile (and group) size
    # sees every tile list and pixel group of that window unchanged (x' moves by the window
    # origin, up to the rounding of one float64 addition)
    scene = synthetic.ball_scene(13, 300, log_scale_mu=-3.0)
    full = synthetic.look_at((0.3, -0.2, -3.0), width=80, height=64)
    crop = synthetic.crop_camera(full, 16, 32, 48, 32)
    for mode in ("plain", "cr"):
        a = blend.render_view(project.project_view(scene, full, tile=16), mode=mode)
        b = blend.render_view(project.project_view(scene, crop, tile=16), mode=mode)
        np.testing.assert_allclose(b["image"], a["image"][:, 32:64, 16:64], rtol=0, atol=1e-12)
        np.testing.assert_allclose(b["final_T"], a["final_T"][32:64, 16:64], rtol=0, atol=1e-12)
        np.testing.assert_array_equal(b["n_contrib"], a["n_contrib"][32:64, 16:64])
