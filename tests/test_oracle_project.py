"""Pins for the oracle's preprocessing (CPU only): closed forms, library
routines and brute force, independent of the formulas being tested."""
import json
import math
import os

import numpy as np
import pytest
import scipy.special as sps
from scipy.spatial.transform import Rotation

import synthetic
from oracle import project, sh

HERE = os.path.dirname(__file__)
CONST = json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))


def _scene(means, log_scales, quats, logits, sh_coef=None):
    n = len(logits)
    shc = np.zeros((16, 3, n), np.float32) if sh_coef is None else sh_coef
    return synthetic.Scene(np.asarray(means, np.float32).T.copy(),
                           np.asarray(log_scales, np.float32).T.copy(),
                           np.asarray(quats, np.float32).T.copy(),
                           np.asarray(logits, np.float32), shc)


def test_constants_match_paper():
    assert project.ALPHA_THETA == pytest.approx(CONST["alpha_theta"]["value"], rel=0, abs=1e-18)


def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    B = sh.basis(d)
    th, ph = np.arccos(d[:, 2]), np.arctan2(d[:, 1], d[:, 0])
    for l in range(4):
        for m in range(-l, l + 1):
            Y = sps.sph_harm_y(l, abs(m), th, ph)
            ref = Y.real if m == 0 else math.sqrt(2) * (Y.real if m > 0 else Y.imag)
            np.testing.assert_allclose(B[:, l * l + l + m], ref, atol=1e-13)


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform in phi integrates degree<=6 products exactly
    x, w = np.polynomial.legendre.leggauss(12)
    ph = np.arange(24) * 2 * np.pi / 24
    Z, P = np.meshgrid(x, ph, indexing="ij")
    W = np.repeat(w[:, None], 24, axis=1) * (2 * np.pi / 24)
    r = np.sqrt(1 - Z ** 2)
    d = np.stack([r * np.cos(P), r * np.sin(P), Z], -1).reshape(-1, 3)
    B = sh.basis(d)
    G = (B * W.reshape(-1, 1)).T @ B
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_grad_fd():
    rng = np.random.default_rng(1)
    d = rng.normal(size=(20, 3))
    G = sh.basis_grad(d)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (sh.basis(d + e) - sh.basis(d - e)) / (2 * h)
        np.testing.assert_allclose(G[..., k], fd, atol=1e-7)


def test_quaternion_rotation_matches_scipy():
    rng = np.random.default_rng(2)
    q = rng.normal(size=(50, 4)) * 3
    R = project.quat_to_rotmat(q)
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()  # scipy: (x, y, z, w)
    np.testing.assert_allclose(R, ref, atol=1e-12)


def test_covariance_eigenvalues_and_sign_invariance():
    rng = np.random.default_rng(3)
    ls = rng.normal(-2, 1, size=(30, 3))
    q = rng.normal(size=(30, 4))
    S = project.covariance3d(ls, q)
    ev = np.linalg.eigvalsh(S)
    np.testing.assert_allclose(np.sort(ev, 1), np.sort(np.exp(2 * ls), 1), rtol=1e-10)
    np.testing.assert_allclose(project.covariance3d(ls, -q), S, atol=1e-15)
    S_id = project.covariance3d(ls, np.tile([1.0, 0, 0, 0], (30, 1)))
    for i in range(30):
        np.testing.assert_allclose(S_id[i], np.diag(np.exp(2 * ls[i])), atol=1e-15)


def test_ewa_jacobian_is_projection_derivative():
    rng = np.random.default_rng(4)
    t = rng.normal(size=(10, 3)) + np.array([0, 0, 5.0])
    fx, fy = 300.0, 280.0
    J = project.ewa_jacobian(t, fx, fy)
    proj = lambda tt: np.stack([fx * tt[:, 0] / tt[:, 2], fy * tt[:, 1] / tt[:, 2]], 1)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        np.testing.assert_allclose(J[:, :, k], (proj(t + e) - proj(t - e)) / (2 * h), atol=1e-6)


@pytest.mark.parametrize("pos", [(0.0, 0.0, 0.0), (0.4, -0.3, 0.5)])
def test_isotropic_gaussian_closed_form(pos):
    s = 0.05
    scene = _scene([pos], [[math.log(s)] * 3], [[0.3, -0.2, 0.9, 0.1]], [2.0])
    cam = synthetic.look_at((0, 0, -3), width=256, height=256)
    p = project.project_view(scene, cam)
    f = cam.fx
    t = np.asarray(pos, np.float32).astype(np.float64) + np.array([0, 0, 3.0])
    # isotropic: R_w Sigma R_w^T = s^2 I, so Sigma' = s^2 J J^T + 0.3 I
    J = np.array([[f / t[2], 0, -f * t[0] / t[2] ** 2], [0, f / t[2], -f * t[1] / t[2] ** 2]])
    s32 = float(np.exp(np.float64(np.float32(math.log(s)))))
    ref = s32 ** 2 * J @ J.T + 0.3 * np.eye(2)
    a, b, c = p["cov2d"][0]
    np.testing.assert_allclose([a, b, c], [ref[0, 0], ref[0, 1], ref[1, 1]], rtol=1e-12, atol=1e-12)
    if pos == (0.0, 0.0, 0.0):
        np.testing.assert_allclose(a, (f * s32 / 3.0) ** 2 + 0.3, rtol=1e-12)
        assert b == pytest.approx(0.0, abs=1e-12)
        np.testing.assert_allclose(p["mean2d"][0], [128.0, 128.0], atol=1e-12)
    # conic is the inverse covariance
    A = p["conic"][0]
    M = np.array([[A[0], A[1]], [A[1], A[2]]]) @ ref
    np.testing.assert_allclose(M, np.eye(2), atol=1e-10)
    # x' = f t_x / t_z + c_x
    np.testing.assert_allclose(p["mean2d"][0], [f * t[0] / t[2] + 128, f * t[1] / t[2] + 128],
                               rtol=1e-12)


def test_dc_colour_and_clamp():
    shc = np.zeros((16, 3, 2), np.float32)
    shc[0, :, 0] = [0.3, -0.1, -2.0]
    shc[0, :, 1] = [1.0, 0.0, 0.0]
    scene = _scene([[0, 0, 0], [0.1, 0, 0]], [[-3] * 3] * 2, [[1, 0, 0, 0]] * 2, [0.0, 0.0], shc)
    cam = synthetic.look_at((0, 0, -3), width=64, height=64)
    p = project.project_view(scene, cam)
    c0 = 1.0 / (2.0 * math.sqrt(math.pi))
    k = shc[0, :, 0].astype(np.float64)
    np.testing.assert_allclose(p["rgb"][0], np.maximum(0.0, 0.5 + c0 * k), atol=1e-15)
    assert p["rgb"][0, 2] == 0.0


def test_degree1_colour_is_direction_linear():
    # l = 1 terms equal (-C1 y, C1 z, -C1 x) with C1 = sqrt(3 / (4 pi)), from scipy's Y_1^m
    shc = np.zeros((16, 3, 1), np.float32)
    shc[1:4, 0, 0] = [0.2, 0.3, -0.4]
    scene = _scene([[0.3, -0.2, 0.1]], [[-3] * 3], [[1, 0, 0, 0]], [0.0], shc)
    cam = synthetic.look_at((0.5, 0.4, -3), width=64, height=64)
    p = project.project_view(scene, cam)
    v = np.array([0.3, -0.2, 0.1], np.float32).astype(np.float64) - cam.center
    d = v / np.linalg.norm(v)
    th, ph = math.acos(d[2]), math.atan2(d[1], d[0])
    y1 = [math.sqrt(2) * sps.sph_harm_y(1, 1, th, ph).imag, sps.sph_harm_y(1, 0, th, ph).real,
          math.sqrt(2) * sps.sph_harm_y(1, 1, th, ph).real]
    ref = 0.5 + float(np.dot(y1, shc[1:4, 0, 0].astype(np.float64)))
    assert p["rgb"][0, 0] == pytest.approx(ref, abs=1e-14)


def test_opacity_aware_extent_and_crossover():
    a_t = 1.0 / 255.0
    # tau = min(2 ln(o / alpha_theta), 9) reaches 9 at o = alpha_theta * e^4.5
    o_cross = a_t * math.exp(4.5)
    assert o_cross == pytest.approx(0.3530, abs=1e-4)
    logits = [math.log(o / (1 - o)) for o in (0.05, 0.2, 0.3, 0.9)]
    scene = _scene([[0, 0, 0]] * 4, [[-2.5, -2.0, -3.0]] * 4, [[0.9, 0.2, -0.3, 0.1]] * 4, logits)
    cam = synthetic.look_at((0, 0, -3), width=256, height=256)
    p = project.project_view(scene, cam, extent="opacity")
    o = p["opacity"]
    # on the ellipse boundary d^T A d = tau, alpha = o exp(-tau/2) = alpha_theta when tau < 9
    for i in range(4):
        tau = p["tau"][i]
        if o[i] < o_cross:
            assert o[i] * math.exp(-tau / 2) == pytest.approx(a_t, rel=1e-12)
        else:
            assert tau == 9.0
        # the box half-widths are the extreme coordinates of the ellipse boundary, by sampling
        a, b, c = p["cov2d"][i]
        L = np.linalg.cholesky(np.array([[a, b], [b, c]]))
        th = np.linspace(0, 2 * np.pi, 200001)
        pts = math.sqrt(tau) * (L @ np.stack([np.cos(th), np.sin(th)]))
        assert np.abs(pts[0]).max() == pytest.approx(p["ex"][i], rel=1e-8)
        assert np.abs(pts[1]).max() == pytest.approx(p["ey"][i], rel=1e-8)
        # and those points satisfy d^T A d = tau
        A = p["conic"][i]
        q = A[0] * pts[0] ** 2 + 2 * A[1] * pts[0] * pts[1] + A[2] * pts[1] ** 2
        np.testing.assert_allclose(q, tau, rtol=1e-9)


def test_three_sigma_circle_contains_three_sigma_ellipse():
    scene = _scene([[0.1, 0, 0]], [[-2.0, -3.5, -2.7]], [[0.5, 0.5, -0.5, 0.2]], [1.0])
    cam = synthetic.look_at((0, 0, -3), width=256, height=256)
    p = project.project_view(scene, cam, extent="3sigma")
    a, b, c = p["cov2d"][0]
    L = np.linalg.cholesky(np.array([[a, b], [b, c]]))
    th = np.linspace(0, 2 * np.pi, 100001)
    pts = 3.0 * (L @ np.stack([np.cos(th), np.sin(th)]))
    r = np.sqrt((pts ** 2).sum(0)).max()
    assert r == pytest.approx(p["ex"][0], rel=1e-8)  # circle touches the ellipse's far point


def test_tile_rect_brute_force():
    rng = np.random.default_rng(5)
    scene = synthetic.ball_scene(11, 300, log_scale_mu=-3.0, log_scale_sigma=0.8, radius=1.2)
    cam = synthetic.look_at((0.2, 0.1, -2.5), width=100, height=70)
    for tile in (8, 16):
        for ext in ("3sigma", "opacity"):
            p = project.project_view(scene, cam, tile=tile, extent=ext)
            gw, gh = -(-100 // tile), -(-70 // tile)
            for i in np.nonzero(p["visible"])[0]:
                lo_x, hi_x = p["mean2d"][i, 0] - p["ex"][i], p["mean2d"][i, 0] + p["ex"][i]
                lo_y, hi_y = p["mean2d"][i, 1] - p["ey"][i], p["mean2d"][i, 1] + p["ey"][i]
                hit = [(tx, ty) for ty in range(gh) for tx in range(gw)
                       if tx * tile <= hi_x and (tx + 1) * tile > lo_x
                       and ty * tile <= hi_y and (ty + 1) * tile > lo_y]
                x0, y0, x1, y1 = p["rect"][i]
                want = [(tx, ty) for ty in range(y0, y1) for tx in range(x0, x1)]
                assert sorted(hit) == sorted(want)
                assert p["n_tiles"][i] == len(hit)
    assert rng is not None


def test_culling_rules():
    means = [[0, 0, -3.5], [0, 0, 0], [np.nan, 0, 0], [0, 0, 0], [50, 0, 0], [0, 0, 0]]
    logits = [0.0, 0.0, 0.0, -8.0, 0.0, math.log((1 / 255) / (1 - 1 / 255)) - 1e-3]
    scene = _scene(means, [[-3] * 3] * 6, [[1, 0, 0, 0]] * 6, logits)
    cam = synthetic.look_at((0, 0, -3), width=64, height=64)
    for ext in ("3sigma", "opacity"):
        p = project.project_view(scene, cam, extent=ext)
        # behind the camera, NaN mean, o < 1/255, off-screen, o just below 1/255
        assert p["visible"].tolist() == [False, True, False, False, False, False]
        assert p["n_tiles"][0] == 0 and p["n_tiles"][1] > 0
