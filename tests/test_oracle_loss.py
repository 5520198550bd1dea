"""Pins for the oracle's fine-tuning loss and optimizer (Sec. 3.5): SSIM of
an image with itself, the closed form on constant images, brute force per
pixel on a tiny image, central differences of the gradient, and Adam's
first step and constant-gradient closed forms (CPU only)."""
import numpy as np
import torch

from oracle import loss as oloss


def test_window_is_normalised_gaussian():
    w = oloss.window()
    assert w.shape == (11, 11) and abs(w.sum() - 1.0) < 1e-15
    g = np.exp(-np.arange(-5, 6) ** 2 / (2 * 1.5 ** 2))
    np.testing.assert_allclose(w, np.outer(g, g) / g.sum() ** 2, rtol=1e-14)


def test_ssim_of_identical_images_is_one():
    rng = np.random.default_rng(0)
    x = torch.tensor(rng.random((3, 20, 17)))
    np.testing.assert_allclose(oloss.ssim_map(x, x).numpy(), 1.0, atol=1e-12)
    assert float(oloss.photometric_loss(x, x)) < 1e-12


def test_ssim_constant_images_closed_form():
    # constant a and b over a 30 x 30 image: at an interior pixel the window
    # moments are a, b, a^2, b^2, ab, so both variances and the covariance
    # vanish and S = (2ab + C1) / (a^2 + b^2 + C1)
    a, b = 0.3, 0.7
    x = torch.full((3, 30, 30), a, dtype=torch.float64)
    y = torch.full((3, 30, 30), b, dtype=torch.float64)
    s = oloss.ssim_map(x, y).numpy()
    want = (2 * a * b + oloss.C1) / (a * a + b * b + oloss.C1)
    np.testing.assert_allclose(s[:, 5:-5, 5:-5], want, rtol=1e-12)


def test_ssim_brute_force_per_pixel():
    rng = np.random.default_rng(1)
    x, y = rng.random((3, 9, 13)), rng.random((3, 9, 13))
    w = oloss.window()
    got = oloss.ssim_map(torch.tensor(x), torch.tensor(y)).numpy()
    for c in range(3):
        for i in range(9):
            for j in range(13):
                mom = np.zeros(5)
                for di in range(-5, 6):
                    for dj in range(-5, 6):
                        ii, jj = i + di, j + dj
                        if 0 <= ii < 9 and 0 <= jj < 13:
                            wt = w[di + 5, dj + 5]
                            a, b = x[c, ii, jj], y[c, ii, jj]
                            mom += wt * np.array([a, b, a * a, b * b, a * b])
                mx, my, exx, eyy, exy = mom
                s = ((2 * mx * my + oloss.C1) * (2 * (exy - mx * my) + oloss.C2)) / (
                    (mx * mx + my * my + oloss.C1) * (exx - mx * mx + eyy - my * my + oloss.C2))
                assert abs(s - got[c, i, j]) < 1e-12


def test_loss_gradient_central_differences():
    rng = np.random.default_rng(2)
    xs = [rng.random((3, 8, 10)), rng.random((3, 6, 7))]
    ys = [rng.random((3, 8, 10)), rng.random((3, 6, 7))]
    loss, grads = oloss.loss_and_grad(xs, ys, 0.2)
    h = 1e-6
    for v in range(2):
        for idx in [(0, 0, 0), (1, 3, 4), (2, 7, 9) if v == 0 else (2, 5, 6), (0, 4, 2)]:
            xp = [a.copy() for a in xs]
            xm = [a.copy() for a in xs]
            xp[v][idx] += h
            xm[v][idx] -= h
            lp = oloss.loss_and_grad(xp, ys, 0.2)[0].mean()
            lm = oloss.loss_and_grad(xm, ys, 0.2)[0].mean()
            assert abs((lp - lm) / (2 * h) - grads[v][idx]) < 1e-7, (v, idx)
    # the L1 part alone: lambda = 0 gives sign(x - y) / (views * elements)
    _, g0 = oloss.loss_and_grad(xs, ys, 0.0)
    np.testing.assert_allclose(g0[1], np.sign(xs[1] - ys[1]) / (2 * xs[1].size), atol=1e-15)


def test_adam_closed_forms():
    rng = np.random.default_rng(3)
    p, g = rng.normal(size=50), rng.normal(size=50)
    z = np.zeros(50)
    # first step: m_hat = g, v_hat = g^2 -> p - lr g / (|g| + eps)
    p1, m, v = oloss.adam_step(p, g, z, z, 0.01, 1, eps=1e-8)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # constant gradient: the bias-corrected moments stay g and g^2
    q, m, v = p.copy(), z, z
    for t in range(1, 20):
        q, m, v = oloss.adam_step(q, g, m, v, 0.01, t, eps=0.0)
    np.testing.assert_allclose(q, p - 19 * 0.01 * np.sign(g), rtol=1e-9)
    # zero gradient from zero state: no move
    p2, _, _ = oloss.adam_step(p, z, z, z, 0.01, 1)
    np.testing.assert_array_equal(p2, p)
