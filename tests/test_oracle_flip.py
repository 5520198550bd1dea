"""Pins for the oracle's FLIP (the view-consistency term of Sec. 3.5):
textbook CIELAB values of the sRGB primaries and white, the maximum of the
colour error (green against blue), the closed form of white against black,
kernel normalisations, the unit response of the edge detector to a unit
step, zero for identical images, and central differences of the gradient
(CPU only)."""
import math

import numpy as np
import torch

from oracle import flip


def _const(rgb, h=8, w=9):
    return np.broadcast_to(np.asarray(rgb, float)[:, None, None], (3, h, w)).copy()


def test_colour_transforms_textbook_values():
    assert abs(float(flip.srgb_to_linear(torch.tensor(0.5, dtype=torch.float64))) -
               0.214041140) < 1e-8
    lab = lambda rgb: flip.linear_to_lab(torch.tensor(np.asarray(rgb, float)[:, None, None])
                                         ).numpy()[:, 0, 0]
    np.testing.assert_allclose(lab([1, 1, 1]), [100, 0, 0], atol=1e-9)
    # CIELAB (D65) of the sRGB primaries, as tabulated (tables differ in the
    # last digits with the white point's precision)
    np.testing.assert_allclose(lab([1, 0, 0]), [53.2408, 80.0925, 67.2032], atol=1e-2)
    np.testing.assert_allclose(lab([0, 1, 0]), [87.7347, -86.1827, 83.1793], atol=1e-2)
    np.testing.assert_allclose(lab([0, 0, 1]), [32.2970, 79.1875, -107.8602], atol=1e-2)


def test_cmax_from_tabulated_primaries():
    g = np.array([87.7347, -86.1827, 83.1793])
    b = np.array([32.2970, 79.1875, -107.8602])
    hg = np.array([g[0], g[0] / 100 * g[1], g[0] / 100 * g[2]])
    hb = np.array([b[0], b[0] / 100 * b[1], b[0] / 100 * b[2]])
    d = hg - hb
    want = (abs(d[0]) + math.hypot(d[1], d[2])) ** 0.7
    assert abs(flip.cmax() - want) < 2e-3 * want


def test_green_blue_is_the_maximum_and_white_black_closed_form():
    v, _ = flip.flip_and_grad([_const([0, 1, 0])], [_const([0, 0, 1])])
    assert abs(v[0] - 1.0) < 1e-9
    v, _ = flip.flip_and_grad([_const([1, 1, 1])], [_const([0, 0, 0])])
    cm = flip.cmax()
    e = (100.0 + math.sqrt(flip.EPS)) ** 0.7
    want = 0.95 + (e - 0.4 * cm) / (cm - 0.4 * cm) * 0.05
    assert abs(v[0] - want) < 1e-9
    # identical images: only the eps floors remain
    rng = np.random.default_rng(1)
    x = rng.random((3, 12, 10))
    v, _ = flip.flip_and_grad([x], [x])
    assert v[0] < 1e-6


def test_kernels():
    for c in ("A", "RG", "BY"):
        k = flip.csf_kernel(c)
        assert k.shape == (21, 21) and abs(k.sum() - 1) < 1e-12
        np.testing.assert_allclose(k, k.T, atol=0)
    for kind in ("edge", "point"):
        k = flip.feature_kernel(kind)
        assert k.shape == (19, 19)
        assert abs(k[k > 0].sum() - 1) < 1e-12 and abs(k[k < 0].sum() + 1) < 1e-12
    # the edge detector answers a unit step with magnitude 1 beside it
    img = torch.zeros((30, 30), dtype=torch.float64)
    img[:, 15:] = 1.0
    ex = flip._filter(img, flip.feature_kernel("edge"))
    np.testing.assert_allclose(ex[10, 14:16].numpy(), [-1.0, -1.0], atol=1e-12)
    assert float(ex[10, 3].abs()) < 1e-12
    # and the point detector is zero on a constant image
    assert float(flip._filter(torch.full((25, 25), 0.3, dtype=torch.float64),
                              flip.feature_kernel("point")).abs().max()) < 1e-12


def test_gradient_central_differences():
    rng = np.random.default_rng(2)
    t = rng.uniform(0.05, 0.95, (3, 14, 13))
    r = np.clip(t + rng.normal(0, 0.1, t.shape), 0.02, 0.98)
    v, g = flip.flip_and_grad([t], [r])
    h = 1e-7
    for idx in [(0, 0, 0), (1, 7, 6), (2, 13, 12), (0, 3, 9), (1, 10, 2)]:
        tp, tm = t.copy(), t.copy()
        tp[idx] += h
        tm[idx] -= h
        fd = (flip.flip_and_grad([tp], [r])[0][0] - flip.flip_and_grad([tm], [r])[0][0]) / (2 * h)
        assert abs(fd - g[0][idx]) < 1e-6 + 1e-4 * abs(fd), (idx, fd, g[0][idx])
