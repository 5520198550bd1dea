"""FLIP (LDR) image difference, in float64 on the CPU with torch autograd for
its gradient (test infrastructure: only the tests, the smoke check and the
benchmark's CPU baseline use the oracle).

Sec. 3.5 adds a view-consistency term gamma * L_consistency (gamma = 0.1) to
the fine-tuning loss, with FLIP [Andersson et al. 2020] over 7 frames.  This
module restates FLIP's published definition:

  colour: sRGB (clamped to [0, 1]) -> linear RGB -> XYZ (D65) -> YCxCz;
    each opponent channel is filtered with its contrast-sensitivity
    Gaussian(s), sum_i a_i sqrt(pi / b_i) exp(-pi^2 d^2 / b_i) over the
    distance d in degrees (1 / ppd per pixel), normalised to sum 1, radius
    ceil(3 sqrt(max b / (2 pi^2)) ppd), edges replicated; back to linear
    RGB, clamped to [0, 1], -> CIELAB -> Hunt adjustment (a, b scaled by
    L / 100) -> HyAB distance |dL| + sqrt(max(da^2 + db^2, eps)), raised to
    qc, then mapped to [0, 1] piecewise linearly: [0, pc cmax) -> [0, pt),
    [pc cmax, cmax] -> [pt, 1], cmax = the same power of the HyAB distance of
    Hunt-adjusted green and blue;
  features: on the normalised luminance (Y + 16) / 116 of the unfiltered
    YCxCz, edge (first derivative of a Gaussian) and point (second
    derivative) detectors along x and y, sd = 0.5 * 0.082 deg * ppd, radius
    ceil(3 sd), positive weights normalised to sum 1 and negative to -1,
    edges replicated; dF = (max(|‖e_ref‖ - ‖e_test‖|, |‖p_ref‖ - ‖p_test‖|)
    clamped below at eps, divided by sqrt 2) ** qf;
  per pixel: dE_c ** (1 - dF); the score is the mean over pixels.
Constants: qc = 0.7, qf = 0.5, pc = 0.4, pt = 0.95, eps = 1e-15; CSF
parameters (a1, b1, a2, b2): A (1, 0.0047, 0, 1e-5), RG (1, 0.0053, 0, 1e-5),
BY (34.1, 0.04, 13.5, 0.025); ppd = 0.7 m * (3840 px / 0.7 m) * pi / 180.

Readings: images are [3][H][W] sRGB; the consistency term of a step is the
mean FLIP between each of 7 consecutive views' render and its target image
(the paper names the metric and the frame count only).

Parity unpinned: the values of the CSF and feature-detector constants above
(restated from FLIP's publication, which is not available here).  The tests
pin the colour chain to tabulated CIELAB values of the sRGB primaries, the
colour-error maximum (green against blue maps to exactly 1), the constants'
normalisations and the unit-step response, and the gradient by central
finite differences; a wrong constant value would pass them.
"""
from __future__ import annotations

import math

import numpy as np
import torch

QC, QF, PC, PT, EPS = 0.7, 0.5, 0.4, 0.95, 1e-15
CSF = {"A": (1.0, 0.0047, 0.0, 1e-5), "RG": (1.0, 0.0053, 0.0, 1e-5),
       "BY": (34.1, 0.04, 13.5, 0.025)}
PPD = 0.7 * (3840 / 0.7) * math.pi / 180.0

# linear sRGB -> XYZ (D65) and its inverse
M_RGB2XYZ = np.array([[10135552 / 24577794, 8788810 / 24577794, 4435075 / 24577794],
                      [2613072 / 12288897, 8788810 / 12288897, 887015 / 12288897],
                      [1425312 / 73733382, 8788810 / 73733382, 70074185 / 73733382]])
M_XYZ2RGB = np.linalg.inv(M_RGB2XYZ)
WHITE = M_RGB2XYZ @ np.ones(3)


def _mat(m, img):
    return torch.einsum("ij,jhw->ihw", torch.from_numpy(m), img)


def srgb_to_linear(x):
    return torch.where(x > 0.04045, ((x + 0.055) / 1.055) ** 2.4, x / 12.92)


def xyz_to_ycxcz(xyz):
    n = xyz / torch.from_numpy(WHITE)[:, None, None]
    return torch.stack([116 * n[1] - 16, 500 * (n[0] - n[1]), 200 * (n[1] - n[2])])


def ycxcz_to_xyz(o):
    y = (o[0] + 16) / 116
    n = torch.stack([o[1] / 500 + y, y, y - o[2] / 200])
    return n * torch.from_numpy(WHITE)[:, None, None]


def xyz_to_lab(xyz):
    n = xyz / torch.from_numpy(WHITE)[:, None, None]
    d = 6.0 / 29.0
    f = torch.where(n > d ** 3, torch.clamp(n, min=d ** 3) ** (1.0 / 3.0), n / (3 * d * d) + 4.0 / 29.0)
    return torch.stack([116 * f[1] - 16, 500 * (f[0] - f[1]), 200 * (f[1] - f[2])])


def linear_to_lab(rgb):
    return xyz_to_lab(_mat(M_RGB2XYZ, rgb))


def srgb_to_ycxcz(x):
    return xyz_to_ycxcz(_mat(M_RGB2XYZ, srgb_to_linear(x)))


def csf_kernel(channel: str, ppd: float = PPD) -> np.ndarray:
    a1, b1, a2, b2 = CSF[channel]
    bmax = max(max(c[1], c[3]) for c in CSF.values())
    r = int(math.ceil(3 * math.sqrt(bmax / (2 * math.pi ** 2)) * ppd))
    x, y = np.meshgrid(np.arange(-r, r + 1), np.arange(-r, r + 1))
    z = (x / ppd) ** 2 + (y / ppd) ** 2
    g = (a1 * math.sqrt(math.pi / b1) * np.exp(-math.pi ** 2 * z / b1) +
         a2 * math.sqrt(math.pi / b2) * np.exp(-math.pi ** 2 * z / b2))
    return g / g.sum()


def feature_kernel(kind: str, ppd: float = PPD) -> np.ndarray:
    """2D kernel along x (transpose for y)."""
    sd = 0.5 * 0.082 * ppd
    r = int(math.ceil(3 * sd))
    x, y = np.meshgrid(np.arange(-r, r + 1), np.arange(-r, r + 1))
    g = np.exp(-(x ** 2 + y ** 2) / (2 * sd * sd))
    k = -x * g if kind == "edge" else (x ** 2 / (sd * sd) - 1) * g
    return np.where(k < 0, k / -k[k < 0].sum(), k / k[k > 0].sum())


def _filter(img, k):
    """2D correlation with edge replication, img [H][W]."""
    r = k.shape[0] // 2
    H, W = img.shape
    yi = torch.clamp(torch.arange(-r, H + r), 0, H - 1)
    xi = torch.clamp(torch.arange(-r, W + r), 0, W - 1)
    pad = img[yi][:, xi]
    out = torch.zeros_like(img)
    kt = torch.from_numpy(k)
    for i in range(k.shape[0]):
        for j in range(k.shape[1]):
            if k[i, j] != 0.0:
                out = out + kt[i, j] * pad[i:i + H, j:j + W]
    return out


def _hunt(lab):
    return torch.stack([lab[0], 0.01 * lab[0] * lab[1], 0.01 * lab[0] * lab[2]])


def _hyab(p, q):
    d = p - q
    return d[0].abs() + torch.sqrt(torch.clamp(d[1] ** 2 + d[2] ** 2, min=EPS))


def cmax() -> float:
    g = _hunt(linear_to_lab(torch.tensor([[[0.0]], [[1.0]], [[0.0]]], dtype=torch.float64)))
    b = _hunt(linear_to_lab(torch.tensor([[[0.0]], [[0.0]], [[1.0]]], dtype=torch.float64)))
    return float(_hyab(g, b)[0, 0]) ** QC


def flip_map(test: torch.Tensor, ref: torch.Tensor, ppd: float = PPD) -> torch.Tensor:
    """Per-pixel FLIP of sRGB images [3][H][W]."""
    t = srgb_to_ycxcz(torch.clamp(test, 0.0, 1.0))
    r = srgb_to_ycxcz(torch.clamp(ref, 0.0, 1.0))
    ks = [csf_kernel(c, ppd) for c in ("A", "RG", "BY")]

    def colour(o):
        f = torch.stack([_filter(o[c], ks[c]) for c in range(3)])
        rgb = torch.clamp(_mat(M_XYZ2RGB, ycxcz_to_xyz(f)), 0.0, 1.0)
        return _hunt(linear_to_lab(rgb))

    e = _hyab(colour(r), colour(t)) ** QC
    cm = cmax()
    dEc = torch.where(e < PC * cm, (PT / (PC * cm)) * e,
                      PT + ((e - PC * cm) / (cm - PC * cm)) * (1.0 - PT))
    ke, kp = feature_kernel("edge", ppd), feature_kernel("point", ppd)

    def feats(o):
        y = (o[0] + 16) / 116
        ex, ey = _filter(y, ke), _filter(y, ke.T.copy())
        px, py = _filter(y, kp), _filter(y, kp.T.copy())
        return torch.sqrt(ex * ex + ey * ey), torch.sqrt(px * px + py * py)

    er, pr = feats(r)
    et, pt_ = feats(t)
    dF = torch.clamp(torch.maximum((er - et).abs(), (pr - pt_).abs()), min=EPS)
    dF = (dF / math.sqrt(2.0)) ** QF
    return dEc ** (1.0 - dF)


def flip_and_grad(tests, refs, ppd: float = PPD):
    """Per-view mean FLIP and the gradient of their mean over the views with
    respect to every test image (lists of [3][H][W] arrays)."""
    ts = [torch.tensor(np.asarray(a, np.float64), requires_grad=True) for a in tests]
    rs = [torch.tensor(np.asarray(b, np.float64)) for b in refs]
    vals = [flip_map(t, r, ppd).mean() for t, r in zip(ts, rs)]
    total = sum(vals) / len(vals)
    grads = torch.autograd.grad(total, ts)
    return np.array([float(v.detach()) for v in vals]), [g.numpy() for g in grads]
