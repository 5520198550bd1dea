"""Fine-tuning loss and optimizer (Sec. 3.5), in float64 on the CPU (test
infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use the oracle).

The fine-tuning keeps the original 3DGS loss, L_3DGS = (1 - lambda) L1 +
lambda (1 - SSIM) with lambda = 0.2, and the 3DGS optimizer, Adam.  Readings
(the paper defers both to 3DGS): L1 is the mean absolute difference over
pixels and channels; SSIM is the mean over pixels and channels of the SSIM
map of each colour channel with an 11 x 11 Gaussian window of standard
deviation 1.5 (normalised to sum 1), out-of-image pixels counting as zero,
C1 = 0.01^2, C2 = 0.03^2; with several views the loss is the mean of the
per-view losses.  The gradient is torch autograd of this definition, in
float64.
"""
from __future__ import annotations

import numpy as np
import torch

C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window(size: int = 11, sigma: float = 1.5) -> np.ndarray:
    d = np.arange(size) - size // 2
    g = np.exp(-d * d / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def _window_sum(a: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """sum_q w[q - p + r] a[q] over the (2r+1)^2 window around every pixel,
    a zero outside the image; a is [C][H][W]."""
    r = w.shape[0] // 2
    C, H, W = a.shape
    pad = torch.zeros((C, H + 2 * r, W + 2 * r), dtype=a.dtype)
    pad[:, r:r + H, r:r + W] = a
    out = torch.zeros_like(a)
    for i in range(2 * r + 1):
        for j in range(2 * r + 1):
            out = out + w[i, j] * pad[:, i:i + H, j:j + W]
    return out


def ssim_map(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    w = torch.from_numpy(window())
    mx, my = _window_sum(x, w), _window_sum(y, w)
    sx = _window_sum(x * x, w) - mx * mx
    sy = _window_sum(y * y, w) - my * my
    sxy = _window_sum(x * y, w) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sx + sy + C2))


def photometric_loss(x: torch.Tensor, y: torch.Tensor, lam: float = 0.2) -> torch.Tensor:
    """L_3DGS of one view, x and y [3][H][W]."""
    return (1.0 - lam) * (x - y).abs().mean() + lam * (1.0 - ssim_map(x, y).mean())


def loss_and_grad(images, targets, lam: float = 0.2):
    """Per-view losses and the gradient of their mean with respect to every
    render (lists of [3][H][W] arrays)."""
    xs = [torch.tensor(np.asarray(a, np.float64), requires_grad=True) for a in images]
    ys = [torch.tensor(np.asarray(b, np.float64)) for b in targets]
    losses = [photometric_loss(x, y, lam) for x, y in zip(xs, ys)]
    total = sum(losses) / len(losses)
    grads = torch.autograd.grad(total, xs)
    return np.array([float(l.detach()) for l in losses]), [g.numpy() for g in grads]


def adam_step(p, g, m, v, lr, step: int, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-15):
    """One Adam step (bias-corrected moments); returns new (p, m, v)."""
    p, g, m, v = (np.asarray(a, np.float64) for a in (p, g, m, v))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    denom = np.sqrt(v) / np.sqrt(1.0 - b2 ** step) + eps
    return p - lr / (1.0 - b1 ** step) * m / denom, m, v
