"""Scene storage order: the Morton order of the means (test infrastructure:
only the tests, the smoke check and the benchmark's CPU baseline use the
oracle).

Not a step of the paper's method: a layout choice.  Written out from its
definition: each coordinate is quantised over the box of the finite
coordinates, q = min(1023, floor((x - lo) * (1024 / (hi - lo)))) in float32
(1023 for a non-finite coordinate, 0 on a flat axis), the three 10-bit
values are interleaved (bit 3k + a of the code is bit k of axis a), and the
Gaussians are stably sorted by code.
"""
from __future__ import annotations

import numpy as np


def interleave(qx: int, qy: int, qz: int) -> int:
    code = 0
    for k in range(10):
        code |= ((qx >> k) & 1) << (3 * k)
        code |= ((qy >> k) & 1) << (3 * k + 1)
        code |= ((qz >> k) & 1) << (3 * k + 2)
    return code


def quantise(means: np.ndarray) -> np.ndarray:
    """[3][n] float32 -> [3][n] uint32 cells."""
    m = np.asarray(means, dtype=np.float32)
    q = np.full(m.shape, 1023, dtype=np.uint32)
    for a in range(3):
        fin = np.isfinite(m[a])
        if not fin.any():
            continue
        lo, hi = m[a][fin].min(), m[a][fin].max()
        ext = np.float32(hi - lo)
        scale = np.float32(1024.0) / ext if ext > 0 and np.isfinite(ext) else np.float32(0.0)
        t = (m[a][fin] - lo).astype(np.float32) * scale
        q[a][fin] = np.where(t >= 1023, 1023, np.floor(t)).astype(np.uint32)
    return q


def morton_order(means: np.ndarray) -> np.ndarray:
    q = quantise(means)
    codes = np.array([interleave(int(a), int(b), int(c)) for a, b, c in zip(*q)], dtype=np.int64)
    return np.argsort(codes, kind="stable")
