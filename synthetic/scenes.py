"""Seeded Gaussian scenes and pinhole cameras (input generation only).

Layouts are structure-of-arrays, float32, matching what the device library
reads: ``means[3][N]``, ``log_scales[3][N]``, ``quats[4][N]`` (w, x, y, z, not
normalised), ``opacity_logits[N]``, ``sh[16][3][N]`` (coefficient, channel,
Gaussian).  Cameras use OpenCV axes (+x right, +y down, +z forward) and a
world-to-camera transform ``x_c = R x_w + t``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

SH_COEFFS = 16


@dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    sh_degree: int = 3

    @property
    def n(self) -> int:
        return int(self.opacity_logits.shape[0])

    def subset(self, idx: np.ndarray) -> "Scene":
        return Scene(
            np.ascontiguousarray(self.means[:, idx]),
            np.ascontiguousarray(self.log_scales[:, idx]),
            np.ascontiguousarray(self.quats[:, idx]),
            np.ascontiguousarray(self.opacity_logits[idx]),
            np.ascontiguousarray(self.sh[:, :, idx]),
            self.sh_degree,
        )

    def arrays(self):
        return dict(
            means=self.means,
            log_scales=self.log_scales,
            quats=self.quats,
            opacity_logits=self.opacity_logits,
            sh=self.sh,
        )


@dataclass
class Camera:
    R: np.ndarray  # (3, 3) float64, rows = camera axes in world coordinates
    t: np.ndarray  # (3,) float64
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def center(self) -> np.ndarray:
        return -self.R.T @ self.t


@dataclass
class HPLayout:
    """Gaussians reordered as [shared | excl_0 | ... | excl_{K-1}].

    ``seg_begin[0], seg_count[0]`` is the shared segment; entry ``1 + c`` is
    cluster ``c``'s exclusive segment.  ``centroids`` are the cluster centres
    in the (normalised camera position, beta * view direction) feature space,
    ``pos_scale`` the normalisation divisor for camera positions.
    """

    seg_begin: np.ndarray
    seg_count: np.ndarray
    centroids: np.ndarray  # (K, 6)
    pos_scale: float
    beta: float = 1.0
    labels: np.ndarray = field(default=None)  # per reordered Gaussian: -1 shared, else cluster


def _soa(means, log_scales, quats, logits, sh, sh_degree=3) -> Scene:
    return Scene(
        np.ascontiguousarray(means.T, dtype=np.float32),
        np.ascontiguousarray(log_scales.T, dtype=np.float32),
        np.ascontiguousarray(quats.T, dtype=np.float32),
        np.ascontiguousarray(logits, dtype=np.float32),
        np.ascontiguousarray(np.transpose(sh, (1, 2, 0)), dtype=np.float32),
        sh_degree,
    )


def _normal_quats(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def ball_scene(seed: int, n: int, log_scale_mu=-4.0, log_scale_sigma=0.5,
               logit_sigma=1.0, sh_sigma=0.3, radius=1.0, sh_degree=3) -> Scene:
    """Means uniform in a ball; log-scales, logits, SH normal (draw order:
    means, log-scales, quaternions, opacity logits, SH)."""
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    u = rng.uniform(size=(n, 1))
    means = radius * d * np.cbrt(u)
    log_scales = rng.normal(log_scale_mu, log_scale_sigma, size=(n, 3))
    quats = _normal_quats(rng, n)
    logits = rng.normal(0.0, logit_sigma, size=n)
    sh = rng.normal(0.0, sh_sigma, size=(n, SH_COEFFS, 3))
    return _soa(means, log_scales, quats, logits, sh, sh_degree)


def _random_rotations(rng, k):
    from scipy.spatial.transform import Rotation
    return Rotation.random(k, random_state=rng).as_matrix()


def cluster_scene(seed: int, n: int, n_clusters=64, bg_frac=0.1, cluster_radius=2.5,
                  sigma_lo=0.05, sigma_hi=0.6, shell_radius=20.0,
                  log_scale_mu=-5.0, log_scale_sigma=1.0, logit_sigma=1.5,
                  sh_sigma=0.3, sh_degree=3) -> Scene:
    """Outdoor-scene-shaped distribution: a mixture of anisotropic Gaussian
    clusters plus a uniform background shell, randomly permuted."""
    rng = np.random.default_rng(seed)
    n_bg = int(round(n * bg_frac))
    n_cl = n - n_bg
    # cluster centres uniform in a ball
    d = rng.normal(size=(n_clusters, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    centres = cluster_radius * d * np.cbrt(rng.uniform(size=(n_clusters, 1)))
    sig = np.exp(rng.uniform(math.log(sigma_lo), math.log(sigma_hi), size=(n_clusters, 3)))
    rot = _random_rotations(rng, n_clusters)
    assign = rng.integers(0, n_clusters, size=n_cl)
    z = rng.normal(size=(n_cl, 3)) * sig[assign]
    pts = centres[assign] + np.einsum("nij,nj->ni", rot[assign], z)
    # background shell
    b = rng.normal(size=(n_bg, 3))
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    means = np.concatenate([pts, shell_radius * b], axis=0)
    means = means[rng.permutation(n)]
    log_scales = rng.normal(log_scale_mu, log_scale_sigma, size=(n, 3))
    quats = _normal_quats(rng, n)
    logits = rng.normal(0.0, logit_sigma, size=n)
    sh = rng.normal(0.0, sh_sigma, size=(n, SH_COEFFS, 3)).astype(np.float32)
    return _soa(means, log_scales, quats, logits, sh, sh_degree)


def perturbed_scene(scene: Scene, seed: int, mean_sigma=0.01, logit_sigma=0.2) -> Scene:
    """Copy of ``scene`` with means + N(0, mean_sigma) and logits + N(0, logit_sigma)."""
    rng = np.random.default_rng(seed)
    means = scene.means + rng.normal(0.0, mean_sigma, size=scene.means.shape).astype(np.float32)
    logits = scene.opacity_logits + rng.normal(0.0, logit_sigma, size=scene.n).astype(np.float32)
    return Scene(np.ascontiguousarray(means, dtype=np.float32), scene.log_scales.copy(),
                 scene.quats.copy(), np.ascontiguousarray(logits, dtype=np.float32),
                 scene.sh.copy(), scene.sh_degree)


def focal_from_hfov(width: int, hfov_deg: float = 60.0) -> float:
    return (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)


def look_at(center, target=(0.0, 0.0, 0.0), width=256, height=256, hfov_deg=60.0,
            up=(0.0, -1.0, 0.0)) -> Camera:
    """Camera at ``center`` looking at ``target``; square pixels, principal
    point at the image centre, horizontal field of view ``hfov_deg``."""
    c = np.asarray(center, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - c
    f /= np.linalg.norm(f)
    x = np.cross(f, np.asarray(up, dtype=np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f])
    t = -R @ c
    fl = float(np.float32(focal_from_hfov(width, hfov_deg)))
    # every camera value is representable in float32, so both consumers of
    # the camera (float32 device path, float64 reference) see the same numbers
    R = R.astype(np.float32).astype(np.float64)
    t = t.astype(np.float32).astype(np.float64)
    return Camera(R, t, fl, fl, width / 2.0, height / 2.0, int(width), int(height))


def crop_camera(cam: Camera, x0: int, y0: int, width: int, height: int) -> Camera:
    """The same pinhole camera restricted to the pixel window [x0, x0 + width)
    x [y0, y0 + height) of its image: the principal point moves by the
    window's origin.  A window whose origin is a multiple of the tile size
    (and of the pixel-group size) renders exactly the same pixels as the full
    view, since every tile list and pixel group is unchanged."""
    return Camera(cam.R.copy(), cam.t.copy(), cam.fx, cam.fy, cam.cx - x0, cam.cy - y0,
                  int(width), int(height))


def orbit_cameras(n_views: int, radius: float, width: int, height: int, hfov_deg=60.0):
    cams = []
    for k in range(n_views):
        th = 2.0 * math.pi * k / n_views
        cams.append(look_at((radius * math.sin(th), 0.0, -radius * math.cos(th)),
                            width=width, height=height, hfov_deg=hfov_deg))
    return cams


def sampled_orbit_poses(seed: int, n_views: int, width: int, height: int, r_lo=3.5, r_hi=4.5,
                        y_max=0.5, hfov_deg=60.0):
    """Random poses around an orbit: angle uniform on the circle, radius
    uniform in [r_lo, r_hi], height uniform in [-y_max, y_max], looking at
    the origin (draw order per pose: angle, radius, height)."""
    rng = np.random.default_rng(seed)
    cams = []
    for _ in range(n_views):
        th = rng.uniform(0.0, 2.0 * math.pi)
        r = rng.uniform(r_lo, r_hi)
        y = rng.uniform(-y_max, y_max)
        cams.append(look_at((r * math.sin(th), y, -r * math.cos(th)), width=width, height=height,
                            hfov_deg=hfov_deg))
    return cams


def sphere_cameras(seed: int, n_views: int, r_lo=3.0, r_hi=6.0,
                   resolutions=((640, 480), (1280, 720), (1920, 1080)), hfov_deg=60.0,
                   max_abs_y=0.9):
    """Random poses on a spherical shell looking at the origin, each with a
    resolution drawn uniformly from ``resolutions``."""
    rng = np.random.default_rng(seed)
    cams = []
    while len(cams) < n_views:
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        r = rng.uniform(r_lo, r_hi)
        k = int(rng.integers(0, len(resolutions)))
        if abs(d[1]) > max_abs_y:
            continue
        w, h = resolutions[k]
        cams.append(look_at(r * d, width=w, height=h, hfov_deg=hfov_deg))
    return cams


def hp_membership(seed: int, n: int, n_clusters=8, shared_p=0.5429):
    """Seed-chosen view-dependent membership: -1 = shared, else the exclusive
    cluster index (uniform over clusters)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(size=n)
    c = rng.integers(0, n_clusters, size=n)
    return np.where(u < shared_p, -1, c).astype(np.int32)


def reorder_segments(scene: Scene, labels: np.ndarray, n_clusters: int, centroids: np.ndarray,
                     pos_scale: float, beta: float = 1.0):
    """Physically reorder Gaussians into [shared | excl_0 | ... | excl_{K-1}]
    (stable within each segment) and return the reordered scene + layout."""
    order = np.argsort(labels, kind="stable")  # -1 (shared) first, then 0..K-1
    lab = labels[order]
    counts = np.array([(lab == -1).sum()] + [(lab == c).sum() for c in range(n_clusters)],
                      dtype=np.int64)
    begins = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)
    layout = HPLayout(begins, counts, np.asarray(centroids, dtype=np.float64), float(pos_scale),
                      float(beta), lab)
    return scene.subset(order), layout
