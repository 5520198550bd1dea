"""Per-view preprocessing in float64 (Sec. 3.1 "Preprocessing"; Eq. 2's
screen-space mean x' and covariance Sigma' via the EWA splatting of
Zwicker et al.; Sec. 3.3 "Online Filtering", Eqs. 3-5).

Steps, in the order the hot path applies them:
  1. activations: s = exp(log_scale), unit quaternion (w, x, y, z) -> R,
     Sigma = R diag(s^2) R^T, opacity o = sigmoid(logit);
  2. camera transform t = R_w x + t_w, cull t_z <= z_near;
  3. EWA: J = d(projection)/dt at t, Sigma' = J R_w Sigma R_w^T J^T + lowpass*I,
     conic A = Sigma'^{-1}, x' = (f_x t_x/t_z + c_x, f_y t_y/t_z + c_y);
  4. extent: plain = circle of radius 3*sqrt(lambda_max(Sigma')) (the 3-sigma
     envelope of Eq. 3); opacity-aware = tight box of the ellipse
     d^T A d <= tau, tau = min(2 ln(o/alpha_theta), 9) (Eq. 5), culled when
     tau <= 0;  plain mode culls o < alpha_theta (such a Gaussian can never
     reach alpha_theta, so the image is unchanged);
  5. tile rectangle [x0, x1) x [y0, y1) of tiles overlapping the extent box;
  6. colour rgb = max(0, 0.5 + sum_lm Y_lm(d) k_lm) with d the unit direction
     from the camera centre to the mean; depth = t_z.
Readings for points the paper leaves open (low-pass 0.3 px^2, z_near 0.2,
no Jacobian clamp, pixel centres at +0.5, SH convention) are listed in the
design notes and the module docstrings.
"""
from __future__ import annotations

import math

import numpy as np

from . import sh as _sh

ALPHA_THETA = 1.0 / 255.0
DEFAULTS = dict(alpha_min=ALPHA_THETA, lowpass=0.3, z_near=0.2, tile=16, extent="3sigma")


def quat_to_rotmat(q: np.ndarray) -> np.ndarray:
    """(N, 4) quaternions (w, x, y, z), any norm -> (N, 3, 3) rotation matrices."""
    q = np.asarray(q, dtype=np.float64)
    n = np.linalg.norm(q, axis=1, keepdims=True)
    with np.errstate(invalid="ignore", divide="ignore"):
        qn = q / n
    w, x, y, z = qn[:, 0], qn[:, 1], qn[:, 2], qn[:, 3]
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1.0 - 2.0 * (y * y + z * z)
    R[:, 0, 1] = 2.0 * (x * y - w * z)
    R[:, 0, 2] = 2.0 * (x * z + w * y)
    R[:, 1, 0] = 2.0 * (x * y + w * z)
    R[:, 1, 1] = 1.0 - 2.0 * (x * x + z * z)
    R[:, 1, 2] = 2.0 * (y * z - w * x)
    R[:, 2, 0] = 2.0 * (x * z - w * y)
    R[:, 2, 1] = 2.0 * (y * z + w * x)
    R[:, 2, 2] = 1.0 - 2.0 * (x * x + y * y)
    return R


def covariance3d(log_scales: np.ndarray, quats: np.ndarray) -> np.ndarray:
    """Sigma = R S S^T R^T with S = diag(exp(log_scales)); inputs (N,3), (N,4)."""
    s = np.exp(np.asarray(log_scales, dtype=np.float64))
    M = quat_to_rotmat(quats) * s[:, None, :]
    return M @ np.transpose(M, (0, 2, 1))


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-np.asarray(x, dtype=np.float64)))


def camera_arrays(cam):
    return (np.asarray(cam.R, dtype=np.float64), np.asarray(cam.t, dtype=np.float64),
            float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy))


def ewa_jacobian(t: np.ndarray, fx: float, fy: float) -> np.ndarray:
    """Jacobian of (f_x t_x/t_z, f_y t_y/t_z) with respect to t: (N, 2, 3)."""
    tx, ty, tz = t[:, 0], t[:, 1], t[:, 2]
    J = np.zeros((t.shape[0], 2, 3))
    J[:, 0, 0] = fx / tz
    J[:, 0, 2] = -fx * tx / (tz * tz)
    J[:, 1, 1] = fy / tz
    J[:, 1, 2] = -fy * ty / (tz * tz)
    return J


def scene_aos(scene):
    """SoA float32 arrays of a ``synthetic.Scene`` -> float64 per-Gaussian rows."""
    return dict(
        means=scene.means.T.astype(np.float64),
        log_scales=scene.log_scales.T.astype(np.float64),
        quats=scene.quats.T.astype(np.float64),
        logits=scene.opacity_logits.astype(np.float64),
        sh=np.transpose(scene.sh, (2, 0, 1)).astype(np.float64),  # (N, 16, 3)
        sh_degree=int(scene.sh_degree),
    )


def project_view(scene, cam, tile: int = 16, extent: str = "3sigma",
                 alpha_min: float = ALPHA_THETA, lowpass: float = 0.3, z_near: float = 0.2,
                 active: np.ndarray | None = None) -> dict:
    """Project every Gaussian of ``scene`` for camera ``cam``.

    Returns float64 per-Gaussian arrays (invisible Gaussians have
    ``n_tiles == 0`` and zero rect) plus decision margins used by the tests
    to recognise float32-vs-float64 borderline cases.
    """
    g = scene_aos(scene)
    n = g["means"].shape[0]
    Rw, tw, fx, fy, cx, cy = camera_arrays(cam)
    W, H = int(cam.width), int(cam.height)
    grid_w, grid_h = -(-W // tile), -(-H // tile)

    with np.errstate(all="ignore"):
        nb_used = (g["sh_degree"] + 1) ** 2
        finite = (np.isfinite(g["means"]).all(1) & np.isfinite(g["log_scales"]).all(1)
                  & np.isfinite(g["quats"]).all(1) & np.isfinite(g["logits"])
                  & np.isfinite(g["sh"][:, :nb_used, :]).all((1, 2))
                  & (np.linalg.norm(g["quats"], axis=1) > 0))
        Sigma = covariance3d(g["log_scales"], g["quats"])
        o = sigmoid(g["logits"])
        t = g["means"] @ Rw.T + tw
        tz = t[:, 2]
        in_front = tz > z_near
        J = ewa_jacobian(t, fx, fy)
        T = J @ Rw  # (N, 2, 3)
        cov2 = T @ Sigma @ np.transpose(T, (0, 2, 1))
        a = cov2[:, 0, 0] + lowpass
        b = cov2[:, 0, 1]
        c = cov2[:, 1, 1] + lowpass
        det = a * c - b * b
        conic = np.stack([c / det, -b / det, a / det], axis=1)
        mean2d = np.stack([fx * t[:, 0] / tz + cx, fy * t[:, 1] / tz + cy], axis=1)

        if extent == "3sigma":
            mid = 0.5 * (a + c)
            lam = mid + np.sqrt(np.maximum(0.0, mid * mid - det))
            r = 3.0 * np.sqrt(lam)
            ex, ey = r, r
            op_ok = o >= alpha_min
            tau = np.full(n, np.nan)
        elif extent == "opacity":
            tau = np.minimum(2.0 * np.log(o / alpha_min), 9.0)
            op_ok = tau > 0
            ex = np.sqrt(tau * a)
            ey = np.sqrt(tau * c)
        else:
            raise ValueError(extent)

        fx0 = np.floor((mean2d[:, 0] - ex) / tile)
        fx1 = np.floor((mean2d[:, 0] + ex) / tile) + 1
        fy0 = np.floor((mean2d[:, 1] - ey) / tile)
        fy1 = np.floor((mean2d[:, 1] + ey) / tile) + 1
        x0 = np.clip(fx0, 0, grid_w)
        x1 = np.clip(fx1, 0, grid_w)
        y0 = np.clip(fy0, 0, grid_h)
        y1 = np.clip(fy1, 0, grid_h)

        ok = finite & in_front & (det > 0) & np.isfinite(conic).all(1) & op_ok
        ok &= np.isfinite(mean2d).all(1) & np.isfinite(ex) & np.isfinite(ey)
        if active is not None:
            ok &= np.asarray(active, dtype=bool)
        ok &= (x1 > x0) & (y1 > y0)

        # colour toward the camera
        centre = -Rw.T @ tw
        v = g["means"] - centre
        dist = np.linalg.norm(v, axis=1, keepdims=True)
        d = v / dist
        deg = g["sh_degree"]
        nb = (deg + 1) ** 2
        Y = _sh.basis(np.where(np.isfinite(d), d, 0.0), deg)  # (N, nb)
        rgb_raw = 0.5 + np.einsum("nk,nkc->nc", Y, g["sh"][:, :nb, :])
        rgb = np.maximum(rgb_raw, 0.0)

        rect = np.stack([x0, y0, x1, y1], axis=1)
        rect = np.where(ok[:, None], rect, 0).astype(np.int64)
        n_tiles = np.where(ok, (rect[:, 2] - rect[:, 0]) * (rect[:, 3] - rect[:, 1]), 0)

        # decision margins (distance from each decision boundary)
        edges = np.stack([(mean2d[:, 0] - ex) / tile, (mean2d[:, 0] + ex) / tile,
                          (mean2d[:, 1] - ey) / tile, (mean2d[:, 1] + ey) / tile], axis=1)
        rect_margin = np.min(np.abs(edges - np.round(edges)), axis=1) * tile  # pixels
        op_margin = np.abs(o - alpha_min) / alpha_min
        near_margin = np.abs(tz - z_near)

    return dict(
        visible=ok, mean2d=mean2d, cov2d=np.stack([a, b, c], axis=1), conic=conic, opacity=o,
        rgb=rgb, rgb_raw=rgb_raw, depth=tz, rect=rect, n_tiles=n_tiles.astype(np.int64),
        t=t, tau=tau, ex=ex, ey=ey, dir=d, dist=dist[:, 0], sh_basis=Y,
        grid_w=grid_w, grid_h=grid_h, tile=tile, width=W, height=H,
        rect_margin=rect_margin, op_margin=op_margin, near_margin=near_margin,
    )
