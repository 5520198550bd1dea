"""Adjoint of the rendering pipeline in float64 (Sec. 3.5: fine-tuning
back-propagates through the unchanged 3DGS pipeline; the hybrid-preprocessing
and contribution-aware decisions are constants of the backward pass).

Blend adjoint (per pixel, entries it blended, last first).  With T_j the
transmittance before entry j, S the colour accumulated behind j (including
T_final * bg) and g = dL/dC:
    dL/dc_j     = T_j alpha_j g
    dL/dalpha_j = sum_ch g_ch (T_j c_j,ch - S_ch / (1 - alpha_j))
then alpha = o exp(-q/2) (zero derivative where the 0.99 clamp is active),
q = d^T A d with d = p - x':  dq/dx' = -2 A d,  dq/d(a, b, c) = (dx^2, 2 dx dy, dy^2).

Preprocess adjoint (per Gaussian and view): conic -> Sigma' (dSigma' = -A dA A),
Sigma' = T Sigma T^T + lowpass I with T = J R_w, through J(t) and x'(t) to
t = R_w x + t_w, Sigma = M M^T with M = R(q) diag(exp(s)) to log-scales and the
normalised quaternion, then the quaternion normalisation; colour
max(0, 0.5 + sum Y k) to the SH coefficients and, through the view direction,
to the mean; sigmoid to the opacity logit.
"""
from __future__ import annotations

import numpy as np

from . import sh as _sh
from .project import quat_to_rotmat, scene_aos, camera_arrays, project_view
from .blend import render_view, splats_from_projection


def blend_adjoint(splats: dict, sorted_ids, ranges, lists: dict, dL_dimage: np.ndarray,
                  width: int, height: int, tile: int, tile_base: int = 0,
                  bg=(0.0, 0.0, 0.0), alpha_max: float = 0.99) -> dict:
    """Gradients with respect to each record's 2D mean, conic (a, b, c),
    opacity and colour.  ``lists[(y, x)]`` holds the list positions the pixel
    blended (from ``render_tiles(collect_lists=True)``)."""
    mean2d = np.asarray(splats["mean2d"], dtype=np.float64)
    conic = np.asarray(splats["conic"], dtype=np.float64)
    opac = np.asarray(splats["opacity"], dtype=np.float64)
    rgb = np.asarray(splats["rgb"], dtype=np.float64)
    R = mean2d.shape[0]
    gm = np.zeros((R, 2))
    gA = np.zeros((R, 3))
    go = np.zeros(R)
    gc = np.zeros((R, 3))
    bg = np.asarray(bg, dtype=np.float64)
    grid_w = -(-width // tile)
    for (y, x), js in lists.items():
        if not js:
            continue
        t = tile_base + (y // tile) * grid_w + (x // tile)
        s, _ = ranges[t]
        px, py = x + 0.5, y + 0.5
        g_pix = dL_dimage[:, y, x]
        recs = [int(sorted_ids[s + j]) for j in js]
        alphas, raws, Ts, ds = [], [], [], []
        T = 1.0
        for r in recs:
            dx, dy = px - mean2d[r, 0], py - mean2d[r, 1]
            a, b, c = conic[r]
            q = max(0.0, a * dx * dx + 2 * b * dx * dy + c * dy * dy)
            raw = opac[r] * np.exp(-0.5 * q)
            al = min(alpha_max, raw)
            alphas.append(al)
            raws.append(raw)
            Ts.append(T)
            ds.append((dx, dy))
            T = T * (1.0 - al)
        S = T * bg  # T is now the final transmittance
        for k in range(len(recs) - 1, -1, -1):
            r, al, Tj = recs[k], alphas[k], Ts[k]
            gc[r] += Tj * al * g_pix
            d_alpha = float(np.sum(g_pix * (Tj * rgb[r] - S / (1.0 - al))))
            S = S + Tj * al * rgb[r]
            if raws[k] > alpha_max:
                continue  # clamped: alpha does not depend on o or q
            G = raws[k] / opac[r]
            go[r] += d_alpha * G
            dq = d_alpha * (-0.5 * al)
            dx, dy = ds[k]
            a, b, c = conic[r]
            gm[r, 0] += dq * (-2.0) * (a * dx + b * dy)
            gm[r, 1] += dq * (-2.0) * (b * dx + c * dy)
            gA[r] += dq * np.array([dx * dx, 2.0 * dx * dy, dy * dy])
    return dict(mean2d=gm, conic=gA, opacity=go, rgb=gc)


def _drot_dq(qn: np.ndarray) -> np.ndarray:
    """d R_ij / d qhat_k for unit quaternions (w, x, y, z): (N, 3, 3, 4)."""
    w, x, y, z = qn[:, 0], qn[:, 1], qn[:, 2], qn[:, 3]
    D = np.zeros((qn.shape[0], 3, 3, 4))
    z0 = np.zeros_like(w)
    D[:, 0, 0] = np.stack([z0, z0, -4 * y, -4 * z], 1)
    D[:, 0, 1] = np.stack([-2 * z, 2 * y, 2 * x, -2 * w], 1)
    D[:, 0, 2] = np.stack([2 * y, 2 * z, 2 * w, 2 * x], 1)
    D[:, 1, 0] = np.stack([2 * z, 2 * y, 2 * x, 2 * w], 1)
    D[:, 1, 1] = np.stack([z0, -4 * x, z0, -4 * z], 1)
    D[:, 1, 2] = np.stack([-2 * x, -2 * w, 2 * z, 2 * y], 1)
    D[:, 2, 0] = np.stack([-2 * y, 2 * z, -2 * w, 2 * x], 1)
    D[:, 2, 1] = np.stack([2 * x, 2 * w, 2 * z, 2 * y], 1)
    D[:, 2, 2] = np.stack([z0, -4 * x, -4 * y, z0], 1)
    return D


def preprocess_adjoint(scene, cam, proj: dict, g2d: dict) -> dict:
    """Chain per-Gaussian 2D gradients of one view back to the raw
    parameters.  Gaussians that are not visible get zero gradient."""
    g = scene_aos(scene)
    n = g["means"].shape[0]
    Rw, tw, fx, fy, cx, cy = camera_arrays(cam)
    vis = proj["visible"]
    out = dict(means=np.zeros((n, 3)), log_scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
               logits=np.zeros(n), sh=np.zeros((n, 16, 3)))
    idx = np.nonzero(vis)[0]
    if idx.size == 0:
        return out
    t = proj["t"][idx]
    tx, ty, tz = t[:, 0], t[:, 1], t[:, 2]
    # colour
    mask = (proj["rgb_raw"][idx] > 0).astype(np.float64)
    graw = g2d["rgb"][idx] * mask  # (k, 3)
    deg = g["sh_degree"]
    nb = (deg + 1) ** 2
    Y = proj["sh_basis"][idx]  # (k, nb)
    out["sh"][idx, :nb, :] = Y[:, :, None] * graw[:, None, :]
    dY = _sh.basis_grad(proj["dir"][idx], deg)  # (k, nb, 3)
    coeff = g["sh"][idx, :nb, :]  # (k, nb, 3)
    g_dir = np.einsum("kc,klc,kld->kd", graw, coeff, dY)
    dvec = proj["dir"][idx]
    dist = proj["dist"][idx][:, None]
    g_mean = (g_dir - dvec * np.sum(dvec * g_dir, 1, keepdims=True)) / dist
    # opacity
    o = proj["opacity"][idx]
    out["logits"][idx] = g2d["opacity"][idx] * o * (1.0 - o)
    # conic -> Sigma'
    A = proj["conic"][idx]
    Am = np.zeros((idx.size, 2, 2))
    Am[:, 0, 0], Am[:, 0, 1], Am[:, 1, 0], Am[:, 1, 1] = A[:, 0], A[:, 1], A[:, 1], A[:, 2]
    gAv = g2d["conic"][idx]
    GA = np.zeros((idx.size, 2, 2))
    GA[:, 0, 0], GA[:, 1, 1] = gAv[:, 0], gAv[:, 2]
    GA[:, 0, 1] = GA[:, 1, 0] = 0.5 * gAv[:, 1]
    Gs2 = -Am @ GA @ Am  # dL/dSigma' (symmetric)
    # Sigma' = T Sigma T^T + lowpass I,  T = J W
    J = np.zeros((idx.size, 2, 3))
    J[:, 0, 0] = fx / tz
    J[:, 0, 2] = -fx * tx / tz ** 2
    J[:, 1, 1] = fy / tz
    J[:, 1, 2] = -fy * ty / tz ** 2
    Tm = J @ Rw
    M = quat_to_rotmat(g["quats"][idx]) * np.exp(g["log_scales"][idx])[:, None, :]
    Sigma = M @ np.transpose(M, (0, 2, 1))
    GSig = np.transpose(Tm, (0, 2, 1)) @ Gs2 @ Tm
    GT = 2.0 * Gs2 @ Tm @ Sigma
    GJ = GT @ Rw.T
    g_t = np.zeros((idx.size, 3))
    g_t[:, 0] += GJ[:, 0, 2] * (-fx / tz ** 2)
    g_t[:, 1] += GJ[:, 1, 2] * (-fy / tz ** 2)
    g_t[:, 2] += (GJ[:, 0, 0] * (-fx / tz ** 2) + GJ[:, 0, 2] * (2 * fx * tx / tz ** 3)
                  + GJ[:, 1, 1] * (-fy / tz ** 2) + GJ[:, 1, 2] * (2 * fy * ty / tz ** 3))
    # 2D mean: x' = (fx tx/tz + cx, fy ty/tz + cy) has Jacobian J
    g_t += np.einsum("kij,ki->kj", J, g2d["mean2d"][idx])
    g_mean += g_t @ Rw
    out["means"][idx] = g_mean
    # Sigma = M M^T, M = R S
    GM = 2.0 * GSig @ M
    s = np.exp(g["log_scales"][idx])
    Rq = quat_to_rotmat(g["quats"][idx])
    gs = np.sum(GM * Rq, axis=1)  # dL/ds_j = sum_i GM_ij R_ij
    out["log_scales"][idx] = gs * s
    GR = GM * s[:, None, :]
    q = g["quats"][idx]
    qnorm = np.linalg.norm(q, axis=1, keepdims=True)
    qn = q / qnorm
    g_qn = np.einsum("kij,kijl->kl", GR, _drot_dq(qn))
    out["quats"][idx] = (g_qn - qn * np.sum(qn * g_qn, 1, keepdims=True)) / qnorm
    return out


def render_and_grad(scene, cams, dL_dimages, tile: int = 16, extent: str = "3sigma",
                    mode: str = "plain", group=(2, 2), bg=(0.0, 0.0, 0.0),
                    alpha_max: float = 0.99, lowpass: float = 0.3, z_near: float = 0.2) -> dict:
    """Full float64 forward and adjoint over several views; gradients summed."""
    n = scene.n
    total = dict(means=np.zeros((n, 3)), log_scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
                 logits=np.zeros(n), sh=np.zeros((n, 16, 3)))
    images = []
    for cam, G in zip(cams, dL_dimages):
        proj = project_view(scene, cam, tile=tile, extent=extent, lowpass=lowpass, z_near=z_near)
        r = render_view(proj, mode=mode, group=group, bg=bg, alpha_max=alpha_max,
                        collect_lists=True)
        images.append(r["image"])
        b = r["binning"]
        g2 = blend_adjoint(splats_from_projection(proj), b["ids"], b["ranges"], r["lists"], G,
                           proj["width"], proj["height"], tile, 0, bg, alpha_max)
        d = preprocess_adjoint(scene, cam, proj, g2)
        for k in total:
            total[k] += d[k]
    total["images"] = images
    return total
