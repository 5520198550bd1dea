"""The five seeded workloads (scene + cameras + render settings).

c1: 10k Gaussians in the unit ball, one 256x256 camera at distance 3.
c2: 3.0M-Gaussian outdoor-shaped scene, 32 orbit views at radius 4, 1920x1080.
c3: the c2 scene with a seed-chosen view-dependent membership (8 clusters,
    ~60% of Gaussians per cluster incl. the shared set), reordered into
    segments; hybrid preprocessing + contribution-aware rasterization.
c4: 1.0M Gaussians (c2 distribution), 8 orbit views at 1280x720, target
    images from a perturbed copy (means + N(0,0.01), logits + N(0,0.2)).
c5: 2.0M Gaussians (c2 distribution), 64 random cameras on a radius 3-6
    shell, resolutions drawn from {640x480, 1280x720, 1920x1080}.

``n`` overrides the Gaussian count (same distribution, smaller scene) so the
oracle can run the same workload shape in seconds.
"""
from __future__ import annotations

import math

import numpy as np

from .scenes import (ball_scene, cluster_scene, look_at, orbit_cameras, perturbed_scene,
                     sphere_cameras, hp_membership, reorder_segments)

ALPHA_MIN = 1.0 / 255.0
T_MIN = 1e-4


def _orbit_centroids(n_clusters: int, n_orbit: int, radius: float, beta: float = 1.0):
    """Cluster centres placed between orbit views (azimuth 2*pi*(s*c+0.5)/n_orbit
    with s = n_orbit / n_clusters) in (position / radius, beta * view dir) space."""
    step = n_orbit // n_clusters
    cents = []
    for c in range(n_clusters):
        phi = 2.0 * math.pi * (step * c + 0.5) / n_orbit
        pos = np.array([math.sin(phi), 0.0, -math.cos(phi)])
        cents.append(np.concatenate([pos, beta * (-pos)]))
    return np.stack(cents)


def config(k: int, n: int | None = None, n_views: int | None = None):
    """Return a dict: scene, cams, tile, and per-config extras."""
    if k == 1:
        scene = ball_scene(1, n or 10_000)
        cams = [look_at((0.0, 0.0, -3.0), width=256, height=256)]
        return dict(name="c1", scene=scene, cams=cams, tile=16)
    if k in (2, 3):
        scene = cluster_scene(2, n or 3_000_000)
        cams = orbit_cameras(32, 4.0, 1920, 1080)
        if n_views is not None:
            cams = cams[:n_views]
        out = dict(name=f"c{k}", scene=scene, cams=cams, tile=16)
        if k == 3:
            labels = hp_membership(3, scene.n, n_clusters=8)
            cents = _orbit_centroids(8, 32, 4.0)
            scene_r, layout = reorder_segments(scene, labels, 8, cents, pos_scale=4.0)
            out.update(scene=scene_r, hp=layout, M=0, group=2)
        return out
    if k == 4:
        scene = cluster_scene(4, n or 1_000_000)
        target = perturbed_scene(scene, 40)
        cams = orbit_cameras(8, 4.0, 1280, 720)
        if n_views is not None:
            cams = cams[:n_views]
        return dict(name="c4", scene=scene, target=target, cams=cams, tile=16)
    if k == 5:
        scene = cluster_scene(5, n or 2_000_000)
        cams = sphere_cameras(50, n_views or 64)
        return dict(name="c5", scene=scene, cams=cams, tile=16)
    raise ValueError(f"unknown config {k}")
