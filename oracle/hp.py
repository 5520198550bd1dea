"""Runtime active-set selection of hybrid preprocessing (Sec. 3.3,
"View-Dependent Scene Representation" and "Algorithm").

The camera feature concatenates the camera position divided by a scene
normalisation constant and beta times the unit view direction (beta = 1 in
the paper).  The nearest cluster centroid (Euclidean distance in that
feature space) is selected, together with the M clusters whose centroids are
nearest to that cluster's centroid (a reading of "this cluster and its M
neighboring clusters"); ties go to the lower cluster index.  The active set
is the shared segment plus the exclusive segments of the selected clusters.
"""
from __future__ import annotations

import numpy as np


def camera_feature(cam, pos_scale: float, beta: float = 1.0) -> np.ndarray:
    R = np.asarray(cam.R, dtype=np.float64)
    t = np.asarray(cam.t, dtype=np.float64)
    centre = -R.T @ t
    view_dir = R[2]  # camera +z axis in world coordinates
    return np.concatenate([centre / pos_scale, beta * view_dir])


def select_clusters(centroids: np.ndarray, feature: np.ndarray, M: int) -> list:
    c = np.asarray(centroids, dtype=np.float64)
    d = np.sqrt(((c - feature[None, :]) ** 2).sum(1))
    nearest = int(min(range(len(c)), key=lambda k: (d[k], k)))
    dn = np.sqrt(((c - c[nearest][None, :]) ** 2).sum(1))
    others = sorted((k for k in range(len(c)) if k != nearest), key=lambda k: (dn[k], k))
    return [nearest] + [int(k) for k in others[:M]]


def active_segments(seg_begin, seg_count, clusters) -> list:
    """(begin, count) segments: shared (entry 0) plus each selected cluster's
    exclusive segment (entry 1 + c), sorted by begin, empty ones dropped."""
    segs = [(int(seg_begin[0]), int(seg_count[0]))]
    segs += [(int(seg_begin[1 + c]), int(seg_count[1 + c])) for c in sorted(set(clusters))]
    return sorted(s for s in segs if s[1] > 0)


def active_mask(n: int, segments) -> np.ndarray:
    m = np.zeros(n, dtype=bool)
    for b, c in segments:
        m[b:b + c] = True
    return m
