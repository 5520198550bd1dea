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


# ---------------------------------------------------------------------------
# Offline construction (Sec. 3.3 "Offline Clustering")
#
# Readings: the sampled poses are clustered with k-means on the same camera
# feature the runtime selection uses; seeding is farthest-point (pose 0, then
# repeatedly the pose whose distance to its nearest chosen centroid is
# largest, the lowest index on ties), then Lloyd iterations (assign to the
# nearest centroid, lowest index on ties; move each centroid to its members'
# mean, an empty cluster keeping its centroid) until no label changes or
# `iters` updates were made.  Per cluster, the union over its views' pixels
# of their top-k contributors (contrib.marks_and_sums) is its important set;
# the shared set is the union of the clusters' important sets.  Every other
# Gaussian with a positive summed contribution in some cluster is exclusive
# to the cluster where that sum is largest (the earlier cluster on ties);
# Gaussians that never blend belong to no segment and are placed last.

def default_pos_scale(cams) -> float:
    """The position normaliser when none is given (a reading: the paper
    normalises the camera position without naming the divisor): the largest
    distance of a sampled camera centre from the world origin."""
    return max(float(np.linalg.norm(-np.asarray(c.R, dtype=np.float64).T
                                     @ np.asarray(c.t, dtype=np.float64))) for c in cams)


def kmeans(features: np.ndarray, K: int, iters: int = 100):
    """(centroids [K, 6] float64, labels [n] int) of the poses' features."""
    f = np.asarray(features, dtype=np.float64)
    n = len(f)
    if not 1 <= K <= n:
        raise ValueError("need 1 <= K <= number of poses")
    chosen = [0]
    for _ in range(1, K):
        d_near = np.array([min(((f[p] - f[c]) ** 2).sum() for c in chosen) for p in range(n)])
        chosen.append(int(np.flatnonzero(d_near == d_near.max())[0]))
    cent = f[chosen].copy()
    labels = None
    for it in range(iters + 1):
        d = ((f[:, None, :] - cent[None, :, :]) ** 2).sum(-1)
        new = np.array([int(np.flatnonzero(d[p] == d[p].min())[0]) for p in range(n)])
        if labels is not None and (new == labels).all():
            break
        labels = new
        if it == iters:
            break
        for k in range(K):
            if (labels == k).any():
                cent[k] = f[labels == k].mean(0)
    return cent, labels


def partition(cluster_marks, cluster_sums, n: int):
    """Segment layout from each cluster's top-k marks (bool [n]) and summed
    contributions ([n]): (perm, seg_begin [1 + K], seg_count [1 + K]) with
    perm[new position] = original index over [shared | excl_0 | ... |
    excl_{K-1} | unused], the original order kept inside each segment."""
    K = len(cluster_marks)
    shared = np.zeros(n, dtype=bool)
    for m in cluster_marks:
        shared |= np.asarray(m, dtype=bool)
    seg = np.full(n, K + 1)
    for i in range(n):
        if shared[i]:
            seg[i] = 0
            continue
        best, best_c = 0.0, -1
        for c in range(K):
            if cluster_sums[c][i] > best:
                best, best_c = cluster_sums[c][i], c
        if best_c >= 0:
            seg[i] = 1 + best_c
    perm = np.concatenate([np.flatnonzero(seg == s) for s in range(K + 2)]).astype(np.int64)
    count = np.array([(seg == s).sum() for s in range(K + 1)], dtype=np.int64)
    begin = np.concatenate([[0], np.cumsum(count)[:-1]]).astype(np.int64)
    return perm, begin, count
