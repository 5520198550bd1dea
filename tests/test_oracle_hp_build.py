"""Pins for the oracle's offline construction of the view-dependent
representation (Sec. 3.3 "Offline Clustering"): k-means on well-separated
blobs, the K = 1 and K = n special cases, the fixed point Lloyd's method
stops at, brute force over every partition of tiny pose sets, and the
segment layout against a hand-worked example and its invariants (CPU only)."""
import itertools

import numpy as np

import synthetic
from oracle import hp


def _same_partition(a, b):
    pairs = {}
    for x, y in zip(a, b):
        if pairs.setdefault(x, y) != y:
            return False
    return len(set(pairs.values())) == len(pairs)


def test_kmeans_separated_blobs():
    rng = np.random.default_rng(1)
    centres = rng.normal(size=(5, 6)) * 20
    truth = rng.integers(0, 5, size=200)
    truth[:5] = np.arange(5)
    f = centres[truth] + rng.normal(size=(200, 6)) * 0.1
    cent, lab = hp.kmeans(f, 5)
    assert _same_partition(lab, truth)
    for k in range(5):
        np.testing.assert_allclose(cent[k], f[lab == k].mean(0), atol=1e-12)


def test_kmeans_special_cases():
    rng = np.random.default_rng(2)
    f = rng.normal(size=(9, 6))
    cent, lab = hp.kmeans(f, 1)
    assert (lab == 0).all()
    np.testing.assert_allclose(cent[0], f.mean(0), atol=1e-12)
    cent, lab = hp.kmeans(f, 9)
    assert sorted(lab) == list(range(9))
    np.testing.assert_allclose(cent[lab], f, atol=0)
    # iters = 0: the centroids are the seeds; seed 1 is the pose farthest
    # from pose 0, seed 2 the one farthest from both
    cent, _ = hp.kmeans(f, 3, iters=0)
    d0 = [np.linalg.norm(f[p] - f[0]) for p in range(9)]
    s1 = int(np.argmax(d0))
    d01 = [min(d0[p], np.linalg.norm(f[p] - f[s1])) for p in range(9)]
    s2 = int(np.argmax(d01))
    np.testing.assert_array_equal(cent, f[[0, s1, s2]])


def test_kmeans_stops_at_a_fixed_point_and_tiny_optimum():
    rng = np.random.default_rng(3)
    for trial in range(20):
        n, K = int(rng.integers(3, 8)), int(rng.integers(1, 4))
        K = min(K, n)
        f = rng.normal(size=(n, 6))
        cent, lab = hp.kmeans(f, K)
        # fixed point: every pose sits with its nearest centroid, every
        # non-empty centroid is the mean of its poses
        for p in range(n):
            d = [np.linalg.norm(f[p] - c) for c in cent]
            assert d[lab[p]] <= min(d) + 1e-12
        for k in set(lab.tolist()):
            np.testing.assert_allclose(cent[k], f[lab == k].mean(0), atol=1e-12)
        # it is never worse than the seeds and, on two well-separated groups,
        # equals the best of every K = 2 partition (brute force)
        if K == 2:
            g = np.concatenate([rng.normal(size=(3, 6)), rng.normal(size=(3, 6)) + 50])
            _, lab2 = hp.kmeans(g, 2)
            best = min(
                (sum(((g[[i for i in range(6) if a[i] == k]] -
                       g[[i for i in range(6) if a[i] == k]].mean(0)) ** 2).sum()
                     for k in (0, 1) if k in a), a)
                for a in itertools.product((0, 1), repeat=6) if 0 < sum(a) < 6)
            assert _same_partition(lab2, best[1])


def test_kmeans_on_orbit_cameras_groups_neighbours():
    # 24 views on an orbit, 4 clusters: every cluster is 6 consecutive views
    cams = synthetic.orbit_cameras(24, 4.0, 64, 64)
    f = np.stack([hp.camera_feature(c, 4.0) for c in cams])
    _, lab = hp.kmeans(f, 4)
    changes = sum(lab[i] != lab[(i + 1) % 24] for i in range(24))
    assert changes == 4 and np.bincount(lab).tolist() == [6, 6, 6, 6]


def test_partition_hand_example():
    # 7 Gaussians, 2 clusters
    marks = [np.array([1, 0, 0, 0, 0, 0, 0], bool), np.array([0, 0, 1, 0, 0, 0, 0], bool)]
    sums = [np.array([.9, .2, .1, .0, .3, .0, .5]), np.array([.1, .4, .8, .0, .3, .0, .0])]
    perm, begin, count = hp.partition(marks, sums, 7)
    # shared {0, 2}; 1 -> cluster 1 (.4 > .2); 4 -> cluster 0 (tie keeps the
    # earlier); 6 -> cluster 0; 3, 5 never blend
    assert perm.tolist() == [0, 2, 4, 6, 1, 3, 5]
    assert begin.tolist() == [0, 2, 4] and count.tolist() == [2, 2, 1]


def test_partition_invariants():
    rng = np.random.default_rng(4)
    n, K = 500, 5
    marks = [rng.random(n) < 0.05 for _ in range(K)]
    sums = [np.where(rng.random(n) < 0.5, rng.integers(0, 4, n) / 4.0, 0.0) for _ in range(K)]
    perm, begin, count = hp.partition(marks, sums, n)
    assert sorted(perm.tolist()) == list(range(n))
    shared = np.any(marks, axis=0)
    S = np.stack(sums)
    for s in range(K + 1):
        seg = perm[begin[s]:begin[s] + count[s]]
        assert (np.diff(seg) > 0).all()
        if s == 0:
            assert set(seg.tolist()) == set(np.flatnonzero(shared).tolist())
        else:
            for i in seg:
                assert not shared[i] and S[s - 1, i] == S[:, i].max() > 0
                assert (S[:s - 1, i] < S[s - 1, i]).all()
    rest = perm[begin[-1] + count[-1]:]
    assert all(not shared[i] and S[:, i].max() == 0 for i in rest)


def test_default_pos_scale_is_the_farthest_camera_centre():
    # orbit cameras all sit at radius 4; a camera placed at (3, 4, 12) is 13 from the origin
    cams = synthetic.orbit_cameras(8, 4.0, 64, 64)
    assert abs(hp.default_pos_scale(cams) - 4.0) < 1e-6
    far = synthetic.look_at((3.0, 4.0, 12.0))
    assert abs(hp.default_pos_scale(cams + [far]) - 13.0) < 1e-5
    assert abs(hp.default_pos_scale([far]) - 13.0) < 1e-5
