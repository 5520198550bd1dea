"""Pins for the oracle's per-pixel contributions and top-k ranking (Sec. 3.3
"Offline Clustering"): closed forms, the telescoping identity of Eq. 1's
weights, and brute force on tiny scenes (CPU only)."""
import math

import numpy as np

import synthetic
from oracle import binning, blend, contrib, project

A_T = 1.0 / 255.0


def _tile(mean2d, conic, opacity, size=16):
    L = len(opacity)
    sp = dict(mean2d=np.asarray(mean2d, float), conic=np.asarray(conic, float),
              opacity=np.asarray(opacity, float), rgb=np.full((L, 3), 0.5))
    return sp, np.array([[0, L]]), np.arange(L)


def test_single_gaussian_weight_is_its_alpha():
    # one Gaussian, T = 1 in front of it: the weight is alpha itself,
    # o * exp(-q/2) with q = d^T A d, written out here per pixel
    a, b, c, o = 0.05, 0.01, 0.08, 0.7
    sp, rng, ids = _tile([[7.3, 8.9]], [[a, b, c]], [o])
    con = contrib.contributions(sp, rng, ids, 16, 16, 16)
    for (y, x), (gid, w, _, _) in con.items():
        dx, dy = x + 0.5 - 7.3, y + 0.5 - 8.9
        al = min(0.99, o * math.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy)))
        if al >= A_T:
            assert list(gid) == [0] and abs(w[0] - al) < 1e-15
        else:
            assert len(gid) == 0


def test_two_flat_layers_in_order():
    # flat layers (q = 0): weights o1 and (1 - o1) o2, front first
    sp, rng, ids = _tile([[8, 8], [8, 8]], [[0, 0, 0], [0, 0, 0]], [0.4, 0.5])
    con = contrib.contributions(sp, rng, ids, 16, 16, 16)
    gid, w, _, T = con[(3, 4)]
    assert list(gid) == [0, 1]
    np.testing.assert_allclose(w, [0.4, 0.6 * 0.5], rtol=0, atol=1e-15)
    assert abs(T - 0.6 * 0.5) < 1e-15


def test_weights_telescope_to_one_minus_final_T():
    # sum_i T_i alpha_i = 1 - prod_i (1 - alpha_i) = 1 - T_final, and T_final
    # equals the blend oracle's
    scene = synthetic.ball_scene(3, 400, log_scale_mu=-2.5)
    cam = synthetic.look_at((0.0, 0.0, -3.0), width=64, height=48)
    p = project.project_view(scene, cam, tile=16)
    sp = blend.splats_from_projection(p)
    b = binning.bin_and_sort([dict(rect=p["rect"], n_tiles=p["n_tiles"], depth_f32=p["depth"]
                                   .astype(np.float32), grid_w=p["grid_w"],
                                   grid_h=p["grid_h"])], scene.n)
    con = contrib.contributions(sp, b["ranges"], b["ids"], 64, 48, 16)
    ref = blend.render_tiles(sp, b["ranges"], b["ids"], 64, 48, 16)
    n_multi = 0
    for (y, x), (gid, w, _, T) in con.items():
        assert abs(T - ref["final_T"][y, x]) < 1e-12
        assert abs(w.sum() - (1.0 - T)) < 1e-12
        # blended entries sit at list positions up to the last one (n_contrib)
        assert len(gid) <= ref["n_contrib"][y, x] and (len(gid) == 0) == (ref["n_contrib"][y, x] == 0)
        n_multi += len(gid) > 3
    assert n_multi > 100


def test_topk_ranking_brute_force():
    rng = np.random.default_rng(5)
    for _ in range(50):
        n = int(rng.integers(1, 40))
        ids = rng.permutation(200)[:n].astype(np.int64)
        w = rng.choice([0.1, 0.2, 0.25, 0.3], size=n)  # many exact ties
        for k in (1, 3, 32):
            got = contrib.topk(ids, w, k)
            want = sorted(range(n), key=lambda i: (-w[i], ids[i]))[:k]
            assert list(got) == [int(ids[i]) for i in want]


def test_marks_sums_and_stability_sets():
    # a scene with deep per-pixel lists: with k larger than every list all
    # blended records are marked; stable <= mark <= possible
    scene = synthetic.ball_scene(4, 600, log_scale_mu=-2.0)
    cam = synthetic.look_at((0.0, 0.0, -3.0), width=48, height=48)
    p = project.project_view(scene, cam, tile=16)
    sp = blend.splats_from_projection(p)
    b = binning.bin_and_sort([dict(rect=p["rect"], n_tiles=p["n_tiles"], depth_f32=p["depth"]
                                   .astype(np.float32), grid_w=p["grid_w"],
                                   grid_h=p["grid_h"])], scene.n)
    con = contrib.contributions(sp, b["ranges"], b["ids"], 48, 48, 16)
    blended = np.zeros(scene.n, dtype=bool)
    for gid, _, _, _ in con.values():
        blended[gid] = True
    mark_all, sums, _, _ = contrib.marks_and_sums(con, 10_000, scene.n)
    assert (mark_all == blended).all() and (sums[~blended] == 0).all()
    mark, sums2, stable, possible = contrib.marks_and_sums(con, 2, scene.n, 1e-6, 1e-5)
    assert (stable <= mark).all() and (mark <= possible).all()
    assert 0 < mark.sum() < blended.sum()
    np.testing.assert_allclose(sums, sums2)
    # the sum of all weights is the frame's total coverage
    total = sum(1.0 - T for _, _, _, T in con.values())
    assert abs(sums.sum() - total) < 1e-9
