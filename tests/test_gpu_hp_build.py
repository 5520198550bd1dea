"""Offline construction of the view-dependent representation on the GPU
(Sec. 3.3 "Offline Clustering") against the oracle: the per-cluster fold and
the segment layout bit-exactly on exactly summable inputs, the gather of the
reordered scene, and the whole builder on a small scene, its shared set
between the oracle's stable and possible top-k unions, its exclusive
assignment within the float32 uncertainty of the oracle's contributions, and
its all-cluster render equal to the reordered full scene's on the sampled
poses."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import contrib as ocon
from oracle import hp as ohp
from paper_2503_05168_amd import GaussianTensors, Renderer, Settings
from paper_2503_05168_amd import seele_hp_segments, seele_hp_select
from paper_2503_05168_amd.hp_build import (build_view_dependent, seele_gather_gaussians,
                                           seele_hp_accumulate, seele_hp_partition)

pytestmark = pytest.mark.gpu

import gpu_util as gu  # noqa: E402


@pytest.mark.parametrize("n,K,V", [(1, 1, 1), (100_003, 4, 3), (4096, 9, 1)])
def test_accumulate_and_partition_match_oracle(n, K, V):
    gu.log(f"[case] hp accumulate n={n} K={K} V={V}")
    rng = np.random.default_rng(n + K)
    marks = [(rng.random((V, n)) < 0.02).astype(np.uint8) for _ in range(K)]
    # multiples of 1/16 below 1/2: every float32 partial sum is exact
    sums = [np.where(rng.random((V, n)) < 0.5, rng.integers(0, 8, (V, n)) / 16.0, 0.0)
            .astype(np.float32) for _ in range(K)]
    dev = "cuda"
    shared = torch.zeros(n, dtype=torch.uint8, device=dev)
    best = torch.zeros(n, dtype=torch.float32, device=dev)
    bc = torch.full((n,), -1, dtype=torch.int32, device=dev)
    for c in range(K):
        seele_hp_accumulate(torch.from_numpy(marks[c]).to(dev).ravel(),
                            torch.from_numpy(sums[c]).to(dev).ravel(), V, n, c, shared, best, bc)
    torch.cuda.synchronize()
    S = np.stack([s.astype(np.float64).sum(0) for s in sums])
    np.testing.assert_array_equal(best.cpu().numpy(), S.max(0))
    perm, begin, count = seele_hp_partition(shared.cpu().numpy(), best.cpu().numpy(),
                                            bc.cpu().numpy(), K)
    op, ob, oc = ohp.partition([m.any(0) for m in marks], list(S), n)
    assert perm.tolist() == op.tolist()
    assert begin.tolist() == ob.tolist() and count.tolist() == oc.tolist()


def test_gather_gaussians():
    gu.log("[case] hp gather")
    scene = synthetic.ball_scene(7, 5000)
    g = GaussianTensors.from_arrays(scene)
    rng = np.random.default_rng(7)
    for perm in (rng.permutation(5000), rng.integers(0, 5000, 777), np.array([4999])):
        p = torch.from_numpy(perm.astype(np.int64)).cuda()
        out = seele_gather_gaussians(g, p)
        torch.cuda.synchronize()
        for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
            assert torch.equal(getattr(out, name), getattr(g, name)[..., p]), name
        assert out.sh_degree == g.sh_degree


def _oracle_cluster_state(scene, poses, labels, K, k, st):
    """Per cluster: the oracle's summed contributions per Gaussian, the stable
    and possible top-k unions over all poses, and a bound on how far the
    float32 sums may lie from the oracle's (pixels with a near-threshold
    decision can blend or skip an entry of weight at most about 1/255 and
    rescale the weights behind it by about as much)."""
    n = scene.n
    S = np.zeros((K, n))
    B = np.zeros((K, n))
    stable = np.zeros(n, dtype=bool)
    possible = np.zeros(n, dtype=bool)
    for cam, c in zip(poses, labels):
        f = gu.run(scene, [cam], st)
        sp = gu.splats_np(f)
        ids = f.sorted_ids.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
        ranges = f.tile_ranges.cpu().numpy().astype(np.int64)
        con = ocon.contributions(sp, ranges, ids, cam.width, cam.height, st.tile)
        _, s_v, st_v, po_v = ocon.marks_and_sums(con, k, n, tie_rel=1e-5,
                                                 margin_min=gu.ALPHA_MARGIN)
        S[c] += s_v
        stable |= st_v
        possible |= po_v
        gw = -(-cam.width // st.tile)
        shaky = np.zeros(len(ranges), dtype=np.int64)
        for (y, x), (_, _, marg, _) in con.items():
            if marg < gu.ALPHA_MARGIN:
                shaky[(y // st.tile) * gw + x // st.tile] += 1
        for t in np.nonzero(shaky)[0]:
            s, e = ranges[t]
            B[c, ids[s:e]] += 0.01 * shaky[t]
    B += 2e-4 * S + 1e-6
    return S, B, stable, possible


def test_build_view_dependent_end_to_end():
    gu.log("[case] hp build end-to-end")
    scene = synthetic.cluster_scene(5, 12_000, n_clusters=24)
    poses = synthetic.orbit_cameras(9, 4.0, 96, 72)
    K, k = 3, 8
    st = Settings(tile=16)
    g = GaussianTensors.from_arrays(scene)
    vd = build_view_dependent(g, poses, K, k=k, settings=st, views_per_call=2)
    torch.cuda.synchronize()
    n = scene.n
    # clustering: the oracle's k-means over the same features
    f = np.stack([ohp.camera_feature(c, vd.pos_scale, vd.beta) for c in poses])
    oc, ol = ohp.kmeans(f, K)
    assert vd.labels.tolist() == ol.tolist()
    np.testing.assert_allclose(vd.centroids, oc, rtol=0, atol=1e-6)
    # layout: a permutation, contiguous segments, the gathered scene
    perm = vd.perm.cpu().numpy()
    assert sorted(perm.tolist()) == list(range(n))
    assert vd.seg_begin[0] == 0 and (vd.seg_begin[1:] == vd.seg_begin[:-1] + vd.seg_count[:-1]).all()
    for name in ("means", "opacity_logits", "sh"):
        assert torch.equal(getattr(vd.gaussians, name), getattr(g, name)[..., vd.perm])
    seg = np.full(n, K + 1)
    for s in range(K + 1):
        seg[perm[vd.seg_begin[s]:vd.seg_begin[s] + vd.seg_count[s]]] = s
    shared = vd.shared.cpu().numpy().astype(bool)
    bc = vd.best_cluster.cpu().numpy()
    bs = vd.best_sum.cpu().numpy().astype(np.float64)
    assert ((seg == 0) == shared).all()
    assert (seg[~shared] == np.where(bc >= 0, bc + 1, K + 1)[~shared]).all()
    # against the oracle's contributions
    S, B, stable, possible = _oracle_cluster_state(scene, poses, vd.labels, K, k, st)
    assert stable.sum() > 0
    missing = np.nonzero(stable & ~shared)[0]
    extra = np.nonzero(shared & ~possible)[0]
    assert len(missing) == 0 and len(extra) == 0, (missing[:10], extra[:10])
    excl = np.nonzero(~shared & (bc >= 0))[0]
    unused = np.nonzero(~shared & (bc < 0))[0]
    assert len(excl) > 100 and len(unused) > 0, (len(excl), len(unused))
    for i in unused:
        assert (S[:, i] <= B[:, i]).all(), i
    for i in excl:
        c = bc[i]
        assert S[c, i] + B[c, i] >= (S[:, i] - B[:, i]).max(), i
        assert abs(bs[i] - S[c, i]) <= B[c, i], (i, bs[i], S[c, i])
    # rendering every segment reproduces the scene on the sampled poses
    r_full, r_vd = Renderer(st), Renderer(st)
    ties = 0
    for cam in poses:
        sel = seele_hp_select(vd.centroids, cam, vd.pos_scale, vd.beta, K - 1)
        segs = seele_hp_segments(vd.seg_begin, vd.seg_count, sel)
        fa = r_full.render(g, [cam])
        a = fa.image.clone()
        b = r_vd.render(vd.gaussians, [cam], segs).image.clone()
        b_all = r_vd.render(vd.gaussians, [cam]).image.clone()
        torch.cuda.synchronize()
        # dropping the unused Gaussians changes nothing
        assert torch.equal(b, b_all)
        # reordering changes only the order of records with equal depth keys
        # (ties go to the lower record id): any pixel that differs from the
        # original scene's lies in a tile whose list holds such a tie
        d = (a - b_all).abs().view(3, cam.height, cam.width).amax(0)
        depth = fa.splats[:, 12].cpu().numpy()
        gw = -(-cam.width // st.tile)
        for t in {(int(y) // st.tile) * gw + int(x) // st.tile
                  for y, x in zip(*np.nonzero(d.cpu().numpy() > 0))}:
            s_, e_ = fa.tile_ranges[t].tolist()
            lst = fa.sorted_ids[s_:e_].cpu().numpy().astype(np.int64) & 0xFFFFFFFF
            assert len(np.unique(depth[lst])) < len(lst), t
            ties += 1
        sel0 = seele_hp_select(vd.centroids, cam, vd.pos_scale, vd.beta, 0)
        b0 = r_vd.render(vd.gaussians, [cam], seele_hp_segments(vd.seg_begin, vd.seg_count, sel0))
        mse = ((a - b0.image) ** 2).mean().item()
        gu.log(f"  pose M=0 PSNR {10 * np.log10(1 / max(mse, 1e-20)):.1f} dB")
    gu.log(f"[done] hp build stats={vd.stats} tiles with depth ties that moved pixels={ties}")
