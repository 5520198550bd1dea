"""Scene prefetching on the GPU (Sec. 3.3 "Scene Prefetching"): segment
copies against torch indexing, and a prefetching renderer with fewer slots
than clusters along a camera path, whose frames equal the all-resident
hybrid-preprocessing frames (up to the order of depth ties, which follows
record positions) and whose pool holds exactly the host columns of the
clusters its slot table names."""
import math

import numpy as np
import pytest
import torch

import synthetic
from paper_2503_05168_amd import GaussianTensors, Renderer, Settings
from paper_2503_05168_amd import seele_hp_segments, seele_hp_select
from paper_2503_05168_amd.hp_build import build_view_dependent
from paper_2503_05168_amd.prefetch import PrefetchingRenderer, seele_load_segments

pytestmark = pytest.mark.gpu

import gpu_util as gu  # noqa: E402


def test_load_segments_matches_indexing():
    gu.log("[case] prefetch load_segments")
    rng = np.random.default_rng(1)
    host = torch.randn((59, 5003)).pin_memory()
    pool = torch.zeros((59, 2000), device="cuda")
    sb, db, ct = [0, 4000, 1234, 5002], [0, 100, 1500, 1999], [100, 1003, 0, 1]
    s = torch.cuda.Stream()
    seele_load_segments(host, pool, sb, db, ct, s)
    s.synchronize()
    want = torch.zeros((59, 2000))
    for a, b, c in zip(sb, db, ct):
        want[:, b:b + c] = host[:, a:a + c]
    assert torch.equal(pool.cpu(), want)


def _orbit_path(n, radius, w, h, wobble=0.3):
    cams = []
    for k in range(n):
        th = 2.0 * math.pi * k / n
        y = wobble * math.sin(3 * th)
        cams.append(synthetic.look_at((radius * math.sin(th), y, -radius * math.cos(th)),
                                      width=w, height=h))
    return cams


@pytest.mark.parametrize("lookahead,slots,preload",
                         [(1.0, 6, False), (None, 4, False), (2.0, 9, False), (None, 8, True)])
def test_prefetching_renderer_matches_all_resident(lookahead, slots, preload):
    gu.log(f"[case] prefetch renderer lookahead={lookahead} slots={slots} preload={preload}")
    scene = synthetic.cluster_scene(5, 12_000, n_clusters=24)
    g = GaussianTensors.from_arrays(scene)
    poses = synthetic.sampled_orbit_poses(8, 40, 96, 72)
    K, M = 8, 2
    vd = build_view_dependent(g, poses, K, k=8, settings=Settings(), views_per_call=8)
    st = Settings(extent="opacity")
    pr = PrefetchingRenderer(vd, st, M=M, n_slots=slots, lookahead=lookahead, lists="super",
                             preload=preload)
    ref = Renderer(st, lists="super")
    path = _orbit_path(36, 4.0, 96, 72)
    ties = 0
    for cam in path:
        f = pr.render(cam)
        sel = seele_hp_select(vd.centroids, cam, vd.pos_scale, vd.beta, M)
        fr = ref.render(vd.gaussians, [cam], seele_hp_segments(vd.seg_begin, vd.seg_count, sel))
        torch.cuda.synchronize()
        d = (f.image - fr.image).abs().view(3, cam.height, cam.width).amax(0)
        if d.max().item() > 0:
            # only where a tile's list holds two records of equal depth
            depth = fr.splats[:, 12].cpu().numpy()
            ids = fr.sorted_ids.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
            rng_ = fr.tile_ranges.cpu().numpy()
            gw = -(-cam.width // 16)
            sw = -(-gw // 4)
            for y, x in zip(*np.nonzero(d.cpu().numpy() > 0)):
                tx, ty = x // 16, y // 16
                s_, e_ = rng_[(ty // 4) * sw + tx // 4]
                lst = ids[s_:e_]
                assert len(np.unique(depth[lst])) < len(lst), (y, x)
            ties += 1
    torch.cuda.synchronize()
    # the pool holds the host columns of every resident cluster
    for s, c in enumerate(pr.slot_cluster):
        if c < 0:
            continue
        b, n = int(pr.begins[c]), int(pr.counts[c])
        o = pr.n_shared + s * pr.slot_cap
        assert torch.equal(pr.pool[:, o:o + n].cpu(), pr.host[:, b:b + n])
    assert torch.equal(pr.pool[:, :pr.n_shared].cpu(), pr.host[:, :pr.n_shared])
    gu.log(f"[done] prefetch stats={pr.stats} resident={pr.resident_bytes} "
           f"frames with tie differences={ties}")
    assert (pr.stats["loads"] == 0) == preload
    if lookahead is not None:
        assert pr.stats["demand_loads"] < pr.stats["loads"]
