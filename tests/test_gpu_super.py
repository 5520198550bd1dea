"""Super-tile lists on the GPU: seele_bin_sort_super's entries, expanded by
their clipped rectangles, are exactly seele_bin_sort's per-tile lists, and
seele_rasterize_fwd_super writes the same bits (image, final T, n_contrib and
work counters) as seele_rasterize_fwd over those lists -- on small ragged and
multi-view cases, both tile sizes and both rasterizer forms, and on the full
3.0M-Gaussian 1080p frame, where sampled tiles are also checked against the
float64 oracle."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import blend as oblend
from paper_2503_05168_amd import (GaussianTensors, Renderer, Settings, seele_bin_sort_super,
                                  seele_spatial_order,
                                  seele_preprocess, seele_rasterize_fwd_counted,
                                  seele_rasterize_fwd_super, total_super_tiles, total_tiles)

pytestmark = pytest.mark.gpu

import gpu_util as gu  # noqa: E402


def expand_super(keys, ids, st_ranges, cams, tile):
    """Per-tile lists (ids, [TT][2] ranges) from super-tile entries: tile t's
    list is its super-tile's entries whose clip covers t, in entry order."""
    n_ent = int(st_ranges[:, 1].max(initial=0))
    keys = keys[:n_ent].astype(np.int64) & 0xFFFFFFFF
    ids = ids[:n_ent].astype(np.int64) & 0xFFFFFFFF
    st = keys & 0xFFFFFF
    clip = keys >> 24
    x0, x1, y0, y1 = clip & 3, (clip >> 2) & 3, (clip >> 4) & 3, (clip >> 6) & 3
    # per super-tile: view tile base, grid width, origin tile
    s_tb, s_gw, s_ox, s_oy = [], [], [], []
    tb = 0
    for c in cams:
        gw, gh = -(-c.width // tile), -(-c.height // tile)
        sgw, sgh = -(-gw // 4), -(-gh // 4)
        loc = np.arange(sgw * sgh)
        s_tb.append(np.full(loc.size, tb))
        s_gw.append(np.full(loc.size, gw))
        s_ox.append((loc % sgw) * 4)
        s_oy.append((loc // sgw) * 4)
        tb += gw * gh
    s_tb, s_gw, s_ox, s_oy = (np.concatenate(a) for a in (s_tb, s_gw, s_ox, s_oy))
    assert st.max(initial=0) < s_tb.size
    gt, pos = [], []
    for ly in range(4):
        for lx in range(4):
            p = np.nonzero((x0 <= lx) & (lx <= x1) & (y0 <= ly) & (ly <= y1))[0]
            s = st[p]
            gt.append(s_tb[s] + (s_oy[s] + ly) * s_gw[s] + s_ox[s] + lx)
            pos.append(p)
    gt, pos = np.concatenate(gt), np.concatenate(pos)
    order = np.lexsort((pos, gt))
    out_ids = ids[pos[order]]
    cnt = np.bincount(gt, minlength=tb)
    assert cnt.size == tb
    end = np.cumsum(cnt)
    start = end - cnt
    ranges = np.where((cnt > 0)[:, None], np.stack([start, end], 1), 0)
    return out_ids, ranges


def super_frame(scene, cams, st, capacity=1 << 22, segments=None):
    g = GaussianTensors.from_arrays(scene)
    splats, n_tiles = seele_preprocess(g, cams, st, segments)
    keys, ids, rng, npairs, ws = seele_bin_sort_super(splats, n_tiles, g.n, cams, st.tile,
                                                      capacity)
    need = int(npairs[1].item())  # entries
    if need > capacity:  # the frame reported its need: sort again with room for it
        keys, ids, rng, npairs, _ = seele_bin_sort_super(splats, n_tiles, g.n, cams, st.tile,
                                                         need)
    img, T, nc = seele_rasterize_fwd_super(splats, keys, ids, rng, cams, st)
    torch.cuda.synchronize()
    return g, splats, n_tiles, keys, ids, rng, npairs, img, T, nc


def check_against_tile_path(scene, cams, st, counters=True, segments=None):
    g, splats, n_tiles, keys, ids, rng, npairs, img, T, nc = super_frame(scene, cams, st,
                                                                         segments=segments)
    f = gu.run(scene, cams, st, capacity=1 << 22, segments=segments)
    P = int(f.num_pairs.item())
    assert int(npairs[0].item()) == P
    assert int(npairs[1].item()) == int(rng[:, 1].max().item()) <= P
    assert rng.shape == (total_super_tiles(cams, st.tile), 2)
    # the super-tile lists expand to the per-tile lists exactly
    e_ids, e_ranges = expand_super(keys.cpu().numpy(), ids.cpu().numpy(), rng.cpu().numpy(),
                                   cams, st.tile)
    assert e_ranges.shape == (total_tiles(cams, st.tile), 2)
    np.testing.assert_array_equal(e_ids, f.sorted_ids.cpu().numpy()[:P].astype(np.int64) &
                                  0xFFFFFFFF)
    np.testing.assert_array_equal(e_ranges, f.tile_ranges.cpu().numpy().astype(np.int64))
    # and rasterize to the same bits
    assert torch.equal(img, f.image) and torch.equal(T, f.final_T)
    assert torch.equal(nc, f.n_contrib)
    if counters:
        c_s = torch.zeros(6, dtype=torch.int64, device="cuda")
        img2, T2, nc2 = seele_rasterize_fwd_super(splats, keys, ids, rng, cams, st, counters=c_s)
        _, _, _, c_t = seele_rasterize_fwd_counted(f.splats, f.sorted_ids, f.tile_ranges, cams, st)
        torch.cuda.synchronize()
        assert torch.equal(img2, f.image) and torch.equal(nc2, f.n_contrib)
        assert c_s.cpu().tolist() == c_t.cpu().tolist()
    return f, P


CASES = [
    ("c1-plain", lambda: (synthetic.config(1)["scene"], synthetic.config(1)["cams"]),
     Settings()),
    ("c1-cr-2x4-tile8", lambda: (synthetic.config(1)["scene"], synthetic.config(1)["cams"]),
     Settings(mode="contrib", group=(2, 4), tile=8, bg=(0.2, 0.5, 0.1))),
    ("c2shape-ragged-2views-opacity", lambda: (synthetic.cluster_scene(2, 40_000),
                                               [synthetic.look_at((0, 0, -4), width=500, height=333),
                                                synthetic.look_at((4, 0, 0), width=331,
                                                                  height=197)]),
     Settings(extent="opacity")),
    ("c5shape-mixed-12views-cr", lambda: (synthetic.cluster_scene(5, 60_000),
                                          synthetic.sphere_cameras(50, 12, resolutions=(
                                              (160, 120), (320, 180), (480, 270)))),
     Settings(mode="contrib")),
    ("c2shape-tile8-plain-1080p", lambda: (synthetic.cluster_scene(2, 200_000),
                                           synthetic.orbit_cameras(2, 4.0, 1920, 1080)),
     Settings(tile=8)),
    ("c1-cr-4x4", lambda: (synthetic.config(1)["scene"], synthetic.config(1)["cams"]),
     Settings(mode="contrib", group=(4, 4))),
    ("c2shape-cr-2x4-tile16-2views", lambda: (synthetic.cluster_scene(2, 60_000),
                                              synthetic.orbit_cameras(2, 4.0, 640, 360)),
     Settings(mode="contrib", group=(2, 4))),
    # a grid wider than 256 tiles: the rectangles are gathered by id
    ("c2shape-wide-strip-tile8", lambda: (synthetic.cluster_scene(2, 40_000),
                                          [synthetic.look_at((0.5, 0.2, -3.5), width=2112,
                                                             height=96)]),
     Settings(tile=8)),
]


@pytest.mark.parametrize("name,build,settings", CASES, ids=[c[0] for c in CASES])
def test_super_lists_equal_tile_lists_and_render_the_same_bits(name, build, settings):
    gu.log(f"[case] super {name}")
    scene, cams = build()
    _, P = check_against_tile_path(scene, cams, settings)
    gu.log(f"[done] super {name} pairs={P}")


def test_super_overflow_and_empty_scene():
    scene = synthetic.config(1)["scene"]
    cams = synthetic.config(1)["cams"]
    st = Settings()
    g = GaussianTensors.from_arrays(scene)
    splats, n_tiles = seele_preprocess(g, cams, st)
    keys, ids, rng, npairs, _ = seele_bin_sort_super(splats, n_tiles, g.n, cams, st.tile, 64)
    img, T, nc = seele_rasterize_fwd_super(splats, keys, ids, rng, cams, st)
    torch.cuda.synchronize()
    pairs, entries = int(npairs[0].item()), int(npairs[1].item())
    assert pairs >= entries > 64
    assert int(rng.abs().sum().item()) == 0  # every super-tile list left empty
    assert torch.all(nc == 0) and torch.all(T == 1.0)
    # the capacity bounds the entries: exactly the entry count fits although
    # the pairs exceed it, and the lists equal those sorted with room to spare
    assert pairs > entries
    big = seele_bin_sort_super(splats, n_tiles, g.n, cams, st.tile, pairs)
    exact = seele_bin_sort_super(splats, n_tiles, g.n, cams, st.tile, entries)
    torch.cuda.synchronize()
    assert torch.equal(big[3], exact[3])
    assert torch.equal(big[2], exact[2]) and int(exact[2][:, 1].max().item()) == entries
    assert torch.equal(big[0][:entries], exact[0][:entries])
    assert torch.equal(big[1][:entries], exact[1][:entries])
    short = seele_bin_sort_super(splats, n_tiles, g.n, cams, st.tile, entries - 1)
    torch.cuda.synchronize()
    assert torch.equal(short[3], big[3]) and int(short[2].abs().sum().item()) == 0
    # nothing visible: all lists empty, background everywhere
    far = [synthetic.look_at((0.0, 0.0, 30.0), target=(0.0, 0.0, 60.0), width=96, height=64)]
    st2 = Settings(bg=(0.25, 0.5, 0.75))
    _, _, _, keys, ids, rng, npairs, img, T, nc = super_frame(scene, far, st2)
    assert int(npairs.abs().sum().item()) == 0 and int(rng.abs().sum().item()) == 0
    assert torch.all(T == 1.0) and torch.all(nc == 0)
    im = img.reshape(3, -1)
    for ch, b in enumerate(st2.bg):
        assert torch.all(im[ch] == b)


def test_super_default_batch_only():
    scene = synthetic.config(1)["scene"]
    cams = synthetic.config(1)["cams"]
    g, splats, n_tiles, keys, ids, rng, *_ = super_frame(scene, cams, Settings())
    with pytest.raises(Exception, match="default LDS batch"):
        seele_rasterize_fwd_super(splats, keys, ids, rng, cams, Settings(lds_batch=128))
    with pytest.raises(ValueError):
        Renderer(Settings(), lists="super", schedule="queue")


FULL_FRAMES = [("morton", "plain"), ("generated", "plain"), ("morton", "contrib"),
               ("c3-segments", "hp_contrib")]


@pytest.mark.parametrize("order,form", FULL_FRAMES, ids=[f"{a}-{b}" for a, b in FULL_FRAMES])
def test_full_frame_3m_1080p_super_matches_tile_path_and_oracle_samples(order, form):
    """The benchmark's frames (3.0M Gaussians, 1920x1080, 16x16 tiles) in the
    launch configuration it times: the plain form in the storage order it
    uses (Morton order of the means) and in the generator's order, the
    contribution-aware form (2x2 groups), and hybrid preprocessing (the c3
    layout's nearest cluster, opacity-aware extent) with contribution-aware
    rasterization.  Each is bit-identical to the per-tile path, the
    instrumented kernel (which visits every listed record) writes the same
    bits as the culled ones, and sampled tiles match the float64 oracle over
    the GPU's own splats."""
    segs = None
    if order == "c3-segments":
        from oracle import hp as ohp
        cfg = synthetic.config(3)
        lay, scene, cams = cfg["hp"], cfg["scene"], cfg["cams"][:1]
        sel = ohp.select_clusters(lay.centroids, ohp.camera_feature(cams[0], lay.pos_scale),
                                  cfg["M"])
        segs = ohp.active_segments(lay.seg_begin, lay.seg_count, sel)
    else:
        cfg = synthetic.config(2, n_views=1)
        scene, cams = cfg["scene"], cfg["cams"]
    if order == "morton":
        perm, _ = seele_spatial_order(GaussianTensors.from_arrays(scene))
        scene = scene.subset(perm.cpu().numpy())
    st = {"plain": Settings(), "contrib": Settings(mode="contrib"),
          "hp_contrib": Settings(mode="contrib", extent="opacity")}[form]
    gu.log(f"[case] super full frame 3.0M 1080p, {order} order, {form}")
    f, P = check_against_tile_path(scene, cams, st, counters=True, segments=segs)
    gu.log(f"[step] full frame lists, bits and counters equal, pairs={P}")
    # the staged path the benchmark times gives the same lists and bits
    _, _, _, keys, eids, rng, _, img, T, nc = super_frame(scene, cams, st, segments=segs)
    fs = Renderer(st, capacity=1 << 22, lists="super").render(GaussianTensors.from_arrays(scene),
                                                               cams, segs)
    torch.cuda.synchronize()
    E = int(rng[:, 1].max().item())
    assert torch.equal(fs.entry_keys[:E], keys[:E]) and torch.equal(fs.sorted_ids[:E], eids[:E])
    assert torch.equal(fs.tile_ranges, rng)
    assert torch.equal(fs.image, img) and torch.equal(fs.final_T, T)
    assert torch.equal(fs.n_contrib, nc)
    del fs
    gu.log("[step] staged full frame equal")
    sp = gu.splats_np(f)
    ids = f.sorted_ids.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    ranges = f.tile_ranges.cpu().numpy().astype(np.int64)
    cam = cams[0]
    gw = -(-cam.width // 16)
    ntl = gw * (-(-cam.height // 16))
    # the heaviest tiles and a random sample
    lens = ranges[:, 1] - ranges[:, 0]
    tiles = sorted(set(np.argsort(-lens)[:3].tolist() +
                       np.random.default_rng(7).integers(0, ntl, 5).tolist()))
    # the oracle's own order for the sampled tiles' lists
    rect, nt, depth = sp["rect"], sp["n_tiles"], sp["depth_f32"].astype(np.float64)
    for t in tiles:
        tx, ty = t % gw, t // gw
        cov = np.nonzero((nt > 0) & (rect[:, 0] <= tx) & (tx < rect[:, 2]) & (rect[:, 1] <= ty) &
                         (ty < rect[:, 3]))[0]
        want = cov[np.lexsort((cov, depth[cov]))]
        np.testing.assert_array_equal(ids[ranges[t, 0]:ranges[t, 1]], want)
    mode = "plain" if st.mode == "plain" else "cr"
    r = oblend.render_tiles(sp, ranges, ids, cam.width, cam.height, 16, 0, mode, st.group,
                            st.bg, st.alpha_min, st.alpha_max, st.T_min, tiles=tiles)
    imgs, Ts, ncs = gu.outputs_np(f)
    for t in tiles:
        ty, tx = divmod(t, gw)
        sl = (slice(ty * 16, (ty + 1) * 16), slice(tx * 16, (tx + 1) * 16))
        safe = r["margin"][sl] >= gu.ALPHA_MARGIN
        err = np.abs(imgs[0][(slice(None),) + sl] - r["image"][(slice(None),) + sl]).max(0)
        assert err[safe].max(initial=0) <= 1e-5, t
        np.testing.assert_array_equal(ncs[0][sl][safe], r["n_contrib"][sl][safe])
        assert safe.mean() > 0.9, t
    gu.log(f"[done] super full frame, oracle tiles {tiles}")


STAGED_CASES = [
    ("c2shape-1080p-super", lambda: (synthetic.cluster_scene(2, 200_000),
                                     synthetic.orbit_cameras(1, 4.0, 1920, 1080)), Settings(), True),
    ("c5shape-mixed-12views-n-not-256-super", lambda: (synthetic.cluster_scene(5, 60_001),
                                                       synthetic.sphere_cameras(50, 12)),
     Settings(mode="contrib"), True),
    ("c2shape-3views-tile8-tilelists", lambda: (synthetic.cluster_scene(2, 50_003),
                                                synthetic.orbit_cameras(3, 4.0, 640, 480)),
     Settings(tile=8), False),
    # very small near planes: depth keys over many binades (the shell at
    # radius 20 against z_near 2e-4, a ratio above 2^16) and records just
    # past the near plane whose footprints cover the view
    ("c2shape-znear-2e-4-wide-depth-ratio-super",
     lambda: (synthetic.cluster_scene(2, 100_001), synthetic.orbit_cameras(2, 4.0, 960, 540)),
     Settings(z_near=2e-4), True),
    ("c2shape-znear-1e-6-super",
     lambda: (synthetic.cluster_scene(3, 60_000), synthetic.orbit_cameras(1, 4.0, 960, 540)),
     Settings(z_near=1e-6), True),
    ("c2shape-znear-2e-4-tilelists",
     lambda: (synthetic.cluster_scene(2, 40_000), synthetic.orbit_cameras(1, 4.0, 640, 480)),
     Settings(z_near=2e-4), False),
]


@pytest.mark.parametrize("name,build,settings,sup", STAGED_CASES, ids=[c[0] for c in STAGED_CASES])
def test_staged_preprocessing_bins_identically(name, build, settings, sup):
    """seele_preprocess_staged + seele_bin_sort_ex(STAGED) write the same
    splats, counts, lists and ranges as seele_preprocess + the unstaged sort,
    for both list forms, several views and n not a multiple of 256."""
    from paper_2503_05168_amd import seele_bin_sort_ex, seele_preprocess_staged
    from paper_2503_05168_amd.pipeline import bin_sort_workspace_size
    gu.log(f"[case] staged {name}")
    scene, cams = build()
    st = settings
    g = GaussianTensors.from_arrays(scene)
    n, V = g.n, len(cams)
    TT = total_tiles(cams, st.tile)
    NR = total_super_tiles(cams, st.tile) if sup else TT
    sp0, nt0 = seele_preprocess(g, cams, st)
    out = {}
    for staged in (False, True):
        cap = 1 << 22
        for _ in range(2):  # second round with the capacity the frame reported
            ws = torch.zeros(bin_sort_workspace_size(V * n, cap, TT), dtype=torch.uint8,
                             device="cuda")
            keys = torch.empty(cap, dtype=torch.int32, device="cuda")
            ids = torch.empty(cap, dtype=torch.int32, device="cuda")
            rng = torch.empty((NR, 2), dtype=torch.int32, device="cuda")
            npairs = torch.empty(2 if sup else 1, dtype=torch.int64, device="cuda")
            if staged:
                sp, nt = seele_preprocess_staged(g, cams, st, cap, ws)
            else:
                sp, nt = sp0, nt0
            seele_bin_sort_ex(sp, nt, n, cams, st.tile, cap, ws, ids, rng, npairs, keys,
                              super_lists=sup, staged=staged)
            torch.cuda.synchronize()
            need = int(npairs[-1].item())  # the stored list length
            if need <= cap:
                break
            cap = need
        out[staged] = (sp, nt, keys, ids, rng, need)
    a, b = out[False], out[True]
    assert a[5] == b[5] and a[5] > 0
    assert torch.equal(a[1], b[1])
    vis = (a[1] > 0).repeat_interleave(16).view(-1, 16)
    assert torch.equal(a[0][vis], b[0][vis])  # records of visible Gaussians
    ne = int(a[4][:, 1].max().item()) if sup else a[5]
    assert torch.equal(a[3][:ne], b[3][:ne]) and torch.equal(a[4], b[4])
    if sup:
        assert torch.equal(a[2][:ne], b[2][:ne])
    gu.log(f"[done] staged {name} pairs={a[5]}")


def test_staged_preprocessing_with_inactive_segments():
    """Hybrid-preprocessing segments leave most records inactive: the staged
    path still bins exactly like the unstaged one."""
    from paper_2503_05168_amd import seele_bin_sort_ex, seele_preprocess_staged
    from paper_2503_05168_amd.pipeline import bin_sort_workspace_size
    scene = synthetic.cluster_scene(3, 70_000)
    cams = synthetic.orbit_cameras(2, 4.0, 800, 600)
    st = Settings()
    g = GaussianTensors.from_arrays(scene)
    segs = [(1000, 20_000), (33_333, 5_000), (60_000, 7_777)]
    n, V = g.n, len(cams)
    TT, NS = total_tiles(cams, st.tile), total_super_tiles(cams, st.tile)
    cap = 1 << 22
    res = []
    for staged in (False, True):
        ws = torch.zeros(bin_sort_workspace_size(V * n, cap, TT), dtype=torch.uint8,
                         device="cuda")
        keys = torch.empty(cap, dtype=torch.int32, device="cuda")
        ids = torch.empty(cap, dtype=torch.int32, device="cuda")
        rng = torch.empty((NS, 2), dtype=torch.int32, device="cuda")
        npairs = torch.empty(2, dtype=torch.int64, device="cuda")
        if staged:
            sp, nt = seele_preprocess_staged(g, cams, st, cap, ws, segs)
        else:
            sp, nt = seele_preprocess(g, cams, st, segs)
        seele_bin_sort_ex(sp, nt, n, cams, st.tile, cap, ws, ids, rng, npairs, keys,
                          super_lists=True, staged=staged)
        torch.cuda.synchronize()
        res.append((nt, keys, ids, rng, int(npairs[0].item())))
    (nt0, k0, i0, r0, p0), (nt1, k1, i1, r1, p1) = res
    assert p0 == p1 and 0 < p0 <= cap and torch.equal(nt0, nt1) and torch.equal(r0, r1)
    ne = int(r0[:, 1].max().item())
    assert torch.equal(k0[:ne], k1[:ne]) and torch.equal(i0[:ne], i1[:ne])
