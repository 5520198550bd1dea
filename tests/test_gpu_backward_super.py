"""The blend backward over super-tile lists (one workgroup per 2 x 2-tile
quadrant, Sec. 3.5) against the per-tile backward and the FP64 oracle's
adjoint: same gradients up to the order of the float sums; and the
forward's last-entry indices it reads, against the per-tile n_contrib."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import adjoint as oadj
from oracle import blend as oblend
from oracle import project as oproj
from paper_2503_05168_amd import GaussianTensors, Renderer, SeeleError, Settings
from paper_2503_05168_amd import seele_rasterize_bwd

import gpu_util as gu
from test_gpu_backward import _soa_grads, assert_grad_close

pytestmark = pytest.mark.gpu

CASES = [
    ("plain-c2shape-320x180",
     lambda: (synthetic.cluster_scene(2, 20_000),
              [synthetic.look_at((0.5, -0.3, -4.0), width=320, height=180)]), Settings()),
    ("cr-opacity-ragged",
     lambda: (synthetic.ball_scene(32, 3000, log_scale_mu=-3.0),
              [synthetic.look_at((0.0, 0.0, -3.0), width=100, height=72)]),
     Settings(mode="contrib", extent="opacity")),
    ("plain-mixed-views-bg",
     lambda: (synthetic.cluster_scene(5, 30_000), synthetic.sphere_cameras(50, 5)),
     Settings(bg=(0.1, 0.2, 0.3))),
    ("cr-2x4-mixed-views",
     lambda: (synthetic.cluster_scene(5, 30_000), synthetic.sphere_cameras(51, 4)),
     Settings(mode="contrib", group=(2, 4))),
    ("plain-70-views-chunks",
     lambda: (synthetic.ball_scene(41, 500, log_scale_mu=-2.8),
              synthetic.orbit_cameras(70, 3.0, 48, 40)), Settings()),
]


def _frames(scene, cams, st):
    g = GaussianTensors.from_arrays(scene)
    ft = Renderer(st, capacity=1 << 22, lists="tile").render(g, cams)
    fs = Renderer(st, capacity=1 << 22, lists="super", last_entry=True).render(g, cams)
    torch.cuda.synchronize()
    # the forward over super-tile lists writes the same bits, with or
    # without the last-entry output
    assert torch.equal(ft.image, fs.image) and torch.equal(ft.n_contrib, fs.n_contrib)
    check_last_entry(ft, fs, cams, st.tile)
    return g, ft, fs


def check_last_entry(ft, fs, cams, tile, sample=None):
    """Every pixel's last_entry names, in its super-tile list, the entry that
    holds the record at position n_contrib of its tile's own list: the same
    record id, an entry covering the tile, and exactly n_contrib covering
    entries up to it (0 where n_contrib is 0).  The count is checked for
    every distinct (tile, entry), or for `sample` seeded pixels per view.
    Integer work: bit-exact."""
    le = fs.last_entry.cpu().numpy().astype(np.int64)
    nc = ft.n_contrib.cpu().numpy().astype(np.int64)
    tid = ft.sorted_ids.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    tr = ft.tile_ranges.cpu().numpy().astype(np.int64).reshape(-1, 2)
    eid = fs.sorted_ids.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    clip_all = (fs.entry_keys.cpu().numpy().astype(np.int64) & 0xFFFFFFFF) >> 24
    sr = fs.tile_ranges.cpu().numpy().astype(np.int64).reshape(-1, 2)
    assert ((le == 0) == (nc == 0)).all()
    rng = np.random.default_rng(11)

    def covers(c, lx, ly):
        return ((c & 3) <= lx) & (lx <= ((c >> 2) & 3)) & (((c >> 4) & 3) <= ly) \
            & (ly <= ((c >> 6) & 3))

    pix = tb = sb = 0
    for cam in cams:
        W, H = cam.width, cam.height
        gw, gh = -(-W // tile), -(-H // tile)
        sgw, sgh = -(-gw // 4), -(-gh // 4)
        yy, xx = np.mgrid[0:H, 0:W]
        tx, ty = (xx // tile).ravel(), (yy // tile).ravel()
        t = tb + ty * gw + tx
        s = sb + (ty // 4) * sgw + (tx // 4)
        lev, ncv = le[pix:pix + W * H], nc[pix:pix + W * H]
        on = np.flatnonzero(lev > 0)
        e = sr[s[on], 0] + lev[on] - 1
        assert (e < sr[s[on], 1]).all()
        assert (eid[e] == tid[tr[t[on], 0] + ncv[on] - 1]).all()
        assert covers(clip_all[e], tx[on] % 4, ty[on] % 4).all()
        if sample is None:
            picks = {}
            for k, ek in zip(on.tolist(), e.tolist()):
                picks.setdefault((t[k], ek), k)
            picks = list(picks.values())
        else:
            picks = rng.choice(on, size=min(sample, on.size), replace=False).tolist()
        for k in picks:
            c = clip_all[sr[s[k], 0]:sr[s[k], 0] + lev[k]]
            assert int(covers(c, tx[k] % 4, ty[k] % 4).sum()) == ncv[k], (cam.width, k)
        pix += W * H
        tb += gw * gh
        sb += sgw * sgh


@pytest.mark.parametrize("name,build,st", CASES, ids=[c[0] for c in CASES])
def test_super_backward_equals_tile_backward(name, build, st):
    gu.log(f"[case] bwd-super {name}")
    scene, cams = build()
    g, ft, fs = _frames(scene, cams, st)
    dL = torch.randn(ft.image.numel(), device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    gt, g2t = seele_rasterize_bwd(g, cams, st, ft.splats, ft.n_tiles, ft.sorted_ids,
                                  ft.tile_ranges, ft.final_T, ft.n_contrib, dL)
    gs, g2s = seele_rasterize_bwd(g, cams, st, fs.splats, fs.n_tiles, fs.sorted_ids,
                                  fs.tile_ranges, fs.final_T, fs.n_contrib, dL,
                                  entry_keys=fs.entry_keys, last_entry=fs.last_entry)
    torch.cuda.synchronize()
    a = g2t.cpu().numpy().astype(np.float64)
    b = g2s.cpu().numpy().astype(np.float64)
    vis = (ft.n_tiles > 0).cpu().numpy()
    assert np.abs(b[~vis]).max(initial=0) == 0.0
    # the same float32 terms summed in another order (per quadrant in LDS,
    # wave arrival order unspecified): the backward's bar against the oracle
    for lo, hi, what in ((0, 2, "dmean2d"), (2, 5, "dconic"), (5, 6, "dopacity"), (6, 9, "drgb")):
        assert_grad_close(b[:, lo:hi], a[:, lo:hi], what)
    # the chain to the raw parameters: the oracle's preprocess adjoint of this
    # path's own 2D gradients (comparing the two paths' chained gradients
    # directly would amplify float sum-order noise where views cancel)
    n = scene.n
    sp = gu.splats_np(fs)
    tot, agree = None, np.ones(n, dtype=bool)
    for v, cam in enumerate(cams):
        proj = oproj.project_view(scene, cam, tile=st.tile, extent=st.extent)
        agree &= proj["visible"] == (sp["n_tiles"][v * n:(v + 1) * n] > 0)
        sl = slice(v * n, (v + 1) * n)
        d = oadj.preprocess_adjoint(scene, cam, proj, dict(mean2d=b[sl, 0:2], conic=b[sl, 2:5],
                                                           opacity=b[sl, 5], rgb=b[sl, 6:9]))
        tot = d if tot is None else {k: tot[k] + d[k] for k in tot}
    got = _soa_grads(gs, n)
    for k in ("means", "log_scales", "quats", "logits", "sh"):
        assert_grad_close(got[k][agree], tot[k][agree], k)
    gu.log(f"[done] bwd-super {name} visible={int(vis.sum())} disagree={int((~agree).sum())}")


def test_super_backward_against_oracle_adjoint():
    """Stage-wise against the oracle's blend adjoint over the tile lists that
    the super-tile lists expand to."""
    scene = synthetic.cluster_scene(2, 20_000)
    cams = [synthetic.look_at((0.5, -0.3, -4.0), width=320, height=180),
            synthetic.look_at((-0.4, 0.2, -3.8), width=144, height=112)]
    st = Settings(mode="contrib")
    g, ft, fs = _frames(scene, cams, st)
    sp = gu.splats_np(ft)
    ids = ft.sorted_ids.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    ranges = ft.tile_ranges.cpu().numpy().astype(np.int64)
    rng = np.random.default_rng(9)
    n = scene.n
    ref = dict(mean2d=np.zeros((len(cams) * n, 2)), conic=np.zeros((len(cams) * n, 3)),
               opacity=np.zeros(len(cams) * n), rgb=np.zeros((len(cams) * n, 3)))
    Gs, base = [], 0
    for cam in cams:
        r = oblend.render_tiles(sp, ranges, ids, cam.width, cam.height, st.tile, base, "cr",
                                st.group, st.bg, st.alpha_min, st.alpha_max, st.T_min,
                                collect_lists=True)
        G = rng.normal(size=(3, cam.height, cam.width))
        G[:, r["margin"] < gu.ALPHA_MARGIN] = 0.0
        Gs.append(G)
        a = oadj.blend_adjoint(sp, ids, ranges, r["lists"], G, cam.width, cam.height, st.tile,
                               base, st.bg, st.alpha_max)
        for k in ref:
            ref[k] += a[k]
        base += (-(-cam.width // st.tile)) * (-(-cam.height // st.tile))
    dL = torch.cat([torch.as_tensor(G, dtype=torch.float32).reshape(-1) for G in Gs]).cuda()
    _, g2 = seele_rasterize_bwd(g, cams, st, fs.splats, fs.n_tiles, fs.sorted_ids,
                                fs.tile_ranges, fs.final_T, fs.n_contrib, dL,
                                entry_keys=fs.entry_keys, last_entry=fs.last_entry)
    torch.cuda.synchronize()
    g2 = g2.cpu().numpy().astype(np.float64)
    assert_grad_close(g2[:, 0:2], ref["mean2d"], "dmean2d")
    assert_grad_close(g2[:, 2:5], ref["conic"], "dconic")
    assert_grad_close(g2[:, 5], ref["opacity"], "dopacity")
    assert_grad_close(g2[:, 6:9], ref["rgb"], "drgb")


def test_super_backward_empty_and_tile8():
    scene = synthetic.ball_scene(1, 500)
    far = [synthetic.look_at((0.0, 0.0, 30.0), target=(0.0, 0.0, 60.0), width=64, height=48)]
    st = Settings()
    g, ft, fs = _frames(scene, far, st)
    dL = torch.ones(fs.image.numel(), device="cuda")
    gs, g2 = seele_rasterize_bwd(g, far, st, fs.splats, fs.n_tiles, fs.sorted_ids, fs.tile_ranges,
                                 fs.final_T, fs.n_contrib, dL, entry_keys=fs.entry_keys,
                                 last_entry=fs.last_entry)
    torch.cuda.synchronize()
    assert float(g2.abs().max().item()) == 0.0 and float(gs.means.abs().max().item()) == 0.0
    st8 = Settings(tile=8)
    f8 = Renderer(st8, capacity=1 << 20, lists="super", last_entry=True).render(g, far)
    with pytest.raises(SeeleError):
        seele_rasterize_bwd(g, far, st8, f8.splats, f8.n_tiles, f8.sorted_ids, f8.tile_ranges,
                            f8.final_T, f8.n_contrib, dL, entry_keys=f8.entry_keys,
                            last_entry=f8.last_entry)
    with pytest.raises(ValueError):  # the super-tile backward reads last_entry
        seele_rasterize_bwd(g, far, st, fs.splats, fs.n_tiles, fs.sorted_ids, fs.tile_ranges,
                            fs.final_T, fs.n_contrib, dL, entry_keys=fs.entry_keys)


def test_last_entry_at_full_size():
    """The 8 x 720p fine-tuning frame (1.0M Gaussians): last_entry against the
    per-tile n_contrib on every pixel (record and coverage), the
    covering-entry count on 64 seeded pixels per view."""
    gu.log("[case] last_entry 8 x 1280x720, 1.0M Gaussians")
    scene = synthetic.cluster_scene(4, 1_000_000)
    cams = synthetic.orbit_cameras(8, 4.0, 1280, 720)
    g = GaussianTensors.from_arrays(scene)
    st = Settings()
    ft = Renderer(st, capacity=1 << 25, lists="tile").render(g, cams)
    fs = Renderer(st, capacity=1 << 25, lists="super", last_entry=True).render(g, cams)
    torch.cuda.synchronize()
    assert torch.equal(ft.image, fs.image) and torch.equal(ft.n_contrib, fs.n_contrib)
    check_last_entry(ft, fs, cams, st.tile, sample=64)
