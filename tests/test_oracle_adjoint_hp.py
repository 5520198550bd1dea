"""Pins for the oracle's adjoint (central finite differences in float64 on
tiny scenes whose decisions cannot flip under the step) and for the
hybrid-preprocessing active-set selection (brute force, constructed cases)."""
import copy

import numpy as np
import pytest

import synthetic
from oracle import adjoint, blend, hp, project

FIELDS = [("means", "means"), ("log_scales", "log_scales"), ("quats", "quats"),
          ("opacity_logits", "logits"), ("sh", "sh")]


def _f64(scene):
    s = copy.deepcopy(scene)
    for k, _ in FIELDS:
        setattr(s, k, getattr(scene, k).astype(np.float64))
    return s


def _loss(scene, cams, Gs, tile, extent, mode):
    tot, margins = 0.0, []
    for cam, G in zip(cams, Gs):
        p = project.project_view(scene, cam, tile=tile, extent=extent)
        r = blend.render_view(p, mode=mode)
        tot += float((r["image"] * G).sum())
        margins.append((r["margin"].min(), p["rect_margin"][p["visible"]].min()))
    return tot, margins


@pytest.mark.parametrize("mode,extent,seed", [("plain", "3sigma", 7), ("cr", "opacity", 8),
                                              ("plain", "opacity", 9)])
def test_adjoint_matches_central_differences(mode, extent, seed):
    cams = [synthetic.look_at((0.3, 0.2, -3.0), width=32, height=32),
            synthetic.look_at((-0.8, 0.1, -2.8), width=32, height=24)]
    rng = np.random.default_rng(seed)
    Gs = [rng.normal(size=(3, c.height, c.width)) for c in cams]
    # take the first scene (deterministic seed sequence) whose every blending decision is at
    # least 1e-3 (relative) and every rect edge 1e-2 px from its boundary, so that a step of
    # 1e-6 cannot flip any decision
    for s in range(seed * 100, seed * 100 + 100):
        scene = _f64(synthetic.ball_scene(s, 12, log_scale_mu=-1.6, log_scale_sigma=0.2,
                                          radius=0.5))
        _, margins = _loss(scene, cams, Gs, 8, extent, mode)
        if min(m[0] for m in margins) > 1e-3 and min(m[1] for m in margins) > 1e-2:
            break
    else:
        pytest.fail("no scene with safe decision margins")
    res = adjoint.render_and_grad(scene, cams, Gs, tile=8, extent=extent, mode=mode)
    h = 1e-6
    for attr, key in FIELDS:
        arr = getattr(scene, attr)
        g = res[key]
        for flat in range(0, arr.size, max(1, arr.size // 25)):
            ix = np.unravel_index(flat, arr.shape)
            sp, sm = copy.deepcopy(scene), copy.deepcopy(scene)
            getattr(sp, attr)[ix] += h
            getattr(sm, attr)[ix] -= h
            fd = (_loss(sp, cams, Gs, 8, extent, mode)[0] - _loss(sm, cams, Gs, 8, extent,
                                                                  mode)[0]) / (2 * h)
            if attr == "sh":
                an = g[ix[2], ix[0], ix[1]]
            elif attr == "opacity_logits":
                an = g[ix[0]]
            else:
                an = g[ix[1], ix[0]]
            assert an == pytest.approx(fd, abs=2e-6, rel=1e-5), (attr, ix)


def test_blend_adjoint_2d_matches_central_differences():
    scene = synthetic.ball_scene(21, 10, log_scale_mu=-1.7, log_scale_sigma=0.2, radius=0.5)
    cam = synthetic.look_at((0.1, 0.0, -3.0), width=24, height=24)
    p = project.project_view(scene, cam, tile=8)
    r = blend.render_view(p, mode="cr", collect_lists=True, bg=(0.2, 0.1, 0.4))
    b = r["binning"]
    G = np.random.default_rng(1).normal(size=(3, 24, 24))
    sp = blend.splats_from_projection(p)
    g2 = adjoint.blend_adjoint(sp, b["ids"], b["ranges"], r["lists"], G, 24, 24, 8,
                               bg=(0.2, 0.1, 0.4))

    def L(s):
        o = blend.render_tiles(s, b["ranges"], b["ids"], 24, 24, 8, mode="cr",
                               bg=(0.2, 0.1, 0.4))
        return float((o["image"] * G).sum())

    h = 1e-7
    for key in ("mean2d", "conic", "opacity", "rgb"):
        for g in np.nonzero(p["visible"])[0][:6]:
            for k in range(sp[key][g].size if np.ndim(sp[key][g]) else 1):
                s1 = {kk: np.array(v, copy=True) for kk, v in sp.items()}
                s2 = {kk: np.array(v, copy=True) for kk, v in sp.items()}
                if np.ndim(sp[key][g]):
                    s1[key][g, k] += h
                    s2[key][g, k] -= h
                    an = g2[key][g, k]
                else:
                    s1[key][g] += h
                    s2[key][g] -= h
                    an = g2[key][g]
                fd = (L(s1) - L(s2)) / (2 * h)
                assert an == pytest.approx(fd, abs=1e-5, rel=1e-5), (key, g, k)


def test_hp_nearest_cluster_brute_force():
    rng = np.random.default_rng(3)
    cents = rng.normal(size=(24, 6))
    for _ in range(50):
        f = rng.normal(size=6)
        sel = hp.select_clusters(cents, f, 3)
        d = [float(np.linalg.norm(cents[k] - f)) for k in range(24)]
        assert sel[0] == int(np.argmin(d))
        dn = [float(np.linalg.norm(cents[k] - cents[sel[0]])) for k in range(24)]
        rest = sorted([k for k in range(24) if k != sel[0]], key=lambda k: dn[k])[:3]
        assert sel[1:] == rest and len(set(sel)) == 4


def test_hp_orbit_views_pick_adjacent_cluster():
    cfg = synthetic.config(3, n=2000)
    lay = cfg["hp"]
    for k, cam in enumerate(cfg["cams"]):
        f = hp.camera_feature(cam, lay.pos_scale, lay.beta)
        sel = hp.select_clusters(lay.centroids, f, 0)
        # centroids sit between views 4c and 4c+1; views 4c+2 -> c, 4c+3 -> c+1 (mod 8)
        want = {0: k // 4, 1: k // 4, 2: k // 4, 3: (k // 4 + 1) % 8}[k % 4]
        assert sel == [want]
        segs = hp.active_segments(lay.seg_begin, lay.seg_count, sel)
        m = hp.active_mask(cfg["scene"].n, segs)
        assert m.sum() == lay.seg_count[0] + lay.seg_count[1 + want]
        assert (lay.labels[m] == -1).sum() == lay.seg_count[0]


def test_hp_camera_at_centroid():
    cam = synthetic.look_at((4.0, 0.0, 0.0))
    f = hp.camera_feature(cam, 4.0)
    np.testing.assert_allclose(f, [1, 0, 0, -1, 0, 0], atol=1e-7)
    cents = np.array([[1, 0, 0, -1, 0, 0], [0, 0, 1, 0, 0, -1], [-1, 0, 0, 1, 0, 0.0]])
    assert hp.select_clusters(cents, f, 1) == [0, 1]
