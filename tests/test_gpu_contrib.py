"""The offline contribution pass on the GPU (seele_contrib_topk) against the
float64 oracle over the GPU's own splats and tile lists: every record that a
stable pixel ranks among its top k is marked, nothing outside what some pixel
could rank there is, and the per-record sums of T alpha agree."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import contrib as ocon
from paper_2503_05168_amd import Settings, seele_contrib_topk

pytestmark = pytest.mark.gpu

import gpu_util as gu  # noqa: E402

CASES = [
    ("c1-k32", lambda: (synthetic.config(1)["scene"], synthetic.config(1)["cams"]), 16, 32),
    ("c1-k4-tile8", lambda: (synthetic.config(1)["scene"], synthetic.config(1)["cams"]), 8, 4),
    ("c2shape-2views-k8", lambda: (synthetic.cluster_scene(2, 30_000),
                                   [synthetic.look_at((0, 0, -4), width=320, height=180),
                                    synthetic.look_at((3, 1, -2), width=200, height=136)]),
     16, 8),
]


@pytest.mark.parametrize("name,build,tile,k", CASES, ids=[c[0] for c in CASES])
def test_contrib_topk_matches_oracle(name, build, tile, k):
    gu.log(f"[case] contrib {name}")
    scene, cams = build()
    st = Settings(tile=tile)
    f = gu.run(scene, cams, st)
    n = scene.n
    mark, sums = seele_contrib_topk(f.splats, f.sorted_ids, f.tile_ranges, cams, st, n, k)
    # a second call accumulates: marks stay, sums double
    mark2, sums2 = seele_contrib_topk(f.splats, f.sorted_ids, f.tile_ranges, cams, st, n, k,
                                      mark.clone(), sums.clone())
    torch.cuda.synchronize()
    assert torch.equal(mark2, mark)
    torch.testing.assert_close(sums2, 2 * sums, rtol=1e-6, atol=1e-7)
    got = mark.cpu().numpy().astype(bool)
    gsum = sums.cpu().numpy().astype(np.float64)
    sp = gu.splats_np(f)
    ids = f.sorted_ids.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    ranges = f.tile_ranges.cpu().numpy().astype(np.int64)
    R = len(cams) * n
    stable = np.zeros(R, dtype=bool)
    possible = np.zeros(R, dtype=bool)
    osum = np.zeros(R)
    shaky = np.zeros(R, dtype=bool)  # records blended by a pixel with a near-threshold decision
    base = 0
    for cam in cams:
        con = ocon.contributions(sp, ranges, ids, cam.width, cam.height, tile, tile_base=base)
        _, s_v, st_v, po_v = ocon.marks_and_sums(con, k, R, tie_rel=1e-5,
                                                 margin_min=gu.ALPHA_MARGIN)
        stable |= st_v
        possible |= po_v
        osum += s_v
        for gid, _, marg, _ in con.values():
            if marg < gu.ALPHA_MARGIN:
                shaky[gid] = True
        base += -(-cam.width // tile) * -(-cam.height // tile)
    assert stable.sum() > 0
    missing = np.nonzero(stable & ~got)[0]
    extra = np.nonzero(got & ~possible)[0]
    assert len(missing) == 0, missing[:10]
    assert len(extra) == 0, extra[:10]
    ok = ~shaky
    np.testing.assert_allclose(gsum[ok], osum[ok], rtol=2e-4, atol=1e-5)
    gu.log(f"[done] contrib {name} marked={int(got.sum())} stable={int(stable.sum())} "
           f"possible={int(possible.sum())}")


def test_contrib_topk_rejects_cr_and_bad_k():
    scene = synthetic.config(1)["scene"]
    cams = synthetic.config(1)["cams"]
    f = gu.run(scene, cams, Settings())
    with pytest.raises(Exception, match="plain"):
        seele_contrib_topk(f.splats, f.sorted_ids, f.tile_ranges, cams, Settings(mode="contrib"),
                           scene.n)
    with pytest.raises(Exception, match="k must be"):
        seele_contrib_topk(f.splats, f.sorted_ids, f.tile_ranges, cams, Settings(), scene.n, 33)
