"""seele_bin_sort_noalloc (binning on the library's per-device scratch array)
against seele_bin_sort_ex with a caller workspace: identical lists, ranges and
pair counts for both list forms, over two calls in a row on one GPU, the
second with a smaller input (the scratch array keeps the first call's
contents)."""
import numpy as np
import pytest
import torch

import synthetic
from paper_2503_05168_amd import (GaussianTensors, Settings, seele_bin_sort_ex,
                                  seele_bin_sort_noalloc, seele_preprocess, total_super_tiles,
                                  total_tiles)
from paper_2503_05168_amd import _abi as A
from paper_2503_05168_amd.pipeline import bin_sort_workspace_size

import gpu_util as gu

pytestmark = pytest.mark.gpu

CALLS = [  # larger input first, then a smaller one on the same scratch array
    ("c2shape-2views-640x480-tile16", lambda: (synthetic.cluster_scene(2, 50_003),
                                               synthetic.orbit_cameras(2, 4.0, 640, 480)), 16),
    ("c1-256x256-tile8", lambda: (synthetic.ball_scene(1, 10_000),
                                  [synthetic.look_at((0.0, 0.0, -3.0), width=256, height=256)]), 8),
]


def _buffers(cap, nr, sup):
    return (torch.full((cap,), -7, dtype=torch.int32, device="cuda"),
            torch.full((cap,), -7, dtype=torch.int32, device="cuda"),
            torch.full((nr, 2), -7, dtype=torch.int32, device="cuda"),
            torch.full((2 if sup else 1,), -7, dtype=torch.int64, device="cuda"))


def _with_workspace(sp, nt, n, cams, tile, cap, sup):
    TT = total_tiles(cams, tile)
    nr = total_super_tiles(cams, tile) if sup else TT
    ws = torch.empty(bin_sort_workspace_size(len(cams) * n, cap, TT), dtype=torch.uint8,
                     device="cuda")
    keys, ids, rng, npairs = _buffers(cap, nr, sup)
    seele_bin_sort_ex(sp, nt, n, cams, tile, cap, ws, ids, rng, npairs, keys, super_lists=sup)
    return keys, ids, rng, npairs


def _noalloc(sp, nt, n, cams, tile, cap, sup):
    TT = total_tiles(cams, tile)
    nr = total_super_tiles(cams, tile) if sup else TT
    keys, ids, rng, npairs = _buffers(cap, nr, sup)
    seele_bin_sort_noalloc(sp, nt, n, cams, tile, cap, ids, rng, npairs, keys, super_lists=sup)
    return keys, ids, rng, npairs


@pytest.mark.parametrize("sup", [False, True], ids=["tile-lists", "super-lists"])
def test_noalloc_bin_sort_matches_workspace_entry_point(sup):
    for name, build, tile in CALLS:
        gu.log(f"[case] noalloc {name} super={sup}")
        scene, cams = build()
        g = GaussianTensors.from_arrays(scene)
        n = g.n
        sp, nt = seele_preprocess(g, cams, Settings(tile=tile))
        # the frame's pair count from the workspace entry point, then both at that capacity
        probe = _with_workspace(sp, nt, n, cams, tile, 1, sup)
        torch.cuda.synchronize()
        cap = int(probe[3][-1].item())  # the stored list length: entries or pairs
        assert cap > 0
        need = bin_sort_workspace_size(len(cams) * n, cap, total_tiles(cams, tile))
        assert need <= A.SEELE_NOALLOC_SCRATCH_BYTES, (name, need)
        ref = _with_workspace(sp, nt, n, cams, tile, cap, sup)
        got = _noalloc(sp, nt, n, cams, tile, cap, sup)
        torch.cuda.synchronize()
        assert torch.equal(got[3], ref[3]) and int(ref[3][-1].item()) == cap
        assert torch.equal(got[2], ref[2])
        ne = int(ref[2][:, 1].max().item()) if sup else cap
        assert ne > 0
        assert torch.equal(got[1][:ne], ref[1][:ne])
        if sup:
            assert torch.equal(got[0][:ne], ref[0][:ne])
        gu.log(f"[done] noalloc {name} super={sup} pairs={cap} listed={ne}")


def test_noalloc_bin_sort_overflow_and_oversize():
    """Overflow behaves as with a workspace (every range empty, the count
    reported); a frame whose workspace would exceed the scratch array is
    refused before anything runs."""
    gu.log("[case] noalloc overflow/oversize")
    scene = synthetic.ball_scene(1, 10_000)
    cams = [synthetic.look_at((0.0, 0.0, -3.0), width=256, height=256)]
    g = GaussianTensors.from_arrays(scene)
    sp, nt = seele_preprocess(g, cams, Settings())
    ref = _with_workspace(sp, nt, g.n, cams, 16, 100, True)
    got = _noalloc(sp, nt, g.n, cams, 16, 100, True)
    torch.cuda.synchronize()
    assert torch.equal(got[3], ref[3]) and int(ref[3][-1].item()) > 100
    assert torch.equal(got[2], ref[2]) and int(got[2].abs().sum().item()) == 0
    big = 4 << 20  # 4M records: far more workspace than the scratch array holds
    assert bin_sort_workspace_size(big, 1, total_tiles(cams, 16)) > A.SEELE_NOALLOC_SCRATCH_BYTES
    L = A.lib()
    st = L.seele_bin_sort_noalloc(0, None, None, big, A.camera_array(cams), 1, 16, None, None, 1,
                                  None, None, None)
    assert st == A.SEELE_ERR_CAPACITY
    assert b"scratch" in L.seele_last_error()
    gu.log("[done] noalloc overflow/oversize")
