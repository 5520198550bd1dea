"""Frames in flight on several HIP streams: every entry point launches on the
stream it is given (the current torch stream), so frames whose stages run on
different streams, ordered only by events and each on its own buffers, equal
the same views rendered one by one on one stream."""
import pytest
import torch

import synthetic
import gpu_util as gu
from paper_2503_05168_amd import (GaussianTensors, Renderer, Settings, seele_bin_sort_ex,
                                  seele_preprocess_staged, seele_rasterize_fwd_super,
                                  pixel_count, total_super_tiles, total_tiles)
from paper_2503_05168_amd.pipeline import SPLAT_FLOATS, bin_sort_workspace_size

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["plain", "contrib"])
def test_frames_in_flight_on_two_streams_equal_single_renders(mode):
    st = Settings(mode=mode)
    scene = synthetic.cluster_scene(2, 120_000)
    cams = synthetic.orbit_cameras(6, 4.0, 640, 480)
    g = GaussianTensors.from_arrays(scene)
    n = g.n
    gu.log(f"[case] two streams, {mode}, {len(cams)} frames")
    ref = []
    for cam in cams:
        f = Renderer(st, capacity=1 << 22, lists="super").render(g, [cam])
        ref.append(f.image.clone())
    torch.cuda.synchronize()
    cap = 1 << 22
    TT, NS, npix = total_tiles(cams[:1], 16), total_super_tiles(cams[:1], 16), pixel_count(cams[:1])
    bufs = [dict(splats=torch.empty((n, SPLAT_FLOATS), dtype=torch.float32, device="cuda"),
                 n_tiles=torch.empty(n, dtype=torch.int32, device="cuda"),
                 ws=torch.empty(bin_sort_workspace_size(n, cap, TT), dtype=torch.uint8,
                                device="cuda"),
                 ids=torch.empty(cap, dtype=torch.int32, device="cuda"),
                 keys=torch.empty(cap, dtype=torch.int32, device="cuda"),
                 ranges=torch.empty((NS, 2), dtype=torch.int32, device="cuda"),
                 npairs=torch.empty(2, dtype=torch.int64, device="cuda"))
            for _ in range(2)]
    out = [torch.empty(3 * npix, dtype=torch.float32, device="cuda") for _ in cams]
    T = torch.empty(npix, dtype=torch.float32, device="cuda")
    nc = torch.empty(npix, dtype=torch.int32, device="cuda")
    front, back = torch.cuda.Stream(), torch.cuda.Stream()
    binned = [torch.cuda.Event() for _ in range(2)]
    rastered = [torch.cuda.Event() for _ in range(2)]
    for i, cam in enumerate(cams):
        b = bufs[i & 1]
        with torch.cuda.stream(front):
            if i >= 2:
                front.wait_event(rastered[i & 1])
            seele_preprocess_staged(g, [cam], st, cap, b["ws"], None, b["splats"], b["n_tiles"])
            seele_bin_sort_ex(b["splats"], b["n_tiles"], n, [cam], 16, cap, b["ws"], b["ids"],
                              b["ranges"], b["npairs"], b["keys"], super_lists=True, staged=True)
            binned[i & 1].record(front)
        with torch.cuda.stream(back):
            back.wait_event(binned[i & 1])
            seele_rasterize_fwd_super(b["splats"], b["keys"], b["ids"], b["ranges"], [cam], st,
                                      out[i], T, nc)
            rastered[i & 1].record(back)
    torch.cuda.synchronize()
    for i in range(len(cams)):
        assert torch.equal(out[i], ref[i]), i
    gu.log("[done] two streams")
