#!/usr/bin/env python3
"""Benchmark: 1080p frames/s at 3.0M Gaussians, plain vs contribution-aware.

Workload (default): the outdoor-scene-shaped 3.0M-Gaussian scene (64
anisotropic clusters + 10% background shell, seed 2; stored in Morton order
of the means, a one-time layout choice at load), 32 orbit views at
radius 4, 1920x1080, 60 deg horizontal FOV, 16x16 tiles, alpha_theta = 1/255,
T_min = 1e-4.  One step = one frame: preprocess + bin/sort + rasterize of one
orbit view (views cycle), inputs resident in HBM, no host synchronisation
inside the timed region.  ``value`` is the plain form's frames/s; the other
forms are reported beside it:
  contrib     contribution-aware rasterization (2x2 groups), 3-sigma extent
  hp          hybrid preprocessing: nearest view cluster (8 clusters, each
              ~60% of the Gaussians incl. the shared set) + opacity-aware extent
  hp_contrib  both.
  hp_built    hybrid preprocessing over a representation built by the
              offline construction of Sec. 3.3 from 128 sampled poses around
              the orbit (24 pose clusters, top-32 contributors, nearest
              cluster + 3 neighbours) + opacity-aware extent; its PSNR against
              the plain full-scene image is reported beside its speed.
Per-stage times come from HIP events recorded on the launch stream.  The
roofline object covers the dominant kernel of the plain form; its work counts
come from the library's instrumented rasterizer (run once per view, untimed).
The CPU baseline times the float64 oracle on a bounded sample of one view.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz FP32 lane-ops (packed FP32 not used)
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
PEAK_HBM = 8.0e12
# algorithmic FP32 lane operations per alpha evaluation (the quadratic form,
# opacity and clamp: 12, plus the exp) and per blend (weight, transmittance,
# three colour FMAs, termination test: 9)
OPS_EVAL = 13
OPS_BLEND = 9
# backward: lane-ops per blended (pixel, Gaussian) and per visible record
OPS_BWD_BLEND = 40
OPS_BWD_RECORD = 300


def measured_traffic(kernel_key):
    """HBM bytes per launch of the rasterizer from the committed rocprofv3
    counter summary, if the kernel source is still the one that was
    profiled (otherwise None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel_key}.traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    h = hashlib.sha256()
    for f in ("paper_2503_05168_amd/csrc/raster_fwd.hip",
              "paper_2503_05168_amd/csrc/seele_internal.h"):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest()[:16] != d.get("source_sha256_16"):
        return None
    return d["hbm_read_bytes_per_launch"] + d["hbm_write_bytes_per_launch"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=32)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--n", type=int, default=3_000_000, help="Gaussian count (default 3.0M)")
    ap.add_argument("--forms",
                    default="plain,contrib,hp,hp_contrib,hp_built,plain_generator_order")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-tiles", type=int, default=120,
                    help="tiles of view 0 each CPU oracle worker blends (about 10-30 s)")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="(internal) run the CPU oracle baseline alone and print it as JSON")
    ap.add_argument("--no-bwd", action="store_true", help="skip the fwd+bwd measurement")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-view batched run")
    ap.add_argument("--no-pipelined", action="store_true",
                    help="skip the plain frames with two in flight")
    ap.add_argument("--no-prefetch", action="store_true",
                    help="skip the scene-prefetching measurement (needs the hp_built form)")
    ap.add_argument("--ft-steps", type=int, default=1000,
                    help="steps of the integrated fine-tuning run (0 skips it; needs hp_built)")
    ap.add_argument("--ft-gamma", type=float, default=0.1,
                    help="weight of the FLIP term in the integrated fine-tuning run")
    ap.add_argument("--ft-lr-scale", type=float, default=1.0,
                    help="scale of the 3DGS learning rates in the integrated fine-tuning run")
    ap.add_argument("--no-cluster-sweep", action="store_true",
                    help="skip the cluster-count x neighbour-count sweep")
    ap.add_argument("--no-groups", action="store_true",
                    help="skip the contribution-aware group-size sweep")
    ap.add_argument("--lists", choices=("super", "tile"), default="super",
                    help="list form of the timed frame: super-tile lists read by each tile "
                         "(default) or per-tile lists")
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="first copy 256 MiB device to device (a known-size kernel that "
                         "scales hardware byte counters)")
    return ap.parse_args()


def load_scene(scene):
    """The scene in its storage order on the device: Gaussians sorted by the
    Morton code of their means (a one-time layout choice at load, untimed;
    the host copy is permuted alike).  Returns (host scene, GaussianTensors)."""
    import paper_2503_05168_amd as P
    g0 = P.GaussianTensors.from_arrays(scene)
    perm, _ = P.seele_spatial_order(g0)
    g = P.seele_gather_gaussians(g0, perm)
    del g0
    return scene.subset(perm.cpu().numpy()), g


def build_forms(names, n):
    import numpy as np
    import synthetic
    from synthetic.configs import _orbit_centroids
    from paper_2503_05168_amd import GaussianTensors, Settings

    log(f"[bench] generating scene n={n}")
    t = time.time()
    scene = synthetic.cluster_scene(2, n)
    cams = synthetic.orbit_cameras(32, 4.0, 1920, 1080)
    log(f"[bench] scene ready in {time.time() - t:.1f}s")
    forms = {}
    if "plain_generator_order" in names:
        g0 = GaussianTensors.from_arrays(scene)
        forms["plain_generator_order"] = dict(g=g0, st=Settings(), hp=None)
    scene, g = load_scene(scene)
    if "plain_generator_order" in forms:  # differs from the stored order's image by tie swaps
        forms["plain_generator_order"]["full_g"] = g
    if "plain" in names:
        forms["plain"] = dict(g=g, st=Settings(), hp=None)
    if "contrib" in names:
        forms["contrib"] = dict(g=g, st=Settings(mode="contrib"), hp=None, full_g=g)
    if "hp" in names or "hp_contrib" in names:
        labels = synthetic.hp_membership(3, scene.n, n_clusters=8)
        cents = _orbit_centroids(8, 32, 4.0)
        scene_r, lay = synthetic.reorder_segments(scene, labels, 8, cents, pos_scale=4.0)
        g3 = GaussianTensors.from_arrays(scene_r)
        del scene_r
        if "hp" in names:
            forms["hp"] = dict(g=g3, st=Settings(extent="opacity"), hp=lay, full_g=g)
        if "hp_contrib" in names:
            forms["hp_contrib"] = dict(g=g3, st=Settings(extent="opacity", mode="contrib"),
                                       hp=lay, full_g=g)
    if "hp_built" in names:
        import torch
        from paper_2503_05168_amd import build_view_dependent
        poses = synthetic.sampled_orbit_poses(6, 128, 1920, 1080)
        t = time.time()
        vd = build_view_dependent(g, poses, 24, k=32, settings=Settings(), views_per_call=8)
        torch.cuda.synchronize()
        build_s = time.time() - t
        log(f"[bench] view-dependent representation built in {build_s:.1f}s: {vd.stats}")
        forms["hp_built"] = dict(g=vd.gaussians, st=Settings(extent="opacity"), hp=vd, M=3,
                                 full_g=g,
                                 extra=dict(build_s=build_s, sampled_poses=len(poses),
                                            clusters=24, M=3, k=32, shared=vd.stats["shared"],
                                            exclusive_total=sum(vd.stats["exclusive"]),
                                            unused=vd.stats["unused"]))
    return scene, cams, forms


def form_quality(full_g, form, cams):
    """Image error of a form against the plain full-scene image over the
    first four orbit views: PSNR and max abs per channel (the plain GPU image
    equals the float64 oracle's within 1e-5, checked by the tests)."""
    import paper_2503_05168_amd as P
    lay = form["hp"]
    ref = P.Renderer(P.Settings(), capacity=1 << 26, lists="super")
    r = P.Renderer(form["st"], capacity=1 << 26, lists="super")
    mse, mx = 0.0, 0.0
    views = cams[:4]
    for c in views:
        segs = None
        if lay is not None:
            cl = P.seele_hp_select(lay.centroids, c, lay.pos_scale, lay.beta, form.get("M", 0))
            segs = P.seele_hp_segments(lay.seg_begin, lay.seg_count, cl)
        d = r.render(form["g"], [c], segs).image - ref.render(full_g, [c]).image
        mse += float((d * d).mean().item()) / len(views)
        mx = max(mx, float(d.abs().max().item()))
    psnr = float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)
    return dict(psnr_vs_plain_full=psnr, max_abs_vs_plain_full=mx, quality_views=len(views))


def run_form(name, form, cams, steps, warmup, lists="super"):
    import torch
    import paper_2503_05168_amd as P

    g, st, lay = form["g"], form["st"], form["hp"]
    n = g.n
    V = len(cams)
    # active segments per view (hybrid preprocessing, host-side C calls)
    segs = [None] * V
    if lay is not None:
        for v, cam in enumerate(cams):
            cl = P.seele_hp_select(lay.centroids, cam, lay.pos_scale, lay.beta,
                                   form.get("M", 0))
            segs[v] = P.seele_hp_segments(lay.seg_begin, lay.seg_count, cl)
    dev = g.means.device
    one = [cams[0]]
    TT = P.total_tiles(one, st.tile)
    NS = P.total_super_tiles(one, st.tile)
    sup = lists == "super"
    npix = P.pixel_count(one)
    splats = torch.empty((n, P.pipeline.SPLAT_FLOATS), dtype=torch.float32, device=dev)
    n_tiles = torch.empty(n, dtype=torch.int32, device=dev)
    ranges = torch.empty((NS if sup else TT, 2), dtype=torch.int32, device=dev)
    image = torch.empty(3 * npix, dtype=torch.float32, device=dev)
    final_T = torch.empty(npix, dtype=torch.float32, device=dev)
    n_contrib = torch.empty(npix, dtype=torch.int32, device=dev)

    # size the pair buffer from the views themselves (one synchronising pass)
    need = []
    for v in range(V):
        P.seele_preprocess(g, [cams[v]], st, segs[v], splats, n_tiles)
        need.append(int(n_tiles.sum(dtype=torch.int64).item()))
    capacity = int(max(need) * 1.02) + 4096
    ws = torch.empty(P.pipeline.bin_sort_workspace_size(n, capacity, TT), dtype=torch.uint8,
                     device=dev)
    ids = torch.empty(capacity, dtype=torch.int32, device=dev)
    keys = torch.empty(capacity if sup else 1, dtype=torch.int32, device=dev)
    npairs_log = torch.zeros(steps, dtype=torch.int64, device=dev)
    npairs = torch.empty(2 if sup else 1, dtype=torch.int64, device=dev)

    def preprocess(v):
        if sup:  # the binning's first step is staged by preprocessing
            P.seele_preprocess_staged(g, [cams[v]], st, capacity, ws, segs[v], splats, n_tiles)
        else:
            P.seele_preprocess(g, [cams[v]], st, segs[v], splats, n_tiles)

    def binning(cam):
        if sup:
            P.seele_bin_sort_ex(splats, n_tiles, n, cam, st.tile, capacity, ws, ids, ranges,
                                npairs, keys, super_lists=True, staged=True)
        else:
            P.seele_bin_sort(splats, n_tiles, n, cam, st.tile, capacity, ws, ids, ranges, npairs)

    def raster(cam, counters=None):
        if sup:
            P.seele_rasterize_fwd_super(splats, keys, ids, ranges, cam, st, image, final_T,
                                        n_contrib, counters)
        elif counters is not None:
            counters.copy_(P.seele_rasterize_fwd_counted(splats, ids, ranges, cam, st)[3])
        else:
            P.seele_rasterize_fwd(splats, ids, ranges, cam, st, image, final_T, n_contrib)

    def step(v, ev=None):
        cam = [cams[v]]
        if ev is not None:
            ev[0].record()
        preprocess(v)
        if ev is not None:
            ev[1].record()
        binning(cam)
        if ev is not None:
            ev[2].record()
        raster(cam)
        if ev is not None:
            ev[3].record()

    for i in range(warmup):
        step(i % V)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        step(i % V, evs[i])
        # the stored list length (super-tile entries, or pairs)
        npairs_log[i:i + 1].copy_(npairs[-1:], non_blocking=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert int(npairs_log.max().item()) <= capacity, "pair buffer overflow in the timed region"
    stage = {"preprocess": 0.0, "bin_sort": 0.0, "raster": 0.0}
    for e in evs:
        stage["preprocess"] += e[0].elapsed_time(e[1])
        stage["bin_sort"] += e[1].elapsed_time(e[2])
        stage["raster"] += e[2].elapsed_time(e[3])
    stage = {k: v / steps for k, v in stage.items()}

    # work counters and visible counts for the views that were timed (untimed pass)
    vis, act, pairs, ents, cnt = [], [], [], [], []
    c = torch.zeros(6, dtype=torch.int64, device=dev)
    for i in range(min(steps, V)):
        v = i % V
        preprocess(v)
        vis.append(int((n_tiles > 0).sum().item()))
        act.append(n if segs[v] is None else sum(c_ for _, c_ in segs[v]))
        binning([cams[v]])
        pairs.append(int(npairs[0].item()))
        ents.append(int(ranges[:, 1].max().item()) if sup else 0)
        raster([cams[v]], c)
        cnt.append([int(x) for x in c.cpu().tolist()])
    torch.cuda.synchronize()
    k = len(cnt)
    mean = lambda xs: sum(xs) / len(xs)
    evals = mean([c[0] + c[2] for c in cnt])  # per-pixel evaluations + leader tests
    blends = mean([c[1] for c in cnt])
    need = mean([c[4] + c[2] for c in cnt])  # evaluations left to the culled kernel
    ms = 1000.0 * wall / steps
    out = dict(fps=1000.0 / ms, ms_per_frame=ms, stage_ms=stage, capacity=capacity,
               lists=lists, super_tiles=NS, tiles=TT, pairs=mean(pairs),
               entries=mean(ents) if sup else None,
               visible=mean(vis), active=mean(act),
               evals=evals, blends=blends, evals_needed=need,
               block_visits=mean([c[5] for c in cnt]),
               leader_tests=mean([c[2] for c in cnt]), leader_pass=mean([c[3] for c in cnt]),
               views_counted=k)
    log(f"[bench] {name}: {out['fps']:.1f} fps ({ms:.3f} ms/frame) stages="
        + ", ".join(f"{a}={b:.3f}" for a, b in stage.items())
        + f" pairs={out['pairs']:.3e} vis={out['visible']:.3e} evals={evals:.3e}")
    return out


def run_form_pipelined(name, form, cams, steps, warmup, stages=2):
    """The same frames with several in flight: with stages=2, frame i+1's
    preprocessing and binning (one stream) run while frame i is rasterised
    (a second stream); with stages=3, preprocessing, binning and
    rasterisation each have a stream, so three frames overlap.  Each frame in
    flight has its own set of buffers; events order the stages of a frame and
    the reuse of a set.  Every frame still does all of its work; only
    throughput is reported."""
    import torch
    import paper_2503_05168_amd as P

    g, st = form["g"], form["st"]
    assert form["hp"] is None, "pipelined frames take the full scene"
    n = g.n
    V = len(cams)
    dev = g.means.device
    one = [cams[0]]
    TT = P.total_tiles(one, st.tile)
    NS = P.total_super_tiles(one, st.tile)
    npix = P.pixel_count(one)
    splats0 = torch.empty((n, P.pipeline.SPLAT_FLOATS), dtype=torch.float32, device=dev)
    nt0 = torch.empty(n, dtype=torch.int32, device=dev)
    need = []
    for v in range(V):
        P.seele_preprocess(g, [cams[v]], st, None, splats0, nt0)
        need.append(int(nt0.sum(dtype=torch.int64).item()))
    del splats0, nt0
    capacity = int(max(need) * 1.02) + 4096
    K = stages
    bufs = []
    for _ in range(K):
        bufs.append(dict(
            splats=torch.empty((n, P.pipeline.SPLAT_FLOATS), dtype=torch.float32, device=dev),
            n_tiles=torch.empty(n, dtype=torch.int32, device=dev),
            ws=torch.empty(P.pipeline.bin_sort_workspace_size(n, capacity, TT),
                           dtype=torch.uint8, device=dev),
            ids=torch.empty(capacity, dtype=torch.int32, device=dev),
            keys=torch.empty(capacity, dtype=torch.int32, device=dev),
            ranges=torch.empty((NS, 2), dtype=torch.int32, device=dev),
            npairs=torch.empty(2, dtype=torch.int64, device=dev),
            image=torch.empty(3 * npix, dtype=torch.float32, device=dev),
            final_T=torch.empty(npix, dtype=torch.float32, device=dev),
            n_contrib=torch.empty(npix, dtype=torch.int32, device=dev)))
    npairs_log = torch.zeros(steps, dtype=torch.int64, device=dev)
    # default-priority streams: preprocessing, binning (the first one when
    # stages=2), rasterisation
    s_pre = torch.cuda.Stream()
    s_bin = torch.cuda.Stream() if K == 3 else s_pre
    s_ras = torch.cuda.Stream()
    prepped = [torch.cuda.Event() for _ in range(K)]
    binned = [torch.cuda.Event() for _ in range(K)]
    rastered = [torch.cuda.Event() for _ in range(K)]
    torch.cuda.synchronize()

    def frame(i, log_i=None):
        k = i % K
        b = bufs[k]
        cam = [cams[i % V]]
        with torch.cuda.stream(s_pre):
            if i >= K:
                s_pre.wait_event(rastered[k])  # frame i - K is done with b
            P.seele_preprocess_staged(g, cam, st, capacity, b["ws"], None, b["splats"],
                                      b["n_tiles"])
            prepped[k].record(s_pre)
        with torch.cuda.stream(s_bin):
            s_bin.wait_event(prepped[k])
            P.seele_bin_sort_ex(b["splats"], b["n_tiles"], n, cam, st.tile, capacity, b["ws"],
                                b["ids"], b["ranges"], b["npairs"], b["keys"],
                                super_lists=True, staged=True)
            if log_i is not None:
                npairs_log[log_i:log_i + 1].copy_(b["npairs"][-1:], non_blocking=True)
            binned[k].record(s_bin)
        with torch.cuda.stream(s_ras):
            s_ras.wait_event(binned[k])
            P.seele_rasterize_fwd_super(b["splats"], b["keys"], b["ids"], b["ranges"], cam, st,
                                        b["image"], b["final_T"], b["n_contrib"], None)
            rastered[k].record(s_ras)

    for i in range(warmup):
        frame(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        frame(warmup + i, i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert int(npairs_log.max().item()) <= capacity, "pair buffer overflow in the timed region"
    # the last frame equals the same view rendered alone on one stream
    last = bufs[(warmup + steps - 1) % K]
    ref = P.Renderer(st, capacity=capacity, lists="super").render(
        g, [cams[(warmup + steps - 1) % V]])
    torch.cuda.synchronize()
    same = bool(torch.equal(ref.image, last["image"]))
    ms = 1000.0 * wall / steps
    out = dict(fps=1000.0 / ms, ms_per_frame=ms, frames_in_flight=K, equal_to_sequential=same)
    log(f"[bench] {name} ({K} frames in flight): {out['fps']:.1f} fps ({ms:.3f} ms/frame), "
        f"last frame equal to a single render: {same}")
    del bufs, ref
    torch.cuda.empty_cache()
    return out


def run_prefetch(vd, frames=240, slots=8, M=3):
    """Scene prefetching (Sec. 3.3) over the built representation along a
    smooth 1080p camera path (an orbit of radius 4 with a vertical wobble of
    0.3, `frames` frames, none of them a sampled pose): ms/frame with every
    cluster resident (one preloaded slot per cluster, the same code path),
    with `slots` cluster slots and prediction one frame
    ahead, and with the same slots but demand loads only; resident bytes and
    copies.  Each is timed over the whole path after an untimed pass, in two
    modes: streaming (the host runs ahead of the GPU) and interactive (each
    frame waits for the previous one, so a copy the frame needs is not
    hidden behind earlier frames); three interleaved rounds, the best
    counts.  The pair capacity is sized on an all-resident
    pass over the path and checked on the device after every timed run."""
    import torch
    import synthetic
    import paper_2503_05168_amd as P
    from paper_2503_05168_amd.prefetch import ROWS, PrefetchingRenderer

    path = []
    for k in range(frames):
        th = 2.0 * math.pi * k / frames
        path.append(synthetic.look_at((4.0 * math.sin(th), 0.3 * math.sin(3 * th),
                                       -4.0 * math.cos(th)), width=1920, height=1080))
    st = P.Settings(extent="opacity")
    ref = P.Renderer(st, capacity=1 << 24, lists="super")
    for c in path:  # sizes the pair buffer
        ref.render(vd.gaussians, [c], P.seele_hp_segments(
            vd.seg_begin, vd.seg_count, P.seele_hp_select(vd.centroids, c, vd.pos_scale, vd.beta,
                                                          M)))
    cap = int(ref.capacity * 1.05) + 4096
    del ref

    def listed(f):  # stored list length: super-tile entries
        return f.num_entries if f.num_entries is not None else f.num_pairs

    def timed(fn, interactive):
        mx = torch.zeros(1, dtype=torch.int64, device="cuda")
        for i in range(len(path)):  # the same host work as the timed pass
            torch.maximum(mx, listed(fn(i)), out=mx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(len(path)):
            torch.maximum(mx, listed(fn(i)), out=mx)
            if interactive:
                torch.cuda.current_stream().synchronize()
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - t0) / len(path)
        assert int(mx.item()) <= cap, "list buffer overflow in the timed region"
        return ms

    K = len(vd.seg_begin) - 1
    cfgs = {"all_resident": dict(n_slots=K, lookahead=None, preload=True),
            "prefetch": dict(n_slots=slots, lookahead=1.0),
            "demand_only": dict(n_slots=slots, lookahead=None)}
    prs, host = {}, None
    for name, kw in cfgs.items():
        prs[name] = PrefetchingRenderer(vd, st, M=M, capacity=cap, lists="super", host=host,
                                        **kw)
        host = prs[name].host
    # three interleaved rounds of every configuration; the best round counts
    ms = {name: {"streaming": [], "interactive": []} for name in cfgs}
    for _ in range(3):
        for mode in ("streaming", "interactive"):
            for name, pr in prs.items():
                ms[name][mode].append(timed(lambda i: pr.render(path[i], check=False),
                                            mode == "interactive"))
    best = {name: {m: min(v) for m, v in d.items()} for name, d in ms.items()}
    out = dict(frames=frames, slots=slots, M=M, rounds=3,
               model_bytes=ROWS * 4 * int(vd.gaussians.n),
               all_clusters_bytes=ROWS * 4 * int(vd.seg_count.sum()))
    assert prs["all_resident"].stats["loads"] == 0
    for name, pr in prs.items():
        n = pr.stats["frames"]
        out[name] = dict(ms=best[name], resident_bytes=pr.resident_bytes,
                         loads_per_frame=pr.stats["loads"] / n,
                         demand_loads_per_frame=pr.stats["demand_loads"] / n,
                         mb_loaded_per_frame=pr.stats["bytes_loaded"] / n / 1e6)
        if name != "all_resident":
            out[name]["overhead"] = {m: best[name][m] / best["all_resident"][m] - 1.0
                                     for m in best[name]}
        log(f"[bench] {name}: {best[name]['streaming']:.3f} / {best[name]['interactive']:.3f} "
            f"ms/frame streaming / interactive, resident {pr.resident_bytes / 1e6:.0f} MB "
            f"(all clusters {out['all_clusters_bytes'] / 1e6:.0f} MB), "
            f"{out[name]['loads_per_frame']:.2f} loads/frame "
            f"({out[name]['demand_loads_per_frame']:.2f} demand)")
    del prs, host
    return out


def run_integrated_finetune(vd, full_g, start_g, steps=1000, window=7, M=3, frames=240,
                            lr_scale=1.0, gamma=0.1):
    """The integrated fine-tuning of Sec. 3.5 in the built representation's
    layout: a model to fine-tune (start_g: the scene with perturbed means
    and opacities, standing in for a converted model that lost quality) is
    trained towards the plain full-scene renders of the scene.  Each step
    renders `window` consecutive 1080p frames of a camera path (orbit radius
    4, vertical wobble 0.3) with Seele's pipeline (hybrid preprocessing over
    the union of the frames' selected clusters, opacity-aware extent,
    contribution-aware rasterization), takes L_3DGS + gamma FLIP, the
    backward and Adam.  Reports ms per step and the PSNR of Seele's render
    against the plain full-scene image on 8 orbit views (not on the path)
    before and after."""
    import torch
    import synthetic
    import paper_2503_05168_amd as P

    path = []
    for k in range(frames):
        th = 2.0 * math.pi * k / frames
        path.append(synthetic.look_at((4.0 * math.sin(th), 0.3 * math.sin(3 * th),
                                       -4.0 * math.cos(th)), width=1920, height=1080))
    held = synthetic.orbit_cameras(32, 4.0, 1920, 1080)
    plain = P.Renderer(P.Settings(), capacity=1 << 26, lists="super")
    npx = 3 * 1920 * 1080
    targets = torch.empty((frames, npx), dtype=torch.float32, device="cuda")
    for i, c in enumerate(path):
        targets[i].copy_(plain.render(full_g, [c]).image)
    held_ref = [plain.render(full_g, [c]).image.clone() for c in held[::4]]
    g = start_g
    st = P.Settings(mode="contrib", extent="opacity")

    def segs(cams):
        cl = sorted({c for cam in cams for c in P.seele_hp_select(vd.centroids, cam, vd.pos_scale,
                                                                  vd.beta, M)})
        return P.seele_hp_segments(vd.seg_begin, vd.seg_count, cl)

    def psnr_held():
        r = P.Renderer(st, capacity=1 << 26, lists="super")
        mse = 0.0
        for c, ref in zip(held[::4], held_ref):
            d = r.render(g, [c], segs([c])).image - ref
            mse += float((d * d).mean().item()) / len(held_ref)
        return 10.0 * math.log10(1.0 / mse)

    before = psnr_held()
    o = P.AdamOpts()
    opts = P.AdamOpts(*(lr_scale * getattr(o, k) for k in
                        ("lr_means", "lr_log_scales", "lr_quats", "lr_opacity", "lr_sh_dc",
                         "lr_sh_rest")))
    ft = P.FineTuner(g, st, gamma=gamma, opts=opts, extent=vd.pos_scale, capacity=1 << 26)
    starts = [(s_ * window) % (frames - window + 1) for s_ in range(steps)]
    loss0 = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, s0 in enumerate(starts):
        cams = path[s0:s0 + window]
        l = ft.step(cams, targets[s0:s0 + window].reshape(-1), segs(cams))
        if i == 0:
            loss0 = float(l.mean().item())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    loss1 = float(l.mean().item())
    after = psnr_held()
    out = dict(steps=steps, window=window, lr_scale=lr_scale, gamma=gamma,
               ms_per_step=1000.0 * wall / max(steps, 1),
               ms_per_view=1000.0 * wall / max(steps * window, 1), loss_first=loss0,
               loss_last=loss1, psnr_before=before, psnr_after=after)
    log(f"[bench] integrated fine-tuning: {steps} steps x {window} frames, "
        f"{out['ms_per_step']:.2f} ms/step; loss {loss0:.5f} -> {loss1:.5f}; PSNR vs the plain "
        f"full scene {before:.2f} -> {after:.2f} dB")
    del ft, targets
    return out


def run_group_sweep(g, cams, steps, warmup, groups=((1, 1), (2, 2), (2, 4), (4, 4))):
    """Contribution-aware form with pixel groups of several sizes (Fig. 7's
    sweep on the synthetic 1080p scene): frames/s, and the PSNR of its image
    against the plain form's over the first four orbit views."""
    import torch
    import paper_2503_05168_amd as P

    views = cams[:4]
    ref = P.Renderer(P.Settings(), capacity=1 << 26, lists="super")
    plain = [ref.render(g, [c]).image.clone() for c in views]
    out = []
    for gw, gh in groups:
        st = P.Settings(mode="contrib", group=(gw, gh))
        res = run_form(f"contrib-{gw}x{gh}", dict(g=g, st=st, hp=None), cams, steps, warmup)
        r = P.Renderer(st, capacity=ref.capacity, lists="super")
        mse = 0.0
        for c, im in zip(views, plain):
            d = r.render(g, [c]).image - im
            mse += float((d * d).mean().item()) / len(views)
        psnr = float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)
        out.append(dict(group=f"{gw}x{gh}", fps=res["fps"], raster_ms=res["stage_ms"]["raster"],
                        psnr_vs_plain=psnr, leader_tests=res["leader_tests"],
                        leader_pass=res["leader_pass"], blends=res["blends"]))
        log(f"[bench] CR group {gw}x{gh}: {res['fps']:.1f} fps, PSNR vs plain {psnr:.2f} dB")
    return out


def run_cluster_sweep(g, cams, steps, warmup, clusters=(8, 16, 24, 32), Ms=(0, 1, 3, 7)):
    """Sensitivity of hybrid preprocessing to the number of view clusters
    and of neighbouring clusters M (the structure of Fig. 6, on the
    synthetic 1080p scene): the view-dependent representation is built from
    the 128 sampled orbit poses for each cluster count, then rendered with
    the nearest cluster + M neighbours and the opacity-aware extent;
    frames/s, active Gaussians, and the image error against the plain
    full-scene image over the first four orbit views."""
    import torch
    import synthetic
    import paper_2503_05168_amd as P

    poses = synthetic.sampled_orbit_poses(6, 128, 1920, 1080)
    out = []
    for K in clusters:
        t = time.time()
        vd = P.build_view_dependent(g, poses, K, k=32, settings=P.Settings(), views_per_call=8)
        torch.cuda.synchronize()
        build_s = time.time() - t
        for M in Ms:
            if M >= K:
                continue
            form = dict(g=vd.gaussians, st=P.Settings(extent="opacity"), hp=vd, M=M)
            res = run_form(f"built-K{K}-M{M}", form, cams, steps, warmup)
            q = form_quality(g, form, cams)
            out.append(dict(clusters=K, M=M, fps=res["fps"], active=res["active"],
                            visible=res["visible"], build_s=build_s,
                            shared=vd.stats["shared"], unused=vd.stats["unused"], **q))
            log(f"[bench] clusters={K} M={M}: {res['fps']:.1f} fps, active {res['active']:.3e}, "
                f"PSNR vs plain full {q['psnr_vs_plain_full']:.2f} dB")
        del vd
        torch.cuda.empty_cache()
    return out


def run_fwd_bwd(n, n_views, steps, warmup, mode):
    """Fine-tuning step of the paper's Sec. 3.5 on the 1.0M-Gaussian workload:
    the 8 views rendered in one batched call, the loss L_3DGS (0.8 L1 + 0.2
    D-SSIM) + 0.1 FLIP against images of a perturbed copy of the scene, the
    batched backward to every raw parameter, then one Adam step.
    Returns ms per view: forward, photometric loss, FLIP, backward, Adam
    (stream time from events); forward + backward (render and the library's
    backward: the "fwd+bwd" figure) and the whole step (wall clock)."""
    import torch
    import synthetic
    import paper_2503_05168_amd as P

    scene = synthetic.cluster_scene(4, n)
    target_scene = synthetic.perturbed_scene(scene, 40)
    cams = synthetic.orbit_cameras(n_views, 4.0, 1280, 720)
    st = P.Settings(mode=mode)
    _, g = load_scene(scene)
    gt = P.GaussianTensors.from_arrays(target_scene)
    r = P.Renderer(P.Settings(), capacity=1 << 24)
    target = r.render(gt, cams).image.clone()
    del r, gt
    ft = P.FineTuner(g, st, extent=4.0, capacity=1 << 24)
    ft.renderer.render(g, cams)  # sizes the pair buffer (one synchronising pass)
    ft.renderer.capacity = int(ft.renderer.capacity * 1.05) + 4096
    npairs = torch.zeros(1, dtype=torch.int64, device="cuda")

    def step(ev=None):
        loss = ft.step(cams, target, check=False, events=None if ev is None else ev[1:])
        return loss

    for _ in range(warmup):  # the same host work as a timed step (first launches load code)
        step()
        torch.maximum(npairs, ft.renderer_last_pairs(), out=npairs)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
    losses = []
    t0 = time.perf_counter()
    for i in range(steps):
        evs[i][0].record()
        losses.append(step(evs[i]))
        torch.maximum(npairs, ft.renderer_last_pairs(), out=npairs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert int(npairs.item()) <= ft.renderer.capacity, "pair buffer overflow"
    ph = [sum(e[k].elapsed_time(e[k + 1]) for e in evs) / steps / n_views for k in range(5)]
    # work of the backward (untimed): blends of the 8 views from the
    # instrumented forward, and the visible records
    f = ft.renderer.render(g, cams)
    if f.entry_keys is not None:  # super-tile lists
        cnt = torch.zeros(6, dtype=torch.int64, device="cuda")
        P.seele_rasterize_fwd_super(f.splats, f.entry_keys, f.sorted_ids, f.tile_ranges, cams, st,
                                    counters=cnt)
    else:
        cnt = P.seele_rasterize_fwd_counted(f.splats, f.sorted_ids, f.tile_ranges, cams, st)[3]
    blends = int(cnt[1].item())
    n_vis = int((f.n_tiles > 0).sum().item())
    del f
    out = dict(ms_per_view=ph[0] + ph[3], fwd_ms_per_view=ph[0], loss_ms_per_view=ph[1],
               flip_ms_per_view=ph[2], bwd_ms_per_view=ph[3], adam_ms_per_view=ph[4],
               finetune_step_ms_per_view=1000.0 * wall / steps / n_views,
               loss_first=float(losses[0].mean().item()), loss_last=float(losses[-1].mean().item()),
               gaussians=n, views=n_views, width=1280, height=720, blends=blends,
               visible_records=n_vis)
    log(f"[bench] fwd+bwd {mode}: {out['ms_per_view']:.3f} ms/view (fwd {ph[0]:.3f}, bwd "
        f"{ph[3]:.3f}); loss {ph[1]:.3f}, FLIP {ph[2]:.3f}, Adam {ph[4]:.3f}; whole step "
        f"{out['finetune_step_ms_per_view']:.3f} ms/view; loss {out['loss_first']:.5f} -> "
        f"{out['loss_last']:.5f}")
    return out


def run_batched(n, n_views, mode, reps=3):
    """64 cameras of mixed resolution (640x480 / 1280x720 / 1920x1080, radius
    3-6 shell) over 2.0M Gaussians: sequential per-view frames vs one batched
    call (autotuned tile size, LDS batch depth and schedule) vs the batched
    frame captured in a HIP graph and replayed.  Returns ms per view."""
    import torch
    import synthetic
    import paper_2503_05168_amd as P
    from paper_2503_05168_amd.autotune import autotune
    from paper_2503_05168_amd.pipeline import bin_sort_workspace_size

    scene = synthetic.cluster_scene(5, n)
    cams = synthetic.sphere_cameras(50, n_views)
    _, g = load_scene(scene)
    del scene
    base = P.Settings(mode=mode)
    tuned = autotune(g, cams, base, reps=reps, log=log)
    st, sch, lists = tuned["settings"], tuned["schedule"], tuned["lists"]
    log(f"[bench] batched {mode}: autotuned tile={st.tile} lds_batch={st.lds_batch} "
        f"schedule={sch} lists={lists} ({tuned['ms']:.2f} ms/frame of {n_views} views)")

    # sequential: one frame per camera, default settings, super-tile lists
    seq = P.Renderer(base, capacity=1 << 22, lists="super")
    for cam in cams:
        seq.render(g, [cam])
    seq.capacity = int(seq.capacity * 1.05) + 4096
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for cam in cams:
            seq.render(g, [cam], check=False)
    torch.cuda.synchronize()
    seq_ms = 1000.0 * (time.perf_counter() - t0) / reps / n_views

    # batched eager, tuned
    r = P.Renderer(st, capacity=1 << 24, schedule=sch, lists=lists)
    f = r.render(g, cams)
    r.capacity = int(r.capacity * 1.05) + 4096
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        f = r.render(g, cams, check=False)
    torch.cuda.synchronize()
    eager_ms = 1000.0 * (time.perf_counter() - t0) / reps / n_views
    assert f.list_need() <= r.capacity

    # batched frame in a HIP graph (static buffers, device-side counts)
    V = len(cams)
    TT = P.total_tiles(cams, st.tile)
    NS = P.total_super_tiles(cams, st.tile)
    sup = lists == "super"
    npix = P.pixel_count(cams)
    cap = r.capacity
    splats = torch.empty((V * n, P.pipeline.SPLAT_FLOATS), dtype=torch.float32, device="cuda")
    n_tiles = torch.empty(V * n, dtype=torch.int32, device="cuda")
    ws = torch.empty(bin_sort_workspace_size(V * n, cap, TT), dtype=torch.uint8, device="cuda")
    ids = torch.empty(cap, dtype=torch.int32, device="cuda")
    keys = torch.empty(cap if sup else 1, dtype=torch.int32, device="cuda")
    ranges = torch.empty((NS if sup else TT, 2), dtype=torch.int32, device="cuda")
    npairs = torch.empty(2 if sup else 1, dtype=torch.int64, device="cuda")
    image = torch.empty(3 * npix, dtype=torch.float32, device="cuda")
    final_T = torch.empty(npix, dtype=torch.float32, device="cuda")
    n_contrib = torch.empty(npix, dtype=torch.int32, device="cuda")
    del f
    qws = None
    if sch != "grid":
        qws = torch.empty(int(P.lib().seele_raster_queue_workspace_size(TT)), dtype=torch.uint8,
                          device="cuda")

    def frame():
        P.seele_preprocess(g, cams, st, None, splats, n_tiles)
        if sup:
            P.seele_bin_sort_super(splats, n_tiles, n, cams, st.tile, cap, ws, keys, ids, ranges,
                                   npairs)
            P.seele_rasterize_fwd_super(splats, keys, ids, ranges, cams, st, image, final_T,
                                        n_contrib)
            return
        P.seele_bin_sort(splats, n_tiles, n, cams, st.tile, cap, ws, ids, ranges, npairs)
        if sch == "grid":
            P.seele_rasterize_fwd(splats, ids, ranges, cams, st, image, final_T, n_contrib)
        else:
            P.seele_rasterize_fwd_queue(splats, ids, ranges, cams, st,
                                        "heaviest" if sch == "queue_heavy" else "list", qws,
                                        image, final_T, n_contrib)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        frame()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        frame()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        graph.replay()
    torch.cuda.synchronize()
    graph_ms = 1000.0 * (time.perf_counter() - t0) / reps / n_views
    assert int(npairs[-1].item()) <= cap, "list buffer overflow in the graph"
    out = dict(sequential_ms_per_view=seq_ms, batched_ms_per_view=eager_ms,
               graph_ms_per_view=graph_ms, tile=st.tile, lds_batch=st.lds_batch, schedule=sch,
               lists=lists,
               pairs=int(npairs[0].item()),
               entries=int(npairs[1].item()) if sup else None, views=n_views, gaussians=n,
               autotune=[dict(t) for t in tuned["table"]])
    log(f"[bench] batched {mode}: sequential {seq_ms:.3f} ms/view, batched {eager_ms:.3f}, "
        f"graph {graph_ms:.3f}")
    del graph, splats, ws, ids, g
    torch.cuda.empty_cache()
    return out


# The CPU baseline runs in a child process of its own (started with the
# interpreter, never a fork of this GPU process); its workers are forks of
# that child and read the shared inputs from here.
_CPU = {}
_PROJ_KEYS = ("visible", "mean2d", "conic", "opacity", "rgb", "depth", "rect", "n_tiles")


def _cpu_project(chunk):
    """Worker: the float64 oracle's projection of one chunk of Gaussians."""
    import numpy as np
    from oracle import project
    lo, hi = chunk
    t0 = time.perf_counter()
    p = project.project_view(_CPU["scene"].subset(np.arange(lo, hi)), _CPU["cam"], tile=16)
    dt = time.perf_counter() - t0
    return {k: p[k] for k in _PROJ_KEYS}, dt


def _cpu_blend(tiles):
    """Worker: the float64 oracle's blending of a list of tiles."""
    from oracle import blend
    t0 = time.perf_counter()
    blend.render_tiles(_CPU["splats"], _CPU["ranges"], _CPU["ids"], _CPU["W"], _CPU["H"], 16,
                       tiles=tiles)
    return time.perf_counter() - t0


def cpu_baseline(n, n_tiles_per_worker):
    """Float64 oracle on the host cores (one thread per worker process), view
    0 of the 1080p orbit: preprocessing of every Gaussian split over the
    workers; binning (one thread) of every pair of the Gaussians that touch a
    random sample of tiles, scaled to all pairs; blending of those sampled
    tiles split over the workers, scaled to all tiles.  A phase's time is its
    slowest worker's; the binning is timed on its second call (the first
    pays this fresh process's page faults)."""
    import multiprocessing as mp
    import numpy as np
    import synthetic
    from threadpoolctl import threadpool_limits
    from oracle import binning, blend

    workers = max(1, min(16, os.cpu_count() or 1))
    scene = synthetic.cluster_scene(2, n)
    cam = synthetic.orbit_cameras(32, 4.0, 1920, 1080)[0]
    _CPU.update(scene=scene, cam=cam)
    ctx = mp.get_context("fork")
    with threadpool_limits(1):
        bounds = np.linspace(0, n, workers + 1).astype(np.int64)
        with ctx.Pool(workers) as pool:
            parts = pool.map(_cpu_project, [(int(bounds[k]), int(bounds[k + 1]))
                                            for k in range(workers)])
        t_pre = max(dt for _, dt in parts)
        p = {k: np.concatenate([q[k] for q, _ in parts]) for k in _PROJ_KEYS}
        del parts
        gw, gh = -(-cam.width // 16), -(-cam.height // 16)
        rng = np.random.default_rng(0)
        n_sample = min(gw * gh, n_tiles_per_worker * workers)
        tiles = sorted(rng.choice(gw * gh, n_sample, replace=False).tolist())
        r = p["rect"]
        touch = np.zeros(n, dtype=bool)
        for t in tiles:
            tx, ty = t % gw, t // gw
            touch |= (r[:, 0] <= tx) & (tx < r[:, 2]) & (r[:, 1] <= ty) & (ty < r[:, 3])
        nt = np.where(touch, p["n_tiles"], 0)
        all_pairs = int(p["n_tiles"].sum())
        bin_in = [dict(rect=r, n_tiles=nt, depth_f32=p["depth"].astype(np.float32), grid_w=gw,
                       grid_h=gh)]
        binning.bin_and_sort(bin_in, n)  # untimed: this process's first large allocations
        t0 = time.perf_counter()
        b = binning.bin_and_sort(bin_in, n)
        t_bin = (time.perf_counter() - t0) * all_pairs / max(1, b["n_pairs"])
        _CPU.update(splats=blend.splats_from_projection(p), ranges=b["ranges"], ids=b["ids"],
                    W=cam.width, H=cam.height)
        with ctx.Pool(workers) as pool:
            times = pool.map(_cpu_blend, [tiles[k::workers] for k in range(workers)])
        t_blend = max(times) * (gw * gh) / len(tiles)
    total = t_pre + t_bin + t_blend
    return dict(value=1.0 / total, unit="frames/s", cores=workers, kind="oracle",
                sample=(f"view 0 of the 1080p orbit, {workers} worker processes of one thread: "
                        f"float64 preprocessing of all {n} Gaussians split over the workers "
                        f"({t_pre:.1f}s); binning (one thread) of the {b['n_pairs']} pairs of "
                        f"Gaussians touching {len(tiles)} random tiles, scaled to all "
                        f"{all_pairs} pairs ({t_bin:.1f}s est.); blending of those "
                        f"{len(tiles)} tiles split over the workers, scaled to {gw * gh} "
                        f"tiles ({t_blend:.1f}s est.)"),
                seconds_per_frame=total)


def run_cpu_baseline(n, n_tiles_per_worker):
    """The CPU baseline in a child process that never touches the GPU."""
    import subprocess
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only",
                          "--n", str(n), "--cpu-tiles", str(n_tiles_per_worker)],
                         capture_output=True, text=True, timeout=600)
    if out.returncode != 0:
        raise RuntimeError(f"cpu baseline failed: {out.stderr[-2000:]}")
    return json.loads(out.stdout.strip().splitlines()[-1])


def main():
    args = parse()
    if args.cpu_baseline_only:  # the child process of run_cpu_baseline: no GPU
        print(json.dumps(cpu_baseline(args.n, args.cpu_tiles)))
        return
    if args.gpus != 1:
        print("this benchmark runs on one GPU only: the renderer shards by view with no "
              "exchange between GPUs, and only the one-GPU path is implemented and measured",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    import paper_2503_05168_amd as P
    P.lib()
    if args.pmc_calibrate:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 268435456 bytes read, 268435456 bytes written")
        del src, dst
    t_start = time.time()
    names = [s.strip() for s in args.forms.split(",") if s.strip()]
    scene, cams, forms = build_forms(names, args.n)
    results = {}
    for name in names:
        results[name] = run_form(name, forms[name], cams, args.steps, args.warmup, args.lists)
        if name == "plain" and args.lists == "super" and not args.no_pipelined:
            results[name]["pipelined"] = run_form_pipelined(name, forms[name], cams, args.steps,
                                                            args.warmup, 2)
        if "extra" in forms[name]:
            results[name].update(forms[name]["extra"])
        if "full_g" in forms[name]:
            results[name].update(form_quality(forms[name]["full_g"], forms[name], cams))
            log(f"[bench] {name}: vs the plain full-scene image PSNR "
                f"{results[name]['psnr_vs_plain_full']:.2f} dB, max abs "
                f"{results[name]['max_abs_vs_plain_full']:.3e}")
        log(f"[bench] t+{time.time() - t_start:.0f}s form {name} done")
    prefetch = None
    if not args.no_prefetch and "hp_built" in forms:
        prefetch = run_prefetch(forms["hp_built"]["hp"])
        log(f"[bench] t+{time.time() - t_start:.0f}s prefetch done")
    finetune = None
    if args.ft_steps > 0 and "hp_built" in forms:
        import synthetic
        vd = forms["hp_built"]["hp"]
        start = P.seele_gather_gaussians(
            P.GaussianTensors.from_arrays(synthetic.perturbed_scene(scene, 40)), vd.perm)
        finetune = run_integrated_finetune(vd, forms["hp_built"]["full_g"], start,
                                           args.ft_steps, lr_scale=args.ft_lr_scale,
                                           gamma=args.ft_gamma)
        del start
        log(f"[bench] t+{time.time() - t_start:.0f}s integrated fine-tuning done")
    groups = None
    if not args.no_groups and "plain" in forms:
        groups = run_group_sweep(forms["plain"]["g"], cams, max(8, args.steps // 2),
                                 max(2, args.warmup // 2))
        log(f"[bench] t+{time.time() - t_start:.0f}s group sweep done")
    clusters = None
    if not args.no_cluster_sweep and "plain" in forms:
        clusters = run_cluster_sweep(forms["plain"]["g"], cams, max(8, args.steps // 2),
                                     max(2, args.warmup // 2))
        log(f"[bench] t+{time.time() - t_start:.0f}s cluster sweep done")
    fwd_bwd = None
    if not args.no_bwd:
        del forms
        torch.cuda.empty_cache()
        fwd_bwd = {m: run_fwd_bwd(1_000_000, 8, 6, 2, m) for m in ("plain", "contrib")}
        log(f"[bench] t+{time.time() - t_start:.0f}s fwd+bwd done")
    batched = None
    if not args.no_batched:
        torch.cuda.empty_cache()
        batched = {m: run_batched(2_000_000, 64, m) for m in ("plain", "contrib")}
        log(f"[bench] t+{time.time() - t_start:.0f}s batched done")
    head = results.get("plain") or results[names[0]]
    st = head["stage_ms"]
    # Per-stage rooflines.  The rasterizer is priced on the evaluations its
    # culled loop must do (live pixels x records that can reach their 8x8
    # block) and the blends; preprocessing and binning on their algorithmic
    # HBM bytes (binning is a pipeline of ~30 kernels).
    r_ops = head["evals_needed"] * OPS_EVAL + head["blends"] * OPS_BLEND
    r_ach = r_ops / (st["raster"] * 1e-3) / 1e12
    p_bytes = 48 * head["active"] + 256 * head["visible"]
    if head.get("lists") == "super":  # staged: (depth key, id) per visible, rectangle per record
        p_bytes += 8 * head["visible"] + 8 * args.n
    p_ach = p_bytes / (st["preprocess"] * 1e-3) / 1e9
    # binning: 16 B per visible record (depth key, id, rectangle) plus its
    # output -- 8 B per super-tile entry (key, id) and 8 B per super-tile
    # range, or 4 B per pair and 8 B per tile range for per-tile lists
    if head.get("lists") == "super":
        b_bytes = 16 * head["visible"] + 8 * head["entries"] + 8 * head["super_tiles"]
    else:
        b_bytes = 16 * head["visible"] + 4 * head["pairs"] + 8 * head["tiles"]
    b_ach = b_bytes / (st["bin_sort"] * 1e-3) / 1e9
    stage_roof = {
        "raster": dict(bound="alu", achieved=r_ach, peak=PEAK_LANE_OPS / 1e12,
                       unit="Tlane-op/s", frac=r_ach / (PEAK_LANE_OPS / 1e12)),
        "preprocess": dict(bound="hbm", achieved=p_ach, peak=PEAK_HBM / 1e9, unit="GB/s",
                           frac=p_ach / (PEAK_HBM / 1e9)),
        "bin_sort": dict(bound="hbm", achieved=b_ach, peak=PEAK_HBM / 1e9, unit="GB/s",
                         frac=b_ach / (PEAK_HBM / 1e9)),
    }
    if fwd_bwd is not None:
        # backward of the 8-view 720p fine-tuning frame: per blend ~40 lane-ops,
        # per visible record ~300 (the preprocessing chain), per Gaussian 236 B
        # of gradients written; priced against the VALU peak
        fb = fwd_bwd["plain"]
        b_ops = OPS_BWD_BLEND * fb["blends"] + OPS_BWD_RECORD * fb["visible_records"]
        b_s = fb["bwd_ms_per_view"] * fb["views"] * 1e-3
        stage_roof["raster_bwd"] = dict(
            bound="alu", achieved=b_ops / b_s / 1e12, peak=PEAK_LANE_OPS / 1e12,
            unit="Tlane-op/s", frac=b_ops / b_s / PEAK_LANE_OPS,
            grad_bytes_GBps=236 * fb["gaussians"] / b_s / 1e9,
            workload="1.0M Gaussians, 8 x 1280x720, plain")
    # the dominant single kernel: the rasterizer or the preprocessing kernel
    if st["raster"] >= st["preprocess"]:
        kname = "raster_fwd_super" if head.get("lists") == "super" else "raster_fwd"
        roof = dict(stage_roof["raster"], kernel=kname,
                    traffic=measured_traffic(f"{kname}_plain_c2_1080p_3M"),
                    traffic_unit="bytes/launch")
    else:
        roof = dict(stage_roof["preprocess"], kernel="preprocess", traffic=None)
    cpu = None
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle) ...")
        cpu = run_cpu_baseline(args.n, args.cpu_tiles)
        log(f"[bench] t+{time.time() - t_start:.0f}s cpu baseline {cpu['value']:.3e} frames/s")
    line = {
        "metric": "1080p FPS @3M Gaussians, plain vs contribution-aware; fwd+bwd ms/view",
        "value": head["fps"],
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_frame"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"outdoor-shaped scene, {args.n} Gaussians (64 clusters + 10% "
                                f"shell, seed 2, stored in Morton order of the means), 32-view "
                                f"orbit r=4, 1920x1080, 16x16 tiles, plain 3DGS forward "
                                f"(preprocess + bin/sort + raster), {args.lists} lists"),
                   "gaussians": args.n, "views": 32, "width": 1920, "height": 1080, "tile": 16},
        "forms": {k: {kk: vv for kk, vv in v.items()} for k, v in results.items()},
        "fwd_bwd_ms_per_view": (None if fwd_bwd is None else
                                {k: v["ms_per_view"] for k, v in fwd_bwd.items()}),
        "fwd_bwd": fwd_bwd,
        "batched_64_views": batched,
        "contrib_group_sweep": groups,
        "hp_cluster_sweep": clusters,
        "scene_prefetch": prefetch,
        "integrated_finetune": finetune,
        "roofline": roof,
        "stage_roofline": stage_roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
