"""Autotuner for the batched renderer: tile size x LDS batch depth x raster
schedule x list form, timed on the caller's own workload.

Each candidate renders the full frame (all views, preprocess + sort +
raster) a few times with HIP events on the current stream; the fastest is
returned and cached as JSON, keyed by the GPU name and a workload signature
(Gaussian count, camera sizes, mode).  Changing the tile size changes which
tiles a Gaussian's extent covers, so images may differ between tile sizes in
the last few of a Gaussian's pixels; the batch depth, the schedule and the
list form (per-tile or super-tile lists, the latter with the grid schedule
and the default batch depth) never change a result.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import os

import torch

from .pipeline import CapacityError, Renderer, Settings

CANDIDATE_BATCH = {16: (256, 128, 64), 8: (64,)}
SCHEDULES = ("grid", "queue", "queue_heavy")


def workload_key(g, cams, settings: Settings) -> str:
    sig = json.dumps(dict(n=int(g.n), cams=[(int(c.width), int(c.height)) for c in cams],
                          mode=settings.mode, extent=settings.extent,
                          group=list(settings.group)), sort_keys=True)
    return hashlib.sha256(sig.encode()).hexdigest()[:16]


def _candidates(tiles, schedules):
    """(tile, lds_batch, schedule, lists) in trial order."""
    out = []
    for tile in tiles:
        for batch in CANDIDATE_BATCH[tile]:
            for sch in schedules:
                out.append((tile, batch, sch, "tile"))
            if batch == tile * tile and "grid" in schedules:
                out.append((tile, batch, "grid", "super"))
    return out


def _time_frame(renderer: Renderer, g, cams, segments, reps: int) -> float:
    f = renderer.render(g, cams, segments)  # sizes the pair buffer
    renderer.capacity = int(renderer.capacity * 1.05) + 4096
    renderer.render(g, cams, segments, check=False)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        f = renderer.render(g, cams, segments, check=False)
    stop.record()
    torch.cuda.synchronize()
    assert f.list_need() <= renderer.capacity
    return start.elapsed_time(stop) / reps


def autotune(g, cams, settings: Settings | None = None, segments=None, reps: int = 3,
             tiles=(16, 8), schedules=SCHEDULES, cache_path: str | None = None,
             log=None) -> dict:
    """Return {"settings": Settings, "schedule": str, "lists": str, "ms": float,
    "table": [...]}."""
    settings = settings or Settings()
    dev = torch.cuda.get_device_name()
    key = f"{dev}|{workload_key(g, cams, settings)}"
    cache = {}
    if cache_path and os.path.exists(cache_path):
        cache = json.load(open(cache_path))
        if key in cache:
            c = cache[key]
            st = dataclasses.replace(settings, tile=c["tile"], lds_batch=c["lds_batch"])
            return dict(settings=st, schedule=c["schedule"], lists=c.get("lists", "tile"),
                        ms=c["ms"], table=c["table"], cached=True)
    table = []
    best = None
    skipped = set()  # (tile, lists) whose lists do not fit one call
    for tile, batch, sch, lists in _candidates(tiles, schedules):
        if (tile, lists) in skipped:
            continue
        st = dataclasses.replace(settings, tile=tile, lds_batch=batch)
        try:
            ms = _time_frame(Renderer(st, capacity=1 << 22, schedule=sch, lists=lists), g, cams,
                             segments, reps)
        except CapacityError as e:
            table.append(dict(tile=tile, lds_batch=batch, schedule=sch, lists=lists, ms=None,
                              skipped=str(e)))
            if log:
                log(f"[autotune] tile={tile} batch={batch}: skipped ({e})")
            # the list length depends on the tile size and the list form only
            skipped.add((tile, lists))
            continue
        table.append(dict(tile=tile, lds_batch=batch, schedule=sch, lists=lists, ms=ms))
        if log:
            log(f"[autotune] tile={tile} batch={batch} schedule={sch} lists={lists}: {ms:.3f} ms")
        if best is None or ms < best[0]:
            best = (ms, st, sch, lists)
    ms, st, sch, lists = best
    if cache_path:
        cache[key] = dict(tile=st.tile, lds_batch=st.lds_batch, schedule=sch, lists=lists, ms=ms,
                          table=table)
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        json.dump(cache, open(cache_path, "w"), indent=1)
    return dict(settings=st, schedule=sch, lists=lists, ms=ms, table=table, cached=False)
