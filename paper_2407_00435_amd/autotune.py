"""Autotuner for the batched step: tile size, views per sub-batch, the
number of streams the sub-batches alternate over, the sort's partition size
and the compositor's scheduling (one workgroup per tile or the persistent
work queue).

Candidates are measured, not modelled: each is built (buffers, a recorded
graph), replayed a few times on the device, and timed with events on its
stream.  The search is coordinate descent from (tile 16, all views in one
sub-batch, one stream, partition 8192, one workgroup per tile): first the
tile size, then the sub-batch size (on one and on two streams) at the best
tile, then the partition size, then the persistent work-queue compositor.  A candidate that does not fit in
device memory is skipped.  Results can be cached in a JSON file keyed by the
workload's shape (point count, SH degree, view sizes, device name).
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import binding as B
from .batched import BatchedStep


def _signature(scene, cams, eyes):
    sizes = [(int(c.width), int(c.height)) for c in cams]
    esz = [(int(c.width), int(c.height)) for c in (eyes or [])]
    return json.dumps(dict(n=scene.n, sh=scene.sh_degree, levels=scene.n_levels, views=sizes, eyes=esz,
                           device=torch.cuda.get_device_name()), sort_keys=True)


def time_step(step: BatchedStep, reps: int = 3) -> float:
    """Mean milliseconds of a graph replay of ``step`` (records it if needed)."""
    if step.graph is None:
        step.capture()
    step.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(step.stream)
    for _ in range(reps):
        step.graph.launch(step.stream)
    e1.record(step.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(scene, cams, target, eyes=None, foveae=None, tiles=(16, 32, 8), reps=3, cache_path=None,
         log=None):
    """Returns (best config dict, list of (config, ms) tried)."""
    sig = _signature(scene, cams, eyes)
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if sig in cache:
            return cache[sig], []
    V = len(cams)
    tried = []

    def measure(cfg):
        for c, ms in tried:
            if c == cfg:
                return ms
        B.gs_set_tuning("radix_part", cfg["radix_part"])
        B.gs_set_tuning("raster_queue", cfg["raster_queue"])
        step = None
        try:
            step = BatchedStep(scene, cams, target, cfg["tile"], cfg["batch_views"], eyes, foveae,
                               lanes=cfg.get("lanes", 1))
            ms = time_step(step, reps)
            if not step.keys_ok():
                ms = math.inf
        except (torch.cuda.OutOfMemoryError, B.GsError) as e:
            if log:
                log(f"  {cfg}: skipped ({type(e).__name__})")
            ms = math.inf
        finally:
            del step
            torch.cuda.empty_cache()
        tried.append((dict(cfg), ms))
        if log:
            log(f"  {cfg}: {ms:.3f} ms")
        return ms

    best = dict(tile=16, batch_views=V, lanes=1, radix_part=8192, raster_queue=0)
    best_ms = measure(best)
    for t in tiles:
        c = dict(best, tile=t)
        ms = measure(c)
        if ms < best_ms:
            best, best_ms = c, ms
    for bv in sorted({max(1, math.ceil(V / 2)), max(1, math.ceil(V / 4))}):
        for ln in (1, 2):
            c = dict(best, batch_views=bv, lanes=ln)
            ms = measure(c)
            if ms < best_ms:
                best, best_ms = c, ms
    for key, alt in (("radix_part", 16384), ("raster_queue", 1)):
        c = dict(best, **{key: alt})
        ms = measure(c)
        if ms < best_ms:
            best, best_ms = c, ms
    B.gs_set_tuning("radix_part", best["radix_part"])
    B.gs_set_tuning("raster_queue", best["raster_queue"])
    best = dict(best, ms=best_ms)
    if cache_path:
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        cache[sig] = best
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best, tried
