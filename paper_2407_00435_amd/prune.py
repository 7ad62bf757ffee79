"""Efficiency-aware pruning round (Section 3) on the library's kernels.

``ce_over_views`` renders every view of a camera set once (projection,
binning with per-point hit counts, compositing with dominated-pixel counts)
and reduces them to one computational efficiency per point;
``prune_round`` then selects the R = 10 % of points with the lowest CE.
Torch only provides memory and the stream.
"""
from __future__ import annotations

import torch

from . import binding as B


def ce_over_views(scene: B.SceneTensors, cams: B.Cameras, tile_size: int = 16, foveated_filter=None):
    """CE per point over the views of ``cams``; also returns the hit counts
    [V, n] (the U of the weighted scale).  ``foveated_filter`` = (tile_level,
    qbound) applies the level filter of Section 4.2 to the hit counts."""
    splats = B.gs_project(scene, cams, tile_size)
    tl, qb = foveated_filter if foveated_filter is not None else (None, None)
    bs = B.gs_bin_sort(splats, scene.n, cams, tile_size, tile_level=tl, qbound=qb, want_hits=True)
    out = B.gs_rasterize_fwd(splats, scene.n, cams, tile_size, bs["vals"], bs["ranges"], want_dominated=True)
    ce = B.gs_ce_score(out["dominated"], bs["hits"])
    return ce, bs["hits"], out["dominated"]


def prune_round(scene: B.SceneTensors, cams: B.Cameras, tile_size: int = 16, fraction: float = 0.10):
    """(keep mask [n] bool, removed indices [k] ascending, CE [n]) for one
    pruning round removing ``fraction`` of the points with the lowest CE."""
    ce, _, _ = ce_over_views(scene, cams, tile_size)
    k = int(fraction * scene.n)
    mask, idx = B.gs_select_lowest(ce, k)
    return mask == 0, idx, ce
