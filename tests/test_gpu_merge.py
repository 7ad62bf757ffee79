"""Tile merging (the Tile Merge Unit of Section 5.2, on the GPU) through the
C ABI: with the "raster_merge" knob at beta, consecutive tiles whose keys
total at most beta form one merged tile (a heavier tile alone) and a
persistent compositor's workgroups take merged tiles whole.

- The groups the GPU forms equal a plain host greedy over the tile loads
  (read back from the workspace).
- Images, final transmittance and last contributors equal those of one
  workgroup per tile bit for bit (each pixel runs the same arithmetic), for
  the plain and the foveated compositor, at several beta and tile sizes;
  the per-tile results are held to the oracle in the parity tests, and one
  case here checks the merged image against the oracle directly.
"""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from gpu_util import check_envelope, image_views, need_gpu, say, splat_np, view_slice

pytestmark = pytest.mark.gpu

WS_HEADER = 256


def gs():
    need_gpu()
    import paper_2407_00435_amd as g
    return g


def greedy_groups(loads, beta):
    groups, i, T = [], 0, len(loads)
    while i < T:
        j, tot = i + 1, int(loads[i])
        while j < T and tot + int(loads[j]) <= beta:
            tot += int(loads[j])
            j += 1
        groups.append((i, j))
        i = j
    return groups


def read_groups(ws, n_tiles):
    t, ptr, _ = ws
    off = ptr.value - t.data_ptr() + WS_HEADER
    w = t[off:].cpu().numpy().view(np.uint32)
    n1 = n_tiles + 1
    ng = int(w[0])
    g0 = 16 + 5 * n1 + (1 if n1 % 2 else 0)
    gr = w[g0:g0 + 2 * ng].reshape(ng, 2)
    return [(int(a), int(b)) for a, b in gr]


def plain_case(seed=61):
    sc = scenegen.small_scene(4000, seed=seed, sh_degree=3, log_scale_mu=-3.4, log_scale_sigma=0.6)
    cams = [scenegen.pinhole(203, 157, 60.0, t=(0.0, 0.0, 4.0)),
            scenegen.look_at((1.2, -0.6, -3.3), (0.1, 0.0, 0.0), 131, 97, 55.0)]
    return sc, cams


@pytest.mark.parametrize("tile,beta", [(16, 1), (16, 300), (16, 4000), (8, 700), (32, 2000), (16, 1 << 30)])
def test_merged_plain_equals_per_tile(tile, beta):
    g = gs()
    sc, cams = plain_case()
    say("merged plain", tile, beta)
    C, S = g.Cameras(cams), g.SceneTensors(sc)
    splats = g.gs_project(S, C, tile)
    bs = g.gs_bin_sort(splats, sc.n, C, tile, check=True)
    ref = g.gs_rasterize_fwd(splats, sc.n, C, tile, bs["vals"], bs["ranges"], (0.1, 0.2, 0.3))
    n_tiles, _ = C.tiles(tile)
    ctx = g.context()
    ctx.set_tuning("raster_merge", beta)
    try:
        ws = g.binding._ws(g.gs_workspace_bytes(C, sc.n, tile, bs["capacity"]))
        out = g.gs_rasterize_fwd(splats, sc.n, C, tile, bs["vals"], bs["ranges"], (0.1, 0.2, 0.3), workspace=ws)
        torch.cuda.synchronize()
    finally:
        ctx.set_tuning("raster_merge", 0)
    for k in ("image", "final_T", "n_contrib"):
        assert torch.equal(out[k], ref[k]), k
    r = bs["ranges"].cpu().numpy().astype(np.int64)
    expect = greedy_groups(r[:, 1] - r[:, 0], beta)
    got = read_groups(ws, n_tiles)
    assert got == expect
    say(f"{n_tiles} tiles in {len(got)} merged tiles")


@pytest.mark.parametrize("tile,beta", [(16, 512), (8, 2048), (16, 1)])
def test_merged_foveated_equals_per_tile(tile, beta):
    g = gs()
    sc = scenegen.small_scene(5000, seed=62, sh_degree=3, fr_levels=4, log_scale_mu=-3.4, log_scale_sigma=0.6)
    cams = [scenegen.pinhole(300, 170, scenegen.FR_FOV_DEG, t=(0.03, 0.0, 2.0)),
            scenegen.pinhole(280, 190, scenegen.FR_FOV_DEG, t=(-0.03, 0.0, 2.0))]
    fov = [scenegen.Fovea(150.0, 85.0), scenegen.Fovea(120.0, 100.0)]
    say("merged foveated", tile, beta)
    C, S = g.Cameras(cams), g.SceneTensors(sc)
    t = g.gs_fovea_prep(C, fov, tile, 4)
    splats, lvl = g.gs_project(S, C, tile, levels=True)
    bs = g.gs_bin_sort(splats, sc.n, C, tile, tile_level=t["tile_level"], qbound=S.t["qbound"], check=True)
    ref = g.gs_rasterize_foveated(splats, lvl, sc.n, S.t["qbound"], 4, C, tile, bs["vals"], bs["ranges"],
                                  t["pix_level"], t["pix_weight"])
    ctx = g.context()
    ctx.set_tuning("raster_merge", beta)
    try:
        ws = g.binding._ws(g.gs_workspace_bytes(C, sc.n, tile, bs["capacity"]))
        img = g.gs_rasterize_foveated(splats, lvl, sc.n, S.t["qbound"], 4, C, tile, bs["vals"], bs["ranges"],
                                      t["pix_level"], t["pix_weight"], workspace=ws)
        one, _, _ = g.gs_render_foveated(S, C, fov, tile, key_capacity=bs["capacity"])
        torch.cuda.synchronize()
    finally:
        ctx.set_tuning("raster_merge", 0)
    assert torch.equal(img, ref)
    assert torch.equal(one, ref)
    n_tiles, _ = C.tiles(tile)
    r = bs["ranges"].cpu().numpy().astype(np.int64)
    assert read_groups(ws, n_tiles) == greedy_groups(r[:, 1] - r[:, 0], beta)


def test_merged_image_matches_oracle():
    g = gs()
    sc, cams = plain_case(seed=63)
    say("merged against the oracle")
    C, S = g.Cameras(cams), g.SceneTensors(sc)
    ctx = g.context()
    ctx.set_tuning("raster_merge", 1500)
    try:
        out = g.gs_render_fwd(S, C, 16, key_capacity=200_000, check=True)
        torch.cuda.synchronize()
    finally:
        ctx.set_tuning("raster_merge", 0)
    sp = splat_np(out["splats"])
    imgs = image_views(out["image"], [(c.width, c.height) for c in cams])
    for v, cam in enumerate(cams):
        ref = oracle.composite(oracle.splats_to_proj(view_slice(sp, v)), cam.width, cam.height)
        err, namb = check_envelope(imgs[v], ref)
        say(f"view {v}: max err {err:.3g}, ambiguous {namb}")
