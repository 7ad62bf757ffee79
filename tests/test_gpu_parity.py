"""Parity of the HIP path against the FP64 oracle, stage by stage, through the
C ABI (projection, binning, compositing, foveation, reverse pass).

Sizes are small enough for the oracle to finish in seconds but span many
tiles with ragged image borders.  Bars: binning outputs bit-exact; images
within 2e-4 per channel of the oracle's branch envelope (threshold-ambiguous
pixels may land on either side of a cut-off); projection within float32
rounding of the FP64 values; gradients within 1e-3 relative L2.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import scenegen
from gpu_util import (IMG_TOL, check_envelope, conic_rounding_bound, image_views, need_gpu, per_point_check,
                      pixel_views, rel_l2, say, splat_np, view_slice)

pytestmark = pytest.mark.gpu


def gs():
    need_gpu()
    import paper_2407_00435_amd as g
    return g


def two_views():
    return [scenegen.pinhole(203, 157, 60.0, t=(0.0, 0.0, 4.0)),
            scenegen.look_at((1.2, -0.6, -3.3), (0.1, 0.0, 0.0), 131, 97, 55.0)]


def scene_small(seed=7, n=3000, deg=3, fr=0):
    return scenegen.small_scene(n, seed=seed, sh_degree=deg, fr_levels=fr, log_scale_mu=-3.4,
                                log_scale_sigma=0.6)


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_projection_matches_oracle(deg):
    g = gs()
    sc = scene_small(seed=10 + deg, deg=deg)
    cams = two_views()
    say("projection", deg)
    C = g.Cameras(cams)
    S = g.SceneTensors(sc)
    sp = splat_np(g.gs_project(S, C, 16))
    for v, cam in enumerate(cams):
        ref = oracle.project(sc, cam)
        s = view_slice(sp, v)
        vis = ref["visible"] > 0
        np.testing.assert_array_equal(s["radius"] > 0, vis)
        # radius: ceil of 3 sqrt(lambda_max) -- equal unless the argument sits
        # within float32 rounding of an integer
        mid = 0.5 * (ref["cov2d"][:, 0] + ref["cov2d"][:, 2])
        det = ref["cov2d"][:, 0] * ref["cov2d"][:, 2] - ref["cov2d"][:, 1] ** 2
        arg = 3.0 * np.sqrt(mid + np.sqrt(np.maximum(mid * mid - det, 0.0)))
        near_int = np.abs(arg - np.round(arg)) < 1e-4 * arg
        ok = vis & ~near_int
        np.testing.assert_array_equal(s["radius"][ok], ref["radius"][ok])
        m = ref["mean2d"][vis]
        assert np.all(np.abs(s["mean2d"][vis] - m) <= 1e-4 * (1 + np.abs(m))), "mean2d"
        cn = ref["conic"][vis]
        scale = np.abs(cn).max(axis=1, keepdims=True)
        # conic: within float32 rounding of the FP64 inverse, as propagated
        # through the determinant's cancellation
        dc = np.abs(s["conic"][vis] - cn)
        bound = conic_rounding_bound(ref["cov2d"][vis], cn)
        say(f"view {v}: conic error / row max {float((dc / scale).max()):.2e}, "
            f"/ rounding bound {float((dc / bound).max()):.3f}")
        assert np.all(dc <= bound), "conic"
        np.testing.assert_allclose(s["depth"][vis], ref["depth"][vis], rtol=2e-6)
        np.testing.assert_allclose(s["opacity"], ref["opacity"], atol=2e-6)
        np.testing.assert_allclose(s["color"][vis], ref["color"][vis], atol=2e-5)
        # the unfiltered rectangle tile count is the float32 binning rule
        b = oracle.bin_f32(s["mean2d"], s["radius"], s["depth"], [cam.width], [cam.height], 16)
        np.testing.assert_array_equal(s["tiles_touched"].astype(np.uint32), b["hits"][0])


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_binning_bit_exact(tile):
    g = gs()
    sc = scene_small(seed=21)
    cams = two_views()
    say("binning", tile)
    C = g.Cameras(cams)
    S = g.SceneTensors(sc)
    splats = g.gs_project(S, C, tile)
    out = g.gs_bin_sort(splats, sc.n, C, tile, want_keys=True, want_hits=True)
    torch.cuda.synchronize()
    sp = splat_np(splats)
    ref = oracle.bin_f32(sp["mean2d"], sp["radius"], sp["depth"], [c.width for c in cams],
                         [c.height for c in cams], tile)
    nk = int(out["num_keys"].item())
    assert nk == ref["num_keys"] > 1000
    np.testing.assert_array_equal(out["keys"].cpu().numpy()[:nk].view(np.uint64), ref["keys"])
    np.testing.assert_array_equal(out["vals"].cpu().numpy()[:nk].view(np.uint32), ref["vals"])
    np.testing.assert_array_equal(out["ranges"].cpu().numpy().view(np.uint32), ref["ranges"])
    np.testing.assert_array_equal(out["hits"].cpu().numpy().view(np.uint32), ref["hits"])


# coarse pairs carry their rectangle in the sort key (ids below 2^17) or in an
# 8-byte value (the form used above 2^17 super-tiles); both give the oracle's
# keys, with and without the level filter (whose bound rides in the pair)
@pytest.mark.parametrize("packed", [1, 0])
@pytest.mark.parametrize("filtered", [False, True])
def test_binning_coarse_pair_forms(packed, filtered):
    g = gs()
    tile = 16
    sc = scene_small(seed=53, n=4000, fr=4)
    cams = [scenegen.pinhole(300, 170, scenegen.FR_FOV_DEG, t=(0.03, 0.0, 2.0)),
            scenegen.pinhole(280, 190, scenegen.FR_FOV_DEG, t=(-0.03, 0.0, 2.0))]
    say("coarse pairs", packed, filtered)
    C = g.Cameras(cams)
    S = g.SceneTensors(sc)
    splats = g.gs_project(S, C, tile)
    kw = {}
    tl = None
    if filtered:
        fov = [scenegen.Fovea(150.0, 85.0)] * 2
        t = g.gs_fovea_prep(C, fov, tile, 4)
        kw = dict(tile_level=t["tile_level"], qbound=S.t["qbound"])
        tl = t["tile_level"][:, 0].cpu().numpy()
    g.gs_set_tuning("coarse_packed", packed)
    try:
        bs = g.gs_bin_sort(splats, sc.n, C, tile, want_keys=True, want_hits=True, **kw)
        torch.cuda.synchronize()
    finally:
        g.gs_set_tuning("coarse_packed", 1)
    sp = splat_np(splats)
    ref = oracle.bin_f32(sp["mean2d"], sp["radius"], sp["depth"], [c.width for c in cams],
                         [c.height for c in cams], tile,
                         **(dict(tile_level_lo=tl, qbound=sc.qbound) if filtered else {}))
    nk = int(bs["num_keys"].item())
    assert nk == ref["num_keys"] > 1000
    np.testing.assert_array_equal(bs["keys"].cpu().numpy()[:nk].view(np.uint64), ref["keys"])
    np.testing.assert_array_equal(bs["vals"].cpu().numpy()[:nk].view(np.uint32), ref["vals"])
    np.testing.assert_array_equal(bs["ranges"].cpu().numpy().view(np.uint32), ref["ranges"])
    # per-point hit counts after the level filter (Comp_i of Eq. 3 after the
    # Section 4.2 filter) are bit-exact too
    np.testing.assert_array_equal(bs["hits"].cpu().numpy().view(np.uint32), ref["hits"])


def _raster_case(g, sc, cams, tile, bg=(0.0, 0.0, 0.0), dominated=True):
    C = g.Cameras(cams)
    S = g.SceneTensors(sc)
    splats = g.gs_project(S, C, tile)
    bs = g.gs_bin_sort(splats, sc.n, C, tile)
    out = g.gs_rasterize_fwd(splats, sc.n, C, tile, bs["vals"], bs["ranges"], bg,
                             want_dominated=dominated)
    torch.cuda.synchronize()
    return C, splats, bs, out


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_rasterize_matches_oracle_composite(tile):
    g = gs()
    sc = scene_small(seed=31)
    cams = two_views()
    bg = (0.1, 0.25, 0.05)
    say("raster", tile)
    C, splats, bs, out = _raster_case(g, sc, cams, tile, bg)
    sp = splat_np(splats)
    sizes = [(c.width, c.height) for c in cams]
    imgs = image_views(out["image"], sizes)
    Ts = pixel_views(out["final_T"], sizes)
    ncs = pixel_views(out["n_contrib"], sizes)
    dom = out["dominated"].cpu().numpy()
    vals = bs["vals"].cpu().numpy()
    ranges = bs["ranges"].cpu().numpy()
    tile_off = 0
    for v, cam in enumerate(cams):
        ref = oracle.composite(oracle.splats_to_proj(view_slice(sp, v)), cam.width, cam.height, bg=bg)
        err, namb = check_envelope(imgs[v], ref)
        say(f"view {v}: max err {err:.3g}, ambiguous {namb}")
        amb = ref["amb"] != 0
        np.testing.assert_allclose(Ts[v][~amb], ref["T"][~amb], atol=2e-5, rtol=1e-4)
        # last blended point: the GPU's position in the tile run names a point id
        W, H = cam.width, cam.height
        tx_n = (W + tile - 1) // tile
        yy, xx = np.mgrid[:H, :W]
        gt = tile_off + (yy // tile) * tx_n + (xx // tile)
        nc = ncs[v].astype(np.int64)
        start = ranges[gt, 0].astype(np.int64)
        last = np.where(nc > 0, vals[np.clip(start + nc - 1, 0, len(vals) - 1)], -1)
        ok = (ref["last_set"] == last[..., None]).any(-1)
        assert ok[~amb].all(), f"last contributor differs at {np.argwhere(~ok & ~amb)[:5]}"
        assert ok.mean() > 0.999
        # Val_i: per point counts between the unambiguous and the possible dominations
        sure = np.zeros(sc.n, np.int64)
        maybe = np.zeros(sc.n, np.int64)
        ds = ref["dom_set"].reshape(-1, 4)
        single = (ds[:, 1] == -2) & (ds[:, 0] >= 0)
        np.add.at(sure, ds[single, 0], 1)
        for row in ds[~single]:
            for i in row:
                if i >= 0:
                    maybe[i] += 1
        assert np.all(dom[v] >= sure) and np.all(dom[v] <= sure + maybe)
        tile_off += tx_n * ((H + tile - 1) // tile)


def test_end_to_end_image_matches_fp64_oracle():
    g = gs()
    sc = scene_small(seed=41)
    cams = two_views()
    say("end-to-end")
    C, splats, bs, out = _raster_case(g, sc, cams, 16, dominated=False)
    imgs = image_views(out["image"], [(c.width, c.height) for c in cams])
    for v, cam in enumerate(cams):
        ref = oracle.render(sc, cam, margins=(2e-4, 2e-4, 1e-4, 1e-4))
        err, namb = check_envelope(imgs[v], ref, max_unresolved_frac=1e-3)
        say(f"view {v}: max err vs fp64 {err:.3g}, ambiguous {namb}")


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_foveation_tables(tile):
    """Per-pixel levels and weights and per-tile level ranges; the widths
    leave a partial strip of tiles at the right edge at every tile size (the
    kernel takes 64-pixel-wide strips of tiles) and partial tiles below."""
    g = gs()
    cams = [scenegen.pinhole(320, 180, scenegen.FR_FOV_DEG, t=(0.03, 0.0, 2.0)),
            scenegen.pinhole(232, 170, scenegen.FR_FOV_DEG, t=(-0.03, 0.0, 2.0)),
            scenegen.pinhole(200, 90, scenegen.FR_FOV_DEG, t=(0.0, 0.02, 2.0))]
    fov = [scenegen.Fovea(140.0, 95.0), scenegen.Fovea(120.3, 70.7), scenegen.Fovea(90.0, 40.0)]
    say(f"fovea tables, tile {tile}")
    C = g.Cameras(cams)
    t = g.gs_fovea_prep(C, fov, tile, 4)
    sizes = [(c.width, c.height) for c in cams]
    lv = pixel_views(t["pix_level"], sizes)
    wt = pixel_views(t["pix_weight"], sizes)
    tl = t["tile_level"].cpu().numpy()
    off = 0
    for v, cam in enumerate(cams):
        ref = oracle.fovea(cam, fov[v], 4, tile, eps=1e-3)
        amb = ref["pix_amb"].reshape(cam.height, cam.width) > 0
        np.testing.assert_array_equal(lv[v][~amb], ref["pix_lo"].reshape(cam.height, cam.width)[~amb])
        np.testing.assert_allclose(wt[v], ref["pix_w"].reshape(cam.height, cam.width), atol=2e-3 / 3.5)
        nt = len(ref["tile_lo"])
        tamb = ref["tile_amb"] > 0
        np.testing.assert_array_equal(tl[off:off + nt, 0][~tamb], ref["tile_lo"][~tamb])
        np.testing.assert_array_equal(tl[off:off + nt, 1][~tamb], ref["tile_hi"][~tamb])
        off += nt


def _fr_case(g, sc, cams, fov, tile):
    C = g.Cameras(cams)
    S = g.SceneTensors(sc)
    t = g.gs_fovea_prep(C, fov, tile, 4)
    splats, lvl = g.gs_project(S, C, tile, levels=True)
    bs = g.gs_bin_sort(splats, sc.n, C, tile, tile_level=t["tile_level"], qbound=S.t["qbound"],
                       want_keys=True, want_hits=True)
    img = g.gs_rasterize_foveated(splats, lvl, sc.n, S.t["qbound"], 4, C, tile, bs["vals"],
                                  bs["ranges"], t["pix_level"], t["pix_weight"])
    torch.cuda.synchronize()
    return C, S, t, splats, lvl, bs, img


def _max_block_span(pl, pw):
    """Largest number of levels the pixels of one 8 x 8 block use."""
    hi = pl.astype(np.int32) + (pw > 0)
    H, W = pl.shape
    span = 0
    for y in range(0, H, 8):
        for x in range(0, W, 8):
            span = max(span, int(hi[y:y + 8, x:x + 8].max() - pl[y:y + 8, x:x + 8].min()) + 1)
    return span


# the last case puts rings 2 degrees (about 6 pixels) apart: 8 x 8 blocks then
# need up to four levels, the compositor's path for blocks wider than two
@pytest.mark.parametrize("tile,rings,band", [(8, (12.0, 24.0, 33.0), 3.5), (16, (12.0, 24.0, 33.0), 3.5),
                                             (16, (10.0, 12.0, 14.0), 1.0)])
def test_foveated_matches_oracle(tile, rings, band):
    g = gs()
    sc = scene_small(seed=51, n=4000, fr=4)
    cams = [scenegen.pinhole(300, 170, scenegen.FR_FOV_DEG, t=(0.03, 0.0, 2.0)),
            scenegen.pinhole(300, 170, scenegen.FR_FOV_DEG, t=(-0.03, 0.0, 2.0))]
    fov = [scenegen.Fovea(160.0, 80.0, rings_deg=rings, band_deg=band)] * 2
    say("foveated", tile, rings, band)
    C, S, t, splats, lvl, bs, img = _fr_case(g, sc, cams, fov, tile)
    sp = splat_np(splats)
    lvn = lvl.cpu().numpy()
    sizes = [(c.width, c.height) for c in cams]
    # filtered binning is bit-exact given the GPU's level table
    ref_b = oracle.bin_f32(sp["mean2d"], sp["radius"], sp["depth"], [c.width for c in cams],
                           [c.height for c in cams], tile,
                           tile_level_lo=t["tile_level"][:, 0].cpu().numpy(), qbound=sc.qbound)
    nk = int(bs["num_keys"].item())
    assert nk == ref_b["num_keys"]
    np.testing.assert_array_equal(bs["keys"].cpu().numpy()[:nk].view(np.uint64), ref_b["keys"])
    np.testing.assert_array_equal(bs["vals"].cpu().numpy()[:nk].view(np.uint32), ref_b["vals"])
    np.testing.assert_array_equal(bs["ranges"].cpu().numpy().view(np.uint32), ref_b["ranges"])
    # filtered per-point hit counts (Comp_i after the level filter) bit for bit
    np.testing.assert_array_equal(bs["hits"].cpu().numpy().view(np.uint32), ref_b["hits"])
    # fewer keys than the unfiltered rectangle count
    assert nk < int(sp["tiles_touched"].sum())
    imgs = image_views(img, sizes)
    pl = pixel_views(t["pix_level"], sizes)
    pw = pixel_views(t["pix_weight"], sizes)
    spans = [_max_block_span(pl[v], pw[v]) for v in range(len(cams))]
    assert (max(spans) == 2) if band > 2.0 else (max(spans) >= 3), spans
    for v, cam in enumerate(cams):
        proj = oracle.splats_to_proj(view_slice(sp, v))
        proj["lvl_opacity"] = lvn[v, :, :, 3].T.astype(np.float64).copy()
        proj["lvl_color"] = lvn[v, :, :, 0:3].transpose(1, 0, 2).astype(np.float64).copy()
        ref = oracle.composite(proj, cam.width, cam.height, qbound=sc.qbound,
                               pix_lo=pl[v].ravel(), pix_w=pw[v].ravel().astype(np.float64),
                               levels=True)
        err, namb = check_envelope(imgs[v], ref)
        say(f"eye {v}: max err {err:.3g}, ambiguous {namb}, blended {(pw[v] > 0).mean():.3f}")
    # the per-level values follow the oracle's projection of the level versions
    ref_p = oracle.project(sc, cams[0], levels=True)
    vis = ref_p["visible"] > 0
    np.testing.assert_allclose(lvn[0, vis, :, 3], ref_p["lvl_opacity"].T[vis], atol=2e-6)
    np.testing.assert_allclose(lvn[0, vis, :, 0:3], ref_p["lvl_color"].transpose(1, 0, 2)[vis], atol=2e-5)


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_render_fwd_one_call_equals_stages(tile):
    """The plain one-call render (its projection counts each entry's tiles and
    the binning compacts what it wrote) gives exactly the splats, keys, tile
    ranges, image, final T and contributor counts of gs_project +
    gs_bin_sort + gs_rasterize_fwd, over views of mixed sizes."""
    g = gs()
    sc = scene_small(seed=57, n=4000)
    cams = two_views() + [scenegen.pinhole(213, 121, 60.0, t=(0.0, 0.05, 1.8))]
    say(f"render_fwd one call, tile {tile}")
    C, splats, bs, out = _raster_case(g, sc, cams, tile, dominated=False)
    S = g.SceneTensors(sc)
    one = g.gs_render_fwd(S, C, tile, key_capacity=int(bs["num_keys"].item()) + 5)
    torch.cuda.synchronize()
    nk = int(bs["num_keys"].item())
    assert int(one["num_keys"].item()) == nk
    assert torch.equal(one["splats"], splats)
    assert torch.equal(one["vals"][:nk], bs["vals"][:nk])
    assert torch.equal(one["ranges"], bs["ranges"])
    for k in ("image", "final_T", "n_contrib"):
        assert torch.equal(one[k], out[k]), k


@pytest.mark.parametrize("n", [700_000, 1_400_000, 2_700_000])
def test_render_fwd_one_call_compaction_block_sizes(n):
    """Entry counts on each side of the compaction's block-size thresholds
    (4096, 8192 and 16384 entries per block): the one-call keys, ranges and
    image equal those of the counting pass (blocks of 4096)."""
    g = gs()
    sc = scene_small(seed=59, n=n, deg=0)
    cams = [scenegen.pinhole(320, 240, 60.0, t=(0.0, 0.0, 4.0))]
    say(f"render_fwd one call, {n} entries")
    C, splats, bs, out = _raster_case(g, sc, cams, 16, dominated=False)
    one = g.gs_render_fwd(g.SceneTensors(sc), C, 16, key_capacity=int(bs["num_keys"].item()) + 5)
    torch.cuda.synchronize()
    nk = int(bs["num_keys"].item())
    assert int(one["num_keys"].item()) == nk
    assert torch.equal(one["vals"][:nk], bs["vals"][:nk])
    assert torch.equal(one["ranges"], bs["ranges"])
    assert torch.equal(one["image"], out["image"])


@pytest.mark.parametrize("tile,eyes", [(16, 2), (8, 3), (32, 3)])
def test_render_foveated_one_call_equals_stages(tile, eyes):
    """The one-call render (its projection counts each entry's kept tiles and
    the binning compacts what it wrote) gives the image and key count of the
    separate stages (counting pass over the splat records)."""
    g = gs()
    sc = scene_small(seed=52, n=3000, fr=4)
    cams = [scenegen.pinhole(300, 170, scenegen.FR_FOV_DEG, t=(0.03, 0.0, 2.0)),
            scenegen.pinhole(300, 170, scenegen.FR_FOV_DEG, t=(-0.03, 0.0, 2.0)),
            scenegen.pinhole(213, 121, scenegen.FR_FOV_DEG, t=(0.0, 0.05, 1.8))][:eyes]
    fov = [scenegen.Fovea(150.0, 90.0), scenegen.Fovea(150.0, 90.0), scenegen.Fovea(60.0, 100.0)][:eyes]
    say(f"render_foveated one call, tile {tile}, {eyes} eyes")
    C, S, t, splats, lvl, bs, img = _fr_case(g, sc, cams, fov, tile)
    img2, num, _ = g.gs_render_foveated(S, C, fov, tile, key_capacity=int(bs["num_keys"].item()) + 7)
    torch.cuda.synchronize()
    assert int(num.item()) == int(bs["num_keys"].item())
    assert torch.equal(img, img2)


def test_concurrent_streams_give_the_sequential_frames():
    """Two stereo frames (different gazes) rendered at the same time on two
    streams, each with its own workspace and image, equal the same frames
    rendered one after the other: no entry point shares device state between
    calls (the frame pipelining of bench.py relies on this)."""
    g = gs()
    sc = scene_small(seed=61, n=6000, fr=4)
    cams = [scenegen.pinhole(320, 180, scenegen.FR_FOV_DEG, t=(0.03, 0.0, 2.0)),
            scenegen.pinhole(320, 180, scenegen.FR_FOV_DEG, t=(-0.03, 0.0, 2.0))]
    gazes = [[scenegen.Fovea(150.0, 90.0)] * 2, [scenegen.Fovea(60.0, 120.0)] * 2]
    say("two streams")
    C = g.Cameras(cams)
    S = g.SceneTensors(sc)
    cap = 400_000
    refs = []
    for fov in gazes:
        img, num, _ = g.gs_render_foveated(S, C, fov, 16, key_capacity=cap)
        torch.cuda.synchronize()
        assert 0 < int(num.item()) <= cap
        refs.append(img.clone())
    assert not torch.equal(refs[0], refs[1])
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    imgs = [torch.empty_like(refs[0]), torch.empty_like(refs[1])]
    wss = [None, None]
    for rep in range(3):
        cur = torch.cuda.current_stream()
        for k, st in enumerate(streams):
            st.wait_stream(cur)
            with torch.cuda.stream(st):
                _, _, wss[k] = g.gs_render_foveated(S, C, gazes[k], 16, key_capacity=cap, image=imgs[k],
                                                    workspace=wss[k])
        for st in streams:
            cur.wait_stream(st)
        torch.cuda.synchronize()
        assert torch.equal(imgs[0], refs[0]) and torch.equal(imgs[1], refs[1]), rep
        imgs[0].fill_(float("nan"))
        imgs[1].fill_(float("nan"))
        torch.cuda.synchronize()


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_backward_stagewise_matches_oracle(tile):
    g = gs()
    sc = scene_small(seed=61, n=1500)
    cams = two_views()
    bg = (0.2, 0.1, 0.3)
    say(f"backward stage-wise tile {tile}")
    C, splats, bs, out = _raster_case(g, sc, cams, tile, bg, dominated=False)
    sizes = [(c.width, c.height) for c in cams]
    rng = np.random.default_rng(0)
    dimg = rng.uniform(-1.0, 1.0, out["image"].shape[0]).astype(np.float32)
    dimg_t = torch.from_numpy(dimg).cuda()
    grads = g.gs_rasterize_bwd(splats, sc.n, C, tile, bs["vals"], bs["ranges"], out["final_T"],
                               out["n_contrib"], dimg_t, bg)
    S = g.SceneTensors(sc)
    pg = g.gs_project_bwd(S, C, splats, grads)
    torch.cuda.synchronize()
    sp = splat_np(splats)
    gn = grads.cpu().numpy()
    off = 0
    acc = None
    for v, cam in enumerate(cams):
        W, H = cam.width, cam.height
        gv = dimg[off:off + 3 * W * H].reshape(3, H, W)
        off += 3 * W * H
        ref = oracle.composite_bwd(oracle.splats_to_proj(view_slice(sp, v)), W, H, gv, bg)
        for name, sl in (("mean2d", slice(0, 2)), ("conic", slice(2, 5)), ("opacity", slice(5, 6)),
                         ("color", slice(6, 9))):
            r = rel_l2(gn[v][:, sl], ref[name].reshape(sc.n, -1))
            # point by point as well: at most 0.2 % of the points may differ
            # by more than 1e-3 of their own norm + 1e-4 of the rms norm (a
            # pair at a cut-off flips between float32 and float64 and moves
            # its point by a whole contribution)
            nbad, worst = per_point_check(gn[v][:, sl], ref[name].reshape(sc.n, -1))
            say(f"view {v} {name}: rel L2 {r:.2e}, points over the per-point bar {nbad}, worst {worst:.2e}")
            assert r < 1e-3, (v, name, r)
            assert nbad <= 0.002 * sc.n, (v, name, nbad)
        # projection reverse fed with the same (GPU) splat gradients
        gsplat = dict(mean2d=gn[v][:, 0:2].astype(np.float64), conic=gn[v][:, 2:5].astype(np.float64),
                      opacity=gn[v][:, 5].astype(np.float64), color=gn[v][:, 6:9].astype(np.float64))
        acc = oracle.project_bwd(sc, cam, gsplat, acc)
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        r = rel_l2(pg[name].cpu().numpy(), acc[name])
        nbad, worst = per_point_check(pg[name].cpu().numpy(), acc[name])
        say(f"project_bwd {name}: rel L2 {r:.2e}, points over the per-point bar {nbad}, worst {worst:.2e}")
        assert r < 1e-4, (name, r)
        assert nbad == 0, (name, nbad)


def test_autograd_matches_oracle_reverse_fd_subcase():
    g = gs()
    wl = scenegen.fd_subcase()
    sc, cam = wl.scene, wl.cams[0]
    say("autograd fd subcase")
    C = g.Cameras([cam])
    S = g.SceneTensors(sc)
    params = {k: S.t[k].clone().requires_grad_(True)
              for k in ("means", "log_scales", "quats", "opacity_logits", "sh")}
    img = g.render(params["means"], params["log_scales"], params["quats"], params["opacity_logits"],
                   params["sh"], C, sc.sh_degree)
    rng = np.random.default_rng(3)
    target = torch.from_numpy(rng.uniform(0, 1, img.shape[0]).astype(np.float32)).cuda()
    loss = (img - target).abs().mean()
    loss.backward()
    torch.cuda.synchronize()
    # L1 gradient sign(I - I*) / (3 H W) with the GPU image deciding the sign
    gimg = (torch.sign(img.detach() - target) / img.shape[0]).cpu().numpy().reshape(3, 32, 32)
    ref = oracle.reverse(sc, [cam], [gimg])
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        r = rel_l2(params[name].grad.cpu().numpy(), ref[name])
        nbad, worst = per_point_check(params[name].grad.cpu().numpy(), ref[name])
        say(f"autograd {name}: rel L2 {r:.2e}, points over the per-point bar {nbad}, worst {worst:.2e}")
        assert r < 1e-3, (name, r)
        assert nbad <= 0.002 * sc.n, (name, nbad)


def test_empty_and_culled_scenes_give_background():
    g = gs()
    cams = [scenegen.pinhole(70, 50, 60.0, t=(0.0, 0.0, 4.0))]
    bg = (0.3, 0.6, 0.9)
    say("empty / culled")
    C = g.Cameras(cams)
    for n, z in ((0, 0.0), (50, -10.0)):
        sc = scene_small(seed=70, n=max(n, 1), deg=0)
        if n == 0:
            sc = sc.subset(np.arange(0))
        else:
            sc.means[:, 2] = z  # behind the camera
        S = g.SceneTensors(sc)
        splats = g.gs_project(S, C, 16)
        bs = g.gs_bin_sort(splats, sc.n, C, 16, key_capacity=16)
        out = g.gs_rasterize_fwd(splats, sc.n, C, 16, bs["vals"], bs["ranges"], bg)
        torch.cuda.synchronize()
        assert int(bs["num_keys"].item()) == 0
        img = image_views(out["image"], [(70, 50)])[0]
        np.testing.assert_array_equal(img, np.broadcast_to(np.float32(bg), img.shape))
        assert torch.all(out["final_T"] == 1) and torch.all(out["n_contrib"] == 0)


def test_capacity_overflow_reports_required_count():
    g = gs()
    sc = scene_small(seed=71, n=2000)
    cams = [scenegen.pinhole(160, 120, 60.0, t=(0.0, 0.0, 4.0))]
    say("capacity overflow")
    C = g.Cameras(cams)
    S = g.SceneTensors(sc)
    splats = g.gs_project(S, C, 16)
    need = int(splat_np(splats)["tiles_touched"].sum())
    bs = g.gs_bin_sort(splats, sc.n, C, 16, key_capacity=need // 2)
    out = g.gs_rasterize_fwd(splats, sc.n, C, 16, bs["vals"], bs["ranges"])
    torch.cuda.synchronize()
    assert int(bs["num_keys"].item()) == need
    # truncated lists are never read: every tile is empty
    assert int(bs["ranges"].abs().sum().item()) == 0
    assert torch.all(out["final_T"] == 1)
