"""Degenerate shapes through the C ABI, against the oracle.

- Views smaller than a tile (1 x 1, one row, one column, 5 x 3) beside a
  17 x 17 view, in one call: binning bit-exact against the oracle's float32
  binning, images within its envelope, the compositing reverse within
  1e-3 relative L2 per view (views where nothing contributes: exactly zero).
- One Gaussian covering every tile of two views (its rectangle spans many
  super-tiles): every tile holds its key, image within the envelope.
- The foveated path on the tiny views (the gaze inside each), binning
  bit-exact with the level filter, images within the envelope; and an empty
  foveated scene renders the background.
- Points that are all behind the cameras: both one-call renders give no
  keys and the background.
"""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from gpu_util import check_envelope, image_views, need_gpu, pixel_views, rel_l2, say, splat_np, view_slice

pytestmark = pytest.mark.gpu

TINY = [(1, 1), (1, 37), (23, 1), (5, 3), (17, 17)]


def gs():
    need_gpu()
    import paper_2407_00435_amd as g
    return g


def tiny_cams():
    return [scenegen.pinhole(w, h, 60.0, t=(0.02 * k, -0.01 * k, 3.0)) for k, (w, h) in enumerate(TINY)]


def scene(seed, n=1200, fr=0):
    return scenegen.small_scene(n, seed=seed, sh_degree=3, fr_levels=fr, log_scale_mu=-2.8, log_scale_sigma=0.5)


@pytest.mark.parametrize("tile", [8, 16])
def test_tiny_views_forward_and_reverse(tile):
    g = gs()
    sc = scene(91)
    cams = tiny_cams()
    bg = (0.2, 0.4, 0.6)
    say("tiny views", tile)
    C, S = g.Cameras(cams), g.SceneTensors(sc)
    splats = g.gs_project(S, C, tile)
    bs = g.gs_bin_sort(splats, sc.n, C, tile, want_keys=True, want_hits=True, check=True)
    out = g.gs_rasterize_fwd(splats, sc.n, C, tile, bs["vals"], bs["ranges"], bg)
    rng = np.random.default_rng(4)
    dimg = rng.uniform(-1.0, 1.0, out["image"].shape[0]).astype(np.float32)
    grads = g.gs_rasterize_bwd(splats, sc.n, C, tile, bs["vals"], bs["ranges"], out["final_T"], out["n_contrib"],
                               torch.from_numpy(dimg).cuda(), bg)
    torch.cuda.synchronize()
    sp = splat_np(splats)
    ref_b = oracle.bin_f32(sp["mean2d"], sp["radius"], sp["depth"], [c.width for c in cams],
                           [c.height for c in cams], tile)
    nk = int(bs["num_keys"].item())
    assert nk == ref_b["num_keys"] and nk > 0
    np.testing.assert_array_equal(bs["keys"].cpu().numpy()[:nk].view(np.uint64), ref_b["keys"])
    np.testing.assert_array_equal(bs["vals"].cpu().numpy()[:nk].view(np.uint32), ref_b["vals"])
    np.testing.assert_array_equal(bs["ranges"].cpu().numpy().view(np.uint32), ref_b["ranges"])
    np.testing.assert_array_equal(bs["hits"].cpu().numpy().view(np.uint32), ref_b["hits"])
    imgs = image_views(out["image"], TINY)
    gn = grads.cpu().numpy()
    off = 0
    for v, cam in enumerate(cams):
        W, H = cam.width, cam.height
        proj = oracle.splats_to_proj(view_slice(sp, v))
        err, namb = check_envelope(imgs[v], oracle.composite(proj, W, H, bg))
        ref = oracle.composite_bwd(proj, W, H, dimg[off:off + 3 * W * H].reshape(3, H, W), bg)
        off += 3 * W * H
        for name, sl in (("mean2d", slice(0, 2)), ("conic", slice(2, 5)), ("opacity", slice(5, 6)),
                         ("color", slice(6, 9))):
            r_ = ref[name].reshape(sc.n, -1)
            if not np.any(r_):
                assert not np.any(gn[v][:, sl]), (v, name)
                continue
            r = rel_l2(gn[v][:, sl], r_)
            assert r < 1e-3, (v, name, r)
        say(f"view {W}x{H}: max err {err:.3g}, ambiguous {namb}")


def test_one_gaussian_covering_every_tile():
    g = gs()
    sc = scenegen.Scene(np.array([[0.05, -0.03, 0.0]], np.float32), np.array([[-0.2, -0.4, -0.3]], np.float32),
                        np.array([[0.9, 0.2, -0.1, 0.3]], np.float32), np.array([1.5], np.float32),
                        np.random.default_rng(2).normal(0.0, 0.3, (1, 16, 3)).astype(np.float32) + 0.5, 3)
    cams = [scenegen.pinhole(300, 200, 60.0, t=(0.0, 0.0, 1.2)), scenegen.pinhole(130, 257, 50.0, t=(0.0, 0.0, 1.4))]
    say("one Gaussian over every tile")
    C, S = g.Cameras(cams), g.SceneTensors(sc)
    splats = g.gs_project(S, C, 16)
    bs = g.gs_bin_sort(splats, sc.n, C, 16, want_keys=True, check=True)
    out = g.gs_rasterize_fwd(splats, sc.n, C, 16, bs["vals"], bs["ranges"])
    torch.cuda.synchronize()
    n_tiles, _ = C.tiles(16)
    assert int(bs["num_keys"].item()) == n_tiles
    r = bs["ranges"].cpu().numpy().astype(np.int64)
    assert np.all(r[:, 1] - r[:, 0] == 1)
    sp = splat_np(splats)
    imgs = image_views(out["image"], [(c.width, c.height) for c in cams])
    for v, cam in enumerate(cams):
        err, namb = check_envelope(imgs[v], oracle.composite(oracle.splats_to_proj(view_slice(sp, v)), cam.width,
                                                             cam.height))
        say(f"view {v}: max err {err:.3g}, ambiguous {namb}")


def test_foveated_tiny_views_and_empty_scene():
    g = gs()
    sc = scene(93, fr=4)
    cams = [scenegen.pinhole(w, h, scenegen.FR_FOV_DEG, t=(0.02 * k, 0.0, 2.5)) for k, (w, h) in enumerate(TINY)]
    fov = [scenegen.Fovea(0.5 * (w - 1), 0.5 * (h - 1)) for w, h in TINY]
    say("foveated tiny views")
    C, S = g.Cameras(cams), g.SceneTensors(sc)
    t = g.gs_fovea_prep(C, fov, 16, 4)
    splats, lvl = g.gs_project(S, C, 16, levels=True)
    bs = g.gs_bin_sort(splats, sc.n, C, 16, tile_level=t["tile_level"], qbound=S.t["qbound"], want_keys=True,
                       want_hits=True, check=True)
    img = g.gs_rasterize_foveated(splats, lvl, sc.n, S.t["qbound"], 4, C, 16, bs["vals"], bs["ranges"],
                                  t["pix_level"], t["pix_weight"])
    one, _, _ = g.gs_render_foveated(S, C, fov, 16, key_capacity=bs["capacity"])
    torch.cuda.synchronize()
    assert torch.equal(one, img)
    sp = splat_np(splats)
    ref_b = oracle.bin_f32(sp["mean2d"], sp["radius"], sp["depth"], [c.width for c in cams],
                           [c.height for c in cams], 16, tile_level_lo=t["tile_level"][:, 0].cpu().numpy(),
                           qbound=sc.qbound)
    nk = int(bs["num_keys"].item())
    assert nk == ref_b["num_keys"]
    np.testing.assert_array_equal(bs["vals"].cpu().numpy()[:nk].view(np.uint32), ref_b["vals"])
    np.testing.assert_array_equal(bs["ranges"].cpu().numpy().view(np.uint32), ref_b["ranges"])
    np.testing.assert_array_equal(bs["hits"].cpu().numpy().view(np.uint32), ref_b["hits"])
    lvn = lvl.cpu().numpy()
    imgs = image_views(img, TINY)
    pl, pw = pixel_views(t["pix_level"], TINY), pixel_views(t["pix_weight"], TINY)
    for v, cam in enumerate(cams):
        proj = oracle.splats_to_proj(view_slice(sp, v))
        proj["lvl_opacity"] = lvn[v, :, :, 3].T.astype(np.float64).copy()
        proj["lvl_color"] = lvn[v, :, :, 0:3].transpose(1, 0, 2).astype(np.float64).copy()
        ref = oracle.composite(proj, cam.width, cam.height, qbound=sc.qbound, pix_lo=pl[v].ravel(),
                               pix_w=pw[v].ravel().astype(np.float64), levels=True)
        check_envelope(imgs[v], ref)
    # an empty foveated scene: the background everywhere, no keys
    say("foveated empty scene")
    bg = (0.3, 0.5, 0.7)
    E = g.SceneTensors(sc.subset(np.arange(0)))
    img0, num0, _ = g.gs_render_foveated(E, C, fov, 16, bg=bg, key_capacity=16)
    torch.cuda.synchronize()
    assert int(num0.item()) == 0
    for im in image_views(img0, TINY):
        np.testing.assert_array_equal(im, np.broadcast_to(np.float32(bg), im.shape))


def test_one_call_renders_with_every_point_behind_the_camera():
    """Points exist but none is in front of any camera: the one-call renders
    (whose projection writes every entry's key word as 'no keys') give zero
    keys and the background, as the stage calls do."""
    g = gs()
    sc = scene(97, fr=4)
    cams = [scenegen.pinhole(40, 30, 60.0, t=(0.0, 0.0, -10.0)), scenegen.pinhole(33, 17, 60.0, t=(0.1, 0.0, -12.0))]
    C, S = g.Cameras(cams), g.SceneTensors(sc)
    bg = (0.2, 0.4, 0.6)
    say("every point behind the camera")
    plain = g.gs_render_fwd(S, C, 16, bg=bg, key_capacity=64)
    fov = [scenegen.Fovea(20.0, 15.0), scenegen.Fovea(16.0, 8.0)]
    img, num, _ = g.gs_render_foveated(S, C, fov, 16, bg=bg, key_capacity=64)
    torch.cuda.synchronize()
    assert int(plain["num_keys"].item()) == 0 and int(num.item()) == 0
    sizes = [(c.width, c.height) for c in cams]
    for im in image_views(plain["image"], sizes):
        np.testing.assert_array_equal(im, np.broadcast_to(np.float32(bg), im.shape))
    # band pixels blend two background values, (1 - w) bg + w bg: within an ulp of bg
    for im in image_views(img, sizes):
        np.testing.assert_allclose(im, np.broadcast_to(np.float32(bg), im.shape), rtol=0, atol=2e-7)
    assert torch.all(plain["final_T"] == 1.0) and torch.all(plain["n_contrib"] == 0)
