"""Reverse of the foveated render on the GPU (through the C ABI) against the
oracle: stage-wise (compositing reverse per level, given the GPU's splats
and level tables) and end to end (parameters, against the oracle's
weighted sum of level-scene reverses).  Bar: 1e-3 relative L2, as for the
plain reverse (decisions near a threshold may differ between float32 and
float64)."""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from gpu_util import need_gpu, per_point_check, pixel_views, rel_l2, say, splat_np, view_slice

pytestmark = pytest.mark.gpu


def gs():
    need_gpu()
    import paper_2407_00435_amd as g
    return g


def case(seed=91, n=2500):
    sc = scenegen.small_scene(n, seed=seed, sh_degree=3, fr_levels=4, log_scale_mu=-3.2, log_scale_sigma=0.5)
    cams = [scenegen.pinhole(150, 96, scenegen.FR_FOV_DEG, t=(0.03, 0.0, 2.2)),
            scenegen.pinhole(150, 96, scenegen.FR_FOV_DEG, t=(-0.03, 0.0, 2.2))]
    fov = [scenegen.Fovea(70.0, 45.0, rings_deg=(12.0, 22.0, 32.0), band_deg=4.0),
           scenegen.Fovea(80.0, 50.0, rings_deg=(12.0, 22.0, 32.0), band_deg=4.0)]
    return sc, cams, fov


def forward(g, sc, cams, fov, tile=16):
    C, S = g.Cameras(cams), g.SceneTensors(sc)
    t = g.gs_fovea_prep(C, fov, tile, 4)
    splats, lvl = g.gs_project(S, C, tile, levels=True)
    bs = g.gs_bin_sort(splats, sc.n, C, tile, tile_level=t["tile_level"], qbound=S.t["qbound"])
    _, n_px = C.tiles(tile)
    fT2 = torch.empty((n_px, 2), dtype=torch.float32, device="cuda")
    nc2 = torch.empty((n_px, 2), dtype=torch.int32, device="cuda")
    img = g.gs_rasterize_foveated(splats, lvl, sc.n, S.t["qbound"], 4, C, tile, bs["vals"], bs["ranges"],
                                  t["pix_level"], t["pix_weight"], keep=(fT2, nc2))
    grid = g.gs_rasterize_foveated(splats, lvl, sc.n, S.t["qbound"], 4, C, tile, bs["vals"], bs["ranges"],
                                   t["pix_level"], t["pix_weight"])
    torch.cuda.synchronize()
    assert torch.equal(img, grid)  # keeping the reverse state does not change the image
    return C, S, t, splats, lvl, bs, img, fT2, nc2


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_fr_reverse_stagewise_matches_oracle(tile):
    g = gs()
    sc, cams, fov = case()
    say("fr reverse stage-wise", tile)
    C, S, t, splats, lvl, bs, img, fT2, nc2 = forward(g, sc, cams, fov, tile)
    rng = np.random.default_rng(3)
    dimg = torch.from_numpy(rng.uniform(-1, 1, img.shape[0]).astype(np.float32)).cuda()
    grads, lgr = g.gs_rasterize_foveated_bwd(splats, lvl, sc.n, S.t["qbound"], 4, C, tile, bs["vals"],
                                             bs["ranges"], t["pix_level"], t["pix_weight"], fT2, nc2, dimg)
    torch.cuda.synchronize()
    sp = splat_np(splats)
    lvn = lvl.cpu().numpy().astype(np.float64)
    gn = grads.cpu().numpy().astype(np.float64)
    lgn = lgr.cpu().numpy().astype(np.float64)
    sizes = [(c.width, c.height) for c in cams]
    pl = pixel_views(t["pix_level"], sizes)
    pw = pixel_views(t["pix_weight"], sizes)
    dn = dimg.cpu().numpy().astype(np.float64)
    off = 0
    for v, cam in enumerate(cams):
        W, H = cam.width, cam.height
        dv = dn[3 * off:3 * (off + W * H)].reshape(3, H, W)
        geo_m = np.zeros((sc.n, 2))
        geo_c = np.zeros((sc.n, 3))
        for lev in range(1, 5):
            proj = oracle.splats_to_proj(view_slice(sp, v))
            proj["opacity"] = lvn[v, :, lev - 1, 3].copy()
            proj["color"] = lvn[v, :, lev - 1, 0:3].copy()
            proj["radius"] = np.where(sc.qbound >= lev, proj["radius"], 0).astype(np.int32)
            wt = oracle.level_weights(pl[v].ravel(), pw[v].ravel().astype(np.float64), lev).reshape(H, W)
            ref = oracle.composite_bwd(proj, W, H, dv * wt[None])
            geo_m += ref["mean2d"]
            geo_c += ref["conic"]
            e_op = rel_l2(lgn[v, :, lev - 1, 3], ref["opacity"])
            e_col = rel_l2(lgn[v, :, lev - 1, 0:3], ref["color"])
            say(f"eye {v} level {lev}: opacity {e_op:.2e} colour {e_col:.2e}")
            if np.abs(ref["opacity"]).sum() > 0:
                assert e_op < 1e-3 and e_col < 1e-3
        assert rel_l2(gn[v, :, 0:2], geo_m) < 1e-3
        assert rel_l2(gn[v, :, 2:5], geo_c) < 1e-3
        assert np.all(gn[v, :, 5:9] == 0)
        off += W * H


def test_fr_reverse_parameters_match_oracle():
    g = gs()
    sc, cams, fov = case(seed=92, n=1500)
    C, S, t, splats, lvl, bs, img, fT2, nc2 = forward(g, sc, cams, fov)
    rng = np.random.default_rng(4)
    dimg = torch.from_numpy(rng.uniform(-1, 1, img.shape[0]).astype(np.float32)).cuda()
    grads, lgr = g.gs_rasterize_foveated_bwd(splats, lvl, sc.n, S.t["qbound"], 4, C, 16, bs["vals"], bs["ranges"],
                                             t["pix_level"], t["pix_weight"], fT2, nc2, dimg)
    pg = g.gs_project_bwd_levels(S, C, splats, grads, lgr)
    torch.cuda.synchronize()
    sizes = [(c.width, c.height) for c in cams]
    pl = pixel_views(t["pix_level"], sizes)
    pw = pixel_views(t["pix_weight"], sizes)
    dn = dimg.cpu().numpy().astype(np.float64)
    dls, tabs, off = [], [], 0
    for v, cam in enumerate(cams):
        W, H = cam.width, cam.height
        dls.append(dn[3 * off:3 * (off + W * H)].reshape(3, H, W))
        tabs.append((pl[v].ravel(), pw[v].ravel().astype(np.float64)))
        off += W * H
    sc64 = scenegen.Scene(*(np.asarray(getattr(sc, k), np.float64) for k in ("means", "log_scales", "quats",
                                                                             "opacity_logits", "sh")),
                          sc.sh_degree, sc.qbound, np.asarray(sc.lvl_opacity_logits, np.float64),
                          np.asarray(sc.lvl_sh_dc, np.float64))
    ref = oracle.fr_reverse(sc64, cams, tabs, dls)
    for k in ("means", "log_scales", "quats", "sh", "lvl_opacity_logits", "lvl_sh_dc"):
        gpu, r = pg[k].cpu().numpy().astype(np.float64), ref[k]
        e = rel_l2(gpu, r)
        if k.startswith("lvl_"):  # [L][n][...] -> points first
            gpu, r = np.moveaxis(gpu, 1, 0), np.moveaxis(r, 1, 0)
        # point by point: at most 0.2 % of the points beyond 1e-3 of their
        # own norm + 1e-4 of the rms norm (threshold flips between float32
        # and float64 move a point's gradient by a whole pair's contribution)
        nbad, worst = per_point_check(gpu, r)
        say(f"{k}: rel L2 {e:.2e}, points over the per-point bar {nbad}, worst {worst:.2e}")
        assert e < 1e-3, k
        assert nbad <= 0.002 * sc.n, (k, nbad)
    # base logit and DC are unused when every level has its own version
    assert float(pg["opacity_logits"].abs().max()) == 0.0
    assert float(pg["sh"][:, 0, :].abs().max()) == 0.0


def test_render_foveated_autograd():
    g = gs()
    sc, cams, fov = case(seed=93, n=1200)
    S = g.SceneTensors(sc)
    C = g.Cameras(cams)
    names = ("means", "log_scales", "quats", "opacity_logits", "sh", "lvl_opacity_logits", "lvl_sh_dc")
    params = [S.t[k].clone().requires_grad_(True) for k in names]
    img = g.render_foveated(*params, S.t["qbound"], C, fov, sc.sh_degree, 16)
    rng = np.random.default_rng(5)
    w = torch.from_numpy(rng.uniform(-1, 1, img.shape[0]).astype(np.float32)).cuda()
    (img * w).sum().backward()
    torch.cuda.synchronize()
    # the same chain called stage by stage
    C2, S2, t, splats, lvl, bs, img2, fT2, nc2 = forward(g, sc, cams, fov)
    assert torch.equal(img.detach(), img2)
    grads, lgr = g.gs_rasterize_foveated_bwd(splats, lvl, sc.n, S2.t["qbound"], 4, C2, 16, bs["vals"], bs["ranges"],
                                             t["pix_level"], t["pix_weight"], fT2, nc2, w)
    pg = g.gs_project_bwd_levels(S2, C2, splats, grads, lgr)
    torch.cuda.synchronize()
    for p, k in zip(params, names):
        assert rel_l2(p.grad.cpu().numpy(), pg[k].cpu().numpy()) < 1e-5, k
