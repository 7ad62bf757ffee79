"""HVSQ (Section 2.2, Eq. 2) on the GPU against the oracle, through the C ABI.

The setting is the paper's (Section 4.3): the reference image is the full
render of the scene, the altered image the foveated render of the same eye,
the regions are the quality rings.  Pooling radii: equal to the oracle's
except where rho * eccentricity lies within 1e-4 of an integer (the float32
eccentricity may round across it).  Given the same radii: per-region pixel
counts exact; per-pixel terms and per-region sums within 1e-9 relative (the
tables are double-double, the oracle sums every window directly); the
gradient (float32) within 1e-6 of the largest component plus 1e-6 relative.
"""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from gpu_util import need_gpu, pixel_views, say

pytestmark = pytest.mark.gpu


def gs():
    need_gpu()
    import paper_2407_00435_amd as g
    return g


def eyes_case(W=240, H=135, n=4000, seed=95):
    sc = scenegen.small_scene(n, seed=seed, sh_degree=3, fr_levels=4, log_scale_mu=-3.2, log_scale_sigma=0.5)
    cams = [scenegen.pinhole(W, H, scenegen.FR_FOV_DEG, t=(0.03, 0.0, 2.2)),
            scenegen.pinhole(W - 30, H + 10, scenegen.FR_FOV_DEG, t=(-0.03, 0.0, 2.2))]
    fov = [scenegen.Fovea(0.4 * W, 0.45 * H, rings_deg=(12.0, 22.0, 32.0), band_deg=3.0),
           scenegen.Fovea(0.6 * W, 0.5 * H, rings_deg=(12.0, 22.0, 32.0), band_deg=3.0)]
    return sc, cams, fov


def images(g, sc, cams, fov):
    """(altered = foveated render, reference = full render, region map)."""
    S, C = g.SceneTensors(sc), g.Cameras(cams)
    alt, _, _ = g.gs_render_foveated(S, C, fov, 16, key_capacity=3_000_000, check=True)
    ref = g.gs_render_fwd(S, C, 16, key_capacity=3_000_000, check=True)["image"]
    region = g.gs_fovea_prep(C, fov, 16, 4)["pix_level"]
    return C, alt, ref, region


def test_pooling_radius_matches_oracle():
    g = gs()
    sc, cams, fov = eyes_case()
    say("hvsq pooling radius")
    C = g.Cameras(cams)
    rad = g.gs_hvsq_pooling(C, fov, 0.37).cpu().numpy()
    off = 0
    for v, cam in enumerate(cams):
        n = cam.width * cam.height
        ref, amb = oracle.hvsq_radius(cam, fov[v], 0.37)
        ok = amb == 0
        np.testing.assert_array_equal(rad[off:off + n][ok], ref[ok])
        assert amb.mean() < 1e-2
        off += n


@pytest.mark.parametrize("grad_region", [0, 2])
def test_hvsq_matches_oracle(grad_region):
    g = gs()
    sc, cams, fov = eyes_case()
    say("hvsq against the oracle, gradient of region", grad_region)
    C, alt, ref, region = images(g, sc, cams, fov)
    rad = g.gs_hvsq_pooling(C, fov, 0.37)
    out = g.gs_hvsq(alt, ref, C, rad, region=region, n_regions=4, grad_region=grad_region, want_terms=True)
    torch.cuda.synchronize()
    sizes = [(c.width, c.height) for c in cams]
    a_n, r_n = alt.cpu().numpy(), ref.cpu().numpy()
    rad_n, reg_n = rad.cpu().numpy(), region.cpu().numpy()
    terms = out["terms"].cpu().numpy()
    grad = out["grad"].cpu().numpy()
    off = 0
    for v, (W, H) in enumerate(sizes):
        n = W * H
        sl, sl3 = slice(off, off + n), slice(3 * off, 3 * (off + n))
        o = oracle.hvsq(a_n[sl3], r_n[sl3], rad_n[sl], W, H, region=reg_n[sl], n_regions=4,
                        grad_region=grad_region, want_terms=True)
        np.testing.assert_array_equal(out["counts"][v].cpu().numpy(), o["counts"])
        np.testing.assert_allclose(terms[sl], o["terms"], rtol=1e-9, atol=1e-13)
        np.testing.assert_allclose(out["sums"][v].cpu().numpy(), o["sums"], rtol=1e-9, atol=1e-12)
        gref = o["grad"].reshape(-1)
        scale = float(np.abs(gref).max())
        assert scale > 0
        err = np.abs(grad[sl3] - gref)
        say(f"view {v}: hvsq per region {np.round(o['hvsq'], 6).tolist()}, gradient max err / scale "
            f"{float(err.max()) / scale:.2e}")
        assert np.all(err <= 1e-6 * scale + 1e-6 * np.abs(gref))
        off += n


def test_identical_images_give_zero():
    g = gs()
    sc, cams, fov = eyes_case(W=96, H=64)
    C, alt, ref, region = images(g, sc, cams, fov)
    rad = g.gs_hvsq_pooling(C, fov, 0.5)
    out = g.gs_hvsq(ref, ref, C, rad, region=region, n_regions=4, grad_region=0)
    torch.cuda.synchronize()
    assert float(out["sums"].abs().max()) == 0.0
    assert float(out["grad"].abs().max()) == 0.0


def test_hvsq_stereo_1080p_sampled():
    """The bench's stereo eyes at 1920x1080 (1.5M Gaussians): per-region counts
    against the ring map, and per-pixel terms at sampled pixels (windows up
    to about 190 pixels half-width at the periphery) against the oracle."""
    g = gs()
    from bench import Foveated
    say("hvsq stereo 1080p")
    wl = scenegen.config3()
    fr = Foveated(g, wl, 16)
    for s in fr.STAGES:
        getattr(fr, s)()
    ref = g.gs_render_fwd(fr.S, fr.C, 16, key_capacity=fr.cap, check=True)["image"]
    rho = 0.25 * float(wl.cams[0].fx) * np.pi / 180.0  # half of a pooling diameter of 0.5 x eccentricity
    rad = g.gs_hvsq_pooling(fr.C, wl.foveae, rho)
    out = g.gs_hvsq(fr.image, ref, fr.C, rad, region=fr.pix_level, n_regions=4, grad_region=0, want_terms=True)
    torch.cuda.synchronize()
    sizes = [(c.width, c.height) for c in wl.cams]
    lv = pixel_views(fr.pix_level, sizes)
    rng = np.random.default_rng(8)
    a_n, r_n, rad_n = fr.image.cpu().numpy(), ref.cpu().numpy(), rad.cpu().numpy()
    terms = out["terms"].cpu().numpy()
    off = 0
    for v, (W, H) in enumerate(sizes):
        n = W * H
        counts = out["counts"][v].cpu().numpy()
        np.testing.assert_array_equal(counts[:4], np.bincount(lv[v].ravel(), minlength=5)[1:])
        assert counts[4] == n
        pix = np.stack([rng.integers(0, W, 600), rng.integers(0, H, 600)], 1).astype(np.int32)
        o = oracle.hvsq_at(a_n[3 * off:3 * (off + n)], r_n[3 * off:3 * (off + n)], rad_n[off:off + n], W, H, pix)
        gpu = terms[off:off + n][pix[:, 1] * W + pix[:, 0]]
        np.testing.assert_allclose(gpu, o, rtol=1e-9, atol=1e-13)
        say(f"eye {v}: hvsq per ring {np.round(out['hvsq'][v].cpu().numpy(), 7).tolist()}, max radius "
            f"{int(rad_n[off:off + n].max())}")
        off += n
    assert torch.isfinite(out["grad"]).all()
