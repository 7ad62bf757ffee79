"""Pins for the oracle's foveated form (Section 4.1 regions and blending,
Section 4.2 nested subsets and multi-versioning, Section 6 ring layout).

- Ring starts at 0/18/27/33 degrees cover about 13/17/21/49 % of pixels
  (Section 6); with a centred gaze and a 94 degree horizontal field of view
  the reading gives 12.8/18.7/18.5/49.9 %.
- About a quarter of the pixels are blended (Section 4.1); the 3.5 degree
  band gives that.
- All quality bounds at the top level with no per-level versions reduces to
  the plain render; a single level reduces to a plain render of the subset
  {i : m_i >= t}.
- A point has no version above its quality bound (Section 4.2): its level
  opacity there is zero, elsewhere the logistic of its level logit.
"""
import math

import numpy as np

import scenegen


def centred_eye(w=1920, h=1080):
    cam = scenegen.pinhole(w, h, scenegen.FR_FOV_DEG, t=(0.0, 0.0, 2.0))
    return cam, scenegen.Fovea(cam.cx, cam.cy)


def test_ring_fractions_match_section6(oracle_lib):
    cam, fov = centred_eye()
    no_band = scenegen.Fovea(fov.gaze_x, fov.gaze_y, band_deg=0.0)
    f = oracle_lib.fovea(cam, no_band, 4, 16)
    frac = np.bincount(f["pix_lo"], minlength=5)[1:] / f["pix_lo"].size
    paper = np.array([0.13, 0.17, 0.21, 0.49])
    assert np.all(np.abs(frac - paper) <= 0.03), frac
    # eccentricity is an angle: the gaze pixel is 0 and the corner is the widest
    assert f["ecc"].min() < 0.05
    half_diag = np.degrees(np.arctan(np.hypot(959.5, 539.5) / cam.fx))
    assert abs(f["ecc"].max() - half_diag) < 1e-9


def test_blended_fraction_about_a_quarter(oracle_lib):
    cam, fov = centred_eye()
    f = oracle_lib.fovea(cam, fov, 4, 16)
    blended = (f["pix_w"] > 0).mean()
    assert 0.22 <= blended <= 0.28, blended
    assert np.all((f["pix_w"] >= 0) & (f["pix_w"] < 1))


def test_weights_are_a_linear_ramp_in_eccentricity(oracle_lib):
    cam, fov = centred_eye(640, 360)
    f = oracle_lib.fovea(cam, fov, 4, 16)
    ecc, lo, w = f["ecc"], f["pix_lo"], f["pix_w"]
    for j, b in enumerate(fov.rings_deg, start=1):
        band = (ecc > b - 1.75) & (ecc < b + 1.75)
        assert np.all(lo[band] == j)
        np.testing.assert_allclose(w[band], (ecc[band] - (b - 1.75)) / 3.5, rtol=1e-12)


def test_tile_level_range(oracle_lib):
    cam, fov = centred_eye(320, 180)
    T = 16
    f = oracle_lib.fovea(cam, fov, 4, T)
    lo = f["pix_lo"].reshape(180, 320)
    hi = lo + (f["pix_w"].reshape(180, 320) > 0)
    tx, ty = 20, 12
    for y in range(ty):
        for x in range(tx):
            blk = (slice(y * T, (y + 1) * T), slice(x * T, (x + 1) * T))
            assert f["tile_lo"][y * tx + x] == lo[blk].min()
            assert f["tile_hi"][y * tx + x] == hi[blk].max()


def _fr_scene(seed):
    sc = scenegen.small_scene(400, seed=seed, sh_degree=1, fr_levels=4, log_scale_mu=-2.6)
    cam = scenegen.pinhole(48, 32, scenegen.FR_FOV_DEG, t=(0.0, 0.0, 2.0))
    fov = scenegen.Fovea(20.0, 14.0, rings_deg=(10.0, 20.0, 30.0), band_deg=3.0)
    return sc, cam, fov


def test_all_top_level_reduces_to_plain(oracle_lib):
    sc, cam, fov = _fr_scene(21)
    sc.qbound[:] = 4
    sc.lvl_opacity_logits = None
    sc.lvl_sh_dc = None
    pr = oracle_lib.project(sc, cam, levels=True)
    f = oracle_lib.fovea(cam, fov, 4, 16)
    fr = oracle_lib.composite(pr, 48, 32, qbound=sc.qbound, pix_lo=f["pix_lo"], pix_w=f["pix_w"],
                              levels=True)
    plain = oracle_lib.composite(pr, 48, 32)
    np.testing.assert_allclose(fr["rgb"], plain["rgb"], rtol=1e-12, atol=1e-14)


def test_single_level_is_plain_render_of_subset(oracle_lib):
    sc, cam, _ = _fr_scene(22)
    pr = oracle_lib.project(sc, cam, levels=True)
    for t in (1, 2, 3, 4):
        lo = np.full(48 * 32, t, np.uint8)
        w = np.zeros(48 * 32)
        fr = oracle_lib.composite(pr, 48, 32, qbound=sc.qbound, pix_lo=lo, pix_w=w, levels=True)
        keep = np.nonzero(sc.qbound >= t)[0]
        sub = {k: pr[k][keep] for k in ("mean2d", "conic", "depth", "radius")}
        sub["opacity"] = pr["lvl_opacity"][t - 1][keep]
        sub["color"] = pr["lvl_color"][t - 1][keep]
        plain = oracle_lib.composite(sub, 48, 32)
        np.testing.assert_allclose(fr["rgb"], plain["rgb"], rtol=1e-12, atol=1e-14)


def test_level_opacity_is_zero_above_the_quality_bound(oracle_lib):
    sc, cam, _ = _fr_scene(24)
    pr = oracle_lib.project(sc, cam, levels=True)
    logits = np.asarray(sc.lvl_opacity_logits, np.float64)
    qb = np.asarray(sc.qbound).astype(np.int64)
    vis = pr["radius"] > 0
    assert vis.sum() > 50 and len(set(qb[vis].tolist())) >= 3
    for t in range(1, 5):
        want = np.where(qb >= t, 1.0 / (1.0 + np.exp(-logits[t - 1])), 0.0)
        np.testing.assert_allclose(pr["lvl_opacity"][t - 1][vis], want[vis], rtol=1e-13, atol=0.0)


def test_blend_is_weighted_sum_of_levels(oracle_lib):
    sc, cam, fov = _fr_scene(23)
    pr = oracle_lib.project(sc, cam, levels=True)
    f = oracle_lib.fovea(cam, fov, 4, 16)
    fr = oracle_lib.composite(pr, 48, 32, qbound=sc.qbound, pix_lo=f["pix_lo"], pix_w=f["pix_w"],
                              levels=True)
    per_level = []
    for t in (1, 2, 3, 4):
        lo = np.full(48 * 32, t, np.uint8)
        per_level.append(oracle_lib.composite(pr, 48, 32, qbound=sc.qbound, pix_lo=lo,
                                              pix_w=np.zeros(48 * 32), levels=True)["rgb"])
    lo = f["pix_lo"].reshape(32, 48)
    w = f["pix_w"].reshape(32, 48, 1)
    stack = np.stack(per_level)  # (4, H, W, 3)
    yy, xx = np.mgrid[:32, :48]
    a = stack[lo - 1, yy, xx]
    b = stack[np.minimum(lo, 3), yy, xx]
    np.testing.assert_allclose(fr["rgb"], (1 - w) * a + w * b, rtol=1e-12, atol=1e-14)
    assert (f["pix_w"] > 0).any()


def test_eccentricity_about_an_off_centre_gaze(oracle_lib):
    # rays through one image row (or one image column) lie in a plane
    # through the camera centre, so their angles add there.  On the gaze's
    # row, in the plane y_cam = b z_cam with b = (gy - cy)/f, the in-plane
    # distance to the axis is f sqrt(1 + b^2), so
    # ecc = |atan((x - cx)/(f sqrt(1 + b^2))) - atan((gx - cx)/(f sqrt(1 + b^2)))|;
    # on the gaze's column likewise with a = (gx - cx)/f.  On the principal
    # row (odd height puts it on a pixel row) b = 0.
    cam = scenegen.pinhole(321, 181, scenegen.FR_FOV_DEG, t=(0.0, 0.0, 2.0))
    gx, gy = 251.0, 40.0
    f = oracle_lib.fovea(cam, scenegen.Fovea(gx, gy), 4, 16)
    ecc = f["ecc"].reshape(181, 321)
    assert ecc[int(gy), int(gx)] < 1e-9
    xs = np.arange(321)
    b = (gy - cam.cy) / cam.fy
    fx = cam.fx * math.sqrt(1 + b * b)
    row = np.degrees(np.abs(np.arctan((xs - cam.cx) / fx) - np.arctan((gx - cam.cx) / fx)))
    np.testing.assert_allclose(ecc[int(gy)], row, atol=1e-9)
    f0 = oracle_lib.fovea(cam, scenegen.Fovea(gx, cam.cy), 4, 16)
    row0 = np.degrees(np.abs(np.arctan((xs - cam.cx) / cam.fx) - np.arctan((gx - cam.cx) / cam.fx)))
    np.testing.assert_allclose(f0["ecc"].reshape(181, 321)[int(cam.cy)], row0, atol=1e-9)
    a = (gx - cam.cx) / cam.fx
    fy = cam.fy * math.sqrt(1 + a * a)
    ys = np.arange(181)
    col = np.degrees(np.abs(np.arctan((ys - cam.cy) / fy) - np.arctan((gy - cam.cy) / fy)))
    np.testing.assert_allclose(ecc[:, int(gx)], col, atol=1e-9)
    # any pixel: rotate the gaze ray onto the optical axis, the eccentricity
    # is then the polar angle of the rotated pixel ray
    g = np.array([(gx - cam.cx) / cam.fx, (gy - cam.cy) / cam.fy, 1.0])
    e3 = g / np.linalg.norm(g)
    e1 = np.cross([0.0, 1.0, 0.0], e3)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(e3, e1)
    Rg = np.stack([e1, e2, e3])
    rng = np.random.default_rng(2)
    for x, y in zip(rng.integers(0, 321, 50), rng.integers(0, 181, 50)):
        r = Rg @ np.array([(x - cam.cx) / cam.fx, (y - cam.cy) / cam.fy, 1.0])
        assert abs(ecc[y, x] - math.degrees(math.atan2(math.hypot(r[0], r[1]), r[2]))) < 1e-9
    # the levels follow the gaze: the gaze pixel is in the fovea and the
    # pixel farthest from it is in the outer ring
    lo = f["pix_lo"].reshape(181, 321)
    assert lo[int(gy), int(gx)] == 1
    far = np.unravel_index(np.argmax(ecc), ecc.shape)
    assert far == (180, 0) and lo[far] == 4
