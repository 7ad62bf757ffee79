"""Pins for the oracle's reverse of the foveated render (Section 4.1 blend,
Section 4.2 filter and per-level opacity / DC): central finite differences
of the oracle's FP64 foveated forward, including the level versions, and
the reduction to the plain reverse when every pixel sits in one level."""
import numpy as np
import pytest

import scenegen


def fr_case(seed=12, n=70, W=40, H=30):
    sc = scenegen.small_scene(n, seed=seed, sh_degree=2, fr_levels=4, log_scale_mu=-2.3,
                              log_scale_sigma=0.35)
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "lvl_opacity_logits", "lvl_sh_dc"):
        setattr(sc, k, np.asarray(getattr(sc, k), dtype=np.float64))
    cam = scenegen.pinhole(W, H, scenegen.FR_FOV_DEG, t=(0.0, 0.0, 2.6))
    fov = scenegen.Fovea(19.0, 14.0, rings_deg=(8.0, 16.0, 24.0), band_deg=4.0)
    return sc, cam, fov


def fr_loss(oracle_lib, sc, cam, lo, w, wts):
    img = oracle_lib.fr_render(sc, cam, lo, w).transpose(2, 0, 1)
    return float((img * wts).sum())


def test_fr_reverse_matches_finite_differences(oracle_lib):
    sc, cam, fov = fr_case()
    f = oracle_lib.fovea(cam, fov, 4, 8)
    lo, w = f["pix_lo"], f["pix_w"]
    assert len(set(lo.tolist())) >= 3 and (w > 0).mean() > 0.1  # several levels and bands
    rng = np.random.default_rng(1)
    wts = rng.uniform(-1.0, 1.0, (3, cam.height, cam.width))
    g = oracle_lib.fr_reverse(sc, [cam], [(lo, w)], [wts])
    arrays = {k: getattr(sc, k) for k in ("means", "log_scales", "quats", "sh", "lvl_opacity_logits",
                                          "lvl_sh_dc", "opacity_logits")}
    # points that blend somewhere
    live = np.nonzero(np.abs(g["lvl_opacity_logits"]).sum(0) > 1e-9)[0]
    assert len(live) > 20
    picks = []
    for i in rng.choice(live, 14, replace=False):
        for a in range(3):
            picks.append(("means", (i, a)))
            picks.append(("log_scales", (i, a)))
        picks.append(("quats", (i, int(rng.integers(0, 4)))))
        picks.append(("sh", (i, int(rng.integers(1, 9)), int(rng.integers(0, 3)))))
        m = int(sc.qbound[i])
        for t in range(m):
            picks.append(("lvl_opacity_logits", (t, i)))
            picks.append(("lvl_sh_dc", (t, i, int(rng.integers(0, 3)))))
    checked = dropped = 0
    for name, idx in picks:
        arr = arrays[name]
        theta = arr[idx]
        h = 1e-6 * max(1.0, abs(theta))
        arr[idx] = theta + h
        lp = fr_loss(oracle_lib, sc, cam, lo, w, wts)
        arr[idx] = theta - h
        lm = fr_loss(oracle_lib, sc, cam, lo, w, wts)
        arr[idx] = theta
        l0 = fr_loss(oracle_lib, sc, cam, lo, w, wts)
        fwd, bwd = (lp - l0) / h, (l0 - lm) / h
        if abs(fwd - bwd) > 0.1 * max(abs(fwd), abs(bwd), 1e-6):
            dropped += 1  # a skip / stop / clamp kink between the two sides
            continue
        fd = (lp - lm) / (2 * h)
        gv = g[name][idx]
        assert abs(fd - gv) <= 5e-6 * max(abs(fd), abs(gv), 1e-3), (name, idx, fd, gv)
        checked += 1
    assert checked >= 0.9 * len(picks), (checked, dropped)
    # the base opacity logit and DC are not used by the foveated render when
    # every level has its own version
    assert np.all(g["opacity_logits"] == 0) and np.all(g["sh"][:, 0, :] == 0)


def test_fr_reverse_single_level_is_plain_reverse(oracle_lib):
    sc, cam, _ = fr_case(seed=13)
    n_px = cam.width * cam.height
    rng = np.random.default_rng(2)
    wts = rng.uniform(-1.0, 1.0, (3, cam.height, cam.width))
    for t in (1, 3):
        lo = np.full(n_px, t, np.uint8)
        w = np.zeros(n_px)
        g = oracle_lib.fr_reverse(sc, [cam], [(lo, w)], [wts])
        sub, idx = oracle_lib.level_scene(sc, t)
        ref = oracle_lib.reverse(sub, [cam], [wts])
        np.testing.assert_allclose(g["means"][idx], ref["means"], rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(g["lvl_opacity_logits"][t - 1][idx], ref["opacity_logits"], rtol=1e-12,
                                   atol=1e-15)
        rest = np.setdiff1d(np.arange(sc.n), idx)
        assert np.all(g["means"][rest] == 0)
