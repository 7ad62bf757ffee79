"""Pins for the oracle's HVSQ (Section 2.2, Eq. 2) on the stated feature
reading: colour channels as features, square pooling windows of half-width
radius[i] centred on each pixel and clipped to the image, population mean
and standard deviation, the per-pixel term averaged over the channels, and
the mean over a region's pixels (Section 4.3).

- Identical images give 0 and a zero gradient.
- Windows of one pixel reduce the metric to the mean squared error (the
  standard deviation of one value is 0).
- Constant images: the term is the mean over channels of the squared
  difference of the constants.
- A window of known composition (two-valued stripes) against a constant:
  mean k/n, standard deviation sqrt(p (1 - p)) with p = k/n (population, not
  n - 1), also in a window clipped at the image corner.
- The gradient agrees with central finite differences of the metric.
- Regions partition the image: their sums and counts add up to the whole.
- The pooling radius is zero at the gaze pixel and grows with eccentricity.
- The terms at sampled pixels equal brute-force windows with numpy's
  population statistics (borders, and a window over the whole image).
"""
import math

import numpy as np
import pytest

import scenegen


def rnd(rng, H, W):
    return rng.uniform(0.0, 1.0, (3, H, W))


def test_identical_images_give_zero(oracle_lib):
    rng = np.random.default_rng(1)
    a = rnd(rng, 9, 13)
    rad = rng.integers(0, 4, 9 * 13)
    out = oracle_lib.hvsq(a, a, rad, 13, 9, grad_region=0)
    assert out["hvsq"][0] == 0.0 and np.all(out["grad"] == 0.0)


def test_single_pixel_windows_reduce_to_mse(oracle_lib):
    rng = np.random.default_rng(2)
    a, r = rnd(rng, 7, 11), rnd(rng, 7, 11)
    out = oracle_lib.hvsq(a, r, np.zeros(77, np.int32), 11, 7, grad_region=0)
    assert out["hvsq"][0] == pytest.approx(np.mean((a - r) ** 2), rel=1e-13)
    # d/da of mean((a - r)^2) over 3 N values
    np.testing.assert_allclose(out["grad"], 2.0 * (a - r) / a.size, rtol=1e-12)


def test_constant_images(oracle_lib):
    ca, cr = np.array([0.2, 0.7, 0.4]), np.array([0.5, 0.1, 0.4])
    a = np.broadcast_to(ca[:, None, None], (3, 6, 8)).copy()
    r = np.broadcast_to(cr[:, None, None], (3, 6, 8)).copy()
    rad = np.random.default_rng(3).integers(0, 5, 48)
    out = oracle_lib.hvsq(a, r, rad, 8, 6, want_terms=True)
    np.testing.assert_allclose(out["terms"], np.mean((ca - cr) ** 2), rtol=1e-13)


def test_known_window_composition(oracle_lib):
    # vertical stripes of 1 and 0 in every channel (columns x % 3 == 0 are 1)
    H, W = 10, 12
    a = np.zeros((3, H, W))
    a[:, :, 0::3] = 1.0
    r = np.full((3, H, W), 0.25)
    rad = np.zeros(H * W, np.int32)
    rad[4 * W + 5] = 2   # interior: columns 3..7 (ones at 3 and 6), rows 2..6 -> k = 10 of n = 25
    rad[0] = 2           # corner: columns 0..2, rows 0..2 -> k = 3 of n = 9
    out = oracle_lib.hvsq(a, r, rad, W, H, want_terms=True)
    for idx, k, n in ((4 * W + 5, 10, 25), (0, 3, 9)):
        p = k / n
        mu, sd = p, math.sqrt(p * (1 - p))
        assert out["terms"][idx] == pytest.approx((mu - 0.25) ** 2 + sd ** 2, rel=1e-13), idx


def test_gradient_matches_finite_differences(oracle_lib):
    rng = np.random.default_rng(4)
    H, W = 8, 10
    a, r = rnd(rng, H, W), rnd(rng, H, W)
    rad = rng.integers(0, 4, H * W).astype(np.int32)
    region = rng.integers(1, 4, H * W).astype(np.uint8)
    for gr in (0, 2):
        g = oracle_lib.hvsq(a, r, rad, W, H, region=region, n_regions=3, grad_region=gr)["grad"]
        idx = gr if gr else 3
        h = 1e-6
        for c, y, x in zip(rng.integers(0, 3, 25), rng.integers(0, H, 25), rng.integers(0, W, 25)):
            ap, am = a.copy(), a.copy()
            ap[c, y, x] += h
            am[c, y, x] -= h
            fp = oracle_lib.hvsq(ap, r, rad, W, H, region=region, n_regions=3)["hvsq"][idx - 1 if gr else 3]
            fm = oracle_lib.hvsq(am, r, rad, W, H, region=region, n_regions=3)["hvsq"][idx - 1 if gr else 3]
            fd = (fp - fm) / (2 * h)
            assert abs(fd - g[c, y, x]) <= 1e-6 * max(abs(fd), 1e-3), (gr, c, y, x, fd, g[c, y, x])


def test_regions_partition_the_image(oracle_lib):
    rng = np.random.default_rng(5)
    H, W = 9, 14
    a, r = rnd(rng, H, W), rnd(rng, H, W)
    rad = rng.integers(0, 6, H * W).astype(np.int32)
    region = rng.integers(1, 5, H * W).astype(np.uint8)
    out = oracle_lib.hvsq(a, r, rad, W, H, region=region, n_regions=4)
    assert out["sums"][:4].sum() == pytest.approx(out["sums"][4], rel=1e-13)
    assert out["counts"][:4].sum() == out["counts"][4] == H * W
    np.testing.assert_array_equal(out["counts"][:4], np.bincount(region, minlength=5)[1:])


def test_pooling_radius_grows_with_eccentricity(oracle_lib):
    cam = scenegen.pinhole(161, 91, scenegen.FR_FOV_DEG, t=(0.0, 0.0, 2.0))
    fov = scenegen.Fovea(40.0, 45.0)
    rho = 0.8
    rad, amb = oracle_lib.hvsq_radius(cam, fov, rho)
    rad = rad.reshape(91, 161)
    assert rad[45, 40] == 0
    ecc = oracle_lib.fovea(cam, fov, 1, 16)["ecc"].reshape(91, 161)
    np.testing.assert_array_equal(rad, np.floor(rho * ecc).astype(np.int32))
    row = rad[45, 40:]
    assert np.all(np.diff(row) >= 0) and row[-1] > 20


def test_sampled_terms_match_brute_force_windows(oracle_lib):
    # hvsq_at (the per-pixel terms at chosen pixels) against windows sliced
    # out by hand and numpy's population statistics, including windows
    # clipped at every border and one covering the whole image
    rng = np.random.default_rng(11)
    H, W = 9, 13
    a, r = rnd(rng, H, W), rnd(rng, H, W)
    rad = rng.integers(0, 5, H * W).astype(np.int32)
    rad[4 * W + 6] = 20
    pix = np.array([[0, 0], [12, 8], [6, 4], [12, 0], [0, 8], [3, 5], [9, 2]], np.int32)
    got = oracle_lib.hvsq_at(a, r, rad, W, H, pix)
    for k, (x, y) in enumerate(pix):
        h = int(rad[y * W + x])
        ys, xs = slice(max(0, y - h), min(H, y + h + 1)), slice(max(0, x - h), min(W, x + h + 1))
        wa, wr = a[:, ys, xs].reshape(3, -1), r[:, ys, xs].reshape(3, -1)
        term = np.mean((wa.mean(1) - wr.mean(1)) ** 2 + (wa.std(1) - wr.std(1)) ** 2)
        assert got[k] == pytest.approx(term, rel=1e-12, abs=1e-15), (x, y)
