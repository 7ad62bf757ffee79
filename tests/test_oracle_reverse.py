"""Pins for the oracle's reverse pass (the gradient of the forward as
defined: the training loops of Section 3.4 and Section 4.3 differentiate the
renderer of Eq. 1).

FP64 central finite differences of the oracle's full forward on the
256-Gaussian 32x32 case, and a single-Gaussian analytic derivative.
Parameters whose two one-sided differences disagree straddle a kink of
the piecewise-smooth forward (a skip, stop or clamp) and are dropped.
"""
import math

import numpy as np
import pytest

import scenegen


def loss(oracle_lib, sc, cam, wts):
    out = oracle_lib.render(sc, cam, nthreads=1)
    img = out["rgb"].transpose(2, 0, 1)  # (3, H, W)
    return float((img * wts).sum())


def fd_check(oracle_lib, sc, cam, wts, grads, picks, rel=5e-6):
    arrays = {"means": sc.means, "log_scales": sc.log_scales, "quats": sc.quats,
              "opacity_logits": sc.opacity_logits, "sh": sc.sh}
    checked = dropped = 0
    for name, idx in picks:
        arr = arrays[name]
        theta = arr[idx]
        h = 1e-6 * max(1.0, abs(theta))
        arr[idx] = theta + h
        lp = loss(oracle_lib, sc, cam, wts)
        arr[idx] = theta - h
        lm = loss(oracle_lib, sc, cam, wts)
        arr[idx] = theta
        l0 = loss(oracle_lib, sc, cam, wts)
        fwd, bwd = (lp - l0) / h, (l0 - lm) / h
        if abs(fwd - bwd) > 0.1 * max(abs(fwd), abs(bwd), 1e-6):
            dropped += 1
            continue
        fd = (lp - lm) / (2 * h)
        g = grads[name][idx]
        scale = max(abs(fd), abs(g), 1e-3)
        assert abs(fd - g) <= rel * scale, (name, idx, fd, g)
        checked += 1
    return checked, dropped


def as_f64(sc):
    return scenegen.Scene(sc.means.astype(np.float64), sc.log_scales.astype(np.float64),
                          sc.quats.astype(np.float64), sc.opacity_logits.astype(np.float64),
                          sc.sh.astype(np.float64), sc.sh_degree)


def test_reverse_matches_finite_differences(oracle_lib):
    wl = scenegen.fd_subcase()
    sc = as_f64(wl.scene)
    cam = wl.cams[0]
    rng = np.random.default_rng(0)
    wts = rng.uniform(-1.0, 1.0, (3, cam.height, cam.width))
    g = oracle_lib.reverse(sc, [cam], [wts])
    # Gaussians that actually cover pixels
    pr = oracle_lib.project(sc, cam)
    live = np.nonzero(np.abs(g["opacity_logits"]) > 1e-8)[0]
    assert len(live) > 50
    picks = []
    for i in rng.choice(live, 24, replace=False):
        for a in range(3):
            picks.append(("means", (i, a)))
            picks.append(("log_scales", (i, a)))
        for a in range(4):
            picks.append(("quats", (i, a)))
        picks.append(("opacity_logits", (i,)))
        for k in rng.choice(16, 3, replace=False):
            picks.append(("sh", (i, k, rng.integers(0, 3))))
    checked, dropped = fd_check(oracle_lib, sc, cam, wts, g, picks)
    assert checked >= 0.9 * len(picks), (checked, dropped)
    assert pr["visible"].sum() == sc.n


def test_single_gaussian_opacity_and_colour_derivative(oracle_lib):
    # one Gaussian over a black background: I(p) = c alpha(p), so
    # dL/dc = sum_p w(p) alpha(p) and dL/dlogit = sum_p w(p) c alpha(p) (1 - o)
    sc = scenegen.Scene(np.array([[0.0, 0.0, 0.0]]), np.array([[-1.6] * 3]),
                        np.array([[1.0, 0.0, 0.0, 0.0]]), np.array([0.4]),
                        np.array([[[0.5, -0.2, 0.3]]]), 0)
    cam = scenegen.pinhole(24, 24, 60.0, t=(0.0, 0.0, 4.0))
    wts = np.ones((3, 24, 24))
    g = oracle_lib.reverse(sc, [cam], [wts])
    pr = oracle_lib.project(sc, cam)
    o = pr["opacity"][0]
    c = pr["color"][0]
    yy, xx = np.mgrid[:24, :24]
    A, B, C = pr["conic"][0]
    dx, dy = xx - pr["mean2d"][0][0], yy - pr["mean2d"][0][1]
    q = A * dx * dx + 2 * B * dx * dy + C * dy * dy
    alpha = np.minimum(0.99, o * np.exp(-0.5 * q))
    use = (q <= 9) & (alpha >= 1 / 255)
    assert not (o * np.exp(-0.5 * q) > 0.99).any()
    sum_a = alpha[use].sum()
    Y00 = 0.5 / math.sqrt(math.pi)
    np.testing.assert_allclose(g["sh"][0, 0], Y00 * sum_a * np.ones(3), rtol=1e-12)
    assert g["opacity_logits"][0] == pytest.approx(c.sum() * sum_a * (1 - o), rel=1e-12)


def test_reverse_beyond_the_tangent_clamp_matches_finite_differences(oracle_lib):
    # two large Gaussians whose centres lie beyond the Jacobian's tangent
    # limit (one horizontally, one vertically) but whose extents reach the
    # image: the clamped tangent makes the covariance independent of the
    # clamped coordinate, and the reverse must agree with the forward there
    cam = scenegen.pinhole(64, 48, 60.0, t=(0.0, 0.0, 4.0))
    limx = 1.3 * 32.0 / cam.fx
    limy = 1.3 * 24.0 / cam.fy
    means = np.array([[3.3, 0.1, 0.0], [0.2, 2.6, 0.0]])
    assert means[0, 0] / 4.0 > limx and means[1, 1] / 4.0 > limy
    sc = scenegen.Scene(means, np.array([[-0.8, -0.9, -0.85], [-0.85, -0.8, -0.9]]),
                        np.array([[0.9, 0.1, -0.2, 0.3], [0.8, -0.3, 0.2, 0.1]]), np.array([0.6, 0.9]),
                        np.random.default_rng(3).normal(0.0, 0.3, (2, 16, 3)) + 0.2, 3)
    rng = np.random.default_rng(5)
    wts = rng.uniform(-1.0, 1.0, (3, cam.height, cam.width))
    g = oracle_lib.reverse(sc, [cam], [wts])
    out = oracle_lib.render(sc, cam, nthreads=1)
    assert (out["n_blend"] > 0).sum() > 40
    picks = []
    for i in range(2):
        assert abs(g["opacity_logits"][i]) > 1e-6
        for a in range(3):
            picks += [("means", (i, a)), ("log_scales", (i, a))]
        for a in range(4):
            picks.append(("quats", (i, a)))
        picks.append(("opacity_logits", (i,)))
        picks += [("sh", (i, k, k % 3)) for k in (0, 3, 9, 15)]
    checked, dropped = fd_check(oracle_lib, sc, cam, wts, g, picks)
    assert checked >= len(picks) - 2, (checked, dropped)
