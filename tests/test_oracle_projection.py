"""Pins for the oracle's projection and colour (Section 2.1, Eq. 1b/1c).

Each check is against something other than the oracle's own formula:
closed forms, finite differences of the pinhole map, rotation invariance,
and numerical quadrature of the spherical-harmonic basis.
"""
import math

import numpy as np
import pytest

import scenegen


def one(mean, log_scale, quat=(1.0, 0.0, 0.0, 0.0), logit=0.0, sh=None, deg=0):
    K = (deg + 1) ** 2
    sh = np.zeros((1, K, 3)) if sh is None else np.asarray(sh, np.float64).reshape(1, K, 3)
    return scenegen.Scene(np.array([mean], np.float64), np.array([log_scale], np.float64),
                          np.array([quat], np.float64), np.array([logit], np.float64), sh, deg)


CAM = scenegen.pinhole(64, 48, 60.0, t=(0.0, 0.0, 4.0))


def test_isotropic_on_axis_closed_form(oracle_lib):
    # on the optical axis J = [diag(f/z, f/z), 0], so the 2D covariance is
    # ((f s / z)^2 + 0.3) I exactly; the mean lands on the principal point
    s = 0.05
    for z in (0.5, 1.0, 3.0):
        pr = oracle_lib.project(one((0.0, 0.0, z), [math.log(s)] * 3), CAM)
        zc = z + 4.0
        var = (CAM.fx * s / zc) ** 2 + 0.3
        np.testing.assert_allclose(pr["cov2d"][0], [var, 0.0, var], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(pr["mean2d"][0], [CAM.cx, CAM.cy], atol=1e-12)
        assert pr["depth"][0] == pytest.approx(zc)
        assert pr["radius"][0] == math.ceil(3.0 * math.sqrt(var))


def test_conic_is_inverse(oracle_lib):
    sc = scenegen.small_scene(200, seed=5, sh_degree=0)
    pr = oracle_lib.project(sc, CAM)
    vis = pr["visible"] > 0
    a, b, c = pr["cov2d"][vis].T
    A, B, C = pr["conic"][vis].T
    np.testing.assert_allclose(a * A + b * B, 1.0, rtol=1e-10)
    np.testing.assert_allclose(a * B + b * C, 0.0, atol=1e-10 * np.abs(a * B).max())
    np.testing.assert_allclose(b * B + c * C, 1.0, rtol=1e-10)


def test_jacobian_matches_finite_difference_of_pinhole(oracle_lib):
    # a tiny isotropic Gaussian off axis (inside the tangent clamp) has
    # cov2d - 0.3 I = s^2 J J^T, J the Jacobian of world -> pixel
    s = 1e-3
    R = scenegen.look_at((0.7, -0.4, -3.0), (0.1, 0.2, 0.0), 64, 48, 60.0).R
    cam = scenegen.look_at((0.7, -0.4, -3.0), (0.1, 0.2, 0.0), 64, 48, 60.0)
    assert np.allclose(R @ R.T, np.eye(3))
    mu = np.array([0.3, -0.2, 0.4])
    pr = oracle_lib.project(one(mu, [math.log(s)] * 3), cam)

    def pix(p):
        u = cam.R @ p + cam.t
        return np.array([cam.fx * u[0] / u[2] + cam.cx, cam.fy * u[1] / u[2] + cam.cy])

    h = 1e-6
    J = np.stack([(pix(mu + h * e) - pix(mu - h * e)) / (2 * h) for e in np.eye(3)], 1)
    cov = s * s * J @ J.T
    np.testing.assert_allclose(pr["cov2d"][0] - [0.3, 0.0, 0.3], [cov[0, 0], cov[0, 1], cov[1, 1]],
                               rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(pr["mean2d"][0], pix(mu), atol=1e-9)


def test_isotropic_is_rotation_invariant(oracle_lib):
    rng = np.random.default_rng(0)
    base = oracle_lib.project(one((0.2, 0.1, 0.3), [-2.0] * 3), CAM)
    for _ in range(5):
        q = rng.standard_normal(4)
        pr = oracle_lib.project(one((0.2, 0.1, 0.3), [-2.0] * 3, quat=q), CAM)
        np.testing.assert_allclose(pr["cov2d"], base["cov2d"], rtol=1e-12)


def test_quaternion_rotation_about_z(oracle_lib):
    # scales (sa, sb, sc) rotated 90 degrees about z swap the x and y extents
    sa, sb = 0.08, 0.02
    ls = [math.log(sa), math.log(sb), math.log(0.01)]
    q90 = (math.cos(math.pi / 4), 0.0, 0.0, math.sin(math.pi / 4))
    pr0 = oracle_lib.project(one((0.0, 0.0, 0.0), ls), CAM)
    pr1 = oracle_lib.project(one((0.0, 0.0, 0.0), ls, quat=q90), CAM)
    f = CAM.fx / 4.0
    np.testing.assert_allclose(pr0["cov2d"][0], [(f * sa) ** 2 + 0.3, 0.0, (f * sb) ** 2 + 0.3], rtol=1e-12)
    np.testing.assert_allclose(pr1["cov2d"][0], [(f * sb) ** 2 + 0.3, 0.0, (f * sa) ** 2 + 0.3],
                               rtol=1e-12, atol=1e-15)
    # an unnormalised quaternion is normalised first
    pr2 = oracle_lib.project(one((0.0, 0.0, 0.0), ls, quat=[3 * v for v in q90]), CAM)
    np.testing.assert_allclose(pr2["cov2d"], pr1["cov2d"], rtol=1e-12, atol=1e-15)


def test_near_plane_cull(oracle_lib):
    pr = oracle_lib.project(one((0.0, 0.0, -3.85), [-3.0] * 3), CAM)  # camera z = 0.15
    assert pr["visible"][0] == 0 and pr["radius"][0] == 0
    pr = oracle_lib.project(one((0.0, 0.0, -3.7), [-3.0] * 3), CAM)   # camera z = 0.3
    assert pr["visible"][0] == 1 and pr["radius"][0] > 0


def test_opacity_is_sigmoid(oracle_lib):
    for lg in (-3.0, 0.0, 2.5):
        pr = oracle_lib.project(one((0.0, 0.0, 0.0), [-3.0] * 3, logit=lg), CAM)
        assert pr["opacity"][0] == pytest.approx(1.0 / (1.0 + math.exp(-lg)), rel=1e-14)


def _sphere_quadrature(n_theta=24, n_phi=48):
    # Gauss-Legendre in cos(theta) x uniform phi: exact for polynomials of
    # degree < 2 n_theta in z and trigonometric degree < n_phi in phi
    z, wz = np.polynomial.legendre.leggauss(n_theta)
    phi = np.arange(n_phi) * 2 * math.pi / n_phi
    pts, wts = [], []
    for zi, wi in zip(z, wz):
        r = math.sqrt(1 - zi * zi)
        for p in phi:
            pts.append((r * math.cos(p), r * math.sin(p), zi))
            wts.append(wi * 2 * math.pi / n_phi)
    return np.array(pts), np.array(wts)


def test_sh_orthonormal_by_quadrature(oracle_lib):
    pts, wts = _sphere_quadrature()
    Y = np.stack([oracle_lib.sh_basis(3, p) for p in pts])  # (P, 16)
    gram = (Y * wts[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-12)


def test_sh_low_order_cartesian_forms(oracle_lib):
    # textbook Cartesian forms of the real basis for l <= 1 (no phase factor)
    rng = np.random.default_rng(1)
    for _ in range(10):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        Y = oracle_lib.sh_basis(1, d)
        c0 = 0.5 / math.sqrt(math.pi)
        c1 = math.sqrt(3.0 / (4.0 * math.pi))
        np.testing.assert_allclose(Y, [c0, c1 * d[1], c1 * d[2], c1 * d[0]], rtol=1e-12)


def test_dc_only_colour(oracle_lib):
    dc = np.array([0.7, -1.2, 2.0])
    sh = np.zeros((1, 3))
    sh[0] = dc
    pr = oracle_lib.project(one((0.1, 0.2, 0.3), [-3.0] * 3, sh=sh, deg=0), CAM)
    expect = np.maximum(0.0, 0.28209479177387814 * dc + 0.5)
    np.testing.assert_allclose(pr["color"][0], expect, rtol=1e-14)


def test_level_versions_replace_dc_and_opacity(oracle_lib):
    sc = scenegen.small_scene(64, seed=9, fr_levels=4)
    pr = oracle_lib.project(sc, CAM, levels=True)
    np.testing.assert_allclose(pr["lvl_opacity"][0], pr["opacity"], rtol=1e-14)
    np.testing.assert_allclose(pr["lvl_color"][0], pr["color"], rtol=1e-14)
    # level t differs from the base only through DC (a shift of Y00 * delta before the clamp)
    raw = pr["color"]
    for t in range(1, 4):
        delta = (sc.lvl_sh_dc[t].astype(np.float64) - sc.sh[:, 0, :]) * 0.28209479177387814
        ok = (raw > 0) & (pr["lvl_color"][t] > 0)
        np.testing.assert_allclose(pr["lvl_color"][t][ok], (raw + delta)[ok], rtol=1e-9, atol=1e-12)
        # the logistic of the level logit where the point has a level-(t + 1)
        # version (quality bound >= t + 1, Section 4.2), zero above its bound
        op = 1.0 / (1.0 + np.exp(-sc.lvl_opacity_logits[t].astype(np.float64)))
        op = np.where(np.asarray(sc.qbound) >= t + 1, op, 0.0)
        np.testing.assert_allclose(pr["lvl_opacity"][t], op, rtol=1e-13)


def test_sh_basis_gradient_is_the_derivative(oracle_lib):
    # the reverse pass's analytic derivative of Y(d / |d|) against central
    # differences of the basis itself, at random directions and near and at
    # the poles (where the angle form of the basis has no derivative in phi)
    # (the angle form takes sqrt(1 - z^2), which keeps few digits within
    # 1e-4 of a pole, so the differences there are only good to about 1e-5,
    # and at the pole itself to about 1e-4: still far below any wrong sign,
    # factor or dropped term, which are of order 0.1)
    rng = np.random.default_rng(4)
    dirs = [(rng.standard_normal(3), 2e-8) for _ in range(12)]
    dirs += [(np.array([1e-4, -2e-4, 1.0]), 1e-5), (np.array([3e-5, 1e-5, -1.0]), 1e-5),
             (np.array([0.0, 0.0, 1.0]), 1e-4), (np.array([1.0, 0.0, 0.0]), 2e-8),
             (np.array([0.0, -1.0, 0.0]), 2e-8)]
    h = 1e-6
    for d, tol in dirs:
        d = d / np.linalg.norm(d)
        Y, dY = oracle_lib.sh_basis_grad(3, d)
        np.testing.assert_allclose(Y, oracle_lib.sh_basis(3, d), atol=1e-13)
        fd = np.zeros((16, 3))
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            yp = oracle_lib.sh_basis(3, (d + e) / np.linalg.norm(d + e))
            ym = oracle_lib.sh_basis(3, (d - e) / np.linalg.norm(d - e))
            fd[:, a] = (yp - ym) / (2 * h)
        np.testing.assert_allclose(dY, fd, atol=tol)
        # a radial change of d does not change Y(d / |d|)
        np.testing.assert_allclose(dY @ d, 0.0, atol=1e-13)


def test_tangent_clamp_closed_form(oracle_lib):
    # a small isotropic Gaussian beyond the Jacobian's tangent limits: with
    # R = I, Sigma = s^2 I, J = [[f/z, 0, -f tx/z], [0, f/z, -f ty/z]] and the
    # tangents tx, ty clamped to 1.3 tan(fov/2) on each axis, the 2D
    # covariance is (f s / z)^2 [[1 + tx^2, tx ty], [tx ty, 1 + ty^2]] + 0.3 I
    s = 0.05
    f = CAM.fx
    limx = 1.3 * (CAM.width / 2.0) / CAM.fx
    limy = 1.3 * (CAM.height / 2.0) / CAM.fy
    for mean, tx, ty in (((4.5, 3.0, 0.0), limx, limy),       # both clamped
                         ((-4.5, 0.8, 0.0), -limx, 0.2),      # x clamped only
                         ((0.4, -3.2, 0.0), 0.1, -limy)):     # y clamped only
        z = mean[2] + 4.0
        pr = oracle_lib.project(one(mean, [math.log(s)] * 3), CAM)
        k = (f * s / z) ** 2
        expect = [k * (1 + tx * tx) + 0.3, k * tx * ty, k * (1 + ty * ty) + 0.3]
        np.testing.assert_allclose(pr["cov2d"][0], expect, rtol=1e-12, atol=1e-14)
        # the unclamped tangents would give a clearly different covariance
        ux, uy = mean[0] / z, mean[1] / z
        free = [k * (1 + ux * ux) + 0.3, k * ux * uy, k * (1 + uy * uy) + 0.3]
        assert np.max(np.abs(np.subtract(free, expect))) > 0.05 * k
        # the mean is not clamped
        np.testing.assert_allclose(pr["mean2d"][0], [f * ux + CAM.cx, f * uy + CAM.cy], rtol=1e-13)


def test_sh_direction_from_the_camera_centre(oracle_lib):
    # rotated cameras: the colour direction runs from the camera centre (the
    # eye position the camera was built from, not its translation vector) to
    # the mean, in world space; the degree-1 basis is c1 (y, z, x) there
    c0 = 0.5 / math.sqrt(math.pi)
    c1 = math.sqrt(3.0 / (4.0 * math.pi))
    rng = np.random.default_rng(11)
    for eye in ((1.2, -0.6, -3.3), (-2.5, 1.5, 2.0), (0.0, 3.5, 0.5)):
        cam = scenegen.look_at(eye, (0.1, 0.0, 0.0), 64, 48, 60.0)
        assert np.abs(np.asarray(cam.t) + np.asarray(eye)).max() > 0.1  # -t is not the centre
        mu = np.array([0.3, -0.2, 0.4])
        sh = rng.normal(0.0, 0.3, (4, 3))
        sh[0] = 1.0
        pr = oracle_lib.project(one(mu, [-3.0] * 3, sh=sh, deg=1), cam)
        assert pr["visible"][0]
        d = (mu - np.asarray(eye)) / np.linalg.norm(mu - np.asarray(eye))
        expect = 0.5 + c0 * sh[0] + c1 * (sh[1] * d[1] + sh[2] * d[2] + sh[3] * d[0])
        assert np.all(expect > 0)
        np.testing.assert_allclose(pr["color"][0], expect, rtol=1e-12)
