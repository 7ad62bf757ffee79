"""Pins for the oracle's per-pixel compositing (Section 2.1, Eq. 1a) and the
dominated-pixel count Val_i (Section 3.2, Eq. 3).

Closed forms: a single isotropic Gaussian, a stack of identical Gaussians
(analytic transmittance product and stop index), unequal alphas by hand.
Brute force: a pure-Python all-pairs renderer on a tiny scene.
Invariants: input permutation, Sum Val_i, hand-made dominance scenes.
"""
import math

import numpy as np
import pytest

import scenegen


def splats(mean2d, sigma, opacity, color, depth):
    """Isotropic screen-space splats with covariance sigma^2 I."""
    n = len(depth)
    s2 = np.asarray(sigma, np.float64) ** 2 * np.ones(n)
    return dict(mean2d=np.asarray(mean2d, np.float64).reshape(n, 2),
                conic=np.stack([1 / s2, np.zeros(n), 1 / s2], 1),
                depth=np.asarray(depth, np.float64),
                opacity=np.asarray(opacity, np.float64) * np.ones(n),
                color=np.asarray(color, np.float64).reshape(n, 3),
                radius=np.ceil(3 * np.sqrt(s2)).astype(np.int32))


def test_single_isotropic_gaussian_image(oracle_lib):
    W, H = 40, 30
    mx, my, sig, o = 17.3, 12.6, 3.1, 0.8
    c = np.array([0.9, 0.4, 0.1])
    bg = np.array([0.05, 0.1, 0.2])
    out = oracle_lib.composite(splats([mx, my], sig, o, c, [2.0]), W, H, bg=bg)
    for y in range(H):
        for x in range(W):
            d2 = ((x - mx) ** 2 + (y - my) ** 2) / sig ** 2
            a = min(0.99, o * math.exp(-0.5 * d2))
            if d2 <= 9.0 and a >= 1.0 / 255.0:
                expect = c * a + (1 - a) * bg
            else:
                expect = bg
            np.testing.assert_allclose(out["rgb"][y, x], expect, rtol=1e-13, atol=1e-15)


def stacked_expectation(a, K, c, bg):
    # blending continues while the transmittance after the next Gaussian stays >= 1e-4
    k = 0
    while k < K and (1 - a) ** (k + 1) >= 1e-4:
        k += 1
    return c * (1 - (1 - a) ** k) + bg * (1 - a) ** k, k


@pytest.mark.parametrize("a,K", [(0.3, 10), (0.5, 40), (0.9, 8), (0.99, 5), (0.02, 100)])
def test_stacked_identical_gaussians(oracle_lib, a, K):
    c = np.array([0.2, 0.6, 1.0])
    bg = np.array([0.3, 0.3, 0.3])
    sp = splats(np.tile([[5.0, 5.0]], (K, 1)), 2.0, min(a, 0.99) if a < 0.99 else 1.0,
                np.tile(c, (K, 1)), np.arange(K) + 1.0)
    out = oracle_lib.composite(sp, 11, 11, bg=bg, pixels=np.array([[5, 5]]))
    expect, k = stacked_expectation(a, K, c, bg)
    np.testing.assert_allclose(out["rgb"][0], expect, rtol=1e-12)
    assert out["n_blend"][0] == k
    assert out["last_id"][0] == (k - 1 if k > 0 else -1)


def test_unequal_alphas_by_hand(oracle_lib):
    # three centred Gaussians (front to back) with alphas 0.5, 0.25, 0.8
    a = [0.5, 0.25, 0.8]
    cols = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    sp = splats(np.tile([[3.0, 3.0]], (3, 1)), 1.5, 1.0, cols, [1.0, 2.0, 3.0])
    sp["opacity"] = np.array(a)
    bg = np.array([1.0, 1.0, 1.0])
    out = oracle_lib.composite(sp, 7, 7, bg=bg, pixels=np.array([[3, 3]]))
    # T: 1, 0.5, 0.375, final 0.075
    expect = 0.5 * cols[0] + 0.5 * 0.25 * cols[1] + 0.375 * 0.8 * cols[2] + 0.075 * bg
    np.testing.assert_allclose(out["rgb"][0], expect, rtol=1e-14)
    assert out["T"][0] == pytest.approx(0.075, rel=1e-14)
    # contributions T*alpha: 0.5, 0.125, 0.3 -> the first dominates
    assert out["dom_id"][0] == 0


def brute_force(sp, W, H, bg):
    """All pairs, pure Python: for every pixel, every Gaussian in (depth, index) order."""
    n = len(sp["depth"])
    order = sorted(range(n), key=lambda i: (sp["depth"][i], i))
    img = np.zeros((H, W, 3))
    dom = -np.ones((H, W), int)
    for y in range(H):
        for x in range(W):
            C = [0.0, 0.0, 0.0]
            T = 1.0
            best, best_i = -1.0, -1
            for i in order:
                if sp["radius"][i] <= 0:
                    continue
                dx = x - sp["mean2d"][i][0]
                dy = y - sp["mean2d"][i][1]
                A, B, Cc = sp["conic"][i]
                q = A * dx * dx + 2 * B * dx * dy + Cc * dy * dy
                if q > 9.0:
                    continue
                alpha = min(0.99, sp["opacity"][i] * math.exp(-0.5 * q))
                if alpha < 1.0 / 255.0:
                    continue
                Tn = T * (1 - alpha)
                if Tn < 1e-4:
                    break
                for ch in range(3):
                    C[ch] += sp["color"][i][ch] * alpha * T
                if alpha * T > best:
                    best, best_i = alpha * T, i
                T = Tn
            img[y, x] = [C[ch] + T * bg[ch] for ch in range(3)]
            dom[y, x] = best_i
    return img, dom


def test_brute_force_tiny_scene(oracle_lib):
    sc = scenegen.small_scene(60, seed=3, sh_degree=1, log_scale_mu=-2.2, log_scale_sigma=0.5)
    cam = scenegen.pinhole(26, 20, 60.0, t=(0.0, 0.0, 4.0))
    pr = oracle_lib.project(sc, cam)
    bg = (0.1, 0.2, 0.3)
    out = oracle_lib.composite(pr, 26, 20, bg=bg)
    img, dom = brute_force(pr, 26, 20, bg)
    np.testing.assert_allclose(out["rgb"], img, rtol=1e-13, atol=1e-15)
    np.testing.assert_array_equal(out["dom_id"], dom)


def test_permutation_invariance(oracle_lib):
    sc = scenegen.small_scene(300, seed=4, sh_degree=2)
    cam = scenegen.pinhole(48, 40, 60.0, t=(0.0, 0.0, 4.0))
    base = oracle_lib.render(sc, cam)
    perm = np.random.default_rng(0).permutation(sc.n)
    other = oracle_lib.render(sc.subset(perm), cam)
    np.testing.assert_allclose(other["rgb"], base["rgb"], rtol=1e-12, atol=1e-14)
    ok = base["dom_id"] >= 0
    np.testing.assert_array_equal(perm[other["dom_id"][ok]], base["dom_id"][ok])


def test_dominance_two_gaussians(oracle_lib):
    # a faint front Gaussian over a strong back one: the back one dominates
    # at the centre (0.8 * 0.9 > 0.1); with a strong front one it flips
    sp = splats([[4.0, 4.0], [4.0, 4.0]], 2.0, 1.0, np.ones((2, 3)), [1.0, 2.0])
    sp["opacity"] = np.array([0.1, 0.8])
    out = oracle_lib.composite(sp, 9, 9, pixels=np.array([[4, 4]]))
    assert out["dom_id"][0] == 1
    sp["opacity"] = np.array([0.6, 0.8])
    out = oracle_lib.composite(sp, 9, 9, pixels=np.array([[4, 4]]))
    assert out["dom_id"][0] == 0


def test_val_sum_counts_covered_pixels(oracle_lib):
    sc = scenegen.small_scene(500, seed=6, sh_degree=0)
    cam = scenegen.pinhole(64, 64, 60.0, t=(0.0, 0.0, 4.0))
    out = oracle_lib.render(sc, cam)
    covered = (out["n_blend"] > 0).sum()
    val = np.bincount(out["dom_id"][out["dom_id"] >= 0], minlength=sc.n)
    assert val.sum() == covered
    assert covered > 0.3 * 64 * 64


def test_threshold_ambiguity_is_flagged(oracle_lib):
    # a pixel exactly on the 3-sigma ellipse: q = 9 within the margin
    sp = splats([[3.0, 0.0]], 1.0, 0.9, [[1.0, 1.0, 1.0]], [1.0])
    out = oracle_lib.composite(sp, 7, 1, pixels=np.array([[0, 0], [6, 0], [3, 0]]))
    assert out["amb"][0] & 1 and out["amb"][1] & 1 and not out["amb"][2] & 1
    a = 0.9 * math.exp(-4.5)
    # envelope spans both decisions
    assert out["rgb_min"][0][0] == pytest.approx(0.0, abs=1e-15)
    assert out["rgb_max"][0][0] == pytest.approx(a, rel=1e-12)
