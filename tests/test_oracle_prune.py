"""Pins of the oracle's pruning metrics (Section 3) against hand-computed
values, brute force and finite differences."""
import math

import numpy as np

import oracle


def test_ce_hand_example():
    # two views, four points; CE = max over views of dominated / tiles used
    dom = [[3, 0, 5, 7], [1, 2, 0, 0]]
    hits = [[2, 0, 10, 0], [1, 4, 1, 0]]
    ce = oracle.ce_score(dom, hits)
    assert ce.dtype == np.float32
    np.testing.assert_array_equal(ce, np.array([1.5, 0.5, 0.5, 0.0], np.float32))


def test_ce_single_view_and_rounding():
    # one view given as 1-D arrays; 1/3 is the float32 nearest to the ratio
    ce = oracle.ce_score([1, 2, 0], [3, 3, 5])
    np.testing.assert_array_equal(ce, np.array([np.float32(1) / np.float32(3), np.float32(2) / np.float32(3), 0.0],
                                               np.float32))
    assert ce[0] == np.float32(1.0 / 3.0)


def test_select_lowest_brute_force():
    rng = np.random.default_rng(3)
    for n, k in ((1, 0), (1, 1), (17, 5), (200, 20), (1000, 999)):
        # few distinct values so that ties are common
        ce = rng.integers(0, 6, n).astype(np.float32) / np.float32(4)
        mask, idx = oracle.select_lowest(ce, k)
        want = sorted(range(n), key=lambda i: (float(ce[i]), i))[:k]
        assert list(idx) == sorted(want)
        assert mask.sum() == k and all(mask[i] == 1 for i in want)


def test_select_lowest_clamps_k():
    mask, idx = oracle.select_lowest(np.array([0.5, 0.25], np.float32), 5)
    assert list(idx) == [0, 1] and mask.tolist() == [1, 1]
    mask, idx = oracle.select_lowest(np.array([0.5, 0.25], np.float32), -1)
    assert len(idx) == 0 and mask.sum() == 0


def test_weighted_scale_hand_example():
    # scales (world units): point 0 longest axis e^0 = 1 -> S = 3;
    # point 1 longest axis e^-1 -> S = 3 e^-1; point 2 uses few tiles
    ls = np.array([[0.0, -2.0, -1.0], [-3.0, -1.0, -2.0], [1.0, 1.0, 1.0]])
    hits = np.array([[10, 4, 3], [6, 12, 1]])
    T = 5.0
    ws, grad = oracle.weighted_scale(ls, hits, T, gamma=2.0)
    G = np.array([(10 - 5) + (6 - 5), 0 + (12 - 5), 0])
    S = np.array([3.0, 3.0 * math.exp(-1.0), 3.0 * math.e])
    want = 2.0 * (S * G).sum() / (3 * 2)
    assert abs(ws - want) < 1e-12
    assert grad[0, 0] == 2.0 * G[0] * S[0] / 6 and grad[0, 1] == 0 and grad[0, 2] == 0
    assert grad[1, 1] == 2.0 * G[1] * S[1] / 6 and grad[1, 0] == 0
    assert np.all(grad[2] == 0)  # G = 0 (uses no more than T tiles)


def test_weighted_scale_gradient_finite_difference():
    rng = np.random.default_rng(5)
    n, V = 40, 3
    ls = rng.normal(-3.0, 0.7, (n, 3))
    hits = rng.integers(0, 30, (V, n))
    T = 8.0
    _, grad = oracle.weighted_scale(ls, hits, T, gamma=0.7)
    h = 1e-6
    for i in range(0, n, 7):
        for k in range(3):
            a, b = ls.copy(), ls.copy()
            a[i, k] += h
            b[i, k] -= h
            fd = (oracle.weighted_scale(a, hits, T, 0.7)[0] - oracle.weighted_scale(b, hits, T, 0.7)[0]) / (2 * h)
            assert abs(fd - grad[i, k]) <= 1e-6 * max(1.0, abs(grad[i, k]))
