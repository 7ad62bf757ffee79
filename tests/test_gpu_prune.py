"""Pruning metrics on the GPU (through the C ABI) against the oracle.

CE is a float32 ratio of integer counts and must match bit for bit given
the GPU's own hit and dominated counts (those are checked against the
oracle by the binning and compositing parity tests); the selection of the
lowest-CE points is integer work and must match exactly, ties included;
the weighted scale and its gradient are float32 sums, within 1e-5
relative of the FP64 values.
"""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def gs():
    need_gpu()
    import paper_2407_00435_amd as g
    return g


def views():
    return [scenegen.pinhole(203, 157, 60.0, t=(0.0, 0.0, 4.0)),
            scenegen.look_at((1.2, -0.6, -3.3), (0.1, 0.0, 0.0), 131, 97, 55.0),
            scenegen.look_at((-2.8, 0.3, 2.2), (0.0, 0.0, 0.0), 160, 90, 60.0)]


def test_ce_matches_oracle():
    g = gs()
    from paper_2407_00435_amd import prune
    sc = scenegen.small_scene(4000, seed=81, sh_degree=3, log_scale_mu=-3.4, log_scale_sigma=0.6)
    S, C = g.SceneTensors(sc), g.Cameras(views())
    ce, hits, dom = prune.ce_over_views(S, C, 16)
    torch.cuda.synchronize()
    ref = oracle.ce_score(dom.cpu().numpy(), hits.cpu().numpy())
    np.testing.assert_array_equal(ce.cpu().numpy(), ref)
    assert (ref > 0).sum() > 100
    # one pruning round: 10 % with the lowest CE
    keep, idx, ce2 = prune.prune_round(S, C, 16, 0.10)
    torch.cuda.synchronize()
    m_ref, i_ref = oracle.select_lowest(ref, int(0.10 * sc.n))
    np.testing.assert_array_equal(idx.cpu().numpy().view(np.uint32), i_ref)
    np.testing.assert_array_equal((~keep).cpu().numpy().astype(np.uint8), m_ref)


@pytest.mark.parametrize("n", [1, 5, 4096, 4097, 100003, (1 << 20) + 17])
def test_select_lowest_matches_oracle(n):
    g = gs()
    rng = np.random.default_rng(n)
    # quantised values: many ties, including at the threshold
    ce = (rng.integers(0, 50, n).astype(np.float32) / np.float32(7)).astype(np.float32)
    ce[rng.random(n) < 0.3] = 0.0
    t = torch.from_numpy(ce).cuda()
    for k in sorted({0, 1, n // 10, n // 2, max(n - 1, 0), n}):
        say("select", n, k)
        mask, idx = g.gs_select_lowest(t, k)
        torch.cuda.synchronize()
        m_ref, i_ref = oracle.select_lowest(ce, k)
        np.testing.assert_array_equal(mask.cpu().numpy(), m_ref)
        if k:
            np.testing.assert_array_equal(idx.cpu().numpy().view(np.uint32), i_ref)


def test_weighted_scale_matches_oracle():
    g = gs()
    rng = np.random.default_rng(9)
    n, V = 50000, 3
    ls = rng.normal(-3.5, 0.8, (n, 3)).astype(np.float32)
    hits = rng.integers(0, 40, (V, n)).astype(np.int32)
    T, gamma = 10.0, 0.25
    ws_ref, grad_ref = oracle.weighted_scale(ls.astype(np.float64), hits, T, gamma)
    lt, ht = torch.from_numpy(ls).cuda(), torch.from_numpy(hits).cuda()
    ws, grad = g.gs_weighted_scale(lt, ht, T, gamma)
    torch.cuda.synchronize()
    assert abs(ws.item() - ws_ref) <= 1e-5 * abs(ws_ref)
    np.testing.assert_allclose(grad.cpu().numpy(), grad_ref, rtol=1e-5, atol=1e-12)
    # accumulate adds to an existing gradient
    base = torch.full((n, 3), 0.5, dtype=torch.float32, device="cuda")
    _, acc = g.gs_weighted_scale(lt, ht, T, gamma, d_log_scales=base, accumulate=True)
    torch.cuda.synchronize()
    np.testing.assert_allclose(acc.cpu().numpy(), grad_ref + 0.5, rtol=1e-5, atol=1e-7)


def test_weighted_scale_threshold_edges():
    g = gs()
    # U equal to T gives G = 0; a single view given as [1, n]
    ls = torch.zeros((3, 3), dtype=torch.float32, device="cuda")
    hits = torch.tensor([[5, 6, 4]], dtype=torch.int32, device="cuda")
    ws, grad = g.gs_weighted_scale(ls, hits, 5.0, 1.0)
    torch.cuda.synchronize()
    # only point 1 counts: S = 3, G = 1, WS = 3 / 3
    assert abs(ws.item() - 1.0) < 1e-6
    np.testing.assert_allclose(grad.cpu().numpy(), [[0, 0, 0], [1.0, 0, 0], [0, 0, 0]], atol=1e-7)
