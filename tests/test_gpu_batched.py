"""Batched multi-view step and its graph replay (through the C ABI).

The batched schedule (all views of a sub-batch in one call per stage) must
give the per-view schedule's results: images, final transmittance and
last-contributor indices bit for bit (each tile sees the same sorted list),
the loss and the parameter gradients up to float32 reassociation (the
gradients are summed over views in a different order and with atomics).
A recorded graph is replayed several times, with eager work and host
synchronisation between replays, and every replay is checked against the
eager step.  Per-view parity with the oracle is covered by the parity tests.
"""
import numpy as np
import pytest
import torch

import scenegen
from gpu_util import need_gpu, rel_l2, say

pytestmark = pytest.mark.gpu

GRAD_RTOL = 1e-5  # relative L2 between schedules (float32 reassociation only)


def gs():
    need_gpu()
    import paper_2407_00435_amd as g
    return g


def views():
    return [scenegen.pinhole(203, 157, 60.0, t=(0.0, 0.0, 4.0)),
            scenegen.look_at((1.2, -0.6, -3.3), (0.1, 0.0, 0.0), 131, 97, 55.0),
            scenegen.look_at((-2.5, 0.4, -2.9), (0.0, 0.1, 0.0), 96, 64, 62.0),
            scenegen.look_at((0.3, 2.2, -3.1), (0.0, 0.0, 0.2), 160, 90, 58.0),
            scenegen.look_at((3.0, -0.2, 2.4), (0.0, 0.0, 0.0), 77, 121, 65.0)]


def setup(g, n=3000, seed=21, fr=4):
    sc = scenegen.small_scene(n, seed=seed, sh_degree=3, fr_levels=fr, log_scale_mu=-3.4,
                              log_scale_sigma=0.6)
    cams = views()
    S = g.SceneTensors(sc)
    px = sum(c.width * c.height for c in cams)
    rng = np.random.default_rng(seed)
    target = torch.from_numpy(rng.uniform(0.0, 1.0, 3 * px).astype(np.float32)).cuda()
    eyes = [scenegen.pinhole(96, 64, 94.0, t=(0.03, 0.0, 4.0)), scenegen.pinhole(96, 64, 94.0, t=(-0.03, 0.0, 4.0))]
    fov = [scenegen.Fovea(40.0, 30.0), scenegen.Fovea(44.0, 31.0)]
    return sc, S, cams, target, eyes, fov


def snapshot(step):
    torch.cuda.synchronize()
    out = dict(image=step.image.clone(), final_T=step.final_T.clone(), n_contrib=step.n_contrib.clone(),
               dL=step.dL.clone(), loss=step.loss.clone(),
               grads={k: v.clone() for k, v in step.grads.items() if v is not None})
    if step.eye_image is not None:
        out["eyes"] = step.eye_image.clone()
    return out


def assert_same(a, b, exact_grads=False):
    assert torch.equal(a["image"], b["image"])
    assert torch.equal(a["final_T"], b["final_T"])
    assert torch.equal(a["n_contrib"], b["n_contrib"])
    assert torch.equal(a["dL"], b["dL"])
    assert abs(a["loss"].item() - b["loss"].item()) <= 1e-6 * max(1.0, abs(a["loss"].item()))
    for k in a["grads"]:
        if exact_grads:
            assert torch.equal(a["grads"][k], b["grads"][k]), k
        else:
            assert rel_l2(a["grads"][k].cpu().numpy(), b["grads"][k].cpu().numpy()) < GRAD_RTOL, k
    if "eyes" in a:
        assert torch.equal(a["eyes"], b["eyes"])


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_batched_equals_per_view(tile):
    g = gs()
    from paper_2407_00435_amd.batched import BatchedStep
    sc, S, cams, target, eyes, fov = setup(g)
    say("batched vs per view", tile)
    full = BatchedStep(S, cams, target, tile, None, eyes, fov)
    full.step()
    a = snapshot(full)
    assert full.keys_ok()
    for bv in (1, 2):
        part = BatchedStep(S, cams, target, tile, bv, eyes, fov, eye_batch=bv)
        part.step()
        b = snapshot(part)
        assert part.keys_ok()
        assert_same(a, b)
    # the loss and its gradient are the L1 definition on the rendered image
    img, tg = a["image"].cpu().numpy().astype(np.float64), target.cpu().numpy().astype(np.float64)
    ref = np.abs(img - tg).sum() / img.size
    assert abs(a["loss"].item() - ref) < 1e-5 * ref
    np.testing.assert_array_equal(a["dL"].cpu().numpy(), (np.sign(img - tg) / img.size).astype(np.float32))


def test_batched_step_matches_separate_calls():
    """The step's forward pieces equal the standalone one-call renders."""
    g = gs()
    from paper_2407_00435_amd.batched import BatchedStep
    sc, S, cams, target, eyes, fov = setup(g, seed=23)
    step = BatchedStep(S, cams, target, 16, None, eyes, fov)
    step.step()
    a = snapshot(step)
    C = g.Cameras(cams)
    out = g.gs_render_fwd(S, C, 16, key_capacity=step.groups[0]["cap"])
    torch.cuda.synchronize()
    assert torch.equal(out["image"], a["image"])
    img, _, _ = g.gs_render_foveated(S, g.Cameras(eyes), fov, 16, key_capacity=step.eye_groups[0]["cap"])
    torch.cuda.synchronize()
    assert torch.equal(img, a["eyes"])
    # parameter gradients: reverse passes called one by one
    grads = g.gs_rasterize_bwd(out["splats"], S.n, C, 16, out["vals"], out["ranges"], out["final_T"],
                               out["n_contrib"], a["dL"])
    pg = g.gs_project_bwd(S, C, out["splats"], grads)
    torch.cuda.synchronize()
    for k in pg:
        assert rel_l2(pg[k].cpu().numpy(), a["grads"][k].cpu().numpy()) < GRAD_RTOL, k


@pytest.mark.parametrize("bv,lanes", [(None, 1), (2, 1), (2, 2), (1, 2)])
def test_graph_replays_match_eager(bv, lanes):
    g = gs()
    from paper_2407_00435_amd.batched import BatchedStep
    sc, S, cams, target, eyes, fov = setup(g, seed=25)
    say("graph replay", bv, lanes)
    step = BatchedStep(S, cams, target, 16, bv, eyes, fov, lanes=lanes)
    step.step()
    eager = snapshot(step)
    step.capture()
    for rep in range(4):
        # eager work on the default stream and a host synchronisation between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        step.replay()
        got = snapshot(step)
        assert_same(eager, got)
        assert torch.isfinite(junk)
    # the replay reads the target's current contents
    target.mul_(0.5)
    step.step()
    eager2 = snapshot(step)
    step.replay()
    got2 = snapshot(step)
    assert_same(eager2, got2)
    assert not torch.equal(eager2["dL"], eager["dL"]) or not torch.equal(eager2["loss"], eager["loss"])
    step.graph.close()


@pytest.mark.parametrize("bv", [1, 2])
def test_two_lanes_equal_one_lane(bv):
    """Sub-batches alternating over two streams (one's binning beside the
    other's compositing) give the one-stream step: the same images and
    compositing state, the same loss and, up to the order of float atomics,
    the same parameter gradients (the projection reverses accumulate in
    sub-batch order)."""
    g = gs()
    from paper_2407_00435_amd.batched import BatchedStep
    sc, S, cams, target, eyes, fov = setup(g, seed=27)
    say("two lanes", bv)
    one = BatchedStep(S, cams, target, 16, bv, eyes, fov, lanes=1)
    one.step()
    a = snapshot(one)
    two = BatchedStep(S, cams, target, 16, bv, eyes, fov, lanes=2)
    assert two.lanes == 2
    for rep in range(2):
        two.step()
        assert_same(a, snapshot(two))


def test_autotune_small():
    g = gs()
    from paper_2407_00435_amd import autotune
    from paper_2407_00435_amd.batched import BatchedStep
    sc, S, cams, target, eyes, fov = setup(g, n=2000, seed=27)
    best, tried = autotune.tune(S, cams, target, eyes, fov, reps=2)
    assert best["tile"] in (8, 16, 32) and 1 <= best["batch_views"] <= len(cams)
    assert best["radix_part"] in (8192, 16384) and np.isfinite(best["ms"])
    assert best["raster_queue"] in (0, 1)
    assert len(tried) >= 5
    step = BatchedStep(S, cams, target, best["tile"], best["batch_views"], eyes, fov)
    step.step()
    ref = BatchedStep(S, cams, target, best["tile"], None, eyes, fov)
    ref.step()
    assert_same(snapshot(ref), snapshot(step))
    g.gs_set_tuning("radix_part", 8192)
    g.gs_set_tuning("raster_queue", 0)


def eye_target(g, S, eyes, fov, seed=31):
    C = g.Cameras(eyes)
    _, n_px = C.tiles(16)
    rng = np.random.default_rng(seed)
    return torch.from_numpy(rng.uniform(0.0, 1.0, 3 * n_px).astype(np.float32)).cuda()


def test_eye_training_matches_autograd():
    """Eyes only: the step's foveated forward, L1 loss and reverse give the
    gradients of the autograd foveated render under the same loss."""
    g = gs()
    from paper_2407_00435_amd.batched import BatchedStep
    sc, S, cams, target, eyes, fov = setup(g, seed=33)
    et = eye_target(g, S, eyes, fov)
    step = BatchedStep(S, [], target[:0], 16, None, eyes, fov, eye_target=et)
    step.step()
    a = snapshot(step)
    names = ("means", "log_scales", "quats", "opacity_logits", "sh", "lvl_opacity_logits", "lvl_sh_dc")
    params = [S.t[k].clone().requires_grad_(True) for k in names]
    img = g.render_foveated(*params, S.t["qbound"], g.Cameras(eyes), fov, sc.sh_degree, 16)
    loss = (img - et).abs().mean()
    loss.backward()
    torch.cuda.synchronize()
    assert torch.equal(img.detach(), a["eyes"])
    assert abs(loss.item() - a["loss"].item()) <= 1e-5 * loss.item()
    for p, k in zip(params, names):
        assert rel_l2(p.grad.cpu().numpy(), a["grads"][k].cpu().numpy()) < 1e-5, k


@pytest.mark.parametrize("bv", [None, 1])
def test_views_and_eyes_training_graph(bv):
    """Views and trained eyes in one step: per-view schedule = batched, and
    graph replays = eager."""
    g = gs()
    from paper_2407_00435_amd.batched import BatchedStep
    sc, S, cams, target, eyes, fov = setup(g, seed=35)
    et = eye_target(g, S, eyes, fov, seed=36)
    ref = BatchedStep(S, cams, target, 16, None, eyes, fov, eye_target=et)
    ref.step()
    a = snapshot(ref)
    step = BatchedStep(S, cams, target, 16, bv, eyes, fov, eye_batch=bv, eye_target=et)
    step.step()
    assert_same(a, snapshot(step))
    step.capture()
    for _ in range(3):
        torch.cuda.synchronize()
        step.replay()
        assert_same(a, snapshot(step))
    assert step.keys_ok()
    step.graph.close()
