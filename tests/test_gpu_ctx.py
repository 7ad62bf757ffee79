"""Library contexts and key-capacity handling on the GPU (through the C ABI).

- Two host threads, each with its own context (different sort partitions
  and coarse-pair forms) and stream, render stereo frames at the same time;
  every frame equals the one rendered sequentially with the default
  context, bit for bit (tuning changes launch shapes, never results, and
  no call shares device state).
- gs_poll_status reports a binning's required key count and flags an
  overflow; the binding's checked calls retry once with the reported count
  and then equal a render with ample capacity.
- The autograd path plans its capacity without host syncs; a forward that
  overflowed is reported by the next one, which raises and grows the plan.
- The batched step's checked form raises on an overflowed sub-batch.
"""
import ctypes
import threading

import numpy as np
import pytest
import torch

import scenegen
from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def gs():
    need_gpu()
    import paper_2407_00435_amd as g
    return g


def fr_case(seed=81, n=5000):
    sc = scenegen.small_scene(n, seed=seed, sh_degree=3, fr_levels=4, log_scale_mu=-3.4, log_scale_sigma=0.6)
    cams = [scenegen.pinhole(320, 180, scenegen.FR_FOV_DEG, t=(0.03, 0.0, 2.0)),
            scenegen.pinhole(320, 180, scenegen.FR_FOV_DEG, t=(-0.03, 0.0, 2.0))]
    return sc, cams


def test_two_threads_two_contexts_give_the_sequential_frames():
    g = gs()
    sc, cams = fr_case()
    say("two threads, two contexts")
    S, C = g.SceneTensors(sc), g.Cameras(cams)
    gazes = [[scenegen.Fovea(150.0 + 7 * k, 90.0 - 5 * k)] * 2 for k in range(6)]
    cap = 600_000
    refs = []
    for fov in gazes:
        img, num, _ = g.gs_render_foveated(S, C, fov, 16, key_capacity=cap, check=True)
        refs.append(img.clone())
    torch.cuda.synchronize()
    tunings = [dict(radix_part=4096, coarse_packed=0), dict(radix_part=16384, coarse_packed=1)]
    results = [[None] * len(gazes) for _ in tunings]
    errors = []

    def worker(k):
        try:
            ctx = g.binding.Context(torch.cuda.current_device())
            for name, v in tunings[k].items():
                ctx.set_tuning(name, v)
            st = torch.cuda.Stream()
            ws = None
            with ctx, torch.cuda.stream(st):
                for rep in range(2):
                    for j, fov in enumerate(gazes):
                        img = torch.empty_like(refs[0])
                        _, num, ws = g.gs_render_foveated(S, C, fov, 16, key_capacity=cap, image=img,
                                                          workspace=ws)
                        results[k][j] = img
                st.synchronize()
                status, need = ctx.poll_status(ws)
                assert status == 0 and 0 < need <= cap
            ctx.close()
        except Exception as e:  # reported in the main thread
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(len(tunings))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    torch.cuda.synchronize()
    for k in range(len(tunings)):
        for j in range(len(gazes)):
            assert torch.equal(results[k][j], refs[j]), (k, j)


def test_poll_status_and_checked_retry():
    g = gs()
    sc = scenegen.small_scene(3000, seed=82, sh_degree=1, log_scale_mu=-3.3)
    cams = [scenegen.pinhole(200, 140, 60.0, t=(0.0, 0.0, 4.0))]
    say("poll status and retry")
    S, C = g.SceneTensors(sc), g.Cameras(cams)
    splats = g.gs_project(S, C, 16)
    need = int(g.splat_fields(splats)["tiles_touched"].to(torch.int64).sum().item())
    ref = g.gs_render_fwd(S, C, 16, key_capacity=need + 10)
    small = g.gs_render_fwd(S, C, 16, key_capacity=need // 3)
    torch.cuda.synchronize()
    ctx = g.binding.context()
    st, req = ctx.poll_status(small["workspace"])
    assert st == g.binding.GS_ERR_CAPACITY and req == need
    st, req = ctx.poll_status(ref["workspace"])
    assert st == 0 and req == need
    # the overflowed render shows the background and keeps no keys
    assert torch.all(small["image"] == 0) and int(small["ranges"].abs().sum().item()) == 0
    # checked calls retry once with the reported count
    out = g.gs_render_fwd(S, C, 16, key_capacity=need // 3, check=True)
    assert out["capacity"] == need and torch.equal(out["image"], ref["image"])
    bs = g.gs_bin_sort(splats, sc.n, C, 16, key_capacity=100, check=True)
    assert bs["capacity"] == need and torch.equal(bs["ranges"], ref["ranges"])
    assert torch.equal(bs["vals"][:need], ref["vals"][:need])
    fr, fcams = fr_case(seed=83, n=3000)
    SF, CF = g.SceneTensors(fr), g.Cameras(fcams)
    fov = [scenegen.Fovea(150.0, 90.0)] * 2
    big, _, _ = g.gs_render_foveated(SF, CF, fov, 16, key_capacity=2_000_000)
    img, num, ws = g.gs_render_foveated(SF, CF, fov, 16, key_capacity=50, check=True)
    torch.cuda.synchronize()
    assert torch.equal(img, big)
    # a context for a device that does not exist is refused
    h = ctypes.c_void_p()
    assert g.binding.raw_lib().gs_create(ctypes.byref(h), torch.cuda.device_count()) == g.binding.GS_ERR_INVALID


def test_autograd_planned_capacity_reports_an_overflow():
    g = gs()
    sc = scenegen.small_scene(3000, seed=84, sh_degree=3, log_scale_mu=-3.3)
    cams = [scenegen.pinhole(160, 120, 60.0, t=(0.0, 0.0, 4.0))]
    say("planned capacity")
    S, C = g.SceneTensors(sc), g.Cameras(cams)
    names = ("means", "log_scales", "quats", "opacity_logits", "sh")
    params = [S.t[k].clone().requires_grad_(True) for k in names]
    img = g.render(*params, C, 3)
    plan = ("plain", sc.n, 16)
    cap0 = C.key_capacity[plan]
    img.sum().backward()
    img2 = g.render(*params, C, 3)
    torch.cuda.synchronize()
    assert torch.equal(img, img2) and C.key_capacity[plan] == cap0
    # shrink the plan below the keys needed: the forward's image is invalid,
    # and the next forward (after its count has landed) says so
    C.key_capacity[plan] = 64
    bad = g.render(*params, C, 3)
    torch.cuda.synchronize()
    assert torch.all(bad == 0)
    with pytest.raises(g.GsError, match="needed"):
        bad.sum().backward()
    with pytest.raises(g.GsError, match="earlier render"):
        g.render(*params, C, 3)
    assert C.key_capacity[plan] > 64
    img3 = g.render(*params, C, 3)
    torch.cuda.synchronize()
    assert torch.equal(img3, img)


def test_batched_step_checked_form_raises_on_overflow():
    g = gs()
    from paper_2407_00435_amd.batched import BatchedStep
    sc = scenegen.small_scene(4000, seed=85, sh_degree=1, log_scale_mu=-3.0)
    cams = [scenegen.pinhole(160, 120, 60.0, t=(0.0, 0.0, 4.0)),
            scenegen.look_at((1.2, -0.6, -3.3), (0.1, 0.0, 0.0), 131, 97, 55.0)]
    say("batched step overflow")
    S = g.SceneTensors(sc)
    px = sum(c.width * c.height for c in cams)
    target = torch.zeros(3 * px, device="cuda")
    ok = BatchedStep(S, cams, target, 16)
    ok.step(check=True)
    tight = BatchedStep(S, cams, target, 16, key_margin=0.01)
    with pytest.raises(g.GsError, match="capacity"):
        tight.step(check=True)
