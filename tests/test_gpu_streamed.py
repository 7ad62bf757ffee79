"""Eye-by-eye foveated rendering (the "stream_views" knob of a context):
each eye is binned on the caller's stream and composited on the context's
second stream, so that eye e's compositing overlaps eye e + 1's binning (the
incremental pipelining of Section 5.2 at view granularity).

- Images equal those of the joint one-call render bit for bit (two and
  three eyes of different sizes, tiles 8 and 16), and the reported key count
  is the joint total.
- Each eye gets key_capacity / n_eyes keys: a capacity that holds the total
  but not one eye's share is reported by gs_poll_status as n_eyes times the
  largest per-eye need, and the checked call succeeds after one retry.
- The image lies in the oracle's envelope.
- A graph captured on the caller's stream records both streams' work: its
  replays equal the eager image.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import scenegen
from gpu_util import check_envelope, image_views, need_gpu, pixel_views, say, splat_np, view_slice

pytestmark = pytest.mark.gpu


def gs():
    need_gpu()
    import paper_2407_00435_amd as g
    return g


def eyes_case(n_eyes, seed):
    sc = scenegen.small_scene(5000, seed=seed, sh_degree=3, fr_levels=4, log_scale_mu=-3.4, log_scale_sigma=0.6)
    sizes = [(300, 170), (256, 200), (190, 150)][:n_eyes]
    cams = [scenegen.pinhole(w, h, scenegen.FR_FOV_DEG, t=(0.03 * (1 - 2 * (k % 2)), 0.01 * k, 2.0))
            for k, (w, h) in enumerate(sizes)]
    fov = [scenegen.Fovea(0.5 * w + 10 * k, 0.45 * h) for k, (w, h) in enumerate(sizes)]
    return sc, cams, fov


def streamed(g, on):
    g.context().set_tuning("stream_views", 1 if on else 0)


@pytest.mark.parametrize("n_eyes,tile", [(2, 16), (3, 16), (2, 8)])
def test_streamed_equals_joint(n_eyes, tile):
    g = gs()
    sc, cams, fov = eyes_case(n_eyes, 71 + n_eyes + tile)
    say("streamed eyes", n_eyes, tile)
    C, S = g.Cameras(cams), g.SceneTensors(sc)
    cap = 600_000
    ref, num_ref, _ = g.gs_render_foveated(S, C, fov, tile, key_capacity=cap, check=True)
    try:
        streamed(g, True)
        img, num, ws = g.gs_render_foveated(S, C, fov, tile, key_capacity=cap, check=True)
        img2, num2, _ = g.gs_render_foveated(S, C, fov, tile, key_capacity=cap, workspace=ws)
        torch.cuda.synchronize()
    finally:
        streamed(g, False)
    assert int(num.item()) == int(num_ref.item())
    assert torch.equal(img, ref)
    assert torch.equal(img2, ref)
    say(f"{int(num.item())} keys")


def test_streamed_capacity_is_per_eye():
    g = gs()
    sc, cams, fov = eyes_case(2, 81)
    # the left eye sees the scene, the right one mostly empty space
    cams[1] = scenegen.look_at((0.0, 0.0, 2.0), (0.0, 0.0, 9.0), 256, 200, scenegen.FR_FOV_DEG)
    C, S = g.Cameras(cams), g.SceneTensors(sc)
    say("streamed per-eye capacity")
    ref, num_ref, _ = g.gs_render_foveated(S, C, fov, 16, key_capacity=600_000)
    torch.cuda.synchronize()
    total = int(num_ref.item())
    per_eye = [int(g.gs_render_foveated(S, g.Cameras([c]), [f], 16, key_capacity=600_000)[1].item())
               for c, f in zip(cams, fov)]
    assert sum(per_eye) == total and max(per_eye) > 0.6 * total, per_eye
    cap = total + 16  # holds the total, not twice the larger eye
    try:
        streamed(g, True)
        _, num, ws = g.gs_render_foveated(S, C, fov, 16, key_capacity=cap)
        torch.cuda.synchronize()
        st, need = g.context().poll_status(ws)
        assert st == g.binding.GS_ERR_CAPACITY
        assert need == 2 * max(per_eye)
        assert int(num.item()) == total
        img, num, _ = g.gs_render_foveated(S, C, fov, 16, key_capacity=cap, check=True)
        torch.cuda.synchronize()
    finally:
        streamed(g, False)
    assert torch.equal(img, ref)


def test_streamed_matches_oracle():
    g = gs()
    sc, cams, fov = eyes_case(2, 83)
    say("streamed against the oracle")
    C, S = g.Cameras(cams), g.SceneTensors(sc)
    t = g.gs_fovea_prep(C, fov, 16, 4)
    splats, lvl = g.gs_project(S, C, 16, levels=True)
    try:
        streamed(g, True)
        img, _, _ = g.gs_render_foveated(S, C, fov, 16, key_capacity=600_000, check=True)
        torch.cuda.synchronize()
    finally:
        streamed(g, False)
    sp = splat_np(splats)
    lvn = lvl.cpu().numpy()
    sizes = [(c.width, c.height) for c in cams]
    imgs = image_views(img, sizes)
    pl = pixel_views(t["pix_level"], sizes)
    pw = pixel_views(t["pix_weight"], sizes)
    for v, cam in enumerate(cams):
        proj = oracle.splats_to_proj(view_slice(sp, v))
        proj["lvl_opacity"] = lvn[v, :, :, 3].T.astype(np.float64).copy()
        proj["lvl_color"] = lvn[v, :, :, 0:3].transpose(1, 0, 2).astype(np.float64).copy()
        ref = oracle.composite(proj, cam.width, cam.height, qbound=sc.qbound, pix_lo=pl[v].ravel(),
                               pix_w=pw[v].ravel().astype(np.float64), levels=True)
        err, namb = check_envelope(imgs[v], ref)
        say(f"eye {v}: max err {err:.3g}, ambiguous {namb}")


def test_streamed_graph_replays():
    g = gs()
    B = g.binding
    sc, cams, fov = eyes_case(2, 85)
    say("streamed under graph capture")
    C, S = g.Cameras(cams), g.SceneTensors(sc)
    cap = 600_000
    ref, _, _ = g.gs_render_foveated(S, C, fov, 16, key_capacity=cap)
    torch.cuda.synchronize()
    nb = g.gs_render_workspace_bytes(C, S.n, S.n_levels, 16, cap)
    ws = B._ws(nb)
    _, n_px = C.tiles(16)
    img = torch.zeros(3 * n_px, dtype=torch.float32, device="cuda")
    num = torch.zeros(1, dtype=torch.int64, device="cuda")
    fa = B._foveae(fov)
    bg = (ctypes.c_float * 3)(0.0, 0.0, 0.0)
    st = S.struct(levels=True)
    stream = torch.cuda.Stream()

    def call():
        B._check(g.lib().gs_render_foveated(ctypes.byref(st), C.hp, C.dp, ctypes.cast(fa, B._PF), C.n, 16,
                                            ctypes.cast(bg, B._VP), B._ptr(img), cap, B._ptr(num), ws[1], ws[2],
                                            ctypes.c_void_p(stream.cuda_stream)))

    try:
        streamed(g, True)
        torch.cuda.synchronize()
        call()  # eager first: makes the context's second stream
        stream.synchronize()
        assert torch.equal(img, ref)
        with g.Graph.capture(stream) as cap_g:
            call()
        for k in range(3):
            img.zero_()
            torch.cuda.synchronize()
            cap_g.graph.launch(stream)
            stream.synchronize()
            assert torch.equal(img, ref), k
            _ = (img * 2.0).sum().item()  # eager work between replays
        cap_g.graph.close()
    finally:
        streamed(g, False)
