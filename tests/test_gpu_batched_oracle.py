"""The batched training step against the FP64 oracle (through the C ABI).

Five views of mixed resolution and two foveated eyes, every stage of each
batched in one call (projection reads each point once for all views, one
global tile space, one sort, one compositing launch, one reverse launch),
replayed from a recorded graph: the views' images against the oracle's full
FP64 render (projection and compositing), the eyes' images against the
oracle's FP64 foveated compositing given the GPU's fovea tables (the tables
themselves are checked against the oracle in the parity tests), and the
parameter gradients of the step's L1 loss against the oracle's reverse of
the views plus its foveated reverse of the eyes, fed with the step's own
dL/dimage (the sign of each pixel's residual is the GPU image's).

Bars: images within 2e-4 of the oracle's branch envelope; gradients within
1e-3 relative L2 per parameter group and, point by point, within 1e-3 of the
point's own gradient norm plus 1e-4 of the root mean square norm, except
for at most 0.2 % of the points (a pair whose alpha or extent decision sits at
its threshold flips between float32 and float64, and a flipped pair moves
its point's gradient by its whole contribution).
"""
import numpy as np
import pytest
import torch

import oracle
import scenegen
from gpu_util import check_envelope, image_views, need_gpu, per_point_check, pixel_views, rel_l2, say

pytestmark = pytest.mark.gpu


def gs():
    need_gpu()
    import paper_2407_00435_amd as g
    return g


def views():
    return [scenegen.pinhole(120, 68, 60.0, t=(0.0, 0.0, 4.0)),
            scenegen.look_at((1.2, -0.6, -3.3), (0.1, 0.0, 0.0), 96, 54, 55.0),
            scenegen.look_at((-2.5, 0.4, -2.9), (0.0, 0.1, 0.0), 64, 36, 62.0),
            scenegen.look_at((0.3, 2.2, -3.1), (0.0, 0.0, 0.2), 80, 45, 58.0),
            scenegen.look_at((3.0, -0.2, 2.4), (0.0, 0.0, 0.0), 77, 101, 65.0)]


def as_f64(sc):
    return scenegen.Scene(*(np.asarray(getattr(sc, k), np.float64)
                            for k in ("means", "log_scales", "quats", "opacity_logits", "sh")),
                          sc.sh_degree, sc.qbound, np.asarray(sc.lvl_opacity_logits, np.float64),
                          np.asarray(sc.lvl_sh_dc, np.float64))


@pytest.mark.parametrize("batch_views", [None, 2])
def test_batched_step_matches_oracle(batch_views):
    g = gs()
    from paper_2407_00435_amd.batched import BatchedStep
    sc = scenegen.small_scene(2500, seed=33, sh_degree=3, fr_levels=4, log_scale_mu=-3.3, log_scale_sigma=0.5)
    cams = views()
    eyes = [scenegen.pinhole(112, 64, scenegen.FR_FOV_DEG, t=(0.03, 0.0, 2.5)),
            scenegen.pinhole(112, 64, scenegen.FR_FOV_DEG, t=(-0.03, 0.0, 2.5))]
    fov = [scenegen.Fovea(50.0, 30.0, rings_deg=(10.0, 20.0, 30.0), band_deg=3.5),
           scenegen.Fovea(62.0, 33.0, rings_deg=(10.0, 20.0, 30.0), band_deg=3.5)]
    say("batched step against the oracle", batch_views)
    S = g.SceneTensors(sc)
    rng = np.random.default_rng(7)
    px = sum(c.width * c.height for c in cams)
    epx = sum(c.width * c.height for c in eyes)
    target = torch.from_numpy(rng.uniform(0.0, 1.0, 3 * px).astype(np.float32)).cuda()
    eye_target = torch.from_numpy(rng.uniform(0.0, 1.0, 3 * epx).astype(np.float32)).cuda()
    step = BatchedStep(S, cams, target, 16, batch_views, eyes, fov, eye_target=eye_target)
    step.capture()
    step.replay()
    torch.cuda.synchronize()
    assert step.keys_ok()
    # views: full FP64 render
    imgs = image_views(step.image, [(c.width, c.height) for c in cams])
    for v, cam in enumerate(cams):
        ref = oracle.render(sc, cam, margins=(2e-4, 2e-4, 1e-4, 1e-4))
        err, namb = check_envelope(imgs[v], ref, max_unresolved_frac=1e-3)
        say(f"view {v} {cam.width}x{cam.height}: max err {err:.3g}, ambiguous {namb}")
    # eyes: FP64 projection with the level versions, foveated compositing
    # with the GPU's tables
    esz = [(c.width, c.height) for c in eyes]
    eimgs = image_views(step.eye_image, esz)
    pl = pixel_views(step.eye_bufs["pix_level"][:epx], esz)
    pw = pixel_views(step.eye_bufs["pix_weight"][:epx], esz)
    for v, cam in enumerate(eyes):
        pr = oracle.project(sc, cam, levels=True)
        ref = oracle.composite(pr, cam.width, cam.height, qbound=sc.qbound, pix_lo=pl[v].ravel(),
                               pix_w=pw[v].ravel().astype(np.float64), levels=True,
                               margins=(2e-4, 2e-4, 1e-4, 1e-4))
        err, namb = check_envelope(eimgs[v], ref, max_unresolved_frac=1e-3)
        say(f"eye {v}: max err {err:.3g}, ambiguous {namb}")
    # gradients of the step's loss: the views' reverse plus the eyes'
    # foveated reverse, with the step's own dL/dimage
    dl = step.dL.cpu().numpy().astype(np.float64)
    dls, off = [], 0
    for cam in cams:
        W, H = cam.width, cam.height
        dls.append(dl[3 * off:3 * (off + W * H)].reshape(3, H, W))
        off += W * H
    sc64 = as_f64(sc)
    ref = oracle.reverse(sc64, cams, dls)
    edl = step.eye_dL.cpu().numpy().astype(np.float64)
    edls, tabs, off = [], [], 0
    for v, cam in enumerate(eyes):
        W, H = cam.width, cam.height
        edls.append(edl[3 * off:3 * (off + W * H)].reshape(3, H, W))
        tabs.append((pl[v].ravel(), pw[v].ravel().astype(np.float64)))
        off += W * H
    fref = oracle.fr_reverse(sc64, eyes, tabs, edls)
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        ref[k] = ref[k] + fref[k]
    for k in ("lvl_opacity_logits", "lvl_sh_dc"):
        ref[k] = fref[k]
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "lvl_opacity_logits", "lvl_sh_dc"):
        gpu = step.grads[k].cpu().numpy().astype(np.float64)
        r = ref[k]
        if k.startswith("lvl_"):  # [L][n][...] -> points first
            gpu, r = np.moveaxis(gpu, 1, 0), np.moveaxis(r, 1, 0)
        e = rel_l2(gpu, r)
        nbad, worst = per_point_check(gpu, r)
        say(f"{k}: rel L2 {e:.2e}, points over the per-point bar {nbad} of {sc.n}, worst {worst:.2e}")
        assert e < 1e-3, (k, e)
        assert nbad <= 0.002 * sc.n, (k, nbad)
