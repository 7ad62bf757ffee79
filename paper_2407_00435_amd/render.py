"""Differentiable render: a torch.autograd.Function over the C ABI.

Forward runs projection, binning/sort and compositing in the HIP library
and keeps what the reverse pass needs (splats, sorted ids, tile ranges,
final transmittance and last-contributor index); backward runs the
compositing reverse and the projection reverse in the library.  Torch only
supplies memory and the stream.

Key capacity: given, it is used as is; else it is planned per camera set
(``Cameras.planned_capacity``: one host read the first time, none after) and
every forward leaves a deferred overflow check behind it.  A check that has
found an overflow raises GsError at the next forward with these cameras, or
at this forward's backward if the count has landed by then, and the plan
grows; no forward waits for the device.
"""
from __future__ import annotations

import torch

from . import binding as B


class GaussianRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, cams, sh_degree, tile_size, bg,
                key_capacity):
        scene = B.SceneTensors(means=means.detach(), log_scales=log_scales.detach(),
                               quats=quats.detach(), opacity_logits=opacity_logits.detach(),
                               sh=sh.detach(), sh_degree=sh_degree)
        plan = ("plain", scene.n, tile_size)
        if key_capacity is not None:
            cap = key_capacity
        else:
            # the first render of these cameras projects once to size the capacity
            planned = plan in cams.key_capacity
            cap = cams.planned_capacity(plan, None if planned else B.gs_project(scene, cams, tile_size))
        out = B.gs_render_fwd(scene, cams, tile_size, bg, key_capacity=cap)
        ctx.scene, ctx.cams, ctx.tile, ctx.bg = scene, cams, tile_size, bg
        ctx.save_for_backward(out["splats"], out["vals"], out["ranges"], out["final_T"], out["n_contrib"])
        ctx.num_keys, ctx.capacity = out["num_keys"], out["capacity"]
        ctx.watch = cams.watch(plan, out["num_keys"], out["capacity"]) if key_capacity is None else None
        return out["image"]

    @staticmethod
    def backward(ctx, dL_dimage):
        _raise_if_overflowed(ctx.watch)
        splats, vals, ranges, final_T, n_contrib = ctx.saved_tensors
        g = B.gs_rasterize_bwd(splats, ctx.scene.n, ctx.cams, ctx.tile, vals, ranges, final_T,
                               n_contrib, dL_dimage.contiguous(), ctx.bg)
        pg = B.gs_project_bwd(ctx.scene, ctx.cams, splats, g)
        return (pg["means"], pg["log_scales"], pg["quats"], pg["opacity_logits"], pg["sh"],
                None, None, None, None, None)


def _raise_if_overflowed(watch):
    if watch is not None and watch.overflowed():
        raise B.GsError(B.GS_ERR_CAPACITY, f"the forward needed {watch.required()} keys but had capacity for "
                                           f"{watch.capacity}: its image is invalid (render again)")


def render(means, log_scales, quats, opacity_logits, sh, cams, sh_degree, tile_size=16,
           bg=(0.0, 0.0, 0.0), key_capacity=None):
    """Render all views of ``cams``; returns the planar image buffer
    (view v occupies 3 * W_v * H_v floats, channel-major)."""
    return GaussianRender.apply(means, log_scales, quats, opacity_logits, sh, cams, sh_degree,
                                tile_size, tuple(bg), key_capacity)


class FoveatedRender(torch.autograd.Function):
    """Foveated render (Section 4.1 rings and blend, Section 4.2 filter and
    level versions) with its reverse: gradients for the base parameters and
    the per-level opacity logits and DC colours."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, lvl_opacity_logits, lvl_sh_dc, qbound, cams,
                foveae, sh_degree, tile_size, bg, key_capacity):
        scene = B.SceneTensors(means=means.detach(), log_scales=log_scales.detach(), quats=quats.detach(),
                               opacity_logits=opacity_logits.detach(), sh=sh.detach(), qbound=qbound,
                               lvl_opacity_logits=lvl_opacity_logits.detach(), lvl_sh_dc=lvl_sh_dc.detach(),
                               sh_degree=sh_degree)
        L = scene.n_levels
        t = B.gs_fovea_prep(cams, foveae, tile_size, L)
        splats, lvl = B.gs_project(scene, cams, tile_size, levels=True)
        plan = ("foveated", scene.n, tile_size, L)
        cap = key_capacity if key_capacity is not None else cams.planned_capacity(plan, splats)
        bs = B.gs_bin_sort(splats, scene.n, cams, tile_size, tile_level=t["tile_level"], qbound=scene.t["qbound"],
                           key_capacity=cap)
        _, n_px = cams.tiles(tile_size)
        fT2 = torch.empty((n_px, 2), dtype=torch.float32, device=means.device)
        nc2 = torch.empty((n_px, 2), dtype=torch.int32, device=means.device)
        image = B.gs_rasterize_foveated(splats, lvl, scene.n, scene.t["qbound"], L, cams, tile_size, bs["vals"],
                                        bs["ranges"], t["pix_level"], t["pix_weight"], bg, keep=(fT2, nc2))
        ctx.scene, ctx.cams, ctx.tile, ctx.bg, ctx.tables = scene, cams, tile_size, bg, t
        ctx.save_for_backward(splats, lvl, bs["vals"], bs["ranges"], fT2, nc2)
        ctx.num_keys = bs["num_keys"]
        ctx.watch = cams.watch(plan, bs["num_keys"], bs["capacity"]) if key_capacity is None else None
        return image

    @staticmethod
    def backward(ctx, dL_dimage):
        _raise_if_overflowed(ctx.watch)
        splats, lvl, vals, ranges, fT2, nc2 = ctx.saved_tensors
        sc, t = ctx.scene, ctx.tables
        g, lg = B.gs_rasterize_foveated_bwd(splats, lvl, sc.n, sc.t["qbound"], sc.n_levels, ctx.cams, ctx.tile, vals,
                                            ranges, t["pix_level"], t["pix_weight"], fT2, nc2,
                                            dL_dimage.contiguous(), ctx.bg)
        pg = B.gs_project_bwd_levels(sc, ctx.cams, splats, g, lg)
        return (pg["means"], pg["log_scales"], pg["quats"], pg["opacity_logits"], pg["sh"],
                pg["lvl_opacity_logits"], pg["lvl_sh_dc"], None, None, None, None, None, None, None)


def render_foveated(means, log_scales, quats, opacity_logits, sh, lvl_opacity_logits, lvl_sh_dc, qbound, cams,
                    foveae, sh_degree, tile_size=16, bg=(0.0, 0.0, 0.0), key_capacity=None):
    """Foveated render of the eyes in ``cams`` (planar image buffer)."""
    return FoveatedRender.apply(means, log_scales, quats, opacity_logits, sh, lvl_opacity_logits, lvl_sh_dc,
                                qbound, cams, foveae, sh_degree, tile_size, tuple(bg), key_capacity)


class L1Loss(torch.autograd.Function):
    """Mean absolute error between a render and its target, the training
    objective used with the reverse pass, through the library's fused kernel:
    one pass over both images gives the loss and dL/dimage = sign / n."""

    @staticmethod
    def forward(ctx, image, target):
        image, target = image.detach().contiguous(), target.detach().contiguous()
        grad = torch.empty_like(image)
        loss = torch.empty(1, dtype=torch.float32, device=image.device)
        B.gs_l1_grad(image, target, 1.0 / image.numel(), grad, loss, reset=True)
        ctx.save_for_backward(grad)
        return loss.reshape(())

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return grad * g, None


def l1_loss(image, target):
    """Mean |image - target| (a 0-d tensor) with its reverse."""
    return L1Loss.apply(image, target)
