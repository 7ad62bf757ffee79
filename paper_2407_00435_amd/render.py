"""Differentiable render: a torch.autograd.Function over the C ABI.

Forward runs projection, binning/sort and compositing in the HIP library
and keeps what the reverse pass needs (splats, sorted ids, tile ranges,
final transmittance and last-contributor index); backward runs the
compositing reverse and the projection reverse in the library.  Torch only
supplies memory and the stream.
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
        splats = B.gs_project(scene, cams, tile_size)
        bs = B.gs_bin_sort(splats, scene.n, cams, tile_size, key_capacity=key_capacity)
        out = B.gs_rasterize_fwd(splats, scene.n, cams, tile_size, bs["vals"], bs["ranges"], bg)
        ctx.scene, ctx.cams, ctx.tile, ctx.bg = scene, cams, tile_size, bg
        ctx.save_for_backward(splats, bs["vals"], bs["ranges"], out["final_T"], out["n_contrib"])
        ctx.num_keys, ctx.capacity = bs["num_keys"], bs["capacity"]
        return out["image"]

    @staticmethod
    def backward(ctx, dL_dimage):
        splats, vals, ranges, final_T, n_contrib = ctx.saved_tensors
        g = B.gs_rasterize_bwd(splats, ctx.scene.n, ctx.cams, ctx.tile, vals, ranges, final_T,
                               n_contrib, dL_dimage.contiguous(), ctx.bg)
        pg = B.gs_project_bwd(ctx.scene, ctx.cams, splats, g)
        return (pg["means"], pg["log_scales"], pg["quats"], pg["opacity_logits"], pg["sh"],
                None, None, None, None, None)


def render(means, log_scales, quats, opacity_logits, sh, cams, sh_degree, tile_size=16,
           bg=(0.0, 0.0, 0.0), key_capacity=None):
    """Render all views of ``cams``; returns the planar image buffer
    (view v occupies 3 * W_v * H_v floats, channel-major)."""
    return GaussianRender.apply(means, log_scales, quats, opacity_logits, sh, cams, sh_degree,
                                tile_size, tuple(bg), key_capacity)
