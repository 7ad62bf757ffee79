"""MI355X (gfx950) Gaussian-splatting rasterizer: thin Python binding over the
C ABI of ``libgsmi.so`` (see ``include/gs.h``).

Every step of the render runs in the library's HIP kernels; this package only
marshals torch device tensors into the C calls.  Importing it loads the
library and fails loudly if it has not been built.
"""
from .binding import (  # noqa: F401
    Cameras, SceneTensors, GsError, lib, raw_lib, lib_path, Context, context, gs_get_tuning,
    gs_project, gs_bin_sort, gs_rasterize_fwd, gs_rasterize_bwd, gs_project_bwd,
    gs_fovea_prep, gs_rasterize_foveated, gs_render_foveated, gs_render_fwd,
    gs_workspace_bytes, gs_render_workspace_bytes, gs_tile_count, splat_fields, gs_sort_pairs, gs_set_tuning,
    gs_sort_pairs_static, gs_hvsq_pooling, gs_hvsq,
    gs_l1_grad, gs_ce_score, gs_select_lowest, gs_weighted_scale, Graph,
    gs_rasterize_foveated_bwd, gs_project_bwd_levels,
)
from .render import GaussianRender, render, FoveatedRender, render_foveated, L1Loss, l1_loss  # noqa: F401
