"""FP64 CPU oracle (test infrastructure only).

Plain, slow reference for the Gaussian-splatting hot path; see the header of
``gs_oracle.c`` for what each routine follows in the paper.  Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import this package.
It shares no code with the HIP library and does not import it.

Parity unpinned: none of the routines below; each is pinned by the
``tests/test_oracle_*.py`` suite against closed forms, brute force or
finite differences.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB = os.path.join(_HERE, "libgs_oracle.so")
_lib = None

DEFAULT_MARGINS = (2e-5, 2e-5, 1e-5, 1e-5)  # dq, de, dT, ddom


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, FP64, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB)
        _lib.oc_bin_f32.restype = ctypes.c_int64
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, np.float32)


def _f64(a):
    return np.ascontiguousarray(a, np.float64)


def cam_row(cam) -> np.ndarray:
    return np.ascontiguousarray(cam.as_row() if hasattr(cam, "as_row") else cam, np.float64)


def sh_basis(degree: int, direction) -> np.ndarray:
    d = _f64(direction)
    Y = np.zeros((degree + 1) ** 2)
    lib().oc_sh_basis(ctypes.c_int(degree), _p(d), _p(Y))
    return Y


def sh_basis_grad(degree: int, direction):
    """(Y [K], dY/d dir [K, 3]) of the real SH basis at a unit direction, from
    the polynomial form of the basis (the reverse pass's derivative)."""
    d = _f64(direction)
    K = (degree + 1) ** 2
    Y = np.zeros(K)
    dY = np.zeros((K, 3))
    lib().oc_sh_basis_grad(ctypes.c_int(degree), _p(d), _p(Y), _p(dY))
    return Y, dY


def project(scene, cam, levels: bool = False) -> dict:
    """FP64 projection of every Gaussian for one camera."""
    n = scene.n
    out = dict(mean2d=np.zeros((n, 2)), cov2d=np.zeros((n, 3)), conic=np.zeros((n, 3)),
               depth=np.zeros(n), opacity=np.zeros(n), color=np.zeros((n, 3)),
               radius=np.zeros(n, np.int32), visible=np.zeros(n, np.uint8))
    L = 0
    lo = lc = None
    if levels and scene.qbound is not None:
        L = (scene.lvl_opacity_logits.shape[0] if scene.lvl_opacity_logits is not None
             else int(scene.qbound.max()))
        out["lvl_opacity"] = lo = np.zeros((L, n))
        out["lvl_color"] = lc = np.zeros((L, n, 3))
    lvl_logits = None if scene.lvl_opacity_logits is None else _f64(scene.lvl_opacity_logits)
    lvl_dc = None if scene.lvl_sh_dc is None else _f64(scene.lvl_sh_dc)
    args = [_f64(scene.means), _f64(scene.log_scales), _f64(scene.quats),
            _f64(scene.opacity_logits), _f64(scene.sh)]
    crow = cam_row(cam)
    lib().oc_project(ctypes.c_int(n), ctypes.c_int(scene.sh_degree), *[_p(a) for a in args],
                     _p(crow), _p(out["mean2d"]), _p(out["cov2d"]), _p(out["conic"]),
                     _p(out["depth"]), _p(out["opacity"]), _p(out["color"]), _p(out["radius"]),
                     _p(out["visible"]), ctypes.c_int(L), _p(lvl_logits if L else None),
                     _p(lvl_dc if L else None), _p(lo), _p(lc))
    if L:
        # Section 4.2: a point has a version only at the levels t <= m_i (its
        # quality bound); at the levels above, its opacity is zero
        qb = np.asarray(scene.qbound).astype(np.int64)
        for t in range(1, L + 1):
            lo[t - 1][qb < t] = 0.0
    return out


def bin_f32(mean2d, radius, depth, widths, heights, tile: int,
            tile_level_lo=None, qbound=None) -> dict:
    """Stage-wise binning on float32 inputs ([V][n] arrays)."""
    mean2d = _f32(mean2d)
    radius = np.ascontiguousarray(radius, np.int32)
    depth = _f32(depth)
    V = len(widths)
    n = radius.size // V
    widths = np.ascontiguousarray(widths, np.int32)
    heights = np.ascontiguousarray(heights, np.int32)
    tll = None if tile_level_lo is None else np.ascontiguousarray(tile_level_lo, np.uint8)
    qb = None if qbound is None else np.ascontiguousarray(qbound, np.uint8)
    hits = np.zeros(V * n, np.uint32)
    total = lib().oc_bin_f32(V, n, _p(mean2d), _p(radius), _p(depth), _p(widths), _p(heights),
                             tile, _p(tll), _p(qb), _p(hits), None, None, None, ctypes.c_int64(0))
    tiles = int(sum(((w + tile - 1) // tile) * ((h + tile - 1) // tile)
                    for w, h in zip(widths, heights)))
    keys = np.zeros(max(total, 1), np.uint64)
    vals = np.zeros(max(total, 1), np.uint32)
    ranges = np.zeros((tiles, 2), np.uint32)
    got = lib().oc_bin_f32(V, n, _p(mean2d), _p(radius), _p(depth), _p(widths), _p(heights),
                           tile, _p(tll), _p(qb), _p(hits), _p(keys), _p(vals), _p(ranges),
                           ctypes.c_int64(total))
    assert got == total
    return dict(hits=hits.reshape(V, n), keys=keys[:total], vals=vals[:total], ranges=ranges,
                num_keys=int(total))


def composite(proj: dict, W: int, H: int, bg=(0.0, 0.0, 0.0), pixels=None,
              margins=DEFAULT_MARGINS, max_leaves: int = 64, nthreads: int = 0,
              qbound=None, pix_lo=None, pix_w=None, levels: bool = False) -> dict:
    """Per-pixel compositing (Eq. 1a) of projected splats given as float64
    arrays (mean2d, conic, depth, opacity, color, radius).  ``pixels`` is an
    (m, 2) array of (x, y) or None for the full image (returned as (H, W, 3))."""
    n = proj["depth"].shape[0]
    m2, cn, dp, op, cl = (_f64(proj[k]) for k in ("mean2d", "conic", "depth", "opacity", "color"))
    rad = np.ascontiguousarray(proj["radius"], np.int32)
    lo = lc = None
    if levels:
        lo = _f64(proj["lvl_opacity"]) if proj.get("lvl_opacity") is not None else None
        lc = _f64(proj["lvl_color"]) if proj.get("lvl_color") is not None else None
    px = None if pixels is None else np.ascontiguousarray(pixels, np.int32)
    npx = W * H if px is None else px.shape[0]
    out = dict(rgb=np.zeros((npx, 3)), rgb_min=np.zeros((npx, 3)), rgb_max=np.zeros((npx, 3)),
               T=np.zeros(npx), last_id=np.zeros(npx, np.int32), dom_id=np.zeros(npx, np.int32),
               amb=np.zeros(npx, np.int32), n_blend=np.zeros(npx, np.int32),
               last_set=np.zeros((npx, 4), np.int32), dom_set=np.zeros((npx, 4), np.int32))
    bgv = _f64(bg)
    mg = _f64(margins)
    qb = None if qbound is None else np.ascontiguousarray(qbound, np.uint8)
    plo = None if pix_lo is None else np.ascontiguousarray(pix_lo, np.uint8)
    pw = None if pix_w is None else _f64(pix_w)
    lib().oc_composite(ctypes.c_int(n), _p(m2), _p(cn), _p(dp), _p(op), _p(cl), _p(rad),
                       ctypes.c_int(W), ctypes.c_int(H), _p(bgv), _p(qb), _p(lo), _p(lc),
                       _p(plo), _p(pw), ctypes.c_int(npx), _p(px), _p(mg),
                       ctypes.c_int(max_leaves),
                       _p(out["rgb"]), _p(out["rgb_min"]), _p(out["rgb_max"]), _p(out["T"]),
                       _p(out["last_id"]), _p(out["dom_id"]), _p(out["amb"]), _p(out["n_blend"]),
                       _p(out["last_set"]), _p(out["dom_set"]), ctypes.c_int(nthreads))
    if px is None:
        for k in ("rgb", "rgb_min", "rgb_max"):
            out[k] = out[k].reshape(H, W, 3)
        for k in ("T", "last_id", "dom_id", "amb", "n_blend"):
            out[k] = out[k].reshape(H, W)
        for k in ("last_set", "dom_set"):
            out[k] = out[k].reshape(H, W, 4)
    return out


def render(scene, cam, bg=(0.0, 0.0, 0.0), pixels=None, **kw) -> dict:
    """O1: full FP64 render (projection then compositing)."""
    pr = project(scene, cam)
    out = composite(pr, int(cam.width), int(cam.height), bg=bg, pixels=pixels, **kw)
    out["proj"] = pr
    return out


def fovea(cam, fov, n_levels: int, tile: int, eps: float = 1e-3) -> dict:
    W, H = int(cam.width), int(cam.height)
    tiles = ((W + tile - 1) // tile) * ((H + tile - 1) // tile)
    out = dict(pix_lo=np.zeros(W * H, np.uint8), pix_w=np.zeros(W * H), ecc=np.zeros(W * H),
               pix_amb=np.zeros(W * H, np.uint8), tile_lo=np.zeros(tiles, np.uint8),
               tile_hi=np.zeros(tiles, np.uint8), tile_amb=np.zeros(tiles, np.uint8))
    crow = cam_row(cam)
    frow = _f64(fov.as_row() if hasattr(fov, "as_row") else fov)
    lib().oc_fovea(_p(crow), _p(frow), ctypes.c_int(n_levels), ctypes.c_int(tile),
                   ctypes.c_double(eps), _p(out["pix_lo"]), _p(out["pix_w"]), _p(out["ecc"]),
                   _p(out["pix_amb"]), _p(out["tile_lo"]), _p(out["tile_hi"]), _p(out["tile_amb"]))
    return out


def composite_bwd(proj: dict, W: int, H: int, dL_dimg, bg=(0.0, 0.0, 0.0)) -> dict:
    """Reverse of the compositing: per-Gaussian d mean2d, d conic, d opacity,
    d colour for dL/dI given as (3, H, W)."""
    n = proj["depth"].shape[0]
    m2, cn, dp, op, cl = (_f64(proj[k]) for k in ("mean2d", "conic", "depth", "opacity", "color"))
    rad = np.ascontiguousarray(proj["radius"], np.int32)
    g = _f64(dL_dimg)
    out = dict(mean2d=np.zeros((n, 2)), conic=np.zeros((n, 3)), opacity=np.zeros(n),
               color=np.zeros((n, 3)))
    bgv = _f64(bg)
    lib().oc_composite_bwd(ctypes.c_int(n), _p(m2), _p(cn), _p(dp), _p(op), _p(cl), _p(rad),
                           ctypes.c_int(W), ctypes.c_int(H), _p(bgv), _p(g),
                           _p(out["mean2d"]), _p(out["conic"]), _p(out["opacity"]),
                           _p(out["color"]))
    return out


def project_bwd(scene, cam, g: dict, acc: dict | None = None) -> dict:
    """Reverse of the projection for one camera; adds into ``acc``."""
    n = scene.n
    K = (scene.sh_degree + 1) ** 2
    if acc is None:
        acc = dict(means=np.zeros((n, 3)), log_scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
                   opacity_logits=np.zeros(n), sh=np.zeros((n, K, 3)))
    args = [_f64(scene.means), _f64(scene.log_scales), _f64(scene.quats),
            _f64(scene.opacity_logits), _f64(scene.sh)]
    crow = cam_row(cam)
    gm, gc, go, gcl = (_f64(g[k]) for k in ("mean2d", "conic", "opacity", "color"))
    lib().oc_project_bwd(ctypes.c_int(n), ctypes.c_int(scene.sh_degree), *[_p(a) for a in args],
                         _p(crow), _p(gm), _p(gc), _p(go), _p(gcl),
                         _p(acc["means"]), _p(acc["log_scales"]), _p(acc["quats"]),
                         _p(acc["opacity_logits"]), _p(acc["sh"]))
    return acc


def reverse(scene, cams, dL_dimgs, bg=(0.0, 0.0, 0.0)) -> dict:
    """O4: gradients of sum_v <dL_dimg_v, I_v> w.r.t. all parameters."""
    acc = None
    for cam, g in zip(cams, dL_dimgs):
        pr = project(scene, cam)
        gs = composite_bwd(pr, int(cam.width), int(cam.height), g, bg)
        acc = project_bwd(scene, cam, gs, acc)
    return acc


def splats_to_proj(splats: dict) -> dict:
    """Upcast float32 splat fields (as returned by the HIP path) to the float64
    dict the compositing routines take."""
    return dict(mean2d=_f64(splats["mean2d"]), conic=_f64(splats["conic"]),
                depth=_f64(splats["depth"]), opacity=_f64(splats["opacity"]),
                color=_f64(splats["color"]),
                radius=np.ascontiguousarray(splats["radius"], np.int32),
                lvl_opacity=None if splats.get("lvl_opacity") is None else _f64(splats["lvl_opacity"]),
                lvl_color=None if splats.get("lvl_color") is None else _f64(splats["lvl_color"]))


# ---------------------------------------------------------------------------
# Efficiency-aware pruning (Section 3).  Plain numpy, written from the
# definitions; the point of these is to be read against the paper.

def ce_score(dominated, hits) -> np.ndarray:
    """Computational efficiency of every point (Section 3.2, the CE equation):
    CE_i = Val_i / Comp_i per view -- Val the pixels the point dominates,
    Comp the tiles that intersect and use it -- and the final CE is the
    maximum over the views (Section 3.2 prefers the maximum to the mean).
    A view in which the point uses no tile contributes 0.  The ratio is
    taken in float32 (correctly rounded division of exactly representable
    counts), the precision the selection below orders by."""
    dom = np.asarray(dominated, dtype=np.int64)
    hit = np.asarray(hits, dtype=np.int64)
    if dom.ndim == 1:
        dom, hit = dom[None], hit[None]
    V, n = dom.shape
    out = np.zeros(n, dtype=np.float32)
    for v in range(V):
        used = hit[v] > 0
        ratio = np.zeros(n, dtype=np.float32)
        ratio[used] = dom[v, used].astype(np.float32) / hit[v, used].astype(np.float32)
        out = np.maximum(out, ratio)
    return out


def select_lowest(ce, k: int):
    """The k points with the lowest CE, removed first by the pruning step of
    Section 3.4 (R = 10 % of the points per round there).  Ties in CE are
    broken by the lower point index.  Returns (mask [n] uint8, indices [k]
    ascending)."""
    ce = np.asarray(ce, dtype=np.float32)
    n = ce.shape[0]
    k = max(0, min(int(k), n))
    order = np.lexsort((np.arange(n), ce))  # by CE, then by index
    chosen = np.sort(order[:k]).astype(np.uint32)
    mask = np.zeros(n, dtype=np.uint8)
    mask[chosen] = 1
    return mask, chosen


def weighted_scale(log_scales, hits, threshold: float, gamma: float = 1.0):
    """Weighted Scale (Section 3.3): WS = (1/N) sum_i S_i G_i with
    G_i = [U_i > T] (U_i - T), U_i the tiles point i is used in.  Readings:
    S_i, the largest span of the point's ellipse, is three standard
    deviations along its longest axis, 3 max_k exp(log_scale_ik); with a
    batch of V views, U is taken per view and WS is averaged over the views.
    Returns (gamma * WS, d(gamma * WS)/d log_scales) in float64; the
    gradient flows through S only (G is a count), to the axis attaining the
    maximum (the first one on ties)."""
    ls = np.asarray(log_scales, dtype=np.float64).reshape(-1, 3)
    U = np.asarray(hits, dtype=np.float64)
    if U.ndim == 1:
        U = U[None]
    V, n = U.shape
    sc = np.exp(ls)
    axis = np.argmax(sc, axis=1)
    S = 3.0 * sc[np.arange(n), axis]
    G = np.where(U > threshold, U - threshold, 0.0).sum(axis=0)
    ws = gamma * float((S * G).sum()) / (n * V)
    grad = np.zeros_like(ls)
    grad[np.arange(n), axis] = gamma * G * S / (n * V)
    return ws, grad


# ---------------------------------------------------------------------------
# Reverse of the foveated render (Section 4.1 blending, Section 4.2 filtering
# and selective multi-versioning), as a composition of the plain reverse.

def level_scene(scene, t: int):
    """Level t (1-based) of a foveated scene as a plain scene: the points
    with quality bound m >= t (Section 4.2: a point takes part in level t iff
    t <= m), with the level's opacity logit and DC colour (the non-DC SH
    coefficients, position and shape are shared).  Returns (scene_t,
    indices into the full scene)."""
    idx = np.nonzero(np.asarray(scene.qbound) >= t)[0]
    sub = scene.subset(idx)
    if scene.lvl_opacity_logits is not None:
        sub.opacity_logits = np.asarray(scene.lvl_opacity_logits[t - 1][idx], dtype=np.float64)
    sub.sh = np.array(sub.sh, dtype=np.float64)
    if scene.lvl_sh_dc is not None:
        sub.sh[:, 0, :] = np.asarray(scene.lvl_sh_dc[t - 1][idx], dtype=np.float64)
    return sub, idx


def level_weights(pix_lo, pix_w, t: int) -> np.ndarray:
    """Per-pixel weight of level t in the blended image: 1 - w at the pixel's
    lower level and w at the next one (Section 4.1), 1 at the lower level
    outside the bands."""
    lo = np.asarray(pix_lo, dtype=np.int64)
    w = np.asarray(pix_w, dtype=np.float64)
    return np.where(lo == t, 1.0 - w, 0.0) + np.where((lo + 1 == t) & (w > 0), w, 0.0)


def fr_reverse(scene, cams, tables, dL_dimgs, bg=(0.0, 0.0, 0.0)) -> dict:
    """Gradients of sum_v <dL_v, I_v> for the foveated images I_v, with
    tables[v] = (pix_lo [H*W], pix_w [H*W]).  The blended image is
    sum_t weight_t(p) * (the plain render of level t's scene) at p, so the
    gradient is the sum over levels of the plain reverse of level t's scene
    under dL * weight_t, scattered back to the full scene: shared parameters
    (means, log-scales, quaternions, non-DC SH) sum over levels; opacity
    logits and DC go to the level versions when the scene has them (else to
    the base).  Returns the five base arrays plus lvl_opacity_logits and
    lvl_sh_dc (None when the scene shares the base)."""
    n, K = scene.n, (scene.sh_degree + 1) ** 2
    L = int(np.max(scene.qbound))
    out = dict(means=np.zeros((n, 3)), log_scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
               opacity_logits=np.zeros(n), sh=np.zeros((n, K, 3)),
               lvl_opacity_logits=None if scene.lvl_opacity_logits is None
               else np.zeros(np.asarray(scene.lvl_opacity_logits).shape),
               lvl_sh_dc=None if scene.lvl_sh_dc is None else np.zeros(np.asarray(scene.lvl_sh_dc).shape))
    for t in range(1, L + 1):
        sub, idx = level_scene(scene, t)
        if len(idx) == 0:
            continue
        dls = []
        for cam, (lo, w), g in zip(cams, tables, dL_dimgs):
            wt = level_weights(lo, w, t).reshape(int(cam.height), int(cam.width))
            dls.append(np.asarray(g, dtype=np.float64) * wt[None])
        gt = reverse(sub, cams, dls, bg)
        for k in ("means", "log_scales", "quats"):
            out[k][idx] += gt[k]
        out["sh"][idx, 1:, :] += gt["sh"][:, 1:, :]
        if out["lvl_sh_dc"] is not None:
            out["lvl_sh_dc"][t - 1][idx] += gt["sh"][:, 0, :]
        else:
            out["sh"][idx, 0, :] += gt["sh"][:, 0, :]
        if out["lvl_opacity_logits"] is not None:
            out["lvl_opacity_logits"][t - 1][idx] += gt["opacity_logits"]
        else:
            out["opacity_logits"][idx] += gt["opacity_logits"]
    return out


def fr_render(scene, cam, pix_lo, pix_w, bg=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Foveated FP64 render (projection with the level versions, then the
    per-level compositing and blend); (H, W, 3)."""
    pr = project(scene, cam, levels=True)
    out = composite(pr, int(cam.width), int(cam.height), bg=bg, qbound=scene.qbound, pix_lo=pix_lo,
                    pix_w=np.asarray(pix_w, dtype=np.float64), levels=True, nthreads=1)
    return out["rgb"]


# ---------------------------------------------------------------------------
# HVSQ (Section 2.2, Eq. 2) on the stated feature reading (colour channels,
# square windows whose half-width grows linearly with eccentricity).

def hvsq_radius(cam, fov, rho: float, eps: float = 1e-4):
    """Pooling half-width of every pixel: floor(rho * eccentricity in
    degrees), with the eccentricity of Section 4.1 (the angle between the
    pixel's and the gaze pixel's rays).  Returns (radius int32 [H*W],
    ambiguous uint8 [H*W]: rho * ecc within eps of an integer, where a
    float32 evaluation may land on the other side)."""
    f = fovea(cam, fov, 1, 16)
    x = rho * f["ecc"]
    rad = np.floor(x).astype(np.int32)
    frac = x - np.floor(x)
    amb = ((frac < eps) | (frac > 1.0 - eps)).astype(np.uint8)
    return rad, amb


def hvsq(img_a, img_r, radius, W: int, H: int, region=None, n_regions: int = 0, grad_region=None,
         want_terms: bool = False) -> dict:
    """HVSQ of altered image img_a against reference img_r, both [3][H][W]
    (any array shape with 3*H*W elements), radius [H*W] pooling half-widths,
    region [H*W] (1..n_regions, optional).  Returns per-region sums and
    counts of the per-pixel terms (index n_regions = the whole image), the
    means ("hvsq"), optionally per-pixel terms and the gradient of the mean
    over region grad_region (0 = whole image) with respect to img_a."""
    a = _f64(img_a).reshape(3, H, W)
    r = _f64(img_r).reshape(3, H, W)
    rad = np.ascontiguousarray(radius, np.int32).reshape(-1)
    reg = None if region is None else np.ascontiguousarray(region, np.uint8).reshape(-1)
    sums = np.zeros(n_regions + 1)
    counts = np.zeros(n_regions + 1)
    terms = np.zeros(W * H) if want_terms else None
    grad = np.zeros((3, H, W)) if grad_region is not None else None
    lib().oc_hvsq(ctypes.c_int(W), ctypes.c_int(H), _p(a), _p(r), _p(rad), _p(reg), ctypes.c_int(n_regions),
                  ctypes.c_int(0 if grad_region is None else int(grad_region)), _p(sums), _p(counts), _p(terms),
                  _p(grad))
    with np.errstate(invalid="ignore", divide="ignore"):
        means = np.where(counts > 0, sums / np.maximum(counts, 1), 0.0)
    return dict(sums=sums, counts=counts, hvsq=means, terms=terms, grad=grad)


def hvsq_at(img_a, img_r, radius, W: int, H: int, pixels) -> np.ndarray:
    """Per-pixel HVSQ terms at the (x, y) rows of ``pixels`` only."""
    a = _f64(img_a).reshape(3, H, W)
    r = _f64(img_r).reshape(3, H, W)
    rad = np.ascontiguousarray(radius, np.int32).reshape(-1)
    px = np.ascontiguousarray(pixels, np.int32)
    out = np.zeros(px.shape[0])
    lib().oc_hvsq_at(ctypes.c_int(W), ctypes.c_int(H), _p(a), _p(r), _p(rad), ctypes.c_int(px.shape[0]), _p(px),
                     _p(out))
    return out
