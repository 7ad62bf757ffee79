"""Helpers shared by the GPU parity tests (no renderer arithmetic here)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

IMG_TOL = 2e-4  # per-channel absolute image tolerance against the oracle


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs an MI355X")


def say(*a):
    print("[case]", *a, flush=True)


def splat_np(splats: torch.Tensor) -> dict:
    """float32 splat tensor [V, n, 12] -> numpy fields (float32 / int32)."""
    s = splats.detach().cpu().contiguous()
    f = s.numpy()
    i = s.view(torch.int32).numpy()
    return dict(mean2d=f[..., 0:2].copy(), conic=f[..., 2:5].copy(), opacity=f[..., 5].copy(),
                color=f[..., 6:9].copy(), depth=f[..., 9].copy(), radius=i[..., 10].copy(),
                tiles_touched=i[..., 11].copy())


def view_slice(sp: dict, v: int) -> dict:
    return {k: a[v] for k, a in sp.items()}


def image_views(img: torch.Tensor, sizes) -> list:
    """Planar global image buffer -> list of (H, W, 3) numpy arrays."""
    a = img.detach().cpu().numpy()
    out, off = [], 0
    for w, h in sizes:
        out.append(a[off:off + 3 * w * h].reshape(3, h, w).transpose(1, 2, 0))
        off += 3 * w * h
    return out


def pixel_views(buf: torch.Tensor, sizes) -> list:
    a = buf.detach().cpu().numpy()
    out, off = [], 0
    for w, h in sizes:
        out.append(a[off:off + w * h].reshape(h, w))
        off += w * h
    return out


def check_envelope(gpu_rgb, ref: dict, tol=IMG_TOL, max_unresolved_frac=1e-4):
    """GPU pixel values must lie within tol of the oracle's envelope over all
    threshold-consistent branches.  Returns (max error vs primary branch,
    #ambiguous pixels)."""
    lo = ref["rgb_min"] - tol
    hi = ref["rgb_max"] + tol
    bad = (gpu_rgb < lo) | (gpu_rgb > hi)
    unresolved = (ref["amb"] & 4) != 0
    bad_px = bad.any(axis=-1) & ~unresolved
    n_bad = int(bad_px.sum())
    if n_bad:
        idx = np.argwhere(bad_px)[:5]
        detail = [(tuple(int(x) for x in ij), gpu_rgb[tuple(ij)].tolist(), ref["rgb"][tuple(ij)].tolist())
                  for ij in idx]
        raise AssertionError(f"{n_bad} pixels outside the oracle envelope (+-{tol}): {detail}")
    assert unresolved.sum() <= max(1, max_unresolved_frac * unresolved.size)
    amb = (ref["amb"] & 1) != 0
    err = np.abs(gpu_rgb - ref["rgb"])
    return float(err[~amb].max(initial=0.0)), int(amb.sum())


def rel_l2(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def per_point_check(gpu, ref, rtol=1e-3, floor=1e-4):
    """Per-point gradient check beside a relative L2 bar: point i (a row of
    the [n, ...] arrays) passes if ||g_i - r_i|| <= rtol ||r_i|| + floor *
    rms_i ||r_i||.  Returns (number of failing points, the largest ratio of
    error to bound)."""
    g = np.asarray(gpu, np.float64).reshape(len(gpu), -1)
    r = np.asarray(ref, np.float64).reshape(len(ref), -1)
    nr = np.linalg.norm(r, axis=1)
    rms = float(np.sqrt(np.mean(nr * nr))) if len(nr) else 0.0
    bound = rtol * nr + floor * rms + 1e-30
    ratio = np.linalg.norm(g - r, axis=1) / bound
    return int((ratio > 1.0).sum()), float(ratio.max(initial=0.0))


EPS32 = 2.0 ** -24  # unit roundoff of float32


def conic_rounding_bound(cov2d, conic_ref):
    """Per-point bound on a float32 conic against the FP64 one, [n, 1]:
    conic = adj(S') / det(S') with det = a c - b^2, whose absolute rounding
    error is of order eps (a c + b^2); relative to det that is eps times
    kappa = (a c + b^2) / (a c - b^2), and it carries over to every conic
    entry relative to the largest one.  The factor 64 covers the chain of
    roundings before S' (rotation, scales, the Jacobian and the mean)."""
    a, b, c = (np.asarray(cov2d, np.float64)[:, k] for k in range(3))
    kappa = (a * c + b * b) / (a * c - b * b)
    return 64.0 * EPS32 * kappa[:, None] * np.abs(conic_ref).max(axis=1, keepdims=True)
