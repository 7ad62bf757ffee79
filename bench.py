#!/usr/bin/env python3
"""Benchmark of the foveated stereo render on one MI355X.

Workload: 1.5M clustered Gaussians with degree-3 SH, nested quality subsets
(100/40/15/5 %) with per-level opacity and DC, two eyes at 1920x1080 with a
shared gaze, four eccentricity rings with 3.5 degree blend bands, 16x16 tiles.
One step = one pass of the whole path over both eyes: foveation tables,
projection (with per-level versions), filtered binning and (tile, depth)
sort, foveated compositing.  Inputs are resident in HBM before timing.

Prints ONE JSON line (stdout).  Also reported, untimed in the headline:
plain forward at 1280x720 / 500k, forward+backward at 1280x720 / 1M, the
FP64 oracle's rate on the host (bounded sample), and the roofline of the
dominant kernel (foveated compositing) from live HIP-event timings.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FPS & Mpix/s fwd, 1080p 1.5M Gaussians; fwd+bwd it/s; batched vs plain"
# published dense fp32 vector peak of MI355X (256 CUs, 2.4 GHz, packed fp32 counted as two)
FP32_PEAK_TFLOPS = 157.3
# algorithmic fp32 flops of one (pixel, point) pair of the forward compositing
# (FMA = 2): offsets 2, quadratic falloff 8, exp2 1, clamp 1, cut-off test 1,
# transmittance 2, stop test 1, weight 1, colour 6
FLOPS_PER_BLEND = 23
# ... and of one blended pair of its reverse: offsets 2, quadratic falloff 8,
# exp2 1, clamp 1, 1/(1 - alpha) 2, transmittance recovery 1, blend weight 1,
# g . colour 5, dL/dalpha 3, light-behind update 2, w = alpha dL/dalpha 1,
# the six moments of w in the pixel offset 11, colour gradients 6
FLOPS_PER_BLEND_BWD = 44


# HBM traffic of one k_raster_fov launch on this workload, from two
# rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch,
# averaged over the dispatches), each scaled by the ratio of known bytes to
# the same counter on a plain device copy (bench.py --copy-probe).  Valid
# only for the kernel sources they were taken on (sha256 below).
TRAFFIC = {"kernel": "k_raster_fov", "fetch_kib": 360724.9, "write_kib": 88878.7, "fetch_scale": 2.0,
           "write_scale": 1.0, "sha256": "66dce30ac61ade92b2d34b0355baebc59c3d18623c6fb84d8f264e095baaf491"}
# The same for the compositing reverse on the 1280x720 1M-Gaussian frame.
TRAFFIC_BWD = {"kernel": "k_raster_bwd", "fetch_kib": 55507.6, "write_kib": 29395.7, "fetch_scale": 2.0,
               "write_scale": 1.0, "sha256": "66dce30ac61ade92b2d34b0355baebc59c3d18623c6fb84d8f264e095baaf491"}

def kernel_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("raster.hip", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2407_00435_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_bytes(t=None):
    t = t or TRAFFIC
    if not t or t["sha256"] != kernel_sha():
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024


def copy_probe(mib=1024, reps=5):
    """Plain device copy of a known size, for scaling the memory counters."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "dispatches": reps}),
          flush=True)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Foveated:
    """Preallocated buffers and stage calls for the foveated stereo render."""

    def __init__(self, g, wl, tile=16):
        import torch
        self.g, self.torch, self.tile = g, torch, tile
        self.S = g.SceneTensors(wl.scene)
        self.C = g.Cameras(wl.cams)
        self.fov = g.binding._foveae(wl.foveae)
        self.L = self.S.n_levels
        self.n = self.S.n
        dev = self.S.t["means"].device
        self.n_tiles, self.n_px = self.C.tiles(tile)
        V = self.C.n
        self.splats = torch.empty((V, self.n, 12), dtype=torch.float32, device=dev)
        self.lvl = torch.empty((V, self.n, self.L, 4), dtype=torch.float32, device=dev)
        self.pix_level = torch.empty(self.n_px, dtype=torch.uint8, device=dev)
        self.pix_weight = torch.empty(self.n_px, dtype=torch.float32, device=dev)
        self.tile_level = torch.empty((self.n_tiles, 2), dtype=torch.uint8, device=dev)
        self.ranges = torch.empty((self.n_tiles, 2), dtype=torch.int32, device=dev)
        self.num = torch.zeros(1, dtype=torch.int64, device=dev)
        self.image = torch.empty(3 * self.n_px, dtype=torch.float32, device=dev)
        self.scene_struct = self.S.struct(levels=True)
        # key capacity: the unfiltered rectangle count bounds the filtered keys
        self.project()
        torch.cuda.synchronize()
        tt = self.splats[..., 11].view(torch.int32).to(torch.int64).sum().item()
        self.cap = int(tt)
        self.vals = torch.empty(self.cap, dtype=torch.int32, device=dev)
        nb = g.gs_workspace_bytes(self.C, self.n, tile, self.cap)
        self.ws_t, self.ws, self.wsn = g.binding._ws(nb)
        self.bg = (ctypes.c_float * 3)(0.0, 0.0, 0.0)
        self.stream = g.binding._stream()
        # per-point filtered hit counts ([views][n] uint32): off in the timed
        # step, set to a buffer by the full-size parity test
        self.hits = None

    def fovea(self):
        L, B, g = self.g.lib(), self.g.binding, self
        B._check(L.gs_fovea_prep(g.C.hp, g.C.dp, ctypes.cast(g.fov, B._PF), g.C.n, g.tile, g.L,
                                 B._ptr(g.pix_level), B._ptr(g.pix_weight), B._ptr(g.tile_level),
                                 g.stream))

    def project(self):
        L, B = self.g.lib(), self.g.binding
        # the constructor's first projection runs before the stream is set
        st = getattr(self, "stream", None) or B._stream()
        B._check(L.gs_project(ctypes.byref(self.scene_struct), self.C.hp, self.C.dp, self.C.n, self.tile,
                              B._ptr(self.splats), B._ptr(self.lvl), st))

    def binsort(self):
        L, B, g = self.g.lib(), self.g.binding, self
        B._check(L.gs_bin_sort(B._ptr(g.splats), g.n, g.C.hp, g.C.dp, g.C.n, g.tile,
                               B._ptr(g.tile_level), B._ptr(g.S.t["qbound"]), B._ptr(g.vals), None,
                               g.cap, B._ptr(g.ranges), B._ptr(g.hits), B._ptr(g.num), g.ws, g.wsn,
                               g.stream))

    def raster(self, stats=None):
        L, B, g = self.g.lib(), self.g.binding, self
        B._check(L.gs_rasterize_foveated(B._ptr(g.splats), B._ptr(g.lvl), g.n, B._ptr(g.S.t["qbound"]),
                                         g.L, g.C.hp, g.C.dp, g.C.n, g.tile, B._ptr(g.vals),
                                         B._ptr(g.ranges), B._ptr(g.pix_level), B._ptr(g.pix_weight),
                                         ctypes.cast(g.bg, B._VP), B._ptr(g.image), B._ptr(stats), None,
                                         None, g.ws, g.wsn, g.stream))

    STAGES = ("fovea", "project", "binsort", "raster")

    def one_call(self):
        """The whole frame through the library's one-call entry point (fovea
        tables, projection, binning, compositing in one call), into its own
        preallocated image and workspace."""
        L, B, g = self.g.lib(), self.g.binding, self
        if not hasattr(self, "rws"):
            torch = self.torch
            dev = self.image.device
            nb = g.g.gs_render_workspace_bytes(g.C, g.n, g.L, g.tile, g.cap)
            self.rws_t, self.rws, self.rwsn = B._ws(nb)
            self.image1 = torch.empty_like(self.image)
            self.num1 = torch.zeros(1, dtype=torch.int64, device=dev)
        B._check(L.gs_render_foveated(ctypes.byref(g.scene_struct), g.C.hp, g.C.dp, ctypes.cast(g.fov, B._PF), g.C.n,
                                      g.tile, ctypes.cast(g.bg, B._VP), B._ptr(g.image1), g.cap, B._ptr(g.num1),
                                      g.rws, g.rwsn, g.stream))


def time_foveated(fr, steps, warmup):
    torch = fr.torch
    for _ in range(warmup):
        for s in fr.STAGES:
            getattr(fr, s)()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(fr.STAGES) + 1)]
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        for j, s in enumerate(fr.STAGES):
            getattr(fr, s)()
            ev[k][j + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms = {s: sum(ev[k][j].elapsed_time(ev[k][j + 1]) for k in range(steps)) / steps
                for j, s in enumerate(fr.STAGES)}
    return wall, stage_ms


def time_one_call(fr, steps, warmup):
    """Wall time of `steps` one-call frames after `warmup` untimed ones,
    bracketed by device synchronisations."""
    torch = fr.torch
    for _ in range(warmup):
        fr.one_call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fr.one_call()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def raster_stats(fr):
    torch = fr.torch
    st = torch.zeros(4, dtype=torch.int64, device=fr.image.device)
    fr.raster(stats=st)
    torch.cuda.synchronize()
    return [int(x) for x in st.cpu().tolist()]


def timed_windows(fn, steps, warmup, windows=5, min_warm_s=0.3):
    """Seconds per call of fn: `warmup` calls and at least `min_warm_s` of
    calls untimed (the GPU has idled while the host built the workload),
    then `windows` timed windows of `steps` calls each; returns (median,
    fastest, slowest) window averages."""
    import statistics

    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < min_warm_s:
        fn()
        torch.cuda.synchronize()
    per = []
    for _ in range(windows):
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        per.append((time.perf_counter() - t0) / steps)
    return statistics.median(per), min(per), max(per)


def plain_fwd_rate(g, wl, steps, warmup, tile=16):
    """Plain forward (projection, binning/sort, compositing) of one view."""
    import torch
    S, C = g.SceneTensors(wl.scene), g.Cameras(wl.cams)
    splats = g.gs_project(S, C, tile)
    cap = int(splats[..., 11].view(torch.int32).to(torch.int64).sum().item())
    state = {"ws": None}

    def frame():
        state["out"] = g.gs_render_fwd(S, C, tile, key_capacity=cap, workspace=state["ws"])
        state["ws"] = state["out"]["workspace"]

    dt, lo, hi = timed_windows(frame, steps, warmup)
    px = sum(w * h for w, h in C.sizes)
    return dict(fps=1.0 / dt, mpix_s=px / dt / 1e6, ms=dt * 1e3, ms_range=[lo * 1e3, hi * 1e3],
                keys=int(state["out"]["num_keys"].item()), timing=f"median of 5 windows of {steps} frames")


def fwd_bwd_rate(g, wl, steps, warmup, tile=16):
    """Forward + backward (L1 loss against a target render, the fused loss
    kernel) through autograd."""
    import torch
    S, C = g.SceneTensors(wl.scene), g.Cameras(wl.cams)
    tgt_S = g.SceneTensors(wl.extra["target_scene"])
    with torch.no_grad():
        target = g.render(*(tgt_S.t[k] for k in ("means", "log_scales", "quats", "opacity_logits", "sh")),
                          C, tgt_S.sh_degree, tile)
    params = [S.t[k].clone().requires_grad_(True)
              for k in ("means", "log_scales", "quats", "opacity_logits", "sh")]
    splats = g.gs_project(S, C, tile)
    cap = int(splats[..., 11].view(torch.int32).to(torch.int64).sum().item())

    def it():
        img = g.render(*params, C, S.sh_degree, tile, key_capacity=cap)
        loss = g.l1_loss(img, target)
        loss.backward()
        for p in params:
            p.grad = None

    dt, lo, hi = timed_windows(it, steps, warmup)
    out = dict(it_s=1.0 / dt, ms=dt * 1e3, ms_range=[lo * 1e3, hi * 1e3],
               timing=f"median of 5 windows of {steps} iterations")
    # the compositing reverse on its own, timed live with events on the
    # stream it runs on, against the blended pairs of the forward (the
    # reverse takes the forward's decisions, pair for pair)
    fw = g.gs_render_fwd(S, C, tile, key_capacity=cap)
    st = torch.zeros(4, dtype=torch.int64, device="cuda")
    g.gs_rasterize_fwd(fw["splats"], S.n, C, tile, fw["vals"], fw["ranges"], stats=st)
    img = fw["image"]
    dL = torch.sign(img - target) / img.numel()
    grads = torch.empty((1, S.n, 12), dtype=torch.float32, device="cuda")
    B = g.binding
    L = g.lib()
    bg = (ctypes.c_float * 3)(0.0, 0.0, 0.0)

    def bwd():
        B._check(L.gs_rasterize_bwd(B._ptr(fw["splats"]), S.n, C.hp, C.dp, C.n, tile, B._ptr(fw["vals"]),
                                    B._ptr(fw["ranges"]), ctypes.cast(bg, B._VP), B._ptr(fw["final_T"]),
                                    B._ptr(fw["n_contrib"]), B._ptr(dL), B._ptr(grads), None, 0, B._stream()))

    for _ in range(3):
        bwd()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        bwd()
    e1.record()
    torch.cuda.synchronize()
    t_b = e0.elapsed_time(e1) * 1e-3 / reps
    blended = int(st[0].item())
    ach = blended * FLOPS_PER_BLEND_BWD / t_b / 1e12
    out["roofline_bwd"] = {"bound": "alu", "kernel": "k_raster_bwd", "unit": "TFLOP/s", "achieved": ach,
                           "peak": FP32_PEAK_TFLOPS, "frac": ach / FP32_PEAK_TFLOPS,
                           "frac_of_nonpacked": ach / (FP32_PEAK_TFLOPS / 2), "ms": t_b * 1e3,
                           "traffic": traffic_bytes(TRAFFIC_BWD), "unit_of_work": "blended (pixel, point) pair",
                           "blended_pairs": blended, "flops_per_pair": FLOPS_PER_BLEND_BWD}
    return out


TILE_SCHEDULES = (
    ("per_tile", {}),
    ("merge_256", {"raster_merge": 256}),
    ("merge_1024", {"raster_merge": 1024}),
    ("merge_4096", {"raster_merge": 4096}),
    ("merge_16384", {"raster_merge": 16384}),
    ("queue", {"raster_queue": 1}),
    ("queue_heavy_4096", {"raster_queue": 1, "raster_heavy": 4096}),
    ("queue_heavy_16384", {"raster_queue": 1, "raster_heavy": 16384}),
    ("queue_split_4096", {"raster_queue": 1, "raster_split": 4096}),
)


def greedy_group_count(ranges, beta):
    """Merged tiles of the greedy rule (consecutive tiles while their keys
    total at most beta) over a [tiles, 2] range table."""
    import numpy as np
    loads = (ranges[:, 1] - ranges[:, 0]).astype(np.int64)
    groups, tot = 0, None
    for x in loads:
        if tot is None or tot + x > beta:
            groups += 1
            tot = int(x)
        else:
            tot += int(x)
    return groups


def tile_schedules(g, fr, wl2, tile=16, reps=20):
    """Compositing time of the foveated stereo frame and of the 1280x720
    500k-Gaussian plain frame under each tile schedule: one workgroup per
    tile, light tiles merged up to beta keys, the persistent work queue, and
    the queue with runs longer than 4096 keys split.  Events around the
    compositing call, on the stream it runs on (median over calls); each
    image is compared with the per-tile one (merged and queued: bit for bit;
    split: reassociated)."""
    import torch
    B = g.binding
    S2, C2 = g.SceneTensors(wl2.scene), g.Cameras(wl2.cams)
    splats2 = g.gs_project(S2, C2, tile)
    bs2 = g.gs_bin_sort(splats2, S2.n, C2, tile, check=True)
    saved = (fr.ws_t, fr.ws, fr.wsn)
    cases = {"foveated_stereo_1080p_1.5M": {}, "plain_720p_500k": {}}
    ranges = {"foveated_stereo_1080p_1.5M": fr.ranges.cpu().numpy(),
              "plain_720p_500k": bs2["ranges"].cpu().numpy()}
    refs = {}

    def ev_ms(fn):
        # per-call event pairs, median: a host stall (allocator, collector)
        # inside the window would otherwise count as compositing time
        import statistics
        for _ in range(3):
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        torch.cuda.synchronize()
        for e0, e1 in ev:
            e0.record()
            fn()
            e1.record()
        torch.cuda.synchronize()
        return statistics.median(e0.elapsed_time(e1) for e0, e1 in ev)

    try:
        for name, knobs in TILE_SCHEDULES:
            for k, v in knobs.items():
                g.gs_set_tuning(k, v)
            try:
                fr.ws_t, fr.ws, fr.wsn = B._ws(g.gs_workspace_bytes(fr.C, fr.n, tile, fr.cap))
                ws2 = B._ws(g.gs_workspace_bytes(C2, S2.n, tile, bs2["capacity"]))
                st = {}

                def plain():
                    st["out"] = g.gs_rasterize_fwd(splats2, S2.n, C2, tile, bs2["vals"], bs2["ranges"],
                                                   workspace=ws2)

                for case, fn, img in (("foveated_stereo_1080p_1.5M", fr.raster, lambda: fr.image),
                                      ("plain_720p_500k", plain, lambda: st["out"]["image"])):
                    ms = ev_ms(fn)
                    im = img().clone()
                    if name == "per_tile":
                        refs[case] = im
                    r = {"ms": ms, "bit_equal": bool(torch.equal(im, refs[case])),
                         "max_abs_diff": float((im - refs[case]).abs().max().item())}
                    if "raster_merge" in knobs:
                        r["merged_tiles"] = greedy_group_count(ranges[case], knobs["raster_merge"])
                        r["tiles"] = int(len(ranges[case]))
                    cases[case][name] = r
            finally:
                for k in knobs:
                    g.gs_set_tuning(k, 0)
    finally:
        fr.ws_t, fr.ws, fr.wsn = saved
    return cases


def batched_vs_plain(g, steps=3, log=None, fixed=None, plain_too=True):
    """3M Gaussians, 32 orbit views at mixed resolutions (forward + L1 loss +
    backward) plus the foveated forward of two eyes, as one step.  Batched:
    the autotuned schedule replayed from a recorded graph.  Plain: one view
    per call (and one eye per call), run eagerly, tile 16."""
    import torch
    import scenegen
    from paper_2407_00435_amd import autotune
    from paper_2407_00435_amd.batched import BatchedStep

    wl = scenegen.config5()
    S = g.SceneTensors(wl.scene)
    cams, eyes, fov = wl.cams, wl.extra["eyes"], wl.extra["eye_foveae"]
    C = g.Cameras(cams)
    tgt_S = g.SceneTensors(scenegen.perturbed(wl.scene, 1006))
    sp = g.gs_project(tgt_S, C, 16)
    cap = int(sp[..., 11].view(torch.int32).to(torch.int64).sum().item()) + 1024
    del sp
    target = g.gs_render_fwd(tgt_S, C, 16, key_capacity=cap)["image"].clone()
    del tgt_S
    torch.cuda.empty_cache()
    px = sum(c.width * c.height for c in cams) + sum(c.width * c.height for c in eyes)
    if log:
        log(f"batched: autotuning ({len(cams)} views + {len(eyes)} eyes, {px / 1e6:.1f} Mpix) ...")
    if fixed:
        best, tried = dict(fixed), []
        g.gs_set_tuning("radix_part", best["radix_part"])
        g.gs_set_tuning("raster_queue", best.get("raster_queue", 0))
    else:
        best, tried = autotune.tune(S, cams, target, eyes, fov, reps=2, log=log)
    step = BatchedStep(S, cams, target, best["tile"], best["batch_views"], eyes, fov, lanes=best.get("lanes", 1))
    ms_b = autotune.time_step(step, steps)
    keys_b = int(step.num_keys.sum().item())
    ok_b = step.keys_ok()
    del step
    torch.cuda.empty_cache()
    g.gs_set_tuning("radix_part", 8192)
    g.gs_set_tuning("raster_queue", 0)
    if not plain_too:
        return dict(batched_it_s=1e3 / ms_b, batched_ms=ms_b, config=best, keys=keys_b, capacity_ok=bool(ok_b))
    plain = BatchedStep(S, cams, target, 16, 1, eyes, fov, eye_batch=1)
    plain.step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(plain.stream)
    for _ in range(steps):
        plain._enqueue()
    e1.record(plain.stream)
    torch.cuda.synchronize()
    ms_p = e0.elapsed_time(e1) / steps
    ok_p = plain.keys_ok()
    return dict(workload="3M Gaussians SH3; 32 orbit views (640x360..1920x1080) fwd + L1 + bwd; "
                         "2 foveated 1080p eyes fwd",
                megapixels=px / 1e6, batched_it_s=1e3 / ms_b, batched_ms=ms_b, plain_it_s=1e3 / ms_p,
                plain_ms=ms_p, speedup=ms_p / ms_b, autotuned=best, keys=keys_b,
                capacity_ok=bool(ok_b and ok_p),
                tried=[dict(c, ms=round(m, 3)) for c, m in tried])


def host_threads():
    """Threads the oracle runs on: the CPUs this process may use, at most the
    16 a one-GPU machine shares out."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def cpu_baseline(fr, wl, n_gauss_sample=12000, px_sample=(3000, 9000), threads=None):
    """FP64 oracle on the host, on a bounded sample of the same workload:
    projection (with the four level versions) of a random subset of the
    Gaussians for both eyes, and per-pixel foveated compositing of random
    pixels over the full projected splat set, each on `threads` threads.  The
    per-Gaussian and per-pixel costs are extrapolated to a whole stereo
    frame."""
    import concurrent.futures as cf

    import numpy as np
    import oracle
    threads = threads or host_threads()
    rng = np.random.default_rng(0)
    sub = wl.scene.subset(rng.choice(wl.scene.n, n_gauss_sample, replace=False))
    parts = [sub.subset(np.arange(a, min(a + -(-sub.n // threads), sub.n)))
             for a in range(0, sub.n, -(-sub.n // threads))]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:  # the oracle's C code runs without the GIL
        for cam in wl.cams:
            list(ex.map(lambda sc: oracle.project(sc, cam, levels=True), parts))
    t_proj = (time.perf_counter() - t0) / (n_gauss_sample * len(wl.cams))
    sp = fr.splats.cpu().numpy()
    spi = fr.splats.cpu().view(fr.torch.int32).numpy()
    lv = fr.lvl.cpu().numpy()
    pl = fr.pix_level.cpu().numpy()
    pw = fr.pix_weight.cpu().numpy().astype(np.float64)
    per_px, fixed = [], []
    off = 0
    for v, cam in enumerate(wl.cams):
        W, H = cam.width, cam.height
        proj = dict(mean2d=sp[v, :, 0:2], conic=sp[v, :, 2:5], depth=sp[v, :, 9], opacity=sp[v, :, 5],
                    color=sp[v, :, 6:9], radius=spi[v, :, 10],
                    lvl_opacity=lv[v, :, :, 3].T.copy(), lvl_color=lv[v, :, :, 0:3].transpose(1, 0, 2).copy())
        proj = oracle.splats_to_proj(proj)
        ts = []
        for k in px_sample:
            pix = np.stack([rng.integers(0, W, k), rng.integers(0, H, k)], 1)
            t0 = time.perf_counter()
            oracle.composite(proj, W, H, qbound=wl.scene.qbound, pix_lo=pl[off:off + W * H],
                             pix_w=pw[off:off + W * H], levels=True, pixels=pix, nthreads=threads)
            ts.append(time.perf_counter() - t0)
        a = (ts[1] - ts[0]) / (px_sample[1] - px_sample[0])
        per_px.append(max(a, 0.0))
        fixed.append(max(ts[0] - a * px_sample[0], 0.0))
        off += W * H
    frame = t_proj * wl.scene.n * len(wl.cams) + sum(
        f + a * c.width * c.height for f, a, c in zip(fixed, per_px, wl.cams))
    px = sum(c.width * c.height for c in wl.cams)
    return dict(value=px / frame / 1e6, unit="Mpix/s", cores=threads, kind="oracle",
                host_cpus=len(os.sched_getaffinity(0)),
                sample=(f"projection of {n_gauss_sample} random Gaussians x {len(wl.cams)} eyes x "
                        f"(base + {wl.scene.lvl_opacity_logits.shape[0]} levels), and foveated compositing "
                        f"of {px_sample[0]}+{px_sample[1]} random pixels per eye over all projected splats, "
                        f"both on {threads} threads; extrapolated to one full stereo frame "
                        f"({frame:.1f} s/frame)"),
                frame_s=frame)


def cpu_full_frames(threads=None, reps=3):
    """The oracle's full render (FP64 projection, then per-pixel compositing)
    of whole frames of the two plain workloads: 4096 Gaussians at 128x128
    and 500k Gaussians at 1280x720, on all the threads it may use and on one.
    Median of `reps` runs, except that the single-threaded 1280x720 frame is
    timed on every 8th pixel row and scaled by 8 (about 75 s whole)."""
    import numpy as np
    import oracle
    import scenegen
    threads = threads or host_threads()
    out = {"host_cpus": len(os.sched_getaffinity(0)), "threads": threads}
    for label, wl, r in (("128x128_4k", scenegen.config1(), reps), ("1280x720_500k", scenegen.config2(), 1)):
        cam = wl.cams[0]
        W, H = cam.width, cam.height
        rec = {}
        for th in (threads, 1):
            sub_rows = th == 1 and H > 128
            pix = None
            if sub_rows:
                ys = np.arange(0, H, 8)
                pix = np.stack(np.meshgrid(np.arange(W), ys), -1).reshape(-1, 2).astype(np.int32)
            ts = []
            for _ in range(r):
                t0 = time.perf_counter()
                oracle.render(wl.scene, cam, pixels=pix, nthreads=th)
                ts.append(time.perf_counter() - t0)
            t = float(np.median(ts))
            if sub_rows:
                t *= H / len(np.arange(0, H, 8))
            rec[f"{th}_threads"] = {"s_per_frame": t, "fps": 1.0 / t, "mpix_s": W * H / t / 1e6,
                                    "measured_on": "every 8th row, scaled" if sub_rows else "full frame"}
        out[label] = rec
    return out


def pipelined_frames(g, wl, tile, frames=40, warmup=6):
    """Throughput of consecutive stereo frames issued alternately to two
    streams with two buffer sets: a frame's binning overlaps the previous
    frame's compositing (a GPU analogue of the paper's incremental
    pipelining).  Every frame still runs all four stages; per-frame latency
    is the sequential frame time, not this figure."""
    import torch
    sts = [torch.cuda.Stream(), torch.cuda.Stream()]
    frs = []
    for st in sts:
        with torch.cuda.stream(st):
            frs.append(Foveated(g, wl, tile))
    torch.cuda.synchronize()

    def frame(f):
        for s in f.STAGES:
            getattr(f, s)()

    for k in range(warmup):
        frame(frs[k % 2])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(frames):
        frame(frs[k % 2])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / frames
    same = bool(torch.equal(frs[0].image, frs[1].image))
    return {"streams": 2, "frames": frames, "ms_per_frame": dt * 1e3, "fps": 1.0 / dt,
            "mpix_s": frs[0].n_px / dt / 1e6, "frames_identical": same}


def one_call_frames(g, fr, wl, tile, steps=20, warmup=5):
    """The stereo frame through the one-call gs_render_foveated: joint (both
    eyes per stage) and eye by eye on two streams (stream_views: eye 0's
    compositing overlaps eye 1's binning), with one workspace sized for
    each, median of timed windows; the two images are compared bit for
    bit."""
    import torch
    B = g.binding
    out = {}
    imgs = {}
    for name, on in (("joint", 0), ("eye_streamed", 1)):
        g.gs_set_tuning("stream_views", on)
        try:
            state = {"ws": None}

            def frame():
                img, num, ws = g.gs_render_foveated(fr.S, fr.C, wl.foveae, tile, key_capacity=fr.cap,
                                                    workspace=state["ws"])
                state.update(ws=ws, img=img, num=num)

            frame()
            torch.cuda.synchronize()
            st, need = g.context().poll_status(state["ws"])
            dt, lo, hi = timed_windows(frame, steps, warmup)
            imgs[name] = state["img"].clone()
            out[name] = {"ms": dt * 1e3, "ms_range": [lo * 1e3, hi * 1e3], "mpix_s": fr.n_px / dt / 1e6,
                         "keys": int(state["num"].item()), "capacity_ok": st == B.GS_OK}
        finally:
            g.gs_set_tuning("stream_views", 0)
    out["bit_equal"] = bool(torch.equal(imgs["joint"], imgs["eye_streamed"]))
    out["timing"] = f"median of 5 windows of {steps} frames"
    return out


def hbm_bandwidth(g, fr, stage_ms, reps=10):
    """Achieved HBM bandwidth of the projection and of the radix sort, against a
    plain device copy on the same GPU (the achievable reference) and the
    published 8 TB/s.  Projection bytes are algorithmic: per Gaussian 236 B of
    SH3 parameters + 65 B of level data read, per (Gaussian, eye) 48 B of splat +
    4 x 16 B of level colour/opacity written.  Sort bytes: one 4 B key read for
    the histogram, then per 8-bit pass an 8 B (key, value) read and write."""
    import torch
    B = g.binding
    src = torch.ones(256 << 20, dtype=torch.float32, device="cuda")  # 1 GiB
    dst = torch.empty_like(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    out = {"copy_gbs": copy_gbs, "peak_gbs": 8000.0}
    eyes = fr.C.n
    proj_bytes = fr.n * (236 + 65) + fr.n * eyes * (48 + 4 * 16)
    gbs = proj_bytes / (stage_ms["project"] * 1e-3) / 1e9
    out["project"] = {"bytes": proj_bytes, "gbs": gbs, "frac_of_copy": gbs / copy_gbs, "frac_of_peak": gbs / 8000.0}
    L = B.lib()
    for label, count in (("sort_2.9M", int(fr.n * eyes * 0.955)), ("sort_64M", 64 << 20)):
        gen = torch.Generator(device="cuda").manual_seed(7)
        k0 = torch.randint(0, 2 ** 31 - 1, (count,), dtype=torch.int32, device="cuda", generator=gen)
        v0 = torch.arange(count, dtype=torch.int32, device="cuda")
        k, v, kt, vt = k0.clone(), v0.clone(), torch.empty_like(k0), torch.empty_like(v0)
        ws = B._ws(int(L.gs_sort_workspace_bytes(count)))
        t = 0.0
        for r in range(reps + 1):
            k.copy_(k0)
            v.copy_(v0)
            e0.record()
            B._check(L.gs_sort_pairs(B._ptr(k), B._ptr(v), B._ptr(kt), B._ptr(vt), count, 32, ws[1], ws[2],
                                     B._stream()))
            e1.record()
            torch.cuda.synchronize()
            if r:
                t += e0.elapsed_time(e1) * 1e-3
        t /= reps
        nbytes = count * (4 + 4 * 16)
        gbs = nbytes / t / 1e9
        out[label] = {"keys": count, "bits": 32, "ms": t * 1e3, "bytes": nbytes, "gbs": gbs,
                      "frac_of_copy": gbs / copy_gbs, "frac_of_peak": gbs / 8000.0}
        del k0, v0, k, v, kt, vt, ws
    return out


def hvsq_rate(g, fr, wl, reps=10):
    """HVSQ (Eq. 2) of the foveated stereo frame against the full render of
    the same eyes, per ring, with the gradient of the whole-frame metric
    (pooling half-width 0.25 x eccentricity in degrees, in pixels), timed
    with events on the library's stream."""
    import numpy as np
    import torch
    ref = g.gs_render_fwd(fr.S, fr.C, fr.tile, key_capacity=fr.cap, check=True)["image"]
    rho = 0.25 * float(wl.cams[0].fx) * np.pi / 180.0
    rad = g.gs_hvsq_pooling(fr.C, wl.foveae, rho)
    out = g.gs_hvsq(fr.image, ref, fr.C, rad, region=fr.pix_level, n_regions=fr.L, grad_region=0)
    ws = out["workspace"]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    for label, gr in (("metric", -1), ("metric_and_gradient", 0)):
        g.gs_hvsq(fr.image, ref, fr.C, rad, region=fr.pix_level, n_regions=fr.L, grad_region=gr, workspace=ws)
        e0.record()
        for _ in range(reps):
            out = g.gs_hvsq(fr.image, ref, fr.C, rad, region=fr.pix_level, n_regions=fr.L, grad_region=gr,
                            workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        res[label + "_ms"] = e0.elapsed_time(e1) / reps
    res["hvsq_per_ring"] = [[round(float(x), 7) for x in row] for row in out["hvsq"].cpu().numpy()]
    res["max_radius_px"] = int(rad.max().item())
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched step (3M Gaussians, 32 views + 2 eyes) at a fixed schedule: "
                         "--tile, --batch-views, --lanes, --radix-part; for profiling")
    ap.add_argument("--batch-views", type=int, default=32)
    ap.add_argument("--lanes", type=int, default=1, help="streams the sub-batches alternate over")
    ap.add_argument("--radix-part", type=int, default=16384)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (memory-counter calibration)")
    ap.add_argument("--only", choices=("fwdbwd", "plain", "schedules", "streamed", "hvsq"),
                    help="only the 1280x720 1M-Gaussian forward+backward, only the 1280x720 500k plain "
                         "forward (for profiling one kernel), only the tile-schedule comparison, only the one-call "
                         "frame joint and eye by eye, or only the HVSQ of the stereo frame")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the renderer has no multi-GPU path "
              "(its views would shard across GPUs with one gradient all-reduce).", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_probe:
        copy_probe()
        return
    import paper_2407_00435_amd as g
    import scenegen

    if args.only == "fwdbwd":
        print(json.dumps(fwd_bwd_rate(g, scenegen.config4(), args.steps, args.warmup)), flush=True)
        return
    if args.only == "plain":
        print(json.dumps(plain_fwd_rate(g, scenegen.config2(), args.steps, args.warmup)), flush=True)
        return
    if args.only == "hvsq":
        torch.cuda.set_device(0)
        wl = scenegen.config3()
        fr = Foveated(g, wl, args.tile)
        time_foveated(fr, 1, 1)
        print(json.dumps(hvsq_rate(g, fr, wl)), flush=True)
        return
    if args.only == "streamed":
        torch.cuda.set_device(0)
        wl = scenegen.config3()
        fr = Foveated(g, wl, args.tile)
        print(json.dumps(one_call_frames(g, fr, wl, args.tile)), flush=True)
        return
    if args.only == "schedules":
        torch.cuda.set_device(0)
        fr = Foveated(g, scenegen.config3(), args.tile)
        time_foveated(fr, 3, 2)
        print(json.dumps(tile_schedules(g, fr, scenegen.config2(), args.tile)), flush=True)
        return
    if args.batched_only:
        r = batched_vs_plain(g, args.steps, log, fixed=dict(tile=args.tile, batch_views=args.batch_views,
                                                             lanes=args.lanes, radix_part=args.radix_part,
                                                             raster_queue=0),
                             plain_too=False)
        print(json.dumps(r), flush=True)
        return

    torch.cuda.set_device(0)
    log("generating the 1.5M-Gaussian foveated scene ...")
    wl = scenegen.config3()
    fr = Foveated(g, wl, args.tile)
    log(f"key capacity {fr.cap}; warmup {args.warmup}, steps {args.steps}")
    # per-stage times from the stages issued as separate calls with events
    # between them; the step itself is the library's one-call frame
    wall_staged, stage_ms = time_foveated(fr, args.steps, args.warmup)
    wall = time_one_call(fr, args.steps, args.warmup)
    ms = wall / args.steps * 1e3
    same = bool(torch.equal(fr.image1, fr.image))
    px = fr.n_px
    keys = int(fr.num.item())
    stats = raster_stats(fr)
    t_r = stage_ms["raster"] * 1e-3
    # the algorithmic unit is the evaluated (pixel, point) pair; the
    # blended pairs (those that change the pixel) are reported beside it
    achieved = stats[1] * FLOPS_PER_BLEND / t_r / 1e12
    achieved_bl = stats[0] * FLOPS_PER_BLEND / t_r / 1e12
    line = {
        "metric": METRIC,
        "value": px / (wall / args.steps) / 1e6,
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "foveated stereo forward, 1.5M Gaussians SH3, 2 eyes 1920x1080, "
                               "4 levels (100/40/15/5 %), 3.5 deg bands, 16x16 tiles",
                   "gaussians": fr.n, "eyes": 2, "width": 1920, "height": 1080, "tile": args.tile,
                   "levels": fr.L},
        "fps": 1e3 / ms,
        "step": "gs_render_foveated (one call: fovea tables, projection, binning + sort, compositing)",
        "staged_ms_per_step": wall_staged / args.steps * 1e3,
        "one_call_equals_stages": same,
        "stage_ms": stage_ms,
        "keys": keys,
        "raster_pairs": {"blended": stats[0], "evaluated": stats[1], "staged": stats[2], "kept": stats[3]},
        "roofline": {"bound": "alu", "kernel": "k_raster_fov", "achieved": achieved,
                     "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": traffic_bytes(), "unit_of_work": "evaluated (pixel, point) pair",
                     "flops_per_pair": FLOPS_PER_BLEND, "pairs": stats[1], "ms": stage_ms["raster"],
                     "frac_of_nonpacked": achieved / (FP32_PEAK_TFLOPS / 2),
                     "achieved_blended": achieved_bl, "frac_blended": achieved_bl / FP32_PEAK_TFLOPS},
    }
    if not args.no_extras:
        log("HBM bandwidth of projection and sort ...")
        line["hbm"] = hbm_bandwidth(g, fr, stage_ms)
        log("one-call frame: joint and eye by eye on two streams ...")
        line["one_call_frames"] = one_call_frames(g, fr, wl, args.tile)
        log("consecutive frames on two streams ...")
        line["pipelined_frames"] = pipelined_frames(g, wl, args.tile)
        log("plain forward, 4096 Gaussians, 128x128 ...")
        line["plain_fwd_128_4k"] = plain_fwd_rate(g, scenegen.config1(), 50, 5)
        log("plain forward, 500k Gaussians, 1280x720 ...")
        line["plain_fwd_720p_500k"] = plain_fwd_rate(g, scenegen.config2(), 20, 3)
        log("tile schedules: per tile, merged, queue, split ...")
        line["tile_schedules"] = tile_schedules(g, fr, scenegen.config2(), args.tile)
        log("forward+backward, 1M Gaussians, 1280x720 ...")
        line["fwd_bwd_720p_1M"] = fwd_bwd_rate(g, scenegen.config4(), 10, 3)
        log("HVSQ of the stereo frame ...")
        line["hvsq_stereo_1080p"] = hvsq_rate(g, fr, wl)
        log("batched vs plain, 3M Gaussians, 32 views + 2 eyes ...")
        line["batched_vs_plain"] = batched_vs_plain(g, 3, log)
    if not args.no_cpu_baseline:
        log("oracle on the host (bounded sample) ...")
        line["cpu_baseline"] = cpu_baseline(fr, wl)
        log("oracle on whole 128x128 and 1280x720 frames ...")
        line["cpu_oracle_frames"] = cpu_full_frames()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
