"""Batched multi-view forward + backward, recorded once as a graph.

One training step over a fixed camera set: projection, binning/sort and
compositing of every view, the L1 loss against per-view targets, the
compositing reverse and the projection reverse (gradients summed over
views), plus the foveated eyes: forward only, or, given eye targets, forward,
L1 loss and the foveated reverse into the base and per-level parameters
(the loss is the mean over the views' pixels plus the mean over the eyes'
pixels).  Views are processed in
sub-batches of ``batch_views`` consecutive views; within a sub-batch every
stage is one library call over all its views (each Gaussian is read once
for all of them, one global tile space, one sort, one compositing launch
and one reverse launch).  ``batch_views = 1`` is the plain
one-view-per-launch schedule (``eye_batch = 1`` likewise renders one eye
per call).  All buffers are allocated up front, so the
whole step is a fixed sequence of kernel launches on one stream and is
captured with the library's graph calls and replayed.

Torch only provides device memory and the stream; every step runs in the
library's kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import binding as B


class BatchedStep:
    def __init__(self, scene: B.SceneTensors, cams: list, target: torch.Tensor, tile_size: int = 16,
                 batch_views: int | None = None, eyes: list | None = None, foveae: list | None = None,
                 key_margin: float = 1.05, stream: torch.cuda.Stream | None = None,
                 eye_batch: int | None = None, eye_target: torch.Tensor | None = None, lanes: int = 1):
        dev = scene.t["means"].device
        self.scene, self.tile = scene, tile_size
        self.stream = stream or torch.cuda.Stream(device=dev)
        V = len(cams)
        bv = max(1, V if not batch_views else min(int(batch_views), V))
        self.batch_views = bv
        self.groups = []
        px_off = 0
        cap_max, n_px_max, tiles_max, ws_max = 1, 1, 1, 256
        for a in range(0, V, bv):
            C = B.Cameras(cams[a:a + bv], device=dev)
            n_tiles, n_px = C.tiles(tile_size)
            splats = B.gs_project(scene, C, tile_size)
            cap = int(B.splat_fields(splats)["tiles_touched"].to(torch.int64).sum().item())
            cap = max(int(cap * key_margin) + 1024, 1)
            self.groups.append(dict(C=C, n_tiles=n_tiles, n_px=n_px, px_off=px_off, cap=cap))
            px_off += n_px
            cap_max, n_px_max, tiles_max = max(cap_max, cap), max(n_px_max, n_px), max(tiles_max, n_tiles)
            ws_max = max(ws_max, B.gs_workspace_bytes(C, scene.n, tile_size, cap))
            del splats
        self.n_px = px_off
        if target.numel() != 3 * self.n_px:
            raise ValueError(f"target has {target.numel()} floats, the views need {3 * self.n_px}")
        self.target = target.contiguous()
        n, Vb = scene.n, bv
        f32 = dict(dtype=torch.float32, device=dev)
        i32 = dict(dtype=torch.int32, device=dev)
        # lanes: sub-batches alternate over this many streams, each with its
        # own scratch, so that one sub-batch's binning runs beside another's
        # compositing (the eyes' reverse, when trained, keeps one lane)
        nl = 1 if (eyes and eye_target is not None) else max(1, min(int(lanes), len(self.groups)))
        self.lanes = nl
        self.lane_streams = [self.stream] + [torch.cuda.Stream(device=dev) for _ in range(nl - 1)]
        # per-sub-batch scratch of each lane, reused by the lane's sub-batches
        self.lane_bufs = []
        for _ in range(nl):
            ws_t, ws, wsn = B._ws(ws_max)
            self.lane_bufs.append(dict(splats=torch.empty((Vb, n, 12), **f32), sgrads=torch.empty((Vb, n, 12), **f32),
                                       vals=torch.empty(cap_max, **i32), ranges=torch.empty((tiles_max, 2), **i32),
                                       ws_t=ws_t, ws=ws, wsn=wsn))
        self.splats, self.sgrads = self.lane_bufs[0]["splats"], self.lane_bufs[0]["sgrads"]
        self.vals, self.ranges = self.lane_bufs[0]["vals"], self.lane_bufs[0]["ranges"]
        self.ws_t, self.ws, self.wsn = self.lane_bufs[0]["ws_t"], self.lane_bufs[0]["ws"], self.lane_bufs[0]["wsn"]
        # a sub-batch's projection reverse accumulates into the parameter
        # gradients after the previous sub-batch's (one event per sub-batch)
        self.pb_events = [torch.cuda.Event() for _ in self.groups]
        self.num_keys = torch.zeros(len(self.groups), dtype=torch.int64, device=dev)
        # whole-step outputs
        self.image = torch.empty(3 * self.n_px, **f32)
        self.final_T = torch.empty(self.n_px, **f32)
        self.n_contrib = torch.empty(self.n_px, **i32)
        self.dL = torch.empty(3 * self.n_px, **f32)
        self.loss = torch.zeros(1, **f32)
        self.grads = {k: torch.empty_like(scene.t[k]) for k in B.PARAM_NAMES}
        self.scale = 1.0 / (3 * self.n_px) if self.n_px else 0.0
        self.bg = (ctypes.c_float * 3)(0.0, 0.0, 0.0)
        self.scene_struct = scene.struct(levels=False)
        # foveated eyes (forward), in groups of eye_batch eyes per call
        self.eye_groups = []
        self.eye_image = None
        if eyes:
            if scene.n_levels == 0:
                raise ValueError("foveated eyes need a scene with quality levels")
            eb = len(eyes) if not eye_batch else max(1, min(int(eye_batch), len(eyes)))
            e_off, e_ws = 0, 256
            for a in range(0, len(eyes), eb):
                E = B.Cameras(eyes[a:a + eb], device=dev)
                _, e_px = E.tiles(tile_size)
                probe = B.gs_project(scene, E, tile_size)
                e_cap = int(B.splat_fields(probe)["tiles_touched"].to(torch.int64).sum().item()) + 1024
                del probe
                e_ws = max(e_ws, B.gs_render_workspace_bytes(E, scene.n, scene.n_levels, tile_size, e_cap))
                self.eye_groups.append(dict(C=E, fov=B._foveae(foveae[a:a + eb]), cap=e_cap, px_off=e_off,
                                            n_px=e_px))
                e_off += e_px
            self.eye_ws = B._ws(e_ws)
            self.eye_image = torch.empty(3 * e_off, **f32)
            self.eye_num = torch.zeros(len(self.eye_groups), dtype=torch.int64, device=dev)
            self.eye_struct = scene.struct(levels=True)
            self.eye_train = eye_target is not None
            if self.eye_train:
                if eye_target.numel() != 3 * e_off:
                    raise ValueError(f"eye target has {eye_target.numel()} floats, the eyes need {3 * e_off}")
                self.eye_target = eye_target.contiguous()
                self.eye_dL = torch.empty(3 * e_off, **f32)
                self.eye_scale = 1.0 / (3 * e_off)
                L = scene.n_levels
                eb_max = max(e["C"].n for e in self.eye_groups)
                e_tiles = max(e["C"].tiles(tile_size)[0] for e in self.eye_groups)
                e_cap = max(e["cap"] for e in self.eye_groups)
                e_px_max = max(e["n_px"] for e in self.eye_groups)
                self.eye_bufs = dict(
                    pix_level=torch.empty(e_px_max, dtype=torch.uint8, device=dev),
                    pix_weight=torch.empty(e_px_max, **f32),
                    tile_level=torch.empty((e_tiles, 2), dtype=torch.uint8, device=dev),
                    splats=torch.empty((eb_max, n, 12), **f32), lvl=torch.empty((eb_max, n, L, 4), **f32),
                    vals=torch.empty(e_cap, **i32), ranges=torch.empty((e_tiles, 2), **i32),
                    fT2=torch.empty((e_px_max, 2), **f32), nc2=torch.empty((e_px_max, 2), **i32),
                    grads=torch.empty((eb_max, n, 12), **f32), lvl_grads=torch.empty((eb_max, n, L, 4), **f32))
                self.eye_bin_ws = B._ws(max(B.gs_workspace_bytes(e["C"], n, tile_size, e["cap"])
                                            for e in self.eye_groups))
                for k in ("lvl_opacity_logits", "lvl_sh_dc"):
                    self.grads[k] = torch.empty_like(scene.t[k]) if scene.t.get(k) is not None else None
        else:
            self.eye_train = False
        # eyes rendered forward only depend on the scene, not on the views'
        # forward and reverse: they run on a second stream beside them
        self.eye_stream = (torch.cuda.Stream(device=dev) if self.eye_groups and not self.eye_train else None)
        self.graph = None

    def _enqueue(self):
        L, g = B.lib(), self
        st = ctypes.c_void_p(self.stream.cuda_stream)
        P = B._ptr
        gr = g.grads
        first = True  # the first gradient writer overwrites, the others add
        if self.eye_train:
            # eyes first: their reverse is the only writer of the level arrays
            eb = self.eye_bufs
            nl = g.scene.n_levels
            for k, e in enumerate(self.eye_groups):
                C, o, npx = e["C"], e["px_off"], e["n_px"]
                img = self.eye_image[3 * o:3 * (o + npx)]
                dL = self.eye_dL[3 * o:3 * (o + npx)]
                tg = self.eye_target[3 * o:3 * (o + npx)]
                B._check(L.gs_fovea_prep(C.hp, C.dp, ctypes.cast(e["fov"], B._PF), C.n, g.tile, nl,
                                         P(eb["pix_level"]), P(eb["pix_weight"]), P(eb["tile_level"]), st))
                B._check(L.gs_project(ctypes.byref(self.eye_struct), C.hp, C.dp, C.n, g.tile, P(eb["splats"]),
                                      P(eb["lvl"]), st))
                B._check(L.gs_bin_sort(P(eb["splats"]), g.scene.n, C.hp, C.dp, C.n, g.tile, P(eb["tile_level"]),
                                       P(g.scene.t["qbound"]), P(eb["vals"]), None, e["cap"], P(eb["ranges"]),
                                       None, P(self.eye_num[k:k + 1]), self.eye_bin_ws[1], self.eye_bin_ws[2],
                                       st))
                B._check(L.gs_rasterize_foveated(P(eb["splats"]), P(eb["lvl"]), g.scene.n, P(g.scene.t["qbound"]),
                                                 nl, C.hp, C.dp, C.n, g.tile, P(eb["vals"]), P(eb["ranges"]),
                                                 P(eb["pix_level"]), P(eb["pix_weight"]),
                                                 ctypes.cast(g.bg, B._VP), P(img), None, P(eb["fT2"]),
                                                 P(eb["nc2"]), None, 0, st))
                B._check(L.gs_l1_grad(P(img), P(tg), 3 * npx, ctypes.c_float(self.eye_scale), P(dL), P(g.loss),
                                      1 if first else 0, st))
                B._check(L.gs_rasterize_foveated_bwd(P(eb["splats"]), P(eb["lvl"]), g.scene.n,
                                                     P(g.scene.t["qbound"]), nl, C.hp, C.dp, C.n, g.tile,
                                                     P(eb["vals"]), P(eb["ranges"]), P(eb["pix_level"]),
                                                     P(eb["pix_weight"]), ctypes.cast(g.bg, B._VP), P(eb["fT2"]),
                                                     P(eb["nc2"]), P(dL), P(eb["grads"]), P(eb["lvl_grads"]), st))
                B._check(L.gs_project_bwd_levels(ctypes.byref(self.eye_struct), C.hp, C.dp, C.n,
                                                 P(eb["splats"]), P(eb["grads"]), P(eb["lvl_grads"]),
                                                 P(gr["means"]), P(gr["log_scales"]), P(gr["quats"]),
                                                 P(gr["opacity_logits"]), P(gr["sh"]),
                                                 P(gr.get("lvl_opacity_logits")), P(gr.get("lvl_sh_dc")),
                                                 0 if first else 1, st))
                first = False
        if self.eye_stream is not None:
            # fork: the eyes' forward renders beside the views' work
            es = self.eye_stream
            es.wait_stream(self.stream)
            est = ctypes.c_void_p(es.cuda_stream)
            for k, e in enumerate(self.eye_groups):
                o, npx = e["px_off"], e["n_px"]
                B._check(L.gs_render_foveated(ctypes.byref(self.eye_struct), e["C"].hp, e["C"].dp,
                                              ctypes.cast(e["fov"], B._PF), e["C"].n, g.tile,
                                              ctypes.cast(g.bg, B._VP), P(self.eye_image[3 * o:3 * (o + npx)]),
                                              e["cap"], P(self.eye_num[k:k + 1]), self.eye_ws[1], self.eye_ws[2],
                                              est))
        multi = self.lanes > 1
        if multi:
            # the loss is cleared before the lanes add to it
            if first:
                B._check(L.gs_l1_grad(None, None, 0, ctypes.c_float(g.scale), None, P(g.loss), 1, st))
            for ls in self.lane_streams[1:]:
                ls.wait_stream(self.stream)
        for k, grp in enumerate(self.groups):
            C, o, npx = grp["C"], grp["px_off"], grp["n_px"]
            img = self.image[3 * o:3 * (o + npx)]
            fT = self.final_T[o:o + npx]
            nc = self.n_contrib[o:o + npx]
            dL = self.dL[3 * o:3 * (o + npx)]
            tg = self.target[3 * o:3 * (o + npx)]
            lane = k % self.lanes
            lb = self.lane_bufs[lane]
            lst = self.lane_streams[lane]
            sl = ctypes.c_void_p(lst.cuda_stream)
            B._check(L.gs_render_fwd(ctypes.byref(self.scene_struct), C.hp, C.dp, C.n, g.tile,
                                     ctypes.cast(g.bg, B._VP), P(lb["splats"]), P(lb["vals"]), P(lb["ranges"]),
                                     grp["cap"], P(g.num_keys[k:k + 1]), P(img), P(fT), P(nc), lb["ws"],
                                     lb["wsn"], sl))
            B._check(L.gs_l1_grad(P(img), P(tg), 3 * npx, ctypes.c_float(g.scale), P(dL), P(g.loss),
                                  1 if first and k == 0 and not multi else 0, sl))
            B._check(L.gs_rasterize_bwd(P(lb["splats"]), g.scene.n, C.hp, C.dp, C.n, g.tile, P(lb["vals"]),
                                        P(lb["ranges"]), ctypes.cast(g.bg, B._VP), P(fT), P(nc), P(dL),
                                        P(lb["sgrads"]), None, 0, sl))
            if multi and k > 0 and (k - 1) % self.lanes != lane:
                lst.wait_event(self.pb_events[k - 1])
            B._check(L.gs_project_bwd(ctypes.byref(self.scene_struct), C.hp, C.dp, C.n, P(lb["splats"]),
                                      P(lb["sgrads"]), P(gr["means"]), P(gr["log_scales"]), P(gr["quats"]),
                                      P(gr["opacity_logits"]), P(gr["sh"]), 0 if first else 1, sl))
            if multi:
                self.pb_events[k].record(lst)
            first = False
        if multi:
            for ls in self.lane_streams[1:]:
                self.stream.wait_stream(ls)
        if self.eye_stream is not None:
            # join the eyes' branch
            self.stream.wait_stream(self.eye_stream)

    def step(self, check: bool = False):
        """Run one step eagerly on this object's stream.  check: synchronise
        and raise GsError if a sub-batch or eye group needed more keys than
        its capacity (its images and gradients are then invalid)."""
        self.stream.wait_stream(torch.cuda.current_stream())
        self._enqueue()
        torch.cuda.current_stream().wait_stream(self.stream)
        if check and not self.keys_ok():
            raise B.GsError(B.GS_ERR_CAPACITY, "a sub-batch needed more keys than its capacity: "
                                               f"required {self.num_keys.cpu().tolist()}, capacities "
                                               f"{[g['cap'] for g in self.groups]}")

    def capture(self):
        """Record one step as a graph (nothing runs during the recording)."""
        torch.cuda.synchronize()
        with B.Graph.capture(self.stream) as cap:
            self._enqueue()
        self.graph = cap.graph
        return self.graph

    def replay(self):
        """Replay the recorded step.  Capacities are those of the recording:
        callers whose scene moves read keys_ok() after synchronising (or
        rebuild the step) to find an overflowed sub-batch."""
        self.stream.wait_stream(torch.cuda.current_stream())
        self.graph.launch(self.stream)
        torch.cuda.current_stream().wait_stream(self.stream)

    def keys_ok(self):
        """True if no sub-batch needed more keys than its capacity (reads back)."""
        caps = torch.tensor([g["cap"] for g in self.groups], dtype=torch.int64)
        ok = bool((self.num_keys.cpu() <= caps).all())
        if self.eye_groups:
            ecaps = torch.tensor([e["cap"] for e in self.eye_groups], dtype=torch.int64)
            ok = ok and bool((self.eye_num.cpu() <= ecaps).all())
        return ok
