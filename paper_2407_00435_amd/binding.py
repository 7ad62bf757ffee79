"""ctypes binding of the C ABI in ``include/gs.h``.

Argument marshalling only: torch tensors supply device pointers and the
current HIP stream; every computation happens in ``libgsmi.so``.  Function
names match the C entry points.

Contexts: the C calls that launch work take a ``gs_ctx`` first.  Each host
thread has a current :class:`Context` (one per thread and device, made on
first use, or the one entered with ``with Context(...)``); :func:`lib`
returns the library with that context bound as the first argument of every
call that takes one, so the wrappers below and their callers pass the other
arguments only.  :func:`raw_lib` is the unbound library.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libgsmi.so")

GS_OK, GS_ERR_INVALID, GS_ERR_UNSUPPORTED, GS_ERR_CAPACITY, GS_ERR_HIP = 0, -1, -2, -3, -4


class GsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gs error {code}: {msg}")
        self.code = code


class GsCamera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3),
                ("near_z", ctypes.c_float)]


class GsScene(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("sh_degree", ctypes.c_int32),
                ("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacity_logits", ctypes.c_void_p),
                ("sh", ctypes.c_void_p), ("qbound", ctypes.c_void_p),
                ("n_levels", ctypes.c_int32),
                ("lvl_opacity_logits", ctypes.c_void_p), ("lvl_sh_dc", ctypes.c_void_p)]


class GsFovea(ctypes.Structure):
    _fields_ = [("gaze_x", ctypes.c_float), ("gaze_y", ctypes.c_float),
                ("ring_deg", ctypes.c_float * 3), ("band_deg", ctypes.c_float)]


assert ctypes.sizeof(GsCamera) == 76
assert ctypes.sizeof(GsFovea) == 24

_lib = None
_VP = ctypes.c_void_p
_I = ctypes.c_int
_I32 = ctypes.c_int32
_U64 = ctypes.c_uint64
_SZ = ctypes.c_size_t
_PC = ctypes.POINTER(GsCamera)
_PS = ctypes.POINTER(GsScene)
_PF = ctypes.POINTER(GsFovea)

_SIGS = {
    "gs_last_error": ([], ctypes.c_char_p),
    "gs_version": ([], _I),
    "gs_create": ([ctypes.POINTER(_VP), _I], _I),
    "gs_destroy": ([_VP], _I),
    "gs_poll_status": ([_VP, ctypes.POINTER(_I), ctypes.POINTER(_U64)], _I),
    "gs_get_tuning": ([ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)], _I),
    "gs_tile_count": ([_PC, _I, _I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], _I),
    "gs_workspace_bytes": ([_PC, _I, _I32, _I, _U64], _SZ),
    "gs_render_workspace_bytes": ([_PC, _I, _I32, _I, _I, _U64], _SZ),
    "gs_project": ([_PS, _PC, _VP, _I, _I, _VP, _VP, _VP], _I),
    "gs_bin_sort": ([_VP, _I32, _PC, _VP, _I, _I, _VP, _VP, _VP, _VP, _U64, _VP, _VP, _VP, _VP, _SZ,
                     _VP], _I),
    "gs_rasterize_fwd": ([_VP, _I32, _PC, _VP, _I, _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                          _SZ, _VP], _I),
    "gs_rasterize_bwd": ([_VP, _I32, _PC, _VP, _I, _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _SZ,
                          _VP], _I),
    "gs_project_bwd": ([_PS, _PC, _VP, _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _I, _VP], _I),
    "gs_fovea_prep": ([_PC, _VP, _PF, _I, _I, _I, _VP, _VP, _VP, _VP], _I),
    "gs_rasterize_foveated": ([_VP, _VP, _I32, _VP, _I, _PC, _VP, _I, _I, _VP, _VP, _VP, _VP, _VP,
                               _VP, _VP, _VP, _VP, _VP, _SZ, _VP], _I),
    "gs_rasterize_foveated_bwd": ([_VP, _VP, _I32, _VP, _I, _PC, _VP, _I, _I, _VP, _VP, _VP, _VP, _VP,
                                   _VP, _VP, _VP, _VP, _VP, _VP], _I),
    "gs_project_bwd_levels": ([_PS, _PC, _VP, _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _I,
                               _VP], _I),
    "gs_render_foveated": ([_PS, _PC, _VP, _PF, _I, _I, _VP, _VP, _U64, _VP, _VP, _SZ, _VP], _I),
    "gs_render_fwd": ([_PS, _PC, _VP, _I, _I, _VP, _VP, _VP, _VP, _U64, _VP, _VP, _VP, _VP, _VP, _SZ,
                       _VP], _I),
    "gs_sort_workspace_bytes": ([_U64], _SZ),
    "gs_set_tuning": ([ctypes.c_char_p, ctypes.c_int64], _I),
    "gs_sort_pairs": ([_VP, _VP, _VP, _VP, _U64, _I, _VP, _SZ, _VP], _I),
    "gs_sort_pairs_static": ([_VP, _VP, _VP, _VP, _U64, _I, _VP], _I),
    "gs_l1_grad": ([_VP, _VP, _U64, ctypes.c_float, _VP, _VP, _I, _VP], _I),
    "gs_ce_score": ([_VP, _VP, _I32, _I, _VP, _VP], _I),
    "gs_select_workspace_bytes": ([_I32], _SZ),
    "gs_select_lowest": ([_VP, _I32, _I32, _VP, _VP, _VP, _SZ, _VP], _I),
    "gs_weighted_scale": ([_VP, _VP, _I32, _I, ctypes.c_float, ctypes.c_float, _VP, _VP, _I, _VP], _I),
    "gs_hvsq_pooling": ([_PC, _VP, _PF, _I, ctypes.c_float, _VP, _VP], _I),
    "gs_hvsq_workspace_bytes": ([_PC, _I, _I], _SZ),
    "gs_hvsq": ([_PC, _VP, _I, _VP, _VP, _VP, _VP, _I, _VP, _VP, _VP, _I, _VP, _VP, _SZ, _VP], _I),
    "gs_graph_begin": ([_VP], _I),
    "gs_graph_end": ([_VP, ctypes.POINTER(_VP)], _I),
    "gs_graph_launch": ([_VP, _VP], _I),
    "gs_graph_destroy": ([_VP], _I),
}
# calls whose first C argument is the context (the signatures above list the
# other arguments; the context pointer is prepended here)
CTX_FIRST = frozenset((
    "gs_workspace_bytes", "gs_render_workspace_bytes", "gs_project", "gs_bin_sort", "gs_rasterize_fwd",
    "gs_rasterize_bwd", "gs_project_bwd", "gs_fovea_prep", "gs_rasterize_foveated",
    "gs_rasterize_foveated_bwd", "gs_project_bwd_levels", "gs_render_foveated", "gs_render_fwd",
    "gs_l1_grad", "gs_ce_score", "gs_select_lowest", "gs_weighted_scale", "gs_sort_pairs",
    "gs_sort_pairs_static", "gs_set_tuning", "gs_get_tuning", "gs_poll_status", "gs_hvsq_pooling",
    "gs_hvsq_workspace_bytes", "gs_hvsq"))
for _name in CTX_FIRST:
    _a, _r = _SIGS[_name]
    _SIGS[_name] = ([_VP] + list(_a), _r)
EXPORTED = tuple(_SIGS)


def raw_lib():
    """Load libgsmi.so (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path):
            raise RuntimeError(f"{lib_path} is missing; build it with "
                               "paper_2407_00435_amd/build.py (hipcc, gfx950)")
        L = ctypes.CDLL(lib_path)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


class Context:
    """A library context (``gs_ctx``) for one device: its tuning applies to
    the calls made with it.  ``with Context(...) as c:`` makes it the calling
    thread's current context for the block."""

    def __init__(self, device: int | None = None):
        if device is None:
            device = torch.cuda.current_device() if torch.cuda.is_available() else 0
        self.device = int(device)
        h = _VP()
        _check(raw_lib().gs_create(ctypes.byref(h), self.device))
        self._h = h

    @property
    def handle(self):
        return self._h

    def set_tuning(self, name: str, value: int):
        _check(raw_lib().gs_set_tuning(self._h, name.encode(), int(value)))

    def get_tuning(self, name: str) -> int:
        v = ctypes.c_int64()
        _check(raw_lib().gs_get_tuning(self._h, name.encode(), ctypes.byref(v)))
        return int(v.value)

    def poll_status(self, workspace) -> tuple[int, int]:
        """(status, required keys) of the last binning that used
        ``workspace`` (a tuple from ``_ws``); synchronises the current
        stream first."""
        torch.cuda.current_stream().synchronize()
        st, req = _I(), _U64()
        _check(raw_lib().gs_poll_status(self._h, workspace[1], ctypes.byref(st), ctypes.byref(req)))
        return int(st.value), int(req.value)

    def close(self):
        if getattr(self, "_h", None):
            raw_lib().gs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        _tls.__dict__.setdefault("stack", []).append(self)
        return self

    def __exit__(self, et, ev, tb):
        _tls.stack.pop()
        return False


_tls = threading.local()


def context() -> Context:
    """The calling thread's current context: the innermost ``with Context``,
    else the thread's own context for the current device (made on first
    use)."""
    stack = getattr(_tls, "stack", None)
    if stack:
        return stack[-1]
    dev = torch.cuda.current_device() if torch.cuda.is_available() else 0
    own = _tls.__dict__.setdefault("own", {})
    if dev not in own:
        own[dev] = Context(dev)
    return own[dev]


class _Bound:
    """The library with the current context bound as the first argument of
    the calls that take one."""

    def __init__(self, L):
        self._L = L

    def __getattr__(self, name):
        fn = getattr(self._L, name)
        if name in CTX_FIRST:
            h = context().handle
            return lambda *a: fn(h, *a)
        return fn


def lib():
    return _Bound(raw_lib())


def _check(code: int):
    if code != GS_OK:
        raise GsError(code, raw_lib().gs_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev():
    return torch.device("cuda", torch.cuda.current_device())


def _ws(nbytes: int):
    """A workspace: (tensor, 256-byte aligned pointer, usable bytes).  Its
    status header starts zeroed (no binning has used it)."""
    t = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=_dev())
    off = (-t.data_ptr()) % 256
    t[off:off + 256].zero_()
    return t, ctypes.c_void_p(t.data_ptr() + off), int(nbytes)


def _grown(required: int) -> int:
    """Key capacity after an overflow: the reported count plus a margin for
    later calls whose scene has moved a little."""
    return int(required * 1.25) + 1024


class KeyWatch:
    """Deferred overflow check of one binning call: its required key count is
    copied to pinned host memory behind it on the stream, and read once that
    copy has landed (never waiting for it)."""

    def __init__(self, num_keys: torch.Tensor, capacity: int):
        self.capacity = int(capacity)
        self.host = torch.empty(1, dtype=torch.int64, pin_memory=True)
        self.host.copy_(num_keys.view(1), non_blocking=True)
        self.event = torch.cuda.Event()
        self.event.record()

    def required(self):
        """The call's required key count, or None while not yet known."""
        if not self.event.query():
            return None
        return int(self.host[0])

    def overflowed(self) -> bool:
        r = self.required()
        return r is not None and r > self.capacity


class Cameras:
    """n_views cameras on the host (ctypes array) and the device (uint8 tensor)."""

    def __init__(self, cams, device=None):
        self.n = len(cams)
        self.host = (GsCamera * self.n)()
        for k, c in enumerate(cams):
            row = c.as_row() if hasattr(c, "as_row") else np.asarray(c, np.float64)
            h = self.host[k]
            h.width, h.height = int(row[0]), int(row[1])
            h.fx, h.fy, h.cx, h.cy = (float(x) for x in row[2:6])
            for j in range(9):
                h.R[j] = float(row[6 + j])
            for j in range(3):
                h.t[j] = float(row[15 + j])
            h.near_z = float(row[18])
        raw = bytes(self.host)
        self.dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device or _dev())
        self.sizes = [(int(c.width), int(c.height)) for c in self.host]
        # key capacity planned per (form, points, tile size) for calls that
        # do not give one, and the pending overflow checks of those calls
        self.key_capacity = {}
        self.key_watch = {}

    def planned_capacity(self, key, splats: torch.Tensor) -> int:
        """Key capacity for a binning of these cameras without a host sync:
        the first call per key reads the rectangle tile count of ``splats``
        once (an upper bound of the keys, exact without the level filter) and
        keeps it with a margin; later calls reuse it.  A pending check that
        has found an earlier call over its capacity raises GsError (that
        call's outputs were invalid) after raising the planned capacity."""
        pending = self.key_watch.get(key, [])
        for w in pending:
            if w.overflowed():
                self.key_watch[key] = []
                self.key_capacity[key] = max(self.key_capacity.get(key, 0), _grown(w.required()))
                raise GsError(GS_ERR_CAPACITY,
                              f"an earlier render of these cameras needed {w.required()} keys but had "
                              f"capacity for {w.capacity}: its image and gradients are invalid; the "
                              f"planned capacity is now {self.key_capacity[key]}")
        self.key_watch[key] = [w for w in pending if w.required() is None]
        if key not in self.key_capacity:
            bound = int(splat_fields(splats)["tiles_touched"].to(torch.int64).sum().item())
            self.key_capacity[key] = _grown(bound)
        return self.key_capacity[key]

    def watch(self, key, num_keys: torch.Tensor, capacity: int) -> KeyWatch:
        w = KeyWatch(num_keys, capacity)
        self.key_watch.setdefault(key, []).append(w)
        return w

    @property
    def hp(self):
        return ctypes.cast(self.host, _PC)

    @property
    def dp(self):
        return ctypes.c_void_p(self.dev.data_ptr())

    def tiles(self, tile_size: int):
        nt, npx = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().gs_tile_count(self.hp, self.n, tile_size, ctypes.byref(nt), ctypes.byref(npx)))
        return int(nt.value), int(npx.value)


class SceneTensors:
    """Device copies of a scene's parameter arrays (float32, contiguous)."""

    def __init__(self, scene=None, device=None, **tensors):
        dev = device or _dev()
        if scene is not None:
            tensors = dict(means=scene.means, log_scales=scene.log_scales, quats=scene.quats,
                           opacity_logits=scene.opacity_logits, sh=scene.sh,
                           qbound=scene.qbound, lvl_opacity_logits=scene.lvl_opacity_logits,
                           lvl_sh_dc=scene.lvl_sh_dc, sh_degree=scene.sh_degree)
        self.sh_degree = int(tensors.pop("sh_degree"))
        self.t = {}
        for k, v in tensors.items():
            if v is None:
                self.t[k] = None
                continue
            if not torch.is_tensor(v):
                v = torch.from_numpy(np.ascontiguousarray(v))
            dt = torch.uint8 if k == "qbound" else torch.float32
            self.t[k] = v.to(device=dev, dtype=dt).contiguous()
        self.n = int(self.t["means"].shape[0])
        self.n_levels = 0
        if self.t.get("qbound") is not None:
            if self.t.get("lvl_opacity_logits") is not None:
                self.n_levels = int(self.t["lvl_opacity_logits"].shape[0])
            elif self.t.get("lvl_sh_dc") is not None:
                self.n_levels = int(self.t["lvl_sh_dc"].shape[0])
            else:
                self.n_levels = 4

    def struct(self, levels: bool = True) -> GsScene:
        g = self.t.get
        s = GsScene()
        s.n, s.sh_degree = self.n, self.sh_degree
        s.means, s.log_scales, s.quats = (g("means").data_ptr(), g("log_scales").data_ptr(),
                                          g("quats").data_ptr())
        s.opacity_logits, s.sh = g("opacity_logits").data_ptr(), g("sh").data_ptr()
        if levels and g("qbound") is not None:
            s.qbound = g("qbound").data_ptr()
            s.n_levels = self.n_levels
            s.lvl_opacity_logits = g("lvl_opacity_logits").data_ptr() if g("lvl_opacity_logits") is not None else None
            s.lvl_sh_dc = g("lvl_sh_dc").data_ptr() if g("lvl_sh_dc") is not None else None
        return s


def splat_fields(splats: torch.Tensor) -> dict:
    """View a [V, n, 12] float32 splat tensor as named fields."""
    f = splats
    return dict(mean2d=f[..., 0:2], conic=f[..., 2:5], opacity=f[..., 5], color=f[..., 6:9],
                depth=f[..., 9], radius=f[..., 10].view(torch.int32),
                tiles_touched=f[..., 11].view(torch.int32))


def gs_tile_count(cams: Cameras, tile_size: int):
    return cams.tiles(tile_size)


def gs_workspace_bytes(cams: Cameras, n: int, tile_size: int, key_capacity: int) -> int:
    return int(lib().gs_workspace_bytes(cams.hp, cams.n, n, tile_size, key_capacity))


def gs_render_workspace_bytes(cams: Cameras, n: int, n_levels: int, tile_size: int,
                              key_capacity: int) -> int:
    return int(lib().gs_render_workspace_bytes(cams.hp, cams.n, n, n_levels, tile_size, key_capacity))


def gs_project(scene: SceneTensors, cams: Cameras, tile_size: int = 16, levels: bool = False):
    """Projection; returns splats [V, n, 12] (and lvl_rgba [V, n, L, 4] if levels)."""
    dev = scene.t["means"].device
    splats = torch.empty((cams.n, scene.n, 12), dtype=torch.float32, device=dev)
    lvl = None
    if levels:
        lvl = torch.empty((cams.n, scene.n, scene.n_levels, 4), dtype=torch.float32, device=dev)
    st = scene.struct(levels=levels)
    _check(lib().gs_project(ctypes.byref(st), cams.hp, cams.dp, cams.n, tile_size, _ptr(splats),
                            _ptr(lvl), _stream()))
    return (splats, lvl) if levels else splats


def gs_bin_sort(splats: torch.Tensor, n: int, cams: Cameras, tile_size: int = 16,
                tile_level=None, qbound=None, key_capacity: int | None = None,
                want_keys: bool = False, want_hits: bool = False, check: bool = False):
    """Binning + (tile, depth) sort.  key_capacity defaults to the sum of the
    unfiltered rectangle tile counts (exact for the plain path, an upper bound
    with the level filter); that default reads one scalar back from the device.
    check: synchronise, read the workspace status and, if the capacity was
    too small, run once more with the reported count (GsError if that fails
    too)."""
    if key_capacity is None:
        key_capacity = int(splat_fields(splats)["tiles_touched"].to(torch.int64).sum().item())

    def once(cap):
        dev = splats.device
        n_tiles, _ = cams.tiles(tile_size)
        cap = max(int(cap), 1)
        vals = torch.empty(cap, dtype=torch.int32, device=dev)
        keys = torch.empty(cap, dtype=torch.int64, device=dev) if want_keys else None
        ranges = torch.empty((n_tiles, 2), dtype=torch.int32, device=dev)
        hits = torch.empty((cams.n, n), dtype=torch.int32, device=dev) if want_hits else None
        num = torch.zeros(1, dtype=torch.int64, device=dev)
        ws = _ws(gs_workspace_bytes(cams, n, tile_size, cap))
        _check(lib().gs_bin_sort(_ptr(splats), n, cams.hp, cams.dp, cams.n, tile_size, _ptr(tile_level),
                                 _ptr(qbound), _ptr(vals), _ptr(keys), cap, _ptr(ranges), _ptr(hits),
                                 _ptr(num), ws[1], ws[2], _stream()))
        return dict(vals=vals, keys=keys, ranges=ranges, hits=hits, num_keys=num, capacity=cap, _ws=ws[0],
                    workspace=ws)

    return _checked(once, key_capacity, check)


def _checked(once, cap, check: bool):
    """Runs once(cap); with check, polls the status of its workspace and runs
    once more with the reported key count after an overflow."""
    out = once(cap)
    if not check:
        return out
    st, need = context().poll_status(out["workspace"])
    if st == GS_ERR_CAPACITY:
        out = once(need)
        st, need = context().poll_status(out["workspace"])
        if st == GS_ERR_CAPACITY:
            raise GsError(st, f"binning needs {need} keys, more than the capacity {out['capacity']} of the retry")
    return out


def gs_rasterize_fwd(splats, n, cams: Cameras, tile_size, vals, ranges, bg=(0.0, 0.0, 0.0),
                     want_dominated: bool = False, stats=None, workspace=None):
    """Forward compositing.  With ``workspace`` (a tuple from ``_ws``) the
    library runs its persistent work-queue compositor; without, one
    workgroup per tile."""
    dev = splats.device
    _, n_px = cams.tiles(tile_size)
    image = torch.empty(3 * n_px, dtype=torch.float32, device=dev)
    final_T = torch.empty(n_px, dtype=torch.float32, device=dev)
    n_contrib = torch.empty(n_px, dtype=torch.int32, device=dev)
    dom = torch.empty((cams.n, n), dtype=torch.int32, device=dev) if want_dominated else None
    bgc = (ctypes.c_float * 3)(*bg)
    ws, wsn = (workspace[1], workspace[2]) if workspace is not None else (None, 0)
    _check(lib().gs_rasterize_fwd(_ptr(splats), n, cams.hp, cams.dp, cams.n, tile_size, _ptr(vals),
                                  _ptr(ranges), ctypes.cast(bgc, _VP), _ptr(image), _ptr(final_T),
                                  _ptr(n_contrib), _ptr(dom), _ptr(stats), ws, wsn, _stream()))
    return dict(image=image, final_T=final_T, n_contrib=n_contrib, dominated=dom)


def gs_rasterize_bwd(splats, n, cams: Cameras, tile_size, vals, ranges, final_T, n_contrib,
                     dL_dimage, bg=(0.0, 0.0, 0.0)):
    grads = torch.empty((cams.n, n, 12), dtype=torch.float32, device=splats.device)
    bgc = (ctypes.c_float * 3)(*bg)
    _check(lib().gs_rasterize_bwd(_ptr(splats), n, cams.hp, cams.dp, cams.n, tile_size, _ptr(vals),
                                  _ptr(ranges), ctypes.cast(bgc, _VP), _ptr(final_T), _ptr(n_contrib),
                                  _ptr(dL_dimage.contiguous()), _ptr(grads), None, 0, _stream()))
    return grads


PARAM_NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh")


def gs_project_bwd(scene: SceneTensors, cams: Cameras, splats, grads, out=None, accumulate=False):
    """Parameter gradients summed over the views; written into ``out`` (a dict
    of tensors shaped like the parameters) when given, added to it if
    ``accumulate``."""
    t = scene.t
    if out is None:
        out = {k: torch.empty_like(t[k]) for k in PARAM_NAMES}
    st = scene.struct(levels=False)
    _check(lib().gs_project_bwd(ctypes.byref(st), cams.hp, cams.dp, cams.n, _ptr(splats), _ptr(grads),
                                _ptr(out["means"]), _ptr(out["log_scales"]), _ptr(out["quats"]),
                                _ptr(out["opacity_logits"]), _ptr(out["sh"]), int(bool(accumulate)),
                                _stream()))
    return out


def gs_l1_grad(image, target, scale, dL_dimage, loss, reset=True):
    """loss (+)= scale * sum|image - target|; dL_dimage = scale * sign(image - target)."""
    _check(lib().gs_l1_grad(_ptr(image), _ptr(target), image.numel(), float(scale), _ptr(dL_dimage),
                            _ptr(loss), int(bool(reset)), _stream()))


def gs_ce_score(dominated, hits):
    """CE per point from dominated [V, n] and hits [V, n] (int32/uint32 device tensors)."""
    V, n = dominated.shape
    ce = torch.empty(n, dtype=torch.float32, device=dominated.device)
    _check(lib().gs_ce_score(_ptr(dominated.contiguous()), _ptr(hits.contiguous()), n, V, _ptr(ce), _stream()))
    return ce


def gs_select_lowest(ce, k: int, want_indices: bool = True):
    """(mask uint8 [n], indices int32 [k] ascending) of the k lowest CE values."""
    n = ce.numel()
    kk = max(0, min(int(k), n))
    mask = torch.empty(n, dtype=torch.uint8, device=ce.device)
    idx = torch.empty(kk, dtype=torch.int32, device=ce.device) if want_indices else None
    ws = _ws(int(lib().gs_select_workspace_bytes(n)))
    _check(lib().gs_select_lowest(_ptr(ce.contiguous()), n, int(k), _ptr(mask), _ptr(idx) if kk else None, ws[1],
                                  ws[2], _stream()))
    return mask, idx


def gs_weighted_scale(log_scales, hits, threshold: float, gamma: float = 1.0, d_log_scales=None,
                      accumulate: bool = False):
    """(gamma * WS as a 1-element device tensor, d/d log_scales)."""
    V, n = hits.shape
    ws = torch.empty(1, dtype=torch.float32, device=hits.device)
    if d_log_scales is None:
        d_log_scales = torch.empty((n, 3), dtype=torch.float32, device=hits.device)
    _check(lib().gs_weighted_scale(_ptr(log_scales.contiguous()), _ptr(hits.contiguous()), n, V, float(threshold),
                                   float(gamma), _ptr(ws), _ptr(d_log_scales), int(bool(accumulate)), _stream()))
    return ws, d_log_scales


class Graph:
    """A recorded sequence of library calls on one stream, replayed with
    ``launch``.  Record with ``with Graph.capture(stream) as g: ...``."""

    def __init__(self, handle):
        self._h = handle

    @staticmethod
    def capture(stream):
        return _Capture(stream)

    def launch(self, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().gs_graph_launch(self._h, ctypes.c_void_p(s.cuda_stream)))

    def close(self):
        if self._h:
            _check(lib().gs_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Capture:
    def __init__(self, stream):
        self.stream = stream
        self.graph = None

    def __enter__(self):
        _check(lib().gs_graph_begin(ctypes.c_void_p(self.stream.cuda_stream)))
        return self

    def __exit__(self, et, ev, tb):
        h = ctypes.c_void_p()
        rc = lib().gs_graph_end(ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if et is None:
            _check(rc)
            self.graph = Graph(h)
        return False


def _foveae(foveae):
    arr = (GsFovea * len(foveae))()
    for k, f in enumerate(foveae):
        row = f.as_row() if hasattr(f, "as_row") else np.asarray(f, np.float64)
        arr[k].gaze_x, arr[k].gaze_y = float(row[0]), float(row[1])
        for j in range(3):
            arr[k].ring_deg[j] = float(row[2 + j])
        arr[k].band_deg = float(row[5])
    return arr


def gs_fovea_prep(cams: Cameras, foveae, tile_size: int = 16, n_levels: int = 4):
    dev = cams.dev.device
    n_tiles, n_px = cams.tiles(tile_size)
    pl = torch.empty(n_px, dtype=torch.uint8, device=dev)
    pw = torch.empty(n_px, dtype=torch.float32, device=dev)
    tl = torch.empty((n_tiles, 2), dtype=torch.uint8, device=dev)
    fa = _foveae(foveae)
    _check(lib().gs_fovea_prep(cams.hp, cams.dp, ctypes.cast(fa, _PF), cams.n, tile_size, n_levels,
                               _ptr(pl), _ptr(pw), _ptr(tl), _stream()))
    return dict(pix_level=pl, pix_weight=pw, tile_level=tl)


def gs_rasterize_foveated(splats, lvl_rgba, n, qbound, n_levels, cams: Cameras, tile_size, vals,
                          ranges, pix_level, pix_weight, bg=(0.0, 0.0, 0.0), stats=None, image=None,
                          workspace=None, keep=None):
    """Foveated compositing; returns the image.  ``keep`` = (final_T2, n_contrib2)
    tensors ([n_pixels, 2] float32 / int32) receive the reverse pass's start."""
    _, n_px = cams.tiles(tile_size)
    if image is None:
        image = torch.empty(3 * n_px, dtype=torch.float32, device=splats.device)
    bgc = (ctypes.c_float * 3)(*bg)
    ws, wsn = (workspace[1], workspace[2]) if workspace is not None else (None, 0)
    fT2, nc2 = keep if keep is not None else (None, None)
    _check(lib().gs_rasterize_foveated(_ptr(splats), _ptr(lvl_rgba), n, _ptr(qbound), n_levels, cams.hp,
                                       cams.dp, cams.n, tile_size, _ptr(vals), _ptr(ranges),
                                       _ptr(pix_level), _ptr(pix_weight), ctypes.cast(bgc, _VP),
                                       _ptr(image), _ptr(stats), _ptr(fT2), _ptr(nc2), ws, wsn, _stream()))
    return image


def gs_rasterize_foveated_bwd(splats, lvl_rgba, n, qbound, n_levels, cams: Cameras, tile_size, vals, ranges,
                              pix_level, pix_weight, final_T2, n_contrib2, dL_dimage, bg=(0.0, 0.0, 0.0)):
    """Reverse of the foveated compositing: (grads [V, n, 12], lvl_grads [V, n, L, 4])."""
    dev = splats.device
    grads = torch.empty((cams.n, n, 12), dtype=torch.float32, device=dev)
    lvl_grads = torch.empty((cams.n, n, n_levels, 4), dtype=torch.float32, device=dev)
    bgc = (ctypes.c_float * 3)(*bg)
    _check(lib().gs_rasterize_foveated_bwd(_ptr(splats), _ptr(lvl_rgba), n, _ptr(qbound), n_levels, cams.hp,
                                           cams.dp, cams.n, tile_size, _ptr(vals), _ptr(ranges), _ptr(pix_level),
                                           _ptr(pix_weight), ctypes.cast(bgc, _VP), _ptr(final_T2),
                                           _ptr(n_contrib2), _ptr(dL_dimage.contiguous()), _ptr(grads),
                                           _ptr(lvl_grads), _stream()))
    return grads, lvl_grads


LEVEL_PARAM_NAMES = PARAM_NAMES + ("lvl_opacity_logits", "lvl_sh_dc")


def gs_project_bwd_levels(scene: SceneTensors, cams: Cameras, splats, grads, lvl_grads, out=None,
                          accumulate=False):
    """Parameter gradients of the foveated render (base arrays plus the level
    versions present in the scene), summed over the eyes."""
    t = scene.t
    if out is None:
        out = {k: torch.empty_like(t[k]) for k in PARAM_NAMES}
        for k in ("lvl_opacity_logits", "lvl_sh_dc"):
            out[k] = torch.empty_like(t[k]) if t.get(k) is not None else None
    st = scene.struct(levels=True)
    _check(lib().gs_project_bwd_levels(ctypes.byref(st), cams.hp, cams.dp, cams.n, _ptr(splats), _ptr(grads),
                                       _ptr(lvl_grads), _ptr(out["means"]), _ptr(out["log_scales"]),
                                       _ptr(out["quats"]), _ptr(out["opacity_logits"]), _ptr(out["sh"]),
                                       _ptr(out.get("lvl_opacity_logits")), _ptr(out.get("lvl_sh_dc")),
                                       int(bool(accumulate)), _stream()))
    return out


def gs_render_foveated(scene: SceneTensors, cams: Cameras, foveae, tile_size: int = 16,
                       bg=(0.0, 0.0, 0.0), key_capacity: int = 0, image=None, workspace=None,
                       check: bool = False):
    """One-call foveated render; returns (image, num_keys tensor, workspace).
    check as in gs_bin_sort (a retry sizes a new workspace)."""
    dev = scene.t["means"].device
    _, n_px = cams.tiles(tile_size)
    if image is None:
        image = torch.empty(3 * n_px, dtype=torch.float32, device=dev)
    num = torch.zeros(1, dtype=torch.int64, device=dev)
    fa = _foveae(foveae)
    bgc = (ctypes.c_float * 3)(*bg)
    st = scene.struct(levels=True)

    def once(cap):
        nonlocal workspace
        need = gs_render_workspace_bytes(cams, scene.n, scene.n_levels, tile_size, cap)
        if workspace is None or workspace[2] < need:
            workspace = _ws(need)
        _check(lib().gs_render_foveated(ctypes.byref(st), cams.hp, cams.dp, ctypes.cast(fa, _PF), cams.n,
                                        tile_size, ctypes.cast(bgc, _VP), _ptr(image), int(cap),
                                        _ptr(num), workspace[1], workspace[2], _stream()))
        return dict(workspace=workspace, capacity=int(cap))

    out = _checked(once, key_capacity, check)
    return image, num, out["workspace"]


def gs_set_tuning(name: str, value: int):
    """Sets a tuning knob of the calling thread's current context."""
    context().set_tuning(name, value)


def gs_get_tuning(name: str) -> int:
    return context().get_tuning(name)


def gs_sort_pairs(keys: torch.Tensor, vals: torch.Tensor, bits: int, workspace=None):
    """Stable radix sort of int32 (uint32 bit pattern) keys and values, in place."""
    n = keys.numel()
    kt, vt = torch.empty_like(keys), torch.empty_like(vals)
    need = int(lib().gs_sort_workspace_bytes(n))
    if workspace is None or workspace[2] < need:
        workspace = _ws(need)
    _check(lib().gs_sort_pairs(_ptr(keys), _ptr(vals), _ptr(kt), _ptr(vt), n, bits, workspace[1],
                               workspace[2], _stream()))
    return workspace


def gs_hvsq_pooling(cams: Cameras, foveae, rho: float):
    """Pooling half-widths floor(rho * eccentricity) of every pixel (int32 [n_pixels])."""
    _, n_px = cams.tiles(16)
    radius = torch.empty(n_px, dtype=torch.int32, device=cams.dev.device)
    fa = _foveae(foveae)
    _check(lib().gs_hvsq_pooling(cams.hp, cams.dp, ctypes.cast(fa, _PF), cams.n, float(rho), _ptr(radius),
                                 _stream()))
    return radius


def gs_hvsq(img_a, img_r, cams: Cameras, radius, region=None, n_regions: int = 0, grad_region: int = -1,
            want_terms: bool = False, workspace=None):
    """HVSQ of img_a against img_r (planar float images of ``cams``): per view
    and region the sums and counts of the per-pixel terms, their means
    ("hvsq", [n_views][n_regions + 1], the last column the whole view),
    optionally the per-pixel terms and, for grad_region >= 0, the gradient of
    the sum over views of the region's HVSQ with respect to img_a."""
    dev = img_a.device
    _, n_px = cams.tiles(16)
    sums = torch.empty((cams.n, n_regions + 1), dtype=torch.float64, device=dev)
    counts = torch.empty_like(sums)
    terms = torch.empty(n_px, dtype=torch.float64, device=dev) if want_terms else None
    grad = torch.empty_like(img_a) if grad_region >= 0 else None
    need = int(lib().gs_hvsq_workspace_bytes(cams.hp, cams.n, int(grad_region >= 0)))
    if workspace is None or workspace[2] < need:
        workspace = _ws(need)
    _check(lib().gs_hvsq(cams.hp, cams.dp, cams.n, _ptr(img_a.contiguous()), _ptr(img_r.contiguous()),
                         _ptr(radius), _ptr(region), int(n_regions), _ptr(sums), _ptr(counts), _ptr(terms),
                         int(grad_region), _ptr(grad), workspace[1], workspace[2], _stream()))
    return dict(sums=sums, counts=counts, hvsq=sums / counts.clamp(min=1), terms=terms, grad=grad,
                workspace=workspace)


SORT_STATIC_MAX_KEYS = 1 << 24


def gs_sort_pairs_static(keys: torch.Tensor, vals: torch.Tensor, bits: int, tmp=None):
    """gs_sort_pairs without a workspace (the library's static scratch): in
    place, n <= SORT_STATIC_MAX_KEYS.  ``tmp`` = (keys_tmp, vals_tmp)
    preallocated by the caller, or None to allocate them here."""
    n = keys.numel()
    kt, vt = tmp if tmp is not None else (torch.empty_like(keys), torch.empty_like(vals))
    _check(lib().gs_sort_pairs_static(_ptr(keys), _ptr(vals), _ptr(kt), _ptr(vt), n, bits, _stream()))


def gs_render_fwd(scene: SceneTensors, cams: Cameras, tile_size: int = 16, bg=(0.0, 0.0, 0.0),
                  key_capacity: int = 0, workspace=None, check: bool = False):
    """One-call plain render; check as in gs_bin_sort (a retry allocates new
    buffers and workspace)."""
    dev = scene.t["means"].device
    n_tiles, n_px = cams.tiles(tile_size)

    def once(cap):
        nonlocal workspace
        cap = max(int(cap), 1)
        out = dict(splats=torch.empty((cams.n, scene.n, 12), dtype=torch.float32, device=dev),
                   vals=torch.empty(cap, dtype=torch.int32, device=dev),
                   ranges=torch.empty((n_tiles, 2), dtype=torch.int32, device=dev),
                   num_keys=torch.zeros(1, dtype=torch.int64, device=dev),
                   image=torch.empty(3 * n_px, dtype=torch.float32, device=dev),
                   final_T=torch.empty(n_px, dtype=torch.float32, device=dev),
                   n_contrib=torch.empty(n_px, dtype=torch.int32, device=dev), capacity=cap)
        need = gs_workspace_bytes(cams, scene.n, tile_size, cap)
        if workspace is None or workspace[2] < need:
            workspace = _ws(need)
        bgc = (ctypes.c_float * 3)(*bg)
        st = scene.struct(levels=False)
        _check(lib().gs_render_fwd(ctypes.byref(st), cams.hp, cams.dp, cams.n, tile_size,
                                   ctypes.cast(bgc, _VP), _ptr(out["splats"]), _ptr(out["vals"]),
                                   _ptr(out["ranges"]), cap, _ptr(out["num_keys"]), _ptr(out["image"]),
                                   _ptr(out["final_T"]), _ptr(out["n_contrib"]), workspace[1], workspace[2],
                                   _stream()))
        out["workspace"] = workspace
        return out

    return _checked(once, key_capacity, check)
