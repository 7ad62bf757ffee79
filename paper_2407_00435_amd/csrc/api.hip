// C ABI of the library: argument checks, workspace layout and the
// composition of the stages.  Every entry point only enqueues on the given
// stream and never allocates device memory.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>

#include "common.hpp"
#include "kernels.hpp"
#include <new>

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok()
{
    g_err.clear();
    return GS_OK;
}

int hip_fail(hipError_t e, const char *where)
{
    return fail(GS_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

bool tile_ok(int T) { return T == 8 || T == 16 || T == 32; }

int check_cams(const gs_camera *ch, const gs_camera *cd, int V, int T, int64_t *tiles,
               int64_t *pixels)
{
    if (V < 1) return fail(GS_ERR_INVALID, "n_views must be >= 1 (got %d)", V);
    if (!ch || !cd) return fail(GS_ERR_INVALID, "camera arrays must not be NULL");
    if (!tile_ok(T)) return fail(GS_ERR_UNSUPPORTED, "tile size %d not in {8, 16, 32}", T);
    int64_t t = 0, p = 0;
    for (int v = 0; v < V; ++v) {
        const gs_camera &c = ch[v];
        if (c.width <= 0 || c.height <= 0 || c.width > 65536 || c.height > 65536)
            return fail(GS_ERR_INVALID, "camera %d: bad size %dx%d", v, c.width, c.height);
        if (!(c.fx > 0.f) || !(c.fy > 0.f) || !std::isfinite(c.cx) || !std::isfinite(c.cy))
            return fail(GS_ERR_INVALID, "camera %d: bad intrinsics", v);
        t += (int64_t)((c.width + T - 1) / T) * ((c.height + T - 1) / T);
        p += (int64_t)c.width * c.height;
    }
    if (t >= (1ll << 32)) return fail(GS_ERR_UNSUPPORTED, "too many tiles (%lld)", (long long)t);
    if (tiles) *tiles = t;
    if (pixels) *pixels = p;
    return GS_OK;
}

int check_scene(const gs_scene *s, bool levels)
{
    if (!s) return fail(GS_ERR_INVALID, "scene is NULL");
    if (s->n < 0) return fail(GS_ERR_INVALID, "n must be >= 0");
    if (s->sh_degree < 0 || s->sh_degree > 3)
        return fail(GS_ERR_UNSUPPORTED, "sh_degree %d not in 0..3", s->sh_degree);
    if (s->n > 0 && (!s->means || !s->log_scales || !s->quats || !s->opacity_logits || !s->sh))
        return fail(GS_ERR_INVALID, "scene parameter pointer is NULL");
    if (!aligned(s->quats, 16)) return fail(GS_ERR_INVALID, "quats must be 16-byte aligned");
    if ((s->sh_degree == 1 || s->sh_degree == 3) && !aligned(s->sh, 16))
        return fail(GS_ERR_INVALID, "sh must be 16-byte aligned");
    if (levels) {
        if (s->n_levels < 1 || s->n_levels > 4)
            return fail(GS_ERR_UNSUPPORTED, "n_levels %d not in 1..4", s->n_levels);
        if (s->n > 0 && !s->qbound) return fail(GS_ERR_INVALID, "qbound is NULL");
    }
    return GS_OK;
}

// ---------------------------------------------------------------------------
// Workspace layout (256-byte aligned sub-buffers).
struct Carve {
    size_t off = 0;
    char *base = nullptr;
    template <class P>
    P *take(size_t bytes)
    {
        off = (off + 255) & ~size_t(255);
        P *p = base ? reinterpret_cast<P *>(base + off) : nullptr;
        off += bytes;
        return p;
    }
};

void carve_bin(Carve &c, int V, int64_t E, uint64_t cap, int64_t tiles, BinScratch &bs)
{
    bs.dkey_a = c.take<uint32_t>(4 * E);
    bs.dval_a = c.take<uint32_t>(4 * E);
    bs.dkey_b = c.take<uint32_t>(4 * E);
    bs.dval_b = c.take<uint32_t>(4 * E);
    bs.rec = c.take<uint4>(16 * E);
    bs.rec_s = c.take<uint4>(16 * E);
    bs.cc_s = c.take<uint32_t>(4 * E);
    int64_t nb = (E + ENTRY_BLOCK - 1) / ENTRY_BLOCK + 1;
    bs.block_sums = c.take<uint64_t>(8 * nb);
    bs.block_sums2 = c.take<uint64_t>(8 * nb);
    bs.block_vis = c.take<uint32_t>(4 * nb);
    bs.vtab = c.take<int64_t>(16 * (int64_t)V);
    bs.stab = c.take<int4>(16 * (int64_t)V);
    bs.bbox = c.take<int32_t>(64 * (int64_t)V);
    bs.tkey_a = c.take<uint32_t>(4 * cap);
    bs.tkey_b = c.take<uint32_t>(4 * cap);
    bs.cpay_a = c.take<uint2>(8 * cap);
    bs.cpay_b = c.take<uint2>(8 * cap);
    const uint64_t chunks = bin_max_chunks(cap, tiles);
    bs.st_ranges = c.take<uint32_t>(8 * tiles);
    bs.st_cls = c.take<uint8_t>(4 * tiles);
    bs.chunk_off = c.take<uint32_t>(4 * (tiles + 1));
    bs.chunk = c.take<uint4>(16 * chunks);
    bs.ccnt = c.take<uint32_t>(4 * BIN_SUPER_TILE * BIN_SUPER_TILE * chunks);
    bs.tot = c.take<uint32_t>(4 * tiles);
    bs.tsum = c.take<uint64_t>(8 * (tiles / (SCAN_THREADS * SCAN_ITEMS) + 1));
    bs.counts = c.take<uint64_t>(8 * 8);
    bs.sat = c.take<uint32_t>(4 * 4 * tiles);
    bs.rs.hist = c.take<uint32_t>(4 * 4 * 256);
    uint64_t big = cap > (uint64_t)E ? cap : (uint64_t)E;
    bs.rs.status_words = radix_status_words(big);
    bs.rs.status = c.take<uint64_t>(2 * 8 * bs.rs.status_words);
    bs.rs.tickets = c.take<uint32_t>(4 * 4);
}

struct RenderBufs {
    gs_splat *splats;
    float *lvl;
    uint32_t *vals;
    uint32_t *ranges;
    uint8_t *pix_level;
    float *pix_weight;
    uint8_t *tile_level;
};

void carve_render(Carve &c, int64_t E, int L, uint64_t cap, int64_t tiles, int64_t pixels,
                  RenderBufs &rb)
{
    rb.splats = c.take<gs_splat>(sizeof(gs_splat) * E);
    rb.lvl = L > 0 ? c.take<float>(16 * E * L) : nullptr;
    rb.vals = c.take<uint32_t>(4 * cap);
    rb.ranges = c.take<uint32_t>(8 * tiles);
    rb.pix_level = L > 0 ? c.take<uint8_t>(pixels) : nullptr;
    rb.pix_weight = L > 0 ? c.take<float>(4 * pixels) : nullptr;
    rb.tile_level = L > 0 ? c.take<uint8_t>(2 * tiles) : nullptr;
}

// Compositing work queue (see raster.hip): off by default -- on MI355X the
// hardware dispatcher, one workgroup per tile in tile order, measured faster
// than the persistent queue on the foveated stereo frame (0.63-0.67 ms
// against 0.79 ms) -- and, when on, no split by default (tiles with the
// longest runs saturate within their first chunks, so splitting composites
// chunks that are then discarded).

// chunk partial per task: T*T pixels x 3 float4
size_t queue_task_bytes(const Tuning &tn, int T) { return 8 + 4 + (tn.raster_beta ? (size_t)T * T * 48 : 0); }

size_t queue_fixed_bytes(int64_t tiles) { return 256 + 8 * (size_t)tiles + 4 * 256; }

// Workspace for the queue of a compositing call over `tiles` tiles and at
// most `cap` keys (0 when the queue is switched off).
size_t raster_queue_bytes(const Tuning &tn, int64_t tiles, int T, uint64_t cap)
{
    if (!tn.raster_queue) return tn.raster_merge ? 4 * merge_scratch_words(tiles) + 256 : 0;
    return queue_fixed_bytes(tiles) + raster_queue_heavy_cap(tiles, T, cap, tn.raster_beta) * queue_task_bytes(tn, T);
}

// Tile-merging scratch at [base, base + bytes) (false when merging is off,
// the queue is on, or the space is too small).
bool carve_merge(const Tuning &tn, char *base, size_t bytes, int64_t tiles, MergeArgs &ma)
{
    if (tn.raster_queue || !tn.raster_merge || !base || bytes < 4 * merge_scratch_words(tiles)) return false;
    ma.scratch = reinterpret_cast<uint32_t *>(base);
    ma.beta = tn.raster_merge;
    return true;
}

// Lays the queue out in [base, base + bytes); the heavy-task capacity is what
// fits (tiles that do not fit are queued unsplit).  False if the queue is off
// or the space does not hold the fixed part.
bool carve_queue(const Tuning &tn, char *base, size_t bytes, int64_t tiles, int T, RasterQueueArgs &q)
{
    if (!tn.raster_queue || !base) return false;
    const size_t fixed = queue_fixed_bytes(tiles);
    if (bytes < fixed) return false;
    const size_t per = queue_task_bytes(tn, T);
    uint64_t hc = (bytes - fixed) / per;
    if (hc > (1u << 30)) hc = 1u << 30;
    for (;;) {
        Carve c;
        c.base = base;
        q.counts = c.take<uint32_t>(16);
        q.light = c.take<uint32_t>(8 * tiles);
        q.heavy = c.take<uint32_t>(8 * hc);
        q.merge_cnt = c.take<uint32_t>(4 * hc);
        q.part = tn.raster_beta ? c.take<float>((size_t)T * T * 48 * hc) : nullptr;
        if (c.off <= bytes || hc == 0) break;
        // alignment padding ate into the heavy part: shrink it
        const uint64_t over = (c.off - bytes + per - 1) / per;
        hc = hc > over ? hc - over : 0;
    }
    q.heavy_cap = (uint32_t)hc;
    q.light_cap = (uint32_t)tiles;
    q.beta = tn.raster_beta;
    q.heavy_min = tn.raster_heavy;
    q.grab = tn.raster_grab;
    return true;
}

// Every workspace starts with a status header (WS_HEADER bytes): the
// required key count and the capacity of the last binning that used it,
// read back by gs_poll_status.  A compositing call's work queue and every
// scratch area come after it.
constexpr size_t WS_HEADER = 256;

size_t bin_bytes(int V_, int64_t E, uint64_t cap, int64_t tiles)
{
    Carve c;
    c.take<uint64_t>(WS_HEADER);
    BinScratch bs;
    carve_bin(c, V_, E, cap, tiles, bs);
    return c.off + 256;
}

// The queue of a compositing call sits after the header of its workspace.
bool carve_queue_ws(const Tuning &tn, void *ws, size_t bytes, int64_t tiles, int T, RasterQueueArgs &q)
{
    if (!ws || bytes <= WS_HEADER) return false;
    return carve_queue(tn, (char *)ws + WS_HEADER, bytes - WS_HEADER, tiles, T, q);
}

bool carve_merge_ws(const Tuning &tn, void *ws, size_t bytes, int64_t tiles, MergeArgs &ma)
{
    if (!ws || bytes <= WS_HEADER) return false;
    return carve_merge(tn, (char *)ws + WS_HEADER, bytes - WS_HEADER, tiles, ma);
}

int check_ws(const void *ws, size_t have, size_t need)
{
    if (!ws) return fail(GS_ERR_INVALID, "workspace is NULL");
    if (!aligned(ws, 256)) return fail(GS_ERR_INVALID, "workspace must be 256-byte aligned");
    if (have < need)
        return fail(GS_ERR_CAPACITY, "workspace too small: %zu bytes given, %zu needed", have, need);
    return GS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Static scratch of gs_sort_pairs_static: the sort's digit counts, tickets,
// key count and lookback words for up to GS_SORT_STATIC_MAX_KEYS keys live
// in this array, one copy per device, held until the process ends.  Host code
// never uses the array's name (a host-side stand-in): its device address on
// each device is resolved once, when the first context for that device is
// created, and kept in g_scratch_ptr.
constexpr size_t SORT_STATIC_BYTES = 17u << 20;
static __device__ __align__(256) unsigned char scratch[SORT_STATIC_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Resolves the device address of `scratch` on `device` (once per device),
// with that device current; restores the caller's current device.
int setup_static_scratch(int device)
{
    if (device >= MAX_DEVICES) return fail(GS_ERR_UNSUPPORTED, "device %d: at most %d devices", device, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return GS_OK;
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (prev != device) hipSetDevice(prev);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress (static sort scratch)");
    g_scratch_ptr[device] = ptr;
    return GS_OK;
}

void *static_scratch(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace

// A library context: the device it was made for and the launch choices of
// the calls made with it.  Host state only.
struct gs_ctx {
    uint32_t magic;
    int device;
    Tuning tn;
    // view-by-view rendering: the second stream and its two events, made on
    // the first such call (on `side_device`), released by gs_destroy
    hipStream_t side = nullptr;
    hipEvent_t ev_bin = nullptr, ev_join = nullptr;
    int side_device = -1;
};

namespace {

constexpr uint32_t CTX_MAGIC = 0x67736374u;  // "gsct"

// The context is valid; checked before any other argument.
int check_ctx(const gs_ctx *ctx)
{
    if (!ctx) return fail(GS_ERR_INVALID, "context is NULL");
    if (ctx->magic != CTX_MAGIC) return fail(GS_ERR_INVALID, "not a live context (destroyed or corrupt)");
    return GS_OK;
}

// The context's device is the calling thread's current device; checked
// after the arguments, before anything is enqueued.
int check_device(const gs_ctx *ctx)
{
    int d = -1;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (d != ctx->device)
        return fail(GS_ERR_INVALID, "context is for device %d, the current device is %d", ctx->device, d);
    return GS_OK;
}

}  // namespace

extern "C" {

int gs_create(gs_ctx **out, int device)
{
    if (!out) return fail(GS_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (device < 0) return fail(GS_ERR_INVALID, "device %d < 0", device);
    int count = 0;
    // without a usable runtime the context still serves host-only calls
    // (workspace sizes, argument checks); a call that launches work checks
    // the device then
    if (hipGetDeviceCount(&count) == hipSuccess) {
        if (device >= count) return fail(GS_ERR_INVALID, "device %d does not exist (%d devices)", device, count);
        int r;
        if ((r = setup_static_scratch(device))) return r;
    }
    gs_ctx *c = new (std::nothrow) gs_ctx;
    if (!c) return fail(GS_ERR_INVALID, "out of host memory");
    c->magic = CTX_MAGIC;
    c->device = device;
    if (const char *s = std::getenv("GS_RADIX_PART")) {
        const int v = std::atoi(s);
        if (radix_part_ok(v)) c->tn.radix_part = v;
    }
    *out = c;
    return ok();
}

int gs_destroy(gs_ctx *ctx)
{
    if (!ctx) return ok();
    int r;
    if ((r = check_ctx(ctx))) return r;
    ctx->magic = 0;
    if (ctx->side) {
        int cur = 0;
        const bool have = hipGetDevice(&cur) == hipSuccess;
        if (hipSetDevice(ctx->side_device) == hipSuccess) {
            (void)hipStreamSynchronize(ctx->side);
            (void)hipStreamDestroy(ctx->side);
            (void)hipEventDestroy(ctx->ev_bin);
            (void)hipEventDestroy(ctx->ev_join);
        }
        if (have) (void)hipSetDevice(cur);
    }
    delete ctx;
    return ok();
}

int gs_poll_status(gs_ctx *ctx, const void *workspace, int *status, uint64_t *required_keys)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    if (!workspace || !status) return fail(GS_ERR_INVALID, "NULL workspace or status");
    if (!aligned(workspace, 256)) return fail(GS_ERR_INVALID, "workspace must be 256-byte aligned");
    if ((r = check_device(ctx))) return r;
    uint64_t h[2] = {0, 0};
    hipError_t e = hipMemcpy(h, workspace, sizeof(h), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "gs_poll_status");
    *status = h[0] > h[1] ? GS_ERR_CAPACITY : GS_OK;
    if (required_keys) *required_keys = h[0];
    return ok();
}

const char *gs_last_error(void) { return g_err.c_str(); }

int gs_version(void) { return 2; }

int gs_tile_count(const gs_camera *cams_host, int n_views, int tile_size, int64_t *n_tiles,
                  int64_t *n_pixels)
{
    int r = check_cams(cams_host, cams_host, n_views, tile_size, n_tiles, n_pixels);
    return r ? r : ok();
}

size_t gs_workspace_bytes(gs_ctx *ctx, const gs_camera *cams_host, int n_views, int32_t n, int tile_size,
                          uint64_t key_capacity)
{
    int64_t tiles = 0;
    if (check_ctx(ctx) || check_cams(cams_host, cams_host, n_views, tile_size, &tiles, nullptr)) return 0;
    return bin_bytes(n_views, (int64_t)n_views * (n > 0 ? n : 0), key_capacity, tiles) + WS_HEADER +
           raster_queue_bytes(ctx->tn, tiles, tile_size, key_capacity);
}

size_t gs_render_workspace_bytes(gs_ctx *ctx, const gs_camera *cams_host, int n_views, int32_t n, int n_levels,
                                 int tile_size, uint64_t key_capacity)
{
    int64_t tiles = 0, pixels = 0;
    if (check_ctx(ctx) || check_cams(cams_host, cams_host, n_views, tile_size, &tiles, &pixels)) return 0;
    int64_t E = (int64_t)n_views * (n > 0 ? n : 0);
    Carve c;
    c.take<uint64_t>(WS_HEADER);
    BinScratch bs;
    RenderBufs rb;
    carve_render(c, E, n_levels, key_capacity, tiles, pixels, rb);
    carve_bin(c, n_views, E, key_capacity, tiles, bs);
    return c.off + 512 + raster_queue_bytes(ctx->tn, tiles, tile_size, key_capacity);
}

int gs_project(gs_ctx *ctx, const gs_scene *scene, const gs_camera *cams_host, const gs_camera *cams_dev,
               int n_views, int tile_size, gs_splat *splats, float *lvl_rgba, void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    if ((r = check_scene(scene, false))) return r;
    if ((r = check_cams(cams_host, cams_dev, n_views, tile_size, nullptr, nullptr))) return r;
    if ((int64_t)n_views * scene->n >= (1ll << 32))
        return fail(GS_ERR_UNSUPPORTED, "n_views * n must be < 2^32");
    if (scene->n > 0 && !splats) return fail(GS_ERR_INVALID, "splats is NULL");
    if (!aligned(splats, 16) || !aligned(lvl_rgba, 16))
        return fail(GS_ERR_INVALID, "splats and lvl_rgba must be 16-byte aligned");
    if (lvl_rgba && (scene->n_levels < 1 || scene->n_levels > 4))
        return fail(GS_ERR_INVALID, "lvl_rgba given but n_levels = %d", scene->n_levels);
    if ((r = check_device(ctx))) return r;
    hipError_t e = launch_project(*scene, cams_dev, n_views, tile_size, splats, lvl_rgba,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gs_project");
    return ok();
}

int gs_bin_sort(gs_ctx *ctx, const gs_splat *splats, int32_t n, const gs_camera *cams_host,
                const gs_camera *cams_dev, int n_views, int tile_size,
                const uint8_t *tile_level, const uint8_t *qbound, uint32_t *vals,
                uint64_t *keys, uint64_t key_capacity, uint32_t *tile_ranges, uint32_t *hits,
                uint64_t *num_keys, void *workspace, size_t workspace_bytes, void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    int64_t tiles = 0;
    if ((r = check_cams(cams_host, cams_dev, n_views, tile_size, &tiles, nullptr))) return r;
    if (n < 0) return fail(GS_ERR_INVALID, "n must be >= 0");
    int64_t E = (int64_t)n_views * n;
    if (E >= (1ll << 32)) return fail(GS_ERR_UNSUPPORTED, "n_views * n must be < 2^32");
    if (key_capacity >= (1ull << 32)) return fail(GS_ERR_UNSUPPORTED, "key_capacity must be < 2^32");
    if ((n > 0 && !splats) || !tile_ranges || !num_keys || (key_capacity > 0 && !vals))
        return fail(GS_ERR_INVALID, "NULL output or input pointer");
    if (!aligned(splats, 16)) return fail(GS_ERR_INVALID, "splats must be 16-byte aligned");
    if ((tile_level != nullptr) != (qbound != nullptr))
        return fail(GS_ERR_INVALID, "tile_level and qbound go together");
    if ((r = check_ws(workspace, workspace_bytes, bin_bytes(n_views, E, key_capacity, tiles)))) return r;
    Carve c;
    c.base = (char *)workspace;
    uint64_t *status = c.take<uint64_t>(WS_HEADER);
    BinScratch bs;
    carve_bin(c, n_views, E, key_capacity, tiles, bs);
    bs.rs.part = ctx->tn.radix_part;
    if ((r = check_device(ctx))) return r;
    hipError_t e = launch_bin_sort(splats, n, cams_dev, cams_host, n_views, tiles,
                                   tile_size,
                                   tile_level, qbound, 4, vals, keys, key_capacity, tile_ranges,
                                   hits, num_keys, bs, ctx->tn.coarse_packed, status, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gs_bin_sort");
    return ok();
}

int gs_rasterize_fwd(gs_ctx *ctx, const gs_splat *splats, int32_t n, const gs_camera *cams_host,
                     const gs_camera *cams_dev, int n_views, int tile_size, const uint32_t *vals,
                     const uint32_t *tile_ranges, const float *bg, float *image, float *final_T,
                     uint32_t *n_contrib, uint32_t *dominated_px, uint64_t *stats,
                     void *workspace, size_t workspace_bytes, void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    int64_t tiles = 0;
    if ((r = check_cams(cams_host, cams_dev, n_views, tile_size, &tiles, nullptr))) return r;
    if (n < 0) return fail(GS_ERR_INVALID, "n must be >= 0");
    if (!tile_ranges || !image || !final_T || !n_contrib || (n > 0 && (!splats || !vals)))
        return fail(GS_ERR_INVALID, "NULL output or input pointer");
    if (!aligned(splats, 16)) return fail(GS_ERR_INVALID, "splats must be 16-byte aligned");
    if (workspace && !aligned(workspace, 256)) return fail(GS_ERR_INVALID, "workspace must be 256-byte aligned");
    RasterQueueArgs q;
    const bool queued = carve_queue_ws(ctx->tn, workspace, workspace_bytes, tiles, tile_size, q);
    MergeArgs ma;
    const bool merged = carve_merge_ws(ctx->tn, workspace, workspace_bytes, tiles, ma);
    const float zero[3] = {0.f, 0.f, 0.f};
    if ((r = check_device(ctx))) return r;
    hipError_t e = launch_raster_fwd(splats, n, cams_dev, n_views, tile_size, tiles, vals, tile_ranges,
                                     bg ? bg : zero, image, final_T, n_contrib, dominated_px, stats,
                                     queued ? &q : nullptr, (hipStream_t)stream, merged ? &ma : nullptr);
    if (e != hipSuccess) return hip_fail(e, "gs_rasterize_fwd");
    return ok();
}

int gs_rasterize_bwd(gs_ctx *ctx, const gs_splat *splats, int32_t n, const gs_camera *cams_host,
                     const gs_camera *cams_dev, int n_views, int tile_size, const uint32_t *vals,
                     const uint32_t *tile_ranges, const float *bg, const float *final_T,
                     const uint32_t *n_contrib, const float *dL_dimage, gs_splat_grad *grads,
                     void *workspace, size_t workspace_bytes, void *stream)
{
    (void)workspace;
    (void)workspace_bytes;
    int r;
    if ((r = check_ctx(ctx))) return r;
    int64_t tiles = 0;
    if ((r = check_cams(cams_host, cams_dev, n_views, tile_size, &tiles, nullptr))) return r;
    if (n < 0) return fail(GS_ERR_INVALID, "n must be >= 0");
    if (!tile_ranges || !final_T || !n_contrib || !dL_dimage ||
        (n > 0 && (!splats || !vals || !grads)))
        return fail(GS_ERR_INVALID, "NULL output or input pointer");
    if (!aligned(splats, 16)) return fail(GS_ERR_INVALID, "splats must be 16-byte aligned");
    const float zero[3] = {0.f, 0.f, 0.f};
    if ((r = check_device(ctx))) return r;
    hipError_t e = launch_raster_bwd(splats, n, cams_dev, n_views, tile_size, tiles, vals, tile_ranges,
                                     bg ? bg : zero, final_T, n_contrib, dL_dimage, grads,
                                     (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gs_rasterize_bwd");
    return ok();
}

int gs_project_bwd(gs_ctx *ctx, const gs_scene *scene, const gs_camera *cams_host, const gs_camera *cams_dev,
                   int n_views, const gs_splat *splats, const gs_splat_grad *grads, float *d_means,
                   float *d_log_scales, float *d_quats, float *d_opacity_logits, float *d_sh,
                   int accumulate, void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    if ((r = check_scene(scene, false))) return r;
    if (accumulate != 0 && accumulate != 1) return fail(GS_ERR_INVALID, "accumulate must be 0 or 1");
    if ((r = check_cams(cams_host, cams_dev, n_views, 16, nullptr, nullptr))) return r;
    if (scene->n > 0 &&
        (!splats || !grads || !d_means || !d_log_scales || !d_quats || !d_opacity_logits || !d_sh))
        return fail(GS_ERR_INVALID, "NULL output or input pointer");
    if (!aligned(d_quats, 16)) return fail(GS_ERR_INVALID, "d_quats must be 16-byte aligned");
    if ((scene->sh_degree == 1 || scene->sh_degree == 3) && !aligned(d_sh, 16))
        return fail(GS_ERR_INVALID, "d_sh must be 16-byte aligned");
    if ((r = check_device(ctx))) return r;
    hipError_t e = launch_project_bwd(*scene, cams_dev, n_views, splats, grads, d_means, d_log_scales,
                                      d_quats, d_opacity_logits, d_sh, accumulate, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gs_project_bwd");
    return ok();
}

int gs_fovea_prep(gs_ctx *ctx, const gs_camera *cams_host, const gs_camera *cams_dev, const gs_fovea *fov_host,
                  int n_eyes, int tile_size, int n_levels, uint8_t *pix_level, float *pix_weight,
                  uint8_t *tile_level, void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    int64_t tiles = 0, pixels = 0;
    if ((r = check_cams(cams_host, cams_dev, n_eyes, tile_size, &tiles, &pixels))) return r;
    if (n_eyes > 8) return fail(GS_ERR_UNSUPPORTED, "at most 8 eyes (got %d)", n_eyes);
    if (n_levels < 1 || n_levels > 4) return fail(GS_ERR_UNSUPPORTED, "n_levels %d not in 1..4", n_levels);
    if (!fov_host || !pix_level || !pix_weight || !tile_level)
        return fail(GS_ERR_INVALID, "NULL output or input pointer");
    for (int i = 0; i < n_eyes; ++i) {
        const gs_fovea &f = fov_host[i];
        if (!(f.band_deg >= 0.f) || !std::isfinite(f.gaze_x) || !std::isfinite(f.gaze_y))
            return fail(GS_ERR_INVALID, "eye %d: bad fovea parameters", i);
        for (int j = 0; j + 1 < n_levels; ++j) {
            if (j > 0 && !(f.ring_deg[j] - 0.5f * f.band_deg >= f.ring_deg[j - 1] + 0.5f * f.band_deg))
                return fail(GS_ERR_INVALID, "eye %d: ring bands overlap or are unordered", i);
        }
        if (n_levels > 1 && f.band_deg > 0.f && !(f.ring_deg[0] - 0.5f * f.band_deg >= 0.f))
            return fail(GS_ERR_INVALID, "eye %d: first band starts below 0 degrees", i);
    }
    if ((r = check_device(ctx))) return r;
    hipError_t e = launch_fovea_prep(cams_host, cams_dev, fov_host, n_eyes, tile_size, n_levels, pixels, tiles,
                                     pix_level, pix_weight, tile_level, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gs_fovea_prep");
    return ok();
}

int gs_rasterize_foveated(gs_ctx *ctx, const gs_splat *splats, const float *lvl_rgba, int32_t n,
                          const uint8_t *qbound, int n_levels, const gs_camera *cams_host,
                          const gs_camera *cams_dev, int n_eyes, int tile_size, const uint32_t *vals,
                          const uint32_t *tile_ranges, const uint8_t *pix_level,
                          const float *pix_weight, const float *bg, float *image, uint64_t *stats,
                          float *final_T2, uint32_t *n_contrib2, void *workspace, size_t workspace_bytes,
                          void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    int64_t tiles = 0;
    if ((r = check_cams(cams_host, cams_dev, n_eyes, tile_size, &tiles, nullptr))) return r;
    if (n < 0) return fail(GS_ERR_INVALID, "n must be >= 0");
    if (n_levels < 1 || n_levels > 4) return fail(GS_ERR_UNSUPPORTED, "n_levels %d not in 1..4", n_levels);
    if (!tile_ranges || !pix_level || !pix_weight || !image ||
        (n > 0 && (!splats || !lvl_rgba || !qbound || !vals)))
        return fail(GS_ERR_INVALID, "NULL output or input pointer");
    if (!aligned(splats, 16) || !aligned(lvl_rgba, 16))
        return fail(GS_ERR_INVALID, "splats and lvl_rgba must be 16-byte aligned");
    if (workspace && !aligned(workspace, 256)) return fail(GS_ERR_INVALID, "workspace must be 256-byte aligned");
    RasterQueueArgs q;
    const bool queued = carve_queue_ws(ctx->tn, workspace, workspace_bytes, tiles, tile_size, q);
    MergeArgs ma;
    const bool merged = carve_merge_ws(ctx->tn, workspace, workspace_bytes, tiles, ma);
    const float zero[3] = {0.f, 0.f, 0.f};
    if ((final_T2 != nullptr) != (n_contrib2 != nullptr))
        return fail(GS_ERR_INVALID, "final_T2 and n_contrib2 go together");
    if (!aligned(final_T2, 8) || !aligned(n_contrib2, 8))
        return fail(GS_ERR_INVALID, "final_T2 and n_contrib2 must be 8-byte aligned");
    if ((r = check_device(ctx))) return r;
    hipError_t e = launch_raster_fov(splats, lvl_rgba, n, qbound, n_levels, cams_dev, n_eyes, tile_size,
                                     tiles, vals, tile_ranges, pix_level, pix_weight, bg ? bg : zero,
                                     image, stats, final_T2, n_contrib2, queued ? &q : nullptr, (hipStream_t)stream,
                                     merged ? &ma : nullptr);
    if (e != hipSuccess) return hip_fail(e, "gs_rasterize_foveated");
    return ok();
}

int gs_rasterize_foveated_bwd(gs_ctx *ctx, const gs_splat *splats, const float *lvl_rgba, int32_t n, const uint8_t *qbound,
                              int n_levels, const gs_camera *cams_host, const gs_camera *cams_dev, int n_eyes,
                              int tile_size, const uint32_t *vals, const uint32_t *tile_ranges,
                              const uint8_t *pix_level, const float *pix_weight, const float *bg,
                              const float *final_T2, const uint32_t *n_contrib2, const float *dL_dimage,
                              gs_splat_grad *grads, float *lvl_grads, void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    int64_t tiles = 0;
    if ((r = check_cams(cams_host, cams_dev, n_eyes, tile_size, &tiles, nullptr))) return r;
    if (n < 0) return fail(GS_ERR_INVALID, "n must be >= 0");
    if (n_levels < 1 || n_levels > 4) return fail(GS_ERR_UNSUPPORTED, "n_levels %d not in 1..4", n_levels);
    if (!tile_ranges || !pix_level || !pix_weight || !final_T2 || !n_contrib2 || !dL_dimage ||
        (n > 0 && (!splats || !lvl_rgba || !qbound || !vals || !grads || !lvl_grads)))
        return fail(GS_ERR_INVALID, "NULL output or input pointer");
    if (!aligned(splats, 16) || !aligned(lvl_rgba, 16) || !aligned(lvl_grads, 16) || !aligned(grads, 16))
        return fail(GS_ERR_INVALID, "splats, lvl_rgba, grads and lvl_grads must be 16-byte aligned");
    if (!aligned(final_T2, 8) || !aligned(n_contrib2, 8))
        return fail(GS_ERR_INVALID, "final_T2 and n_contrib2 must be 8-byte aligned");
    const float zero[3] = {0.f, 0.f, 0.f};
    if ((r = check_device(ctx))) return r;
    hipError_t e = launch_raster_fov_bwd(splats, lvl_rgba, n, qbound, n_levels, cams_dev, n_eyes, tile_size, tiles,
                                         vals, tile_ranges, pix_level, pix_weight, bg ? bg : zero, final_T2,
                                         n_contrib2, dL_dimage, grads, lvl_grads, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gs_rasterize_foveated_bwd");
    return ok();
}

int gs_project_bwd_levels(gs_ctx *ctx, const gs_scene *scene, const gs_camera *cams_host, const gs_camera *cams_dev,
                          int n_views, const gs_splat *splats, const gs_splat_grad *grads, const float *lvl_grads,
                          float *d_means, float *d_log_scales, float *d_quats, float *d_opacity_logits,
                          float *d_sh, float *d_lvl_opacity_logits, float *d_lvl_sh_dc, int accumulate,
                          void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    if ((r = check_scene(scene, true))) return r;
    if ((r = check_cams(cams_host, cams_dev, n_views, 16, nullptr, nullptr))) return r;
    if (accumulate != 0 && accumulate != 1) return fail(GS_ERR_INVALID, "accumulate must be 0 or 1");
    if (scene->n_levels < 1 || scene->n_levels > 4)
        return fail(GS_ERR_UNSUPPORTED, "n_levels %d not in 1..4", scene->n_levels);
    if (scene->n > 0 && (!splats || !grads || !lvl_grads || !d_means || !d_log_scales || !d_quats ||
                         !d_opacity_logits || !d_sh))
        return fail(GS_ERR_INVALID, "NULL output or input pointer");
    if (scene->lvl_opacity_logits && scene->n > 0 && !d_lvl_opacity_logits)
        return fail(GS_ERR_INVALID, "the scene has level opacity logits: d_lvl_opacity_logits is needed");
    if (scene->lvl_sh_dc && scene->n > 0 && !d_lvl_sh_dc)
        return fail(GS_ERR_INVALID, "the scene has level DC colours: d_lvl_sh_dc is needed");
    if (!aligned(d_quats, 16) || !aligned(lvl_grads, 16)) return fail(GS_ERR_INVALID, "d_quats and lvl_grads must be 16-byte aligned");
    if ((scene->sh_degree == 1 || scene->sh_degree == 3) && !aligned(d_sh, 16))
        return fail(GS_ERR_INVALID, "d_sh must be 16-byte aligned");
    if ((r = check_device(ctx))) return r;
    hipError_t e = launch_project_bwd(*scene, cams_dev, n_views, splats, grads, d_means, d_log_scales, d_quats,
                                      d_opacity_logits, d_sh, accumulate, (hipStream_t)stream, lvl_grads,
                                      scene->lvl_opacity_logits ? d_lvl_opacity_logits : nullptr,
                                      scene->lvl_sh_dc ? d_lvl_sh_dc : nullptr);
    if (e != hipSuccess) return hip_fail(e, "gs_project_bwd_levels");
    return ok();
}

namespace {

// The context's second stream and events, made on the first call that needs
// them; a context keeps them on that device.
int side_stream(gs_ctx *ctx)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (ctx->side) {
        if (dev != ctx->side_device)
            return fail(GS_ERR_INVALID, "view-by-view rendering of one context stays on device %d (now on %d)",
                        ctx->side_device, dev);
        return GS_OK;
    }
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "hipStreamCreate");
    if ((e = hipEventCreateWithFlags(&a, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&b, hipEventDisableTiming)) != hipSuccess) {
        (void)hipStreamDestroy(s);
        if (a) (void)hipEventDestroy(a);
        return hip_fail(e, "hipEventCreate");
    }
    ctx->side = s;
    ctx->ev_bin = a;
    ctx->ev_join = b;
    ctx->side_device = dev;
    return GS_OK;
}

// Per-view slots of the workspace status header (in 8-byte words): the
// (required, capacity) pair each view's binning writes, then its key count.
constexpr int STATUS_VIEW_REQ = 4;
constexpr int STATUS_VIEW_NUM = 20;

// The incremental pipelining of Section 5.2 at view granularity: each view is
// binned on the caller's stream into its own cap / V slice of the keys, and
// composited on the context's second stream once its binning is done, so
// that view v's compositing overlaps view v + 1's binning.  Each view's keys,
// ranges and pixels are exactly those of the joint call (bit-identical
// images); the caller's stream waits for the last compositing.  The
// compositing work queue and tile merging are not used here (their scratch
// would be shared by the concurrent binning).
int render_views_streamed(gs_ctx *ctx, const gs_scene *scene, const gs_camera *cams_host, const gs_camera *cams_dev,
                          int V, int T, const float *bg, float *image, uint64_t key_capacity, uint64_t *num_keys,
                          uint64_t *status, const RenderBufs &rb, BinScratch &bs, hipStream_t st)
{
    int r;
    if ((r = side_stream(ctx))) return r;
    const int n = scene->n, L = scene->n_levels;
    const uint64_t cap_v = key_capacity / (uint64_t)V;
    const float zero[3] = {0.f, 0.f, 0.f};
    int64_t toff = 0, poff = 0;
    hipError_t e;
    for (int v = 0; v < V; ++v) {
        const int W = cams_host[v].width, H = cams_host[v].height;
        const int64_t tv = (int64_t)((W + T - 1) / T) * ((H + T - 1) / T);
        const gs_splat *sp = rb.splats + (int64_t)v * n;
        const float *lv = rb.lvl + (int64_t)v * n * L * 4;
        uint32_t *vals = rb.vals + (int64_t)v * cap_v;
        uint32_t *ranges = rb.ranges + 2 * toff;
        e = launch_bin_sort(sp, n, cams_dev + v, cams_host + v, 1, tv, T, rb.tile_level + 2 * toff, scene->qbound, L,
                            vals, nullptr, cap_v, ranges, nullptr, status + STATUS_VIEW_NUM + v, bs,
                            ctx->tn.coarse_packed, status + STATUS_VIEW_REQ + 2 * v, st);
        if (e != hipSuccess) return hip_fail(e, "gs_render_foveated (binning of a view)");
        if ((e = hipEventRecord(ctx->ev_bin, st)) != hipSuccess ||
            (e = hipStreamWaitEvent(ctx->side, ctx->ev_bin, 0)) != hipSuccess)
            return hip_fail(e, "gs_render_foveated (stream order)");
        e = launch_raster_fov(sp, lv, n, scene->qbound, L, cams_dev + v, 1, T, tv, vals, ranges, rb.pix_level + poff,
                              rb.pix_weight + poff, bg ? bg : zero, image + 3 * poff, nullptr, nullptr, nullptr,
                              nullptr, ctx->side, nullptr);
        if (e != hipSuccess) return hip_fail(e, "gs_render_foveated (compositing of a view)");
        toff += tv;
        poff += (int64_t)W * H;
    }
    if ((e = launch_status_views(status + STATUS_VIEW_REQ, status + STATUS_VIEW_NUM, V, key_capacity, status,
                                 num_keys, st)) != hipSuccess)
        return hip_fail(e, "gs_render_foveated (status)");
    if ((e = hipEventRecord(ctx->ev_join, ctx->side)) != hipSuccess ||
        (e = hipStreamWaitEvent(st, ctx->ev_join, 0)) != hipSuccess)
        return hip_fail(e, "gs_render_foveated (stream join)");
    return ok();
}

}  // namespace

int gs_render_foveated(gs_ctx *ctx, const gs_scene *scene, const gs_camera *cams_host, const gs_camera *cams_dev,
                       const gs_fovea *fov_host, int n_eyes, int tile_size, const float *bg,
                       float *image, uint64_t key_capacity, uint64_t *num_keys, void *workspace,
                       size_t workspace_bytes, void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    int64_t tiles = 0, pixels = 0;
    if ((r = check_scene(scene, true))) return r;
    if ((r = check_cams(cams_host, cams_dev, n_eyes, tile_size, &tiles, &pixels))) return r;
    if (n_eyes > 8) return fail(GS_ERR_UNSUPPORTED, "at most 8 eyes (got %d)", n_eyes);
    if (key_capacity >= (1ull << 32)) return fail(GS_ERR_UNSUPPORTED, "key_capacity must be < 2^32");
    if (!image || !num_keys || !fov_host) return fail(GS_ERR_INVALID, "NULL output or input pointer");
    int64_t E = (int64_t)n_eyes * scene->n;
    if (E >= (1ll << 32)) return fail(GS_ERR_UNSUPPORTED, "n_eyes * n must be < 2^32");
    int L = scene->n_levels;
    size_t need = gs_render_workspace_bytes(ctx, cams_host, n_eyes, scene->n, L, tile_size, key_capacity);
    if ((r = check_ws(workspace, workspace_bytes, need))) return r;
    Carve c;
    c.base = (char *)workspace;
    uint64_t *status = c.take<uint64_t>(WS_HEADER);
    RenderBufs rb;
    carve_render(c, E, L, key_capacity, tiles, pixels, rb);
    const size_t scratch_off = (c.off + 255) & ~size_t(255);  // binning scratch, then the compositing queue
    BinScratch bs;
    carve_bin(c, n_eyes, E, key_capacity, tiles, bs);
    bs.rs.part = ctx->tn.radix_part;
    if ((r = gs_fovea_prep(ctx, cams_host, cams_dev, fov_host, n_eyes, tile_size, L, rb.pix_level,
                           rb.pix_weight, rb.tile_level, stream)))
        return r;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (ctx->tn.stream_views && n_eyes > 1) {
        if ((r = gs_project(ctx, scene, cams_host, cams_dev, n_eyes, tile_size, rb.splats, rb.lvl, stream)))
            return r;
        return render_views_streamed(ctx, scene, cams_host, cams_dev, n_eyes, tile_size, bg, image, key_capacity,
                                     num_keys, status, rb, bs, st);
    }
    // The binning's set-up and level-filter tables go first, so that the
    // projection counts each entry's kept tiles while it has the splat in
    // registers; the binning then compacts the key words it wrote instead of
    // reading the splat records again.  Keys and ranges are those of the
    // separate stages.
    e = launch_bin_sort(rb.splats, scene->n, cams_dev, cams_host, n_eyes, tiles, tile_size, rb.tile_level,
                        scene->qbound, L, rb.vals, nullptr, key_capacity, rb.ranges, nullptr, num_keys, bs,
                        ctx->tn.coarse_packed, status, st, BIN_SETUP);
    if (e != hipSuccess) return hip_fail(e, "gs_render_foveated (binning set-up)");
    const ProjBin pb = bin_counting_args(bs, tiles);
    e = launch_project(*scene, cams_dev, n_eyes, tile_size, rb.splats, rb.lvl, st, &pb);
    if (e != hipSuccess) return hip_fail(e, "gs_render_foveated (projection)");
    e = launch_bin_sort(rb.splats, scene->n, cams_dev, cams_host, n_eyes, tiles, tile_size, rb.tile_level,
                        scene->qbound, L, rb.vals, nullptr, key_capacity, rb.ranges, nullptr, num_keys, bs,
                        ctx->tn.coarse_packed, status, st, BIN_COUNTED);
    if (e != hipSuccess) return hip_fail(e, "gs_render_foveated (binning)");
    const float zero[3] = {0.f, 0.f, 0.f};
    RasterQueueArgs q;
    const bool queued = carve_queue(ctx->tn, (char *)workspace + scratch_off, workspace_bytes - scratch_off,
                                    tiles, tile_size, q);
    MergeArgs ma;
    const bool merged = carve_merge(ctx->tn, (char *)workspace + scratch_off, workspace_bytes - scratch_off, tiles, ma);
    e = launch_raster_fov(rb.splats, rb.lvl, scene->n, scene->qbound, L, cams_dev, n_eyes, tile_size,
                          tiles, rb.vals, rb.ranges, rb.pix_level, rb.pix_weight, bg ? bg : zero, image,
                          nullptr, nullptr, nullptr, queued ? &q : nullptr, st, merged ? &ma : nullptr);
    if (e != hipSuccess) return hip_fail(e, "gs_render_foveated (compositing)");
    return ok();
}

int gs_render_fwd(gs_ctx *ctx, const gs_scene *scene, const gs_camera *cams_host, const gs_camera *cams_dev,
                  int n_views, int tile_size, const float *bg, gs_splat *splats, uint32_t *vals,
                  uint32_t *tile_ranges, uint64_t key_capacity, uint64_t *num_keys, float *image,
                  float *final_T, uint32_t *n_contrib, void *workspace, size_t workspace_bytes,
                  void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    int64_t tiles = 0;
    if ((r = check_scene(scene, false))) return r;
    if ((r = check_cams(cams_host, cams_dev, n_views, tile_size, &tiles, nullptr))) return r;
    const int64_t E = (int64_t)n_views * scene->n;
    if (E >= (1ll << 32)) return fail(GS_ERR_UNSUPPORTED, "n_views * n must be < 2^32");
    if (key_capacity >= (1ull << 32)) return fail(GS_ERR_UNSUPPORTED, "key_capacity must be < 2^32");
    if ((scene->n > 0 && !splats) || !tile_ranges || !num_keys || (key_capacity > 0 && !vals))
        return fail(GS_ERR_INVALID, "NULL output or input pointer");
    if (!aligned(splats, 16)) return fail(GS_ERR_INVALID, "splats must be 16-byte aligned");
    if ((r = check_ws(workspace, workspace_bytes, bin_bytes(n_views, E, key_capacity, tiles)))) return r;
    if ((r = check_device(ctx))) return r;
    Carve c;
    c.base = (char *)workspace;
    uint64_t *status = c.take<uint64_t>(WS_HEADER);
    BinScratch bs;
    carve_bin(c, n_views, E, key_capacity, tiles, bs);
    bs.rs.part = ctx->tn.radix_part;
    hipStream_t st = (hipStream_t)stream;
    // as in gs_render_foveated: the binning's set-up first, the projection
    // counts each entry's tiles, the binning compacts its key words (keys
    // and ranges are those of gs_project + gs_bin_sort)
    hipError_t e = launch_bin_sort(splats, scene->n, cams_dev, cams_host, n_views, tiles, tile_size, nullptr,
                                   nullptr, 4, vals, nullptr, key_capacity, tile_ranges, nullptr, num_keys, bs,
                                   ctx->tn.coarse_packed, status, st, BIN_SETUP);
    if (e != hipSuccess) return hip_fail(e, "gs_render_fwd (binning set-up)");
    const ProjBin pb = bin_counting_args(bs, tiles);
    e = launch_project(*scene, cams_dev, n_views, tile_size, splats, nullptr, st, &pb);
    if (e != hipSuccess) return hip_fail(e, "gs_render_fwd (projection)");
    e = launch_bin_sort(splats, scene->n, cams_dev, cams_host, n_views, tiles, tile_size, nullptr, nullptr, 4, vals,
                        nullptr, key_capacity, tile_ranges, nullptr, num_keys, bs, ctx->tn.coarse_packed, status, st,
                        BIN_COUNTED);
    if (e != hipSuccess) return hip_fail(e, "gs_render_fwd (binning)");
    return gs_rasterize_fwd(ctx, splats, scene->n, cams_host, cams_dev, n_views, tile_size, vals, tile_ranges,
                            bg, image, final_T, n_contrib, nullptr, nullptr, workspace, workspace_bytes,
                            stream);
}

size_t gs_sort_workspace_bytes(uint64_t n) { return radix_sort_scratch_bytes(n); }

int gs_l1_grad(gs_ctx *ctx, const float *image, const float *target, uint64_t n, float scale, float *dL_dimage,
               float *loss, int reset, void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    if (!loss || (n > 0 && (!image || !target || !dL_dimage)))
        return fail(GS_ERR_INVALID, "NULL output or input pointer");
    if (reset != 0 && reset != 1) return fail(GS_ERR_INVALID, "reset must be 0 or 1");
    if ((r = check_device(ctx))) return r;
    hipError_t e;
    if (reset && (e = launch_fill_u32(reinterpret_cast<uint32_t *>(loss), 0u, 1, (hipStream_t)stream)) !=
                     hipSuccess)
        return hip_fail(e, "gs_l1_grad");
    if ((e = launch_l1_grad(image, target, n, scale, dL_dimage, loss, (hipStream_t)stream)) != hipSuccess)
        return hip_fail(e, "gs_l1_grad");
    return ok();
}

int gs_ce_score(gs_ctx *ctx, const uint32_t *dominated, const uint32_t *hits, int32_t n, int n_views, float *ce, void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    if (n < 0 || n_views < 1) return fail(GS_ERR_INVALID, "n must be >= 0 and n_views >= 1");
    if ((int64_t)n * n_views >= (1ll << 32)) return fail(GS_ERR_UNSUPPORTED, "n_views * n must be < 2^32");
    if (n > 0 && (!dominated || !hits || !ce)) return fail(GS_ERR_INVALID, "NULL output or input pointer");
    if ((r = check_device(ctx))) return r;
    hipError_t e = launch_ce_score(dominated, hits, n, n_views, ce, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gs_ce_score");
    return ok();
}

size_t gs_select_workspace_bytes(int32_t n) { return select_scratch_bytes(n > 0 ? n : 0) + 256; }

int gs_select_lowest(gs_ctx *ctx, const float *ce, int32_t n, int32_t k, uint8_t *mask, uint32_t *idx, void *workspace,
                     size_t workspace_bytes, void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    if (n < 0) return fail(GS_ERR_INVALID, "n must be >= 0");
    if (n > 0 && (!ce || !mask)) return fail(GS_ERR_INVALID, "NULL output or input pointer");
    if (k < 0) k = 0;
    if (k > n) k = n;
    if (k > 0 && (r = check_ws(workspace, workspace_bytes, gs_select_workspace_bytes(n)))) return r;
    if ((r = check_device(ctx))) return r;
    if (k == 0) {
        hipError_t e = launch_fill_u8(mask, 0, n, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "gs_select_lowest");
        return ok();
    }
    hipError_t e = launch_select_lowest(ce, n, k, mask, idx, workspace, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gs_select_lowest");
    return ok();
}

int gs_weighted_scale(gs_ctx *ctx, const float *log_scales, const uint32_t *hits, int32_t n, int n_views, float threshold,
                      float gamma, float *ws, float *d_log_scales, int accumulate, void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    if (n < 0 || n_views < 1) return fail(GS_ERR_INVALID, "n must be >= 0 and n_views >= 1");
    if ((int64_t)n * n_views >= (1ll << 32)) return fail(GS_ERR_UNSUPPORTED, "n_views * n must be < 2^32");
    if (!ws || (n > 0 && (!log_scales || !hits))) return fail(GS_ERR_INVALID, "NULL output or input pointer");
    if (accumulate != 0 && accumulate != 1) return fail(GS_ERR_INVALID, "accumulate must be 0 or 1");
    if ((r = check_device(ctx))) return r;
    hipError_t e = launch_weighted_scale(log_scales, hits, n, n_views, threshold, gamma, ws, d_log_scales,
                                         accumulate, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gs_weighted_scale");
    return ok();
}

struct gs_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

int gs_graph_begin(void *stream)
{
    if (!stream) return fail(GS_ERR_INVALID, "graph capture needs a non-default stream");
    hipError_t e = hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "gs_graph_begin");
    return ok();
}

int gs_graph_end(void *stream, gs_graph **graph)
{
    if (!stream || !graph) return fail(GS_ERR_INVALID, "NULL stream or graph pointer");
    *graph = nullptr;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture((hipStream_t)stream, &g);
    if (e != hipSuccess) return hip_fail(e, "gs_graph_end (capture)");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(g);
        return hip_fail(e, "gs_graph_end (instantiate)");
    }
    gs_graph *out = new (std::nothrow) gs_graph{g, x};
    if (!out) {
        hipGraphExecDestroy(x);
        hipGraphDestroy(g);
        return fail(GS_ERR_INVALID, "out of host memory");
    }
    *graph = out;
    return ok();
}

int gs_graph_launch(gs_graph *graph, void *stream)
{
    if (!graph) return fail(GS_ERR_INVALID, "NULL graph");
    hipError_t e = hipGraphLaunch(graph->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gs_graph_launch");
    return ok();
}

int gs_graph_destroy(gs_graph *graph)
{
    if (!graph) return ok();
    hipGraphExecDestroy(graph->exec);
    hipGraphDestroy(graph->graph);
    delete graph;
    return ok();
}

int gs_hvsq_pooling(gs_ctx *ctx, const gs_camera *cams_host, const gs_camera *cams_dev, const gs_fovea *fov_host,
                    int n_views, float rho, int32_t *radius, void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    if ((r = check_cams(cams_host, cams_dev, n_views, 16, nullptr, nullptr))) return r;
    if (n_views > 8) return fail(GS_ERR_UNSUPPORTED, "at most 8 views (got %d)", n_views);
    if (!fov_host || !radius) return fail(GS_ERR_INVALID, "NULL output or input pointer");
    if (!(rho >= 0.f) || !std::isfinite(rho)) return fail(GS_ERR_INVALID, "rho must be finite and >= 0");
    if ((r = check_device(ctx))) return r;
    hipError_t e = launch_hvsq_radius(cams_host, cams_dev, fov_host, n_views, rho, radius, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gs_hvsq_pooling");
    return ok();
}

size_t gs_hvsq_workspace_bytes(gs_ctx *ctx, const gs_camera *cams_host, int n_views, int want_grad)
{
    if (check_ctx(ctx) || check_cams(cams_host, cams_host, n_views, 16, nullptr, nullptr)) return 0;
    return hvsq_scratch_bytes(cams_host, n_views, want_grad != 0);
}

int gs_hvsq(gs_ctx *ctx, const gs_camera *cams_host, const gs_camera *cams_dev, int n_views, const float *img_a,
            const float *img_r, const int32_t *radius, const uint8_t *region, int n_regions, double *sums,
            double *counts, double *terms, int grad_region, float *dL_da, void *workspace, size_t workspace_bytes,
            void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    if ((r = check_cams(cams_host, cams_dev, n_views, 16, nullptr, nullptr))) return r;
    if (n_regions < 0 || n_regions > GS_HVSQ_MAX_REGIONS)
        return fail(GS_ERR_UNSUPPORTED, "n_regions %d not in 0..%d", n_regions, GS_HVSQ_MAX_REGIONS);
    if (!img_a || !img_r || !radius || !sums || !counts) return fail(GS_ERR_INVALID, "NULL output or input pointer");
    if (n_regions > 0 && !region) return fail(GS_ERR_INVALID, "n_regions > 0 needs the region map");
    if (grad_region < -1 || grad_region > n_regions)
        return fail(GS_ERR_INVALID, "grad_region %d not in -1..n_regions", grad_region);
    if (grad_region >= 0 && !dL_da) return fail(GS_ERR_INVALID, "grad_region >= 0 needs dL_da");
    const bool grad = grad_region >= 0;
    if ((r = check_ws(workspace, workspace_bytes, hvsq_scratch_bytes(cams_host, n_views, grad)))) return r;
    if ((r = check_device(ctx))) return r;
    hipError_t e = launch_hvsq(cams_host, cams_dev, n_views, img_a, img_r, radius, region, n_regions, sums, counts,
                               terms, grad ? grad_region : -1, grad ? dL_da : nullptr, workspace, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gs_hvsq");
    return ok();
}

int gs_set_tuning(gs_ctx *ctx, const char *name, int64_t value)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    if (!name) return fail(GS_ERR_INVALID, "tuning name is NULL");
    Tuning &tn = ctx->tn;
    std::string k(name);
    if (k == "raster_queue") {
        if (value != 0 && value != 1) return fail(GS_ERR_INVALID, "raster_queue must be 0 or 1");
        tn.raster_queue = (int)value;
        return ok();
    }
    if (k == "raster_grab") {
        if (value < 1 || value > 64) return fail(GS_ERR_INVALID, "raster_grab must be in 1..64");
        tn.raster_grab = (uint32_t)value;
        return ok();
    }
    if (k == "raster_heavy") {
        if (value < 0 || value > (1ll << 31)) return fail(GS_ERR_INVALID, "raster_heavy must be in 0..2^31");
        tn.raster_heavy = (uint32_t)value;
        return ok();
    }
    if (k == "raster_split") {
        if (value != 0 && (value < 256 || value > (1 << 24)))
            return fail(GS_ERR_INVALID, "raster_split must be 0 or in 256..2^24");
        tn.raster_beta = (uint32_t)value;
        return ok();
    }
    if (k == "raster_merge") {
        if (value < 0 || value > (1ll << 31)) return fail(GS_ERR_INVALID, "raster_merge must be in 0..2^31");
        tn.raster_merge = (uint32_t)value;
        return ok();
    }
    if (k == "stream_views") {
        if (value != 0 && value != 1) return fail(GS_ERR_INVALID, "stream_views must be 0 or 1");
        tn.stream_views = (int)value;
        return ok();
    }
    if (k == "coarse_packed") {
        if (value != 0 && value != 1) return fail(GS_ERR_INVALID, "coarse_packed must be 0 or 1");
        tn.coarse_packed = value != 0;
        return ok();
    }
    if (k == "radix_part") {
        if (!radix_part_ok((int)value)) return fail(GS_ERR_INVALID, "radix_part must be 4096, 8192 or 16384");
        tn.radix_part = (int)value;
        return ok();
    }
    return fail(GS_ERR_INVALID, "unknown tuning knob '%s'", name);
}

int gs_get_tuning(gs_ctx *ctx, const char *name, int64_t *value)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    if (!name || !value) return fail(GS_ERR_INVALID, "NULL name or value");
    const Tuning &tn = ctx->tn;
    std::string k(name);
    if (k == "raster_queue") *value = tn.raster_queue;
    else if (k == "raster_grab") *value = tn.raster_grab;
    else if (k == "raster_heavy") *value = tn.raster_heavy;
    else if (k == "raster_split") *value = tn.raster_beta;
    else if (k == "raster_merge") *value = tn.raster_merge;
    else if (k == "coarse_packed") *value = tn.coarse_packed ? 1 : 0;
    else if (k == "stream_views") *value = tn.stream_views;
    else if (k == "radix_part") *value = tn.radix_part;
    else return fail(GS_ERR_INVALID, "unknown tuning knob '%s'", name);
    return ok();
}

}  // extern "C"

namespace {

// The sort of gs_sort_pairs / gs_sort_pairs_static with its scratch at ws.
int sort_pairs_with(gs_ctx *ctx, uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp, uint32_t *vals_tmp, uint64_t n,
                    int bits, void *ws, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    bool in_tmp = false;
    hipError_t e = radix_sort_standalone(keys, vals, keys_tmp, vals_tmp, n, bits, ws, ctx->tn.radix_part, &in_tmp,
                                         st);
    if (e == hipSuccess && in_tmp) {
        e = hipMemcpyAsync(keys, keys_tmp, 4 * n, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(vals, vals_tmp, 4 * n, hipMemcpyDeviceToDevice, st);
    }
    if (e != hipSuccess) return hip_fail(e, "sort");
    return ok();
}

}  // namespace

extern "C" {

int gs_sort_pairs(gs_ctx *ctx, uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp, uint32_t *vals_tmp, uint64_t n,
                  int bits, void *workspace, size_t workspace_bytes, void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    if (bits < 0 || bits > 32) return fail(GS_ERR_INVALID, "bits %d not in 0..32", bits);
    if (n >= (1ull << 32)) return fail(GS_ERR_UNSUPPORTED, "n must be < 2^32");
    if (n > 0 && (!keys || !vals || !keys_tmp || !vals_tmp))
        return fail(GS_ERR_INVALID, "NULL key or value array");
    if ((r = check_ws(workspace, workspace_bytes, radix_sort_scratch_bytes(n)))) return r;
    if (n == 0 || bits == 0) return ok();
    if ((r = check_device(ctx))) return r;
    return sort_pairs_with(ctx, keys, vals, keys_tmp, vals_tmp, n, bits, workspace, stream);
}

int gs_sort_pairs_static(gs_ctx *ctx, uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp, uint32_t *vals_tmp,
                         uint64_t n, int bits, void *stream)
{
    int r;
    if ((r = check_ctx(ctx))) return r;
    if (bits < 0 || bits > 32) return fail(GS_ERR_INVALID, "bits %d not in 0..32", bits);
    if (n > GS_SORT_STATIC_MAX_KEYS)
        return fail(GS_ERR_CAPACITY, "n = %llu keys exceeds the static scratch's maximum of %llu keys",
                    (unsigned long long)n, (unsigned long long)GS_SORT_STATIC_MAX_KEYS);
    if (n > 0 && (!keys || !vals || !keys_tmp || !vals_tmp))
        return fail(GS_ERR_INVALID, "NULL key or value array");
    if (n == 0 || bits == 0) return ok();
    if ((r = check_device(ctx))) return r;
    void *ws = static_scratch(ctx->device);
    if (!ws)
        return fail(GS_ERR_HIP, "no static scratch on device %d (its context was made without a HIP runtime)",
                    ctx->device);
    if (radix_sort_scratch_bytes(n) > SORT_STATIC_BYTES)
        return fail(GS_ERR_CAPACITY, "static scratch too small for %llu keys", (unsigned long long)n);
    return sort_pairs_with(ctx, keys, vals, keys_tmp, vals_tmp, n, bits, ws, stream);
}

}  // extern "C"
