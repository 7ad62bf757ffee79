/*
 * gs.h -- C ABI of the MI355X (gfx950) Gaussian-splatting rasterizer.
 *
 * The library renders images from 3D Gaussian points in the three stages of
 * the point-based neural rendering pipeline (Section 2.1): projection of each
 * ellipsoid to a screen-space ellipse with a spherical-harmonic colour
 * (Eq. 1b, 1c), per-tile depth sorting, and per-pixel front-to-back
 * integration (Eq. 1a).  The foveated form (Section 4.1, 4.2) renders
 * eccentricity rings from nested point subsets with per-level opacity and DC
 * colour and blends the rings at their borders.
 *
 * Conventions shared by every entry point
 *   - Calls that launch work, or whose result depends on launch choices,
 *     take a context (gs_ctx, from gs_create) first.  A context holds host
 *     state only: the device it was made for and its tuning (launch choices
 *     that never change results).  Use one context per host thread; calls
 *     with different contexts may run concurrently on different threads.
 *     The context's device must be the calling thread's current device.
 *   - All arrays named "device" are device (HBM) pointers owned by the
 *     caller; the library never allocates, frees or retains them.  Scratch
 *     memory comes in through `workspace` (device, 256-byte aligned, at least
 *     gs_workspace_bytes() bytes).  No entry point allocates device memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *     enqueues work on it and returns; there is no host synchronisation, so
 *     every call can be captured into a HIP graph.
 *   - Arguments are validated on the host before anything is enqueued.  On
 *     error a negative status is returned, nothing is enqueued, and
 *     gs_last_error() returns a message (thread-local, valid until the next
 *     call on the same thread).
 *   - Every workspace begins with a 256-byte status header: the key count
 *     the last binning that used the workspace required and the capacity it
 *     had.  A capacity overflow is found on the device, so it cannot be a
 *     return status of the (asynchronous) call; gs_poll_status reads it.
 *   - Views: `cams_host` and `cams_dev` hold the same `n_views` cameras, on
 *     the host (read for validation and launch sizes) and on the device
 *     (read by kernels).  Tiles of all views form one global tile space:
 *     view v owns tiles [off_v, off_v + tx_v * ty_v), tx_v = ceil(W_v / T),
 *     ty_v = ceil(H_v / T), off_v = sum of the tile counts of views < v;
 *     tile (tx, ty) of view v is global tile off_v + ty * tx_v + tx.
 *     Pixels likewise: view v owns pixels [P_v, P_v + W_v H_v), row-major.
 *   - Images are planar float32: view v occupies 3 * W_v * H_v floats
 *     starting at 3 * P_v, channel-major ([3][H_v][W_v]).
 *   - Tile size T is 8, 16 or 32.
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GS_OK = 0,
    GS_ERR_INVALID = -1,     /* bad argument (null pointer, size, alignment, context) */
    GS_ERR_UNSUPPORTED = -2, /* valid but unsupported (SH degree > 3, tile size) */
    GS_ERR_CAPACITY = -3,    /* workspace too small, or (gs_poll_status) key capacity exceeded */
    GS_ERR_HIP = -4          /* a HIP runtime call or launch failed */
};

/* Library context (opaque; host state only). */
typedef struct gs_ctx gs_ctx;

/* Pinhole camera, OpenCV frame (x right, y down, z forward).  A world point x
 * maps to camera space as R x + t (R row-major).  Pixel (i, j) is sampled at
 * its integer coordinates; fx, fy in pixels; the projection Jacobian's
 * tangent clamp uses tan(fov_x / 2) = width / (2 fx).  Points with camera
 * depth <= near_z are culled.  Size 76 bytes, arrays tightly packed. */
typedef struct gs_camera {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float near_z;
} gs_camera;

/* Scene (Section 2.1 point parameters; Section 4.2 nested subsets).  All
 * pointers are device pointers, float32, structure of arrays:
 *   means [n][3], log_scales [n][3] (scale = exp), quats [n][4] as
 *   (w, x, y, z) (normalised in the kernel), opacity_logits [n]
 *   (opacity = sigmoid), sh [n][K][3] with K = (sh_degree + 1)^2.
 * Foveated rendering only (NULL / 0 otherwise):
 *   qbound [n] uint8 in 1..n_levels, the quality bound m: point i is used by
 *   levels t <= m_i;  lvl_opacity_logits [n_levels][n] and
 *   lvl_sh_dc [n_levels][n][3], the per-level versions of opacity and DC
 *   colour (selective multi-versioning); NULL means every level shares the
 *   base parameter. */
typedef struct gs_scene {
    int32_t n;
    int32_t sh_degree;
    const float *means;
    const float *log_scales;
    const float *quats;
    const float *opacity_logits;
    const float *sh;
    const uint8_t *qbound;
    int32_t n_levels;
    const float *lvl_opacity_logits;
    const float *lvl_sh_dc;
} gs_scene;

/* Projected splat, one per (view, point): 48 bytes.
 *   mean_x, mean_y   screen position (pixels)
 *   conic_a/b/c      inverse 2D covariance [[a, b], [b, c]]
 *   opacity, r, g, b activated opacity and colour
 *   depth            camera-space z
 *   radius           ceil(3 sqrt(largest eigenvalue)), 0 if culled
 *   tiles_touched    tiles of the clipped pixel rectangle
 *                    [ceil(x - r), floor(x + r)] x [ceil(y - r), floor(y + r)],
 *                    computed in float32 (Comp_i of Eq. 3 before filtering) */
typedef struct gs_splat {
    float mean_x, mean_y;
    float conic_a, conic_b, conic_c;
    float opacity;
    float r, g, b;
    float depth;
    int32_t radius;
    uint32_t tiles_touched;
} gs_splat;

/* Gradient of a loss with respect to a splat's screen-space quantities
 * (48 bytes; the three pad floats are written as zero). */
typedef struct gs_splat_grad {
    float mean_x, mean_y;
    float conic_a, conic_b, conic_c;
    float opacity;
    float r, g, b;
    float pad[3];
} gs_splat_grad;

/* Foveation parameters of one eye (Section 4.1, Section 6): gaze pixel, the
 * eccentricities (degrees) where rings 2..n_levels start, and the total width
 * (degrees) of the blend band centred on each ring start. */
typedef struct gs_fovea {
    float gaze_x, gaze_y;
    float ring_deg[3];
    float band_deg;
} gs_fovea;

/* Message for the last non-zero status on this thread ("" if none). */
const char *gs_last_error(void);

/* ABI version (bumped on any layout change). */
int gs_version(void);

/* Creates a context for HIP device `device` with the default tuning (the
 * GS_RADIX_PART environment variable, if 4096, 8192 or 16384, sets the sort
 * partition).  *out is owned by the caller and released with gs_destroy.
 * Fails with GS_ERR_INVALID for a device that does not exist.  Without a
 * usable HIP runtime the context still serves host-only calls (workspace
 * sizes, argument checks); calls that launch work then fail. */
int gs_create(gs_ctx **out, int device);

/* Releases a context (NULL is a no-op).  Calls already enqueued with it are
 * unaffected: a context holds no device state. */
int gs_destroy(gs_ctx *ctx);

/* Status of the last binning (gs_bin_sort, gs_render_fwd,
 * gs_render_foveated) that used `workspace` (device, the call's workspace):
 * *status = GS_OK, or GS_ERR_CAPACITY if it needed more keys than its
 * key_capacity (its outputs are then invalid: ranges are empty and images
 * show the background); *required_keys (nullable) = the keys it needed.
 * Reads the workspace's header with a blocking copy: call it after the
 * stream that ran the binning has been synchronised, outside graph capture.
 * The header of a workspace no binning has used is undefined. */
int gs_poll_status(gs_ctx *ctx, const void *workspace, int *status, uint64_t *required_keys);

/* Host helper: total tiles and pixels of the global spaces. */
int gs_tile_count(const gs_camera *cams_host, int n_views, int tile_size,
                  int64_t *n_tiles, int64_t *n_pixels);

/* Bytes of workspace needed by gs_bin_sort / gs_rasterize_* / gs_render_*
 * for these views, n points and a key capacity. */
size_t gs_workspace_bytes(gs_ctx *ctx, const gs_camera *cams_host, int n_views, int32_t n,
                          int tile_size, uint64_t key_capacity);

/* Projection (Section 2.1 "Projection"; Eq. 1b, 1c).
 * Writes splats [n_views][n] (device).  For each point and view: camera-space
 * mean u = R mu + t; culled if u_z <= near_z; 2D covariance
 * J R Sigma R^T J^T + 0.3 I with Sigma = Rot(q) diag(exp(2 log_scale))
 * Rot(q)^T and J the perspective Jacobian (tangent clamped to 1.3x the half
 * field of view); colour max(0, sum_k sh_k Y_k(dir) + 1/2) with Y the real
 * orthonormal SH basis of the unit direction from the camera centre to mu.
 * lvl_rgba (device, nullable) [n_views][n][n_levels][4]: per-level colour
 * and opacity (rgb, opacity) when the scene has n_levels > 0.  A point has no
 * version at the levels above its quality bound (Section 4.2): where the
 * scene gives qbound, level t's opacity is 0 for the points with
 * qbound < t. */
int gs_project(gs_ctx *ctx, const gs_scene *scene, const gs_camera *cams_host, const gs_camera *cams_dev,
               int n_views, int tile_size, gs_splat *splats, float *lvl_rgba, void *stream);

/* Tile binning and (tile, depth) sort (Section 2.1 "Sorting"; Section 4.2
 * filtering).  For every view v and point i with a visible splat, one key per
 * tile of its pixel rectangle (row-major), kept only if tile_level is NULL or
 * tile_level[tile][0] <= qbound[i] (tile_level: the [n_tiles][2] uint8 table
 * of gs_fovea_prep; its first column is the tile's lowest level).  The list is sorted by
 * (global tile, float32 depth bits), ties by (view, i).
 * Outputs (device):
 *   vals [key_capacity]        point index i of each sorted key
 *   keys [key_capacity]        nullable; (global tile << 32) | depth bits
 *   tile_ranges [n_tiles][2]   [begin, end) of each tile's run in vals
 *   hits [n_views][n]          nullable; keys emitted per point (Comp_i)
 *   num_keys [1] (uint64)      total keys required.  If it exceeds
 *                              key_capacity the outputs are invalid (no
 *                              tile has keys); the caller re-runs with a
 *                              larger capacity (read num_keys, or
 *                              gs_poll_status on the workspace, after
 *                              synchronising).
 * key_capacity must be < 2^32. */
int gs_bin_sort(gs_ctx *ctx, const gs_splat *splats, int32_t n, const gs_camera *cams_host,
                const gs_camera *cams_dev, int n_views, int tile_size,
                const uint8_t *tile_level, const uint8_t *qbound,
                uint32_t *vals, uint64_t *keys, uint64_t key_capacity,
                uint32_t *tile_ranges, uint32_t *hits, uint64_t *num_keys,
                void *workspace, size_t workspace_bytes, void *stream);

/* Per-pixel front-to-back compositing (Eq. 1a) over each tile's sorted run.
 * A point contributes to pixel p if its Mahalanobis distance d satisfies
 * d^2 <= 9 and alpha = min(0.99, opacity exp(-d^2 / 2)) >= 1/255; before
 * blending it, T' = T (1 - alpha) is formed and the pixel stops (without
 * blending it) once T' < 1e-4.  Output I = sum T_i alpha_i c_i + T bg.
 * Outputs (device): image (planar, see above), final_T [n_pixels],
 * n_contrib [n_pixels] (1-based position in the tile run of the last blended
 * point, 0 if none), dominated_px (nullable) [n_views][n]: number of pixels
 * whose largest T_i alpha_i is point i's (Val_i of Eq. 3; first maximum in
 * depth order).  bg is a host float[3] (NULL = black).
 * stats (device, nullable, uint64[4], accumulated, caller zeroes): blended
 * (pixel, point) pairs, evaluated pairs, staged list entries and entries kept
 * by the per-wave footprint test; a separate instrumented kernel runs when
 * stats is non-NULL. */
int gs_rasterize_fwd(gs_ctx *ctx, const gs_splat *splats, int32_t n, const gs_camera *cams_host,
                     const gs_camera *cams_dev, int n_views, int tile_size,
                     const uint32_t *vals, const uint32_t *tile_ranges, const float *bg,
                     float *image, float *final_T, uint32_t *n_contrib, uint32_t *dominated_px,
                     uint64_t *stats, void *workspace, size_t workspace_bytes, void *stream);

/* Reverse of gs_rasterize_fwd: given dL/dimage (planar, device) and the
 * forward's final_T and n_contrib, writes grads [n_views][n] (device,
 * overwritten): the gradient of L with respect to each splat's mean, conic,
 * opacity and colour.  The per-pixel decisions (extent, skip, stop, the alpha
 * clamp) are held constant.  A splat's sums over the tiles it reaches are
 * added with float atomics, so their last bits depend on scheduling. */
int gs_rasterize_bwd(gs_ctx *ctx, const gs_splat *splats, int32_t n, const gs_camera *cams_host,
                     const gs_camera *cams_dev, int n_views, int tile_size,
                     const uint32_t *vals, const uint32_t *tile_ranges, const float *bg,
                     const float *final_T, const uint32_t *n_contrib, const float *dL_dimage,
                     gs_splat_grad *grads, void *workspace, size_t workspace_bytes,
                     void *stream);

/* Reverse of gs_project: from grads [n_views][n] to the scene parameters,
 * summed over views.  Outputs (device): d_means [n][3], d_log_scales [n][3],
 * d_quats [n][4], d_opacity_logits [n], d_sh [n][K][3]; overwritten when
 * accumulate is 0, added to when it is 1 (views rendered by separate calls
 * sum their gradients this way).  The projection is recomputed from the
 * scene; splats (the forward's output) is accepted for interface symmetry and
 * not read.  A (view, point) whose gradient record is all zero, or that the
 * forward culls (near plane, degenerate covariance), contributes nothing. */
int gs_project_bwd(gs_ctx *ctx, const gs_scene *scene, const gs_camera *cams_host, const gs_camera *cams_dev,
                   int n_views, const gs_splat *splats, const gs_splat_grad *grads,
                   float *d_means, float *d_log_scales, float *d_quats,
                   float *d_opacity_logits, float *d_sh, int accumulate, void *stream);

/* Foveation tables (Section 4.1; ring layout of Section 6).  For every pixel
 * of every eye: eccentricity = angle between the pinhole rays through the
 * pixel and through the gaze pixel; lower level lo (1-based) and weight w of
 * level lo + 1, a linear ramp across the band of total width band_deg centred
 * on each ring start (w = 0 outside bands).  Per tile: the lowest and highest
 * level with non-zero weight over its pixels.
 * fov_host: n_eyes structs (host).  Outputs (device): pix_level [n_pixels]
 * uint8, pix_weight [n_pixels] float, tile_level [n_tiles][2] uint8 (lo, hi).
 * n_levels is 1..4. */
int gs_fovea_prep(gs_ctx *ctx, const gs_camera *cams_host, const gs_camera *cams_dev, const gs_fovea *fov_host,
                  int n_eyes, int tile_size, int n_levels, uint8_t *pix_level, float *pix_weight,
                  uint8_t *tile_level, void *stream);

/* Foveated compositing (Section 4.1 blending, 4.2 filtering and
 * multi-versioning).  Keys must come from gs_bin_sort with the same tile
 * level table (so each tile's run holds the points of its lowest level,
 * the superset of its other levels).  Each pixel composites level lo and, if its
 * weight is non-zero, level lo + 1; level t uses only points with
 * qbound >= t and their level-t colour and opacity (lvl_rgba from
 * gs_project of a scene with these quality bounds: the filter relies on its
 * zero opacity above each point's bound, qbound is read only where a pixel
 * block spans more than two levels); output (1 - w) I_lo + w I_(lo+1).  Same cut-offs as
 * gs_rasterize_fwd, applied per level; stats as in gs_rasterize_fwd
 * (blended pairs count each level's blend).  final_T2 (float [n_pixels][2])
 * and n_contrib2 (uint32 [n_pixels][2]), both nullable and given together,
 * receive per pixel the final transmittance and the last blended run
 * position of the two accumulators (levels lo and lo + 1): the start of
 * gs_rasterize_foveated_bwd. */
int gs_rasterize_foveated(gs_ctx *ctx, const gs_splat *splats, const float *lvl_rgba, int32_t n,
                          const uint8_t *qbound, int n_levels, const gs_camera *cams_host,
                          const gs_camera *cams_dev, int n_eyes, int tile_size,
                          const uint32_t *vals, const uint32_t *tile_ranges,
                          const uint8_t *pix_level, const float *pix_weight, const float *bg,
                          float *image, uint64_t *stats, float *final_T2, uint32_t *n_contrib2,
                          void *workspace, size_t workspace_bytes, void *stream);

/* Reverse of gs_rasterize_foveated (the differentiable form of the blend of
 * Section 4.1 with the per-level opacity and colour of Section 4.2): given
 * dL/dimage and the forward's final_T2 / n_contrib2, each accumulator is
 * walked back to front from its last blended splat with dL scaled by its
 * blend weight.  Outputs (device, overwritten): grads [n_eyes][n]: the
 * gradient with respect to each splat's mean and conic (summed over the
 * levels; the opacity and colour fields are zero); lvl_grads [n_eyes][n]
 * [n_levels][4]: per level, the gradient with respect to its colour (r, g,
 * b) and opacity.  Decisions (extent, filter, skip, stop, clamp) are held
 * constant. */
int gs_rasterize_foveated_bwd(gs_ctx *ctx, const gs_splat *splats, const float *lvl_rgba, int32_t n,
                              const uint8_t *qbound, int n_levels, const gs_camera *cams_host,
                              const gs_camera *cams_dev, int n_eyes, int tile_size,
                              const uint32_t *vals, const uint32_t *tile_ranges,
                              const uint8_t *pix_level, const float *pix_weight, const float *bg,
                              const float *final_T2, const uint32_t *n_contrib2, const float *dL_dimage,
                              gs_splat_grad *grads, float *lvl_grads, void *stream);

/* Reverse of gs_project with the level versions (Section 4.2): from grads
 * and lvl_grads of gs_rasterize_foveated_bwd to the scene parameters,
 * summed over the eyes.  Level t's colour is max(0, DC_t Y_0 + sum_{k>=1}
 * sh_k Y_k + 1/2) and its opacity sigmoid(lvl_opacity_logits[t]): the level
 * DC and logit gradients go to d_lvl_sh_dc [n_levels][n][3] and
 * d_lvl_opacity_logits [n_levels][n] (or, when the scene shares the base
 * parameters, to the base DC and logit), the non-DC SH, position and shape
 * gradients sum over the levels.  Outputs as in gs_project_bwd, plus the two
 * level arrays (nullable when the scene has no level versions);
 * accumulate = 1 adds to the outputs. */
int gs_project_bwd_levels(gs_ctx *ctx, const gs_scene *scene, const gs_camera *cams_host, const gs_camera *cams_dev,
                          int n_views, const gs_splat *splats, const gs_splat_grad *grads,
                          const float *lvl_grads, float *d_means, float *d_log_scales, float *d_quats,
                          float *d_opacity_logits, float *d_sh, float *d_lvl_opacity_logits,
                          float *d_lvl_sh_dc, int accumulate, void *stream);

/* One-call foveated render of n_eyes views: fovea tables, projection with
 * per-level versions, filtered binning and sort, foveated compositing.
 * Intermediate buffers live in the workspace; size it with
 * gs_render_workspace_bytes().  num_keys (device, uint64) receives the
 * required key count as in gs_bin_sort (outputs are invalid if it exceeds
 * key_capacity).  The projection also counts each entry's kept tiles, so
 * the binning does not read the splat records again; image and key count
 * equal those of the stage calls. */
size_t gs_render_workspace_bytes(gs_ctx *ctx, const gs_camera *cams_host, int n_views, int32_t n,
                                 int n_levels, int tile_size, uint64_t key_capacity);
int gs_render_foveated(gs_ctx *ctx, const gs_scene *scene, const gs_camera *cams_host,
                       const gs_camera *cams_dev, const gs_fovea *fov_host, int n_eyes,
                       int tile_size, const float *bg, float *image, uint64_t key_capacity,
                       uint64_t *num_keys, void *workspace, size_t workspace_bytes,
                       void *stream);

/* One-call plain render of n_views views: projection, binning and sort,
 * compositing.  Same workspace rule as gs_render_foveated (n_levels = 0).
 * splats, vals, tile_ranges, final_T, n_contrib are outputs kept for a
 * backward pass (device; n_contrib/final_T [n_pixels], vals [key_capacity]),
 * equal to those of gs_project + gs_bin_sort + gs_rasterize_fwd (the
 * projection also counts each entry's tiles). */
int gs_render_fwd(gs_ctx *ctx, const gs_scene *scene, const gs_camera *cams_host, const gs_camera *cams_dev,
                  int n_views, int tile_size, const float *bg, gs_splat *splats,
                  uint32_t *vals, uint32_t *tile_ranges, uint64_t key_capacity,
                  uint64_t *num_keys, float *image, float *final_T, uint32_t *n_contrib,
                  void *workspace, size_t workspace_bytes, void *stream);

/* L1 photometric loss, the training objective used with the reverse pass
 * (Section 3 trains against captured images; the scale sets the mean):
 * loss += scale * sum_k |image[k] - target[k]| and dL_dimage[k] =
 * scale * sign(image[k] - target[k]) (0 where equal).  image, target,
 * dL_dimage: device float [n]; loss: device float, added to (reset = 1
 * zeroes it first).  The sum is taken in float32 with block partials added
 * atomically, so its last bits depend on scheduling.  Launches kernels
 * only, so it may be captured in a graph. */
int gs_l1_grad(gs_ctx *ctx, const float *image, const float *target, uint64_t n, float scale, float *dL_dimage,
               float *loss, int reset, void *stream);

/* Computational efficiency of every point (Section 3.2, the CE equation):
 * per view, Val / Comp with Val = the pixels the point dominates
 * (dominated_px of gs_rasterize_fwd) and Comp = the tiles that intersect and
 * use it (hits of gs_bin_sort, after the level filter when there is one);
 * CE = the maximum over the views (0 for views where it uses no tile).  The
 * ratio is a correctly rounded float32 division.  dominated, hits: device
 * uint32 [n_views][n]; ce: device float [n]. */
int gs_ce_score(gs_ctx *ctx, const uint32_t *dominated, const uint32_t *hits, int32_t n, int n_views, float *ce,
                void *stream);

/* Selection of the k points with the lowest CE for removal (the pruning
 * rounds of Section 3.4 remove R = 10 % per round): a radix select on the
 * float bits (CE >= 0), ties broken by the lower index.  ce: device float
 * [n] (non-negative, no NaN); mask: device uint8 [n], 1 for selected points;
 * idx (nullable): device uint32 [k], the selected indices ascending.  k is
 * clamped to [0, n].  Workspace: gs_select_workspace_bytes(n) bytes, 256-byte
 * aligned (not needed when k = 0). */
size_t gs_select_workspace_bytes(int32_t n);
int gs_select_lowest(gs_ctx *ctx, const float *ce, int32_t n, int32_t k, uint8_t *mask, uint32_t *idx, void *workspace,
                     size_t workspace_bytes, void *stream);

/* Weighted scale and its gradient (Section 3.3): ws = gamma / (N V) *
 * sum_v sum_i S_i G_iv, S_i = 3 max_k exp(log_scales[i][k]) (three standard
 * deviations along the longest axis), G_iv = [U > T] (U - T) with U =
 * hits[v][i] (tiles the point is used in) and T = threshold.  The gradient
 * with respect to log_scales flows through S to the longest axis (the first
 * on ties); d_log_scales (nullable, device float [n][3]) is overwritten
 * (accumulate = 0) or added to (1), e.g. on top of the render's gradient to
 * form the composite loss of Section 3.3.  ws: device float, overwritten;
 * summed in float32 with atomics (last bits depend on scheduling). */
int gs_weighted_scale(gs_ctx *ctx, const float *log_scales, const uint32_t *hits, int32_t n, int n_views, float threshold,
                      float gamma, float *ws, float *d_log_scales, int accumulate, void *stream);

/* Graph capture of a sequence of calls on one stream (every entry point
 * above except gs_sort_pairs and gs_poll_status launches kernels only: no
 * allocation, host synchronisation or host copies, so a fixed sequence of them on
 * preallocated buffers can be recorded once and replayed).
 * gs_graph_begin starts capture on `stream` (not the legacy default
 * stream); the calls that follow on that stream are recorded, not run;
 * gs_graph_end stops capture and instantiates the graph into *graph (owned
 * by the caller, released with gs_graph_destroy).  gs_graph_launch replays
 * it on a stream: pointers, sizes and host-side arguments (cameras, tile
 * size, capacities) are those of the capture; the contents of device
 * buffers are read afresh at each replay. */
typedef struct gs_graph gs_graph;
int gs_graph_begin(void *stream);
int gs_graph_end(void *stream, gs_graph **graph);
int gs_graph_launch(gs_graph *graph, void *stream);
int gs_graph_destroy(gs_graph *graph);

/* Tuning of a context (launch choices; results do not depend on them):
 *   "radix_part": keys per sort workgroup, 4096, 8192 (default) or 16384.
 *   "raster_queue": 0 (default): one workgroup per tile; 1: when the call
 *                   has a workspace, the forward compositors run as a
 *                   persistent grid whose workgroups pop tile tasks from a
 *                   work queue.
 *   "raster_heavy": with the queue and no split, tiles whose run is longer
 *                   than this go first (default 0: tile order).
 *   "raster_grab":  tasks a workgroup takes per pop (1..64, default 1).
 *   "raster_split": 0 (default) or beta in 256..2^24: with the queue, tile
 *                   runs longer than beta are cut into chunks of beta
 *                   entries composited in parallel and merged front to back
 *                   (chunks whose pixels reach the stop threshold are
 *                   composited again from the running state, so the result
 *                   is the sequential one up to float reassociation).
 *   "raster_merge": 0 (default) or beta >= 1: with the queue off and a
 *                   workspace, consecutive tiles are merged while their keys
 *                   total at most beta (a tile with more stands alone; the
 *                   Tile Merging of Section 5.2), and the workgroups of a
 *                   persistent forward compositor take merged tiles whole;
 *                   results are those of one workgroup per tile.
 *   "stream_views": 0 (default) or 1: gs_render_foveated with two or more
 *                   eyes bins and composites eye by eye, the binning on the
 *                   caller's stream and the compositing on a second stream
 *                   of the context, so that eye e's compositing overlaps eye
 *                   e + 1's binning (the incremental pipelining of Section
 *                   5.2 at view granularity).  Each eye gets key_capacity /
 *                   n_eyes keys; gs_poll_status then reports n_eyes times the
 *                   largest per-eye requirement and *num_keys the total.
 *                   Images are those of the joint call.  The second stream
 *                   (default priority) and its two events are made on the
 *                   first such call and bound to that device until
 *                   gs_destroy; the caller's stream waits for them, so a
 *                   graph captured on it records both branches.  The
 *                   compositing queue and tile merging are not used here.
 *   "coarse_packed": 1 (default): coarse (super-tile, entry) pairs carry
 *                   their tile rectangle in the sort key above the
 *                   super-tile id when the ids fit in 17 bits; 0: always in
 *                   an 8-byte value (the form used above 2^17 super-tiles).
 *                   The keys and ranges are identical either way.
 * Workspace sizes returned by gs_workspace_bytes / gs_render_workspace_bytes
 * depend on these settings: size workspaces after setting them.  The
 * setting applies to the calls made afterwards with this context (a graph
 * keeps the launches it recorded). */
int gs_set_tuning(gs_ctx *ctx, const char *name, int64_t value);
int gs_get_tuning(gs_ctx *ctx, const char *name, int64_t *value);

/* Stable LSD radix sort of n (uint32 key, uint32 value) pairs by the low
 * `bits` bits of the key (1..32) -- the sort of gs_bin_sort's depth and tile
 * passes (Section 2.1 "Sorting").  keys, vals (device, [n]) are sorted in
 * place; keys_tmp, vals_tmp (device, [n]) are scratch; equal keys keep their
 * input order.  Key bits above `bits` must be zero.  n < 2^32. */
size_t gs_sort_workspace_bytes(uint64_t n);
int gs_sort_pairs(gs_ctx *ctx, uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp, uint32_t *vals_tmp,
                  uint64_t n, int bits, void *workspace, size_t workspace_bytes, void *stream);

/* HVSQ, the eccentricity-aware quality metric (Section 2.2, Eq. 2), per
 * quality region as the foveated training uses it (Section 4.3).  The
 * paper takes the features and pooling from the cited HVSQ work; this
 * library reads them as: features = the three colour channels; the pooling
 * of pixel i = the square window of half-width radius[i] centred on it,
 * clipped to the image; statistics = mean and population standard deviation
 * per channel.  term_i = (1/3) sum over channels of (M_a - M_r)^2 +
 * (S_a - S_r)^2; the HVSQ of a region = the mean of term_i over its pixels.
 *
 * gs_hvsq_pooling: radius[p] = floor(rho * eccentricity of p in degrees)
 * (the eccentricity of gs_fovea_prep; a pooling whose area grows
 * quadratically with eccentricity) for the n_views (<= 8) views and their
 * gazes; radius: device int32 [n_pixels].
 *
 * gs_hvsq: img_a (altered), img_r (reference): device planar float images
 * as everywhere in this library; radius: device int32 [n_pixels] (negative
 * values count as 0); region: device uint8 [n_pixels] in 1..n_regions
 * (nullable when n_regions = 0), e.g. the pix_level of gs_fovea_prep.
 * Outputs (device, overwritten): sums, counts: double [n_views][n_regions + 1],
 * per view the sum of term_i and the pixel count of each region (index
 * t - 1) and of the whole view (index n_regions); terms (nullable): double
 * [n_pixels], term_i.  grad_region = -1: no gradient; 0 or t in
 * 1..n_regions: dL_da (device float, planar like img_a) receives the
 * gradient of L = sum over views of the view's HVSQ over the whole view (0)
 * or over region t, with respect to img_a (where the altered window's
 * standard deviation is 0 only its mean contributes).  Double-precision
 * accumulations use atomics, so the last bits depend on scheduling.
 * Workspace: gs_hvsq_workspace_bytes(want_grad) bytes, 256-byte aligned.
 * At most GS_HVSQ_MAX_REGIONS (8) regions. */
int gs_hvsq_pooling(gs_ctx *ctx, const gs_camera *cams_host, const gs_camera *cams_dev, const gs_fovea *fov_host,
                    int n_views, float rho, int32_t *radius, void *stream);
size_t gs_hvsq_workspace_bytes(gs_ctx *ctx, const gs_camera *cams_host, int n_views, int want_grad);
int gs_hvsq(gs_ctx *ctx, const gs_camera *cams_host, const gs_camera *cams_dev, int n_views, const float *img_a,
            const float *img_r, const int32_t *radius, const uint8_t *region, int n_regions, double *sums,
            double *counts, double *terms, int grad_region, float *dL_da, void *workspace, size_t workspace_bytes,
            void *stream);

/* Largest n of gs_sort_pairs_static. */
#define GS_SORT_STATIC_MAX_KEYS (1u << 24)

/* gs_sort_pairs without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same sort, arguments and result as
 * gs_sort_pairs; its scratch (digit counts, tickets, lookback words) is a
 * static 17 MiB array in the library, one per device, held until the
 * process ends, so n is at most GS_SORT_STATIC_MAX_KEYS (GS_ERR_CAPACITY
 * beyond, found on the host).  It allocates and frees nothing.  Every call
 * on a device uses that device's one array: calls that overlap on one
 * device (other streams, other threads, other contexts) race and must be
 * ordered by the caller; each call clears what it needs. */
int gs_sort_pairs_static(gs_ctx *ctx, uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp, uint32_t *vals_tmp,
                         uint64_t n, int bits, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
