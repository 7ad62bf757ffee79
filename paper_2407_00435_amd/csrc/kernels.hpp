// Host-side launchers of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs.h"

// projection
// The binning's counting step folded into the projection (the one-call
// renders): per entry e = v n + i, the count of its tiles (with level
// versions: kept after the level filter) in its rectangle record (rec[e]),
// and its depth key or KEY_NONE (kw[e]).  The tables (sat, bbox, vtab) are
// the binning's, built before.
constexpr uint32_t KEY_NONE = 0xFFFFFFFFu;  // no keys: never the bits of a positive depth
struct ProjBin {
    const uint32_t *sat;
    const int32_t *bbox;
    const int64_t *vtab;
    int64_t n_tiles;
    uint4 *rec;
    uint32_t *kw;
};
hipError_t launch_project(const gs_scene &sc, const gs_camera *cams_dev, int V, int T,
                          gs_splat *out, float *lvl_rgba, hipStream_t st, const ProjBin *pb = nullptr);
hipError_t launch_project_bwd(const gs_scene &sc, const gs_camera *cams_dev, int V,
                              const gs_splat *splats, const gs_splat_grad *grads, float *g_means,
                              float *g_ls, float *g_q, float *g_logit, float *g_sh, int accumulate,
                              hipStream_t st, const float *lvl_grads = nullptr, float *g_lvl_logit = nullptr,
                              float *g_lvl_dc = nullptr);

// pruning metrics
hipError_t launch_ce_score(const uint32_t *dominated, const uint32_t *hits, int n, int V, float *ce,
                           hipStream_t st);
size_t select_scratch_bytes(int n);
hipError_t launch_fill_u8(uint8_t *p, uint8_t v, int n, hipStream_t st);
hipError_t launch_select_lowest(const float *ce, int n, int k, uint8_t *mask, uint32_t *idx, void *scratch,
                                hipStream_t st);
hipError_t launch_weighted_scale(const float *log_scales, const uint32_t *hits, int n, int V, float thr,
                                 float gamma, float *ws, float *d_log_scales, int accumulate, hipStream_t st);

// losses
hipError_t launch_l1_grad(const float *image, const float *target, uint64_t n, float scale,
                          float *dL_dimage, float *loss, hipStream_t st);

// Launch choices of one library context (gs_ctx), read on the host while a
// call enqueues its kernels; they change launch shapes, never results.
struct Tuning {
    int radix_part = 8192;       // keys per sort workgroup: 4096, 8192 or 16384
    bool coarse_packed = true;   // coarse pairs carry their rectangle in the key
    int raster_queue = 0;        // persistent work-queue compositors
    uint32_t raster_beta = 0;    // heavy-tile split length (0: no split)
    uint32_t raster_heavy = 0;   // without split: runs longer than this go first
    uint32_t raster_grab = 1;    // tasks per pop
    uint32_t raster_merge = 0;   // tile merging threshold beta (0: one workgroup per tile)
    int stream_views = 0;        // one-call foveated render: bin and composite view by view on two streams
};

// radix sort of (u32 key, u32 value) pairs, LSD over bits [0, bits)
struct RadixScratch {
    uint32_t *hist;     // [4][256] digit counts, then exclusive bases
    uint64_t *status;   // [2][status_words] lookback words, two buffers
    uint32_t *tickets;  // [4] partition tickets, one per pass
    uint64_t status_words;  // words per buffer (radix_status_words)
    int part = 8192;        // keys per workgroup (4096, 8192 or 16384)
};
// partitions the lookback status must hold for `cap` keys (smallest partition)
uint64_t radix_max_parts(uint64_t cap);
// lookback words per buffer for sorts of up to `cap` keys (any radix)
uint64_t radix_status_words(uint64_t cap);
// passes a sort of `bits`-bit keys with vbytes-byte values runs with
// partitions of `part` keys (its result is in the second buffer pair when odd)
int radix_pass_count(int bits, int vbytes, int part);
inline int radix_passes(int bits) { return (bits + 7) / 8; }
// digit width of each pass for a key of `bits` bits (equal widths, <= 8)
int radix_digit_bits(int bits);
// Sorts count (device, clamped to cap) pairs.  Input in (ka, va); the result
// is in (ka, va) if radix_pass_count(bits, value bytes) is even, else in (kb,
// vb).  With hist_ready (keys of more than 9 bits) the caller has called
// radix_sort_prepare and accumulated the per-pass digit counts into rs.hist
// ([pass][256], pass p = bits [p d, (p + 1) d) with d = radix_digit_bits(bits)).
// With `cleared` (and not hist_ready) the caller has zeroed what
// radix_sort_prepare would (digit counts, tickets, first-pass lookback words)
// and the sort only counts the digits.
hipError_t radix_sort_pairs(uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb,
                            const uint64_t *d_count, uint64_t cap, int bits,
                            const RadixScratch &rs, hipStream_t st, bool hist_ready, bool cleared = false);

// The same with 8-byte values (partitions of at most 8192 keys).
hipError_t radix_sort_pairs_v2(uint32_t *ka, uint2 *va, uint32_t *kb, uint2 *vb, const uint64_t *d_count,
                               uint64_t cap, int bits, const RadixScratch &rs, hipStream_t st,
                               bool hist_ready = false, bool cleared = false);

// How a sort of `bits`-bit keys with vbytes-byte values runs: partitions of
// `part` keys, `passes` passes of `dbits`-bit digits (pass p sorts on the
// digit (key >> (dbits * p)) & ((1 << dbits) - 1), counted at
// hist[p * radix + digit]); its first pass's lookback words for `count` pairs
// are ceil(count / part) * radix (what radix_prepare_words returns).
struct RadixShape {
    int part;
    int radix;
    int passes;
    int dbits;
};
RadixShape radix_shape(const RadixScratch &rs, int vbytes, int bits);

// zeroes the digit counts, tickets and first-pass lookback words of a sort
// of min(*d_count, cap) pairs with vbytes-byte values; a caller that builds
// the digit counts itself (hist_ready) calls it first
hipError_t radix_sort_prepare(const RadixScratch &rs, const uint64_t *d_count, uint64_t cap, int vbytes, int bits,
                              hipStream_t st);
// the lookback words radix_sort_prepare clears for a sort of `count` pairs
// (a caller clearing them itself, with the digit counts and tickets, may
// skip radix_sort_prepare)
uint64_t radix_prepare_words(const RadixScratch &rs, uint64_t count, int vbytes, int bits);
size_t radix_sort_scratch_bytes(uint64_t n);
inline bool radix_part_ok(int p) { return p == 4096 || p == 8192 || p == 16384; }
// sorts n pairs with its own scratch at ws (radix_sort_scratch_bytes(n)
// bytes) in partitions of `part` keys; *in_tmp tells where the result is
hipError_t radix_sort_standalone(uint32_t *keys, uint32_t *vals, uint32_t *kt, uint32_t *vt, uint64_t n,
                                 int bits, void *ws, int part, bool *in_tmp, hipStream_t st);

// binning
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
// (view, point) entries per block of the counting, gather and coarse-emission
// passes (1024-thread workgroups, two entries a thread): blocks of 4096 kept
// one 1024-thread workgroup per CU for the gather and the emission, whose
// latency then set their time (binning of the stereo 1080p frame 0.478 ->
// 0.444 ms at 2048; 1024 was slower again, 0.463 ms)
constexpr int ENTRY_BLOCK = 2048;
constexpr int BIN_SUPER_TILE = 8;   // super-tile side in tiles (BIN_SUPER_TILE^2 <= 64)
constexpr uint32_t BIN_CHUNK = 256; // coarse pairs per chunk of the per-tile counting passes
// chunks of the counting passes: each super-tile's run of coarse pairs (at
// most the keys) is cut into chunks of BIN_CHUNK, and there are at most
// n_tiles super-tiles
inline uint64_t bin_max_chunks(uint64_t cap, int64_t n_tiles) { return cap / BIN_CHUNK + (uint64_t)n_tiles + 1; }
struct BinScratch {
    uint32_t *dkey_a, *dval_a, *dkey_b, *dval_b;  // [E] depth sort ping-pong
    uint4 *rec;                                   // [E] rectangle, count, quality bound (entries with keys)
    uint4 *rec_s;                                 // [E] rectangle, entry, view and quality bound in depth order
    uint32_t *cc_s;                               // [E] coarse pairs of each entry in depth order
    uint32_t *block_vis;                          // [0]: ticket of the counting pass
    uint64_t *block_sums, *block_sums2;           // [E / ENTRY_BLOCK + 1] (block_sums: the counting pass's lookback words first)
    int64_t *vtab;                                // [2V] first tile and tiles_x of each view
    int4 *stab;                                   // [V] first super-tile, super-tiles per row, tiles_x, tiles_y
    uint32_t *tkey_a, *tkey_b;                    // [cap] coarse-pair sort keys (super-tile ids), ping-pong
    uint2 *cpay_a, *cpay_b;                       // [cap] coarse-pair payloads, ping-pong
    uint32_t *st_ranges;                          // [n_tiles][2] run of each super-tile in the sorted pairs
    uint8_t *st_cls;                              // [n_tiles][4] per super-tile and level: keeps none/all/part
    uint32_t *chunk_off;                          // [n_tiles + 1] first chunk of each super-tile
    uint4 *chunk;                                 // [bin_max_chunks] first pair, end pair, super-tile, view
    uint32_t *ccnt;                               // [bin_max_chunks][BIN_SUPER_TILE^2] per-chunk tile counts, then prefixes
    uint32_t *tot;                                // [n_tiles] keys per tile
    uint64_t *tsum;                               // [n_tiles / SCAN_ITEMS + 1] block sums of tot
    uint64_t *counts;                             // [8]: entries, keys, capacity, coarse pairs, chunks, keys
    uint32_t *sat;                                // [4][n_tiles] level summed-area tables
    int32_t *bbox;                                // [V][4][4] bounding box of each level's kept tiles
    RadixScratch rs;
};
// Binning and sort.  coarse_packed: coarse pairs carry their rectangle in
// the sort key where the super-tile ids leave room, else an 8-byte value
// (same keys either way).  status (device, nullable, 2 words): the required
// key count and the capacity, for gs_poll_status.
// mode: BIN_ALL runs every step; BIN_SETUP only the set-up and the level
// filter's tables (before a projection that counts, launch_project with
// bin_counting_args); BIN_COUNTED the rest, compacting the key words that
// projection wrote instead of counting from the splat records.
enum BinMode { BIN_ALL = 0, BIN_SETUP = 1, BIN_COUNTED = 2 };
hipError_t launch_bin_sort(const gs_splat *splats, int n, const gs_camera *cams_dev,
                           const gs_camera *cams_host, int V, int64_t n_tiles, int T,
                           const uint8_t *tile_level, const uint8_t *qbound, int n_levels,
                           uint32_t *vals, uint64_t *keys, uint64_t cap,
                           uint32_t *ranges, uint32_t *hits_out, uint64_t *num_keys,
                           const BinScratch &bs, bool coarse_packed, uint64_t *status, hipStream_t st,
                           BinMode mode = BIN_ALL);
// The projection's counting arguments over a binning scratch (kw in the depth
// sort's second key buffer, free until the sort's first pass).
ProjBin bin_counting_args(const BinScratch &bs, int64_t n_tiles);

// Status of a binning done view by view: status[0] = V * the largest per-view
// required key count (the capacity that fits every view when each has
// cap / V), status[1] = cap, *num_keys = the total; req_cap: [V][2] (required,
// capacity) as each binning wrote it, nums: [V] per-view key counts.
hipError_t launch_status_views(const uint64_t *req_cap, const uint64_t *nums, int V, uint64_t cap,
                               uint64_t *status, uint64_t *num_keys, hipStream_t st);

// compositing
// Work-queue scratch of the persistent compositors (carved from a workspace).
struct RasterQueueArgs {
    uint32_t *counts;     // [4]
    uint32_t *heavy;      // [heavy_cap][2]
    uint32_t *light;      // [light_cap][2]
    uint32_t *merge_cnt;  // [heavy_cap]
    float *part;          // [heavy_cap][64][12] when beta > 0
    uint32_t heavy_cap, light_cap;
    uint32_t beta;
    uint32_t heavy_min;  // without splitting, runs longer than this go first (0: tile order)
    uint32_t grab;       // consecutive tasks a workgroup takes per pop
};
uint64_t raster_queue_heavy_cap(int64_t n_tiles, int T, uint64_t cap, uint32_t beta);
// Tile merging (carved from a workspace): groups of consecutive tiles whose
// intersections total at most beta (a heavier tile alone), popped whole by
// the workgroups of a persistent compositor.
struct MergeArgs {
    uint32_t *scratch;  // merge_scratch_words(n_tiles) words
    uint32_t beta;
};
inline size_t merge_scratch_words(int64_t n_tiles) { return 16 + 8 * (size_t)(n_tiles + 1); }
hipError_t launch_raster_fwd(const gs_splat *splats, int n, const gs_camera *cams_dev, int V, int T,
                             int64_t n_tiles, const uint32_t *vals, const uint32_t *ranges,
                             const float bg[3], float *image, float *final_T, uint32_t *n_contrib,
                             uint32_t *dominated, uint64_t *stats, const RasterQueueArgs *qa, hipStream_t st,
                             const MergeArgs *ma = nullptr);
hipError_t launch_raster_bwd(const gs_splat *splats, int n, const gs_camera *cams_dev, int V, int T,
                             int64_t n_tiles, const uint32_t *vals, const uint32_t *ranges,
                             const float bg[3], const float *final_T, const uint32_t *n_contrib,
                             const float *dL_dimage, gs_splat_grad *grads, hipStream_t st);
hipError_t launch_raster_fov_bwd(const gs_splat *splats, const float *lvl_rgba, int n, const uint8_t *qbound,
                                 int n_levels, const gs_camera *cams_dev, int V, int T, int64_t n_tiles,
                                 const uint32_t *vals, const uint32_t *ranges, const uint8_t *pix_level,
                                 const float *pix_weight, const float bg[3], const float *final_T2,
                                 const uint32_t *n_contrib2, const float *dL_dimage, gs_splat_grad *grads,
                                 float *lvl_grads, hipStream_t st);
hipError_t launch_fovea_prep(const gs_camera *cams_host, const gs_camera *cams_dev, const gs_fovea *fov_host,
                             int n_eyes, int T, int n_levels, int64_t n_pixels, int64_t n_tiles,
                             uint8_t *pix_level, float *pix_weight, uint8_t *tile_level, hipStream_t st);
hipError_t launch_raster_fov(const gs_splat *splats, const float *lvl_rgba, int n,
                             const uint8_t *qbound, int n_levels, const gs_camera *cams_dev, int V,
                             int T, int64_t n_tiles, const uint32_t *vals, const uint32_t *ranges,
                             const uint8_t *pix_level, const float *pix_weight, const float bg[3],
                             float *image, uint64_t *stats, float *final_T2, uint32_t *n_contrib2,
                             const RasterQueueArgs *qa, hipStream_t st, const MergeArgs *ma = nullptr);

// HVSQ (hvsq.hip)
constexpr int GS_HVSQ_MAX_REGIONS = 8;
struct FoveaGazes {
    float x[8], y[8];
};
int64_t hvsq_padded_pixels(const gs_camera *cams_host, int V);
size_t hvsq_scratch_bytes(const gs_camera *cams_host, int V, bool grad);
hipError_t launch_hvsq_radius(const gs_camera *cams_host, const gs_camera *cams_dev, const gs_fovea *fov_host, int V,
                              float rho, int32_t *radius, hipStream_t st);
hipError_t launch_hvsq(const gs_camera *cams_host, const gs_camera *cams_dev, int V, const float *img_a,
                       const float *img_r, const int32_t *radius, const uint8_t *region, int R, double *sums,
                       double *counts, double *terms, int grad_region, float *dL_da, void *ws, hipStream_t st);

// utilities
hipError_t launch_fill_u32(uint32_t *p, uint32_t value, uint64_t count, hipStream_t st);
