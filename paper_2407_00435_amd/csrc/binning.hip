// Tile binning (Section 2.1 "Sorting"; Section 4.2 filtering).
//
// Depth-first construction of the (tile, depth)-sorted key list:
//   1. count:  per (view, point) the number of kept tiles of its rectangle
//              (tile t kept iff its lower level tile_level[t][0] <= the
//              point's quality bound).  With the level filter the count comes
//              from per-level summed-area tables over the tile grid, O(1)
//              per point whatever its size;
//   2. compact the entries that emit at least one key, in index order, and
//      count their depth digits on the way;
//   3. sort them by float32 depth bits (stable radix, 4 passes);
//   4. gather the entry records in depth order and put the keys in
//      (tile, depth, view, point) order with a two-level stable counting
//      sort (super-tiles of 8 x 8 tiles, one wave lane per tile; see
//      "Tile order" below), which writes every key once at its final
//      position and yields the tile ranges from per-tile counts.
// Sorting by depth over the points (millions) and counting per tile over the
// keys (tens of millions) moves far fewer bytes than a 64-bit key sort.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr int SAT_LDS_TILES = 16384;      // views up to this many tiles build their tables in LDS (80 KB)
constexpr int ST = BIN_SUPER_TILE;        // super-tile side in tiles
constexpr int TST = ST * ST;              // tiles per super-tile (<= wave size)
constexpr int MS = 4;                     // coarse masks cover spans of up to MS x MS super-tiles
constexpr uint32_t CHUNK = BIN_CHUNK;     // coarse pairs per chunk

__global__ void __launch_bounds__(256)
k_fill_u32(uint32_t *__restrict__ p, uint32_t value, uint64_t count)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        p[i] = value;
}

// Bitwise OR over the 64 lanes of a wave, in every lane: DPP ORs inside each
// 16-lane row (complete in lane 15 of the row), then the four row results.
__device__ __forceinline__ uint32_t wave_or(uint32_t x)
{
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);  // row_shr:2
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);  // row_shr:4
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);  // row_shr:8
    return (uint32_t)(__builtin_amdgcn_readlane((int)x, 15) | __builtin_amdgcn_readlane((int)x, 31) |
                      __builtin_amdgcn_readlane((int)x, 47) | __builtin_amdgcn_readlane((int)x, 63));
}

__device__ __forceinline__ int64_t view_tile_off(const gs_camera *__restrict__ cams, int v, int T)
{
    int64_t toff = 0;
    for (int u = 0; u < v; ++u) toff += (int64_t)div_up(cams[u].width, T) * div_up(cams[u].height, T);
    return toff;
}

// Set-up of one binning call: the tile offset and grid width of every view,
// vtab[v] = {first tile, tiles_x}, stab[v] = {first super-tile, super-tiles
// per row, tiles_x, tiles_y}; the key capacity in *cap_out; zeroed tile and
// super-tile ranges (a tile without keys keeps (0, 0)); and, when given,
// *num_keys = 0 (no entries at all).
// Also cleared here: the lookback words and ticket of the counting pass
// (lb[nb], *tick) and the depth sort's digit counts, tickets and first-pass
// lookback words (what radix_sort_prepare would clear).
struct SetupClears {
    uint64_t *lb;
    int64_t nb;
    uint32_t *tick;
    uint32_t *hist;     // [4][256]
    uint32_t *tickets;  // [4]
    uint64_t *status;
    uint64_t status_words;
};

__global__ void __launch_bounds__(256)
k_bin_setup(const gs_camera *__restrict__ cams, int V, int T, int64_t *__restrict__ vtab, int4 *__restrict__ stab,
            uint64_t *__restrict__ cap_out, uint64_t cap, uint32_t *__restrict__ ranges, int64_t n_tiles,
            uint32_t *__restrict__ st_ranges, int64_t n_st, uint64_t *__restrict__ num_keys,
            uint64_t *__restrict__ status, SetupClears z)
{
    const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = i0; i < 2 * (uint64_t)n_tiles; i += stride) ranges[i] = 0;
    for (uint64_t i = i0; i < 2 * (uint64_t)n_st; i += stride) st_ranges[i] = 0;
    for (uint64_t i = i0; i < (uint64_t)z.nb; i += stride) z.lb[i] = 0;
    for (uint64_t i = i0; i < z.status_words; i += stride) z.status[i] = 0;
    for (uint64_t i = i0; i < 4 * 256; i += stride) z.hist[i] = 0;
    if (i0 < 4) z.tickets[i0] = 0;
    if (i0 == 4) *z.tick = 0;
    if (i0 != 0) return;
    *cap_out = cap;
    if (num_keys) *num_keys = 0;
    if (status) {
        status[0] = 0;  // required keys (k_scan_pair writes the total)
        status[1] = cap;
    }
    int64_t toff = 0;
    int soff = 0;
    for (int v = 0; v < V; ++v) {
        const int tx = div_up(cams[v].width, T), ty = div_up(cams[v].height, T);
        const int sx = div_up(tx, ST), sy = div_up(ty, ST);
        vtab[2 * v] = toff;
        vtab[2 * v + 1] = tx;
        stab[v] = make_int4(soff, sx, tx, ty);
        toff += (int64_t)tx * ty;
        soff += sx * sy;
    }
}

// Class of every (super-tile, level): 0 if the level keeps none of the
// super-tile's tiles, 1 if it keeps all of them, 2 otherwise.  One wave per
// super-tile s, lane = tile.
__device__ __forceinline__ void st_class(const int64_t *__restrict__ vtab, const int4 *__restrict__ stab, int V,
                                         int64_t s, int L, const uint8_t *__restrict__ tl,
                                         uint8_t *__restrict__ cls)
{
    const int lane = threadIdx.x & 63;
    int v = 0;
    while (v + 1 < V && stab[v + 1].x <= (int)s) ++v;
    const int4 sb = stab[v];
    const int sl = (int)s - sb.x, sy = sl / sb.y, sx = sl - sy * sb.y;
    const int tx = sx * ST + lane % ST, ty = sy * ST + lane / ST;
    const bool valid = lane < TST && tx < sb.z && ty < sb.w;
    const uint32_t lvl = valid ? tl[2 * (vtab[2 * v] + (int64_t)ty * sb.z + tx)] : 255u;
    const int nv = __popcll(ballot64(valid));
    for (int m = 1; m <= L; ++m) {
        const int nk = __popcll(ballot64(valid && lvl <= (uint32_t)m));
        if (lane == 0) cls[s * 4 + m - 1] = (uint8_t)(nk == 0 ? 0 : (nk == nv ? 1 : 2));
    }
}

// Summed-area table of [lower level of tile <= m] over each view's tile grid,
// one table per level m = 1..L: sat[(m-1) * n_tiles + g] counts the tiles
// (x', y') <= (x, y) of g's view.  One workgroup per (view, level), built in
// LDS (dynamic size, with the tiles' lower levels staged beside it) when the
// view's grid fits, else in place in memory: row sums (a wave per row), then
// column sums (a wave per column).
// Also the bounding box of those tiles, bbox[(v * L + m - 1) * 4 +
// {x0, y0, x1, y1}] (x0 > x1 when there are none).  The workgroups after the
// first V * L classify the super-tiles, 16 per workgroup (st_class).
__global__ void __launch_bounds__(1024)
k_level_sat(const gs_camera *__restrict__ cams, int V, int T, int L, int64_t n_tiles,
            const uint8_t *__restrict__ tl, uint32_t *__restrict__ sat, int32_t *__restrict__ bbox, int use_lds,
            const int64_t *__restrict__ vtab, const int4 *__restrict__ stab, int64_t n_st,
            uint8_t *__restrict__ cls)
{
    extern __shared__ uint32_t s_sat[];
    __shared__ int s_box[4];
    if ((int)blockIdx.x >= V * L) {
        const int64_t st_id = (int64_t)(blockIdx.x - V * L) * 16 + (threadIdx.x >> 6);
        if (st_id < n_st) st_class(vtab, stab, V, st_id, L, tl, cls);
        return;
    }
    const int v = blockIdx.x / L, m = blockIdx.x % L + 1;
    const int64_t toff = view_tile_off(cams, v, T);
    const int tx = div_up(cams[v].width, T), ty = div_up(cams[v].height, T);
    const int nt = tx * ty;
    if (threadIdx.x == 0) {
        s_box[0] = tx;
        s_box[1] = ty;
        s_box[2] = -1;
        s_box[3] = -1;
    }
    uint32_t *g = sat + (int64_t)(m - 1) * n_tiles + toff;
    uint32_t *s = use_lds ? s_sat : g;
    const uint16_t *lv = reinterpret_cast<const uint16_t *>(tl + 2 * toff);  // {lower, upper} level per tile
    // in LDS mode the lower levels are staged first, every load in flight at once
    uint8_t *s_lv = reinterpret_cast<uint8_t *>(s_sat + nt);
    if (use_lds) {
        constexpr int U = 8;
        for (int k0 = threadIdx.x; k0 < nt; k0 += U * blockDim.x) {
            uint16_t r[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int k = k0 + j * blockDim.x;
                r[j] = k < nt ? lv[k] : (uint16_t)0;
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int k = k0 + j * blockDim.x;
                if (k < nt) s_lv[k] = (uint8_t)(r[j] & 0xff);
            }
        }
    }
    __syncthreads();
    // row sums: a wave per row, 64 columns per step (ballot prefix counts)
    const int lane = threadIdx.x & 63, waves = blockDim.x / 64, wave = threadIdx.x >> 6;
    for (int y = wave; y < ty; y += waves) {
        uint32_t run = 0;
        int xl = tx, xr = -1;
        for (int x0 = 0; x0 < tx; x0 += 64) {
            const int x = x0 + lane;
            const int k = y * tx + x;
            const bool kept = x < tx && (use_lds ? (int)s_lv[k] : (int)(lv[k] & 0xff)) <= m;
            const uint64_t bal = __builtin_amdgcn_ballot_w64(kept);
            const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            if (x < tx) s[k] = run + below + (kept ? 1u : 0u);
            run += (uint32_t)__popcll(bal);
            if (bal) {
                xl = min(xl, x0 + __ffsll((unsigned long long)bal) - 1);
                xr = max(xr, x0 + 63 - __clzll((long long)bal));
            }
        }
        if (xr >= 0 && lane == 0) {
            atomicMin(&s_box[0], xl);
            atomicMin(&s_box[1], y);
            atomicMax(&s_box[2], xr);
            atomicMax(&s_box[3], y);
        }
    }
    __syncthreads();
    if (threadIdx.x < 4) bbox[((int64_t)v * L + m - 1) * 4 + threadIdx.x] = s_box[threadIdx.x];
    // column sums: a wave per column, 64 rows per step (wave prefix sums)
    for (int x = wave; x < tx; x += waves) {
        uint32_t run = 0;
        for (int y0 = 0; y0 < ty; y0 += 64) {
            const int y = y0 + lane;
            const uint32_t c = wave_incl_scan(y < ty ? s[(int64_t)y * tx + x] : 0u);
            if (y < ty) s[(int64_t)y * tx + x] = run + c;
            run += __shfl(c, 63);
        }
    }
    if (use_lds) {
        __syncthreads();
        for (int64_t k = threadIdx.x; k < nt; k += blockDim.x) g[k] = s[k];
    }
}

__device__ __forceinline__ uint32_t sat_at(const uint32_t *__restrict__ s, int tiles_x, int x, int y)
{
    return (x < 0 || y < 0) ? 0u : s[(int64_t)y * tiles_x + x];
}

__device__ __forceinline__ uint32_t sat_rect(const uint32_t *__restrict__ s, int tiles_x, int x0,
                                             int x1, int y0, int y1)
{
    return sat_at(s, tiles_x, x1, y1) - sat_at(s, tiles_x, x0 - 1, y1) - sat_at(s, tiles_x, x1, y0 - 1) +
           sat_at(s, tiles_x, x0 - 1, y0 - 1);
}

// 1-2. per-entry counts (culled / empty entries count 0, to hits_out when
//    given) and, for the entries with keys, rec[e] = {x0 | y0 << 16,
//    x1 | y1 << 16, count, quality bound} with the rectangle clipped to the
//    bounding box of the tiles its level keeps (the kept tiles and their
//    row-major order are unchanged); then the stable compaction of those
//    entries, (float32 depth bits, entry) to (dkey, dval), counting the depth
//    digits of every sort pass into hist.  Workgroups take their blocks of
//    entries in ticket order and find their output offset by decoupled
//    lookback over the blocks before (lb: flag | count words); the block with
//    the last ticket writes the total to *total.
constexpr int COUNT_THREADS = 1024;
// The counting pass keeps blocks of 4096 entries: its blocks find their
// output offsets by a lookback chain over the blocks before and add their
// digit counts with global atomics, and twice as many blocks made it slower
// (78 -> 88 us on the stereo 1080p frame) where the gather and the emission
// gained from blocks of ENTRY_BLOCK.
constexpr int COUNT_BLOCK = 4096;
constexpr int COUNT_ITEMS = COUNT_BLOCK / COUNT_THREADS;
// The compaction of a counting projection's key words takes blocks of up to
// 16384 entries while that leaves at least KEYW_MIN_BLOCKS of them (one-call
// stereo 1080p frame, 3M entries: 1.041 ms at 4096, 1.037 at 8192, 1.034 at
// 16384; a 500k-entry view was slower at 16384 than at 4096, with 31 blocks).
constexpr int KEYW_MIN_BLOCKS = 160;
static_assert(COUNT_BLOCK == 4096, "the set-up clears lookback words for blocks of at least 4096 entries");
constexpr uint64_t LB_AGG = 1ull << 62;
constexpr uint64_t LB_INC = 2ull << 62;
constexpr uint64_t LB_VAL = (1ull << 62) - 1;
constexpr int LB_BATCH = 8;  // lookback words read per round

// Exclusive prefix of `tot` over the blocks before `blk` (ticket order), by
// decoupled lookback: a batch of predecessors' words is read at once and
// taken in order until an inclusive prefix; an unpublished word ends the
// batch.  One thread.
__device__ __forceinline__ uint64_t block_lookback(uint64_t *__restrict__ lb, int64_t blk, uint64_t tot)
{
    if (blk == 0) {
        __hip_atomic_store(lb, LB_INC | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return 0;
    }
    __hip_atomic_store(lb + blk, LB_AGG | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t prefix = 0;
    int64_t q = blk - 1;
    for (;;) {
        uint64_t w[LB_BATCH];
#pragma unroll
        for (int k = 0; k < LB_BATCH; ++k)
            w[k] = q - k >= 0 ? __hip_atomic_load(lb + (q - k), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : LB_INC;
        int used = LB_BATCH;
        bool done = false;
#pragma unroll
        for (int k = 0; k < LB_BATCH; ++k) {
            if (used < LB_BATCH || done) continue;
            const uint64_t flag = w[k] & ~LB_VAL;
            if (flag == 0) {
                used = k;
                continue;
            }
            prefix += w[k] & LB_VAL;
            if (flag == LB_INC) done = true;
        }
        if (done) break;
        if (used == 0) __builtin_amdgcn_s_sleep(1);
        q -= used;
    }
    __hip_atomic_store(lb + blk, LB_INC | (prefix + tot), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return prefix;
}

// The stable compaction of one block's entries with keys (item j of thread t
// is entry base + j * COUNT_THREADS + t; bal[j] = the wave's ballot of item j
// having keys): (depth bits, entry) to (dkey, dval) at the block's offset,
// found by lookback, and the depth digits of every sort pass into hist.  The
// per-(item, wave) counts are scanned once in entry order (item-major) by
// the first IT waves, so each item's offset is one LDS read.  Called by
// every thread of the block after s_h is zeroed.
template <int IT>
__device__ __forceinline__ void compact_block(const uint64_t (&bal)[IT], const uint32_t (&key)[IT],
                                              int64_t base, int64_t blk, uint64_t *__restrict__ lb,
                                              uint64_t *__restrict__ total, uint32_t *__restrict__ dkey,
                                              uint32_t *__restrict__ dval, uint32_t *__restrict__ hist,
                                              uint32_t (*s_w)[COUNT_THREADS / 64], uint32_t (*s_h)[256],
                                              uint64_t *s_off)
{
    constexpr int W = COUNT_THREADS / 64;
    constexpr int NF = IT * W;  // (item, wave) counts
    static_assert(NF % 64 == 0 && NF <= COUNT_THREADS, "whole waves scan the counts");
    __shared__ uint32_t s_wp[NF / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < IT; ++j) s_w[j][wave] = (uint32_t)__popcll(bal[j]);
    }
    __syncthreads();
    uint32_t *flat = &s_w[0][0];  // index j * W + w
    if (threadIdx.x < NF) {
        const uint32_t x = flat[threadIdx.x];
        const uint32_t inc = wave_incl_scan(x);
        flat[threadIdx.x] = inc - x;
        if (lane == 63) s_wp[wave] = inc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t tot = 0;
        for (int q = 0; q < NF / 64; ++q) {
            const uint32_t c = s_wp[q];
            s_wp[q] = (uint32_t)tot;
            tot += c;
        }
        const uint64_t pre = block_lookback(lb, blk, tot);
        *s_off = pre;
        if (blk == (int64_t)gridDim.x - 1) *total = pre + tot;
    }
    __syncthreads();
    // entries with keys in entry order
    const uint64_t off = *s_off;
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        if ((bal[j] >> lane) & 1ull) {
            const int f = j * W + wave;
            const int64_t e = base + (int64_t)j * COUNT_THREADS + threadIdx.x;
            const uint64_t pos = off + s_wp[f >> 6] + flat[f] + (uint32_t)__popcll(bal[j] & lanemask_lt());
            const uint32_t k = key[j];
            dkey[pos] = k;
            dval[pos] = (uint32_t)e;
#pragma unroll
            for (int p = 0; p < 4; ++p) atomicAdd(&s_h[p][(k >> (8 * p)) & 255u], 1u);
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 4 * 256; q += COUNT_THREADS) {
        const uint32_t x = (&s_h[0][0])[q];
        if (x) atomicAdd(&hist[q], x);
    }
}

template <bool FILT>
__global__ void __launch_bounds__(COUNT_THREADS)
k_count(const gs_splat *__restrict__ splats, int n, const gs_camera *__restrict__ cams, int V, int T,
        const int64_t *__restrict__ vtab, const uint32_t *__restrict__ sat, const int32_t *__restrict__ bbox, int L, int64_t n_tiles,
        const uint8_t *__restrict__ qbound, uint4 *__restrict__ rec, uint32_t *__restrict__ hits_out,
        uint32_t *__restrict__ tick, uint64_t *__restrict__ lb, uint64_t *__restrict__ total,
        uint32_t *__restrict__ dkey, uint32_t *__restrict__ dval, uint32_t *__restrict__ hist)
{
    constexpr int W = COUNT_THREADS / 64;
    __shared__ uint32_t s_blk;
    __shared__ uint32_t s_w[COUNT_ITEMS][W];
    __shared__ uint32_t s_h[4][256];
    __shared__ uint64_t s_off;
    if (threadIdx.x == 0) s_blk = atomicAdd(tick, 1u);
    for (int q = threadIdx.x; q < 4 * 256; q += COUNT_THREADS) (&s_h[0][0])[q] = 0;
    __syncthreads();
    const int64_t blk = s_blk;
    const int64_t E = (int64_t)V * n;
    const int64_t base = blk * (COUNT_THREADS * COUNT_ITEMS);
    // Three rounds of loads over all items, each round issued before any of
    // its values is used: (1) splat fields, quality bound, view sizes; (2)
    // the level's bounding box; (3) the four summed-area corners.  Indices
    // are clamped in bounds (items past E read entry 0, empty rectangles
    // read corner (0, 0)) and the results selected afterwards, so no load
    // sits behind a branch.
    float4 a[COUNT_ITEMS], c[COUNT_ITEMS];
    int vq[COUNT_ITEMS], iq[COUNT_ITEMS], mq[COUNT_ITEMS], Wq[COUNT_ITEMS], Hq[COUNT_ITEMS];
    int64_t toffq[COUNT_ITEMS];
    int txq[COUNT_ITEMS];
#pragma unroll
    for (int j = 0; j < COUNT_ITEMS; ++j) {
        const int64_t e = base + (int64_t)j * COUNT_THREADS + threadIdx.x;
        const int64_t ec = e < E ? e : 0;
        const float4 *s4 = reinterpret_cast<const float4 *>(splats + ec);
        a[j] = s4[0];
        c[j] = s4[2];
        vq[j] = (int)(ec / n);
        iq[j] = (int)(ec - (int64_t)vq[j] * n);
        Wq[j] = cams[vq[j]].width;
        Hq[j] = cams[vq[j]].height;
        mq[j] = FILT ? (int)qbound[iq[j]] : 255;
        toffq[j] = FILT ? vtab[2 * vq[j]] : 0;
        txq[j] = FILT ? (int)vtab[2 * vq[j] + 1] : 0;
    }
    TileRect r[COUNT_ITEMS];
    bool has[COUNT_ITEMS];
    int mlq[COUNT_ITEMS];
    int4 bb[COUNT_ITEMS];
#pragma unroll
    for (int j = 0; j < COUNT_ITEMS; ++j) {
        const int64_t e = base + (int64_t)j * COUNT_THREADS + threadIdx.x;
        has[j] = e < E && tile_rect(a[j].x, a[j].y, __float_as_int(c[j].z), Wq[j], Hq[j], T, r[j]);
        if (!has[j]) r[j].tx0 = r[j].tx1 = r[j].ty0 = r[j].ty1 = 0;
        mlq[j] = mq[j] < 1 ? 1 : (mq[j] < L ? mq[j] : L);
        if (FILT) bb[j] = reinterpret_cast<const int4 *>(bbox)[(int64_t)vq[j] * L + mlq[j] - 1];
    }
    uint32_t cnt[COUNT_ITEMS];
    if (!FILT) {
#pragma unroll
        for (int j = 0; j < COUNT_ITEMS; ++j)
            cnt[j] = has[j] ? (uint32_t)(r[j].tx1 - r[j].tx0 + 1) * (uint32_t)(r[j].ty1 - r[j].ty0 + 1) : 0u;
    } else {
        // kept tiles lie in the level's bounding box: clip to it
        bool ne[COUNT_ITEMS];
        uint32_t s11[COUNT_ITEMS], s01[COUNT_ITEMS], s10[COUNT_ITEMS], s00[COUNT_ITEMS];
#pragma unroll
        for (int j = 0; j < COUNT_ITEMS; ++j) {
            r[j].tx0 = r[j].tx0 > bb[j].x ? r[j].tx0 : bb[j].x;
            r[j].ty0 = r[j].ty0 > bb[j].y ? r[j].ty0 : bb[j].y;
            r[j].tx1 = r[j].tx1 < bb[j].z ? r[j].tx1 : bb[j].z;
            r[j].ty1 = r[j].ty1 < bb[j].w ? r[j].ty1 : bb[j].w;
            ne[j] = has[j] && mq[j] >= 1 && r[j].tx0 <= r[j].tx1 && r[j].ty0 <= r[j].ty1;
            const uint32_t *sp = sat + (int64_t)(mlq[j] - 1) * n_tiles + toffq[j];
            const int x1 = ne[j] ? r[j].tx1 : 0, y1 = ne[j] ? r[j].ty1 : 0;
            const int x0 = ne[j] && r[j].tx0 > 0 ? r[j].tx0 - 1 : 0;
            const int y0 = ne[j] && r[j].ty0 > 0 ? r[j].ty0 - 1 : 0;
            s11[j] = sp[(int64_t)y1 * txq[j] + x1];
            s01[j] = sp[(int64_t)y1 * txq[j] + x0];
            s10[j] = sp[(int64_t)y0 * txq[j] + x1];
            s00[j] = sp[(int64_t)y0 * txq[j] + x0];
        }
#pragma unroll
        for (int j = 0; j < COUNT_ITEMS; ++j) {
            // sat_rect: corners left of column 0 or above row 0 count zero
            const bool lx = r[j].tx0 > 0, ly = r[j].ty0 > 0;
            cnt[j] = ne[j] ? s11[j] - (lx ? s01[j] : 0u) - (ly ? s10[j] : 0u) + (lx && ly ? s00[j] : 0u) : 0u;
        }
    }
    uint64_t bal[COUNT_ITEMS];
    uint32_t key[COUNT_ITEMS];
#pragma unroll
    for (int j = 0; j < COUNT_ITEMS; ++j) {
        const int64_t e = base + (int64_t)j * COUNT_THREADS + threadIdx.x;
        if (e < E) {
            // every entry's record is written (whole cache lines), read only for entries with keys
            rec[e] = make_uint4((uint32_t)r[j].tx0 | ((uint32_t)r[j].ty0 << 16),
                                (uint32_t)r[j].tx1 | ((uint32_t)r[j].ty1 << 16), cnt[j],
                                (uint32_t)(FILT ? mq[j] : 255));
            if (hits_out) hits_out[e] = cnt[j];
        }
        bal[j] = ballot64(e < E && cnt[j] > 0);
        key[j] = __float_as_uint(c[j].y);
    }
    compact_block(bal, key, base, blk, lb, total, dkey, dval, hist, s_w, s_h, &s_off);
}

// The compaction alone, over the key words a counting projection wrote
// (kw[e] = depth bits, or KEY_NONE for an entry without keys): the counting
// pass's tickets, lookback and outputs over blocks of KEYW_BLOCK entries
// (fewer blocks than the counting pass: a shorter lookback chain and fewer
// digit-count atomics per histogram word; the set-up clears the counting
// pass's larger number of lookback words).
template <int IT>
__global__ void __launch_bounds__(COUNT_THREADS)
k_compact_keys(const uint32_t *__restrict__ kw, int64_t E, uint32_t *__restrict__ tick, uint64_t *__restrict__ lb,
               uint64_t *__restrict__ total, uint32_t *__restrict__ dkey, uint32_t *__restrict__ dval,
               uint32_t *__restrict__ hist)
{
    __shared__ uint32_t s_blk;
    __shared__ uint32_t s_w[IT][COUNT_THREADS / 64];
    __shared__ uint32_t s_h[4][256];
    __shared__ uint64_t s_off;
    if (threadIdx.x == 0) s_blk = atomicAdd(tick, 1u);
    for (int q = threadIdx.x; q < 4 * 256; q += COUNT_THREADS) (&s_h[0][0])[q] = 0;
    __syncthreads();
    const int64_t blk = s_blk;
    const int64_t base = blk * (COUNT_THREADS * IT);
    uint64_t bal[IT];
    uint32_t key[IT];
#pragma unroll
    for (int j = 0; j < IT; ++j) {
        const int64_t e = base + (int64_t)j * COUNT_THREADS + threadIdx.x;
        key[j] = e < E ? kw[e] : KEY_NONE;
    }
#pragma unroll
    for (int j = 0; j < IT; ++j) bal[j] = ballot64(key[j] != KEY_NONE);
    compact_block(bal, key, base, blk, lb, total, dkey, dval, hist, s_w, s_h, &s_off);
}

// Exclusive scan of nb block values in place by one workgroup of 1024
// threads (block_u32, when given, holds the values as u32); returns the
// total to every thread.
__device__ uint64_t scan_blocks_body(uint64_t *__restrict__ s, uint64_t *__restrict__ block_sums,
                                     const uint32_t *__restrict__ block_u32, int64_t nb)
{
    const int t = threadIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b0 = t * per, b1 = b0 + per < nb ? b0 + per : nb;
    uint64_t local = 0;
    for (int64_t b = b0; b < b1; ++b) local += block_u32 ? block_u32[b] : block_sums[b];
    __syncthreads();  // s may still be read by a previous scan
    s[t] = local;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint64_t add = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    uint64_t run = s[t] - local;
    for (int64_t b = b0; b < b1; ++b) {
        uint64_t x = block_u32 ? block_u32[b] : block_sums[b];
        block_sums[b] = run;
        run += x;
    }
    return s[1023];
}

// Exclusive scan of nb block values in place (one workgroup); the total goes
// to *total.
__global__ void __launch_bounds__(1024)
k_scan_blocks(uint64_t *__restrict__ block_sums, const uint32_t *__restrict__ block_u32, int64_t nb,
              uint64_t *__restrict__ total)
{
    __shared__ uint64_t s[1024];
    const uint64_t tot = scan_blocks_body(s, block_sums, block_u32, nb);
    if (threadIdx.x == 1023) *total = tot;
}

// The two scans after the gather, in one workgroup: block key counts (total
// to *keys_total, or 0 when it exceeds *cap_ptr; the unclamped total to
// *num_keys) and block coarse-pair counts (total to *pairs_total, or 0 when
// the key total was 0: coarse pairs never outnumber keys, so this is the
// overflow case).  On overflow nothing downstream reads the partial lists.
__global__ void __launch_bounds__(1024)
k_scan_pair(uint64_t *__restrict__ key_sums, uint64_t *__restrict__ pair_sums, int64_t nb,
            uint64_t *__restrict__ keys_total, const uint64_t *__restrict__ cap_ptr,
            uint64_t *__restrict__ num_keys, uint64_t *__restrict__ pairs_total, uint64_t *__restrict__ status)
{
    __shared__ uint64_t s[1024];
    const uint64_t kt = scan_blocks_body(s, key_sums, nullptr, nb);
    const uint64_t kc = kt <= *cap_ptr ? kt : 0;
    const uint64_t pt = scan_blocks_body(s, pair_sums, nullptr, nb);
    if (threadIdx.x == 1023) {
        *keys_total = kc;
        if (num_keys) *num_keys = kt;
        if (status) status[0] = kt;
        *pairs_total = pt <= kc ? pt : 0;
    }
}

// ---------------------------------------------------------------------------
// Tile order by a two-level stable counting sort.  The tiles of each view are
// grouped into super-tiles of ST x ST tiles, so that the 64 lanes of a wave
// own the 64 tiles of one super-tile.
//   a. every depth-ordered entry lists the super-tiles that hold at least one
//      of its kept tiles (coarse pairs, in depth order), and a stable radix
//      sort on the super-tile id groups them: each super-tile's run is in
//      depth order;
//   b. each run is cut into chunks of CHUNK entries, one wave per chunk: the
//      lanes walk the chunk's entries in order and each counts the entries
//      that keep its own tile;
//   c. per tile, an exclusive scan of its counts over the chunks of its
//      super-tile and, over all tiles in global tile order, of its totals
//      (the tile ranges);
//   d. the same walk again writes each kept (entry, tile) key at its tile's
//      start + chunk prefix + running count: the (tile, depth, view, point)
//      order, with every key written once at its final position.

// What a coarse pair carries besides its entry (view * n + point): relative
// to super-tile (sx, sy), the entry's clipped tile rectangle (3 bits per
// bound) and min(quality bound, 4) (3 bits; the tile pass tells no higher
// bound apart), 15 bits.  With super-tile ids below 2^ST_ID_BITS they ride
// in the sort key above the id (PACKED: key = id | info << ST_ID_BITS, 4-byte
// value e); else the value is (e, info).
constexpr int ST_ID_BITS = 17;
static_assert(ST == 8, "3 bits per bound");
__device__ __forceinline__ uint32_t coarse_info(uint32_t rx, uint32_t ry, uint32_t m, int sx, int sy)
{
    const int x0 = (int)(rx & 0xffffu) - sx * ST, y0 = (int)(rx >> 16) - sy * ST;
    const int x1 = (int)(ry & 0xffffu) - sx * ST, y1 = (int)(ry >> 16) - sy * ST;
    const uint32_t cx0 = (uint32_t)max(x0, 0), cy0 = (uint32_t)max(y0, 0);
    const uint32_t cx1 = (uint32_t)min(x1, ST - 1), cy1 = (uint32_t)min(y1, ST - 1);
    return cx0 | (cy0 << 3) | (cx1 << 6) | (cy1 << 9) | (min(m, 4u) << 12);
}

// The super-tile sort's digit counts of the pairs a workgroup emits, in LDS
// (sh[p * radix + digit], pass p's digit of the super-tile id: the packed
// info above the id lies past every digit).
struct DigitCount {
    uint32_t *sh;
    int passes, dbits, radix;
    __device__ __forceinline__ void add(uint32_t st_id) const
    {
        const uint32_t mask = (1u << dbits) - 1u;
        for (int p = 0; p < passes; ++p) atomicAdd(&sh[p * radix + ((st_id >> (dbits * p)) & mask)], 1u);
    }
};

template <bool PACKED>
__device__ __forceinline__ void coarse_put(uint32_t *__restrict__ ck, void *__restrict__ cv, uint64_t pos,
                                           uint32_t st_id, uint32_t info, uint32_t e, const DigitCount &dc)
{
    dc.add(st_id);
    if (PACKED) {
        ck[pos] = st_id | (info << ST_ID_BITS);
        reinterpret_cast<uint32_t *>(cv)[pos] = e;
    } else {
        ck[pos] = st_id;
        reinterpret_cast<uint2 *>(cv)[pos] = make_uint2(e, info);
    }
}

// Super-tiles of the entry's view that its tile rectangle [x0, x1] x [y0, y1]
// overlaps and that hold at least one of its kept tiles (with the level
// filter: the class table, and a summed-area count over rectangle and
// super-tile > 0 where the level keeps part of the super-tile), in row-major
// order.  With EMIT, (super-tile id, payload) pairs of entry e are written
// from position pos on.  Returns their number.
template <bool EMIT, bool PACKED = false>
__device__ __forceinline__ uint32_t coarse_walk(uint32_t rx, uint32_t ry, uint32_t m, int v, uint32_t e,
                                                const int64_t *__restrict__ vtab, const int4 *__restrict__ stab,
                                                const uint32_t *__restrict__ sat, const uint8_t *__restrict__ cls,
                                                int L, int64_t n_tiles, uint32_t *__restrict__ ck,
                                                void *__restrict__ cv, uint64_t pos, const DigitCount *dc)
{
    const int x0 = (int)(rx & 0xffffu), y0 = (int)(rx >> 16), x1 = (int)(ry & 0xffffu), y1 = (int)(ry >> 16);
    const int sx0 = x0 / ST, sx1 = x1 / ST, sy0 = y0 / ST, sy1 = y1 / ST;
    const int4 sb = stab[v];
    if (sx0 == sx1 && sy0 == sy1) {
        // one super-tile: it holds all the entry's kept tiles (there is one)
        if (EMIT)
            coarse_put<PACKED>(ck, cv, pos, (uint32_t)(sb.x + sy0 * sb.y + sx0), coarse_info(rx, ry, m, sx0, sy0), e,
                               *dc);
        return 1u;
    }
    const uint32_t *s = nullptr;
    const int ml = (int)m < L ? (int)m : L;
    if (sat) s = sat + (int64_t)(ml - 1) * n_tiles + vtab[2 * v];
    uint32_t c = 0;
    for (int sy = sy0; sy <= sy1; ++sy) {
        const int by0 = y0 > sy * ST ? y0 : sy * ST, by1 = y1 < sy * ST + ST - 1 ? y1 : sy * ST + ST - 1;
        for (int sx = sx0; sx <= sx1; ++sx) {
            const uint32_t st_id = (uint32_t)(sb.x + sy * sb.y + sx);
            bool keep = true;
            if (s) {
                const uint8_t k = cls[(uint64_t)st_id * 4 + ml - 1];
                if (k == 2) {
                    const int bx0 = x0 > sx * ST ? x0 : sx * ST;
                    const int bx1 = x1 < sx * ST + ST - 1 ? x1 : sx * ST + ST - 1;
                    keep = sat_rect(s, sb.z, bx0, bx1, by0, by1) != 0u;
                } else {
                    keep = k == 1;
                }
            }
            if (keep) {
                if (EMIT) coarse_put<PACKED>(ck, cv, pos + c, st_id, coarse_info(rx, ry, m, sx, sy), e, *dc);
                ++c;
            }
        }
    }
    return c;
}

// Coarse pairs of an entry whose rectangle spans at most MS x MS super-tiles,
// as a mask: bit dy * MS + dx for super-tile (sx0 + dx, sy0 + dy).  Larger
// spans have no mask (coarse_walk is run again to emit them).  Encoded count:
// bit 31 set -> mask in bits 0..15 and count in bits 16..20; else the count.
__device__ __forceinline__ uint32_t cc_count(uint32_t cc) { return (cc >> 31) ? (cc >> 16) & 31u : cc; }

__device__ __forceinline__ uint32_t coarse_code(uint32_t rx, uint32_t ry, uint32_t m, int v,
                                                const int64_t *__restrict__ vtab, const int4 *__restrict__ stab,
                                                const uint32_t *__restrict__ sat, const uint8_t *__restrict__ cls,
                                                int L, int64_t n_tiles)
{
    const int x0 = (int)(rx & 0xffffu), y0 = (int)(rx >> 16), x1 = (int)(ry & 0xffffu), y1 = (int)(ry >> 16);
    const int sx0 = x0 / ST, sx1 = x1 / ST, sy0 = y0 / ST, sy1 = y1 / ST;
    if (sx1 - sx0 >= MS || sy1 - sy0 >= MS)
        return coarse_walk<false>(rx, ry, m, v, 0u, vtab, stab, sat, cls, L, n_tiles, nullptr, nullptr, 0, nullptr);
    if (sx0 == sx1 && sy0 == sy1) return 0x80000000u | (1u << 16) | 1u;
    const int4 sb = stab[v];
    const int ml = (int)m < L ? (int)m : L;
    const uint32_t *s = sat ? sat + (int64_t)(ml - 1) * n_tiles + vtab[2 * v] : nullptr;
    uint32_t mask = 0;
    for (int dy = 0; dy <= sy1 - sy0; ++dy) {
        const int sy = sy0 + dy;
        const int by0 = y0 > sy * ST ? y0 : sy * ST, by1 = y1 < sy * ST + ST - 1 ? y1 : sy * ST + ST - 1;
        for (int dx = 0; dx <= sx1 - sx0; ++dx) {
            const int sx = sx0 + dx;
            bool keep = true;
            if (s) {
                const uint8_t k = cls[(uint64_t)(sb.x + sy * sb.y + sx) * 4 + ml - 1];
                if (k == 2) {
                    const int bx0 = x0 > sx * ST ? x0 : sx * ST;
                    const int bx1 = x1 < sx * ST + ST - 1 ? x1 : sx * ST + ST - 1;
                    keep = sat_rect(s, sb.z, bx0, bx1, by0, by1) != 0u;
                } else {
                    keep = k == 1;
                }
            }
            mask |= keep ? 1u << (dy * MS + dx) : 0u;
        }
    }
    return 0x80000000u | ((uint32_t)__popc(mask) << 16) | mask;
}

// 4a. gather the records in depth order: rec_s[r] = {x0 | y0 << 16,
// x1 | y1 << 16, entry, view << 8 | quality bound}; cc_s[r] = its coarse
// pairs (count, or count and mask, as coarse_code); per-block sums of key counts and
// coarse pairs.  A block takes ENTRY_BLOCK entries with
// GATHER_THREADS threads, each issuing its loads for all its entries first.
// The depth sort is done by now: the first block zeroes the sort's digit
// counts and tickets for the super-tile sort (see k_coarse_emit).
constexpr int GATHER_THREADS = 1024;
constexpr int GATHER_ITEMS = ENTRY_BLOCK / GATHER_THREADS;
__global__ void __launch_bounds__(GATHER_THREADS)
k_gather(const uint32_t *__restrict__ order, const uint4 *__restrict__ rec, const uint64_t *__restrict__ d_count,
         int n, const int64_t *__restrict__ vtab, const int4 *__restrict__ stab, const uint32_t *__restrict__ sat,
         const uint8_t *__restrict__ cls, int L, int64_t n_tiles, uint4 *__restrict__ rec_s,
         uint32_t *__restrict__ cc_s, uint64_t *__restrict__ bsum_h, uint64_t *__restrict__ bsum_c,
         uint32_t *__restrict__ sort_hist, uint32_t *__restrict__ sort_tickets)
{
    __shared__ uint64_t s_h[GATHER_THREADS / 64], s_c[GATHER_THREADS / 64];
    if (blockIdx.x == 0) {
        sort_hist[threadIdx.x] = 0u;  // [4][256]: one word per thread
        if (threadIdx.x < 4) sort_tickets[threadIdx.x] = 0u;
    }
    const uint64_t E = *d_count;
    const int64_t base = (int64_t)blockIdx.x * (GATHER_THREADS * GATHER_ITEMS);
    uint32_t e[GATHER_ITEMS];
    uint4 q[GATHER_ITEMS];
#pragma unroll
    for (int j = 0; j < GATHER_ITEMS; ++j) {
        const int64_t r = base + (int64_t)j * GATHER_THREADS + threadIdx.x;
        e[j] = (uint64_t)r < E ? order[r] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int j = 0; j < GATHER_ITEMS; ++j) q[j] = e[j] != 0xFFFFFFFFu ? rec[e[j]] : make_uint4(0u, 0u, 0u, 0u);
    uint64_t acc_h = 0, acc_c = 0;
#pragma unroll
    for (int j = 0; j < GATHER_ITEMS; ++j) {
        if (e[j] == 0xFFFFFFFFu) continue;
        const int64_t r = base + (int64_t)j * GATHER_THREADS + threadIdx.x;
        const int v = (int)(e[j] / (uint32_t)n);
        const uint32_t m = q[j].w & 255u;
        const uint32_t code = coarse_code(q[j].x, q[j].y, m, v, vtab, stab, sat, cls, L, n_tiles);
        rec_s[r] = make_uint4(q[j].x, q[j].y, e[j], ((uint32_t)v << 8) | m);
        cc_s[r] = code;
        acc_h += q[j].z;
        acc_c += cc_count(code);
    }
    for (int off = 32; off > 0; off >>= 1) {
        acc_h += __shfl_xor(acc_h, off);
        acc_c += __shfl_xor(acc_c, off);
    }
    if ((threadIdx.x & 63) == 0) {
        s_h[threadIdx.x >> 6] = acc_h;
        s_c[threadIdx.x >> 6] = acc_c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t th = 0, tc = 0;
        for (int w = 0; w < GATHER_THREADS / 64; ++w) {
            th += s_h[w];
            tc += s_c[w];
        }
        bsum_h[blockIdx.x] = th;
        bsum_c[blockIdx.x] = tc;
    }
}

// 4b. coarse pairs of every depth-ordered entry at its scanned offset (from
// the mask when there is one).  The super-tile sort needs no set-up launch of
// its own: each workgroup counts the digits of the super-tile ids it emits
// into the sort's digit counts (zeroed by k_gather), and the grid zeroes the
// sort's first-pass lookback words for the pairs' count, counts[3] (clamped
// to cap): ceil(count / part) * radix words.
template <bool PACKED>
__global__ void __launch_bounds__(GATHER_THREADS)
k_coarse_emit(const uint4 *__restrict__ rec_s, const uint32_t *__restrict__ cc_s, const uint64_t *__restrict__ counts,
              const uint64_t *__restrict__ boff, const int64_t *__restrict__ vtab, const int4 *__restrict__ stab,
              const uint32_t *__restrict__ sat, const uint8_t *__restrict__ cls, int L, int64_t n_tiles,
              uint32_t *__restrict__ ck, void *__restrict__ cv, uint64_t *__restrict__ sort_status, uint64_t cap,
              RadixShape shape, uint32_t *__restrict__ sort_hist)
{
    constexpr int W = GATHER_THREADS / 64;
    __shared__ uint32_t s_w[GATHER_ITEMS][W];
    __shared__ uint32_t s_dig[4 * 256];
    const int part = shape.part, radix = shape.radix;
    for (int q = threadIdx.x; q < 4 * 256; q += GATHER_THREADS) s_dig[q] = 0u;  // (visible after the barrier below)
    const DigitCount dc{s_dig, shape.passes, shape.dbits, radix};
    {
        const uint64_t np = counts[3] < cap ? counts[3] : cap;
        const uint64_t words = ((np + part - 1) / part) * (uint64_t)radix;
        const uint64_t stride = (uint64_t)gridDim.x * GATHER_THREADS;
        for (uint64_t i = (uint64_t)blockIdx.x * GATHER_THREADS + threadIdx.x; i < words; i += stride)
            sort_status[i] = 0;
    }
    const uint64_t E = counts[0];
    if (counts[1] == 0) return;  // no keys, or more than the capacity
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * (GATHER_THREADS * GATHER_ITEMS);
    if ((uint64_t)base >= E) return;
    uint32_t c[GATHER_ITEMS], x[GATHER_ITEMS];
    uint4 q[GATHER_ITEMS];
#pragma unroll
    for (int j = 0; j < GATHER_ITEMS; ++j) {
        const int64_t r = base + (int64_t)j * GATHER_THREADS + threadIdx.x;
        const bool ok = (uint64_t)r < E;
        c[j] = ok ? cc_s[r] : 0u;
        q[j] = ok ? rec_s[r] : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int j = 0; j < GATHER_ITEMS; ++j) {
        x[j] = wave_incl_scan(cc_count(c[j]));
        if (lane == 63) s_w[j][wave] = x[j];
    }
    __syncthreads();
    // the (item, wave) totals scanned once in entry order (item-major) by
    // the first wave, so that an item's offset is one LDS read
    static_assert(GATHER_ITEMS * W <= 64, "one wave scans the (item, wave) totals");
    uint32_t *flat = &s_w[0][0];  // index j * W + w
    if (wave == 0) {
        const uint32_t v = lane < GATHER_ITEMS * W ? flat[lane] : 0u;
        const uint32_t inc = wave_incl_scan(v);
        if (lane < GATHER_ITEMS * W) flat[lane] = inc - v;
    }
    __syncthreads();
    const uint64_t run = boff[blockIdx.x];
#pragma unroll
    for (int j = 0; j < GATHER_ITEMS; ++j) {
        const int64_t r = base + (int64_t)j * GATHER_THREADS + threadIdx.x;
        const uint32_t cnt = cc_count(c[j]);
        const uint64_t pos = run + flat[j * W + wave] + x[j] - cnt;
        if (cnt) {
            const int v = (int)(q[j].w >> 8);
            if (c[j] >> 31) {
                const int4 sb = stab[v];
                const int sx0 = (int)(q[j].x & 0xffffu) / ST, sy0 = (int)(q[j].x >> 16) / ST;
                uint32_t mask = c[j] & 0xffffu, k = 0;
                while (mask) {
                    const int bit = __ffs(mask) - 1;
                    mask &= mask - 1u;
                    const int sx = sx0 + bit % MS, sy = sy0 + bit / MS;
                    coarse_put<PACKED>(ck, cv, pos + k, (uint32_t)(sb.x + sy * sb.y + sx),
                                       coarse_info(q[j].x, q[j].y, q[j].w & 255u, sx, sy), q[j].z, dc);
                    ++k;
                }
            } else {
                coarse_walk<true, PACKED>(q[j].x, q[j].y, q[j].w & 255u, v, q[j].z, vtab, stab, sat, cls, L,
                                          n_tiles, ck, cv, pos, &dc);
            }
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < shape.passes * radix; q += GATHER_THREADS)
        if (s_dig[q]) atomicAdd(&sort_hist[q], s_dig[q]);
}

// View of a super-tile: the last view whose first super-tile is <= s.
__device__ __forceinline__ int view_of_st(const int4 *__restrict__ stab, int V, int s)
{
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (stab[mid].x <= s)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Chunks of every super-tile's run: chunk_off[s] = first chunk of s
// (chunk_off[n_st] = their number, also in *n_chunks).  One workgroup; each
// thread takes consecutive super-tiles.  With FILL (n_st <= 1024, one
// super-tile per thread) the same workgroup also writes the chunk records,
// chunk[c] = {first pair, end pair, super-tile, view}, a wave per super-tile.
template <bool FILL>
__global__ void __launch_bounds__(1024)
k_chunk_table(const uint32_t *__restrict__ st_ranges, int64_t n_st, uint32_t *__restrict__ chunk_off,
              uint64_t *__restrict__ n_chunks, const int4 *__restrict__ stab, int V, uint4 *__restrict__ chunk)
{
    // with FILL, each thread's super-tile run (first, end pair) and view stay
    // in LDS for the fill, so no wave waits on a global load per super-tile
    __shared__ uint32_t s[1024];
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_b[FILL ? 1024 : 1], s_e[FILL ? 1024 : 1], s_v[FILL ? 1024 : 1];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int64_t per = (n_st + 1023) / 1024;
    const int64_t b0 = t * per < n_st ? t * per : n_st, b1 = b0 + per < n_st ? b0 + per : n_st;
    uint32_t local = 0;
    if constexpr (FILL) {
        // per == 1: super-tile t
        if (b0 < b1) {
            const uint32_t bq = st_ranges[2 * b0], eq = st_ranges[2 * b0 + 1];
            s_b[t] = bq;
            s_e[t] = eq;
            s_v[t] = (uint32_t)view_of_st(stab, V, (int)b0);
            local = (eq - bq + CHUNK - 1) / CHUNK;
        }
    } else {
        for (int64_t q = b0; q < b1; ++q) local += (st_ranges[2 * q + 1] - st_ranges[2 * q] + CHUNK - 1) / CHUNK;
    }
    // inclusive prefix over the threads: a scan per wave, then the wave totals
    const uint32_t x = wave_incl_scan(local);
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    uint32_t add = 0, all = 0;
    for (int w = 0; w < 16; ++w) {
        const uint32_t y = s_w[w];
        if (w < wave) add += y;
        all += y;
    }
    s[t] = add + x;
    uint32_t run = add + x - local;
    if constexpr (FILL) {
        if (b0 < b1) chunk_off[b0] = run;
    } else {
        for (int64_t q = b0; q < b1; ++q) {
            chunk_off[q] = run;
            run += (st_ranges[2 * q + 1] - st_ranges[2 * q] + CHUNK - 1) / CHUNK;
        }
    }
    if (t == 1023) {
        chunk_off[n_st] = all;
        *n_chunks = all;
    }
    if constexpr (FILL) {
        __syncthreads();
        // s[q] is the inclusive chunk prefix of super-tile q; a wave per super-tile
        for (int64_t q = wave; q < n_st; q += 1024 / 64) {
            const uint32_t c1 = s[q], c0 = q > 0 ? s[q - 1] : 0u;
            if (c1 == c0) continue;
            const uint32_t bq = s_b[q], eq = s_e[q], v = s_v[q];
            for (uint32_t c = c0 + lane; c < c1; c += 64) {
                const uint32_t bb = bq + (c - c0) * CHUNK;
                chunk[c] = make_uint4(bb, eq < bb + CHUNK ? eq : bb + CHUNK, (uint32_t)q, v);
            }
        }
    }
}

// Chunk records: chunk[c] = {first pair, end pair, super-tile, view}.  One
// workgroup per super-tile.
__global__ void __launch_bounds__(256)
k_chunk_fill(const uint32_t *__restrict__ st_ranges, const uint32_t *__restrict__ chunk_off,
             const int4 *__restrict__ stab, int V, uint4 *__restrict__ chunk)
{
    const uint32_t s = blockIdx.x;
    const uint32_t c0 = chunk_off[s], nch = chunk_off[s + 1] - c0;
    if (nch == 0) return;
    const uint32_t b0 = st_ranges[2 * s], e0 = st_ranges[2 * s + 1];
    const uint32_t v = (uint32_t)view_of_st(stab, V, (int)s);
    for (uint32_t t = threadIdx.x; t < nch; t += blockDim.x) {
        const uint32_t b = b0 + t * CHUNK;
        chunk[c0 + t] = make_uint4(b, e0 < b + CHUNK ? e0 : b + CHUNK, s, v);
    }
}

// 4c/4e. One wave per chunk of a super-tile's run.  Lane j of batch q holds
// entry b + 64 q + j of the chunk as a mask of the super-tile's tiles it keeps
// (bit l = tile (l % ST, l / ST): inside its rectangle and, with the level
// filter, of lower level <= its quality bound).  The wave visits the tiles
// in the union of the masks; per tile and batch a ballot of the mask bits
// gives the covering entries in order.  COUNT: ccnt[c][l] = entries of the
// chunk that keep tile l.  WRITE: their point indices (and optional 64-bit
// keys), ranked by mbcnt, at the tile's start + the chunk's exclusive prefix
// (ccnt after k_col_scan) + the running count: a tile's keys of one batch
// are one contiguous store.
constexpr int NB = CHUNK / 64;  // batches of 64 entries per chunk
// bit y * ST of every row y < ST: spreads an ST-bit row mask over all rows
__host__ __device__ constexpr uint64_t row_spread()
{
    uint64_t r = 0;
    for (int y = 0; y < ST; ++y) r |= 1ull << (y * ST);
    return r;
}
template <bool WRITE, bool PACKED, bool KEYS>
__global__ void __launch_bounds__(256)
k_tile_pass(const uint32_t *__restrict__ ck, const void *__restrict__ cv, const uint4 *__restrict__ chunk,
            const uint64_t *__restrict__ counts,
            const int64_t *__restrict__ vtab,
            const int4 *__restrict__ stab, int V, int n, const uint8_t *__restrict__ tl, uint32_t *__restrict__ ccnt,
            const uint32_t *__restrict__ ranges, uint32_t *__restrict__ vals, uint64_t *__restrict__ keys,
            const gs_splat *__restrict__ splats)
{
    // output position of each tile of the wave's super-tile, read back with
    // uniform LDS loads inside the tile loop (a register loaded from memory
    // would make every iteration wait for the stores before it)
    __shared__ uint32_t s_pos[4][TST];
    if (counts[1] == 0) return;  // no keys, or more than the capacity
    const uint64_t nc = counts[4];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
    for (uint64_t c = (uint64_t)blockIdx.x * (blockDim.x / 64) + wave; c < nc; c += waves) {
        const uint4 ch = chunk[c];
        const uint32_t b = ch.x, e_end = ch.y, s = ch.z;
        const int v = (int)ch.w;
        // the chunk's pairs early (entry, info): they do not depend on the view
        uint2 pj[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const uint32_t j = b + 64u * q + (uint32_t)lane;
            if (j < e_end) {
                if (PACKED)
                    pj[q] = make_uint2(reinterpret_cast<const uint32_t *>(cv)[j], ck[j] >> ST_ID_BITS);
                else
                    pj[q] = reinterpret_cast<const uint2 *>(cv)[j];
            } else {
                pj[q] = make_uint2(0u, 0xFFFFFFFFu);  // no entry (info never has bit 31)
            }
        }
        const int4 sb = stab[v];
        const int sl = (int)s - sb.x, sy = sl / sb.y, sx = sl - sy * sb.y;
        const int bx = sx * ST, by = sy * ST;
        const int64_t toff = vtab[2 * v];
        // per level m: the super-tile's tiles whose lower level is <= m
        uint64_t lvm1 = ~0ull, lvm2 = ~0ull, lvm3 = ~0ull, lvm4 = ~0ull;
        {
            const int mtx = bx + lane % ST, mty = by + lane / ST;
            const bool mvalid = lane < TST && mtx < sb.z && mty < sb.w;
            const int64_t mg = toff + (int64_t)mty * sb.z + mtx;
            if (tl) {
                const uint32_t lvl = mvalid ? (uint32_t)tl[2 * mg] : 255u;
                lvm1 = __builtin_amdgcn_ballot_w64(lvl <= 1u);
                lvm2 = __builtin_amdgcn_ballot_w64(lvl <= 2u);
                lvm3 = __builtin_amdgcn_ballot_w64(lvl <= 3u);
                lvm4 = __builtin_amdgcn_ballot_w64(lvl <= 4u);
            }
            if (WRITE && lane < TST) s_pos[wave][lane] = mvalid ? ranges[2 * mg] + ccnt[c * TST + lane] : 0u;
        }
        // the chunk's entries as tile masks, and their union
        uint32_t mlo[NB], mhi[NB], ez[NB];
        uint64_t uni = 0;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            uint64_t tm = 0;
            ez[q] = 0u;
            if (pj[q].y != 0xFFFFFFFFu) {
                const uint32_t w = pj[q].y;
                const int cx0 = (int)(w & 7u), cy0 = (int)((w >> 3) & 7u);
                const int cx1 = (int)((w >> 6) & 7u), cy1 = (int)((w >> 9) & 7u);
                const uint64_t cols = (2ull << cx1) - (1ull << cx0);
                const int hb = (cy1 + 1) * ST;
                const uint64_t rows = (hb >= 64 ? ~0ull : (1ull << hb) - 1ull) & ~((1ull << (cy0 * ST)) - 1ull);
                tm = cols * row_spread() & rows;
                const uint32_t m = w >> 12;
                tm &= m >= 4u ? lvm4 : (m == 3u ? lvm3 : (m == 2u ? lvm2 : lvm1));
                ez[q] = pj[q].x;
            }
            mlo[q] = (uint32_t)tm;
            mhi[q] = (uint32_t)(tm >> 32);
            uni |= tm;
        }
        const uint32_t ulo = wave_or((uint32_t)uni), uhi = wave_or((uint32_t)(uni >> 32));
        const uint32_t vbase = (uint32_t)v * (uint32_t)n;
        wave_lds_sync();
        uint32_t mcnt = 0;
        // batches past the chunk's end hold empty masks: their ballots are
        // zero, so no batch needs a bounds test; a batch's store is skipped by
        // the empty exec mask
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            uint32_t um = half ? uhi : ulo;
            while (um) {
                const int l32 = __builtin_ctz(um);
                um &= um - 1u;
                const int l = half * 32 + l32;
                uint32_t pos = 0;
                if (WRITE) pos = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_pos[wave][l]);
                uint32_t tot = 0;
#pragma unroll
                for (int q = 0; q < NB; ++q) {
                    const bool cov = (((half ? mhi[q] : mlo[q]) >> l32) & 1u) != 0u;
                    const uint64_t bal = __builtin_amdgcn_ballot_w64(cov);
                    if (WRITE) {
                        if (cov) {
                            const uint32_t at = pos + __builtin_amdgcn_mbcnt_hi(
                                                          (uint32_t)(bal >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                            vals[at] = ez[q] - vbase;
                            if (KEYS)
                                keys[at] = ((uint64_t)(toff + (int64_t)(by + l / ST) * sb.z + bx + l % ST) << 32) |
                                           __float_as_uint(splats[ez[q]].depth);
                        }
                        pos += (uint32_t)__popcll(bal);
                    } else {
                        tot += (uint32_t)__popcll(bal);
                    }
                }
                if (!WRITE) mcnt = lane == l ? tot : mcnt;
            }
        }
        if (!WRITE && lane < TST) ccnt[c * TST + lane] = mcnt;
        // the next chunk rewrites the wave's LDS row
        wave_lds_sync();
    }
}

// 4d. per super-tile and lane (tile): exclusive prefix of the chunk counts
// in place, and the tile's total.  COL_WAVES waves split the chunks.
constexpr int COL_WAVES = 16;
__global__ void __launch_bounds__(COL_WAVES * 64)
k_col_scan(const uint32_t *__restrict__ chunk_off, const int64_t *__restrict__ vtab, const int4 *__restrict__ stab,
           int V, uint32_t *__restrict__ ccnt, uint32_t *__restrict__ tot)
{
    __shared__ uint32_t s_part[COL_WAVES][64];
    const bool tile_lane = (threadIdx.x & 63) < TST;
    const uint32_t s = blockIdx.x;
    const uint32_t c0 = chunk_off[s], nch = chunk_off[s + 1] - c0;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t per = (nch + COL_WAVES - 1) / COL_WAVES;
    const uint32_t a = c0 + (wave * per < nch ? wave * per : nch);
    const uint32_t z = c0 + ((wave + 1) * per < nch ? (wave + 1) * per : nch);
    uint32_t sum = 0;
    if (tile_lane)
        for (uint32_t c = a; c < z; ++c) sum += ccnt[(uint64_t)c * TST + lane];
    s_part[wave][lane] = sum;
    __syncthreads();
    uint32_t run = 0, total = 0;
    for (int w = 0; w < COL_WAVES; ++w) {
        const uint32_t x = s_part[w][lane];
        if (w < wave) run += x;
        total += x;
    }
    if (tile_lane) {
        for (uint32_t c = a; c < z; ++c) {
            const uint32_t x = ccnt[(uint64_t)c * TST + lane];
            ccnt[(uint64_t)c * TST + lane] = run;
            run += x;
        }
    }
    if (wave == 0 && tile_lane) {
        const int v = view_of_st(stab, V, (int)s);
        const int4 sb = stab[v];
        const int sl = (int)s - sb.x, sy = sl / sb.y, sx = sl - sy * sb.y;
        const int tx = sx * ST + lane % ST, ty = sy * ST + lane / ST;
        if (tx < sb.z && ty < sb.w) tot[vtab[2 * v] + (int64_t)ty * sb.z + tx] = total;
    }
}

// Block sums of the per-tile totals (blocks of SCAN_THREADS * SCAN_ITEMS tiles).
__global__ void __launch_bounds__(SCAN_THREADS)
k_tile_reduce(const uint32_t *__restrict__ tot, int64_t n_tiles, uint64_t *__restrict__ bsum)
{
    __shared__ uint64_t s_w[SCAN_THREADS / 64];
    const int64_t base = (int64_t)blockIdx.x * (SCAN_THREADS * SCAN_ITEMS);
    uint64_t acc = 0;
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const int64_t g = base + (int64_t)j * SCAN_THREADS + threadIdx.x;
        if (g < n_tiles) acc += tot[g];
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < SCAN_THREADS / 64; ++w) t += s_w[w];
        bsum[blockIdx.x] = t;
    }
}

// 4d. tile ranges from the totals: thread t of a block takes SCAN_ITEMS
// consecutive tiles; an empty tile gets (0, 0).
__global__ void __launch_bounds__(SCAN_THREADS)
k_tile_ranges(const uint32_t *__restrict__ tot, int64_t n_tiles, const uint64_t *__restrict__ boff,
              const uint64_t *__restrict__ counts, uint32_t *__restrict__ ranges)
{
    __shared__ uint64_t s_w[SCAN_THREADS / 64];
    if (counts[1] == 0) return;  // ranges stay zero
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t g0 = (int64_t)blockIdx.x * (SCAN_THREADS * SCAN_ITEMS) + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t t[SCAN_ITEMS];
    uint64_t local = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        t[j] = g0 + j < n_tiles ? tot[g0 + j] : 0u;
        local += t[j];
    }
    uint64_t x = local;
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    uint64_t run = boff[blockIdx.x] + x - local;
    for (int w = 0; w < wave; ++w) run += s_w[w];
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        if (g0 + j < n_tiles)
            reinterpret_cast<uint2 *>(ranges)[g0 + j] =
                t[j] ? make_uint2((uint32_t)run, (uint32_t)(run + t[j])) : make_uint2(0u, 0u);
        run += t[j];
    }
}

// 4d in one workgroup (grids of up to TILE_SCAN1_MAX tiles): tile ranges
// from the totals.  Segment after segment (with a running carry), wave w
// takes 1024 consecutive tiles as SCAN_ITEMS rows of 64, lane l of row j
// holding tile 64 j + l (coalesced loads and stores); the rows are scanned
// in order by wave prefix sums.  An empty tile gets (0, 0).
constexpr int TS1_THREADS = 1024;
constexpr int64_t TILE_SCAN1_MAX = 4 * TS1_THREADS * SCAN_ITEMS;
__global__ void __launch_bounds__(TS1_THREADS)
k_tile_scan1(const uint32_t *__restrict__ tot, int64_t n_tiles, const uint64_t *__restrict__ counts,
             uint32_t *__restrict__ ranges)
{
    constexpr int WAVES = TS1_THREADS / 64;
    __shared__ uint64_t s_w[WAVES];
    if (counts[1] == 0) return;  // ranges stay zero
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t carry = 0;
    for (int64_t seg = 0; seg < n_tiles; seg += TS1_THREADS * SCAN_ITEMS) {
        const int64_t g0 = seg + (int64_t)wave * (64 * SCAN_ITEMS) + lane;
        uint32_t t[SCAN_ITEMS];
        uint32_t local = 0;
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            t[j] = g0 + 64 * j < n_tiles ? tot[g0 + 64 * j] : 0u;
            local += t[j];
        }
        uint64_t wt = local;
        for (int off = 32; off > 0; off >>= 1) wt += __shfl_xor(wt, off);
        if (lane == 0) s_w[wave] = wt;
        __syncthreads();
        uint64_t run = carry, segtot = 0;
        for (int w = 0; w < WAVES; ++w) {
            const uint64_t sw = s_w[w];
            run += w < wave ? sw : 0;
            segtot += sw;
        }
#pragma unroll
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            const uint32_t x = wave_incl_scan(t[j]);
            const uint64_t b0 = run + x - t[j];
            if (g0 + 64 * j < n_tiles)
                reinterpret_cast<uint2 *>(ranges)[g0 + 64 * j] =
                    t[j] ? make_uint2((uint32_t)b0, (uint32_t)(b0 + t[j])) : make_uint2(0u, 0u);
            run += __shfl(x, 63);
        }
        carry += segtot;
        __syncthreads();  // s_w is rewritten by the next segment
    }
}

// Super-tile ranges: four sorted ids (the key bits under id_mask) per
// thread; a boundary between k - 1 and k closes one run and opens the next.
__global__ void __launch_bounds__(256)
k_ranges(const uint32_t *__restrict__ tkey, uint32_t id_mask, const uint64_t *__restrict__ d_count, uint64_t cap,
         int64_t n_ids,
         uint32_t *__restrict__ ranges)
{
    uint64_t count = *d_count;
    count = count < cap ? count : cap;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * 4;
    for (uint64_t k0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; k0 < count; k0 += stride) {
        uint32_t t[5];
        t[0] = k0 == 0 ? 0xFFFFFFFFu : tkey[k0 - 1] & id_mask;
        if (k0 + 4 <= count) {
            const uint4 q = *reinterpret_cast<const uint4 *>(tkey + k0);
            t[1] = q.x & id_mask; t[2] = q.y & id_mask; t[3] = q.z & id_mask; t[4] = q.w & id_mask;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) t[j + 1] = k0 + j < count ? tkey[k0 + j] & id_mask : 0xFFFFFFFFu;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t k = k0 + j;
            if (k >= count) break;
            if (t[j + 1] != t[j]) {
                if (t[j + 1] < n_ids) ranges[2 * (uint64_t)t[j + 1]] = (uint32_t)k;
                if (k > 0 && t[j] < n_ids) ranges[2 * (uint64_t)t[j] + 1] = (uint32_t)k;
            }
        }
        if (k0 + 4 >= count) {
            const uint32_t last = t[count - k0];
            if (last < n_ids) ranges[2 * (uint64_t)last + 1] = (uint32_t)count;
        }
    }
}

inline int grid_for(uint64_t work, int per_block, int cap_blocks)
{
    uint64_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > (uint64_t)cap_blocks) b = cap_blocks;
    return (int)b;
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, uint64_t count, hipStream_t st)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(count, 256 * 4, 8192)), dim3(256), 0, st, p, value,
                       count);
    return hipGetLastError();
}

namespace {

__global__ void k_status_views(const uint64_t *__restrict__ req_cap, const uint64_t *__restrict__ nums, int V,
                               uint64_t cap, uint64_t *__restrict__ status, uint64_t *__restrict__ num_keys)
{
    uint64_t most = 0, total = 0;
    for (int v = 0; v < V; ++v) {
        most = max(most, req_cap[2 * v]);
        total += nums[v];
    }
    status[0] = most * (uint64_t)V;
    status[1] = cap;
    if (num_keys) *num_keys = total;
}

}  // namespace

hipError_t launch_status_views(const uint64_t *req_cap, const uint64_t *nums, int V, uint64_t cap,
                               uint64_t *status, uint64_t *num_keys, hipStream_t st)
{
    hipLaunchKernelGGL(k_status_views, dim3(1), dim3(1), 0, st, req_cap, nums, V, cap, status, num_keys);
    return hipGetLastError();
}

ProjBin bin_counting_args(const BinScratch &bs, int64_t n_tiles)
{
    return ProjBin{bs.sat, bs.bbox, bs.vtab, n_tiles, bs.rec, bs.dkey_b};
}

hipError_t launch_bin_sort(const gs_splat *splats, int n, const gs_camera *cams_dev,
                           const gs_camera *cams_host, int V, int64_t n_tiles, int T,
                           const uint8_t *tile_level, const uint8_t *qbound, int n_levels,
                           uint32_t *vals, uint64_t *keys, uint64_t cap, uint32_t *ranges,
                           uint32_t *hits_out, uint64_t *num_keys, const BinScratch &bs,
                           bool coarse_packed, uint64_t *status, hipStream_t st, BinMode mode)
{
    const int64_t E = (int64_t)V * n;
    hipError_t err;
    int64_t n_st = 0;
    int max_view_tiles = 0;
    for (int v = 0; v < V; ++v) {
        const int tx = (cams_host[v].width + T - 1) / T, ty = (cams_host[v].height + T - 1) / T;
        n_st += (int64_t)((tx + ST - 1) / ST) * ((ty + ST - 1) / ST);
        max_view_tiles = tx * ty > max_view_tiles ? tx * ty : max_view_tiles;
    }
    const int64_t nb = (E + ENTRY_BLOCK - 1) / ENTRY_BLOCK;  // gather and emission blocks
    const int64_t nbc = (E + COUNT_BLOCK - 1) / COUNT_BLOCK;  // counting-pass blocks
    // the counting pass's ticket and lookback words, and the depth sort's
    // state for all E entries, are cleared with the rest of the set-up
    SetupClears z;
    z.lb = bs.block_sums;
    z.nb = nbc;
    z.tick = bs.block_vis;
    z.hist = bs.rs.hist;
    z.tickets = bs.rs.tickets;
    z.status = bs.rs.status;
    z.status_words = radix_prepare_words(bs.rs, (uint64_t)E, 4, 32);
    if (z.status_words > bs.rs.status_words) return hipErrorInvalidValue;
    const uint64_t setup_n = std::max<uint64_t>(2 * (uint64_t)(n_tiles > n_st ? n_tiles : n_st), z.status_words);
    const bool filt = tile_level != nullptr;
    const int L = n_levels < 1 ? 1 : (n_levels > 4 ? 4 : n_levels);
    if (mode != BIN_COUNTED) {
        hipLaunchKernelGGL(k_bin_setup, dim3(grid_for(setup_n, 256 * 4, 256)), dim3(256), 0, st, cams_dev, V, T,
                           bs.vtab, bs.stab, bs.counts + 2, cap, ranges, n_tiles, bs.st_ranges, n_st,
                           E == 0 ? num_keys : nullptr, status, z);
        if (E == 0) return hipGetLastError();
        if (filt) {
            const int lds = max_view_tiles <= SAT_LDS_TILES;
            const unsigned cls_blocks = (unsigned)((n_st + 15) / 16);
            hipLaunchKernelGGL(k_level_sat, dim3(V * L + cls_blocks), dim3(1024), lds ? 5 * max_view_tiles + 16 : 0,
                               st, cams_dev, V, T, L, n_tiles, tile_level, bs.sat, bs.bbox, lds, bs.vtab, bs.stab,
                               n_st, bs.st_cls);
        }
        if (mode == BIN_SETUP) return hipGetLastError();
    } else if (E == 0) {
        return hipSuccess;
    }
    const uint32_t *sat = filt ? bs.sat : nullptr;
    // 1-2: counts, and the stable compaction of the entries with keys (depth
    // digits counted, the total to counts[0]); after a counting projection
    // only the compaction of its key words
#define GS_CK(IT)                                                                                         \
    hipLaunchKernelGGL(k_compact_keys<IT>, dim3((unsigned)((E + IT * COUNT_THREADS - 1) / (IT * COUNT_THREADS))), \
                       dim3(COUNT_THREADS), 0, st, bs.dkey_b, E, bs.block_vis, bs.block_sums, bs.counts, bs.dkey_a,  \
                       bs.dval_a, bs.rs.hist)
    if (mode == BIN_COUNTED) {
        if (E >= (int64_t)KEYW_MIN_BLOCKS * 16 * COUNT_THREADS)
            GS_CK(16);
        else if (E >= (int64_t)KEYW_MIN_BLOCKS * 8 * COUNT_THREADS)
            GS_CK(8);
        else
            GS_CK(4);
    } else if (filt) {
        hipLaunchKernelGGL(k_count<true>, dim3((unsigned)nbc), dim3(COUNT_THREADS), 0, st, splats, n, cams_dev, V, T,
                           bs.vtab, sat, bs.bbox, L, n_tiles, qbound, bs.rec, hits_out, bs.block_vis,
                           bs.block_sums, bs.counts, bs.dkey_a, bs.dval_a, bs.rs.hist);
    } else {
        hipLaunchKernelGGL(k_count<false>, dim3((unsigned)nbc), dim3(COUNT_THREADS), 0, st, splats, n, cams_dev, V, T,
                           bs.vtab, sat, bs.bbox, L, n_tiles, qbound, bs.rec, hits_out, bs.block_vis,
                           bs.block_sums, bs.counts, bs.dkey_a, bs.dval_a, bs.rs.hist);
    }
#undef GS_CK
    // 3: depth sort of the entries with keys (4 x 8-bit passes), result back in (dkey_a, dval_a)
    if ((err = radix_sort_pairs(bs.dkey_a, bs.dval_a, bs.dkey_b, bs.dval_b, bs.counts, (uint64_t)E, 32, bs.rs, st,
                                true)) != hipSuccess)
        return err;
    // 4a: records in depth order; totals of keys (capacity rule) and coarse pairs
    static_assert(GATHER_THREADS == 4 * 256, "k_gather zeroes the sort's digit counts with a word per thread");
    hipLaunchKernelGGL(k_gather, dim3((unsigned)nb), dim3(GATHER_THREADS), 0, st, bs.dval_a, bs.rec, bs.counts, n,
                       bs.vtab, bs.stab, sat, bs.st_cls, L, n_tiles, bs.rec_s, bs.cc_s, bs.block_sums, bs.block_sums2,
                       bs.rs.hist, bs.rs.tickets);
    hipLaunchKernelGGL(k_scan_pair, dim3(1), dim3(1024), 0, st, bs.block_sums, bs.block_sums2, nb, bs.counts + 1,
                       bs.counts + 2, num_keys, bs.counts + 3, status);
    // 4b: coarse pairs with their payloads, stably sorted by super-tile
    int st_bits = 1;
    while ((int64_t(1) << st_bits) < n_st) ++st_bits;
    // the pair's info rides in the sort key when the super-tile ids leave room
    // (and only while every digit of the sort lies below the packed info:
    // three 6-bit digits of a 17-bit id would reach its lowest bit)
    const bool packed = coarse_packed && st_bits <= 16;
    const bool even = radix_pass_count(st_bits, packed ? 4 : 8, bs.rs.part) % 2 == 0;
    // the super-tile sort's digit counts and tickets were zeroed by k_gather;
    // k_coarse_emit zeroes its first-pass lookback words and counts its digits
    const RadixShape shape = radix_shape(bs.rs, packed ? 4 : 8, st_bits);
    if (radix_prepare_words(bs.rs, cap, packed ? 4 : 8, st_bits) > bs.rs.status_words ||
        shape.passes * shape.radix > 4 * 256)
        return hipErrorInvalidValue;
    if (packed) {
        hipLaunchKernelGGL(k_coarse_emit<true>, dim3((unsigned)nb), dim3(GATHER_THREADS), 0, st, bs.rec_s, bs.cc_s,
                           bs.counts, bs.block_sums2, bs.vtab, bs.stab, sat, bs.st_cls, L, n_tiles, bs.tkey_a,
                           (void *)bs.cpay_a, bs.rs.status, cap, shape, bs.rs.hist);
        if ((err = radix_sort_pairs(bs.tkey_a, reinterpret_cast<uint32_t *>(bs.cpay_a), bs.tkey_b,
                                    reinterpret_cast<uint32_t *>(bs.cpay_b), bs.counts + 3, cap, st_bits, bs.rs, st,
                                    true)) != hipSuccess)
            return err;
    } else {
        hipLaunchKernelGGL(k_coarse_emit<false>, dim3((unsigned)nb), dim3(GATHER_THREADS), 0, st, bs.rec_s, bs.cc_s,
                           bs.counts, bs.block_sums2, bs.vtab, bs.stab, sat, bs.st_cls, L, n_tiles, bs.tkey_a,
                           (void *)bs.cpay_a, bs.rs.status, cap, shape, bs.rs.hist);
        if ((err = radix_sort_pairs_v2(bs.tkey_a, bs.cpay_a, bs.tkey_b, bs.cpay_b, bs.counts + 3, cap, st_bits, bs.rs,
                                       st, true, true)) != hipSuccess)
            return err;
    }
    const uint32_t *sk = even ? bs.tkey_a : bs.tkey_b;
    const void *sv = even ? (const void *)bs.cpay_a : (const void *)bs.cpay_b;
    const uint32_t id_mask = packed ? (1u << ST_ID_BITS) - 1u : 0xFFFFFFFFu;
    hipLaunchKernelGGL(k_ranges, dim3(grid_for(cap, 256 * 16, 8192)), dim3(256), 0, st, sk, id_mask, bs.counts + 3,
                       cap, n_st, bs.st_ranges);
    if (n_st <= 1024) {
        hipLaunchKernelGGL(k_chunk_table<true>, dim3(1), dim3(1024), 0, st, bs.st_ranges, n_st, bs.chunk_off,
                           bs.counts + 4, bs.stab, V, bs.chunk);
    } else {
        hipLaunchKernelGGL(k_chunk_table<false>, dim3(1), dim3(1024), 0, st, bs.st_ranges, n_st, bs.chunk_off,
                           bs.counts + 4, bs.stab, V, bs.chunk);
        hipLaunchKernelGGL(k_chunk_fill, dim3((unsigned)n_st), dim3(256), 0, st, bs.st_ranges, bs.chunk_off, bs.stab,
                           V, bs.chunk);
    }
    // 4c-4e: per-tile counts, their scans (tile ranges), keys at their final positions
    const int pass_blocks = grid_for(bin_max_chunks(cap, n_tiles), 4, 2048);
#define GS_TP(W, PK, KY)                                                                                   \
    hipLaunchKernelGGL((k_tile_pass<W, PK, KY>), dim3(pass_blocks), dim3(256), 0, st, sk, sv, bs.chunk,         \
                       bs.counts, bs.vtab, bs.stab, V, n, tile_level, bs.ccnt, ranges, vals, keys, splats)
    if (packed)
        GS_TP(false, true, false);
    else
        GS_TP(false, false, false);
    hipLaunchKernelGGL(k_col_scan, dim3((unsigned)n_st), dim3(COL_WAVES * 64), 0, st, bs.chunk_off, bs.vtab, bs.stab, V,
                       bs.ccnt, bs.tot);
    if (n_tiles <= TILE_SCAN1_MAX) {
        hipLaunchKernelGGL(k_tile_scan1, dim3(1), dim3(TS1_THREADS), 0, st, bs.tot, n_tiles, bs.counts, ranges);
    } else {
        const int64_t nbt = (n_tiles + SCAN_THREADS * SCAN_ITEMS - 1) / (SCAN_THREADS * SCAN_ITEMS);
        hipLaunchKernelGGL(k_tile_reduce, dim3((unsigned)nbt), dim3(SCAN_THREADS), 0, st, bs.tot, n_tiles, bs.tsum);
        hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, bs.tsum, nullptr, nbt, bs.counts + 5);
        hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)nbt), dim3(SCAN_THREADS), 0, st, bs.tot, n_tiles, bs.tsum,
                           bs.counts, ranges);
    }
    if (packed) {
        if (keys)
            GS_TP(true, true, true);
        else
            GS_TP(true, true, false);
    } else {
        if (keys)
            GS_TP(true, false, true);
        else
            GS_TP(true, false, false);
    }
#undef GS_TP
    return hipGetLastError();
}
