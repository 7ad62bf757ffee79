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
//   4. gather the entry records in depth order, scan their counts and
//      rectangle areas, and emit each entry's kept tile ids (row-major) at its
//      offset -- the emitted list is in (depth, view, point) order.  The
//      emission is load-balanced over the concatenated rectangles (fixed
//      slices of tiles per wave, coalesced stores), so one huge rectangle
//      costs no more than many small ones;
//   5. a stable radix sort on the tile id alone (ceil(log2 tiles) bits)
//      then yields (tile, depth, view, point) order;
//   6. tile ranges from the boundaries of the sorted tile ids.
// Sorting by depth first over the points (millions) and by tile over the
// keys (tens of millions) moves far fewer bytes than a 64-bit key sort.
#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr int SAT_LDS_TILES = 16384;      // views up to this many tiles build their tables in LDS (64 KB)
constexpr uint64_t SLICE_MIN = 1024;       // rectangle tiles per emission task (at least)
constexpr uint64_t MAX_SLICES = BIN_MAX_SLICES;  // emission tasks (at most)

__global__ void k_set_u64(uint64_t *__restrict__ p, uint64_t value) { *p = value; }

__global__ void __launch_bounds__(256)
k_fill_u32(uint32_t *__restrict__ p, uint32_t value, uint64_t count)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        p[i] = value;
}

__device__ __forceinline__ int64_t view_tile_off(const gs_camera *__restrict__ cams, int v, int T)
{
    int64_t toff = 0;
    for (int u = 0; u < v; ++u) toff += (int64_t)div_up(cams[u].width, T) * div_up(cams[u].height, T);
    return toff;
}

// Tile offset and grid width of every view: vtab[v] = {first tile, tiles_x}.
__global__ void __launch_bounds__(256)
k_view_table(const gs_camera *__restrict__ cams, int V, int T, int64_t *__restrict__ vtab)
{
    if (threadIdx.x != 0) return;
    int64_t toff = 0;
    for (int v = 0; v < V; ++v) {
        const int tx = div_up(cams[v].width, T), ty = div_up(cams[v].height, T);
        vtab[2 * v] = toff;
        vtab[2 * v + 1] = tx;
        toff += (int64_t)tx * ty;
    }
}

// Summed-area table of [lower level of tile <= m] over each view's tile grid,
// one table per level m = 1..L: sat[(m-1) * n_tiles + g] counts the tiles
// (x', y') <= (x, y) of g's view.  One workgroup per (view, level), built in
// LDS (dynamic size) when the view's grid fits, else in place in memory:
// row sums (a thread per row), then column sums (a thread per column).
// Also the bounding box of those tiles, bbox[(v * L + m - 1) * 4 +
// {x0, y0, x1, y1}] (x0 > x1 when there are none).
__global__ void __launch_bounds__(256)
k_level_sat(const gs_camera *__restrict__ cams, int V, int T, int L, int64_t n_tiles,
            const uint8_t *__restrict__ tl, uint32_t *__restrict__ sat, int32_t *__restrict__ bbox, int use_lds)
{
    extern __shared__ uint32_t s_sat[];
    __shared__ int s_box[4];
    const int v = blockIdx.x / L, m = blockIdx.x % L + 1;
    const int64_t toff = view_tile_off(cams, v, T);
    const int tx = div_up(cams[v].width, T), ty = div_up(cams[v].height, T);
    if (threadIdx.x == 0) {
        s_box[0] = tx;
        s_box[1] = ty;
        s_box[2] = -1;
        s_box[3] = -1;
    }
    __syncthreads();
    uint32_t *g = sat + (int64_t)(m - 1) * n_tiles + toff;
    uint32_t *s = use_lds ? s_sat : g;
    const uint8_t *lv = tl + 2 * toff;
    for (int y = threadIdx.x; y < ty; y += blockDim.x) {
        uint32_t run = 0;
        int xl = tx, xr = -1;
        for (int x = 0; x < tx; ++x) {
            const bool kept = lv[2 * ((int64_t)y * tx + x)] <= m;
            run += kept;
            if (kept) {
                xl = x < xl ? x : xl;
                xr = x;
            }
            s[(int64_t)y * tx + x] = run;
        }
        if (xr >= 0) {
            atomicMin(&s_box[0], xl);
            atomicMin(&s_box[1], y);
            atomicMax(&s_box[2], xr);
            atomicMax(&s_box[3], y);
        }
    }
    __syncthreads();
    if (threadIdx.x < 4) bbox[((int64_t)v * L + m - 1) * 4 + threadIdx.x] = s_box[threadIdx.x];
    for (int x = threadIdx.x; x < tx; x += blockDim.x) {
        uint32_t run = 0;
        for (int y = 0; y < ty; ++y) {
            run += s[(int64_t)y * tx + x];
            s[(int64_t)y * tx + x] = run;
        }
    }
    if (use_lds) {
        __syncthreads();
        for (int64_t k = threadIdx.x; k < (int64_t)tx * ty; k += blockDim.x) g[k] = s[k];
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

// 1. per-entry counts; culled / empty entries get 0.  Also the float32 depth
//    bits (dkey_all), a per-block count of entries with keys and, for those
//    entries, rec[e] = {x0 | y0 << 16, x1 | y1 << 16, count, quality bound}
//    with the rectangle clipped to the bounding box of the tiles its level
//    keeps (the kept tiles and their row-major order are unchanged).
__global__ void __launch_bounds__(SCAN_THREADS)
k_count(const gs_splat *__restrict__ splats, int n, const gs_camera *__restrict__ cams, int V, int T,
        const int64_t *__restrict__ vtab, const uint32_t *__restrict__ sat, const int32_t *__restrict__ bbox, int L, int64_t n_tiles,
        const uint8_t *__restrict__ qbound, uint32_t *__restrict__ hits, uint4 *__restrict__ rec,
        uint32_t *__restrict__ dkey_all, uint32_t *__restrict__ hits_out, uint32_t *__restrict__ block_vis)
{
    __shared__ uint32_t s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const int64_t E = (int64_t)V * n;
    const int64_t base = (int64_t)blockIdx.x * (SCAN_THREADS * SCAN_ITEMS);
    uint32_t vis = 0;
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const int64_t e = base + (int64_t)j * SCAN_THREADS + threadIdx.x;
        if (e >= E) break;
        const int v = (int)(e / n);
        const int i = (int)(e - (int64_t)v * n);
        const int W = cams[v].width, H = cams[v].height;
        const float4 *s4 = reinterpret_cast<const float4 *>(splats + e);
        const float4 a = s4[0], c = s4[2];
        TileRect r;
        uint32_t cnt = 0;
        int m = 255;
        if (tile_rect(a.x, a.y, __float_as_int(c.z), W, H, T, r)) {
            if (!sat) {
                cnt = (uint32_t)(r.tx1 - r.tx0 + 1) * (uint32_t)(r.ty1 - r.ty0 + 1);
            } else {
                m = qbound[i];
                if (m >= 1) {
                    // kept tiles lie in the level's bounding box: clip to it
                    const int ml = m < L ? m : L;
                    const int4 b = reinterpret_cast<const int4 *>(bbox)[(int64_t)v * L + ml - 1];
                    r.tx0 = r.tx0 > b.x ? r.tx0 : b.x;
                    r.ty0 = r.ty0 > b.y ? r.ty0 : b.y;
                    r.tx1 = r.tx1 < b.z ? r.tx1 : b.z;
                    r.ty1 = r.ty1 < b.w ? r.ty1 : b.w;
                    if (r.tx0 <= r.tx1 && r.ty0 <= r.ty1) {
                        const uint32_t *s = sat + (int64_t)(ml - 1) * n_tiles + vtab[2 * v];
                        cnt = sat_rect(s, (int)vtab[2 * v + 1], r.tx0, r.tx1, r.ty0, r.ty1);
                    }
                }
            }
        }
        hits[e] = cnt;
        if (cnt)
            rec[e] = make_uint4((uint32_t)r.tx0 | ((uint32_t)r.ty0 << 16), (uint32_t)r.tx1 | ((uint32_t)r.ty1 << 16),
                                cnt, (uint32_t)m);
        if (hits_out) hits_out[e] = cnt;
        dkey_all[e] = __float_as_uint(c.y);
        vis += cnt > 0;
    }
    for (int off = 32; off > 0; off >>= 1) vis += __shfl_xor(vis, off);
    if ((threadIdx.x & 63) == 0) atomicAdd(&s_cnt, vis);
    __syncthreads();
    if (threadIdx.x == 0) block_vis[blockIdx.x] = s_cnt;
}

// Exclusive scan of nb block values in place (one workgroup); the total goes
// to *total (and, if given, the keys-needed output with the capacity rule).
__global__ void __launch_bounds__(1024)
k_scan_blocks(uint64_t *__restrict__ block_sums, const uint32_t *__restrict__ block_u32, int64_t nb,
              uint64_t *__restrict__ total, const uint64_t *__restrict__ cap_ptr,
              uint64_t *__restrict__ num_keys)
{
    __shared__ uint64_t s[1024];
    int t = threadIdx.x;
    int64_t per = (nb + 1023) / 1024;
    int64_t b0 = t * per, b1 = b0 + per < nb ? b0 + per : nb;
    uint64_t local = 0;
    for (int64_t b = b0; b < b1; ++b) local += block_u32 ? block_u32[b] : block_sums[b];
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
    if (t == 1023) {
        uint64_t tot = s[1023];
        if (num_keys) {
            // on overflow nothing downstream reads the (partial) key list: the
            // sort and the ranges see zero keys; num_keys reports what is needed
            *total = tot <= *cap_ptr ? tot : 0;
            *num_keys = tot;
        } else {
            *total = tot;
        }
    }
}

// 2. stable compaction of the entries with keys, counting depth digits.
__global__ void __launch_bounds__(SCAN_THREADS)
k_compact(const uint32_t *__restrict__ hits, const uint32_t *__restrict__ dkey_all, int64_t E,
          const uint64_t *__restrict__ block_off, uint32_t *__restrict__ dkey,
          uint32_t *__restrict__ dval, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t s_w[SCAN_THREADS / 64];
    __shared__ uint32_t s_h[4][256];
    for (int q = threadIdx.x; q < 4 * 256; q += SCAN_THREADS) (&s_h[0][0])[q] = 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * (SCAN_THREADS * SCAN_ITEMS);
    uint64_t run = block_off[blockIdx.x];
    __syncthreads();
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const int64_t e = base + (int64_t)j * SCAN_THREADS + threadIdx.x;
        const bool vis = e < E && hits[e] > 0;
        const uint64_t bal = ballot64(vis);
        if (lane == 0) s_w[wave] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t wpre = 0, tot = 0;
        for (int w = 0; w < SCAN_THREADS / 64; ++w) {
            const uint32_t c = s_w[w];
            if (w < wave) wpre += c;
            tot += c;
        }
        if (vis) {
            const uint64_t pos = run + wpre + (uint32_t)__popcll(bal & lanemask_lt());
            const uint32_t k = dkey_all[e];
            dkey[pos] = k;
            dval[pos] = (uint32_t)e;
#pragma unroll
            for (int p = 0; p < 4; ++p) atomicAdd(&s_h[p][(k >> (8 * p)) & 255u], 1u);
        }
        run += tot;
        __syncthreads();
    }
    for (int q = threadIdx.x; q < 4 * 256; q += SCAN_THREADS) {
        const uint32_t c = (&s_h[0][0])[q];
        if (c) atomicAdd(&hist[q], c);
    }
}

// Depth-ordered entry record: x = first tile id of the rectangle,
// y = w | h << 14 | (x0 == 0) << 28 | (y0 == 0) << 29, z = point index,
// w = tiles_x << 8 | quality bound.
struct SortedRec {
    uint32_t gid0, w, h, tiles_x, m, i;
    bool x0_zero, y0_zero;
};

__device__ __forceinline__ SortedRec unpack_rec(uint4 q)
{
    SortedRec r;
    r.gid0 = q.x;
    r.w = q.y & 0x3fffu;
    r.h = (q.y >> 14) & 0x3fffu;
    r.x0_zero = (q.y >> 28) & 1u;
    r.y0_zero = (q.y >> 29) & 1u;
    r.i = q.z;
    r.tiles_x = q.w >> 8;
    r.m = q.w & 255u;
    return r;
}

// 4a. gather the records in depth order and sum counts and areas per block.
__global__ void __launch_bounds__(SCAN_THREADS)
k_gather(const uint32_t *__restrict__ order, const uint4 *__restrict__ rec, const uint64_t *__restrict__ d_count,
         int n, const int64_t *__restrict__ vtab, uint4 *__restrict__ rec_s, uint32_t *__restrict__ hits_s,
         uint64_t *__restrict__ bsum_h, uint64_t *__restrict__ bsum_a)
{
    __shared__ uint64_t s_h[SCAN_THREADS / 64], s_a[SCAN_THREADS / 64];
    const uint64_t E = *d_count;
    const int64_t base = (int64_t)blockIdx.x * (SCAN_THREADS * SCAN_ITEMS);
    uint64_t acc_h = 0, acc_a = 0;
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const int64_t r = base + (int64_t)j * SCAN_THREADS + threadIdx.x;
        if ((uint64_t)r >= E) break;
        const uint32_t e = order[r];
        const uint4 q = rec[e];
        const uint32_t v = e / (uint32_t)n;
        const uint32_t i = e - v * (uint32_t)n;
        const uint32_t x0 = q.x & 0xffffu, y0 = q.x >> 16, x1 = q.y & 0xffffu, y1 = q.y >> 16;
        const uint32_t w = x1 - x0 + 1, h = y1 - y0 + 1;
        const int64_t tx = vtab[2 * v + 1];
        const uint32_t gid0 = (uint32_t)(vtab[2 * v] + (int64_t)y0 * tx + x0);
        rec_s[r] = make_uint4(gid0, w | (h << 14) | ((uint32_t)(x0 == 0) << 28) | ((uint32_t)(y0 == 0) << 29), i,
                              ((uint32_t)tx << 8) | q.w);
        hits_s[r] = q.z;
        acc_h += q.z;
        acc_a += (uint64_t)w * h;
    }
    for (int off = 32; off > 0; off >>= 1) {
        acc_h += __shfl_xor(acc_h, off);
        acc_a += __shfl_xor(acc_a, off);
    }
    if ((threadIdx.x & 63) == 0) {
        s_h[threadIdx.x >> 6] = acc_h;
        s_a[threadIdx.x >> 6] = acc_a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t th = 0, ta = 0;
        for (int w = 0; w < SCAN_THREADS / 64; ++w) {
            th += s_h[w];
            ta += s_a[w];
        }
        bsum_h[blockIdx.x] = th;
        bsum_a[blockIdx.x] = ta;
    }
}

__device__ __forceinline__ uint64_t slice_len(uint64_t area_total)
{
    uint64_t s = (area_total + MAX_SLICES - 1) / MAX_SLICES;
    s = (s + 63) & ~uint64_t(63);
    return s > SLICE_MIN ? s : SLICE_MIN;
}

// 4b. scan down-sweep: key offset and area offset of every sorted entry, and
// the entry in which each emission slice of the area starts.
__global__ void __launch_bounds__(SCAN_THREADS)
k_scan_down(const uint4 *__restrict__ rec_s, const uint32_t *__restrict__ hits_s,
            const uint64_t *__restrict__ counts, const uint64_t *__restrict__ boff_h,
            const uint64_t *__restrict__ boff_a, uint64_t *__restrict__ hpre, uint64_t *__restrict__ apre,
            uint32_t *__restrict__ slice)
{
    __shared__ uint64_t s_h[SCAN_THREADS / 64], s_a[SCAN_THREADS / 64];
    const uint64_t E = counts[0];
    const uint64_t S = slice_len(counts[3]);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * (SCAN_THREADS * SCAN_ITEMS);
    if ((uint64_t)base >= E) return;
    uint64_t run_h = boff_h[blockIdx.x], run_a = boff_a[blockIdx.x];
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const int64_t r = base + (int64_t)j * SCAN_THREADS + threadIdx.x;
        const bool ok = (uint64_t)r < E;
        uint64_t ch = 0, ca = 0;
        if (ok) {
            const uint32_t y = rec_s[r].y;
            ch = hits_s[r];
            ca = (uint64_t)(y & 0x3fffu) * ((y >> 14) & 0x3fffu);
        }
        uint64_t xh = ch, xa = ca;
        for (int off = 1; off < 64; off <<= 1) {
            const uint64_t yh = __shfl_up(xh, off), ya = __shfl_up(xa, off);
            if (lane >= off) {
                xh += yh;
                xa += ya;
            }
        }
        if (lane == 63) {
            s_h[wave] = xh;
            s_a[wave] = xa;
        }
        __syncthreads();
        uint64_t ph = 0, pa = 0, th = 0, ta = 0;
        for (int w = 0; w < SCAN_THREADS / 64; ++w) {
            const uint64_t vh = s_h[w], va = s_a[w];
            if (w < wave) {
                ph += vh;
                pa += va;
            }
            th += vh;
            ta += va;
        }
        __syncthreads();
        if (ok) {
            const uint64_t a0 = run_a + pa + xa - ca;
            hpre[r] = run_h + ph + xh - ch;
            apre[r] = a0;
            for (uint64_t k = (a0 + S - 1) / S; k * S < a0 + ca; ++k) slice[k] = (uint32_t)r;
        }
        run_h += th;
        run_a += ta;
    }
}

// Value of a level summed-area table at (x0 + dx, y0 + dy) of a rectangle.
__device__ __forceinline__ uint32_t sat_rel(const uint32_t *__restrict__ s, const SortedRec &q, int dx, int dy)
{
    if ((dx < 0 && q.x0_zero) || (dy < 0 && q.y0_zero)) return 0u;
    return s[(int64_t)q.gid0 + (int64_t)dy * q.tiles_x + dx];
}

__device__ __forceinline__ uint32_t sat_rel_rect(const uint32_t *__restrict__ s, const SortedRec &q, int dx0,
                                                 int dx1, int dy0, int dy1)
{
    return sat_rel(s, q, dx1, dy1) - sat_rel(s, q, dx0 - 1, dy1) - sat_rel(s, q, dx1, dy0 - 1) +
           sat_rel(s, q, dx0 - 1, dy0 - 1);
}

// Inclusive max-scan over the 64 lanes of a wave (values >= 0): row
// shifts within each row of 16 lanes, then row broadcasts across rows.
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t x)
{
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true));  // row_shr:1
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true));  // row_shr:2
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true));  // row_shr:4
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true));  // row_shr:8
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false));  // row_bcast:15
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return x;
}

// floor(l / w) and l mod w for l < w * 2^14, w >= 1 (reciprocal estimate,
// one correction step: the quotient is below 2^14).
__device__ __forceinline__ void divmod_small(uint32_t l, uint32_t w, uint32_t &q, uint32_t &rem)
{
    uint32_t qq = (uint32_t)((float)l * __builtin_amdgcn_rcpf((float)w));
    int32_t rr = (int32_t)(l - qq * w);
    if (rr < 0) {
        --qq;
        rr += (int32_t)w;
    } else if (rr >= (int32_t)w) {
        ++qq;
        rr -= (int32_t)w;
    }
    q = qq;
    rem = (uint32_t)rr;
}

// 4c. load-balanced emission.  The rectangles of the depth-sorted entries,
// concatenated in row-major order, form one sequence of (entry, tile) items
// whose kept tiles are exactly the key list in order.  Each wave takes slices
// of that sequence, 64 items per step: an entry that starts inside the step
// marks its first item in a wave-private LDS row, a max-scan over the lanes
// hands every item its entry, the tile level is tested, and kept keys are
// compacted with a ballot, so every store is coalesced.
__global__ void __launch_bounds__(256)
k_emit(const uint4 *__restrict__ rec_s, const uint64_t *__restrict__ hpre, const uint64_t *__restrict__ apre,
       const uint32_t *__restrict__ slice, const uint64_t *__restrict__ counts, const uint8_t *__restrict__ tl,
       const uint32_t *__restrict__ sat, int L, int64_t n_tiles, uint64_t cap, uint32_t *__restrict__ tkey,
       uint32_t *__restrict__ tval)
{
    __shared__ uint32_t s_mark[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    s_mark[wave][lane] = 0;
    wave_lds_sync();
    const uint64_t E = counts[0], A = counts[3];
    if (counts[1] == 0 || E == 0) return;  // no keys, or more than the capacity
    const uint64_t S = slice_len(A);
    const uint64_t n_slices = (A + S - 1) / S;
    const uint64_t lt = lanemask_lt();
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
    for (uint64_t sl = (uint64_t)blockIdx.x * (blockDim.x / 64) + wave; sl < n_slices; sl += waves) {
        const uint64_t a_beg = sl * S;
        const uint64_t a_end = a_beg + S < A ? a_beg + S : A;
        uint64_t r = slice[sl];
        uint32_t base0 = (uint32_t)(a_beg - apre[r]);  // items of entry r before the step
        uint64_t o = hpre[r];
        {
            const SortedRec q = unpack_rec(rec_s[r]);
            if (!tl) {
                o += base0;
            } else {
                uint32_t ly, lx;
                divmod_small(base0, q.w, ly, lx);
                const uint32_t ml = q.m < (uint32_t)L ? q.m : (uint32_t)L;
                const uint32_t *s = sat + (int64_t)(ml - 1) * n_tiles;
                if (ly) o += sat_rel_rect(s, q, 0, (int)q.w - 1, 0, (int)ly - 1);
                if (lx) o += sat_rel_rect(s, q, 0, (int)lx - 1, (int)ly, (int)ly);
            }
        }
        for (uint64_t c0 = a_beg; c0 < a_end; c0 += 64) {
            // entries r+1 .. r+63 that start inside this step mark their first item
            const uint64_t rj = r + lane;
            if (lane > 0 && rj < E) {
                const uint64_t d = apre[rj] - c0;
                if (d < 64) s_mark[wave][d] = ((uint32_t)lane << 6) | (uint32_t)d;
            }
            wave_lds_sync();
            const uint32_t mark = s_mark[wave][lane];
            wave_lds_sync();
            s_mark[wave][lane] = 0;
            const uint32_t km = wave_incl_max(mark);
            uint32_t k = km >> 6;
            const uint32_t l = k == 0 ? base0 + (uint32_t)lane : (uint32_t)lane - (km & 63u);
            uint64_t re = r + k;
            re = re < E ? re : E - 1;
            const bool valid = c0 + lane < a_end;
            const SortedRec q = unpack_rec(rec_s[re]);
            uint32_t ly, lx;
            divmod_small(l, q.w, ly, lx);
            const uint32_t gid = q.gid0 + ly * q.tiles_x + lx;
            const bool keep = valid && (!tl || (gid < (uint64_t)n_tiles && tl[2 * (uint64_t)gid] <= q.m));
            const uint64_t bal = ballot64(keep);
            if (keep) {
                const uint64_t pos = o + (uint32_t)__popcll(bal & lt);
                if (pos < cap) {
                    tkey[pos] = gid;
                    tval[pos] = q.i;
                }
            }
            o += (uint32_t)__popcll(bal);
            // the next step starts one item after lane 63's
            const uint32_t k63 = __builtin_amdgcn_readlane(k, 63);
            const uint32_t l63 = __builtin_amdgcn_readlane(l, 63);
            const uint32_t area63 = __builtin_amdgcn_readlane(q.w * q.h, 63);
            if (l63 + 1 < area63) {
                r += k63;
                base0 = l63 + 1;
            } else {
                r += k63 + 1;
                base0 = 0;
            }
            wave_lds_sync();
        }
    }
}

// 6. tile ranges: four sorted ids per thread; a boundary between k - 1 and k
// closes one tile's run and opens the next.
__global__ void __launch_bounds__(256)
k_ranges(const uint32_t *__restrict__ tkey, const uint64_t *__restrict__ counts, uint64_t cap,
         int64_t n_tiles, uint32_t *__restrict__ ranges)
{
    uint64_t count = counts[1];
    count = count < cap ? count : cap;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * 4;
    for (uint64_t k0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; k0 < count; k0 += stride) {
        uint32_t t[5];
        t[0] = k0 == 0 ? 0xFFFFFFFFu : tkey[k0 - 1];
        if (k0 + 4 <= count) {
            const uint4 q = *reinterpret_cast<const uint4 *>(tkey + k0);
            t[1] = q.x; t[2] = q.y; t[3] = q.z; t[4] = q.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) t[j + 1] = k0 + j < count ? tkey[k0 + j] : 0xFFFFFFFFu;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t k = k0 + j;
            if (k >= count) break;
            if (t[j + 1] != t[j]) {
                if (t[j + 1] < n_tiles) ranges[2 * (uint64_t)t[j + 1]] = (uint32_t)k;
                if (k > 0 && t[j] < n_tiles) ranges[2 * (uint64_t)t[j] + 1] = (uint32_t)k;
            }
        }
        if (k0 + 4 >= count) {
            const uint32_t last = t[count - k0];
            if (last < n_tiles) ranges[2 * (uint64_t)last + 1] = (uint32_t)count;
        }
    }
}

__global__ void __launch_bounds__(256)
k_keys64(const uint32_t *__restrict__ tkey, const uint32_t *__restrict__ vals,
         const uint64_t *__restrict__ counts, uint64_t cap, const gs_splat *__restrict__ splats,
         int n, const gs_camera *__restrict__ cams, int V, int T, int64_t n_tiles,
         uint64_t *__restrict__ keys)
{
    uint64_t count = counts[1];
    count = count < cap ? count : cap;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride) {
        uint32_t t = tkey[k];
        if (t >= n_tiles) continue;
        ViewInfo vi = view_of_tile(cams, V, T, t);
        float d = splats[(int64_t)vi.v * n + vals[k]].depth;
        keys[k] = ((uint64_t)t << 32) | __float_as_uint(d);
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

hipError_t launch_bin_sort(const gs_splat *splats, int n, const gs_camera *cams_dev,
                           const gs_camera *cams_host, int V, int64_t n_tiles, int tile_bits, int T,
                           const uint8_t *tile_level, const uint8_t *qbound, int n_levels,
                           uint32_t *vals, uint64_t *keys, uint64_t cap, uint32_t *ranges,
                           uint32_t *hits_out, uint64_t *num_keys, const BinScratch &bs,
                           hipStream_t st)
{
    const int64_t E = (int64_t)V * n;
    hipError_t err;
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, bs.counts + 2, cap);
    if ((err = launch_fill_u32(ranges, 0u, 2 * (uint64_t)n_tiles, st)) != hipSuccess) return err;
    if (E == 0) {
        hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, num_keys, (uint64_t)0);
        return hipGetLastError();
    }
    const bool filt = tile_level != nullptr;
    const int L = n_levels < 1 ? 1 : (n_levels > 4 ? 4 : n_levels);
    hipLaunchKernelGGL(k_view_table, dim3(1), dim3(64), 0, st, cams_dev, V, T, bs.vtab);
    if (filt) {
        int max_view_tiles = 0;
        for (int v = 0; v < V; ++v) {
            int t = ((cams_host[v].width + T - 1) / T) * ((cams_host[v].height + T - 1) / T);
            max_view_tiles = t > max_view_tiles ? t : max_view_tiles;
        }
        const int lds = max_view_tiles <= SAT_LDS_TILES;
        hipLaunchKernelGGL(k_level_sat, dim3(V * L), dim3(256), lds ? 4 * max_view_tiles : 0, st, cams_dev,
                           V, T, L, n_tiles, tile_level, bs.sat, bs.bbox, lds);
    }
    const int64_t nb = (E + SCAN_THREADS * SCAN_ITEMS - 1) / (SCAN_THREADS * SCAN_ITEMS);
    // 1-2: counts, then stable compaction of entries with keys (depth digits counted)
    hipLaunchKernelGGL(k_count, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, splats, n, cams_dev, V, T, bs.vtab,
                       filt ? bs.sat : nullptr, bs.bbox, L, n_tiles, qbound, bs.hits, bs.rec, bs.dkey_b, hits_out,
                       bs.block_vis);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, bs.block_sums, bs.block_vis, nb, bs.counts,
                       nullptr, nullptr);
    if ((err = launch_fill_u32(bs.rs.hist, 0u, 4 * 256, st)) != hipSuccess) return err;
    hipLaunchKernelGGL(k_compact, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, bs.hits, bs.dkey_b, E,
                       bs.block_sums, bs.dkey_a, bs.dval_a, bs.rs.hist);
    // 3: depth sort of the entries with keys (4 x 8-bit passes), result back in (dkey_a, dval_a)
    if ((err = radix_sort_pairs(bs.dkey_a, bs.dval_a, bs.dkey_b, bs.dval_b, bs.counts, (uint64_t)E, 32, bs.rs, st,
                                true)) != hipSuccess)
        return err;
    // 4: records in depth order, scans of counts and areas, emission
    hipLaunchKernelGGL(k_gather, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, bs.dval_a, bs.rec, bs.counts, n,
                       bs.vtab, bs.rec_s, bs.hits_s, bs.block_sums, bs.block_sums2);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, bs.block_sums, nullptr, nb, bs.counts + 1,
                       bs.counts + 2, num_keys);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, bs.block_sums2, nullptr, nb, bs.counts + 3,
                       nullptr, nullptr);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, bs.rec_s, bs.hits_s, bs.counts,
                       bs.block_sums, bs.block_sums2, bs.hpre, bs.apre, bs.slice);
    const int passes = radix_passes(tile_bits);
    // emission goes to the buffer from which an even/odd number of passes
    // ends in the caller's vals
    uint32_t *ek = bs.tkey_a, *ev = (passes % 2 == 0) ? vals : bs.tval_b;
    uint32_t *ok = bs.tkey_b, *ov = (passes % 2 == 0) ? bs.tval_b : vals;
    hipLaunchKernelGGL(k_emit, dim3(2048), dim3(256), 0, st, bs.rec_s, bs.hpre, bs.apre, bs.slice, bs.counts,
                       tile_level, filt ? bs.sat : nullptr, L, n_tiles, cap, ek, ev);
    // 5: tile sort
    if ((err = radix_sort_pairs(ek, ev, ok, ov, bs.counts + 1, cap, tile_bits, bs.rs, st, false)) !=
        hipSuccess)
        return err;
    const uint32_t *sorted_t = (passes % 2 == 0) ? ek : ok;
    // 6: ranges
    hipLaunchKernelGGL(k_ranges, dim3(grid_for(cap, 256 * 16, 8192)), dim3(256), 0, st, sorted_t, bs.counts,
                       cap, n_tiles, ranges);
    if (keys)
        hipLaunchKernelGGL(k_keys64, dim3(grid_for(cap, 256 * 8, 8192)), dim3(256), 0, st, sorted_t, vals,
                           bs.counts, cap, splats, n, cams_dev, V, T, n_tiles, keys);
    return hipGetLastError();
}
