// Tile binning (Section 2.1 "Sorting"; Section 4.2 filtering).
//
// Depth-first construction of the (tile, depth)-sorted key list:
//   1. count:  per (view, point) the number of kept tiles of its rectangle
//              (tile t kept iff its lower level tile_level[t][0] <= the
//              point's quality bound) and the float32 depth bits as a sort
//              key (no tile -> max).  With the level filter the count comes
//              from per-level summed-area tables over the tile grid, O(1)
//              per point whatever its size;
//   2. sort the (view, point) entries by depth (stable radix, 4 passes);
//   3. scan the counts in depth order and emit each entry's tile ids
//      (row-major) at its offset -- the emitted list is in (depth, view,
//      point) order.  Points with small rectangles emit from their own
//      thread; larger rectangles are queued and expanded by one wave each, so
//      a few very large splats cannot serialise the kernel;
//   4. a stable radix sort on the tile id alone (ceil(log2 tiles) bits)
//      then yields (tile, depth, view, point) order;
//   5. tile ranges from the boundaries of the sorted tile ids.
// Sorting by depth first over the points (millions) and by tile over the
// keys (tens of millions) moves far fewer bytes than a 64-bit key sort.
#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr uint32_t HEAVY_KEYS = 32;  // larger rectangles are expanded by a wave

__global__ void k_set_u64(uint64_t *__restrict__ p, uint64_t value) { *p = value; }

__global__ void __launch_bounds__(256)
k_fill_u32(uint32_t *__restrict__ p, uint32_t value, uint64_t count)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        p[i] = value;
}

// Summed-area table of [lower level of tile <= m] over each view's tile grid,
// one table per level m = 1..L: sat[(m-1) * n_tiles + g] counts the tiles
// (x', y') <= (x, y) of g's view.  One workgroup per (view, level).
__global__ void __launch_bounds__(256)
k_level_sat(const gs_camera *__restrict__ cams, int V, int T, int L, int64_t n_tiles,
            const uint8_t *__restrict__ tl, uint32_t *__restrict__ sat)
{
    const int v = blockIdx.x / L, m = blockIdx.x % L + 1;
    int64_t toff = 0;
    for (int u = 0; u < v; ++u) toff += (int64_t)div_up(cams[u].width, T) * div_up(cams[u].height, T);
    const int tx = div_up(cams[v].width, T), ty = div_up(cams[v].height, T);
    uint32_t *s = sat + (int64_t)(m - 1) * n_tiles + toff;
    const uint8_t *lv = tl + 2 * toff;
    for (int y = threadIdx.x; y < ty; y += blockDim.x) {
        uint32_t run = 0;
        for (int x = 0; x < tx; ++x) {
            run += lv[2 * ((int64_t)y * tx + x)] <= m;
            s[(int64_t)y * tx + x] = run;
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < tx; x += blockDim.x) {
        uint32_t run = 0;
        for (int y = 0; y < ty; ++y) {
            run += s[(int64_t)y * tx + x];
            s[(int64_t)y * tx + x] = run;
        }
    }
}

__device__ __forceinline__ uint32_t sat_at(const uint32_t *__restrict__ s, int tiles_x, int x, int y)
{
    return (x < 0 || y < 0) ? 0u : s[(int64_t)y * tiles_x + x];
}

__global__ void __launch_bounds__(256)
k_count(const gs_splat *__restrict__ splats, int n, const gs_camera *__restrict__ cams, int V, int T,
        const uint32_t *__restrict__ sat, int L, int64_t n_tiles, const uint8_t *__restrict__ qbound,
        uint32_t *__restrict__ hits, uint32_t *__restrict__ area, uint32_t *__restrict__ dkey,
        uint32_t *__restrict__ dval, uint32_t *__restrict__ hits_out)
{
    int64_t E = (int64_t)V * n;
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    int v = (int)(e / n);
    int i = (int)(e - (int64_t)v * n);
    int64_t toff = 0;
    for (int u = 0; u < v; ++u) toff += (int64_t)div_up(cams[u].width, T) * div_up(cams[u].height, T);
    int W = cams[v].width, H = cams[v].height;
    const float4 *s4 = reinterpret_cast<const float4 *>(splats + e);
    float4 a = s4[0], c = s4[2];
    int radius = __float_as_int(c.z);
    TileRect r;
    uint32_t cnt = 0, ar = 0;
    if (tile_rect(a.x, a.y, radius, W, H, T, r)) {
        ar = (uint32_t)(r.tx1 - r.tx0 + 1) * (uint32_t)(r.ty1 - r.ty0 + 1);
        if (!sat) {
            cnt = ar;
        } else {
            int m = qbound[i];
            if (m >= 1) {
                m = m < L ? m : L;
                const uint32_t *s = sat + (int64_t)(m - 1) * n_tiles + toff;
                int tx = div_up(W, T);
                cnt = sat_at(s, tx, r.tx1, r.ty1) - sat_at(s, tx, r.tx0 - 1, r.ty1) -
                      sat_at(s, tx, r.tx1, r.ty0 - 1) + sat_at(s, tx, r.tx0 - 1, r.ty0 - 1);
            }
        }
    }
    hits[e] = cnt;
    area[e] = ar;
    if (hits_out) hits_out[e] = cnt;
    dkey[e] = cnt ? __float_as_uint(c.y) : 0xFFFFFFFFu;
    dval[e] = (uint32_t)e;
}

// Scan phase 1: per-block sums of the counts taken in depth order.
__global__ void __launch_bounds__(SCAN_THREADS)
k_scan_reduce(const uint32_t *__restrict__ order, const uint32_t *__restrict__ hits, int64_t E,
              uint64_t *__restrict__ block_sums)
{
    __shared__ uint64_t s[SCAN_THREADS / 64];
    int64_t base = (int64_t)blockIdx.x * (SCAN_THREADS * SCAN_ITEMS);
    uint64_t acc = 0;
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t r = base + (int64_t)j * SCAN_THREADS + threadIdx.x;
        if (r < E) acc += hits[order[r]];
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t tot = 0;
        for (int w = 0; w < SCAN_THREADS / 64; ++w) tot += s[w];
        block_sums[blockIdx.x] = tot;
    }
}

// Scan phase 2: exclusive scan of the block sums (one block), total -> counts[1].
__global__ void __launch_bounds__(1024)
k_scan_blocks(uint64_t *__restrict__ block_sums, int64_t nb, uint64_t *__restrict__ counts,
              uint64_t *__restrict__ num_keys)
{
    __shared__ uint64_t s[1024];
    int t = threadIdx.x;
    int64_t per = (nb + 1023) / 1024;
    int64_t b0 = t * per, b1 = b0 + per < nb ? b0 + per : nb;
    uint64_t local = 0;
    for (int64_t b = b0; b < b1; ++b) local += block_sums[b];
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
        uint64_t x = block_sums[b];
        block_sums[b] = run;
        run += x;
    }
    if (t == 1023) {
        // on overflow nothing downstream reads the (partial) key list: the
        // sort and the ranges see zero keys; num_keys reports what is needed
        uint64_t total = s[1023];
        counts[1] = total <= counts[2] ? total : 0;
        *num_keys = total;
    }
}

struct EntryRect {
    TileRect r;
    int64_t toff;
    int tiles_x;
    int i;
    uint8_t m;
};

__device__ __forceinline__ EntryRect entry_rect(uint32_t e, const gs_splat *__restrict__ splats, int n,
                                                const gs_camera *__restrict__ cams, int T,
                                                const uint8_t *__restrict__ qbound)
{
    EntryRect er;
    int v = (int)(e / (uint32_t)n);
    er.i = (int)(e - (uint32_t)v * (uint32_t)n);
    er.toff = 0;
    for (int u = 0; u < v; ++u) er.toff += (int64_t)div_up(cams[u].width, T) * div_up(cams[u].height, T);
    int W = cams[v].width, H = cams[v].height;
    er.tiles_x = div_up(W, T);
    const float4 *s4 = reinterpret_cast<const float4 *>(splats + e);
    float4 a = s4[0], c = s4[2];
    if (!tile_rect(a.x, a.y, __float_as_int(c.z), W, H, T, er.r)) {
        er.r.tx0 = er.r.ty0 = 0;
        er.r.tx1 = er.r.ty1 = -1;
    }
    er.m = qbound ? qbound[er.i] : (uint8_t)255;
    return er;
}

// Scan phase 3 + emission.  Entries whose rectangle has at most HEAVY_KEYS
// tiles are expanded by their own thread; larger rectangles (whatever the
// level filter keeps of them) are queued for k_emit_heavy, where one wave
// expands one rectangle.
__global__ void __launch_bounds__(SCAN_THREADS)
k_scan_emit(const uint32_t *__restrict__ order, const uint32_t *__restrict__ hits,
            const uint32_t *__restrict__ area, int64_t E, const uint64_t *__restrict__ block_sums,
            const gs_splat *__restrict__ splats, int n, const gs_camera *__restrict__ cams, int V,
            int T, const uint8_t *__restrict__ tl, const uint8_t *__restrict__ qbound, uint64_t cap,
            uint32_t *__restrict__ tkey, uint32_t *__restrict__ tval, uint32_t *__restrict__ heavy_n,
            uint32_t *__restrict__ heavy_e, uint64_t *__restrict__ heavy_off)
{
    __shared__ uint64_t s_w[SCAN_THREADS / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t base = (int64_t)blockIdx.x * (SCAN_THREADS * SCAN_ITEMS);
    uint64_t run = block_sums[blockIdx.x];
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t r = base + (int64_t)j * SCAN_THREADS + threadIdx.x;
        uint32_t e = 0, cnt = 0;
        if (r < E) {
            e = order[r];
            cnt = hits[e];
        }
        // exclusive scan of cnt across the block (in r order)
        uint64_t x = cnt;
        for (int off = 1; off < 64; off <<= 1) {
            uint64_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) s_w[wave] = x;
        __syncthreads();
        uint64_t wpre = 0, tot = 0;
        for (int w = 0; w < SCAN_THREADS / 64; ++w) {
            uint64_t sw = s_w[w];
            if (w < wave) wpre += sw;
            tot += sw;
        }
        __syncthreads();
        const uint64_t off = run + wpre + x - cnt;
        run += tot;
        if (cnt == 0 || off + cnt > cap) continue;
        if (area[e] > HEAVY_KEYS) {
            const uint32_t h = atomicAdd(heavy_n, 1u);
            heavy_e[h] = e;
            heavy_off[h] = off;
            continue;
        }
        const EntryRect er = entry_rect(e, splats, n, cams, T, qbound);
        uint64_t o = off;
        for (int ty = er.r.ty0; ty <= er.r.ty1; ++ty) {
            const int64_t rowt = er.toff + (int64_t)ty * er.tiles_x;
            for (int tx = er.r.tx0; tx <= er.r.tx1; ++tx) {
                const int64_t g = rowt + tx;
                if (tl && !(tl[2 * g] <= er.m)) continue;
                tkey[o] = (uint32_t)g;
                tval[o] = (uint32_t)er.i;
                ++o;
            }
        }
    }
}

// One wave per queued rectangle: 64 tiles at a time in row-major order,
// kept tiles compacted with a ballot so the run stays in order.
__global__ void __launch_bounds__(256)
k_emit_heavy(const uint32_t *__restrict__ heavy_n, const uint32_t *__restrict__ heavy_e,
             const uint64_t *__restrict__ heavy_off, const gs_splat *__restrict__ splats, int n,
             const gs_camera *__restrict__ cams, int T, const uint8_t *__restrict__ tl,
             const uint8_t *__restrict__ qbound, uint32_t *__restrict__ tkey,
             uint32_t *__restrict__ tval)
{
    const int lane = threadIdx.x & 63;
    const uint32_t nh = *heavy_n;
    const uint32_t waves = gridDim.x * (blockDim.x / 64);
    for (uint32_t h = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); h < nh; h += waves) {
        const EntryRect er = entry_rect(heavy_e[h], splats, n, cams, T, qbound);
        const uint64_t off = heavy_off[h];
        const int w = er.r.tx1 - er.r.tx0 + 1;
        const int64_t total = (int64_t)w * (er.r.ty1 - er.r.ty0 + 1);
        uint64_t pos = 0;
        for (int64_t b0 = 0; b0 < total; b0 += 64) {
            const int64_t jj = b0 + lane;
            const bool valid = jj < total;
            int64_t g = 0;
            if (valid)
                g = er.toff + (int64_t)(er.r.ty0 + (int)(jj / w)) * er.tiles_x + er.r.tx0 + (int)(jj % w);
            const bool keep = valid && (!tl || tl[2 * g] <= er.m);
            const uint64_t bal = ballot64(keep);
            if (keep) {
                const uint64_t o = off + pos + (uint32_t)__popcll(bal & lanemask_lt());
                tkey[o] = (uint32_t)g;
                tval[o] = (uint32_t)er.i;
            }
            pos += (uint32_t)__popcll(bal);
        }
    }
}

__global__ void __launch_bounds__(256)
k_ranges(const uint32_t *__restrict__ tkey, const uint64_t *__restrict__ counts, uint64_t cap,
         int64_t n_tiles, uint32_t *__restrict__ ranges)
{
    uint64_t count = counts[1];
    count = count < cap ? count : cap;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride) {
        uint32_t t = tkey[k];
        if (t >= n_tiles) continue;
        if (k == 0 || tkey[k - 1] != t) ranges[2 * (uint64_t)t] = (uint32_t)k;
        if (k + 1 == count || tkey[k + 1] != t) ranges[2 * (uint64_t)t + 1] = (uint32_t)(k + 1);
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

hipError_t launch_bin_sort(const gs_splat *splats, int n, const gs_camera *cams_dev, int V,
                           int64_t n_tiles, int tile_bits, int T, const uint8_t *tile_level,
                           const uint8_t *qbound, int n_levels, uint32_t *vals, uint64_t *keys,
                           uint64_t cap, uint32_t *ranges, uint32_t *hits_out, uint64_t *num_keys,
                           const BinScratch &bs, hipStream_t st)
{
    int64_t E = (int64_t)V * n;
    hipError_t err;
    uint64_t hostE = (uint64_t)E;
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, bs.counts, hostE);
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, bs.counts + 2, cap);
    if ((err = launch_fill_u32(ranges, 0u, 2 * (uint64_t)n_tiles, st)) != hipSuccess) return err;
    if (E == 0) {
        hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, num_keys, (uint64_t)0);
        return hipGetLastError();
    }
    const bool filt = tile_level != nullptr;
    int L = n_levels < 1 ? 1 : (n_levels > 4 ? 4 : n_levels);
    if (filt)
        hipLaunchKernelGGL(k_level_sat, dim3(V * L), dim3(256), 0, st, cams_dev, V, T, L, n_tiles,
                           tile_level, bs.sat);
    hipLaunchKernelGGL(k_count, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, st, splats, n,
                       cams_dev, V, T, filt ? bs.sat : nullptr, L, n_tiles, qbound, bs.hits,
                       bs.area, bs.dkey_a, bs.dval_a, hits_out);
    // depth sort of the entries: 32 bits -> 4 passes, result back in (dkey_a, dval_a)
    if ((err = radix_sort_pairs(bs.dkey_a, bs.dval_a, bs.dkey_b, bs.dval_b, bs.counts, hostE, 32,
                                bs.rs, st)) != hipSuccess)
        return err;
    const uint32_t *order = bs.dval_a;
    int64_t nb = (E + SCAN_THREADS * SCAN_ITEMS - 1) / (SCAN_THREADS * SCAN_ITEMS);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, order, bs.hits, E,
                       bs.block_sums);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, bs.block_sums, nb, bs.counts,
                       num_keys);
    // emission goes to the buffer from which an even/odd number of passes
    // ends in the caller's vals
    int passes = radix_passes(tile_bits);
    uint32_t *ek = bs.tkey_a, *ev = (passes % 2 == 0) ? vals : bs.tval_b;
    uint32_t *ok = bs.tkey_b, *ov = (passes % 2 == 0) ? bs.tval_b : vals;
    if ((err = launch_fill_u32(bs.heavy_n, 0u, 1, st)) != hipSuccess) return err;
    hipLaunchKernelGGL(k_scan_emit, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, order, bs.hits,
                       bs.area, E, bs.block_sums, splats, n, cams_dev, V, T, tile_level, qbound, cap, ek,
                       ev, bs.heavy_n, bs.heavy_e, bs.heavy_off);
    hipLaunchKernelGGL(k_emit_heavy, dim3(2048), dim3(256), 0, st, bs.heavy_n, bs.heavy_e, bs.heavy_off,
                       splats, n, cams_dev, T, tile_level, qbound, ek, ev);
    if ((err = radix_sort_pairs(ek, ev, ok, ov, bs.counts + 1, cap, tile_bits, bs.rs, st)) !=
        hipSuccess)
        return err;
    const uint32_t *sorted_t = (passes % 2 == 0) ? ek : ok;
    int rg = grid_for(cap, 256 * 8, 8192);
    hipLaunchKernelGGL(k_ranges, dim3(rg), dim3(256), 0, st, sorted_t, bs.counts, cap, n_tiles, ranges);
    if (keys)
        hipLaunchKernelGGL(k_keys64, dim3(rg), dim3(256), 0, st, sorted_t, vals, bs.counts, cap, splats,
                           n, cams_dev, V, T, n_tiles, keys);
    return hipGetLastError();
}
