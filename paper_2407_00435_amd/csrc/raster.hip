// Per-pixel front-to-back compositing (Eq. 1a), its foveated form
// (Section 4.1 blending, Section 4.2 filtering and multi-versioning) and its
// reverse.
//
// Work decomposition for gfx950: a workgroup per tile; each wave64 owns an
// 8x8 pixel sub-block of the tile and works independently of the others (no
// workgroup barriers).  A wave walks its tile's sorted run 64 entries at a
// time: every lane gathers one splat, tests conservatively whether its
// 3-sigma / 1/255 footprint can reach any pixel of the sub-block, and the
// survivors are compacted in order into the wave's LDS slice.  The lanes then
// composite their pixel against the survivors (LDS broadcast reads) and the
// wave leaves as soon as all 64 of its pixels have saturated.  Skipping a
// splat whose footprint misses the sub-block does not change any result.
#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr float NEG_HALF_LOG2E = -0.5f * GS_LOG2E;
constexpr float LOG2_ALPHA_MIN = -7.9943534368588578f;  // log2(1/255)
constexpr float EXTENT_LOG2 = -4.5f * GS_LOG2E;         // log2 exp(-9/2)

// Forward record of a splat, 48 bytes in LDS:
//   a: mean x, mean y, qa, qb     (log2 of the Gaussian falloff is
//   b: qc, log2 opacity, thr, pos  qa dx^2 + qb dx dy + qc dy^2)
//   c: r, g, b, point id
// A pair (pixel, splat) contributes iff e2 = falloff + log2 opacity >= thr,
// thr = max(log2 opacity + log2 e^-4.5, log2 1/255): that is d^2 <= 9 and
// alpha >= 1/255 at once.
struct FwdRec {
    float4 a, b, c;
};

__device__ __forceinline__ FwdRec make_rec(const float4 s0, const float4 s1, const float4 s2,
                                           uint32_t pos, uint32_t id)
{
    FwdRec r;
    float lop = __log2f(s1.y);
    r.a = make_float4(s0.x, s0.y, NEG_HALF_LOG2E * s0.z, -GS_LOG2E * s0.w);
    r.b = make_float4(NEG_HALF_LOG2E * s1.x, lop, fmaxf(lop + EXTENT_LOG2, LOG2_ALPHA_MIN),
                      __uint_as_float(pos));
    r.c = make_float4(s1.z, s1.w, s2.x, __uint_as_float(id));
    return r;
}

__device__ __forceinline__ FwdRec zero_rec()
{
    FwdRec r;
    r.a = r.b = r.c = make_float4(0.f, 0.f, 0.f, 0.f);
    return r;
}

__device__ __forceinline__ float pair_e2(const float4 &a, const float4 &b, float px, float py)
{
    float dx = px - a.x, dy = py - a.y;
    float u = fmaf(a.z, dx, a.w * dy);
    float w = fmaf(b.x * dy, dy, b.y);
    return fmaf(u, dx, w);
}

// Conservative test: can the splat (conic A, B, C; mean m; extent q <= qmax)
// reach any point of the pixel rectangle [x0, x1] x [y0, y1]?  Minimises
// q(d) = A dx^2 + 2 B dx dy + C dy^2 over the rectangle (continuous), which
// is no larger than the minimum over its pixel centres.
__device__ __forceinline__ bool reaches_rect(float mx, float my, float A, float B, float C,
                                             float qmax, float x0, float x1, float y0, float y1)
{
    if (!(qmax >= 0.0f)) return false;
    if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return true;
    float lx = x0 - mx, hx = x1 - mx, ly = y0 - my, hy = y1 - my;
    float best = 3.0e38f;
    // edges x = const: minimise over dy in [ly, hy]
    float iC = 1.0f / C, iA = 1.0f / A;
    {
        float dx = lx;
        float dy = fminf(hy, fmaxf(ly, -B * dx * iC));
        best = fminf(best, A * dx * dx + 2.0f * B * dx * dy + C * dy * dy);
        dx = hx;
        dy = fminf(hy, fmaxf(ly, -B * dx * iC));
        best = fminf(best, A * dx * dx + 2.0f * B * dx * dy + C * dy * dy);
    }
    {
        float dy = ly;
        float dx = fminf(hx, fmaxf(lx, -B * dy * iA));
        best = fminf(best, A * dx * dx + 2.0f * B * dx * dy + C * dy * dy);
        dy = hy;
        dx = fminf(hx, fmaxf(lx, -B * dy * iA));
        best = fminf(best, A * dx * dx + 2.0f * B * dx * dy + C * dy * dy);
    }
    return best <= qmax;
}

// Largest Mahalanobis q at which a splat of opacity o can still pass both
// cut-offs, with a relative margin that covers float32 rounding.
__device__ __forceinline__ float qmax_of(float opacity)
{
    float qa = 2.0f * __logf(255.0f * opacity);
    float q = fminf(9.0f, qa);
    return q * 1.001f + 1e-3f;
}

// ---------------------------------------------------------------------------
// Optional statistics (STATS): [0] blended pairs, [1] evaluated (pixel,
// splat) pairs, [2] staged records, [3] records kept by the cull.
__device__ __forceinline__ void stats_add(unsigned long long *stats, float blended, float evaluated,
                                          float staged, float kept)
{
    blended = wave_sum(blended);
    evaluated = wave_sum(evaluated);
    if (__lane_id() == 0) {
        atomicAdd(stats + 0, (unsigned long long)blended);
        atomicAdd(stats + 1, (unsigned long long)evaluated);
        atomicAdd(stats + 2, (unsigned long long)staged);
        atomicAdd(stats + 3, (unsigned long long)kept);
    }
}

template <int T, bool DOM, bool STATS>
__global__ void __launch_bounds__(T *T)
k_raster_fwd(const gs_splat *__restrict__ splats, int n, const gs_camera *__restrict__ cams, int V,
             const uint32_t *__restrict__ vals, const uint32_t *__restrict__ ranges, float bg0,
             float bg1, float bg2, float *__restrict__ image, float *__restrict__ final_T,
             uint32_t *__restrict__ n_contrib, uint32_t *__restrict__ dominated,
             unsigned long long *__restrict__ stats)
{
    float st_blend = 0.f, st_eval = 0.f, st_staged = 0.f, st_kept = 0.f;
    constexpr int WAVES = T * T / 64;
    constexpr int SUB = T / 8;
    __shared__ FwdRec s_rec[WAVES][64];
    const int64_t gtile = blockIdx.x;
    const ViewInfo vi = view_of_tile(cams, V, T, gtile);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t lt = gtile - vi.tile_off;
    const int tx = (int)(lt % vi.tiles_x), ty = (int)(lt / vi.tiles_x);
    const int sx0 = tx * T + (wave % SUB) * 8, sy0 = ty * T + (wave / SUB) * 8;
    const int px = sx0 + (lane & 7), py = sy0 + (lane >> 3);
    const bool inside = px < vi.W && py < vi.H;
    const float fpx = (float)px, fpy = (float)py;
    // the sub-block clipped to the image (empty sub-blocks skip all work)
    const float rx0 = (float)sx0, ry0 = (float)sy0;
    const float rx1 = (float)min(sx0 + 7, vi.W - 1), ry1 = (float)min(sy0 + 7, vi.H - 1);
    const uint32_t start = ranges[2 * gtile], end = ranges[2 * gtile + 1];
    const gs_splat *__restrict__ vsp = splats + (int64_t)vi.v * n;

    float Tr = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
    uint32_t last = 0;
    float best = 0.0f;
    int best_id = -1;
    bool done = !inside;

    for (uint32_t c0 = start; c0 < end; c0 += 64) {
        if (ballot64(!done) == 0) break;
        const uint32_t idx = c0 + lane;
        bool keep = false;
        // the record is fully defined on every lane before the cull decision
        FwdRec rec = zero_rec();
        if (idx < end) {
            const uint32_t id = vals[idx];
            const float4 *s4 = reinterpret_cast<const float4 *>(vsp + id);
            const float4 s0 = s4[0], s1 = s4[1], s2 = s4[2];
            rec = make_rec(s0, s1, s2, idx - start + 1, id);
            keep = reaches_rect(s0.x, s0.y, s0.z, s0.w, s1.x, qmax_of(s1.y), rx0, rx1, ry0, ry1);
        }
        const uint64_t m = ballot64(keep);
        if (keep) s_rec[wave][__popcll(m & lanemask_lt())] = rec;
        wave_lds_sync();
        const int cnt = __popcll(m);
        if (STATS) {
            st_staged += (float)min(64u, end - c0);
            st_kept += (float)cnt;
        }
        for (int j = 0; j < cnt; ++j) {
            // branch-free: every lane evaluates, selects take the decisions
            const float4 a = s_rec[wave][j].a, b = s_rec[wave][j].b, c = s_rec[wave][j].c;
            if (STATS) st_eval += done ? 0.0f : 1.0f;
            const float e2 = pair_e2(a, b, fpx, fpy);
            const float alpha = fminf(GS_ALPHA_MAX, fast_exp2(e2));
            const bool use = !done && e2 >= b.z;
            const float Tn = fmaf(-alpha, Tr, Tr);
            const bool stop = use && Tn < GS_T_STOP;
            const bool blend = use && !stop;
            const float w = blend ? alpha * Tr : 0.0f;
            C0 = fmaf(w, c.x, C0);
            C1 = fmaf(w, c.y, C1);
            C2 = fmaf(w, c.z, C2);
            Tr = blend ? Tn : Tr;
            last = blend ? __float_as_uint(b.w) : last;
            done = done || stop;
            if (STATS) st_blend += blend ? 1.0f : 0.0f;
            if (DOM && blend && w > best) {
                best = w;
                best_id = (int)__float_as_uint(c.w);
            }
            if ((j & 7) == 7 && ballot64(!done) == 0) break;
        }
        wave_lds_sync();
    }
    if (inside) {
        const int64_t pix = vi.pix_off + (int64_t)py * vi.W + px;
        const int64_t plane = (int64_t)vi.W * vi.H;
        float *img = image + 3 * vi.pix_off + (int64_t)py * vi.W + px;
        img[0] = fmaf(Tr, bg0, C0);
        img[plane] = fmaf(Tr, bg1, C1);
        img[2 * plane] = fmaf(Tr, bg2, C2);
        final_T[pix] = Tr;
        n_contrib[pix] = last;
        if (DOM && best_id >= 0) atomicAdd(dominated + (int64_t)vi.v * n + best_id, 1u);
    }
    if (STATS) stats_add(stats, st_blend, st_eval, st_staged, st_kept);
}

// ---------------------------------------------------------------------------
// Foveated compositing.  Record: geometry (mean, qa, qb | qc, quality bound,
// unused, unused) and per level (r, g, b, opacity).  Each pixel runs the
// accumulator of its lower level and, if blended, of the next one; level t
// takes a splat only if its quality bound is >= t and uses that level's
// opacity and colour.
constexpr int MAXL = 4;
struct FovRec {
    float4 a, b;
    float4 lv[MAXL];
};

template <int T, bool STATS>
__global__ void __launch_bounds__(T *T)
k_raster_fov(const gs_splat *__restrict__ splats, const float4 *__restrict__ lvl, int n,
             const uint8_t *__restrict__ qbound, int L, const gs_camera *__restrict__ cams, int V,
             const uint32_t *__restrict__ vals, const uint32_t *__restrict__ ranges,
             const uint8_t *__restrict__ pix_level, const float *__restrict__ pix_weight, float bg0,
             float bg1, float bg2, float *__restrict__ image, unsigned long long *__restrict__ stats)
{
    float st_blend = 0.f, st_eval = 0.f, st_staged = 0.f, st_kept = 0.f;
    constexpr int WAVES = T * T / 64;
    constexpr int SUB = T / 8;
    __shared__ FovRec s_rec[WAVES][64];
    const int64_t gtile = blockIdx.x;
    const ViewInfo vi = view_of_tile(cams, V, T, gtile);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t lt = gtile - vi.tile_off;
    const int tx = (int)(lt % vi.tiles_x), ty = (int)(lt / vi.tiles_x);
    const int sx0 = tx * T + (wave % SUB) * 8, sy0 = ty * T + (wave / SUB) * 8;
    const int px = sx0 + (lane & 7), py = sy0 + (lane >> 3);
    const bool inside = px < vi.W && py < vi.H;
    const float fpx = (float)px, fpy = (float)py;
    const float rx0 = (float)sx0, ry0 = (float)sy0;
    const float rx1 = (float)min(sx0 + 7, vi.W - 1), ry1 = (float)min(sy0 + 7, vi.H - 1);
    const uint32_t start = ranges[2 * gtile], end = ranges[2 * gtile + 1];
    const int64_t pix = vi.pix_off + (int64_t)py * vi.W + px;

    int lo = 1;
    float wup = 0.0f;
    if (inside) {
        lo = pix_level[pix];
        wup = pix_weight[pix];
    }
    const bool two = wup > 0.0f;
    // lowest level any pixel of the wave needs: splats bounded below it are skipped
    int wave_lo = inside ? lo : 255;
    for (int off = 32; off > 0; off >>= 1) wave_lo = min(wave_lo, __shfl_xor(wave_lo, off));
    const bool any_two = ballot64(two) != 0;

    float Ta = 1.f, A0 = 0.f, A1 = 0.f, A2 = 0.f;
    float Tb = 1.f, B0 = 0.f, B1 = 0.f, B2 = 0.f;
    bool done_a = !inside, done_b = !inside || !two;
    const int64_t vbase = (int64_t)vi.v * n;

    for (uint32_t c0 = start; c0 < end; c0 += 64) {
        if (ballot64(!(done_a && done_b)) == 0) break;
        const uint32_t idx = c0 + lane;
        bool keep = false;
        // the record is fully defined on every lane before the cull decision
        FovRec rec;
        rec.a = rec.b = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int t = 0; t < MAXL; ++t) rec.lv[t] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (idx < end) {
            const uint32_t id = vals[idx];
            const int m = qbound[id];
            const float4 *s4 = reinterpret_cast<const float4 *>(splats + vbase + id);
            const float4 s0 = s4[0], s1 = s4[1];
            rec.a = make_float4(s0.x, s0.y, NEG_HALF_LOG2E * s0.z, -GS_LOG2E * s0.w);
            rec.b = make_float4(NEG_HALF_LOG2E * s1.x, 0.0f, __int_as_float(m), 0.0f);
            const float4 *lp = lvl + (vbase + id) * L;
#pragma unroll
            for (int t = 0; t < MAXL; ++t)
                if (t < L) rec.lv[t] = lp[t];
            keep = m >= wave_lo &&
                   reaches_rect(s0.x, s0.y, s0.z, s0.w, s1.x, 9.001f, rx0, rx1, ry0, ry1);
        }
        const uint64_t msk = ballot64(keep);
        if (keep) s_rec[wave][__popcll(msk & lanemask_lt())] = rec;
        wave_lds_sync();
        const int cnt = __popcll(msk);
        if (STATS) {
            st_staged += (float)min(64u, end - c0);
            st_kept += (float)cnt;
        }
        for (int j = 0; j < cnt; ++j) {
            // branch-free: every lane evaluates, selects take the decisions
            const float4 a = s_rec[wave][j].a, b = s_rec[wave][j].b;
            if (STATS) st_eval += (done_a && done_b) ? 0.0f : 1.0f;
            const float p2 = pair_e2(a, b, fpx, fpy);  // b.y = 0: falloff only
            const int m = __float_as_int(b.z);
            const float G = fast_exp2(p2);
            const bool incl = p2 >= EXTENT_LOG2;
            {
                const float4 lv = s_rec[wave][j].lv[lo - 1];
                const float alpha = fminf(GS_ALPHA_MAX, lv.w * G);
                const bool use = incl && !done_a && m >= lo && alpha >= GS_ALPHA_MIN;
                const float Tn = fmaf(-alpha, Ta, Ta);
                const bool stop = use && Tn < GS_T_STOP;
                const bool blend = use && !stop;
                const float w = blend ? alpha * Ta : 0.0f;
                A0 = fmaf(w, lv.x, A0);
                A1 = fmaf(w, lv.y, A1);
                A2 = fmaf(w, lv.z, A2);
                Ta = blend ? Tn : Ta;
                done_a = done_a || stop;
                if (STATS) st_blend += blend ? 1.0f : 0.0f;
            }
            if (any_two) {
                const float4 lv = s_rec[wave][j].lv[lo < MAXL ? lo : MAXL - 1];
                const float alpha = fminf(GS_ALPHA_MAX, lv.w * G);
                const bool use = incl && !done_b && m >= lo + 1 && alpha >= GS_ALPHA_MIN;
                const float Tn = fmaf(-alpha, Tb, Tb);
                const bool stop = use && Tn < GS_T_STOP;
                const bool blend = use && !stop;
                const float w = blend ? alpha * Tb : 0.0f;
                B0 = fmaf(w, lv.x, B0);
                B1 = fmaf(w, lv.y, B1);
                B2 = fmaf(w, lv.z, B2);
                Tb = blend ? Tn : Tb;
                done_b = done_b || stop;
                if (STATS) st_blend += blend ? 1.0f : 0.0f;
            }
            if ((j & 7) == 7 && ballot64(!(done_a && done_b)) == 0) break;
        }
        wave_lds_sync();
    }
    if (inside) {
        const int64_t plane = (int64_t)vi.W * vi.H;
        float *img = image + 3 * vi.pix_off + (int64_t)py * vi.W + px;
        float ra = fmaf(Ta, bg0, A0), ga = fmaf(Ta, bg1, A1), ba = fmaf(Ta, bg2, A2);
        if (two) {
            float rb = fmaf(Tb, bg0, B0), gb = fmaf(Tb, bg1, B1), bb = fmaf(Tb, bg2, B2);
            ra = (1.0f - wup) * ra + wup * rb;
            ga = (1.0f - wup) * ga + wup * gb;
            ba = (1.0f - wup) * ba + wup * bb;
        }
        img[0] = ra;
        img[plane] = ga;
        img[2 * plane] = ba;
    }
    if (STATS) stats_add(stats, st_blend, st_eval, st_staged, st_kept);
}

// ---------------------------------------------------------------------------
// Reverse of the forward compositing.  Per pixel, back to front from its last
// blended splat: T_i = T_(i+1) / (1 - alpha_i) starting from final_T, and the
// light behind i (including the background) is accumulated on the way, so
//   dL/dc_i = g alpha_i T_i,  dL/dalpha_i = sum_ch g (c_i T_i - B_i / (1 - alpha_i)).
// The tile's list is walked in chunks of 64 positions by all its waves
// together.  Gradients of one splat are summed over a wave's 64 pixels with
// DPP reductions, then over the tile's waves in LDS, and leave the tile as
// one float atomic per quantity per chunk: the global atomics, not the
// arithmetic, bound this kernel.
struct BwdRec {
    float4 a, b, c;   // forward record (identical decisions)
    float4 raw;       // conic A, B, C, opacity
};

// Sum over the 64 lanes of a wave, complete in lane 63 only: row sums, then
// row broadcasts (lane 15 of row 0 into row 1 and of row 2 into row 3, then
// lane 31 into row 3) -- six DPP adds, no lane reads.
__device__ __forceinline__ float wave_total_63(float x)
{
    x = row_sum16(x);
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x142, 0xA, 0xF, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x143, 0x8, 0xF, false));
    return x;
}

template <int T>
__global__ void __launch_bounds__(T *T)
k_raster_bwd(const gs_splat *__restrict__ splats, int n, const gs_camera *__restrict__ cams, int V,
             const uint32_t *__restrict__ vals, const uint32_t *__restrict__ ranges, float bg0,
             float bg1, float bg2, const float *__restrict__ final_T,
             const uint32_t *__restrict__ n_contrib, const float *__restrict__ dL_dimage,
             gs_splat_grad *__restrict__ grads)
{
    constexpr int WAVES = T * T / 64;
    constexpr int SUB = T / 8;
    constexpr int NG = 9;  // mean x, y, conic A, B, C, opacity, colour r, g, b
    __shared__ BwdRec s_rec[WAVES][64];
    __shared__ float s_grad[NG][64];
    __shared__ uint32_t s_id[64];
    __shared__ uint32_t s_maxnc;
    const int64_t gtile = blockIdx.x;
    const ViewInfo vi = view_of_tile(cams, V, T, gtile);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t lt = gtile - vi.tile_off;
    const int tx = (int)(lt % vi.tiles_x), ty = (int)(lt / vi.tiles_x);
    const int sx0 = tx * T + (wave % SUB) * 8, sy0 = ty * T + (wave / SUB) * 8;
    const int px = sx0 + (lane & 7), py = sy0 + (lane >> 3);
    const bool inside = px < vi.W && py < vi.H;
    const float fpx = (float)px, fpy = (float)py;
    const float rx0 = (float)sx0, ry0 = (float)sy0;
    const float rx1 = (float)min(sx0 + 7, vi.W - 1), ry1 = (float)min(sy0 + 7, vi.H - 1);
    const uint32_t start = ranges[2 * gtile];
    const int64_t pix = vi.pix_off + (int64_t)py * vi.W + px;
    const int64_t vbase = (int64_t)vi.v * n;

    if (threadIdx.x == 0) s_maxnc = 0;
    for (int q = threadIdx.x; q < NG * 64; q += T * T) (&s_grad[0][0])[q] = 0.f;
    uint32_t nc = 0;
    float Tr = 1.0f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
    if (inside) {
        nc = n_contrib[pix];
        Tr = final_T[pix];
        const int64_t plane = (int64_t)vi.W * vi.H;
        const float *gi = dL_dimage + 3 * vi.pix_off + (int64_t)py * vi.W + px;
        g0 = gi[0];
        g1 = gi[plane];
        g2 = gi[2 * plane];
    }
    // light from behind the current splat, starting with the background
    float B0 = Tr * bg0, B1 = Tr * bg1, B2 = Tr * bg2;
    uint32_t maxnc = nc;
    for (int off = 32; off > 0; off >>= 1) maxnc = max(maxnc, (uint32_t)__shfl_xor((int)maxnc, off));
    __syncthreads();
    if (lane == 0) atomicMax(&s_maxnc, maxnc);
    __syncthreads();
    const uint32_t maxnc_tile = s_maxnc;

    // chunks of 64 positions back to front: positions [p0, p1], 1-based
    for (int64_t p1 = maxnc_tile; p1 >= 1; p1 -= 64) {
        const int64_t p0 = p1 - 63 >= 1 ? p1 - 63 : 1;
        if (threadIdx.x < 64) {
            const int64_t pos = p0 + threadIdx.x;
            s_id[threadIdx.x] = pos <= p1 ? vals[start + (uint32_t)(pos - 1)] : 0u;
        }
        if ((uint32_t)p0 <= maxnc) {
            const int64_t pos = p0 + lane;
            bool keep = false;
            // the record is fully defined on every lane before the cull decision
            BwdRec rec;
            rec.a = rec.b = rec.c = rec.raw = make_float4(0.f, 0.f, 0.f, 0.f);
            if (pos <= p1 && pos <= (int64_t)maxnc) {
                const uint32_t idx = start + (uint32_t)(pos - 1);
                const uint32_t id = vals[idx];
                const float4 *s4 = reinterpret_cast<const float4 *>(splats + vbase + id);
                const float4 s0 = s4[0], s1 = s4[1], s2 = s4[2];
                const FwdRec f = make_rec(s0, s1, s2, (uint32_t)pos, id);
                rec.a = f.a;
                rec.b = f.b;
                rec.c = f.c;
                rec.raw = make_float4(s0.z, s0.w, s1.x, s1.y);
                keep = reaches_rect(s0.x, s0.y, s0.z, s0.w, s1.x, qmax_of(s1.y), rx0, rx1, ry0, ry1);
            }
            const uint64_t msk = ballot64(keep);
            if (keep) s_rec[wave][__popcll(msk & lanemask_lt())] = rec;
            wave_lds_sync();
            const int cnt = __popcll(msk);
            for (int j = cnt - 1; j >= 0; --j) {
                const float4 a = s_rec[wave][j].a, b = s_rec[wave][j].b;
                const uint32_t ppos = __float_as_uint(b.w);
                float gmx = 0.f, gmy = 0.f, gA = 0.f, gB = 0.f, gC = 0.f, gop = 0.f;
                float gr = 0.f, gg = 0.f, gb = 0.f;
                bool contrib = false;
                if (ppos <= nc) {
                    const float e2 = pair_e2(a, b, fpx, fpy);
                    if (e2 >= b.z) {
                        contrib = true;
                        const float4 c = s_rec[wave][j].c, raw = s_rec[wave][j].raw;
                        const float araw = fast_exp2(e2);
                        const float alpha = fminf(GS_ALPHA_MAX, araw);
                        const float oma = 1.0f - alpha;
                        const float ioma = __builtin_amdgcn_rcpf(oma);
                        Tr = Tr * ioma;
                        const float wT = alpha * Tr;
                        gr = g0 * wT;
                        gg = g1 * wT;
                        gb = g2 * wT;
                        const float dLda = g0 * (c.x * Tr - B0 * ioma) + g1 * (c.y * Tr - B1 * ioma) +
                                           g2 * (c.z * Tr - B2 * ioma);
                        B0 = fmaf(c.x, wT, B0);
                        B1 = fmaf(c.y, wT, B1);
                        B2 = fmaf(c.z, wT, B2);
                        if (araw <= GS_ALPHA_MAX) {
                            gop = dLda * alpha * __builtin_amdgcn_rcpf(raw.w);
                            const float dLdq = -0.5f * alpha * dLda;
                            const float dx = fpx - a.x, dy = fpy - a.y;
                            gA = dLdq * dx * dx;
                            gB = dLdq * 2.0f * dx * dy;
                            gC = dLdq * dy * dy;
                            gmx = -2.0f * dLdq * (raw.x * dx + raw.y * dy);
                            gmy = -2.0f * dLdq * (raw.y * dx + raw.z * dy);
                        }
                    }
                }
                if (ballot64(contrib) != 0) {
                    gmx = wave_total_63(gmx);
                    gmy = wave_total_63(gmy);
                    gA = wave_total_63(gA);
                    gB = wave_total_63(gB);
                    gC = wave_total_63(gC);
                    gop = wave_total_63(gop);
                    gr = wave_total_63(gr);
                    gg = wave_total_63(gg);
                    gb = wave_total_63(gb);
                    if (lane == 63) {
                        const int q = (int)(ppos - (uint32_t)p0);
                        atomicAdd(&s_grad[0][q], gmx);
                        atomicAdd(&s_grad[1][q], gmy);
                        atomicAdd(&s_grad[2][q], gA);
                        atomicAdd(&s_grad[3][q], gB);
                        atomicAdd(&s_grad[4][q], gC);
                        atomicAdd(&s_grad[5][q], gop);
                        atomicAdd(&s_grad[6][q], gr);
                        atomicAdd(&s_grad[7][q], gg);
                        atomicAdd(&s_grad[8][q], gb);
                    }
                }
            }
        }
        __syncthreads();
        // the tile's sums of this chunk leave with one atomic per quantity
        for (int q = threadIdx.x; q < NG * 64; q += T * T) {
            const int k = q >> 6, jj = q & 63;
            const float v = s_grad[k][jj];
            if (v != 0.f) {
                atomicAdd(reinterpret_cast<float *>(grads + vbase + s_id[jj]) + k, v);
                s_grad[k][jj] = 0.f;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Foveation tables.
struct FovArgs {
    gs_fovea f[8];
};

__global__ void __launch_bounds__(256)
k_fovea_pix(const gs_camera *__restrict__ cams, int V, int T, int L, int64_t n_pixels, FovArgs fa,
            uint8_t *__restrict__ pix_level, float *__restrict__ pix_weight)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_pixels) return;
    const ViewInfo vi = view_of_pixel(cams, V, T, p);
    const gs_camera &c = cams[vi.v];
    const gs_fovea f = fa.f[vi.v];
    int64_t lp = p - vi.pix_off;
    int x = (int)(lp % vi.W), y = (int)(lp / vi.W);
    float rx = ((float)x - c.cx) / c.fx, ry = ((float)y - c.cy) / c.fy;
    float gx = (f.gaze_x - c.cx) / c.fx, gy = (f.gaze_y - c.cy) / c.fy;
    // angle between (rx, ry, 1) and (gx, gy, 1)
    float cx_ = ry - gy, cy_ = gx - rx, cz_ = rx * gy - ry * gx;
    float cn = sqrtf(cx_ * cx_ + cy_ * cy_ + cz_ * cz_);
    float dt = rx * gx + ry * gy + 1.0f;
    float ecc = atan2f(cn, dt) * 57.29577951308232f;
    int lo = 1;
    float w = 0.0f;
    float hb = 0.5f * f.band_deg;
    for (int j = 0; j < L - 1; ++j) {
        float e0 = f.ring_deg[j] - hb, e1 = f.ring_deg[j] + hb;
        if (ecc < e0) break;
        if (ecc < e1) {
            lo = j + 1;
            w = (ecc - e0) / f.band_deg;
            break;
        }
        lo = j + 2;
    }
    pix_level[p] = (uint8_t)lo;
    pix_weight[p] = w;
}

// one wave per tile: lowest and highest level with non-zero weight
__global__ void __launch_bounds__(256)
k_fovea_tile(const gs_camera *__restrict__ cams, int V, int T, int64_t n_tiles,
             const uint8_t *__restrict__ pix_level, const float *__restrict__ pix_weight,
             uint8_t *__restrict__ tile_level)
{
    int64_t gt = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (gt >= n_tiles) return;
    const ViewInfo vi = view_of_tile(cams, V, T, gt);
    int64_t lt = gt - vi.tile_off;
    int tx = (int)(lt % vi.tiles_x), ty = (int)(lt / vi.tiles_x);
    int lo = 255, hi = 0;
    for (int k = lane; k < T * T; k += 64) {
        int x = tx * T + (k % T), y = ty * T + (k / T);
        if (x < vi.W && y < vi.H) {
            int64_t p = vi.pix_off + (int64_t)y * vi.W + x;
            int l = pix_level[p];
            lo = min(lo, l);
            hi = max(hi, l + (pix_weight[p] > 0.0f ? 1 : 0));
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo = min(lo, __shfl_xor(lo, off));
        hi = max(hi, __shfl_xor(hi, off));
    }
    if (lane == 0) {
        tile_level[2 * gt] = (uint8_t)lo;
        tile_level[2 * gt + 1] = (uint8_t)hi;
    }
}

}  // namespace

hipError_t launch_raster_fwd(const gs_splat *splats, int n, const gs_camera *cams_dev, int V, int T,
                             int64_t n_tiles, const uint32_t *vals, const uint32_t *ranges,
                             const float bg[3], float *image, float *final_T, uint32_t *n_contrib,
                             uint32_t *dominated, uint64_t *stats, hipStream_t st)
{
    if (n_tiles == 0) return hipSuccess;
    hipError_t e;
    if (dominated && (e = launch_fill_u32(dominated, 0u, (uint64_t)V * n, st)) != hipSuccess) return e;
    unsigned long long *sp = reinterpret_cast<unsigned long long *>(stats);
#define GS_RF(TS)                                                                                  \
    if (stats)                                                                                     \
        hipLaunchKernelGGL((k_raster_fwd<TS, false, true>), dim3((unsigned)n_tiles), dim3(TS * TS), \
                           0, st, splats, n, cams_dev, V, vals, ranges, bg[0], bg[1], bg[2], image, \
                           final_T, n_contrib, dominated, sp);                                     \
    else if (dominated)                                                                            \
        hipLaunchKernelGGL((k_raster_fwd<TS, true, false>), dim3((unsigned)n_tiles), dim3(TS * TS), \
                           0, st, splats, n, cams_dev, V, vals, ranges, bg[0], bg[1], bg[2], image, \
                           final_T, n_contrib, dominated, sp);                                     \
    else                                                                                           \
        hipLaunchKernelGGL((k_raster_fwd<TS, false, false>), dim3((unsigned)n_tiles),              \
                           dim3(TS * TS), 0, st, splats, n, cams_dev, V, vals, ranges, bg[0],      \
                           bg[1], bg[2], image, final_T, n_contrib, dominated, sp);
    switch (T) {
    case 8: GS_RF(8); break;
    case 16: GS_RF(16); break;
    default: GS_RF(32); break;
    }
#undef GS_RF
    return hipGetLastError();
}

hipError_t launch_raster_bwd(const gs_splat *splats, int n, const gs_camera *cams_dev, int V, int T,
                             int64_t n_tiles, const uint32_t *vals, const uint32_t *ranges,
                             const float bg[3], const float *final_T, const uint32_t *n_contrib,
                             const float *dL_dimage, gs_splat_grad *grads, hipStream_t st)
{
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(grads), 0u, (uint64_t)V * n * 12, st);
    if (e != hipSuccess || n_tiles == 0) return e;
#define GS_RB(TS)                                                                                    \
    hipLaunchKernelGGL((k_raster_bwd<TS>), dim3((unsigned)n_tiles), dim3(TS * TS), 0, st, splats, n, \
                       cams_dev, V, vals, ranges, bg[0], bg[1], bg[2], final_T, n_contrib, dL_dimage, \
                       grads);
    switch (T) {
    case 8: GS_RB(8); break;
    case 16: GS_RB(16); break;
    default: GS_RB(32); break;
    }
#undef GS_RB
    return hipGetLastError();
}

hipError_t launch_fovea_prep(const gs_camera *cams_dev, const gs_fovea *fov_host, int n_eyes, int T,
                             int n_levels, int64_t n_pixels, int64_t n_tiles, uint8_t *pix_level,
                             float *pix_weight, uint8_t *tile_level, hipStream_t st)
{
    FovArgs fa;
    for (int i = 0; i < 8; ++i) fa.f[i] = fov_host[i < n_eyes ? i : 0];
    hipLaunchKernelGGL(k_fovea_pix, dim3((unsigned)((n_pixels + 255) / 256)), dim3(256), 0, st,
                       cams_dev, n_eyes, T, n_levels, n_pixels, fa, pix_level, pix_weight);
    hipLaunchKernelGGL(k_fovea_tile, dim3((unsigned)((n_tiles + 3) / 4)), dim3(256), 0, st, cams_dev,
                       n_eyes, T, n_tiles, pix_level, pix_weight, tile_level);
    return hipGetLastError();
}

hipError_t launch_raster_fov(const gs_splat *splats, const float *lvl_rgba, int n,
                             const uint8_t *qbound, int n_levels, const gs_camera *cams_dev, int V,
                             int T, int64_t n_tiles, const uint32_t *vals, const uint32_t *ranges,
                             const uint8_t *pix_level, const float *pix_weight, const float bg[3],
                             float *image, uint64_t *stats, hipStream_t st)
{
    if (n_tiles == 0) return hipSuccess;
    const float4 *lv = reinterpret_cast<const float4 *>(lvl_rgba);
    unsigned long long *sp = reinterpret_cast<unsigned long long *>(stats);
#define GS_RV(TS)                                                                                    \
    if (stats)                                                                                       \
        hipLaunchKernelGGL((k_raster_fov<TS, true>), dim3((unsigned)n_tiles), dim3(TS * TS), 0, st,   \
                           splats, lv, n, qbound, n_levels, cams_dev, V, vals, ranges, pix_level,    \
                           pix_weight, bg[0], bg[1], bg[2], image, sp);                              \
    else                                                                                             \
        hipLaunchKernelGGL((k_raster_fov<TS, false>), dim3((unsigned)n_tiles), dim3(TS * TS), 0, st,  \
                           splats, lv, n, qbound, n_levels, cams_dev, V, vals, ranges, pix_level,    \
                           pix_weight, bg[0], bg[1], bg[2], image, sp);
    switch (T) {
    case 8: GS_RV(8); break;
    case 16: GS_RV(16); break;
    default: GS_RV(32); break;
    }
#undef GS_RV
    return hipGetLastError();
}
