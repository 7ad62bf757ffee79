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
// staging slots per wave: a chunk's 64 records after up to 3 carried ones,
// padded to a group of 4
constexpr int FWD_SLOTS = 68;

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

// The same falloff exponent qa dx^2 + qb dx dy + qc dy^2 expanded about the
// centre (cx, cy) of a wave's 8 x 8 block.  With (mu, mv) the mean's offset
// from the centre and (u, v) the pixel's,
//   e = F + u (D + qa u + qb v) + v (E + qc v),
//   D = -(2 qa mu + qb mv),  E = -(2 qc mv + qb mu),
//   F = qa mu^2 + qb mu mv + qc mv^2,
// five FMAs per pair instead of the two differences and five products and
// sums of the direct form (the mean is folded into F, D, E once per splat).
// The cancellation between the terms is the one the direct form has between
// qa dx^2, qb dx dy and qc dy^2: both lose accuracy with the conic's
// condition, not with the expansion.  Explicit fmaf throughout, so that
// every kernel that evaluates a pair this way rounds identically.
struct Quad {
    float F, D, E;
};

__device__ __forceinline__ Quad quad_about(float mx, float my, float qa, float qb, float qc, float cx, float cy)
{
    const float mu = mx - cx, mv = my - cy;
    Quad q;
    q.D = -fmaf(qb, mv, (2.0f * qa) * mu);
    q.E = -fmaf(qb, mu, (2.0f * qc) * mv);
    q.F = fmaf(mu, fmaf(qa, mu, qb * mv), (qc * mv) * mv);
    return q;
}

__device__ __forceinline__ float quad_eval(float F, float D, float E, float qa, float qb, float qc, float u,
                                           float v)
{
    const float t1 = fmaf(qa, u, fmaf(qb, v, D));
    const float t2 = fmaf(v, fmaf(qc, v, E), F);
    return fmaf(u, t1, t2);
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

// Where a wave works: its 8x8 sub-block of a tile, its pixel, and the
// sub-block rectangle clipped to the image (for the footprint cull).
struct WaveCtx {
    ViewInfo vi;
    int px, py;
    bool inside;
    float fpx, fpy, rx0, rx1, ry0, ry1;
    uint32_t start, end;  // the tile's run in the sorted list
    int64_t pix;
};

template <int T>
__device__ __forceinline__ WaveCtx wave_ctx(const gs_camera *__restrict__ cams, int V, int64_t gtile, int sub,
                                            int lane, const uint32_t *__restrict__ ranges)
{
    constexpr int SUB = T / 8;
    WaveCtx w;
    w.vi = view_of_tile(cams, V, T, gtile);
    const int64_t lt = gtile - w.vi.tile_off;
    const int tx = (int)(lt % w.vi.tiles_x), ty = (int)(lt / w.vi.tiles_x);
    const int sx0 = tx * T + (sub % SUB) * 8, sy0 = ty * T + (sub / SUB) * 8;
    w.px = sx0 + (lane & 7);
    w.py = sy0 + (lane >> 3);
    w.inside = w.px < w.vi.W && w.py < w.vi.H;
    w.fpx = (float)w.px;
    w.fpy = (float)w.py;
    w.rx0 = (float)sx0;
    w.ry0 = (float)sy0;
    w.rx1 = (float)min(sx0 + 7, w.vi.W - 1);
    w.ry1 = (float)min(sy0 + 7, w.vi.H - 1);
    w.start = ranges[2 * gtile];
    w.end = ranges[2 * gtile + 1];
    w.pix = w.vi.pix_off + (int64_t)w.py * w.vi.W + w.px;
    return w;
}

// Per-pixel state of the plain compositor.
struct FwdState {
    float Tr, C0, C1, C2, best;
    uint32_t last;
    int best_id;
    bool done;
};

__device__ __forceinline__ FwdState fwd_init(bool inside)
{
    FwdState s;
    s.Tr = 1.0f;
    s.C0 = s.C1 = s.C2 = 0.0f;
    s.best = 0.0f;
    s.last = 0;
    s.best_id = -1;
    s.done = !inside;
    return s;
}

// Front-to-back over list positions [b, e) of the tile (absolute indices into
// vals): 64 entries at a time are gathered, culled against the sub-block and
// compacted into the wave's LDS slice, then composited.
template <bool DOM, bool STATS>
__device__ __forceinline__ void fwd_walk(const gs_splat *__restrict__ vsp, const uint32_t *__restrict__ vals,
                                         const WaveCtx &w, uint32_t b, uint32_t e, FwdRec *__restrict__ srec,
                                         FwdState &s, float *st)
{
    const int lane = __lane_id();
    // the next chunk's point indices load while this chunk composites (an
    // unconditional load clamped to the run's last entry, so that waiting
    // for the records never waits for it)
    uint32_t id_next = b < e ? vals[min(b + lane, e - 1)] : 0u;
    int carry = 0;  // records carried over from the chunk before, at srec[0, carry)
    for (uint32_t c0 = b; c0 < e; c0 += 64) {
        if (ballot64(!s.done) == 0) break;
        const uint32_t idx = c0 + lane;
        const uint32_t id = id_next;
        id_next = vals[min(c0 + 64 + lane, e - 1)];
        bool keep = false;
        // the record is fully defined on every lane before the cull decision
        FwdRec rec = zero_rec();
        if (idx < e) {
            const float4 *s4 = reinterpret_cast<const float4 *>(vsp + id);
            const float4 s0 = s4[0], s1 = s4[1], s2 = s4[2];
            rec = make_rec(s0, s1, s2, idx - w.start + 1, id);
            keep = reaches_rect(s0.x, s0.y, s0.z, s0.w, s1.x, qmax_of(s1.y), w.rx0, w.rx1, w.ry0, w.ry1);
        }
        const uint64_t m = ballot64(keep);
        const int cnt = __popcll(m);
        // kept records go after the 0-3 carried from the chunk before; the
        // loop below runs in groups of 4 with one exit test per group, and
        // the records past the last full group wait for the next chunk --
        // after the last chunk they are padded to a group with null records
        // (an infinite alpha threshold: no pixel uses them)
        if (keep) srec[carry + __popcll(m & lanemask_lt())] = rec;
        const int total = carry + cnt;
        const bool last_chunk = c0 + 64 >= e;
        const int full = total & ~3;
        const int upto = last_chunk ? (total + 3) & ~3 : full;
        if (last_chunk && lane < 4 && full + lane >= total && full + lane < upto) {
            FwdRec z = zero_rec();
            z.b.z = __builtin_inff();
            srec[full + lane] = z;
        }
        wave_lds_sync();
        if (STATS) {
            st[2] += (float)min(64u, e - c0);
            st[3] += (float)cnt;
        }
        for (int j0 = 0; j0 < upto; j0 += 4) {
#pragma unroll
            for (int j = j0; j < j0 + 4; ++j) {
                // branch-free: every lane evaluates, selects take the decisions
                const float4 a = srec[j].a, bb = srec[j].b, c = srec[j].c;
                if (STATS) st[1] += (j >= total || s.done) ? 0.0f : 1.0f;
                const float e2 = pair_e2(a, bb, w.fpx, w.fpy);
                const float alpha = fminf(GS_ALPHA_MAX, fast_exp2(e2));
                const bool use = !s.done && e2 >= bb.z;
                const float Tn = fmaf(-alpha, s.Tr, s.Tr);
                const bool stop = use && Tn < GS_T_STOP;
                const bool blend = use && !stop;
                const float wt = blend ? alpha * s.Tr : 0.0f;
                s.C0 = fmaf(wt, c.x, s.C0);
                s.C1 = fmaf(wt, c.y, s.C1);
                s.C2 = fmaf(wt, c.z, s.C2);
                s.Tr = blend ? Tn : s.Tr;
                s.last = blend ? __float_as_uint(bb.w) : s.last;
                s.done = s.done || stop;
                if (STATS) st[0] += blend ? 1.0f : 0.0f;
                if (DOM && blend && wt > s.best) {
                    s.best = wt;
                    s.best_id = (int)__float_as_uint(c.w);
                }
            }
            if (ballot64(!s.done) == 0) break;
        }
        wave_lds_sync();
        // the records past the last full group move to the front (they do
        // not overlap their new place when there was a full group): lane k
        // moves part k % 3 of record k / 3
        const int left = total - full;
        if (!last_chunk && full > 0) {
            float4 *v4 = reinterpret_cast<float4 *>(srec);
            const bool mv = lane < 3 * left;
            const float4 t = v4[mv ? 3 * full + lane : 0];
            wave_lds_sync();
            if (mv) v4[lane] = t;
            wave_lds_sync();
        }
        carry = left;
    }
}

template <bool DOM>
__device__ __forceinline__ void fwd_finish(const WaveCtx &w, const FwdState &s, int n, float bg0, float bg1,
                                           float bg2, float *__restrict__ image, float *__restrict__ final_T,
                                           uint32_t *__restrict__ n_contrib, uint32_t *__restrict__ dominated)
{
    if (!w.inside) return;
    const int64_t plane = (int64_t)w.vi.W * w.vi.H;
    float *img = image + 3 * w.vi.pix_off + (int64_t)w.py * w.vi.W + w.px;
    img[0] = fmaf(s.Tr, bg0, s.C0);
    img[plane] = fmaf(s.Tr, bg1, s.C1);
    img[2 * plane] = fmaf(s.Tr, bg2, s.C2);
    final_T[w.pix] = s.Tr;
    n_contrib[w.pix] = s.last;
    if (DOM && s.best_id >= 0) atomicAdd(dominated + (int64_t)w.vi.v * n + s.best_id, 1u);
}

template <int T, bool DOM, bool STATS>
__global__ void __launch_bounds__(T *T)
k_raster_fwd(const gs_splat *__restrict__ splats, int n, const gs_camera *__restrict__ cams, int V,
             const uint32_t *__restrict__ vals, const uint32_t *__restrict__ ranges, float bg0,
             float bg1, float bg2, float *__restrict__ image, float *__restrict__ final_T,
             uint32_t *__restrict__ n_contrib, uint32_t *__restrict__ dominated,
             unsigned long long *__restrict__ stats)
{
    float st[4] = {0.f, 0.f, 0.f, 0.f};
    constexpr int WAVES = T * T / 64;
    __shared__ FwdRec s_rec[WAVES][FWD_SLOTS];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const WaveCtx w = wave_ctx<T>(cams, V, blockIdx.x, wave, lane, ranges);
    FwdState s = fwd_init(w.inside);
    fwd_walk<DOM, STATS>(splats + (int64_t)w.vi.v * n, vals, w, w.start, w.end, s_rec[wave], s, st);
    fwd_finish<DOM>(w, s, n, bg0, bg1, bg2, image, final_T, n_contrib, dominated);
    if (STATS) stats_add(stats, st[0], st[1], st[2], st[3]);
}

// ---------------------------------------------------------------------------
// Foveated compositing.  Record: the falloff about the wave's block centre
// (F, D, E, qa | qb, qc, point index, list position) and (r, g, b, opacity)
// of the two levels the wave's pixels use (wave_lo and wave_lo + 1); a wave
// that reads its levels from memory keeps the quality bound in the first
// level slot instead.  Each pixel runs the
// accumulator of its lower level and, if blended, of the next one; level t
// takes a splat only if its quality bound is >= t and uses that level's
// opacity and colour.  An 8 x 8 block needs more than two levels only when
// ring bands are closer than the block; such a wave reads the level data
// from memory instead.
constexpr int MAXL = 4;
struct FovRec {
    float4 a, b;
    float4 lv[2];
};
// staging slots per wave: a chunk's 64 records after up to 3 carried ones,
// padded to a group of 4
constexpr int FOV_SLOTS = 68;

struct FovPix {
    int lo;          // lower level of the pixel
    float wup;       // weight of level lo + 1
    bool two;        // the pixel blends two levels
    int wave_lo;     // lowest level any pixel of the wave needs
    bool any_two;    // some pixel of the wave blends two levels
    bool one;        // every pixel of the wave uses level wave_lo alone
    bool wide;       // the wave's pixels need more than two levels
};

__device__ __forceinline__ FovPix fov_pix(const WaveCtx &w, const uint8_t *__restrict__ pix_level,
                                          const float *__restrict__ pix_weight)
{
    FovPix f;
    f.lo = 1;
    f.wup = 0.0f;
    if (w.inside) {
        f.lo = pix_level[w.pix];
        f.wup = pix_weight[w.pix];
    }
    f.two = f.wup > 0.0f;
    int wl = w.inside ? f.lo : 255;
    for (int off = 32; off > 0; off >>= 1) wl = min(wl, __shfl_xor(wl, off));
    int wh = w.inside ? f.lo + (f.two ? 1 : 0) : 0;
    for (int off = 32; off > 0; off >>= 1) wh = max(wh, __shfl_xor(wh, off));
    f.wave_lo = wl;
    f.any_two = ballot64(f.two) != 0;
    f.one = wh == wl;
    f.wide = wh - wl >= 2;
    return f;
}

struct FovState {
    float Ta, A0, A1, A2, Tb, B0, B1, B2;
    uint32_t last_a, last_b;  // 1-based run position of the last blended splat (kept on request)
    bool done_a, done_b;
};

__device__ __forceinline__ FovState fov_init(bool inside, bool two)
{
    FovState s;
    s.Ta = s.Tb = 1.0f;
    s.A0 = s.A1 = s.A2 = s.B0 = s.B1 = s.B2 = 0.0f;
    s.last_a = s.last_b = 0u;
    s.done_a = !inside;
    s.done_b = !inside || !two;
    return s;
}

// One lane's share of a chunk's staging loads: the point's geometry and the
// level records the wave uses (one or two).  A level above the point's
// quality bound has zero opacity in the level records, which no cull or
// alpha test passes, so the quality bound itself is loaded only by a wave
// that reads its levels from memory.
struct FovFetch {
    uint32_t id;
    int m;
    float4 s0, l0, l1;
    float c;  // the conic's third coefficient (first word of the second vector)
};

template <bool WIDE>
__device__ __forceinline__ FovFetch fov_fetch(const gs_splat *__restrict__ splats, const float4 *__restrict__ lvl,
                                              const uint8_t *__restrict__ qbound, int L, int64_t vbase, uint32_t id,
                                              bool ok, int wave_lo, bool one)
{
    FovFetch r;
    r.id = id;
    r.m = 0;
    r.s0 = r.l0 = r.l1 = make_float4(0.f, 0.f, 0.f, 0.f);
    r.c = 0.0f;
    if (ok) {
        // only the words the compositor uses: a wider load would hold
        // registers that the compiler reuses at once, waiting for the load
        const float4 *s4 = reinterpret_cast<const float4 *>(splats + vbase + id);
        r.s0 = s4[0];
        r.c = reinterpret_cast<const float *>(s4 + 1)[0];
        if (WIDE) {
            r.m = qbound[id];
        } else {
            const float4 *lp = lvl + (vbase + id) * L;
            r.l0 = lp[min(max(wave_lo - 1, 0), L - 1)];
            if (!one) r.l1 = lp[min(wave_lo, L - 1)];
        }
    }
    return r;
}

template <bool STATS, bool KEEP, bool WIDE>
__device__ __forceinline__ void fov_walk_impl(const gs_splat *__restrict__ splats, const float4 *__restrict__ lvl,
                                         int n, const uint8_t *__restrict__ qbound, int L,
                                         const uint32_t *__restrict__ vals, const WaveCtx &w, const FovPix &f,
                                         uint32_t b, uint32_t e, FovRec *__restrict__ srec, FovState &s,
                                         float *st)
{
    const int lane = __lane_id();
    const int64_t vbase = (int64_t)w.vi.v * n;
    // the next chunk's point indices are loaded while this chunk is
    // composited, so that staging a chunk waits for one memory latency (its
    // records) instead of two dependent ones; prefetching the records too
    // holds more registers than the occupancy it costs is worth
    // (the index load is unconditional -- clamped to the run's last entry,
    // in bounds whenever the run is not empty -- so that waiting for the
    // records never has to wait for it)
    uint32_t id_next = b < e ? vals[min(b + lane, e - 1)] : 0u;
    // the block centre, and the pixel's offset from it (exact in float)
    const float cx = w.rx0 + 3.5f, cy = w.ry0 + 3.5f;
    const float pu = (float)(lane & 7) - 3.5f, pv = (float)(lane >> 3) - 3.5f;
    int carry = 0;  // records carried over from the chunk before, at srec[0, carry)
    for (uint32_t c0 = b; c0 < e; c0 += 64) {
        if (ballot64(!(s.done_a && s.done_b)) == 0) break;
        const uint32_t idx = c0 + lane;
        const FovFetch cur = fov_fetch<WIDE>(splats, lvl, qbound, L, vbase, id_next, idx < e, f.wave_lo, f.one);
        id_next = vals[min(c0 + 64 + lane, e - 1)];
        bool keep = false;
        // the record is fully defined on every lane before the cull decision
        FovRec rec;
        rec.a = rec.b = rec.lv[0] = rec.lv[1] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (idx < e) {
            const uint32_t id = cur.id;
            const int m = cur.m;
            const float4 s0 = cur.s0;
            const float c = cur.c;
            const float qa = NEG_HALF_LOG2E * s0.z, qb = -GS_LOG2E * s0.w, qc = NEG_HALF_LOG2E * c;
            const Quad q = quad_about(s0.x, s0.y, qa, qb, qc, cx, cy);
            rec.a = make_float4(q.F, q.D, q.E, qa);
            rec.b = make_float4(qb, qc, __uint_as_float(id), __uint_as_float(idx - w.start + 1));
            float qcull = 9.001f;
            if (WIDE) rec.lv[0].x = __int_as_float(m);
            if (!WIDE) {
                // (a level above the splat's quality bound has zero opacity:
                // no alpha test passes, so the loop needs no level test)
                rec.lv[0] = cur.l0;
                rec.lv[1] = cur.l1;
                // no pixel of the wave blends the splat where opacity * G
                // stays below the alpha floor (at every level the wave uses;
                // a splat filtered out of them has no reach at all)
                qcull = qmax_of(fmaxf(rec.lv[0].w, rec.lv[1].w));
            }
            keep = (!WIDE || m >= f.wave_lo) &&
                   reaches_rect(s0.x, s0.y, s0.z, s0.w, c, qcull, w.rx0, w.rx1, w.ry0, w.ry1);
        }
        const uint64_t msk = ballot64(keep);
        const int cnt = __popcll(msk);
        // kept records go after the 0-3 carried from the chunk before; the
        // loop below runs in groups of 4 with one exit test per group, and
        // the records past the last full group wait for the next chunk --
        // after the last chunk they are padded to a group with null records
        // (opacity 0, quality bound -1: no pixel uses them)
        if (keep) srec[carry + __popcll(msk & lanemask_lt())] = rec;
        const int total = carry + cnt;
        const bool last_chunk = c0 + 64 >= e;
        const int full = total & ~3;
        const int upto = last_chunk ? (total + 3) & ~3 : full;
        if (last_chunk && lane < 4 && full + lane >= total && full + lane < upto) {
            FovRec z;
            z.a = z.b = z.lv[1] = make_float4(0.f, 0.f, 0.f, 0.f);
            z.lv[0] = make_float4(WIDE ? __int_as_float(-1) : 0.f, 0.f, 0.f, 0.f);
            srec[full + lane] = z;
        }
        wave_lds_sync();
        if (STATS) {
            st[2] += (float)min(64u, e - c0);
            st[3] += (float)cnt;
        }
        for (int j0 = 0; j0 < upto; j0 += 4) {
#pragma unroll
            for (int j = j0; j < j0 + 4; ++j) {
                // branch-free: every lane evaluates, selects take the decisions
                const float4 a = srec[j].a, bb = srec[j].b;
                if (STATS) st[1] += (j >= total || (s.done_a && s.done_b)) ? 0.0f : 1.0f;
                const float p2 = quad_eval(a.x, a.y, a.z, a.w, bb.x, bb.y, pu, pv);  // falloff only
                const float G = fast_exp2(p2);
                const bool incl = p2 >= EXTENT_LOG2;
                float4 lva, lvb;
                int m = 0;
                if (!WIDE) {
                    // 0 or 1 inside the image; pixels outside (level 1, done) are clamped
                    lva = srec[j].lv[min(max(f.lo - f.wave_lo, 0), 1)];
                    lvb = srec[j].lv[1];
                } else {
                    m = __float_as_int(srec[j].lv[0].x);
                    const float4 *lp = lvl + (vbase + __float_as_uint(bb.z)) * L;
                    lva = lp[f.lo - 1];
                    lvb = lp[f.lo < L ? f.lo : L - 1];
                }
                {
                    const float4 lv = lva;
                    const float alpha = fminf(GS_ALPHA_MAX, lv.w * G);
                    const bool use = incl && !s.done_a && (!WIDE || m >= f.lo) && alpha >= GS_ALPHA_MIN;
                    const float Tn = fmaf(-alpha, s.Ta, s.Ta);
                    const bool stop = use && Tn < GS_T_STOP;
                    const bool blend = use && !stop;
                    const float wt = blend ? alpha * s.Ta : 0.0f;
                    s.A0 = fmaf(wt, lv.x, s.A0);
                    s.A1 = fmaf(wt, lv.y, s.A1);
                    s.A2 = fmaf(wt, lv.z, s.A2);
                    s.Ta = blend ? Tn : s.Ta;
                    if (KEEP) s.last_a = blend ? __float_as_uint(bb.w) : s.last_a;
                    s.done_a = s.done_a || stop;
                    if (STATS) st[0] += blend ? 1.0f : 0.0f;
                }
                if (f.any_two) {
                    const float4 lv = lvb;
                    const float alpha = fminf(GS_ALPHA_MAX, lv.w * G);
                    const bool use = incl && !s.done_b && (!WIDE || m >= f.lo + 1) && alpha >= GS_ALPHA_MIN;
                    const float Tn = fmaf(-alpha, s.Tb, s.Tb);
                    const bool stop = use && Tn < GS_T_STOP;
                    const bool blend = use && !stop;
                    const float wt = blend ? alpha * s.Tb : 0.0f;
                    s.B0 = fmaf(wt, lv.x, s.B0);
                    s.B1 = fmaf(wt, lv.y, s.B1);
                    s.B2 = fmaf(wt, lv.z, s.B2);
                    s.Tb = blend ? Tn : s.Tb;
                    if (KEEP) s.last_b = blend ? __float_as_uint(bb.w) : s.last_b;
                    s.done_b = s.done_b || stop;
                    if (STATS) st[0] += blend ? 1.0f : 0.0f;
                }
            }
            if (ballot64(!(s.done_a && s.done_b)) == 0) break;
        }
        wave_lds_sync();
        // the records past the last full group move to the front (they do
        // not overlap their new place when there was a full group)
        const int left = total - full;
        if (!last_chunk && full > 0) {
            // one float4 per lane: lane k moves part k % 4 of record k / 4
            float4 *v4 = reinterpret_cast<float4 *>(srec);
            const bool mv = lane < 4 * left;
            const float4 t = v4[mv ? 4 * full + lane : 0];
            wave_lds_sync();
            if (mv) v4[lane] = t;
            wave_lds_sync();
        }
        carry = left;
    }
}

// The two-level records serve every wave whose pixels need at most two
// levels; the rest read level data from memory (separate instantiations keep
// memory loads out of the common loop).
template <bool STATS, bool KEEP = false>
__device__ __forceinline__ void fov_walk(const gs_splat *__restrict__ splats, const float4 *__restrict__ lvl,
                                         int n, const uint8_t *__restrict__ qbound, int L,
                                         const uint32_t *__restrict__ vals, const WaveCtx &w, const FovPix &f,
                                         uint32_t b, uint32_t e, FovRec *__restrict__ srec, FovState &s,
                                         float *st)
{
    if (f.wide)
        fov_walk_impl<STATS, KEEP, true>(splats, lvl, n, qbound, L, vals, w, f, b, e, srec, s, st);
    else
        fov_walk_impl<STATS, KEEP, false>(splats, lvl, n, qbound, L, vals, w, f, b, e, srec, s, st);
}

__device__ __forceinline__ void fov_finish(const WaveCtx &w, const FovPix &f, const FovState &s, float bg0,
                                           float bg1, float bg2, float *__restrict__ image)
{
    if (!w.inside) return;
    const int64_t plane = (int64_t)w.vi.W * w.vi.H;
    float *img = image + 3 * w.vi.pix_off + (int64_t)w.py * w.vi.W + w.px;
    float ra = fmaf(s.Ta, bg0, s.A0), ga = fmaf(s.Ta, bg1, s.A1), ba = fmaf(s.Ta, bg2, s.A2);
    if (f.two) {
        // written out with fmaf so that every kernel sharing this epilogue
        // rounds the blend identically (left to contraction, the compiler
        // fuses a different product in different kernels)
        const float rb = fmaf(s.Tb, bg0, s.B0), gb = fmaf(s.Tb, bg1, s.B1), bb = fmaf(s.Tb, bg2, s.B2);
        const float wl = 1.0f - f.wup;
        ra = fmaf(f.wup, rb, wl * ra);
        ga = fmaf(f.wup, gb, wl * ga);
        ba = fmaf(f.wup, bb, wl * ba);
    }
    img[0] = ra;
    img[plane] = ga;
    img[2 * plane] = ba;
}

// Eight waves per SIMD (at most 64 registers) composite faster than the six
// the compiler's own choice of 73 allows: 0.484 -> 0.463 ms at seven waves,
// 0.451 ms at eight, on the stereo 1080p frame.  At eight, one 64-bit value
// is kept in scratch across the chunk loop (and one record per chunk in the
// rare walk that reads levels from memory); the record loop itself spills
// nothing.  The statistics and reverse-state instantiations keep the
// compiler's choice.
template <int T, bool STATS, bool KEEP>
__global__ void __launch_bounds__(T *T) __attribute__((amdgpu_waves_per_eu(STATS || KEEP ? 1 : 8)))
k_raster_fov(const gs_splat *__restrict__ splats, const float4 *__restrict__ lvl, int n,
             const uint8_t *__restrict__ qbound, int L, const gs_camera *__restrict__ cams, int V,
             const uint32_t *__restrict__ vals, const uint32_t *__restrict__ ranges,
             const uint8_t *__restrict__ pix_level, const float *__restrict__ pix_weight, float bg0,
             float bg1, float bg2, float *__restrict__ image, unsigned long long *__restrict__ stats,
             float2 *__restrict__ final_T2, uint2 *__restrict__ n_contrib2)
{
    float st[4] = {0.f, 0.f, 0.f, 0.f};
    constexpr int WAVES = T * T / 64;
    __shared__ FovRec s_rec[WAVES][FOV_SLOTS];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const WaveCtx w = wave_ctx<T>(cams, V, blockIdx.x, wave, lane, ranges);
    const FovPix f = fov_pix(w, pix_level, pix_weight);
    FovState s = fov_init(w.inside, f.two);
    fov_walk<STATS, KEEP>(splats, lvl, n, qbound, L, vals, w, f, w.start, w.end, s_rec[wave], s, st);
    fov_finish(w, f, s, bg0, bg1, bg2, image);
    if (KEEP && w.inside) {
        // the reverse pass starts from these: per accumulator, the final T and
        // the last blended position
        final_T2[w.pix] = make_float2(s.Ta, s.Tb);
        n_contrib2[w.pix] = make_uint2(s.last_a, s.last_b);
    }
    if (STATS) stats_add(stats, st[0], st[1], st[2], st[3]);
}

// ---------------------------------------------------------------------------
// Persistent work queue (load balance across tiles).  A task is a tile, or,
// for a tile whose run is longer than the split length beta, one chunk of
// beta entries of it; a workgroup takes one task at a time and its waves
// cover the tile's 8x8 sub-blocks as in the one-workgroup-per-tile kernels
// (so they share the gathered splats in cache).  Tasks of tiles with long
// runs are queued first (longest work first); the workgroups of a persistent
// grid pop tasks from one atomic counter until the queue is empty.  A chunk
// composites its entries from T = 1 and stores (C, T, stopped) per pixel;
// the workgroup that finishes a tile's last chunk merges the chunks front to
// back with (C, T)_a + (C, T)_b = (C_a + T_a C_b, T_a T_b).  Where the running
// T reaches the stop threshold inside a chunk (or the chunk stopped on its
// own), the product would overshoot the sequential stop, so that chunk is
// composited again for those pixels from the running state -- the
// sequential result, up to float reassociation of the T products.
struct RasterQueue {
    uint32_t *counts;     // [4]: head, heavy tasks, light tasks, spare
    uint2 *heavy;         // [heavy_cap] (tile, chunk)
    uint2 *light;         // [light_cap]
    uint32_t *merge_cnt;  // [heavy_cap] chunks finished, at each tile's first chunk
    float4 *part;         // [heavy_cap][T*T][3] chunk partials (split only)
    uint32_t heavy_cap, light_cap;
    uint32_t beta;        // split length (0: no split)
    uint32_t heavy_min;   // runs longer than this are queued first
    uint32_t grab;        // tasks taken per pop
    int64_t n_tiles;
};

__device__ __forceinline__ uint32_t n_chunks_of(uint32_t len, uint32_t beta)
{
    return (beta && len > beta) ? (len + beta - 1) / beta : 1u;
}

// One thread per tile; block-level aggregation of the queue reservations.
__global__ void __launch_bounds__(256)
k_build_queue(const uint32_t *__restrict__ ranges, int64_t n_tiles, RasterQueue q)
{
    __shared__ uint32_t s_h[4], s_l[4], s_bh, s_bl;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t nch = 1, nh = 0, nl = 0;
    if (t < n_tiles) {
        const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
        nch = n_chunks_of(len, q.beta);
        if (nch > 1 || len > q.heavy_min)
            nh = nch;
        else
            nl = 1;
    }
    // exclusive prefix of nh and nl over the block
    uint32_t ih = nh, il = nl;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t a = __shfl_up(ih, off), b = __shfl_up(il, off);
        if (lane >= off) {
            ih += a;
            il += b;
        }
    }
    if (lane == 63) {
        s_h[wave] = ih;
        s_l[wave] = il;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t th = 0, tl = 0;
        for (int k = 0; k < 4; ++k) {
            const uint32_t a = s_h[k], b = s_l[k];
            s_h[k] = th;
            s_l[k] = tl;
            th += a;
            tl += b;
        }
        s_bh = th ? atomicAdd(q.counts + 1, th) : 0u;
        s_bl = tl ? atomicAdd(q.counts + 2, tl) : 0u;
    }
    __syncthreads();
    if (t >= n_tiles) return;
    if (nh) {
        const uint32_t base = s_bh + s_h[wave] + ih - nh;
        if (base + nh <= q.heavy_cap) {
            for (uint32_t c = 0; c < nh; ++c) q.heavy[base + c] = make_uint2((uint32_t)t, c);
            q.merge_cnt[base] = 0u;
            return;
        }
        // no room among the heavy tasks: blank the reserved slots that exist
        // and queue the tile unsplit with the light ones (which always fit)
        for (uint32_t k = base; k < base + nh && k < q.heavy_cap; ++k) q.heavy[k] = make_uint2(0xFFFFFFFFu, 0u);
        const uint32_t lb = atomicAdd(q.counts + 2, 1u);
        if (lb < q.light_cap) q.light[lb] = make_uint2((uint32_t)t, 0u);
        return;
    }
    const uint32_t base = s_bl + s_l[wave] + il - nl;
    if (base < q.light_cap) q.light[base] = make_uint2((uint32_t)t, 0u);
}

// Pops the next task for the calling workgroup (uniform over the block).
__device__ __forceinline__ uint32_t pop_task(uint32_t *head, uint32_t *s_slot, uint32_t grab)
{
    if (threadIdx.x == 0) *s_slot = atomicAdd(head, grab);
    __syncthreads();
    const uint32_t v = *s_slot;
    __syncthreads();
    return v;
}

// After a chunk's partials are stored: counts the chunk as finished and
// returns true (uniform over the block) in the workgroup that finished last.
__device__ __forceinline__ bool last_chunk(uint32_t *cnt, uint32_t nch, uint32_t *s_slot)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) *s_slot = atomicAdd(cnt, 1u);
    __syncthreads();
    const bool last = *s_slot == nch - 1;
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// One task of the plain compositor (every thread of the block calls it).
template <int T, bool DOM>
__device__ __forceinline__ void fwd_task(const gs_splat *__restrict__ splats, int n,
                                         const gs_camera *__restrict__ cams, int V,
                                         const uint32_t *__restrict__ vals, const uint32_t *__restrict__ ranges,
                                         float bg0, float bg1, float bg2, float *__restrict__ image,
                                         float *__restrict__ final_T, uint32_t *__restrict__ n_contrib,
                                         uint32_t *__restrict__ dominated, const RasterQueue &q, uint32_t nh,
                                         uint32_t it, FwdRec *__restrict__ srec, uint32_t *s_slot)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint2 task = it < nh ? q.heavy[it] : q.light[it - nh];
    if ((int64_t)task.x >= q.n_tiles) return;
    const uint32_t c = task.y;
    const WaveCtx w = wave_ctx<T>(cams, V, task.x, wave, lane, ranges);
    const gs_splat *vsp = splats + (int64_t)w.vi.v * n;
    // tasks from the light list (including heavy tiles that did not fit
    // among the heavy tasks) are never split
    const uint32_t nch = it < nh ? n_chunks_of(w.end - w.start, q.beta) : 1u;
    FwdState s = fwd_init(w.inside);
    if (nch == 1) {
        fwd_walk<DOM, false>(vsp, vals, w, w.start, w.end, srec, s, nullptr);
        fwd_finish<DOM>(w, s, n, bg0, bg1, bg2, image, final_T, n_contrib, dominated);
        return;
    }
    if (c >= nch || it - c + nch > nh) return;
    const uint32_t b = w.start + c * q.beta, e = min(w.end, b + q.beta);
    fwd_walk<DOM, false>(vsp, vals, w, b, e, srec, s, nullptr);
    float4 *pp = q.part + ((int64_t)it * (T * T) + threadIdx.x) * 3;
    pp[0] = make_float4(s.C0, s.C1, s.C2, s.Tr);
    pp[1] = make_float4(__uint_as_float(s.last), s.best, __int_as_float(s.best_id),
                        __uint_as_float(s.done ? 1u : 0u));
    const uint32_t first = it - c;
    if (!last_chunk(q.merge_cnt + first, nch, s_slot)) return;
    // last chunk of this tile: merge front to back
    FwdState m = fwd_init(w.inside);
    for (uint32_t k = 0; k < nch; ++k) {
        const float4 *pk = q.part + ((int64_t)(first + k) * (T * T) + threadIdx.x) * 3;
        const float4 p0 = pk[0], p1 = pk[1];
        const bool pdone = __float_as_uint(p1.w) != 0u;
        const bool fix = !m.done && (pdone || m.Tr * p0.w < GS_T_STOP);
        if (!m.done && !fix) {
            m.C0 = fmaf(m.Tr, p0.x, m.C0);
            m.C1 = fmaf(m.Tr, p0.y, m.C1);
            m.C2 = fmaf(m.Tr, p0.z, m.C2);
            const uint32_t pl = __float_as_uint(p1.x);
            if (pl) m.last = pl;
            if (DOM && __float_as_int(p1.z) >= 0 && m.Tr * p1.y > m.best) {
                m.best = m.Tr * p1.y;
                m.best_id = __float_as_int(p1.z);
            }
            m.Tr *= p0.w;
        }
        if (ballot64(fix) != 0) {
            // composite this chunk again from the running state
            FwdState r = m;
            r.done = m.done || !fix;
            const uint32_t kb = w.start + k * q.beta, ke = min(w.end, kb + q.beta);
            fwd_walk<DOM, false>(vsp, vals, w, kb, ke, srec, r, nullptr);
            if (fix) m = r;
        }
    }
    fwd_finish<DOM>(w, m, n, bg0, bg1, bg2, image, final_T, n_contrib, dominated);
}

template <int T, bool DOM>
__global__ void __launch_bounds__(T *T)
k_raster_fwd_q(const gs_splat *__restrict__ splats, int n, const gs_camera *__restrict__ cams, int V,
               const uint32_t *__restrict__ vals, const uint32_t *__restrict__ ranges, float bg0, float bg1,
               float bg2, float *__restrict__ image, float *__restrict__ final_T,
               uint32_t *__restrict__ n_contrib, uint32_t *__restrict__ dominated, RasterQueue q)
{
    constexpr int WAVES = T * T / 64;
    __shared__ FwdRec s_rec[WAVES][FWD_SLOTS];
    __shared__ uint32_t s_slot;
    const uint32_t nh = min(q.counts[1], q.heavy_cap), total = nh + min(q.counts[2], q.light_cap);
    // q.grab consecutive tasks per pop (neighbouring tiles share splats in cache)
    uint32_t it = pop_task(q.counts, &s_slot, q.grab);
    while (it < total) {
        for (uint32_t k = 0; k < q.grab && it + k < total; ++k) {
            fwd_task<T, DOM>(splats, n, cams, V, vals, ranges, bg0, bg1, bg2, image, final_T, n_contrib,
                             dominated, q, nh, it + k, s_rec[threadIdx.x >> 6], &s_slot);
            __syncthreads();
        }
        it = pop_task(q.counts, &s_slot, q.grab);
    }
}

// One task of the foveated compositor (every thread of the block calls it).
template <int T>
__device__ __forceinline__ void fov_task(const gs_splat *__restrict__ splats, const float4 *__restrict__ lvl,
                                         int n, const uint8_t *__restrict__ qbound, int L,
                                         const gs_camera *__restrict__ cams, int V,
                                         const uint32_t *__restrict__ vals, const uint32_t *__restrict__ ranges,
                                         const uint8_t *__restrict__ pix_level,
                                         const float *__restrict__ pix_weight, float bg0, float bg1, float bg2,
                                         float *__restrict__ image, const RasterQueue &q, uint32_t nh,
                                         uint32_t it, FovRec *__restrict__ srec, uint32_t *s_slot)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint2 task = it < nh ? q.heavy[it] : q.light[it - nh];
    if ((int64_t)task.x >= q.n_tiles) return;
    const uint32_t c = task.y;
    const WaveCtx w = wave_ctx<T>(cams, V, task.x, wave, lane, ranges);
    const FovPix f = fov_pix(w, pix_level, pix_weight);
    // tasks from the light list (including heavy tiles that did not fit
    // among the heavy tasks) are never split
    const uint32_t nch = it < nh ? n_chunks_of(w.end - w.start, q.beta) : 1u;
    FovState s = fov_init(w.inside, f.two);
    if (nch == 1) {
        fov_walk<false>(splats, lvl, n, qbound, L, vals, w, f, w.start, w.end, srec, s, nullptr);
        fov_finish(w, f, s, bg0, bg1, bg2, image);
        return;
    }
    if (c >= nch || it - c + nch > nh) return;
    const uint32_t b = w.start + c * q.beta, e = min(w.end, b + q.beta);
    fov_walk<false>(splats, lvl, n, qbound, L, vals, w, f, b, e, srec, s, nullptr);
    float4 *pp = q.part + ((int64_t)it * (T * T) + threadIdx.x) * 3;
    pp[0] = make_float4(s.A0, s.A1, s.A2, s.Ta);
    pp[1] = make_float4(s.B0, s.B1, s.B2, s.Tb);
    pp[2] = make_float4(__uint_as_float(s.done_a ? 1u : 0u), __uint_as_float(s.done_b ? 1u : 0u), 0.f, 0.f);
    const uint32_t first = it - c;
    if (!last_chunk(q.merge_cnt + first, nch, s_slot)) return;
    // last chunk of this tile: merge front to back
    FovState m = fov_init(w.inside, f.two);
    for (uint32_t k = 0; k < nch; ++k) {
        const float4 *pk = q.part + ((int64_t)(first + k) * (T * T) + threadIdx.x) * 3;
        const float4 pa = pk[0], pb = pk[1], pf = pk[2];
        const bool fix_a = !m.done_a && (__float_as_uint(pf.x) != 0u || m.Ta * pa.w < GS_T_STOP);
        const bool fix_b = !m.done_b && (__float_as_uint(pf.y) != 0u || m.Tb * pb.w < GS_T_STOP);
        if (!m.done_a && !fix_a) {
            m.A0 = fmaf(m.Ta, pa.x, m.A0);
            m.A1 = fmaf(m.Ta, pa.y, m.A1);
            m.A2 = fmaf(m.Ta, pa.z, m.A2);
            m.Ta *= pa.w;
        }
        if (!m.done_b && !fix_b) {
            m.B0 = fmaf(m.Tb, pb.x, m.B0);
            m.B1 = fmaf(m.Tb, pb.y, m.B1);
            m.B2 = fmaf(m.Tb, pb.z, m.B2);
            m.Tb *= pb.w;
        }
        if (ballot64(fix_a || fix_b) != 0) {
            // composite this chunk again from the running state
            FovState r = m;
            r.done_a = m.done_a || !fix_a;
            r.done_b = m.done_b || !fix_b;
            const uint32_t kb = w.start + k * q.beta, ke = min(w.end, kb + q.beta);
            fov_walk<false>(splats, lvl, n, qbound, L, vals, w, f, kb, ke, srec, r, nullptr);
            if (fix_a) {
                m.Ta = r.Ta;
                m.A0 = r.A0;
                m.A1 = r.A1;
                m.A2 = r.A2;
                m.done_a = r.done_a;
            }
            if (fix_b) {
                m.Tb = r.Tb;
                m.B0 = r.B0;
                m.B1 = r.B1;
                m.B2 = r.B2;
                m.done_b = r.done_b;
            }
        }
    }
    fov_finish(w, f, m, bg0, bg1, bg2, image);
}

template <int T>
__global__ void __launch_bounds__(T *T)
k_raster_fov_q(const gs_splat *__restrict__ splats, const float4 *__restrict__ lvl, int n,
               const uint8_t *__restrict__ qbound, int L, const gs_camera *__restrict__ cams, int V,
               const uint32_t *__restrict__ vals, const uint32_t *__restrict__ ranges,
               const uint8_t *__restrict__ pix_level, const float *__restrict__ pix_weight, float bg0, float bg1,
               float bg2, float *__restrict__ image, RasterQueue q)
{
    constexpr int WAVES = T * T / 64;
    __shared__ FovRec s_rec[WAVES][FOV_SLOTS];
    __shared__ uint32_t s_slot;
    const uint32_t nh = min(q.counts[1], q.heavy_cap), total = nh + min(q.counts[2], q.light_cap);
    // q.grab consecutive tasks per pop (neighbouring tiles share splats in cache)
    uint32_t it = pop_task(q.counts, &s_slot, q.grab);
    while (it < total) {
        for (uint32_t k = 0; k < q.grab && it + k < total; ++k) {
            fov_task<T>(splats, lvl, n, qbound, L, cams, V, vals, ranges, pix_level, pix_weight, bg0, bg1, bg2,
                        image, q, nh, it + k, s_rec[threadIdx.x >> 6], &s_slot);
            __syncthreads();
        }
        it = pop_task(q.counts, &s_slot, q.grab);
    }
}

// ---------------------------------------------------------------------------
// Tile merging (the Tile Merge Unit of Section 5.2, on the GPU): consecutive
// tiles are merged while their intersections (keys) total at most beta; a
// tile with more stands alone.  Greedy from the first tile: the group that
// starts at tile i ends before next(i), the last j with S(j) - S(i) <= beta
// (S the exclusive prefix of the tile loads; at least i + 1).  The group
// starts are the chain 0, next(0), next(next(0)), ...: found by pointer
// doubling (round r marks the chain nodes 2^r steps beyond the marked ones),
// then compacted in order.  One workgroup does it all; a persistent
// compositor's workgroups then pop whole groups and composite their tiles
// one after another (per pixel exactly as one workgroup per tile).
struct MergeView {
    uint32_t *counts;  // [16]: groups, pop head
    uint32_t *S, *nxt, *J0, *J1, *mark;  // [n_tiles + 1]
    uint2 *groups;     // [n_tiles + 1] (first tile, end tile)
};

__host__ __device__ __forceinline__ MergeView merge_view(uint32_t *base, int64_t n_tiles)
{
    MergeView m;
    const int64_t n1 = n_tiles + 1;
    m.counts = base;
    m.S = base + 16;
    m.nxt = m.S + n1;
    m.J0 = m.nxt + n1;
    m.J1 = m.J0 + n1;
    m.mark = m.J1 + n1;
    m.groups = reinterpret_cast<uint2 *>(m.mark + n1 + ((n1 & 1) ? 1 : 0));
    return m;
}

constexpr int MERGE_THREADS = 1024;

// Exclusive scan of f(i), i < n, into out[0..n] (out[n] = total), by the
// whole workgroup: contiguous segments per thread, segment totals in LDS.
template <class F>
__device__ __forceinline__ void block_exclusive_scan(int64_t n, F f, uint32_t *__restrict__ out, uint32_t *s_tot)
{
    const int t = threadIdx.x;
    const int64_t seg = (n + MERGE_THREADS - 1) / MERGE_THREADS;
    const int64_t b = t * seg, e = min(b + seg, n);
    uint32_t acc = 0;
    for (int64_t i = b; i < e; ++i) acc += f(i);
    s_tot[t] = acc;
    __syncthreads();
    for (int off = 1; off < MERGE_THREADS; off <<= 1) {
        const uint32_t add = t >= off ? s_tot[t - off] : 0u;
        __syncthreads();
        s_tot[t] += add;
        __syncthreads();
    }
    uint32_t run = t ? s_tot[t - 1] : 0u;
    for (int64_t i = b; i < e; ++i) {
        out[i] = run;
        run += f(i);
    }
    if (t == MERGE_THREADS - 1) out[n] = s_tot[t];
    __syncthreads();
}

__global__ void __launch_bounds__(MERGE_THREADS)
k_merge_groups_global(const uint32_t *__restrict__ ranges, int64_t n_tiles, uint32_t beta, uint32_t *scratch)
{
    __shared__ uint32_t s_tot[MERGE_THREADS];
    const MergeView m = merge_view(scratch, n_tiles);
    const int64_t T = n_tiles;
    block_exclusive_scan(T, [&](int64_t i) { return ranges[2 * i + 1] - ranges[2 * i]; }, m.S, s_tot);
    for (int64_t i = threadIdx.x; i < T; i += MERGE_THREADS) {
        const uint64_t target = (uint64_t)m.S[i] + beta;
        int64_t lo = i + 1, hi = T;
        if ((uint64_t)m.S[lo] <= target) {
            // last j in [lo, T] with S(j) <= target
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if ((uint64_t)m.S[mid] <= target) lo = mid;
                else hi = mid - 1;
            }
        }
        m.nxt[i] = (uint32_t)lo;
        m.J0[i] = (uint32_t)lo;
        m.mark[i] = i == 0 ? 1u : 0u;
    }
    __syncthreads();
    uint32_t *J = m.J0, *Jn = m.J1;
    for (int64_t span = 1; span <= T; span <<= 1) {
        for (int64_t i = threadIdx.x; i < T; i += MERGE_THREADS)
            if (m.mark[i] && J[i] < (uint32_t)T) m.mark[J[i]] = 1u;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < T; i += MERGE_THREADS) Jn[i] = J[i] < (uint32_t)T ? J[J[i]] : (uint32_t)T;
        __syncthreads();
        uint32_t *tmp = J;
        J = Jn;
        Jn = tmp;
    }
    // group starts in order: the exclusive scan of the marks reuses J0 / J1
    block_exclusive_scan(T, [&](int64_t i) { return m.mark[i]; }, Jn, s_tot);
    for (int64_t i = threadIdx.x; i < T; i += MERGE_THREADS)
        if (m.mark[i]) m.groups[Jn[i]] = make_uint2((uint32_t)i, m.nxt[i]);
    if (threadIdx.x == 0) {
        m.counts[0] = Jn[T];
        m.counts[1] = 0u;
    }
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t a = __shfl_up(v, off);
        if (lane >= off) v += a;
    }
    return v;
}

// Exclusive prefix, over the workgroup, of x (one value per thread, in
// thread order) after `carry`; carry becomes carry + the workgroup's total.
__device__ __forceinline__ uint32_t block_scan_step(uint32_t x, uint32_t &carry, uint32_t *s_tot)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan(x);
    if (lane == 63) s_tot[wave] = incl;
    __syncthreads();
    uint32_t off = carry, all = carry;
    for (int w = 0; w < MERGE_THREADS / 64; ++w) {
        const uint32_t y = s_tot[w];
        off += w < wave ? y : 0u;
        all += y;
    }
    carry = all;
    __syncthreads();
    return off + incl - x;
}

// The grouping of k_merge_groups_global with every array in LDS (up to
// MERGE_LDS_TILES tiles): the loads are staged in LDS and scanned in place
// a workgroup-width chunk at a time, each tile's reach is found by a
// galloping search of the prefix, and the doubling rounds stop once a round
// marks no new group start.  The jump arrays are 16-bit; the second reuses
// the prefix's space, and so do the group starts at the end.
constexpr int MERGE_LDS_TILES = 16384;

__global__ void __launch_bounds__(MERGE_THREADS)
k_merge_groups(const uint32_t *__restrict__ ranges, int T, uint32_t beta, uint32_t *scratch)
{
    __shared__ uint32_t s_S[MERGE_LDS_TILES + 2];
    __shared__ uint16_t s_J[MERGE_LDS_TILES];
    __shared__ uint8_t s_mark[MERGE_LDS_TILES];
    __shared__ uint32_t s_tot[MERGE_THREADS / 64];
    const MergeView m = merge_view(scratch, T);
    const int t = threadIdx.x;
    const uint2 *rg = reinterpret_cast<const uint2 *>(ranges);
#pragma unroll 4
    for (int i = t; i < T; i += MERGE_THREADS) {
        const uint2 r = rg[i];
        s_S[i] = r.y - r.x;
    }
    __syncthreads();
    uint32_t carry = 0;
    for (int base = 0; base < T; base += MERGE_THREADS) {
        const int i = base + t;
        const uint32_t x = i < T ? s_S[i] : 0u;
        const uint32_t ex = block_scan_step(x, carry, s_tot);
        if (i < T) s_S[i] = ex;
    }
    if (t == 0) s_S[T] = carry;
    __syncthreads();
    // reach: the last j in [i + 1, T] with S(j) <= S(i) + beta
    for (int i = t; i < T; i += MERGE_THREADS) {
        const uint64_t target = (uint64_t)s_S[i] + beta;
        int lo = i + 1;
        if ((uint64_t)s_S[lo] <= target) {
            int step = 1, hi;
            for (;;) {
                const int nx = lo + step;
                if (nx > T || (uint64_t)s_S[nx] > target) {
                    hi = min(nx, T + 1) - 1;
                    break;
                }
                lo = nx;
                step <<= 1;
            }
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if ((uint64_t)s_S[mid] <= target) lo = mid;
                else hi = mid - 1;
            }
        }
        s_J[i] = (uint16_t)lo;
        s_mark[i] = i == 0 ? 1u : 0u;
    }
    __syncthreads();
    uint16_t *J = s_J, *Jn = reinterpret_cast<uint16_t *>(s_S);
    for (int span = 1; span < T; span <<= 1) {
        int fresh = 0;
#pragma unroll 4
        for (int i = t; i < T; i += MERGE_THREADS) {
            const int j = J[i];
            if (s_mark[i] && j < T && !s_mark[j]) {
                s_mark[j] = 1u;
                fresh = 1;
            }
        }
        if (!__syncthreads_or(fresh)) break;
#pragma unroll 4
        for (int i = t; i < T; i += MERGE_THREADS) {
            const int j = J[i];
            Jn[i] = j < T ? J[j] : (uint16_t)T;
        }
        __syncthreads();
        uint16_t *tmp = J;
        J = Jn;
        Jn = tmp;
    }
    // group starts in order; a group ends where the next one starts
    uint16_t *start = s_J;
    __syncthreads();
    carry = 0;
    for (int base = 0; base < T; base += MERGE_THREADS) {
        const int i = base + t;
        const uint32_t x = i < T ? s_mark[i] : 0u;
        const uint32_t pos = block_scan_step(x, carry, s_tot);
        if (x) start[pos] = (uint16_t)i;
    }
    const uint32_t ng = carry;
    __syncthreads();
    for (uint32_t g = t; g < ng; g += MERGE_THREADS)
        m.groups[g] = make_uint2(start[g], g + 1 < ng ? (uint32_t)start[g + 1] : (uint32_t)T);
    if (t == 0) {
        m.counts[0] = ng;
        m.counts[1] = 0u;
    }
}

template <int T, bool DOM>
__global__ void __launch_bounds__(T *T)
k_raster_fwd_m(const gs_splat *__restrict__ splats, int n, const gs_camera *__restrict__ cams, int V,
               const uint32_t *__restrict__ vals, const uint32_t *__restrict__ ranges, float bg0, float bg1,
               float bg2, float *__restrict__ image, float *__restrict__ final_T,
               uint32_t *__restrict__ n_contrib, uint32_t *__restrict__ dominated, uint32_t *merge, int64_t n_tiles)
{
    constexpr int WAVES = T * T / 64;
    __shared__ FwdRec s_rec[WAVES][FWD_SLOTS];
    __shared__ uint32_t s_slot;
    const MergeView m = merge_view(merge, n_tiles);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t ng = m.counts[0];
    uint32_t g = pop_task(m.counts + 1, &s_slot, 1);
    while (g < ng) {
        const uint2 gr = m.groups[g];
        for (uint32_t t = gr.x; t < gr.y; ++t) {
            const WaveCtx w = wave_ctx<T>(cams, V, t, wave, lane, ranges);
            FwdState s = fwd_init(w.inside);
            fwd_walk<DOM, false>(splats + (int64_t)w.vi.v * n, vals, w, w.start, w.end, s_rec[wave], s, nullptr);
            fwd_finish<DOM>(w, s, n, bg0, bg1, bg2, image, final_T, n_contrib, dominated);
        }
        g = pop_task(m.counts + 1, &s_slot, 1);
    }
}

template <int T>
__global__ void __launch_bounds__(T *T)
k_raster_fov_m(const gs_splat *__restrict__ splats, const float4 *__restrict__ lvl, int n,
               const uint8_t *__restrict__ qbound, int L, const gs_camera *__restrict__ cams, int V,
               const uint32_t *__restrict__ vals, const uint32_t *__restrict__ ranges,
               const uint8_t *__restrict__ pix_level, const float *__restrict__ pix_weight, float bg0, float bg1,
               float bg2, float *__restrict__ image, uint32_t *merge, int64_t n_tiles)
{
    constexpr int WAVES = T * T / 64;
    __shared__ FovRec s_rec[WAVES][FOV_SLOTS];
    __shared__ uint32_t s_slot;
    const MergeView m = merge_view(merge, n_tiles);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t ng = m.counts[0];
    uint32_t g = pop_task(m.counts + 1, &s_slot, 1);
    while (g < ng) {
        const uint2 gr = m.groups[g];
        for (uint32_t t = gr.x; t < gr.y; ++t) {
            const WaveCtx w = wave_ctx<T>(cams, V, t, wave, lane, ranges);
            const FovPix f = fov_pix(w, pix_level, pix_weight);
            FovState s = fov_init(w.inside, f.two);
            fov_walk<false>(splats, lvl, n, qbound, L, vals, w, f, w.start, w.end, s_rec[wave], s, nullptr);
            fov_finish(w, f, s, bg0, bg1, bg2, image);
        }
        g = pop_task(m.counts + 1, &s_slot, 1);
    }
}

// ---------------------------------------------------------------------------
// Reverse of the forward compositing.  Per pixel, back to front from its last
// blended splat: T_i = T_(i+1) / (1 - alpha_i) starting from final_T, and the
// light behind i (including the background) is accumulated on the way, so
//   dL/dc_i = g alpha_i T_i,  dL/dalpha_i = sum_ch g (c_i T_i - B_i / (1 - alpha_i)).
// The tile's list is walked in chunks of 64 positions by all its waves
// together.  Gradients of one splat are summed over each 16-lane row of a
// wave with DPP reduce-scatters, then over rows and the tile's waves in LDS,
// and leave the tile as one float atomic per quantity per chunk.
struct BwdRec {
    float4 a, b, c;   // forward record (identical decisions)
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

// Sum over each octet of lanes (8 k .. 8 k + 7), in every lane of the octet:
// quad exchanges, then the half-row mirror (lane i <-> 7 - i within 8).
__device__ __forceinline__ float octet_sum(float x)
{
    x += dpp_f<0xB1>(x);   // quad_perm [1,0,3,2]
    x += dpp_f<0x4E>(x);   // quad_perm [2,3,0,1]
    x += dpp_f<0x141>(x);  // row_half_mirror
    return x;
}

template <int T>
__global__ void __launch_bounds__(T *T) __attribute__((amdgpu_waves_per_eu(5)))
k_raster_bwd(const gs_splat *__restrict__ splats, int n, const gs_camera *__restrict__ cams, int V,
             const uint32_t *__restrict__ vals, const uint32_t *__restrict__ ranges, float bg0,
             float bg1, float bg2, const float *__restrict__ final_T,
             const uint32_t *__restrict__ n_contrib, const float *__restrict__ dL_dimage,
             gs_splat_grad *__restrict__ grads)
{
    constexpr int WAVES = T * T / 64;
    constexpr int SUB = T / 8;
    constexpr int NG = 9;  // sums of w, w dx, w dy, w dx^2, w dx dy, w dy^2, colour r, g, b
    __shared__ BwdRec s_rec[WAVES][64];
    // (w, alpha T) of 8 records x 64 pixels per wave; record r's row is
    // rotated by r pairs so that the regrouped reads (lanes 8 r + y, column
    // x) of the 8 records fall in different LDS banks
    __shared__ float2 s_m[WAVES][8][64];
    __shared__ float s_grad[NG][73];  // row stride 73: the flush reads 9 rows of 7 positions with few bank conflicts
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
    for (int q = threadIdx.x; q < NG * 73; q += T * T) (&s_grad[0][0])[q] = 0.f;
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
    // light from behind the current splat enters dL/dalpha only as
    // sum_ch g_ch B_ch: that one sum is carried, starting with the background
    float gB = Tr * fmaf(g0, bg0, fmaf(g1, bg1, g2 * bg2));
    // dL/dimage of the 8 pixels of row (lane & 7) of the wave's block, for
    // the per-record row sums
    float grow0[8], grow1[8], grow2[8];
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        const int src = 8 * (lane & 7) + x;
        grow0[x] = __shfl(g0, src);
        grow1[x] = __shfl(g1, src);
        grow2[x] = __shfl(g2, src);
    }
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
            rec.a = rec.b = rec.c = make_float4(0.f, 0.f, 0.f, 0.f);
            if (pos <= p1 && pos <= (int64_t)maxnc) {
                const uint32_t idx = start + (uint32_t)(pos - 1);
                const uint32_t id = vals[idx];
                const float4 *s4 = reinterpret_cast<const float4 *>(splats + vbase + id);
                const float4 s0 = s4[0], s1 = s4[1], s2 = s4[2];
                const FwdRec f = make_rec(s0, s1, s2, (uint32_t)pos, id);
                rec.a = f.a;
                rec.b = f.b;
                rec.c = f.c;
                keep = reaches_rect(s0.x, s0.y, s0.z, s0.w, s1.x, qmax_of(s1.y), rx0, rx1, ry0, ry1);
            }
            const uint64_t msk = ballot64(keep);
            const int cnt = __popcll(msk);
            // padded to a multiple of 8 with null records (an infinite alpha
            // threshold: no pixel takes them), walked back to front in groups of 8
            const int cnt8 = (cnt + 7) & ~7;
            if (keep) s_rec[wave][__popcll(msk & lanemask_lt())] = rec;
            if (lane >= cnt && lane < cnt8) {
                BwdRec z;
                z.a = z.b = z.c = make_float4(0.f, 0.f, 0.f, 0.f);
                z.b.z = __builtin_inff();
                s_rec[wave][lane] = z;
            }
            wave_lds_sync();
            for (int j0 = cnt8 - 8; j0 >= 0; j0 -= 8) {
                // (1) lanes are pixels: per record w = alpha dL/dalpha and the
                // blend weight alpha T into the wave's LDS block.  Branch-free:
                // every lane evaluates, selects take the forward's decisions.
                bool any = false;
#pragma unroll 2
                for (int r = 7; r >= 0; --r) {
                    const int j = j0 + r;
                    const float4 a = s_rec[wave][j].a, b = s_rec[wave][j].b;
                    const uint32_t ppos = __float_as_uint(b.w);
                    const float e2 = pair_e2(a, b, fpx, fpy);
                    const bool contrib = ppos <= nc && e2 >= b.z;
                    const float4 c = s_rec[wave][j].c;
                    const float araw = fast_exp2(e2);
                    const float alpha = fminf(GS_ALPHA_MAX, araw);
                    const float ioma = __builtin_amdgcn_rcpf(1.0f - alpha);
                    const float Tn = Tr * ioma;
                    const float wT = contrib ? alpha * Tn : 0.f;
                    const float gc = fmaf(g0, c.x, fmaf(g1, c.y, g2 * c.z));
                    const float dLda = fmaf(gc, Tn, -gB * ioma);
                    gB = fmaf(gc, wT, gB);
                    Tr = contrib ? Tn : Tr;
                    const float w = (contrib && araw <= GS_ALPHA_MAX) ? alpha * dLda : 0.f;
                    s_m[wave][r][(lane + r) & 63] = make_float2(w, wT);
                    any = any || contrib;
                }
                if (ballot64(any) == 0) continue;  // none of the 8 reaches the wave's pixels
                wave_lds_sync();
                // (2) lane 8 r + y sums record j0 + r over pixel row y in
                // registers: w and its moments in the pixel offsets (x, y)
                // from the block corner, colour as g alpha T.  The 8 rows
                // of a record add up by DPP within the lane octet; one lane
                // per record moves the moments to the record's mean,
                //   sum w dx = Mx - u M, sum w dx^2 = (Mxx - u Mx) - u sum w dx,
                //   sum w dx dy = (Mxy - v Mx) - u sum w dy, ...
                // with (u, v) the mean's offset from the corner, and adds the
                // nine sums to the tile's slots of the record's list position
                {
                    const int r = lane >> 3, y = lane & 7;
                    float M0 = 0.f, Mx = 0.f, Mxx = 0.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
#pragma unroll
                    for (int x = 0; x < 8; ++x) {
                        const float2 m = s_m[wave][r][(8 * y + x + r) & 63];
                        M0 += m.x;
                        Mx = fmaf(m.x, (float)x, Mx);
                        Mxx = fmaf(m.x, (float)(x * x), Mxx);
                        C0 = fmaf(grow0[x], m.y, C0);
                        C1 = fmaf(grow1[x], m.y, C1);
                        C2 = fmaf(grow2[x], m.y, C2);
                    }
                    const float fy = (float)y;
                    float S[NG] = {M0, Mx, fy * M0, Mxx, fy * Mx, fy * fy * M0, C0, C1, C2};
#pragma unroll
                    for (int k = 0; k < NG; ++k) S[k] = octet_sum(S[k]);
                    if (y == 0 && j0 + r < cnt) {
                        const float4 a = s_rec[wave][j0 + r].a;
                        const int q = (int)(__float_as_uint(s_rec[wave][j0 + r].b.w) - (uint32_t)p0);
                        const float u = a.x - rx0, v = a.y - ry0;
                        const float sdx = fmaf(-u, S[0], S[1]), sdy = fmaf(-v, S[0], S[2]);
                        S[3] = fmaf(-u, sdx, fmaf(-u, S[1], S[3]));
                        S[4] = fmaf(-u, sdy, fmaf(-v, S[1], S[4]));
                        S[5] = fmaf(-v, sdy, fmaf(-v, S[2], S[5]));
                        S[1] = sdx;
                        S[2] = sdy;
#pragma unroll
                        for (int k = 0; k < NG; ++k) atomicAdd(&s_grad[k][q], S[k]);
                    }
                }
                wave_lds_sync();  // the next group rewrites the wave's LDS block
            }
        }
        __syncthreads();
        // the tile's sums of this chunk leave with global atomics: with q =
        // the Mahalanobis form and dL/dq = -w / 2,
        //   dL/dmean = (A S_wdx + B S_wdy, B S_wdx + C S_wdy),
        //   dL/d(A, B, C) = (-S_wdx2 / 2, -S_wdxdy, -S_wdy2 / 2),
        //   dL/dopacity = S_w / opacity.
        // Lane 9 i + k of an instruction adds quantity k of position 7 rnd + i,
        // so the lanes of one position add to one 36-byte run of its
        // gradient record; the ten rounds of 7 positions go round the waves
        {
            // recomputed per chunk rather than held across the record loop
            int ln = lane;
            asm volatile("" : "+v"(ln));
            const int pl = (ln * 57) >> 9;  // ln / 9 for ln < 64
            const int k = ln - 9 * pl;
            for (int rnd = wave; rnd < 10; rnd += WAVES) {
                const int q = 7 * rnd + pl;
                if (ln < 63 && q < 64) {
                    // quantities 2..4 (the conic) come from the second moments 3..5
                    const float v = s_grad[k >= 2 && k <= 4 ? k + 1 : k][q];
                    const float S0 = s_grad[0][q], S1 = s_grad[1][q], S2 = s_grad[2][q];
                    float out = k == 2 || k == 4 ? -0.5f * v : (k == 3 ? -v : v);
                    if (k == 0 || k == 1 || k == 5) {
                        out = 0.f;
                        if (S0 != 0.f || S1 != 0.f || S2 != 0.f) {
                            const float *sp = reinterpret_cast<const float *>(splats + vbase + s_id[q]);
                            const float2 ab = *reinterpret_cast<const float2 *>(sp + 2);
                            const float2 co = *reinterpret_cast<const float2 *>(sp + 4);
                            out = k == 0 ? fmaf(ab.x, S1, ab.y * S2)
                                         : (k == 1 ? fmaf(ab.y, S1, co.x * S2) : S0 * __builtin_amdgcn_rcpf(co.y));
                        }
                    }
                    s_grad[k][q] = 0.f;
                    if (out != 0.f) atomicAdd(reinterpret_cast<float *>(grads + vbase + s_id[q]) + k, out);
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Reverse of the foveated compositing.  Per pixel, each accumulator (level lo
// with weight 1 - w, level lo + 1 with weight w in a band) is walked back to
// front from its last blended splat exactly as the plain reverse, with that
// level's opacity and colour and the level filter.  Gradients with respect to
// mean and conic are summed over the levels; colour and opacity gradients
// are kept per level.  The tile's waves walk the list in chunks of 64
// positions together and sum per splat in LDS before one atomic per quantity.
struct FovBwdRec {
    float4 a, b;      // mean x, mean y, qa, qb | qc, 0, quality bound, position
    float4 raw;       // conic A, B, C, unused
    float4 lv[MAXL];  // per level r, g, b, opacity
};

template <int T>
__global__ void __launch_bounds__(T *T)
k_raster_fov_bwd(const gs_splat *__restrict__ splats, const float4 *__restrict__ lvl, int n,
                 const uint8_t *__restrict__ qbound, int L, const gs_camera *__restrict__ cams, int V,
                 const uint32_t *__restrict__ vals, const uint32_t *__restrict__ ranges,
                 const uint8_t *__restrict__ pix_level, const float *__restrict__ pix_weight, float bg0,
                 float bg1, float bg2, const float2 *__restrict__ final_T2, const uint2 *__restrict__ n_contrib2,
                 const float *__restrict__ dL_dimage, gs_splat_grad *__restrict__ grads,
                 float4 *__restrict__ lvl_grads)
{
    constexpr int WAVES = T * T / 64;
    constexpr int NG = 5 + 4 * MAXL;  // mean x, y, conic A, B, C; per level r, g, b, opacity
    __shared__ FovBwdRec s_rec[WAVES][64];
    __shared__ float s_grad[NG][64];
    __shared__ uint32_t s_id[64];
    __shared__ uint32_t s_maxnc;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const WaveCtx w = wave_ctx<T>(cams, V, blockIdx.x, wave, lane, ranges);
    const FovPix f = fov_pix(w, pix_level, pix_weight);
    const int64_t vbase = (int64_t)w.vi.v * n;
    const float cx = w.rx0 + 3.5f, cy = w.ry0 + 3.5f;
    const float pu = (float)(lane & 7) - 3.5f, pv = (float)(lane >> 3) - 3.5f;

    if (threadIdx.x == 0) s_maxnc = 0;
    for (int q = threadIdx.x; q < NG * 64; q += T * T) (&s_grad[0][0])[q] = 0.f;
    uint32_t nca = 0, ncb = 0;
    float Ta = 1.0f, Tb = 1.0f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
    if (w.inside) {
        const float2 ft = final_T2[w.pix];
        const uint2 nc = n_contrib2[w.pix];
        Ta = ft.x;
        Tb = ft.y;
        nca = nc.x;
        ncb = f.two ? nc.y : 0u;
        const int64_t plane = (int64_t)w.vi.W * w.vi.H;
        const float *gi = dL_dimage + 3 * w.vi.pix_off + (int64_t)w.py * w.vi.W + w.px;
        g0 = gi[0];
        g1 = gi[plane];
        g2 = gi[2 * plane];
    }
    const float wa = f.two ? 1.0f - f.wup : 1.0f, wb = f.two ? f.wup : 0.0f;
    const float ga0 = g0 * wa, ga1 = g1 * wa, ga2 = g2 * wa;
    const float gb0 = g0 * wb, gb1 = g1 * wb, gb2 = g2 * wb;
    // light from behind the current splat, starting with the background
    float Ba0 = Ta * bg0, Ba1 = Ta * bg1, Ba2 = Ta * bg2;
    float Bb0 = Tb * bg0, Bb1 = Tb * bg1, Bb2 = Tb * bg2;
    const int lob = f.lo < MAXL ? f.lo : MAXL - 1;  // index of level lo + 1
    int wave_hi = w.inside ? f.lo + (f.two ? 1 : 0) : 0;
    uint32_t maxnc = max(nca, ncb);
    for (int off = 32; off > 0; off >>= 1) {
        maxnc = max(maxnc, (uint32_t)__shfl_xor((int)maxnc, off));
        wave_hi = max(wave_hi, __shfl_xor(wave_hi, off));
    }
    __syncthreads();
    if (lane == 0) atomicMax(&s_maxnc, maxnc);
    __syncthreads();
    const uint32_t maxnc_tile = s_maxnc;

    for (int64_t p1 = maxnc_tile; p1 >= 1; p1 -= 64) {
        const int64_t p0 = p1 - 63 >= 1 ? p1 - 63 : 1;
        if (threadIdx.x < 64) {
            const int64_t pos = p0 + threadIdx.x;
            s_id[threadIdx.x] = pos <= p1 ? vals[w.start + (uint32_t)(pos - 1)] : 0u;
        }
        if ((uint32_t)p0 <= maxnc) {
            const int64_t pos = p0 + lane;
            bool keep = false;
            // the record is fully defined on every lane before the cull decision
            FovBwdRec rec;
            rec.a = rec.b = rec.raw = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int t = 0; t < MAXL; ++t) rec.lv[t] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (pos <= p1 && pos <= (int64_t)maxnc) {
                const uint32_t id = vals[w.start + (uint32_t)(pos - 1)];
                const int m = qbound[id];
                const float4 *s4 = reinterpret_cast<const float4 *>(splats + vbase + id);
                const float4 s0 = s4[0], s1 = s4[1];
                rec.a = make_float4(s0.x, s0.y, NEG_HALF_LOG2E * s0.z, -GS_LOG2E * s0.w);
                rec.b = make_float4(NEG_HALF_LOG2E * s1.x, 0.0f, __int_as_float(m), __uint_as_float((uint32_t)pos));
                rec.raw = make_float4(s0.z, s0.w, s1.x, 0.0f);
                const float4 *lp = lvl + (vbase + id) * L;
#pragma unroll
                for (int t = 0; t < MAXL; ++t)
                    if (t < L) rec.lv[t] = lp[t];
                keep = m >= f.wave_lo &&
                       reaches_rect(s0.x, s0.y, s0.z, s0.w, s1.x, 9.001f, w.rx0, w.rx1, w.ry0, w.ry1);
            }
            const uint64_t msk = ballot64(keep);
            if (keep) s_rec[wave][__popcll(msk & lanemask_lt())] = rec;
            wave_lds_sync();
            const int cnt = __popcll(msk);
            for (int j = cnt - 1; j >= 0; --j) {
                const float4 a = s_rec[wave][j].a, b = s_rec[wave][j].b;
                const uint32_t ppos = __float_as_uint(b.w);
                const int m = __float_as_int(b.z);
                // the forward's falloff, bit for bit: the same expansion
                // about the block centre
                const Quad qd = quad_about(a.x, a.y, a.z, a.w, b.x, cx, cy);
                const float p2 = quad_eval(qd.F, qd.D, qd.E, a.z, a.w, b.x, pu, pv);
                const float G = fast_exp2(p2);
                const bool incl = p2 >= EXTENT_LOG2;
                const float4 raw = s_rec[wave][j].raw;
                const float dx = w.fpx - a.x, dy = w.fpy - a.y;
                float dLdq = 0.f;
                float ca0 = 0.f, ca1 = 0.f, ca2 = 0.f, cao = 0.f;  // level lo: colour, opacity
                float cb0 = 0.f, cb1 = 0.f, cb2 = 0.f, cbo = 0.f;  // level lo + 1
                bool ca = false, cb = false;
                {
                    const float4 lv = s_rec[wave][j].lv[f.lo - 1];
                    const float araw = lv.w * G;
                    const float alpha = fminf(GS_ALPHA_MAX, araw);
                    if (ppos <= nca && incl && m >= f.lo && alpha >= GS_ALPHA_MIN) {
                        ca = true;
                        const float oma = 1.0f - alpha;
                        const float ioma = __builtin_amdgcn_rcpf(oma);
                        Ta = Ta * ioma;
                        const float wT = alpha * Ta;
                        ca0 = ga0 * wT;
                        ca1 = ga1 * wT;
                        ca2 = ga2 * wT;
                        const float dLda = ga0 * (lv.x * Ta - Ba0 * ioma) + ga1 * (lv.y * Ta - Ba1 * ioma) +
                                           ga2 * (lv.z * Ta - Ba2 * ioma);
                        Ba0 = fmaf(lv.x, wT, Ba0);
                        Ba1 = fmaf(lv.y, wT, Ba1);
                        Ba2 = fmaf(lv.z, wT, Ba2);
                        if (araw <= GS_ALPHA_MAX) {
                            cao = dLda * G;
                            dLdq += -0.5f * alpha * dLda;
                        }
                    }
                }
                if (f.two) {
                    const float4 lv = s_rec[wave][j].lv[lob];
                    const float araw = lv.w * G;
                    const float alpha = fminf(GS_ALPHA_MAX, araw);
                    if (ppos <= ncb && incl && m >= f.lo + 1 && alpha >= GS_ALPHA_MIN) {
                        cb = true;
                        const float oma = 1.0f - alpha;
                        const float ioma = __builtin_amdgcn_rcpf(oma);
                        Tb = Tb * ioma;
                        const float wT = alpha * Tb;
                        cb0 = gb0 * wT;
                        cb1 = gb1 * wT;
                        cb2 = gb2 * wT;
                        const float dLda = gb0 * (lv.x * Tb - Bb0 * ioma) + gb1 * (lv.y * Tb - Bb1 * ioma) +
                                           gb2 * (lv.z * Tb - Bb2 * ioma);
                        Bb0 = fmaf(lv.x, wT, Bb0);
                        Bb1 = fmaf(lv.y, wT, Bb1);
                        Bb2 = fmaf(lv.z, wT, Bb2);
                        if (araw <= GS_ALPHA_MAX) {
                            cbo = dLda * G;
                            dLdq += -0.5f * alpha * dLda;
                        }
                    }
                }
                if (ballot64(ca || cb) == 0) continue;
                const int q = (int)(ppos - (uint32_t)p0);
                float gA = dLdq * dx * dx, gB = dLdq * 2.0f * dx * dy, gC = dLdq * dy * dy;
                float gmx = -2.0f * dLdq * (raw.x * dx + raw.y * dy);
                float gmy = -2.0f * dLdq * (raw.y * dx + raw.z * dy);
                gmx = wave_total_63(gmx);
                gmy = wave_total_63(gmy);
                gA = wave_total_63(gA);
                gB = wave_total_63(gB);
                gC = wave_total_63(gC);
                if (lane == 63) {
                    atomicAdd(&s_grad[0][q], gmx);
                    atomicAdd(&s_grad[1][q], gmy);
                    atomicAdd(&s_grad[2][q], gA);
                    atomicAdd(&s_grad[3][q], gB);
                    atomicAdd(&s_grad[4][q], gC);
                }
                // per level: the lanes whose lower level (or next level) it is
                for (int t = f.wave_lo; t <= wave_hi && t <= MAXL; ++t) {
                    float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f;
                    if (ca && f.lo == t) {
                        v0 += ca0;
                        v1 += ca1;
                        v2 += ca2;
                        v3 += cao;
                    }
                    if (cb && f.lo + 1 == t) {
                        v0 += cb0;
                        v1 += cb1;
                        v2 += cb2;
                        v3 += cbo;
                    }
                    if (ballot64(v0 != 0.f || v1 != 0.f || v2 != 0.f || v3 != 0.f) == 0) continue;
                    v0 = wave_total_63(v0);
                    v1 = wave_total_63(v1);
                    v2 = wave_total_63(v2);
                    v3 = wave_total_63(v3);
                    if (lane == 63) {
                        const int k0 = 5 + 4 * (t - 1);
                        atomicAdd(&s_grad[k0][q], v0);
                        atomicAdd(&s_grad[k0 + 1][q], v1);
                        atomicAdd(&s_grad[k0 + 2][q], v2);
                        atomicAdd(&s_grad[k0 + 3][q], v3);
                    }
                }
            }
        }
        __syncthreads();
        // the tile's sums of this chunk leave with one atomic per quantity
        for (int qq = threadIdx.x; qq < NG * 64; qq += T * T) {
            const int k = qq >> 6, jj = qq & 63;
            const float v = s_grad[k][jj];
            if (v != 0.f) {
                const int64_t e = vbase + s_id[jj];
                if (k < 5) {
                    atomicAdd(reinterpret_cast<float *>(grads + e) + k, v);
                } else {
                    const int t = (k - 5) >> 2, c = (k - 5) & 3;
                    if (t < L) atomicAdd(reinterpret_cast<float *>(lvl_grads + e * L + t) + c, v);
                }
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

// Level and blend weight of pixel (x, y) of a view: the eccentricity is the
// angle between the pixel's ray and the gaze ray (through the gaze pixel);
// the level is the first ring the pixel lies inside, and within a ring's
// blend band the weight of the next level rises linearly from 0 to 1.
__device__ __forceinline__ void fovea_level(const gs_camera &c, const gs_fovea &f, int L, int x, int y, int &lo,
                                            float &w)
{
    const float ecc = pixel_ecc_deg(c, f.gaze_x, f.gaze_y, x, y);
    lo = 1;
    w = 0.0f;
    const float hb = 0.5f * f.band_deg;
    for (int j = 0; j < L - 1; ++j) {
        const float e0 = f.ring_deg[j] - hb, e1 = f.ring_deg[j] + hb;
        if (ecc < e0) break;
        if (ecc < e1) {
            lo = j + 1;
            w = (ecc - e0) / f.band_deg;
            break;
        }
        lo = j + 2;
    }
}

// One workgroup per strip of G = 64 / T horizontally adjacent tiles of one
// view (64 pixels wide, T rows): its four waves take the strip's rows in
// turn, a lane per pixel, so each row's levels and weights are written as 64
// contiguous pixels.  Each lane keeps the lowest level and the highest level
// with non-zero weight of its column; the T lanes of a tile's columns and the
// four waves then give the tile's (tile_level[2 g], tile_level[2 g + 1]).
template <int T>
__global__ void __launch_bounds__(256)
k_fovea_prep(const gs_camera *__restrict__ cams, int V, int L, FovArgs fa, uint8_t *__restrict__ pix_level,
             float *__restrict__ pix_weight, uint8_t *__restrict__ tile_level)
{
    constexpr int G = 64 / T;
    static_assert(G * T == 64 && T >= 4, "a strip is 64 pixels wide");
    __shared__ int s_lo[4][G], s_hi[4][G];
    // the strip's view: strips are numbered view by view, row-major within one
    const int64_t gs = blockIdx.x;
    int v = 0, W = 0, H = 0, ntx = 0;
    int64_t soff = 0, toff = 0, poff = 0;
    for (;; ++v) {
        W = cams[v].width;
        H = cams[v].height;
        ntx = div_up(W, T);
        const int nty = div_up(H, T);
        const int64_t ns = (int64_t)div_up(ntx, G) * nty;
        if (gs < soff + ns || v == V - 1) break;
        soff += ns;
        toff += (int64_t)ntx * nty;
        poff += (int64_t)W * H;
    }
    const int nsx = div_up(ntx, G);
    const int sx = (int)((gs - soff) % nsx), ty = (int)((gs - soff) / nsx);
    const int col = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x = sx * 64 + col;
    int lo = 255, hi = 0;
    for (int r = wave; r < T; r += 4) {
        const int y = ty * T + r;
        if (x < W && y < H) {
            int l;
            float w;
            fovea_level(cams[v], fa.f[v], L, x, y, l, w);
            const int64_t p = poff + (int64_t)y * W + x;
            pix_level[p] = (uint8_t)l;
            pix_weight[p] = w;
            lo = min(lo, l);
            hi = max(hi, l + (w > 0.0f ? 1 : 0));
        }
    }
    for (int off = T / 2; off > 0; off >>= 1) {
        lo = min(lo, __shfl_xor(lo, off));
        hi = max(hi, __shfl_xor(hi, off));
    }
    if (col % T == 0) {
        s_lo[wave][col / T] = lo;
        s_hi[wave][col / T] = hi;
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < G && sx * G + t < ntx) {
        int a = s_lo[0][t], b = s_hi[0][t];
        for (int q = 1; q < 4; ++q) {
            a = min(a, s_lo[q][t]);
            b = max(b, s_hi[q][t]);
        }
        const int64_t gt = toff + (int64_t)ty * ntx + sx * G + t;
        tile_level[2 * gt] = (uint8_t)a;
        tile_level[2 * gt + 1] = (uint8_t)b;
    }
}

}  // namespace

namespace {

// Persistent grid: as many workgroups per CU as its thread slots hold, on
// every CU.  No workgroup of a persistent compositor waits on another, so
// workgroups beyond what registers or LDS let reside only start late and find
// the task list drained; asking for fewer (the occupancy query's answer is
// conservative here) would leave slots idle for the whole launch.
template <class K>
unsigned persistent_blocks(K kernel, int threads)
{
    (void)kernel;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 2048;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxThreadsPerMultiProcessor, dev) != hipSuccess ||
        per_cu < threads)
        per_cu = 2048;
    return (unsigned)(cus * std::max(1, per_cu / threads));
}

void launch_merge_groups(const uint32_t *ranges, int64_t n_tiles, const MergeArgs *ma, hipStream_t st)
{
    if (n_tiles <= MERGE_LDS_TILES)
        hipLaunchKernelGGL(k_merge_groups, dim3(1), dim3(MERGE_THREADS), 0, st, ranges, (int)n_tiles, ma->beta,
                           ma->scratch);
    else
        hipLaunchKernelGGL(k_merge_groups_global, dim3(1), dim3(MERGE_THREADS), 0, st, ranges, n_tiles, ma->beta,
                           ma->scratch);
}

hipError_t build_queue(const uint32_t *ranges, int64_t n_tiles, int T, const RasterQueueArgs &qa, RasterQueue &q,
                       hipStream_t st)
{
    q.counts = qa.counts;
    q.heavy = reinterpret_cast<uint2 *>(qa.heavy);
    q.light = reinterpret_cast<uint2 *>(qa.light);
    q.merge_cnt = qa.merge_cnt;
    q.part = reinterpret_cast<float4 *>(qa.part);
    q.heavy_cap = qa.heavy_cap;
    q.light_cap = qa.light_cap;
    q.beta = qa.beta;
    // split tiles are the heavy ones; without splitting, runs longer than
    // heavy_min go first (0: plain tile order)
    q.heavy_min = qa.beta ? qa.beta : (qa.heavy_min ? qa.heavy_min : 0xFFFFFFFFu);
    q.grab = qa.grab ? qa.grab : 1;
    q.n_tiles = n_tiles;
    hipError_t e = launch_fill_u32(q.counts, 0u, 4, st);
    if (e != hipSuccess) return e;
    const unsigned blocks = (unsigned)((n_tiles + 255) / 256);
    (void)T;
    hipLaunchKernelGGL(k_build_queue, dim3(blocks), dim3(256), 0, st, ranges, n_tiles, q);
    return hipGetLastError();
}

}  // namespace

uint64_t raster_queue_heavy_cap(int64_t n_tiles, int T, uint64_t cap, uint32_t beta)
{
    (void)T;
    return (uint64_t)n_tiles + (beta ? cap / beta + 1 : 0);
}

hipError_t launch_raster_fwd(const gs_splat *splats, int n, const gs_camera *cams_dev, int V, int T,
                             int64_t n_tiles, const uint32_t *vals, const uint32_t *ranges,
                             const float bg[3], float *image, float *final_T, uint32_t *n_contrib,
                             uint32_t *dominated, uint64_t *stats, const RasterQueueArgs *qa, hipStream_t st,
                             const MergeArgs *ma)
{
    if (n_tiles == 0) return hipSuccess;
    hipError_t e;
    if (dominated && (e = launch_fill_u32(dominated, 0u, (uint64_t)V * n, st)) != hipSuccess) return e;
    unsigned long long *sp = reinterpret_cast<unsigned long long *>(stats);
    if (ma && !qa && !stats) {
        launch_merge_groups(ranges, n_tiles, ma, st);
#define GS_RM(TS, DM)                                                                                  \
    {                                                                                                  \
        static unsigned blocks = 0;                                                                    \
        if (!blocks) blocks = persistent_blocks(k_raster_fwd_m<TS, DM>, TS * TS);                     \
        hipLaunchKernelGGL((k_raster_fwd_m<TS, DM>), dim3(blocks), dim3(TS * TS), 0, st, splats, n, cams_dev, \
                           V, vals, ranges, bg[0], bg[1], bg[2], image, final_T, n_contrib, dominated,  \
                           ma->scratch, n_tiles);                                                      \
    }
        if (dominated) {
            switch (T) {
            case 8: GS_RM(8, true); break;
            case 16: GS_RM(16, true); break;
            default: GS_RM(32, true); break;
            }
        } else {
            switch (T) {
            case 8: GS_RM(8, false); break;
            case 16: GS_RM(16, false); break;
            default: GS_RM(32, false); break;
            }
        }
#undef GS_RM
        return hipGetLastError();
    }
    if (qa && !stats) {
        RasterQueue q;
        if ((e = build_queue(ranges, n_tiles, T, *qa, q, st)) != hipSuccess) return e;
#define GS_RQ(TS, DM)                                                                                  \
    {                                                                                                  \
        static unsigned blocks = 0;                                                                    \
        if (!blocks) blocks = persistent_blocks(k_raster_fwd_q<TS, DM>, TS * TS);                     \
        hipLaunchKernelGGL((k_raster_fwd_q<TS, DM>), dim3(blocks), dim3(TS * TS), 0, st, splats, n, cams_dev, \
                           V, vals, ranges, bg[0], bg[1], bg[2], image, final_T, n_contrib, dominated, q); \
    }
        if (dominated) {
            switch (T) {
            case 8: GS_RQ(8, true); break;
            case 16: GS_RQ(16, true); break;
            default: GS_RQ(32, true); break;
            }
        } else {
            switch (T) {
            case 8: GS_RQ(8, false); break;
            case 16: GS_RQ(16, false); break;
            default: GS_RQ(32, false); break;
            }
        }
#undef GS_RQ
        return hipGetLastError();
    }
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

hipError_t launch_raster_fov_bwd(const gs_splat *splats, const float *lvl_rgba, int n, const uint8_t *qbound,
                                 int n_levels, const gs_camera *cams_dev, int V, int T, int64_t n_tiles,
                                 const uint32_t *vals, const uint32_t *ranges, const uint8_t *pix_level,
                                 const float *pix_weight, const float bg[3], const float *final_T2,
                                 const uint32_t *n_contrib2, const float *dL_dimage, gs_splat_grad *grads,
                                 float *lvl_grads, hipStream_t st)
{
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(grads), 0u, (uint64_t)V * n * 12, st);
    if (e != hipSuccess) return e;
    e = launch_fill_u32(reinterpret_cast<uint32_t *>(lvl_grads), 0u, (uint64_t)V * n * n_levels * 4, st);
    if (e != hipSuccess || n_tiles == 0) return e;
    const float4 *lv = reinterpret_cast<const float4 *>(lvl_rgba);
    const float2 *fT2 = reinterpret_cast<const float2 *>(final_T2);
    const uint2 *nc2 = reinterpret_cast<const uint2 *>(n_contrib2);
    float4 *lg = reinterpret_cast<float4 *>(lvl_grads);
#define GS_FB(TS)                                                                                      \
    hipLaunchKernelGGL((k_raster_fov_bwd<TS>), dim3((unsigned)n_tiles), dim3(TS * TS), 0, st, splats, lv, n,   \
                       qbound, n_levels, cams_dev, V, vals, ranges, pix_level, pix_weight, bg[0], bg[1], bg[2], \
                       fT2, nc2, dL_dimage, grads, lg);
    switch (T) {
    case 8: GS_FB(8); break;
    case 16: GS_FB(16); break;
    default: GS_FB(32); break;
    }
#undef GS_FB
    return hipGetLastError();
}

hipError_t launch_fovea_prep(const gs_camera *cams_host, const gs_camera *cams_dev, const gs_fovea *fov_host,
                             int n_eyes, int T, int n_levels, int64_t n_pixels, int64_t n_tiles,
                             uint8_t *pix_level, float *pix_weight, uint8_t *tile_level, hipStream_t st)
{
    (void)n_pixels;
    if (n_tiles == 0) return hipSuccess;
    FovArgs fa;
    for (int i = 0; i < 8; ++i) fa.f[i] = fov_host[i < n_eyes ? i : 0];
    // strips of 64 / T tiles, view by view
    const int Tc = T == 8 || T == 16 ? T : 32;
    int64_t strips = 0;
    for (int v = 0; v < n_eyes; ++v) {
        const int64_t ntx = (cams_host[v].width + Tc - 1) / Tc, nty = (cams_host[v].height + Tc - 1) / Tc;
        strips += (ntx + 64 / Tc - 1) / (64 / Tc) * nty;
    }
    if (strips == 0) return hipSuccess;
#define GS_FP(TS)                                                                                      \
    hipLaunchKernelGGL((k_fovea_prep<TS>), dim3((unsigned)strips), dim3(256), 0, st, cams_dev, n_eyes,     \
                       n_levels, fa, pix_level, pix_weight, tile_level)
    switch (T) {
    case 8: GS_FP(8); break;
    case 16: GS_FP(16); break;
    default: GS_FP(32); break;
    }
#undef GS_FP
    return hipGetLastError();
}

hipError_t launch_raster_fov(const gs_splat *splats, const float *lvl_rgba, int n,
                             const uint8_t *qbound, int n_levels, const gs_camera *cams_dev, int V,
                             int T, int64_t n_tiles, const uint32_t *vals, const uint32_t *ranges,
                             const uint8_t *pix_level, const float *pix_weight, const float bg[3],
                             float *image, uint64_t *stats, float *final_T2, uint32_t *n_contrib2,
                             const RasterQueueArgs *qa, hipStream_t st, const MergeArgs *ma)
{
    if (n_tiles == 0) return hipSuccess;
    const float4 *lv = reinterpret_cast<const float4 *>(lvl_rgba);
    unsigned long long *sp = reinterpret_cast<unsigned long long *>(stats);
    float2 *fT2 = reinterpret_cast<float2 *>(final_T2);
    uint2 *nc2 = reinterpret_cast<uint2 *>(n_contrib2);
    if (fT2 && nc2) {
        // the reverse pass needs per-accumulator state: one workgroup per tile
#define GS_RK(TS)                                                                                    \
    hipLaunchKernelGGL((k_raster_fov<TS, false, true>), dim3((unsigned)n_tiles), dim3(TS * TS), 0, st,    \
                       splats, lv, n, qbound, n_levels, cams_dev, V, vals, ranges, pix_level, pix_weight,  \
                       bg[0], bg[1], bg[2], image, sp, fT2, nc2);
        switch (T) {
        case 8: GS_RK(8); break;
        case 16: GS_RK(16); break;
        default: GS_RK(32); break;
        }
#undef GS_RK
        return hipGetLastError();
    }
    if (ma && !qa && !stats) {
        launch_merge_groups(ranges, n_tiles, ma, st);
#define GS_RM(TS)                                                                                      \
    {                                                                                                  \
        static unsigned blocks = 0;                                                                    \
        if (!blocks) blocks = persistent_blocks(k_raster_fov_m<TS>, TS * TS);                         \
        hipLaunchKernelGGL((k_raster_fov_m<TS>), dim3(blocks), dim3(TS * TS), 0, st, splats, lv, n, qbound, \
                           n_levels, cams_dev, V, vals, ranges, pix_level, pix_weight, bg[0], bg[1],    \
                           bg[2], image, ma->scratch, n_tiles);                                        \
    }
        switch (T) {
        case 8: GS_RM(8); break;
        case 16: GS_RM(16); break;
        default: GS_RM(32); break;
        }
#undef GS_RM
        return hipGetLastError();
    }
    if (qa && !stats) {
        RasterQueue q;
        hipError_t e;
        if ((e = build_queue(ranges, n_tiles, T, *qa, q, st)) != hipSuccess) return e;
#define GS_RQ(TS)                                                                                      \
    {                                                                                                  \
        static unsigned blocks = 0;                                                                    \
        if (!blocks) blocks = persistent_blocks(k_raster_fov_q<TS>, TS * TS);                         \
        hipLaunchKernelGGL((k_raster_fov_q<TS>), dim3(blocks), dim3(TS * TS), 0, st, splats, lv, n, qbound, \
                           n_levels, cams_dev, V, vals, ranges, pix_level, pix_weight, bg[0], bg[1],    \
                           bg[2], image, q);                                                           \
    }
        switch (T) {
        case 8: GS_RQ(8); break;
        case 16: GS_RQ(16); break;
        default: GS_RQ(32); break;
        }
#undef GS_RQ
        return hipGetLastError();
    }
#define GS_RV(TS)                                                                                    \
    if (stats)                                                                                       \
        hipLaunchKernelGGL((k_raster_fov<TS, true, false>), dim3((unsigned)n_tiles), dim3(TS * TS), 0, st, \
                           splats, lv, n, qbound, n_levels, cams_dev, V, vals, ranges, pix_level,    \
                           pix_weight, bg[0], bg[1], bg[2], image, sp, nullptr, nullptr);            \
    else                                                                                             \
        hipLaunchKernelGGL((k_raster_fov<TS, false, false>), dim3((unsigned)n_tiles), dim3(TS * TS), 0, st, \
                           splats, lv, n, qbound, n_levels, cams_dev, V, vals, ranges, pix_level,    \
                           pix_weight, bg[0], bg[1], bg[2], image, sp, nullptr, nullptr);
    switch (T) {
    case 8: GS_RV(8); break;
    case 16: GS_RV(16); break;
    default: GS_RV(32); break;
    }
#undef GS_RV
    return hipGetLastError();
}
