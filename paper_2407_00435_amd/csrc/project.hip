// Projection of 3D Gaussians to screen-space splats (Section 2.1, Eq. 1b/1c)
// and its reverse.  One thread per Gaussian; the thread loops over the views,
// so each Gaussian's parameters are read from HBM once for all views.
#include "common.hpp"
#include "kernels.hpp"

namespace {

struct Cov3 {
    float xx, xy, xz, yy, yz, zz;
};

struct Rot {
    float m[9];
};

__device__ __forceinline__ Rot quat_rot(float w, float x, float y, float z)
{
    float inv = rsqrtf(w * w + x * x + y * y + z * z);
    w *= inv; x *= inv; y *= inv; z *= inv;
    Rot R;
    R.m[0] = 1.f - 2.f * (y * y + z * z); R.m[1] = 2.f * (x * y - w * z);       R.m[2] = 2.f * (x * z + w * y);
    R.m[3] = 2.f * (x * y + w * z);       R.m[4] = 1.f - 2.f * (x * x + z * z); R.m[5] = 2.f * (y * z - w * x);
    R.m[6] = 2.f * (x * z - w * y);       R.m[7] = 2.f * (y * z + w * x);       R.m[8] = 1.f - 2.f * (x * x + y * y);
    return R;
}

// Sigma = Rot diag(s^2) Rot^T
__device__ __forceinline__ Cov3 cov3d(const Rot &R, float s0, float s1, float s2)
{
    float a0 = s0 * s0, a1 = s1 * s1, a2 = s2 * s2;
    const float *m = R.m;
    Cov3 c;
    c.xx = m[0] * m[0] * a0 + m[1] * m[1] * a1 + m[2] * m[2] * a2;
    c.xy = m[0] * m[3] * a0 + m[1] * m[4] * a1 + m[2] * m[5] * a2;
    c.xz = m[0] * m[6] * a0 + m[1] * m[7] * a1 + m[2] * m[8] * a2;
    c.yy = m[3] * m[3] * a0 + m[4] * m[4] * a1 + m[5] * m[5] * a2;
    c.yz = m[3] * m[6] * a0 + m[4] * m[7] * a1 + m[5] * m[8] * a2;
    c.zz = m[6] * m[6] * a0 + m[7] * m[7] * a1 + m[8] * m[8] * a2;
    return c;
}

struct CamF {
    int W, H;
    float fx, fy, cx, cy, near_z;
    float R[9], t[3];
    float pos[3];  // camera centre -R^T t
    float limx, limy;
};

__device__ __forceinline__ CamF load_cam(const gs_camera *__restrict__ cams, int v)
{
    CamF c;
    const gs_camera &g = cams[v];
    c.W = g.width; c.H = g.height;
    c.fx = g.fx; c.fy = g.fy; c.cx = g.cx; c.cy = g.cy; c.near_z = g.near_z;
#pragma unroll
    for (int k = 0; k < 9; ++k) c.R[k] = g.R[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) c.t[k] = g.t[k];
#pragma unroll
    for (int j = 0; j < 3; ++j) c.pos[j] = -(c.R[j] * c.t[0] + c.R[3 + j] * c.t[1] + c.R[6 + j] * c.t[2]);
    c.limx = 1.3f * (0.5f * (float)c.W / c.fx);
    c.limy = 1.3f * (0.5f * (float)c.H / c.fy);
    return c;
}

// Load the (DEG+1)^2 x 3 SH coefficients of one Gaussian.
template <int DEG>
__device__ __forceinline__ void load_sh(const float *__restrict__ sh, int64_t i, float *c)
{
    constexpr int NC = (DEG + 1) * (DEG + 1) * 3;
    const float *p = sh + i * NC;
    if constexpr (NC % 4 == 0) {
        const float4 *p4 = reinterpret_cast<const float4 *>(p);
#pragma unroll
        for (int k = 0; k < NC / 4; ++k) {
            float4 q = p4[k];
            c[4 * k] = q.x; c[4 * k + 1] = q.y; c[4 * k + 2] = q.z; c[4 * k + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < NC; ++k) c[k] = p[k];
    }
}

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + __expf(-x)); }

// BIN: also the binning's count of each entry, written as the counting pass
// of the binning writes it: with LEVELS, after the level filter (the tile
// rectangle clipped to the bounding box of the tiles whose lower level is at
// most the point's quality bound, then that level's summed-area table over
// the clipped rectangle); without, the rectangle's tiles.
template <int DEG, bool LEVELS, bool BIN>
__global__ void __launch_bounds__(256)
k_project(const float *__restrict__ means, const float *__restrict__ log_scales,
          const float *__restrict__ quats, const float *__restrict__ logits,
          const float *__restrict__ sh, const float *__restrict__ lvl_logits,
          const float *__restrict__ lvl_dc, int L, const uint8_t *__restrict__ qbound,
          const gs_camera *__restrict__ cams, int V, int T, int n, gs_splat *__restrict__ out,
          float4 *__restrict__ lvl_out, ProjBin pb)
{
    constexpr int K = (DEG + 1) * (DEG + 1);
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float mx = means[3 * (int64_t)i], my = means[3 * (int64_t)i + 1], mz = means[3 * (int64_t)i + 2];
    float4 q = reinterpret_cast<const float4 *>(quats)[i];
    Rot Rq = quat_rot(q.x, q.y, q.z, q.w);
    Cov3 S = cov3d(Rq, __expf(log_scales[3 * (int64_t)i]), __expf(log_scales[3 * (int64_t)i + 1]),
                   __expf(log_scales[3 * (int64_t)i + 2]));
    float opacity = sigmoidf(logits[i]);
    float coef[K * 3];
    load_sh<DEG>(sh, i, coef);
    float lvl_op[4], lvl_dcv[4][3];
    const int qm = LEVELS && qbound ? (int)qbound[i] : 255;
    if (LEVELS) {
        // every level's loads first, unconditional (levels past L read level
        // L - 1, which is in bounds) so that they are in flight together,
        // then their use
        float raw[4], rdc[4][3];
        const bool hl = lvl_logits != nullptr, hd = lvl_dc != nullptr;
        if (hl && hd) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t tl = (int64_t)min(t, L - 1) * n + i;
                raw[t] = lvl_logits[tl];
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) rdc[t][ch] = lvl_dc[tl * 3 + ch];
            }
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t tl = (int64_t)min(t, L - 1) * n + i;
                raw[t] = hl ? lvl_logits[tl] : 0.f;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) rdc[t][ch] = hd ? lvl_dc[tl * 3 + ch] : 0.f;
            }
        }
        // a point has no version at the levels above its quality bound
        // (Section 4.2): there its level opacity is zero
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            lvl_op[t] = t + 1 > qm ? 0.0f : ((hl && t < L) ? sigmoidf(raw[t]) : opacity);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) lvl_dcv[t][ch] = (hd && t < L) ? rdc[t][ch] : coef[ch];
        }
    }
    const int mlq = qm < 1 ? 1 : (qm < L ? qm : L);  // the level filter's table for this point
    for (int v = 0; v < V; ++v) {
        CamF c = load_cam(cams, v);
        int64_t e = (int64_t)v * n + i;
        float4 *o4 = reinterpret_cast<float4 *>(out + e);
        // the level's bounding box, loaded before the projection needs it
        const int4 bb = BIN && LEVELS ? reinterpret_cast<const int4 *>(pb.bbox)[(int64_t)v * L + mlq - 1] : int4{};
        float ux = c.R[0] * mx + c.R[1] * my + c.R[2] * mz + c.t[0];
        float uy = c.R[3] * mx + c.R[4] * my + c.R[5] * mz + c.t[1];
        float uz = c.R[6] * mx + c.R[7] * my + c.R[8] * mz + c.t[2];
        bool ok = uz > c.near_z;
        float a = 0.f, b = 0.f, cc = 0.f, det = 0.f;
        if (ok) {
            float iz = 1.0f / uz;
            float tx = fminf(c.limx, fmaxf(-c.limx, ux * iz));
            float ty = fminf(c.limy, fmaxf(-c.limy, uy * iz));
            float j00 = c.fx * iz, j02 = -c.fx * tx * iz;
            float j11 = c.fy * iz, j12 = -c.fy * ty * iz;
            // T = J Rc (2x3)
            float t00 = j00 * c.R[0] + j02 * c.R[6], t01 = j00 * c.R[1] + j02 * c.R[7],
                  t02 = j00 * c.R[2] + j02 * c.R[8];
            float t10 = j11 * c.R[3] + j12 * c.R[6], t11 = j11 * c.R[4] + j12 * c.R[7],
                  t12 = j11 * c.R[5] + j12 * c.R[8];
            // rows of T Sigma
            float p0 = t00 * S.xx + t01 * S.xy + t02 * S.xz;
            float p1 = t00 * S.xy + t01 * S.yy + t02 * S.yz;
            float p2 = t00 * S.xz + t01 * S.yz + t02 * S.zz;
            float r0 = t10 * S.xx + t11 * S.xy + t12 * S.xz;
            float r1 = t10 * S.xy + t11 * S.yy + t12 * S.yz;
            float r2 = t10 * S.xz + t11 * S.yz + t12 * S.zz;
            a = p0 * t00 + p1 * t01 + p2 * t02 + 0.3f;
            b = p0 * t10 + p1 * t11 + p2 * t12;
            cc = r0 * t10 + r1 * t11 + r2 * t12 + 0.3f;
            det = a * cc - b * b;
            ok = det > 0.0f;
        }
        if (!ok) {
            float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
            o4[0] = z;
            o4[1] = z;
            o4[2] = z;
            if (LEVELS)
                for (int t = 0; t < L; ++t) lvl_out[e * L + t] = z;
            if (BIN) {
                pb.rec[e] = make_uint4(0u, 0u, 0u, 0u);
                pb.kw[e] = KEY_NONE;
            }
            continue;
        }
        float idet = 1.0f / det;
        float mid = 0.5f * (a + cc);
        float lmax = mid + sqrtf(fmaxf(mid * mid - det, 0.0f));
        int radius = (int)ceilf(3.0f * sqrtf(lmax));
        float px = c.fx * ux / uz + c.cx;
        float py = c.fy * uy / uz + c.cy;
        TileRect rect{};
        uint32_t tiles = 0;
        if (tile_rect(px, py, radius, c.W, c.H, T, rect))
            tiles = (uint32_t)(rect.tx1 - rect.tx0 + 1) * (uint32_t)(rect.ty1 - rect.ty0 + 1);
        // the filtered count: the level's summed-area table over the
        // rectangle clipped to that level's bounding box (the four corners
        // are loaded here and used after the colour)
        bool ne = false, lx = false, ly = false;
        uint32_t s11 = 0, s01 = 0, s10 = 0, s00 = 0;
        if (BIN && LEVELS) {
            rect.tx0 = rect.tx0 > bb.x ? rect.tx0 : bb.x;
            rect.ty0 = rect.ty0 > bb.y ? rect.ty0 : bb.y;
            rect.tx1 = rect.tx1 < bb.z ? rect.tx1 : bb.z;
            rect.ty1 = rect.ty1 < bb.w ? rect.ty1 : bb.w;
            ne = tiles && qm >= 1 && rect.tx0 <= rect.tx1 && rect.ty0 <= rect.ty1;
            const int64_t ntx = pb.vtab[2 * v + 1];
            const uint32_t *sp = pb.sat + (int64_t)(mlq - 1) * pb.n_tiles + pb.vtab[2 * v];
            lx = rect.tx0 > 0;
            ly = rect.ty0 > 0;
            const int x1 = ne ? rect.tx1 : 0, y1 = ne ? rect.ty1 : 0;
            const int x0 = ne && lx ? rect.tx0 - 1 : 0, y0 = ne && ly ? rect.ty0 - 1 : 0;
            s11 = sp[(int64_t)y1 * ntx + x1];
            s01 = sp[(int64_t)y1 * ntx + x0];
            s10 = sp[(int64_t)y0 * ntx + x1];
            s00 = sp[(int64_t)y0 * ntx + x0];
        }
        // colour from the unit direction camera -> mean
        float dx = mx - c.pos[0], dy = my - c.pos[1], dz = mz - c.pos[2];
        float inv = rsqrtf(dx * dx + dy * dy + dz * dz);
        dx *= inv; dy *= inv; dz *= inv;
        float Y[K];
        sh_basis<DEG>(dx, dy, dz, Y);
        float rest[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float s = 0.f;
#pragma unroll
            for (int k = 1; k < K; ++k) s += coef[3 * k + ch] * Y[k];
            rest[ch] = s + 0.5f;
        }
        float col[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) col[ch] = fmaxf(0.0f, coef[ch] * SH_C0 + rest[ch]);
        o4[0] = make_float4(px, py, cc * idet, -b * idet);
        o4[1] = make_float4(a * idet, opacity, col[0], col[1]);
        o4[2] = make_float4(col[2], uz, __int_as_float(radius), __uint_as_float(tiles));
        if (LEVELS) {
            for (int t = 0; t < L; ++t) {
                lvl_out[e * L + t] = make_float4(fmaxf(0.0f, lvl_dcv[t][0] * SH_C0 + rest[0]),
                                                 fmaxf(0.0f, lvl_dcv[t][1] * SH_C0 + rest[1]),
                                                 fmaxf(0.0f, lvl_dcv[t][2] * SH_C0 + rest[2]),
                                                 lvl_op[t]);
            }
        }
        if (BIN) {
            const uint32_t cnt =
                !LEVELS ? tiles : (ne ? s11 - (lx ? s01 : 0u) - (ly ? s10 : 0u) + (lx && ly ? s00 : 0u) : 0u);
            // every entry's record is written (whole cache lines), read only for entries with keys
            pb.rec[e] = make_uint4((uint32_t)rect.tx0 | ((uint32_t)rect.ty0 << 16),
                                   (uint32_t)rect.tx1 | ((uint32_t)rect.ty1 << 16), cnt, (uint32_t)qm);
            pb.kw[e] = cnt ? __float_as_uint(uz) : KEY_NONE;
        }
    }
}

// ---------------------------------------------------------------------------
// Reverse of the projection.  For every view the forward quantities are
// recomputed and the splat gradient is pushed back through
//   conic = inverse(S'), S' = T Sigma T^T + 0.3 I, T = J Rc,
//   J(u) with the clamped tangents, mean2d(u), u = Rc mu + t,
//   Sigma = (Rq S)(Rq S)^T, Rq of the normalised quaternion,
//   colour = max(0, sum sh Y(dir) + 1/2), opacity = sigmoid(logit).
// LEVELS: the splat gradient carries only mean and conic; colour and opacity
// gradients come per level (lvl_g [V][n][L]: r, g, b, opacity) and go through
// level t's colour max(0, DC_t Y_0 + sum_{k>=1} sh_k Y_k + 1/2) and opacity
// sigmoid(logit_t) to the level DC / logit (or the base ones when the scene
// shares them), the non-DC SH and the direction.
template <int DEG, bool LEVELS>
__global__ void __launch_bounds__(256)
k_project_bwd(const float *__restrict__ means, const float *__restrict__ log_scales,
              const float *__restrict__ quats, const float *__restrict__ logits,
              const float *__restrict__ sh, const gs_camera *__restrict__ cams, int V, int n,
              const gs_splat *__restrict__ splats, const gs_splat_grad *__restrict__ grads,
              float *__restrict__ g_means, float *__restrict__ g_ls, float *__restrict__ g_q,
              float *__restrict__ g_logit, float *__restrict__ g_sh, int acc,
              const float *__restrict__ lvl_logits, const float *__restrict__ lvl_dc, int L,
              const uint8_t *__restrict__ qbound, const float4 *__restrict__ lvl_g,
              float *__restrict__ g_lvl_logit, float *__restrict__ g_lvl_dc)
{
    constexpr int K = (DEG + 1) * (DEG + 1);
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float mx = means[3 * (int64_t)i], my = means[3 * (int64_t)i + 1], mz = means[3 * (int64_t)i + 2];
    float4 q4 = reinterpret_cast<const float4 *>(quats)[i];
    float qn_inv = rsqrtf(q4.x * q4.x + q4.y * q4.y + q4.z * q4.z + q4.w * q4.w);
    float qw = q4.x * qn_inv, qx = q4.y * qn_inv, qy = q4.z * qn_inv, qz = q4.w * qn_inv;
    Rot Rq = quat_rot(q4.x, q4.y, q4.z, q4.w);
    float s[3] = {__expf(log_scales[3 * (int64_t)i]), __expf(log_scales[3 * (int64_t)i + 1]),
                  __expf(log_scales[3 * (int64_t)i + 2])};
    // M = Rq diag(s); Sigma = M M^T
    float M[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) M[r * 3 + k] = Rq.m[r * 3 + k] * s[k];
    float Sg[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            Sg[r * 3 + k] = M[r * 3] * M[k * 3] + M[r * 3 + 1] * M[k * 3 + 1] + M[r * 3 + 2] * M[k * 3 + 2];
    float coef[K * 3];
    load_sh<DEG>(sh, i, coef);
    float opacity = sigmoidf(logits[i]);
    // level versions (LEVELS only)
    const int qm = (LEVELS && qbound) ? (int)qbound[i] : 255;
    constexpr int ML = LEVELS ? 4 : 1;
    float lvl_op[ML], lvl_dcv[ML][3], g_lop[ML], g_ldc[ML][3];
#pragma unroll
    for (int t = 0; t < ML; ++t) {
        lvl_op[t] = opacity;
        g_lop[t] = 0.f;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            lvl_dcv[t][ch] = coef[ch];
            g_ldc[t][ch] = 0.f;
        }
        if (LEVELS && t < L) {
            if (lvl_logits) lvl_op[t] = sigmoidf(lvl_logits[(int64_t)t * n + i]);
            if (lvl_dc)
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) lvl_dcv[t][ch] = lvl_dc[((int64_t)t * n + i) * 3 + ch];
        }
    }

    float gm[3] = {0.f, 0.f, 0.f};
    float dSig[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) dSig[k] = 0.f;
    float gsh[K * 3];
#pragma unroll
    for (int k = 0; k < K * 3; ++k) gsh[k] = 0.f;
    float glogit = 0.f;

    // the SH coefficients are complete before the view loop: their waits
    // would otherwise sit inside it and also wait for the next view's loads
#pragma unroll
    for (int k = 0; k < K * 3; ++k) __asm__ volatile("" ::"v"(coef[k]));
    // the view's 48-byte gradient record as three vector loads, the next
    // view's issued before this view's work (one thread walks all views)
    const float4 *g4 = reinterpret_cast<const float4 *>(grads);
    float4 ga = make_float4(0.f, 0.f, 0.f, 0.f), gb = ga, gc3 = ga;
    if (V > 0) {
        ga = g4[3 * (int64_t)i];
        gb = g4[3 * (int64_t)i + 1];
        gc3 = g4[3 * (int64_t)i + 2];
    }
    // (and so is the first view's record, for the same reason)
    __asm__ volatile("" ::"v"(ga.x), "v"(ga.y), "v"(ga.z), "v"(ga.w), "v"(gb.x), "v"(gb.y), "v"(gb.z), "v"(gb.w),
                     "v"(gc3.x));
    for (int v = 0; v < V; ++v) {
        int64_t e = (int64_t)v * n + i;
        gs_splat_grad g;
        g.mean_x = ga.x; g.mean_y = ga.y; g.conic_a = ga.z; g.conic_b = ga.w;
        g.conic_c = gb.x; g.opacity = gb.y; g.r = gb.z; g.g = gb.w;
        g.b = gc3.x;
        if (v + 1 < V) {
            const int64_t en = e + n;
            ga = g4[3 * en];
            gb = g4[3 * en + 1];
            gc3 = g4[3 * en + 2];
        }
        // keeps the next view's loads here, ahead of this view's work (the
        // scheduler would otherwise sink them to the end of the iteration)
        __asm__ volatile("" ::: "memory");
        // splats culled by the forward carry no gradient, and a visible
        // splat that no pixel blended (occluded, or outside every tile's
        // stop point) has an all-zero gradient: nothing to push back (the
        // forward's records are not read)
        bool zero = (g.mean_x == 0.f) & (g.mean_y == 0.f) & (g.conic_a == 0.f) & (g.conic_b == 0.f) &
                    (g.conic_c == 0.f) & (g.opacity == 0.f) & (g.r == 0.f) & (g.g == 0.f) & (g.b == 0.f);
        float4 lg[ML];
#pragma unroll
        for (int t = 0; t < ML; ++t) {
            lg[t] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (LEVELS && t < L) {
                lg[t] = lvl_g[e * L + t];
                zero = zero && lg[t].x == 0.f && lg[t].y == 0.f && lg[t].z == 0.f && lg[t].w == 0.f;
            }
        }
        if (zero) continue;
        CamF c = load_cam(cams, v);
        float ux = c.R[0] * mx + c.R[1] * my + c.R[2] * mz + c.t[0];
        float uy = c.R[3] * mx + c.R[4] * my + c.R[5] * mz + c.t[1];
        float uz = c.R[6] * mx + c.R[7] * my + c.R[8] * mz + c.t[2];
        if (!(uz > c.near_z)) continue;  // the forward's near cull
        // T = J Rc, T Sigma and the conic, as the forward computes them
        const float iz = 1.0f / uz;
        const float rx = ux * iz, ry = uy * iz;
        const float tx = fminf(c.limx, fmaxf(-c.limx, rx));
        const float ty = fminf(c.limy, fmaxf(-c.limy, ry));
        const float j00 = c.fx * iz, j02 = -c.fx * tx * iz;
        const float j11 = c.fy * iz, j12 = -c.fy * ty * iz;
        const float T0[3] = {j00 * c.R[0] + j02 * c.R[6], j00 * c.R[1] + j02 * c.R[7], j00 * c.R[2] + j02 * c.R[8]};
        const float T1[3] = {j11 * c.R[3] + j12 * c.R[6], j11 * c.R[4] + j12 * c.R[7], j11 * c.R[5] + j12 * c.R[8]};
        float TS0[3], TS1[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            TS0[k] = T0[0] * Sg[k] + T0[1] * Sg[3 + k] + T0[2] * Sg[6 + k];
            TS1[k] = T1[0] * Sg[k] + T1[1] * Sg[3 + k] + T1[2] * Sg[6 + k];
        }
        const float ca = TS0[0] * T0[0] + TS0[1] * T0[1] + TS0[2] * T0[2] + 0.3f;
        const float cb = TS0[0] * T1[0] + TS0[1] * T1[1] + TS0[2] * T1[2];
        const float cc_ = TS1[0] * T1[0] + TS1[1] * T1[1] + TS1[2] * T1[2] + 0.3f;
        const float cdet = ca * cc_ - cb * cb;
        if (!(cdet > 0.0f)) continue;  // the forward's degenerate-covariance cull
        const float cidet = 1.0f / cdet;
        // opacity
        if (!LEVELS) {
            glogit += g.opacity * opacity * (1.0f - opacity);
        } else {
#pragma unroll
            for (int t = 0; t < ML; ++t)
                if (t < L && t + 1 <= qm) {  // zero opacity above the quality bound
                    const float d = lg[t].w * lvl_op[t] * (1.0f - lvl_op[t]);
                    if (lvl_logits)
                        g_lop[t] += d;
                    else
                        glogit += d;
                }
        }
        // colour -> SH coefficients and direction
        float ddx = mx - c.pos[0], ddy = my - c.pos[1], ddz = mz - c.pos[2];
        float dist_inv = rsqrtf(ddx * ddx + ddy * ddy + ddz * ddz);
        float dx = ddx * dist_inv, dy = ddy * dist_inv, dz = ddz * dist_inv;
        float Y[K];
        sh_basis<DEG>(dx, dy, dz, Y);
        float gdir[3] = {0.f, 0.f, 0.f};
        float Yx[K], Yy[K], Yz[K];
        if (DEG > 0) sh_basis_grad<DEG>(dx, dy, dz, Yx, Yy, Yz);
#pragma unroll
        for (int t = 0; t < ML; ++t) {
            if (LEVELS && t >= L) continue;
            const float gc[3] = {LEVELS ? lg[t].x : g.r, LEVELS ? lg[t].y : g.g, LEVELS ? lg[t].z : g.b};
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const float dc = LEVELS ? lvl_dcv[t][ch] : coef[ch];
                float raw = 0.5f + dc * Y[0];
#pragma unroll
                for (int k = 1; k < K; ++k) raw += coef[3 * k + ch] * Y[k];
                if (!(raw > 0.0f)) continue;
                if (LEVELS && lvl_dc)
                    g_ldc[t][ch] += gc[ch] * Y[0];
                else
                    gsh[ch] += gc[ch] * Y[0];
#pragma unroll
                for (int k = 1; k < K; ++k) gsh[3 * k + ch] += gc[ch] * Y[k];
                if (DEG > 0) {
                    gdir[0] += gc[ch] * dc * Yx[0];
                    gdir[1] += gc[ch] * dc * Yy[0];
                    gdir[2] += gc[ch] * dc * Yz[0];
#pragma unroll
                    for (int k = 1; k < K; ++k) {
                        gdir[0] += gc[ch] * coef[3 * k + ch] * Yx[k];
                        gdir[1] += gc[ch] * coef[3 * k + ch] * Yy[k];
                        gdir[2] += gc[ch] * coef[3 * k + ch] * Yz[k];
                    }
                }
            }
        }
        if (DEG > 0) {
            float pr = dx * gdir[0] + dy * gdir[1] + dz * gdir[2];
            gm[0] += (gdir[0] - dx * pr) * dist_inv;
            gm[1] += (gdir[1] - dy * pr) * dist_inv;
            gm[2] += (gdir[2] - dz * pr) * dist_inv;
        }
        // conic (A, B, C) -> S' = [[a, b], [b, cc]]
        const float A = cc_ * cidet, B = -cb * cidet, C = ca * cidet;
        // dL/dS' = -M G M with G the symmetric gradient of [[A, B], [B, C]]
        float GA = g.conic_a, GB = 0.5f * g.conic_b, GC = g.conic_c;
        // M G
        float mg00 = A * GA + B * GB, mg01 = A * GB + B * GC;
        float mg10 = B * GA + C * GB, mg11 = B * GB + C * GC;
        float dS00 = -(mg00 * A + mg01 * B);
        float dS01 = -(mg00 * B + mg01 * C);
        float dS11 = -(mg10 * B + mg11 * C);
        // dSigma += T^T dS T  (dS symmetric)
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                dSig[r * 3 + k] += T0[r] * (dS00 * T0[k] + dS01 * T1[k]) + T1[r] * (dS01 * T0[k] + dS11 * T1[k]);
        // dT = 2 dS T Sigma
        float dT0[3], dT1[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            dT0[k] = 2.0f * (dS00 * TS0[k] + dS01 * TS1[k]);
            dT1[k] = 2.0f * (dS01 * TS0[k] + dS11 * TS1[k]);
        }
        // dJ = dT Rc^T: J entries (0,0), (0,2), (1,1), (1,2)
        float dJ00 = dT0[0] * c.R[0] + dT0[1] * c.R[1] + dT0[2] * c.R[2];
        float dJ02 = dT0[0] * c.R[6] + dT0[1] * c.R[7] + dT0[2] * c.R[8];
        float dJ11 = dT1[0] * c.R[3] + dT1[1] * c.R[4] + dT1[2] * c.R[5];
        float dJ12 = dT1[0] * c.R[6] + dT1[1] * c.R[7] + dT1[2] * c.R[8];
        float iz2 = iz * iz;
        float gux = 0.f, guy = 0.f, guz = 0.f;
        guz += -dJ00 * c.fx * iz2 - dJ11 * c.fy * iz2;
        bool inx = rx > -c.limx && rx < c.limx;
        bool iny = ry > -c.limy && ry < c.limy;
        // J02 = -fx tx / z, tx = x / z when not clamped
        if (inx) {
            gux += dJ02 * (-c.fx * iz2);
            guz += dJ02 * (2.0f * c.fx * ux * iz2 * iz);
        } else {
            guz += dJ02 * (c.fx * tx * iz2);
        }
        if (iny) {
            guy += dJ12 * (-c.fy * iz2);
            guz += dJ12 * (2.0f * c.fy * uy * iz2 * iz);
        } else {
            guz += dJ12 * (c.fy * ty * iz2);
        }
        // mean2d = (fx x / z + cx, fy y / z + cy)
        gux += g.mean_x * c.fx * iz;
        guy += g.mean_y * c.fy * iz;
        guz += -(g.mean_x * c.fx * ux + g.mean_y * c.fy * uy) * iz2;
        // u = Rc mu + t
        gm[0] += c.R[0] * gux + c.R[3] * guy + c.R[6] * guz;
        gm[1] += c.R[1] * gux + c.R[4] * guy + c.R[7] * guz;
        gm[2] += c.R[2] * gux + c.R[5] * guy + c.R[8] * guz;
    }
    // Sigma = M M^T: dM = (dSig + dSig^T) M
    float dM[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float acc = 0.f;
#pragma unroll
            for (int l = 0; l < 3; ++l) acc += (dSig[r * 3 + l] + dSig[l * 3 + r]) * M[l * 3 + k];
            dM[r * 3 + k] = acc;
        }
    // M = Rq diag(s)
    float dR[9];
    float ols[3] = {0.f, 0.f, 0.f};
    if (acc) {
        ols[0] = g_ls[3 * (int64_t)i];
        ols[1] = g_ls[3 * (int64_t)i + 1];
        ols[2] = g_ls[3 * (int64_t)i + 2];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float ds = dM[k] * Rq.m[k] + dM[3 + k] * Rq.m[3 + k] + dM[6 + k] * Rq.m[6 + k];
        g_ls[3 * (int64_t)i + k] = ols[k] + ds * s[k];
#pragma unroll
        for (int r = 0; r < 3; ++r) dR[r * 3 + k] = dM[r * 3 + k] * s[k];
    }
    float w = qw, x = qx, y = qy, z = qz;
    float dw = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    float dxq = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] +
                       w * dR[7] - 2.f * x * dR[8]);
    float dyq = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                       z * dR[7] - 2.f * y * dR[8]);
    float dzq = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] +
                       y * dR[5] + x * dR[6] + y * dR[7]);
    float pr = w * dw + x * dxq + y * dyq + z * dzq;
    float4 gq = make_float4((dw - w * pr) * qn_inv, (dxq - x * pr) * qn_inv, (dyq - y * pr) * qn_inv,
                            (dzq - z * pr) * qn_inv);
    // accumulating: the old values are read in batches (one wait per batch,
    // not one round trip per value)
    if (acc) {
        const float4 o = reinterpret_cast<const float4 *>(g_q)[i];
        const float om0 = g_means[3 * (int64_t)i], om1 = g_means[3 * (int64_t)i + 1];
        const float om2 = g_means[3 * (int64_t)i + 2], ol = g_logit[i];
        gq = make_float4(o.x + gq.x, o.y + gq.y, o.z + gq.z, o.w + gq.w);
        gm[0] += om0;
        gm[1] += om1;
        gm[2] += om2;
        glogit += ol;
    }
    reinterpret_cast<float4 *>(g_q)[i] = gq;
    g_means[3 * (int64_t)i] = gm[0];
    g_means[3 * (int64_t)i + 1] = gm[1];
    g_means[3 * (int64_t)i + 2] = gm[2];
    g_logit[i] = glogit;
    float *gs_out = g_sh + (int64_t)i * K * 3;
    if constexpr ((K * 3) % 4 == 0) {
        float4 *p4 = reinterpret_cast<float4 *>(gs_out);
        constexpr int N4 = K * 3 / 4;
#pragma unroll
        for (int k0 = 0; k0 < N4; k0 += 4) {
            float4 o[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                o[j] = (acc && k0 + j < N4) ? p4[k0 + j] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = k0 + j;
                if (k < N4)
                    p4[k] = make_float4(o[j].x + gsh[4 * k], o[j].y + gsh[4 * k + 1], o[j].z + gsh[4 * k + 2],
                                        o[j].w + gsh[4 * k + 3]);
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < K * 3; ++k) gs_out[k] = (acc ? gs_out[k] : 0.f) + gsh[k];
    }
    if (LEVELS) {
#pragma unroll
        for (int t = 0; t < ML; ++t) {
            if (t >= L) continue;
            if (g_lvl_logit) {
                float *p = g_lvl_logit + (int64_t)t * n + i;
                *p = (acc ? *p : 0.f) + g_lop[t];
            }
            if (g_lvl_dc) {
                float *p = g_lvl_dc + ((int64_t)t * n + i) * 3;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) p[ch] = (acc ? p[ch] : 0.f) + g_ldc[t][ch];
            }
        }
    }
}

}  // namespace

hipError_t launch_project(const gs_scene &sc, const gs_camera *cams_dev, int V, int T,
                          gs_splat *out, float *lvl_rgba, hipStream_t st, const ProjBin *pb)
{
    int n = sc.n;
    if (n == 0) return hipSuccess;
    dim3 grid((n + 255) / 256), block(256);
    int L = sc.n_levels;
    bool lv = lvl_rgba != nullptr && L > 0;
    if (pb && lv && !sc.qbound) return hipErrorInvalidValue;  // the level filter needs the quality bounds
    float4 *lo = reinterpret_cast<float4 *>(lvl_rgba);
    const ProjBin none{};
#define GS_PROJ(DEG)                                                                                   \
    if (pb && lv)                                                                                      \
        hipLaunchKernelGGL((k_project<DEG, true, true>), grid, block, 0, st, sc.means, sc.log_scales, \
                           sc.quats, sc.opacity_logits, sc.sh, sc.lvl_opacity_logits, sc.lvl_sh_dc,  \
                           L, sc.qbound, cams_dev, V, T, n, out, lo, *pb);                             \
    else if (pb)                                                                                       \
        hipLaunchKernelGGL((k_project<DEG, false, true>), grid, block, 0, st, sc.means, sc.log_scales,\
                           sc.quats, sc.opacity_logits, sc.sh, nullptr, nullptr, 0, nullptr, cams_dev, \
                           V, T, n, out, nullptr, *pb);                                                \
    else if (lv)                                                                                       \
        hipLaunchKernelGGL((k_project<DEG, true, false>), grid, block, 0, st, sc.means, sc.log_scales,\
                           sc.quats, sc.opacity_logits, sc.sh, sc.lvl_opacity_logits, sc.lvl_sh_dc,  \
                           L, sc.qbound, cams_dev, V, T, n, out, lo, none);                            \
    else                                                                                               \
        hipLaunchKernelGGL((k_project<DEG, false, false>), grid, block, 0, st, sc.means, sc.log_scales,\
                           sc.quats, sc.opacity_logits, sc.sh, nullptr, nullptr, 0, nullptr, cams_dev, \
                           V, T, n, out, nullptr, none);
    switch (sc.sh_degree) {
    case 0: GS_PROJ(0); break;
    case 1: GS_PROJ(1); break;
    case 2: GS_PROJ(2); break;
    default: GS_PROJ(3); break;
    }
#undef GS_PROJ
    return hipGetLastError();
}

hipError_t launch_project_bwd(const gs_scene &sc, const gs_camera *cams_dev, int V,
                              const gs_splat *splats, const gs_splat_grad *grads, float *g_means,
                              float *g_ls, float *g_q, float *g_logit, float *g_sh, int accumulate,
                              hipStream_t st, const float *lvl_grads, float *g_lvl_logit, float *g_lvl_dc)
{
    int n = sc.n;
    if (n == 0) return hipSuccess;
    dim3 grid((n + 255) / 256), block(256);
    const float4 *lg = reinterpret_cast<const float4 *>(lvl_grads);
    const int L = sc.n_levels;
#define GS_PB(DEG)                                                                                     \
    if (lg)                                                                                            \
        hipLaunchKernelGGL((k_project_bwd<DEG, true>), grid, block, 0, st, sc.means, sc.log_scales,   \
                           sc.quats, sc.opacity_logits, sc.sh, cams_dev, V, n, splats, grads, g_means, \
                           g_ls, g_q, g_logit, g_sh, accumulate, sc.lvl_opacity_logits, sc.lvl_sh_dc, L, \
                           sc.qbound, lg, g_lvl_logit, g_lvl_dc);                                     \
    else                                                                                               \
        hipLaunchKernelGGL((k_project_bwd<DEG, false>), grid, block, 0, st, sc.means, sc.log_scales,  \
                           sc.quats, sc.opacity_logits, sc.sh, cams_dev, V, n, splats, grads, g_means, \
                           g_ls, g_q, g_logit, g_sh, accumulate, nullptr, nullptr, 0, nullptr, nullptr, \
                           nullptr, nullptr);
    switch (sc.sh_degree) {
    case 0: GS_PB(0); break;
    case 1: GS_PB(1); break;
    case 2: GS_PB(2); break;
    default: GS_PB(3); break;
    }
#undef GS_PB
    return hipGetLastError();
}
