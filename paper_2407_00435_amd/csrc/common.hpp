// Shared device helpers for the gfx950 Gaussian-splatting kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs.h"

#define GS_LOG2E 1.4426950408889634f
#define GS_ALPHA_MIN (1.0f / 255.0f)
#define GS_ALPHA_MAX 0.99f
#define GS_T_STOP 1e-4f

// ---------------------------------------------------------------------------
// Views and the global tile / pixel spaces.
struct ViewInfo {
    int v;
    int W, H;
    int tiles_x, tiles_y;
    int64_t tile_off;  // first global tile of the view
    int64_t pix_off;   // first global pixel of the view
};

__device__ __forceinline__ int div_up(int a, int b) { return (a + b - 1) / b; }

// Eccentricity of pixel (x, y) in degrees (Section 4.1): the angle between
// the pinhole rays through the pixel and through the gaze pixel.
__device__ __forceinline__ float pixel_ecc_deg(const gs_camera &c, float gaze_x, float gaze_y, int x, int y)
{
    const float ifx = 1.0f / c.fx, ify = 1.0f / c.fy;
    const float rx = ((float)x - c.cx) * ifx, ry = ((float)y - c.cy) * ify;
    const float gx = (gaze_x - c.cx) * ifx, gy = (gaze_y - c.cy) * ify;
    // angle between (rx, ry, 1) and (gx, gy, 1)
    const float cx_ = ry - gy, cy_ = gx - rx, cz_ = rx * gy - ry * gx;
    const float cn = sqrtf(cx_ * cx_ + cy_ * cy_ + cz_ * cz_);
    const float dt = rx * gx + ry * gy + 1.0f;
    return atan2f(cn, dt) * 57.29577951308232f;
}

// Linear walk over the (few) views; every lane of a block does the same walk.
__device__ __forceinline__ ViewInfo view_of_tile(const gs_camera *__restrict__ cams, int V, int T,
                                                 int64_t gtile)
{
    ViewInfo vi;
    int64_t toff = 0, poff = 0;
    for (int v = 0; v < V; ++v) {
        int W = cams[v].width, H = cams[v].height;
        int tx = div_up(W, T), ty = div_up(H, T);
        int64_t nt = (int64_t)tx * ty;
        if (gtile < toff + nt || v == V - 1) {
            vi.v = v; vi.W = W; vi.H = H; vi.tiles_x = tx; vi.tiles_y = ty;
            vi.tile_off = toff; vi.pix_off = poff;
            return vi;
        }
        toff += nt;
        poff += (int64_t)W * H;
    }
    vi.v = 0; vi.W = vi.H = vi.tiles_x = vi.tiles_y = 0; vi.tile_off = vi.pix_off = 0;
    return vi;
}

// ---------------------------------------------------------------------------
// Pixel rectangle of a splat in float32: [ceil(x - r), floor(x + r)] clipped
// to the image, likewise in y; tile rectangle = pixel rectangle / T.  Only
// IEEE subtract, ceil, floor and compares are used, so contraction cannot
// change the result.  Returns false for an empty rectangle or r <= 0.
struct TileRect {
    int tx0, tx1, ty0, ty1;
};

__device__ __forceinline__ bool tile_rect(float mx, float my, int r, int W, int H, int T,
                                          TileRect &out)
{
    if (r <= 0) return false;
    float fr = (float)r;
    float x0 = ceilf(__fsub_rn(mx, fr)), x1 = floorf(__fadd_rn(mx, fr));
    float y0 = ceilf(__fsub_rn(my, fr)), y1 = floorf(__fadd_rn(my, fr));
    if (!(x0 <= x1) || !(y0 <= y1)) return false;
    x0 = x0 < 0.0f ? 0.0f : x0;
    y0 = y0 < 0.0f ? 0.0f : y0;
    x1 = x1 > (float)(W - 1) ? (float)(W - 1) : x1;
    y1 = y1 > (float)(H - 1) ? (float)(H - 1) : y1;
    if (!(x0 <= x1) || !(y0 <= y1)) return false;
    out.tx0 = (int)x0 / T;
    out.tx1 = (int)x1 / T;
    out.ty0 = (int)y0 / T;
    out.ty1 = (int)y1 / T;
    return true;
}

// ---------------------------------------------------------------------------
// Real orthonormal spherical harmonics for l <= 3 in Cartesian form on the
// unit sphere, without the Condon-Shortley phase; index k = l^2 + l + m.
// Constants: N_lm from sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times sqrt(2)
// for m != 0 and the polynomial factor of P_l^|m|.
#define SH_C0 0.28209479177387814f   // 1/(2 sqrt(pi))
#define SH_C1 0.4886025119029199f    // sqrt(3/(4 pi))
#define SH_C2A 1.0925484305920792f   // sqrt(15/pi)/2      xy, yz, xz
#define SH_C2B 0.31539156525252005f  // sqrt(5/pi)/4       3z^2 - 1
#define SH_C2C 0.5462742152960396f   // sqrt(15/pi)/4      x^2 - y^2
#define SH_C3A 0.5900435899266435f   // sqrt(35/(2 pi))/4  y(3x^2 - y^2), x(x^2 - 3y^2)
#define SH_C3B 2.890611442640554f    // sqrt(105/pi)/2     xyz
#define SH_C3C 0.4570457994644658f   // sqrt(21/(2 pi))/4  y(5z^2 - 1), x(5z^2 - 1)
#define SH_C3D 0.3731763325901154f   // sqrt(7/pi)/4       z(5z^2 - 3)
#define SH_C3E 1.445305721320277f    // sqrt(105/pi)/4     z(x^2 - y^2)

template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float *Y)
{
    Y[0] = SH_C0;
    if (DEG >= 1) {
        Y[1] = SH_C1 * y;
        Y[2] = SH_C1 * z;
        Y[3] = SH_C1 * x;
    }
    if (DEG >= 2) {
        float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = SH_C2A * x * y;
        Y[5] = SH_C2A * y * z;
        Y[6] = SH_C2B * (3.0f * zz - 1.0f);
        Y[7] = SH_C2A * x * z;
        Y[8] = SH_C2C * (xx - yy);
        if (DEG >= 3) {
            Y[9] = SH_C3A * y * (3.0f * xx - yy);
            Y[10] = SH_C3B * x * y * z;
            Y[11] = SH_C3C * y * (5.0f * zz - 1.0f);
            Y[12] = SH_C3D * z * (5.0f * zz - 3.0f);
            Y[13] = SH_C3C * x * (5.0f * zz - 1.0f);
            Y[14] = SH_C3E * z * (xx - yy);
            Y[15] = SH_C3A * x * (xx - 3.0f * yy);
        }
    }
}

// Partial derivatives of the Cartesian forms above with respect to x, y, z
// (the radial part is removed by the caller's projection onto the sphere).
template <int DEG>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, float *dx, float *dy,
                                              float *dz)
{
    dx[0] = dy[0] = dz[0] = 0.0f;
    if (DEG >= 1) {
        dx[1] = 0.0f;  dy[1] = SH_C1; dz[1] = 0.0f;
        dx[2] = 0.0f;  dy[2] = 0.0f;  dz[2] = SH_C1;
        dx[3] = SH_C1; dy[3] = 0.0f;  dz[3] = 0.0f;
    }
    if (DEG >= 2) {
        float xx = x * x, yy = y * y, zz = z * z;
        dx[4] = SH_C2A * y;               dy[4] = SH_C2A * x;                dz[4] = 0.0f;
        dx[5] = 0.0f;                     dy[5] = SH_C2A * z;                dz[5] = SH_C2A * y;
        dx[6] = 0.0f;                     dy[6] = 0.0f;                      dz[6] = SH_C2B * 6.0f * z;
        dx[7] = SH_C2A * z;               dy[7] = 0.0f;                      dz[7] = SH_C2A * x;
        dx[8] = SH_C2C * 2.0f * x;        dy[8] = -SH_C2C * 2.0f * y;        dz[8] = 0.0f;
        if (DEG >= 3) {
            dx[9] = SH_C3A * 6.0f * x * y;  dy[9] = SH_C3A * (3.0f * xx - 3.0f * yy);  dz[9] = 0.0f;
            dx[10] = SH_C3B * y * z;        dy[10] = SH_C3B * x * z;                   dz[10] = SH_C3B * x * y;
            dx[11] = 0.0f;                  dy[11] = SH_C3C * (5.0f * zz - 1.0f);      dz[11] = SH_C3C * 10.0f * y * z;
            dx[12] = 0.0f;                  dy[12] = 0.0f;                             dz[12] = SH_C3D * (15.0f * zz - 3.0f);
            dx[13] = SH_C3C * (5.0f * zz - 1.0f); dy[13] = 0.0f;                       dz[13] = SH_C3C * 10.0f * x * z;
            dx[14] = SH_C3E * 2.0f * x * z; dy[14] = -SH_C3E * 2.0f * y * z;           dz[14] = SH_C3E * (xx - yy);
            dx[15] = SH_C3A * (3.0f * xx - 3.0f * yy); dy[15] = -SH_C3A * 6.0f * x * y; dz[15] = 0.0f;
        }
    }
}

// ---------------------------------------------------------------------------
// Wave helpers (wave64).
__device__ __forceinline__ uint64_t lanemask_lt()
{
    uint32_t lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// Orders LDS traffic of the lanes of one wave (all lanes of the wave run in
// lock step; this stops the compiler from moving LDS accesses across it).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// Sum over the 16 lanes of each DPP row; every lane of the row gets the sum.
__device__ __forceinline__ float row_sum16(float x)
{
    x += dpp_f<0xB1>(x);   // quad_perm [1,0,3,2]
    x += dpp_f<0x4E>(x);   // quad_perm [2,3,0,1]
    x += dpp_f<0x141>(x);  // row_half_mirror
    x += dpp_f<0x140>(x);  // row_mirror
    return x;
}

// Inclusive prefix sum over the 64 lanes of a wave: shifts by 1, 2, 4 and 8
// inside each 16-lane row, then lane 15 of rows 0 and 2 into rows 1 and 3,
// then lane 31 into rows 2 and 3 -- six DPP adds, no round trip through LDS.  Every
// lane of the wave must be active.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return x;
}

// Sum over all 64 lanes, result in every lane (wave-uniform).
__device__ __forceinline__ float wave_sum(float x)
{
    x = row_sum16(x);
    float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
    float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 16));
    float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32));
    float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 48));
    return (a + b) + (c + d);
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
