// HVSQ (Section 2.2, Eq. 2): the eccentricity-aware quality metric that the
// foveated training of Section 4.3 uses per quality region, and its
// gradient with respect to the altered image.
//
// Per pixel i: the mean and the population standard deviation of each colour
// channel over its pooling window (the square of half-width radius[i]
// centred on it, clipped to the image) in the altered image a and the
// reference r; term_i = mean over channels of (M_a - M_r)^2 + (S_a - S_r)^2;
// the metric of a region is the mean of term_i over its pixels.
//
// Window sums come from summed-area tables, so a pixel costs the same
// whatever its window: the tables hold, per view, channel and image, the
// prefix sums of x and of x^2.  They are double-double (a pair of doubles
// per value): a window's variance is a difference of two such sums, and in
// one double the rounding of sums over a whole frame would swamp the
// variance of a small window.  The gradient of the metric over a region,
//   dL/da_j = sum over windows i containing j of A_i + B_i a_j,
//   A_i = k (2 (M_a - M_r) / n - 2 (S_a - S_r) M_a / (n S_a)),
//   B_i = k 2 (S_a - S_r) / (n S_a),  k = 1 / (3 N_region)
// (B_i = 0 where S_a = 0, where the square root has no derivative), is a
// sum of per-window constants over rectangles: each window adds A_i and B_i
// at its four corners of a difference array (double atomics), and a 2D
// prefix sum of that array gives every pixel's sums (k is applied last: it
// needs the region's pixel count, which the scatter's own pass counts).
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace {

// --- double-double arithmetic (value = hi + lo, |lo| <= ulp(hi) / 2) -------
struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd quick_two_sum(double a, double b)
{
    const double s = a + b;
    return {s, b - (s - a)};
}

__device__ __forceinline__ dd dd_add(dd x, dd y)
{
    const double s = x.hi + y.hi;
    const double bb = s - x.hi;
    const double e = (x.hi - (s - bb)) + (y.hi - bb) + x.lo + y.lo;
    return quick_two_sum(s, e);
}

__device__ __forceinline__ dd dd_neg(dd x) { return {-x.hi, -x.lo}; }

__device__ __forceinline__ dd dd_mul_d(dd x, double d)
{
    const double p = x.hi * d;
    const double e = fma(x.hi, d, -p) + x.lo * d;
    return quick_two_sum(p, e);
}

__device__ __forceinline__ dd dd_sqr(dd x)
{
    const double p = x.hi * x.hi;
    const double e = fma(x.hi, x.hi, -p) + 2.0 * x.hi * x.lo;
    return quick_two_sum(p, e);
}

// Where view v's rows and pixels start: a linear walk over the (few) views.
struct HvView {
    int v, W, H;
    int64_t pix_off;  // first pixel of the view
    int64_t pad_off;  // first entry of the view's (H + 1) x (W + 1) table
    int64_t row_off;  // first global row of the view
};

__device__ __forceinline__ HvView hv_view(const gs_camera *__restrict__ cams, int V, int v)
{
    HvView h;
    h.pix_off = h.pad_off = h.row_off = 0;
    for (int u = 0; u < v; ++u) {
        const int W = cams[u].width, H = cams[u].height;
        h.pix_off += (int64_t)W * H;
        h.pad_off += (int64_t)(W + 1) * (H + 1);
        h.row_off += H;
    }
    h.v = v;
    h.W = cams[v].width;
    h.H = cams[v].height;
    return h;
}

// Pooling half-width of every pixel: floor(rho * eccentricity in degrees).
__global__ void __launch_bounds__(256)
k_hvsq_radius(const gs_camera *__restrict__ cams, int V, FoveaGazes gz, float rho, int32_t *__restrict__ radius)
{
    const HvView h = hv_view(cams, V, blockIdx.y);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)h.W * h.H) return;
    const int x = (int)(i % h.W), y = (int)(i / h.W);
    const float ecc = pixel_ecc_deg(cams[h.v], gz.x[h.v], gz.y[h.v], x, y);
    radius[h.pix_off + i] = (int32_t)floorf(rho * ecc);
}

constexpr int PLANES = 12;  // image (a, r) x channel (3) x power (x, x^2)
constexpr int ROW_THREADS = 256;

// Row pass: one workgroup per (view row, image, channel) makes the row of
// both powers' tables (x and x^2).  The row is read in chunks of
// 4 * ROW_THREADS values, four consecutive ones per thread (coalesced); each
// chunk is scanned in double-double -- within the thread, across the wave by
// shuffles, across the workgroup through LDS -- after the running total of
// the chunks before, and stored as contiguous runs; table column 0 is zero.
__device__ __forceinline__ dd dd_shfl_up(dd x, int off)
{
    return {__shfl_up(x.hi, off), __shfl_up(x.lo, off)};
}

__global__ void __launch_bounds__(ROW_THREADS)
k_hvsq_sat_rows(const gs_camera *__restrict__ cams, int V, const float *__restrict__ img_a,
                const float *__restrict__ img_r, int64_t P, double *__restrict__ hi, double *__restrict__ lo)
{
    constexpr int WAVES = ROW_THREADS / 64;
    __shared__ dd s_w[2][WAVES];
    const int q = blockIdx.y, img = q / 3, ch = q % 3;
    // the view of global row blockIdx.x
    int v = 0;
    int64_t rows = 0;
    for (; v < V - 1; ++v) {
        if ((int64_t)blockIdx.x < rows + cams[v].height) break;
        rows += cams[v].height;
    }
    const HvView h = hv_view(cams, V, v);
    const int y = (int)(blockIdx.x - h.row_off);
    const float *src = (img ? img_r : img_a) + 3 * h.pix_off + (int64_t)ch * h.W * h.H + (int64_t)y * h.W;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // planes img * 6 + ch * 2 + power
    const int64_t row0 = (int64_t)(img * 6 + ch * 2) * P + h.pad_off + (int64_t)(y + 1) * (h.W + 1);
    const int64_t row1 = row0 + P;
    if (threadIdx.x == 0) {
        hi[row0] = lo[row0] = 0.0;
        hi[row1] = lo[row1] = 0.0;
    }
    dd carry0 = {0.0, 0.0}, carry1 = {0.0, 0.0};
    for (int c0 = 0; c0 < h.W; c0 += 4 * ROW_THREADS) {
        const int x = c0 + 4 * (int)threadIdx.x;
        dd a[4], b[4];  // the thread's inclusive prefixes of x and x^2
        dd s0 = {0.0, 0.0}, s1 = {0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double e = x + k < h.W ? (double)src[x + k] : 0.0;
            s0 = dd_add(s0, {e, 0.0});
            s1 = dd_add(s1, {e * e, 0.0});  // a float's square is exact in a double
            a[k] = s0;
            b[k] = s1;
        }
        dd t0 = s0, t1 = s1;
        for (int off = 1; off < 64; off <<= 1) {
            const dd u0 = dd_shfl_up(t0, off), u1 = dd_shfl_up(t1, off);
            if (lane >= off) {
                t0 = dd_add(t0, u0);
                t1 = dd_add(t1, u1);
            }
        }
        if (lane == 63) {
            s_w[0][wave] = t0;
            s_w[1][wave] = t1;
        }
        __syncthreads();
        dd w0 = carry0, w1 = carry1, n0 = carry0, n1 = carry1;
        for (int k = 0; k < WAVES; ++k) {
            if (k < wave) {
                w0 = dd_add(w0, s_w[0][k]);
                w1 = dd_add(w1, s_w[1][k]);
            }
            n0 = dd_add(n0, s_w[0][k]);
            n1 = dd_add(n1, s_w[1][k]);
        }
        dd e0 = dd_shfl_up(t0, 1), e1 = dd_shfl_up(t1, 1);
        if (lane == 0) e0 = e1 = {0.0, 0.0};
        w0 = dd_add(w0, e0);
        w1 = dd_add(w1, e1);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (x + k < h.W) {
                const dd r0 = dd_add(w0, a[k]), r1 = dd_add(w1, b[k]);
                hi[row0 + x + k + 1] = r0.hi;
                lo[row0 + x + k + 1] = r0.lo;
                hi[row1 + x + k + 1] = r1.hi;
                lo[row1 + x + k + 1] = r1.lo;
            }
        }
        carry0 = n0;
        carry1 = n1;
        __syncthreads();  // s_w is written again by the next chunk
    }
}

// Column pass: thread (plane, view column) accumulates down the rows; table
// row 0 is zero.  Adjacent threads take adjacent columns (coalesced).
__global__ void __launch_bounds__(256)
k_hvsq_sat_cols(const gs_camera *__restrict__ cams, int V, int64_t P, double *__restrict__ hi,
                double *__restrict__ lo)
{
    const int p = blockIdx.y;
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int v = 0;
    for (; v < V; ++v) {
        if (c < cams[v].width + 1) break;
        c -= cams[v].width + 1;
    }
    if (v >= V) return;
    const HvView h = hv_view(cams, V, v);
    const int64_t W1 = h.W + 1;
    const int64_t base = (int64_t)p * P + h.pad_off + c;
    hi[base] = 0.0;
    lo[base] = 0.0;
    dd acc = {0.0, 0.0};
    // rows in batches of CB: the next batch's loads are issued before this
    // batch's stores (a load waits for every store issued before it), then
    // the rows left over one by one
    constexpr int CB = 8;
    const int full = h.H / CB * CB;
    double nh[CB], nl[CB];
    if (full > 0) {
#pragma unroll
        for (int k = 0; k < CB; ++k) {
            nh[k] = hi[base + (int64_t)(1 + k) * W1];
            nl[k] = lo[base + (int64_t)(1 + k) * W1];
        }
    }
    for (int y0 = 1; y0 <= full; y0 += CB) {
        double ch[CB], cl[CB];
#pragma unroll
        for (int k = 0; k < CB; ++k) {
            ch[k] = nh[k];
            cl[k] = nl[k];
        }
        if (y0 + CB <= full) {
#pragma unroll
            for (int k = 0; k < CB; ++k) {
                nh[k] = hi[base + (int64_t)(y0 + CB + k) * W1];
                nl[k] = lo[base + (int64_t)(y0 + CB + k) * W1];
            }
        }
#pragma unroll
        for (int k = 0; k < CB; ++k) {
            acc = dd_add(acc, {ch[k], cl[k]});
            hi[base + (int64_t)(y0 + k) * W1] = acc.hi;
            lo[base + (int64_t)(y0 + k) * W1] = acc.lo;
        }
    }
    for (int y = full + 1; y <= h.H; ++y) {
        const int64_t q = base + (int64_t)y * W1;
        acc = dd_add(acc, {hi[q], lo[q]});
        hi[q] = acc.hi;
        lo[q] = acc.lo;
    }
}

struct WinStats {
    double mu[2][3], sd[2][3];  // [image][channel]
    int n;
    int x0, x1, y0, y1;         // the clipped window
};

__device__ __forceinline__ dd table_at(const double *__restrict__ hi, const double *__restrict__ lo, int64_t q)
{
    return {hi[q], lo[q]};
}

// Mean and population standard deviation over pixel (x, y)'s window, from
// the tables: window sum = S(x1+1, y1+1) - S(x0, y1+1) - S(x1+1, y0) + S(x0, y0);
// variance = (n S2 - S1^2) / n^2, formed in double-double.
__device__ __forceinline__ WinStats win_stats(const HvView &h, int64_t P, const double *__restrict__ hi,
                                              const double *__restrict__ lo, int x, int y, int rad)
{
    WinStats w;
    w.x0 = max(x - rad, 0);
    w.x1 = min(x + rad, h.W - 1);
    w.y0 = max(y - rad, 0);
    w.y1 = min(y + rad, h.H - 1);
    w.n = (w.x1 - w.x0 + 1) * (w.y1 - w.y0 + 1);
    const int64_t W1 = h.W + 1;
    const int64_t q11 = (int64_t)(w.y1 + 1) * W1 + w.x1 + 1, q01 = (int64_t)(w.y1 + 1) * W1 + w.x0;
    const int64_t q10 = (int64_t)w.y0 * W1 + w.x1 + 1, q00 = (int64_t)w.y0 * W1 + w.x0;
    const double n = (double)w.n;
    for (int img = 0; img < 2; ++img)
        for (int ch = 0; ch < 3; ++ch) {
            dd S[2];
            for (int sq = 0; sq < 2; ++sq) {
                const int64_t b = (int64_t)(img * 6 + ch * 2 + sq) * P + h.pad_off;
                S[sq] = dd_add(dd_add(table_at(hi, lo, b + q11), dd_neg(table_at(hi, lo, b + q01))),
                               dd_add(dd_neg(table_at(hi, lo, b + q10)), table_at(hi, lo, b + q00)));
            }
            const dd nvar = dd_add(dd_mul_d(S[1], n), dd_neg(dd_sqr(S[0])));  // n^2 variance
            w.mu[img][ch] = (S[0].hi + S[0].lo) / n;
            w.sd[img][ch] = sqrt(fmax(nvar.hi + nvar.lo, 0.0)) / n;
        }
    return w;
}

__device__ __forceinline__ double pixel_term(const WinStats &w)
{
    double t = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
        const double dm = w.mu[0][ch] - w.mu[1][ch], ds = w.sd[0][ch] - w.sd[1][ch];
        t += dm * dm + ds * ds;
    }
    return t / 3.0;
}

__device__ __forceinline__ double wave_sum_d(double x)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// Per pixel: the term; per view: sums and counts per region and over the
// whole view (wave sums, one LDS atomic per wave and region, one double
// atomic per block and region).  terms (nullable): the per-pixel terms.
// With GRAD, the pixels of grad_region (0: every pixel) also add their
// window's gradient constants, without the factor 1 / (3 N) (N the region's
// pixel count, known only when every block is done; k_hvsq_grad applies it),
// at the four corners of the window in the view's difference arrays D
// ([channel][A, B] planes of (H + 1) x (W + 1) doubles): the metric over a
// region is (1 / N) sum_i t_i, and for pixel j of window i and channel c,
//   d t_i / d a_jc = (1 / 3) (2 (M_a - M_r) / n + 2 (S_a - S_r) (a_jc - M_a) / (n S_a))
//                  = (1 / 3) (A + B a_jc),
// B = 2 (S_a - S_r) / (n S_a) (0 where S_a = 0), A = 2 (M_a - M_r) / n - B M_a,
// the statistics being those of channel c; summed over the windows that
// contain j.
template <bool GRAD>
__global__ void __launch_bounds__(256)
k_hvsq_terms(const gs_camera *__restrict__ cams, int V, int64_t P, const double *__restrict__ hi,
             const double *__restrict__ lo, const int32_t *__restrict__ radius, const uint8_t *__restrict__ region,
             int R, double *__restrict__ sums, double *__restrict__ counts, double *__restrict__ terms,
             int grad_region, double *__restrict__ D)
{
    __shared__ double s_sum[GS_HVSQ_MAX_REGIONS + 1], s_cnt[GS_HVSQ_MAX_REGIONS + 1];
    if (threadIdx.x <= R) {
        s_sum[threadIdx.x] = 0.0;
        s_cnt[threadIdx.x] = 0.0;
    }
    __syncthreads();
    const HvView h = hv_view(cams, V, blockIdx.y);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool valid = i < (int64_t)h.W * h.H;
    double t = 0.0;
    int rg = 0;  // the pixel's region (0: none)
    if (valid) {
        const int x = (int)(i % h.W), y = (int)(i / h.W);
        const WinStats w = win_stats(h, P, hi, lo, x, y, max(radius[h.pix_off + i], 0));
        t = pixel_term(w);
        if (terms) terms[h.pix_off + i] = t;
        if (region) {
            const int r = region[h.pix_off + i];
            rg = r >= 1 && r <= R ? r : 0;
        }
        if (GRAD && (grad_region == 0 || rg == grad_region)) {
            const double n = (double)w.n;
            const int64_t W1 = h.W + 1;
            const int64_t c00 = (int64_t)w.y0 * W1 + w.x0, c10 = (int64_t)w.y0 * W1 + w.x1 + 1;
            const int64_t c01 = (int64_t)(w.y1 + 1) * W1 + w.x0, c11 = (int64_t)(w.y1 + 1) * W1 + w.x1 + 1;
            for (int ch = 0; ch < 3; ++ch) {
                const double dm = w.mu[0][ch] - w.mu[1][ch], ds = w.sd[0][ch] - w.sd[1][ch];
                const double B = w.sd[0][ch] > 0.0 ? 2.0 * ds / (n * w.sd[0][ch]) : 0.0;
                const double A = 2.0 * dm / n - B * w.mu[0][ch];
                for (int q = 0; q < 2; ++q) {
                    const double val = q ? B : A;
                    double *pl = D + (int64_t)(ch * 2 + q) * P + h.pad_off;
                    atomicAdd(pl + c00, val);
                    atomicAdd(pl + c10, -val);
                    atomicAdd(pl + c01, -val);
                    atomicAdd(pl + c11, val);
                }
            }
        }
    }
    // the whole view
    const uint64_t vm = ballot64(valid);
    const double tv = wave_sum_d(t);
    if (lane == 0 && vm) {
        atomicAdd(&s_sum[R], tv);
        atomicAdd(&s_cnt[R], (double)__popcll(vm));
    }
    // each region present in the wave
    uint64_t left = ballot64(rg != 0);
    while (left) {
        const int leader = __ffsll((unsigned long long)left) - 1;
        const int cur = __shfl(rg, leader);
        const bool mine = rg == cur;
        const uint64_t m = ballot64(mine);
        const double x = wave_sum_d(mine ? t : 0.0);
        if (lane == leader) {
            atomicAdd(&s_sum[cur - 1], x);
            atomicAdd(&s_cnt[cur - 1], (double)__popcll(m));
        }
        left &= ~m;
    }
    __syncthreads();
    if (threadIdx.x <= R && s_cnt[threadIdx.x] > 0.0) {
        atomicAdd(&sums[(int64_t)h.v * (R + 1) + threadIdx.x], s_sum[threadIdx.x]);
        atomicAdd(&counts[(int64_t)h.v * (R + 1) + threadIdx.x], s_cnt[threadIdx.x]);
    }
}

__global__ void __launch_bounds__(256) k_fill_f64(double *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// In-place inclusive prefix of the difference arrays along rows (block per
// (global row, plane); rows of W + 1 entries, the view's first H rows),
// then along columns (thread per (plane, view column)).
__global__ void __launch_bounds__(ROW_THREADS)
k_hvsq_prefix_rows(const gs_camera *__restrict__ cams, int V, int64_t P, double *__restrict__ D)
{
    constexpr int WAVES = ROW_THREADS / 64;
    __shared__ double s_w[WAVES];
    int v = 0;
    int64_t rows = 0;
    for (; v < V - 1; ++v) {
        if ((int64_t)blockIdx.x < rows + cams[v].height) break;
        rows += cams[v].height;
    }
    const HvView h = hv_view(cams, V, v);
    const int y = (int)(blockIdx.x - h.row_off);
    double *row = D + (int64_t)blockIdx.y * P + h.pad_off + (int64_t)y * (h.W + 1);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // chunks of 4 * ROW_THREADS values, four consecutive ones per thread, as
    // in the table's row pass
    double carry = 0.0;
    for (int c0 = 0; c0 < h.W; c0 += 4 * ROW_THREADS) {
        const int x = c0 + 4 * (int)threadIdx.x;
        double a[4], t = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            t += x + k < h.W ? row[x + k] : 0.0;
            a[k] = t;
        }
        double wt = t;
        for (int off = 1; off < 64; off <<= 1) {
            const double u = __shfl_up(wt, off);
            if (lane >= off) wt += u;
        }
        if (lane == 63) s_w[wave] = wt;
        __syncthreads();
        double w = carry, n = carry;
        for (int k = 0; k < WAVES; ++k) {
            if (k < wave) w += s_w[k];
            n += s_w[k];
        }
        const double ex = __shfl_up(wt, 1);
        w += lane ? ex : 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (x + k < h.W) row[x + k] = w + a[k];
        carry = n;
        __syncthreads();  // s_w is written again by the next chunk
    }
}

__global__ void __launch_bounds__(256)
k_hvsq_prefix_cols(const gs_camera *__restrict__ cams, int V, int64_t P, double *__restrict__ D)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int v = 0;
    for (; v < V; ++v) {
        if (c < cams[v].width) break;
        c -= cams[v].width;
    }
    if (v >= V) return;
    const HvView h = hv_view(cams, V, v);
    double *col = D + (int64_t)blockIdx.y * P + h.pad_off + c;
    const int64_t W1 = h.W + 1;
    double acc = 0.0;
    // batches of CB rows, the next batch's loads issued before this batch's
    // stores (as in the table's column pass), then the rows left over
    constexpr int CB = 8;
    const int full = h.H / CB * CB;
    double nx[CB];
    if (full > 0) {
#pragma unroll
        for (int k = 0; k < CB; ++k) nx[k] = col[(int64_t)k * W1];
    }
    for (int y0 = 0; y0 < full; y0 += CB) {
        double cx[CB];
#pragma unroll
        for (int k = 0; k < CB; ++k) cx[k] = nx[k];
        if (y0 + CB < full) {
#pragma unroll
            for (int k = 0; k < CB; ++k) nx[k] = col[(int64_t)(y0 + CB + k) * W1];
        }
#pragma unroll
        for (int k = 0; k < CB; ++k) {
            acc += cx[k];
            col[(int64_t)(y0 + k) * W1] = acc;
        }
    }
    for (int y = full; y < h.H; ++y) {
        acc += col[(int64_t)y * W1];
        col[(int64_t)y * W1] = acc;
    }
}

// dL/da = G_A + a G_B per pixel and channel (float).
__global__ void __launch_bounds__(256)
k_hvsq_grad(const gs_camera *__restrict__ cams, int V, int64_t P, const double *__restrict__ D,
            const float *__restrict__ img_a, const double *__restrict__ counts, int R, int grad_region,
            float *__restrict__ dL_da)
{
    const HvView h = hv_view(cams, V, blockIdx.y);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)h.W * h.H) return;
    // the factor 1 / (3 N) of the view's region, left out of the scatter
    const double N = counts[(int64_t)h.v * (R + 1) + (grad_region > 0 ? grad_region - 1 : R)];
    const double k = N > 0.0 ? 1.0 / (3.0 * N) : 0.0;
    const int x = (int)(i % h.W), y = (int)(i / h.W);
    const int64_t q = h.pad_off + (int64_t)y * (h.W + 1) + x;
    for (int ch = 0; ch < 3; ++ch) {
        const int64_t px = 3 * h.pix_off + (int64_t)ch * h.W * h.H + i;
        const double g = D[(int64_t)(ch * 2) * P + q] + (double)img_a[px] * D[(int64_t)(ch * 2 + 1) * P + q];
        dL_da[px] = (float)(k * g);
    }
}

}  // namespace

int64_t hvsq_padded_pixels(const gs_camera *cams_host, int V)
{
    int64_t P = 0;
    for (int v = 0; v < V; ++v) P += (int64_t)(cams_host[v].width + 1) * (cams_host[v].height + 1);
    return P;
}

size_t hvsq_scratch_bytes(const gs_camera *cams_host, int V, bool grad)
{
    const int64_t P = hvsq_padded_pixels(cams_host, V);
    return (size_t)8 * P * (2 * PLANES + (grad ? 6 : 0)) + 512;
}

hipError_t launch_hvsq_radius(const gs_camera *cams_host, const gs_camera *cams_dev, const gs_fovea *fov_host, int V,
                              float rho, int32_t *radius, hipStream_t st)
{
    FoveaGazes gz;
    int64_t maxpx = 1;
    for (int v = 0; v < V; ++v) {
        gz.x[v] = fov_host[v].gaze_x;
        gz.y[v] = fov_host[v].gaze_y;
        maxpx = std::max(maxpx, (int64_t)cams_host[v].width * cams_host[v].height);
    }
    hipLaunchKernelGGL(k_hvsq_radius, dim3((unsigned)((maxpx + 255) / 256), V), dim3(256), 0, st, cams_dev, V, gz,
                       rho, radius);
    return hipGetLastError();
}

hipError_t launch_hvsq(const gs_camera *cams_host, const gs_camera *cams_dev, int V, const float *img_a,
                       const float *img_r, const int32_t *radius, const uint8_t *region, int R, double *sums,
                       double *counts, double *terms, int grad_region, float *dL_da, void *ws, hipStream_t st)
{
    const int64_t P = hvsq_padded_pixels(cams_host, V);
    int64_t rows = 0, cols = 0, colsD = 0, maxpx = 1;
    for (int v = 0; v < V; ++v) {
        rows += cams_host[v].height;
        cols += cams_host[v].width + 1;
        colsD += cams_host[v].width;
        maxpx = std::max(maxpx, (int64_t)cams_host[v].width * cams_host[v].height);
    }
    char *base = (char *)(((uintptr_t)ws + 255) & ~uintptr_t(255));
    double *hi = (double *)base;
    double *lo = hi + (int64_t)PLANES * P;
    double *D = lo + (int64_t)PLANES * P;
    const int64_t nsum = (int64_t)V * (R + 1);
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(256), 0, st, sums, nsum);
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(256), 0, st, counts, nsum);
    hipLaunchKernelGGL(k_hvsq_sat_rows, dim3((unsigned)rows, PLANES / 2), dim3(ROW_THREADS), 0, st, cams_dev, V, img_a,
                       img_r, P, hi, lo);
    hipLaunchKernelGGL(k_hvsq_sat_cols, dim3((unsigned)((cols + 255) / 256), PLANES), dim3(256), 0, st, cams_dev, V,
                       P, hi, lo);
    const dim3 pgrid((unsigned)((maxpx + 255) / 256), V);
    const bool grad = grad_region >= 0 && dL_da;
    if (grad) {
        const int64_t nD = 6 * P;
        const int64_t fb = (nD + 255) / 256 < 8192 ? (nD + 255) / 256 : 8192;
        hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)fb), dim3(256), 0, st, D, nD);
        hipLaunchKernelGGL(k_hvsq_terms<true>, pgrid, dim3(256), 0, st, cams_dev, V, P, hi, lo, radius, region, R,
                           sums, counts, terms, grad_region, D);
        hipLaunchKernelGGL(k_hvsq_prefix_rows, dim3((unsigned)rows, 6), dim3(ROW_THREADS), 0, st, cams_dev, V, P, D);
        hipLaunchKernelGGL(k_hvsq_prefix_cols, dim3((unsigned)((colsD + 255) / 256), 6), dim3(256), 0, st, cams_dev,
                           V, P, D);
        hipLaunchKernelGGL(k_hvsq_grad, pgrid, dim3(256), 0, st, cams_dev, V, P, D, img_a, counts, R, grad_region,
                           dL_da);
    } else {
        hipLaunchKernelGGL(k_hvsq_terms<false>, pgrid, dim3(256), 0, st, cams_dev, V, P, hi, lo, radius, region, R,
                           sums, counts, terms, -1, nullptr);
    }
    return hipGetLastError();
}
