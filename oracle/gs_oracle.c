/*
 * FP64 CPU oracle for the tile-based Gaussian-splatting rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * HIP path is checked against.  It shares no code, header, table or constant
 * with the HIP library, and nothing in the product path may link or call it.
 *
 * What it computes (Section 2.1, Eq. 1a-1c; Section 3.2, Eq. 3; Section 4.1-4.2).
 * Scene parameters are taken as float64 (a float32 scene upcasts exactly):
 *   - projection of each 3D Gaussian to a screen-space ellipse with a
 *     view-dependent spherical-harmonic colour (the f and g of Eq. 1b/1c, which
 *     the paper defers to 3DGS; written here from first principles),
 *   - the tile/depth binning of the ellipses (Section 2.1, "Sorting"), in IEEE
 *     float32 on float32 inputs so that it is reproducible bit for bit,
 *   - per-pixel front-to-back compositing over every Gaussian covering the
 *     pixel in increasing depth (Eq. 1a) with the 3-sigma extent, the 1/255
 *     alpha skip, the 0.99 alpha clamp and the 1e-4 transmittance stop,
 *   - the dominated-pixel count Val_i of the efficiency metric (Eq. 3),
 *   - the foveated form: eccentricity rings with blend bands, per-level
 *     nested point subsets and per-level opacity/DC versions (Section 4.1-4.2),
 *   - the exact reverse pass of the compositing and of the projection.
 *
 * Where the paper is silent this file takes these readings: OpenCV camera
 * frame with pixel centres at integer coordinates; EWA projection with the
 * tangent clamped at 1.3x the half field of view inside the Jacobian and a
 * 0.3 px^2 low-pass added to the 2D covariance; a 3-sigma extent tested as
 * Mahalanobis distance <= 3; real orthonormal SH without the Condon-Shortley
 * phase, colour = max(0, SH . Y(dir) + 1/2); ties in depth ordered by
 * Gaussian index.
 *
 * Compositing decisions that sit within a small margin of a threshold
 * (Mahalanobis distance vs 3 sigma, alpha vs 1/255, transmittance vs 1e-4)
 * are flagged; for such pixels every consistent choice of those decisions is
 * enumerated and the envelope of the results is returned, because a float32
 * renderer may legitimately land on either side.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define OC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* camera: double row [19] = W, H, fx, fy, cx, cy, R[9] (row-major), t[3], near */
typedef struct {
    int w, h;
    double fx, fy, cx, cy, R[9], t[3], near_z;
} ocam;

static ocam cam_from_row(const double *r)
{
    ocam c;
    c.w = (int)r[0];
    c.h = (int)r[1];
    c.fx = r[2]; c.fy = r[3]; c.cx = r[4]; c.cy = r[5];
    for (int i = 0; i < 9; i++) c.R[i] = r[6 + i];
    for (int i = 0; i < 3; i++) c.t[i] = r[15 + i];
    c.near_z = r[18];
    return c;
}

/* camera centre in world space: -R^T t */
static void cam_center(const ocam *c, double o[3])
{
    for (int j = 0; j < 3; j++)
        o[j] = -(c->R[0 * 3 + j] * c->t[0] + c->R[1 * 3 + j] * c->t[1] + c->R[2 * 3 + j] * c->t[2]);
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics, l <= 3, orthonormal on the sphere, no
 * Condon-Shortley phase.  Y_lm = N_lm P_l^|m|(cos th) * {sqrt2 cos(m ph),
 * 1, sqrt2 sin(|m| ph)} for m > 0, m = 0, m < 0, with
 * N_lm = sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) and P_l^m the associated
 * Legendre function without the (-1)^m factor.  Index k = l^2 + l + m. */
static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; i++) f *= i;
    return f;
}

/* associated Legendre P_l^m(x), m >= 0, by the standard three-term recurrence */
static double assoc_legendre(int l, int m, double x)
{
    double s = sqrt(fmax(0.0, 1.0 - x * x));
    double pmm = 1.0;
    for (int i = 1; i <= m; i++) pmm *= (2.0 * i - 1.0) * s;
    if (l == m) return pmm;
    double pm1 = x * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return pm1;
    double pl = 0.0;
    for (int ll = m + 2; ll <= l; ll++) {
        pl = ((2.0 * ll - 1.0) * x * pm1 - (ll + m - 1.0) * pmm) / (ll - m);
        pmm = pm1;
        pm1 = pl;
    }
    return pl;
}

void oc_sh_basis(int degree, const double dir[3], double *Y)
{
    double x = dir[0], y = dir[1], z = dir[2];
    double ct = z;
    double ph = atan2(y, x);
    for (int l = 0; l <= degree; l++) {
        for (int m = -l; m <= l; m++) {
            int am = m < 0 ? -m : m;
            double N = sqrt((2.0 * l + 1.0) / (4.0 * OC_PI) * factorial(l - am) / factorial(l + am));
            double P = assoc_legendre(l, am, ct);
            double v;
            if (m > 0) v = sqrt(2.0) * N * P * cos(m * ph);
            else if (m < 0) v = sqrt(2.0) * N * P * sin(am * ph);
            else v = N * P;
            Y[l * l + l + m] = v;
        }
    }
}

/* Legendre polynomial P_l (l <= 3) as coefficients c[j] of z^j, from
 * Bonnet's recurrence (k + 1) P_{k+1} = (2k + 1) z P_k - k P_{k-1}. */
static void legendre_coeffs(int l, double c[4])
{
    double pm[4] = {1, 0, 0, 0}, p[4] = {0, 1, 0, 0};
    if (l == 0) { memcpy(c, pm, sizeof(pm)); return; }
    for (int k = 1; k < l; k++) {
        double nx[4] = {0, 0, 0, 0};
        for (int j = 0; j < 3; j++) nx[j + 1] += (2.0 * k + 1.0) * p[j];
        for (int j = 0; j < 4; j++) nx[j] = (nx[j] - k * pm[j]) / (k + 1.0);
        memcpy(pm, p, sizeof(p));
        memcpy(p, nx, sizeof(nx));
    }
    memcpy(c, p, sizeof(p));
}

/* d^m/dz^m of the polynomial sum_j c[j] z^j, evaluated at z */
static double poly_deriv(const double c[4], int m, double z)
{
    double s = 0.0;
    for (int j = m; j < 4; j++) {
        double f = c[j];
        for (int k = 0; k < m; k++) f *= (double)(j - k);
        double zp = 1.0;
        for (int k = 0; k < j - m; k++) zp *= z;
        s += f * zp;
    }
    return s;
}

/* Analytic derivative of Y_k(d / |d|) with respect to d at a unit d (3
 * partials per basis function).  On the unit sphere the basis above equals
 * the polynomial N_lm Q(z) A(x, y) with Q = d^|m| P_l / dz^|m| and A =
 * sqrt2 Re (x + iy)^m for m > 0, 1 for m = 0, sqrt2 Im (x + iy)^|m| for
 * m < 0, because (1 - z^2)^(|m|/2) e^(i |m| phi) = (x + iy)^|m| there.  The
 * derivative of Y(d / |d|) is that polynomial's Euclidean gradient with its
 * radial part removed, (I - d d^T) grad.  Used by the reverse pass.
 * Y (nullable) receives the polynomial form's values. */
void oc_sh_basis_grad(int degree, const double dir[3], double *Y, double *dY /* [K][3] */)
{
    double x = dir[0], y = dir[1], z = dir[2];
    for (int l = 0; l <= degree; l++) {
        double pc[4] = {0, 0, 0, 0};
        legendre_coeffs(l, pc);
        for (int m = -l; m <= l; m++) {
            int am = m < 0 ? -m : m;
            double N = sqrt((2.0 * l + 1.0) / (4.0 * OC_PI) * factorial(l - am) / factorial(l + am));
            double Q = poly_deriv(pc, am, z), dQ = poly_deriv(pc, am + 1, z);
            /* (x + iy)^am and (x + iy)^(am - 1) */
            double re = 1.0, im = 0.0, re1 = 1.0, im1 = 0.0;
            for (int k = 0; k < am; k++) {
                re1 = re; im1 = im;
                double r2 = re * x - im * y, i2 = re * y + im * x;
                re = r2; im = i2;
            }
            double A, Ax, Ay;
            if (m > 0) {
                A = sqrt(2.0) * re;
                Ax = sqrt(2.0) * am * re1;    /* d/dx (x+iy)^m = m (x+iy)^(m-1) */
                Ay = -sqrt(2.0) * am * im1;   /* d/dy = i m (x+iy)^(m-1) */
            } else if (m < 0) {
                A = sqrt(2.0) * im;
                Ax = sqrt(2.0) * am * im1;
                Ay = sqrt(2.0) * am * re1;
            } else {
                A = 1.0; Ax = 0.0; Ay = 0.0;
            }
            int k = l * l + l + m;
            double g[3] = {N * Ax * Q, N * Ay * Q, N * A * dQ};
            double rad = g[0] * x + g[1] * y + g[2] * z;
            for (int a = 0; a < 3; a++) dY[k * 3 + a] = g[a] - dir[a] * rad;
            if (Y) Y[k] = N * A * Q;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* rotation from a (w, x, y, z) quaternion, normalised first */
static void quat_to_rot(const double qi[4], double R[9])
{
    double n = sqrt(qi[0] * qi[0] + qi[1] * qi[1] + qi[2] * qi[2] + qi[3] * qi[3]);
    double w = qi[0] / n, x = qi[1] / n, y = qi[2] / n, z = qi[3] / n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static void matmul(const double *A, const double *B, double *C, int n, int k, int m)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < m; j++) {
            double s = 0.0;
            for (int l = 0; l < k; l++) s += A[i * k + l] * B[l * m + j];
            C[i * m + j] = s;
        }
}

static void transpose(const double *A, double *At, int n, int m)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < m; j++) At[j * n + i] = A[i * m + j];
}

/* ------------------------------------------------------------------------ */
/* Projection of one Gaussian, in float64.
 * Outputs: mean2d, cov2d (a, b, c of the dilated 2x2 covariance), conic
 * (A, B, C of its inverse), depth, opacity, colour, integer radius.
 * Returns 1 if visible, 0 if culled (then outputs are zero). */
typedef struct {
    double mean2d[2], cov2d[3], conic[3], depth, opacity, color[3], color_raw[3], radius;
    double u[3];          /* camera-space mean */
    double dir[3], dist;  /* unit view direction and distance, for SH */
    int visible;
} oproj;

static void project_one(const ocam *c, int sh_degree,
                        const double *mean, const double *log_scale, const double *quat,
                        double logit, const double *sh, const double *dc_override,
                        oproj *o)
{
    memset(o, 0, sizeof(*o));
    double mu[3] = {mean[0], mean[1], mean[2]};
    double u[3];
    for (int i = 0; i < 3; i++)
        u[i] = c->R[i * 3 + 0] * mu[0] + c->R[i * 3 + 1] * mu[1] + c->R[i * 3 + 2] * mu[2] + c->t[i];
    if (!(u[2] > c->near_z)) return;
    double z = u[2];
    double limx = 1.3 * (0.5 * c->w / c->fx), limy = 1.3 * (0.5 * c->h / c->fy);
    double tx = fmin(limx, fmax(-limx, u[0] / z));
    double ty = fmin(limy, fmax(-limy, u[1] / z));
    double J[6] = {c->fx / z, 0.0, -c->fx * tx / z,
                   0.0, c->fy / z, -c->fy * ty / z};
    double Rq[9], q[4] = {quat[0], quat[1], quat[2], quat[3]};
    quat_to_rot(q, Rq);
    double S2[9] = {0};
    for (int i = 0; i < 3; i++) {
        double s = exp((double)log_scale[i]);
        S2[i * 4] = s * s;
    }
    double tmp[9], RqT[9], Sig[9];
    matmul(Rq, S2, tmp, 3, 3, 3);
    transpose(Rq, RqT, 3, 3);
    matmul(tmp, RqT, Sig, 3, 3, 3);
    double T[6], Tt[6], TS[6], Cov[4];
    matmul(J, c->R, T, 2, 3, 3);
    transpose(T, Tt, 2, 3);
    matmul(T, Sig, TS, 2, 3, 3);
    matmul(TS, Tt, Cov, 2, 3, 2);
    double a = Cov[0] + 0.3, b = Cov[1], cc = Cov[3] + 0.3;
    double det = a * cc - b * b;
    if (!(det > 0.0)) return;
    o->cov2d[0] = a; o->cov2d[1] = b; o->cov2d[2] = cc;
    o->conic[0] = cc / det; o->conic[1] = -b / det; o->conic[2] = a / det;
    double mid = 0.5 * (a + cc);
    double lmax = mid + sqrt(fmax(mid * mid - det, 0.0));
    o->radius = ceil(3.0 * sqrt(lmax));
    o->mean2d[0] = c->fx * u[0] / z + c->cx;
    o->mean2d[1] = c->fy * u[1] / z + c->cy;
    o->depth = z;
    o->opacity = 1.0 / (1.0 + exp(-(double)logit));
    o->u[0] = u[0]; o->u[1] = u[1]; o->u[2] = u[2];
    /* colour */
    double cc3[3];
    cam_center(c, cc3);
    double d[3] = {mu[0] - cc3[0], mu[1] - cc3[1], mu[2] - cc3[2]};
    double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int i = 0; i < 3; i++) o->dir[i] = d[i] / n;
    o->dist = n;
    int K = (sh_degree + 1) * (sh_degree + 1);
    double Y[16];
    oc_sh_basis(sh_degree, o->dir, Y);
    for (int ch = 0; ch < 3; ch++) {
        double s = 0.0;
        for (int k = 0; k < K; k++) {
            double coef = (k == 0 && dc_override) ? dc_override[ch] : sh[k * 3 + ch];
            s += coef * Y[k];
        }
        o->color_raw[ch] = s + 0.5;
        o->color[ch] = fmax(0.0, s + 0.5);
    }
    o->visible = 1;
}

/* Batch projection for one camera.  Per-level outputs (lvl_opacity [L][n],
 * lvl_color [L][n][3]) are written when n_levels > 0; a NULL per-level array
 * means the level shares the base parameter. */
int oc_project(int n, int sh_degree, const double *means, const double *log_scales,
               const double *quats, const double *logits, const double *sh,
               const double *cam_row,
               double *mean2d, double *cov2d, double *conic, double *depth,
               double *opacity, double *color, int32_t *radius, uint8_t *visible,
               int n_levels, const double *lvl_logits, const double *lvl_dc,
               double *lvl_opacity, double *lvl_color)
{
    ocam c = cam_from_row(cam_row);
    int K = (sh_degree + 1) * (sh_degree + 1);
    for (int i = 0; i < n; i++) {
        oproj o;
        project_one(&c, sh_degree, means + 3 * i, log_scales + 3 * i, quats + 4 * i,
                    logits[i], sh + (size_t)i * K * 3, NULL, &o);
        mean2d[2 * i] = o.mean2d[0]; mean2d[2 * i + 1] = o.mean2d[1];
        for (int j = 0; j < 3; j++) {
            if (cov2d) cov2d[3 * i + j] = o.cov2d[j];
            conic[3 * i + j] = o.conic[j];
            color[3 * i + j] = o.color[j];
        }
        depth[i] = o.depth;
        opacity[i] = o.opacity;
        radius[i] = (int32_t)o.radius;
        visible[i] = (uint8_t)o.visible;
        for (int t = 0; t < n_levels; t++) {
            double lg = lvl_logits ? lvl_logits[(size_t)t * n + i] : logits[i];
            const double *dc = lvl_dc ? lvl_dc + ((size_t)t * n + i) * 3 : NULL;
            oproj ol;
            project_one(&c, sh_degree, means + 3 * i, log_scales + 3 * i, quats + 4 * i,
                        lg, sh + (size_t)i * K * 3, dc, &ol);
            lvl_opacity[(size_t)t * n + i] = ol.opacity;
            for (int j = 0; j < 3; j++) lvl_color[((size_t)t * n + i) * 3 + j] = ol.color[j];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Binning in IEEE float32 (stage-wise contract).
 * Pixel column range of Gaussian i: [ceil(mx - r), floor(mx + r)] clipped to
 * [0, W-1], evaluated in float32 from the float32 mean and the integer
 * radius; same for rows.  Tile range = pixel range / tile size.  A Gaussian
 * with radius 0 or an empty range touches no tile.  With a tile level table
 * and quality bounds, tile g is kept for Gaussian i only if
 * level_lo[g] <= m_i (Section 4.2, filtering).
 * Keys: (global tile << 32) | float32 bits of depth; value i.  Emission order
 * is (view, i, tile row-major); the output is that list stably sorted by key. */
static int rect_f32(float mx, float my, int r, int W, int H, int T,
                    int *tx0, int *tx1, int *ty0, int *ty1)
{
    if (r <= 0) return 0;
    float fr = (float)r;
    volatile float xl = mx - fr, xh = mx + fr, yl = my - fr, yh = my + fr;
    float x0 = ceilf(xl), x1 = floorf(xh), y0 = ceilf(yl), y1 = floorf(yh);
    if (!(x0 <= x1) || !(y0 <= y1)) return 0;
    if (x0 < 0.0f) x0 = 0.0f;
    if (y0 < 0.0f) y0 = 0.0f;
    if (x1 > (float)(W - 1)) x1 = (float)(W - 1);
    if (y1 > (float)(H - 1)) y1 = (float)(H - 1);
    if (!(x0 <= x1) || !(y0 <= y1)) return 0;
    *tx0 = (int)x0 / T; *tx1 = (int)x1 / T;
    *ty0 = (int)y0 / T; *ty1 = (int)y1 / T;
    return 1;
}

typedef struct { uint64_t key; uint64_t order; uint32_t val; } okey;

static int okey_cmp(const void *a, const void *b)
{
    const okey *x = (const okey *)a, *y = (const okey *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->order < y->order ? -1 : (x->order > y->order);
}

/* Pass keys == NULL to get only the count (returned).  widths/heights per view. */
int64_t oc_bin_f32(int V, int n, const float *mean2d /*[V][n][2]*/,
                   const int32_t *radius /*[V][n]*/, const float *depth /*[V][n]*/,
                   const int32_t *widths, const int32_t *heights, int T,
                   const uint8_t *tile_level_lo /*[tiles] or NULL*/,
                   const uint8_t *qbound /*[n] or NULL*/,
                   uint32_t *hits /*[V][n]*/, uint64_t *keys, uint32_t *vals,
                   uint32_t *ranges /*[tiles][2] or NULL*/, int64_t capacity)
{
    int64_t total = 0;
    int64_t tile_off = 0;
    /* pass 1: counts */
    for (int v = 0; v < V; v++) {
        int W = widths[v], H = heights[v];
        int tiles_x = (W + T - 1) / T;
        for (int i = 0; i < n; i++) {
            size_t e = (size_t)v * n + i;
            int tx0, tx1, ty0, ty1;
            uint32_t cnt = 0;
            if (rect_f32(mean2d[2 * e], mean2d[2 * e + 1], radius[e], W, H, T, &tx0, &tx1, &ty0, &ty1)) {
                for (int ty = ty0; ty <= ty1; ty++)
                    for (int tx = tx0; tx <= tx1; tx++) {
                        int64_t g = tile_off + (int64_t)ty * tiles_x + tx;
                        if (tile_level_lo && qbound && !(tile_level_lo[g] <= qbound[i])) continue;
                        cnt++;
                    }
            }
            hits[e] = cnt;
            total += cnt;
        }
        tile_off += (int64_t)tiles_x * ((H + T - 1) / T);
    }
    if (!keys) return total;
    if (total > capacity) return -total;
    okey *buf = (okey *)malloc(sizeof(okey) * (size_t)(total ? total : 1));
    int64_t k = 0;
    tile_off = 0;
    for (int v = 0; v < V; v++) {
        int W = widths[v], H = heights[v];
        int tiles_x = (W + T - 1) / T;
        for (int i = 0; i < n; i++) {
            size_t e = (size_t)v * n + i;
            int tx0, tx1, ty0, ty1;
            if (!rect_f32(mean2d[2 * e], mean2d[2 * e + 1], radius[e], W, H, T, &tx0, &tx1, &ty0, &ty1))
                continue;
            uint32_t dbits;
            memcpy(&dbits, &depth[e], 4);
            for (int ty = ty0; ty <= ty1; ty++)
                for (int tx = tx0; tx <= tx1; tx++) {
                    int64_t g = tile_off + (int64_t)ty * tiles_x + tx;
                    if (tile_level_lo && qbound && !(tile_level_lo[g] <= qbound[i])) continue;
                    buf[k].key = ((uint64_t)g << 32) | dbits;
                    buf[k].order = (uint64_t)k;
                    buf[k].val = (uint32_t)i;
                    k++;
                }
        }
        tile_off += (int64_t)tiles_x * ((H + T - 1) / T);
    }
    qsort(buf, (size_t)total, sizeof(okey), okey_cmp);
    for (int64_t j = 0; j < total; j++) {
        keys[j] = buf[j].key;
        vals[j] = buf[j].val;
    }
    if (ranges) {
        memset(ranges, 0, sizeof(uint32_t) * 2 * (size_t)tile_off);
        for (int64_t j = 0; j < total; j++) {
            uint64_t g = buf[j].key >> 32;
            if (j == 0 || (buf[j - 1].key >> 32) != g) ranges[2 * g] = (uint32_t)j;
            if (j == total - 1 || (buf[j + 1].key >> 32) != g) ranges[2 * g + 1] = (uint32_t)(j + 1);
        }
    }
    free(buf);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Per-pixel compositing (Eq. 1a) with branch enumeration at thresholds.    */

typedef struct {
    /* splats, float64, one view */
    int n;
    const double *mean2d, *conic, *depth, *opacity, *color;
    const int32_t *radius;
    /* optional: level filter and per-level parameters */
    const uint8_t *qbound;
    const double *lvl_opacity, *lvl_color; /* [L][n], [L][n][3] or NULL */
    int W, H;
    double bg[3];
    double dq, de, dT, ddom; /* ambiguity margins */
    int max_leaves;
    /* candidate rows (CSR): for row y, ids in depth order */
    const int64_t *row_ptr;
    const int32_t *row_ids;
} cctx;

typedef struct {
    double rgb_min[3], rgb_max[3];
    double T_min, T_max;
    int leaves, unresolved;
    /* primary branch (fp64 decisions) */
    double rgb[3], T;
    int last_id;   /* id of the last blended Gaussian, -1 if none */
    int n_blend;
    int dom_id;    /* argmax of T*alpha, -1 if none */
    double dom_val, second_val;
    int amb;       /* bit0: threshold branch, bit1: dominance tie */
    int last_ids[4], n_last;   /* distinct last ids over branches */
    int dom_ids[4], n_dom;     /* distinct dominators over branches (incl. ties) */
} cres;

typedef struct {
    int k;               /* position in candidate list */
    double C[3], T, Terr;
    int last_id, n_blend;
    int dom_id, second_id;
    double dom_val, second_val;
    int primary;
} cstate;

static void add_id(int *arr, int *n, int id)
{
    for (int i = 0; i < *n; i++) if (arr[i] == id) return;
    if (*n < 4) arr[(*n)++] = id;
}

static void finish_leaf(const cctx *X, cres *R, const cstate *s)
{
    double out[3];
    for (int ch = 0; ch < 3; ch++) out[ch] = s->C[ch] + s->T * X->bg[ch];
    if (R->leaves == 0) {
        for (int ch = 0; ch < 3; ch++) R->rgb_min[ch] = R->rgb_max[ch] = out[ch];
        R->T_min = R->T_max = s->T;
    } else {
        for (int ch = 0; ch < 3; ch++) {
            R->rgb_min[ch] = fmin(R->rgb_min[ch], out[ch]);
            R->rgb_max[ch] = fmax(R->rgb_max[ch], out[ch]);
        }
        R->T_min = fmin(R->T_min, s->T);
        R->T_max = fmax(R->T_max, s->T);
    }
    R->leaves++;
    add_id(R->last_ids, &R->n_last, s->last_id);
    add_id(R->dom_ids, &R->n_dom, s->dom_id);
    /* a near-tie for the largest contribution admits the runner-up too */
    if (s->dom_id >= 0 && s->second_id >= 0 && s->dom_val - s->second_val <= X->ddom * s->dom_val)
        add_id(R->dom_ids, &R->n_dom, s->second_id);
    if (s->primary) {
        for (int ch = 0; ch < 3; ch++) R->rgb[ch] = out[ch];
        R->T = s->T;
        R->last_id = s->last_id;
        R->n_blend = s->n_blend;
        R->dom_id = s->dom_id;
        R->dom_val = s->dom_val;
        R->second_val = s->second_val;
        if (s->dom_id >= 0 && s->dom_val - s->second_val <= X->ddom * s->dom_val) R->amb |= 2;
    }
}

/* Walk the candidate list from state s.  'level' >= 1 selects the FR level
 * (filter m_i >= level and use that level's opacity/colour); 0 = plain. */
static void walk(const cctx *X, cres *R, cstate s, double px, double py,
                 const int32_t *cand, int ncand, int level)
{
    for (; s.k < ncand; s.k++) {
        int i = cand[s.k];
        if (level > 0 && X->qbound && !(X->qbound[i] >= level)) continue;
        double dx = px - X->mean2d[2 * i], dy = py - X->mean2d[2 * i + 1];
        /* outside the bounding square (half-width r, plus one pixel): the
         * 3-sigma ellipse cannot cover this pixel */
        if (fabs(dx) > X->radius[i] + 1.0) continue;
        double A = X->conic[3 * i], B = X->conic[3 * i + 1], Cc = X->conic[3 * i + 2];
        double q = A * dx * dx + 2.0 * B * dx * dy + Cc * dy * dy;
        double sabs = fabs(A * dx * dx) + fabs(2.0 * B * dx * dy) + fabs(Cc * dy * dy);
        double o = X->opacity[i];
        const double *col = X->color + 3 * i;
        if (level > 0 && X->lvl_opacity) o = X->lvl_opacity[(size_t)(level - 1) * X->n + i];
        if (level > 0 && X->lvl_color) col = X->lvl_color + ((size_t)(level - 1) * X->n + i) * 3;
        /* decision 1: inside the 3-sigma ellipse (q <= 9) */
        int inc = q <= 9.0;
        int amb_inc = fabs(q - 9.0) <= X->dq * (sabs + 1e-30);
        if (!inc && !amb_inc) continue;
        double e = log(o) - 0.5 * q;            /* ln(o G) */
        double a_raw = exp(e);
        double alpha = fmin(0.99, a_raw);
        double err_e = X->de * (1.0 + 0.5 * sabs);
        /* decision 2: alpha >= 1/255 */
        int pass = alpha >= 1.0 / 255.0;
        int amb_pass = a_raw < 0.99 && fabs(e - log(1.0 / 255.0)) <= err_e;
        int use = inc && pass;
        int amb_use = amb_inc || amb_pass;
        if (amb_use && R->leaves + 1 < X->max_leaves) {
            /* explore the flipped branch as a non-primary path */
            cstate alt = s;
            alt.primary = 0;
            R->amb |= 1;
            if (use) {
                /* flipped: skip this Gaussian */
                alt.k = s.k + 1;
                walk(X, R, alt, px, py, cand, ncand, level);
            } else {
                /* flipped: blend it (with the value the formula gives) */
                double Tn = alt.T * (1.0 - alpha);
                if (Tn < 1e-4) {
                    finish_leaf(X, R, &alt);
                } else {
                    double w = alpha * alt.T;
                    for (int ch = 0; ch < 3; ch++) alt.C[ch] += col[ch] * w;
                    if (w > alt.dom_val) { alt.second_val = alt.dom_val; alt.second_id = alt.dom_id; alt.dom_val = w; alt.dom_id = i; }
                    else if (w > alt.second_val) { alt.second_val = w; alt.second_id = i; }
                    alt.T = Tn;
                    alt.last_id = i;
                    alt.n_blend++;
                    alt.k = s.k + 1;
                    walk(X, R, alt, px, py, cand, ncand, level);
                }
            }
        } else if (amb_use) {
            R->unresolved = 1;
        }
        if (!use) continue;
        /* decision 3: transmittance stop */
        double Tn = s.T * (1.0 - alpha);
        int stop = Tn < 1e-4;
        double relerr = s.Terr + alpha / fmax(1e-12, 1.0 - alpha) * err_e;
        int amb_stop = fabs(Tn - 1e-4) <= (relerr + X->dT) * 1e-4;
        if (amb_stop && R->leaves + 1 < X->max_leaves) {
            cstate alt = s;
            alt.primary = 0;
            R->amb |= 1;
            if (stop) {
                /* flipped: continue blending */
                double w = alpha * alt.T;
                for (int ch = 0; ch < 3; ch++) alt.C[ch] += col[ch] * w;
                if (w > alt.dom_val) { alt.second_val = alt.dom_val; alt.second_id = alt.dom_id; alt.dom_val = w; alt.dom_id = i; }
                else if (w > alt.second_val) { alt.second_val = w; alt.second_id = i; }
                alt.T = Tn;
                alt.Terr = relerr;
                alt.last_id = i;
                alt.n_blend++;
                alt.k = s.k + 1;
                walk(X, R, alt, px, py, cand, ncand, level);
            } else {
                finish_leaf(X, R, &alt);
            }
        } else if (amb_stop) {
            R->unresolved = 1;
        }
        if (stop) {
            finish_leaf(X, R, &s);
            return;
        }
        double w = alpha * s.T;
        for (int ch = 0; ch < 3; ch++) s.C[ch] += col[ch] * w;
        if (w > s.dom_val) { s.second_val = s.dom_val; s.second_id = s.dom_id; s.dom_val = w; s.dom_id = i; }
        else if (w > s.second_val) { s.second_val = w; s.second_id = i; }
        s.T = Tn;
        s.Terr = relerr;
        s.last_id = i;
        s.n_blend++;
    }
    finish_leaf(X, R, &s);
}

static void composite_pixel(const cctx *X, int px, int py, int level, cres *R)
{
    memset(R, 0, sizeof(*R));
    R->last_id = -1;
    R->dom_id = -1;
    cstate s;
    memset(&s, 0, sizeof(s));
    s.T = 1.0;
    s.last_id = -1;
    s.dom_id = -1;
    s.second_id = -1;
    s.primary = 1;
    s.Terr = 1e-7;
    const int32_t *cand = X->row_ids + X->row_ptr[py];
    int ncand = (int)(X->row_ptr[py + 1] - X->row_ptr[py]);
    /* candidates for this row; the x-range filter is applied per Gaussian
     * inside walk() through the ellipse test, the row list only prunes
     * Gaussians whose bounding square misses this row */
    walk(X, R, s, (double)px, (double)py, cand, ncand, level);
}

/* Build per-row candidate lists in (depth, index) order: Gaussian i is a
 * candidate for rows [ceil(my - r - 1), floor(my + r + 1)]; the 3-sigma
 * ellipse lies inside the square of half-width r, so no pixel it covers is
 * missed. */
typedef struct { double d; int32_t i; } didx;

static int didx_cmp(const void *a, const void *b)
{
    const didx *x = (const didx *)a, *y = (const didx *)b;
    if (x->d != y->d) return x->d < y->d ? -1 : 1;
    return x->i - y->i;
}

static void build_rows(int n, const double *mean2d, const double *depth, const int32_t *radius,
                       int W, int H, const uint8_t *qbound, int min_level,
                       int64_t **row_ptr_out, int32_t **row_ids_out)
{
    (void)W;
    didx *ord = (didx *)malloc(sizeof(didx) * (size_t)(n ? n : 1));
    int nv = 0;
    for (int i = 0; i < n; i++) {
        if (radius[i] <= 0) continue;
        if (qbound && min_level > 0 && !(qbound[i] >= min_level)) continue;
        ord[nv].d = depth[i];
        ord[nv].i = i;
        nv++;
    }
    qsort(ord, (size_t)nv, sizeof(didx), didx_cmp);
    int64_t *cnt = (int64_t *)calloc((size_t)H + 1, sizeof(int64_t));
    for (int j = 0; j < nv; j++) {
        int i = ord[j].i;
        double r = radius[i] + 1.0;
        double y0 = ceil(mean2d[2 * i + 1] - r), y1 = floor(mean2d[2 * i + 1] + r);
        if (y0 < 0) y0 = 0;
        if (y1 > H - 1) y1 = H - 1;
        for (int y = (int)y0; y <= (int)y1; y++) cnt[y + 1]++;
    }
    for (int y = 0; y < H; y++) cnt[y + 1] += cnt[y];
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cnt[H] ? cnt[H] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(H ? H : 1));
    for (int y = 0; y < H; y++) fill[y] = cnt[y];
    for (int j = 0; j < nv; j++) {
        int i = ord[j].i;
        double r = radius[i] + 1.0;
        double y0 = ceil(mean2d[2 * i + 1] - r), y1 = floor(mean2d[2 * i + 1] + r);
        if (y0 < 0) y0 = 0;
        if (y1 > H - 1) y1 = H - 1;
        for (int y = (int)y0; y <= (int)y1; y++) ids[fill[y]++] = i;
    }
    free(fill);
    free(ord);
    *row_ptr_out = cnt;
    *row_ids_out = ids;
}

typedef struct {
    const cctx *X;
    int npx;
    const int32_t *px;      /* [npx][2] or NULL for all pixels */
    const uint8_t *pix_lo;  /* FR: per-pixel lower level (1-based) or NULL */
    const double *pix_w;    /* FR: per-pixel weight of level lo+1 */
    /* outputs per pixel */
    double *rgb, *rgb_min, *rgb_max, *T;
    int32_t *last_id, *dom_id, *amb, *n_blend;
    int32_t *last_set, *dom_set; /* [npx][4], -2 padded */
    int next;
    pthread_mutex_t mu;
} cjob;

static void write_res(cjob *J, int p, const cres *R)
{
    for (int ch = 0; ch < 3; ch++) {
        J->rgb[3 * p + ch] = R->rgb[ch];
        if (J->rgb_min) J->rgb_min[3 * p + ch] = R->rgb_min[ch];
        if (J->rgb_max) J->rgb_max[3 * p + ch] = R->rgb_max[ch];
    }
    if (J->T) J->T[p] = R->T;
    if (J->last_id) J->last_id[p] = R->last_id;
    if (J->dom_id) J->dom_id[p] = R->dom_id;
    if (J->n_blend) J->n_blend[p] = R->n_blend;
    if (J->amb) J->amb[p] = R->amb | (R->unresolved ? 4 : 0);
    if (J->last_set)
        for (int j = 0; j < 4; j++) J->last_set[4 * p + j] = j < R->n_last ? R->last_ids[j] : -2;
    if (J->dom_set) {
        int ids[4], nd = R->n_dom;
        memcpy(ids, R->dom_ids, sizeof(ids));
        for (int j = 0; j < 4; j++) J->dom_set[4 * p + j] = j < nd ? ids[j] : -2;
    }
}

static void *cworker(void *arg)
{
    cjob *J = (cjob *)arg;
    const cctx *X = J->X;
    for (;;) {
        pthread_mutex_lock(&J->mu);
        int p0 = J->next;
        J->next += 64;
        pthread_mutex_unlock(&J->mu);
        if (p0 >= J->npx) break;
        int p1 = p0 + 64 < J->npx ? p0 + 64 : J->npx;
        for (int p = p0; p < p1; p++) {
            int x = J->px ? J->px[2 * p] : p % X->W;
            int y = J->px ? J->px[2 * p + 1] : p / X->W;
            cres R;
            if (!J->pix_lo) {
                composite_pixel(X, x, y, 0, &R);
            } else {
                /* FR: blend the composites of level lo and (if weighted) lo+1 */
                size_t pp = (size_t)y * X->W + x;
                int lo = J->pix_lo[pp];
                double w = J->pix_w[pp];
                cres Ra, Rb;
                composite_pixel(X, x, y, lo, &Ra);
                R = Ra;
                if (w > 0.0) {
                    composite_pixel(X, x, y, lo + 1, &Rb);
                    for (int ch = 0; ch < 3; ch++) {
                        R.rgb[ch] = (1.0 - w) * Ra.rgb[ch] + w * Rb.rgb[ch];
                        double m1 = (1.0 - w) * Ra.rgb_min[ch] + w * Rb.rgb_min[ch];
                        double m2 = (1.0 - w) * Ra.rgb_max[ch] + w * Rb.rgb_max[ch];
                        R.rgb_min[ch] = m1;
                        R.rgb_max[ch] = m2;
                    }
                    R.amb |= Rb.amb;
                    R.unresolved |= Rb.unresolved;
                }
            }
            write_res(J, p, &R);
        }
    }
    return NULL;
}

static int nthreads_default(int nt)
{
    if (nt > 0) return nt;
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    return c > 0 ? (int)c : 1;
}

static void run_jobs(cjob *J, int nthreads)
{
    nthreads = nthreads_default(nthreads);
    pthread_mutex_init(&J->mu, NULL);
    J->next = 0;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, cworker, J);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&J->mu);
}

/* Composite an image (px == NULL: all W*H pixels, row-major) or a pixel list.
 * margins: dq (relative, on the 3-sigma test), de (on ln alpha), dT (on the
 * stop), ddom (relative dominance tie).  For FR pass qbound, the per-level
 * parameters and the per-pixel level table (pix_lo 1-based, pix_w). */
int oc_composite(int n, const double *mean2d, const double *conic, const double *depth,
                 const double *opacity, const double *color, const int32_t *radius,
                 int W, int H, const double *bg,
                 const uint8_t *qbound, const double *lvl_opacity, const double *lvl_color,
                 const uint8_t *pix_lo, const double *pix_w,
                 int npx, const int32_t *px,
                 const double *margins, int max_leaves,
                 double *rgb, double *rgb_min, double *rgb_max, double *T,
                 int32_t *last_id, int32_t *dom_id, int32_t *amb, int32_t *n_blend,
                 int32_t *last_set, int32_t *dom_set, int nthreads)
{
    cctx X;
    memset(&X, 0, sizeof(X));
    X.n = n;
    X.mean2d = mean2d; X.conic = conic; X.depth = depth; X.opacity = opacity; X.color = color;
    X.radius = radius;
    X.qbound = qbound;
    X.lvl_opacity = lvl_opacity;
    X.lvl_color = lvl_color;
    X.W = W; X.H = H;
    for (int ch = 0; ch < 3; ch++) X.bg[ch] = bg[ch];
    X.dq = margins[0]; X.de = margins[1]; X.dT = margins[2]; X.ddom = margins[3];
    X.max_leaves = max_leaves;
    int64_t *row_ptr;
    int32_t *row_ids;
    build_rows(n, mean2d, depth, radius, W, H, NULL, 0, &row_ptr, &row_ids);
    X.row_ptr = row_ptr;
    X.row_ids = row_ids;
    cjob J;
    memset(&J, 0, sizeof(J));
    J.X = &X;
    J.npx = px ? npx : W * H;
    J.px = px;
    J.pix_lo = pix_lo;
    J.pix_w = pix_w;
    J.rgb = rgb; J.rgb_min = rgb_min; J.rgb_max = rgb_max; J.T = T;
    J.last_id = last_id; J.dom_id = dom_id; J.amb = amb; J.n_blend = n_blend;
    J.last_set = last_set; J.dom_set = dom_set;
    run_jobs(&J, nthreads);
    free(row_ptr);
    free(row_ids);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Foveation (Section 4.1, Section 6).  Eccentricity of pixel p = angle
 * between the pinhole ray through p and the ray through the gaze pixel.
 * Ring boundaries b_1 < ... < b_{L-1} (degrees); around each boundary a band
 * of total width w blends level j and j+1 with a linear ramp in
 * eccentricity.  Per pixel: lower level lo (1-based) and weight of lo+1.
 * Per tile: lowest and highest level with non-zero weight over its pixels.
 * 'amb' marks pixels within eps degrees of a band edge. */
int oc_fovea(const double *cam_row, const double *fov_row /* gx, gy, b1..b_{L-1}, band */,
             int n_levels, int T, double eps,
             uint8_t *pix_lo, double *pix_w, double *ecc_out, uint8_t *pix_amb,
             uint8_t *tile_lo, uint8_t *tile_hi, uint8_t *tile_amb)
{
    ocam c = cam_from_row(cam_row);
    double gx = fov_row[0], gy = fov_row[1];
    const double *b = fov_row + 2;
    double band = fov_row[2 + n_levels - 1];
    double g[3] = {(gx - c.cx) / c.fx, (gy - c.cy) / c.fy, 1.0};
    int tiles_x = (c.w + T - 1) / T, tiles_y = (c.h + T - 1) / T;
    for (int t = 0; t < tiles_x * tiles_y; t++) {
        tile_lo[t] = 255;
        tile_hi[t] = 0;
        tile_amb[t] = 0;
    }
    for (int y = 0; y < c.h; y++)
        for (int x = 0; x < c.w; x++) {
            double r[3] = {(x - c.cx) / c.fx, (y - c.cy) / c.fy, 1.0};
            double cr[3] = {r[1] * g[2] - r[2] * g[1], r[2] * g[0] - r[0] * g[2], r[0] * g[1] - r[1] * g[0]};
            double cn = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
            double dt = r[0] * g[0] + r[1] * g[1] + r[2] * g[2];
            double ecc = atan2(cn, dt) * 180.0 / OC_PI;
            int lo = 1;
            double w = 0.0;
            int amb = 0;
            for (int j = 0; j < n_levels - 1; j++) {
                double e0 = b[j] - 0.5 * band, e1 = b[j] + 0.5 * band;
                if (fabs(ecc - e0) <= eps || fabs(ecc - e1) <= eps) amb = 1;
                if (ecc < e0) break;
                if (ecc < e1) {
                    lo = j + 1;
                    w = (ecc - e0) / band;
                    break;
                }
                lo = j + 2;
            }
            size_t p = (size_t)y * c.w + x;
            pix_lo[p] = (uint8_t)lo;
            pix_w[p] = w;
            if (ecc_out) ecc_out[p] = ecc;
            if (pix_amb) pix_amb[p] = (uint8_t)amb;
            int hi = lo + (w > 0.0 ? 1 : 0);
            int t = (y / T) * tiles_x + x / T;
            if (lo < tile_lo[t]) tile_lo[t] = (uint8_t)lo;
            if (hi > tile_hi[t]) tile_hi[t] = (uint8_t)hi;
            if (amb) tile_amb[t] = 1;
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Reverse pass.                                                            */
/* Stage 1: compositing backward.  For every pixel, the forward is re-run in
 * FP64 and the blended Gaussians (id, alpha, T, G, dx, dy, clamped) are kept
 * in order; gradients of I = sum c_k a_k T_k + T_end bg then follow from
 * dI/dc_k = a_k T_k and dI/da_k = c_k T_k - B_k / (1 - a_k), with B_k the
 * light arriving from behind k (including the background).  No per-pixel
 * decision is differentiated (skip, extent, stop are constant).
 * Outputs per Gaussian: d mean2d (2), d conic (A, B, C), d opacity, d colour (3). */
typedef struct { int id; double a, T, G, dx, dy; int clamped; } contrib;

int oc_composite_bwd(int n, const double *mean2d, const double *conic, const double *depth,
                     const double *opacity, const double *color, const int32_t *radius,
                     int W, int H, const double *bg, const double *dL_dimg /* [3][H][W] */,
                     double *d_mean2d, double *d_conic, double *d_opacity, double *d_color)
{
    int64_t *row_ptr;
    int32_t *row_ids;
    build_rows(n, mean2d, depth, radius, W, H, NULL, 0, &row_ptr, &row_ids);
    memset(d_mean2d, 0, sizeof(double) * 2 * (size_t)n);
    memset(d_conic, 0, sizeof(double) * 3 * (size_t)n);
    memset(d_opacity, 0, sizeof(double) * (size_t)n);
    memset(d_color, 0, sizeof(double) * 3 * (size_t)n);
    int cap = 1024;
    contrib *list = (contrib *)malloc(sizeof(contrib) * (size_t)cap);
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            const int32_t *cand = row_ids + row_ptr[y];
            int ncand = (int)(row_ptr[y + 1] - row_ptr[y]);
            int m = 0;
            double T = 1.0;
            for (int k = 0; k < ncand; k++) {
                int i = cand[k];
                double dx = x - mean2d[2 * i], dy = y - mean2d[2 * i + 1];
                if (fabs(dx) > radius[i] + 1.0) continue;
                double A = conic[3 * i], B = conic[3 * i + 1], C = conic[3 * i + 2];
                double q = A * dx * dx + 2.0 * B * dx * dy + C * dy * dy;
                if (!(q <= 9.0)) continue;
                double G = exp(-0.5 * q);
                double a = opacity[i] * G;
                int clamped = a > 0.99;
                if (clamped) a = 0.99;
                if (a < 1.0 / 255.0) continue;
                double Tn = T * (1.0 - a);
                if (Tn < 1e-4) break;
                if (m == cap) {
                    cap *= 2;
                    list = (contrib *)realloc(list, sizeof(contrib) * (size_t)cap);
                }
                list[m].id = i; list[m].a = a; list[m].T = T; list[m].G = G;
                list[m].dx = dx; list[m].dy = dy; list[m].clamped = clamped;
                m++;
                T = Tn;
            }
            double g[3];
            for (int ch = 0; ch < 3; ch++) g[ch] = dL_dimg[(size_t)ch * W * H + (size_t)y * W + x];
            double Bk[3] = {bg[0] * T, bg[1] * T, bg[2] * T}; /* behind the last one */
            for (int k = m - 1; k >= 0; k--) {
                contrib *c = &list[k];
                int i = c->id;
                double dLda = 0.0;
                for (int ch = 0; ch < 3; ch++) {
                    double cc = color[3 * i + ch];
                    d_color[3 * i + ch] += g[ch] * c->a * c->T;
                    dLda += g[ch] * (cc * c->T - Bk[ch] / (1.0 - c->a));
                }
                for (int ch = 0; ch < 3; ch++) Bk[ch] += color[3 * i + ch] * c->a * c->T;
                if (c->clamped) continue;
                /* a = o G, G = exp(-q/2) */
                d_opacity[i] += dLda * c->G;
                double dLdq = dLda * opacity[i] * c->G * (-0.5);
                double dx = c->dx, dy = c->dy;
                double A = conic[3 * i], B = conic[3 * i + 1], C = conic[3 * i + 2];
                /* q = A dx^2 + 2 B dx dy + C dy^2, dx = px - mean */
                d_conic[3 * i] += dLdq * dx * dx;
                d_conic[3 * i + 1] += dLdq * 2.0 * dx * dy;
                d_conic[3 * i + 2] += dLdq * dy * dy;
                d_mean2d[2 * i] += dLdq * -(2.0 * A * dx + 2.0 * B * dy);
                d_mean2d[2 * i + 1] += dLdq * -(2.0 * B * dx + 2.0 * C * dy);
            }
        }
    free(list);
    free(row_ptr);
    free(row_ids);
    return 0;
}

/* Stage 2: projection backward for one camera.  From per-Gaussian gradients
 * of (mean2d, conic, opacity, colour) to the parameters, in matrix form:
 *   conic = S'^-1           -> dS' = -M G M  (G the symmetric conic gradient)
 *   S' = T Sig T^T + 0.3 I  -> dSig = T^T dS' T,  dT = 2 dS' T Sig
 *   T = J Rc                -> dJ = dT Rc^T
 *   J(u), mean2d(u)         -> du (through the clamped tan terms)
 *   u = Rc mu + t           -> dmu += Rc^T du
 *   Sig = M M^T, M = Rq S   -> dM = 2 dSig M, ds, dRq
 *   Rq(q / |q|)             -> dq
 *   colour = max(0, sum sh Y(dir) + 1/2), dir = (mu - c)/|mu - c|
 *   opacity = sigmoid(logit)
 * Gradients are ADDED into the outputs (so views can be summed). */
int oc_project_bwd(int n, int sh_degree, const double *means, const double *log_scales,
                   const double *quats, const double *logits, const double *sh,
                   const double *cam_row,
                   const double *d_mean2d, const double *d_conic, const double *d_opacity,
                   const double *d_color,
                   double *g_means, double *g_log_scales, double *g_quats, double *g_logits,
                   double *g_sh)
{
    ocam c = cam_from_row(cam_row);
    int K = (sh_degree + 1) * (sh_degree + 1);
    for (int i = 0; i < n; i++) {
        oproj o;
        project_one(&c, sh_degree, means + 3 * i, log_scales + 3 * i, quats + 4 * i, logits[i],
                    sh + (size_t)i * K * 3, NULL, &o);
        if (!o.visible) continue;
        /* opacity */
        g_logits[i] += d_opacity[i] * o.opacity * (1.0 - o.opacity);
        /* colour -> SH and direction */
        double Y[16], dY[48];
        oc_sh_basis(sh_degree, o.dir, Y);
        oc_sh_basis_grad(sh_degree, o.dir, NULL, dY);
        double ddir[3] = {0, 0, 0};
        for (int ch = 0; ch < 3; ch++) {
            if (!(o.color_raw[ch] > 0.0)) continue;
            double gc = d_color[3 * i + ch];
            for (int k = 0; k < K; k++) {
                g_sh[((size_t)i * K + k) * 3 + ch] += gc * Y[k];
                for (int a = 0; a < 3; a++) ddir[a] += gc * sh[((size_t)i * K + k) * 3 + ch] * dY[k * 3 + a];
            }
        }
        /* dir = d / |d| -> dd = (ddir - dir (dir . ddir)) / |d| */
        double dd = o.dir[0] * ddir[0] + o.dir[1] * ddir[1] + o.dir[2] * ddir[2];
        for (int a = 0; a < 3; a++) g_means[3 * i + a] += (ddir[a] - o.dir[a] * dd) / o.dist;
        /* conic -> cov2d */
        double M[4] = {o.conic[0], o.conic[1], o.conic[1], o.conic[2]};
        double G[4] = {d_conic[3 * i], 0.5 * d_conic[3 * i + 1], 0.5 * d_conic[3 * i + 1], d_conic[3 * i + 2]};
        double MG[4], dS[4];
        matmul(M, G, MG, 2, 2, 2);
        matmul(MG, M, dS, 2, 2, 2);
        for (int k = 0; k < 4; k++) dS[k] = -dS[k];
        /* dS is the gradient w.r.t. the full symmetric matrix S' (entries
         * counted once each); S' = T Sig T^T + 0.3 I */
        double z = o.u[2];
        double limx = 1.3 * (0.5 * c.w / c.fx), limy = 1.3 * (0.5 * c.h / c.fy);
        double rx = o.u[0] / z, ry = o.u[1] / z;
        double tx = fmin(limx, fmax(-limx, rx)), ty = fmin(limy, fmax(-limy, ry));
        double J[6] = {c.fx / z, 0.0, -c.fx * tx / z, 0.0, c.fy / z, -c.fy * ty / z};
        double Rq[9], q[4] = {quats[4 * i], quats[4 * i + 1], quats[4 * i + 2], quats[4 * i + 3]};
        quat_to_rot(q, Rq);
        double s[3], S[9] = {0};
        for (int k = 0; k < 3; k++) {
            s[k] = exp((double)log_scales[3 * i + k]);
            S[k * 4] = s[k];
        }
        double Mq[9], MqT[9], Sig[9];
        matmul(Rq, S, Mq, 3, 3, 3);
        transpose(Mq, MqT, 3, 3);
        matmul(Mq, MqT, Sig, 3, 3, 3);
        double T[6], Tt[6];
        matmul(J, c.R, T, 2, 3, 3);
        transpose(T, Tt, 2, 3);
        double tmp6[6], dSig[9], dT[6];
        matmul(Tt, dS, tmp6, 3, 2, 2);       /* 3x2 */
        matmul(tmp6, T, dSig, 3, 2, 3);      /* 3x3 */
        double dST[6];
        matmul(dS, T, dST, 2, 2, 3);         /* 2x3 */
        matmul(dST, Sig, dT, 2, 3, 3);
        for (int k = 0; k < 6; k++) dT[k] *= 2.0;
        double RcT[9], dJ[6];
        transpose(c.R, RcT, 3, 3);
        matmul(dT, RcT, dJ, 2, 3, 3);
        /* J entries depend on u: J00 = fx/z, J02 = -fx tx/z, J11 = fy/z, J12 = -fy ty/z */
        double du[3] = {0, 0, 0};
        du[2] += dJ[0] * (-c.fx / (z * z));
        du[2] += dJ[4] * (-c.fy / (z * z));
        double dtx_dx = (rx > -limx && rx < limx) ? 1.0 / z : 0.0;
        double dtx_dz = (rx > -limx && rx < limx) ? -o.u[0] / (z * z) : 0.0;
        double dty_dy = (ry > -limy && ry < limy) ? 1.0 / z : 0.0;
        double dty_dz = (ry > -limy && ry < limy) ? -o.u[1] / (z * z) : 0.0;
        /* J02 = -fx tx / z */
        du[0] += dJ[2] * (-c.fx / z) * dtx_dx;
        du[2] += dJ[2] * (-c.fx * (dtx_dz / z - tx / (z * z)));
        du[1] += dJ[5] * (-c.fy / z) * dty_dy;
        du[2] += dJ[5] * (-c.fy * (dty_dz / z - ty / (z * z)));
        /* mean2d = (fx x/z + cx, fy y/z + cy) */
        double gmx = d_mean2d[2 * i], gmy = d_mean2d[2 * i + 1];
        du[0] += gmx * c.fx / z;
        du[1] += gmy * c.fy / z;
        du[2] += -gmx * c.fx * o.u[0] / (z * z) - gmy * c.fy * o.u[1] / (z * z);
        for (int a = 0; a < 3; a++)
            g_means[3 * i + a] += c.R[0 * 3 + a] * du[0] + c.R[1 * 3 + a] * du[1] + c.R[2 * 3 + a] * du[2];
        /* Sig = Mq Mq^T with Mq = Rq S */
        double dMq[9];
        matmul(dSig, Mq, dMq, 3, 3, 3);
        /* dSig is symmetric and counts each entry once: dL/dMq = (dSig + dSig^T) Mq */
        for (int k = 0; k < 9; k++) dMq[k] *= 2.0;
        for (int k = 0; k < 3; k++) {
            double ds = 0.0;
            for (int r = 0; r < 3; r++) ds += dMq[r * 3 + k] * Rq[r * 3 + k];
            g_log_scales[3 * i + k] += ds * s[k];
        }
        double dR[9];
        for (int r = 0; r < 3; r++)
            for (int k = 0; k < 3; k++) dR[r * 3 + k] = dMq[r * 3 + k] * s[k];
        /* R(w,x,y,z) of the normalised quaternion */
        double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        double w = q[0] / nq, x = q[1] / nq, y = q[2] / nq, zz = q[3] / nq;
        double dw = 2 * (-zz * dR[1] + y * dR[2] + zz * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
        double dx = 2 * (y * dR[1] + zz * dR[2] + y * dR[3] - 2 * x * dR[4] - w * dR[5] + zz * dR[6] + w * dR[7] - 2 * x * dR[8]);
        double dy = 2 * (-2 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + zz * dR[5] - w * dR[6] + zz * dR[7] - 2 * y * dR[8]);
        double dz = 2 * (-2 * zz * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2 * zz * dR[4] + y * dR[5] + x * dR[6] + y * dR[7]);
        double dqn[4] = {dw, dx, dy, dz}, qn[4] = {w, x, y, zz};
        double proj = 0.0;
        for (int k = 0; k < 4; k++) proj += qn[k] * dqn[k];
        for (int k = 0; k < 4; k++) g_quats[4 * i + k] += (dqn[k] - qn[k] * proj) / nq;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* HVSQ (Section 2.2, Eq. 2): mean over the pixels of a region of
 * (M(I^a_i) - M(I^r_i))^2 + (sigma(I^a_i) - sigma(I^r_i))^2, the pooled
 * statistics of the altered and reference images around each pixel i.
 * The paper takes the features and the pooling shape from the cited HVSQ
 * work; the readings here: the features are the three colour channels (the
 * term is averaged over them); the pooling of pixel i is the square window
 * of half-width radius[i] centred on it, clipped to the image (its area
 * grows quadratically when the radius grows linearly with eccentricity);
 * M is the mean and sigma the population standard deviation over the
 * window.  Region restriction (Section 4.3): the mean runs over the pixels
 * of one quality region.  Every window is summed directly, two passes
 * (mean, then squared deviations).
 *
 * a, r: [3][H][W]; radius: [H*W] (>= 0); region (nullable): [H*W] in
 * 1..n_regions.  sums[t - 1], counts[t - 1]: the sum of the per-pixel terms
 * and the pixel count of region t; sums[n_regions], counts[n_regions]: the
 * whole image.  terms (nullable): [H*W] per-pixel term.  grad (nullable):
 * [3][H][W], d(mean over region grad_region, or the whole image when 0, of
 * the per-pixel terms) / d a; where sigma(I^a_i) = 0 its term contributes
 * only through the mean (the square root has no derivative there). */
static void window_stats(int W, int H, const double *img, int x, int y, int rad, double mu[3], double sd[3], int *n)
{
    int x0 = x - rad < 0 ? 0 : x - rad, x1 = x + rad > W - 1 ? W - 1 : x + rad;
    int y0 = y - rad < 0 ? 0 : y - rad, y1 = y + rad > H - 1 ? H - 1 : y + rad;
    int cnt = (x1 - x0 + 1) * (y1 - y0 + 1);
    for (int c = 0; c < 3; c++) {
        const double *pl = img + (size_t)c * W * H;
        double s = 0.0;
        for (int yy = y0; yy <= y1; yy++)
            for (int xx = x0; xx <= x1; xx++) s += pl[(size_t)yy * W + xx];
        double m = s / cnt, v = 0.0;
        for (int yy = y0; yy <= y1; yy++)
            for (int xx = x0; xx <= x1; xx++) {
                double d = pl[(size_t)yy * W + xx] - m;
                v += d * d;
            }
        mu[c] = m;
        sd[c] = sqrt(v / cnt);
    }
    *n = cnt;
}

int oc_hvsq(int W, int H, const double *a, const double *r, const int32_t *radius, const uint8_t *region,
            int n_regions, int grad_region, double *sums, double *counts, double *terms, double *grad)
{
    for (int t = 0; t <= n_regions; t++) sums[t] = counts[t] = 0.0;
    if (grad) memset(grad, 0, sizeof(double) * 3 * (size_t)W * H);
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            size_t i = (size_t)y * W + x;
            double ma[3], sa[3], mr[3], sr[3];
            int n;
            window_stats(W, H, a, x, y, radius[i], ma, sa, &n);
            window_stats(W, H, r, x, y, radius[i], mr, sr, &n);
            double term = 0.0;
            for (int c = 0; c < 3; c++) term += (ma[c] - mr[c]) * (ma[c] - mr[c]) + (sa[c] - sr[c]) * (sa[c] - sr[c]);
            term /= 3.0;
            int t = region ? region[i] : 0;
            if (t >= 1 && t <= n_regions) {
                sums[t - 1] += term;
                counts[t - 1] += 1.0;
            }
            sums[n_regions] += term;
            counts[n_regions] += 1.0;
            if (terms) terms[i] = term;
        }
    if (!grad) return 0;
    double N = grad_region == 0 ? counts[n_regions] : counts[grad_region - 1];
    if (N <= 0.0) return 0;
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            size_t i = (size_t)y * W + x;
            if (grad_region != 0 && (!region || region[i] != grad_region)) continue;
            double ma[3], sa[3], mr[3], sr[3];
            int n;
            window_stats(W, H, a, x, y, radius[i], ma, sa, &n);
            window_stats(W, H, r, x, y, radius[i], mr, sr, &n);
            int rad = radius[i];
            int x0 = x - rad < 0 ? 0 : x - rad, x1 = x + rad > W - 1 ? W - 1 : x + rad;
            int y0 = y - rad < 0 ? 0 : y - rad, y1 = y + rad > H - 1 ? H - 1 : y + rad;
            for (int c = 0; c < 3; c++) {
                /* d term / d a_j = (1/3) [2 (ma - mr) / n + 2 (sa - sr) (a_j - ma) / (n sa)] */
                double k = 1.0 / (3.0 * N);
                double gm = k * 2.0 * (ma[c] - mr[c]) / n;
                double gs = sa[c] > 0.0 ? k * 2.0 * (sa[c] - sr[c]) / (n * sa[c]) : 0.0;
                const double *pl = a + (size_t)c * W * H;
                double *gp = grad + (size_t)c * W * H;
                for (int yy = y0; yy <= y1; yy++)
                    for (int xx = x0; xx <= x1; xx++) {
                        size_t j = (size_t)yy * W + xx;
                        gp[j] += gm + gs * (pl[j] - ma[c]);
                    }
            }
        }
    return 0;
}

/* Per-pixel HVSQ terms at listed pixels px [npx][2] = (x, y) only (for
 * sampled checks of large images). */
int oc_hvsq_at(int W, int H, const double *a, const double *r, const int32_t *radius, int npx, const int32_t *px,
               double *terms)
{
    for (int k = 0; k < npx; k++) {
        int x = px[2 * k], y = px[2 * k + 1];
        double ma[3], sa[3], mr[3], sr[3];
        int n;
        int rad = radius[(size_t)y * W + x];
        window_stats(W, H, a, x, y, rad, ma, sa, &n);
        window_stats(W, H, r, x, y, rad, mr, sr, &n);
        double term = 0.0;
        for (int c = 0; c < 3; c++) term += (ma[c] - mr[c]) * (ma[c] - mr[c]) + (sa[c] - sr[c]) * (sa[c] - sr[c]);
        terms[k] = term / 3.0;
    }
    return 0;
}

int oc_version(void) { return 1; }
