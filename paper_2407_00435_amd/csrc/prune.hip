// Efficiency-aware pruning metrics (Section 3): computational efficiency per
// point (Section 3.2), selection of the lowest-CE points for removal (Section
// 3.4), and the weighted-scale penalty with its gradient (Section 3.3).
#include "common.hpp"
#include "kernels.hpp"

namespace {

// CE_i = max over views of dominated_i,v / tiles_i,v (views where the point
// uses no tile give 0).  The ratio is a correctly rounded float32 division
// of two exactly representable counts.
__global__ void __launch_bounds__(256)
k_ce_score(const uint32_t *__restrict__ dominated, const uint32_t *__restrict__ hits, int n, int V,
           float *__restrict__ ce)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float best = 0.0f;
    for (int v = 0; v < V; ++v) {
        const int64_t e = (int64_t)v * n + i;
        const uint32_t h = hits[e];
        if (h) best = fmaxf(best, __fdiv_rn((float)dominated[e], (float)h));
    }
    ce[i] = best;
}

// --- radix select of the k smallest keys (float bits of CE >= 0 order like
// the values), most significant digit first, then a stable compaction in
// index order: keys below the threshold, and the first (k - below) keys
// equal to it.
constexpr int SEL_THREADS = 256;
constexpr int SEL_ITEMS = 16;
constexpr int SEL_CHUNK = SEL_THREADS * SEL_ITEMS;

// state: [0] threshold prefix, [1] keys still to take at the threshold
__global__ void k_sel_init(uint32_t *__restrict__ state, uint32_t k)
{
    state[0] = 0u;
    state[1] = k;
}

__global__ void __launch_bounds__(SEL_THREADS)
k_sel_hist(const uint32_t *__restrict__ keys, int n, const uint32_t *__restrict__ state, int shift,
           uint32_t *__restrict__ hist)
{
    __shared__ uint32_t sh[256];
    sh[threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t prefix = state[0];
    const uint32_t hi_mask = shift >= 24 ? 0u : (0xFFFFFFFFu << (shift + 8));
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t key = keys[i];
        if ((key & hi_mask) == (prefix & hi_mask)) atomicAdd(&sh[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    const uint32_t c = sh[threadIdx.x];
    if (c) atomicAdd(&hist[threadIdx.x], c);
}

// one workgroup of 256: picks the digit at which the count of smaller keys
// reaches the number still to take
__global__ void __launch_bounds__(256) k_sel_pick(uint32_t *__restrict__ hist, uint32_t *__restrict__ state, int shift)
{
    __shared__ uint32_t s[256];
    const int t = threadIdx.x;
    const uint32_t h = hist[t];
    s[t] = h;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t a = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += a;
        __syncthreads();
    }
    const uint32_t incl = s[t], excl = incl - h;
    const uint32_t rem = state[1];
    __syncthreads();
    if (excl < rem && rem <= incl) {
        state[0] |= (uint32_t)t << shift;
        state[1] = rem - excl;
    }
    hist[t] = 0u;  // ready for the next digit
}

// per chunk: keys below the threshold and keys equal to it
__global__ void __launch_bounds__(SEL_THREADS)
k_sel_count(const uint32_t *__restrict__ keys, int n, const uint32_t *__restrict__ state,
            uint32_t *__restrict__ below, uint32_t *__restrict__ equal)
{
    __shared__ uint32_t s_b, s_e;
    if (threadIdx.x == 0) s_b = s_e = 0u;
    __syncthreads();
    const uint32_t t = state[0];
    uint32_t cb = 0, ce = 0;
    const int64_t base = (int64_t)blockIdx.x * SEL_CHUNK;
    for (int j = 0; j < SEL_ITEMS; ++j) {
        const int64_t i = base + (int64_t)j * SEL_THREADS + threadIdx.x;
        if (i < n) {
            const uint32_t key = keys[i];
            cb += key < t;
            ce += key == t;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        cb += __shfl_xor(cb, off);
        ce += __shfl_xor(ce, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&s_b, cb);
        atomicAdd(&s_e, ce);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        below[blockIdx.x] = s_b;
        equal[blockIdx.x] = s_e;
    }
}

// one workgroup: exclusive offsets of equal keys, then of selected keys
__global__ void __launch_bounds__(1024)
k_sel_scan(uint32_t *__restrict__ below, uint32_t *__restrict__ equal, int nb, const uint32_t *__restrict__ state)
{
    __shared__ uint32_t s[1024];
    const int t = threadIdx.x;
    const int per = (nb + 1023) / 1024;
    const int b0 = t * per, b1 = min(b0 + per, nb);
    const uint32_t take = state[1];
    // pass 1: equal keys before each chunk
    uint32_t loc = 0;
    for (int b = b0; b < b1; ++b) loc += equal[b];
    s[t] = loc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t a = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += a;
        __syncthreads();
    }
    uint32_t run = s[t] - loc;
    __syncthreads();
    // selected per chunk: all below plus the equal ones still within `take`
    uint32_t sel_loc = 0;
    for (int b = b0; b < b1; ++b) {
        const uint32_t e = equal[b];
        const uint32_t eq_take = run >= take ? 0u : min(e, take - run);
        equal[b] = run;  // exclusive offset of equal keys
        run += e;
        below[b] += eq_take;  // now: selected keys in the chunk
        sel_loc += below[b];
    }
    s[t] = sel_loc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t a = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += a;
        __syncthreads();
    }
    uint32_t srun = s[t] - sel_loc;
    for (int b = b0; b < b1; ++b) {
        const uint32_t c = below[b];
        below[b] = srun;  // exclusive offset of selected keys
        srun += c;
    }
}

__global__ void __launch_bounds__(SEL_THREADS)
k_sel_write(const uint32_t *__restrict__ keys, int n, const uint32_t *__restrict__ state,
            const uint32_t *__restrict__ sel_off, const uint32_t *__restrict__ eq_off, uint8_t *__restrict__ mask,
            uint32_t *__restrict__ idx)
{
    __shared__ uint32_t s_we[SEL_THREADS / 64], s_ws[SEL_THREADS / 64];
    const uint32_t t = state[0], take = state[1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lt = lanemask_lt();
    const int64_t base = (int64_t)blockIdx.x * SEL_CHUNK;
    uint32_t erun = eq_off[blockIdx.x], srun = sel_off[blockIdx.x];
    for (int j = 0; j < SEL_ITEMS; ++j) {
        const int64_t i = base + (int64_t)j * SEL_THREADS + threadIdx.x;
        const bool ok = i < n;
        const uint32_t key = ok ? keys[i] : 0xFFFFFFFFu;
        const bool eq = ok && key == t;
        const uint64_t beq = ballot64(eq);
        if (lane == 0) s_we[wave] = (uint32_t)__popcll(beq);
        __syncthreads();
        uint32_t epre = 0, etot = 0;
        for (int w = 0; w < SEL_THREADS / 64; ++w) {
            if (w < wave) epre += s_we[w];
            etot += s_we[w];
        }
        const uint32_t erank = erun + epre + (uint32_t)__popcll(beq & lt);
        const bool sel = ok && (key < t || (eq && erank < take));
        const uint64_t bsel = ballot64(sel);
        if (lane == 0) s_ws[wave] = (uint32_t)__popcll(bsel);
        __syncthreads();
        uint32_t spre = 0, stot = 0;
        for (int w = 0; w < SEL_THREADS / 64; ++w) {
            if (w < wave) spre += s_ws[w];
            stot += s_ws[w];
        }
        if (ok) mask[i] = sel ? 1 : 0;
        if (sel && idx) idx[srun + spre + (uint32_t)__popcll(bsel & lt)] = (uint32_t)i;
        erun += etot;
        srun += stot;
        __syncthreads();
    }
}

// Weighted scale: per point S = 3 max_k exp(ls_k) (first maximum), summed
// G over the views, contribution S G; gradient coef G S to the longest axis.
__global__ void __launch_bounds__(256)
k_weighted_scale(const float *__restrict__ log_scales, const uint32_t *__restrict__ hits, int n, int V,
                 float thr, float coef, float *__restrict__ ws, float *__restrict__ d_ls, int accumulate)
{
    __shared__ float s_part[4];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float contrib = 0.0f;
    if (i < n) {
        const float l0 = log_scales[3 * (int64_t)i], l1 = log_scales[3 * (int64_t)i + 1],
                    l2 = log_scales[3 * (int64_t)i + 2];
        int ax = 0;
        float lm = l0;
        if (l1 > lm) {
            lm = l1;
            ax = 1;
        }
        if (l2 > lm) {
            lm = l2;
            ax = 2;
        }
        const float S = 3.0f * __expf(lm);
        float G = 0.0f;
        for (int v = 0; v < V; ++v) {
            const float U = (float)hits[(int64_t)v * n + i];
            if (U > thr) G += U - thr;
        }
        contrib = S * G;
        if (d_ls) {
            float *g = d_ls + 3 * (int64_t)i;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float add = k == ax ? coef * G * S : 0.0f;
                g[k] = accumulate ? g[k] + add : add;
            }
        }
    }
    contrib = wave_sum(contrib);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = contrib;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float b = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
        if (b != 0.0f) atomicAdd(ws, b * coef);
    }
}

__global__ void __launch_bounds__(256) k_fill_u8(uint8_t *__restrict__ p, uint8_t v, int n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

}  // namespace

hipError_t launch_fill_u8(uint8_t *p, uint8_t v, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    int b = (n + 1023) / 1024;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_fill_u8, dim3(b), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t launch_ce_score(const uint32_t *dominated, const uint32_t *hits, int n, int V, float *ce,
                           hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ce_score, dim3((n + 255) / 256), dim3(256), 0, st, dominated, hits, n, V, ce);
    return hipGetLastError();
}

size_t select_scratch_bytes(int n)
{
    const size_t nb = ((size_t)n + SEL_CHUNK - 1) / SEL_CHUNK + 1;
    return 256 * 4 + 4 * 4 + 2 * 4 * nb + 4 * 256;
}

hipError_t launch_select_lowest(const float *ce, int n, int k, uint8_t *mask, uint32_t *idx, void *scratch,
                                hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const int nb = (n + SEL_CHUNK - 1) / SEL_CHUNK;
    char *p = (char *)scratch;
    uint32_t *hist = (uint32_t *)p;
    uint32_t *state = (uint32_t *)(p + 256 * 4);
    uint32_t *below = (uint32_t *)(p + 256 * 4 + 4 * 4);
    uint32_t *equal = below + nb + 1;
    const uint32_t *keys = reinterpret_cast<const uint32_t *>(ce);
    hipError_t e = launch_fill_u32(hist, 0u, 256, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(1), 0, st, state, (uint32_t)k);
    int hb = (n + SEL_CHUNK - 1) / SEL_CHUNK;
    if (hb > 1024) hb = 1024;
    for (int shift = 24; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_sel_hist, dim3(hb), dim3(SEL_THREADS), 0, st, keys, n, state, shift, hist);
        hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(256), 0, st, hist, state, shift);
    }
    hipLaunchKernelGGL(k_sel_count, dim3(nb), dim3(SEL_THREADS), 0, st, keys, n, state, below, equal);
    hipLaunchKernelGGL(k_sel_scan, dim3(1), dim3(1024), 0, st, below, equal, nb, state);
    hipLaunchKernelGGL(k_sel_write, dim3(nb), dim3(SEL_THREADS), 0, st, keys, n, state, below, equal, mask, idx);
    return hipGetLastError();
}

hipError_t launch_weighted_scale(const float *log_scales, const uint32_t *hits, int n, int V, float thr,
                                 float gamma, float *ws, float *d_log_scales, int accumulate, hipStream_t st)
{
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(ws), 0u, 1, st);
    if (e != hipSuccess || n == 0) return e;
    const float coef = gamma / ((float)n * (float)V);
    hipLaunchKernelGGL(k_weighted_scale, dim3((n + 255) / 256), dim3(256), 0, st, log_scales, hits, n, V, thr, coef,
                       ws, d_log_scales, accumulate);
    return hipGetLastError();
}
