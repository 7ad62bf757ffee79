// Stable LSD radix sort of (u32 key, u32 value) pairs for gfx950.
//
// One histogram pass over the keys computes the digit counts of every pass;
// then each pass is a single "onesweep" kernel: a workgroup takes the next
// partition ticket from an atomic counter (so partitions are processed in
// ticket order and every predecessor is already resident), ranks its 4096
// keys stably with wave64 ballot matching, publishes its per-digit counts,
// and resolves its global offsets by decoupled lookback over predecessor
// partitions before scattering through LDS in coalesced runs.
#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr int RS_WAVES = RS_THREADS / 64;
constexpr uint64_t FLAG_AGG = 1ull << 62;
constexpr uint64_t FLAG_INC = 2ull << 62;
constexpr uint64_t VAL_MASK = (1ull << 62) - 1;

__global__ void __launch_bounds__(256)
k_radix_hist(const uint32_t *__restrict__ keys, const uint64_t *__restrict__ d_count, uint64_t cap,
             int passes, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t sh[4][256];
    for (int j = threadIdx.x; j < 4 * 256; j += blockDim.x) (&sh[0][0])[j] = 0;
    __syncthreads();
    uint64_t count = *d_count;
    count = count < cap ? count : cap;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        uint32_t k = keys[i];
        for (int p = 0; p < passes; ++p) atomicAdd(&sh[p][(k >> (8 * p)) & 255u], 1u);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < passes * 256; j += blockDim.x) {
        uint32_t c = (&sh[0][0])[j];
        if (c) atomicAdd(&hist[j], c);
    }
}

// exclusive prefix over the 256 digits of each pass (one block per pass)
__global__ void __launch_bounds__(256) k_radix_prefix(uint32_t *__restrict__ hist)
{
    __shared__ uint32_t s[256];
    uint32_t *h = hist + blockIdx.x * 256;
    int t = threadIdx.x;
    uint32_t v = h[t];
    s[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t add = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    h[t] = s[t] - v;
}

__global__ void __launch_bounds__(256)
k_radix_clear(uint64_t *__restrict__ status, uint32_t *__restrict__ ticket,
              const uint64_t *__restrict__ d_count, uint64_t cap)
{
    uint64_t count = *d_count;
    count = count < cap ? count : cap;
    uint64_t words = ((count + RS_PART - 1) / RS_PART) * 256;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
        status[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *ticket = 0;
}

__global__ void __launch_bounds__(RS_THREADS)
k_radix_onesweep(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                 uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                 const uint64_t *__restrict__ d_count, uint64_t cap, int shift,
                 const uint32_t *__restrict__ gbase, uint64_t *__restrict__ status,
                 uint32_t *__restrict__ ticket)
{
    __shared__ uint32_t s_keys[RS_PART];
    __shared__ uint32_t s_vals[RS_PART];
    __shared__ uint32_t s_whist[RS_WAVES][256];
    __shared__ uint32_t s_bexcl[256];  // exclusive prefix over digits of the block counts
    __shared__ uint64_t s_dbase[256];  // global position of the digit's first key of this block
    __shared__ uint32_t s_part;

    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    if (t == 0) s_part = atomicAdd(ticket, 1u);
    for (int j = t; j < RS_WAVES * 256; j += RS_THREADS) (&s_whist[0][0])[j] = 0;
    __syncthreads();
    const uint64_t part = s_part;
    uint64_t count = *d_count;
    count = count < cap ? count : cap;
    const uint64_t nparts = (count + RS_PART - 1) / RS_PART;
    if (part >= nparts) return;

    const uint64_t pbase = part * RS_PART;
    const uint64_t wbase = pbase + (uint64_t)wave * (RS_ITEMS * 64);
    uint32_t k[RS_ITEMS], v[RS_ITEMS], rk[RS_ITEMS];
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        uint64_t idx = wbase + (uint64_t)r * 64 + lane;
        bool ok = idx < count;
        k[r] = ok ? kin[idx] : 0xFFFFFFFFu;
        v[r] = ok ? vin[idx] : 0u;
    }
    const uint64_t lt = lanemask_lt();
    // stable rank within the wave: items in (round, lane) order
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        uint64_t idx = wbase + (uint64_t)r * 64 + lane;
        bool ok = idx < count;
        uint32_t d = (k[r] >> shift) & 255u;
        uint64_t peers = ballot64(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t bb = ballot64(bit);
            peers &= bit ? bb : ~bb;
        }
        uint32_t before = (uint32_t)__popcll(peers & lt);
        uint32_t prev = s_whist[wave][d];
        rk[r] = prev + before;
        wave_lds_sync();
        if (ok && before == 0) s_whist[wave][d] = prev + (uint32_t)__popcll(peers);
        wave_lds_sync();
    }
    __syncthreads();
    // per digit: exclusive over waves, block total
    uint32_t total = 0;
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) {
        uint32_t c = s_whist[w][t];
        s_whist[w][t] = total;
        total += c;
    }
    // publish this partition's counts, then look back for the prefix
    uint64_t *my = status + part * 256 + t;
    if (part == 0) {
        __hip_atomic_store(my, FLAG_INC | (uint64_t)total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        __hip_atomic_store(my, FLAG_AGG | (uint64_t)total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    uint64_t prefix = 0;
    if (part > 0) {
        int64_t q = (int64_t)part - 1;
        for (;;) {
            uint64_t st = __hip_atomic_load(status + q * 256 + t, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
            uint64_t flag = st & ~VAL_MASK;
            if (flag == 0) {
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            prefix += st & VAL_MASK;
            if (flag == FLAG_INC) break;
            --q;
        }
        __hip_atomic_store(my, FLAG_INC | (prefix + total), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    // block-local exclusive prefix over digits (Hillis-Steele in LDS)
    s_bexcl[t] = total;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        uint32_t add = t >= off ? s_bexcl[t - off] : 0u;
        __syncthreads();
        s_bexcl[t] += add;
        __syncthreads();
    }
    uint32_t bexcl = s_bexcl[t] - total;
    __syncthreads();
    s_bexcl[t] = bexcl;
    s_dbase[t] = (uint64_t)gbase[t] + prefix;
    __syncthreads();
    // scatter into LDS in digit order
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        uint64_t idx = wbase + (uint64_t)r * 64 + lane;
        if (idx < count) {
            uint32_t d = (k[r] >> shift) & 255u;
            uint32_t pos = s_bexcl[d] + s_whist[wave][d] + rk[r];
            s_keys[pos] = k[r];
            s_vals[pos] = v[r];
        }
    }
    __syncthreads();
    uint32_t pcount = (uint32_t)((count - pbase) < (uint64_t)RS_PART ? (count - pbase) : RS_PART);
    for (uint32_t j = t; j < pcount; j += RS_THREADS) {
        uint32_t key = s_keys[j];
        uint32_t d = (key >> shift) & 255u;
        uint64_t dst = s_dbase[d] + (j - s_bexcl[d]);
        kout[dst] = key;
        vout[dst] = s_vals[j];
    }
}

}  // namespace

hipError_t radix_sort_pairs(uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb,
                            const uint64_t *d_count, uint64_t cap, int bits,
                            const RadixScratch &rs, hipStream_t st)
{
    int passes = radix_passes(bits);
    if (passes == 0 || cap == 0) return hipSuccess;
    hipError_t e = launch_fill_u32(rs.hist, 0u, 4 * 256, st);
    if (e != hipSuccess) return e;
    uint64_t max_parts = radix_max_parts(cap);
    int hist_blocks = (int)((cap + 256 * 32 - 1) / (256 * 32));
    if (hist_blocks > 2048) hist_blocks = 2048;
    if (hist_blocks < 1) hist_blocks = 1;
    hipLaunchKernelGGL(k_radix_hist, dim3(hist_blocks), dim3(256), 0, st, ka, d_count, cap, passes,
                       rs.hist);
    hipLaunchKernelGGL(k_radix_prefix, dim3(passes), dim3(256), 0, st, rs.hist);
    uint32_t *src_k = ka, *src_v = va, *dst_k = kb, *dst_v = vb;
    int clear_blocks = (int)((max_parts * 256 + 255) / 256);
    if (clear_blocks > 4096) clear_blocks = 4096;
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(k_radix_clear, dim3(clear_blocks), dim3(256), 0, st, rs.status,
                           rs.tickets + p, d_count, cap);
        hipLaunchKernelGGL(k_radix_onesweep, dim3((unsigned)max_parts), dim3(RS_THREADS), 0, st,
                           src_k, src_v, dst_k, dst_v, d_count, cap, 8 * p, rs.hist + 256 * p,
                           rs.status, rs.tickets + p);
        uint32_t *tk = src_k, *tv = src_v;
        src_k = dst_k; src_v = dst_v;
        dst_k = tk; dst_v = tv;
    }
    return hipGetLastError();
}
