// Stable LSD radix sort of (u32 key, u32 value) pairs for gfx950.
//
// One histogram pass over the keys computes the digit counts of every pass;
// then each pass is a single "onesweep" kernel: a workgroup takes the next
// partition ticket from an atomic counter (so partitions are processed in
// ticket order and every predecessor is already resident), ranks its keys
// stably with wave64 ballot matching, publishes its per-digit counts, and
// resolves its global offsets by decoupled lookback over predecessor
// partitions before scattering through LDS in coalesced runs.  The grid is
// persistent: a workgroup takes tickets until the partitions run out, so
// every partition it waits on belongs to a workgroup that is already running.
//
// Digits are at most 8 bits wide and equal across passes (a 14-bit key sorts
// in two 7-bit passes).  The partition size (keys per workgroup) trades the
// length of the lookback chain against occupancy; it is 8192 by default and
// can be set to 4096, 8192 or 16384 with the GS_RADIX_PART environment
// variable or gs_set_tuning("radix_part", ...).
#include <cstdlib>

#include "common.hpp"
#include "kernels.hpp"

namespace {

constexpr uint64_t FLAG_AGG = 1ull << 62;
constexpr uint64_t FLAG_INC = 2ull << 62;
constexpr uint64_t VAL_MASK = (1ull << 62) - 1;
constexpr int MIN_PART = 4096;
constexpr uint64_t SWEEP_BLOCKS = 1024;  // persistent onesweep workgroups (at most)
// lookback words read per round (1024-thread workgroups holding 16 keys a
// thread have no registers to spare for more than one)
template <int THREADS, int ITEMS>
constexpr int lookback_batch() { return THREADS >= 1024 && ITEMS >= 16 ? 1 : 8; }

// Digit counts of every pass.  Each thread takes HIST_RUN consecutive keys
// and adds one per key and digit into its wave's own LDS counters (the
// waves' counters are summed once at the end); a plain increment is a few
// instructions, where detecting runs of equal digits cost about 24 per key
// and digit and the keys sorted here rarely repeat.
constexpr int HIST_RUN = 16;
constexpr int HIST_THREADS = 1024;

__global__ void __launch_bounds__(HIST_THREADS)
k_radix_hist(const uint32_t *__restrict__ keys, const uint64_t *__restrict__ d_count, uint64_t cap,
             int passes, int dbits, int radix, uint32_t *__restrict__ hist)
{
    // counts of pass p at shw[wave][p * radix + digit] (radix 256, or 512 for one 9-bit pass)
    constexpr int WAVES = HIST_THREADS / 64;
    __shared__ uint32_t shw[WAVES][4 * 256];
    for (int j = threadIdx.x; j < WAVES * 4 * 256; j += blockDim.x) (&shw[0][0])[j] = 0;
    __syncthreads();
    uint32_t *sh = shw[threadIdx.x >> 6];
    uint64_t count = *d_count;
    count = count < cap ? count : cap;
    const uint32_t mask = (1u << dbits) - 1u;
    const bool vec_ok = (reinterpret_cast<uintptr_t>(keys) & 15) == 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * HIST_RUN;
    for (uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * HIST_RUN; i < count; i += stride) {
        uint32_t k[HIST_RUN];
        const uint32_t nk = count - i < (uint64_t)HIST_RUN ? (uint32_t)(count - i) : (uint32_t)HIST_RUN;
        if (vec_ok && nk == HIST_RUN) {
#pragma unroll
            for (int q = 0; q < HIST_RUN / 4; ++q) {
                const uint4 v = reinterpret_cast<const uint4 *>(keys + i)[q];
                k[4 * q] = v.x;
                k[4 * q + 1] = v.y;
                k[4 * q + 2] = v.z;
                k[4 * q + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < HIST_RUN; ++j) k[j] = j < (int)nk ? keys[i + j] : 0u;
        }
        for (int p = 0; p < passes; ++p) {
            const int sh_p = dbits * p;
#pragma unroll
            for (int j = 0; j < HIST_RUN; ++j)
                if (j < (int)nk) atomicAdd(&sh[p * radix + ((k[j] >> sh_p) & mask)], 1u);
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < passes * radix; j += blockDim.x) {
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) c += shw[w][j];
        if (c) atomicAdd(&hist[j], c);
    }
}

// Prepares one sort: zeroes the digit counts and the partition tickets of
// every pass, and the lookback words of the first pass's partitions (the
// key count read on the device).  Each pass clears the words of the next.
__global__ void __launch_bounds__(256)
k_radix_init(uint32_t *__restrict__ hist, uint32_t *__restrict__ tickets, uint64_t *__restrict__ status,
             const uint64_t *__restrict__ d_count, uint64_t cap, int part, int radix)
{
    uint64_t count = *d_count;
    count = count < cap ? count : cap;
    const uint64_t words = ((count + part - 1) / part) * radix;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = i0; i < words; i += stride) status[i] = 0;
    for (uint64_t i = i0; i < 4 * 256; i += stride) hist[i] = 0;
    if (i0 < 4) tickets[i0] = 0;
}

template <int THREADS, int ITEMS, typename VT, int RB>
__global__ void __launch_bounds__(THREADS)
k_radix_onesweep(const uint32_t *__restrict__ kin, const VT *__restrict__ vin,
                 uint32_t *__restrict__ kout, VT *__restrict__ vout,
                 const uint64_t *__restrict__ d_count, uint64_t cap, int shift, uint32_t mask,
                 int dbits, const uint32_t *__restrict__ dcount, uint64_t *__restrict__ status,
                 uint64_t *__restrict__ status_next, uint32_t *__restrict__ ticket)
{
    constexpr int WAVES = THREADS / 64;
    constexpr int PART = THREADS * ITEMS;
    constexpr int R = 1 << RB;  // digits of the pass, one thread each
    static_assert(R <= THREADS, "a thread per digit");
    __shared__ uint32_t s_keys[PART];
    __shared__ VT s_vals[PART];
    __shared__ uint32_t s_whist[WAVES][R];
    __shared__ uint32_t s_bexcl[R];  // exclusive prefix over digits of the block counts
    __shared__ uint64_t s_dbase[R];  // global position of the digit's first key of this block
    __shared__ uint32_t s_gbase[R];  // exclusive prefix of this pass's digit counts
    __shared__ uint32_t s_wsum[R / 64];
    __shared__ uint32_t s_part;

    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    // digit bases of the pass, once per workgroup (the first R / 64 waves
    // take 64 digits each)
    uint32_t dc = 0, dx = 0;
    if (t < R) {
        dc = dcount[t];
        dx = wave_incl_scan(dc);
        if (lane == 63) s_wsum[wave] = dx;
    }
    __syncthreads();
    if (t < R) {
        uint32_t add = 0;
        for (int w = 0; w < wave; ++w) add += s_wsum[w];
        s_gbase[t] = add + dx - dc;
    }
    uint64_t count = *d_count;
    count = count < cap ? count : cap;
    const uint64_t nparts = (count + PART - 1) / PART;
    // persistent: partitions are taken in ticket order until none is left
    for (;;) {
        if (t == 0) s_part = atomicAdd(ticket, 1u);
        for (int j = t; j < WAVES * R; j += THREADS) (&s_whist[0][0])[j] = 0;
        __syncthreads();
        const uint64_t part = s_part;
        if (part >= nparts) return;
        // the next pass finds its partition's lookback words cleared
        if (status_next && t < R) status_next[part * R + t] = 0;

        const uint64_t pbase = part * PART;
        const uint64_t wbase = pbase + (uint64_t)wave * (ITEMS * 64);
        uint32_t k[ITEMS], rk[ITEMS];
        VT v[ITEMS];
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            uint64_t idx = wbase + (uint64_t)r * 64 + lane;
            bool ok = idx < count;
            k[r] = ok ? kin[idx] : 0xFFFFFFFFu;
            v[r] = ok ? vin[idx] : VT{};
        }
        const uint64_t lt = lanemask_lt();
        // stable rank within the wave: items in (round, lane) order
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            uint64_t idx = wbase + (uint64_t)r * 64 + lane;
            bool ok = idx < count;
            uint32_t d = (k[r] >> shift) & mask;
            uint64_t peers = ballot64(ok);
            for (int b = 0; b < dbits; ++b) {
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
        // per digit (threads < R): exclusive over waves, block total, lookback
        const bool dig = t < R;
        uint32_t total = 0, inc = 0;
        uint64_t prefix = 0;
        if (dig) {
#pragma unroll
            for (int w = 0; w < WAVES; ++w) {
                uint32_t c = s_whist[w][t];
                s_whist[w][t] = total;
                total += c;
            }
            uint64_t *my = status + part * R + t;
            if (part == 0) {
                __hip_atomic_store(my, FLAG_INC | (uint64_t)total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                __hip_atomic_store(my, FLAG_AGG | (uint64_t)total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (part > 0 && (uint32_t)t <= mask) {
                // a batch of predecessors' words is read at once and taken in
                // order (aggregates added until an inclusive prefix); an
                // unpublished word ends the batch and is read again next
                // round.  Partition 0 always ends the walk, so words before
                // it are never taken.
                constexpr int LOOKBACK = lookback_batch<THREADS, ITEMS>();
                int64_t q = (int64_t)part - 1;
                for (;;) {
                    uint64_t w[LOOKBACK];
#pragma unroll
                    for (int j = 0; j < LOOKBACK; ++j)
                        w[j] = q - j >= 0 ? __hip_atomic_load(status + (q - j) * R + t, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT)
                                          : FLAG_INC;
                    int used = LOOKBACK;
                    bool done = false;
#pragma unroll
                    for (int j = 0; j < LOOKBACK; ++j) {
                        if (used < LOOKBACK || done) continue;
                        const uint64_t flag = w[j] & ~VAL_MASK;
                        if (flag == 0) {
                            used = j;
                            continue;
                        }
                        prefix += w[j] & VAL_MASK;
                        if (flag == FLAG_INC) done = true;
                    }
                    if (done) break;
                    if (used == 0) __builtin_amdgcn_s_sleep(1);
                    q -= used;
                }
                __hip_atomic_store(my, FLAG_INC | (prefix + total), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            // block-local prefix over the digits: a wave scan in each of
            // the first R / 64 waves, then the totals of the waves before
            inc = wave_incl_scan(total);
            if (lane == 63) s_wsum[wave] = inc;
        }
        __syncthreads();
        if (dig) {
            uint32_t add = 0;
            for (int w = 0; w < wave; ++w) add += s_wsum[w];
            s_bexcl[t] = add + inc - total;
            s_dbase[t] = (uint64_t)s_gbase[t] + prefix;
        }
        __syncthreads();
        // scatter into LDS in digit order
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            uint64_t idx = wbase + (uint64_t)r * 64 + lane;
            if (idx < count) {
                uint32_t d = (k[r] >> shift) & mask;
                uint32_t pos = s_bexcl[d] + s_whist[wave][d] + rk[r];
                s_keys[pos] = k[r];
                s_vals[pos] = v[r];
            }
        }
        __syncthreads();
        uint32_t pcount = (uint32_t)((count - pbase) < (uint64_t)PART ? (count - pbase) : PART);
        for (uint32_t j = t; j < pcount; j += THREADS) {
            uint32_t key = s_keys[j];
            uint32_t d = (key >> shift) & mask;
            uint64_t dst = s_dbase[d] + (j - s_bexcl[d]);
            kout[dst] = key;
            vout[dst] = s_vals[j];
        }
        // the next partition reuses every LDS array
        __syncthreads();
    }
}

__global__ void k_set_count(uint64_t *__restrict__ p, uint64_t value) { *p = value; }

}  // namespace

uint64_t radix_max_parts(uint64_t cap) { return (cap + MIN_PART - 1) / MIN_PART; }

// 256 words per partition of 4096 keys also hold 512 per partition of 8192
uint64_t radix_status_words(uint64_t cap) { return 256 * (radix_max_parts(cap ? cap : 1) + 1); }

int radix_digit_bits(int bits)
{
    const int passes = radix_passes(bits);
    return passes ? (bits + passes - 1) / passes : 0;
}

// partition size of a sort with values of vbytes bytes given the context's
// choice (the LDS holds keys and values: 8-byte values take partitions of at
// most 8192 keys)
static int part_for(int vbytes, int part) { return vbytes > 4 && part > 8192 ? 8192 : part; }

// A 9-bit key sorts in one pass of 512 digits where the workgroup has a
// thread per digit (512 threads: partitions of 8192 keys).
static bool one_wide_pass(int bits, int P) { return bits == 9 && P == 8192; }

int radix_pass_count(int bits, int vbytes, int part)
{
    return one_wide_pass(bits, part_for(vbytes, part)) ? 1 : radix_passes(bits);
}

RadixShape radix_shape(const RadixScratch &rs, int vbytes, int bits)
{
    const int P = part_for(vbytes, rs.part);
    const bool wide = one_wide_pass(bits, P);
    // equal digit widths <= 8 bits (fewer buckets give longer runs per
    // digit), or one 9-bit digit
    return RadixShape{P, wide ? 512 : 256, wide ? 1 : radix_passes(bits), wide ? 9 : radix_digit_bits(bits)};
}

uint64_t radix_prepare_words(const RadixScratch &rs, uint64_t count, int vbytes, int bits)
{
    const RadixShape sh = radix_shape(rs, vbytes, bits);
    return ((count + sh.part - 1) / sh.part) * sh.radix;
}

hipError_t radix_sort_prepare(const RadixScratch &rs, const uint64_t *d_count, uint64_t cap, int vbytes, int bits,
                              hipStream_t st)
{
    const int P = part_for(vbytes, rs.part);
    const int R = one_wide_pass(bits, P) ? 512 : 256;
    const uint64_t words = ((cap + P - 1) / P) * R;
    if (words > rs.status_words) return hipErrorInvalidValue;
    uint64_t blocks = (words + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
    hipLaunchKernelGGL(k_radix_init, dim3((unsigned)blocks), dim3(256), 0, st, rs.hist, rs.tickets, rs.status,
                       d_count, cap, P, R);
    return hipGetLastError();
}

template <typename VT>
static hipError_t sort_pairs_impl(uint32_t *ka, VT *va, uint32_t *kb, VT *vb,
                            const uint64_t *d_count, uint64_t cap, int bits,
                            const RadixScratch &rs, hipStream_t st, bool hist_ready, bool cleared)
{
    if (radix_passes(bits) == 0 || cap == 0) return hipSuccess;
    const RadixShape shape = radix_shape(rs, (int)sizeof(VT), bits);
    const int P = shape.part;
    const bool wide = shape.radix == 512;
    const int passes = shape.passes;
    const int dbits = shape.dbits;
    const int R = shape.radix;
    const uint32_t mask = (1u << dbits) - 1u;
    hipError_t e;
    const uint64_t parts = (cap + P - 1) / P;
    if (!hist_ready) {
        if (!cleared && (e = radix_sort_prepare(rs, d_count, cap, (int)sizeof(VT), bits, st)) != hipSuccess)
            return e;
        // few large blocks: each adds its counts to the global histogram
        // with one atomic per digit, and same-address atomics from
        // thousands of blocks would serialise in L2
        int hist_blocks = (int)((cap + 1024 * HIST_RUN * 4 - 1) / (1024 * HIST_RUN * 4));
        if (hist_blocks > 256) hist_blocks = 256;
        if (hist_blocks < 1) hist_blocks = 1;
        hipLaunchKernelGGL(k_radix_hist, dim3(hist_blocks), dim3(HIST_THREADS), 0, st, ka, d_count, cap, passes,
                           dbits, R, rs.hist);
    }
    uint32_t *src_k = ka, *dst_k = kb;
    VT *src_v = va, *dst_v = vb;
    // a persistent grid of at most SWEEP_BLOCKS workgroups keeps the cost
    // of an over-sized capacity (workgroups that start only to find no
    // partition) bounded
    const unsigned sweep_blocks = (unsigned)(parts < SWEEP_BLOCKS ? parts : SWEEP_BLOCKS);
    for (int p = 0; p < passes; ++p) {
        // lookback words alternate between two buffers; pass p clears the
        // buffer of pass p + 1 as it goes
        uint64_t *cur = rs.status + (p & 1) * rs.status_words;
        uint64_t *next = p + 1 < passes ? rs.status + ((p + 1) & 1) * rs.status_words : nullptr;
#define GS_OS(TH, IT, RB)                                                                            \
    hipLaunchKernelGGL((k_radix_onesweep<TH, IT, VT, RB>), dim3(sweep_blocks), dim3(TH), 0, st, src_k, \
                       src_v, dst_k, dst_v, d_count, cap, dbits * p, mask, dbits,                  \
                       rs.hist + R * p, cur, next, rs.tickets + p)
        if (wide) {
            GS_OS(1024, 8, 9);
        } else if (P == 4096) {
            GS_OS(512, 8, 8);
        } else if (P == 16384) {
            if constexpr (sizeof(VT) == 4) GS_OS(1024, 16, 8);
        } else {
            GS_OS(1024, 8, 8);
        }
#undef GS_OS
        uint32_t *tk = src_k;
        VT *tv = src_v;
        src_k = dst_k; src_v = dst_v;
        dst_k = tk; dst_v = tv;
    }
    return hipGetLastError();
}

hipError_t radix_sort_pairs(uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb,
                            const uint64_t *d_count, uint64_t cap, int bits,
                            const RadixScratch &rs, hipStream_t st, bool hist_ready, bool cleared)
{
    return sort_pairs_impl<uint32_t>(ka, va, kb, vb, d_count, cap, bits, rs, st, hist_ready, cleared);
}

hipError_t radix_sort_pairs_v2(uint32_t *ka, uint2 *va, uint32_t *kb, uint2 *vb, const uint64_t *d_count,
                               uint64_t cap, int bits, const RadixScratch &rs, hipStream_t st, bool hist_ready,
                               bool cleared)
{
    return sort_pairs_impl<uint2>(ka, va, kb, vb, d_count, cap, bits, rs, st, hist_ready, cleared);
}

size_t radix_sort_scratch_bytes(uint64_t n)
{
    // hist [4][256] u32 | tickets [4] u32 | count u64 | status [2][status words] u64
    return 4 * 256 * 4 + 4 * 4 + 8 + 256 + 2 * 8 * radix_status_words(n) + 256;
}

hipError_t radix_sort_standalone(uint32_t *keys, uint32_t *vals, uint32_t *kt, uint32_t *vt, uint64_t n,
                                 int bits, void *ws, int part, bool *in_tmp, hipStream_t st)
{
    char *base = (char *)ws;
    RadixScratch rs;
    rs.hist = (uint32_t *)base;
    rs.tickets = (uint32_t *)(base + 4 * 256 * 4);
    uint64_t *count = (uint64_t *)(base + 4 * 256 * 4 + 4 * 4 + 8);  // 8-byte aligned
    rs.status = (uint64_t *)(base + 4 * 256 * 4 + 4 * 4 + 8 + 256);
    rs.status = (uint64_t *)(((uintptr_t)rs.status + 255) & ~uintptr_t(255));
    rs.status_words = radix_status_words(n);
    rs.part = part;
    hipLaunchKernelGGL(k_set_count, dim3(1), dim3(1), 0, st, count, n);
    *in_tmp = radix_pass_count(bits, 4, part) % 2 == 1;
    return radix_sort_pairs(keys, vals, kt, vt, count, n, bits, rs, st, false);
}
