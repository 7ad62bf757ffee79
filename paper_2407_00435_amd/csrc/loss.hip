// L1 photometric loss and its gradient with respect to the image.
#include "common.hpp"
#include "kernels.hpp"

namespace {

__device__ __forceinline__ float l1_sign(float d, float scale) { return d > 0.f ? scale : (d < 0.f ? -scale : 0.f); }

__device__ __forceinline__ void l1_block_add(float acc, float scale, float *__restrict__ loss)
{
    __shared__ float s_part[4];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float b = s_part[0] + s_part[1] + s_part[2] + s_part[3];
        if (b != 0.f) atomicAdd(loss, b * scale);
    }
}

// Unaligned buffers: a grid-stride loop over single floats.
__global__ void __launch_bounds__(256)
k_l1_grad(const float *__restrict__ image, const float *__restrict__ target, uint64_t n, float scale,
          float *__restrict__ dL, float *__restrict__ loss)
{
    float acc = 0.f;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const float d = image[k] - target[k];
        acc += fabsf(d);
        dL[k] = l1_sign(d, scale);
    }
    l1_block_add(acc, scale, loss);
}

// 16-byte aligned buffers of at least 4 floats: each thread takes L1_VEC
// float4 of its block's span, all loads issued before the first use
// (clamped in bounds, selected after), and block 0 also takes the n % 4 tail.
constexpr int L1_VEC = 4;
__global__ void __launch_bounds__(256)
k_l1_grad4(const float4 *__restrict__ image, const float4 *__restrict__ target, uint64_t n, float scale,
           float4 *__restrict__ dL, float *__restrict__ loss)
{
    const uint64_t n4 = n / 4;
    const uint64_t base = (uint64_t)blockIdx.x * (256 * L1_VEC) + threadIdx.x;
    float4 a[L1_VEC], b[L1_VEC];
#pragma unroll
    for (int j = 0; j < L1_VEC; ++j) {
        const uint64_t k = base + (uint64_t)j * 256;
        const uint64_t kc = k < n4 ? k : 0;
        a[j] = image[kc];
        b[j] = target[kc];
    }
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < L1_VEC; ++j) {
        const uint64_t k = base + (uint64_t)j * 256;
        if (k < n4) {
            const float4 d = make_float4(a[j].x - b[j].x, a[j].y - b[j].y, a[j].z - b[j].z, a[j].w - b[j].w);
            acc += (fabsf(d.x) + fabsf(d.y)) + (fabsf(d.z) + fabsf(d.w));
            dL[k] = make_float4(l1_sign(d.x, scale), l1_sign(d.y, scale), l1_sign(d.z, scale), l1_sign(d.w, scale));
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < (n & 3)) {
        const uint64_t k = n4 * 4 + threadIdx.x;
        const float d = reinterpret_cast<const float *>(image)[k] - reinterpret_cast<const float *>(target)[k];
        acc += fabsf(d);
        reinterpret_cast<float *>(dL)[k] = l1_sign(d, scale);
    }
    l1_block_add(acc, scale, loss);
}

}  // namespace

hipError_t launch_l1_grad(const float *image, const float *target, uint64_t n, float scale,
                          float *dL_dimage, float *loss, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const bool aligned = ((reinterpret_cast<uintptr_t>(image) | reinterpret_cast<uintptr_t>(target) |
                           reinterpret_cast<uintptr_t>(dL_dimage)) & 15) == 0;
    if (aligned && n >= 4) {
        const uint64_t blocks = (n / 4 + 256 * L1_VEC - 1) / (256 * L1_VEC);
        hipLaunchKernelGGL(k_l1_grad4, dim3((unsigned)(blocks ? blocks : 1)), dim3(256), 0, st,
                           reinterpret_cast<const float4 *>(image), reinterpret_cast<const float4 *>(target), n,
                           scale, reinterpret_cast<float4 *>(dL_dimage), loss);
    } else {
        uint64_t blocks = (n + 256 * 8 - 1) / (256 * 8);
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(k_l1_grad, dim3((unsigned)blocks), dim3(256), 0, st, image, target, n, scale,
                           dL_dimage, loss);
    }
    return hipGetLastError();
}
