// L1 photometric loss and its gradient with respect to the image.
#include "common.hpp"
#include "kernels.hpp"

namespace {

__global__ void __launch_bounds__(256)
k_l1_grad(const float *__restrict__ image, const float *__restrict__ target, uint64_t n, float scale,
          float *__restrict__ dL, float *__restrict__ loss)
{
    __shared__ float s_part[4];
    float acc = 0.f;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const float d = image[k] - target[k];
        acc += fabsf(d);
        dL[k] = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float b = s_part[0] + s_part[1] + s_part[2] + s_part[3];
        if (b != 0.f) atomicAdd(loss, b * scale);
    }
}

}  // namespace

hipError_t launch_l1_grad(const float *image, const float *target, uint64_t n, float scale,
                          float *dL_dimage, float *loss, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 256 * 8 - 1) / (256 * 8);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_l1_grad, dim3((unsigned)blocks), dim3(256), 0, st, image, target, n, scale, dL_dimage,
                       loss);
    return hipGetLastError();
}
