// Photometric losses: the L1 form L = mean over B x 3 of |rgb - target| with
// dL/drgb = sign(rgb - target) / (3B), sign(0) = 0; and the paper's relatively
// weighted L2 (Eq. photo_loss).
#include "device.h"
#include "kernels.h"

namespace psdf {

constexpr int LBLOCK = 256;
constexpr int kPer = 4;  // float4 per thread on the vector path, all loaded before use

__device__ __forceinline__ float l1_grad(float d, float scale) {
  return d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
}

// VEC: n is a multiple of 4 and the three arrays are 16-byte aligned
template <bool VEC>
__global__ void __launch_bounds__(LBLOCK) l1_loss_kernel(int64_t n, float scale, const float* rgb,
                                                         const float* target, float* dL,
                                                         float* loss) {
  __shared__ float part[LBLOCK / 64];
  float acc = 0.f;
  if constexpr (VEC) {
    const int64_t n4 = n >> 2;
    const float4* r4 = reinterpret_cast<const float4*>(rgb);
    const float4* t4 = reinterpret_cast<const float4*>(target);
    float4* d4 = reinterpret_cast<float4*>(dL);
    const int64_t base = (int64_t)blockIdx.x * (LBLOCK * kPer) + threadIdx.x;
    float4 x[kPer], y[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int64_t i = base + (int64_t)j * LBLOCK;
      if (i < n4) {
        x[j] = r4[i];
        y[j] = t4[i];
      }
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int64_t i = base + (int64_t)j * LBLOCK;
      if (i < n4) {
        const float dx = x[j].x - y[j].x, dy = x[j].y - y[j].y;
        const float dz = x[j].z - y[j].z, dw = x[j].w - y[j].w;
        acc += fabsf(dx) + fabsf(dy) + fabsf(dz) + fabsf(dw);
        d4[i] = make_float4(l1_grad(dx, scale), l1_grad(dy, scale), l1_grad(dz, scale),
                            l1_grad(dw, scale));
      }
    }
  } else {
    for (int64_t i = (int64_t)blockIdx.x * LBLOCK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * LBLOCK) {
      const float d = rgb[i] - target[i];
      acc += fabsf(d);
      dL[i] = l1_grad(d, scale);
    }
  }
  if (loss) {
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      float s = 0.f;
      for (int w = 0; w < LBLOCK / 64; ++w) s += part[w];
      atomic_add_f32(loss, s * scale);
    }
  }
}

__global__ void zero1_kernel(float* p) {
  if (threadIdx.x == 0) p[0] = 0.f;
}

hipError_t launch_l1_loss(int64_t B, const float* rgb, const float* target, float* dL, float* loss,
                          hipStream_t s) {
  const int64_t n = 3 * B;
  if (loss) hipLaunchKernelGGL(zero1_kernel, dim3(1), dim3(64), 0, s, loss);
  const float scale = (float)(1.0 / (3.0 * (double)B));
  const auto al16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  if (n % 4 == 0 && al16(rgb) && al16(target) && al16(dL)) {
    const int64_t per = (int64_t)LBLOCK * kPer, blocks = (n / 4 + per - 1) / per;
    if (blocks > 0)
      hipLaunchKernelGGL(l1_loss_kernel<true>, dim3((unsigned)blocks), dim3(LBLOCK), 0, s, n,
                         scale, rgb, target, dL, loss);
  } else {
    // every block adds its partial sum to the one loss value, and same-address
    // atomics serialise: few blocks, each looping
    int64_t blocks = (n + 8 * LBLOCK - 1) / (8 * LBLOCK);
    if (blocks > 256) blocks = 256;
    if (blocks > 0)
      hipLaunchKernelGGL(l1_loss_kernel<false>, dim3((unsigned)blocks), dim3(LBLOCK), 0, s, n,
                         scale, rgb, target, dL, loss);
  }
  return hipGetLastError();
}

// Relatively weighted L2 (Eq. photo_loss with the per-pixel weight (max(c, c_gt) +
// eps)^-1 on its gradient, scaled by lambda / n_images): per channel
//   L = sc * sum (c - c_gt)^2 / (max(c, c_gt) + eps),  dL/dc = 2 sc (c - c_gt) / (max + eps),
// the weight held constant.  Grid-stride over the 3B values, one atomic per block.
__global__ void __launch_bounds__(LBLOCK) l2rel_loss_kernel(int64_t n, float sc, float eps,
                                                            const float* rgb, const float* target,
                                                            float* dL, float* loss) {
  __shared__ float part[LBLOCK / 64];
  float acc = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * LBLOCK + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * LBLOCK) {
    const float c = rgb[i], t = target[i];
    const float d = c - t;
    const float w = 1.0f / (fmaxf(c, t) + eps);
    acc += d * d * w;
    dL[i] = 2.0f * sc * d * w;
  }
  if (loss) {
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      float s = 0.f;
      for (int w = 0; w < LBLOCK / 64; ++w) s += part[w];
      atomic_add_f32(loss, s * sc);
    }
  }
}

hipError_t launch_l2rel_loss(int64_t B, const float* rgb, const float* target, float* dL,
                             float* loss, float lambda, float eps, float n_images, hipStream_t s) {
  const int64_t n = 3 * B;
  if (loss) hipLaunchKernelGGL(zero1_kernel, dim3(1), dim3(64), 0, s, loss);
  int64_t blocks = (n + 8 * LBLOCK - 1) / (8 * LBLOCK);
  if (blocks > 1024) blocks = 1024;
  if (blocks > 0)
    hipLaunchKernelGGL(l2rel_loss_kernel, dim3((unsigned)blocks), dim3(LBLOCK), 0, s, n,
                       lambda / n_images, eps, rgb, target, dL, loss);
  return hipGetLastError();
}

}  // namespace psdf
