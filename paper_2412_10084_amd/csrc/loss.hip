// Photometric loss.  The paper uses a relatively weighted L2 (Eq. photo_loss);
// this kernel computes its L1 form: L = mean over B x 3 of |rgb - target| and
// dL/drgb = sign(rgb - target) / (3B), sign(0) = 0.
#include "device.h"
#include "kernels.h"

namespace psdf {

constexpr int LBLOCK = 256;

__global__ void __launch_bounds__(LBLOCK) l1_loss_kernel(int64_t n, float scale, const float* rgb,
                                                         const float* target, float* dL,
                                                         float* loss) {
  __shared__ float part[LBLOCK / 64];
  float acc = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * LBLOCK + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * LBLOCK) {
    const float d = rgb[i] - target[i];
    acc += fabsf(d);
    dL[i] = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
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
  // every block adds its partial sum to the one loss value, and same-address
  // atomics serialise: few blocks, each looping
  int64_t blocks = (n + 8 * LBLOCK - 1) / (8 * LBLOCK);
  if (blocks > 256) blocks = 256;
  hipLaunchKernelGGL(l1_loss_kernel, dim3((unsigned)blocks), dim3(LBLOCK), 0, s, n,
                     (float)(1.0 / (3.0 * (double)B)), rgb, target, dL, loss);
  return hipGetLastError();
}

}  // namespace psdf
