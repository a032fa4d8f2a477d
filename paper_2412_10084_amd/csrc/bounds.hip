// Brick bounds of an SDF grid: for every block of 8^3 cells, the min and max of
// the nodes those cells interpolate (nodes [8b, min(8b+8, R-1)] per axis).  The
// renderers use them to skip samples that the skip rule (Sec. 3.3) would leave
// inactive without reading their corners.
//
// One workgroup per (y, z) brick pair: each thread reduces one x column over the
// (up to) 9 x 9 node rows of the pair with coalesced row reads, then the brick
// ranges along x are reduced from LDS.
#include "device.h"
#include "kernels.h"

namespace psdf {

constexpr int BBLOCK = 256;
constexpr int BMAX_R = 1024;

template <typename T>
__global__ void __launch_bounds__(BBLOCK) sdf_bounds_kernel(const T* __restrict__ sdf, int R, int nb,
                                                            float2* __restrict__ out) {
  __shared__ float cmin[BMAX_R], cmax[BMAX_R];
  const int by = (int)blockIdx.x % nb, bz = (int)blockIdx.x / nb;
  const int y0 = by * 8, y1 = min(y0 + 8, R - 1), z0 = bz * 8, z1 = min(z0 + 8, R - 1);
  for (int x = threadIdx.x; x < R; x += BBLOCK) {
    float mn = INFINITY, mx = -INFINITY;
    for (int z = z0; z <= z1; ++z)
      for (int y = y0; y <= y1; ++y) {
        const float v = ld1(sdf, (z * R + y) * R + x);
        mn = fminf(mn, v);
        mx = fmaxf(mx, v);
      }
    cmin[x] = mn;
    cmax[x] = mx;
  }
  __syncthreads();
  for (int bx = threadIdx.x; bx < nb; bx += BBLOCK) {
    const int x0 = bx * 8, x1 = min(x0 + 8, R - 1);
    float mn = INFINITY, mx = -INFINITY;
    for (int x = x0; x <= x1; ++x) {
      mn = fminf(mn, cmin[x]);
      mx = fmaxf(mx, cmax[x]);
    }
    out[(bz * nb + by) * nb + bx] = make_float2(mn, mx);
  }
}

hipError_t launch_sdf_bounds(const void* sdf, int R, int sdf_dt, float* bounds, hipStream_t s) {
  const int nb = ((R - 2) >> 3) + 1;
  const dim3 grid((unsigned)(nb * nb));
  float2* out = reinterpret_cast<float2*>(bounds);
  if (sdf_dt == 0)
    hipLaunchKernelGGL(sdf_bounds_kernel<float>, grid, dim3(BBLOCK), 0, s,
                       static_cast<const float*>(sdf), R, nb, out);
  else
    hipLaunchKernelGGL(sdf_bounds_kernel<_Float16>, grid, dim3(BBLOCK), 0, s,
                       static_cast<const _Float16*>(sdf), R, nb, out);
  return hipGetLastError();
}

}  // namespace psdf
