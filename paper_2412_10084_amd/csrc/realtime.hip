// Real-time render of the supplementary "Performance Analysis": a shading pass
// assigns a colour to every voxel near the surface, then a volume-rendering pass
// samples the SDF and that colour field along the pixel rays.
//   voxel_list_kernel    the nodes with |s| <= band, compacted (one atomic per
//                        block of 16384 nodes); view-independent, built once per SDF;
//   voxel_shade_kernel   one listed node per lane: view direction from the node to
//                        the camera centre, FD normal, F_s, F_a, MLP (per lane, or
//                        FP16 / BF16 MFMA over the wave) -> colour grid;
//   volume_render_kernel one pixel ray per lane (16 x 16 pixel tiles), the same
//                        march, skip rule, brick skipping and NeuS weights as the
//                        training forward, colour = trilinear of the colour grid.
#include "dispatch.h"
#include "shade.h"

namespace psdf {

__global__ void zero_count_kernel(int* c) {
  if (threadIdx.x == 0) c[0] = 0;
}

// One block lists VL_IT x VL_CHUNK consecutive nodes: each thread tests VL_V
// consecutive nodes per round (one 16- or 32-byte load when the grid is 16-byte
// aligned), keeps the in-band bits, and the block reserves its whole range with a
// single atomic before writing the indices, in node order within the block.
constexpr int VL_V = 8, VL_IT = 8, VL_CHUNK = 256 * VL_V;
typedef _Float16 h8v __attribute__((ext_vector_type(8)));

template <typename ST, bool VEC>
__device__ __forceinline__ unsigned band_bits(const ST* __restrict__ sdf, int64_t n0, int64_t n3,
                                              float band) {
  float v[VL_V];
  if (VEC && n0 + VL_V <= n3) {
    if constexpr (sizeof(ST) == 2) {
      const h8v h = *reinterpret_cast<const h8v*>(sdf + n0);
#pragma unroll
      for (int j = 0; j < VL_V; ++j) v[j] = (float)h[j];
    } else {
      const float4 a = reinterpret_cast<const float4*>(sdf + n0)[0];
      const float4 b = reinterpret_cast<const float4*>(sdf + n0)[1];
      v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w;
      v[4] = b.x, v[5] = b.y, v[6] = b.z, v[7] = b.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < VL_V; ++j) v[j] = n0 + j < n3 ? ld1(sdf, (int)(n0 + j)) : INFINITY;
  }
  unsigned m = 0;
#pragma unroll
  for (int j = 0; j < VL_V; ++j) m |= (fabsf(v[j]) <= band ? 1u : 0u) << j;
  return m;
}

template <typename ST, bool VEC>
__global__ void __launch_bounds__(256) voxel_list_kernel(int64_t n3, const ST* __restrict__ sdf,
                                                         float band, int* __restrict__ list,
                                                         int64_t cap, int* __restrict__ count) {
  __shared__ int woff[VL_IT][4];
  __shared__ int bbase;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t b0 = (int64_t)blockIdx.x * (VL_CHUNK * VL_IT) + threadIdx.x * VL_V;
  unsigned bits[VL_IT];
  int pre[VL_IT];
#pragma unroll
  for (int k = 0; k < VL_IT; ++k) bits[k] = band_bits<ST, VEC>(sdf, b0 + (int64_t)k * VL_CHUNK, n3, band);
#pragma unroll
  for (int k = 0; k < VL_IT; ++k) {
    const int c = __popc(bits[k]);
    int x = c;  // inclusive prefix over the wave's lanes
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(x, d);
      if (lane >= d) x += y;
    }
    pre[k] = x - c;
    if (lane == 63) woff[k][wv] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int k = 0; k < VL_IT; ++k)
      for (int w = 0; w < 4; ++w) {
        const int t = woff[k][w];
        woff[k][w] = tot;
        tot += t;
      }
    bbase = tot ? atomicAdd(count, tot) : 0;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < VL_IT; ++k) {
    int64_t slot = (int64_t)bbase + woff[k][wv] + pre[k];
    const int64_t n0 = b0 + (int64_t)k * VL_CHUNK;
    for (unsigned m = bits[k]; m; m &= m - 1, ++slot)
      if (slot < cap) list[slot] = (int)(n0 + __ffs(m) - 1);
  }
}

// colour grid element: FP32 (r, g, b, 0) or FP16 (r, g, b, 0), 16 or 8 bytes
__device__ __forceinline__ void store_colour(float* g, int64_t n, float r, float gg, float b) {
  reinterpret_cast<float4*>(g)[n] = make_float4(r, gg, b, 0.f);
}
__device__ __forceinline__ void store_colour(_Float16* g, int64_t n, float r, float gg, float b) {
  h4 v = {(_Float16)r, (_Float16)gg, (_Float16)b, (_Float16)0.f};
  reinterpret_cast<h4*>(g)[n] = v;
}
__device__ __forceinline__ float4 load_colour(const float* g, int n) {
  return reinterpret_cast<const float4*>(g)[n];
}
__device__ __forceinline__ float4 load_colour(const _Float16* g, int n) {
  const h4 v = reinterpret_cast<const h4*>(g)[n];
  return make_float4((float)v.x, (float)v.y, (float)v.z, 0.f);
}

template <typename ST, typename FT, int NSH, int M, typename CT>
__global__ void __launch_bounds__(BLOCK) voxel_shade_kernel(RealtimeArgs a) {
  __shared__ MlpLds<M> mlds[M == MLP_F32 ? 1 : WAVES];
  const int lane = threadIdx.x & 63;
  MlpLds<M>& ML = mlds[M == MLP_F32 ? 0 : (threadIdx.x >> 6)];
  const ST* __restrict__ sdf = static_cast<const ST*>(a.sdf);
  const FT* __restrict__ feat = static_cast<const FT*>(a.feat);
  const FT* __restrict__ probes = static_cast<const FT*>(a.probes);
  CT* __restrict__ colour = static_cast<CT*>(a.colour);
  const Geo G{a.R, a.P, 2.0 / (a.R - 1), 0.5 * (a.R - 1), 0.5 * (a.P - 1), a.flags};
  MlpFrag<M> frag;
  if constexpr (M != MLP_F32) mlp_frag_load<M>(a.mlp, lane, frag);
  const double c[3] = {a.cam[3], a.cam[7], a.cam[11]};
  const int64_t n_list = min((int64_t)*a.count, a.cap);
  const int R = a.R;
  // every wave runs the same number of rounds (the MFMA path needs whole waves)
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t base = (int64_t)blockIdx.x * BLOCK + (threadIdx.x & ~63); base < n_list;
       base += stride) {
    const int64_t e = base + lane;
    const bool ve = e < n_list;
    const int n = ve ? a.list[e] : 0;
    float z[NIN];
#pragma unroll
    for (int j = 0; j < NIN; ++j) z[j] = 0.f;
    if (ve) {
      const int i = n % R, jy = (n / R) % R, k = n / (R * R);
      const double x[3] = {-1.0 + i * G.h, -1.0 + jy * G.h, -1.0 + k * G.h};
      double v[3], vn = 0.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        v[q] = c[q] - x[q];
        vn += v[q] * v[q];
      }
      vn = sqrt(vn);
      const float vf[3] = {(float)(v[0] / vn), (float)(v[1] / vn), (float)(v[2] / vn)};
      float Y[NSH];
      sh_basis<NSH>(vf[0], vf[1], vf[2], Y);
      Normal nm;
      shade_inputs<ST, FT, NSH>(sdf, feat, probes, G, x, vf, Y, z, nm);
    }
    float out[3];
    if constexpr (M == MLP_F32) {
      float pre[HID], hid[HID];
      mlp_lane<M>(const_mlp(a.mlp), z, pre, hid, out);
    } else {
      mlp_wave<M>(frag, ML, lane, z, out);
    }
    if (ve) store_colour(colour, n, sigmoidf(out[0]), sigmoidf(out[1]), sigmoidf(out[2]));
  }
}

// pixel ray of a pinhole camera in FP64 (the camera layout of the sphere tracer)
__device__ __forceinline__ bool pixel_ray(const float* __restrict__ cam, int px, int py, int N,
                                          RayD& r) {
  const double dcx = ((double)px + 0.5 - (double)cam[14]) / (double)cam[12];
  const double dcy = ((double)py + 0.5 - (double)cam[15]) / (double)cam[13];
  double d[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    d[k] = (double)cam[4 * k + 0] * dcx + (double)cam[4 * k + 1] * dcy + (double)cam[4 * k + 2];
    r.o[k] = cam[4 * k + 3];
  }
  const double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double t0 = -INFINITY, t1 = INFINITY;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r.d[k] = d[k] / dn;
    const double ta = (-1.0 - r.o[k]) / r.d[k];
    const double tb = (1.0 - r.o[k]) / r.d[k];
    t0 = fmax(t0, fmin(ta, tb));
    t1 = fmin(t1, fmax(ta, tb));
  }
  t0 = fmax(t0, 0.0);
  const bool hit = t1 > t0;
  r.tn = t0;
  r.dt = hit ? (t1 - t0) / (double)N : 0.0;
  return hit;
}

template <typename ST, typename CT>
__global__ void __launch_bounds__(BLOCK) volume_render_kernel(RealtimeArgs a) {
  unsigned bx, by, bz;
  xcd_block3(bx, by, bz);
  const int px = bx * 16 + (threadIdx.x & 15);
  const int py = by * 16 + (threadIdx.x >> 4);
  const bool valid = px < a.W && py < a.H;
  const ST* __restrict__ sdf = static_cast<const ST*>(a.sdf);
  const CT* __restrict__ colour = static_cast<const CT*>(a.colour);
  const double inv_h = 0.5 * (a.R - 1);
  RayD r;
  const bool hit = pixel_ray(a.cam, px, py, a.N, r) && valid;
  const Bricks K = make_bricks(a.bounds, a.R, a.skip_thr);
  float rgb[3] = {0.f, 0.f, 0.f}, logT = 0.f;
  MarchState ms;
  march_begin(sdf, a.R, K, r, inv_h, hit, a.N, ms);
  for (int i = 0; i < a.N - 1; ++i) {  // wave-uniform
    float s_i, s_n;
    bool may;
    march_next(sdf, a.R, K, hit, i, a.N, ms, s_i, s_n, may);
    const bool active = may && (a.skip_thr <= 0.f || fabsf(s_i) <= a.skip_thr);
    if (active) {
      const float dl = log_sigmoid(a.tau * s_n) - log_sigmoid(a.tau * s_i);
      if (dl < 0.f) {
        const float w = expf(logT) * -expm1f(dl);
        logT += dl;
        double x[3];
        sample_pos(r, sample_t(r, i), x);
        const Cell cc = cell_d(x, a.R, inv_h);
        float wc[8];
        corner_w(cc, wc);
        float c0 = 0.f, c1 = 0.f, c2 = 0.f;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float4 col = load_colour(colour, cc.base + corner_off(q, a.R));
          c0 = fmaf(wc[q], col.x, c0);
          c1 = fmaf(wc[q], col.y, c1);
          c2 = fmaf(wc[q], col.z, c2);
        }
        rgb[0] = fmaf(w, c0, rgb[0]);
        rgb[1] = fmaf(w, c1, rgb[1]);
        rgb[2] = fmaf(w, c2, rgb[2]);
      }
    }
  }
  if (valid) {
    float* po = a.out + ((int64_t)py * a.W + px) * 3;
    po[0] = rgb[0];
    po[1] = rgb[1];
    po[2] = rgb[2];
  }
}

hipError_t launch_voxel_list(int R, int sdf_dt, const void* sdf, float band, int* list,
                             int64_t cap, int* count, hipStream_t s) {
  hipLaunchKernelGGL(zero_count_kernel, dim3(1), dim3(64), 0, s, count);
  const int64_t n3 = (int64_t)R * R * R;
  const dim3 grid((unsigned)((n3 + VL_CHUNK * VL_IT - 1) / (VL_CHUNK * VL_IT)));
  const bool vec = reinterpret_cast<uintptr_t>(sdf) % 16 == 0;
  if (sdf_dt == 0) {
    const float* p = static_cast<const float*>(sdf);
    if (vec)
      hipLaunchKernelGGL((voxel_list_kernel<float, true>), grid, dim3(256), 0, s, n3, p, band, list, cap, count);
    else
      hipLaunchKernelGGL((voxel_list_kernel<float, false>), grid, dim3(256), 0, s, n3, p, band, list, cap, count);
  } else {
    const _Float16* p = static_cast<const _Float16*>(sdf);
    if (vec)
      hipLaunchKernelGGL((voxel_list_kernel<_Float16, true>), grid, dim3(256), 0, s, n3, p, band, list, cap, count);
    else
      hipLaunchKernelGGL((voxel_list_kernel<_Float16, false>), grid, dim3(256), 0, s, n3, p, band, list, cap, count);
  }
  return hipGetLastError();
}

hipError_t launch_voxel_shade(const RealtimeArgs& a, int sdf_dt, int feat_dt, int mlp_dt, int n_sh,
                              int colour_dt, hipStream_t s) {
  // enough waves for the listed nodes of a surface band, each looping
  const int64_t blocks = min((a.cap + BLOCK - 1) / BLOCK, (int64_t)16384);
  const dim3 grid((unsigned)(blocks > 0 ? blocks : 1));
  if (colour_dt == 0) {
    typedef float CT;
    PSDF_DT_SWITCH(sdf_dt, feat_dt, PSDF_SH_SWITCH(n_sh, PSDF_MLP_SWITCH(mlp_dt,
        hipLaunchKernelGGL((voxel_shade_kernel<ST, FT, NSH, M, CT>), grid, dim3(BLOCK), 0, s, a))));
  } else {
    typedef _Float16 CT;
    PSDF_DT_SWITCH(sdf_dt, feat_dt, PSDF_SH_SWITCH(n_sh, PSDF_MLP_SWITCH(mlp_dt,
        hipLaunchKernelGGL((voxel_shade_kernel<ST, FT, NSH, M, CT>), grid, dim3(BLOCK), 0, s, a))));
  }
  return hipGetLastError();
}

hipError_t launch_volume_render(const RealtimeArgs& a, int sdf_dt, int colour_dt, hipStream_t s) {
  const dim3 grid((unsigned)((a.W + 15) / 16), (unsigned)((a.H + 15) / 16), 1);
  if (sdf_dt == 0 && colour_dt == 0)
    hipLaunchKernelGGL((volume_render_kernel<float, float>), grid, dim3(BLOCK), 0, s, a);
  else if (sdf_dt == 0)
    hipLaunchKernelGGL((volume_render_kernel<float, _Float16>), grid, dim3(BLOCK), 0, s, a);
  else if (colour_dt == 0)
    hipLaunchKernelGGL((volume_render_kernel<_Float16, float>), grid, dim3(BLOCK), 0, s, a);
  else
    hipLaunchKernelGGL((volume_render_kernel<_Float16, _Float16>), grid, dim3(BLOCK), 0, s, a);
  return hipGetLastError();
}

}  // namespace psdf
