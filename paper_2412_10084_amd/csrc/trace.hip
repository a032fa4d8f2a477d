// Sphere-traced inference render.  The paper's real-time renderer shades voxels
// and volume renders them (supplementary "Performance Analysis"); this path
// marches t <- t + s(x) from the cube entry until s < eps (hit) or t > t_f
// (miss), at most max_steps evaluations (positions and step lengths in FP64),
// then shades the hit point once with the same colour model (Sec. 3.1-3.2, Sec. 4).  Rays are generated in the
// kernel from the pinhole cameras; a block covers a 16 x 16 pixel tile of one
// view so that a wave's rays (4 rows of 16) stay spatially coherent.
#include "dispatch.h"
#include "shade.h"

namespace psdf {

// Trilinear SDF at an FP64 point, interpolated in FP64 from the stored nodes.  The
// trace sums its step lengths (t <- t + s over tens of steps), so an FP32
// interpolation error of each s would accumulate in the hit point; in FP64 the hit
// decisions and the hit point agree with an FP64 evaluation to rounding.
template <typename T>
__device__ __forceinline__ double tri1_d(const T* __restrict__ g, int R, double inv_h,
                                         const double x[3]) {
  int k[3];
  double f[3];
  const double kmax = (double)(R - 2);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double u = (x[a] + 1.0) * inv_h;
    const double fl = fmin(fmax(floor(u), 0.0), kmax);
    k[a] = (int)fl;
    f[a] = u - fl;
  }
  const int b = (k[2] * R + k[1]) * R + k[0], RR = R * R;
  const float2 p00 = ld2(g, b), p10 = ld2(g, b + R), p01 = ld2(g, b + RR), p11 = ld2(g, b + RR + R);
  auto lerp = [](double a, double c, double t) { return fma(t, c - a, a); };
  const double a0 = lerp(p00.x, p00.y, f[0]), a1 = lerp(p10.x, p10.y, f[0]);
  const double a2 = lerp(p01.x, p01.y, f[0]), a3 = lerp(p11.x, p11.y, f[0]);
  return lerp(lerp(a0, a1, f[1]), lerp(a2, a3, f[1]), f[2]);
}

template <typename ST, typename FT, int NSH, int M>
__global__ void __launch_bounds__(BLOCK) sphere_trace_kernel(TraceArgs a) {
  __shared__ MlpLds<M> mlds[M == MLP_F32 ? 1 : WAVES];
  const int lane = threadIdx.x & 63;
  MlpLds<M>& ML = mlds[M == MLP_F32 ? 0 : (threadIdx.x >> 6)];
  const int px = blockIdx.x * 16 + (threadIdx.x & 15);
  const int py = blockIdx.y * 16 + (threadIdx.x >> 4);
  const int vi = blockIdx.z;
  const bool valid = px < a.W && py < a.H;
  const ST* __restrict__ sdf = static_cast<const ST*>(a.sdf);
  const FT* __restrict__ feat = static_cast<const FT*>(a.feat);
  const FT* __restrict__ probes = static_cast<const FT*>(a.probes);
  const float* __restrict__ cam = a.cams + 16 * vi;
  const Geo G{a.R, a.P, 2.0 / (a.R - 1), 0.5 * (a.R - 1), 0.5 * (a.P - 1), a.flags};
  MlpFrag<M> frag;
  if constexpr (M != MLP_F32) mlp_frag_load<M>(a.mlp, lane, frag);

  // pixel ray in FP64
  const double dcx = ((double)px + 0.5 - (double)cam[14]) / (double)cam[12];
  const double dcy = ((double)py + 0.5 - (double)cam[15]) / (double)cam[13];
  double d[3], o[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    d[k] = (double)cam[4 * k + 0] * dcx + (double)cam[4 * k + 1] * dcy + (double)cam[4 * k + 2];
    o[k] = cam[4 * k + 3];
  }
  const double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  d[0] /= dn;
  d[1] /= dn;
  d[2] /= dn;
  double t0 = -INFINITY, t1 = INFINITY;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double ta = (-1.0 - o[k]) / d[k];
    const double tb = (1.0 - o[k]) / d[k];
    t0 = fmax(t0, fmin(ta, tb));
    t1 = fmin(t1, fmax(ta, tb));
  }
  t0 = fmax(t0, 0.0);
  bool hit = false;
  double x[3] = {0.0, 0.0, 0.0};
  if (valid && t1 > t0) {
    double t = t0;
    for (int k = 0; k < a.max_steps; ++k) {
#pragma unroll
      for (int q = 0; q < 3; ++q) x[q] = fmin(fmax(fma(t, d[q], o[q]), -1.0), 1.0);
      const double s = tri1_d(sdf, a.R, G.inv_h, x);
      if (s < (double)a.eps) {
        hit = true;
        break;
      }
      t += s;
      if (t > t1) break;
    }
  }
  float out[3] = {0.f, 0.f, 0.f};
  if (__ballot(hit)) {
    const float v[3] = {(float)-d[0], (float)-d[1], (float)-d[2]};
    float z[NIN];
#pragma unroll
    for (int j = 0; j < NIN; ++j) z[j] = 0.f;
    if (hit) {
      float Y[NSH];
      sh_basis<NSH>(v[0], v[1], v[2], Y);
      Normal nm;
      shade_inputs<ST, FT, NSH>(sdf, feat, probes, G, x, v, Y, z, nm);
    }
    if constexpr (M == MLP_F32) {
      float pre[HID], hid[HID];
      mlp_lane<M>(const_mlp(a.mlp), z, pre, hid, out);
    } else {
      mlp_wave<M>(frag, ML, lane, z, out);
    }
    if (hit) {
      out[0] = sigmoidf(out[0]);
      out[1] = sigmoidf(out[1]);
      out[2] = sigmoidf(out[2]);
    } else {
      out[0] = out[1] = out[2] = 0.f;
    }
  }
  if (valid) {
    float* po = a.out + (((int64_t)vi * a.H + py) * a.W + px) * 3;
    po[0] = out[0];
    po[1] = out[1];
    po[2] = out[2];
  }
}

hipError_t launch_sphere_trace(const TraceArgs& a, int sdf_dt, int feat_dt, int mlp_dt, int n_sh,
                               hipStream_t s) {
  const dim3 grid((unsigned)((a.W + 15) / 16), (unsigned)((a.H + 15) / 16), (unsigned)a.V);
  PSDF_DT_SWITCH(sdf_dt, feat_dt, PSDF_SH_SWITCH(n_sh, PSDF_MLP_SWITCH(mlp_dt,
      hipLaunchKernelGGL((sphere_trace_kernel<ST, FT, NSH, M>), grid, dim3(BLOCK), 0, s, a))));
  return hipGetLastError();
}

}  // namespace psdf
