// Fused optimiser step over the ProbeSDF parameters: regulariser gradients
// (eikonal on the SDF, squared-difference smoothness on the features and on the
// probe coefficients; Sec. 3.3, Eqs. eikonal_reg, smooth_features,
// smooth_probes) added to the accumulated render gradient, then Adam (Sec. 3.4;
// moments as in the supplementary scheduling section).
//
// The feature and probe grids are streaming passes launched as (row chunk, j,
// k): a thread owns four parameters, gathers the regulariser gradient of each
// from its stencil (no scatter, no atomics), applies Adam, writes the new value
// to a separate output buffer (neighbours still read the old one), writes the
// moments back, zeroes the gradient and optionally writes an FP16 copy.  The
// SDF pass (eikonal) is tiled through LDS (step_sdf.hip).
#include "device.h"
#include "kernels.h"

namespace psdf {

constexpr int SBLOCK = 256;

// (blocks of up to SBLOCK threads, a multiple of 64)
__device__ __forceinline__ void block_add(float val, float* dst) {
  __shared__ float part[SBLOCK / 64];
  val = wave_sum(val);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = val;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += part[w];
    if (s != 0.f) atomic_add_f32(dst, s);
  }
}

// ---------------------------------------------------------------------------
// smoothness + Adam on a grid with C channels per node:
// dL/dF_{m,c} = 2 lambda / (3 R^2 (R-1) C) * sum over existing neighbours nb of (F_m - F_nb)
// ---------------------------------------------------------------------------
struct TvArgs {
  int R;
  float lambda, lr;
  const float* F_in;
  float* F_out;
  float* g;
  float* m;
  float* v;
  _Float16* half_out;
  float* loss_dst;
};

template <int C>  // channels per node; one float per thread
__global__ void __launch_bounds__(SBLOCK) step_tv_kernel(TvArgs t, StepArgs a) {
  const int R = t.R, rowlen = R * C;
  unsigned bx, by, bz;
  xcd_block3(bx, by, bz);
  const int xi = bx * SBLOCK + threadIdx.x, j = by, k = bz;
  const bool valid = xi < rowlen;
  const float npairs = 3.0f * (float)R * (float)R * (float)(R - 1);
  const float scale = t.lambda / (npairs * (float)C);
  float loss = 0.f;
  if (valid) {
    const int i = xi / C;
    const int e = (k * R + j) * rowlen + xi;
    const int sy = rowlen, sz = R * rowlen;
    const float* __restrict__ F = t.F_in;
    const float f = F[e];
    float acc = 0.f;
    if (i > 0) acc += f - F[e - C];
    if (i < R - 1) { const float d = F[e + C] - f; acc -= d; loss += d * d; }
    if (j > 0) acc += f - F[e - sy];
    if (j < R - 1) { const float d = F[e + sy] - f; acc -= d; loss += d * d; }
    if (k > 0) acc += f - F[e - sz];
    if (k < R - 1) { const float d = F[e + sz] - f; acc -= d; loss += d * d; }
    const float g = t.g[e];
    const float G = g + 2.0f * scale * acc;
    float m = t.m[e], v = t.v[e];
    const float p = adam_update_f(f, G, m, v, t.lr, a.beta1, a.beta2, a.eps, a.bc1, a.bc2);
    t.F_out[e] = p;
    t.m[e] = m;
    t.v[e] = v;
    if (g != 0.f) t.g[e] = 0.f;  // the render gradient is sparse
    if (t.half_out) t.half_out[e] = (_Float16)p;
  }
  if (t.loss_dst) block_add(loss * scale, t.loss_dst);
}

// four consecutive channels of one node per thread (C a multiple of 4)
__device__ __forceinline__ float4 ld4g(const float* p, int e) {
  return *reinterpret_cast<const float4*>(p + e);
}
__device__ __forceinline__ void st4g(float* p, int e, float4 v) {
  *reinterpret_cast<float4*>(p + e) = v;
}
// streaming (non-temporal) access for the optimiser state and the gradient: each
// is touched once per step, so it should not displace cached grid data
typedef float nf4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld4s(const float* p, int e) {
  const nf4 v = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(p + e));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st4s(float* p, int e, float4 v) {
  const nf4 w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, reinterpret_cast<nf4*>(p + e));
}

template <int C>
__global__ void __launch_bounds__(SBLOCK) step_tv4_kernel(TvArgs t, StepArgs a) {
  static_assert(C % 4 == 0, "vector path needs C % 4 == 0");
  const int R = t.R, rowlen = R * C;
  unsigned bx, by, bz;
  xcd_block3(bx, by, bz);
  const int xi = (bx * SBLOCK + threadIdx.x) * 4, j = by, k = bz;
  const bool valid = xi < rowlen;
  const float npairs = 3.0f * (float)R * (float)R * (float)(R - 1);
  const float scale = t.lambda / (npairs * (float)C);
  float loss = 0.f;
  if (valid) {
    const int i = xi / C;
    const int e = (k * R + j) * rowlen + xi;
    const int sy = rowlen, sz = R * rowlen;
    const float* __restrict__ F = t.F_in;
    const float4 f = ld4g(F, e);
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    auto back = [&](int off) {
      const float4 b = ld4g(F, e - off);
      acc.x += f.x - b.x; acc.y += f.y - b.y; acc.z += f.z - b.z; acc.w += f.w - b.w;
    };
    auto fwd = [&](int off) {
      const float4 b = ld4g(F, e + off);
      const float dx = b.x - f.x, dy = b.y - f.y, dz = b.z - f.z, dw = b.w - f.w;
      acc.x -= dx; acc.y -= dy; acc.z -= dz; acc.w -= dw;
      loss += dx * dx + dy * dy + dz * dz + dw * dw;
    };
    if (i > 0) back(C);
    if (i < R - 1) fwd(C);
    if (j > 0) back(sy);
    if (j < R - 1) fwd(sy);
    if (k > 0) back(sz);
    if (k < R - 1) fwd(sz);
    const float4 g = ld4s(t.g, e);
    float4 m = ld4s(t.m, e), v = ld4s(t.v, e);
    const float s2 = 2.0f * scale;
    float4 p;
    p.x = adam_update_f(f.x, g.x + s2 * acc.x, m.x, v.x, t.lr, a.beta1, a.beta2, a.eps, a.bc1, a.bc2);
    p.y = adam_update_f(f.y, g.y + s2 * acc.y, m.y, v.y, t.lr, a.beta1, a.beta2, a.eps, a.bc1, a.bc2);
    p.z = adam_update_f(f.z, g.z + s2 * acc.z, m.z, v.z, t.lr, a.beta1, a.beta2, a.eps, a.bc1, a.bc2);
    p.w = adam_update_f(f.w, g.w + s2 * acc.w, m.w, v.w, t.lr, a.beta1, a.beta2, a.eps, a.bc1, a.bc2);
    st4g(t.F_out, e, p);
    st4s(t.m, e, m);
    st4s(t.v, e, v);
    // the render gradient is sparse: only nonzero entries are cleared
    if (g.x != 0.f || g.y != 0.f || g.z != 0.f || g.w != 0.f)
      st4g(t.g, e, make_float4(0.f, 0.f, 0.f, 0.f));
    if (t.half_out) {
      h4 hv = {(_Float16)p.x, (_Float16)p.y, (_Float16)p.z, (_Float16)p.w};
      *reinterpret_cast<h4*>(t.half_out + e) = hv;
    }
  }
  if (t.loss_dst) block_add(loss * scale, t.loss_dst);
}

// three channels per node, four consecutive floats per thread (R % 4 == 0, so a
// row of 3R floats is whole float4s): the x-neighbours of element k are k -/+ 3
// floats away and come from the previous / current / next float4 of the row.
__global__ void __launch_bounds__(SBLOCK) step_tv3v_kernel(TvArgs t, StepArgs a) {
  constexpr int C = 3;
  const int R = t.R, rowlen = R * C;
  unsigned bx, by, bz;
  xcd_block3(bx, by, bz);
  const int xi = (bx * blockDim.x + threadIdx.x) * 4, j = by, k = bz;
  const bool valid = xi < rowlen;
  const float npairs = 3.0f * (float)R * (float)R * (float)(R - 1);
  const float scale = t.lambda / (npairs * (float)C);
  float loss = 0.f;
  if (valid) {
    const int e = (k * R + j) * rowlen + xi;
    const int sy = rowlen, sz = R * rowlen;
    const float* __restrict__ F = t.F_in;
    const float4 f4v = ld4g(F, e);
    const float4 pv = xi >= 4 ? ld4g(F, e - 4) : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 nv = xi + 8 <= rowlen ? ld4g(F, e + 4) : make_float4(0.f, 0.f, 0.f, 0.f);
    const float f[4] = {f4v.x, f4v.y, f4v.z, f4v.w};
    const float xm[4] = {pv.y, pv.z, pv.w, f4v.x};  // element q - 3
    const float xp[4] = {f4v.w, nv.x, nv.y, nv.z};  // element q + 3
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = (xi + q) / C;
      if (i > 0) acc[q] += f[q] - xm[q];
      if (i < R - 1) { const float d = xp[q] - f[q]; acc[q] -= d; loss += d * d; }
    }
    auto yz = [&](int off, bool back, bool fwd) {
      if (back) {
        const float4 b = ld4g(F, e - off);
        acc[0] += f[0] - b.x; acc[1] += f[1] - b.y; acc[2] += f[2] - b.z; acc[3] += f[3] - b.w;
      }
      if (fwd) {
        const float4 b = ld4g(F, e + off);
        const float d0 = b.x - f[0], d1 = b.y - f[1], d2 = b.z - f[2], d3 = b.w - f[3];
        acc[0] -= d0; acc[1] -= d1; acc[2] -= d2; acc[3] -= d3;
        loss += d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3;
      }
    };
    yz(sy, j > 0, j < R - 1);
    yz(sz, k > 0, k < R - 1);
    const float4 g = ld4s(t.g, e);
    float4 m = ld4s(t.m, e), v = ld4s(t.v, e);
    const float s2 = 2.0f * scale;
    float4 p;
    p.x = adam_update_f(f[0], g.x + s2 * acc[0], m.x, v.x, t.lr, a.beta1, a.beta2, a.eps, a.bc1, a.bc2);
    p.y = adam_update_f(f[1], g.y + s2 * acc[1], m.y, v.y, t.lr, a.beta1, a.beta2, a.eps, a.bc1, a.bc2);
    p.z = adam_update_f(f[2], g.z + s2 * acc[2], m.z, v.z, t.lr, a.beta1, a.beta2, a.eps, a.bc1, a.bc2);
    p.w = adam_update_f(f[3], g.w + s2 * acc[3], m.w, v.w, t.lr, a.beta1, a.beta2, a.eps, a.bc1, a.bc2);
    st4g(t.F_out, e, p);
    st4s(t.m, e, m);
    st4s(t.v, e, v);
    // the render gradient is sparse: only nonzero entries are cleared
    if (g.x != 0.f || g.y != 0.f || g.z != 0.f || g.w != 0.f)
      st4g(t.g, e, make_float4(0.f, 0.f, 0.f, 0.f));
    if (t.half_out) {
      h4 hv = {(_Float16)p.x, (_Float16)p.y, (_Float16)p.z, (_Float16)p.w};
      *reinterpret_cast<h4*>(t.half_out + e) = hv;
    }
  }
  if (t.loss_dst) block_add(loss * scale, t.loss_dst);
}

__global__ void __launch_bounds__(SBLOCK) step_mlp_kernel(StepArgs a) {
  const int e = blockIdx.x * SBLOCK + threadIdx.x;
  if (e < a.n_mlp) {
    float m = a.m_mlp[e], v = a.v_mlp[e];
    a.mlp[e] = adam_update_f(a.mlp[e], a.g_mlp[e], m, v, a.lr_mlp, a.beta1, a.beta2, a.eps, a.bc1,
                           a.bc2);
    a.m_mlp[e] = m;
    a.v_mlp[e] = v;
    a.g_mlp[e] = 0.f;
  }
}

__global__ void zero3_kernel(float* p) {
  if (threadIdx.x < 3) p[threadIdx.x] = 0.f;
}

// any channel count: one float per thread, runtime division
__global__ void __launch_bounds__(SBLOCK) step_tv_any_kernel(TvArgs t, int C, StepArgs a) {
  const int R = t.R, rowlen = R * C;
  unsigned bx, by, bz;
  xcd_block3(bx, by, bz);
  const int xi = bx * SBLOCK + threadIdx.x, j = by, k = bz;
  const bool valid = xi < rowlen;
  const float npairs = 3.0f * (float)R * (float)R * (float)(R - 1);
  const float scale = t.lambda / (npairs * (float)C);
  float loss = 0.f;
  if (valid) {
    const int i = xi / C;
    const int e = (k * R + j) * rowlen + xi;
    const int sy = rowlen, sz = R * rowlen;
    const float* __restrict__ F = t.F_in;
    const float f = F[e];
    float acc = 0.f;
    if (i > 0) acc += f - F[e - C];
    if (i < R - 1) { const float d = F[e + C] - f; acc -= d; loss += d * d; }
    if (j > 0) acc += f - F[e - sy];
    if (j < R - 1) { const float d = F[e + sy] - f; acc -= d; loss += d * d; }
    if (k > 0) acc += f - F[e - sz];
    if (k < R - 1) { const float d = F[e + sz] - f; acc -= d; loss += d * d; }
    const float g = t.g[e];
    float m = t.m[e], v = t.v[e];
    const float p = adam_update_f(f, g + 2.0f * scale * acc, m, v, t.lr, a.beta1, a.beta2,
                                a.eps, a.bc1, a.bc2);
    t.F_out[e] = p;
    t.m[e] = m;
    t.v[e] = v;
    if (g != 0.f) t.g[e] = 0.f;  // the render gradient is sparse
    if (t.half_out) t.half_out[e] = (_Float16)p;
  }
  if (t.loss_dst) block_add(loss * scale, t.loss_dst);
}

static void launch_tv(const TvArgs& t, int C, const StepArgs& a, hipStream_t s) {
  const unsigned R = (unsigned)t.R;
  const unsigned rowlen = R * (unsigned)C;
  if (C % 4 == 0 && (C == 4 || C == 16 || C == 36 || C == 64)) {
    const dim3 grid((rowlen / 4 + SBLOCK - 1) / SBLOCK, R, R);
    switch (C) {
      case 4: hipLaunchKernelGGL(step_tv4_kernel<4>, grid, dim3(SBLOCK), 0, s, t, a); break;
      case 16: hipLaunchKernelGGL(step_tv4_kernel<16>, grid, dim3(SBLOCK), 0, s, t, a); break;
      case 36: hipLaunchKernelGGL(step_tv4_kernel<36>, grid, dim3(SBLOCK), 0, s, t, a); break;
      default: hipLaunchKernelGGL(step_tv4_kernel<64>, grid, dim3(SBLOCK), 0, s, t, a); break;
    }
    return;
  }
  if (C == 3 && R % 4 == 0) {
    // a row of 3R/4 float4s per block when it fits (no idle lanes at R = 256)
    const unsigned n4 = rowlen / 4;
    const unsigned threads = min((unsigned)SBLOCK, (n4 + 63) / 64 * 64);
    const dim3 grid4((n4 + threads - 1) / threads, R, R);
    hipLaunchKernelGGL(step_tv3v_kernel, grid4, dim3(threads), 0, s, t, a);
    return;
  }
  const dim3 grid((rowlen + SBLOCK - 1) / SBLOCK, R, R);
  if (C == 3) hipLaunchKernelGGL(step_tv_kernel<3>, grid, dim3(SBLOCK), 0, s, t, a);
  else hipLaunchKernelGGL(step_tv_any_kernel, grid, dim3(SBLOCK), 0, s, t, C, a);
}

__global__ void zero2_kernel(float* p) {
  if (threadIdx.x < 2) p[threadIdx.x] = 0.f;
}

hipError_t launch_grid_step(const StepArgs& a, hipStream_t s) {
  if (a.losses) hipLaunchKernelGGL(zero3_kernel, dim3(1), dim3(64), 0, s, a.losses);
  hipError_t e;
  if (a.ext) {
    if (a.losses_ext) hipLaunchKernelGGL(zero2_kernel, dim3(1), dim3(64), 0, s, a.losses_ext);
    e = launch_step_sdf_reg(a, s);
  } else {
    e = launch_step_sdf(a, s);
  }
  if (e != hipSuccess) return e;
  TvArgs tf{a.R, a.lambda_tv_feat, a.lr_feat, a.feat_in, a.feat_out, a.g_feat, a.m_feat, a.v_feat,
            static_cast<_Float16*>(a.feat_half), a.losses ? a.losses + 1 : nullptr};
  launch_tv(tf, a.n_feat, a, s);
  TvArgs tp{a.P, a.lambda_tv_probe, a.lr_probe, a.probes_in, a.probes_out, a.g_probes, a.m_probes,
            a.v_probes, static_cast<_Float16*>(a.probes_half), a.losses ? a.losses + 2 : nullptr};
  launch_tv(tp, a.n_pc, a, s);
  if (a.n_mlp > 0)
    hipLaunchKernelGGL(step_mlp_kernel, dim3((unsigned)((a.n_mlp + SBLOCK - 1) / SBLOCK)),
                       dim3(SBLOCK), 0, s, a);
  return hipGetLastError();
}

}  // namespace psdf
