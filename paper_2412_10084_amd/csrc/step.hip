// Fused optimiser step over the ProbeSDF parameters: regulariser gradients
// (eikonal on the SDF, squared-difference smoothness on the features and on
// the probe coefficients; Sec. 3.3, Eqs. eikonal_reg, smooth_features,
// smooth_probes) added to the accumulated render gradient, then Adam
// (Sec. 3.4; moments as in the supplementary scheduling section).
//
// Each grid is one streaming pass: a thread owns one parameter, gathers the
// regulariser gradient of that parameter from its stencil (so no scatter and no
// atomics), applies Adam, writes the new value to a separate output buffer
// (neighbours still read the old one), writes the moments back, zeroes the
// gradient and optionally writes an FP16 copy.
#include "device.h"
#include "kernels.h"

namespace psdf {

constexpr int SBLOCK = 256;

__device__ __forceinline__ float adam_update(float p, float G, float& m, float& v, float lr, float b1,
                                             float b2, float eps, float bc1, float bc2) {
  m = b1 * m + (1.0f - b1) * G;
  v = b2 * v + (1.0f - b2) * G * G;
  const float mh = m / bc1;
  const float vh = v / bc2;
  return p - lr * mh / (sqrtf(vh) + eps);
}

__device__ __forceinline__ void block_add(float val, float* dst) {
  __shared__ float part[SBLOCK / 64];
  val = wave_sum(val);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = val;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int w = 0; w < SBLOCK / 64; ++w) s += part[w];
    if (s != 0.f) atomic_add_f32(dst, s);
  }
}

// central-difference gradient of node (i,j,k); valid only for interior nodes
__device__ __forceinline__ void cd_grad(const float* __restrict__ s, int R, int n, float inv2h,
                                        float g[3]) {
  const int RR = R * R;
  g[0] = (s[n + 1] - s[n - 1]) * inv2h;
  g[1] = (s[n + R] - s[n - R]) * inv2h;
  g[2] = (s[n + RR] - s[n - RR]) * inv2h;
}

// dL_eik/dg at node (i,j,k) times 1/(coef): 2(|g|-1)/|g| g, zero off the interior
__device__ __forceinline__ float eik_q(const float* __restrict__ s, int R, int i, int j, int k,
                                       float inv2h, int axis) {
  if (i < 1 || j < 1 || k < 1 || i > R - 2 || j > R - 2 || k > R - 2) return 0.f;
  float g[3];
  cd_grad(s, R, (k * R + j) * R + i, inv2h, g);
  const float gn = sqrtf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  if (!(gn > 0.f)) return 0.f;
  return 2.0f * (gn - 1.0f) / gn * g[axis];
}

__global__ void __launch_bounds__(SBLOCK) step_sdf_kernel(StepArgs a) {
  const int R = a.R;
  const int64_t n_nodes = (int64_t)R * R * R;
  const int64_t n64 = (int64_t)blockIdx.x * SBLOCK + threadIdx.x;
  const bool valid = n64 < n_nodes;
  const int n = valid ? (int)n64 : 0;
  const int i = n % R, j = (n / R) % R, k = n / (R * R);
  const float inv2h = 0.5f / a.h;
  const float M = (float)(R - 2) * (float)(R - 2) * (float)(R - 2);
  const float coef = a.lambda_eik / M;
  float loss = 0.f;
  if (valid) {
    const float* __restrict__ s = a.sdf_in;
    float G = a.g_sdf[n];
    if (a.lambda_eik != 0.f && R >= 3) {
      float ge = eik_q(s, R, i - 1, j, k, inv2h, 0) - eik_q(s, R, i + 1, j, k, inv2h, 0) +
                 eik_q(s, R, i, j - 1, k, inv2h, 1) - eik_q(s, R, i, j + 1, k, inv2h, 1) +
                 eik_q(s, R, i, j, k - 1, inv2h, 2) - eik_q(s, R, i, j, k + 1, inv2h, 2);
      G += coef * ge * inv2h;
      if (i >= 1 && j >= 1 && k >= 1 && i <= R - 2 && j <= R - 2 && k <= R - 2) {
        float g[3];
        cd_grad(s, R, n, inv2h, g);
        const float e = sqrtf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) - 1.0f;
        loss = e * e;
      }
    }
    float m = a.m_sdf[n], v = a.v_sdf[n];
    const float p = adam_update(s[n], G, m, v, a.lr_sdf, a.beta1, a.beta2, a.eps, a.bc1, a.bc2);
    a.sdf_out[n] = p;
    a.m_sdf[n] = m;
    a.v_sdf[n] = v;
    a.g_sdf[n] = 0.f;
    if (a.sdf_half) static_cast<_Float16*>(a.sdf_half)[n] = (_Float16)p;
  }
  if (a.losses) block_add(loss * coef, a.losses + 0);
}

// smoothness + Adam on a grid with C channels per node
__global__ void __launch_bounds__(SBLOCK) step_tv_kernel(int R, int C, float lambda, float lr,
                                                         const float* __restrict__ F_in,
                                                         float* F_out, float* g, float* m_, float* v_,
                                                         _Float16* half_out, float* loss_dst,
                                                         StepArgs a) {
  const int64_t n_el = (int64_t)R * R * R * C;
  const int64_t e64 = (int64_t)blockIdx.x * SBLOCK + threadIdx.x;
  const bool valid = e64 < n_el;
  const int e = valid ? (int)e64 : 0;
  const int node = e / C;
  const int i = node % R, j = (node / R) % R, k = node / (R * R);
  const float npairs = 3.0f * (float)R * (float)R * (float)(R - 1);
  const float scale = lambda / (npairs * (float)C);
  float loss = 0.f;
  if (valid) {
    const float f = F_in[e];
    float acc = 0.f;
    const int sx = C, sy = R * C, sz = R * R * C;
    if (i > 0) acc += f - F_in[e - sx];
    if (i < R - 1) { const float d = F_in[e + sx] - f; acc -= d; loss += d * d; }
    if (j > 0) acc += f - F_in[e - sy];
    if (j < R - 1) { const float d = F_in[e + sy] - f; acc -= d; loss += d * d; }
    if (k > 0) acc += f - F_in[e - sz];
    if (k < R - 1) { const float d = F_in[e + sz] - f; acc -= d; loss += d * d; }
    const float G = g[e] + 2.0f * scale * acc;
    float m = m_[e], v = v_[e];
    const float p = adam_update(f, G, m, v, lr, a.beta1, a.beta2, a.eps, a.bc1, a.bc2);
    F_out[e] = p;
    m_[e] = m;
    v_[e] = v;
    g[e] = 0.f;
    if (half_out) half_out[e] = (_Float16)p;
  }
  if (loss_dst) block_add(loss * scale, loss_dst);
}

__global__ void __launch_bounds__(SBLOCK) step_mlp_kernel(StepArgs a) {
  const int e = blockIdx.x * SBLOCK + threadIdx.x;
  if (e < a.n_mlp) {
    float m = a.m_mlp[e], v = a.v_mlp[e];
    a.mlp[e] = adam_update(a.mlp[e], a.g_mlp[e], m, v, a.lr_mlp, a.beta1, a.beta2, a.eps, a.bc1,
                           a.bc2);
    a.m_mlp[e] = m;
    a.v_mlp[e] = v;
    a.g_mlp[e] = 0.f;
  }
}

__global__ void zero3_kernel(float* p) {
  if (threadIdx.x < 3) p[threadIdx.x] = 0.f;
}

hipError_t launch_grid_step(const StepArgs& a, hipStream_t s) {
  if (a.losses) hipLaunchKernelGGL(zero3_kernel, dim3(1), dim3(64), 0, s, a.losses);
  const int64_t ns = (int64_t)a.R * a.R * a.R;
  hipLaunchKernelGGL(step_sdf_kernel, dim3((unsigned)((ns + SBLOCK - 1) / SBLOCK)), dim3(SBLOCK), 0,
                     s, a);
  const int64_t nf = ns * a.n_feat;
  hipLaunchKernelGGL(step_tv_kernel, dim3((unsigned)((nf + SBLOCK - 1) / SBLOCK)), dim3(SBLOCK), 0,
                     s, a.R, a.n_feat, a.lambda_tv_feat, a.lr_feat, a.feat_in, a.feat_out, a.g_feat,
                     a.m_feat, a.v_feat, static_cast<_Float16*>(a.feat_half),
                     a.losses ? a.losses + 1 : nullptr, a);
  const int64_t np = (int64_t)a.P * a.P * a.P * a.n_pc;
  hipLaunchKernelGGL(step_tv_kernel, dim3((unsigned)((np + SBLOCK - 1) / SBLOCK)), dim3(SBLOCK), 0,
                     s, a.P, a.n_pc, a.lambda_tv_probe, a.lr_probe, a.probes_in, a.probes_out,
                     a.g_probes, a.m_probes, a.v_probes, static_cast<_Float16*>(a.probes_half),
                     a.losses ? a.losses + 2 : nullptr, a);
  hipLaunchKernelGGL(step_mlp_kernel, dim3((unsigned)((a.n_mlp + SBLOCK - 1) / SBLOCK)),
                     dim3(SBLOCK), 0, s, a);
  return hipGetLastError();
}

}  // namespace psdf
