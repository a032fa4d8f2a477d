// Host-side launch interface between the C ABI (abi.cpp) and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psdf {

struct RenderArgs {
  int64_t B;
  const float* rays_o;
  const float* rays_d;
  // field
  int R, P;
  float h, inv_h, inv_hp;
  const void* sdf;
  const void* feat;
  const void* probes;
  const float* mlp;
  const float* bounds;  // brick bounds of sdf, nullable
  // options
  int N;
  float tau;
  float skip_thr;  // absolute threshold (skip_voxels * h); <= 0 disables
  int flags;
  // forward outputs
  float* rgb;
  float* aux;
  float* depth_wsum;
  // backward inputs / outputs
  const float* aux_in;
  const float* dL;
  float* g_sdf;
  float* g_feat;
  float* g_probes;
  float* g_mlp;
};

struct TraceArgs {
  int R, P;
  float h, inv_h, inv_hp;
  const void* sdf;
  const void* feat;
  const void* probes;
  const float* mlp;
  float eps;
  int max_steps;
  int flags;
  int V, W, H;
  const float* cams;
  float* out;
};

struct StepArgs {
  int R, P, n_feat, n_pc, n_mlp;
  float h;
  float lr_sdf, lr_feat, lr_probe, lr_mlp;
  float beta1, beta2, eps;
  float bc1, bc2;  // 1 - beta^step
  float lambda_eik, lambda_tv_feat, lambda_tv_probe;
  const float* sdf_in;
  float* sdf_out;
  const float* feat_in;
  float* feat_out;
  const float* probes_in;
  float* probes_out;
  float* mlp;
  float* g_sdf;
  float* g_feat;
  float* g_probes;
  float* g_mlp;
  float* m_sdf;
  float* v_sdf;
  float* m_feat;
  float* v_feat;
  float* m_probes;
  float* v_probes;
  float* m_mlp;
  float* v_mlp;
  void* sdf_half;
  void* feat_half;
  void* probes_half;
  float* losses;
  float* sdf_bounds;  // brick bounds of the new sdf (of sdf_half when set), nullable
};

// dtype codes as in the public header
hipError_t launch_render_forward(const RenderArgs& a, int sdf_dt, int feat_dt, int mlp_dt,
                                 int n_sh, hipStream_t s);
hipError_t launch_render_backward(const RenderArgs& a, int sdf_dt, int feat_dt, int mlp_dt,
                                  int n_sh, hipStream_t s);
hipError_t launch_sphere_trace(const TraceArgs& a, int sdf_dt, int feat_dt, int mlp_dt, int n_sh,
                               hipStream_t s);
hipError_t launch_l1_loss(int64_t B, const float* rgb, const float* target, float* dL,
                          float* loss, hipStream_t s);
hipError_t launch_grid_step(const StepArgs& a, hipStream_t s);
hipError_t launch_sdf_bounds(const void* sdf, int R, int sdf_dt, float* bounds, hipStream_t s);

}  // namespace psdf
