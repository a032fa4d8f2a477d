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
  const int* todo;  // backward: nonzero entries select the 64-ray waves to run; nullptr = all
  // sparse tiles with tri-plane features (paper-model kernels): feat holds the planes
  const int* tile_index;  // [T^3] slot or -1; nullptr = dense features
  int tile_T;
};

// One shaded sample of the entry-parallel backward (160 bytes).
struct BwdEntry {
  double x[3];    // sample position
  float v[3];     // view direction (-unit ray direction)
  float w, T;     // compositing weight T_i alpha_i and transmittance T_i
  float s0, s1;   // s_i, s_{i+1}
  int ray;        // ray index
  int key;        // (sample index << 6) | lane of the ray in its wave
  int lw;         // the ray's 64-ray wave; -1: a slot that holds no sample
  int prev;       // first slot of the previous chunk of the same wave, -1 if none
  float C[3];     // colour of the sample
  // recorded by a forward that writes a tape
  float z[10];    // MLP inputs [F_s, F_a, c, c^2, c^4]
  float nrm[3];   // unit FD normal
  float gn;       // |FD gradient|
  // written by the per-ray walk of a taped backward
  float gdl;      // dL/d dl_i
  float gdl_prev; // dL/d dl_{i-1} when sample i-1 of the ray is an entry, else 0
  int pkey;       // key of the probe cell of x (the binning order of the backward)
  float nx_off[3];// x_{i+1} - x_i when sample i+1 of the ray is not an entry (the
                  // opacity gradient at s_{i+1} goes with this sample), else 0
};

// Gradient record of one shaded sample for the probe grid, placed in probe-cell order.
struct ProbeRec {
  int cell;       // probe cell (flat index of its lower corner node)
  float f[3];     // trilinear fractions in the cell
  float v[3];     // view direction (the SH argument)
  float dfa[4];   // dL/dF_a
  float pad;
};

// SDF and feature cotangents of one shaded sample, in probe-cell order (taped
// schedule): written by the shading pass, scattered by the box pass.
struct ScatRec {
  double x[3];    // sample position
  float dg[3];    // dL/d(FD gradient of the SDF at x) through the normal
  float a0;       // dL/ds_i through the opacities of samples i and i-1
  float df[3];    // dL/d(spatial features at x)
  int valid;      // 0: the slot holds no sample to scatter
  float off[3];   // x_{i+1} - x_i when the opacity gradient at s_{i+1} goes here
  float a1;       // dL/ds_{i+1} (trilinear at x + off), else 0
  float pad[2];
};

// most waves a shading pass launches (1024 blocks of 4 waves)
constexpr int kMlpWaves = 4096;

// Device workspace of the entry-parallel backward, carved from one caller buffer.
struct BwdWs {
  unsigned long long* counter;  // [1] slots handed out (may pass cap)
  int* overflow;       // [n_waves] 1: the wave did not fit and runs the fused kernel
  int* count;          // [n_waves] samples of the wave
  int* last;           // [n_waves] first slot of the wave's last chunk, -1 if none
  int* pcount;         // [P^3] samples per probe cell
  int* pcursor;        // [P^3] exclusive offsets, advanced by the placement
  int* psum;           // [nsum] scan partials
  int* plist;          // [P^3] occupied probe cells (first *pocc entries)
  int* pocc;           // [1]
  int* nbatch;         // [1] batches of the box pass
  int2* bdesc;         // [ndesc] (first sorted slot, samples): up to 64 samples of one
                       // block of 2x2x2 probe cells
  int* nsorted;        // [1] samples filed in probe-cell order (taped schedule)
  int* mbox;           // [6] brick box (min x, y, z, max x, y, z) of the bricks that may pass
                       // the skip rule (taped forward with brick bounds)
  float* mlp_part;     // [kMlpWaves][227] MLP gradient partials of the shading waves
  float* mlp_r;        // [227] the MLP with its weights rounded as the shading pass rounds them
  BwdEntry* entries;   // [cap]
  ProbeRec* precs;     // [cap] in probe-cell order
  ScatRec* srecs;      // [cap] in probe-cell order (taped schedule)
  int64_t cap, ndesc;
  int64_t n_waves;
  int64_t nkeys, nsum;  // probe-cell keys (bins) and scan blocks
  int probe_bins;      // 1: the probe gradient goes through the cell bins
  int bins;            // 1: samples are counted per probe cell (probe bins or taped order)
  int range;           // 1: the taped forward marches each wave over the samples in mbox
};

// bytes of a workspace with room for `cap` samples; carve() lays it out
int64_t bwd_ws_bytes(int64_t B, int P, int64_t cap);
int64_t bwd_ws_capacity(int64_t B, int P, int64_t bytes);
BwdWs bwd_ws_carve(void* base, int64_t B, int P, int64_t bytes);

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

// 5 taps of the Gaussian G of the smoothed SDF
struct SmoothTaps {
  float w[5];
};

// SDF regularisers of Sec. 3.3 on the smoothed SDF (step_reg.hip)
struct SdfRegArgs {
  int R;
  float h;
  int smooth;    // 1: the parameters are shat, rendering reads s = G(shat)
  int weighted;  // 1: (1 + 5 |s|)^-1 on the regularisers' gradients
  float lam_sdf, lam_eik, lam_nrm;  // lambda divided by the count of its sum
  SmoothTaps taps;
  const float* s_in;   // G(shat) as rendered (smooth)
  float* s_out;        // G(shat_out) (smooth)
  void* work;          // 8 R^3 floats
  // filled by the launcher
  const float* shat;
  const float* s;
  const float* g_s;
  float* nrm;
  float* dg;
  float* y;
  float* t;
  float* loss_eik;
  float* loss_sdf;
  float* loss_nrm;
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
  int ext;            // 1: the SDF goes through the Sec. 3.3 regularisers of `reg`
  SdfRegArgs reg;
  float* losses_ext;  // nullable [2]: L_sdf, L_normal
};

// real-time render: per-voxel shading and volume rendering (realtime.hip)
struct RealtimeArgs {
  int R, P, flags;
  const void* sdf;
  const void* feat;
  const void* probes;
  const float* mlp;
  const float* bounds;  // brick bounds of sdf, nullable
  const float* cam;     // [16] device: c2w (3x4), fx, fy, cx, cy
  const int* list;      // nodes to shade, *count of them (at most cap)
  const int* count;
  int64_t cap;
  void* colour;         // [R^3][4] FP32 or FP16 (r, g, b, 0)
  int N;
  float tau, skip_thr;
  int W, H;
  float* out;           // [H][W][3]
};

// optimiser step of the tri-plane features of sparse tiles
struct PlaneStepArgs {
  int64_t n_planes;  // 3 per allocated tile
  float scale;       // lambda / (slots 3 2 16 15 NF)
  float lr, beta1, beta2, eps, bc1, bc2;
  const float* in;
  float* out;
  float* g;
  float* m;
  float* v;
  _Float16* half;  // nullable
  float* loss;     // nullable [1]
};

// dtype codes as in the public header
hipError_t launch_render_forward(const RenderArgs& a, const BwdWs* tape, int sdf_dt, int feat_dt,
                                 int mlp_dt, int n_sh, hipStream_t s);
hipError_t launch_bwd_ws_clear(const BwdWs& ws, hipStream_t s);
hipError_t launch_render_backward(const RenderArgs& a, int sdf_dt, int feat_dt, int mlp_dt,
                                  int n_sh, hipStream_t s);
hipError_t launch_render_backward_split(const RenderArgs& a, const BwdWs& ws, bool from_tape,
                                        int sdf_dt, int feat_dt, int mlp_dt, int n_sh,
                                        hipStream_t s);
// the paper's colour model (model.h): forward (backward = false) or reverse mode
hipError_t launch_render_model(const RenderArgs& a, bool backward, int sdf_dt, int feat_dt,
                               int mlp_dt, int n_sh, int hidden, int layers, hipStream_t s);
hipError_t launch_sphere_trace(const TraceArgs& a, int sdf_dt, int feat_dt, int mlp_dt, int n_sh,
                               hipStream_t s);
hipError_t launch_l1_loss(int64_t B, const float* rgb, const float* target, float* dL,
                          float* loss, hipStream_t s);
hipError_t launch_grid_step(const StepArgs& a, hipStream_t s);
hipError_t launch_step_sdf(const StepArgs& a, hipStream_t s);
hipError_t launch_l2rel_loss(int64_t B, const float* rgb, const float* target, float* dL,
                             float* loss, float lambda, float eps, float n_images, hipStream_t s);
hipError_t launch_step_sdf_reg(const StepArgs& a, hipStream_t s);
hipError_t launch_smooth(int R, const SmoothTaps& w, const float* in, float* out, _Float16* half,
                         bool transpose, hipStream_t s);
hipError_t launch_voxel_list(int R, int sdf_dt, const void* sdf, float band, int* list,
                             int64_t cap, int* count, hipStream_t s);
hipError_t launch_voxel_shade(const RealtimeArgs& a, int sdf_dt, int feat_dt, int mlp_dt, int n_sh,
                              int colour_dt, hipStream_t s);
hipError_t launch_volume_render(const RealtimeArgs& a, int sdf_dt, int colour_dt, hipStream_t s);
hipError_t launch_plane_step(const PlaneStepArgs& a, hipStream_t s);
hipError_t launch_sdf_bounds(const void* sdf, int R, int sdf_dt, float* bounds, hipStream_t s);

}  // namespace psdf
