/*
 * probesdf.h -- C ABI of the MI355X (gfx950) ProbeSDF render-step library.
 *
 * Method: Toussaint, Thomas, Franco, "ProbeSDF: Light Field Probes For Neural
 * Surface Reconstruction", CVPR 2025 (arXiv 2412.10084).  The library computes
 * the fused per-ray render step of that method on an explicit SDF voxel grid:
 *   - a dense SDF grid s and spatial features F_s (Sec. 3.1), sampled by
 *     trilinear interpolation;
 *   - a lower-resolution grid of light-field probes, each holding l^2
 *     spherical-harmonic coefficient vectors b_j (Sec. 3.2, Eqs.
 *     spherical_harmonics, sh_eval1, sh_eval2), interpolated and evaluated in the
 *     view direction;
 *   - incidence inputs from n.v with n the normalised SDF gradient
 *     (Sec. 3.1, Eq. newparametrization);
 *   - a tiny MLP that decodes colour (Sec. 4);
 *   - NeuS SDF-to-opacity compositing along the ray (Sec. 3.3, Eq. neus).
 *
 * Common conventions
 *   Grids are align-corners over the cube [-1,1]^3: R nodes per axis, node
 *   (i,j,k) at (-1 + i h, -1 + j h, -1 + k h), h = 2/(R-1); stored x fastest,
 *   flat index (k*R + j)*R + i.  Trilinear interpolation takes, per axis,
 *   u = (x+1)/h, cell k0 = clamp(floor(u), 0, R-2), weight f = u - k0; sample
 *   positions are clamped to the cube.
 *     sdf     [R][R][R]                      FP32 or FP16
 *     feat    [R][R][R][n_feat]              FP32 or FP16   (F_s)
 *     probes  [P][P][P][sh_coeffs][n_ang]    FP32 or FP16   (b_ij)
 *     mlp     W1[hidden][n_in] row-major, b1[hidden], W2[3][hidden], b2[3],
 *             FP32, n_in = n_feat + n_ang + 3; MLP input z = [F_s, F_a, c, c^2, c^4]
 *             (the workload colour model; the paper's own is described at
 *             psdf_field)
 *             with c = n.v (v = -ray direction), hidden ReLU, sigmoid output.
 *   Rays: origins and directions [B][3] FP32 (directions need not be unit).
 *   Per ray: interval [t_n, t_f] = ray / cube intersection (t >= 0); N samples
 *   t_i = t_n + (i + 1/2)(t_f - t_n)/N; alpha_i from s_i and s_{i+1}; the last
 *   sample has alpha 0.  A sample is active iff |s_i| <= skip_voxels * h
 *   (skip_voxels <= 0: every sample).  Rays that miss the cube render 0.
 *
 * Memory and streams
 *   Every pointer argument except the descriptor structs themselves is DEVICE
 *   memory owned by the caller; descriptor structs are host memory read during
 *   the call only.  Calls enqueue work on `stream` (a hipStream_t; NULL = the
 *   null stream) and return without synchronising.  The library allocates no
 *   device memory and keeps no per-call state; its one piece of device memory,
 *   the static scratch of psdf_render_backward_noalloc, is reset by each call of
 *   that entry point before use.  Gradient buffers are
 *   accumulated into (+=); the caller zeroes them, or psdf_grid_step does.
 *
 * Errors
 *   Every entry point returns PSDF_OK (0) or a negative code; arguments are
 *   validated on the host before anything is enqueued, and on error nothing
 *   is enqueued.  psdf_last_error() returns a thread-local message for the last
 *   failing call on this thread.  B = 0 (or an empty image) is a no-op that
 *   returns PSDF_OK.  NaN/Inf inputs are propagated, never trapped; every
 *   memory access is clamped into the grids, so no input can make a kernel
 *   read or write out of bounds.  Faults inside a kernel surface at the
 *   caller's next synchronisation of the stream.
 */
#ifndef PROBESDF_H
#define PROBESDF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PSDF_ABI_VERSION 5

#define PSDF_OK 0
#define PSDF_EINVAL (-1)       /* null pointer, bad size or shape, aliasing */
#define PSDF_EALIGN (-2)       /* a pointer is not aligned as documented */
#define PSDF_EUNSUPPORTED (-3) /* a shape or dtype combination not compiled in */
#define PSDF_EHIP (-4)         /* the HIP runtime reported an error */

typedef enum { PSDF_F32 = 0, PSDF_F16 = 1, PSDF_BF16 = 2 } psdf_dtype;

/* render flags: ablations of the colour model (Sec. 5 "Ablations") and the
 * paper's own form of its inputs */
#define PSDF_FLAG_NO_FS 1  /* F_s := 0 */
#define PSDF_FLAG_NO_FA 2  /* F_a := 0 */
#define PSDF_FLAG_NV_ONE 4 /* n.v := 1 in the incidence inputs (no incidence dependence) */
/* SH evaluated at the reflection of v about the normal, r = 2 (n.v) n - v
 * (Sec. 3.1 Eq. newparametrization, Sec. 3.2), instead of at v */
#define PSDF_FLAG_SH_REFLECT 8
/* incidence inputs (1 - n.v)^0 .. (1 - n.v)^5 (Eq. newparametrization) instead of
 * (n.v, (n.v)^2, (n.v)^4); the MLP then has n_in = n_feat + n_ang + 6 inputs */
#define PSDF_FLAG_FRESNEL_PAPER 16

/* Most samples per ray of the paper colour model's kernels, which hold a ray's
 * shaded samples in LDS. */
#define PSDF_MODEL_MAX_SAMPLES 513

/*
 * The scene parameters (Sec. 3.4: raw SDF values, spatial features, probe
 * coefficients and MLP weights).  Supported shapes: n_feat = 3, n_ang = 4,
 * sh_coeffs in {1, 4, 9, 16}, 2 <= R, P <= 1024 with R^3 * n_feat and
 * P^3 * sh_coeffs * n_ang below 2^31, and an MLP of (mlp_layers, mlp_hidden) =
 * (1, 16) or (2, 32) hidden layers (Sec. 4 uses two of 32).
 *
 * Colour models.  The workload model -- one hidden layer of 16, SH at v, inputs
 * (c, c^2, c^4) -- runs on the kernels described at each entry point.  The
 * paper's own model -- any of PSDF_FLAG_SH_REFLECT, PSDF_FLAG_FRESNEL_PAPER or
 * two hidden layers of 32 -- runs on kernels that take one ray per wave and one
 * sample per lane, with these limits (else PSDF_EUNSUPPORTED): FP32 sdf;
 * FP32 features with the FP32 MLP, or FP16 features with the FP16 / BF16 MLP;
 * sh_coeffs 9 or 16; n_samples <= PSDF_MODEL_MAX_SAMPLES; no sphere tracing.
 * Its forward records no tape, and its backward re-marches (a workspace or
 * PSDF_BWD_FROM_TAPE is accepted and left unused).
 * MLP packing for n_in inputs (n_in = n_feat + n_ang + 3, or + 6 with
 * PSDF_FLAG_FRESNEL_PAPER), hidden width H, L hidden layers: W_0[H][n_in],
 * b_0[H], (W_1[H][H], b_1[H] if L = 2), W_o[3][H], b_o[3]; psdf_grads.mlp has
 * the same size.
 * Dtypes: sdf_dtype F32 | F16, feat_dtype F32 | F16 (features and probes),
 * mlp_dtype F32 | F16 | BF16 (the precision the MLP computes in; weights are
 * always passed FP32 and rounded to nearest-even on use).
 * Alignment: sdf, feat 4 bytes (2 for FP16); probes 16 bytes (8 for FP16);
 * mlp 4 bytes; sdf_bounds 8 bytes.
 *
 * sdf_bounds (nullable) enables empty-space skipping of the march: FP32
 * [nb][nb][nb][2] with nb = PSDF_BRICKS(R), x fastest; entry (bx, by, bz)
 * holds the min and max of the sdf nodes [8b, min(8b + 8, R - 1)] on each
 * axis, i.e. of every node that the cells [8b, 8b + 7] interpolate.  A sample
 * whose brick has min > thr or max < -thr (thr = skip_voxels * h, widened by a
 * 1e-6 relative margin that covers FP32 interpolation rounding) cannot pass the
 * skip rule, so its corners are not read.  Results are identical with and
 * without bounds.  They must describe exactly the sdf array they travel with
 * (as read, i.e. after FP16 rounding): write them with psdf_sdf_bounds or with
 * psdf_grid_step's sdf_bounds_out; stale bounds give wrong images.
 */
#define PSDF_BRICK 8
#define PSDF_BRICKS(R) (((R) - 2) / PSDF_BRICK + 1)

typedef struct psdf_field {
  uint32_t struct_size; /* sizeof(psdf_field) */
  int32_t R;
  int32_t P;
  int32_t n_feat;
  int32_t sh_coeffs;
  int32_t n_ang;
  int32_t mlp_hidden;
  int32_t sdf_dtype;
  int32_t feat_dtype;
  int32_t mlp_dtype;
  const void* sdf;
  const void* feat;
  const void* probes;
  const float* mlp;
  const float* sdf_bounds; /* nullable, see above */
  int32_t mlp_layers;      /* hidden layers of the MLP: 1 (mlp_hidden 16) or 2 (mlp_hidden 32) */
  /* Sparse tiles (Sec. 3.1, Sec. 4).  tile_T > 0: the domain is T^3 tiles of 16^3
   * cells (R = 16 T + 1); tile_index [T][T][T] (int32, device) gives each tile's
   * slot or -1 for an empty tile; samples in empty tiles are inactive; the spatial
   * features are tri-planes and `feat` points to [n_tiles][3][16][16][n_feat]:
   * planes F_x over (y, z), F_y over (x, z), F_z over (x, y), rows [v][u], texels at
   * the tile's cell centres, bilinear and clamped inside the tile, and
   * F_s = F_x * F_y * F_z channel by channel.  The SDF stays dense, the probes sit
   * at the tile corners (P = T + 1 is the paper's layout).  Tiled fields run on the
   * paper colour model's kernels (its limits apply); the feature gradient has the
   * plane layout.  tile_T = 0: dense features. */
  int32_t tile_T;
  const int32_t* tile_index;
  int64_t n_tiles;
} psdf_field;

typedef struct psdf_render_opts {
  uint32_t struct_size; /* sizeof(psdf_render_opts) */
  int32_t n_samples;    /* N, 2 <= N <= 4096 */
  float tau;            /* NeuS sharpness of Phi_tau (Eq. neus), > 0 */
  float skip_voxels;    /* skip rule threshold in voxels; <= 0 disables */
  int32_t flags;        /* PSDF_FLAG_* */
} psdf_render_opts;

/* FP32 gradient accumulators, same layouts as the parameters.  A NULL member
 * skips that group (its scatter is not performed). */
typedef struct psdf_grads {
  float* sdf;
  float* feat;
  float* probes;
  float* mlp;
} psdf_grads;

/*
 * psdf_render_forward -- colour of B rays (Sec. 3.3): c = sum_i T_i alpha_i C_i,
 * T_i = prod_{j<i} (1 - alpha_j), alpha_i = max((Phi(s_i) - Phi(s_{i+1}))/Phi(s_i), 0),
 * C_i = MLP(F_s(x_i), F_a(x_i, v), c, c^2, c^4).
 *   rgb         [B][3] out
 *   aux         [B][4] out, nullable: (rgb, log T_final); required by the backward
 *   depth_wsum  [B][2] out, nullable: (sum_i w_i (t_i + dt/2), sum_i w_i), w_i = T_i alpha_i
 *   tape, tape_bytes: nullable device buffer laid out as a backward workspace
 *     (see psdf_render_backward); when given, the forward also records every
 *     shaded sample there (position, weights, s_i, s_{i+1}, colour, MLP inputs,
 *     normal, about 160 bytes each) for a backward called with
 *     PSDF_BWD_FROM_TAPE.  Waves of 64 rays whose samples do not fit are
 *     flagged and re-marched by that backward.  The outputs do not depend on it.
 */
int psdf_render_forward(const psdf_field* field, const psdf_render_opts* opts, int64_t B,
                        const float* rays_o, const float* rays_d, float* rgb, float* aux,
                        float* depth_wsum, void* tape, int64_t tape_bytes, void* stream);

/*
 * psdf_render_backward -- reverse mode of psdf_render_forward for the same
 * field, opts and rays: given dL/drgb [B][3] and the forward's aux [B][4], ADDS
 * dL/d(sdf, feat, probes, mlp) into `grads` (Sec. 3.3: the SDF and appearance
 * are optimised by back-propagating the colour loss through the rendering
 * equation).  Without PSDF_BWD_FROM_TAPE the march is recomputed; with it the
 * backward reads the samples the forward recorded in the workspace.
 * Gradients are summed in FP32: global FP32 atomics, and in the taped
 * schedule's SDF / feature box pass LDS boxes of 32-bit fixed point per batch of
 * up to 64 samples (scale 2^30 / (64 B), B the batch's largest contribution of
 * one sample to one node, so each add is within B / 2^25 of its FP32 value; a
 * batch with a non-finite or huge B, or with samples at the grid boundary, adds
 * in FP32).  The summation order (and the last bits) varies from run to run.
 * The single-kernel schedule forms the colour remaining after sample i as the
 * forward's rgb minus the colours before i, clamped to its exact range [0, T_i].
 * Gradients are defined with respect to the values the forward reads (FP16
 * storage: the rounded values).
 *   workspace, workspace_bytes: optional device buffer (256-byte aligned, at
 *     least psdf_backward_workspace_bytes(B, P, 0) bytes) for the
 *     entry-parallel schedule: a march pass writes the shaded samples there
 *     (and counts them per probe cell), a shading pass processes them 64 per
 *     wave whatever ray they come from and files their probe gradients by
 *     probe cell, a pass per probe cell sums its records and adds them to the
 *     cell's 8 corner nodes, and a per-ray pass adds the opacity gradient.
 *     Waves of 64 rays whose samples do not fit are run by the fused schedule
 *     afterwards, so any size gives the same gradients.  NULL: the fused
 *     single-kernel schedule for every wave.  Calls that share a workspace
 *     must not overlap.
 *   flags: PSDF_BWD_FROM_TAPE -- the workspace holds the tape that
 *     psdf_render_forward recorded for the same field, opts and rays (the
 *     reserve-space contract: nothing may touch it in between).  The march and
 *     the re-read of the shading inputs are skipped, the per-ray walk runs
 *     first on the recorded colours, and the opacity gradient at s_i joins the
 *     sample's SDF patch.  Waves the forward flagged as not fitting are
 *     re-marched by the fused schedule.  0: the workspace is scratch.
 */
#define PSDF_BWD_FROM_TAPE 1

int psdf_render_backward(const psdf_field* field, const psdf_render_opts* opts, int64_t B,
                         const float* rays_o, const float* rays_d, const float* aux,
                         const float* dL_drgb, const psdf_grads* grads, void* workspace,
                         int64_t workspace_bytes, int32_t flags, void* stream);

/*
 * psdf_render_backward_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): psdf_render_backward with flags = 0 and, as its workspace, a
 * static device array of the library of PSDF_NOALLOC_SCRATCH_BYTES (128 MiB),
 * so the call allocates nothing (no hipMalloc, no hipFree, no allocating library
 * routine).  Same arguments, results and accumulation (+=) as
 * psdf_render_backward; waves of 64 rays whose shaded samples do not fit the
 * scratch (about 360 000 samples at P = 128 beside the fixed part) run the
 * fused schedule, so any batch gives the same gradients.
 *   Limit: the fixed part of the workspace (12 bytes per 64 rays, about 12
 *   bytes per probe cell of the P^3 grid, 3.6 MiB of MLP partials) must fit
 *   the scratch; larger B or P return PSDF_EINVAL with a message.
 *   Each GPU holds its own copy of the scratch from the first call made with
 *   that device current until the process ends; the call uses the copy of the
 *   current device.  Every call on one GPU shares that copy, and each call
 *   resets the counters it relies on before use: calls that overlap on one
 *   GPU (other streams, other host threads) race and give wrong gradients.
 */
#define PSDF_NOALLOC_SCRATCH_BYTES 134217728

int psdf_render_backward_noalloc(const psdf_field* field, const psdf_render_opts* opts, int64_t B,
                                 const float* rays_o, const float* rays_d, const float* aux,
                                 const float* dL_drgb, const psdf_grads* grads, void* stream);

/* Bytes of a backward workspace (or forward tape) for B rays and a P^3 probe
 * grid with room for `max_samples` shaded samples (288 bytes each, plus 12
 * bytes per 64 rays, about 12 bytes per probe cell and 3.6 MiB for the MLP
 * gradient partials of the shading waves); -1 if an argument is out of range. */
int64_t psdf_backward_workspace_bytes(int64_t B, int32_t P, int64_t max_samples);

/*
 * psdf_l1_loss -- photometric loss.  The paper uses a relatively weighted L2
 * (Eq. photo_loss); this is its L1 form L = mean over B x 3 of |rgb - target|.
 *   dL_drgb [B][3] out = sign(rgb - target) / (3B), sign(0) = 0
 *   loss    [1] out, nullable: L (overwritten)
 */
int psdf_l1_loss(int64_t B, const float* rgb, const float* target, float* dL_drgb, float* loss,
                 void* stream);

/*
 * psdf_grid_step -- one optimiser step over all parameters (Sec. 3.4: Adam over
 * the raw SDF, features, probes and MLP; moments beta1, beta2 as in the
 * supplementary scheduling section).  For each group the total gradient is the
 * accumulated render gradient plus the regulariser gradient:
 *   eikonal (Eq. eikonal_reg):  lambda_eik / (R-2)^3 * sum over interior nodes of
 *       (|grad s| - 1)^2, grad s by central differences (s[n+e]-s[n-e])/2h;
 *   feature smoothness (Eq. smooth_features) and probe smoothness
 *       (Eq. smooth_probes): lambda / (3 R^2 (R-1) C) * sum over axis-adjacent
 *       node pairs and the C channels of squared differences;
 * then bias-corrected Adam (Kingma & Ba, Algorithm 1) with `step` >= 1.
 * Grids are updated OUT OF PLACE (the stencils read neighbours): *_in and
 * *_out must not overlap; the MLP is updated in place.  Gradients are zeroed.
 * Alignment: the grid buffers (params, gradients, moments) 16 bytes, FP16
 * copies 8 bytes, MLP buffers 4 bytes.
 * Optional FP16 render copies (round to nearest even) of the new sdf, feat
 * and probes are written when their pointers are non-NULL.  `losses` [3]
 * (nullable, device) receives (L_eik, L_feat, L_probe) of the input
 * parameters.  `sdf_bounds_out` (nullable, [PSDF_BRICKS(R)^3][2], 8-byte
 * aligned) receives the brick bounds of the new sdf as the renderer will read
 * it: of the FP16 copy when sdf_half_out is set, else of sdf_out.
 * Sec. 3.3's remaining regularisers: with any of sdf_reg_flags, lambda_sdf or
 * lambda_normal set, the SDF part of the step instead
 *   - with PSDF_STEP_SMOOTH, takes sdf_in / sdf_out as the raw values shat, g_sdf
 *     as the render gradient with respect to s = G(shat) (s_in), and writes
 *     s_out = G(sdf_out) (its FP16 copy in sdf_half_out, its bounds in
 *     sdf_bounds_out);
 *   - evaluates on s: L_sdf = lambda_sdf / R^3 * sum (s - shat)^2, the eikonal
 *     term above, and L_normal = lambda_normal / (3 (R-2)^2 (R-3)) * sum over
 *     axis-adjacent pairs of interior nodes |n_a - n_b|^2 (n = g / |g|, g the
 *     central differences), with PSDF_STEP_REG_WEIGHT weighting their gradient at
 *     node m by 1 / (1 + 5 |s_m|);
 *   - takes the gradient back to shat through G^T, then Adam as above.
 * It needs `work` (psdf_step_work_bytes(R) bytes); losses[0] is L_Eik of s and
 * losses_ext receives (L_sdf, L_normal).
 */
typedef struct psdf_step_args {
  uint32_t struct_size; /* sizeof(psdf_step_args) */
  int32_t R, P, n_feat, n_pc; /* n_pc = sh_coeffs * n_ang */
  int32_t n_mlp;
  int64_t step;
  float lr_sdf, lr_feat, lr_probe, lr_mlp;
  float beta1, beta2, eps;
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
  void* sdf_half_out;    /* nullable FP16 copies */
  void* feat_half_out;
  void* probes_half_out;
  float* losses;         /* nullable [3] */
  float* sdf_bounds_out; /* nullable */
  /* Sec. 3.3's smoothed SDF and remaining regularisers (all zero / NULL: unused; see
   * psdf_grid_step) */
  int32_t sdf_reg_flags; /* PSDF_STEP_SMOOTH | PSDF_STEP_REG_WEIGHT */
  float lambda_sdf;      /* L_sdf (Eq. smooth_sdf) */
  float lambda_normal;   /* L_normal (Eq. smmoth_normals) */
  float smooth_sigma;    /* width of the Gaussian, voxels (> 0 with PSDF_STEP_SMOOTH) */
  const float* s_in;     /* PSDF_STEP_SMOOTH: G(sdf_in), the field the renderer read */
  float* s_out;          /* PSDF_STEP_SMOOTH: receives G(sdf_out) */
  void* work;            /* psdf_step_work_bytes(R) bytes, 16-byte aligned */
  int64_t work_bytes;
  float* losses_ext;     /* nullable [2]: (L_sdf, L_normal) of the input parameters */
} psdf_step_args;

/* sdf_reg_flags */
#define PSDF_STEP_SMOOTH 1     /* the sdf parameters are raw values shat; rendering reads
                                  s = G(shat), G the 5^3 Gaussian of Sec. 3.3 */
#define PSDF_STEP_REG_WEIGHT 2 /* the SDF regularisers' gradient at node m is weighted
                                  by 1 / (1 + 5 |s_m|) (Sec. 3.3) */

/*
 * psdf_plane_step -- optimiser step of the tri-plane features of sparse tiles:
 * the smoothness of the factorised features (Eq. smooth_features), mean-
 * normalised, L = lambda / (n_tiles 3 2 16 15 n_feat) * sum over every plane, both
 * of its axes and channels of squared differences of neighbouring texels, plus the
 * accumulated render gradient g, then bias-corrected Adam (as psdf_grid_step);
 * out of place (in and out must not overlap); g is cleared.
 *   in, out, g, m, v [n_tiles][3][16][16][n_feat] FP32 (n_feat = 3), 16-byte aligned
 *   half_out nullable FP16 copy of out; loss nullable [1] (L of `in`)
 */
int psdf_plane_step(int64_t n_tiles, int32_t n_feat, const float* in, float* out, float* g,
                    float* m, float* v, int64_t step, float lr, float beta1, float beta2,
                    float eps, float lambda, void* half_out, float* loss, void* stream);

/* Bytes of the workspace of a grid step that uses the Sec. 3.3 regularisers:
 * 8 R^3 floats; -1 if R is out of range. */
int64_t psdf_step_work_bytes(int32_t R);

/*
 * psdf_smooth_sdf -- s = G(shat), the 5^3 Gaussian of Sec. 3.3 (Eq. smooth_sdf):
 * 5 taps per axis proportional to exp(-k^2 / (2 sigma^2)), k = -2..2, normalised,
 * nodes beyond the grid reading the edge node.  The field the renderer reads
 * when the SDF is trained as raw values (the grid step writes the next one).
 *   shat, s [R][R][R] FP32 (4-byte aligned, not overlapping); s_half nullable
 *   FP16 copy of s (2-byte aligned); 2 <= R <= 1024, sigma > 0.
 */
int psdf_smooth_sdf(int32_t R, float sigma, const float* shat, float* s, void* s_half,
                    void* stream);

/*
 * psdf_l2rel_loss -- the paper's photometric loss (Eq. photo_loss): L2 with the
 * per-pixel weight (max(c, c_gt) + eps)^-1 on its gradient, scaled by lambda and
 * divided by the number of images of the batch (supplementary "Scheduling"); the
 * weight is held constant and applies per channel:
 *   loss = lambda / n_images * sum (c - c_gt)^2 / (max(c, c_gt) + eps)   (nullable, overwritten)
 *   dL_drgb = 2 lambda / n_images * (c - c_gt) / (max(c, c_gt) + eps)
 * rgb, target, dL_drgb [B][3] FP32.  eps > 0, n_images > 0.
 */
int psdf_l2rel_loss(int64_t B, const float* rgb, const float* target, float* dL_drgb, float* loss,
                    float lambda, float eps, float n_images, void* stream);

int psdf_grid_step(const psdf_step_args* args, void* stream);

/*
 * psdf_sdf_bounds -- brick bounds of an sdf grid for psdf_field.sdf_bounds (an
 * acceleration structure for the skip rule of Sec. 3.3; not part of the model).
 *   sdf     [R][R][R] FP32 or FP16 (sdf_dtype), 2 <= R <= 1024
 *   bounds  [PSDF_BRICKS(R)^3][2] FP32 out, 8-byte aligned
 * NaN nodes are ignored (an all-NaN brick gets min = +inf, max = -inf, so its
 * samples are skipped, as the skip rule leaves a NaN sample inactive).
 */
int psdf_sdf_bounds(int32_t R, int32_t sdf_dtype, const void* sdf, float* bounds, void* stream);

/*
 * psdf_render_sphere_trace -- inference render of V pinhole views.  The paper
 * renders in real time by shading voxels and volume rendering them
 * (supplementary "Performance Analysis"); this entry point instead sphere-traces
 * the SDF (t <- t + s(x) from the cube entry until s < eps: hit, t > t_f: miss,
 * at most max_steps evaluations) and shades the hit point once with the same
 * colour model.  Misses render 0.
 *   cams  [V][16] device FP32: c2w (3x4 row-major; columns = camera x (right),
 *         y (down), z (forward) axes and the centre), fx, fy, cx, cy; pixel
 *         (px, py) looks along c2w[:, :3] . ((px+.5-cx)/fx, (py+.5-cy)/fy, 1)
 *   out   [V][H][W][3] FP32
 */
typedef struct psdf_trace_opts {
  uint32_t struct_size; /* sizeof(psdf_trace_opts) */
  float eps;            /* hit threshold, > 0 */
  int32_t max_steps;    /* >= 1 */
  int32_t flags;        /* PSDF_FLAG_* */
} psdf_trace_opts;

int psdf_render_sphere_trace(const psdf_field* field, const psdf_trace_opts* opts, int32_t V,
                             const float* cams, int32_t W, int32_t H, float* out, void* stream);

/*
 * Real-time render (supplementary "Performance Analysis": a shading pass assigns
 * a colour to every voxel, a volume-rendering pass samples the SDF and the colour
 * field along the rays).  Voxels are the grid nodes; only those near the surface
 * are shaded.
 *
 * psdf_voxel_list -- the nodes with |sdf| <= band (FP32 comparison), as flat
 * indices in list[0 .. *count) (order unspecified; at most `capacity` written,
 * *count may exceed it).  View-independent: build it once per SDF.
 *   sdf [R][R][R] FP32 or FP16 (sdf_dtype); list int32 [capacity]; count int32 [1]
 *
 * psdf_voxel_shade -- colour of each listed node seen from the camera centre
 * (c2w[:, 3] of cam): v = (c - x) / |c - x|, the colour model of the field (FD
 * normal, F_s, F_a(v), n.v, MLP, sigmoid) at the node.  Writes only the listed
 * nodes of colour [R^3][4] (r, g, b, 0): FP32 (colour_dtype PSDF_F32, 16-byte
 * aligned) or FP16 (PSDF_F16, 8-byte aligned); the caller zeroes it once, since
 * nodes outside the band keep their values.  The workload colour model only.
 *   cam [16] device FP32 (the layout of psdf_render_sphere_trace); list, count as
 *   written by psdf_voxel_list with the same capacity
 *
 * psdf_volume_render -- one view of W x H pinhole pixels (camera layout of
 * psdf_render_sphere_trace): per pixel ray, the samples, skip rule, brick skipping
 * (field->sdf_bounds) and NeuS weights of psdf_render_forward, with the colour of
 * sample i the trilinear interpolation of the colour grid at x_i.
 *   out [H][W][3] FP32
 */
int psdf_voxel_list(int32_t R, int32_t sdf_dtype, const void* sdf, float band, int32_t* list,
                    int64_t capacity, int32_t* count, void* stream);
int psdf_voxel_shade(const psdf_field* field, int32_t flags, const float* cam, const int32_t* list,
                     const int32_t* count, int64_t capacity, void* colour, int32_t colour_dtype,
                     void* stream);
int psdf_volume_render(const psdf_field* field, const psdf_render_opts* opts, const void* colour,
                       int32_t colour_dtype, const float* cam, int32_t W, int32_t H, float* out,
                       void* stream);

/* Thread-local text of the last error on this thread ("" if none). */
const char* psdf_last_error(void);

/* PSDF_ABI_VERSION of the loaded library. */
int psdf_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PROBESDF_H */
