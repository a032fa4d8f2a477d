/*
 * FP64 reference ("oracle") of the ProbeSDF per-ray render step.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, scalar C in double precision.  It is
 * called by the tests, by the smoke check and by the benchmark's CPU-baseline
 * leg, never by the product path, and it shares no code, header, table or
 * constant with the HIP library.
 *
 * Paper: Toussaint, Thomas, Franco, "ProbeSDF: Light Field Probes For Neural
 * Surface Reconstruction", CVPR 2025 (arXiv 2412.10084).  Every function cites
 * the passage it follows.  Where the paper is silent, the reading used is
 * stated at the function.
 *
 * All arrays are double.  Grids are align-corners over [-1,1]^3 (R nodes per
 * axis, h = 2/(R-1)), x fastest: index (k*R + j)*R + i.
 */
#ifndef PROBESDF_ORACLE_H
#define PROBESDF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t R;            /* spatial nodes per axis */
  int32_t P;            /* probe nodes per axis */
  int32_t n_feat;       /* spatial feature channels n_s */
  int32_t n_sh;         /* SH coefficients per probe: 1, 4, 9, 16 */
  int32_t n_ang;        /* angular feature channels n_a */
  int32_t hidden;       /* MLP hidden width */
  int32_t mlp_layers;   /* hidden layers: 1, or 2 (Sec. 4) */
  const double* sdf;    /* [R][R][R] */
  const double* feat;   /* [R][R][R][n_feat] */
  const double* probes; /* [P][P][P][n_sh][n_ang] */
  const double* mlp;    /* per hidden layer W_l[hidden][n_prev], b_l[hidden]; Wo[3][hidden], bo[3] */
  /* sparse tiles (Sec. 3.1, Sec. 4): tile_T > 0 selects tri-plane spatial features on
   * tiles of 16^3 cells, R = 16 tile_T + 1; feat is then unused */
  int32_t tile_T;              /* tiles per axis, 0: dense features */
  const int32_t* tile_index;   /* [T][T][T] slot of each tile, -1: empty (not allocated) */
  const double* tile_feat;     /* [slots][3][16][16][n_feat]: planes F_x(y,z), F_y(x,z), F_z(x,y) */
} orc_field;

/* flags */
#define ORC_NO_FS 1       /* F_s := 0 (visual ablation, Fig. "MLP components") */
#define ORC_NO_FA 2       /* F_a := 0 */
#define ORC_NV_ONE 4      /* n.v := 1 in the incidence inputs (Fresnel ablation, Table "Ablation") */
#define ORC_SH_REFLECT 8  /* SH evaluated at the reflected vector r (Sec. 3.1, Fig. overview) */
#define ORC_FRESNEL_PAPER 16 /* incidence inputs (1-n.v)^0..5 (Eq. newparametrization) */

typedef struct {
  int32_t n_samples;    /* N */
  double tau;           /* NeuS sharpness */
  double skip_voxels;   /* sample active iff |s| <= skip_voxels*h; <= 0 disables */
  int32_t flags;
} orc_render_opts;

typedef struct {
  double lr_sdf, lr_feat, lr_probe, lr_mlp;
  double beta1, beta2, eps;
  double lambda_eik, lambda_tv_feat, lambda_tv_probe;
} orc_step_opts;

typedef struct {
  orc_step_opts base;
  double lambda_sdf, lambda_normal;
  double sigma;        /* width of the 5-tap Gaussian, in voxels */
  int32_t smooth;      /* 1: the SDF parameters are shat, rendering reads s = G(shat) */
  int32_t weighted;    /* 1: (1 + 5 |s|)^-1 on the SDF regulariser gradients */
} orc_step_ext;

/* ---- building blocks, each pinned separately by the tests ---- */
int orc_ray_box(const double o[3], const double d[3], double* tn, double* tf);
void orc_trilinear(const double* grid, int R, int C, const double x[3], double* out);
void orc_tri_corners(int R, const double x[3], int64_t idx[8], double w[8]);
void orc_sdf_gradient(const double* sdf, int R, const double x[3], double g[3]);
int orc_sh_basis(int n_sh, const double v[3], double* Y);
double orc_logsigmoid(double x);
int orc_sh_grad(int n_sh, const double v[3], double* dY);
int64_t orc_mlp_size(int n_in, int hidden, int layers);
void orc_mlp_forward(const double* mlp, int n_in, int hidden, int layers, const double* z,
                     double* pre, double* hid, double out[3], double C[3]);
int orc_n_inputs(const orc_field* f, int32_t flags);
int orc_field_check(const orc_field* f, int32_t flags);
double orc_composite(int N, const double* s, const int32_t* active, double tau,
                     double* alpha, double* T, double* w);
void orc_shade(const orc_field* f, int32_t flags, const double x[3], const double v[3],
               double C[3], double* z_out);

/* ---- the render step ---- */
/* the render entry points return 0, or -1 for N outside [2, 2^20], a field
 * shape outside the supported set, or an allocation failure */
int orc_render_forward(const orc_field* f, const orc_render_opts* opt, int64_t B,
                       const double* rays_o, const double* rays_d, double* rgb,
                       double* aux, double* depth_wsum, double* margin,
                       int32_t* n_shaded);
int orc_render_backward(const orc_field* f, const orc_render_opts* opt, int64_t B,
                        const double* rays_o, const double* rays_d,
                        const double* dL_drgb, double* g_sdf, double* g_feat,
                        double* g_probes, double* g_mlp);
double orc_l1_loss(int64_t B, const double* rgb, const double* target, double* dL_drgb);
void orc_regularizers(int R, int P, int n_feat, int n_pc, const double* sdf,
                      const double* feat, const double* probes, double lambda_eik,
                      double lambda_tv_feat, double lambda_tv_probe, double* g_sdf,
                      double* g_feat, double* g_probes, double losses[3]);
void orc_adam(int64_t n, double* p, const double* g, double* m, double* v, int64_t step,
              double lr, double beta1, double beta2, double eps);
void orc_grid_step(int R, int P, int n_feat, int n_pc, int n_mlp, double* sdf, double* feat,
                   double* probes, double* mlp, const double* g_sdf, const double* g_feat,
                   const double* g_probes, const double* g_mlp, double* m, double* v,
                   int64_t step, const orc_step_opts* opt, double losses[3]);
void orc_gauss5(double sigma, double w[5]);
void orc_smooth(int R, double sigma, const double* shat, double* s);
void orc_smooth_T(int R, double sigma, const double* y, double* out);
void orc_sdf_regs(int R, const double* shat, int smooth, double sigma, int weighted,
                  double lambda_sdf, double lambda_eik, double lambda_normal, const double* g_s,
                  double* g_shat, double* s_out, double losses[3]);
void orc_grid_step_ext(int R, int P, int n_feat, int n_pc, int n_mlp, double* sdf, double* feat,
                       double* probes, double* mlp, const double* g_s, const double* g_feat,
                       const double* g_probes, const double* g_mlp, double* m, double* v,
                       int64_t step, const orc_step_ext* opt, double losses[5], double* s_new);
double orc_l2rel_loss(int64_t B, const double* rgb, const double* target, double lambda,
                      double eps, double n_images, double* dL_drgb);
void orc_voxel_shade(const orc_field* f, int32_t flags, const double cam_centre[3], double band,
                     double* col);
int orc_volume_render(const orc_field* f, const double* col, const orc_render_opts* opt,
                      const double* cam, int32_t W, int32_t H, const int64_t* pixel_ids,
                      int64_t n_pix, double* out, double* margin);
int orc_tile_of(const orc_field* f, const double x[3], double loc[3]);
int orc_triplane(const orc_field* f, const double x[3], double* out);
double orc_plane_smooth(int64_t n_slots, int n_feat, const double* planes, double lambda,
                        double* g);
void orc_set_threads(int n);
int orc_max_threads(void);
int orc_sphere_trace(const orc_field* f, int32_t flags, double eps, int32_t max_steps,
                     int32_t V, const double* cams, int32_t W, int32_t H,
                     const int64_t* pixel_ids, int64_t n_pix, double* out, double* t_hit,
                     int32_t* steps, double* margin);

#ifdef __cplusplus
}
#endif
#endif
