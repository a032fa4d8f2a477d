/*
 * FP64 reference ("oracle") of the ProbeSDF per-ray render step.
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code
 * with the HIP library.  Everything is double precision, scalar, and follows
 * the paper's equations in the paper's order; OpenMP only spreads rays over
 * cores.
 *
 * Paper sections cited: Sec. 3.1 "Decoupled Parametrization of Radiance"
 * (Eqs. rendering/classic/shlick/newparametrization), Sec. 3.2 "Light Field
 * Probes on a Coarse Grid" (Eqs. spherical_harmonics, sh_eval1, sh_eval2),
 * Sec. 3.3 "SDF Estimation Approach" (Eq. neus and the loss Eqs. smooth_sdf ..
 * photo_loss), Sec. 3.4 "Training", Sec. 4 "Implementation Details",
 * Supplementary Sec. A "Scheduling" (Adam moments).
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_N 1048576 /* largest N the render entry points accept */
#define MAXIN 64    /* max MLP inputs */
#define MAXH 128    /* max MLP hidden width */
#define MAXSH 16

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* ---------------------------------------------------------------------------
 * Ray / box interval.  The paper renders pixel-aligned rays (Sec. 3.3); the
 * sampling interval is the ray's intersection with the grid's domain
 * [-1,1]^3 (slab test), clipped to t >= 0.  Returns 1 iff t_f > t_n.
 * ------------------------------------------------------------------------- */
int orc_ray_box(const double o[3], const double d[3], double* tn, double* tf) {
  double t0 = -INFINITY, t1 = INFINITY;
  for (int a = 0; a < 3; ++a) {
    double ta = (-1.0 - o[a]) / d[a];
    double tb = (1.0 - o[a]) / d[a];
    t0 = fmax(t0, fmin(ta, tb));
    t1 = fmin(t1, fmax(ta, tb));
  }
  t0 = fmax(t0, 0.0);
  *tn = t0;
  *tf = t1;
  return t1 > t0;
}

/* ---------------------------------------------------------------------------
 * Trilinear interpolation on an align-corners grid (Sec. 3.2, Eqs.
 * sh_eval1/sh_eval2: a point blends its 8 surrounding probes with trilinear
 * weights w_i; the same operator serves the SDF and spatial features).  Reading: per axis u = (x+1)/h,
 * k0 = clamp(floor(u), 0, R-2), f = u - k0; weight of corner (dx,dy,dz) is the
 * product over axes of (f if d=1 else 1-f).
 * ------------------------------------------------------------------------- */
static void cell_coord(int R, double x, int* k0, double* f) {
  double h = 2.0 / (double)(R - 1);
  double u = (x + 1.0) / h;
  double fl = floor(u);
  if (fl < 0.0) fl = 0.0;
  if (fl > (double)(R - 2)) fl = (double)(R - 2);
  *k0 = (int)fl;
  *f = u - fl;
}

void orc_tri_corners(int R, const double x[3], int64_t idx[8], double w[8]) {
  int k[3];
  double f[3];
  for (int a = 0; a < 3; ++a) cell_coord(R, x[a], &k[a], &f[a]);
  for (int c = 0; c < 8; ++c) {
    int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
    double wx = dx ? f[0] : 1.0 - f[0];
    double wy = dy ? f[1] : 1.0 - f[1];
    double wz = dz ? f[2] : 1.0 - f[2];
    idx[c] = ((int64_t)(k[2] + dz) * R + (k[1] + dy)) * R + (k[0] + dx);
    w[c] = wx * wy * wz;
  }
}

void orc_trilinear(const double* grid, int R, int C, const double x[3], double* out) {
  int64_t idx[8];
  double w[8];
  orc_tri_corners(R, x, idx, w);
  for (int ch = 0; ch < C; ++ch) out[ch] = 0.0;
  for (int c = 0; c < 8; ++c)
    for (int ch = 0; ch < C; ++ch) out[ch] += w[c] * grid[idx[c] * C + ch];
}

/* ---------------------------------------------------------------------------
 * SDF gradient for the normal n = grad s / |grad s| (Sec. 3.3, Eq.
 * smmoth_normals defines n this way; the gradient operator is not given).
 * Reading: central difference of the trilinear SDF with step h along each
 * axis; both stencil points are clamped to the domain and the difference is
 * divided by the actual distance between them.
 * ------------------------------------------------------------------------- */
void orc_sdf_gradient(const double* sdf, int R, const double x[3], double g[3]) {
  double h = 2.0 / (double)(R - 1);
  for (int a = 0; a < 3; ++a) {
    double xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]};
    xp[a] = clampd(x[a] + h, -1.0, 1.0);
    xm[a] = clampd(x[a] - h, -1.0, 1.0);
    double sp, sm;
    orc_trilinear(sdf, R, 1, xp, &sp);
    orc_trilinear(sdf, R, 1, xm, &sm);
    g[a] = (sp - sm) / (xp[a] - xm[a]);
  }
}

/* ---------------------------------------------------------------------------
 * Real spherical-harmonic basis Y_j (Sec. 3.2, Eq. spherical_harmonics: l^2
 * coefficients with one-indexed l).  Reading: orthonormal real SH on the unit
 * sphere, no Condon-Shortley phase, ordered (0,0), (1,-1), (1,0), (1,1),
 * (2,-2) .. (2,2), (3,-3) .. (3,3).  Constants are computed here from their
 * closed forms.
 * ------------------------------------------------------------------------- */
int orc_sh_basis(int n_sh, const double v[3], double* Y) {
  const double pi = acos(-1.0);
  double x = v[0], y = v[1], z = v[2];
  if (n_sh != 1 && n_sh != 4 && n_sh != 9 && n_sh != 16) return -1;
  Y[0] = 0.5 * sqrt(1.0 / pi);
  if (n_sh >= 4) {
    double c1 = sqrt(3.0 / (4.0 * pi));
    Y[1] = c1 * y;
    Y[2] = c1 * z;
    Y[3] = c1 * x;
  }
  if (n_sh >= 9) {
    double c2 = 0.5 * sqrt(15.0 / pi);
    Y[4] = c2 * x * y;
    Y[5] = c2 * y * z;
    Y[6] = 0.25 * sqrt(5.0 / pi) * (3.0 * z * z - 1.0);
    Y[7] = c2 * x * z;
    Y[8] = 0.25 * sqrt(15.0 / pi) * (x * x - y * y);
  }
  if (n_sh >= 16) {
    Y[9] = 0.25 * sqrt(35.0 / (2.0 * pi)) * y * (3.0 * x * x - y * y);
    Y[10] = 0.5 * sqrt(105.0 / pi) * x * y * z;
    Y[11] = 0.25 * sqrt(21.0 / (2.0 * pi)) * y * (5.0 * z * z - 1.0);
    Y[12] = 0.25 * sqrt(7.0 / pi) * z * (5.0 * z * z - 3.0);
    Y[13] = 0.25 * sqrt(21.0 / (2.0 * pi)) * x * (5.0 * z * z - 1.0);
    Y[14] = 0.25 * sqrt(105.0 / pi) * z * (x * x - y * y);
    Y[15] = 0.25 * sqrt(35.0 / (2.0 * pi)) * x * (x * x - 3.0 * y * y);
  }
  return 0;
}

/* ---------------------------------------------------------------------------
 * log Phi_tau(s) with Phi the logistic of Eq. neus: log(1/(1+e^{-x})) written
 * as min(x,0) - log1p(e^{-|x|}), which is the same function without overflow.
 * ------------------------------------------------------------------------- */
double orc_logsigmoid(double x) { return fmin(x, 0.0) - log1p(exp(-fabs(x))); }

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* ---------------------------------------------------------------------------
 * Colour MLP (Sec. 4: ReLU hidden layers, sigmoid output layer).  `layers`
 * hidden layers of `hidden` units: a_0 = z, pre_l = W_l a_{l-1} + b_l,
 * a_l = max(pre_l, 0), out = Wo a_L + bo, C = sigmoid(out).  Packed weights, in
 * this order: for each hidden layer W_l[hidden][n_{l-1}] row-major (n_0 = n_in,
 * else hidden) and b_l[hidden]; then Wo[3][hidden] and bo[3].  pre and hid hold
 * layers x hidden values (layer-major).
 * ------------------------------------------------------------------------- */
int64_t orc_mlp_size(int n_in, int hidden, int layers) {
  int64_t n = 0;
  for (int l = 0; l < layers; ++l) n += (int64_t)hidden * (l == 0 ? n_in : hidden) + hidden;
  return n + 3 * (int64_t)hidden + 3;
}

void orc_mlp_forward(const double* mlp, int n_in, int hidden, int layers, const double* z,
                     double* pre, double* hid, double out[3], double C[3]) {
  const double* p = mlp;
  const double* a = z;
  int n_prev = n_in;
  for (int l = 0; l < layers; ++l) {
    const double* W = p;
    const double* b = W + hidden * n_prev;
    for (int k = 0; k < hidden; ++k) {
      double acc = b[k];
      for (int j = 0; j < n_prev; ++j) acc += W[k * n_prev + j] * a[j];
      pre[l * hidden + k] = acc;
      hid[l * hidden + k] = acc > 0.0 ? acc : 0.0;
    }
    p = b + hidden;
    a = hid + l * hidden;
    n_prev = hidden;
  }
  const double* Wo = p;
  const double* bo = Wo + 3 * hidden;
  for (int c = 0; c < 3; ++c) {
    double acc = bo[c];
    for (int k = 0; k < hidden; ++k) acc += Wo[c * hidden + k] * a[k];
    out[c] = acc;
    C[c] = sigmoid(acc);
  }
}

/* ---------------------------------------------------------------------------
 * NeuS compositing weights (Sec. 3.3, Eq. neus):
 *   alpha_i = max((Phi(s_i) - Phi(s_{i+1})) / Phi(s_i), 0),
 *   T_i = prod_{j<i} (1 - alpha_j),  weight w_i = T_i alpha_i.
 * Evaluated in the log domain: 1 - Phi(s_{i+1})/Phi(s_i) = -expm1(dl) with
 * dl = log Phi(s_{i+1}) - log Phi(s_i), and log(1 - alpha_i) = min(dl, 0).
 * Reading: alpha of the last sample is 0 (it has no successor), inactive
 * samples (skip rule) have alpha 0.  Returns log T after the last sample.
 * ------------------------------------------------------------------------- */
double orc_composite(int N, const double* s, const int32_t* active, double tau, double* alpha,
                     double* T, double* w) {
  double logT = 0.0;
  for (int i = 0; i < N; ++i) {
    double a = 0.0;
    double dl = 0.0;
    if (i + 1 < N && active[i]) {
      dl = orc_logsigmoid(tau * s[i + 1]) - orc_logsigmoid(tau * s[i]);
      a = dl < 0.0 ? -expm1(dl) : 0.0;
    }
    alpha[i] = a;
    T[i] = exp(logT);
    w[i] = T[i] * a;
    if (a > 0.0) logT += dl;
  }
  return logT;
}

/* ---------------------------------------------------------------------------
 * Gradient of each real SH polynomial of orc_sh_basis with respect to its
 * argument (x, y, z), taken on the polynomials themselves: dY[j][a] = dY_j/dx_a.
 * Needed where the SH argument depends on the normal (reflected vector).
 * ------------------------------------------------------------------------- */
int orc_sh_grad(int n_sh, const double v[3], double* dY) {
  const double pi = acos(-1.0);
  double x = v[0], y = v[1], z = v[2];
  if (n_sh != 1 && n_sh != 4 && n_sh != 9 && n_sh != 16) return -1;
  for (int q = 0; q < 3 * n_sh; ++q) dY[q] = 0.0;
  if (n_sh >= 4) {
    double c1 = sqrt(3.0 / (4.0 * pi));
    dY[3 * 1 + 1] = c1;
    dY[3 * 2 + 2] = c1;
    dY[3 * 3 + 0] = c1;
  }
  if (n_sh >= 9) {
    double c2 = 0.5 * sqrt(15.0 / pi), c6 = 0.25 * sqrt(5.0 / pi), c8 = 0.25 * sqrt(15.0 / pi);
    dY[3 * 4 + 0] = c2 * y;
    dY[3 * 4 + 1] = c2 * x;
    dY[3 * 5 + 1] = c2 * z;
    dY[3 * 5 + 2] = c2 * y;
    dY[3 * 6 + 2] = 6.0 * c6 * z;
    dY[3 * 7 + 0] = c2 * z;
    dY[3 * 7 + 2] = c2 * x;
    dY[3 * 8 + 0] = 2.0 * c8 * x;
    dY[3 * 8 + 1] = -2.0 * c8 * y;
  }
  if (n_sh >= 16) {
    double a9 = 0.25 * sqrt(35.0 / (2.0 * pi)), a10 = 0.5 * sqrt(105.0 / pi);
    double a11 = 0.25 * sqrt(21.0 / (2.0 * pi)), a12 = 0.25 * sqrt(7.0 / pi);
    double a14 = 0.25 * sqrt(105.0 / pi);
    dY[3 * 9 + 0] = 6.0 * a9 * x * y;
    dY[3 * 9 + 1] = 3.0 * a9 * (x * x - y * y);
    dY[3 * 10 + 0] = a10 * y * z;
    dY[3 * 10 + 1] = a10 * x * z;
    dY[3 * 10 + 2] = a10 * x * y;
    dY[3 * 11 + 1] = a11 * (5.0 * z * z - 1.0);
    dY[3 * 11 + 2] = 10.0 * a11 * y * z;
    dY[3 * 12 + 2] = a12 * (15.0 * z * z - 3.0);
    dY[3 * 13 + 0] = a11 * (5.0 * z * z - 1.0);
    dY[3 * 13 + 2] = 10.0 * a11 * x * z;
    dY[3 * 14 + 0] = 2.0 * a14 * x * z;
    dY[3 * 14 + 1] = -2.0 * a14 * y * z;
    dY[3 * 14 + 2] = a14 * (x * x - y * y);
    dY[3 * 15 + 0] = 3.0 * a9 * (x * x - y * y);
    dY[3 * 15 + 1] = -6.0 * a9 * x * y;
  }
  return 0;
}

/* Number of incidence inputs of the colour model: (c, c^2, c^4), or
 * (1 - c)^0 .. (1 - c)^5 with ORC_FRESNEL_PAPER. */
static int n_incidence(int32_t flags) { return (flags & ORC_FRESNEL_PAPER) ? 6 : 3; }

int orc_n_inputs(const orc_field* f, int32_t flags) {
  return f->n_feat + f->n_ang + n_incidence(flags);
}

/* 0 if the field's shape fits the fixed-size scratch of this file (MLP inputs,
 * hidden width, SH order, layer count), else -1 */
int orc_field_check(const orc_field* f, int32_t flags) {
  if (f->R < 2 || f->P < 2) return -1;
  if (f->n_sh != 1 && f->n_sh != 4 && f->n_sh != 9 && f->n_sh != 16) return -1;
  if (f->n_ang < 1 || f->n_ang > 16 || f->n_feat < 0) return -1;
  if (orc_n_inputs(f, flags) > MAXIN) return -1;
  if (f->hidden < 1 || f->hidden > MAXH || f->mlp_layers < 1 || f->mlp_layers > 2) return -1;
  if (f->tile_T > 0 && (f->R != 16 * f->tile_T + 1 || f->n_feat > 64 || !f->tile_index ||
                        !f->tile_feat))
    return -1;
  return 0;
}

/* ---------------------------------------------------------------------------
 * Colour of one sample (Sec. 3.1 Eqs. classic/newparametrization, Sec. 3.2
 * Eqs. spherical_harmonics, sh_eval1/sh_eval2, Sec. 4):
 *   n = g / |g| with g the SDF gradient, c = n.v (v points from the sample to
 *   the camera);
 *   the SH argument is v, or with ORC_SH_REFLECT the reflection of v about the
 *   normal, r = 2 (n.v) n - v (Sec. 3.1 defines r as the reflected vector for
 *   the view direction v; r = v at normal incidence);
 *   F_s = trilinear spatial features at x;
 *   bhat_j = sum_i w_i b_ij over the 8 probes, F_a = sum_j bhat_j Y_j(arg);
 *   incidence inputs from c' = c (or 1 with ORC_NV_ONE): (c', c'^2, c'^4), or
 *   with ORC_FRESNEL_PAPER the powers (1 - c')^0 .. (1 - c')^5 of Eq.
 *   newparametrization;
 *   C = MLP([F_s, F_a, incidence inputs]).
 * The reflection always uses the true n.v; ORC_NV_ONE only replaces the
 * incidence inputs.
 * ------------------------------------------------------------------------- */
/* ---------------------------------------------------------------------------
 * Sparse tiles with tri-plane spatial features (Sec. 3.1: F_s = F_x (x) F_y (x)
 * F_z from planes of the coarse tile; Sec. 4: tiles of 16^3 voxels holding
 * 3 x 16 x 16 x n_s coefficients).  Readings: R = 16 T + 1 nodes, tile of a point
 * = the tile of its trilinear cell; each plane is a 16 x 16 texture of the tile
 * with texels at the cell centres, bilinear with clamping inside the tile (no
 * reads across tiles); the three interpolated planes are multiplied channel by
 * channel; a point in an empty tile is inactive (the skip rule of the sparse
 * grid).  F_x is a function of (y, z), F_y of (x, z), F_z of (x, y).
 * ------------------------------------------------------------------------- */
/* slot of the tile holding x (-1: empty), and x in the tile's cell units [0, 16] */
int orc_tile_of(const orc_field* f, const double x[3], double loc[3]) {
  double h = 2.0 / (double)(f->R - 1);
  int t[3];
  for (int a = 0; a < 3; ++a) {
    double u = (x[a] + 1.0) / h;
    double k0 = floor(u);
    if (k0 < 0.0) k0 = 0.0;
    if (k0 > f->R - 2) k0 = f->R - 2;
    t[a] = (int)k0 / 16;
    loc[a] = u - 16.0 * t[a];
  }
  int T = f->tile_T;
  return f->tile_index[((int64_t)t[2] * T + t[1]) * T + t[0]];
}

/* texel cell and weight along one plane axis */
static void texel(double l, int* c0, double* w) {
  double tau = clampd(l - 0.5, 0.0, 15.0);
  double c = floor(tau);
  if (c > 14.0) c = 14.0;
  *c0 = (int)c;
  *w = tau - c;
}

/* axes (u, v) of plane a */
static const int plane_axes[3][2] = {{1, 2}, {0, 2}, {0, 1}};

/* bilinear corners of plane a at loc: texel indices and weights */
static void plane_corners(const double loc[3], int a, int idx[4], double w[4]) {
  int cu, cv;
  double fu, fv;
  texel(loc[plane_axes[a][0]], &cu, &fu);
  texel(loc[plane_axes[a][1]], &cv, &fv);
  idx[0] = cv * 16 + cu;
  idx[1] = cv * 16 + cu + 1;
  idx[2] = (cv + 1) * 16 + cu;
  idx[3] = (cv + 1) * 16 + cu + 1;
  w[0] = (1 - fu) * (1 - fv);
  w[1] = fu * (1 - fv);
  w[2] = (1 - fu) * fv;
  w[3] = fu * fv;
}

/* F_s at x into out[n_feat] (0 in an empty tile); returns the tile slot */
int orc_triplane(const orc_field* f, const double x[3], double* out) {
  double loc[3];
  int slot = orc_tile_of(f, x, loc);
  int nf = f->n_feat;
  for (int c = 0; c < nf; ++c) out[c] = slot >= 0 ? 1.0 : 0.0;
  if (slot < 0) return slot;
  for (int a = 0; a < 3; ++a) {
    int idx[4];
    double w[4];
    plane_corners(loc, a, idx, w);
    const double* pl = f->tile_feat + ((int64_t)slot * 3 + a) * 256 * nf;
    for (int c = 0; c < nf; ++c) {
      double v = 0.0;
      for (int q = 0; q < 4; ++q) v += w[q] * pl[idx[q] * nf + c];
      out[c] *= v;
    }
  }
  return slot;
}

static void add_atomic(double* p, double v);

/* reverse mode of orc_triplane: adds dF_s into the plane gradients g (tile layout) */
static void triplane_backward(const orc_field* f, const double x[3], const double* dfs,
                              double* g) {
  double loc[3];
  int slot = orc_tile_of(f, x, loc);
  if (slot < 0) return;
  int nf = f->n_feat;
  double val[3][64];
  int idx[3][4];
  double w[3][4];
  for (int a = 0; a < 3; ++a) {
    plane_corners(loc, a, idx[a], w[a]);
    const double* pl = f->tile_feat + ((int64_t)slot * 3 + a) * 256 * nf;
    for (int c = 0; c < nf; ++c) {
      double v = 0.0;
      for (int q = 0; q < 4; ++q) v += w[a][q] * pl[idx[a][q] * nf + c];
      val[a][c] = v;
    }
  }
  for (int a = 0; a < 3; ++a) {
    double* gp = g + ((int64_t)slot * 3 + a) * 256 * nf;
    for (int c = 0; c < nf; ++c) {
      double other = 1.0;
      for (int b = 0; b < 3; ++b)
        if (b != a) other *= val[b][c];
      for (int q = 0; q < 4; ++q) add_atomic(&gp[idx[a][q] * nf + c], w[a][q] * other * dfs[c]);
    }
  }
}

/* Smoothness of the factorised features (Eq. smooth_features), mean-normalised:
 * lambda / (n_slots 3 2 16 15 n_feat) * sum over every plane, both of its axes and
 * channel of squared differences of neighbouring texels.  Adds the gradient into g;
 * returns the loss. */
double orc_plane_smooth(int64_t n_slots, int n_feat, const double* planes, double lambda,
                        double* g) {
  double sc = lambda / ((double)n_slots * 3 * 2 * 16 * 15 * n_feat);
  double acc = 0.0;
  for (int64_t p = 0; p < n_slots * 3; ++p) {
    const double* pl = planes + p * 256 * n_feat;
    double* gp = g + p * 256 * n_feat;
    for (int v = 0; v < 16; ++v)
      for (int u = 0; u < 16; ++u)
        for (int dir = 0; dir < 2; ++dir) {
          int u2 = u + (dir == 0), v2 = v + (dir == 1);
          if (u2 > 15 || v2 > 15) continue;
          for (int c = 0; c < n_feat; ++c) {
            double d = pl[(v2 * 16 + u2) * n_feat + c] - pl[(v * 16 + u) * n_feat + c];
            acc += d * d;
            gp[(v2 * 16 + u2) * n_feat + c] += 2.0 * sc * d;
            gp[(v * 16 + u) * n_feat + c] -= 2.0 * sc * d;
          }
        }
  }
  return sc * acc;
}

typedef struct {
  double g[3], gn, n[3], c, cin, arg[3];
  double z[MAXIN], pre[2 * MAXH], hid[2 * MAXH], out[3], C[3];
  double Y[MAXSH], bhat[MAXSH * 16];
} shade_state;

static void shade_full(const orc_field* f, int32_t flags, const double x[3], const double v[3],
                       shade_state* st) {
  int nf = f->n_feat, na = f->n_ang, nsh = f->n_sh;
  int n_in = orc_n_inputs(f, flags);
  /* normal and incidence cosine */
  orc_sdf_gradient(f->sdf, f->R, x, st->g);
  st->gn = sqrt(st->g[0] * st->g[0] + st->g[1] * st->g[1] + st->g[2] * st->g[2]);
  double inv = 1.0 / fmax(st->gn, 1e-30);
  for (int a = 0; a < 3; ++a) st->n[a] = st->g[a] * inv;
  st->c = st->n[0] * v[0] + st->n[1] * v[1] + st->n[2] * v[2];
  st->cin = (flags & ORC_NV_ONE) ? 1.0 : st->c;
  /* SH argument */
  for (int a = 0; a < 3; ++a)
    st->arg[a] = (flags & ORC_SH_REFLECT) ? 2.0 * st->c * st->n[a] - v[a] : v[a];
  orc_sh_basis(nsh, st->arg, st->Y);
  /* spatial features */
  if (flags & ORC_NO_FS) {
    for (int k = 0; k < nf; ++k) st->z[k] = 0.0;
  } else {
    if (f->tile_T > 0) orc_triplane(f, x, st->z);
    else orc_trilinear(f->feat, f->R, nf, x, st->z);
  }
  /* angular features: interpolate the coefficients (Eq. sh_eval2), then
   * evaluate the basis */
  if (flags & ORC_NO_FA) {
    for (int a = 0; a < na; ++a) st->z[nf + a] = 0.0;
    for (int q = 0; q < nsh * na; ++q) st->bhat[q] = 0.0;
  } else {
    orc_trilinear(f->probes, f->P, nsh * na, x, st->bhat);
    for (int a = 0; a < na; ++a) {
      double acc = 0.0;
      for (int j = 0; j < nsh; ++j) acc += st->bhat[j * na + a] * st->Y[j];
      st->z[nf + a] = acc;
    }
  }
  double c = st->cin;
  double* zi = st->z + nf + na;
  if (flags & ORC_FRESNEL_PAPER) {
    double p = 1.0;
    for (int m = 0; m < 6; ++m) {
      zi[m] = p;
      p *= 1.0 - c;
    }
  } else {
    zi[0] = c;
    zi[1] = c * c;
    zi[2] = c * c * c * c;
  }
  orc_mlp_forward(f->mlp, n_in, f->hidden, f->mlp_layers, st->z, st->pre, st->hid, st->out,
                  st->C);
}

void orc_shade(const orc_field* f, int32_t flags, const double x[3], const double v[3],
               double C[3], double* z_out) {
  shade_state st;
  shade_full(f, flags, x, v, &st);
  for (int c = 0; c < 3; ++c) C[c] = st.C[c];
  if (z_out)
    for (int j = 0; j < orc_n_inputs(f, flags); ++j) z_out[j] = st.z[j];
}

/* ---------------------------------------------------------------------------
 * Samples along one ray.  Reading (the paper gives no sampler): N cell-centred
 * samples t_i = t_n + (i + 1/2) dt, dt = (t_f - t_n)/N, positions clamped to
 * the domain; s_i is the trilinear SDF.  Skip rule: sample i is active iff
 * |s_i| <= skip_voxels * h (skip_voxels <= 0: always).  margin = distance of
 * the closest |s_i| to the skip threshold (decisions near it may flip between
 * precisions).
 * ------------------------------------------------------------------------- */
typedef struct {
  int hit;
  double o[3], d[3], v[3], tn, tf, dt;
  int N;
  /* per-sample arrays of length N (ray_state_alloc) */
  double *t, (*x)[3], *s, *alpha, *T, *w;
  int32_t* active;
  double logT_final, margin;
} ray_state;

/* One allocation holding a ray_state and its N-sample arrays; NULL if out of
 * memory.  Released with free(). */
static ray_state* ray_state_alloc(int N) {
  size_t n = (size_t)N;
  size_t bytes = sizeof(ray_state) + n * (5 * sizeof(double) + 3 * sizeof(double)) +
                 n * sizeof(int32_t);
  ray_state* r = (ray_state*)calloc(1, bytes);
  if (!r) return NULL;
  double* p = (double*)(r + 1);
  r->t = p;
  p += n;
  r->x = (double(*)[3])p;
  p += 3 * n;
  r->s = p;
  p += n;
  r->alpha = p;
  p += n;
  r->T = p;
  p += n;
  r->w = p;
  p += n;
  r->active = (int32_t*)p;
  return r;
}

static void march(const orc_field* f, const orc_render_opts* opt, const double* o_in,
                  const double* d_in, ray_state* r) {
  int N = opt->n_samples;
  double h = 2.0 / (double)(f->R - 1);
  double dn = sqrt(d_in[0] * d_in[0] + d_in[1] * d_in[1] + d_in[2] * d_in[2]);
  for (int a = 0; a < 3; ++a) {
    r->o[a] = o_in[a];
    r->d[a] = d_in[a] / dn;
    r->v[a] = -r->d[a];
  }
  r->N = N;
  r->margin = INFINITY;
  r->logT_final = 0.0;
  r->hit = orc_ray_box(r->o, r->d, &r->tn, &r->tf);
  if (!r->hit) return;
  r->dt = (r->tf - r->tn) / N;
  double thr = opt->skip_voxels * h;
  for (int i = 0; i < N; ++i) {
    r->t[i] = r->tn + (i + 0.5) * r->dt;
    for (int a = 0; a < 3; ++a) r->x[i][a] = clampd(r->o[a] + r->t[i] * r->d[a], -1.0, 1.0);
    orc_trilinear(f->sdf, f->R, 1, r->x[i], &r->s[i]);
    if (opt->skip_voxels > 0.0) {
      r->active[i] = fabs(r->s[i]) <= thr;
      if (i + 1 < N) r->margin = fmin(r->margin, fabs(fabs(r->s[i]) - thr));
    } else {
      r->active[i] = 1;
    }
    if (f->tile_T > 0) {
      double loc[3];
      if (orc_tile_of(f, r->x[i], loc) < 0) r->active[i] = 0;
    }
  }
  r->logT_final = orc_composite(N, r->s, r->active, opt->tau, r->alpha, r->T, r->w);
}

/* ---------------------------------------------------------------------------
 * Forward render (Sec. 3.3): c = sum_i T_i alpha_i C_i.  Also returned:
 * aux = (c, log T_final), depth_wsum = (sum_i w_i (t_i + dt/2), sum_i w_i),
 * margin (see march), n_shaded = samples with alpha > 0.  Misses give 0
 * (no background term).  Returns 0, or -1 (nothing written) if N is outside
 * [2, ORC_MAX_N] or memory runs out.
 * ------------------------------------------------------------------------- */
int orc_render_forward(const orc_field* f, const orc_render_opts* opt, int64_t B,
                       const double* rays_o, const double* rays_d, double* rgb, double* aux,
                       double* depth_wsum, double* margin, int32_t* n_shaded) {
  if (opt->n_samples < 2 || opt->n_samples > ORC_MAX_N) return -1;
  if (orc_field_check(f, opt->flags)) return -1;
  int failed = 0;
#pragma omp parallel
  {
  ray_state* r = ray_state_alloc(opt->n_samples);
  if (!r) {
#pragma omp atomic write
    failed = 1;
  }
#pragma omp barrier
  if (!failed) {
#pragma omp for schedule(dynamic, 16)
  for (int64_t b = 0; b < B; ++b) {
    march(f, opt, rays_o + 3 * b, rays_d + 3 * b, r);
    double col[3] = {0, 0, 0}, wsum = 0.0, depth = 0.0;
    int ns = 0;
    if (r->hit) {
      for (int i = 0; i < r->N; ++i) {
        if (!(r->alpha[i] > 0.0)) continue;
        double C[3];
        orc_shade(f, opt->flags, r->x[i], r->v, C, NULL);
        for (int c = 0; c < 3; ++c) col[c] += r->w[i] * C[c];
        wsum += r->w[i];
        depth += r->w[i] * (r->t[i] + 0.5 * r->dt);
        ++ns;
      }
    }
    for (int c = 0; c < 3; ++c) rgb[3 * b + c] = col[c];
    if (aux) {
      for (int c = 0; c < 3; ++c) aux[4 * b + c] = col[c];
      aux[4 * b + 3] = r->logT_final;
    }
    if (depth_wsum) {
      depth_wsum[2 * b + 0] = depth;
      depth_wsum[2 * b + 1] = wsum;
    }
    if (margin) margin[b] = r->margin;
    if (n_shaded) n_shaded[b] = ns;
  }
  }
  free(r);
  }
  return failed ? -1 : 0;
}

/* ---------------------------------------------------------------------------
 * Analytic reverse mode of the forward render (Sec. 3.3: the SDF, features,
 * probes and MLP are trained by backpropagating the colour loss through the
 * rendering equation).  Gradients are ADDED to g_* (accumulation over batches,
 * Supplementary Sec. A).  Steps:
 *  d c / d C_i = w_i;
 *  d c / d alpha_i = T_i (C_i - S_i) with the colour behind sample i
 *      S_{N-1} = 0, S_{i-1} = alpha_i C_i + (1 - alpha_i) S_i;
 *  alpha_i = -expm1(dl_i): d alpha_i/d s_i = (1-alpha_i) tau sigma(-tau s_i),
 *      d alpha_i / d s_{i+1} = -(1-alpha_i) tau sigma(-tau s_{i+1}), zero when the
 *      max(., 0) clamp is active or the sample is inactive;
 *  then the MLP, the normal n (through the incidence inputs, d c/d n = v, and
 *  with the reflected SH argument through r = 2 (n.v) n - v), n = g/|g|
 *  (d n/d g = (I - n n^T)/|g|), the finite-difference stencil, and the
 *  trilinear weights scatter into nodes.
 * ------------------------------------------------------------------------- */
static void add_atomic(double* p, double v) {
#pragma omp atomic
  *p += v;
}

static void scatter_tri(double* grid, int R, int C, const double x[3], const double* val) {
  int64_t idx[8];
  double w[8];
  orc_tri_corners(R, x, idx, w);
  for (int c = 0; c < 8; ++c)
    for (int ch = 0; ch < C; ++ch)
      if (val[ch] != 0.0) add_atomic(&grid[idx[c] * C + ch], w[c] * val[ch]);
}

/* reverse mode of orc_mlp_forward: adds the weight gradients into g_mlp and
 * returns dL/dz */
static void mlp_backward(const double* mlp, int n_in, int H, int L, const double* z,
                         const double* pre, const double* hid, const double dout[3],
                         double* g_mlp, double* dz) {
  const double* Wl[2];
  double* gWl[2];
  int64_t off = 0;
  for (int l = 0; l < L; ++l) {
    Wl[l] = mlp + off;
    gWl[l] = g_mlp + off;
    off += (int64_t)H * (l == 0 ? n_in : H) + H;
  }
  const double* Wo = mlp + off;
  double* gWo = g_mlp + off;
  double* gbo = gWo + 3 * H;
  const double* aL = hid + (L - 1) * H;
  double da[MAXH], dpre[MAXH];
  for (int c = 0; c < 3; ++c) {
    add_atomic(&gbo[c], dout[c]);
    for (int k = 0; k < H; ++k) add_atomic(&gWo[c * H + k], dout[c] * aL[k]);
  }
  for (int k = 0; k < H; ++k) {
    double acc = 0.0;
    for (int c = 0; c < 3; ++c) acc += Wo[c * H + k] * dout[c];
    da[k] = acc;
  }
  for (int l = L - 1; l >= 0; --l) {
    int n_prev = l == 0 ? n_in : H;
    const double* a_prev = l == 0 ? z : hid + (l - 1) * H;
    const double* W = Wl[l];
    double* gW = gWl[l];
    double* gb = gW + H * n_prev;
    /* ReLU: derivative 1 iff pre-activation > 0 */
    for (int k = 0; k < H; ++k) dpre[k] = pre[l * H + k] > 0.0 ? da[k] : 0.0;
    for (int k = 0; k < H; ++k) {
      add_atomic(&gb[k], dpre[k]);
      for (int j = 0; j < n_prev; ++j) add_atomic(&gW[k * n_prev + j], dpre[k] * a_prev[j]);
    }
    double* dst = l == 0 ? dz : da;
    double tmp[MAXH > MAXIN ? MAXH : MAXIN];
    for (int j = 0; j < n_prev; ++j) {
      double acc = 0.0;
      for (int k = 0; k < H; ++k) acc += W[k * n_prev + j] * dpre[k];
      tmp[j] = acc;
    }
    for (int j = 0; j < n_prev; ++j) dst[j] = tmp[j];
  }
}

static void shade_backward(const orc_field* f, int32_t flags, const double x[3],
                           const double v[3], const shade_state* st, const double dC[3],
                           double* g_sdf, double* g_feat, double* g_probes, double* g_mlp) {
  int nf = f->n_feat, na = f->n_ang, nsh = f->n_sh;
  int n_in = orc_n_inputs(f, flags);
  /* sigmoid output */
  double dout[3];
  for (int c = 0; c < 3; ++c) dout[c] = dC[c] * st->C[c] * (1.0 - st->C[c]);
  double dz[MAXIN];
  mlp_backward(f->mlp, n_in, f->hidden, f->mlp_layers, st->z, st->pre, st->hid, dout, g_mlp,
               dz);
  /* spatial features */
  if (!(flags & ORC_NO_FS)) {
    if (f->tile_T > 0) triplane_backward(f, x, dz, g_feat);
    else scatter_tri(g_feat, f->R, nf, x, dz);
  }
  /* probes: d/d b_ij = w_i Y_j dF_a */
  if (!(flags & ORC_NO_FA)) {
    double gb[MAXSH * 16];
    for (int j = 0; j < nsh; ++j)
      for (int a = 0; a < na; ++a) gb[j * na + a] = st->Y[j] * dz[nf + a];
    scatter_tri(g_probes, f->P, nsh * na, x, gb);
  }
  /* cotangent of the unit normal n */
  int through_normal = 0;
  double dn[3] = {0.0, 0.0, 0.0};
  if (!(flags & ORC_NV_ONE)) {
    const double* dzi = dz + nf + na;
    double c = st->c, dc = 0.0;
    if (flags & ORC_FRESNEL_PAPER) {
      /* d/dc (1 - c)^m = -m (1 - c)^(m-1) */
      double p = 1.0;
      for (int m = 1; m < 6; ++m) {
        dc -= m * p * dzi[m];
        p *= 1.0 - c;
      }
    } else {
      dc = dzi[0] + 2.0 * c * dzi[1] + 4.0 * c * c * c * dzi[2];
    }
    for (int a = 0; a < 3; ++a) dn[a] += dc * v[a];
    through_normal = 1;
  }
  if ((flags & ORC_SH_REFLECT) && !(flags & ORC_NO_FA)) {
    /* F_a,k = sum_j bhat_jk Y_j(r): dL/dr = sum_j (sum_k bhat_jk dF_a,k) grad Y_j(r);
     * r = 2 (n.v) n - v: dL/dn = 2 (dL/dr . n) v + 2 (n.v) dL/dr */
    double dY[3 * MAXSH], dr[3] = {0.0, 0.0, 0.0};
    orc_sh_grad(nsh, st->arg, dY);
    for (int j = 0; j < nsh; ++j) {
      double e = 0.0;
      for (int a = 0; a < na; ++a) e += st->bhat[j * na + a] * dz[nf + a];
      for (int q = 0; q < 3; ++q) dr[q] += e * dY[3 * j + q];
    }
    double rn = dr[0] * st->n[0] + dr[1] * st->n[1] + dr[2] * st->n[2];
    for (int a = 0; a < 3; ++a) dn[a] += 2.0 * rn * v[a] + 2.0 * st->c * dr[a];
    through_normal = 1;
  }
  if (through_normal) {
    /* n = g / max(|g|, 1e-30) */
    double dg[3];
    if (st->gn >= 1e-30) {
      double nd = dn[0] * st->n[0] + dn[1] * st->n[1] + dn[2] * st->n[2];
      for (int a = 0; a < 3; ++a) dg[a] = (dn[a] - nd * st->n[a]) / st->gn;
    } else {
      for (int a = 0; a < 3; ++a) dg[a] = dn[a] / 1e-30;
    }
    double h = 2.0 / (double)(f->R - 1);
    for (int a = 0; a < 3; ++a) {
      double xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]};
      xp[a] = clampd(x[a] + h, -1.0, 1.0);
      xm[a] = clampd(x[a] - h, -1.0, 1.0);
      double coef = dg[a] / (xp[a] - xm[a]);
      double mc = -coef;
      scatter_tri(g_sdf, f->R, 1, xp, &coef);
      scatter_tri(g_sdf, f->R, 1, xm, &mc);
    }
  }
}

static double sigm_neg(double tau, double s) { return 1.0 / (1.0 + exp(tau * s)); }

int orc_render_backward(const orc_field* f, const orc_render_opts* opt, int64_t B,
                        const double* rays_o, const double* rays_d, const double* dL_drgb,
                        double* g_sdf, double* g_feat, double* g_probes, double* g_mlp) {
  if (opt->n_samples < 2 || opt->n_samples > ORC_MAX_N) return -1;
  if (orc_field_check(f, opt->flags)) return -1;
  const int N = opt->n_samples;
  int failed = 0;
#pragma omp parallel
  {
  ray_state* r = ray_state_alloc(N);
  shade_state* st = (shade_state*)malloc(sizeof(shade_state));
  double(*C)[3] = (double(*)[3])malloc((size_t)N * sizeof(double[3]));
  double* ds = (double*)malloc((size_t)N * sizeof(double));
  if (!r || !st || !C || !ds) {
#pragma omp atomic write
    failed = 1;
  }
#pragma omp barrier
  if (!failed) {
#pragma omp for schedule(dynamic, 16)
  for (int64_t b = 0; b < B; ++b) {
    const double* dL = dL_drgb + 3 * b;
    if (dL[0] == 0.0 && dL[1] == 0.0 && dL[2] == 0.0) continue;
    for (int i = 0; i < N; ++i) {
      ds[i] = 0.0;
      C[i][0] = C[i][1] = C[i][2] = 0.0;
    }
    march(f, opt, rays_o + 3 * b, rays_d + 3 * b, r);
    if (r->hit) {
      for (int i = 0; i < N; ++i) {
        if (!(r->alpha[i] > 0.0)) continue;
        orc_shade(f, opt->flags, r->x[i], r->v, C[i], NULL);
      }
      /* reverse sweep: S_i = colour behind sample i (normalised by T_{i+1}) */
      double S[3] = {0, 0, 0};
      for (int i = N - 1; i >= 0; --i) {
        /* here S = S_i */
        if (r->alpha[i] > 0.0) {
          double dalpha = 0.0;
          for (int c = 0; c < 3; ++c) dalpha += dL[c] * r->T[i] * (C[i][c] - S[c]);
          double one_m = 1.0 - r->alpha[i];
          ds[i] += dalpha * one_m * opt->tau * sigm_neg(opt->tau, r->s[i]);
          ds[i + 1] += -dalpha * one_m * opt->tau * sigm_neg(opt->tau, r->s[i + 1]);
          /* colour path */
          double dC[3];
          for (int c = 0; c < 3; ++c) dC[c] = r->w[i] * dL[c];
          shade_full(f, opt->flags, r->x[i], r->v, st);
          shade_backward(f, opt->flags, r->x[i], r->v, st, dC, g_sdf, g_feat, g_probes, g_mlp);
        }
        /* alpha_i = 0 leaves S unchanged (S_{i-1} = S_i) */
        if (r->alpha[i] > 0.0)
          for (int c = 0; c < 3; ++c) S[c] = r->alpha[i] * C[i][c] + (1.0 - r->alpha[i]) * S[c];
      }
      for (int i = 0; i < N; ++i)
        if (ds[i] != 0.0) scatter_tri(g_sdf, f->R, 1, r->x[i], &ds[i]);
    }
  }
  }
  free(ds);
  free(C);
  free(st);
  free(r);
  }
  return failed ? -1 : 0;
}

/* ---------------------------------------------------------------------------
 * Photometric loss.  The paper uses a relatively weighted L2 (Eq. photo_loss);
 * the reading here is the L1 form L = mean over B x 3 of |c - c_gt|, with
 * dL/dc = sign(c - c_gt)/(3B) and sign(0) = 0.
 * ------------------------------------------------------------------------- */
double orc_l1_loss(int64_t B, const double* rgb, const double* target, double* dL_drgb) {
  double acc = 0.0;
  double inv = 1.0 / (3.0 * (double)B);
  for (int64_t i = 0; i < 3 * B; ++i) {
    double d = rgb[i] - target[i];
    acc += fabs(d);
    dL_drgb[i] = (d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0)) * inv;
  }
  return acc * inv;
}

/* ---------------------------------------------------------------------------
 * Regularisers (Sec. 3.3, Eqs. eikonal_reg, smooth_features, smooth_probes),
 * mean-normalised:
 *   L_Eik   = lambda_eik / M * sum over interior SDF nodes (|grad s| - 1)^2, grad s by
 *             central differences (s[n+e_a] - s[n-e_a]) / 2h, M = (R-2)^3;
 *   L_feat  = lambda / (3 R^2 (R-1) n_feat) * sum over axis-adjacent node pairs and
 *             channels of squared differences (each unordered pair once);
 *   L_probe = the same on the probe grid over its n_sh*n_ang coefficients.
 * Gradients are ADDED to g_*; losses[0..2] receive the three values.  The
 * derivative of |g| at g = 0 is taken as 0.
 * ------------------------------------------------------------------------- */
static double tv_grid(int R, int C, const double* F, double lam, double* gF) {
  double npairs = 3.0 * (double)R * R * (R - 1);
  double scale = lam / (npairs * C);
  double acc = 0.0;
  for (int64_t k = 0; k < R; ++k)
    for (int64_t j = 0; j < R; ++j)
      for (int64_t i = 0; i < R; ++i) {
        int64_t n = (k * R + j) * R + i;
        int64_t nb[3] = {i + 1 < R ? n + 1 : -1, j + 1 < R ? n + R : -1,
                         k + 1 < R ? n + (int64_t)R * R : -1};
        for (int a = 0; a < 3; ++a) {
          if (nb[a] < 0) continue;
          for (int c = 0; c < C; ++c) {
            double d = F[nb[a] * C + c] - F[n * C + c];
            acc += d * d;
            gF[nb[a] * C + c] += 2.0 * scale * d;
            gF[n * C + c] -= 2.0 * scale * d;
          }
        }
      }
  return scale * acc;
}

void orc_regularizers(int R, int P, int n_feat, int n_pc, const double* sdf, const double* feat,
                      const double* probes, double lambda_eik, double lambda_tv_feat,
                      double lambda_tv_probe, double* g_sdf, double* g_feat, double* g_probes,
                      double losses[3]) {
  double h = 2.0 / (double)(R - 1);
  double M = (double)(R - 2) * (R - 2) * (R - 2);
  double acc = 0.0;
  int64_t st[3] = {1, R, (int64_t)R * R};
  for (int64_t k = 1; k < R - 1; ++k)
    for (int64_t j = 1; j < R - 1; ++j)
      for (int64_t i = 1; i < R - 1; ++i) {
        int64_t n = (k * R + j) * R + i;
        double g[3];
        for (int a = 0; a < 3; ++a) g[a] = (sdf[n + st[a]] - sdf[n - st[a]]) / (2.0 * h);
        double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        acc += (gn - 1.0) * (gn - 1.0);
        if (gn > 0.0) {
          double coef = lambda_eik / M * 2.0 * (gn - 1.0) / gn;
          for (int a = 0; a < 3; ++a) {
            g_sdf[n + st[a]] += coef * g[a] / (2.0 * h);
            g_sdf[n - st[a]] -= coef * g[a] / (2.0 * h);
          }
        }
      }
  losses[0] = lambda_eik / M * acc;
  losses[1] = tv_grid(R, n_feat, feat, lambda_tv_feat, g_feat);
  losses[2] = tv_grid(P, n_pc, probes, lambda_tv_probe, g_probes);
}

/* ---------------------------------------------------------------------------
 * Adam (Kingma & Ba 2015, Algorithm 1, bias-corrected), the optimiser named in
 * Sec. 3.4 with the moments of Supplementary Sec. A.  step is 1-based.
 * ------------------------------------------------------------------------- */
void orc_adam(int64_t n, double* p, const double* g, double* m, double* v, int64_t step,
              double lr, double beta1, double beta2, double eps) {
  double bc1 = 1.0 - pow(beta1, (double)step);
  double bc2 = 1.0 - pow(beta2, (double)step);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
    double mh = m[i] / bc1;
    double vh = v[i] / bc2;
    p[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* ---------------------------------------------------------------------------
 * One optimiser step over all trained parameters (Sec. 3.4: raw SDF, spatial
 * features, probe coefficients, MLP weights): total gradient = render
 * gradient + regulariser gradient, then Adam per group with its own learning
 * rate.  m and v are concatenated in the order sdf | feat | probes | mlp.
 * ------------------------------------------------------------------------- */
void orc_grid_step(int R, int P, int n_feat, int n_pc, int n_mlp, double* sdf, double* feat,
                   double* probes, double* mlp, const double* g_sdf, const double* g_feat,
                   const double* g_probes, const double* g_mlp, double* m, double* v,
                   int64_t step, const orc_step_opts* opt, double losses[3]) {
  int64_t ns = (int64_t)R * R * R, nf = ns * n_feat, np = (int64_t)P * P * P * n_pc;
  double* G = (double*)calloc((size_t)(ns + nf + np), sizeof(double));
  memcpy(G, g_sdf, (size_t)ns * sizeof(double));
  memcpy(G + ns, g_feat, (size_t)nf * sizeof(double));
  memcpy(G + ns + nf, g_probes, (size_t)np * sizeof(double));
  orc_regularizers(R, P, n_feat, n_pc, sdf, feat, probes, opt->lambda_eik, opt->lambda_tv_feat,
                   opt->lambda_tv_probe, G, G + ns, G + ns + nf, losses);
  orc_adam(ns, sdf, G, m, v, step, opt->lr_sdf, opt->beta1, opt->beta2, opt->eps);
  orc_adam(nf, feat, G + ns, m + ns, v + ns, step, opt->lr_feat, opt->beta1, opt->beta2,
           opt->eps);
  orc_adam(np, probes, G + ns + nf, m + ns + nf, v + ns + nf, step, opt->lr_probe, opt->beta1,
           opt->beta2, opt->eps);
  orc_adam(n_mlp, mlp, g_mlp, m + ns + nf + np, v + ns + nf + np, step, opt->lr_mlp,
           opt->beta1, opt->beta2, opt->eps);
  free(G);
}

/* ---------------------------------------------------------------------------
 * Sphere-traced inference render.  The paper's real-time path shades voxels
 * and volume-renders them (Supplementary "Performance Analysis"); the reading
 * used here marches t <- t + s(x) from the box entry until s < eps (hit) or
 * t > t_f (miss), at most max_steps evaluations, then shades the hit point
 * once with the same colour model (v = -d).  Pixel rays come from pinhole
 * cameras: cams[v] = c2w (3x4 row-major), fx, fy, cx, cy; the camera-space
 * direction of pixel (px, py) is ((px+.5-cx)/fx, (py+.5-cy)/fy, 1).
 * pixel_ids index views x H x W (v*H*W + py*W + px).  margin = closest
 * approach of a decision to its threshold (|s - eps|, |t - t_f|).
 * ------------------------------------------------------------------------- */
int orc_sphere_trace(const orc_field* f, int32_t flags, double eps, int32_t max_steps,
                     int32_t V, const double* cams, int32_t W, int32_t H,
                     const int64_t* pixel_ids, int64_t n_pix, double* out, double* t_hit,
                     int32_t* steps, double* margin) {
  (void)V;
  if (orc_field_check(f, flags)) return -1;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t q = 0; q < n_pix; ++q) {
    int64_t id = pixel_ids[q];
    int64_t vi = id / ((int64_t)W * H);
    int64_t rem = id % ((int64_t)W * H);
    int py = (int)(rem / W), px = (int)(rem % W);
    const double* cam = cams + 16 * vi;
    double dc[3] = {(px + 0.5 - cam[14]) / cam[12], (py + 0.5 - cam[15]) / cam[13], 1.0};
    double o[3], d[3];
    for (int r = 0; r < 3; ++r) {
      d[r] = cam[4 * r + 0] * dc[0] + cam[4 * r + 1] * dc[1] + cam[4 * r + 2] * dc[2];
      o[r] = cam[4 * r + 3];
    }
    double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int r = 0; r < 3; ++r) d[r] /= dn;
    double tn, tf, mg = INFINITY, th = -1.0;
    int hit = 0, k = 0;
    double x[3];
    if (orc_ray_box(o, d, &tn, &tf)) {
      double t = tn;
      for (k = 0; k < max_steps; ++k) {
        for (int a = 0; a < 3; ++a) x[a] = clampd(o[a] + t * d[a], -1.0, 1.0);
        double s;
        orc_trilinear(f->sdf, f->R, 1, x, &s);
        mg = fmin(mg, fabs(s - eps));
        if (s < eps) {
          hit = 1;
          break;
        }
        t += s;
        mg = fmin(mg, fabs(t - tf));
        if (t > tf) break;
      }
      if (hit) th = t;
    }
    double C[3] = {0, 0, 0};
    if (hit) {
      double v[3] = {-d[0], -d[1], -d[2]};
      orc_shade(f, flags, x, v, C, NULL);
    }
    for (int c = 0; c < 3; ++c) out[3 * q + c] = C[c];
    if (t_hit) t_hit[q] = th;
    if (steps) steps[q] = k;
    if (margin) margin[q] = mg;
  }
  return 0;
}

/* ===========================================================================
 * The smoothed SDF and the remaining regularisers (Sec. 3.3, Eqs. smooth_sdf,
 * eikonal_reg, smmoth_normals, photo_loss).
 * ======================================================================== */

/* 5-tap Gaussian of the 5^3 kernel G (Sec. 3.3 convolves the raw SDF with a 5^3
 * Gaussian; the paper gives no width).  Reading: separable, w[k+2] proportional to
 * exp(-k^2 / (2 sigma^2)) for k = -2..2, normalised to sum 1. */
void orc_gauss5(double sigma, double w[5]) {
  double sum = 0.0;
  for (int k = -2; k <= 2; ++k) {
    w[k + 2] = exp(-(double)(k * k) / (2.0 * sigma * sigma));
    sum += w[k + 2];
  }
  for (int k = 0; k < 5; ++k) w[k] /= sum;
}

static int64_t clampi(int64_t i, int64_t R) { return i < 0 ? 0 : (i >= R ? R - 1 : i); }

/* s = G(shat): every node sums the 125 nodes around it, weight w_a w_b w_c; a node
 * index beyond the grid reads the edge node (reading: replicate, so constants are
 * reproduced). */
void orc_smooth(int R, double sigma, const double* shat, double* s) {
  double w[5];
  orc_gauss5(sigma, w);
  for (int64_t k = 0; k < R; ++k)
    for (int64_t j = 0; j < R; ++j)
      for (int64_t i = 0; i < R; ++i) {
        double acc = 0.0;
        for (int c = -2; c <= 2; ++c)
          for (int b = -2; b <= 2; ++b)
            for (int a = -2; a <= 2; ++a) {
              int64_t n = (clampi(k + c, R) * R + clampi(j + b, R)) * R + clampi(i + a, R);
              acc += w[a + 2] * w[b + 2] * w[c + 2] * shat[n];
            }
        s[(k * R + j) * R + i] = acc;
      }
}

/* out = G^T y: each term of orc_smooth, taken in reverse (y at the output node,
 * added to the node it read). */
void orc_smooth_T(int R, double sigma, const double* y, double* out) {
  double w[5];
  orc_gauss5(sigma, w);
  int64_t n3 = (int64_t)R * R * R;
  for (int64_t q = 0; q < n3; ++q) out[q] = 0.0;
  for (int64_t k = 0; k < R; ++k)
    for (int64_t j = 0; j < R; ++j)
      for (int64_t i = 0; i < R; ++i) {
        double yv = y[(k * R + j) * R + i];
        for (int c = -2; c <= 2; ++c)
          for (int b = -2; b <= 2; ++b)
            for (int a = -2; a <= 2; ++a) {
              int64_t n = (clampi(k + c, R) * R + clampi(j + b, R)) * R + clampi(i + a, R);
              out[n] += w[a + 2] * w[b + 2] * w[c + 2] * yv;
            }
      }
}

/* Regularisers of the raw SDF shat through s = G(shat) (smooth != 0) or s = shat:
 *   L_sdf    = lambda_sdf / R^3 * sum over nodes (s - shat)^2               (Eq. smooth_sdf)
 *   L_Eik    = lambda_eik / (R-2)^3 * sum over interior nodes (|g| - 1)^2    (Eq. eikonal_reg)
 *   L_normal = lambda_normal / Np * sum over axis-adjacent pairs of interior
 *              nodes |n_a - n_b|^2, n = g / |g|, Np = 3 (R-2)^2 (R-3)        (Eq. smmoth_normals)
 * with g the central differences (s[n+e] - s[n-e]) / 2h of s (mean-normalised
 * sums; the normal term reads grad n as forward differences of the unit normal
 * field between neighbouring nodes).  With `weighted`, the gradient of these
 * terms with respect to s at node m (and the direct term of L_sdf with respect
 * to shat_m) is multiplied by 1 / (1 + 5 |s_m|) (Sec. 3.3's factor on the
 * gradients of the per-voxel regularisations).
 *   g_s     [R^3] in:  the render gradient with respect to s
 *   g_shat  [R^3] out: total gradient with respect to shat,
 *           G^T (g_s + weighted dL/ds) + weighted dL/dshat (direct)
 *   s_out   [R^3] out (nullable): s
 *   losses  [3] out: L_sdf, L_Eik, L_normal
 * The derivative of |g| at g = 0 is taken as 0. */
void orc_sdf_regs(int R, const double* shat, int smooth, double sigma, int weighted,
                  double lambda_sdf, double lambda_eik, double lambda_normal, const double* g_s,
                  double* g_shat, double* s_out, double losses[3]) {
  int64_t n3 = (int64_t)R * R * R;
  double h = 2.0 / (double)(R - 1);
  int64_t st[3] = {1, R, (int64_t)R * R};
  double* s = (double*)malloc((size_t)n3 * sizeof(double));
  double* gr = (double*)calloc((size_t)n3, sizeof(double));  /* dL_reg/ds */
  double* gd = (double*)calloc((size_t)n3, sizeof(double));  /* dL_sdf/dshat, direct */
  double* nrm = (double*)calloc((size_t)n3 * 3, sizeof(double));
  double* gnm = (double*)calloc((size_t)n3, sizeof(double));
  double* dn = (double*)calloc((size_t)n3 * 3, sizeof(double));
  if (smooth) orc_smooth(R, sigma, shat, s);
  else memcpy(s, shat, (size_t)n3 * sizeof(double));
  /* L_sdf */
  double acc_sdf = 0.0;
  for (int64_t q = 0; q < n3; ++q) {
    double d = s[q] - shat[q];
    acc_sdf += d * d;
    gr[q] += 2.0 * lambda_sdf / (double)n3 * d;
    gd[q] -= 2.0 * lambda_sdf / (double)n3 * d;
  }
  /* gradients and unit normals at interior nodes */
  double M = (double)(R - 2) * (R - 2) * (R - 2);
  double acc_eik = 0.0;
  for (int64_t k = 1; k < R - 1; ++k)
    for (int64_t j = 1; j < R - 1; ++j)
      for (int64_t i = 1; i < R - 1; ++i) {
        int64_t n = (k * R + j) * R + i;
        double g[3];
        for (int a = 0; a < 3; ++a) g[a] = (s[n + st[a]] - s[n - st[a]]) / (2.0 * h);
        double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        gnm[n] = gn;
        for (int a = 0; a < 3; ++a) nrm[3 * n + a] = g[a] / fmax(gn, 1e-30);
        acc_eik += (gn - 1.0) * (gn - 1.0);
        if (gn > 0.0) {
          double coef = lambda_eik / M * 2.0 * (gn - 1.0) / gn;
          for (int a = 0; a < 3; ++a) {
            gr[n + st[a]] += coef * g[a] / (2.0 * h);
            gr[n - st[a]] -= coef * g[a] / (2.0 * h);
          }
        }
      }
  /* L_normal: pairs (n, n + e_a) with both nodes interior */
  double Np = 3.0 * (double)(R - 2) * (R - 2) * (R - 3);
  double acc_n = 0.0;
  if (R > 3) {
    for (int64_t k = 1; k < R - 1; ++k)
      for (int64_t j = 1; j < R - 1; ++j)
        for (int64_t i = 1; i < R - 1; ++i) {
          int64_t n = (k * R + j) * R + i;
          int64_t idx[3] = {i, j, k};
          for (int a = 0; a < 3; ++a) {
            if (idx[a] + 1 > R - 2) continue;
            int64_t m2 = n + st[a];
            for (int c = 0; c < 3; ++c) {
              double d = nrm[3 * n + c] - nrm[3 * m2 + c];
              acc_n += d * d;
              dn[3 * n + c] += 2.0 * lambda_normal / Np * d;
              dn[3 * m2 + c] -= 2.0 * lambda_normal / Np * d;
            }
          }
        }
    /* through n = g / |g| and the central differences */
    for (int64_t k = 1; k < R - 1; ++k)
      for (int64_t j = 1; j < R - 1; ++j)
        for (int64_t i = 1; i < R - 1; ++i) {
          int64_t n = (k * R + j) * R + i;
          if (gnm[n] <= 0.0) continue;
          double nd = 0.0;
          for (int c = 0; c < 3; ++c) nd += dn[3 * n + c] * nrm[3 * n + c];
          for (int a = 0; a < 3; ++a) {
            double dg = (dn[3 * n + a] - nd * nrm[3 * n + a]) / gnm[n];
            gr[n + st[a]] += dg / (2.0 * h);
            gr[n - st[a]] -= dg / (2.0 * h);
          }
        }
  }
  if (weighted)
    for (int64_t q = 0; q < n3; ++q) {
      double wq = 1.0 / (1.0 + 5.0 * fabs(s[q]));
      gr[q] *= wq;
      gd[q] *= wq;
    }
  /* back to shat */
  for (int64_t q = 0; q < n3; ++q) gr[q] += g_s[q];
  if (smooth) orc_smooth_T(R, sigma, gr, g_shat);
  else memcpy(g_shat, gr, (size_t)n3 * sizeof(double));
  for (int64_t q = 0; q < n3; ++q) g_shat[q] += gd[q];
  if (s_out) memcpy(s_out, s, (size_t)n3 * sizeof(double));
  losses[0] = lambda_sdf / (double)n3 * acc_sdf;
  losses[1] = lambda_eik / M * acc_eik;
  losses[2] = R > 3 ? lambda_normal / Np * acc_n : 0.0;
  free(s);
  free(gr);
  free(gd);
  free(nrm);
  free(gnm);
  free(dn);
}

/* One optimiser step with the smoothed SDF: sdf holds shat; g_s is the render
 * gradient with respect to s = G(shat).  The SDF gradient is orc_sdf_regs's;
 * features and probes take the smoothness terms of orc_regularizers; then Adam
 * per group (as orc_grid_step).  losses[5] = L_sdf, L_Eik, L_normal, L_feat,
 * L_probe; s_new (nullable) receives G of the updated shat (or a copy of it
 * without smoothing). */
void orc_grid_step_ext(int R, int P, int n_feat, int n_pc, int n_mlp, double* sdf, double* feat,
                       double* probes, double* mlp, const double* g_s, const double* g_feat,
                       const double* g_probes, const double* g_mlp, double* m, double* v,
                       int64_t step, const orc_step_ext* opt, double losses[5], double* s_new) {
  const orc_step_opts* b = &opt->base;
  int64_t ns = (int64_t)R * R * R, nf = ns * n_feat, np = (int64_t)P * P * P * n_pc;
  double* G = (double*)calloc((size_t)(ns + nf + np), sizeof(double));
  memcpy(G + ns, g_feat, (size_t)nf * sizeof(double));
  memcpy(G + ns + nf, g_probes, (size_t)np * sizeof(double));
  orc_sdf_regs(R, sdf, opt->smooth, opt->sigma, opt->weighted, opt->lambda_sdf, b->lambda_eik,
               opt->lambda_normal, g_s, G, NULL, losses);
  losses[3] = tv_grid(R, n_feat, feat, b->lambda_tv_feat, G + ns);
  losses[4] = tv_grid(P, n_pc, probes, b->lambda_tv_probe, G + ns + nf);
  orc_adam(ns, sdf, G, m, v, step, b->lr_sdf, b->beta1, b->beta2, b->eps);
  orc_adam(nf, feat, G + ns, m + ns, v + ns, step, b->lr_feat, b->beta1, b->beta2, b->eps);
  orc_adam(np, probes, G + ns + nf, m + ns + nf, v + ns + nf, step, b->lr_probe, b->beta1,
           b->beta2, b->eps);
  orc_adam(n_mlp, mlp, g_mlp, m + ns + nf + np, v + ns + nf + np, step, b->lr_mlp, b->beta1,
           b->beta2, b->eps);
  if (s_new) {
    if (opt->smooth) orc_smooth(R, opt->sigma, sdf, s_new);
    else memcpy(s_new, sdf, (size_t)ns * sizeof(double));
  }
  free(G);
}

/* Relatively weighted L2 photometric loss (Eq. photo_loss with the per-pixel weight
 * (max(c, c_gt) + eps)^-1 on its gradient, the loss scaled by lambda and divided by
 * the number of images in the batch, Supplementary "Scheduling").  Reading: the
 * weight is held constant (its own derivative is not taken) and applies per
 * channel:  L = lambda / n_images * sum (c - c_gt)^2 / (max(c, c_gt) + eps),
 * dL/dc = 2 lambda / n_images * (c - c_gt) / (max(c, c_gt) + eps). */
double orc_l2rel_loss(int64_t B, const double* rgb, const double* target, double lambda,
                      double eps, double n_images, double* dL_drgb) {
  double acc = 0.0, sc = lambda / n_images;
  for (int64_t i = 0; i < 3 * B; ++i) {
    double d = rgb[i] - target[i];
    double wgt = 1.0 / (fmax(rgb[i], target[i]) + eps);
    acc += d * d * wgt;
    dL_drgb[i] = 2.0 * sc * d * wgt;
  }
  return sc * acc;
}

/* threads of the OpenMP loops (the benchmark's CPU baseline times 1 and all) */
void orc_set_threads(int n) { omp_set_num_threads(n); }
int orc_max_threads(void) { return omp_get_max_threads(); }

/* ===========================================================================
 * Real-time render of the supplementary "Performance Analysis": a shading
 * pass assigns a colour to every voxel, then a volume-rendering pass samples
 * the SDF and that colour field along the rays.
 * ======================================================================== */

/* Colour of the voxels seen from a camera centre.  Readings: a voxel is a grid
 * node x_m; it is shaded iff |s_m| <= band (the others hold colour 0); its view
 * direction points from the node to the camera, v = (c - x_m) / |c - x_m|; its
 * colour is the colour model at x_m (orc_shade).
 *   col [R^3][3] out */
void orc_voxel_shade(const orc_field* f, int32_t flags, const double cam_centre[3], double band,
                     double* col) {
  int R = f->R;
  double h = 2.0 / (double)(R - 1);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t k = 0; k < R; ++k)
    for (int64_t j = 0; j < R; ++j)
      for (int64_t i = 0; i < R; ++i) {
        int64_t n = (k * R + j) * R + i;
        double* c = col + 3 * n;
        c[0] = c[1] = c[2] = 0.0;
        if (!(fabs(f->sdf[n]) <= band)) continue;
        double x[3] = {-1.0 + i * h, -1.0 + j * h, -1.0 + k * h};
        double v[3], vn = 0.0;
        for (int a = 0; a < 3; ++a) {
          v[a] = cam_centre[a] - x[a];
          vn += v[a] * v[a];
        }
        vn = sqrt(vn);
        for (int a = 0; a < 3; ++a) v[a] /= vn;
        orc_shade(f, flags, x, v, c, NULL);
      }
}

/* Volume render of pinhole pixels (the camera layout of orc_sphere_trace):
 * samples, skip rule and NeuS weights as orc_render_forward (the field's sdf),
 * C_i = trilinear interpolation of the voxel colours col [R^3][3] at x_i.
 *   out [n_pix][3], margin [n_pix] (nullable, as orc_render_forward) */
int orc_volume_render(const orc_field* f, const double* col, const orc_render_opts* opt,
                      const double* cam, int32_t W, int32_t H, const int64_t* pixel_ids,
                      int64_t n_pix, double* out, double* margin) {
  if (opt->n_samples < 2 || opt->n_samples > ORC_MAX_N) return -1;
  int failed = 0;
#pragma omp parallel
  {
  ray_state* r = ray_state_alloc(opt->n_samples);
  if (!r) {
#pragma omp atomic write
    failed = 1;
  }
#pragma omp barrier
  if (!failed) {
#pragma omp for schedule(dynamic, 16)
  for (int64_t q = 0; q < n_pix; ++q) {
    int64_t id = pixel_ids[q];
    int py = (int)(id / W), px = (int)(id % W);
    (void)H;
    double dc[3] = {(px + 0.5 - cam[14]) / cam[12], (py + 0.5 - cam[15]) / cam[13], 1.0};
    double o[3], d[3];
    for (int a = 0; a < 3; ++a) {
      d[a] = cam[4 * a + 0] * dc[0] + cam[4 * a + 1] * dc[1] + cam[4 * a + 2] * dc[2];
      o[a] = cam[4 * a + 3];
    }
    march(f, opt, o, d, r);
    double c3[3] = {0, 0, 0};
    if (r->hit) {
      for (int i = 0; i < r->N; ++i) {
        if (!(r->alpha[i] > 0.0)) continue;
        double C[3];
        orc_trilinear(col, f->R, 3, r->x[i], C);
        for (int c = 0; c < 3; ++c) c3[c] += r->w[i] * C[c];
      }
    }
    for (int c = 0; c < 3; ++c) out[3 * q + c] = c3[c];
    if (margin) margin[q] = r->hit ? r->margin : INFINITY;
  }
  }
  free(r);
  }
  return failed ? -1 : 0;
}
