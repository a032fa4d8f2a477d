// Per-sample shading of the ProbeSDF render step and its reverse mode, the
// per-ray setup, and the wave-level MLP / weight-gradient helpers shared by the
// forward, backward and sphere-tracing kernels.
//
// Precision: ray parameters, sample positions and cell coordinates are FP64
// (the opacity multiplies SDF errors by tau, so an FP32 position at t ~ 3
// would dominate the error budget); interpolation weights are rounded to FP32
// once; every value read from the grids and every downstream quantity is FP32.
#pragma once

#include "device.h"
#include "kernels.h"

namespace psdf {

constexpr int BLOCK = 256;
constexpr int WAVES = BLOCK / 64;

// ---------------------------------------------------------------------------
// ray setup in FP64: unit direction, ray / cube interval, sample spacing
// ---------------------------------------------------------------------------
struct RayD {
  double o[3], d[3];
  double tn, dt;
};

__device__ __forceinline__ bool ray_setup_d(float ox, float oy, float oz, float dx, float dy,
                                            float dz, int N, RayD& r) {
  const double ddx = dx, ddy = dy, ddz = dz;
  const double dn = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
  r.o[0] = ox;
  r.o[1] = oy;
  r.o[2] = oz;
  r.d[0] = ddx / dn;
  r.d[1] = ddy / dn;
  r.d[2] = ddz / dn;
  double t0 = -INFINITY, t1 = INFINITY;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
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

__device__ __forceinline__ void sample_pos(const RayD& r, double ti, double x[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) x[k] = fmin(fmax(fma(ti, r.d[k], r.o[k]), -1.0), 1.0);
}

__device__ __forceinline__ double sample_t(const RayD& r, int i) {
  return fma((double)i + 0.5, r.dt, r.tn);
}

// March state: the continuous cell coordinate u = (x+1)/h of the current sample,
// advanced by du = dt d / h per sample (FP64; after N <= 4096 steps the drift is
// ~1e-12 of a cell, far below the FP32 rounding of the weights).
struct MarchU {
  double u[3], du[3];
};

__device__ __forceinline__ void march_init(const RayD& r, double inv_h, MarchU& m) {
  double x[3];
  sample_pos(r, sample_t(r, 0), x);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    m.u[k] = (x[k] + 1.0) * inv_h;
    m.du[k] = r.dt * r.d[k] * inv_h;
  }
}

__device__ __forceinline__ Cell march_cell(const MarchU& m, int R) {
  Cell c;
  int k[3];
  float f[3];
  const double umax = (double)(R - 1), kmax = (double)(R - 2);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double u = fmin(fmax(m.u[a], 0.0), umax);  // the cube clamp, in cell units
    const double fl = fmin(floor(u), kmax);
    k[a] = (int)fl;
    f[a] = (float)(u - fl);
  }
  c.fx = f[0];
  c.fy = f[1];
  c.fz = f[2];
  c.base = (k[2] * R + k[1]) * R + k[0];
  return c;
}

__device__ __forceinline__ void march_step(MarchU& m) {
#pragma unroll
  for (int k = 0; k < 3; ++k) m.u[k] += m.du[k];
}

// ---------------------------------------------------------------------------
// Empty-space skipping.  Brick bounds hold, per block of 8^3 cells, the min and
// max of the SDF nodes those cells interpolate.  A trilinear value is a convex
// combination of its corners, so a sample whose brick has min > thr or
// max < -thr cannot pass the skip rule |s| <= thr; its corners are not read
// unless the previous sample is active and needs s_{i+1} for its opacity.
// The FP32 interpolation stays within 9 ulp of max |corner| of the convex
// value, which the 1e-6 relative margin covers, so skipping never changes a
// result.
// ---------------------------------------------------------------------------
constexpr int BRICK_SHIFT = 3;

struct Bricks {
  const float2* __restrict__ b;  // [nb][nb][nb] (min, max); nullptr: no skipping
  int nb;
  float thr;
};

__host__ __device__ inline Bricks make_bricks(const float* bounds, int R, float skip_thr) {
  Bricks k;
  k.b = skip_thr > 0.f ? reinterpret_cast<const float2*>(bounds) : nullptr;
  k.nb = ((R - 2) >> BRICK_SHIFT) + 1;
  k.thr = skip_thr;
  return k;
}

// cell of the march coordinate and the flat index of its brick
__device__ __forceinline__ Cell march_cell_b(const MarchU& m, int R, int nb, int& brick) {
  Cell c;
  int k[3];
  float f[3];
  const double umax = (double)(R - 1), kmax = (double)(R - 2);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double u = fmin(fmax(m.u[a], 0.0), umax);
    const double fl = fmin(floor(u), kmax);
    k[a] = (int)fl;
    f[a] = (float)(u - fl);
  }
  c.fx = f[0];
  c.fy = f[1];
  c.fz = f[2];
  c.base = (k[2] * R + k[1]) * R + k[0];
  brick = ((k[2] >> BRICK_SHIFT) * nb + (k[1] >> BRICK_SHIFT)) * nb + (k[0] >> BRICK_SHIFT);
  return c;
}

__device__ __forceinline__ float2 brick_load(const Bricks& K, bool on, int brick) {
  if (!K.b) return make_float2(0.f, 0.f);
  return K.b[on ? brick : 0];
}

// may a sample in a brick with these bounds pass the skip rule
__device__ __forceinline__ bool brick_may(const Bricks& K, float2 mm) {
  if (!K.b) return true;
  const float t = K.thr + 1e-6f * fmaxf(fabsf(mm.x), fabsf(mm.y));
  return mm.x <= t && mm.y >= -t;
}

// corners of a cell when `need`, else of node 0 (one shared line, value unused)
template <typename T>
__device__ __forceinline__ CellVals fetch_cell_if(const T* __restrict__ g, int R, const Cell& c,
                                                  bool need) {
  Cell q = c;
  q.base = need ? c.base : 0;
  return fetch_cell(g, R, q);
}

// March of one ray per lane over samples i = 0 .. N-1 with loads in flight
// ahead of use: the bounds of sample i+2 and the corners of sample i+1.
//   s0 = s_i (valid when m0), v1 = corners of sample i+1 (fetched when m0 || m1)
// Where no lane of the wave needs the corners of a sample (all in skipped
// bricks), the wave neither fetches nor interpolates them: w1 (wave-uniform)
// says whether v1 holds a fetch.
struct MarchState {
  MarchU mu;
  Cell c2;
  int k2;
  float2 b2;
  CellVals v1;
  float s0;
  bool m0, m1;
  bool w1;
};

// Begin at sample F (wave-uniform): the coordinate is advanced from sample 0 by the
// same F additions a march from sample 0 makes, so every later value is identical.
template <typename ST>
__device__ __forceinline__ void march_begin_at(const ST* __restrict__ sdf, int R, const Bricks& K,
                                               const RayD& r, double inv_h, bool hit, int N, int F,
                                               MarchState& M) {
  march_init(r, inv_h, M.mu);
  for (int j = 0; j < F; ++j) march_step(M.mu);
  int k0, k1;
  const Cell c0 = march_cell_b(M.mu, R, K.nb, k0);
  march_step(M.mu);
  const Cell c1 = march_cell_b(M.mu, R, K.nb, k1);
  const float2 b0 = brick_load(K, hit, k0), b1 = brick_load(K, hit, k1);
  march_step(M.mu);
  M.c2 = march_cell_b(M.mu, R, K.nb, M.k2);
  M.b2 = brick_load(K, hit && N > F + 2, M.k2);
  M.m0 = hit && brick_may(K, b0);
  M.m1 = hit && N > F + 1 && brick_may(K, b1);
  Cell q0 = c0;
  q0.base = M.m0 ? c0.base : 0;
  M.s0 = tri1(sdf, R, q0);
  M.v1 = fetch_cell_if(sdf, R, c1, M.m0 || M.m1);
  M.w1 = true;
}

template <typename ST>
__device__ __forceinline__ void march_begin(const ST* __restrict__ sdf, int R, const Bricks& K,
                                            const RayD& r, double inv_h, bool hit, int N,
                                            MarchState& M) {
  march_begin_at(sdf, R, K, r, inv_h, hit, N, 0, M);
}

// Samples of a ray that may lie in a brick passing the bounds test.  `box` holds
// the brick coordinates (min x, y, z, max x, y, z) of every such brick; the march
// coordinate of sample i is u_0 + i du, so the samples inside the box, widened by
// one cell, form one interval of i, returned widened by one sample (the
// accumulated coordinate differs from u_0 + i du by ~1e-12 of a cell).  Empty:
// lo = N, hi = -1.
__device__ __forceinline__ void may_range(const RayD& r, double inv_h, int N, bool hit,
                                          const int* box, int& lo, int& hi) {
  lo = N;
  hi = -1;
  if (!hit || box[3] < box[0]) return;
  MarchU m;
  march_init(r, inv_h, m);
  double tlo = -1e300, thi = 1e300;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double cells = (double)(1 << BRICK_SHIFT);  // cells per brick edge
    const double blo = cells * box[a] - 1.0, bhi = cells * (box[3 + a] + 1) + 1.0;
    const double u = m.u[a], d = m.du[a];
    if (d > 0.0) {
      tlo = fmax(tlo, (blo - u) / d);
      thi = fmin(thi, (bhi - u) / d);
    } else if (d < 0.0) {
      tlo = fmax(tlo, (bhi - u) / d);
      thi = fmin(thi, (blo - u) / d);
    } else if (u < blo || u > bhi) {
      return;
    }
  }
  const double l = fmax(floor(tlo) - 1.0, 0.0), h = fmin(ceil(thi) + 1.0, (double)(N - 1));
  if (!(l <= h)) return;
  lo = (int)l;
  hi = (int)h;
}

// Step i (0 <= i < N-1): returns s_i, s_{i+1} and whether sample i may be
// active, and moves the state to sample i+1.
template <typename ST>
__device__ __forceinline__ void march_next(const ST* __restrict__ sdf, int R, const Bricks& K,
                                           bool hit, int i, int N, MarchState& M, float& s_i,
                                           float& s_n, bool& may_i) {
  // s_{i+1}, from the corners fetched one step ago (unused where none were)
  s_n = 0.f;
  if (M.w1) s_n = interp_cell(M.v1);  // wave-uniform
  bool m2 = false;
  if (i + 2 < N) {  // wave-uniform
    m2 = hit && brick_may(K, M.b2);
    const bool need = M.m1 || m2;
    const Cell c = M.c2;
    // the bounds of sample i+3 go out before the corners of sample i+2
    if (i + 3 < N) {
      march_step(M.mu);
      M.c2 = march_cell_b(M.mu, R, K.nb, M.k2);
      M.b2 = brick_load(K, hit, M.k2);
    }
    M.w1 = __ballot(need) != 0;
    if (M.w1) M.v1 = fetch_cell_if(sdf, R, c, need);
  }
  s_i = M.s0;
  may_i = M.m0;
  M.s0 = s_n;
  M.m0 = M.m1;
  M.m1 = m2;
}

// align-corners cell of an FP64 point; the weights are rounded to FP32 once
__device__ __forceinline__ void axis_cell_d(double x, double inv_h, double kmax, int& k, float& f) {
  const double u = (x + 1.0) * inv_h;
  const double fl = fmin(fmax(floor(u), 0.0), kmax);
  k = (int)fl;
  f = (float)(u - fl);
}

__device__ __forceinline__ Cell cell_d(const double x[3], int R, double inv_h) {
  Cell c;
  int kx, ky, kz;
  const double kmax = (double)(R - 2);
  axis_cell_d(x[0], inv_h, kmax, kx, c.fx);
  axis_cell_d(x[1], inv_h, kmax, ky, c.fy);
  axis_cell_d(x[2], inv_h, kmax, kz, c.fz);
  c.base = (kz * R + ky) * R + kx;
  return c;
}

// Probe cells are binned (backward, taped forward) under a key that keeps space
// together: blocks of 2x2x2 cells in row-major order, the 8 cells of a block
// consecutive.  Cells span 0..P-2 per axis, so P/2 blocks per axis.
// key of the probe cell with flat corner index `base`
__device__ __forceinline__ int probe_key(int base, int P) {
  const int x = base % P, yz = base / P, y = yz % P, z = yz / P;
  const int nb = P / 2;
  const int blk = ((z >> 1) * nb + (y >> 1)) * nb + (x >> 1);
  return blk * 8 + ((x & 1) | ((y & 1) << 1) | ((z & 1) << 2));
}

// flat corner index of the probe cell with key `key`
__device__ __forceinline__ int probe_cell_of_key(int key, int P) {
  const int nb = P / 2;
  const int blk = key >> 3;
  const int bx = blk % nb, byz = blk / nb, by = byz % nb, bz = byz / nb;
  const int x = 2 * bx + (key & 1), y = 2 * by + ((key >> 1) & 1), z = 2 * bz + ((key >> 2) & 1);
  return (z * P + y) * P + x;
}

// Lanes with `on` set, grouped by equal `key`: returns the group's lane mask
// to every member; the lowest member is the group's leader.  One iteration per
// distinct key of the wave.
template <typename F>
__device__ __forceinline__ void for_each_key_group(bool on, int key, F&& f) {
  uint64_t todo = __ballot(on);
  while (todo) {
    const int leader = __builtin_ctzll(todo);
    const int k = __builtin_amdgcn_readlane(key, leader);
    const uint64_t grp = __ballot(on && key == k);
    f(k, leader, grp);
    todo &= ~grp;
  }
}

// Wave-wide min / max (call with every lane active), on DPP lane moves: a scan
// within each row of 16 lanes (shifts 1, 2, 4, 8), then rows combined by the row
// broadcasts of lanes 15 and 31, so lane 63 holds the result.
__device__ __forceinline__ int wave_min_i(int v) {
  constexpr int kId = 0x7FFFFFFF;
  v = min(v, __builtin_amdgcn_update_dpp(kId, v, 0x111, 0xf, 0xf, false));  // row_shr:1
  v = min(v, __builtin_amdgcn_update_dpp(kId, v, 0x112, 0xf, 0xf, false));  // row_shr:2
  v = min(v, __builtin_amdgcn_update_dpp(kId, v, 0x114, 0xf, 0xf, false));  // row_shr:4
  v = min(v, __builtin_amdgcn_update_dpp(kId, v, 0x118, 0xf, 0xf, false));  // row_shr:8
  v = min(v, __builtin_amdgcn_update_dpp(kId, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = min(v, __builtin_amdgcn_update_dpp(kId, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ int wave_max_i(int v) {
  constexpr int kId = -0x7FFFFFFF - 1;
  v = max(v, __builtin_amdgcn_update_dpp(kId, v, 0x111, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(kId, v, 0x112, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(kId, v, 0x114, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(kId, v, 0x118, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(kId, v, 0x142, 0xa, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(kId, v, 0x143, 0xc, 0xf, false));
  return __builtin_amdgcn_readlane(v, 63);
}

// grid geometry handed to the shading code
struct Geo {
  int R, P;
  double h, inv_h, inv_hp;
  int flags;
};

// ---------------------------------------------------------------------------
// shading inputs z = [F_s, F_a, c, c^2, c^4] of one sample at FP64 position x
// ---------------------------------------------------------------------------
struct Normal {
  float n[3];
  float gn;
  float c;
};

template <typename ST>
__device__ __forceinline__ void sdf_normal(const ST* __restrict__ sdf, const Geo& G,
                                           const double x[3], Normal& nm) {
  float g[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]};
    xp[a] = fmin(x[a] + G.h, 1.0);
    xm[a] = fmax(x[a] - G.h, -1.0);
    const float sp = tri1(sdf, G.R, cell_d(xp, G.R, G.inv_h));
    const float sm = tri1(sdf, G.R, cell_d(xm, G.R, G.inv_h));
    g[a] = (sp - sm) / (float)(xp[a] - xm[a]);
  }
  nm.gn = sqrtf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  const float inv = 1.0f / fmaxf(nm.gn, 1e-30f);
#pragma unroll
  for (int a = 0; a < 3; ++a) nm.n[a] = g[a] * inv;
}

// The same gradient for a sample whose stencil points x -/+ h e_a all lie one
// cell below / above x's cell (k0) with x's fractions (no clamping at the grid
// boundary): the six trilinear values share 32 nodes of the 4x4x4 patch around
// k0 (rows of 4 along x through the central 2x2 in y, z; end pairs along y and z)
// and the bilinear blends of those rows.  Returns false (nothing done) for any
// other sample.
template <typename ST>
__device__ __forceinline__ bool sdf_normal_cross(const ST* __restrict__ sdf, const Geo& G,
                                                 const double x[3], const Cell& c, Normal& nm) {
  const int R = G.R, RR = R * R;
  const int kx = c.base % R, kyz = c.base / R, ky = kyz % R, kz = kyz / R;
  const int kk[3] = {kx, ky, kz};
  bool inner = true;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    inner = inner && kk[a] >= 1 && kk[a] <= R - 3 && x[a] + G.h <= 1.0 && x[a] - G.h >= -1.0;
  if (!inner) return false;
  const int b = c.base;
  // rows along x at (y, z) = (k0 + jj, k0 + kk): nodes k0-1 .. k0+2
  float2 lo[2][2], hi[2][2], yc[2][2], zc[2][2];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int rb = b - 1 + p * R + q * RR;
      lo[p][q] = ld2(sdf, rb);
      hi[p][q] = ld2(sdf, rb + 2);
      // end pairs (x = k0, k0+1) at y = k0-1 / k0+2 (z = k0+q) and z = k0-1 / k0+2 (y = k0+q)
      yc[p][q] = ld2(sdf, b + (p ? 2 : -1) * R + q * RR);
      zc[p][q] = ld2(sdf, b + q * R + (p ? 2 : -1) * RR);
    }
  const float fx = c.fx, fy = c.fy, fz = c.fz;
  auto yzb = [&](float v00, float v10, float v01, float v11) {
    return lerpf(lerpf(v00, v10, fy), lerpf(v01, v11, fy), fz);
  };
  // x: blends of the four rows' nodes x = k0-1 .. k0+2
  const float bx0 = yzb(lo[0][0].x, lo[1][0].x, lo[0][1].x, lo[1][1].x);
  const float bx1 = yzb(lo[0][0].y, lo[1][0].y, lo[0][1].y, lo[1][1].y);
  const float bx2 = yzb(hi[0][0].x, hi[1][0].x, hi[0][1].x, hi[1][1].x);
  const float bx3 = yzb(hi[0][0].y, hi[1][0].y, hi[0][1].y, hi[1][1].y);
  // y: planes y = k0-1 .. k0+2 blended over (x, z) in the central 2x2
  auto xzb = [&](float v00, float v10, float v01, float v11) {
    return lerpf(lerpf(v00, v10, fx), lerpf(v01, v11, fx), fz);
  };
  const float by0 = xzb(yc[0][0].x, yc[0][0].y, yc[0][1].x, yc[0][1].y);
  const float by1 = xzb(lo[0][0].y, hi[0][0].x, lo[0][1].y, hi[0][1].x);
  const float by2 = xzb(lo[1][0].y, hi[1][0].x, lo[1][1].y, hi[1][1].x);
  const float by3 = xzb(yc[1][0].x, yc[1][0].y, yc[1][1].x, yc[1][1].y);
  // z: planes z = k0-1 .. k0+2 blended over (x, y)
  auto xyb = [&](float v00, float v10, float v01, float v11) {
    return lerpf(lerpf(v00, v10, fx), lerpf(v01, v11, fx), fy);
  };
  const float bz0 = xyb(zc[0][0].x, zc[0][0].y, zc[0][1].x, zc[0][1].y);
  const float bz1 = xyb(lo[0][0].y, hi[0][0].x, lo[1][0].y, hi[1][0].x);
  const float bz2 = xyb(lo[0][1].y, hi[0][1].x, lo[1][1].y, hi[1][1].x);
  const float bz3 = xyb(zc[1][0].x, zc[1][0].y, zc[1][1].x, zc[1][1].y);
  float g[3];
  g[0] = (lerpf(bx2, bx3, fx) - lerpf(bx0, bx1, fx)) / (float)((x[0] + G.h) - (x[0] - G.h));
  g[1] = (lerpf(by2, by3, fy) - lerpf(by0, by1, fy)) / (float)((x[1] + G.h) - (x[1] - G.h));
  g[2] = (lerpf(bz2, bz3, fz) - lerpf(bz0, bz1, fz)) / (float)((x[2] + G.h) - (x[2] - G.h));
  nm.gn = sqrtf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  const float inv = 1.0f / fmaxf(nm.gn, 1e-30f);
#pragma unroll
  for (int a = 0; a < 3; ++a) nm.n[a] = g[a] * inv;
  return true;
}

template <typename ST, typename FT, int NSH>
__device__ __forceinline__ void shade_inputs(const ST* __restrict__ sdf, const FT* __restrict__ feat,
                                             const FT* __restrict__ probes, const Geo& G,
                                             const double x[3], const float v[3], const float* Y,
                                             float z[NIN], Normal& nm) {
  const Cell cs = cell_d(x, G.R, G.inv_h);
  if (!sdf_normal_cross(sdf, G, x, cs, nm)) sdf_normal(sdf, G, x, nm);
  nm.c = (G.flags & FLAG_NV_ONE) ? 1.0f : nm.n[0] * v[0] + nm.n[1] * v[1] + nm.n[2] * v[2];
  z[0] = z[1] = z[2] = 0.0f;
  if (!(G.flags & FLAG_NO_FS)) {
    float w[8];
    corner_w(cs, w);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int node = cs.base + corner_off(c, G.R);
#pragma unroll
      for (int ch = 0; ch < NF; ++ch) z[ch] = fmaf(w[c], ld1(feat, node * NF + ch), z[ch]);
    }
  }
  z[3] = z[4] = z[5] = z[6] = 0.0f;
  if (!(G.flags & FLAG_NO_FA)) {
    const Cell cp = cell_d(x, G.P, G.inv_hp);
    float w[8];
    corner_w(cp, w);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int off = (cp.base + corner_off(c, G.P)) * (NSH * NA);
      float q0 = 0.f, q1 = 0.f, q2 = 0.f, q3 = 0.f;
#pragma unroll
      for (int j = 0; j < NSH; ++j) {
        const float4 b = ld4(probes, off + 4 * j);
        q0 = fmaf(Y[j], b.x, q0);
        q1 = fmaf(Y[j], b.y, q1);
        q2 = fmaf(Y[j], b.z, q2);
        q3 = fmaf(Y[j], b.w, q3);
      }
      z[3] = fmaf(w[c], q0, z[3]);
      z[4] = fmaf(w[c], q1, z[4]);
      z[5] = fmaf(w[c], q2, z[5]);
      z[6] = fmaf(w[c], q3, z[6]);
    }
  }
  const float c = nm.c, c2 = c * c;
  z[7] = c;
  z[8] = c2;
  z[9] = c2 * c2;
}

__device__ __forceinline__ void scatter8(float* g, int R, const Cell& c, float val) {
  float w[8];
  corner_w(c, w);
#pragma unroll
  for (int q = 0; q < 8; ++q) atomic_add_f32(g + c.base + corner_off(q, R), val * w[q]);
}

// ---------------------------------------------------------------------------
// Gradient scatter.  FP32 atomics are executed per 64-byte line: a wave
// instruction whose lanes hit consecutive floats costs about as much as one
// whose lanes hit a single float each in different lines, so every scatter
// below arranges its lanes over contiguous runs of the destination grid.
//
// Probes: the grid is coarse, so the shaded samples of one batch (neighbouring
// rays, consecutive samples) share few probe cells.  Each distinct cell of the
// batch gets an LDS slot; for each of the 8 corners the lanes add their
// n_sh x n_ang products w_c Y_j dF_a into the slot with LDS atomics, and the
// slots are flushed coefficient-major, one global atomic per coefficient of
// each distinct node instead of one per sample.
// ---------------------------------------------------------------------------
template <int NSH>
struct ProbeAcc {
  float acc[64][NSH * NA + 1];  // +1: rows start on different banks
  int key[64];                  // base node of the slot's cell
};

template <int NSH>
__device__ __forceinline__ void probe_acc_clear(ProbeAcc<NSH>& A, int lane) {
#pragma unroll
  for (int q = 0; q < NSH * NA; ++q) A.acc[lane][q] = 0.f;
}

// Call with the whole wave.  Leaves the accumulator rows zero.
template <int NSH>
__device__ __forceinline__ void probe_scatter_wave(ProbeAcc<NSH>& A, int lane, bool ve,
                                                   const Cell& cp, int P, const float* Y,
                                                   const float* dFa, float* g_probes) {
  const int mykey = ve ? cp.base : -1;
  int slot = 0, U = 0;
  uint64_t todo = __ballot(ve);
  while (todo) {
    const int leader = __builtin_ctzll(todo);
    const int k = __builtin_amdgcn_readlane(mykey, leader);
    const bool m = ve && mykey == k;
    if (m) slot = U;
    if (lane == leader) A.key[U] = k;
    todo &= ~__ballot(m);
    ++U;
  }
  float w[8];
  corner_w(cp, w);
  wave_sync();
#pragma unroll 1
  for (int c = 0; c < 8; ++c) {
    if (ve) {
#pragma unroll
      for (int j = 0; j < NSH; ++j) {
        const float wy = w[c] * Y[j];
#pragma unroll
        for (int k = 0; k < NA; ++k) atomicAdd(&A.acc[slot][NA * j + k], wy * dFa[k]);
      }
    }
    wave_sync();
    // flush coefficient-major: consecutive lanes hit consecutive floats of a node
    const int nitems = U * (NSH * NA);
    for (int k = lane; k < nitems; k += 64) {
      const int sl = k / (NSH * NA), q = k - sl * (NSH * NA);
      const float val = A.acc[sl][q];
      A.acc[sl][q] = 0.f;
      if (val != 0.f) atomic_add_f32(g_probes + (A.key[sl] + corner_off(c, P)) * (NSH * NA) + q, val);
    }
    wave_sync();
  }
}

// SDF: every node an entry's SDF gradient touches (the 8 corners of its cell
// for the opacity path, the six FD stencil cells for the normal) lies in the
// 4x4x4 node patch [k0-1, k0+2]^3 around its cell k0 (clamped stencil points
// fall back onto k0 or k0+1).  The entry accumulates into its own LDS patch
// row; the patch is flushed one entry per wave instruction (16 x-runs of 4).
__device__ __forceinline__ void cell_k(const double x[3], int R, double inv_h, int k[3]) {
  const double kmax = (double)(R - 2);
#pragma unroll
  for (int a = 0; a < 3; ++a) k[a] = (int)fmin(fmax(floor((x[a] + 1.0) * inv_h), 0.0), kmax);
}

// Destination of SDF-gradient contributions: an LDS block of nodes with origin
// (ox, oy, oz) and strides (1, sy, sz) -- an entry's private 4x4x4 patch, or a
// box shared by the whole wave (then the adds are LDS atomics).
struct PatchDst {
  float* p;
  int ox, oy, oz;
  int sy, sz;
};

__device__ __forceinline__ PatchDst patch_of_row(float* row, const int k0[3]) {
  return PatchDst{row, k0[0] - 1, k0[1] - 1, k0[2] - 1, 4, 16};
}

template <bool SHARED>
__device__ __forceinline__ void dst_add(float* p, float v) {
  if constexpr (SHARED) atomicAdd(p, v);
  else *p += v;
}

// add val * trilinear weights of the cell of point y (kept within one cell of
// k0) into the destination
template <bool SHARED = false>
__device__ __forceinline__ void patch_add(const PatchDst& D, const int k0[3], const double y[3],
                                          int R, double inv_h, float val) {
  int k[3];
  float f[3];
  const double kmax = (double)(R - 2);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // same cell rule as everywhere, then kept within one cell of k0: only an FP64
    // rounding of u at an integer can step further, and moving the cell by one
    // with f shifted by one puts the weights on the same nodes
    const double u = (y[a] + 1.0) * inv_h;
    double fl = fmin(fmax(floor(u), 0.0), kmax);
    fl = fmin(fmax(fl, (double)(k0[a] - 1)), (double)(k0[a] + 1));
    k[a] = (int)fl;
    f[a] = (float)(u - fl);
  }
  // k lies within one cell of k0, so the 8 corners are inside the destination
  float* q = D.p + (k[2] - D.oz) * D.sz + (k[1] - D.oy) * D.sy + (k[0] - D.ox);
  const float gx = 1.0f - f[0], gy = 1.0f - f[1], gz = 1.0f - f[2];
  const int sy = D.sy, sz = D.sz;
  dst_add<SHARED>(q, val * gx * gy * gz);
  dst_add<SHARED>(q + 1, val * f[0] * gy * gz);
  dst_add<SHARED>(q + sy, val * gx * f[1] * gz);
  dst_add<SHARED>(q + sy + 1, val * f[0] * f[1] * gz);
  dst_add<SHARED>(q + sz, val * gx * gy * f[2]);
  dst_add<SHARED>(q + sz + 1, val * f[0] * gy * f[2]);
  dst_add<SHARED>(q + sz + sy, val * gx * f[1] * f[2]);
  dst_add<SHARED>(q + sz + sy + 1, val * f[0] * f[1] * f[2]);
}

// cotangent of the FD gradient g through the normal path (c = n.v, n = g/|g|)
__device__ __forceinline__ void normal_dg(const float v[3], const Normal& nm, const float dz[NIN],
                                          float dg[3]) {
  const float c = nm.c;
  const float dc = dz[7] + 2.0f * c * dz[8] + 4.0f * c * c * c * dz[9];
  if (nm.gn >= 1e-30f) {
    const float sc = dc / nm.gn;
#pragma unroll
    for (int a = 0; a < 3; ++a) dg[a] = sc * (v[a] - c * nm.n[a]);
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) dg[a] = dc * v[a] / 1e-30f;
  }
}

// SDF gradient from the cotangent dg of the central-difference gradient at x
template <bool SHARED = false>
__device__ __forceinline__ void fd_patch(const PatchDst& D, const int k0[3], const Geo& G,
                                         const double x[3], const float dg[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]};
    xp[a] = fmin(x[a] + G.h, 1.0);
    xm[a] = fmax(x[a] - G.h, -1.0);
    const float coef = dg[a] / (float)(xp[a] - xm[a]);
    patch_add<SHARED>(D, k0, xp, G.R, G.inv_h, coef);
    patch_add<SHARED>(D, k0, xm, G.R, G.inv_h, -coef);
  }
}

// SDF gradient of the normal path
template <bool SHARED = false>
__device__ __forceinline__ void normal_backward_patch(const PatchDst& D, const int k0[3],
                                                      const Geo& G, const double x[3],
                                                      const float v[3], const Normal& nm,
                                                      const float dz[NIN]) {
  float dg[3];
  normal_dg(v, nm, dz, dg);
  fd_patch<SHARED>(D, k0, G, x, dg);
}

// ---------------------------------------------------------------------------
// wave-batched MLP on MFMA (reduced precision).  The 64 samples of a batch are
// four 16-sample blocks; with samples on the MFMA's N dimension the first
// layer's output fragment is exactly the second layer's B operand:
//   H^T (16 hidden x 16 samples) = W1 (16 x 16 padded inputs) . Z^T
//   O^T (16 padded out x 16)     = W2 (16 padded x 16 hidden) . relu(H^T + b1)
// ---------------------------------------------------------------------------
template <int M> struct MType;
template <> struct MType<MLP_F16> {
  typedef _Float16 t;
  typedef h4 v;
  static __device__ __forceinline__ f4 mma(h4 a, h4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  }
};
template <> struct MType<MLP_BF16> {
  typedef __bf16 t;
  typedef b4 v;
  static __device__ __forceinline__ f4 mma(b4 a, b4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
};
// F32 mode keeps the per-lane MLP; the fragment types are unused placeholders
template <> struct MType<MLP_F32> : MType<MLP_F16> {};

template <int M>
struct MlpFrag {
  typename MType<M>::v a1, a2;
  float b1r[4], b2r[4];
};

template <int M>
__device__ __forceinline__ void mlp_frag_load(const float* __restrict__ W, int lane, MlpFrag<M>& f) {
  typedef typename MType<M>::t T;
  const int i = lane & 15, g = lane >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int k = 4 * g + r;
    f.a1[r] = (T)(k < NIN ? W[i * NIN + k] : 0.0f);
    f.b1r[r] = W[OFF_B1 + k];
    f.a2[r] = (T)(i < 3 ? W[OFF_W2 + i * HID + k] : 0.0f);
    f.b2r[r] = k < 3 ? W[OFF_B2 + k] : 0.0f;
  }
}

template <int M>
struct MlpLds {
  typename MType<M>::t zs[64][16];
  float cs[64][4];
};

template <int M>
__device__ __forceinline__ void mlp_wave(const MlpFrag<M>& f, MlpLds<M>& L, int lane,
                                         const float z[NIN], float out[3]) {
  typedef typename MType<M>::t T;
  typedef typename MType<M>::v V4;
  const int i = lane & 15, g = lane >> 4;
  const V4 z0 = {(T)z[0], (T)z[1], (T)z[2], (T)z[3]};
  const V4 z1 = {(T)z[4], (T)z[5], (T)z[6], (T)z[7]};
  const V4 z2 = {(T)z[8], (T)z[9], (T)0.0f, (T)0.0f};
  const V4 z3 = {(T)0.0f, (T)0.0f, (T)0.0f, (T)0.0f};
  *reinterpret_cast<V4*>(&L.zs[lane][0]) = z0;
  *reinterpret_cast<V4*>(&L.zs[lane][4]) = z1;
  *reinterpret_cast<V4*>(&L.zs[lane][8]) = z2;
  *reinterpret_cast<V4*>(&L.zs[lane][12]) = z3;
  wave_sync();
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const V4 bz = *reinterpret_cast<const V4*>(&L.zs[16 * b + i][4 * g]);
    f4 d = {0.f, 0.f, 0.f, 0.f};
    d = MType<M>::mma(f.a1, bz, d);
    V4 hb;
#pragma unroll
    for (int r = 0; r < 4; ++r) hb[r] = (T)fmaxf(d[r] + f.b1r[r], 0.0f);
    f4 o = {0.f, 0.f, 0.f, 0.f};
    o = MType<M>::mma(f.a2, hb, o);
    if (g == 0) {
      L.cs[16 * b + i][0] = o[0] + f.b2r[0];
      L.cs[16 * b + i][1] = o[1] + f.b2r[1];
      L.cs[16 * b + i][2] = o[2] + f.b2r[2];
    }
  }
  wave_sync();
  out[0] = L.cs[lane][0];
  out[1] = L.cs[lane][1];
  out[2] = L.cs[lane][2];
  wave_sync();
}

// MLP weight gradients: sum over the batch of (row vector) x (column vector) as
// 16x16 tiles on FP32 MFMA with K = samples.
struct DwLds {
  float st[64][36];  // row stride 36 floats: 16-byte rows, spread banks
};

__device__ __forceinline__ void dw_accumulate(DwLds& L, int lane, const float a[16],
                                              const float b[16], f4& acc) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    *reinterpret_cast<float4*>(&L.st[lane][4 * q]) =
        make_float4(a[4 * q], a[4 * q + 1], a[4 * q + 2], a[4 * q + 3]);
    *reinterpret_cast<float4*>(&L.st[lane][16 + 4 * q]) =
        make_float4(b[4 * q], b[4 * q + 1], b[4 * q + 2], b[4 * q + 3]);
  }
  wave_sync();
  const int i = lane & 15, g = lane >> 4;
#pragma unroll
  for (int t = 0; t < 16; ++t)
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(L.st[4 * t + g][i], L.st[4 * t + g][16 + i], acc, 0,
                                                 0, 0);
  wave_sync();
}

// ---------------------------------------------------------------------------
// per-wave queue of shaded samples (a ring of 128 entries).  A lane pushes at
// most one entry per march step; entries of one ray are linked in order.
// ---------------------------------------------------------------------------
constexpr int RING = 128;

// number of lower lanes set in a wave mask
__device__ __forceinline__ int lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

}  // namespace psdf
