// Reverse-mode pieces of the per-sample shading shared by the fused backward
// kernel and the entry-parallel one: MLP reverse mode, and the wave-level
// gradient scatters into the SDF, the spatial features and the MLP weights.
//
// With dL/dC_i = w_i dL/drgb and C = sigmoid(o): dL/do = dL/dC C (1 - C); the
// MLP and the interpolations are linear in what they scatter, so every lane
// (one shaded sample) produces dL/dz for its inputs z = [F_s, F_a, c, c^2, c^4]
// and spreads them over the grid nodes it read.
#pragma once

#include "shade.h"

namespace psdf {

// dpre (hidden pre-activation) and dz (MLP inputs) of one lane; dz = 0 unless ve
template <int M, bool WR = false, typename WT>
__device__ __forceinline__ void mlp_backward_lane(WT* __restrict__ W, const float dout[3],
                                                  const float pre[HID], bool ve, float dpre[HID],
                                                  float dz[NIN]) {
#pragma unroll
  for (int k = 0; k < HID; ++k) {
    float acc = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) acc = fmaf(wrnd<M, WR>(W[OFF_W2 + c * HID + k]), dout[c], acc);
    dpre[k] = pre[k] > 0.f ? acc : 0.f;
  }
#pragma unroll
  for (int j = 0; j < NIN; ++j) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < HID; ++k) acc = fmaf(wrnd<M, WR>(W[k * NIN + j]), dpre[k], acc);
    dz[j] = ve ? acc : 0.f;
  }
}

// Flush of per-entry 4x4x4 SDF patches (rows sc[e][0..63], origin k0[e] - 1):
// one entry per wave instruction, lanes over the patch (16 x-runs of 4 floats).
// Rows of entries without a gradient must be zero.
__device__ __forceinline__ void sdf_patch_flush(const float (*sc)[65], const int (*k0)[3], int n,
                                                int lane, int R, float* g_sdf) {
  const int px = lane & 3, py = (lane >> 2) & 3, pz = lane >> 4;
  for (int e = 0; e < n; ++e) {
    const float val = sc[e][lane];
    const int nx = k0[e][0] - 1 + px, ny = k0[e][1] - 1 + py, nz = k0[e][2] - 1 + pz;
    if (val != 0.f && nx >= 0 && ny >= 0 && nz >= 0 && nx < R && ny < R && nz < R)
      atomic_add_f32(g_sdf + (nz * R + ny) * R + nx, val);
  }
}

// Spatial-feature gradient: 8 corners x 3 channels per entry, staged in LDS and
// flushed item-major (the two x-neighbour corners are 6 contiguous floats).
// Call with the whole wave; entries e >= n are not read.
__device__ __forceinline__ void feat_scatter_wave(float (*sc)[65], int* fb, bool ve, const Cell& cs,
                                                  const float dz[NIN], int n, int lane, int R,
                                                  float* g_feat) {
  float wc[8];
  corner_w(cs, wc);
  fb[lane] = cs.base;
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int ch = 0; ch < NF; ++ch) sc[lane][c * NF + ch] = ve ? wc[c] * dz[ch] : 0.f;
  wave_sync();
  for (int k = lane; k < n * 8 * NF; k += 64) {
    const int e = k / (8 * NF), q = k - e * (8 * NF);
    const int c = q / NF, ch = q - c * NF;
    const float val = sc[e][q];
    if (val != 0.f) atomic_add_f32(g_feat + (fb[e] + corner_off(c, R)) * NF + ch, val);
  }
  wave_sync();
}

// ---------------------------------------------------------------------------
// Box accumulation: the SDF (or feature) gradients of a spatially compact set of
// samples are added into one LDS box of nodes with LDS atomics, and the box is
// flushed once, each row of nodes as a contiguous run of lanes.  Called with the
// whole wave.
// ---------------------------------------------------------------------------

// zero the first n floats of a 16-byte aligned box whose capacity is a multiple
// of 4 floats (n <= capacity)
__device__ __forceinline__ void box_clear(float* box, int n, int lane) {
  float4* b4 = reinterpret_cast<float4*>(box);
  for (int i = lane; i < (n + 3) / 4; i += 64) b4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// LDS box accumulation.  The LDS executes FP32 atomic adds at a fraction of the
// rate of integer ones, so a box normally holds 32-bit fixed point: each value is
// scaled by sc = 2^30 / (64 B), B a bound on any one lane's contribution to a
// node, and rounded; a node sums at most 64 lanes, so |sum| < 2^30, and the
// rounding error is below B / 2^25 per contribution.  Integer sums are also
// independent of the order of the adds.  Boxes with a non-finite or huge bound
// (or boundary samples, SDF) take FP32 atomics.
template <bool FIXED>
__device__ __forceinline__ void box_add(float* p, float v, float sc) {
  if constexpr (FIXED) atomicAdd(reinterpret_cast<int*>(p), __float2int_rn(v * sc));
  else atomicAdd(p, v);
}

// wave-wide max of a non-negative float (NaN compares above +inf)
__device__ __forceinline__ float wave_max_nonneg(float v) {
  return __int_as_float(wave_max_i(__float_as_int(v)));
}

constexpr float kFixedMaxBound = 1e36f;  // larger bounds use FP32 atomics

__device__ __forceinline__ float fixed_scale(float B) {
  return B > 0.f ? 0x1p30f / (64.f * B) : 1.f;
}

// A box of ex x ey x ez nodes with C channels, origin (ox, oy, oz): rows of
// ex * C values, row r holding nodes (ox + x / C, oy + r % ey, oz + r / ey).  Each
// nonzero value (fixed point: times inv) is added to the grid; a power-of-two
// group of lanes takes a row.
template <int C, bool FIXED>
__device__ __forceinline__ void box_flush(const float* box, float inv, int ex, int ey, int ez,
                                          int ox, int oy, int oz, int R, float* g, int lane) {
  const int row_len = ex * C, nrows = ey * ez;
  int lpr = 1;
  while (lpr < row_len && lpr < 64) lpr <<= 1;  // lanes per row
  const int sh = __builtin_ctz(lpr), rows_per = 64 >> sh;
  const int x0 = lane & (lpr - 1);
  auto value = [&](int i) {
    if constexpr (FIXED) return (float)reinterpret_cast<const int*>(box)[i] * inv;
    else return box[i];
  };
  // this lane's row, advanced by rows_per rows (dz planes + dy rows) per step
  int r = lane >> sh;
  int iz = r / ey, iy = r - iz * ey;
  const int dz = rows_per / ey, dy = rows_per - dz * ey;
  if (row_len <= 64) {
    // one element per lane and step, four steps at a time: the four LDS reads are
    // issued unconditionally (indices inside the box), then the atomics
    const int nstep = (nrows + rows_per - 1) / rows_per;
    const int gx = ox + x0 / C;
    const bool x_in = x0 < row_len && gx >= 0 && gx < R;
    const int64_t rstride = (int64_t)R * C;  // elements per grid row
    const int64_t xoff = (int64_t)ox * C + x0;
    for (int s0 = 0; s0 < nstep; s0 += 4) {
      int ru[4], gy[4], gz[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ru[u] = r;
        gy[u] = oy + iy;
        gz[u] = oz + iz;
        r += rows_per;
        iy += dy;  // dy < ey: one wrap at most
        iz += dz;
        if (iy >= ey) {
          iy -= ey;
          ++iz;
        }
      }
      float v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = value(x_in && ru[u] < nrows ? ru[u] * row_len + x0 : 0);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool in = x_in && ru[u] < nrows && (unsigned)gy[u] < (unsigned)R &&
                        (unsigned)gz[u] < (unsigned)R;
        if (in && v[u] != 0.f)
          atomic_add_f32(g + ((int64_t)gz[u] * R + gy[u]) * rstride + xoff, v[u]);
      }
    }
    return;
  }
  for (int r0 = 0; r0 < nrows; r0 += rows_per) {
    if (r < nrows) {
      const int gy = oy + iy, gz = oz + iz;
      const bool row_in = gy >= 0 && gy < R && gz >= 0 && gz < R;
      float* grow = g + ((int64_t)(gz * R + gy) * R + ox) * C;
      for (int xx = x0; xx < row_len; xx += lpr) {
        const float v = value(r * row_len + xx);
        const int gx = ox + xx / C;
        if (v != 0.f && row_in && gx >= 0 && gx < R) atomic_add_f32(grow + xx, v);
      }
    }
    r += rows_per;
    iy += dy;
    iz += dz;
    if (iy >= ey) {
      iy -= ey;
      ++iz;
    }
  }
}

// The opacity term and the six FD terms of an interior sample, whose stencil
// points x -/+ h e_a lie one cell below / above x's cell with x's fractions: 32
// nodes of the 4x4x4 patch around the cell (its central 2x2x2 and two 2x2 end caps
// per axis).  q points at the patch's lowest node.
template <bool FIXED>
__device__ __forceinline__ void sdf_cross_add(float* q, int sy, int sz, const float f[3],
                                              const float c[3], float a0, float sc) {
  const float wx[2] = {1.f - f[0], f[0]}, wy[2] = {1.f - f[1], f[1]}, wz[2] = {1.f - f[2], f[2]};
#pragma unroll
  for (int kk = 0; kk < 2; ++kk)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
      const float yz = wy[jj] * wz[kk];
      float* row = q + (kk + 1) * sz + (jj + 1) * sy;
      box_add<FIXED>(row, -c[0] * wx[0] * yz, sc);
      box_add<FIXED>(row + 3, c[0] * wx[1] * yz, sc);
      const float yv = jj == 0 ? -c[1] * wy[1] : c[1] * wy[0];
      const float zv = kk == 0 ? -c[2] * wz[1] : c[2] * wz[0];
#pragma unroll
      for (int ii = 0; ii < 2; ++ii) {
        const float xv = ii == 0 ? -c[0] * wx[1] : c[0] * wx[0];
        box_add<FIXED>(row + ii + 1,
                       (a0 * wx[ii] + xv) * yz + yv * wx[ii] * wz[kk] + zv * wx[ii] * wy[jj], sc);
      }
    }
#pragma unroll
  for (int kk = 0; kk < 2; ++kk)
#pragma unroll
    for (int ii = 0; ii < 2; ++ii) {
      const float xz = wx[ii] * wz[kk];
      float* col = q + (kk + 1) * sz + ii + 1;
      box_add<FIXED>(col, -c[1] * wy[0] * xz, sc);
      box_add<FIXED>(col + 3 * sy, c[1] * wy[1] * xz, sc);
    }
#pragma unroll
  for (int jj = 0; jj < 2; ++jj)
#pragma unroll
    for (int ii = 0; ii < 2; ++ii) {
      const float xy = wx[ii] * wy[jj];
      float* col = q + (jj + 1) * sy + ii + 1;
      box_add<FIXED>(col, -c[2] * wz[0] * xy, sc);
      box_add<FIXED>(col + 3 * sz, c[2] * wz[1] * xy, sc);
    }
}

// SDF box pass over the lanes with `part` set: the opacity gradient at s_i
// (coefficient a0, trilinear at x), the central-difference path (cotangent dg of
// the FD gradient at x) and, where sample i+1 is not shaded itself, the opacity
// gradient at s_{i+1} (coefficient a1, trilinear at x + off).  The successor's 8
// corners go into the box when the box of every lane's nodes fits in `cap`
// floats; else the box holds the lanes' own 4x4x4 patches and a successor whose
// corners lie outside it is added to the grid directly (with `direct1` every
// successor is, which a single lane's box always allows).  Returns false, having
// done nothing, when the patches alone do not fit (wave-uniform).
__device__ __forceinline__ bool sdf_box_pass(float* box, int cap, int lane, bool part,
                                             const double x[3], const float dg[3], float a0,
                                             const float off[3], float a1, bool direct1,
                                             const Geo& G, float* g_sdf) {
  int k0[3] = {0, 0, 0}, k1[3] = {0, 0, 0};
  float f1[3] = {0.f, 0.f, 0.f};
  const bool any1 = part && a1 != 0.f;
  if (part) cell_k(x, G.R, G.inv_h, k0);
  if (any1) {
    const double kmax = (double)(G.R - 2);
#pragma unroll
    for (int a = 0; a < 3; ++a) axis_cell_d(x[a] + (double)off[a], G.inv_h, kmax, k1[a], f1[a]);
  }
  // the lanes' own patches: nodes k0-1 .. k0+2
  int lo[3], ext[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = wave_min_i(part ? k0[a] - 1 : 0x7FFFFFFF);
    ext[a] = wave_max_i(part ? k0[a] + 2 : -0x7FFFFFFF) - lo[a] + 1;
  }
  if ((int64_t)ext[0] * ext[1] * ext[2] > cap) return false;
  bool has1 = any1 && !direct1;
  if (wave_any(has1)) {
    // with the successors' corners k1 .. k1+1, if that box fits
    int los[3], exs[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      los[a] = min(lo[a], wave_min_i(has1 ? k1[a] : 0x7FFFFFFF));
      exs[a] = max(lo[a] + ext[a] - 1, wave_max_i(has1 ? k1[a] + 1 : -0x7FFFFFFF)) - los[a] + 1;
    }
    if ((int64_t)exs[0] * exs[1] * exs[2] <= cap) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        lo[a] = los[a];
        ext[a] = exs[a];
      }
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a) has1 = has1 && k1[a] >= lo[a] && k1[a] + 1 < lo[a] + ext[a];
    }
  }
  if (any1 && !has1) {
    const Cell c1{(k1[2] * G.R + k1[1]) * G.R + k1[0], f1[0], f1[1], f1[2]};
    scatter8(g_sdf, G.R, c1, a1);
  }
  const int vol = ext[0] * ext[1] * ext[2];
  const int sy = ext[0], sz = ext[0] * ext[1];
  float f[3] = {0.f, 0.f, 0.f}, c[3] = {0.f, 0.f, 0.f}, bnd = 0.f;
  bool inner = true;
  if (part) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double u = (x[a] + 1.0) * G.inv_h;
      f[a] = (float)(u - (double)k0[a]);
      inner = inner && k0[a] >= 1 && k0[a] <= G.R - 3 && x[a] + G.h <= 1.0 && x[a] - G.h >= -1.0;
      c[a] = dg[a] / (float)((x[a] + G.h) - (x[a] - G.h));
    }
    // every node gets at most |a0| + sum |c_a| + |a1| from a lane (weights <= 1)
    bnd = fabsf(a0) + fabsf(c[0]) + fabsf(c[1]) + fabsf(c[2]) + (has1 ? fabsf(a1) : 0.f);
  }
  const float B = wave_max_nonneg(bnd);
  const bool fixed = !wave_any(part && !inner) && B < kFixedMaxBound;
  const float sc = fixed_scale(B);
  box_clear(box, vol, lane);
  wave_sync();
  float* q = box + (k0[2] - 1 - lo[2]) * sz + (k0[1] - 1 - lo[1]) * sy + (k0[0] - 1 - lo[0]);
  // the successor's 8 corners
  float* q1 = box + (k1[2] - lo[2]) * sz + (k1[1] - lo[1]) * sy + (k1[0] - lo[0]);
  float w1[8];
  corner_w(Cell{0, f1[0], f1[1], f1[2]}, w1);
  if (fixed) {
    if (part) sdf_cross_add<true>(q, sy, sz, f, c, a0, sc);
    if (has1) {
#pragma unroll
      for (int cc = 0; cc < 8; ++cc)
        box_add<true>(q1 + (cc & 1) + ((cc >> 1) & 1) * sy + ((cc >> 2) & 1) * sz, a1 * w1[cc], sc);
    }
    wave_sync();
    box_flush<1, true>(box, 1.f / sc, ext[0], ext[1], ext[2], lo[0], lo[1], lo[2], G.R, g_sdf, lane);
  } else {
    if (part) {
      if (inner) {
        sdf_cross_add<false>(q, sy, sz, f, c, a0, 1.f);
      } else {
        const PatchDst D{box, lo[0], lo[1], lo[2], sy, sz};
        if (a0 != 0.f) patch_add<true>(D, k0, x, G.R, G.inv_h, a0);
        if (dg[0] != 0.f || dg[1] != 0.f || dg[2] != 0.f) fd_patch<true>(D, k0, G, x, dg);
      }
    }
    if (has1) {
#pragma unroll
      for (int cc = 0; cc < 8; ++cc)
        box_add<false>(q1 + (cc & 1) + ((cc >> 1) & 1) * sy + ((cc >> 2) & 1) * sz, a1 * w1[cc], 1.f);
    }
    wave_sync();
    box_flush<1, false>(box, 1.f, ext[0], ext[1], ext[2], lo[0], lo[1], lo[2], G.R, g_sdf, lane);
  }
  wave_sync();
  return true;
}

template <bool FIXED>
__device__ __forceinline__ void feat_corner_add(float* box, int b, int ex, int exy, const float f[3],
                                                const float df[NF], float sc) {
  float wc[8];
  corner_w(Cell{0, f[0], f[1], f[2]}, wc);
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int o = b + (c & 1) + ((c >> 1) & 1) * ex + ((c >> 2) & 1) * exy;
#pragma unroll
    for (int ch = 0; ch < NF; ++ch) box_add<FIXED>(&box[o * NF + ch], wc[c] * df[ch], sc);
  }
}

// spatial-feature box pass: 8 corners x NF channels per lane with `part` set
__device__ __forceinline__ bool feat_box_pass(float* box, int cap, int lane, bool part,
                                              const double x[3], const float df[NF], const Geo& G,
                                              float* g_feat) {
  int k[3] = {0, 0, 0};
  float f[3] = {0.f, 0.f, 0.f};
  if (part) {
    const double kmax = (double)(G.R - 2);
#pragma unroll
    for (int a = 0; a < 3; ++a) axis_cell_d(x[a], G.inv_h, kmax, k[a], f[a]);
  }
  int lo[3], ext[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = wave_min_i(part ? k[a] : 0x7FFFFFFF);  // nodes k .. k+1
    ext[a] = wave_max_i(part ? k[a] : -0x7FFFFFFF) - lo[a] + 2;
  }
  if ((int64_t)ext[0] * ext[1] * ext[2] * NF > cap) return false;
  const int vol = ext[0] * ext[1] * ext[2];
  // a corner weight is at most 1
  float bnd = 0.f;
#pragma unroll
  for (int ch = 0; ch < NF; ++ch) bnd = fmaxf(bnd, part ? fabsf(df[ch]) : 0.f);
  const float B = wave_max_nonneg(bnd);
  const bool fixed = B < kFixedMaxBound;
  const float sc = fixed_scale(B);
  box_clear(box, vol * NF, lane);
  wave_sync();
  const int b = ((k[2] - lo[2]) * ext[1] + (k[1] - lo[1])) * ext[0] + (k[0] - lo[0]);
  if (fixed) {
    if (part) feat_corner_add<true>(box, b, ext[0], ext[0] * ext[1], f, df, sc);
    wave_sync();
    box_flush<NF, true>(box, 1.f / sc, ext[0], ext[1], ext[2], lo[0], lo[1], lo[2], G.R, g_feat,
                        lane);
  } else {
    if (part) feat_corner_add<false>(box, b, ext[0], ext[0] * ext[1], f, df, 1.f);
    wave_sync();
    box_flush<NF, false>(box, 1.f, ext[0], ext[1], ext[2], lo[0], lo[1], lo[2], G.R, g_feat, lane);
  }
  wave_sync();
  return true;
}

// Runs a box pass over the lanes with `ve` set: all of them at once when their
// nodes fit, else in groups of 16 lanes, then 4, then one.  pass(part, single):
// `single` marks the one-lane level, where the pass must fit (its own nodes
// always fit a box of at least 64 floats; farther terms go to the grid).
template <typename Pass>
__device__ __forceinline__ void box_in_groups(bool ve, int lane, Pass pass) {
  if (!wave_any(ve)) return;
  if (pass(ve, false)) return;
  bool pending = ve;
  for (int gs = 16; gs >= 1; gs >>= 2) {
    for (int g0 = 0; g0 < 64; g0 += gs) {
      const bool part = pending && (unsigned)(lane - g0) < (unsigned)gs;
      if (!wave_any(part)) continue;
      if (pass(part, gs == 1)) pending = pending && !part;
    }
    if (!wave_any(pending)) return;
  }
}

// MLP weight gradients of the wave's entries, summed on MFMA (K = samples)
template <int M>
__device__ __forceinline__ void mlp_dw_wave(DwLds& D, int lane, bool ve, const float z[NIN],
                                            const float hid[HID], const float dpre[HID],
                                            const float dout[3], f4& acc_w1, f4& acc_w2,
                                            float db2[3]) {
  float zin[16], hin[16], dop[16];
#pragma unroll
  for (int j = 0; j < NIN; ++j) zin[j] = mrnd<M>(z[j]);
  zin[NIN] = ve ? 1.f : 0.f;
#pragma unroll
  for (int j = NIN + 1; j < 16; ++j) zin[j] = 0.f;
#pragma unroll
  for (int k = 0; k < HID; ++k) hin[k] = mrnd<M>(hid[k]);
#pragma unroll
  for (int k = 0; k < 16; ++k) dop[k] = k < 3 ? dout[k] : 0.f;
  dw_accumulate(D, lane, dpre, zin, acc_w1);
  dw_accumulate(D, lane, dop, hin, acc_w2);
  db2[0] += dout[0];
  db2[1] += dout[1];
  db2[2] += dout[2];
}

// the wave's MLP gradient as one contiguous row of NMLP partials
__device__ __forceinline__ void mlp_grad_store(float* row, int lane, const f4& acc_w1,
                                               const f4& acc_w2, const float db2[3]) {
  const int i = lane & 15, g = lane >> 4;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int r = 4 * g + rr;
    if (i < NIN) row[r * NIN + i] = acc_w1[rr];
    else if (i == NIN) row[OFF_B1 + r] = acc_w1[rr];
    if (r < 3) row[OFF_W2 + r * HID + i] = acc_w2[rr];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float s = wave_sum(db2[c]);
    if (lane == 0) row[OFF_B2 + c] = s;
  }
}

// one global atomic per MLP parameter per wave
__device__ __forceinline__ void mlp_grad_flush(float* g_mlp, int lane, const f4& acc_w1,
                                               const f4& acc_w2, const float db2[3]) {
  const int i = lane & 15, g = lane >> 4;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int row = 4 * g + rr;  // hidden unit for dW1, output for dW2
    if (i < NIN) atomic_add_f32(g_mlp + row * NIN + i, acc_w1[rr]);
    else if (i == NIN) atomic_add_f32(g_mlp + OFF_B1 + row, acc_w1[rr]);
    if (row < 3) atomic_add_f32(g_mlp + OFF_W2 + row * HID + i, acc_w2[rr]);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float s = wave_sum(db2[c]);
    if (lane == 0) atomic_add_f32(g_mlp + OFF_B2 + c, s);
  }
}

}  // namespace psdf
