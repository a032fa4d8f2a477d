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
template <int M>
__device__ __forceinline__ void mlp_backward_lane(const float* __restrict__ W, const float dout[3],
                                                  const float pre[HID], bool ve, float dpre[HID],
                                                  float dz[NIN]) {
#pragma unroll
  for (int k = 0; k < HID; ++k) {
    float acc = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) acc = fmaf(mrnd<M>(W[OFF_W2 + c * HID + k]), dout[c], acc);
    dpre[k] = pre[k] > 0.f ? acc : 0.f;
  }
#pragma unroll
  for (int j = 0; j < NIN; ++j) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < HID; ++k) acc = fmaf(mrnd<M>(W[k * NIN + j]), dpre[k], acc);
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
// Box accumulation: when the wave's samples are spatially compact, their SDF
// (or feature) gradients are added into one LDS box of nodes with LDS atomics,
// and the box is flushed once, each row of nodes as a contiguous run of lanes.
// Call with the whole wave; returns false (nothing done) when the box does not
// fit, and the caller then takes the per-sample path.
// ---------------------------------------------------------------------------
constexpr int BOXCAP = 64 * 65;  // floats

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = min(v, __shfl_xor(v, m, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m, 64));
  return v;
}

// nrows rows of row_len floats; row r holds nodes (ox + x / C, oy + r % ey, oz + r / ey)
__device__ __forceinline__ void box_flush(const float* box, int row_len, int nrows, int ey, int ox,
                                          int oy, int oz, int R, int C, float* g, int lane) {
  int lpr = 1;
  while (lpr < row_len && lpr < 64) lpr <<= 1;  // lanes per row
  const int sh = __builtin_ctz(lpr), rows_per = 64 >> sh;
  for (int r0 = 0; r0 < nrows; r0 += rows_per) {
    const int r = r0 + (lane >> sh);
    if (r < nrows) {
      const int iz = r / ey, iy = r - iz * ey;
      const int gy = oy + iy, gz = oz + iz;
      const bool row_in = gy >= 0 && gy < R && gz >= 0 && gz < R;
      for (int xx = lane & (lpr - 1); xx < row_len; xx += lpr) {
        const float v = box[r * row_len + xx];
        const int gx = ox + xx / C;
        if (v != 0.f && row_in && gx >= 0 && gx < R)
          atomic_add_f32(g + ((int64_t)(gz * R + gy) * R + ox) * C + xx, v);
      }
    }
  }
}

// SDF: the opacity gradient at s_i (coefficient a0) and the normal path
__device__ __forceinline__ bool sdf_box_wave(float* box, int lane, bool ve, const double x[3],
                                             const float v[3], const Normal& nm,
                                             const float dz[NIN], float a0, const Geo& G,
                                             float* g_sdf) {
  if (!wave_any(ve)) return true;
  int k0[3] = {0, 0, 0};
  if (ve) cell_k(x, G.R, G.inv_h, k0);
  int lo[3], ext[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = wave_min_i(ve ? k0[a] : 0x7FFFFFFF);
    ext[a] = wave_max_i(ve ? k0[a] : -0x7FFFFFFF) - lo[a] + 4;  // nodes lo-1 .. hi+2
  }
  if ((int64_t)ext[0] * ext[1] * ext[2] > BOXCAP) return false;
  const int vol = ext[0] * ext[1] * ext[2];
  for (int i = lane; i < vol; i += 64) box[i] = 0.f;
  wave_sync();
  const PatchDst D{box, lo[0] - 1, lo[1] - 1, lo[2] - 1, ext[0], ext[0] * ext[1]};
  if (ve) {
    if (a0 != 0.f) patch_add<true>(D, k0, x, G.R, G.inv_h, a0);
    if (!(G.flags & FLAG_NV_ONE)) normal_backward_patch<true>(D, k0, G, x, v, nm, dz);
  }
  wave_sync();
  box_flush(box, ext[0], ext[1] * ext[2], ext[1], D.ox, D.oy, D.oz, G.R, 1, g_sdf, lane);
  wave_sync();
  return true;
}

// spatial features: 8 corners x 3 channels per sample
__device__ __forceinline__ bool feat_box_wave(float* box, int lane, bool ve, const double x[3],
                                              const Cell& cs, const float dz[NIN], const Geo& G,
                                              float* g_feat) {
  if (!wave_any(ve)) return true;
  int k[3] = {0, 0, 0};
  if (ve) cell_k(x, G.R, G.inv_h, k);
  int lo[3], ext[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = wave_min_i(ve ? k[a] : 0x7FFFFFFF);
    ext[a] = wave_max_i(ve ? k[a] : -0x7FFFFFFF) - lo[a] + 2;  // nodes lo .. hi+1
  }
  if ((int64_t)ext[0] * ext[1] * ext[2] * NF > BOXCAP) return false;
  const int vol = ext[0] * ext[1] * ext[2];
  for (int i = lane; i < vol * NF; i += 64) box[i] = 0.f;
  wave_sync();
  if (ve) {
    float wc[8];
    corner_w(cs, wc);
    const int b = ((k[2] - lo[2]) * ext[1] + (k[1] - lo[1])) * ext[0] + (k[0] - lo[0]);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int o = b + (c & 1) + ((c >> 1) & 1) * ext[0] + ((c >> 2) & 1) * ext[0] * ext[1];
#pragma unroll
      for (int ch = 0; ch < NF; ++ch) atomicAdd(&box[o * NF + ch], wc[c] * dz[ch]);
    }
  }
  wave_sync();
  box_flush(box, ext[0] * NF, ext[1] * ext[2], ext[1], lo[0], lo[1], lo[2], G.R, NF, g_feat, lane);
  wave_sync();
  return true;
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
