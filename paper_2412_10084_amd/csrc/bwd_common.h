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
