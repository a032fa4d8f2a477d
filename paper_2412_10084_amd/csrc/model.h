// The paper's own colour model and its reverse mode, per sample (one lane):
//   - SH evaluated at the view direction v, or at the reflection of v about the
//     normal, r = 2 (n.v) n - v (Sec. 3.1, Sec. 3.2 Eqs. spherical_harmonics,
//     sh_eval1 / sh_eval2), with up to 16 coefficients (bands 0..3, the paper's
//     one-indexed l = 4, Sec. 4);
//   - incidence inputs (c, c^2, c^4) or the powers (1 - c)^0 .. (1 - c)^5 of
//     Eq. newparametrization, c = n.v;
//   - an MLP of one hidden layer of 16 or two hidden layers of 32 (Sec. 4), ReLU,
//     sigmoid output.
// Packed MLP of n_in inputs, hidden width H and L hidden layers: W_0[H][n_in],
// b_0[H], (W_1[H][H], b_1[H] when L = 2), W_o[3][H], b_o[3].
#pragma once

#include "bwd_common.h"

namespace psdf {

constexpr int FLAG_SH_REFLECT = 8;
constexpr int FLAG_FRESNEL_PAPER = 16;
constexpr int MNIN = NF + NA + 6;  // most MLP inputs of any model (13)

__host__ __device__ constexpr int model_n_in(int flags) {
  return NF + NA + ((flags & FLAG_FRESNEL_PAPER) ? 6 : 3);
}
__host__ __device__ constexpr int model_mlp_size(int n_in, int H, int L) {
  return H * n_in + H + (L - 1) * (H * H + H) + 3 * H + 3;
}

// Gradient of the SH polynomials of sh_basis (as functions on R^3): dY[j] = grad Y_j.
template <int NSH>
__device__ __forceinline__ void sh_grad(float x, float y, float z, float (*dY)[3]) {
  dY[0][0] = dY[0][1] = dY[0][2] = 0.f;
  if constexpr (NSH >= 4) {
    constexpr float c1 = 0.4886025119029199f;
    dY[1][0] = 0.f, dY[1][1] = c1, dY[1][2] = 0.f;
    dY[2][0] = 0.f, dY[2][1] = 0.f, dY[2][2] = c1;
    dY[3][0] = c1, dY[3][1] = 0.f, dY[3][2] = 0.f;
  }
  if constexpr (NSH >= 9) {
    constexpr float c2 = 1.0925484305920792f, c20 = 0.31539156525252005f,
                    c22 = 0.5462742152960396f;
    dY[4][0] = c2 * y, dY[4][1] = c2 * x, dY[4][2] = 0.f;
    dY[5][0] = 0.f, dY[5][1] = c2 * z, dY[5][2] = c2 * y;
    dY[6][0] = 0.f, dY[6][1] = 0.f, dY[6][2] = 6.f * c20 * z;
    dY[7][0] = c2 * z, dY[7][1] = 0.f, dY[7][2] = c2 * x;
    dY[8][0] = 2.f * c22 * x, dY[8][1] = -2.f * c22 * y, dY[8][2] = 0.f;
  }
  if constexpr (NSH >= 16) {
    constexpr float a = 0.5900435899266435f, b = 2.890611442640554f, e = 0.4570457994644658f,
                    g = 0.3731763325901154f, k = 1.445305721320277f;
    dY[9][0] = 6.f * a * x * y, dY[9][1] = 3.f * a * (x * x - y * y), dY[9][2] = 0.f;
    dY[10][0] = b * y * z, dY[10][1] = b * x * z, dY[10][2] = b * x * y;
    dY[11][0] = 0.f, dY[11][1] = e * (5.f * z * z - 1.f), dY[11][2] = 10.f * e * y * z;
    dY[12][0] = 0.f, dY[12][1] = 0.f, dY[12][2] = g * (15.f * z * z - 3.f);
    dY[13][0] = e * (5.f * z * z - 1.f), dY[13][1] = 0.f, dY[13][2] = 10.f * e * x * z;
    dY[14][0] = 2.f * k * x * z, dY[14][1] = -2.f * k * y * z, dY[14][2] = k * (x * x - y * y);
    dY[15][0] = 3.f * a * (x * x - y * y), dY[15][1] = -6.f * a * x * y, dY[15][2] = 0.f;
  }
}

// ---------------------------------------------------------------------------
// Sparse tiles of 16^3 cells with tri-plane spatial features (Sec. 3.1, Sec. 4):
// F_s = F_x(y, z) * F_y(x, z) * F_z(x, y) channel by channel, each plane a 16 x 16
// texture of its tile (texels at the cell centres, bilinear, clamped inside the
// tile), planes [slots][3][16][16][NF]; a point lies in the tile of its trilinear
// cell; tile_index [T][T][T] holds each tile's slot or -1 (empty).
// ---------------------------------------------------------------------------
struct Tiles {
  const int* __restrict__ index;  // nullptr: dense features
  int T;
};

// slot of the tile holding x (-1: empty), and x in that tile's cell units
__device__ __forceinline__ int tile_slot(const Tiles& tl, int R, double inv_h, const double x[3],
                                         float loc[3]) {
  int t[3];
  const double kmax = (double)(R - 2);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double u = (x[a] + 1.0) * inv_h;
    const double k0 = fmin(fmax(floor(u), 0.0), kmax);
    t[a] = (int)k0 >> 4;
    loc[a] = (float)(u - 16.0 * t[a]);
  }
  return tl.index[(t[2] * tl.T + t[1]) * tl.T + t[0]];
}

// texel cell and weight of a tile coordinate along one plane axis
__device__ __forceinline__ void plane_texel(float l, int& c0, float& f) {
  const float tau = fminf(fmaxf(l - 0.5f, 0.0f), 15.0f);
  const float c = fminf(floorf(tau), 14.0f);
  c0 = (int)c;
  f = tau - c;
}

// bilinear value of plane a of a tile (all NF channels), its 4 texels and weights
template <typename FT>
__device__ __forceinline__ void plane_lookup(const FT* __restrict__ planes, int slot, int a,
                                             const float loc[3], float val[NF], int idx[4],
                                             float w[4]) {
  const int ua = a == 0 ? 1 : 0, va = a == 2 ? 1 : 2;  // plane axes (y,z), (x,z), (x,y)
  int cu, cv;
  float fu, fv;
  plane_texel(loc[ua], cu, fu);
  plane_texel(loc[va], cv, fv);
  idx[0] = cv * 16 + cu;
  idx[1] = idx[0] + 1;
  idx[2] = idx[0] + 16;
  idx[3] = idx[0] + 17;
  w[0] = (1.f - fu) * (1.f - fv);
  w[1] = fu * (1.f - fv);
  w[2] = (1.f - fu) * fv;
  w[3] = fu * fv;
  const int base = (slot * 3 + a) * 256;
#pragma unroll
  for (int ch = 0; ch < NF; ++ch) {
    float acc = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc = fmaf(w[q], ld1(planes, (base + idx[q]) * NF + ch), acc);
    val[ch] = acc;
  }
}

template <typename FT>
__device__ __forceinline__ void triplane_fs(const FT* __restrict__ planes, int slot,
                                            const float loc[3], float fs[NF]) {
#pragma unroll
  for (int ch = 0; ch < NF; ++ch) fs[ch] = 1.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float val[NF], w[4];
    int idx[4];
    plane_lookup(planes, slot, a, loc, val, idx, w);
#pragma unroll
    for (int ch = 0; ch < NF; ++ch) fs[ch] *= val[ch];
  }
}

// reverse mode: dF_s into the plane gradient g (FP32 atomics, 36 per sample)
template <typename FT>
__device__ __forceinline__ void triplane_scatter(const FT* __restrict__ planes, int slot,
                                                 const float loc[3], const float dfs[NF],
                                                 float* __restrict__ g) {
  float val[3][NF], w[3][4];
  int idx[3][4];
#pragma unroll
  for (int a = 0; a < 3; ++a) plane_lookup(planes, slot, a, loc, val[a], idx[a], w[a]);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int base = (slot * 3 + a) * 256;
#pragma unroll
    for (int ch = 0; ch < NF; ++ch) {
      const float other = val[(a + 1) % 3][ch] * val[(a + 2) % 3][ch];
      const float d = dfs[ch] * other;
      if (d == 0.f) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) atomic_add_f32(g + (base + idx[a][q]) * NF + ch, w[a][q] * d);
    }
  }
}

// shading state of one sample kept for its reverse mode
template <int NSH>
struct ModelShade {
  float z[MNIN];
  Normal nm;     // n, |g|, c = n.v (the true cosine, also under FLAG_NV_ONE)
  float arg[3];  // SH argument: v or r
  float Y[NSH];
};

// MLP inputs z = [F_s, F_a(arg), incidence inputs] of one sample at FP64 position x
template <typename ST, typename FT, int NSH>
__device__ __forceinline__ void model_inputs(const ST* __restrict__ sdf, const FT* __restrict__ feat,
                                             const FT* __restrict__ probes, const Geo& G,
                                             const Tiles& tl, const double x[3], const float v[3],
                                             ModelShade<NSH>& S) {
  const Cell cs = cell_d(x, G.R, G.inv_h);
  if (!sdf_normal_cross(sdf, G, x, cs, S.nm)) sdf_normal(sdf, G, x, S.nm);
  const float c = S.nm.n[0] * v[0] + S.nm.n[1] * v[1] + S.nm.n[2] * v[2];
  S.nm.c = c;
  if (G.flags & FLAG_SH_REFLECT) {
#pragma unroll
    for (int a = 0; a < 3; ++a) S.arg[a] = 2.0f * c * S.nm.n[a] - v[a];
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) S.arg[a] = v[a];
  }
  sh_basis<NSH>(S.arg[0], S.arg[1], S.arg[2], S.Y);
#pragma unroll
  for (int j = 0; j < MNIN; ++j) S.z[j] = 0.0f;
  if (!(G.flags & FLAG_NO_FS) && tl.index) {
    float loc[3];
    const int slot = tile_slot(tl, G.R, G.inv_h, x, loc);
    if (slot >= 0) triplane_fs(feat, slot, loc, S.z);
  } else if (!(G.flags & FLAG_NO_FS)) {
    float w[8];
    corner_w(cs, w);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int node = cs.base + corner_off(q, G.R);
#pragma unroll
      for (int ch = 0; ch < NF; ++ch) S.z[ch] = fmaf(w[q], ld1(feat, node * NF + ch), S.z[ch]);
    }
  }
  if (!(G.flags & FLAG_NO_FA)) {
    const Cell cp = cell_d(x, G.P, G.inv_hp);
    float w[8];
    corner_w(cp, w);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int off = (cp.base + corner_off(q, G.P)) * (NSH * NA);
      float q0 = 0.f, q1 = 0.f, q2 = 0.f, q3 = 0.f;
#pragma unroll
      for (int j = 0; j < NSH; ++j) {
        const float4 b = ld4(probes, off + 4 * j);
        q0 = fmaf(S.Y[j], b.x, q0);
        q1 = fmaf(S.Y[j], b.y, q1);
        q2 = fmaf(S.Y[j], b.z, q2);
        q3 = fmaf(S.Y[j], b.w, q3);
      }
      S.z[3] = fmaf(w[q], q0, S.z[3]);
      S.z[4] = fmaf(w[q], q1, S.z[4]);
      S.z[5] = fmaf(w[q], q2, S.z[5]);
      S.z[6] = fmaf(w[q], q3, S.z[6]);
    }
  }
  const float ci = (G.flags & FLAG_NV_ONE) ? 1.0f : c;
  if (G.flags & FLAG_FRESNEL_PAPER) {
    const float u = 1.0f - ci;
    float p = 1.0f;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      S.z[NF + NA + m] = p;
      p *= u;
    }
  } else {
    const float c2 = ci * ci;
    S.z[7] = ci;
    S.z[8] = c2;
    S.z[9] = c2 * c2;
  }
}

// ---------------------------------------------------------------------------
// MLP, per lane.  Reduced modes round the weights, the inputs and the hidden
// activations to FP16 / BF16 (nearest even) and accumulate in FP32.
// ---------------------------------------------------------------------------
// WR: the weights (not the biases) are already rounded as mrnd<M> rounds them (a
// reduced-precision copy in LDS, model_round_mlp), else they are rounded on use
template <int M, int H, int L, bool WR = false, typename WT>
__device__ __forceinline__ void model_mlp_fwd(WT* __restrict__ W, int nin, const float z[MNIN],
                                              float pre[L * H], float out[3]) {
#pragma unroll
  for (int k = 0; k < H; ++k) {
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < MNIN; ++j)
      if (j < nin) acc = fmaf(wrnd<M, WR>(W[k * nin + j]), mrnd<M>(z[j]), acc);
    pre[k] = acc + W[H * nin + k];
  }
  int off = H * nin + H;
  if constexpr (L == 2) {
#pragma unroll
    for (int k = 0; k < H; ++k) {
      float acc = 0.0f;
#pragma unroll
      for (int j = 0; j < H; ++j)
        acc = fmaf(wrnd<M, WR>(W[off + k * H + j]), mrnd<M>(fmaxf(pre[j], 0.0f)), acc);
      pre[H + k] = acc + W[off + H * H + k];
    }
    off += H * H + H;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < H; ++k)
      acc = fmaf(wrnd<M, WR>(W[off + c * H + k]), mrnd<M>(fmaxf(pre[(L - 1) * H + k], 0.0f)),
                 acc);
    out[c] = acc + W[off + 3 * H + c];
  }
}

// reverse mode: dpre (pre-activation cotangents of every layer) and dz
template <int M, int H, int L, bool WR = false, typename WT>
__device__ __forceinline__ void model_mlp_bwd(WT* __restrict__ W, int nin, const float pre[L * H],
                                              const float dout[3], float dpre[L * H],
                                              float dz[MNIN]) {
  const int off1 = H * nin + H;
  const int offo = off1 + (L - 1) * (H * H + H);
#pragma unroll
  for (int k = 0; k < H; ++k) {
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) acc = fmaf(wrnd<M, WR>(W[offo + c * H + k]), dout[c], acc);
    dpre[(L - 1) * H + k] = pre[(L - 1) * H + k] > 0.0f ? acc : 0.0f;
  }
  if constexpr (L == 2) {
#pragma unroll
    for (int j = 0; j < H; ++j) {
      float acc = 0.0f;
#pragma unroll
      for (int k = 0; k < H; ++k) acc = fmaf(wrnd<M, WR>(W[off1 + k * H + j]), dpre[H + k], acc);
      dpre[j] = pre[j] > 0.0f ? acc : 0.0f;
    }
  }
#pragma unroll
  for (int j = 0; j < MNIN; ++j) {
    float acc = 0.0f;
    if (j < nin) {
#pragma unroll
      for (int k = 0; k < H; ++k) acc = fmaf(wrnd<M, WR>(W[k * nin + j]), dpre[k], acc);
    }
    dz[j] = acc;
  }
}

// largest packed MLP of the paper models (13 inputs, two hidden layers of 32)
constexpr int MODEL_MLP_MAX = model_mlp_size(MNIN, 32, 2);

// copy of the packed MLP with its weights (not its biases) rounded for arithmetic M;
// called by the whole wave, which then reads it from LDS (broadcast reads)
template <int M>
__device__ __forceinline__ void model_round_mlp(const float* __restrict__ W, float* dst, int nin,
                                                int H, int L, int lane) {
  const int n = model_mlp_size(nin, H, L);
  const int b0 = H * nin, w1 = b0 + H, b1 = w1 + (L - 1) * H * H, wo = b1 + (L - 1) * H,
            bo = wo + 3 * H;
  for (int i = lane; i < n; i += 64) {
    const bool bias = (i >= b0 && i < w1) || (L == 2 && i >= b1 && i < wo) || i >= bo;
    dst[i] = bias ? W[i] : mrnd<M>(W[i]);
  }
}

// Probe gradients of a batch of samples (one per lane): dL/db_{node,j,k} = w_c Y_j dL/dF_a,k
// over the 8 corners c of each sample's probe cell.  The samples' corner weights, SH values
// and dL/dF_a are staged in LDS; then, for each distinct cell of the batch, lane q
// (coefficient j = q / 4, k = q % 4) sums its coefficient over the cell's samples in lane
// order for the 8 corners and adds them with one coalesced run of global atomics per
// corner.  No LDS atomics: samples of one cell are common in a batch, and LDS atomics on a
// shared slot serialise.
template <int NSH>
struct ProbeStage {
  int key[64];
  float w8[64][9];
  float y[64][NSH + 1];
  float dfa[64][NA + 1];
};

template <int NSH>
__device__ __forceinline__ void probe_scatter_lanes(ProbeStage<NSH>& S, int lane, bool ve,
                                                    const Cell& cp, int P, const float* Y,
                                                    const float* dFa, float* g_probes) {
  constexpr int NC = NSH * NA;  // coefficients of a probe node
  static_assert(NC <= 64, "one lane per coefficient");
  const int mykey = ve ? cp.base : -1;
  float w[8];
  corner_w(cp, w);
#pragma unroll
  for (int c = 0; c < 8; ++c) S.w8[lane][c] = w[c];
#pragma unroll
  for (int j = 0; j < NSH; ++j) S.y[lane][j] = Y[j];
#pragma unroll
  for (int k = 0; k < NA; ++k) S.dfa[lane][k] = dFa[k];
  wave_sync();
  const int jq = lane / NA, kq = lane - NA * jq;
  uint64_t todo = __ballot(ve);
  while (todo) {  // wave-uniform: one distinct cell per round
    const int leader = __builtin_ctzll(todo);
    const int key = __builtin_amdgcn_readlane(mykey, leader);
    uint64_t mm = __ballot(ve && mykey == key);
    todo &= ~mm;
    if (lane < NC) {
      float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      while (mm) {
        const int sm = __builtin_ctzll(mm);
        mm &= mm - 1;
        const float yd = S.y[sm][jq] * S.dfa[sm][kq];
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = fmaf(S.w8[sm][c], yd, acc[c]);
      }
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (acc[c] != 0.f)
          atomic_add_f32(g_probes + (int64_t)(key + corner_off(c, P)) * NC + lane, acc[c]);
    }
  }
  wave_sync();
}

// The MLP of a wave's 64 samples on MFMA (FP16 or BF16 operands, FP32 accumulation),
// from the rounded copy `Wr` in LDS.  Samples lie on the N dimension, in four blocks
// of 16: a layer's accumulator fragment (lane i + 16 g holds hidden units 4g .. 4g+3
// of sample i of the block) is exactly the B operand of the next layer, so only the
// inputs and the outputs pass through LDS.  Every lane of the wave calls it (lanes
// without a sample pass zero inputs).
//   H0^T = W0 (H x 16 padded inputs) . Z^T,  H1^T = W1 (H x H) . relu(H0^T + b0),
//   O^T = Wo (16 padded outputs x H) . relu(H_{L-1}^T + b_{L-1})
template <int M>
struct ModelMfmaLds {
  typename MType<M>::t zs[64][16];
  float cs[64][4];
};

template <int M, int H, int L>
__device__ __forceinline__ void model_mlp_wave(const float* Wr, int nin, ModelMfmaLds<M>& S,
                                               int lane, const float z[MNIN], float out[3]) {
  typedef typename MType<M>::t T;
  typedef typename MType<M>::v V4;
  constexpr int NT = H / 16;  // 16-row tiles of a hidden layer
  const int i = lane & 15, g = lane >> 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    V4 zq;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = 4 * q + r;
      zq[r] = (T)(k < MNIN && k < nin ? z[k < MNIN ? k : 0] : 0.0f);
    }
    *reinterpret_cast<V4*>(&S.zs[lane][4 * q]) = zq;
  }
  const int ob0 = H * nin, ow1 = ob0 + H, ob1 = ow1 + (L - 1) * H * H, owo = ob1 + (L - 1) * H,
            obo = owo + 3 * H;
  V4 a0[NT], ao[NT];
  float bb0[NT][4], bo[4];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = 4 * g + r;
      a0[t][r] = (T)(k < nin ? Wr[(16 * t + i) * nin + k] : 0.0f);
      bb0[t][r] = Wr[ob0 + 16 * t + k];
      ao[t][r] = (T)(i < 3 ? Wr[owo + i * H + 16 * t + k] : 0.0f);
    }
#pragma unroll
  for (int r = 0; r < 4; ++r) bo[r] = 4 * g + r < 3 ? Wr[obo + 4 * g + r] : 0.0f;
  wave_sync();
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const V4 bz = *reinterpret_cast<const V4*>(&S.zs[16 * b + i][4 * g]);
    V4 h[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      f4 d = {0.f, 0.f, 0.f, 0.f};
      d = MType<M>::mma(a0[t], bz, d);
#pragma unroll
      for (int r = 0; r < 4; ++r) h[t][r] = (T)fmaxf(d[r] + bb0[t][r], 0.0f);
    }
    if constexpr (L == 2) {
      V4 h2[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        f4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < NT; ++kt) {
          V4 a1;
#pragma unroll
          for (int r = 0; r < 4; ++r) a1[r] = (T)Wr[ow1 + (16 * t + i) * H + 16 * kt + 4 * g + r];
          d = MType<M>::mma(a1, h[kt], d);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) h2[t][r] = (T)fmaxf(d[r] + Wr[ob1 + 16 * t + 4 * g + r], 0.0f);
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) h[t] = h2[t];
    }
    f4 o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < NT; ++kt) o = MType<M>::mma(ao[kt], h[kt], o);
    if (g == 0) {
      S.cs[16 * b + i][0] = o[0] + bo[0];
      S.cs[16 * b + i][1] = o[1] + bo[1];
      S.cs[16 * b + i][2] = o[2] + bo[2];
    }
  }
  wave_sync();
  out[0] = S.cs[lane][0];
  out[1] = S.cs[lane][1];
  out[2] = S.cs[lane][2];
  wave_sync();
}

// ---------------------------------------------------------------------------
// MLP weight gradients of a batch of samples (one per lane) as outer-product sums
// on FP32 MFMA, in 16 x 16 tiles (rows: a layer's outputs; columns: its inputs
// followed by a column of ones for the bias).  Accumulated over the batches of a
// wave and flushed with one atomic per parameter.
// ---------------------------------------------------------------------------
template <int H, int L>
struct ModelDw {
  static constexpr int RB = (H + 15) / 16;   // row blocks of a hidden layer
  static constexpr int CBH = (H + 16) / 16;  // column blocks of H inputs + bias
  static constexpr int N0 = RB;              // layer 0: n_in + 1 <= 16 columns
  static constexpr int N1 = L == 2 ? RB * CBH : 0;
  static constexpr int NO = CBH;             // output layer: 3 rows
  f4 t0[N0];
  f4 t1[N1 > 0 ? N1 : 1];
  f4 to[NO];
};

template <int H, int L>
__device__ __forceinline__ void model_dw_zero(ModelDw<H, L>& D) {
  const f4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < ModelDw<H, L>::N0; ++i) D.t0[i] = zero;
#pragma unroll
  for (int i = 0; i < (ModelDw<H, L>::N1 > 0 ? ModelDw<H, L>::N1 : 1); ++i) D.t1[i] = zero;
#pragma unroll
  for (int i = 0; i < ModelDw<H, L>::NO; ++i) D.to[i] = zero;
}

// column block cb of an input vector of n values followed by the bias 1 (ve lanes)
template <int NV>
__device__ __forceinline__ void dw_cols(const float* in, int n, int cb, bool ve, float col[16]) {
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int j = 16 * cb + q;  // a constant once the loops are unrolled
    float val = 0.0f;
    if (j < NV && j < n) val = in[j < NV ? j : 0];
    if (j == n) val = ve ? 1.0f : 0.0f;
    col[q] = val;
  }
}

template <int M, int H, int L>
__device__ __forceinline__ void model_dw_batch(DwLds& lds, int lane, bool ve, int nin,
                                               const float z[MNIN], const float pre[L * H],
                                               const float dpre[L * H], const float dout[3],
                                               ModelDw<H, L>& D) {
  using DW = ModelDw<H, L>;
  float zr[MNIN], h[L * H];
#pragma unroll
  for (int j = 0; j < MNIN; ++j) zr[j] = ve ? mrnd<M>(z[j]) : 0.0f;
#pragma unroll
  for (int k = 0; k < L * H; ++k) h[k] = ve ? mrnd<M>(fmaxf(pre[k], 0.0f)) : 0.0f;
  float row[16], col[16];
  // layer 0: rows = hidden units, columns = inputs + bias
  dw_cols<MNIN>(zr, nin, 0, ve, col);
#pragma unroll
  for (int rb = 0; rb < DW::N0; ++rb) {
#pragma unroll
    for (int q = 0; q < 16; ++q) row[q] = (16 * rb + q < H && ve) ? dpre[16 * rb + q] : 0.0f;
    dw_accumulate(lds, lane, row, col, D.t0[rb]);
  }
  if constexpr (L == 2) {
#pragma unroll
    for (int cb = 0; cb < DW::CBH; ++cb) {
      dw_cols<H>(h, H, cb, ve, col);
#pragma unroll
      for (int rb = 0; rb < DW::RB; ++rb) {
#pragma unroll
        for (int q = 0; q < 16; ++q)
          row[q] = (16 * rb + q < H && ve) ? dpre[H + 16 * rb + q] : 0.0f;
        dw_accumulate(lds, lane, row, col, D.t1[rb * DW::CBH + cb]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) row[q] = (q < 3 && ve) ? dout[q] : 0.0f;
#pragma unroll
  for (int cb = 0; cb < DW::CBH; ++cb) {
    dw_cols<H>(h + (L - 1) * H, H, cb, ve, col);
    dw_accumulate(lds, lane, row, col, D.to[cb]);
  }
}

// adds tile (rows r0.., columns c0..) of a layer with `nr` outputs and `nc` inputs
// (column nc = bias) into the packed gradient at W (weights) and Bv (biases)
__device__ __forceinline__ void dw_tile_flush(const f4& t, int lane, int r0, int c0, int nr, int nc,
                                              float* Wg, float* Bg) {
  const int i = lane & 15, g = lane >> 4;
  const int col = c0 + i;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int row = r0 + 4 * g + rr;
    if (row >= nr || t[rr] == 0.0f) continue;
    if (col < nc) atomic_add_f32(Wg + row * nc + col, t[rr]);
    else if (col == nc) atomic_add_f32(Bg + row, t[rr]);
  }
}

template <int H, int L>
__device__ __forceinline__ void model_dw_flush(const ModelDw<H, L>& D, int lane, int nin,
                                               float* g) {
  using DW = ModelDw<H, L>;
#pragma unroll
  for (int rb = 0; rb < DW::N0; ++rb) dw_tile_flush(D.t0[rb], lane, 16 * rb, 0, H, nin, g, g + H * nin);
  int off = H * nin + H;
  if constexpr (L == 2) {
#pragma unroll
    for (int rb = 0; rb < DW::RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < DW::CBH; ++cb)
        dw_tile_flush(D.t1[rb * DW::CBH + cb], lane, 16 * rb, 16 * cb, H, H, g + off,
                      g + off + H * H);
    off += H * H + H;
  }
#pragma unroll
  for (int cb = 0; cb < DW::CBH; ++cb) dw_tile_flush(D.to[cb], lane, 0, 16 * cb, 3, H, g + off, g + off + 3 * H);
}

// Cotangent of the FD gradient g of the SDF at a sample: through the incidence
// inputs (c = n.v) and, with the reflected SH argument, through r = 2 (n.v) n - v.
//   e: for the reflected argument, e_j = sum_k bhat_jk dF_a,k (else unused)
template <int NSH>
__device__ __forceinline__ void model_normal_dg(const ModelShade<NSH>& S, const float v[3],
                                                const float dz[MNIN], const float e[NSH],
                                                int flags, float dg[3]) {
  float dn[3] = {0.f, 0.f, 0.f};
  const float c = S.nm.c;
  if (!(flags & FLAG_NV_ONE)) {
    float dc;
    if (flags & FLAG_FRESNEL_PAPER) {
      // d/dc (1 - c)^m = -m (1 - c)^(m-1)
      const float u = 1.0f - c;
      float p = 1.0f;
      dc = 0.0f;
#pragma unroll
      for (int m = 1; m < 6; ++m) {
        dc = fmaf(-(float)m * p, dz[NF + NA + m], dc);
        p *= u;
      }
    } else {
      dc = dz[7] + 2.0f * c * dz[8] + 4.0f * c * c * c * dz[9];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) dn[a] = dc * v[a];
  }
  if ((flags & FLAG_SH_REFLECT) && !(flags & FLAG_NO_FA)) {
    float dY[NSH][3];
    sh_grad<NSH>(S.arg[0], S.arg[1], S.arg[2], dY);
    float dr[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < NSH; ++j)
#pragma unroll
      for (int a = 0; a < 3; ++a) dr[a] = fmaf(e[j], dY[j][a], dr[a]);
    const float rn = dr[0] * S.nm.n[0] + dr[1] * S.nm.n[1] + dr[2] * S.nm.n[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) dn[a] += 2.0f * rn * v[a] + 2.0f * c * dr[a];
  }
  if (S.nm.gn >= 1e-30f) {
    const float nd = dn[0] * S.nm.n[0] + dn[1] * S.nm.n[1] + dn[2] * S.nm.n[2];
    const float inv = 1.0f / S.nm.gn;
#pragma unroll
    for (int a = 0; a < 3; ++a) dg[a] = (dn[a] - nd * S.nm.n[a]) * inv;
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) dg[a] = dn[a] / 1e-30f;
  }
}

// e_j = sum_k bhat_jk dF_a,k, with bhat_j the trilinear probe coefficients at x
template <typename FT, int NSH>
__device__ __forceinline__ void probe_contract(const FT* __restrict__ probes, const Geo& G,
                                               const double x[3], const float dfa[NA],
                                               float e[NSH]) {
  const Cell cp = cell_d(x, G.P, G.inv_hp);
  float w[8];
  corner_w(cp, w);
#pragma unroll
  for (int j = 0; j < NSH; ++j) e[j] = 0.f;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int off = (cp.base + corner_off(q, G.P)) * (NSH * NA);
#pragma unroll
    for (int j = 0; j < NSH; ++j) {
      const float4 b = ld4(probes, off + 4 * j);
      const float d = b.x * dfa[0] + b.y * dfa[1] + b.z * dfa[2] + b.w * dfa[3];
      e[j] = fmaf(w[q], d, e[j]);
    }
  }
}

}  // namespace psdf
