// Reverse mode of the ProbeSDF render step (Sec. 3.3: the SDF grid and the
// appearance are optimised by back-propagating the colour loss through the
// rendering equation).  The march is recomputed; nothing is stored per sample.
//
// With log(1 - alpha_i) = dl_i = log Phi(s_{i+1}) - log Phi(s_i) and the colour
// remaining from sample i on, R_i = sum_{j>=i} w_j C_j (R_0 = rgb from the
// forward's aux, R_{i+1} = R_i - w_i C_i; this single-kernel schedule meets the
// samples in march order, so it cannot sum R_i from the back as the workspace
// schedules do, and clamps it to its exact range [0, T_i] instead):
//   dL/dC_i   = w_i dL/drgb,
//   dL/d dl_i = dL/drgb . (R_i - T_i C_i),
//   d dl_i/d s_i = -tau sigma(-tau s_i),  d dl_i/d s_{i+1} = tau sigma(-tau s_{i+1}).
// As in the forward, one ray per lane marches and queues its shaded samples
// (weight, T_i, s_i, s_{i+1}) in a per-wave LDS ring; full batches of 64 are
// shaded one sample per lane; the ray's own lane then walks its entries in
// sample order to produce dL/d dl_i; finally every lane back-propagates its
// sample through the MLP and the interpolations and scatters the gradients
// with FP32 atomics.  MLP weight gradients accumulate as MFMA outer-product
// sums over the batch and are flushed once per wave.
#include "bwd_common.h"
#include "dispatch.h"

namespace psdf {

template <int NSH>
struct BwdLds {
  union {
    DwLds dw;            // MLP weight-gradient staging
    ProbeAcc<NSH> pa;    // probe-gradient aggregation
    float sc[64][65];    // per-entry scatter rows: SDF patch, feature corners
  } u;
  int k0[64][3];         // per entry: SDF cell (patch origin + 1)
  int fb[64];            // per entry: feature cell base node
  RayD ray[64];
  float dL[64][3];
  int next[RING];
  int key[RING];  // (sample index << 6) | ray lane
  float w[RING];
  float T[RING];
  float s0[RING];  // s_i
  float s1[RING];  // s_{i+1}
  float gdl[RING];
  float C[RING][3];
};

template <typename ST, typename FT, int NSH, int M>
__device__ __forceinline__ void bwd_batch(const RenderArgs& a, const Geo& G, BwdLds<NSH>& L,
                                          int lane, int head, int n, float R[3], int& my_first,
                                          int& my_cnt, f4& acc_w1, f4& acc_w2, float db2[3]) {
  const ST* __restrict__ sdf = static_cast<const ST*>(a.sdf);
  const FT* __restrict__ feat = static_cast<const FT*>(a.feat);
  const FT* __restrict__ probes = static_cast<const FT*>(a.probes);
  cfloat* __restrict__ W = const_mlp(a.mlp);  // scalar loads
  wave_sync();
  const bool ve = lane < n;
  const int slot = (head + lane) & (RING - 1);
  float z[NIN];
#pragma unroll
  for (int j = 0; j < NIN; ++j) z[j] = 0.f;
  Normal nm;
  nm.n[0] = nm.n[1] = nm.n[2] = 0.f;
  nm.gn = 1.f;
  nm.c = 0.f;
  int key = 0;
  RayD r;
  float v[3] = {0.f, 0.f, 0.f}, Y[NSH];
  double x[3] = {0.0, 0.0, 0.0};
  if (ve) {
    key = L.key[slot];
    r = L.ray[key & 63];
    sample_pos(r, sample_t(r, key >> 6), x);
    v[0] = (float)-r.d[0];
    v[1] = (float)-r.d[1];
    v[2] = (float)-r.d[2];
    sh_basis<NSH>(v[0], v[1], v[2], Y);
    shade_inputs<ST, FT, NSH>(sdf, feat, probes, G, x, v, Y, z, nm);
  }
  float pre[HID], hid[HID], out[3];
  mlp_lane<M>(W, z, pre, hid, out);
  const float C0 = sigmoidf(out[0]), C1 = sigmoidf(out[1]), C2 = sigmoidf(out[2]);
  if (ve) {
    L.C[slot][0] = C0;
    L.C[slot][1] = C1;
    L.C[slot][2] = C2;
  }
  wave_sync();
  // the ray's lane walks its entries of this batch in sample order
  {
    const float dl0 = L.dL[lane][0], dl1 = L.dL[lane][1], dl2 = L.dL[lane][2];
    while (my_cnt > 0 && my_first < head + n) {
      const int s = my_first & (RING - 1);
      const float w = L.w[s], T = L.T[s];
      const float c0 = L.C[s][0], c1 = L.C[s][1], c2 = L.C[s][2];
      // R_i = rgb - sum_{j<i} w_j C_j cancels where T_i is below the rounding error of
      // rgb; the exact R_i lies in [0, T_i] (0 < C < 1, the weights from i on sum to at
      // most T_i), so the clamp bounds the error of R_i by min(T_i, error of the subtraction)
      const float r0 = fminf(fmaxf(R[0], 0.f), T), r1 = fminf(fmaxf(R[1], 0.f), T),
                  r2 = fminf(fmaxf(R[2], 0.f), T);
      L.gdl[s] = dl0 * (r0 - T * c0) + dl1 * (r1 - T * c1) + dl2 * (r2 - T * c2);
      R[0] -= w * c0;
      R[1] -= w * c1;
      R[2] -= w * c2;
      if (--my_cnt > 0) my_first = L.next[s];
    }
  }
  wave_sync();
  float dout[3] = {0.f, 0.f, 0.f};
  float gs0 = 0.f;  // dL/ds_i through the opacity
  if (ve) {
    const float gdl = L.gdl[slot];
    const float w = L.w[slot];
    const int rl = key & 63, si = key >> 6;
    if (a.g_sdf) {
      gs0 = -a.tau * sigmoidf(-a.tau * L.s0[slot]) * gdl;
      // s_{i+1} lies a sample further along the ray: scattered directly
      double x1[3];
      sample_pos(r, sample_t(r, si + 1), x1);
      scatter8(a.g_sdf, G.R, cell_d(x1, G.R, G.inv_h), a.tau * sigmoidf(-a.tau * L.s1[slot]) * gdl);
    }
    dout[0] = w * L.dL[rl][0] * C0 * (1.f - C0);
    dout[1] = w * L.dL[rl][1] * C1 * (1.f - C1);
    dout[2] = w * L.dL[rl][2] * C2 * (1.f - C2);
  }
  float dpre[HID], dz[NIN];
  mlp_backward_lane<M>(W, dout, pre, ve, dpre, dz);
  // SDF: opacity path at s_i and the normal path, in the entry's 4x4x4 patch
  if (a.g_sdf) {
    float* row = L.u.sc[lane];
#pragma unroll
    for (int q = 0; q < 64; ++q) row[q] = 0.f;
    if (ve) {
      int k0[3];
      cell_k(x, G.R, G.inv_h, k0);
      L.k0[lane][0] = k0[0];
      L.k0[lane][1] = k0[1];
      L.k0[lane][2] = k0[2];
      if (gs0 != 0.f) patch_add(patch_of_row(row, k0), k0, x, G.R, G.inv_h, gs0);
      if (!(G.flags & FLAG_NV_ONE)) normal_backward_patch(patch_of_row(row, k0), k0, G, x, v, nm, dz);
    }
    wave_sync();
    sdf_patch_flush(L.u.sc, L.k0, n, lane, G.R, a.g_sdf);
    wave_sync();
  }
  // spatial features
  if (!(G.flags & FLAG_NO_FS) && a.g_feat)
    feat_scatter_wave(L.u.sc, L.fb, ve, cell_d(x, G.R, G.inv_h), dz, n, lane, G.R, a.g_feat);
  // probes: aggregated per distinct probe cell of the batch
  if (!(G.flags & FLAG_NO_FA) && a.g_probes) {
    probe_acc_clear<NSH>(L.u.pa, lane);
    const float dfa[4] = {dz[3], dz[4], dz[5], dz[6]};
    probe_scatter_wave<NSH>(L.u.pa, lane, ve, ve ? cell_d(x, G.P, G.inv_hp) : Cell{0, 0.f, 0.f, 0.f},
                            G.P, Y, dfa, a.g_probes);
  }
  if (a.g_mlp) mlp_dw_wave<M>(L.u.dw, lane, ve, z, hid, dpre, dout, acc_w1, acc_w2, db2);
  wave_sync();
}

template <typename ST, typename FT, int NSH, int M>
__global__ void __launch_bounds__(BLOCK) render_bwd_kernel(RenderArgs a) {
  __shared__ BwdLds<NSH> lds[WAVES];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  BwdLds<NSH>& L = lds[wv];
  const ST* __restrict__ sdf = static_cast<const ST*>(a.sdf);
  const Geo G{a.R, a.P, 2.0 / (a.R - 1), 0.5 * (a.R - 1), 0.5 * (a.P - 1), a.flags};

  const unsigned lw = xcd_block(blockIdx.x, gridDim.x) * WAVES + wv;  // this wave's 64 rays
  if ((int64_t)lw * 64 >= a.B) return;
  if (a.todo && a.todo[lw] == 0) return;  // only the listed waves (wave-uniform)
  const int64_t ray = (int64_t)lw * 64 + lane;
  const bool valid = ray < a.B;
  float ro[3] = {0.f, 0.f, 0.f}, rd[3] = {0.f, 0.f, 1.f}, dL[3] = {0.f, 0.f, 0.f};
  float R[3] = {0.f, 0.f, 0.f};
  if (valid) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ro[k] = a.rays_o[3 * ray + k];
      rd[k] = a.rays_d[3 * ray + k];
      dL[k] = a.dL[3 * ray + k];
      R[k] = a.aux_in[4 * ray + k];
    }
  }
  RayD r;
  // rays that carry no loss gradient contribute nothing
  const bool hit = ray_setup_d(ro[0], ro[1], ro[2], rd[0], rd[1], rd[2], a.N, r) && valid &&
                   (dL[0] != 0.f || dL[1] != 0.f || dL[2] != 0.f);
  L.ray[lane] = r;
  L.dL[lane][0] = dL[0];
  L.dL[lane][1] = dL[1];
  L.dL[lane][2] = dL[2];

  f4 acc_w1 = {0.f, 0.f, 0.f, 0.f}, acc_w2 = {0.f, 0.f, 0.f, 0.f};
  float db2[3] = {0.f, 0.f, 0.f};
  bool any_batch = false;
  float logT = 0.f;
  int my_first = 0, my_last = 0, my_cnt = 0;
  int head = 0, tail = 0;
  const Bricks K = make_bricks(a.bounds, a.R, a.skip_thr);
  MarchState ms;
  march_begin(sdf, a.R, K, r, G.inv_h, hit, a.N, ms);
  for (int i = 0;; ++i) {
    const bool stepping = i < a.N - 1;  // wave-uniform
    if (stepping) {
      float s_i, s_n;
      bool may;
      march_next(sdf, a.R, K, hit, i, a.N, ms, s_i, s_n, may);
      const bool active = may && (a.skip_thr <= 0.f || fabsf(s_i) <= a.skip_thr);
      bool shaded = false;
      float dl = 0.f;
      if (active) {
        dl = log_sigmoid(a.tau * s_n) - log_sigmoid(a.tau * s_i);
        shaded = dl < 0.f;
      }
      const uint64_t mask = __ballot(shaded);
      if (shaded) {
        const float T = expf(logT);
        const int seq = tail + lane_rank(mask);
        const int slot = seq & (RING - 1);
        L.key[slot] = (i << 6) | lane;
        L.w[slot] = T * -expm1f(dl);
        L.T[slot] = T;
        L.s0[slot] = s_i;
        L.s1[slot] = s_n;
        if (my_cnt > 0) L.next[my_last & (RING - 1)] = seq;
        else my_first = seq;
        my_last = seq;
        ++my_cnt;
        logT += dl;
      }
      tail += __popcll(mask);
    }
    const int pending = tail - head;
    if (pending >= 64 || (!stepping && pending > 0)) {
      const int n = min(64, pending);
      bwd_batch<ST, FT, NSH, M>(a, G, L, lane, head, n, R, my_first, my_cnt, acc_w1, acc_w2,
                                db2);
      head += n;
      any_batch = true;
    } else if (!stepping) {
      break;
    }
  }
  // flush this wave's MLP gradients (any_batch is wave-uniform)
  if (any_batch && a.g_mlp) mlp_grad_flush(a.g_mlp, lane, acc_w1, acc_w2, db2);
}

hipError_t launch_render_backward(const RenderArgs& a, int sdf_dt, int feat_dt, int mlp_dt,
                                  int n_sh, hipStream_t s) {
  const dim3 grid((unsigned)((a.B + BLOCK - 1) / BLOCK));
  PSDF_DT_SWITCH(sdf_dt, feat_dt, PSDF_SH_SWITCH(n_sh, PSDF_MLP_SWITCH(mlp_dt,
      hipLaunchKernelGGL((render_bwd_kernel<ST, FT, NSH, M>), grid, dim3(BLOCK), 0, s, a))));
  return hipGetLastError();
}

}  // namespace psdf
