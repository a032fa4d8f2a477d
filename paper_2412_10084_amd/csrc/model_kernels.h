// Kernels of the render step of the paper's own colour model (model.h): forward
// and reverse mode with one ray per wave and one sample per lane.
//
// A wave marches its rays one at a time.  The 64 lanes evaluate 64 consecutive
// samples of the ray at once (s_i by trilinear interpolation, s_{i+1} from the
// next lane), the NeuS opacity (Sec. 3.3, Eq. neus, log domain) and the
// transmittance as a wavefront prefix sum of log(1 - alpha) carried from chunk to
// chunk.  The shaded samples (active, alpha > 0) are compacted into LDS and shaded
// 64 per wave instruction stream: in the forward, the shaded samples of 64
// consecutive rays share one queue; in the reverse mode, the list holds the whole
// ray, so the colour remaining behind each sample, R_i = sum_{j>=i} w_j C_j, is an
// exact suffix sum (wavefront suffix scans, last batch first), never a difference.
#pragma once

#include "model.h"

namespace psdf {

// shaded samples of one ray that a wave holds: N <= MODEL_EMAX + 1
constexpr int MODEL_EMAX = 512;

struct ModelEntries {
  int i[MODEL_EMAX];      // sample index
  float w[MODEL_EMAX];    // T_i alpha_i
  float T[MODEL_EMAX];    // T_i
  float s0[MODEL_EMAX];   // s_i
  float s1[MODEL_EMAX];   // s_{i+1}
};

__device__ __forceinline__ float wave_prefix_incl(float v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const float y = __shfl_up(v, d, 64);
    if (lane >= d) v += y;
  }
  return v;
}

__device__ __forceinline__ float wave_suffix_incl(float v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const float y = __shfl_down(v, d, 64);
    if (lane + d < 64) v += y;
  }
  return v;
}

// rays [r0, r1) of this wave: contiguous ranges, remapped so that each XCD
// (with its own L2) takes one contiguous part of the batch
__device__ __forceinline__ void wave_rays(int64_t B, int64_t per_wave, int64_t& r0, int64_t& r1) {
  const int64_t w = xcd_block(blockIdx.x, gridDim.x);
  r0 = w * per_wave;
  r1 = r0 + per_wave < B ? r0 + per_wave : B;
}

// One chunk of 64 consecutive samples c0 .. c0+63 of a ray, one per lane: which
// samples may be active (brick bounds of the SDF when given, the tile when the
// features are tiled), s_i where it is needed (for the sample's own opacity, or
// as s_{i+1} of the previous sample), the skip rule, the log-domain opacity and
// the transmittance as a wavefront prefix sum carried in `carry`.  A chunk where
// no sample may be active costs the tests only.  Returns the ballot of the shaded
// samples (active, alpha > 0); a shaded lane gets its position, w = T alpha, T,
// s_i and s_{i+1}.  prev_may carries whether the chunk's last sample may be active.
struct ChunkOut {
  double x[3];
  float w, T, s0, s1;
};

template <typename ST>
__device__ __forceinline__ uint64_t model_chunk(const ST* __restrict__ sdf, const RenderArgs& a,
                                                const Geo& G, const Tiles& tl, const Bricks& K,
                                                const RayD& r, int c0, int lane, float& carry,
                                                ChunkOut& o) {
  const int N = a.N, i = c0 + lane;
  const bool valid = i < N;
  sample_pos(r, sample_t(r, valid ? i : N - 1), o.x);
  int k[3];
  float f[3];
  const double kmax = (double)(G.R - 2);
#pragma unroll
  for (int q = 0; q < 3; ++q) axis_cell_d(o.x[q], G.inv_h, kmax, k[q], f[q]);
  bool may = valid;
  if (K.b && may) {
    const int br = ((k[2] >> BRICK_SHIFT) * K.nb + (k[1] >> BRICK_SHIFT)) * K.nb + (k[0] >> BRICK_SHIFT);
    may = brick_may(K, K.b[br]);
  }
  if (tl.index && may) {
    float loc[3];
    may = tile_slot(tl, G.R, G.inv_h, o.x, loc) >= 0;
  }
  // lane 63 also evaluates sample c0 + 64, its successor, when it may be active
  const bool has_next = lane == 63 && c0 + 64 < N;
  double xn[3] = {0.0, 0.0, 0.0};
  if (has_next) sample_pos(r, sample_t(r, c0 + 64), xn);
  const uint64_t mm = __ballot(may);
  if (mm == 0) return 0;  // wave-uniform: nothing in this chunk can be active
  const bool prev = lane > 0 ? ((mm >> (lane - 1)) & 1ull) != 0 : false;
  float s_i = 0.0f;
  if (may || prev) {
    Cell c;
    c.base = (k[2] * G.R + k[1]) * G.R + k[0];
    c.fx = f[0];
    c.fy = f[1];
    c.fz = f[2];
    s_i = tri1(sdf, G.R, c);
  }
  float s_n = __shfl_down(s_i, 1, 64);
  if (lane == 63) s_n = (may && has_next) ? tri1(sdf, G.R, cell_d(xn, G.R, G.inv_h)) : 0.0f;
  const bool act = may && i < N - 1 && (a.skip_thr <= 0.f || fabsf(s_i) <= a.skip_thr);
  float dl = 0.0f;
  bool sh = false;
  if (act) {
    dl = log_sigmoid(a.tau * s_n) - log_sigmoid(a.tau * s_i);
    sh = dl < 0.0f;
  }
  const float incl = wave_prefix_incl(sh ? dl : 0.0f, lane);
  float excl = __shfl_up(incl, 1, 64);
  if (lane == 0) excl = 0.0f;
  const uint64_t mask = __ballot(sh);
  if (sh) {
    o.T = expf(carry + excl);
    o.w = o.T * -expm1f(dl);
    o.s0 = s_i;
    o.s1 = s_n;
  }
  carry += __shfl(incl, 63, 64);
  return mask;
}

// Forward (Sec. 3.3: c = sum_i T_i alpha_i C_i).  A wave takes its rays in groups of
// 64: each ray is marched chunk by chunk and its shaded samples join one queue
// shared by the group's rays; whenever 64 are queued the wave shades them together
// (one sample per lane, whatever ray it belongs to).  Each ray's weighted colours
// are summed in sample order by the first lane of its run in the batch.
constexpr int MODEL_Q = 128;     // queue: < 64 waiting plus one chunk of 64
constexpr int MODEL_GROUP = 64;  // rays per group

struct ModelFwdLds {
  double x[MODEL_Q][3];
  float w[MODEL_Q], tm[MODEL_Q];
  int rs[MODEL_Q];                // ray of the entry within the group
  float v[MODEL_GROUP][3];        // view direction of each ray
  float acc[MODEL_GROUP][5];      // rgb, depth, weight sum
  float logT[MODEL_GROUP];
  float part[64][5];              // the batch's per-sample terms
};

template <typename ST, typename FT, int NSH, int M, int H, int L>
__global__ void __launch_bounds__(64) model_fwd_kernel(RenderArgs a, int64_t per_wave) {
  __shared__ ModelFwdLds Q;
  __shared__ ModelMfmaLds<M> MM;  // reduced-precision MLP on MFMA
  const int lane = threadIdx.x;
  const ST* __restrict__ sdf = static_cast<const ST*>(a.sdf);
  const FT* __restrict__ feat = static_cast<const FT*>(a.feat);
  const FT* __restrict__ probes = static_cast<const FT*>(a.probes);
  cfloat* __restrict__ W = const_mlp(a.mlp);
  const Geo G{a.R, a.P, 2.0 / (a.R - 1), 0.5 * (a.R - 1), 0.5 * (a.P - 1), a.flags};
  const Tiles tl{a.tile_index, a.tile_T};
  const Bricks K = make_bricks(a.bounds, a.R, a.skip_thr);
  const int nin = model_n_in(a.flags);
  // reduced-precision MLP: a copy with rounded weights in LDS (rounded once, not on
  // every use); FP32 reads the weights with scalar loads
  __shared__ float Wr[M == MLP_F32 ? 1 : MODEL_MLP_MAX];
  if constexpr (M != MLP_F32) {
    model_round_mlp<M>(a.mlp, Wr, nin, H, L, threadIdx.x);
    wave_sync();
  }
  auto mlp_fwd = [&](const float* z, float* pre, float* out) {
    if constexpr (M == MLP_F32) model_mlp_fwd<M, H, L>(W, nin, z, pre, out);
    else model_mlp_fwd<M, H, L, true>(Wr, nin, z, pre, out);
  };
  // shade queue entries [0, nb) and add them to their rays
  auto shade = [&](int nb) {
    wave_sync();
    float t[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    int j = -1;
    ModelShade<NSH> S;
    if (lane < nb) {
      j = Q.rs[lane];
      const double x[3] = {Q.x[lane][0], Q.x[lane][1], Q.x[lane][2]};
      const float v[3] = {Q.v[j][0], Q.v[j][1], Q.v[j][2]};
      model_inputs<ST, FT, NSH>(sdf, feat, probes, G, tl, x, v, S);
    } else {
#pragma unroll
      for (int q = 0; q < MNIN; ++q) S.z[q] = 0.f;
    }
    float out[3] = {0.f, 0.f, 0.f};
    if constexpr (M == MLP_F32) {
      if (lane < nb) {
        float pre[L * H];
        mlp_fwd(S.z, pre, out);
      }
    } else {
      model_mlp_wave<M, H, L>(Wr, nin, MM, lane, S.z, out);
    }
    if (lane < nb) {
      const float w = Q.w[lane];
#pragma unroll
      for (int c = 0; c < 3; ++c) t[c] = w * sigmoidf(out[c]);
      t[3] = w * Q.tm[lane];
      t[4] = w;
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) Q.part[lane][c] = t[c];
    const int jp = __shfl_up(j, 1, 64);
    const bool lead = lane < nb && (lane == 0 || jp != j);
    const uint64_t leads = __ballot(lead);
    wave_sync();
    if (lead) {
      const uint64_t above = lane == 63 ? 0ull : (leads >> (lane + 1)) << (lane + 1);
      const int end = above ? __ffsll((long long)above) - 1 : nb;
      float s[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) s[c] = Q.acc[j][c];
      for (int q = lane; q < end; ++q)
#pragma unroll
        for (int c = 0; c < 5; ++c) s[c] += Q.part[q][c];
#pragma unroll
      for (int c = 0; c < 5; ++c) Q.acc[j][c] = s[c];
    }
    wave_sync();
  };
  int64_t r0, r1;
  wave_rays(a.B, per_wave, r0, r1);
  for (int64_t g0 = r0; g0 < r1; g0 += MODEL_GROUP) {
    const int ng = (int)min((int64_t)MODEL_GROUP, r1 - g0);
#pragma unroll
    for (int c = 0; c < 5; ++c) Q.acc[lane][c] = 0.f;
    Q.logT[lane] = 0.f;
    int qn = 0;  // queued entries (wave-uniform)
    for (int j = 0; j < ng; ++j) {
      const int64_t ray = g0 + j;
      RayD r;
      const bool hit = ray_setup_d(a.rays_o[3 * ray], a.rays_o[3 * ray + 1], a.rays_o[3 * ray + 2],
                                   a.rays_d[3 * ray], a.rays_d[3 * ray + 1], a.rays_d[3 * ray + 2],
                                   a.N, r);
      if (lane == 0) {
        Q.v[j][0] = (float)-r.d[0];
        Q.v[j][1] = (float)-r.d[1];
        Q.v[j][2] = (float)-r.d[2];
      }
      if (!hit) continue;  // wave-uniform
      float carry = 0.0f;
      for (int c0 = 0; c0 < a.N - 1; c0 += 64) {
        ChunkOut o;
        const uint64_t mask = model_chunk(sdf, a, G, tl, K, r, c0, lane, carry, o);
        if (!mask) continue;
        if ((mask >> lane) & 1ull) {
          const int e = qn + lane_rank(mask);
          Q.x[e][0] = o.x[0];
          Q.x[e][1] = o.x[1];
          Q.x[e][2] = o.x[2];
          Q.w[e] = o.w;
          Q.tm[e] = (float)(sample_t(r, c0 + lane) + 0.5 * r.dt);
          Q.rs[e] = j;
        }
        qn += (int)__popcll(mask);
        if (qn >= 64) {
          shade(64);
          // the rest of the queue moves to its front
          const int src = 64 + lane;
          const bool mv = src < qn;
          double x0 = 0.0, x1 = 0.0, x2 = 0.0;
          float w = 0.f, tm = 0.f;
          int rs = 0;
          if (mv) {
            x0 = Q.x[src][0], x1 = Q.x[src][1], x2 = Q.x[src][2];
            w = Q.w[src], tm = Q.tm[src], rs = Q.rs[src];
          }
          wave_sync();
          if (mv) {
            Q.x[lane][0] = x0, Q.x[lane][1] = x1, Q.x[lane][2] = x2;
            Q.w[lane] = w, Q.tm[lane] = tm, Q.rs[lane] = rs;
          }
          qn -= 64;
        }
      }
      if (lane == 0) Q.logT[j] = carry;
    }
    if (qn > 0) shade(qn);
    wave_sync();
    if (lane < ng) {
      const int64_t ray = g0 + lane;
      const float* s = Q.acc[lane];
      a.rgb[3 * ray] = s[0];
      a.rgb[3 * ray + 1] = s[1];
      a.rgb[3 * ray + 2] = s[2];
      if (a.aux) {
        a.aux[4 * ray] = s[0];
        a.aux[4 * ray + 1] = s[1];
        a.aux[4 * ray + 2] = s[2];
        a.aux[4 * ray + 3] = Q.logT[lane];
      }
      if (a.depth_wsum) {
        a.depth_wsum[2 * ray] = s[3];
        a.depth_wsum[2 * ray + 1] = s[4];
      }
    }
    wave_sync();
  }
}

// Reverse mode (gradients added into a.g_*).  A wave collects the shaded samples of
// consecutive rays (at most 64 rays and MODEL_EMAX samples) before it processes
// them, so every batch of the shading and of the reverse mode is full whatever the
// number of shaded samples per ray: the colours of the listed samples, the colour
// behind each sample by a suffix scan segmented by ray (last batch first), then
// per batch of 64 the MLP and the interpolations in reverse, with
//   dL/dC_i = w_i dL/drgb,  dL/d dl_i = dL/drgb . (R_i - T_i C_i),
//   d dl_i/d s_i = -tau sigma(-tau s_i),  d dl_i/d s_{i+1} = tau sigma(-tau s_{i+1}).
template <int NSH>
struct ModelBwdLds {
  ModelEntries E;
  unsigned char rs[MODEL_EMAX];  // ray of the entry within the group
  float C[MODEL_EMAX][3];
  float gdl[MODEL_EMAX];
  RayD ray[MODEL_GROUP];
  float v[MODEL_GROUP][3];
  float dL[MODEL_GROUP][3];
  union {
    DwLds dw;
    ProbeStage<NSH> ps;
    float sc[64][65];
  } u;
  int k0[64][3];
  int fb[64];
};

template <typename ST, typename FT, int NSH, int M, int H, int L>
__global__ void __launch_bounds__(64) model_bwd_kernel(RenderArgs a, int64_t per_wave) {
  __shared__ ModelBwdLds<NSH> S_;
  __shared__ ModelMfmaLds<M> MM;  // the colour pass's reduced-precision MLP on MFMA
  ModelBwdLds<NSH>& Ls = S_;
  ModelEntries& E = Ls.E;
  const int lane = threadIdx.x;
  const ST* __restrict__ sdf = static_cast<const ST*>(a.sdf);
  const FT* __restrict__ feat = static_cast<const FT*>(a.feat);
  const FT* __restrict__ probes = static_cast<const FT*>(a.probes);
  cfloat* __restrict__ W = const_mlp(a.mlp);
  const Geo G{a.R, a.P, 2.0 / (a.R - 1), 0.5 * (a.R - 1), 0.5 * (a.P - 1), a.flags};
  const Tiles tl{a.tile_index, a.tile_T};
  const Bricks K = make_bricks(a.bounds, a.R, a.skip_thr);
  const int nin = model_n_in(a.flags);
  // reduced-precision MLP: a copy with rounded weights in LDS (rounded once, not on
  // every use); FP32 reads the weights with scalar loads
  __shared__ float Wr[M == MLP_F32 ? 1 : MODEL_MLP_MAX];
  if constexpr (M != MLP_F32) {
    model_round_mlp<M>(a.mlp, Wr, nin, H, L, threadIdx.x);
    wave_sync();
  }
  auto mlp_fwd = [&](const float* z, float* pre, float* out) {
    if constexpr (M == MLP_F32) model_mlp_fwd<M, H, L>(W, nin, z, pre, out);
    else model_mlp_fwd<M, H, L, true>(Wr, nin, z, pre, out);
  };
  const bool reflect = (G.flags & FLAG_SH_REFLECT) && !(G.flags & FLAG_NO_FA);
  ModelDw<H, L> D;
  model_dw_zero(D);
  bool any = false;

  // the listed samples of the group: entries [0, n) of rays [0, nr)
  auto process = [&](int n) {
    wave_sync();
    // colours of the listed samples
    for (int b0 = 0; b0 < n; b0 += 64) {
      const int e = b0 + lane;
      ModelShade<NSH> S;
      if (e < n) {
        const int j = Ls.rs[e];
        double x[3];
        sample_pos(Ls.ray[j], sample_t(Ls.ray[j], E.i[e]), x);
        const float v[3] = {Ls.v[j][0], Ls.v[j][1], Ls.v[j][2]};
        model_inputs<ST, FT, NSH>(sdf, feat, probes, G, tl, x, v, S);
      } else {
#pragma unroll
        for (int q = 0; q < MNIN; ++q) S.z[q] = 0.f;
      }
      float out[3] = {0.f, 0.f, 0.f};
      if constexpr (M == MLP_F32) {
        if (e < n) {
          float pre[L * H];
          mlp_fwd(S.z, pre, out);
        }
      } else {
        model_mlp_wave<M, H, L>(Wr, nin, MM, lane, S.z, out);
      }
      if (e < n) {
#pragma unroll
        for (int c = 0; c < 3; ++c) Ls.C[e][c] = sigmoidf(out[c]);
      }
    }
    wave_sync();
    // R_e = sum over the ray's entries e' >= e of w C: a suffix scan segmented by ray,
    // last batch first; `carry` continues the ray that starts the later batch
    {
      float carry[3] = {0.f, 0.f, 0.f};
      int carry_ray = -1;
      for (int b0 = ((n - 1) >> 6) << 6; b0 >= 0; b0 -= 64) {
        const int e = b0 + lane;
        const bool ve = e < n;
        const int j = ve ? Ls.rs[e] : -1 - lane;  // lanes past the end: their own segments
        float Rv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) Rv[c] = ve ? E.w[e] * Ls.C[e][c] : 0.f;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const int jd = __shfl_down(j, d, 64);
          const bool same = lane + d < 64 && jd == j;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float y = __shfl_down(Rv[c], d, 64);
            if (same) Rv[c] += y;
          }
        }
        if (j == carry_ray) {
#pragma unroll
          for (int c = 0; c < 3; ++c) Rv[c] += carry[c];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) carry[c] = __shfl(Rv[c], 0, 64);
        carry_ray = __shfl(j, 0, 64);
        if (ve) {
          const float T = E.T[e];
          const float* dL = Ls.dL[j];
          Ls.gdl[e] = dL[0] * (Rv[0] - T * Ls.C[e][0]) + dL[1] * (Rv[1] - T * Ls.C[e][1]) +
                      dL[2] * (Rv[2] - T * Ls.C[e][2]);
        }
      }
    }
    wave_sync();
    // reverse mode of each batch
    for (int b0 = 0; b0 < n; b0 += 64) {
      const int e = b0 + lane;
      const bool ve = e < n;
      const int nb = min(64, n - b0);
      double x[3] = {0.0, 0.0, 0.0};
      ModelShade<NSH> S;
      float pre[L * H], out[3], dout[3] = {0.f, 0.f, 0.f};
      float gdl = 0.f, s0 = 0.f, s1 = 0.f;
      float v[3] = {0.f, 0.f, 0.f};
      int i = 0, j = 0;
      if (ve) {
        j = Ls.rs[e];
        i = E.i[e];
        sample_pos(Ls.ray[j], sample_t(Ls.ray[j], i), x);
        v[0] = Ls.v[j][0];
        v[1] = Ls.v[j][1];
        v[2] = Ls.v[j][2];
        model_inputs<ST, FT, NSH>(sdf, feat, probes, G, tl, x, v, S);
        mlp_fwd(S.z, pre, out);
        const float w = E.w[e];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float Cc = sigmoidf(out[c]);
          dout[c] = w * Ls.dL[j][c] * Cc * (1.f - Cc);
        }
        gdl = Ls.gdl[e];
        s0 = E.s0[e];
        s1 = E.s1[e];
      } else {
#pragma unroll
        for (int k = 0; k < L * H; ++k) pre[k] = 0.f;
#pragma unroll
        for (int q = 0; q < MNIN; ++q) S.z[q] = 0.f;
#pragma unroll
        for (int q = 0; q < NSH; ++q) S.Y[q] = 0.f;
      }
      float dpre[L * H], dz[MNIN];
      if constexpr (M == MLP_F32) model_mlp_bwd<M, H, L>(W, nin, pre, dout, dpre, dz);
      else model_mlp_bwd<M, H, L, true>(Wr, nin, pre, dout, dpre, dz);
      if (a.g_mlp) model_dw_batch<M, H, L>(Ls.u.dw, lane, ve, nin, S.z, pre, dpre, dout, D);
      wave_sync();
      // SDF: the FD-normal path and the opacity at s_i in the sample's 4x4x4 patch,
      // the opacity at s_{i+1} at the next sample's cell
      if (a.g_sdf) {
        float* row = Ls.u.sc[lane];
#pragma unroll
        for (int q = 0; q < 64; ++q) row[q] = 0.f;
        if (ve) {
          float ev[NSH] = {};
          if (reflect) probe_contract<FT, NSH>(probes, G, x, dz + NF, ev);
          float dg[3] = {0.f, 0.f, 0.f};
          if (!(G.flags & FLAG_NV_ONE) || reflect) model_normal_dg<NSH>(S, v, dz, ev, G.flags, dg);
          int k0[3];
          cell_k(x, G.R, G.inv_h, k0);
          Ls.k0[lane][0] = k0[0];
          Ls.k0[lane][1] = k0[1];
          Ls.k0[lane][2] = k0[2];
          const PatchDst Dp = patch_of_row(row, k0);
          const float gs0 = -a.tau * sigmoidf(-a.tau * s0) * gdl;
          if (gs0 != 0.f) patch_add(Dp, k0, x, G.R, G.inv_h, gs0);
          if (dg[0] != 0.f || dg[1] != 0.f || dg[2] != 0.f) fd_patch(Dp, k0, G, x, dg);
          const float gs1 = a.tau * sigmoidf(-a.tau * s1) * gdl;
          if (gs1 != 0.f) {
            double x1[3];
            sample_pos(Ls.ray[j], sample_t(Ls.ray[j], i + 1), x1);
            scatter8(a.g_sdf, G.R, cell_d(x1, G.R, G.inv_h), gs1);
          }
        }
        wave_sync();
        sdf_patch_flush(Ls.u.sc, Ls.k0, nb, lane, G.R, a.g_sdf);
        wave_sync();
      }
      if (!(G.flags & FLAG_NO_FS) && a.g_feat) {
        if (tl.index) {
          if (ve) {
            float loc[3];
            const int slot = tile_slot(tl, G.R, G.inv_h, x, loc);
            if (slot >= 0) triplane_scatter(feat, slot, loc, dz, a.g_feat);
          }
        } else {
          feat_scatter_wave(Ls.u.sc, Ls.fb, ve, cell_d(x, G.R, G.inv_h), dz, nb, lane, G.R,
                            a.g_feat);
        }
      }
      if (!(G.flags & FLAG_NO_FA) && a.g_probes)
        probe_scatter_lanes<NSH>(Ls.u.ps, lane, ve,
                                 ve ? cell_d(x, G.P, G.inv_hp) : Cell{0, 0.f, 0.f, 0.f}, G.P,
                                 S.Y, dz + NF, a.g_probes);
      wave_sync();
    }
  };

  int n = 0, nr = 0;  // listed samples and rays (wave-uniform)
  int64_t r0, r1;
  wave_rays(a.B, per_wave, r0, r1);
  for (int64_t ray = r0; ray < r1; ++ray) {
    const float dL[3] = {a.dL[3 * ray], a.dL[3 * ray + 1], a.dL[3 * ray + 2]};
    if (dL[0] == 0.f && dL[1] == 0.f && dL[2] == 0.f) continue;  // wave-uniform
    RayD r;
    if (!ray_setup_d(a.rays_o[3 * ray], a.rays_o[3 * ray + 1], a.rays_o[3 * ray + 2],
                     a.rays_d[3 * ray], a.rays_d[3 * ray + 1], a.rays_d[3 * ray + 2], a.N, r))
      continue;
    // room for every sample of this ray
    if (nr == MODEL_GROUP || n + (a.N - 1) > MODEL_EMAX) {
      process(n);
      n = nr = 0;
    }
    wave_sync();
    const int n0 = n;
    float carry = 0.0f;
    for (int c0 = 0; c0 < a.N - 1; c0 += 64) {
      ChunkOut o;
      const uint64_t mask = model_chunk(sdf, a, G, tl, K, r, c0, lane, carry, o);
      if (!mask) continue;
      if ((mask >> lane) & 1ull) {
        const int e = n + lane_rank(mask);
        E.i[e] = c0 + lane;
        E.w[e] = o.w;
        E.T[e] = o.T;
        E.s0[e] = o.s0;
        E.s1[e] = o.s1;
        Ls.rs[e] = (unsigned char)nr;
      }
      n += (int)__popcll(mask);
    }
    if (n == n0) continue;  // no shaded sample: nothing to add
    if (lane == 0) {
      Ls.ray[nr] = r;
      Ls.v[nr][0] = (float)-r.d[0];
      Ls.v[nr][1] = (float)-r.d[1];
      Ls.v[nr][2] = (float)-r.d[2];
      Ls.dL[nr][0] = dL[0];
      Ls.dL[nr][1] = dL[1];
      Ls.dL[nr][2] = dL[2];
    }
    ++nr;
    any = true;
  }
  if (n > 0) process(n);
  if (any && a.g_mlp) model_dw_flush<H, L>(D, lane, nin, a.g_mlp);
}

// Launch of the kernels of one MLP shape (H, L), direction and MLP arithmetic M;
// the instances are spread over several translation units (render_model_*.hip).
template <int H, int L, bool BWD, int M>
hipError_t launch_model_hlm(const RenderArgs& a, int feat_dt, int n_sh, dim3 grid, int64_t per,
                            hipStream_t s) {
  typedef float ST;
  auto go = [&](auto ft, auto nsh) {
    typedef decltype(ft) FT;
    constexpr int NSH = decltype(nsh)::value;
    if constexpr (BWD)
      hipLaunchKernelGGL((model_bwd_kernel<ST, FT, NSH, M, H, L>), grid, dim3(64), 0, s, a, per);
    else
      hipLaunchKernelGGL((model_fwd_kernel<ST, FT, NSH, M, H, L>), grid, dim3(64), 0, s, a, per);
  };
  typedef std::integral_constant<int, 9> S9;
  typedef std::integral_constant<int, 16> S16;
  // storage follows the arithmetic: FP32 features with the FP32 MLP, FP16 features
  // with the FP16 / BF16 MLP
  if (feat_dt != (M == MLP_F32 ? 0 : 1)) return hipErrorInvalidValue;
  if constexpr (M == MLP_F32) {
    if (n_sh == 9) go(float(), S9());
    else if (n_sh == 16) go(float(), S16());
    else return hipErrorInvalidValue;
  } else {
    if (n_sh == 9) go(_Float16(), S9());
    else if (n_sh == 16) go(_Float16(), S16());
    else return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define PSDF_MODEL_INSTANCE(H, L, BWD, M)                                                    \
  template hipError_t launch_model_hlm<H, L, BWD, M>(const RenderArgs&, int, int, dim3, int64_t, \
                                                     hipStream_t);

}  // namespace psdf
