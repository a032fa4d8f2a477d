// Forward render of the ProbeSDF step (Sec. 3.3: c = sum_i T_i alpha_i C_i,
// NeuS opacity of Eq. neus; colour model of Sec. 3.1-3.2 and Sec. 4).
//
// One ray per lane marches its N samples: trilinear SDF, skip rule, log-domain
// opacity and transmittance.  Transmittance and weights depend on the SDF only,
// so the march never waits for colour: each shaded sample (active, alpha > 0)
// is pushed with its weight into a per-wave ring in LDS, and whenever 64 are
// queued the whole wave shades them together, one sample per lane (FD normal,
// spatial features, probe coefficients contracted with the SH basis of the
// ray's view direction, MLP).  The weighted colours are then summed per ray by
// the ray's own lane, in sample order.
//
// Training forwards may record a tape: every batch of shaded samples is written
// to the caller's workspace as one chunk of entries (position, weights, s_i,
// s_{i+1}, colour, MLP inputs and normal), so that the backward neither
// re-marches nor re-reads the shading inputs.
#include "dispatch.h"
#include "shade.h"

namespace psdf {

struct FwdLds {
  RayD ray[64];
  int next[RING];   // sequence number of the same ray's next entry
  int key[RING];    // (sample index << 6) | ray lane
  float w[RING];    // compositing weight T_i alpha_i
  float T[RING];    // transmittance T_i
  float s0[RING];   // s_i
  float s1[RING];   // s_{i+1}
  float wc[RING][3];
};

// tape state of a wave (wave-uniform)
struct TapeW {
  int last = -1, total = 0;
  bool ovf = false;
};

template <typename ST, typename FT, int NSH, int M>
__device__ __forceinline__ void fwd_batch(const RenderArgs& a, const Geo& G, FwdLds& L,
                                          MlpLds<M>& ML, const MlpFrag<M>& frag, int lane, int head,
                                          int n, float rgb[3], int& my_first, int& my_cnt,
                                          const BwdWs& ws, bool tape, unsigned lw, TapeW& tw) {
  const ST* __restrict__ sdf = static_cast<const ST*>(a.sdf);
  const FT* __restrict__ feat = static_cast<const FT*>(a.feat);
  const FT* __restrict__ probes = static_cast<const FT*>(a.probes);
  wave_sync();
  const bool ve = lane < n;
  const int slot = (head + lane) & (RING - 1);
  float z[NIN];
#pragma unroll
  for (int j = 0; j < NIN; ++j) z[j] = 0.f;
  float w = 0.f;
  int key = 0;
  double x[3] = {0.0, 0.0, 0.0};
  float v[3] = {0.f, 0.f, 0.f};
  Normal nm{};
  if (ve) {
    key = L.key[slot];
    const RayD r = L.ray[key & 63];
    w = L.w[slot];
    sample_pos(r, sample_t(r, key >> 6), x);
    v[0] = (float)-r.d[0];
    v[1] = (float)-r.d[1];
    v[2] = (float)-r.d[2];
    float Y[NSH];
    sh_basis<NSH>(v[0], v[1], v[2], Y);
    shade_inputs<ST, FT, NSH>(sdf, feat, probes, G, x, v, Y, z, nm);
  }
  float out[3];
  if constexpr (M == MLP_F32) {
    float pre[HID], hid[HID];
    mlp_lane<M>(const_mlp(a.mlp), z, pre, hid, out);
  } else {
    mlp_wave<M>(frag, ML, lane, z, out);
  }
  const float C0 = sigmoidf(out[0]), C1 = sigmoidf(out[1]), C2 = sigmoidf(out[2]);
  if (ve) {
    L.wc[slot][0] = w * C0;
    L.wc[slot][1] = w * C1;
    L.wc[slot][2] = w * C2;
  }
  if (tape && !tw.ovf) {
    const int pkey = ve ? probe_key(cell_d(x, G.P, G.inv_hp).base, G.P) : 0;
    // one chunk of entries per batch, chunks of the wave linked backwards
    unsigned long long got = 0;
    if (lane == 0) got = atomicAdd(ws.counter, (unsigned long long)n);
    const int64_t base = (int64_t)__shfl(got, 0, 64);
    if (base + n > ws.cap) {
      // no room: the backward runs this wave with the fused kernel
      if (base + lane < ws.cap && lane < n) ws.entries[base + lane].lw = -1;
      tw.ovf = true;
    } else {
      if (ve) {
        BwdEntry e;
        e.x[0] = x[0];
        e.x[1] = x[1];
        e.x[2] = x[2];
        e.v[0] = v[0];
        e.v[1] = v[1];
        e.v[2] = v[2];
        e.w = w;
        e.T = L.T[slot];
        e.s0 = L.s0[slot];
        e.s1 = L.s1[slot];
        e.ray = (int)(lw * 64u) + (key & 63);
        e.key = key;
        e.lw = (int)lw;
        e.prev = tw.last;
        e.C[0] = C0;
        e.C[1] = C1;
        e.C[2] = C2;
#pragma unroll
        for (int j = 0; j < NIN; ++j) e.z[j] = z[j];
        e.nrm[0] = nm.n[0];
        e.nrm[1] = nm.n[1];
        e.nrm[2] = nm.n[2];
        e.gn = nm.gn;
        e.gdl = 0.f;
        e.gdl_prev = 0.f;
        e.pkey = pkey;
        e.nx_off[0] = e.nx_off[1] = e.nx_off[2] = 0.f;
        ws.entries[base + lane] = e;
      }
      // the backward's probe-cell histogram
      for_each_key_group(ve, pkey, [&](int k, int leader, uint64_t grp) {
        if (lane == leader) atomicAdd(ws.pcount + k, (int)__popcll(grp));
      });
      tw.last = (int)base;
      tw.total += n;
    }
  }
  wave_sync();
  // each ray's lane adds its own entries of this batch, in sample order
  while (my_cnt > 0 && my_first < head + n) {
    const int s = my_first & (RING - 1);
    rgb[0] += L.wc[s][0];
    rgb[1] += L.wc[s][1];
    rgb[2] += L.wc[s][2];
    if (--my_cnt > 0) my_first = L.next[s];
  }
  wave_sync();
}

template <typename ST, typename FT, int NSH, int M>
__global__ void __launch_bounds__(BLOCK) render_fwd_kernel(RenderArgs a, BwdWs ws, int tape) {
  __shared__ FwdLds lds[WAVES];
  __shared__ MlpLds<M> mlds[M == MLP_F32 ? 1 : WAVES];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  FwdLds& L = lds[wv];
  MlpLds<M>& ML = mlds[M == MLP_F32 ? 0 : wv];
  const ST* __restrict__ sdf = static_cast<const ST*>(a.sdf);
  const Geo G{a.R, a.P, 2.0 / (a.R - 1), 0.5 * (a.R - 1), 0.5 * (a.P - 1), a.flags};
  MlpFrag<M> frag;
  if constexpr (M != MLP_F32) mlp_frag_load<M>(a.mlp, lane, frag);

  const unsigned lw = xcd_block(blockIdx.x, gridDim.x) * WAVES + wv;  // this wave's 64 rays
  const int64_t ray = (int64_t)lw * 64 + lane;
  const bool valid = ray < a.B;
  TapeW tw;
  float ro[3] = {0.f, 0.f, 0.f}, rd[3] = {0.f, 0.f, 1.f};
  if (valid) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ro[k] = a.rays_o[3 * ray + k];
      rd[k] = a.rays_d[3 * ray + k];
    }
  }
  RayD r;
  const bool hit = ray_setup_d(ro[0], ro[1], ro[2], rd[0], rd[1], rd[2], a.N, r) && valid;
  L.ray[lane] = r;

  float rgb[3] = {0.f, 0.f, 0.f};
  float wsum = 0.f, depth = 0.f, logT = 0.f;
  int my_first = 0, my_last = 0, my_cnt = 0;
  int head = 0, tail = 0;  // wave-uniform ring cursors (sequence numbers)
  const Bricks K = make_bricks(a.bounds, a.R, a.skip_thr);
  // samples first .. last_s are stepped (wave-uniform); outside the interval no
  // lane of the wave can have a sample in a brick that passes the bounds test, so
  // no sample there is active and the march has nothing to compute
  int first = 0, last_s = a.N - 2;
  if (tape && ws.range) {
    int lo, hi;
    may_range(r, G.inv_h, a.N, hit, ws.mbox, lo, hi);
    first = wave_min_i(lo);
    last_s = min(wave_max_i(hi), a.N - 2);
  }
  MarchState ms;
  if (first <= last_s) march_begin_at(sdf, a.R, K, r, G.inv_h, hit, a.N, first, ms);
  for (int i = first;; ++i) {
    const bool stepping = i <= last_s;  // wave-uniform
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
        const float w = T * -expm1f(dl);
        wsum += w;
        depth = fmaf(w, (float)(sample_t(r, i) + 0.5 * r.dt), depth);
        logT += dl;
        const int seq = tail + lane_rank(mask);
        const int slot = seq & (RING - 1);
        L.key[slot] = (i << 6) | lane;
        L.w[slot] = w;
        L.T[slot] = T;
        L.s0[slot] = s_i;
        L.s1[slot] = s_n;
        if (my_cnt > 0) L.next[my_last & (RING - 1)] = seq;
        else my_first = seq;
        my_last = seq;
        ++my_cnt;
      }
      tail += __popcll(mask);
    }
    const int pending = tail - head;
    if (pending >= 64 || (!stepping && pending > 0)) {
      const int n = min(64, pending);
      fwd_batch<ST, FT, NSH, M>(a, G, L, ML, frag, lane, head, n, rgb, my_first, my_cnt, ws,
                                tape != 0, lw, tw);
      head += n;
    } else if (!stepping) {
      break;
    }
  }
  if (valid) {
    a.rgb[3 * ray + 0] = rgb[0];
    a.rgb[3 * ray + 1] = rgb[1];
    a.rgb[3 * ray + 2] = rgb[2];
    if (a.aux) {
      a.aux[4 * ray + 0] = rgb[0];
      a.aux[4 * ray + 1] = rgb[1];
      a.aux[4 * ray + 2] = rgb[2];
      a.aux[4 * ray + 3] = logT;
    }
    if (a.depth_wsum) {
      a.depth_wsum[2 * ray + 0] = depth;
      a.depth_wsum[2 * ray + 1] = wsum;
    }
  }
  if (tape && lane == 0 && lw < ws.n_waves) {
    ws.count[lw] = tw.ovf ? 0 : tw.total;
    ws.last[lw] = tw.ovf ? -1 : tw.last;
    if (tw.ovf) ws.overflow[lw] = 1;
  }
}

// Brick box of the bricks whose bounds pass the skip test (brick_may): 4 bricks
// per thread, a block-wide min / max, six integer atomics per block.
constexpr int kBoxPer = 4;

__global__ void __launch_bounds__(256) may_box_kernel(Bricks K, int* box) {
  __shared__ int red[6][4];
  const int nb = K.nb, n = nb * nb * nb;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int lo[3] = {0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF}, hi[3] = {-1, -1, -1};
  const int base = blockIdx.x * (256 * kBoxPer) + threadIdx.x;
  float2 mm[kBoxPer];
#pragma unroll
  for (int j = 0; j < kBoxPer; ++j) {
    const int b = base + j * 256;
    mm[j] = K.b[b < n ? b : 0];
  }
#pragma unroll
  for (int j = 0; j < kBoxPer; ++j) {
    const int b = base + j * 256;
    if (b < n && brick_may(K, mm[j])) {
      const int c[3] = {b % nb, (b / nb) % nb, b / (nb * nb)};
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        lo[q] = min(lo[q], c[q]);
        hi[q] = max(hi[q], c[q]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    lo[q] = wave_min_i(lo[q]);
    hi[q] = wave_max_i(hi[q]);
  }
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      red[q][wv] = lo[q];
      red[3 + q][wv] = hi[q];
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int q = threadIdx.x;
    int v = red[q][0];
    for (int w = 1; w < 4; ++w) v = q < 3 ? min(v, red[q][w]) : max(v, red[q][w]);
    if (q < 3 ? v != 0x7FFFFFFF : v != -1) {
      if (q < 3) atomicMin(box + q, v);
      else atomicMax(box + q, v);
    }
  }
}

hipError_t launch_render_forward(const RenderArgs& a, const BwdWs* tape, int sdf_dt, int feat_dt,
                                 int mlp_dt, int n_sh, hipStream_t s) {
  const dim3 grid((unsigned)((a.B + BLOCK - 1) / BLOCK));
  BwdWs ws{};
  if (tape) {
    ws = *tape;
    ws.probe_bins = 0;
    ws.bins = 1;  // the forward counts its samples per probe-cell key
    const hipError_t e = launch_bwd_ws_clear(ws, s);
    if (e != hipSuccess) return e;
    const Bricks K = make_bricks(a.bounds, a.R, a.skip_thr);
    ws.range = K.b ? 1 : 0;
    if (ws.range) {
      const int n = K.nb * K.nb * K.nb, per = 256 * kBoxPer;
      hipLaunchKernelGGL(may_box_kernel, dim3((unsigned)((n + per - 1) / per)), dim3(256), 0, s,
                         K, ws.mbox);
    }
  }
  const int on = tape ? 1 : 0;
  PSDF_DT_SWITCH(sdf_dt, feat_dt, PSDF_SH_SWITCH(n_sh, PSDF_MLP_SWITCH(mlp_dt,
      hipLaunchKernelGGL((render_fwd_kernel<ST, FT, NSH, M>), grid, dim3(BLOCK), 0, s, a, ws, on))));
  return hipGetLastError();
}

}  // namespace psdf
