// Entry-parallel schedule of the ProbeSDF backward (same gradients as the
// fused kernel in render_bwd.hip; Sec. 3.3 reverse mode).
//
// The fused kernel keeps a wave's march state live while it shades, so it runs
// at one wave per SIMD, and waves whose rays cross the surface carry all the
// shading work.  Here the work is split into passes over a caller-provided
// workspace:
//   1. march  -- one ray per lane, with brick skipping; the shaded samples
//                (alpha > 0) are written as entries in chunks of 64, the chunks
//                of one wave linked backwards, and counted per probe cell;
//   2. scan   -- exclusive offsets of the probe-cell counts;
//   3. shade  -- every wave takes 64 consecutive entries, whatever their rays:
//                colour C_i (kept for pass 5), MLP reverse mode with
//                dL/dC_i = w_i dL/drgb, the scatters into the features, the SDF
//                (normal path) and the MLP weights, and a record of dL/dF_a filed
//                under the sample's probe cell;
//   4. probes -- one wave per occupied probe cell sums w_c Y_j dL/dF_a,k over
//                the cell's records in registers (lanes = SH x angle
//                coefficients) and adds the result to the cell's 8 corner
//                nodes: one atomic per node coefficient per cell instead of one
//                per sample;
//   5. alpha  -- one wave per 64 rays walks its chunks backwards, forms the
//                remaining colour R_i = sum_{j >= i} w_j C_j and
//                dL/d dl_i = dL/drgb . (R_i - T_i C_i), and scatters the
//                opacity gradient into the corners of s_i and s_{i+1}.
// A wave whose entries do not fit into the workspace is flagged and handled by
// the fused kernel afterwards (its partial entries are skipped; their probe
// records carry zeros).
//
// Taped schedule (the forward recorded its shaded samples with their MLP inputs,
// normal and probe-cell key, and counted them per probe cell): no march.
//   walk   -- per ray, dL/d dl_i of every entry, that of the previous sample when
//             it is an entry, and the offset x_{i+1} - x_i when the next sample
//             is not one (its opacity term then travels with sample i);
//   shade  -- waves take the entries in probe-cell order, 64 slots of one block
//             of 2x2x2 probe cells at a time: MLP reverse mode (weight gradient
//             on MFMA), one probe record and one scatter record per sample;
//   box    -- per block of probe cells, the SDF cotangents (FD normal, opacity
//             at s_i and at x_i + offset) and the feature cotangents are summed
//             in LDS boxes (fixed-point integer adds) and flushed row by row;
//   probes -- as pass 4 above, over the shading pass's records.
#include "bwd_common.h"
#include "dispatch.h"

namespace psdf {

namespace {
constexpr int64_t kHead = 256;
constexpr int kScan = 1024;  // items per scan block
int64_t al256(int64_t b) { return (b + 255) & ~(int64_t)255; }
int64_t n_waves_of(int64_t B) { return (B + 63) / 64; }
// Probe cells are binned under a key that keeps space together: blocks of 2x2x2
// cells in row-major order, the 8 cells of a block consecutive.  Cells span
// 0..P-2 per axis, so P/2 blocks per axis.
int64_t nblk_of(int P) {
  const int64_t nb = P / 2;
  return nb * nb * nb;
}
int64_t nkeys_of(int P) { return 8 * nblk_of(P); }
int64_t nsum_of(int P) { return (nkeys_of(P) + kScan - 1) / kScan; }
constexpr int64_t kMlpPart = (int64_t)NMLP * kMlpWaves * 4;
int64_t fixed_bytes(int64_t B, int P) {
  return kHead + 3 * al256(n_waves_of(B) * 4) + 3 * al256(nkeys_of(P) * 4) + al256(nsum_of(P) * 4) +
         kMlpPart + al256(NMLP * 4);
}
constexpr int64_t kPerSample =
    (int64_t)sizeof(BwdEntry) + (int64_t)sizeof(ProbeRec) + (int64_t)sizeof(ScatRec);
// box-pass batches: each occupied block of cells ends at most one partial batch
int64_t ndesc_of(int P, int64_t cap) { return nblk_of(P) + 1 + cap / 64; }
}  // namespace

int64_t bwd_ws_bytes(int64_t B, int P, int64_t cap) {
  return fixed_bytes(B, P) + cap * kPerSample + al256(ndesc_of(P, cap) * 8);
}

int64_t bwd_ws_capacity(int64_t B, int P, int64_t bytes) {
  // the largest cap whose layout fits (slot indices are 32-bit)
  const int64_t r = bytes - fixed_bytes(B, P) - al256((nblk_of(P) + 1) * 8) - 256;
  if (r <= 0) return 0;
  int64_t cap = min(r * 64 / (64 * kPerSample + 8), (int64_t)INT32_MAX);
  while (cap > 0 && bwd_ws_bytes(B, P, cap) > bytes) --cap;
  return cap;
}

BwdWs bwd_ws_carve(void* base, int64_t B, int P, int64_t bytes) {
  char* p = static_cast<char*>(base);
  const int64_t nw = n_waves_of(B), arr = al256(nw * 4), parr = al256(nkeys_of(P) * 4);
  BwdWs w;
  w.counter = reinterpret_cast<unsigned long long*>(p);
  w.overflow = reinterpret_cast<int*>(p + kHead);
  w.count = reinterpret_cast<int*>(p + kHead + arr);
  w.last = reinterpret_cast<int*>(p + kHead + 2 * arr);
  w.pcount = reinterpret_cast<int*>(p + kHead + 3 * arr);
  w.pcursor = reinterpret_cast<int*>(p + kHead + 3 * arr + parr);
  w.plist = reinterpret_cast<int*>(p + kHead + 3 * arr + 2 * parr);
  w.psum = reinterpret_cast<int*>(p + kHead + 3 * arr + 3 * parr);
  w.mlp_part = reinterpret_cast<float*>(p + kHead + 3 * arr + 3 * parr + al256(nsum_of(P) * 4));
  w.mlp_r = reinterpret_cast<float*>(p + kHead + 3 * arr + 3 * parr + al256(nsum_of(P) * 4) +
                                      kMlpPart);
  w.nbatch = reinterpret_cast<int*>(p + 24);
  w.pocc = reinterpret_cast<int*>(p + 8);
  w.cap = bwd_ws_capacity(B, P, bytes);
  w.entries = reinterpret_cast<BwdEntry*>(p + fixed_bytes(B, P));
  w.precs = reinterpret_cast<ProbeRec*>(p + fixed_bytes(B, P) + w.cap * (int64_t)sizeof(BwdEntry));
  w.srecs = reinterpret_cast<ScatRec*>(p + fixed_bytes(B, P) +
                                       w.cap * (int64_t)(sizeof(BwdEntry) + sizeof(ProbeRec)));
  w.nsorted = reinterpret_cast<int*>(p + 16);
  w.mbox = reinterpret_cast<int*>(p + 32);
  w.ndesc = ndesc_of(P, w.cap);
  w.bdesc = reinterpret_cast<int2*>(p + fixed_bytes(B, P) + w.cap * kPerSample);
  w.n_waves = nw;
  w.nkeys = nkeys_of(P);
  w.nsum = nsum_of(P);
  w.probe_bins = 0;
  w.bins = 0;
  w.range = 0;
  return w;
}

static_assert(sizeof(BwdEntry) == 160 && sizeof(ProbeRec) == 48 && sizeof(ScatRec) == 80,
              "record layouts");

// waves = 1: reset the slot counter and the overflow flags (before a march or a
// taped forward); probe_bins: reset the probe-cell counts
__global__ void __launch_bounds__(256) bwd_ws_clear_kernel(BwdWs ws, int waves) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i == 0) {
    if (waves) *ws.counter = 0;
    *ws.pocc = 0;
    *ws.nbatch = 0;
  }
  if (i < 6) ws.mbox[i] = i < 3 ? 0x7FFFFFFF : -1;
  if (waves && i < ws.n_waves) ws.overflow[i] = 0;
  if (ws.bins && i < ws.nkeys) ws.pcount[i] = 0;
}

static hipError_t launch_clear(const BwdWs& ws, int waves, hipStream_t s) {
  const int64_t n = max(waves ? ws.n_waves : (int64_t)1, ws.bins ? ws.nkeys : (int64_t)1);
  hipLaunchKernelGGL(bwd_ws_clear_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ws,
                     waves);
  return hipGetLastError();
}

hipError_t launch_bwd_ws_clear(const BwdWs& ws, hipStream_t s) { return launch_clear(ws, 1, s); }

// ---------------------------------------------------------------------------
// pass 1: march and emit
// ---------------------------------------------------------------------------
struct EmitLds {
  RayD ray[64];
  int key[RING];  // (sample index << 6) | ray lane
  float w[RING];
  float T[RING];
  float s0[RING];
  float s1[RING];
};

template <typename ST>
__global__ void __launch_bounds__(BLOCK) bwd_march_kernel(RenderArgs a, BwdWs ws) {
  __shared__ EmitLds lds[WAVES];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  EmitLds& L = lds[wv];
  const ST* __restrict__ sdf = static_cast<const ST*>(a.sdf);
  const unsigned lw = xcd_block(blockIdx.x, gridDim.x) * WAVES + wv;
  if (lw >= ws.n_waves) return;
  const int64_t ray = (int64_t)lw * 64 + lane;
  const bool valid = ray < a.B;
  float ro[3] = {0.f, 0.f, 0.f}, rd[3] = {0.f, 0.f, 1.f}, dL[3] = {0.f, 0.f, 0.f};
  if (valid) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ro[k] = a.rays_o[3 * ray + k];
      rd[k] = a.rays_d[3 * ray + k];
      dL[k] = a.dL[3 * ray + k];
    }
  }
  RayD r;
  const bool hit = ray_setup_d(ro[0], ro[1], ro[2], rd[0], rd[1], rd[2], a.N, r) && valid &&
                   (dL[0] != 0.f || dL[1] != 0.f || dL[2] != 0.f);
  L.ray[lane] = r;

  const double inv_h = 0.5 * (a.R - 1), inv_hp = 0.5 * (a.P - 1);
  const Bricks K = make_bricks(a.bounds, a.R, a.skip_thr);
  MarchState ms;
  march_begin(sdf, a.R, K, r, inv_h, hit, a.N, ms);
  float logT = 0.f;
  int head = 0, tail = 0, total = 0, last = -1;
  bool ovf = false;
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
        const int slot = (tail + lane_rank(mask)) & (RING - 1);
        L.key[slot] = (i << 6) | lane;
        L.w[slot] = T * -expm1f(dl);
        L.T[slot] = T;
        L.s0[slot] = s_i;
        L.s1[slot] = s_n;
        logT += dl;
      }
      tail += __popcll(mask);
    }
    const int pending = tail - head;
    if (pending >= 64 || (!stepping && pending > 0)) {
      const int n = min(64, pending);
      wave_sync();
      unsigned long long got = 0;
      if (lane == 0) got = atomicAdd(ws.counter, (unsigned long long)n);
      const int64_t base = (int64_t)__shfl(got, 0, 64);
      if (base + n > ws.cap) {
        // no room: the fused kernel takes this wave; the slots it got hold nothing
        if (base + lane < ws.cap && lane < n) ws.entries[base + lane].lw = -1;
        ovf = true;
        break;
      }
      int pc = 0;
      if (lane < n) {
        const int slot = (head + lane) & (RING - 1);
        const int key = L.key[slot];
        const RayD& rr = L.ray[key & 63];
        BwdEntry e;
        sample_pos(rr, sample_t(rr, key >> 6), e.x);
        pc = probe_key(cell_d(e.x, a.P, inv_hp).base, a.P);
        e.v[0] = (float)-rr.d[0];
        e.v[1] = (float)-rr.d[1];
        e.v[2] = (float)-rr.d[2];
        e.w = L.w[slot];
        e.T = L.T[slot];
        e.s0 = L.s0[slot];
        e.s1 = L.s1[slot];
        e.ray = (int)(lw * 64u) + (key & 63);
        e.key = key;
        e.lw = (int)lw;
        e.prev = last;
        e.C[0] = e.C[1] = e.C[2] = 0.f;
        ws.entries[base + lane] = e;
      }
      if (ws.probe_bins)
        for_each_key_group(lane < n, pc, [&](int k, int leader, uint64_t grp) {
          if (lane == leader) atomicAdd(ws.pcount + k, (int)__popcll(grp));
        });
      last = (int)base;
      total += n;
      head += n;
      wave_sync();
    } else if (!stepping) {
      break;
    }
  }
  if (lane == 0) {
    ws.count[lw] = ovf ? 0 : total;
    ws.last[lw] = ovf ? -1 : last;
    if (ovf) ws.overflow[lw] = 1;
  }
}

// ---------------------------------------------------------------------------
// pass 2: exclusive scan of the probe-cell counts (blocks of 1024 cells)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// block-wide exclusive scan of one int per thread (256 threads); returns the total
__device__ __forceinline__ int block_excl_scan(int v, int* part, int& excl) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int inc = wave_incl_scan(v, lane);
  if (lane == 63) part[wv] = inc;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    off += k < wv ? part[k] : 0;
    tot += part[k];
  }
  __syncthreads();
  excl = off + inc - v;
  return tot;
}

__global__ void __launch_bounds__(256) scan_sums_kernel(BwdWs ws) {
  __shared__ int part[4];
  const int64_t i0 = (int64_t)blockIdx.x * kScan + threadIdx.x * 4;
  int v = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) v += i0 + k < ws.nkeys ? ws.pcount[i0 + k] : 0;
  int excl;
  const int tot = block_excl_scan(v, part, excl);
  if (threadIdx.x == 0) ws.psum[blockIdx.x] = tot;
}

// one block: exclusive scan of the block sums in place
__global__ void __launch_bounds__(256) scan_partials_kernel(BwdWs ws) {
  __shared__ int part[4];
  int carry = 0;
  for (int64_t b0 = 0; b0 < ws.nsum; b0 += 256) {
    const int64_t b = b0 + threadIdx.x;
    const int v = b < ws.nsum ? ws.psum[b] : 0;
    int excl;
    const int tot = block_excl_scan(v, part, excl);
    if (b < ws.nsum) ws.psum[b] = carry + excl;
    carry += tot;
  }
  if (threadIdx.x == 0) *ws.nsorted = carry;
}

// offsets of every cell, the list of occupied cells, and the box-pass batches
// (each block of 2x2x2 cells in runs of up to 64 samples)
__global__ void __launch_bounds__(256) scan_offsets_kernel(BwdWs ws) {
  static_assert(kScan % 8 == 0, "a block of 8 keys is two threads of one scan block");
  __shared__ int part[4];
  __shared__ int lbase, bbase;
  const int64_t i0 = (int64_t)blockIdx.x * kScan + threadIdx.x * 4;
  int c[4], v = 0, occ = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    c[k] = i0 + k < ws.nkeys ? ws.pcount[i0 + k] : 0;
    v += c[k];
    occ += c[k] > 0;
  }
  // keys 8j .. 8j+7 (one block of cells) are threads 2j and 2j+1
  const int bv = v + __shfl_xor(v, 1, 64);
  const int nb = (threadIdx.x & 1) == 0 ? (bv + 63) / 64 : 0;
  int excl, oexcl, bexcl;
  block_excl_scan(v, part, excl);
  const int otot = block_excl_scan(occ, part, oexcl);
  const int btot = block_excl_scan(nb, part, bexcl);
  if (threadIdx.x == 0) {
    lbase = otot > 0 ? atomicAdd(ws.pocc, otot) : 0;
    bbase = btot > 0 ? atomicAdd(ws.nbatch, btot) : 0;
  }
  __syncthreads();
  int o = ws.psum[blockIdx.x] + excl, li = lbase + oexcl;
  for (int q = 0; q < nb; ++q)
    if (bbase + bexcl + q < ws.ndesc)
      ws.bdesc[bbase + bexcl + q] = make_int2(o + 64 * q, min(64, bv - 64 * q));
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (i0 + k < ws.nkeys) ws.pcursor[i0 + k] = o;
    if (c[k] > 0) ws.plist[li++] = (int)(i0 + k);
    o += c[k];
  }
}

// ---------------------------------------------------------------------------
// pass 3: shading reverse mode, 64 entries per wave
// ---------------------------------------------------------------------------
template <int NSH>
struct ShadeLds {
  union {
    DwLds dw;
    float sc[64][65];
  } u;
  int k0[64][3];
  int fb[64];
};

template <typename ST, typename FT, int NSH, int M>
__global__ void __launch_bounds__(BLOCK, 2) bwd_shade_kernel(RenderArgs a, BwdWs ws) {
  __shared__ ShadeLds<NSH> lds[WAVES];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  ShadeLds<NSH>& L = lds[wv];
  const ST* __restrict__ sdf = static_cast<const ST*>(a.sdf);
  const FT* __restrict__ feat = static_cast<const FT*>(a.feat);
  const FT* __restrict__ probes = static_cast<const FT*>(a.probes);
  cfloat* __restrict__ W = const_mlp(a.mlp);  // scalar loads
  const Geo G{a.R, a.P, 2.0 / (a.R - 1), 0.5 * (a.R - 1), 0.5 * (a.P - 1), a.flags};
  // the entries in the order the march wrote them
  const int64_t total = min((int64_t)min(*ws.counter, (unsigned long long)ws.cap), ws.cap);
  const int64_t nbat = (total + 63) / 64;

  f4 acc_w1 = {0.f, 0.f, 0.f, 0.f}, acc_w2 = {0.f, 0.f, 0.f, 0.f};
  float db2[3] = {0.f, 0.f, 0.f};
  const int64_t gw = (int64_t)xcd_block(blockIdx.x, gridDim.x) * WAVES + wv;
  for (int64_t b = gw; b < nbat; b += (int64_t)gridDim.x * WAVES) {
    const int64_t e = b * 64 + lane;
    const int n = (int)min((int64_t)64, total - b * 64);
    BwdEntry E;
    bool counted = false, ve = false;  // counted: holds a sample (has a probe bin slot)
    if (lane < n) {
      E = ws.entries[e];
      counted = E.lw >= 0;
      ve = counted && ws.overflow[E.lw] == 0;
    }
    float z[NIN];
#pragma unroll
    for (int j = 0; j < NIN; ++j) z[j] = 0.f;
    Normal nm;
    nm.n[0] = nm.n[1] = nm.n[2] = 0.f;
    nm.gn = 1.f;
    nm.c = 0.f;
    double x[3] = {0.0, 0.0, 0.0};
    float v[3] = {0.f, 0.f, 0.f}, Y[NSH];
#pragma unroll
    for (int j = 0; j < NSH; ++j) Y[j] = 0.f;
    if (ve) {
      x[0] = E.x[0];
      x[1] = E.x[1];
      x[2] = E.x[2];
      v[0] = E.v[0];
      v[1] = E.v[1];
      v[2] = E.v[2];
      sh_basis<NSH>(v[0], v[1], v[2], Y);
      shade_inputs<ST, FT, NSH>(sdf, feat, probes, G, x, v, Y, z, nm);
    }
    float pre[HID], hid[HID], out[3];
    mlp_lane<M>(W, z, pre, hid, out);
    const float C0 = sigmoidf(out[0]), C1 = sigmoidf(out[1]), C2 = sigmoidf(out[2]);
    float dout[3] = {0.f, 0.f, 0.f};
    if (ve) {
      // the colour, for the per-ray opacity pass
      ws.entries[e].C[0] = C0;
      ws.entries[e].C[1] = C1;
      ws.entries[e].C[2] = C2;
      const float* dLr = a.dL + 3 * (int64_t)E.ray;
      dout[0] = E.w * dLr[0] * C0 * (1.f - C0);
      dout[1] = E.w * dLr[1] * C1 * (1.f - C1);
      dout[2] = E.w * dLr[2] * C2 * (1.f - C2);
    }
    float dpre[HID], dz[NIN];
    mlp_backward_lane<M>(W, dout, pre, ve, dpre, dz);
    // SDF through the normal (the opacity path is scattered by the per-ray pass)
    if (a.g_sdf && !(G.flags & FLAG_NV_ONE)) {
      float* row = L.u.sc[lane];
#pragma unroll
      for (int q = 0; q < 64; ++q) row[q] = 0.f;
      if (ve) {
        int k0[3];
        cell_k(x, G.R, G.inv_h, k0);
        L.k0[lane][0] = k0[0];
        L.k0[lane][1] = k0[1];
        L.k0[lane][2] = k0[2];
        normal_backward_patch(patch_of_row(row, k0), k0, G, x, v, nm, dz);
      }
      wave_sync();
      sdf_patch_flush(L.u.sc, L.k0, n, lane, G.R, a.g_sdf);
      wave_sync();
    }
    if (!(G.flags & FLAG_NO_FS) && a.g_feat) {
      const Cell cs = cell_d(x, G.R, G.inv_h);
      feat_scatter_wave(L.u.sc, L.fb, ve, cs, dz, n, lane, G.R, a.g_feat);
    }
    if (ws.probe_bins) {
      // file dL/dF_a under the probe cell (the cell of the stored position, as
      // counted by the march pass)
      double xs[3] = {0.0, 0.0, 0.0};
      if (counted) {
        xs[0] = E.x[0];
        xs[1] = E.x[1];
        xs[2] = E.x[2];
      }
      const Cell cp = cell_d(xs, G.P, G.inv_hp);
      // the group leaders reserve their slots back to back; each lane then reads
      // its leader's base
      int first = 0, my_leader = 0;
      uint64_t my_grp = 0;
      for_each_key_group(counted, probe_key(cp.base, G.P), [&](int k, int leader, uint64_t grp) {
        if (lane == leader) first = atomicAdd(ws.pcursor + k, (int)__popcll(grp));
        if ((grp >> lane) & 1ull) {
          my_leader = leader;
          my_grp = grp;
        }
      });
      first = __shfl(first, my_leader, 64);
      if (counted) {
        const uint64_t grp = my_grp;
        const int k = cp.base;
        {
          ProbeRec pr;
          pr.cell = k;
          pr.f[0] = cp.fx;
          pr.f[1] = cp.fy;
          pr.f[2] = cp.fz;
          pr.v[0] = E.v[0];
          pr.v[1] = E.v[1];
          pr.v[2] = E.v[2];
          pr.dfa[0] = ve ? dz[3] : 0.f;
          pr.dfa[1] = ve ? dz[4] : 0.f;
          pr.dfa[2] = ve ? dz[5] : 0.f;
          pr.dfa[3] = ve ? dz[6] : 0.f;
          pr.pad = 0.f;
          ws.precs[first + lane_rank(grp)] = pr;
        }
      }
    }
    if (a.g_mlp) mlp_dw_wave<M>(L.u.dw, lane, ve, z, hid, dpre, dout, acc_w1, acc_w2, db2);
    wave_sync();
  }
  // MLP gradient: one row of partials per wave, summed by mlp_reduce_kernel
  if (a.g_mlp) mlp_grad_store(ws.mlp_part + gw * NMLP, lane, acc_w1, acc_w2, db2);
}

// Taped shading pass: everything it needs was recorded by the forward, so it
// depends on the MLP type only.  The weight gradients are summed first, so that
// the MLP's activations are dead before the records are built (the record fields
// are read from the entry there), which keeps the pass free of register spills.
//
// A wave's 64 entries are staged in LDS with full-line loads first: their fields are
// read at scattered points of the pass, and one field loaded across 64 lanes at the
// entry's 160-byte stride touches 80 lines, which other waves evict before the next
// field is loaded (the pass then fetched ~6x the tape from HBM).
constexpr int kEntDw = 42;  // LDS row of an entry: 40 dwords + 2 (8-byte rows, 2-way banks)
static_assert(sizeof(BwdEntry) == 40 * 4, "an entry is 40 dwords (10 x 16 bytes)");

// A wave's staged entries and its MLP-gradient tiles share LDS: the fields the records
// need are read into registers before the tiles are written (three blocks per CU).
union ShadeStage {
  unsigned e[64 * kEntDw];
  DwLds dw;
};

template <int M>
__global__ void __launch_bounds__(BLOCK, 3) tape_shade_kernel(RenderArgs a, BwdWs ws) {
  __shared__ __align__(16) ShadeStage sst[WAVES];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  DwLds& D = sst[wv].dw;
  unsigned* const stage = sst[wv].e;
  // the MLP read through scalar loads; reduced modes use the copy whose weights
  // are already rounded (no per-use conversions to keep in registers)
  cfloat* __restrict__ W = const_mlp(M == MLP_F32 ? a.mlp : ws.mlp_r);
  const Geo G{a.R, a.P, 2.0 / (a.R - 1), 0.5 * (a.R - 1), 0.5 * (a.P - 1), a.flags};
  const int64_t total = min((int64_t)min(*ws.counter, (unsigned long long)ws.cap), ws.cap);
  const int64_t nbat = (total + 63) / 64;
  f4 acc_w1 = {0.f, 0.f, 0.f, 0.f}, acc_w2 = {0.f, 0.f, 0.f, 0.f};
  float db2[3] = {0.f, 0.f, 0.f};
  const int64_t gw = (int64_t)xcd_block(blockIdx.x, gridDim.x) * WAVES + wv;
  for (int64_t b = gw; b < nbat; b += (int64_t)gridDim.x * WAVES) {
    // entries in write order (coalesced); records go to the entry's slot in
    // probe-cell-key order
    const int64_t e = b * 64 + lane;
    {
      const int nchunk = (int)min((int64_t)64, total - b * 64) * 10;
      const uint4* __restrict__ src = reinterpret_cast<const uint4*>(ws.entries + b * 64);
      uint4 v[10];
#pragma unroll
      for (int q = 0; q < 10; ++q) {
        const int c = q * 64 + lane;
        v[q] = c < nchunk ? src[c] : make_uint4(0u, 0u, 0u, 0u);
      }
      wave_sync();  // the previous batch has read its entries
#pragma unroll
      for (int q = 0; q < 10; ++q) {
        const int c = q * 64 + lane, en = c / 10, f = c - 10 * en;
        uint2* dst = reinterpret_cast<uint2*>(stage + en * kEntDw + 4 * f);
        dst[0] = make_uint2(v[q].x, v[q].y);
        dst[1] = make_uint2(v[q].z, v[q].w);
      }
      wave_sync();
    }
    const BwdEntry& E = *reinterpret_cast<const BwdEntry*>(stage + lane * kEntDw);
    bool counted = false, ve = false;
    int pk = 0;
    if (e < total) {
      const int lw = E.lw;
      if (lw >= 0) {
        counted = true;
        pk = E.pkey;
        ve = ws.overflow[lw] == 0;
      }
    }
    // slots: one atomic per distinct key of the batch (the forward counted the
    // samples per key), issued now and read only when the records are written
    bool lead = false;
    int gcount = 0, my_leader = 0;
    uint64_t my_grp = 0;
    for_each_key_group(counted, pk, [&](int k, int leader, uint64_t grp) {
      if (lane == leader) {
        lead = true;
        gcount = (int)__popcll(grp);
      }
      if ((grp >> lane) & 1ull) {
        my_leader = leader;
        my_grp = grp;
      }
    });
    int gbase = 0;
    if (lead) gbase = atomicAdd(ws.pcursor + pk, gcount);
    float z[NIN];
#pragma unroll
    for (int j = 0; j < NIN; ++j) z[j] = ve ? E.z[j] : 0.f;
    float pre[HID], hid[HID], out[3];
    mlp_lane<M, true>(W, z, pre, hid, out);
    float dout[3] = {0.f, 0.f, 0.f};
    if (ve) {
      // the colour the forward composited
      const float C0 = E.C[0], C1 = E.C[1], C2 = E.C[2], w = E.w;
      const float* dLr = a.dL + 3 * (int64_t)E.ray;
      dout[0] = w * dLr[0] * C0 * (1.f - C0);
      dout[1] = w * dLr[1] * C1 * (1.f - C1);
      dout[2] = w * dLr[2] * C2 * (1.f - C2);
    }
    float dpre[HID], dz[NIN];
    mlp_backward_lane<M, true>(W, dout, pre, ve, dpre, dz);
    // the entry's remaining fields, before the MLP-gradient tiles overwrite the stage
    const double x[3] = {E.x[0], E.x[1], E.x[2]};
    const float ev[3] = {E.v[0], E.v[1], E.v[2]};
    const float en[3] = {E.nrm[0], E.nrm[1], E.nrm[2]};
    const float egn = E.gn, es0 = E.s0, es1 = E.s1, egdl = E.gdl, egdl_prev = E.gdl_prev;
    const float eoff[3] = {E.nx_off[0], E.nx_off[1], E.nx_off[2]};
    wave_sync();
    if (a.g_mlp) mlp_dw_wave<M>(D, lane, ve, z, hid, dpre, dout, acc_w1, acc_w2, db2);
    wave_sync();
    const int gb = __shfl(gbase, my_leader, 64);
    if (counted) {
      const int slot = gb + lane_rank(my_grp);
      // SDF and feature cotangents for the box pass: the normal path and the
      // opacity path at s_i, where this sample's alpha and the previous sample's
      // meet (the rest of the opacity path is scattered by the per-ray walk)
      ScatRec r;
      r.x[0] = x[0];
      r.x[1] = x[1];
      r.x[2] = x[2];
      r.dg[0] = r.dg[1] = r.dg[2] = 0.f;
      if (ve && !(G.flags & FLAG_NV_ONE)) {
        Normal nm;
        nm.n[0] = en[0];
        nm.n[1] = en[1];
        nm.n[2] = en[2];
        nm.gn = egn;
        nm.c = z[7];
        normal_dg(ev, nm, dz, r.dg);
      }
      r.a0 = ve ? a.tau * sigmoidf(-a.tau * es0) * (egdl_prev - egdl) : 0.f;
      const bool fs = ve && !(G.flags & FLAG_NO_FS);
      r.df[0] = fs ? dz[0] : 0.f;
      r.df[1] = fs ? dz[1] : 0.f;
      r.df[2] = fs ? dz[2] : 0.f;
      r.valid = ve ? 1 : 0;
      r.off[0] = eoff[0];
      r.off[1] = eoff[1];
      r.off[2] = eoff[2];
      const bool nx = r.off[0] != 0.f || r.off[1] != 0.f || r.off[2] != 0.f;
      r.a1 = ve && nx ? a.tau * sigmoidf(-a.tau * es1) * egdl : 0.f;
      r.pad[0] = r.pad[1] = 0.f;
      ws.srecs[slot] = r;
      if (ws.probe_bins) {
        const Cell cp = cell_d(x, G.P, G.inv_hp);
        ProbeRec pr;
        pr.cell = cp.base;
        pr.f[0] = cp.fx;
        pr.f[1] = cp.fy;
        pr.f[2] = cp.fz;
        pr.v[0] = ev[0];
        pr.v[1] = ev[1];
        pr.v[2] = ev[2];
        pr.dfa[0] = ve ? dz[3] : 0.f;
        pr.dfa[1] = ve ? dz[4] : 0.f;
        pr.dfa[2] = ve ? dz[5] : 0.f;
        pr.dfa[3] = ve ? dz[6] : 0.f;
        pr.pad = 0.f;
        ws.precs[slot] = pr;
      }
    }
  }
  // MLP gradient: the block's four waves add their partials in LDS and the block
  // writes one row, summed by mlp_reduce_kernel
  static_assert(WAVES == 4, "four waves per block");
  if (a.g_mlp) {
    wave_sync();
    mlp_grad_store(&D.st[0][0], lane, acc_w1, acc_w2, db2);
    __syncthreads();
    const int t = threadIdx.x;
    if (t < NMLP) {
      const float s = (sst[0].dw.st[0][t] + sst[1].dw.st[0][t]) + (sst[2].dw.st[0][t] + sst[3].dw.st[0][t]);
      ws.mlp_part[(int64_t)blockIdx.x * NMLP + t] = s;
    }
  }
}

// the MLP with its weights (not its biases) rounded for MLP type M
template <int M>
__global__ void __launch_bounds__(256) mlp_round_kernel(const float* W, float* Wr) {
  const int i = threadIdx.x;
  if (i < NMLP) {
    const bool weight = i < OFF_B1 || (i >= OFF_W2 && i < OFF_B2);
    Wr[i] = weight ? mrnd<M>(W[i]) : W[i];
  }
}

// g_mlp[k] += sum of the rows of partials (one per shading wave or block; fixed order)
__global__ void __launch_bounds__(256) mlp_reduce_kernel(BwdWs ws, int nrows, float* g_mlp) {
  __shared__ float part[4];
  const int k = blockIdx.x;
  float acc = 0.f;
  for (int w = threadIdx.x; w < nrows; w += 256) acc += ws.mlp_part[(int64_t)w * NMLP + k];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) g_mlp[k] += (part[0] + part[1]) + (part[2] + part[3]);
}

// ---------------------------------------------------------------------------
// taped schedule, box pass: a wave takes one occupied block of 2x2x2 probe cells
// (its samples are contiguous in the sorted slots) and scatters their records 64
// at a time; the SDF and feature gradients of a batch are summed in an LDS box and
// each touched node is flushed once, in row-contiguous runs.  A block spans about
// 2 (R-1)/(P-1) grid cells per axis, so a batch's box normally fits; if not, the
// batch is split into groups of lanes.  Few registers and a modest box keep
// several waves resident to cover the latency of the flush atomics.
// ---------------------------------------------------------------------------
constexpr int kBoxCap = 3072;  // floats of a wave's box
static_assert(kBoxCap >= 64 && kBoxCap >= 8 * NF, "one sample's nodes fit a box");
static_assert(kBoxCap % 4 == 0, "boxes are cleared in float4s");

__global__ void __launch_bounds__(BLOCK) bwd_box_kernel(RenderArgs a, BwdWs ws) {
  __shared__ __align__(16) float boxes[WAVES][kBoxCap];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float* box = boxes[wv];
  const Geo G{a.R, a.P, 2.0 / (a.R - 1), 0.5 * (a.R - 1), 0.5 * (a.P - 1), a.flags};
  const int nbat = (int)min((int64_t)*ws.nbatch, ws.ndesc);
  const bool do_f = a.g_feat && !(G.flags & FLAG_NO_FS);
  for (int j0 = xcd_block(blockIdx.x, gridDim.x) * WAVES + wv; j0 < nbat;
       j0 += gridDim.x * WAVES) {
    // batches in a scrambled order (j0 * K mod nbat, K a prime above any batch
    // count): waves running at the same time flush distant parts of the surface
    const int2 bd = ws.bdesc[(int)(((uint64_t)j0 * 2654435761ull) % (uint64_t)nbat)];
    // every load comes before the flush atomics, and one wait here covers them
    // (a first use inside a pass would also wait for the atomics issued so far)
    ScatRec r = ws.srecs[bd.x + min(lane, bd.y - 1)];
    __builtin_amdgcn_s_waitcnt(0);
    const bool ve = lane < bd.y && r.valid != 0;
    if (!ve) {
      r.x[0] = r.x[1] = r.x[2] = 0.0;
      r.dg[0] = r.dg[1] = r.dg[2] = 0.f;
      r.a0 = 0.f;
      r.df[0] = r.df[1] = r.df[2] = 0.f;
      r.off[0] = r.off[1] = r.off[2] = 0.f;
      r.a1 = 0.f;
    }
    if (a.g_sdf)
      box_in_groups(ve, lane, [&](bool part, bool single) {
        return sdf_box_pass(box, kBoxCap, lane, part, r.x, r.dg, r.a0, r.off, r.a1, single, G,
                            a.g_sdf);
      });
    if (do_f)
      box_in_groups(ve, lane, [&](bool part, bool) {
        return feat_box_pass(box, kBoxCap, lane, part, r.x, r.df, G, a.g_feat);
      });
  }
}

// ---------------------------------------------------------------------------
// pass 4: probe gradient per occupied probe cell
// ---------------------------------------------------------------------------
__device__ __forceinline__ float rdlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

template <int NSH>
__global__ void __launch_bounds__(BLOCK) probe_reduce_kernel(RenderArgs a, BwdWs ws) {
  constexpr int NQ = NSH * NA;  // coefficients per node, one per lane
  constexpr int PS = NQ + 1;    // odd row stride: the record lanes' stores hit distinct banks
  __shared__ float prod[WAVES][64 * PS];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float* P = prod[wv];
  const int gw = (int)(blockIdx.x * WAVES + wv);
  const int nw = (int)(gridDim.x * WAVES);
  const int q = lane < NQ ? lane : 0;
  const int nocc = *ws.pocc;
  for (int oi = gw; oi < nocc; oi += nw) {
    const int key = ws.plist[oi];
    const int cell = probe_cell_of_key(key, a.P);
    const int cnt = ws.pcount[key];
    const int end = ws.pcursor[key];  // advanced by the placement to offset + count
    float acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.f;
    for (int r0 = end - cnt; r0 < end; r0 += 64) {
      // one record per lane: its SH x dL/dF_a products go to LDS (row of the
      // record), its 8 corner weights stay in registers
      const int m = __builtin_amdgcn_readfirstlane(min(64, end - r0));
      float wl[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) wl[c] = 0.f;
      if (lane < m) {
        const ProbeRec& pr = ws.precs[r0 + lane];
        float Y[NSH];
        sh_basis<NSH>(pr.v[0], pr.v[1], pr.v[2], Y);
        const float d[NA] = {pr.dfa[0], pr.dfa[1], pr.dfa[2], pr.dfa[3]};
#pragma unroll
        for (int jj = 0; jj < NSH; ++jj)
#pragma unroll
          for (int kk = 0; kk < NA; ++kk) P[lane * PS + jj * NA + kk] = Y[jj] * d[kk];
        corner_w(Cell{0, pr.f[0], pr.f[1], pr.f[2]}, wl);
      }
      wave_sync();
      // coefficient lanes sum the records: one LDS read and the record's weights
      // (broadcast from its lane) per record, eight records' reads in flight
      int t = 0;
      for (; t + 8 <= m; t += 8) {
        float g[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) g[u] = P[(t + u) * PS + q];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int c = 0; c < 8; ++c) acc[c] = fmaf(rdlane(wl[c], t + u), g[u], acc[c]);
      }
      for (; t < m; ++t) {
        const float g = P[t * PS + q];
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = fmaf(rdlane(wl[c], t), g, acc[c]);
      }
      wave_sync();
    }
    if (lane < NQ) {
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (acc[c] != 0.f)
          atomic_add_f32(a.g_probes + (int64_t)(cell + corner_off(c, a.P)) * NQ + lane, acc[c]);
    }
  }
}

// ---------------------------------------------------------------------------
// taped schedule: the per-ray walk that runs before the shading pass (the
// colours come from the forward)
// ---------------------------------------------------------------------------
// The walk reads bytes [32, 96) of each entry (weight, T, s_i, s_{i+1}, ray, key, wave,
// previous chunk, colour): a chunk's spans are staged in LDS with 16-byte loads, 16 lanes
// per 4 entries, instead of one 4-byte load per field and lane at the entry's stride.
constexpr int kSpanB = 32, kSpanDw = 16, kSpanRow = kSpanDw + 1;  // odd row: no bank conflicts
#define PSDF_SPAN_DW(f) ((int)(offsetof(BwdEntry, f) - kSpanB) / 4)
static_assert(offsetof(BwdEntry, w) >= kSpanB && offsetof(BwdEntry, C) + 12 <= kSpanB + 4 * kSpanDw &&
                  offsetof(BwdEntry, key) >= kSpanB && offsetof(BwdEntry, prev) >= kSpanB &&
                  offsetof(BwdEntry, T) >= kSpanB,
              "the walk's fields lie in the staged span");

struct WalkLds {
  RayD ray[64];
  unsigned span[64][kSpanRow];
  float gdl[64];
  int nin[64];
  unsigned long long mine[64];  // entries of the chunk owned by each lane's ray
};

__global__ void __launch_bounds__(BLOCK) tape_walk_kernel(RenderArgs a, BwdWs ws) {
  __shared__ WalkLds lds[WAVES];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  WalkLds& L = lds[wv];
  const unsigned lw = xcd_block(blockIdx.x, gridDim.x) * WAVES + wv;
  if (lw >= ws.n_waves || ws.overflow[lw] != 0) return;
  const int cnt = ws.count[lw];
  if (cnt == 0) return;
  const int64_t ray = (int64_t)lw * 64 + lane;
  const bool valid = ray < a.B;
  float ro[3] = {0.f, 0.f, 0.f}, rd[3] = {0.f, 0.f, 1.f}, dL[3] = {0.f, 0.f, 0.f};
  if (valid) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ro[k] = a.rays_o[3 * ray + k];
      rd[k] = a.rays_d[3 * ray + k];
      dL[k] = a.dL[3 * ray + k];
    }
  }
  RayD r;
  ray_setup_d(ro[0], ro[1], ro[2], rd[0], rd[1], rd[2], a.N, r);
  L.ray[lane] = r;
  float Rc[3] = {0.f, 0.f, 0.f};  // remaining colour of this lane's ray
  int nx_i = -2, nx_slot = -1;    // the ray's entry processed last (the next in sample order)
  int base = ws.last[lw];
  int n = cnt - 64 * ((cnt - 1) / 64);
  while (base >= 0) {  // wave-uniform
    {
      const char* __restrict__ src = reinterpret_cast<const char*>(ws.entries + base) + kSpanB;
      uint4 v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = q * 64 + lane, e = c >> 2, part = c & 3;
        v[q] = e < n ? *reinterpret_cast<const uint4*>(src + (int64_t)e * sizeof(BwdEntry) + 16 * part)
                     : make_uint4(0u, 0u, 0u, 0u);
      }
      wave_sync();  // the previous chunk's walk is done with the stage
      L.mine[lane] = 0ull;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = q * 64 + lane, e = c >> 2, part = c & 3;
        unsigned* d = &L.span[e][4 * part];
        d[0] = v[q].x;
        d[1] = v[q].y;
        d[2] = v[q].z;
        d[3] = v[q].w;
      }
    }
    wave_sync();
    int key = 0, prev = -1;
    if (lane < n) {
      key = (int)L.span[lane][PSDF_SPAN_DW(key)];
      prev = (int)L.span[lane][PSDF_SPAN_DW(prev)];
      atomicOr(&L.mine[key & 63], 1ull << lane);
    }
    wave_sync();
    // each lane walks its own ray's entries of the chunk, last sample first (a
    // ray's entries are stored in sample order)
    for (unsigned long long m = L.mine[lane]; m != 0ull;) {
      const int k = 63 - __clzll(m);
      m &= ~(1ull << k);
      {
        const unsigned* sp = L.span[k];
        const float w = __uint_as_float(sp[PSDF_SPAN_DW(w)]), T = __uint_as_float(sp[PSDF_SPAN_DW(T)]);
        const float c0 = __uint_as_float(sp[PSDF_SPAN_DW(C)]);
        const float c1 = __uint_as_float(sp[PSDF_SPAN_DW(C) + 1]);
        const float c2 = __uint_as_float(sp[PSDF_SPAN_DW(C) + 2]);
        Rc[0] = fmaf(w, c0, Rc[0]);
        Rc[1] = fmaf(w, c1, Rc[1]);
        Rc[2] = fmaf(w, c2, Rc[2]);
        const float g = dL[0] * (Rc[0] - T * c0) + dL[1] * (Rc[1] - T * c1) + dL[2] * (Rc[2] - T * c2);
        const int si = (int)sp[PSDF_SPAN_DW(key)] >> 6;
        const bool nin = nx_i == si + 1;
        if (nin) ws.entries[nx_slot].gdl_prev = g;
        L.gdl[k] = g;
        L.nin[k] = nin ? 1 : 0;
        nx_i = si;
        nx_slot = base + k;
      }
    }
    wave_sync();
    if (lane < n) {
      const float gdl = L.gdl[lane];
      const int nin = L.nin[lane];
      BwdEntry& E = ws.entries[base + lane];
      E.gdl = gdl;
      // s_{i+1} belongs to no entry: its share of the opacity gradient is added
      // with this sample's by the box pass, at x_i + off
      float off[3] = {0.f, 0.f, 0.f};
      if (!nin) {
        const RayD& rr = L.ray[key & 63];
        double x0[3], x1[3];
        sample_pos(rr, sample_t(rr, key >> 6), x0);
        sample_pos(rr, sample_t(rr, (key >> 6) + 1), x1);
#pragma unroll
        for (int c = 0; c < 3; ++c) off[c] = (float)(x1[c] - x0[c]);
      }
      E.nx_off[0] = off[0];
      E.nx_off[1] = off[1];
      E.nx_off[2] = off[2];
    }
    base = __shfl(prev, 0, 64);
    n = 64;
  }
}

// ---------------------------------------------------------------------------
// pass 5: per-ray walk and the opacity gradient
// ---------------------------------------------------------------------------
struct AlphaLds {
  RayD ray[64];
  float w[64];
  float T[64];
  float C[64][3];
  float gdl[64];
  unsigned long long mine[64];  // entries of the chunk owned by each lane's ray
};

__global__ void __launch_bounds__(BLOCK) bwd_alpha_kernel(RenderArgs a, BwdWs ws) {
  __shared__ AlphaLds lds[WAVES];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  AlphaLds& L = lds[wv];
  const unsigned lw = xcd_block(blockIdx.x, gridDim.x) * WAVES + wv;
  if (lw >= ws.n_waves || ws.overflow[lw] != 0) return;
  const int cnt = ws.count[lw];
  if (cnt == 0) return;
  const int64_t ray = (int64_t)lw * 64 + lane;
  const bool valid = ray < a.B;
  float ro[3] = {0.f, 0.f, 0.f}, rd[3] = {0.f, 0.f, 1.f}, dL[3] = {0.f, 0.f, 0.f};
  if (valid) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ro[k] = a.rays_o[3 * ray + k];
      rd[k] = a.rays_d[3 * ray + k];
      dL[k] = a.dL[3 * ray + k];
    }
  }
  RayD r;
  ray_setup_d(ro[0], ro[1], ro[2], rd[0], rd[1], rd[2], a.N, r);
  L.ray[lane] = r;
  const int R = a.R;
  const double inv_h = 0.5 * (a.R - 1);
  float Rc[3] = {0.f, 0.f, 0.f};  // remaining colour of this lane's ray
  int base = ws.last[lw];
  int n = cnt - 64 * ((cnt - 1) / 64);  // the last chunk may be partial
  while (base >= 0) {  // wave-uniform
    wave_sync();
    L.mine[lane] = 0ull;
    wave_sync();
    BwdEntry E;
    E.prev = -1;
    if (lane < n) {
      E = ws.entries[base + lane];
      atomicOr(&L.mine[E.key & 63], 1ull << lane);
      L.w[lane] = E.w;
      L.T[lane] = E.T;
      L.C[lane][0] = E.C[0];
      L.C[lane][1] = E.C[1];
      L.C[lane][2] = E.C[2];
    }
    wave_sync();
    // each lane walks its own ray's entries of the chunk, last sample first (a
    // ray's entries are stored in sample order)
    for (unsigned long long m = L.mine[lane]; m != 0ull;) {
      const int k = 63 - __clzll(m);
      m &= ~(1ull << k);
      {
        const float w = L.w[k], T = L.T[k];
        const float c0 = L.C[k][0], c1 = L.C[k][1], c2 = L.C[k][2];
        Rc[0] = fmaf(w, c0, Rc[0]);
        Rc[1] = fmaf(w, c1, Rc[1]);
        Rc[2] = fmaf(w, c2, Rc[2]);
        L.gdl[k] = dL[0] * (Rc[0] - T * c0) + dL[1] * (Rc[1] - T * c1) + dL[2] * (Rc[2] - T * c2);
      }
    }
    wave_sync();
    if (lane < n) {
      const float gdl = L.gdl[lane];
      const RayD& rr = L.ray[E.key & 63];
      const int si = E.key >> 6;
      double x0[3], x1[3];
      sample_pos(rr, sample_t(rr, si), x0);
      sample_pos(rr, sample_t(rr, si + 1), x1);
      scatter8(a.g_sdf, R, cell_d(x0, R, inv_h), -a.tau * sigmoidf(-a.tau * E.s0) * gdl);
      scatter8(a.g_sdf, R, cell_d(x1, R, inv_h), a.tau * sigmoidf(-a.tau * E.s1) * gdl);
    }
    base = __shfl(E.prev, 0, 64);
    n = 64;
  }
}

hipError_t launch_render_backward_split(const RenderArgs& a, const BwdWs& ws_in, bool from_tape,
                                        int sdf_dt, int feat_dt, int mlp_dt, int n_sh,
                                        hipStream_t s) {
  BwdWs ws = ws_in;
  // probe gradients go through the cell bins (one lane per node coefficient:
  // n_sh * n_ang <= 64 for every compiled SH order)
  ws.probe_bins = (a.g_probes && !(a.flags & FLAG_NO_FA)) ? 1 : 0;
  // a taped backward always files its samples in probe-cell order (locality of
  // the shading pass's scatters)
  ws.bins = (ws.probe_bins || from_tape) ? 1 : 0;
  const dim3 wgrid((unsigned)((a.B + BLOCK - 1) / BLOCK));
  // taped: the forward reset the slot counter and counted its samples per
  // probe-cell key; only the per-call counters are reset here
  BwdWs wc = ws;
  if (from_tape) wc.bins = 0;
  hipError_t e = launch_clear(wc, from_tape ? 0 : 1, s);
  if (e != hipSuccess) return e;
  if (!from_tape) {
    if (sdf_dt == 0)
      hipLaunchKernelGGL(bwd_march_kernel<float>, wgrid, dim3(BLOCK), 0, s, a, ws);
    else
      hipLaunchKernelGGL(bwd_march_kernel<_Float16>, wgrid, dim3(BLOCK), 0, s, a, ws);
  }
  if (ws.bins) {
    hipLaunchKernelGGL(scan_sums_kernel, dim3((unsigned)ws.nsum), dim3(256), 0, s, ws);
    hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(256), 0, s, ws);
    hipLaunchKernelGGL(scan_offsets_kernel, dim3((unsigned)ws.nsum), dim3(256), 0, s, ws);
  }
  if (from_tape && a.g_sdf) hipLaunchKernelGGL(tape_walk_kernel, wgrid, dim3(BLOCK), 0, s, a, ws);
  // enough waves to fill the chip; each loops over batches of 64 entries.  The taped
  // shading pass runs three blocks per CU (its LDS allows three): 768 blocks are all
  // resident at once, with no second round of blocks behind the first
  const int64_t want = (ws.cap + 64 * WAVES - 1) / (64 * WAVES);
  const dim3 sgrid((unsigned)max((int64_t)1, min(want, (int64_t)(from_tape ? 3 * 256 : 1024))));
  if (from_tape) {
    if (mlp_dt != 0)
      PSDF_MLP_SWITCH(mlp_dt, hipLaunchKernelGGL((mlp_round_kernel<M>), dim3(1), dim3(256), 0, s,
                                                 a.mlp, ws.mlp_r));
    PSDF_MLP_SWITCH(mlp_dt, hipLaunchKernelGGL((tape_shade_kernel<M>), sgrid, dim3(BLOCK), 0, s, a,
                                               ws));
  } else {
    PSDF_DT_SWITCH(sdf_dt, feat_dt, PSDF_SH_SWITCH(n_sh, PSDF_MLP_SWITCH(mlp_dt,
        hipLaunchKernelGGL((bwd_shade_kernel<ST, FT, NSH, M>), sgrid, dim3(BLOCK), 0, s, a,
                           ws))));
  }
  if (a.g_mlp)
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3(NMLP), dim3(256), 0, s, ws,
                       (int)(from_tape ? sgrid.x : sgrid.x * WAVES), a.g_mlp);
  if (from_tape && (a.g_sdf || a.g_feat)) {
    const dim3 bgrid((unsigned)max((int64_t)1, min(want, (int64_t)2048)));
    hipLaunchKernelGGL(bwd_box_kernel, bgrid, dim3(BLOCK), 0, s, a, ws);
  }
  if (ws.probe_bins) {
    // one wave per occupied cell (the count is on the device: enough waves for
    // a dense band, each looping)
    const int64_t pw = min(ws.nkeys, (int64_t)16384);
    const dim3 pgrid((unsigned)max((int64_t)1, (pw + WAVES - 1) / WAVES));
    PSDF_SH_SWITCH(n_sh,
        hipLaunchKernelGGL((probe_reduce_kernel<NSH>), pgrid, dim3(BLOCK), 0, s, a, ws));
  }
  if (!from_tape && a.g_sdf) hipLaunchKernelGGL(bwd_alpha_kernel, wgrid, dim3(BLOCK), 0, s, a, ws);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // waves that did not fit
  RenderArgs f = a;
  f.todo = ws.overflow;
  return launch_render_backward(f, sdf_dt, feat_dt, mlp_dt, n_sh, s);
}

}  // namespace psdf
