// SDF part of the optimiser step with the smoothed SDF and the remaining
// regularisers of Sec. 3.3 (Eqs. smooth_sdf, eikonal_reg, smmoth_normals):
// the trained parameters are the raw values shat, rendering reads s = G(shat)
// with G a 5^3 Gaussian (5 taps per axis, replicated edges), and
//   L_sdf    = lambda_sdf / R^3 * sum_nodes (s - shat)^2,
//   L_Eik    = lambda_eik / (R-2)^3 * sum_interior (|g| - 1)^2,
//   L_normal = lambda_normal / Np * sum over axis-adjacent interior pairs |n_a - n_b|^2,
// g the central differences of s, n = g / |g|, Np = 3 (R-2)^2 (R-3); optionally
// the gradient of these terms at node m is weighted by 1 / (1 + 5 |s_m|).
// Passes (one thread per node unless noted):
//   A  n and |g| at interior nodes, L_Eik;
//   B  the cotangent dg of every interior node's central-difference gradient
//      (eikonal and normal terms), L_normal;
//   C  y = g_s + W (dL/ds): the L_sdf term and dg gathered from the six
//      neighbours, L_sdf;
//   D  t = G^T y (LDS tiles, separable, the transposed edge taps);
//   E  Adam on shat with t plus the direct L_sdf term; the render gradient is
//      cleared;
//   F  s_out = G(shat_out) (LDS tiles) and its FP16 copy.
#include "device.h"
#include "kernels.h"

namespace psdf {

namespace {

constexpr int RB = 256;  // threads of the per-node passes

__device__ __forceinline__ int64_t nidx(int i, int j, int k, int R) {
  return ((int64_t)k * R + j) * R + i;
}

__device__ __forceinline__ void node_ijk(int64_t n, int R, int& i, int& j, int& k) {
  i = (int)(n % R);
  const int64_t r = n / R;
  j = (int)(r % R);
  k = (int)(r / R);
}

__device__ __forceinline__ bool interior(int i, int j, int k, int R) {
  return i >= 1 && j >= 1 && k >= 1 && i <= R - 2 && j <= R - 2 && k <= R - 2;
}

// block sum of a per-thread value, added to *dst times `scale`
__device__ __forceinline__ void block_add(float v, float* dst, float scale) {
  __shared__ float part[RB / 64];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
#pragma unroll
    for (int w = 0; w < RB / 64; ++w) s += part[w];
    if (s != 0.f) atomicAdd(dst, s * scale);
  }
}

__global__ void __launch_bounds__(RB) reg_normal_kernel(SdfRegArgs r) {
  const int64_t n = (int64_t)blockIdx.x * RB + threadIdx.x;
  const int R = r.R;
  float eik = 0.f;
  if (n < (int64_t)R * R * R) {
    int i, j, k;
    node_ijk(n, R, i, j, k);
    float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
    if (interior(i, j, k, R)) {
      const float inv2h = 0.5f / r.h;
      const float gx = (r.s[n + 1] - r.s[n - 1]) * inv2h;
      const float gy = (r.s[n + R] - r.s[n - R]) * inv2h;
      const float gz = (r.s[n + (int64_t)R * R] - r.s[n - (int64_t)R * R]) * inv2h;
      const float gn = sqrtf(gx * gx + gy * gy + gz * gz);
      const float inv = 1.0f / fmaxf(gn, 1e-30f);
      out = make_float4(gx * inv, gy * inv, gz * inv, gn);
      eik = (gn - 1.0f) * (gn - 1.0f);
    }
    reinterpret_cast<float4*>(r.nrm)[n] = out;
  }
  if (r.loss_eik) block_add(eik, r.loss_eik, r.lam_eik);
}

__global__ void __launch_bounds__(RB) reg_dg_kernel(SdfRegArgs r) {
  const int64_t n = (int64_t)blockIdx.x * RB + threadIdx.x;
  const int R = r.R;
  float lnrm = 0.f;
  if (n < (int64_t)R * R * R) {
    int i, j, k;
    node_ijk(n, R, i, j, k);
    float dgx = 0.f, dgy = 0.f, dgz = 0.f;
    if (interior(i, j, k, R)) {
      const float4* N = reinterpret_cast<const float4*>(r.nrm);
      const float4 a = N[n];
      float dn[3] = {0.f, 0.f, 0.f};
      if (r.lam_nrm != 0.f && R > 3) {
        const int idx[3] = {i, j, k};
        const int64_t st[3] = {1, R, (int64_t)R * R};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          // neighbours that are interior nodes themselves
          if (idx[ax] + 1 <= R - 2) {
            const float4 b = N[n + st[ax]];
            const float d0 = a.x - b.x, d1 = a.y - b.y, d2 = a.z - b.z;
            lnrm += d0 * d0 + d1 * d1 + d2 * d2;  // each pair once, from its lower node
            dn[0] += d0, dn[1] += d1, dn[2] += d2;
          }
          if (idx[ax] - 1 >= 1) {
            const float4 b = N[n - st[ax]];
            dn[0] += a.x - b.x, dn[1] += a.y - b.y, dn[2] += a.z - b.z;
          }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) dn[c] *= 2.0f * r.lam_nrm;
      }
      const float gn = a.w;
      if (gn > 0.f) {
        // eikonal: d/dg (|g| - 1)^2 = 2 (|g| - 1) g / |g| = 2 (|g| - 1) n
        const float ce = 2.0f * r.lam_eik * (gn - 1.0f);
        // normal: dn / dg = (I - n n^T) / |g|
        const float nd = dn[0] * a.x + dn[1] * a.y + dn[2] * a.z;
        const float inv = 1.0f / gn;
        dgx = ce * a.x + (dn[0] - nd * a.x) * inv;
        dgy = ce * a.y + (dn[1] - nd * a.y) * inv;
        dgz = ce * a.z + (dn[2] - nd * a.z) * inv;
      }
    }
    r.dg[3 * n] = dgx;
    r.dg[3 * n + 1] = dgy;
    r.dg[3 * n + 2] = dgz;
  }
  if (r.loss_nrm) block_add(lnrm, r.loss_nrm, r.lam_nrm);
}

__global__ void __launch_bounds__(RB) reg_gather_kernel(SdfRegArgs r) {
  const int64_t n = (int64_t)blockIdx.x * RB + threadIdx.x;
  const int R = r.R;
  float lsdf = 0.f;
  if (n < (int64_t)R * R * R) {
    int i, j, k;
    node_ijk(n, R, i, j, k);
    const float sv = r.s[n];
    float acc = 0.f;
    if (r.smooth) {
      const float d = sv - r.shat[n];
      lsdf = d * d;
      acc = 2.0f * r.lam_sdf * d;
    }
    const float inv2h = 0.5f / r.h;
    const int idx[3] = {i, j, k};
    const int64_t st[3] = {1, R, (int64_t)R * R};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      // node n is the + stencil point of n - e and the - stencil point of n + e
      if (idx[ax] >= 1) acc += r.dg[3 * (n - st[ax]) + ax] * inv2h;
      if (idx[ax] <= R - 2) acc -= r.dg[3 * (n + st[ax]) + ax] * inv2h;
    }
    const float W = r.weighted ? 1.0f / (1.0f + 5.0f * fabsf(sv)) : 1.0f;
    r.y[n] = r.g_s[n] + W * acc;
  }
  if (r.loss_sdf) block_add(lsdf, r.loss_sdf, r.lam_sdf);
}

// sum_k w_k [clamp(i + k) == j]: the tap of G^T from node i to node j along an axis
__device__ __forceinline__ float tap_T(int i, int j, int R, const float* w) {
  float c = 0.f;
#pragma unroll
  for (int kk = -2; kk <= 2; ++kk) {
    const int q = min(max(i + kk, 0), R - 1);
    if (q == j) c += w[kk + 2];
  }
  return c;
}

// Separable 5^3 Gaussian (TRANS = false: G, edges replicated) or its transpose,
// on tiles of 32 x 8 x 8 nodes: the tile and a halo of 2 are loaded into LDS,
// then filtered along x, y and z in turn.
constexpr int TX = 32, TY = 8, TZ = 8, HX = TX + 4, HY = TY + 4, HZ = TZ + 4;

template <bool TRANS>
__global__ void __launch_bounds__(256) smooth_kernel(int R, SmoothTaps w5, const float* __restrict__ in,
                                                     float* __restrict__ out,
                                                     _Float16* __restrict__ half) {
  __shared__ float a[HZ][HY][HX];   // input tile + halo
  __shared__ float bx[HZ][HY][TX];  // filtered along x
  __shared__ float by[HZ][TY][TX];  // and along y
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * TZ;
  const float* w = w5.w;
  for (int t = threadIdx.x; t < HX * HY * HZ; t += 256) {
    const int xi = t % HX, yi = (t / HX) % HY, zi = t / (HX * HY);
    const int gx = x0 + xi - 2, gy = y0 + yi - 2, gz = z0 + zi - 2;
    float v;
    if (TRANS) {  // the transpose reads only existing nodes
      v = (gx >= 0 && gy >= 0 && gz >= 0 && gx < R && gy < R && gz < R) ? in[nidx(gx, gy, gz, R)]
                                                                         : 0.f;
    } else {  // G replicates the edge nodes
      v = in[nidx(min(max(gx, 0), R - 1), min(max(gy, 0), R - 1), min(max(gz, 0), R - 1), R)];
    }
    a[zi][yi][xi] = v;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < TX * HY * HZ; t += 256) {
    const int xi = t % TX, yi = (t / TX) % HY, zi = t / (TX * HY);
    const int gx = x0 + xi;
    float acc = 0.f;
#pragma unroll
    for (int d = -2; d <= 2; ++d)
      acc += a[zi][yi][xi + 2 + d] * (TRANS ? tap_T(gx + d, gx, R, w) : w[d + 2]);
    bx[zi][yi][xi] = acc;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < TX * TY * HZ; t += 256) {
    const int xi = t % TX, yi = (t / TX) % TY, zi = t / (TX * TY);
    const int gy = y0 + yi;
    float acc = 0.f;
#pragma unroll
    for (int d = -2; d <= 2; ++d)
      acc += bx[zi][yi + 2 + d][xi] * (TRANS ? tap_T(gy + d, gy, R, w) : w[d + 2]);
    by[zi][yi][xi] = acc;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < TX * TY * TZ; t += 256) {
    const int xi = t % TX, yi = (t / TX) % TY, zi = t / (TX * TY);
    const int gx = x0 + xi, gy = y0 + yi, gz = z0 + zi;
    if (gx >= R || gy >= R || gz >= R) continue;
    float acc = 0.f;
#pragma unroll
    for (int d = -2; d <= 2; ++d)
      acc += by[zi + 2 + d][yi][xi] * (TRANS ? tap_T(gz + d, gz, R, w) : w[d + 2]);
    const int64_t n = nidx(gx, gy, gz, R);
    out[n] = acc;
    if (half) half[n] = (_Float16)acc;
  }
}

__global__ void __launch_bounds__(RB) adam_shat_kernel(SdfRegArgs r, StepArgs a) {
  const int64_t n = (int64_t)blockIdx.x * RB + threadIdx.x;
  if (n >= (int64_t)r.R * r.R * r.R) return;
  float G = r.t[n];
  if (r.smooth) {  // direct term of L_sdf: d/dshat (s - shat)^2 = -2 (s - shat)
    const float sv = r.s[n];
    const float W = r.weighted ? 1.0f / (1.0f + 5.0f * fabsf(sv)) : 1.0f;
    G -= W * 2.0f * r.lam_sdf * (sv - r.shat[n]);
  }
  float m = a.m_sdf[n], v = a.v_sdf[n];
  const float p = adam_update_f(a.sdf_in[n], G, m, v, a.lr_sdf, a.beta1, a.beta2, a.eps, a.bc1,
                                a.bc2);
  a.m_sdf[n] = m;
  a.v_sdf[n] = v;
  a.sdf_out[n] = p;
  if (!r.smooth && a.sdf_half) static_cast<_Float16*>(a.sdf_half)[n] = (_Float16)p;
  if (a.g_sdf[n] != 0.f) a.g_sdf[n] = 0.f;
}

}  // namespace

hipError_t launch_smooth(int R, const SmoothTaps& w, const float* in, float* out, _Float16* half,
                         bool transpose, hipStream_t s) {
  const dim3 grid((R + TX - 1) / TX, (R + TY - 1) / TY, (R + TZ - 1) / TZ);
  if (transpose)
    hipLaunchKernelGGL(smooth_kernel<true>, grid, dim3(256), 0, s, R, w, in, out, half);
  else
    hipLaunchKernelGGL(smooth_kernel<false>, grid, dim3(256), 0, s, R, w, in, out, half);
  return hipGetLastError();
}

hipError_t launch_step_sdf_reg(const StepArgs& a, hipStream_t s) {
  const int R = a.R;
  const int64_t n3 = (int64_t)R * R * R;
  const unsigned nblk = (unsigned)((n3 + RB - 1) / RB);
  SdfRegArgs r = a.reg;
  r.R = R;
  r.h = a.h;
  r.shat = a.sdf_in;
  r.s = r.smooth ? r.s_in : a.sdf_in;
  r.g_s = a.g_sdf;
  // workspace: nrm [4 n3] | dg [3 n3] | y [n3]; t reuses nrm once pass C is done
  float* ws = static_cast<float*>(r.work);
  r.nrm = ws;
  r.dg = ws + 4 * n3;
  r.y = ws + 7 * n3;
  r.t = r.smooth ? ws : r.y;
  r.loss_eik = a.losses;
  r.loss_sdf = a.losses_ext;
  r.loss_nrm = a.losses_ext ? a.losses_ext + 1 : nullptr;
  hipLaunchKernelGGL(reg_normal_kernel, dim3(nblk), dim3(RB), 0, s, r);
  hipLaunchKernelGGL(reg_dg_kernel, dim3(nblk), dim3(RB), 0, s, r);
  hipLaunchKernelGGL(reg_gather_kernel, dim3(nblk), dim3(RB), 0, s, r);
  hipError_t e = hipSuccess;
  if (r.smooth) e = launch_smooth(R, r.taps, r.y, r.t, nullptr, true, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adam_shat_kernel, dim3(nblk), dim3(RB), 0, s, r, a);
  if (r.smooth)
    e = launch_smooth(R, r.taps, a.sdf_out, r.s_out, static_cast<_Float16*>(a.sdf_half), false, s);
  if (e != hipSuccess) return e;
  // brick bounds of the field the renderer reads next
  if (a.sdf_bounds) {
    const void* src = a.sdf_half ? a.sdf_half : (r.smooth ? (const void*)r.s_out : a.sdf_out);
    e = launch_sdf_bounds(src, R, a.sdf_half ? 1 : 0, a.sdf_bounds, s);
  }
  return e != hipSuccess ? e : hipGetLastError();
}

}  // namespace psdf

// ---------------------------------------------------------------------------
// Optimiser step of the tri-plane features of sparse tiles: the smoothness of the
// factorised features (Eq. smooth_features: lambda / (slots 3 2 16 15 NF) times the
// squared differences of neighbouring texels of every plane) and Adam; one block
// per 16 x 16 plane, the plane held in LDS.  Out of place (the stencil reads
// neighbours); the gradient is cleared.
// ---------------------------------------------------------------------------
namespace psdf {

__global__ void __launch_bounds__(256) plane_step_kernel(PlaneStepArgs a) {
  constexpr int NT = 256 * NF;  // values of one plane
  __shared__ float pl[NT];
  const int64_t base = (int64_t)blockIdx.x * NT;
  for (int e = threadIdx.x; e < NT; e += 256) pl[e] = a.in[base + e];
  __syncthreads();
  float loss = 0.f;
  for (int e = threadIdx.x; e < NT; e += 256) {
    const int t = e / NF, u = t & 15, v = t >> 4;
    const float val = pl[e];
    float gr = 0.f;
    if (u > 0) gr += val - pl[e - NF];
    if (v > 0) gr += val - pl[e - 16 * NF];
    if (u < 15) {
      const float d = pl[e + NF] - val;
      gr -= d;
      loss += d * d;
    }
    if (v < 15) {
      const float d = pl[e + 16 * NF] - val;
      gr -= d;
      loss += d * d;
    }
    const float G = a.g[base + e] + 2.0f * a.scale * gr;
    float m = a.m[base + e], vv = a.v[base + e];
    const float p = adam_update_f(val, G, m, vv, a.lr, a.beta1, a.beta2, a.eps, a.bc1, a.bc2);
    a.m[base + e] = m;
    a.v[base + e] = vv;
    a.out[base + e] = p;
    if (a.half) a.half[base + e] = (_Float16)p;
    if (a.g[base + e] != 0.f) a.g[base + e] = 0.f;
  }
  if (a.loss) block_add(loss, a.loss, a.scale);
}

__global__ void zero1_plane_kernel(float* p) {
  if (threadIdx.x == 0) p[0] = 0.f;
}

hipError_t launch_plane_step(const PlaneStepArgs& a, hipStream_t s) {
  if (a.loss) hipLaunchKernelGGL(zero1_plane_kernel, dim3(1), dim3(64), 0, s, a.loss);
  if (a.n_planes > 0)
    hipLaunchKernelGGL(plane_step_kernel, dim3((unsigned)a.n_planes), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace psdf
