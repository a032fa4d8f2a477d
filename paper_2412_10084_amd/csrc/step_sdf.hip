// SDF part of the optimiser step: eikonal gradient (Sec. 3.3, Eq. eikonal_reg)
// added to the render gradient, Adam, and optionally the brick bounds of the new
// grid for the renderer's empty-space skipping.
//
// With g_n the central-difference gradient of interior node n and
// q_n = 2 (|g_n| - 1) g_n / |g_n| (0 off the interior or for g_n = 0):
//   dL/ds_m = lambda / M * sum_a (q_{m-e_a,a} - q_{m+e_a,a}) / 2h,  M = (R-2)^3.
// A workgroup owns a 64 x 8 column tile and marches it along z through a chunk
// of 16 planes.  Three s planes (tile + 2 halo) and three q planes (tile + 1
// halo: q_x, q_y of the current and next plane, q_z of three) rotate through
// LDS, so every s
// value is read from memory about 1.6 times (halos) instead of 25 times and
// every q is evaluated once per tile.  The next two s planes and the next two
// planes' gradients and moments are in flight while a plane is processed.
#include "device.h"
#include "kernels.h"

namespace psdf {

namespace {
constexpr int ETX = 64, ETY = 8, ETZ = 16;  // tile and z chunk
constexpr int ETHREADS = 256;
constexpr int SXW = ETX + 4, SYW = ETY + 4, SN = SXW * SYW;  // s plane region (halo 2)
constexpr int SPER = (SN + ETHREADS - 1) / ETHREADS;         // s loads per thread per plane
// bricks a block touches: x 9, y 2, z 9 (node 8b belongs to bricks b-1 and b)
constexpr int BTX = ETX / 8 + 1, BTY = ETY / 8 + 1, BTZ = ETZ / 8 + 1, BTN = BTX * BTY * BTZ;

__device__ __forceinline__ int enc_ord(float f) {
  const int i = __float_as_int(f);
  return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__device__ __forceinline__ float dec_ord(int e) { return __int_as_float(e >= 0 ? e : e ^ 0x7FFFFFFF); }
}  // namespace

constexpr int QXW = ETX + 2, QYW = ETY + 2, QN = QXW * QYW;  // q plane region (halo 1)

struct EikLds {
  float s[3][SN];     // s planes, slot z % 3
  float qxy[2][2][QN];  // q_x, q_y of plane z in slot z % 2 (only plane z needs them)
  float qz[3][QN];      // q_z of plane z in slot z % 3 (planes z-1, z+1 need it)
  int bmin[BTN], bmax[BTN];
  float part[ETHREADS / 64];
};

__device__ __forceinline__ int zslot(int z) { return (z + 3) % 3; }

// Global traffic goes through buffer resources, one per z plane: a plane
// outside the range has no records, and an offset outside the plane is clamped
// by the hardware (loads return 0, stores are dropped).  So no load or store
// sits in a branch, the wait counters stay exact, and the loads of later planes
// remain in flight while the current plane is processed.
constexpr int kOOB = 0x7FFFFFF0;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, int z, int zlim,
                                                           int R, int esize) {
  char* p = const_cast<char*>(static_cast<const char*>(base)) + (int64_t)z * R * R * esize;
  const int bytes = (z >= 0 && z < zlim) ? R * R * esize : 0;
  return __builtin_amdgcn_make_buffer_rsrc(p, 0, bytes, 0x00020000);
}

__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, int off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, int off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, 0);
}
// streaming (non-temporal: cache policy bit 1) forms for the optimiser state and
// the gradient, touched once per step
__device__ __forceinline__ float bload_s(__amdgpu_buffer_rsrc_t r, int off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 2));
}
__device__ __forceinline__ void bstore_s(__amdgpu_buffer_rsrc_t r, int off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, 2);
}

// s plane z of the tile region into registers (0 outside the grid)
__device__ __forceinline__ void s_plane_fetch(const float* __restrict__ s, int R, int x0, int y0,
                                              int z, float v[SPER]) {
  const __amdgpu_buffer_rsrc_t rs = plane_rsrc(s, z, R, R, 4);
#pragma unroll
  for (int u = 0; u < SPER; ++u) {
    const int idx = threadIdx.x + u * ETHREADS;
    const int ly = idx / SXW, lx = idx - ly * SXW;
    const int gx = x0 - 2 + lx, gy = y0 - 2 + ly;
    const bool in = idx < SN && gx >= 0 && gx < R && gy >= 0 && gy < R;
    v[u] = bload(rs, in ? (gy * R + gx) * 4 : kOOB);
  }
}

__device__ __forceinline__ void s_plane_store(EikLds& L, int z, const float v[SPER]) {
#pragma unroll
  for (int u = 0; u < SPER; ++u) {
    const int idx = threadIdx.x + u * ETHREADS;
    if (idx < SN) L.s[zslot(z)][idx] = v[u];
  }
}

// q of plane z over the tile + 1 halo, from s planes z-1, z, z+1
// q of plane z over the tile and its halo; returns this thread's share of the
// eikonal loss of the tile's own nodes when `own_plane`
__device__ __forceinline__ float q_plane(EikLds& L, int R, int x0, int y0, int z, float inv2h,
                                         bool own_plane) {
  float loss = 0.f;
  const float* __restrict__ sm = L.s[zslot(z - 1)];
  const float* __restrict__ s0 = L.s[zslot(z)];
  const float* __restrict__ sp = L.s[zslot(z + 1)];
  float* qxy = &L.qxy[z & 1][0][0];
  float* qz = L.qz[zslot(z)];
  for (int idx = threadIdx.x; idx < QN; idx += ETHREADS) {
    const int ly = idx / QXW, lx = idx - ly * QXW;
    const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
    const int c = (ly + 1) * SXW + (lx + 1);
    const float gxv = (s0[c + 1] - s0[c - 1]) * inv2h;
    const float gyv = (s0[c + SXW] - s0[c - SXW]) * inv2h;
    const float gzv = (sp[c] - sm[c]) * inv2h;
    const float g2 = gxv * gxv + gyv * gyv + gzv * gzv;
    const bool inner = gx >= 1 && gy >= 1 && z >= 1 && gx <= R - 2 && gy <= R - 2 && z <= R - 2;
    // 2 (|g| - 1) / |g| = 2 - 2 / |g| with the hardware reciprocal square root (1 ulp);
    // gradients too small for it (never on an SDF) take the correctly rounded forms
    float gn, f;
    if (g2 >= 1e-30f) {
      const float rg = __builtin_amdgcn_rsqf(g2);
      gn = g2 * rg;
      f = inner ? 2.0f - 2.0f * rg : 0.f;
    } else {
      gn = sqrtf(g2);
      f = inner && gn > 0.f ? 2.0f * (gn - 1.0f) / gn : 0.f;
    }
    const float e = gn - 1.0f;
    qxy[0 * QN + idx] = f * gxv;
    qxy[1 * QN + idx] = f * gyv;
    qz[idx] = f * gzv;
    // own nodes: the tile's columns inside the grid (the loss counts interior ones)
    if (own_plane && inner && lx >= 1 && lx <= ETX && ly >= 1 && ly <= ETY) loss += e * e;
  }
  return loss;
}

__global__ void __launch_bounds__(ETHREADS) step_sdf_tiled_kernel(StepArgs a, int* bounds_enc) {
  __shared__ EikLds L;
  const int R = a.R;
  unsigned bx, by, bz;
  xcd_block3(bx, by, bz);
  const int x0 = bx * ETX, y0 = by * ETY, zs = bz * ETZ, ze = min(zs + ETZ, R);
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // columns (x0+tx, y0+ty) and (.., +4)
  const float inv2h = 0.5f / a.h;
  const float M = (float)(R - 2) * (float)(R - 2) * (float)(R - 2);
  const float coef = (R >= 3 ? a.lambda_eik / M : 0.f) * inv2h;
  const float* __restrict__ s = a.sdf_in;
  const int nb = ((R - 2) >> 3) + 1;
  const bool want_b = bounds_enc != nullptr;
  const int bx0 = (x0 >> 3) - 1, by0 = (y0 >> 3) - 1, bz0 = (zs >> 3) - 1;
  if (want_b) {
    for (int t = threadIdx.x; t < BTN; t += ETHREADS) {
      L.bmin[t] = 0x7FFFFFFF;
      L.bmax[t] = (int)0x80000000;
    }
  }
  // prologue: s planes zs-2 .. zs -> q plane zs-1; s plane zs+1 -> q plane zs;
  // s planes zs+2, zs+3 in flight
  float v[SPER], v2[SPER];
  for (int z = zs - 2; z <= zs; ++z) {
    s_plane_fetch(s, R, x0, y0, z, v);
    s_plane_store(L, z, v);
  }
  s_plane_fetch(s, R, x0, y0, zs + 1, v);
  __syncthreads();
  float loss = q_plane(L, R, x0, y0, zs - 1, inv2h, false);
  __syncthreads();
  s_plane_store(L, zs + 1, v);
  __syncthreads();
  loss += q_plane(L, R, x0, y0, zs, inv2h, true);
  s_plane_fetch(s, R, x0, y0, zs + 2, v);
  s_plane_fetch(s, R, x0, y0, zs + 3, v2);

  int xb[2], nxb = 0;  // x bricks of this thread's column
  const int gx = x0 + tx;
  if (gx < R) {
    if ((gx >> 3) < nb) xb[nxb++] = gx >> 3;
    if ((gx & 7) == 0 && gx > 0) xb[nxb++] = (gx >> 3) - 1;
  }
  float bmn[2] = {INFINITY, INFINITY}, bmx[2] = {-INFINITY, -INFINITY};  // current z brick
  auto flush = [&](int c, int zb, float mn, float mx) {
    const int gy = y0 + ty + 4 * c;
    int yb[2], nyb = 0;
    if ((gy >> 3) < nb) yb[nyb++] = gy >> 3;
    if ((gy & 7) == 0 && gy > 0) yb[nyb++] = (gy >> 3) - 1;
    if (!(mn <= mx) || zb < 0 || zb >= nb) return;
    for (int p = 0; p < nxb; ++p)
      for (int r = 0; r < nyb; ++r) {
        const int t = ((zb - bz0) * BTY + (yb[r] - by0)) * BTX + (xb[p] - bx0);
        atomicMin(&L.bmin[t], enc_ord(mn));
        atomicMax(&L.bmax[t], enc_ord(mx));
      }
  };

  // gradient and moments of this thread's two nodes (0 past the chunk)
  auto gmv_fetch = [&](int z, float g[2], float m[2], float w[2]) {
    const __amdgpu_buffer_rsrc_t rg = plane_rsrc(a.g_sdf, z, ze, R, 4);
    const __amdgpu_buffer_rsrc_t rm = plane_rsrc(a.m_sdf, z, ze, R, 4);
    const __amdgpu_buffer_rsrc_t rv = plane_rsrc(a.v_sdf, z, ze, R, 4);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int gy = y0 + ty + 4 * c;
      const int off = gx < R && gy < R ? (gy * R + gx) * 4 : kOOB;
      g[c] = bload_s(rg, off);
      m[c] = bload_s(rm, off);
      w[c] = bload_s(rv, off);
    }
  };
  // two planes of gradient / moments and two s planes in flight
  float gn_[2], mn_[2], vn_[2], gn2[2], mn2[2], vn2[2];
  gmv_fetch(zs, gn_, mn_, vn_);
  gmv_fetch(zs + 1, gn2, mn2, vn2);

  for (int z = zs; z < ze; ++z) {
    float gc[2] = {gn_[0], gn_[1]}, mc[2] = {mn_[0], mn_[1]}, vc[2] = {vn_[0], vn_[1]};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      gn_[c] = gn2[c];
      mn_[c] = mn2[c];
      vn_[c] = vn2[c];
    }
    gmv_fetch(z + 2, gn2, mn2, vn2);
    __syncthreads();  // everyone is done with s plane z-1 and q plane z-2
    s_plane_store(L, z + 2, v);
#pragma unroll
    for (int u = 0; u < SPER; ++u) v[u] = v2[u];
    if (z + 4 < ze + 2) s_plane_fetch(s, R, x0, y0, z + 4, v2);
    __syncthreads();
    loss += q_plane(L, R, x0, y0, z + 1, inv2h, z + 1 < ze);
    __syncthreads();
    const float* qm = L.qz[zslot(z - 1)];
    const float* q0 = &L.qxy[z & 1][0][0];
    const float* qp = L.qz[zslot(z + 1)];
    const __amdgpu_buffer_rsrc_t wo = plane_rsrc(a.sdf_out, z, R, R, 4);
    const __amdgpu_buffer_rsrc_t wm = plane_rsrc(a.m_sdf, z, R, R, 4);
    const __amdgpu_buffer_rsrc_t wv = plane_rsrc(a.v_sdf, z, R, R, 4);
    const __amdgpu_buffer_rsrc_t wg = plane_rsrc(a.g_sdf, z, R, R, 4);
    const __amdgpu_buffer_rsrc_t wh = plane_rsrc(a.sdf_half, z, a.sdf_half ? R : 0, R, 2);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int gy = y0 + ty + 4 * c;
      const bool own = gx < R && gy < R;
      const int sc = (ty + 4 * c + 2) * SXW + (tx + 2);
      const int qc = (ty + 4 * c + 1) * QXW + (tx + 1);
      const float ge = (q0[0 * QN + qc - 1] - q0[0 * QN + qc + 1]) +
                       (q0[1 * QN + qc - QXW] - q0[1 * QN + qc + QXW]) +
                       (qm[qc] - qp[qc]);
      const float G = gc[c] + coef * ge;
      float m = mc[c], vv = vc[c];
      const float p0 = L.s[zslot(z)][sc];
      const float p = adam_update_f(p0, G, m, vv, a.lr_sdf, a.beta1, a.beta2, a.eps, a.bc1, a.bc2);
      const int off = own ? (gy * R + gx) * 4 : kOOB;
      bstore(wo, off, p);
      bstore_s(wm, off, m);
      bstore_s(wv, off, vv);
      // the render gradient is sparse: only nonzero entries are cleared
      bstore(wg, gc[c] != 0.f ? off : kOOB, 0.f);
      // FP16 copy (a resource without records when there is none)
      const _Float16 hp = (_Float16)p;
      __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, hp), wh,
                                            own ? (gy * R + gx) * 2 : kOOB, 0, 0);
      const float nv = a.sdf_half ? (float)hp : p;
      if (want_b && own && nv == nv) {
        // node z belongs to z brick z/8, and to z/8 - 1 as well when z % 8 == 0
        if ((z & 7) == 0 && z > 0) {
          bmn[c] = fminf(bmn[c], nv);
          bmx[c] = fmaxf(bmx[c], nv);
          flush(c, (z >> 3) - 1, bmn[c], bmx[c]);
          bmn[c] = bmx[c] = nv;
        } else {
          bmn[c] = fminf(bmn[c], nv);
          bmx[c] = fmaxf(bmx[c], nv);
        }
      }
    }
  }
  if (want_b) {
#pragma unroll
    for (int c = 0; c < 2; ++c) flush(c, (ze - 1) >> 3, bmn[c], bmx[c]);
    __syncthreads();
    for (int t = threadIdx.x; t < BTN; t += ETHREADS) {
      if (L.bmin[t] == 0x7FFFFFFF) continue;
      const int bxx = t % BTX + bx0, byy = (t / BTX) % BTY + by0, bzz = t / (BTX * BTY) + bz0;
      if (bxx < 0 || byy < 0 || bzz < 0 || bxx >= nb || byy >= nb || bzz >= nb) continue;
      int* e = bounds_enc + 2 * ((bzz * nb + byy) * nb + bxx);
      atomicMin(e, L.bmin[t]);
      atomicMax(e + 1, L.bmax[t]);
    }
  }
  if (a.losses) {
    const float lc = R >= 3 ? a.lambda_eik / M : 0.f;
    float w = wave_sum(loss);
    if ((threadIdx.x & 63) == 0) L.part[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
      const float t = (L.part[0] + L.part[1] + L.part[2] + L.part[3]) * lc;
      if (t != 0.f) atomic_add_f32(a.losses + 0, t);
    }
  }
}

__global__ void __launch_bounds__(256) bounds_init_kernel(int* e, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    e[2 * i] = enc_ord(INFINITY);
    e[2 * i + 1] = enc_ord(-INFINITY);
  }
}

__global__ void __launch_bounds__(256) bounds_decode_kernel(int* e, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    float* f = reinterpret_cast<float*>(e);
    f[2 * i] = dec_ord(e[2 * i]);
    f[2 * i + 1] = dec_ord(e[2 * i + 1]);
  }
}

hipError_t launch_step_sdf(const StepArgs& a, hipStream_t s) {
  const int R = a.R;
  const int nb = ((R - 2) >> 3) + 1, n3 = nb * nb * nb;
  int* enc = a.sdf_bounds ? reinterpret_cast<int*>(a.sdf_bounds) : nullptr;
  if (enc) hipLaunchKernelGGL(bounds_init_kernel, dim3((n3 + 255) / 256), dim3(256), 0, s, enc, n3);
  const dim3 grid((R + ETX - 1) / ETX, (R + ETY - 1) / ETY, (R + ETZ - 1) / ETZ);
  hipLaunchKernelGGL(step_sdf_tiled_kernel, grid, dim3(ETHREADS), 0, s, a, enc);
  if (enc) hipLaunchKernelGGL(bounds_decode_kernel, dim3((n3 + 255) / 256), dim3(256), 0, s, enc, n3);
  return hipGetLastError();
}

}  // namespace psdf
