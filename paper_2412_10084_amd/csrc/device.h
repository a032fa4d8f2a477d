// Device-side building blocks of the ProbeSDF render step for gfx950.
//
// Method: Toussaint et al., "ProbeSDF: Light Field Probes For Neural Surface
// Reconstruction", CVPR 2025.  Trilinear sampling of the SDF / features /
// probes (Sec. 3.2), real SH basis (Sec. 3.2, Eq. spherical_harmonics), colour
// MLP (Sec. 4), NeuS log-domain opacity (Sec. 3.3, Eq. neus).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psdf {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef __bf16 b4 __attribute__((ext_vector_type(4)));

// Compiled model shape: n_feat = 3, n_ang = 4, hidden = 16, n_in = 10.
constexpr int NF = 3;
constexpr int NA = 4;
constexpr int HID = 16;
constexpr int NIN = NF + NA + 3;
constexpr int NMLP = HID * NIN + HID + 3 * HID + 3;  // 227
constexpr int OFF_B1 = HID * NIN;                    // 160
constexpr int OFF_W2 = OFF_B1 + HID;                 // 176
constexpr int OFF_B2 = OFF_W2 + 3 * HID;             // 224

// MLP arithmetic modes
constexpr int MLP_F32 = 0;   // FP32 FMA per lane
constexpr int MLP_F16 = 1;   // FP16 operands on MFMA, FP32 accumulation
constexpr int MLP_BF16 = 2;  // BF16 operands on MFMA, FP32 accumulation

constexpr int FLAG_NO_FS = 1;
constexpr int FLAG_NO_FA = 2;
constexpr int FLAG_NV_ONE = 4;

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2);
// remap a linear block id so that each XCD works on one contiguous range.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned G) {
  const unsigned x = b & 7u, j = b >> 3, q = G >> 3, r = G & 7u;
  return x * q + (x < r ? x : r) + j;
}

// the same for a 3D grid: returns the remapped (x, y, z) block coordinates
__device__ __forceinline__ void xcd_block3(unsigned& bx, unsigned& by, unsigned& bz) {
  const unsigned G = gridDim.x * gridDim.y * gridDim.z;
  const unsigned L = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const unsigned Lp = xcd_block(L, G);
  bx = Lp % gridDim.x;
  const unsigned t = Lp / gridDim.x;
  by = t % gridDim.y;
  bz = t / gridDim.y;
}

// ---------------------------------------------------------------------------
// storage loads (FP32 or FP16 grids, FP32 math)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float ld1(const float* __restrict__ p, int i) { return p[i]; }
__device__ __forceinline__ float ld1(const _Float16* __restrict__ p, int i) { return (float)p[i]; }

__device__ __forceinline__ float4 ld4(const float* __restrict__ p, int i) {
  return *reinterpret_cast<const float4*>(p + i);
}
__device__ __forceinline__ float4 ld4(const _Float16* __restrict__ p, int i) {
  h4 v = *reinterpret_cast<const h4*>(p + i);
  return make_float4((float)v.x, (float)v.y, (float)v.z, (float)v.w);
}

__device__ __forceinline__ float lerpf(float a, float b, float t) { return fmaf(t, b - a, a); }

// bias-corrected Adam (Kingma & Ba, Algorithm 1) on one parameter; bc = 1 - beta^t
// The bias corrections, the square root and the quotient take the hardware's
// reciprocal and square root (1 ulp each) instead of the correctly rounded forms
// (a third of the instructions): the update's relative error stays within a few
// ulp, and the moments are computed exactly as before.
__device__ __forceinline__ float adam_update_f(float p, float G, float& m, float& v, float lr,
                                               float b1, float b2, float eps, float bc1, float bc2) {
  m = b1 * m + (1.0f - b1) * G;
  v = b2 * v + (1.0f - b2) * G * G;
  const float mh = m * __builtin_amdgcn_rcpf(bc1);
  const float vh = v * __builtin_amdgcn_rcpf(bc2);
  return p - lr * mh * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(vh) + eps);
}

// ---------------------------------------------------------------------------
// align-corners cell of a point: per axis u = (x+1)/h, k0 = clamp(floor u, 0, R-2),
// weights f = u - k0 (computed in FP64, see shade.h)
// ---------------------------------------------------------------------------
struct Cell {
  int base;  // flat index of corner (k0x, k0y, k0z)
  float fx, fy, fz;
};

// corner c = dx + 2 dy + 4 dz
__device__ __forceinline__ int corner_off(int c, int R) {
  return (c & 1) + ((c >> 1) & 1) * R + ((c >> 2) & 1) * R * R;
}

__device__ __forceinline__ void corner_w(const Cell& c, float w[8]) {
  const float gx = 1.0f - c.fx, gy = 1.0f - c.fy, gz = 1.0f - c.fz;
  const float a0 = gy * gz, a1 = c.fy * gz, a2 = gy * c.fz, a3 = c.fy * c.fz;
  w[0] = gx * a0;
  w[1] = c.fx * a0;
  w[2] = gx * a1;
  w[3] = c.fx * a1;
  w[4] = gx * a2;
  w[5] = c.fx * a2;
  w[6] = gx * a3;
  w[7] = c.fx * a3;
}

// two x-adjacent nodes in one load (unaligned 8- or 4-byte global load)
__device__ __forceinline__ float2 ld2(const float* __restrict__ p, int i) {
  float2 v;
  __builtin_memcpy(&v, p + i, sizeof(v));
  return v;
}
__device__ __forceinline__ float2 ld2(const _Float16* __restrict__ p, int i) {
  _Float16 h[2];
  __builtin_memcpy(h, p + i, sizeof(h));
  return make_float2((float)h[0], (float)h[1]);
}

// The four corner pairs of a cell, fetched ahead of their use (software
// pipelining of the march).
struct CellVals {
  float2 p00, p10, p01, p11;
  float fx, fy, fz;
};

template <typename T>
__device__ __forceinline__ CellVals fetch_cell(const T* __restrict__ g, int R, const Cell& c) {
  const int b = c.base, RR = R * R;
  return CellVals{ld2(g, b), ld2(g, b + R), ld2(g, b + RR), ld2(g, b + RR + R), c.fx, c.fy, c.fz};
}

__device__ __forceinline__ float interp_cell(const CellVals& v) {
  const float a0 = lerpf(v.p00.x, v.p00.y, v.fx), a1 = lerpf(v.p10.x, v.p10.y, v.fx);
  const float a2 = lerpf(v.p01.x, v.p01.y, v.fx), a3 = lerpf(v.p11.x, v.p11.y, v.fx);
  const float b0 = lerpf(a0, a1, v.fy), b1 = lerpf(a2, a3, v.fy);
  return lerpf(b0, b1, v.fz);
}

// Scalar trilinear value; x-adjacent corners are neighbours in memory and are
// fetched as pairs (the cell's k0x <= R-2, so b + 1 stays inside the row).
template <typename T>
__device__ __forceinline__ float tri1(const T* __restrict__ g, int R, const Cell& c) {
  const int b = c.base, RR = R * R;
  const float2 p00 = ld2(g, b), p10 = ld2(g, b + R), p01 = ld2(g, b + RR), p11 = ld2(g, b + RR + R);
  const float v000 = p00.x, v100 = p00.y, v010 = p10.x, v110 = p10.y;
  const float v001 = p01.x, v101 = p01.y, v011 = p11.x, v111 = p11.y;
  const float a0 = lerpf(v000, v100, c.fx), a1 = lerpf(v010, v110, c.fx);
  const float a2 = lerpf(v001, v101, c.fx), a3 = lerpf(v011, v111, c.fx);
  const float b0 = lerpf(a0, a1, c.fy), b1 = lerpf(a2, a3, c.fy);
  return lerpf(b0, b1, c.fz);
}

// ---------------------------------------------------------------------------
// Real SH basis, orthonormal, no Condon-Shortley phase, ordered (0,0), (1,-1),
// (1,0), (1,1), (2,-2), ..., (3,3); the argument is a unit vector.
// ---------------------------------------------------------------------------
template <int NSH>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  Y[0] = 0.28209479177387814f;
  if constexpr (NSH >= 4) {
    Y[1] = 0.4886025119029199f * y;
    Y[2] = 0.4886025119029199f * z;
    Y[3] = 0.4886025119029199f * x;
  }
  if constexpr (NSH >= 9) {
    Y[4] = 1.0925484305920792f * x * y;
    Y[5] = 1.0925484305920792f * y * z;
    Y[6] = 0.31539156525252005f * (3.0f * z * z - 1.0f);
    Y[7] = 1.0925484305920792f * x * z;
    Y[8] = 0.5462742152960396f * (x * x - y * y);
  }
  if constexpr (NSH >= 16) {
    Y[9] = 0.5900435899266435f * y * (3.0f * x * x - y * y);
    Y[10] = 2.890611442640554f * x * y * z;
    Y[11] = 0.4570457994644658f * y * (5.0f * z * z - 1.0f);
    Y[12] = 0.3731763325901154f * z * (5.0f * z * z - 3.0f);
    Y[13] = 0.4570457994644658f * x * (5.0f * z * z - 1.0f);
    Y[14] = 1.445305721320277f * z * (x * x - y * y);
    Y[15] = 0.5900435899266435f * x * (x * x - 3.0f * y * y);
  }
}

// log(1 + y) for 0 <= y <= 1 as 2 atanh(t), t = y / (2 + y) <= 1/3: the odd series
// t + t^3/3 + t^5/5 + ... summed to t^15 (the first term left out is below 2^-25 of the
// sum), with the quotient corrected by one Newton step.  Within 2 ulp of log1p for
// normal y, a fifth of the instructions of the library routine, which carries extra
// precision throughout.
__device__ __forceinline__ float log1p_unit(float y) {
  const float d = 2.0f + y;
  const float r = __builtin_amdgcn_rcpf(d);
  float t = y * r;
  t = fmaf(fmaf(-t, d, y), r, t);
  const float s = t * t;
  float q = 2.0f / 15.0f;
  q = fmaf(q, s, 2.0f / 13.0f);
  q = fmaf(q, s, 2.0f / 11.0f);
  q = fmaf(q, s, 2.0f / 9.0f);
  q = fmaf(q, s, 2.0f / 7.0f);
  q = fmaf(q, s, 2.0f / 5.0f);
  q = fmaf(q, s, 2.0f / 3.0f);
  return fmaf(t * s, q, 2.0f * t);
}

// log of the logistic Phi(x) = 1/(1+e^-x), overflow free
__device__ __forceinline__ float log_sigmoid(float x) {
  return fminf(x, 0.0f) - log1p_unit(expf(-fabsf(x)));
}
__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }

// ---------------------------------------------------------------------------
// operand rounding of the reduced-precision MLP modes (round to nearest even)
// ---------------------------------------------------------------------------
template <int M>
__device__ __forceinline__ float mrnd(float x) {
  if constexpr (M == MLP_F16) return (float)(_Float16)x;
  else if constexpr (M == MLP_BF16) return (float)(__bf16)x;
  else return x;
}

// Per-lane colour MLP.  In the reduced modes the operands are rounded exactly as
// the MFMA path rounds them, products are exact in FP32 and sums are FP32, so the
// two differ only in summation order.

// W: the packed MLP, in global memory or (const_mlp) in the constant address
// space, which the compiler reads with scalar loads
typedef const float __attribute__((address_space(4))) cfloat;
__device__ __forceinline__ cfloat* const_mlp(const float* W) {
  return (cfloat*)(W);
}
// WR: the weights (not the biases) are already rounded as mrnd<M> rounds them
template <int M, bool WR>
__device__ __forceinline__ float wrnd(float w) {
  if constexpr (WR) return w;
  else return mrnd<M>(w);
}

template <int M, bool WR = false, typename WT>
__device__ __forceinline__ void mlp_lane(WT* __restrict__ W, const float z[NIN], float pre[HID],
                                         float hid[HID], float out[3]) {
#pragma unroll
  for (int k = 0; k < HID; ++k) {
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < NIN; ++j) acc = fmaf(wrnd<M, WR>(W[k * NIN + j]), mrnd<M>(z[j]), acc);
    acc += W[OFF_B1 + k];
    pre[k] = acc;
    hid[k] = fmaxf(acc, 0.0f);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < HID; ++k)
      acc = fmaf(wrnd<M, WR>(W[OFF_W2 + c * HID + k]), mrnd<M>(hid[k]), acc);
    out[c] = acc + W[OFF_B2 + c];
  }
}

// ---------------------------------------------------------------------------
// wave-level helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

// Orders this wave's LDS traffic across lanes (LDS executes a wave's operations
// in issue order; this keeps the compiler from reordering around the exchange).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ void atomic_add_f32(float* p, float v) {
  // no-return FP32 atomic at L2 (built with -munsafe-fp-atomics)
  atomicAdd(p, v);
}

}  // namespace psdf
