// C ABI of the ProbeSDF render-step library: argument validation on the host,
// then dispatch to the HIP kernels.  No error path enqueues work; no C++
// exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "../../include/probesdf.h"
#include "kernels.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int ok() {
  g_err[0] = '\0';
  return PSDF_OK;
}

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int dt_size(int dt) { return dt == PSDF_F32 ? 4 : 2; }

int check_field(const psdf_field* f) {
  if (!f) return fail(PSDF_EINVAL, "field is NULL");
  if (f->struct_size != sizeof(psdf_field))
    return fail(PSDF_EINVAL, "field.struct_size %u != %zu", f->struct_size, sizeof(psdf_field));
  if (f->R < 2 || f->R > 1024 || f->P < 2 || f->P > 1024)
    return fail(PSDF_EINVAL, "grid sizes R=%d P=%d outside [2, 1024]", f->R, f->P);
  if (f->n_feat != 3 || f->n_ang != 4)
    return fail(PSDF_EUNSUPPORTED, "compiled shape is n_feat=3 n_ang=4 (got %d %d)", f->n_feat,
                f->n_ang);
  if (!((f->mlp_hidden == 16 && f->mlp_layers == 1) || (f->mlp_hidden == 32 && f->mlp_layers == 2)))
    return fail(PSDF_EUNSUPPORTED, "MLP of %d hidden layer(s) of %d: compiled are 1 x 16 and 2 x 32",
                f->mlp_layers, f->mlp_hidden);
  if (f->sh_coeffs != 1 && f->sh_coeffs != 4 && f->sh_coeffs != 9 && f->sh_coeffs != 16)
    return fail(PSDF_EUNSUPPORTED, "sh_coeffs=%d not in {1,4,9,16}", f->sh_coeffs);
  const double r3 = (double)f->R * f->R * f->R, p3 = (double)f->P * f->P * f->P;
  if (r3 * f->n_feat >= 2147483648.0 || p3 * f->sh_coeffs * f->n_ang >= 2147483648.0)
    return fail(PSDF_EINVAL, "grid too large for 32-bit element indices");
  if (f->sdf_dtype != PSDF_F32 && f->sdf_dtype != PSDF_F16)
    return fail(PSDF_EUNSUPPORTED, "sdf_dtype %d", f->sdf_dtype);
  if (f->feat_dtype != PSDF_F32 && f->feat_dtype != PSDF_F16)
    return fail(PSDF_EUNSUPPORTED, "feat_dtype %d", f->feat_dtype);
  if (f->mlp_dtype != PSDF_F32 && f->mlp_dtype != PSDF_F16 && f->mlp_dtype != PSDF_BF16)
    return fail(PSDF_EUNSUPPORTED, "mlp_dtype %d", f->mlp_dtype);
  if (!f->sdf || !f->feat || !f->probes || !f->mlp)
    return fail(PSDF_EINVAL, "field has a NULL array");
  if (!aligned(f->sdf, dt_size(f->sdf_dtype)) || !aligned(f->feat, dt_size(f->feat_dtype)) ||
      !aligned(f->mlp, 4))
    return fail(PSDF_EALIGN, "sdf/feat/mlp misaligned");
  if (!aligned(f->probes, f->feat_dtype == PSDF_F32 ? 16 : 8))
    return fail(PSDF_EALIGN, "probes must be %d-byte aligned", f->feat_dtype == PSDF_F32 ? 16 : 8);
  if (f->sdf_bounds && !aligned(f->sdf_bounds, 8))
    return fail(PSDF_EALIGN, "sdf_bounds must be 8-byte aligned");
  if (f->tile_T < 0) return fail(PSDF_EINVAL, "tile_T must be >= 0");
  if (f->tile_T > 0) {
    if (f->R != 16 * f->tile_T + 1)
      return fail(PSDF_EINVAL, "tiled fields have R = 16 tile_T + 1 (R=%d, tile_T=%d)", f->R,
                  f->tile_T);
    if (!f->tile_index) return fail(PSDF_EINVAL, "tile_index is NULL");
    if (!aligned(f->tile_index, 4)) return fail(PSDF_EALIGN, "tile_index misaligned");
    if (f->n_tiles < 0 || f->n_tiles > (int64_t)f->tile_T * f->tile_T * f->tile_T ||
        (double)f->n_tiles * 3 * 256 * f->n_feat >= 2147483648.0)
      return fail(PSDF_EINVAL, "n_tiles out of range");
  }
  return PSDF_OK;
}

int check_opts(const psdf_render_opts* o) {
  if (!o) return fail(PSDF_EINVAL, "opts is NULL");
  if (o->struct_size != sizeof(psdf_render_opts))
    return fail(PSDF_EINVAL, "opts.struct_size %u != %zu", o->struct_size, sizeof(psdf_render_opts));
  if (o->n_samples < 2 || o->n_samples > 4096)
    return fail(PSDF_EINVAL, "n_samples=%d outside [2, 4096]", o->n_samples);
  if (!(o->tau > 0.f) || !std::isfinite(o->tau)) return fail(PSDF_EINVAL, "tau must be finite > 0");
  if (!std::isfinite(o->skip_voxels)) return fail(PSDF_EINVAL, "skip_voxels must be finite");
  if (o->flags & ~31) return fail(PSDF_EINVAL, "unknown flags 0x%x", o->flags);
  return PSDF_OK;
}

// The paper's colour model (reflected SH argument, (1 - n.v)^0..5 inputs, or the
// two-layer MLP of 32) runs on its own kernels, with these limits.
bool paper_model(const psdf_field* f, int32_t flags) {
  return f->mlp_hidden != 16 || f->mlp_layers != 1 || f->tile_T > 0 ||
         (flags & (PSDF_FLAG_SH_REFLECT | PSDF_FLAG_FRESNEL_PAPER)) != 0;
}

int check_paper_model(const psdf_field* f, const psdf_render_opts* o) {
  if (f->sdf_dtype != PSDF_F32)
    return fail(PSDF_EUNSUPPORTED, "the paper colour model needs an FP32 sdf");
  if (!((f->feat_dtype == PSDF_F32 && f->mlp_dtype == PSDF_F32) ||
        (f->feat_dtype == PSDF_F16 && f->mlp_dtype != PSDF_F32)))
    return fail(PSDF_EUNSUPPORTED,
                "the paper colour model pairs FP32 features with the FP32 MLP and FP16 features "
                "with the FP16 / BF16 MLP (got feat_dtype %d, mlp_dtype %d)",
                f->feat_dtype, f->mlp_dtype);
  if (f->sh_coeffs != 9 && f->sh_coeffs != 16)
    return fail(PSDF_EUNSUPPORTED, "the paper colour model takes sh_coeffs 9 or 16 (got %d)",
                f->sh_coeffs);
  if (o->n_samples > PSDF_MODEL_MAX_SAMPLES)
    return fail(PSDF_EUNSUPPORTED, "the paper colour model takes n_samples <= %d (got %d)",
                PSDF_MODEL_MAX_SAMPLES, o->n_samples);
  return PSDF_OK;
}

int check_f32(const void* p, const char* name) {
  if (!p) return fail(PSDF_EINVAL, "%s is NULL", name);
  if (!aligned(p, 4)) return fail(PSDF_EALIGN, "%s misaligned", name);
  return PSDF_OK;
}

int hip_status(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(PSDF_EHIP, "%s: %s", what, hipGetErrorString(e));
  return ok();
}

psdf::RenderArgs render_args(const psdf_field* f, const psdf_render_opts* o, int64_t B,
                             const float* ro, const float* rd) {
  psdf::RenderArgs a{};
  a.B = B;
  a.rays_o = ro;
  a.rays_d = rd;
  a.R = f->R;
  a.P = f->P;
  a.h = (float)(2.0 / (f->R - 1));
  a.inv_h = (float)((f->R - 1) / 2.0);
  a.inv_hp = (float)((f->P - 1) / 2.0);
  a.sdf = f->sdf;
  a.feat = f->feat;
  a.probes = f->probes;
  a.mlp = f->mlp;
  a.bounds = f->sdf_bounds;
  a.tile_index = f->tile_T > 0 ? f->tile_index : nullptr;
  a.tile_T = f->tile_T;
  a.N = o->n_samples;
  a.tau = o->tau;
  a.skip_thr = o->skip_voxels > 0.f ? (float)(o->skip_voxels * (2.0 / (f->R - 1))) : 0.f;
  a.flags = o->flags;
  return a;
}

const int64_t kMaxRays = (int64_t)1 << 31;

}  // namespace

// Device scratch of psdf_render_backward_noalloc: a workspace of the
// entry-parallel backward that no call allocates.  Every GPU the library runs on
// holds its own copy until the process ends; all calls on one GPU share it.  In
// host code `scratch` names a host-side stand-in, not the device array: kernels
// and copies only ever see the device address taken below.
__device__ __align__(256) unsigned char scratch[PSDF_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call made with that device current and kept for later calls.
int scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(PSDF_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(PSDF_EHIP, "device id %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PSDF_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return PSDF_OK;
}

}  // namespace

extern "C" {

int psdf_abi_version(void) { return PSDF_ABI_VERSION; }

const char* psdf_last_error(void) { return g_err; }

static int check_ws(void* ws, int64_t bytes, int64_t B, int P, const char* what) {
  if (!aligned(ws, 256)) return fail(PSDF_EALIGN, "%s must be 256-byte aligned", what);
  const int64_t need = psdf::bwd_ws_bytes(B, P, 0);
  if (bytes < need || bytes > ((int64_t)1 << 40))
    return fail(PSDF_EINVAL, "%s bytes=%lld outside [%lld, 2^40]", what, (long long)bytes,
                (long long)need);
  return PSDF_OK;
}

int psdf_render_forward(const psdf_field* field, const psdf_render_opts* opts, int64_t B,
                        const float* rays_o, const float* rays_d, float* rgb, float* aux,
                        float* depth_wsum, void* tape, int64_t tape_bytes, void* stream) {
  int rc;
  if ((rc = check_field(field)) || (rc = check_opts(opts))) return rc;
  if (B < 0 || B > kMaxRays) return fail(PSDF_EINVAL, "B=%lld out of range", (long long)B);
  if (B == 0) return ok();
  if ((rc = check_f32(rays_o, "rays_o")) || (rc = check_f32(rays_d, "rays_d")) ||
      (rc = check_f32(rgb, "rgb")))
    return rc;
  if ((aux && !aligned(aux, 4)) || (depth_wsum && !aligned(depth_wsum, 4)))
    return fail(PSDF_EALIGN, "aux/depth_wsum misaligned");
  psdf::RenderArgs a = render_args(field, opts, B, rays_o, rays_d);
  a.rgb = rgb;
  a.aux = aux;
  a.depth_wsum = depth_wsum;
  if (paper_model(field, opts->flags)) {
    if ((rc = check_paper_model(field, opts))) return rc;
    if (tape && (rc = check_ws(tape, tape_bytes, B, field->P, "tape"))) return rc;
    return hip_status(psdf::launch_render_model(a, false, field->sdf_dtype, field->feat_dtype,
                                                field->mlp_dtype, field->sh_coeffs,
                                                field->mlp_hidden, field->mlp_layers,
                                                static_cast<hipStream_t>(stream)),
                      "render_forward launch");
  }
  psdf::BwdWs ws{};
  if (tape) {
    if ((rc = check_ws(tape, tape_bytes, B, field->P, "tape"))) return rc;
    ws = psdf::bwd_ws_carve(tape, B, field->P, tape_bytes);
  }
  return hip_status(psdf::launch_render_forward(a, tape ? &ws : nullptr, field->sdf_dtype,
                                                field->feat_dtype,
                                                field->mlp_dtype, field->sh_coeffs,
                                                static_cast<hipStream_t>(stream)),
                    "render_forward launch");
}

int64_t psdf_backward_workspace_bytes(int64_t B, int32_t P, int64_t max_samples) {
  if (B < 0 || B > kMaxRays || P < 2 || P > 1024 || max_samples < 0 ||
      max_samples > ((int64_t)1 << 31))
    return -1;
  return psdf::bwd_ws_bytes(B, P, max_samples);
}

// Host-side validation shared by the backward entry points; fills `a`.
static int prep_backward(const psdf_field* field, const psdf_render_opts* opts, int64_t B,
                         const float* rays_o, const float* rays_d, const float* aux,
                         const float* dL_drgb, const psdf_grads* grads, psdf::RenderArgs& a) {
  int rc;
  if ((rc = check_field(field)) || (rc = check_opts(opts))) return rc;
  if (B < 0 || B > kMaxRays) return fail(PSDF_EINVAL, "B=%lld out of range", (long long)B);
  if (!grads) return fail(PSDF_EINVAL, "grads is NULL");
  if (B == 0) return PSDF_OK;
  if ((rc = check_f32(rays_o, "rays_o")) || (rc = check_f32(rays_d, "rays_d")) ||
      (rc = check_f32(aux, "aux")) || (rc = check_f32(dL_drgb, "dL_drgb")))
    return rc;
  const float* gp[4] = {grads->sdf, grads->feat, grads->probes, grads->mlp};
  for (const float* p : gp)
    if (p && !aligned(p, 4)) return fail(PSDF_EALIGN, "gradient buffer misaligned");
  a = render_args(field, opts, B, rays_o, rays_d);
  a.aux_in = aux;
  a.dL = dL_drgb;
  a.g_sdf = grads->sdf;
  a.g_feat = grads->feat;
  a.g_probes = grads->probes;
  a.g_mlp = grads->mlp;
  return PSDF_OK;
}

int psdf_render_backward(const psdf_field* field, const psdf_render_opts* opts, int64_t B,
                         const float* rays_o, const float* rays_d, const float* aux,
                         const float* dL_drgb, const psdf_grads* grads, void* workspace,
                         int64_t workspace_bytes, int32_t flags, void* stream) {
  int rc;
  psdf::RenderArgs a{};
  if ((rc = prep_backward(field, opts, B, rays_o, rays_d, aux, dL_drgb, grads, a))) return rc;
  if (B == 0) return ok();
  if (flags & ~PSDF_BWD_FROM_TAPE) return fail(PSDF_EINVAL, "unknown backward flags 0x%x", flags);
  if ((flags & PSDF_BWD_FROM_TAPE) && !workspace)
    return fail(PSDF_EINVAL, "PSDF_BWD_FROM_TAPE needs the workspace the forward recorded");
  if (paper_model(field, opts->flags)) {
    if ((rc = check_paper_model(field, opts))) return rc;
    if (workspace && (rc = check_ws(workspace, workspace_bytes, B, field->P, "workspace")))
      return rc;
    return hip_status(psdf::launch_render_model(a, true, field->sdf_dtype, field->feat_dtype,
                                                field->mlp_dtype, field->sh_coeffs,
                                                field->mlp_hidden, field->mlp_layers,
                                                static_cast<hipStream_t>(stream)),
                      "render_backward launch");
  }
  if (workspace) {
    if ((rc = check_ws(workspace, workspace_bytes, B, field->P, "workspace"))) return rc;
    const psdf::BwdWs ws = psdf::bwd_ws_carve(workspace, B, field->P, workspace_bytes);
    return hip_status(psdf::launch_render_backward_split(a, ws, (flags & PSDF_BWD_FROM_TAPE) != 0,
                                                         field->sdf_dtype,
                                                         field->feat_dtype, field->mlp_dtype,
                                                         field->sh_coeffs,
                                                         static_cast<hipStream_t>(stream)),
                      "render_backward launch");
  }
  return hip_status(psdf::launch_render_backward(a, field->sdf_dtype, field->feat_dtype,
                                                 field->mlp_dtype, field->sh_coeffs,
                                                 static_cast<hipStream_t>(stream)),
                    "render_backward launch");
}

int psdf_render_backward_noalloc(const psdf_field* field, const psdf_render_opts* opts, int64_t B,
                                 const float* rays_o, const float* rays_d, const float* aux,
                                 const float* dL_drgb, const psdf_grads* grads, void* stream) {
  int rc;
  psdf::RenderArgs a{};
  if ((rc = prep_backward(field, opts, B, rays_o, rays_d, aux, dL_drgb, grads, a))) return rc;
  if (B == 0) return ok();
  if (paper_model(field, opts->flags)) {  // its reverse mode uses no workspace
    if ((rc = check_paper_model(field, opts))) return rc;
    return hip_status(psdf::launch_render_model(a, true, field->sdf_dtype, field->feat_dtype,
                                                field->mlp_dtype, field->sh_coeffs,
                                                field->mlp_hidden, field->mlp_layers,
                                                static_cast<hipStream_t>(stream)),
                      "render_backward_noalloc launch");
  }
  const int64_t need = psdf::bwd_ws_bytes(B, field->P, 0);
  if (need > (int64_t)PSDF_NOALLOC_SCRATCH_BYTES)
    return fail(PSDF_EINVAL,
                "B=%lld, P=%d need %lld bytes of fixed workspace, more than the %lld-byte static "
                "scratch of psdf_render_backward_noalloc (use psdf_render_backward with a "
                "workspace)",
                (long long)B, field->P, (long long)need, (long long)PSDF_NOALLOC_SCRATCH_BYTES);
  void* base = nullptr;
  if ((rc = scratch_of_current_device(&base))) return rc;
  const psdf::BwdWs ws = psdf::bwd_ws_carve(base, B, field->P, PSDF_NOALLOC_SCRATCH_BYTES);
  return hip_status(psdf::launch_render_backward_split(a, ws, false, field->sdf_dtype,
                                                       field->feat_dtype, field->mlp_dtype,
                                                       field->sh_coeffs,
                                                       static_cast<hipStream_t>(stream)),
                    "render_backward_noalloc launch");
}

int psdf_l1_loss(int64_t B, const float* rgb, const float* target, float* dL_drgb, float* loss,
                 void* stream) {
  int rc;
  if (B < 0 || B > kMaxRays) return fail(PSDF_EINVAL, "B=%lld out of range", (long long)B);
  if (B == 0) return ok();
  if ((rc = check_f32(rgb, "rgb")) || (rc = check_f32(target, "target")) ||
      (rc = check_f32(dL_drgb, "dL_drgb")))
    return rc;
  if (loss && !aligned(loss, 4)) return fail(PSDF_EALIGN, "loss misaligned");
  return hip_status(psdf::launch_l1_loss(B, rgb, target, dL_drgb, loss,
                                         static_cast<hipStream_t>(stream)),
                    "l1_loss launch");
}

static bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
}

// taps of the 5^3 Gaussian: exp(-k^2 / (2 sigma^2)), k = -2..2, normalised (in FP64)
static psdf::SmoothTaps smooth_taps(float sigma) {
  psdf::SmoothTaps t;
  double w[5], sum = 0.0;
  for (int k = -2; k <= 2; ++k) {
    w[k + 2] = std::exp(-(double)(k * k) / (2.0 * (double)sigma * (double)sigma));
    sum += w[k + 2];
  }
  for (int k = 0; k < 5; ++k) t.w[k] = (float)(w[k] / sum);
  return t;
}

int64_t psdf_step_work_bytes(int32_t R) {
  if (R < 2 || R > 1024) return -1;
  return (int64_t)8 * R * R * R * (int64_t)sizeof(float);
}

int psdf_smooth_sdf(int32_t R, float sigma, const float* shat, float* s, void* s_half,
                    void* stream) {
  if (R < 2 || R > 1024) return fail(PSDF_EINVAL, "R=%d outside [2, 1024]", R);
  if (!(sigma > 0.f) || !std::isfinite(sigma)) return fail(PSDF_EINVAL, "sigma must be finite > 0");
  int rc;
  if ((rc = check_f32(shat, "shat")) || (rc = check_f32(s, "s"))) return rc;
  if (s_half && !aligned(s_half, 2)) return fail(PSDF_EALIGN, "s_half misaligned");
  const size_t bs = (size_t)R * R * R * 4;
  if (overlap(shat, bs, s, bs)) return fail(PSDF_EINVAL, "shat and s must not overlap");
  return hip_status(psdf::launch_smooth(R, smooth_taps(sigma), shat, s,
                                        static_cast<_Float16*>(s_half), false,
                                        static_cast<hipStream_t>(stream)),
                    "smooth_sdf launch");
}

int psdf_l2rel_loss(int64_t B, const float* rgb, const float* target, float* dL_drgb, float* loss,
                    float lambda, float eps, float n_images, void* stream) {
  int rc;
  if (B < 0 || B > kMaxRays) return fail(PSDF_EINVAL, "B=%lld out of range", (long long)B);
  if (!std::isfinite(lambda) || !(eps > 0.f) || !std::isfinite(eps) || !(n_images > 0.f) ||
      !std::isfinite(n_images))
    return fail(PSDF_EINVAL, "lambda finite, eps > 0 and n_images > 0 required");
  if (B == 0) return ok();
  if ((rc = check_f32(rgb, "rgb")) || (rc = check_f32(target, "target")) ||
      (rc = check_f32(dL_drgb, "dL_drgb")))
    return rc;
  if (loss && !aligned(loss, 4)) return fail(PSDF_EALIGN, "loss misaligned");
  return hip_status(psdf::launch_l2rel_loss(B, rgb, target, dL_drgb, loss, lambda, eps, n_images,
                                            static_cast<hipStream_t>(stream)),
                    "l2rel_loss launch");
}

int psdf_plane_step(int64_t n_tiles, int32_t n_feat, const float* in, float* out, float* g,
                    float* m, float* v, int64_t step, float lr, float beta1, float beta2,
                    float eps, float lambda, void* half_out, float* loss, void* stream) {
  if (n_feat != 3) return fail(PSDF_EUNSUPPORTED, "n_feat=%d (compiled: 3)", n_feat);
  if (n_tiles < 0 || (double)n_tiles * 3 * 256 * n_feat >= 2147483648.0)
    return fail(PSDF_EINVAL, "n_tiles out of range");
  if (step < 1) return fail(PSDF_EINVAL, "step must be >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f) ||
      !std::isfinite(lr) || !std::isfinite(lambda))
    return fail(PSDF_EINVAL, "Adam hyper-parameters / lambda out of range");
  if (n_tiles == 0) return ok();
  const void* req[] = {in, out, g, m, v};
  for (const void* p : req) {
    if (!p) return fail(PSDF_EINVAL, "a plane step buffer is NULL");
    if (!aligned(p, 16)) return fail(PSDF_EALIGN, "plane step buffers must be 16-byte aligned");
  }
  const size_t nb = (size_t)n_tiles * 3 * 256 * n_feat * 4;
  if (overlap(in, nb, out, nb)) return fail(PSDF_EINVAL, "the plane step is out of place");
  if (half_out && !aligned(half_out, 8)) return fail(PSDF_EALIGN, "half_out misaligned");
  if (loss && !aligned(loss, 4)) return fail(PSDF_EALIGN, "loss misaligned");
  psdf::PlaneStepArgs a{};
  a.n_planes = 3 * n_tiles;
  a.scale = (float)((double)lambda / ((double)n_tiles * 3 * 2 * 16 * 15 * n_feat));
  a.lr = lr;
  a.beta1 = beta1;
  a.beta2 = beta2;
  a.eps = eps;
  a.bc1 = (float)(1.0 - std::pow((double)beta1, (double)step));
  a.bc2 = (float)(1.0 - std::pow((double)beta2, (double)step));
  a.in = in;
  a.out = out;
  a.g = g;
  a.m = m;
  a.v = v;
  a.half = static_cast<_Float16*>(half_out);
  a.loss = loss;
  return hip_status(psdf::launch_plane_step(a, static_cast<hipStream_t>(stream)),
                    "plane_step launch");
}

int psdf_grid_step(const psdf_step_args* s, void* stream) {
  if (!s) return fail(PSDF_EINVAL, "args is NULL");
  if (s->struct_size != sizeof(psdf_step_args))
    return fail(PSDF_EINVAL, "args.struct_size %u != %zu", s->struct_size, sizeof(psdf_step_args));
  if (s->R < 2 || s->R > 1024 || s->P < 2 || s->P > 1024 || s->n_feat < 1 || s->n_pc < 1 ||
      s->n_mlp < 0)
    return fail(PSDF_EINVAL, "bad sizes R=%d P=%d n_feat=%d n_pc=%d n_mlp=%d", s->R, s->P,
                s->n_feat, s->n_pc, s->n_mlp);
  const double r3 = (double)s->R * s->R * s->R, p3 = (double)s->P * s->P * s->P;
  if (r3 * s->n_feat >= 2147483648.0 || p3 * s->n_pc >= 2147483648.0)
    return fail(PSDF_EINVAL, "grid too large for 32-bit element indices");
  if (s->step < 1) return fail(PSDF_EINVAL, "step must be >= 1 (got %lld)", (long long)s->step);
  if (!(s->beta1 >= 0.f && s->beta1 < 1.f && s->beta2 >= 0.f && s->beta2 < 1.f && s->eps >= 0.f))
    return fail(PSDF_EINVAL, "Adam hyper-parameters out of range");
  const void* req[] = {s->sdf_in, s->sdf_out, s->feat_in, s->feat_out, s->probes_in, s->probes_out,
                       s->g_sdf, s->g_feat, s->g_probes, s->m_sdf, s->v_sdf, s->m_feat, s->v_feat,
                       s->m_probes, s->v_probes};
  for (const void* p : req) {
    if (!p) return fail(PSDF_EINVAL, "a required step buffer is NULL");
    if (!aligned(p, 16)) return fail(PSDF_EALIGN, "step buffers must be 16-byte aligned");
  }
  if (s->n_mlp > 0 && (!s->mlp || !s->g_mlp || !s->m_mlp || !s->v_mlp))
    return fail(PSDF_EINVAL, "MLP step buffers are NULL");
  if (s->n_mlp > 0 && (!aligned(s->mlp, 4) || !aligned(s->g_mlp, 4) || !aligned(s->m_mlp, 4) ||
                       !aligned(s->v_mlp, 4)))
    return fail(PSDF_EALIGN, "MLP step buffers misaligned");
  const size_t bs = (size_t)r3 * 4, bf = (size_t)r3 * s->n_feat * 4, bp = (size_t)p3 * s->n_pc * 4;
  if (overlap(s->sdf_in, bs, s->sdf_out, bs) || overlap(s->feat_in, bf, s->feat_out, bf) ||
      overlap(s->probes_in, bp, s->probes_out, bp))
    return fail(PSDF_EINVAL, "grid step is out of place: *_in and *_out must not overlap");
  const void* halves[] = {s->sdf_half_out, s->feat_half_out, s->probes_half_out};
  for (const void* p : halves)
    if (p && !aligned(p, 8)) return fail(PSDF_EALIGN, "FP16 copies must be 8-byte aligned");
  if (s->losses && !aligned(s->losses, 4)) return fail(PSDF_EALIGN, "losses misaligned");
  if (s->sdf_bounds_out && !aligned(s->sdf_bounds_out, 8))
    return fail(PSDF_EALIGN, "sdf_bounds_out must be 8-byte aligned");
  const bool ext = s->sdf_reg_flags != 0 || s->lambda_sdf != 0.f || s->lambda_normal != 0.f;
  const bool smooth = (s->sdf_reg_flags & PSDF_STEP_SMOOTH) != 0;
  if (ext) {
    if (s->sdf_reg_flags & ~(PSDF_STEP_SMOOTH | PSDF_STEP_REG_WEIGHT))
      return fail(PSDF_EINVAL, "unknown sdf_reg_flags 0x%x", s->sdf_reg_flags);
    if (!std::isfinite(s->lambda_sdf) || !std::isfinite(s->lambda_normal))
      return fail(PSDF_EINVAL, "lambda_sdf / lambda_normal must be finite");
    if (!s->work || s->work_bytes < psdf_step_work_bytes(s->R))
      return fail(PSDF_EINVAL, "the Sec. 3.3 regularisers need a work buffer of %lld bytes",
                  (long long)psdf_step_work_bytes(s->R));
    if (!aligned(s->work, 16)) return fail(PSDF_EALIGN, "work must be 16-byte aligned");
    if (smooth) {
      if (!(s->smooth_sigma > 0.f) || !std::isfinite(s->smooth_sigma))
        return fail(PSDF_EINVAL, "smooth_sigma must be finite > 0");
      if (!s->s_in || !s->s_out) return fail(PSDF_EINVAL, "PSDF_STEP_SMOOTH needs s_in and s_out");
      if (!aligned(s->s_in, 16) || !aligned(s->s_out, 16))
        return fail(PSDF_EALIGN, "s_in / s_out must be 16-byte aligned");
      if (overlap(s->s_out, bs, s->sdf_out, bs) || overlap(s->s_out, bs, s->sdf_in, bs) ||
          overlap(s->s_out, bs, s->s_in, bs))
        return fail(PSDF_EINVAL, "s_out must not overlap sdf_in, sdf_out or s_in");
    } else if (s->lambda_sdf != 0.f) {
      return fail(PSDF_EINVAL, "lambda_sdf needs PSDF_STEP_SMOOTH (without it s = shat)");
    }
    if (s->losses_ext && !aligned(s->losses_ext, 4))
      return fail(PSDF_EALIGN, "losses_ext misaligned");
  }

  psdf::StepArgs a{};
  a.R = s->R;
  a.P = s->P;
  a.n_feat = s->n_feat;
  a.n_pc = s->n_pc;
  a.n_mlp = s->n_mlp;
  a.h = (float)(2.0 / (s->R - 1));
  a.lr_sdf = s->lr_sdf;
  a.lr_feat = s->lr_feat;
  a.lr_probe = s->lr_probe;
  a.lr_mlp = s->lr_mlp;
  a.beta1 = s->beta1;
  a.beta2 = s->beta2;
  a.eps = s->eps;
  a.bc1 = (float)(1.0 - std::pow((double)s->beta1, (double)s->step));
  a.bc2 = (float)(1.0 - std::pow((double)s->beta2, (double)s->step));
  a.lambda_eik = s->lambda_eik;
  a.lambda_tv_feat = s->lambda_tv_feat;
  a.lambda_tv_probe = s->lambda_tv_probe;
  a.sdf_in = s->sdf_in;
  a.sdf_out = s->sdf_out;
  a.feat_in = s->feat_in;
  a.feat_out = s->feat_out;
  a.probes_in = s->probes_in;
  a.probes_out = s->probes_out;
  a.mlp = s->mlp;
  a.g_sdf = s->g_sdf;
  a.g_feat = s->g_feat;
  a.g_probes = s->g_probes;
  a.g_mlp = s->g_mlp;
  a.m_sdf = s->m_sdf;
  a.v_sdf = s->v_sdf;
  a.m_feat = s->m_feat;
  a.v_feat = s->v_feat;
  a.m_probes = s->m_probes;
  a.v_probes = s->v_probes;
  a.m_mlp = s->m_mlp;
  a.v_mlp = s->v_mlp;
  a.sdf_half = s->sdf_half_out;
  a.feat_half = s->feat_half_out;
  a.probes_half = s->probes_half_out;
  a.losses = s->losses;
  a.sdf_bounds = s->sdf_bounds_out;
  if (ext) {
    a.ext = 1;
    a.losses_ext = s->losses_ext;
    psdf::SdfRegArgs& r = a.reg;
    r.smooth = smooth ? 1 : 0;
    r.weighted = (s->sdf_reg_flags & PSDF_STEP_REG_WEIGHT) ? 1 : 0;
    const double R = s->R;
    r.lam_sdf = (float)(s->lambda_sdf / (R * R * R));
    r.lam_eik = (float)(s->lambda_eik / ((R - 2) * (R - 2) * (R - 2)));
    r.lam_nrm = s->R > 3 ? (float)(s->lambda_normal / (3.0 * (R - 2) * (R - 2) * (R - 3))) : 0.f;
    r.taps = smooth_taps(smooth ? s->smooth_sigma : 1.f);
    r.s_in = s->s_in;
    r.s_out = s->s_out;
    r.work = s->work;
  }
  return hip_status(psdf::launch_grid_step(a, static_cast<hipStream_t>(stream)),
                    "grid_step launch");
}

int psdf_sdf_bounds(int32_t R, int32_t sdf_dtype, const void* sdf, float* bounds, void* stream) {
  if (R < 2 || R > 1024) return fail(PSDF_EINVAL, "R=%d outside [2, 1024]", R);
  if (sdf_dtype != PSDF_F32 && sdf_dtype != PSDF_F16)
    return fail(PSDF_EUNSUPPORTED, "sdf_dtype %d", sdf_dtype);
  if (!sdf || !bounds) return fail(PSDF_EINVAL, "sdf/bounds is NULL");
  if (!aligned(sdf, dt_size(sdf_dtype)) || !aligned(bounds, 8))
    return fail(PSDF_EALIGN, "sdf/bounds misaligned");
  return hip_status(psdf::launch_sdf_bounds(sdf, R, sdf_dtype, bounds,
                                            static_cast<hipStream_t>(stream)),
                    "sdf_bounds launch");
}

int psdf_voxel_list(int32_t R, int32_t sdf_dtype, const void* sdf, float band, int32_t* list,
                    int64_t capacity, int32_t* count, void* stream) {
  if (R < 2 || R > 1024) return fail(PSDF_EINVAL, "R=%d outside [2, 1024]", R);
  if (sdf_dtype != PSDF_F32 && sdf_dtype != PSDF_F16)
    return fail(PSDF_EUNSUPPORTED, "sdf_dtype %d", sdf_dtype);
  if (!std::isfinite(band)) return fail(PSDF_EINVAL, "band must be finite");
  if (!sdf || !count || (capacity > 0 && !list)) return fail(PSDF_EINVAL, "NULL argument");
  if (capacity < 0 || capacity > (int64_t)R * R * R)
    return fail(PSDF_EINVAL, "capacity outside [0, R^3]");
  if (!aligned(sdf, sdf_dtype == PSDF_F32 ? 4 : 2) || !aligned(count, 4) ||
      (list && !aligned(list, 4)))
    return fail(PSDF_EALIGN, "sdf / list / count misaligned");
  return hip_status(psdf::launch_voxel_list(R, sdf_dtype, sdf, band, list, capacity, count,
                                            static_cast<hipStream_t>(stream)),
                    "voxel_list launch");
}

static int check_colour(const void* colour, int32_t colour_dtype) {
  if (colour_dtype != PSDF_F32 && colour_dtype != PSDF_F16)
    return fail(PSDF_EUNSUPPORTED, "colour_dtype %d", colour_dtype);
  if (!colour) return fail(PSDF_EINVAL, "colour is NULL");
  if (!aligned(colour, colour_dtype == PSDF_F32 ? 16 : 8))
    return fail(PSDF_EALIGN, "colour must be %d-byte aligned", colour_dtype == PSDF_F32 ? 16 : 8);
  return PSDF_OK;
}

static psdf::RealtimeArgs realtime_args(const psdf_field* f, const float* cam) {
  psdf::RealtimeArgs a{};
  a.R = f->R;
  a.P = f->P;
  a.sdf = f->sdf;
  a.feat = f->feat;
  a.probes = f->probes;
  a.mlp = f->mlp;
  a.bounds = f->sdf_bounds;
  a.cam = cam;
  return a;
}

int psdf_voxel_shade(const psdf_field* field, int32_t flags, const float* cam, const int32_t* list,
                     const int32_t* count, int64_t capacity, void* colour, int32_t colour_dtype,
                     void* stream) {
  int rc;
  if ((rc = check_field(field))) return rc;
  if (flags & ~7) return fail(PSDF_EINVAL, "unknown flags 0x%x (ablation flags only)", flags);
  if (field->mlp_hidden != 16 || field->mlp_layers != 1 || field->tile_T > 0)
    return fail(PSDF_EUNSUPPORTED, "voxel shading takes the one-layer MLP of 16 and dense features");
  if ((rc = check_colour(colour, colour_dtype))) return rc;
  if ((rc = check_f32(cam, "cam"))) return rc;
  if (!count || capacity < 0 || capacity > (int64_t)field->R * field->R * field->R ||
      (capacity > 0 && !list))
    return fail(PSDF_EINVAL, "list / count / capacity out of range");
  if (capacity == 0) return ok();
  psdf::RealtimeArgs a = realtime_args(field, cam);
  a.flags = flags;
  a.list = list;
  a.count = count;
  a.cap = capacity;
  a.colour = colour;
  return hip_status(psdf::launch_voxel_shade(a, field->sdf_dtype, field->feat_dtype,
                                             field->mlp_dtype, field->sh_coeffs, colour_dtype,
                                             static_cast<hipStream_t>(stream)),
                    "voxel_shade launch");
}

int psdf_volume_render(const psdf_field* field, const psdf_render_opts* opts, const void* colour,
                       int32_t colour_dtype, const float* cam, int32_t W, int32_t H, float* out,
                       void* stream) {
  int rc;
  if ((rc = check_field(field)) || (rc = check_opts(opts))) return rc;
  if (opts->flags) return fail(PSDF_EINVAL, "volume rendering takes no render flags");
  if ((rc = check_colour(colour, colour_dtype))) return rc;
  if (W < 0 || H < 0 || W > 65535 * 16 || H > 65535 * 16)
    return fail(PSDF_EINVAL, "bad image size W=%d H=%d", W, H);
  if ((int64_t)W * H == 0) return ok();
  if ((rc = check_f32(cam, "cam")) || (rc = check_f32(out, "out"))) return rc;
  psdf::RealtimeArgs a = realtime_args(field, cam);
  a.colour = const_cast<void*>(colour);
  a.N = opts->n_samples;
  a.tau = opts->tau;
  a.skip_thr = opts->skip_voxels > 0.f ? (float)(opts->skip_voxels * (2.0 / (field->R - 1))) : 0.f;
  a.W = W;
  a.H = H;
  a.out = out;
  return hip_status(psdf::launch_volume_render(a, field->sdf_dtype, colour_dtype,
                                               static_cast<hipStream_t>(stream)),
                    "volume_render launch");
}

int psdf_render_sphere_trace(const psdf_field* field, const psdf_trace_opts* opts, int32_t V,
                             const float* cams, int32_t W, int32_t H, float* out, void* stream) {
  int rc;
  if ((rc = check_field(field))) return rc;
  if (!opts) return fail(PSDF_EINVAL, "opts is NULL");
  if (opts->struct_size != sizeof(psdf_trace_opts))
    return fail(PSDF_EINVAL, "trace opts.struct_size %u != %zu", opts->struct_size,
                sizeof(psdf_trace_opts));
  if (!(opts->eps > 0.f) || !std::isfinite(opts->eps) || opts->max_steps < 1 ||
      opts->max_steps > 100000 || (opts->flags & ~7))
    return fail(PSDF_EINVAL, "trace opts out of range");
  if (V < 0 || W < 0 || H < 0 || V > 65535 || W > 65535 * 16 || H > 65535 * 16)
    return fail(PSDF_EINVAL, "bad image size V=%d W=%d H=%d", V, W, H);
  if (field->mlp_hidden != 16 || field->mlp_layers != 1 || field->tile_T > 0)
    return fail(PSDF_EUNSUPPORTED,
                "sphere tracing shades with the one-layer MLP of 16 and dense features");
  if ((int64_t)V * W * H == 0) return ok();
  if ((rc = check_f32(cams, "cams")) || (rc = check_f32(out, "out"))) return rc;
  psdf::TraceArgs a{};
  a.R = field->R;
  a.P = field->P;
  a.h = (float)(2.0 / (field->R - 1));
  a.inv_h = (float)((field->R - 1) / 2.0);
  a.inv_hp = (float)((field->P - 1) / 2.0);
  a.sdf = field->sdf;
  a.feat = field->feat;
  a.probes = field->probes;
  a.mlp = field->mlp;
  a.eps = opts->eps;
  a.max_steps = opts->max_steps;
  a.flags = opts->flags;
  a.V = V;
  a.W = W;
  a.H = H;
  a.cams = cams;
  a.out = out;
  return hip_status(psdf::launch_sphere_trace(a, field->sdf_dtype, field->feat_dtype,
                                              field->mlp_dtype, field->sh_coeffs,
                                              static_cast<hipStream_t>(stream)),
                    "sphere_trace launch");
}

}  // extern "C"
