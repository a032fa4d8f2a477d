// Render step of the paper's own colour model: host dispatch onto the kernel
// instances of model_kernels.h (compiled in the render_model_*.hip units).
#include "model_kernels.h"
#include "probesdf.h"

namespace psdf {

static_assert(MODEL_EMAX + 1 == PSDF_MODEL_MAX_SAMPLES, "the ABI states the sample limit");
static_assert(FLAG_SH_REFLECT == PSDF_FLAG_SH_REFLECT && FLAG_FRESNEL_PAPER == PSDF_FLAG_FRESNEL_PAPER,
              "flag values of the ABI");

template <int H, int L, bool BWD, int M>
hipError_t launch_model_hlm(const RenderArgs& a, int feat_dt, int n_sh, dim3 grid, int64_t per,
                            hipStream_t s);

hipError_t launch_render_model(const RenderArgs& a, bool backward, int sdf_dt, int feat_dt,
                               int mlp_dt, int n_sh, int hidden, int layers, hipStream_t s) {
  if (a.B == 0) return hipSuccess;
  if (sdf_dt != 0 || a.N > MODEL_EMAX + 1) return hipErrorInvalidValue;
  // each wave takes a contiguous range of rays: one group of MODEL_GROUP rays in the
  // forward; the reverse mode flushes one MLP gradient atomic per parameter per
  // wave, so it runs fewer, longer waves
  const int64_t most = 2048;
  const int64_t waves = backward ? (a.B < most ? a.B : most) : (a.B + MODEL_GROUP - 1) / MODEL_GROUP;
  const int64_t per = (a.B + waves - 1) / waves;
  const dim3 grid((unsigned)((a.B + per - 1) / per));
#define PSDF_MODEL_M(H, L, BWD)                                                       \
  switch (mlp_dt) {                                                                   \
    case MLP_F32: return launch_model_hlm<H, L, BWD, MLP_F32>(a, feat_dt, n_sh, grid, per, s);   \
    case MLP_F16: return launch_model_hlm<H, L, BWD, MLP_F16>(a, feat_dt, n_sh, grid, per, s);   \
    case MLP_BF16: return launch_model_hlm<H, L, BWD, MLP_BF16>(a, feat_dt, n_sh, grid, per, s); \
    default: return hipErrorInvalidValue;                                             \
  }
  if (hidden == 16 && layers == 1) {
    if (backward) PSDF_MODEL_M(16, 1, true) else PSDF_MODEL_M(16, 1, false)
  } else if (hidden == 32 && layers == 2) {
    if (backward) PSDF_MODEL_M(32, 2, true) else PSDF_MODEL_M(32, 2, false)
  }
#undef PSDF_MODEL_M
  return hipErrorInvalidValue;
}

}  // namespace psdf
