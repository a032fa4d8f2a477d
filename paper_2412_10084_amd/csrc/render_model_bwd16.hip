// Instances of the paper-model render kernels: reverse-mode kernels of the one-layer MLP of 16.
#include "model_kernels.h"

namespace psdf {
PSDF_MODEL_INSTANCE(16, 1, true, MLP_F32)
PSDF_MODEL_INSTANCE(16, 1, true, MLP_F16)
PSDF_MODEL_INSTANCE(16, 1, true, MLP_BF16)
}  // namespace psdf
