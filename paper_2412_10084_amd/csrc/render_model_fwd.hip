// Instances of the paper-model render kernels: forward kernels of both MLP shapes.
#include "model_kernels.h"

namespace psdf {
PSDF_MODEL_INSTANCE(16, 1, false, MLP_F32)
PSDF_MODEL_INSTANCE(16, 1, false, MLP_F16)
PSDF_MODEL_INSTANCE(16, 1, false, MLP_BF16)
PSDF_MODEL_INSTANCE(32, 2, false, MLP_F32)
PSDF_MODEL_INSTANCE(32, 2, false, MLP_F16)
PSDF_MODEL_INSTANCE(32, 2, false, MLP_BF16)
}  // namespace psdf
