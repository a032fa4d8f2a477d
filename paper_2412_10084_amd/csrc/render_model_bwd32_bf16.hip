// Instances of the paper-model render kernels: reverse-mode kernels of the two-layer MLP of 32, BF16 arithmetic.
#include "model_kernels.h"

namespace psdf {
PSDF_MODEL_INSTANCE(32, 2, true, MLP_BF16)
}  // namespace psdf
