// MFMA (BF16 / FP16) variant of the operator.
#include "common.h"

namespace tosimp {
hipError_t kv_mfma_launch(const tosimp_ctx*, int, int, const void*, const float*, float*,
                          SolverState*, bool) {
  return hipErrorNotSupported;
}
}  // namespace tosimp
