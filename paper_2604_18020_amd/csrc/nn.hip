// Learned preconditioner (U-Net) state; filled in by the network kernels.
#include "common.h"

extern "C" void tosimp_nn_release(tosimp_ctx* ctx) { (void)ctx; }

extern "C" int tosimp_nn_fcg_solve(tosimp_ctx* ctx, const float*, const float*, float*, double,
                                   int, int, int, int*, int*, int*) {
  return tosimp_fail(ctx, TOSIMP_ESTATE, "no learned preconditioner has been created");
}
