// ecpic_nn.hip -- learned initial guess of the Picard iteration.
#include "ecpic_internal.h"

namespace ecpic {
ecpic_status nn_guess(Ctx& c, bool* used) {
  (void)c;
  *used = false;
  return ECPIC_OK;
}
}  // namespace ecpic

using namespace ecpic;

extern "C" {
int64_t ecpic_nn_param_count(void) { return 0; }
ecpic_status ecpic_nn_set_weights(ecpic_ctx*, const uint16_t*, const float*) {
  return ECPIC_ENOTIMPL;
}
ecpic_status ecpic_nn_forward(ecpic_ctx*, const uint16_t*, const uint16_t*, float*, int32_t) {
  return ECPIC_ENOTIMPL;
}
ecpic_status ecpic_nn_grad(ecpic_ctx*, const uint16_t*, const uint16_t*, const float*, int32_t,
                           float*, float*) {
  return ECPIC_ENOTIMPL;
}
ecpic_status ecpic_nn_adam(ecpic_ctx*, float*, float*, float*, const float*, uint16_t*, float,
                           int32_t) {
  return ECPIC_ENOTIMPL;
}
}
