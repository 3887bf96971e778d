// Reconstruction loss and its gradient (copa_loss_grad).
#include "copa_common.h"

namespace copa {
copa_status launch_loss_grad(copa_plan *, const float *, const float *, const float *,
                             const float *, float *, float *, float *, float *, hipStream_t) {
  set_error("copa_loss_grad is not built yet");
  return COPA_EUNSUPPORTED;
}
}  // namespace copa

using namespace copa;

extern "C" copa_status copa_loss_grad(copa_plan *p, const float *H, const float *V, const float *W,
                                      const float *Qt, float *dH, float *dV, float *dW, float *dS,
                                      double *loss, void *stream) {
  if (!p || !H || !V || !W || !Qt || !dH || !dV || !dW || !loss) {
    set_error("NULL argument");
    return COPA_EINVAL;
  }
  return launch_loss_grad(p, H, V, W, Qt, dH, dV, dW, dS, (hipStream_t)stream);
}
