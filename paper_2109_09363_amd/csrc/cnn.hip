// Multi-scale CNN initial guess (placeholder until the MFMA kernels land).
#include "internal.h"
namespace hyp {
hipError_t run_cnn(const NetShape&, const WsLayout&, int, int, double, const float*, const Ws&,
                   hipStream_t) {
  return hipErrorNotSupported;
}
}  // namespace hyp
