// Adjoint of K steps: not provided yet in this build.
#include "lbm_adjoint.h"

namespace lbm {

hipError_t adjoint_forward(Fields&, AdjointBuffers&, hipStream_t, int, int, int, double, double*) {
  return hipErrorNotSupported;
}
hipError_t adjoint_backward(Fields&, AdjointBuffers&, hipStream_t, int, int, int, double, const double*,
                            const double*, double*, double*, double*) {
  return hipErrorNotSupported;
}

}  // namespace lbm
