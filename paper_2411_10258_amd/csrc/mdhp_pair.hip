// Per-pair decay evaluation (placeholder until the per-pair scan lands).
#include "mdhp_internal.h"

namespace mdhp {

hipError_t pair_eval(const Events&, int, const float*, const float*, const float*, double*,
                     float*, float*, float*, int*, hipStream_t, bool) {
  return hipErrorNotSupported;
}

hipError_t pair_fit(const Events&, int, const FitParams&, float*, float*, float*, double*, int*,
                    int*, int*, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace mdhp
