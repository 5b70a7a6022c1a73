// Wave-per-subcarrier LMMSE detector on the matrix cores (placeholder: not yet eligible).
#include "geom.h"

namespace ranphy {

bool mmse_mfma_eligible(const Geom&) { return false; }

hipError_t launch_mmse_mfma(const Geom&, const float2*, const float2*, int, const float*, float2*,
                            float*, hipStream_t) {
  return hipErrorInvalidValue;
}

}  // namespace ranphy
