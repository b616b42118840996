// Pair weight m (r2)^(-3/2) for the gravity kernels whose force loops are
// bound by FP64 issue (lanes that each hold one body at one or all stages).
#pragma once

#include "device_common.h"

namespace irk {

// m r2^(-3/2) for r2 > 0 in fewer operations than m * rinv3(r2): the hardware
// reciprocal square root y0 refined by one Halley step,
// y = y0 (1 + e/2 + 3 e^2/8) with e = 1 - r2 y0^2 (cubic convergence: within
// 1 ulp of r2^(-1/2), like two Newton steps, in five operations instead of
// seven), then cubed.  The few-body and stage-parallel kernels keep rinv3:
// the few-body kernel's dependent chains ran faster with it, and the
// stage-parallel kernel must match the few-body kernel bit for bit for the
// systems it takes over from it.
__device__ __forceinline__ double mass_rinv3_halley(double r2, double m) {
  const double y0 = __builtin_amdgcn_rsq(r2);
  const double e = fma(-r2, y0 * y0, 1.0);
  const double y = fma(y0, e * fma(e, 0.375, 0.5), y0);
  return m * ((y * y) * y);
}

}  // namespace irk
