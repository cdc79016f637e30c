// Hyperbolic tangent of the hidden layer, shared by the feature, evaluation
// and adjoint-evaluation kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace ddelm {

// tanh through expm1: with e = expm1(2|z|), tanh|z| = e / (e + 2).  expm1
// keeps full relative accuracy for small |z| (no cancellation in 1 - 2/(...)),
// and for |z| > 20 the exact value differs from 1 by less than 1e-17, below
// the double rounding step at 1.  A few ulps, like the library tanh; the
// evaluation kernel takes about half the time with it.
__device__ __forceinline__ double tanh_fast(double z) {
  const double a = fabs(z);
  if (a > 20.0) return copysign(1.0, z);
  const double e = expm1(2.0 * a);
  return copysign(e / (e + 2.0), z);
}

}  // namespace ddelm
