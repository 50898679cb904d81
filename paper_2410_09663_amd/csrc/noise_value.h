// The virtual system's noise for one (row, member, column): row `a` of (L z^i)[:, x] with
// z^i the standard normals of member i, where L is the Cholesky factor of the noise
// covariance (Q for W, R for V; Eqs. (4)-(5)) or its diagonal.  Shared by the noise
// kernels and the rollout kernels that assemble and observe the forecast.
#pragma once

#include "oic_internal.h"

namespace oic {

__device__ __forceinline__ float noise_value(const NoiseRef& nr, int a, int i, int x, int m) {
  const float* z = nr.Z + ((size_t)i * nr.rows) * m + x;
  if (nr.diag) return nr.diag[a] * z[(size_t)a * m];
  float acc = 0.f;
  const float* Lrow = nr.L + (size_t)a * nr.rows;
  for (int b = 0; b <= a; ++b) acc = fmaf(Lrow[b], z[(size_t)b * m], acc);
  return acc;
}

}  // namespace oic
