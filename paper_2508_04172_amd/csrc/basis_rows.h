// Interpolation basis rows at a point of the unit ball (Eq. rbfcoeff): the
// Gaussian kernel exp(-eps^2 |x - x_r|^2) for node rows r < N, the monomials
// p_{r-N}(x) for N <= r < N + M, and zero for the padding rows beyond.
#pragma once
#include <hip/hip_runtime.h>

namespace rbfl {

// Value of basis row `row` at x.  xn: the node's coordinates (row < N);
// poly[p]: the variable indices of monomial p, -1 = unused.
__device__ __forceinline__ double basis_row_fp64(int row, int N, int NM, const double x[4], const double *xn,
                                                 double eps2, const int (*poly)[3]) {
  if (row < N) {
    double d2 = 0.0;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const double t = x[d] - xn[d];
      d2 = fma(t, t, d2);
    }
    return exp(-eps2 * d2);
  }
  if (row < NM) {
    const int p = row - N;
    double v = 1.0;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int id = poly[p][s];
      if (id >= 0) v *= x[id];
    }
    return v;
  }
  return 0.0;
}

__device__ __forceinline__ float basis_row_fp32(int row, int N, int NM, const float x[4], const float *xn,
                                                float eps2, const int (*poly)[3]) {
  if (row < N) {
    float d2 = 0.0f;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const float t = x[d] - xn[d];
      d2 = fmaf(t, t, d2);
    }
    return __expf(-eps2 * d2);
  }
  if (row < NM) {
    const int p = row - N;
    float v = 1.0f;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int id = poly[p][s];
      if (id >= 0) v *= x[id];
    }
    return v;
  }
  return 0.0f;
}

}  // namespace rbfl
