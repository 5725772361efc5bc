// Grid stencils shared by the level-set stage and the band compaction.
#pragma once

#include <hip/hip_runtime.h>

namespace pb {

__device__ __forceinline__ double stencil_sq(double a) { return a * a; }

// ε of the WENO5 weights α_k = d_k/(ε + β_k)², with β_k in units of the divided differences.
constexpr double kWenoEps = 1e-6;

// Fifth-order WENO one-sided derivative from five consecutive differences. The weights
// α_k = d_k/(ε + β_k)² are normalized as α_k/Σα = d_k q_l q_m / Σ d_k q_l q_m with
// q = (ε + β)², the same quotient with one division instead of four; the constant
// coefficients of the three candidate stencils are multiplications. Rounded as written
// (no FMA contraction), like the stencil kernels that call it.
__device__ __forceinline__ double weno5(double v1, double v2, double v3, double v4, double v5) {
#pragma clang fp contract(off)
  const double e = kWenoEps;
  double s1 = 13.0 / 12.0 * stencil_sq(v1 - 2.0 * v2 + v3) + 0.25 * stencil_sq(v1 - 4.0 * v2 + 3.0 * v3);
  double s2 = 13.0 / 12.0 * stencil_sq(v2 - 2.0 * v3 + v4) + 0.25 * stencil_sq(v2 - v4);
  double s3 = 13.0 / 12.0 * stencil_sq(v3 - 2.0 * v4 + v5) + 0.25 * stencil_sq(3.0 * v3 - 4.0 * v4 + v5);
  double q1 = stencil_sq(s1 + e), q2 = stencil_sq(s2 + e), q3 = stencil_sq(s3 + e);
  double w1 = 0.1 * (q2 * q3), w2 = 0.6 * (q1 * q3), w3 = 0.3 * (q1 * q2);
  double p1 = v1 * (1.0 / 3.0) - v2 * (7.0 / 6.0) + v3 * (11.0 / 6.0);
  double p2 = -v2 * (1.0 / 6.0) + v3 * (5.0 / 6.0) + v4 * (1.0 / 3.0);
  double p3 = v3 * (1.0 / 3.0) + v4 * (5.0 / 6.0) - v5 * (1.0 / 6.0);
  return (w1 * p1 + w2 * p2 + w3 * p3) / (w1 + w2 + w3);
}

}  // namespace pb
