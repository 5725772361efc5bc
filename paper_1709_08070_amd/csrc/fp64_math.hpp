// FP64 elementary functions of the pair and energy kernels, written from their
// mathematical definitions (no library call, no branch).
#pragma once

#include <hip/hip_runtime.h>

namespace pb {

// e^{−z} for z ≥ 0 in FP64 without branches (Cody–Waite reduction): k = rint(−z·log2 e),
// t = −z − k·ln2 with ln 2 = L_hi + L_lo (L_hi its nearest double, L_lo the remainder; the
// products are exact inside the FMAs), |t| ≤ ln2/2, e^t by the degree-11 interpolant of e^t at
// the 12 Chebyshev nodes of [−ln2/2, ln2/2] (near-minimax; relative error 1.7e-17 before
// rounding, against 5.2e-18 for the Taylor series to degree 13, two terms longer; the
// coefficients come from exp_coeffs.py beside this file), then scaled by 2^k. For 0 ≤ z ≤ 1e9
// (k fits an int; beyond z ≈ 745 the scaling underflows to 0, as e^{−z} does in FP64): the
// callers' distances stay far below that (the pair kernels' padding records sit 1e6 away).
__device__ __forceinline__ double exp_neg_f64(double z) {
  const double k = __builtin_rint(-z * 1.4426950408889634);
  const double t = fma(-k, 2.3190468138462996e-17, fma(-k, 0.6931471805599453, -z));
  double p = 2.5110037605963777e-08;
  p = fma(p, t, 2.763263963904103e-07);
  p = fma(p, t, 2.755724091857897e-06);
  p = fma(p, t, 2.4801485482328494e-05);
  p = fma(p, t, 0.00019841269890047113);
  p = fma(p, t, 0.0013888888952314775);
  p = fma(p, t, 0.008333333333319601);
  p = fma(p, t, 0.0416666666664881);
  p = fma(p, t, 0.1666666666666668);
  p = fma(p, t, 0.5000000000000019);
  p = fma(p, t, 1.0);
  p = fma(p, t, 1.0);
  return ldexp(p, (int)k);
}

// 1/√x for x > 0: the hardware estimate y (about 2^-24 relative) and one third-order step of
// the series (1 − e)^{−1/2} = 1 + e/2 + 3e²/8 + … with e = 1 − xy², y ← y + ye(½ + 3e/8): the
// truncation leaves about 2.5δ³ for an estimate off by δ, far below an ulp, so the result is
// within an ulp of the correctly rounded value, like two Newton steps, in two fewer
// instructions (checked on the CPU against long-double 1/√x with |δ| up to 2^-20).
__device__ __forceinline__ double rsqrt_f64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-(x * y), y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

}  // namespace pb
