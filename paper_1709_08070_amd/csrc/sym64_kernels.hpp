// Symmetric FP64 operator: every unordered pair {i, j} evaluated once for both directions,
// regularization included (the FP64 path has no near/far split).
//
// With d = x_i − x_j, r = |d|, z = κr, E = e^{−z}, a = E(1 + z), b = E(3 + 3z + z²), the four
// kernels (times 4π) of target i and source j are
//   K11(i,j) = (d·n_j)(1 − θ1 a)/r³,  K12 = (1 − E)/r,
//   K21 = (n_i·n_j)(1 − a)/r³ − (d·n_i)(d·n_j)(3 − b)/r⁵,  K22(i,j) = −(d·n_i)(1 − θ2 a)/r³,
// so K12 and K21 are symmetric and, with d → −d, K11(j,i) = −(d·n_i)(1 − θ1 a)/r³ and
// K22(j,i) = (d·n_j)(1 − θ2 a)/r³. r, E, a, b (one reciprocal square root with two Newton
// steps and one exp) are shared. The regularization predicate of the section
// "Regularization of the singular kernels" measures the tangential distance in the target's
// tangent plane (t² = r² − (d·n_target)²), so each direction takes its own decision; a
// regularized direction gets K11 = K21 = K22 = 0, K12 = K̄12. A pair at r = 0 is regularized in
// both directions under every metric, so the shared radial terms are only used for r > 0.
//
// Work items and partial-sum ownership are those of the symmetric FP32 kernel (chunk pairs,
// one owner per slot, fixed-order FP64 accumulation). The reverse sums travel with their
// source across the lanes of a wave (ds_bpermute on the two halves of each double).
#pragma once

#include "sym_kernels.hpp"

namespace pb {

struct Sym64Shared {
  double2 s0[kSymSub], s1[kSymSub], s2[kSymSub], s3[kSymSub];  // (x, y), (z, nx), (ny, nz), (wψ, wψn)
  double racc[kSymWaves][2][kSymSub];
};

// Regularization decision for the direction whose target has tangential coordinate dn, for
// a metric fixed at compile time.
template <int kMetric>
__device__ __forceinline__ bool reg_f64(double r2, double dn, const KParams& kp) {
  const double t2 = __dadd_rn(r2, -__dmul_rn(dn, dn));
  if (kMetric == PB_REG_EUCLIDEAN) return r2 < kp.tau2;
  if (kMetric == PB_REG_TANGENT) return t2 < kp.tau2;
  return t2 < kp.tau2 && r2 < kp.four_tau2;
}

// e^{−z} for z ≥ 0 in FP64 without branches (Cody–Waite reduction): k = rint(−z·log2 e),
// t = −z − k·ln2 with ln 2 = L_hi + L_lo (L_hi its nearest double, L_lo the remainder; the
// products are exact inside the FMAs), |t| ≤ ln2/2, e^t by its Taylor series to degree 13
// (truncation error below 1e-17 relative), then scaled by 2^k. z is clamped to 745, beyond which
// e^{−z} is 0 in FP64.
__device__ __forceinline__ double exp_neg_f64(double z) {
  z = fmin(z, 745.0);
  const double k = __builtin_rint(-z * 1.4426950408889634);
  const double t = fma(-k, 2.3190468138462996e-17, fma(-k, 0.6931471805599453, -z));
  double p = 1.0 / 6227020800.0;  // 1/13!
  p = fma(p, t, 1.0 / 479001600.0);
  p = fma(p, t, 1.0 / 39916800.0);
  p = fma(p, t, 1.0 / 3628800.0);
  p = fma(p, t, 1.0 / 362880.0);
  p = fma(p, t, 1.0 / 40320.0);
  p = fma(p, t, 1.0 / 5040.0);
  p = fma(p, t, 1.0 / 720.0);
  p = fma(p, t, 1.0 / 120.0);
  p = fma(p, t, 1.0 / 24.0);
  p = fma(p, t, 1.0 / 6.0);
  p = fma(p, t, 0.5);
  p = fma(p, t, 1.0);
  p = fma(p, t, 1.0);
  return ldexp(p, (int)k);
}

// Both directions of one pair. Target i: position xi, normal ni, weights (wψ_i, wψn_i); source j
// likewise. f1/f2 accumulate into i, g1/g2 into j.
template <int kMetric>
__device__ __forceinline__ void pair_sym_f64(double xi, double yi, double zi, double nxi, double nyi, double nzi,
                                             double wpi, double wni, const double2& s0, const double2& s1,
                                             const double2& s2, const double2& s3, const KParams& kp, double& f1,
                                             double& f2, double& g1, double& g2) {
  const double xj = s0.x, yj = s0.y, zj = s1.x, nxj = s1.y, nyj = s2.x, nzj = s2.y, wpj = s3.x, wnj = s3.y;
  const double dx = xi - xj, dy = yi - yj, dz = zi - zj;
  const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
  const double dnx = __dadd_rn(__dadd_rn(__dmul_rn(dx, nxi), __dmul_rn(dy, nyi)), __dmul_rn(dz, nzi));
  const double dny = __dadd_rn(__dadd_rn(__dmul_rn(dx, nxj), __dmul_rn(dy, nyj)), __dmul_rn(dz, nzj));
  const bool rf = reg_f64<kMetric>(r2, dnx, kp), rr = reg_f64<kMetric>(r2, dny, kp);
  // Branch-free: the radial terms are formed for every pair and each direction selects its
  // regularized or regular value. Only a pair regularized both ways can have r = 0; it takes
  // r² = 1 here, whose (finite) radial terms are discarded.
  const double r2s = (rf && rr) ? 1.0 : r2;
  const double nn = nxi * nxj + nyi * nyj + nzi * nzj;
  double rinv = __builtin_amdgcn_rsq(r2s);
  double e = fma(-r2s * rinv, rinv, 1.0);
  rinv = fma(0.5 * rinv, e, rinv);
  e = fma(-r2s * rinv, rinv, 1.0);
  rinv = fma(0.5 * rinv, e, rinv);
  const double r = r2s * rinv;
  const double r3 = rinv * rinv * rinv;
  const double r5 = r3 * rinv * rinv;
  const double z = kp.kappa * r;
  const double E = exp_neg_f64(z);
  const double a = E * (1.0 + z);
  const double b = E * (3.0 + 3.0 * z + z * z);
  const double k12 = (1.0 - E) * rinv;
  const double k21 = nn * (1.0 - a) * r3 - dnx * dny * (3.0 - b) * r5;
  const double f1r = dny * (1.0 - kp.th1 * a) * r3 * wpj - k12 * wnj;
  const double f2r = k21 * wpj + dnx * (1.0 - kp.th2 * a) * r3 * wnj;
  const double g1r = -dnx * (1.0 - kp.th1 * a) * r3 * wpi - k12 * wni;
  const double g2r = k21 * wpi - dny * (1.0 - kp.th2 * a) * r3 * wni;
  f1 += rf ? -kp.k12bar4pi * wnj : f1r;
  f2 += rf ? 0.0 : f2r;
  g1 += rr ? -kp.k12bar4pi * wni : g1r;
  g2 += rr ? 0.0 : g2r;
}

__device__ __forceinline__ double shfl_next(double v, int addr) {
  const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Targets [t0, t0 + 512) (full) against sources [s0, s0 + 512), s0 ≠ t0, both directions;
// adds into fwd (index i − t0) and rev (index j − s0). wpsi/wpsn: h³ωψ/4π, h³ωψn/4π.
template <int kMetric>
__device__ __forceinline__ void sym64_block(const BandDev& b, const double* __restrict__ wpsi,
                                            const double* __restrict__ wpsn, int n, int t0, int s0,
                                            const KParams& kp, Sym64Shared& sh, double* fwd1, double* fwd2,
                                            double* rev1, double* rev2, bool acc) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int q = tid; q < kSymSub; q += kBlock) {
    const int j = s0 + q;
    if (j < n) {
      sh.s0[q] = make_double2(b.px[j], b.py[j]);
      sh.s1[q] = make_double2(b.pz[j], b.nx[j]);
      sh.s2[q] = make_double2(b.ny[j], b.nz[j]);
      sh.s3[q] = make_double2(wpsi[j], wpsn[j]);
    } else {  // padding far away with zero weights: contributes exactly zero both ways
      sh.s0[q] = make_double2(1e30, 1e30);
      sh.s1[q] = make_double2(1e30, 0.0);
      sh.s2[q] = make_double2(0.0, 1.0);
      sh.s3[q] = make_double2(0.0, 0.0);
    }
  }
  const int ia = t0 + w * 128 + lane, ib = ia + 64;
  const double xa = b.px[ia], ya = b.py[ia], za = b.pz[ia], nxa = b.nx[ia], nya = b.ny[ia], nza = b.nz[ia];
  const double xb = b.px[ib], yb = b.py[ib], zb = b.pz[ib], nxb = b.nx[ib], nyb = b.ny[ib], nzb = b.nz[ib];
  const double wpa = wpsi[ia], wna = wpsn[ia], wpb = wpsi[ib], wnb = wpsn[ib];
  __syncthreads();
  double fa1 = 0.0, fa2 = 0.0, fb1 = 0.0, fb2 = 0.0;
  const int next = ((lane + 1) & 63) << 2;
  for (int g = 0; g < kSymSub; g += 64) {
    double ra1 = 0.0, ra2 = 0.0;  // at step s: the reverse sums of source g + ((lane + s) mod 64)
    for (int s = 0; s < 64; ++s) {
      const int q = g + ((lane + s) & 63);
      const double2 c0 = sh.s0[q], c1 = sh.s1[q], c2 = sh.s2[q], c3 = sh.s3[q];
      pair_sym_f64<kMetric>(xa, ya, za, nxa, nya, nza, wpa, wna, c0, c1, c2, c3, kp, fa1, fa2, ra1, ra2);
      pair_sym_f64<kMetric>(xb, yb, zb, nxb, nyb, nzb, wpb, wnb, c0, c1, c2, c3, kp, fb1, fb2, ra1, ra2);
      ra1 = shfl_next(ra1, next);
      ra2 = shfl_next(ra2, next);
    }
    sh.racc[w][0][g + lane] = ra1;
    sh.racc[w][1][g + lane] = ra2;
  }
  __syncthreads();
  fwd1[ia - t0] = fa1 + (acc ? fwd1[ia - t0] : 0.0);
  fwd2[ia - t0] = fa2 + (acc ? fwd2[ia - t0] : 0.0);
  fwd1[ib - t0] = fb1 + (acc ? fwd1[ib - t0] : 0.0);
  fwd2[ib - t0] = fb2 + (acc ? fwd2[ib - t0] : 0.0);
  for (int q = tid; q < kSymSub; q += kBlock) {
    if (s0 + q < n) {
      double x1 = 0.0, x2 = 0.0;
      for (int v = 0; v < kSymWaves; ++v) {
        x1 += sh.racc[v][0][q];
        x2 += sh.racc[v][1][q];
      }
      rev1[q] = x1 + (acc ? rev1[q] : 0.0);
      rev2[q] = x2 + (acc ? rev2[q] : 0.0);
    }
  }
  __syncthreads();
}

// Targets [t0, t0 + 512) against the sources of the same sub-block (self pair included), one
// direction with the per-pair kernel of the one-directional operator; adds into fwd.
__device__ __forceinline__ void diag64_block(const BandDev& b, const double* __restrict__ wpsi,
                                             const double* __restrict__ wpsn, int n, int t0, const KParams& kp,
                                             Sym64Shared& sh, double* fwd1, double* fwd2, bool acc) {
  const int tid = threadIdx.x;
  for (int q = tid; q < kSymSub; q += kBlock) {
    const int j = t0 + q;
    if (j < n) {
      sh.s0[q] = make_double2(b.px[j], b.py[j]);
      sh.s1[q] = make_double2(b.pz[j], b.nx[j]);
      sh.s2[q] = make_double2(b.ny[j], b.nz[j]);
      sh.s3[q] = make_double2(wpsi[j], wpsn[j]);
    }
  }
  __syncthreads();
  const int m = min(kSymSub, n - t0);
  for (int h = 0; h < 2; ++h) {
    const int i = t0 + tid + h * kBlock;
    if (i < n) {
      const double xi = b.px[i], yi = b.py[i], zi = b.pz[i], nxi = b.nx[i], nyi = b.ny[i], nzi = b.nz[i];
      double s1 = 0.0, s2 = 0.0;
      for (int q = 0; q < m; ++q) {
        const double2 c0 = sh.s0[q], c1 = sh.s1[q], c2 = sh.s2[q], c3 = sh.s3[q];
        pair_f64(xi, yi, zi, nxi, nyi, nzi, c0.x, c0.y, c1.x, c1.y, c2.x, c2.y, c3.x, c3.y, kp, 0.0, s1, s2);
      }
      fwd1[i - t0] = s1 + (acc ? fwd1[i - t0] : 0.0);
      fwd2[i - t0] = s2 + (acc ? fwd2[i - t0] : 0.0);
    }
  }
  __syncthreads();
}

// One work item (Ic, Jc), Ic ≤ Jc; partial: the band's chunked partial sums.
__device__ __forceinline__ void sym64_item(const BandDev& b, const double* __restrict__ wpsi,
                                           const double* __restrict__ wpsn, int n, int Ic, int Jc, int nsub,
                                           const KParams& kp, double* __restrict__ partial, Sym64Shared& sh) {
  const int C = nsub * kSymSub;
  const int i0 = Ic * C, i1 = min(n, i0 + C), j0 = Jc * C, j1 = min(n, j0 + C);
  double* rowF = partial + (int64_t)Jc * 2 * n;
  double* rowR = partial + (int64_t)Ic * 2 * n;
  const bool acc = nsub > 1;  // one sub-block per chunk: every owned slot is written once
  if (acc) {
    for (int e = threadIdx.x; e < i1 - i0; e += kBlock) {
      rowF[i0 + e] = 0.0;
      rowF[n + i0 + e] = 0.0;
    }
    if (Ic != Jc)
      for (int e = threadIdx.x; e < j1 - j0; e += kBlock) {
        rowR[j0 + e] = 0.0;
        rowR[n + j0 + e] = 0.0;
      }
    __syncthreads();
  }
  for (int T = i0; T < i1; T += kSymSub)
    for (int S = (Ic == Jc ? T : j0); S < j1; S += kSymSub) {
      if (S == T)
        diag64_block(b, wpsi, wpsn, n, T, kp, sh, rowF + T, rowF + n + T, acc);
      else if (kp.metric == PB_REG_EUCLIDEAN)
        sym64_block<PB_REG_EUCLIDEAN>(b, wpsi, wpsn, n, T, S, kp, sh, rowF + T, rowF + n + T, rowR + S, rowR + n + S,
                                      acc);
      else if (kp.metric == PB_REG_TANGENT)
        sym64_block<PB_REG_TANGENT>(b, wpsi, wpsn, n, T, S, kp, sh, rowF + T, rowF + n + T, rowR + S, rowR + n + S,
                                    acc);
      else
        sym64_block<PB_REG_TANGENT_GUARDED>(b, wpsi, wpsn, n, T, S, kp, sh, rowF + T, rowF + n + T, rowR + S,
                                            rowR + n + S, acc);
    }
}

// Symmetric FP64 operator of one band: one block per work item.
static __global__ void __attribute__((unused)) __launch_bounds__(kBlock)
    k_p2p_f64_sym(BandDev b, const double* __restrict__ wpsi, const double* __restrict__ wpsn, int n, int nsub,
                  const int2* __restrict__ items, int n_items, KParams kp, double* __restrict__ partial,
                  const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ Sym64Shared sh;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int2 w = items[it];
    sym64_item(b, wpsi, wpsn, n, w.x, w.y, nsub, kp, partial, sh);
  }
}

}  // namespace pb
