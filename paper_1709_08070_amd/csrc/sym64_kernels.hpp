// Symmetric FP64 operator: every unordered pair {i, j} evaluated once for both directions,
// regularization included (the FP64 path has no near/far split).
//
// With d = x_i − x_j, r = |d|, z = κr, E = e^{−z}, a = E(1 + z), b = E(3 + 3z + z²), the four
// kernels (times 4π) of target i and source j are
//   K11(i,j) = (d·n_j)(1 − θ1 a)/r³,  K12 = (1 − E)/r,
//   K21 = (n_i·n_j)(1 − a)/r³ − (d·n_i)(d·n_j)(3 − b)/r⁵,  K22(i,j) = −(d·n_i)(1 − θ2 a)/r³,
// so K12 and K21 are symmetric and, with d → −d, K11(j,i) = −(d·n_i)(1 − θ1 a)/r³ and
// K22(j,i) = (d·n_j)(1 − θ2 a)/r³. r, E, a, b (one reciprocal square root with a third-order
// correction and one exp) are shared. The regularization predicate of the section
// "Regularization of the singular kernels" measures the tangential distance in the target's
// tangent plane (t² = r² − (d·n_target)²), so each direction takes its own decision; a
// regularized direction gets K11 = K21 = K22 = 0, K12 = K̄12. A pair at r = 0 is regularized in
// both directions under every metric, so the shared radial terms are only used for r > 0.
//
// Far sub-block pairs. Under the guarded tangent metric no pair with r ≥ 2τ is regularized,
// under the Euclidean one none with r ≥ τ. Sub-block pairs whose exact FP64 bounding boxes
// (block reductions over the staged nodes) are farther apart than that radius, with a
// relative margin of 1e-9 on its square that covers the rounding of the box gap and of r²,
// skip the predicate: none of their pairs can take the regularized branch, so the geometry
// may use fused multiply-adds and the selects drop out. The literal tangent metric can
// regularize pairs at any distance and always runs the predicate.
//
// Work items and partial-sum ownership are those of the symmetric FP32 kernel (chunk pairs,
// one owner per slot, fixed-order FP64 accumulation; forward sums held in registers over a
// target sub-block's sources and stored once, reverse sums stored or added per sub-block
// pair). The reverse sums travel with their source across the lanes of a wave (ds_bpermute
// on the two halves of each double).
#pragma once

#include "fp64_math.hpp"
#include "sym_kernels.hpp"

namespace pb {

struct Sym64Shared {
  double2 s0[kSymSub], s1[kSymSub], s2[kSymSub], s3[kSymSub];  // (x, y), (z, nx), (ny, nz), (wψ, wψn)
  double racc[kSymWaves][2][64];  // one 64-source group's reverse sums per wave
  double box[kSymWaves][6];  // per-wave bounding boxes (lo xyz, hi xyz) of a block reduction
};

// Bounding box over the block: each thread passes the box of its own points (empty: +∞/−∞);
// every thread gets the block's. Every thread of the block calls it (it synchronizes).
__device__ __forceinline__ void block_box(double (&lo)[3], double (&hi)[3], Sym64Shared& sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1)
    for (int c = 0; c < 3; ++c) {
      lo[c] = fmin(lo[c], __shfl_xor(lo[c], off));
      hi[c] = fmax(hi[c], __shfl_xor(hi[c], off));
    }
  if (lane == 0)
    for (int c = 0; c < 3; ++c) {
      sh.box[w][c] = lo[c];
      sh.box[w][3 + c] = hi[c];
    }
  __syncthreads();
  for (int c = 0; c < 3; ++c) {
    lo[c] = sh.box[0][c];
    hi[c] = sh.box[0][3 + c];
    for (int v = 1; v < kSymWaves; ++v) {
      lo[c] = fmin(lo[c], sh.box[v][c]);
      hi[c] = fmax(hi[c], sh.box[v][3 + c]);
    }
  }
  __syncthreads();
}

// Squared gap between two boxes (0 if they overlap), FP64.
__device__ __forceinline__ double box_gap2_f64(const double (&alo)[3], const double (&ahi)[3],
                                               const double (&blo)[3], const double (&bhi)[3]) {
  double g2 = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double g = fmax(0.0, fmax(blo[c] - ahi[c], alo[c] - bhi[c]));
    g2 += g * g;
  }
  return g2;
}

// Regularization decision for the direction whose target has tangential coordinate dn, for
// a metric fixed at compile time.
template <int kMetric>
__device__ __forceinline__ bool reg_f64(double r2, double dn, const KParams& kp) {
  const double t2 = __dadd_rn(r2, -__dmul_rn(dn, dn));
  if (kMetric == PB_REG_EUCLIDEAN) return r2 < kp.tau2;
  if (kMetric == PB_REG_TANGENT) return t2 < kp.tau2;
  return t2 < kp.tau2 && r2 < kp.four_tau2;
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
  const double rinv = rsqrt_f64(r2s);
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

// Both directions of a pair that cannot be regularized (far sub-block pairs): the same
// kernels as pair_sym_f64's regular branch, the products free to fuse. k2 = κ².
__device__ __forceinline__ void pair_sym_f64_far(double xi, double yi, double zi, double nxi, double nyi, double nzi,
                                                 double wpi, double wni, const double2& s0, const double2& s1,
                                                 const double2& s2, const double2& s3, const KParams& kp, double k2,
                                                 double& f1, double& f2, double& g1, double& g2) {
  const double xj = s0.x, yj = s0.y, zj = s1.x, nxj = s1.y, nyj = s2.x, nzj = s2.y, wpj = s3.x, wnj = s3.y;
  const double dx = xi - xj, dy = yi - yj, dz = zi - zj;
  const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
  const double dnx = fma(dz, nzi, fma(dy, nyi, dx * nxi));
  const double dny = fma(dz, nzj, fma(dy, nyj, dx * nxj));
  const double nn = fma(nzi, nzj, fma(nyi, nyj, nxi * nxj));
  const double rinv = rsqrt_f64(r2);
  const double ri2 = rinv * rinv;
  const double r3 = ri2 * rinv;
  const double z = kp.kappa * (r2 * rinv);
  const double E = exp_neg_f64(z);
  const double a = fma(E, z, E);                    // E(1 + z)
  const double k12 = fma(-E, rinv, rinv);           // (1 − E)/r
  // with b = E(3 + 3z + z²) = 3a + Ez²: −(3 − b)/r² = 3(a − 1)/r² + Eκ² (3u as 4u − u keeps
  // every constant inline)
  const double am1 = a - 1.0;
  const double gr = fma(fma(am1, 4.0, -am1), ri2, E * k2);
  const double k21 = r3 * fma(dnx * dny, gr, -nn * am1);
  const double ar3 = a * r3;
  const double c1 = fma(-kp.th1, ar3, r3), c2 = fma(-kp.th2, ar3, r3);  // (1 − θa)/r³
  f1 = fma(dny * c1, wpj, fma(-k12, wnj, f1));
  f2 = fma(k21, wpj, fma(dnx * c2, wnj, f2));
  g1 = fma(-(dnx * c1), wpi, fma(-k12, wni, g1));
  g2 = fma(k21, wpi, fma(-(dny * c2), wni, g2));
}

__device__ __forceinline__ double shfl_next(double v, int addr) {
  const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// One 64-source group g of sym64_block's pair loop: both directions of every pair between the
// thread's two targets and sources g..g+63; forward sums into f, the wave's reverse sums of the
// group into sh.racc[w][·][0..63].
template <int kMetric, bool kFar>
__device__ __forceinline__ void sym64_group(int g, double xa, double ya, double za, double nxa, double nya,
                                            double nza, double wpa, double wna, double xb, double yb, double zb,
                                            double nxb, double nyb, double nzb, double wpb, double wnb,
                                            const KParams& kp, double k2, Sym64Shared& sh, double (&f)[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int next = ((lane + 1) & 63) << 2;
  double ra1 = 0.0, ra2 = 0.0;  // at step s: the reverse sums of source g + ((lane + s) mod 64)
  for (int s = 0; s < 64; ++s) {
    const int q = g + ((lane + s) & 63);
    const double2 c0 = sh.s0[q], c1 = sh.s1[q], c2 = sh.s2[q], c3 = sh.s3[q];
    if (kFar) {
      pair_sym_f64_far(xa, ya, za, nxa, nya, nza, wpa, wna, c0, c1, c2, c3, kp, k2, f[0], f[1], ra1, ra2);
      pair_sym_f64_far(xb, yb, zb, nxb, nyb, nzb, wpb, wnb, c0, c1, c2, c3, kp, k2, f[2], f[3], ra1, ra2);
    } else {
      pair_sym_f64<kMetric>(xa, ya, za, nxa, nya, nza, wpa, wna, c0, c1, c2, c3, kp, f[0], f[1], ra1, ra2);
      pair_sym_f64<kMetric>(xb, yb, zb, nxb, nyb, nzb, wpb, wnb, c0, c1, c2, c3, kp, f[2], f[3], ra1, ra2);
    }
    ra1 = shfl_next(ra1, next);
    ra2 = shfl_next(ra2, next);
  }
  sh.racc[w][0][lane] = ra1;
  sh.racc[w][1][lane] = ra2;
}

// Targets [t0, t0 + 512) (full; two per thread, t0 + 128w + l and 64 further, with bounding
// box tlo/thi) against sources [s0, s0 + 512), s0 ≠ t0, both directions; adds the forward sums
// into f and stores the reverse sums into rev (index j − s0), or adds them when rev_acc.
// wpsi/wpsn: h³ωψ/4π, h³ωψn/4π.
template <int kMetric>
__device__ __forceinline__ void sym64_block(const BandDev& b, const double* __restrict__ wpsi,
                                            const double* __restrict__ wpsn, int n, int t0, int s0,
                                            const KParams& kp, double k2, Sym64Shared& sh, double (&f)[4],
                                            const double (&tlo)[3], const double (&thi)[3], double* rev1,
                                            double* rev2, bool rev_acc) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double slo[3] = {INFINITY, INFINITY, INFINITY}, shi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int q = tid; q < kSymSub; q += kBlock) {
    const int j = s0 + q;
    if (j < n) {
      const double x = b.px[j], y = b.py[j], z = b.pz[j];
      sh.s0[q] = make_double2(x, y);
      sh.s1[q] = make_double2(z, b.nx[j]);
      sh.s2[q] = make_double2(b.ny[j], b.nz[j]);
      sh.s3[q] = make_double2(wpsi[j], wpsn[j]);
      slo[0] = fmin(slo[0], x), slo[1] = fmin(slo[1], y), slo[2] = fmin(slo[2], z);
      shi[0] = fmax(shi[0], x), shi[1] = fmax(shi[1], y), shi[2] = fmax(shi[2], z);
    } else {  // padding far away with zero weights: contributes exactly zero both ways
      sh.s0[q] = make_double2(1e6, 1e6);
      sh.s1[q] = make_double2(1e6, 0.0);
      sh.s2[q] = make_double2(0.0, 1.0);
      sh.s3[q] = make_double2(0.0, 0.0);
    }
  }
  block_box(slo, shi, sh);  // synchronizes: the staged sources are visible after it
  const bool far = kMetric != PB_REG_TANGENT &&
                   box_gap2_f64(tlo, thi, slo, shi) >=
                       (kMetric == PB_REG_EUCLIDEAN ? kp.tau2 : kp.four_tau2) * (1.0 + 1e-9);
  const int ia = t0 + w * 128 + lane, ib = ia + 64;
  const double xa = b.px[ia], ya = b.py[ia], za = b.pz[ia], nxa = b.nx[ia], nya = b.ny[ia], nza = b.nz[ia];
  const double xb = b.px[ib], yb = b.py[ib], zb = b.pz[ib], nxb = b.nx[ib], nyb = b.ny[ib], nzb = b.nz[ib];
  const double wpa = wpsi[ia], wna = wpsn[ia], wpb = wpsi[ib], wnb = wpsn[ib];
  for (int g = 0; g < kSymSub; g += 64) {
    if (far)
      sym64_group<kMetric, true>(g, xa, ya, za, nxa, nya, nza, wpa, wna, xb, yb, zb, nxb, nyb, nzb, wpb, wnb, kp, k2,
                                 sh, f);
    else
      sym64_group<kMetric, false>(g, xa, ya, za, nxa, nya, nza, wpa, wna, xb, yb, zb, nxb, nyb, nzb, wpb, wnb, kp,
                                  k2, sh, f);
    __syncthreads();
    // the four waves' reverse sums of the group, in wave order: threads 0..63 the ψ sums,
    // 64..127 the ψn sums
    if (tid < 128) {
      const int c = tid >> 6, q = g + lane;
      if (s0 + q < n) {
        double x = 0.0;
        for (int v = 0; v < kSymWaves; ++v) x += sh.racc[v][c][lane];
        double* rev = c ? rev2 : rev1;
        rev[q] = x + (rev_acc ? rev[q] : 0.0);
      }
    }
    __syncthreads();
  }
}

// Targets [t0, t0 + 512) (the same two per thread as sym64_block) against the sources of the
// same sub-block (self pair included), one direction with the per-pair kernel of the
// one-directional operator; adds into f.
__device__ __forceinline__ void diag64_block(const BandDev& b, const double* __restrict__ wpsi,
                                             const double* __restrict__ wpsn, int n, int t0, const KParams& kp,
                                             Sym64Shared& sh, double (&f)[4]) {
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
    const int i = t0 + (tid >> 6) * 128 + (tid & 63) + 64 * h;
    if (i < n) {
      const double xi = b.px[i], yi = b.py[i], zi = b.pz[i], nxi = b.nx[i], nyi = b.ny[i], nzi = b.nz[i];
      double s1 = 0.0, s2 = 0.0;
      for (int q = 0; q < m; ++q) {
        const double2 c0 = sh.s0[q], c1 = sh.s1[q], c2 = sh.s2[q], c3 = sh.s3[q];
        pair_f64(xi, yi, zi, nxi, nyi, nzi, c0.x, c0.y, c1.x, c1.y, c2.x, c2.y, c3.x, c3.y, kp, 0.0, s1, s2);
      }
      f[2 * h] += s1;
      f[2 * h + 1] += s2;
    }
  }
  __syncthreads();
}

// One work item (Ic, Jc), Ic ≤ Jc; partial: the band's chunked partial sums; k2 = κ².
__device__ __forceinline__ void sym64_item(const BandDev& b, const double* __restrict__ wpsi,
                                           const double* __restrict__ wpsn, int n, int Ic, int Jc, int nsub,
                                           const KParams& kp, double k2, double* __restrict__ partial,
                                           Sym64Shared& sh) {
  const int C = nsub * kSymSub;
  const int i0 = Ic * C, i1 = min(n, i0 + C), j0 = Jc * C, j1 = min(n, j0 + C);
  double* rowF = partial + (int64_t)Jc * 2 * n;
  double* rowR = partial + (int64_t)Ic * 2 * n;
  const bool diag = Ic == Jc;
  const int tid = threadIdx.x;
  for (int T = i0; T < i1; T += kSymSub) {
    const int ia = T + (tid >> 6) * 128 + (tid & 63), ib = ia + 64;
    // bounding box of the target sub-block (exact FP64)
    double tlo[3] = {INFINITY, INFINITY, INFINITY}, thi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i : {ia, ib})
      if (i < n) {
        const double p3[3] = {b.px[i], b.py[i], b.pz[i]};
        for (int c = 0; c < 3; ++c) {
          tlo[c] = fmin(tlo[c], p3[c]);
          thi[c] = fmax(thi[c], p3[c]);
        }
      }
    block_box(tlo, thi, sh);
    double f[4] = {0.0, 0.0, 0.0, 0.0};
    const bool rev_acc = T != i0;  // the first target sub-block stores the reverse slots
    for (int S = (diag ? T : j0); S < j1; S += kSymSub) {
      if (S == T)
        diag64_block(b, wpsi, wpsn, n, T, kp, sh, f);
      else if (kp.metric == PB_REG_EUCLIDEAN)
        sym64_block<PB_REG_EUCLIDEAN>(b, wpsi, wpsn, n, T, S, kp, k2, sh, f, tlo, thi, rowR + S, rowR + n + S,
                                      rev_acc);
      else if (kp.metric == PB_REG_TANGENT)
        sym64_block<PB_REG_TANGENT>(b, wpsi, wpsn, n, T, S, kp, k2, sh, f, tlo, thi, rowR + S, rowR + n + S, rev_acc);
      else
        sym64_block<PB_REG_TANGENT_GUARDED>(b, wpsi, wpsn, n, T, S, kp, k2, sh, f, tlo, thi, rowR + S, rowR + n + S,
                                            rev_acc);
    }
    // forward sums, once per target sub-block (in a diagonal item the earlier target
    // sub-blocks' reverse sums are already in these slots)
    const bool fwd_acc = diag && T != i0;
    if (ia < n) {
      rowF[ia] = f[0] + (fwd_acc ? rowF[ia] : 0.0);
      rowF[n + ia] = f[1] + (fwd_acc ? rowF[n + ia] : 0.0);
    }
    if (ib < n) {
      rowF[ib] = f[2] + (fwd_acc ? rowF[ib] : 0.0);
      rowF[n + ib] = f[3] + (fwd_acc ? rowF[n + ib] : 0.0);
    }
    __syncthreads();
  }
}

// Symmetric FP64 operator of one band: one block per work item. k2 = κ² (a kernel argument,
// so that it stays in scalar registers). Capped at 168 VGPRs for three waves per SIMD (37 KB
// of LDS per block allows four blocks per CU): the pair loops stay free of spills, which fall
// in the set-up code around them.
static __global__ void __attribute__((unused)) __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
    k_p2p_f64_sym(BandDev b, const double* __restrict__ wpsi, const double* __restrict__ wpsn, int n, int nsub,
                  const int2* __restrict__ items, int n_items, KParams kp, double k2, double* __restrict__ partial,
                  const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ Sym64Shared sh;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int2 w = items[it];
    sym64_item(b, wpsi, wpsn, n, w.x, w.y, nsub, kp, k2, partial, sh);
  }
}

}  // namespace pb
