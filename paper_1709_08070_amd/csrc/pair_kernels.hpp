// Device code shared by the single-molecule and batched operators: the per-pair kernels
// of eq. IBIM-PBE with the regularization subsection, and the LDS-tiled source loops.
//
// With d = x_i* − y_j*, r = |d|, E = e^{−κr}, a = E(1+κr), b = E(3+3κr+κ²r²), the four
// kernels times 4π are
//   4πK11 = (d·n_j)(1 − θ1 a)/r³            4πK12 = (1 − E)/r
//   4πK21 = (n_i·n_j)(1 − a)/r³ − (d·n_i)(d·n_j)(3 − b)/r⁵
//   4πK22 = −(d·n_i)(1 − θ2 a)/r³
// and pairs inside the tangent disc of radius τ take the disc averages (0, K̄12, 0, 0).
#pragma once

#include <hip/hip_runtime.h>

#include "pb_internal.hpp"

namespace pb {

struct KParams {
  double th1, th2, kappa, tau2, four_tau2, k12bar4pi;
  double k11c, k22c, k21bar4pi;  // regularized pairs: 4πK11 = k11c·c_i, 4πK22 = k22c·c_i, 4πK21 = k21bar4pi
  int metric;
  int curved;                     // curvature-corrected disc averages (the kernels then read b.curv)
};

inline KParams kparams(const Derived& d) {
  return KParams{d.th1, d.th2, d.kappa, d.tau2, d.four_tau2, 4.0 * kPi * d.k12bar,
                 d.curved ? d.k11c : 0.0, d.curved ? d.k22c : 0.0, d.curved ? d.k21bar4pi : 0.0, d.metric,
                 d.curved ? 1 : 0};
}

// ---------------------------------------------------------------- FP64

// The four kernels times 4π for one pair in FP64. The regularization predicate uses the
// products and sums exactly as written (no contraction).
__device__ __forceinline__ void kern4_f64(double xi, double yi, double zi, double nxi, double nyi, double nzi,
                                          double xj, double yj, double zj, double nxj, double nyj, double nzj,
                                          const KParams& kp, double ci, double k[4]) {
  double dx = xi - xj, dy = yi - yj, dz = zi - zj;
  double r2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
  double dnx = __dadd_rn(__dadd_rn(__dmul_rn(dx, nxi), __dmul_rn(dy, nyi)), __dmul_rn(dz, nzi));
  double t2 = __dadd_rn(r2, -__dmul_rn(dnx, dnx));
  bool reg;
  if (kp.metric == PB_REG_EUCLIDEAN) reg = r2 < kp.tau2;
  else if (kp.metric == PB_REG_TANGENT) reg = t2 < kp.tau2;
  else reg = t2 < kp.tau2 && r2 < kp.four_tau2;
  if (reg) {  // disc averages; ci = κ1 + κ2 at the target (0 with the paper's averages)
    k[0] = kp.k11c * ci;
    k[1] = kp.k12bar4pi;
    k[2] = kp.k21bar4pi;
    k[3] = kp.k22c * ci;
    return;
  }
  double dny = dx * nxj + dy * nyj + dz * nzj;
  double nn = nxi * nxj + nyi * nyj + nzi * nzj;
  // 1/r from the hardware reciprocal square root refined by two Newton steps
  double rinv = __builtin_amdgcn_rsq(r2);
  double e = fma(-r2 * rinv, rinv, 1.0);
  rinv = fma(0.5 * rinv, e, rinv);
  e = fma(-r2 * rinv, rinv, 1.0);
  rinv = fma(0.5 * rinv, e, rinv);
  double r = r2 * rinv;
  double r3 = rinv * rinv * rinv;
  double r5 = r3 * rinv * rinv;
  double z = kp.kappa * r;
  double E = exp(-z);
  double a = E * (1.0 + z);
  double b = E * (3.0 + 3.0 * z + z * z);
  k[0] = dny * (1.0 - kp.th1 * a) * r3;
  k[1] = (1.0 - E) * rinv;
  k[2] = nn * (1.0 - a) * r3 - dnx * dny * (3.0 - b) * r5;
  k[3] = -dnx * (1.0 - kp.th2 * a) * r3;
}

// s1 += 4πK11·wψ − 4πK12·wψn, s2 += 4πK21·wψ − 4πK22·wψn.
__device__ __forceinline__ void pair_f64(double xi, double yi, double zi, double nxi, double nyi, double nzi,
                                         double xj, double yj, double zj, double nxj, double nyj, double nzj,
                                         double wpsi, double wpsn, const KParams& kp, double ci, double& s1,
                                         double& s2) {
  double k[4];
  kern4_f64(xi, yi, zi, nxi, nyi, nzi, xj, yj, zj, nxj, nyj, nzj, kp, ci, k);
  s1 += k[0] * wpsi - k[1] * wpsn;
  s2 += k[2] * wpsi - k[3] * wpsn;
}

// ---------------------------------------------------------------- FP32

// FP32 records, coordinates centred on the band and scaled by σ = κ (σ = 1 when κ = 0):
//   A_j = (σ(x_j − c), w̃n_j),  M_j = σ·w̃_j·n_j,  N_j = (n_j, σ·w̃_j),
// with w̃_j = h³ω_jψ_j/(4π) and w̃n_j = h³ω_jψn_j/(4π). In scaled coordinates r' = κr = z, so
// e^{−κr} = exp2(−log2(e)·r') needs no extra product, and the sums come out as y1 = σ·S1,
// y2 = σ²·S2 (the scale is applied in FP64 afterwards). Folding the ψ weight into the source
// normal (M) lets one dot product give (d·n_j)·w̃_j and another (n_i·n_j)·w̃_j.
struct F32Params {
  float th1, th2, mlog2e, rc2;  // rc2: squared near-field radius in scaled units
  float far2;                   // rc2·(1 + 1e-3): a tile whose bounding box is at least this far
                                // (squared) from the target block holds no near pair
};

constexpr int kGroup = 256;  // records per bounding box (groups aligned at multiples of kGroup)

// Squared gap between two axis-aligned boxes (0 when they overlap).
__device__ __forceinline__ float box_gap2(const float4& lo1, const float4& hi1, const float4& lo2, const float4& hi2) {
  const float gx = fmaxf(0.f, fmaxf(lo2.x - hi1.x, lo1.x - hi2.x));
  const float gy = fmaxf(0.f, fmaxf(lo2.y - hi1.y, lo1.y - hi2.y));
  const float gz = fmaxf(0.f, fmaxf(lo2.z - hi1.z, lo1.z - hi2.z));
  return gx * gx + gy * gy + gz * gz;
}

// Union of the boxes of groups [g0, g1).
__device__ __forceinline__ void box_union(const float4* __restrict__ box, int g0, int g1, float4& lo, float4& hi) {
  lo = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
  hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.f);
  for (int g = g0; g < g1; ++g) {
    const float4 l = box[2 * g], h = box[2 * g + 1];
    lo.x = fminf(lo.x, l.x); lo.y = fminf(lo.y, l.y); lo.z = fminf(lo.z, l.z);
    hi.x = fmaxf(hi.x, h.x); hi.y = fmaxf(hi.y, h.y); hi.z = fmaxf(hi.z, h.z);
  }
}

// Squared distance in FP32 with a fixed operation sequence; every kernel that separates
// near from far pairs calls it on the same FP32 records.
__device__ __forceinline__ float r2_f32(float xi, float yi, float zi, float xj, float yj, float zj) {
  float dx = xi - xj, dy = yi - yj, dz = zi - zj;
  return __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, __fmul_rn(dx, dx)));
}

// One far pair in FP32 (target record ta with normal tn, source records sa, sm). Near pairs
// (r'² < rc2, which includes the self pair and every regularized pair) contribute exactly
// zero: 1/r' is replaced by 0 and every term carries a factor of it. With d = x_i − x_j,
// D = d·M_j = (d·n_j)σw̃_j, Nw = n_i·M_j = (n_i·n_j)σw̃_j, a = E(1+z):
//   a1 += (1 − θ1 a) D/r'³ − (1 − E) w̃n_j/r'
//   a2 += [(1 − a) Nw + (1 − θ2 a)(d·n_i) w̃n_j + (d·n_i) D (E z² − 3(1 − a))/r'²]/r'³,
// the second line being K21 r'³ = (n_i·n_j)(1 − a) − (d·n_i)(d·n_j)(3 − b)/r'² with
// 3 − b = 3(1 − a) − E z², b = E(3 + 3z + z²).
// kCheck = false is for tiles known to hold no near pair (the predicate is then skipped).
template <bool kScreened, bool kCheck = true>
__device__ __forceinline__ void pair_f32(const float4& ta, const float4& tn, const float4& sa, const float4& sm,
                                         const F32Params& fp, float& a1, float& a2) {
  const float dx = ta.x - sa.x, dy = ta.y - sa.y, dz = ta.z - sa.z;
  const float r2 = r2_f32(ta.x, ta.y, ta.z, sa.x, sa.y, sa.z);
  float rinv = __builtin_amdgcn_rsqf(r2);
  if (kCheck && r2 < fp.rc2) rinv = 0.f;
  float E = 1.f, z = 0.f;
  if (kScreened) {
    z = r2 * rinv;
    E = __builtin_amdgcn_exp2f(fp.mlog2e * z);
  }
  const float a = __fmaf_rn(E, z, E);  // E(1 + r')
  const float dnx = __fmaf_rn(dz, tn.z, __fmaf_rn(dy, tn.y, dx * tn.x));
  const float D = __fmaf_rn(dz, sm.z, __fmaf_rn(dy, sm.y, dx * sm.x));
  const float Nw = __fmaf_rn(tn.z, sm.z, __fmaf_rn(tn.y, sm.y, tn.x * sm.x));
  const float ri2 = rinv * rinv;
  const float r3 = ri2 * rinv;
  const float c1 = __fmaf_rn(-fp.th1, a, 1.f);
  const float c2 = __fmaf_rn(-fp.th2, a, 1.f);
  a1 = __fmaf_rn(c1 * D, r3, a1);
  float t;
  if (kScreened) {
    const float f0w = __fmaf_rn(-E, sa.w, sa.w);  // (1 − E) w̃n_j
    a1 = __fmaf_rn(-f0w, rinv, a1);
    const float gr = __fmaf_rn(__fmaf_rn(3.f, a, -3.f), ri2, E);  // g/r'² = E − 3(1 − a)/r'²
    t = __fmaf_rn(-a, Nw, Nw);
    t = __fmaf_rn(c2 * dnx, sa.w, t);
    t = __fmaf_rn(dnx * D, gr, t);
  } else {  // κ = 0: E = a = 1 and z = 0, so only the θ terms remain
    t = c2 * dnx * sa.w;
  }
  a2 = __fmaf_rn(t, r3, a2);
}

// Targets [t0, t0 + kBlk·TPL) against sources [j0, j1) of the same record arrays; per-tile
// FP32 partial sums flushed into FP64. out1/out2 receive σ·S1 and σ²·S2 for each live target
// (index relative to t0). Every thread of the block must call it (it synchronizes).
// box: bounding boxes of the record groups (k_group_box); full source tiles whose box is
// farther than √far2 from the target block's box skip the near-pair predicate.
template <int kBlk, int TILE, int TPL, bool kScreened>
__device__ __forceinline__ void far_tile_loop(const float4* __restrict__ A, const float4* __restrict__ M,
                                              const float4* __restrict__ N, const float4* __restrict__ box, int t0,
                                              int t_end, int j0, int j1, const F32Params& fp, double sig1,
                                              double sig2, float4* sA, float4* sM, double* __restrict__ out1,
                                              double* __restrict__ out2) {
  static_assert(TILE % kGroup == 0 && (kBlk * TPL) % kGroup == 0, "tiles are whole groups");
  float4 tlo, thi;
  box_union(box, t0 / kGroup, min(t0 + kBlk * TPL, t_end + kGroup - 1) / kGroup, tlo, thi);
  float4 ta[TPL], tn[TPL];
#pragma unroll
  for (int t = 0; t < TPL; ++t) {
    const int i = t0 + t * kBlk + (int)threadIdx.x;
    ta[t] = i < t_end ? A[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    tn[t] = i < t_end ? N[i] : make_float4(0.f, 0.f, 1.f, 0.f);
  }
  double acc1[TPL], acc2[TPL];
#pragma unroll
  for (int t = 0; t < TPL; ++t) acc1[t] = acc2[t] = 0.0;
  for (int base = j0; base < j1; base += TILE) {
    for (int q = threadIdx.x; q < TILE; q += kBlk) {
      const int j = base + q;
      if (j < j1) {
        sA[q] = A[j];
        sM[q] = M[j];
      } else {  // padding: zero weights, every value they meet is finite
        sA[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        sM[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    // block-uniform: the tile is full and its box is clear of the target block's box
    int clear = 0;
    if (base + TILE <= j1) {
      float4 slo, shi;
      box_union(box, base / kGroup, (base + TILE) / kGroup, slo, shi);
      clear = box_gap2(tlo, thi, slo, shi) >= fp.far2;
    }
    clear = __builtin_amdgcn_readfirstlane(clear);
    __syncthreads();
    float a1[TPL], a2[TPL];
#pragma unroll
    for (int t = 0; t < TPL; ++t) a1[t] = a2[t] = 0.f;
    if (clear) {
#pragma unroll 4
      for (int q = 0; q < TILE; ++q) {
        const float4 sa = sA[q], sm = sM[q];
#pragma unroll
        for (int t = 0; t < TPL; ++t) pair_f32<kScreened, false>(ta[t], tn[t], sa, sm, fp, a1[t], a2[t]);
      }
    } else {
#pragma unroll 4
      for (int q = 0; q < TILE; ++q) {
        const float4 sa = sA[q], sm = sM[q];
#pragma unroll
        for (int t = 0; t < TPL; ++t) pair_f32<kScreened, true>(ta[t], tn[t], sa, sm, fp, a1[t], a2[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
      acc1[t] += (double)a1[t];
      acc2[t] += (double)a2[t];
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < TPL; ++t) {
    const int i = t0 + t * kBlk + (int)threadIdx.x;
    if (i < t_end) {
      out1[i - t0] = sig1 * acc1[t];
      out2[i - t0] = sig2 * acc2[t];
    }
  }
}


// ---------------------------------------------------------------- kernels

constexpr int kBlock = 256;

struct BandDev {
  const double *px, *py, *pz, *nx, *ny, *nz;
  const double* curv;  // κ1 + κ2 at the projections, or null (flat disc averages)
};

// The band's geometry; the curvature only where the curvature-corrected averages use it.
inline BandDev band_dev(const pb_band* b, bool with_curv = false) {
  return BandDev{b->px, b->py, b->pz, b->nx, b->ny, b->nz, with_curv ? b->curv : nullptr};
}

// Source weights h³ω_j ψ_j/(4π), h³ω_j ψn_j/(4π) in FP64.
static __global__ void __attribute__((unused)) __launch_bounds__(kBlock) k_weights_f64(int n, const double* __restrict__ w,
                                                               const double* __restrict__ p, double scale,
                                                               double* __restrict__ wpsi, double* __restrict__ wpsn) {
  int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  double s = scale * w[j];
  wpsi[j] = s * p[j];
  wpsn[j] = s * p[n + j];
}

// FP64 targets [t0, t0 + kBlk) against sources [j0, j1) of the band arrays b with source
// weights wpsi/wpsn (h³ωψ/4π, h³ωψn/4π); out1/out2 receive the sums for each live target
// (index relative to t0). Every thread of the block must call it (it synchronizes).
template <int kBlk>
__device__ __forceinline__ void far64_tile_loop(const BandDev& b, const double* __restrict__ wpsi,
                                                const double* __restrict__ wpsn, int t0, int t_end, int j0, int j1,
                                                const KParams& kp, double* smem, double* __restrict__ out1,
                                                double* __restrict__ out2) {
  double *sx = smem, *sy = sx + kBlk, *sz = sy + kBlk, *snx = sz + kBlk, *sny = snx + kBlk, *snz = sny + kBlk,
         *sw1 = snz + kBlk, *sw2 = sw1 + kBlk;
  const int i = t0 + (int)threadIdx.x;
  const bool live = i < t_end;
  double xi = 0, yi = 0, zi = 0, nxi = 0, nyi = 0, nzi = 1, ci = 0;
  if (live) {
    xi = b.px[i]; yi = b.py[i]; zi = b.pz[i];
    nxi = b.nx[i]; nyi = b.ny[i]; nzi = b.nz[i];
    ci = b.curv ? b.curv[i] : 0.0;
  }
  double s1 = 0.0, s2 = 0.0;
  for (int base = j0; base < j1; base += kBlk) {
    const int j = base + (int)threadIdx.x;
    if (j < j1) {
      sx[threadIdx.x] = b.px[j]; sy[threadIdx.x] = b.py[j]; sz[threadIdx.x] = b.pz[j];
      snx[threadIdx.x] = b.nx[j]; sny[threadIdx.x] = b.ny[j]; snz[threadIdx.x] = b.nz[j];
      sw1[threadIdx.x] = wpsi[j]; sw2[threadIdx.x] = wpsn[j];
    }
    __syncthreads();
    const int m = min(kBlk, j1 - base);
    if (live)
      for (int q = 0; q < m; ++q)
        pair_f64(xi, yi, zi, nxi, nyi, nzi, sx[q], sy[q], sz[q], snx[q], sny[q], snz[q], sw1[q], sw2[q], kp, ci, s1,
                 s2);
    __syncthreads();
  }
  if (live) {
    out1[i - t0] = s1;
    out2[i - t0] = s2;
  }
}

// FP64 operator, one target per lane; block (x: target block, y: source chunk).
static __global__ void __attribute__((unused)) __launch_bounds__(kBlock) k_p2p_f64(BandDev b, const double* __restrict__ wpsi,
                                                           const double* __restrict__ wpsn, int n, int chunk,
                                                           double* __restrict__ partial, KParams kp,
                                                           const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double smem[8 * kBlock];
  const int t0 = blockIdx.x * kBlock;
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  double* out = partial + (size_t)blockIdx.y * 2 * n;
  far64_tile_loop<kBlock>(b, wpsi, wpsn, t0, n, j0, j1, kp, smem, out + t0, out + n + t0);
}

// y = Λp + Σ_chunks partial (+ near), in a fixed order.
static __global__ void __attribute__((unused)) __launch_bounds__(kBlock) k_reduce(int n, int n_chunks, const double* __restrict__ partial,
                                                          const double* __restrict__ near,
                                                          const double* __restrict__ p, double lam1, double lam2,
                                                          double* __restrict__ y) {
  int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= 2 * n) return;
  double s = 0.0;
  // unrolled so that eight loads are in flight; the sum keeps its chunk order
#pragma unroll 8
  for (int c = 0; c < n_chunks; ++c) s += partial[(size_t)c * 2 * n + e];
  if (near) s += near[e];
  y[e] = (e < n ? lam1 : lam2) * p[e] + s;
}

// FP32 records of a band (layout above); with p == nullptr only the geometry is written
// (weights zero).
static __global__ void __attribute__((unused)) __launch_bounds__(kBlock) k_pack_f32(int n, BandDev b, const double* __restrict__ w,
                                                            const double* __restrict__ p, double scale, double cx,
                                                            double cy, double cz, double sigma,
                                                            float4* __restrict__ A, float4* __restrict__ M,
                                                            float4* __restrict__ N) {
  int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  const double s = scale * w[j];
  const double w1 = p ? sigma * s * p[j] : 0.0, w2 = p ? s * p[n + j] : 0.0;
  A[j] = make_float4((float)(sigma * (b.px[j] - cx)), (float)(sigma * (b.py[j] - cy)), (float)(sigma * (b.pz[j] - cz)),
                     (float)w2);
  M[j] = make_float4((float)(w1 * b.nx[j]), (float)(w1 * b.ny[j]), (float)(w1 * b.nz[j]), 0.f);
  N[j] = make_float4((float)b.nx[j], (float)b.ny[j], (float)b.nz[j], (float)w1);
}

// Bounding box of each aligned group of kGroup records (one block per group):
// box[2g] = (lo, 0), box[2g + 1] = (hi, 0) over the group's live records.
static __global__ void __attribute__((unused)) __launch_bounds__(kGroup) k_group_box(int n, const float4* __restrict__ A,
                                                                  float4* __restrict__ box) {
  __shared__ float s[6][kGroup];
  const int i = blockIdx.x * kGroup + threadIdx.x;
  float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  if (i < n) {
    const float4 a = A[i];
    v[0] = v[3] = a.x;
    v[1] = v[4] = a.y;
    v[2] = v[5] = a.z;
  }
  for (int q = 0; q < 6; ++q) s[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int off = kGroup / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      for (int q = 0; q < 6; ++q)
        s[q][threadIdx.x] = q < 3 ? fminf(s[q][threadIdx.x], s[q][threadIdx.x + off])
                                  : fmaxf(s[q][threadIdx.x], s[q][threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    box[2 * blockIdx.x] = make_float4(s[0][0], s[1][0], s[2][0], 0.f);
    box[2 * blockIdx.x + 1] = make_float4(s[3][0], s[4][0], s[5][0], 0.f);
  }
}

// FP32 far field of one band: block (x: kBlock·TPL targets, y: source chunk).
template <int TILE, int TPL, bool kScreened>
static __global__ void __attribute__((unused)) __launch_bounds__(kBlock) k_p2p_f32(const float4* __restrict__ A, const float4* __restrict__ M,
                                                           const float4* __restrict__ N,
                                                           const float4* __restrict__ box, int n, int chunk,
                                                           F32Params fp, double sig1, double sig2,
                                                           double* __restrict__ partial,
                                                           const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ float4 sA[TILE], sM[TILE];
  const int t0 = blockIdx.x * kBlock * TPL;
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  double* out = partial + (size_t)blockIdx.y * 2 * n;
  far_tile_loop<kBlock, TILE, TPL, kScreened>(A, M, N, box, t0, n, j0, j1, fp, sig1, sig2, sA, sM, out + t0,
                                              out + n + t0);
}

// ----------------------------------------------------------------- near field (cell list)

struct CellsDev {
  const int64_t* start;  // ncell + 1
  const int* nodes;      // n, sorted within each cell
  const int* cell_of;    // n
  int ncx, ncy, ncz;
};

static __global__ void __attribute__((unused)) __launch_bounds__(kBlock) k_bbox(int n, BandDev b, double* __restrict__ out /*6 per block*/) {
  __shared__ double s[6][kBlock];
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock) {
    v[0] = fmin(v[0], b.px[j]); v[1] = fmin(v[1], b.py[j]); v[2] = fmin(v[2], b.pz[j]);
    v[3] = fmax(v[3], b.px[j]); v[4] = fmax(v[4], b.py[j]); v[5] = fmax(v[5], b.pz[j]);
  }
  for (int q = 0; q < 6; ++q) s[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      for (int q = 0; q < 6; ++q)
        s[q][threadIdx.x] = q < 3 ? fmin(s[q][threadIdx.x], s[q][threadIdx.x + off])
                                  : fmax(s[q][threadIdx.x], s[q][threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 6; ++q) out[6 * blockIdx.x + q] = s[q][0];
}

static __global__ void __attribute__((unused)) __launch_bounds__(kBlock) k_cell_count(int n, BandDev b, double lx, double ly, double lz,
                                                       double inv_cell, int ncx, int ncy, int ncz,
                                                       int* __restrict__ cell_of, int64_t* __restrict__ counts) {
  int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  int cx = min(ncx - 1, max(0, (int)((b.px[j] - lx) * inv_cell)));
  int cy = min(ncy - 1, max(0, (int)((b.py[j] - ly) * inv_cell)));
  int cz = min(ncz - 1, max(0, (int)((b.pz[j] - lz) * inv_cell)));
  int c = (cx * ncy + cy) * ncz + cz;
  cell_of[j] = c;
  atomicAdd((unsigned long long*)&counts[c], 1ull);
}

static __global__ void __attribute__((unused)) __launch_bounds__(kBlock) k_cell_fill(int n, const int* __restrict__ cell_of,
                                                      const int64_t* __restrict__ start, int* __restrict__ cursor,
                                                      int* __restrict__ nodes) {
  int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  int c = cell_of[j];
  int slot = atomicAdd(&cursor[c], 1);
  nodes[start[c] + slot] = j;
}

// Insertion sort of each cell's node list, so the near-field sums run in a fixed order.
static __global__ void __attribute__((unused)) __launch_bounds__(kBlock) k_cell_sort(int64_t ncell, const int64_t* __restrict__ start,
                                                      int* __restrict__ nodes) {
  int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= ncell) return;
  int64_t s = start[c], e = start[c + 1];
  for (int64_t q = s + 1; q < e; ++q) {
    int v = nodes[q];
    int64_t t = q - 1;
    while (t >= s && nodes[t] > v) {
      nodes[t + 1] = nodes[t];
      --t;
    }
    nodes[t + 1] = v;
  }
}

// Visits the near sources of target i (FP32 distance below r_c) in a fixed order: the 27
// neighbouring cells in lexicographic order, each cell's nodes in increasing index. One
// wave per target: the lanes test a cell's candidates 64 at a time and a ballot numbers the
// hits in that order; f(j, slot) runs on each hit lane, and the wave's hit count returns.
template <typename F>
__device__ __forceinline__ int64_t for_near_wave(int i, const float4* __restrict__ A, const CellsDev& cells,
                                                 float rc2, F f) {
  const int lane = threadIdx.x & 63;
  const float4 ta = A[i];
  const int c = cells.cell_of[i];
  const int cz = c % cells.ncz, cy = (c / cells.ncz) % cells.ncy, cx = c / (cells.ncz * cells.ncy);
  int64_t base = 0;
  for (int ax = max(cx - 1, 0); ax <= min(cx + 1, cells.ncx - 1); ++ax)
    for (int ay = max(cy - 1, 0); ay <= min(cy + 1, cells.ncy - 1); ++ay)
      for (int az = max(cz - 1, 0); az <= min(cz + 1, cells.ncz - 1); ++az) {
        const int cc = (ax * cells.ncy + ay) * cells.ncz + az;
        const int64_t e = cells.start[cc + 1];
        for (int64_t q0 = cells.start[cc]; q0 < e; q0 += 64) {
          const int64_t q = q0 + lane;
          int j = -1;
          bool hit = false;
          if (q < e) {
            j = cells.nodes[q];
            const float4 sa = A[j];
            hit = r2_f32(ta.x, ta.y, ta.z, sa.x, sa.y, sa.z) < rc2;
          }
          const unsigned long long mask = __ballot(hit);
          if (hit) f(j, base + __popcll(mask & ((1ull << lane) - 1ull)));
          base += __popcll(mask);
        }
      }
  return base;
}

constexpr int kNearWaves = kBlock / 64;  // targets per block of the near-list kernels

static __global__ void __attribute__((unused)) __launch_bounds__(kBlock) k_near_count(int n, const float4* __restrict__ A, CellsDev cells, float rc2,
                                                       int64_t* __restrict__ counts) {
  const int i = blockIdx.x * kNearWaves + (threadIdx.x >> 6);
  if (i >= n) return;
  const int64_t c = for_near_wave(i, A, cells, rc2, [&](int, int64_t) {});
  if ((threadIdx.x & 63) == 0) counts[i] = c;
}

// Near-field block matrix: for each near pair the FP64 coefficients of
//   y1_i += c0 ψ_j + c1 ψn_j,  y2_i += c2 ψ_j + c3 ψn_j,  with s_j = h³ω_j/(4π)
//   c0 = 4πK11 s_j, c1 = −4πK12 s_j, c2 = 4πK21 s_j, c3 = −4πK22 s_j.
// The coefficients depend on geometry only, so they are built once per band.
static __global__ void __attribute__((unused)) __launch_bounds__(kBlock) k_near_fill(int n, BandDev b, const double* __restrict__ w, double scale,
                                                      const float4* __restrict__ A, CellsDev cells, float rc2,
                                                      KParams kp, const int64_t* __restrict__ row,
                                                      int* __restrict__ col, double4* __restrict__ coef) {
  const int i = blockIdx.x * kNearWaves + (threadIdx.x >> 6);
  if (i >= n) return;
  const double xi = b.px[i], yi = b.py[i], zi = b.pz[i], nxi = b.nx[i], nyi = b.ny[i], nzi = b.nz[i];
  const double ci = b.curv ? b.curv[i] : 0.0;
  const int64_t r0 = row[i];
  // the columns first (a few hits per 64 candidates), then the FP64 coefficients with every
  // lane busy: entry q = r0 + lane, r0 + lane + 64, ... reads back the column its wave wrote
  const int64_t cnt = for_near_wave(i, A, cells, rc2, [&](int j, int64_t slot) { col[r0 + slot] = j; });
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int64_t q = r0 + (threadIdx.x & 63); q < r0 + cnt; q += 64) {
    const int j = col[q];
    double k[4];
    kern4_f64(xi, yi, zi, nxi, nyi, nzi, b.px[j], b.py[j], b.pz[j], b.nx[j], b.ny[j], b.nz[j], kp, ci, k);
    const double sj = scale * w[j];
    coef[q] = make_double4(k[0] * sj, -k[1] * sj, k[2] * sj, -k[3] * sj);
  }
}

constexpr int kRowLanes = 16;  // lanes cooperating on one CSR row

// near = (near block matrix)·p, 16 lanes per row, fixed-order lane reduction.
static __global__ void __attribute__((unused)) __launch_bounds__(kBlock) k_near_spmv(int n, const int64_t* __restrict__ row,
                                                      const int* __restrict__ col, const double4* __restrict__ coef,
                                                      const double* __restrict__ p, double* __restrict__ near) {
  const int i = (blockIdx.x * kBlock + threadIdx.x) / kRowLanes;
  const int lane = threadIdx.x % kRowLanes;
  double s1 = 0.0, s2 = 0.0;
  if (i < n) {
    const int64_t e = row[i + 1];
    for (int64_t q = row[i] + lane; q < e; q += kRowLanes) {
      const int j = col[q];
      const double4 c = coef[q];
      const double ps = p[j], pn = p[n + j];
      s1 += c.x * ps + c.y * pn;
      s2 += c.z * ps + c.w * pn;
    }
  }
  for (int off = kRowLanes / 2; off > 0; off >>= 1) {
    s1 += __shfl_down(s1, off, kRowLanes);
    s2 += __shfl_down(s2, off, kRowLanes);
  }
  if (i < n && lane == 0) {
    near[i] = s1;
    near[n + i] = s2;
  }
}


}  // namespace pb
