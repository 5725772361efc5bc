// The IBIM operator y = Λp + KWp (eq. final-lin-sys) between band nodes.
//
// Per ordered pair (target i, source j), with d = x_i* − y_j*, r = |d|, E = e^{−κr},
// a = E(1+κr), b = E(3+3κr+κ²r²), the four kernels of eq. IBIM-PBE are (times 4π)
//   4πK11 = (d·n_j)(1 − θ1 a)/r³            4πK12 = (1 − E)/r
//   4πK21 = (n_i·n_j)(1 − a)/r³ − (d·n_i)(d·n_j)(3 − b)/r⁵
//   4πK22 = −(d·n_i)(1 − θ2 a)/r³
// and pairs inside the tangent disc of radius τ take the disc averages (0, K̄12, 0, 0)
// (regularization subsection). The source weights carry h³ω_j/(4π), so
//   y1_i = λ1 ψ_i + Σ_j (4πK11 wψ_j − 4πK12 wψn_j),  y2_i = λ2 ψn_i + Σ_j (4πK21 wψ_j − 4πK22 wψn_j).
//
// Two implementations share this file:
//   * FP64: one target per lane, sources staged through LDS in tiles of 256, the source
//     range split into chunks so that small bands still fill 256 CUs; chunk partial sums are
//     reduced in a fixed order (no atomics, bitwise reproducible).
//   * Mixed: the same tiling in FP32 (rsq and exp2 on the transcendental unit, 32 B source
//     records in LDS, FP32 partials per tile flushed to FP64 accumulators). Pairs closer
//     than r_c (≥ 2τ, so every regularized pair) are skipped and evaluated in FP64 by a
//     cell-list near-field kernel. Both kernels decide "near" with the same FP32 function
//     of the same FP32 coordinates, so every pair is counted exactly once.
#include <cmath>

#include "pb_internal.hpp"

namespace pb {

struct KParams {
  double th1, th2, kappa, tau2, four_tau2, k12bar4pi;
  int metric;
};

namespace {

constexpr int kBlock = 256;
constexpr int kTileSrc = 256;

KParams kparams(const Derived& d) {
  return KParams{d.th1, d.th2, d.kappa, d.tau2, d.four_tau2, 4.0 * kPi * d.k12bar, d.metric};
}

// ----------------------------------------------------------------- FP64 pair

// The four kernels times 4π for one pair in FP64: k[0] = 4πK11, k[1] = 4πK12, k[2] = 4πK21,
// k[3] = 4πK22. The regularization predicate uses the products and sums exactly as written
// (no contraction) so that it is decided as in a plain evaluation.
__device__ __forceinline__ void kern4_f64(double xi, double yi, double zi, double nxi, double nyi, double nzi,
                                          double xj, double yj, double zj, double nxj, double nyj, double nzj,
                                          const KParams& kp, double k[4]) {
  double dx = xi - xj, dy = yi - yj, dz = zi - zj;
  double r2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
  double dnx = __dadd_rn(__dadd_rn(__dmul_rn(dx, nxi), __dmul_rn(dy, nyi)), __dmul_rn(dz, nzi));
  double t2 = __dadd_rn(r2, -__dmul_rn(dnx, dnx));
  bool reg;
  if (kp.metric == PB_REG_EUCLIDEAN) reg = r2 < kp.tau2;
  else if (kp.metric == PB_REG_TANGENT) reg = t2 < kp.tau2;
  else reg = t2 < kp.tau2 && r2 < kp.four_tau2;
  if (reg) {
    k[0] = 0.0;
    k[1] = kp.k12bar4pi;
    k[2] = 0.0;
    k[3] = 0.0;
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

// Accumulates one pair: s1 += 4πK11·wψ − 4πK12·wψn, s2 += 4πK21·wψ − 4πK22·wψn.
__device__ __forceinline__ void pair_f64(double xi, double yi, double zi, double nxi, double nyi, double nzi,
                                         double xj, double yj, double zj, double nxj, double nyj, double nzj,
                                         double wpsi, double wpsn, const KParams& kp, double& s1, double& s2) {
  double k[4];
  kern4_f64(xi, yi, zi, nxi, nyi, nzi, xj, yj, zj, nxj, nyj, nzj, kp, k);
  s1 += k[0] * wpsi - k[1] * wpsn;
  s2 += k[2] * wpsi - k[3] * wpsn;
}

// Source weights h³ω_j ψ_j/(4π), h³ω_j ψn_j/(4π) in FP64.
__global__ void __launch_bounds__(kBlock) k_weights_f64(int n, const double* __restrict__ w,
                                                        const double* __restrict__ p, double scale,
                                                        double* __restrict__ wpsi, double* __restrict__ wpsn) {
  int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  double s = scale * w[j];
  wpsi[j] = s * p[j];
  wpsn[j] = s * p[n + j];
}

struct BandDev {
  const double *px, *py, *pz, *nx, *ny, *nz;
};

__global__ void __launch_bounds__(kBlock) k_p2p_f64(BandDev b, const double* __restrict__ wpsi,
                                                    const double* __restrict__ wpsn, int n, int chunk,
                                                    double* __restrict__ partial, KParams kp) {
  __shared__ double sx[kTileSrc], sy[kTileSrc], sz[kTileSrc], snx[kTileSrc], sny[kTileSrc], snz[kTileSrc],
      sw1[kTileSrc], sw2[kTileSrc];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool live = i < n;
  double xi = 0, yi = 0, zi = 0, nxi = 0, nyi = 0, nzi = 1;
  if (live) {
    xi = b.px[i]; yi = b.py[i]; zi = b.pz[i];
    nxi = b.nx[i]; nyi = b.ny[i]; nzi = b.nz[i];
  }
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  double s1 = 0.0, s2 = 0.0;
  for (int base = j0; base < j1; base += kTileSrc) {
    int j = base + threadIdx.x;
    if (j < j1) {
      sx[threadIdx.x] = b.px[j]; sy[threadIdx.x] = b.py[j]; sz[threadIdx.x] = b.pz[j];
      snx[threadIdx.x] = b.nx[j]; sny[threadIdx.x] = b.ny[j]; snz[threadIdx.x] = b.nz[j];
      sw1[threadIdx.x] = wpsi[j]; sw2[threadIdx.x] = wpsn[j];
    }
    __syncthreads();
    const int m = min(kTileSrc, j1 - base);
    if (live)
      for (int q = 0; q < m; ++q)
        pair_f64(xi, yi, zi, nxi, nyi, nzi, sx[q], sy[q], sz[q], snx[q], sny[q], snz[q], sw1[q], sw2[q], kp, s1, s2);
    __syncthreads();
  }
  if (live) {
    partial[(size_t)blockIdx.y * 2 * n + i] = s1;
    partial[(size_t)blockIdx.y * 2 * n + n + i] = s2;
  }
}

// y = Λp + Σ_chunks partial (+ near), in a fixed order.
__global__ void __launch_bounds__(kBlock) k_reduce(int n, int n_chunks, const double* __restrict__ partial,
                                                   const double* __restrict__ near, const double* __restrict__ p,
                                                   double lam1, double lam2, double* __restrict__ y) {
  int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= 2 * n) return;
  double s = 0.0;
  for (int c = 0; c < n_chunks; ++c) s += partial[(size_t)c * 2 * n + e];
  if (near) s += near[e];
  y[e] = (e < n ? lam1 : lam2) * p[e] + s;
}

// ----------------------------------------------------------------- FP32 far field

struct F32Params {
  float th1, th2, kappa, mlog2k;  // mlog2k = −κ·log2(e)
};

// Squared distance in FP32 with a fixed operation sequence; the far and near kernels both
// call it so that they agree on every pair.
__device__ __forceinline__ float r2_f32(float xi, float yi, float zi, float xj, float yj, float zj) {
  float dx = xi - xj, dy = yi - yj, dz = zi - zj;
  return __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, __fmul_rn(dx, dx)));
}

// Source records: A = (x, y, z, h³ωψ/4π), B = (n_x, n_y, n_z, h³ωψn/4π), centroid-relative FP32.
__global__ void __launch_bounds__(kBlock) k_pack_f32(int n, BandDev b, const double* __restrict__ w,
                                                     const double* __restrict__ p, double scale, double cx, double cy,
                                                     double cz, float4* __restrict__ A, float4* __restrict__ B) {
  int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  double s = scale * w[j];
  double w1 = p ? s * p[j] : 0.0, w2 = p ? s * p[n + j] : 0.0;
  A[j] = make_float4((float)(b.px[j] - cx), (float)(b.py[j] - cy), (float)(b.pz[j] - cz), (float)w1);
  B[j] = make_float4((float)b.nx[j], (float)b.ny[j], (float)b.nz[j], (float)w2);
}

__global__ void __launch_bounds__(kBlock) k_p2p_f32(const float4* __restrict__ A, const float4* __restrict__ B, int n,
                                                    int chunk, float rc2, F32Params fp,
                                                    double* __restrict__ partial) {
  __shared__ float4 sA[kTileSrc], sB[kTileSrc];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool live = i < n;
  float4 ta = live ? A[i] : make_float4(0.f, 0.f, 0.f, 0.f);
  float4 tb = live ? B[i] : make_float4(0.f, 0.f, 1.f, 0.f);
  const int j0 = blockIdx.y * chunk;
  const int j1 = min(n, j0 + chunk);
  double acc1 = 0.0, acc2 = 0.0;
  for (int base = j0; base < j1; base += kTileSrc) {
    int j = base + threadIdx.x;
    if (j < j1) {
      sA[threadIdx.x] = A[j];
      sB[threadIdx.x] = B[j];
    } else {
      // padding sources carry zero weights: every kernel value they meet is finite, so they add nothing
      sA[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
      sB[threadIdx.x] = make_float4(0.f, 0.f, 1.f, 0.f);
    }
    __syncthreads();
    float a1 = 0.f, a2 = 0.f;
#pragma unroll 4
    for (int q = 0; q < kTileSrc; ++q) {
      const float4 sa = sA[q], sb = sB[q];
      const float dx = ta.x - sa.x, dy = ta.y - sa.y, dz = ta.z - sa.z;
      const float r2 = r2_f32(ta.x, ta.y, ta.z, sa.x, sa.y, sa.z);
      const bool near = r2 < rc2;
      const float rinv = near ? 0.f : __builtin_amdgcn_rsqf(r2);
      const float r = r2 * rinv;
      const float z = fp.kappa * r;
      const float E = __builtin_amdgcn_exp2f(fp.mlog2k * r);
      const float a = __fmaf_rn(E, z, E);
      const float b = E * __fmaf_rn(z, z + 3.f, 3.f);
      const float dnx = dx * tb.x + dy * tb.y + dz * tb.z;
      const float dny = dx * sb.x + dy * sb.y + dz * sb.z;
      const float nn = tb.x * sb.x + tb.y * sb.y + tb.z * sb.z;
      const float ri2 = rinv * rinv;
      const float r3 = ri2 * rinv;
      const float r5 = r3 * ri2;
      const float k11 = dny * __fmaf_rn(-fp.th1, a, 1.f) * r3;
      const float k12 = (1.f - E) * rinv;
      const float k21 = nn * (1.f - a) * r3 - dnx * dny * (3.f - b) * r5;
      const float k22 = dnx * __fmaf_rn(-fp.th2, a, 1.f) * r3;
      a1 += k11 * sa.w - k12 * sb.w;
      a2 += k21 * sa.w + k22 * sb.w;
    }
    acc1 += (double)a1;
    acc2 += (double)a2;
    __syncthreads();
  }
  if (live) {
    partial[(size_t)blockIdx.y * 2 * n + i] = acc1;
    partial[(size_t)blockIdx.y * 2 * n + n + i] = acc2;
  }
}

// ----------------------------------------------------------------- near field (cell list)

struct CellsDev {
  const int64_t* start;  // ncell + 1
  const int* nodes;      // n, sorted within each cell
  const int* cell_of;    // n
  int ncx, ncy, ncz;
};

__global__ void __launch_bounds__(kBlock) k_bbox(int n, BandDev b, double* __restrict__ out /*6 per block*/) {
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

__global__ void __launch_bounds__(kBlock) k_cell_count(int n, BandDev b, double lx, double ly, double lz,
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

__global__ void __launch_bounds__(kBlock) k_cell_fill(int n, const int* __restrict__ cell_of,
                                                      const int64_t* __restrict__ start, int* __restrict__ cursor,
                                                      int* __restrict__ nodes) {
  int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  int c = cell_of[j];
  int slot = atomicAdd(&cursor[c], 1);
  nodes[start[c] + slot] = j;
}

// Insertion sort of each cell's node list, so the near-field sums run in a fixed order.
__global__ void __launch_bounds__(kBlock) k_cell_sort(int64_t ncell, const int64_t* __restrict__ start,
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

// Visits the near sources of target i (FP32 distance below r_c) in a fixed order: the
// 27 neighbouring cells in lexicographic order, each cell's nodes in increasing index.
template <typename F>
__device__ __forceinline__ void for_near(int i, const float4* __restrict__ A, const CellsDev& cells, float rc2, F f) {
  const float4 ta = A[i];
  const int c = cells.cell_of[i];
  const int cz = c % cells.ncz, cy = (c / cells.ncz) % cells.ncy, cx = c / (cells.ncz * cells.ncy);
  for (int ax = max(cx - 1, 0); ax <= min(cx + 1, cells.ncx - 1); ++ax)
    for (int ay = max(cy - 1, 0); ay <= min(cy + 1, cells.ncy - 1); ++ay)
      for (int az = max(cz - 1, 0); az <= min(cz + 1, cells.ncz - 1); ++az) {
        const int cc = (ax * cells.ncy + ay) * cells.ncz + az;
        for (int64_t q = cells.start[cc]; q < cells.start[cc + 1]; ++q) {
          const int j = cells.nodes[q];
          const float4 sa = A[j];
          if (r2_f32(ta.x, ta.y, ta.z, sa.x, sa.y, sa.z) < rc2) f(j);
        }
      }
}

__global__ void __launch_bounds__(kBlock) k_near_count(int n, const float4* __restrict__ A, CellsDev cells, float rc2,
                                                       int64_t* __restrict__ counts) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int64_t c = 0;
  for_near(i, A, cells, rc2, [&](int) { ++c; });
  counts[i] = c;
}

// Near-field block matrix: for each near pair the FP64 coefficients of
//   y1_i += c0 ψ_j + c1 ψn_j,  y2_i += c2 ψ_j + c3 ψn_j,  with s_j = h³ω_j/(4π)
//   c0 = 4πK11 s_j, c1 = −4πK12 s_j, c2 = 4πK21 s_j, c3 = −4πK22 s_j.
// The coefficients depend on geometry only, so they are built once per band.
__global__ void __launch_bounds__(kBlock) k_near_fill(int n, BandDev b, const double* __restrict__ w, double scale,
                                                      const float4* __restrict__ A, CellsDev cells, float rc2,
                                                      KParams kp, const int64_t* __restrict__ row,
                                                      int* __restrict__ col, double4* __restrict__ coef) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double xi = b.px[i], yi = b.py[i], zi = b.pz[i], nxi = b.nx[i], nyi = b.ny[i], nzi = b.nz[i];
  int64_t q = row[i];
  for_near(i, A, cells, rc2, [&](int j) {
    double k[4];
    kern4_f64(xi, yi, zi, nxi, nyi, nzi, b.px[j], b.py[j], b.pz[j], b.nx[j], b.ny[j], b.nz[j], kp, k);
    const double sj = scale * w[j];
    col[q] = j;
    coef[q] = make_double4(k[0] * sj, -k[1] * sj, k[2] * sj, -k[3] * sj);
    ++q;
  });
}

constexpr int kRowLanes = 16;  // lanes cooperating on one CSR row

// near = (near block matrix)·p, 16 lanes per row, fixed-order lane reduction.
__global__ void __launch_bounds__(kBlock) k_near_spmv(int n, const int64_t* __restrict__ row,
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

// Number of source chunks so that the launch has at least ~8 blocks per CU.
int choose_chunks(pb_ctx* ctx, int n, int* chunk) {
  int tb = (n + kBlock - 1) / kBlock;
  int want = (8 * ctx->n_cu + tb - 1) / tb;
  int max_chunks = (n + kTileSrc - 1) / kTileSrc;
  int s = std::max(1, std::min(want, max_chunks));
  int c = (n + s - 1) / s;
  c = (c + kTileSrc - 1) / kTileSrc * kTileSrc;
  *chunk = c;
  return (n + c - 1) / c;
}

BandDev band_dev(const pb_band* b) { return BandDev{b->px, b->py, b->pz, b->nx, b->ny, b->nz}; }

}  // namespace

pb_status matvec_fp64(pb_ctx* ctx, const pb_band* band, const Derived& d, const double* p, double* y) {
  const int n = (int)band->n;
  int chunk = 0;
  const int S = choose_chunks(ctx, n, &chunk);
  double* wpsi = (double*)workspace(ctx, "mv_wpsi", sizeof(double) * n);
  double* wpsn = (double*)workspace(ctx, "mv_wpsn", sizeof(double) * n);
  double* partial = (double*)workspace(ctx, "mv_partial", sizeof(double) * 2 * (size_t)n * S);
  if (!wpsi || !wpsn || !partial) return PB_ENOMEM;
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  k_weights_f64<<<nb, kBlock, 0, ctx->stream>>>(n, band->w, p, d.h3 / (4.0 * kPi), wpsi, wpsn);
  {
    Scope t(ctx, "p2p_f64");
    k_p2p_f64<<<dim3(nb, S), kBlock, 0, ctx->stream>>>(band_dev(band), wpsi, wpsn, n, chunk, partial, kparams(d));
  }
  {
    Scope t(ctx, "reduce");
    k_reduce<<<(unsigned)((2 * n + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(n, S, partial, nullptr, p, d.lam1,
                                                                                    d.lam2, y);
  }
  return launch_ok(ctx, "matvec_fp64");
}

pb_status mixed_prepare(pb_ctx* ctx, const pb_band* band, const Derived& d) {
  const int n = (int)band->n;
  // bounding box of the projections
  const int nbb = 256;
  double* bb = (double*)workspace(ctx, "mx_bbox", sizeof(double) * 6 * nbb);
  if (!bb) return PB_ENOMEM;
  k_bbox<<<nbb, kBlock, 0, ctx->stream>>>(n, band_dev(band), bb);
  PB_TRY(launch_ok(ctx, "bbox"));
  std::vector<double> hb(6 * nbb);
  PB_HIP(ctx, hipMemcpyAsync(hb.data(), bb, sizeof(double) * 6 * nbb, hipMemcpyDeviceToHost, ctx->stream));
  PB_TRY(sync(ctx, "bbox"));
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int q = 0; q < nbb; ++q)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::fmin(lo[a], hb[6 * q + a]);
      hi[a] = std::fmax(hi[a], hb[6 * q + 3 + a]);
    }
  auto& P = ctx->mixed;
  P.band_key = band->px;
  P.n = n;
  P.cx = 0.5 * (lo[0] + hi[0]);
  P.cy = 0.5 * (lo[1] + hi[1]);
  P.cz = 0.5 * (lo[2] + hi[2]);
  P.rc = d.rc;
  P.rc2f = (float)(d.rc * d.rc);
  // cells at least r_c wide (with margin for FP32 rounding of the coordinates), at most 2^26 cells
  double cell = d.rc * 1.001 + 1e-4;
  for (;;) {
    double nc = 1.0;
    for (int a = 0; a < 3; ++a) nc *= std::floor((hi[a] - lo[a]) / cell) + 1.0;
    if (nc <= 67108864.0) break;
    cell *= 1.25;
  }
  P.cell = cell;
  P.ncx = (int)std::floor((hi[0] - lo[0]) / cell) + 1;
  P.ncy = (int)std::floor((hi[1] - lo[1]) / cell) + 1;
  P.ncz = (int)std::floor((hi[2] - lo[2]) / cell) + 1;
  const int64_t ncell = (int64_t)P.ncx * P.ncy * P.ncz;
  int64_t* start = (int64_t*)workspace(ctx, "mx_cell_start", sizeof(int64_t) * (size_t)(ncell + 1));
  int* cursor = (int*)workspace(ctx, "mx_cell_cursor", sizeof(int) * (size_t)ncell);
  int* nodes = (int*)workspace(ctx, "mx_cell_nodes", sizeof(int) * (size_t)n);
  int* cell_of = (int*)workspace(ctx, "mx_cell_of", sizeof(int) * (size_t)n);
  if (!start || !cursor || !nodes || !cell_of) return PB_ENOMEM;
  PB_HIP(ctx, hipMemsetAsync(start, 0, sizeof(int64_t) * (size_t)(ncell + 1), ctx->stream));
  PB_HIP(ctx, hipMemsetAsync(cursor, 0, sizeof(int) * (size_t)ncell, ctx->stream));
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  k_cell_count<<<nb, kBlock, 0, ctx->stream>>>(n, band_dev(band), lo[0], lo[1], lo[2], 1.0 / cell, P.ncx, P.ncy,
                                               P.ncz, cell_of, start);
  PB_TRY(launch_ok(ctx, "cell count"));
  PB_TRY(exclusive_scan_i64(ctx, start, ncell + 1, nullptr));
  k_cell_fill<<<nb, kBlock, 0, ctx->stream>>>(n, cell_of, start, cursor, nodes);
  k_cell_sort<<<(unsigned)((ncell + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(ncell, start, nodes);
  PB_TRY(launch_ok(ctx, "cell list"));

  // FP32 coordinates (weights zero) for the near predicate, then the near-field block matrix
  float4* A = (float4*)workspace(ctx, "mx_A", sizeof(float4) * n);
  float4* B = (float4*)workspace(ctx, "mx_B", sizeof(float4) * n);
  int64_t* row = (int64_t*)workspace(ctx, "mx_near_row", sizeof(int64_t) * (size_t)(n + 1));
  if (!A || !B || !row) return PB_ENOMEM;
  k_pack_f32<<<nb, kBlock, 0, ctx->stream>>>(n, band_dev(band), band->w, nullptr, 0.0, P.cx, P.cy, P.cz, A, B);
  const CellsDev cells{start, nodes, cell_of, P.ncx, P.ncy, P.ncz};
  PB_HIP(ctx, hipMemsetAsync(row + n, 0, sizeof(int64_t), ctx->stream));
  k_near_count<<<nb, kBlock, 0, ctx->stream>>>(n, A, cells, P.rc2f, row);
  PB_TRY(launch_ok(ctx, "near count"));
  int64_t nnz = 0;
  PB_TRY(exclusive_scan_i64(ctx, row, n + 1, &nnz));
  P.nnz = nnz;
  int* col = (int*)workspace(ctx, "mx_near_col", sizeof(int) * (size_t)std::max<int64_t>(nnz, 1));
  double4* coef = (double4*)workspace(ctx, "mx_near_coef", sizeof(double4) * (size_t)std::max<int64_t>(nnz, 1));
  if (!col || !coef) return PB_ENOMEM;
  k_near_fill<<<nb, kBlock, 0, ctx->stream>>>(n, band_dev(band), band->w, d.h3 / (4.0 * kPi), A, cells, P.rc2f,
                                              kparams(d), row, col, coef);
  return launch_ok(ctx, "near fill");
}

pb_status matvec_mixed(pb_ctx* ctx, const pb_band* band, const Derived& d, const double* p, double* y) {
  const int n = (int)band->n;
  const auto& P = ctx->mixed;
  if (P.band_key != band->px || P.n != n || P.rc != d.rc)
    return ctx->fail(PB_EINVAL, "mixed operator used before its geometry was prepared");
  int chunk = 0;
  const int S = choose_chunks(ctx, n, &chunk);
  float4* A = (float4*)workspace(ctx, "mx_A", sizeof(float4) * n);
  float4* B = (float4*)workspace(ctx, "mx_B", sizeof(float4) * n);
  double* partial = (double*)workspace(ctx, "mv_partial", sizeof(double) * 2 * (size_t)n * S);
  double* near = (double*)workspace(ctx, "mx_near", sizeof(double) * 2 * (size_t)n);
  if (!A || !B || !partial || !near) return PB_ENOMEM;
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  k_pack_f32<<<nb, kBlock, 0, ctx->stream>>>(n, band_dev(band), band->w, p, d.h3 / (4.0 * kPi), P.cx, P.cy, P.cz, A,
                                             B);
  F32Params fp{(float)d.th1, (float)d.th2, (float)d.kappa, (float)(-d.kappa * 1.4426950408889634)};
  {
    Scope t(ctx, "p2p_f32");
    k_p2p_f32<<<dim3(nb, S), kBlock, 0, ctx->stream>>>(A, B, n, chunk, P.rc2f, fp, partial);
  }
  {
    Scope t(ctx, "near_f64");
    k_near_spmv<<<(unsigned)(((int64_t)n * kRowLanes + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(
        n, (const int64_t*)ctx->bufs["mx_near_row"].ptr, (const int*)ctx->bufs["mx_near_col"].ptr,
        (const double4*)ctx->bufs["mx_near_coef"].ptr, p, near);
  }
  {
    Scope t(ctx, "reduce");
    k_reduce<<<(unsigned)((2 * n + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(n, S, partial, near, p, d.lam1,
                                                                                    d.lam2, y);
  }
  return launch_ok(ctx, "matvec_mixed");
}

}  // namespace pb

extern "C" pb_status pb_ibim_matvec(pb_ctx* ctx, const pb_band* band, const pb_params* prm, int precision,
                                    const double* p, double* y) {
  using namespace pb;
  if (!ctx) return PB_EINVAL;
  PB_TRY(check_params(ctx, prm));
  PB_TRY(check_band(ctx, band));
  if (!p || !y) return ctx->fail(PB_EINVAL, "pb_ibim_matvec: NULL vector");
  if (p == y) return ctx->fail(PB_EINVAL, "pb_ibim_matvec: p and y must not alias");
  if (precision != PB_FP64 && precision != PB_MIXED) return ctx->fail(PB_EINVAL, "unknown precision %d", precision);
  if (precision == PB_MIXED && prm->reg_metric == PB_REG_TANGENT)
    return ctx->fail(PB_EINVAL, "the mixed path needs a bounded regularization radius (guarded or Euclidean metric)");
  PB_HIP(ctx, hipSetDevice(ctx->device));
  Derived d = derive(*prm);
  if (precision == PB_MIXED) PB_TRY(mixed_prepare(ctx, band, d));
  PB_TRY(precision == PB_FP64 ? matvec_fp64(ctx, band, d, p, y) : matvec_mixed(ctx, band, d, p, y));
  return sync(ctx, "pb_ibim_matvec");
}
