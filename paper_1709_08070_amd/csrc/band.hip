// Stage 2: order-preserving compaction of the narrow band −ε < φ < ε, with the
// closest-point projection x* = x − φ n, n = ∇φ/|∇φ| (central differences, or the average
// of the two WENO5 one-sided derivatives per axis) and the weight ω = δ_ε(φ)·J
// (eq. cosine-kernel; J ≡ 1 or the explicit J of section "Implicit boundary integral
// methods", read with the adjugate of the Hessian), and, when asked for, the curvature sum
// κ1 + κ2 of the surface at x*.
//
// Three passes over the grid, each block owning one contiguous tile of kTile linear
// indices: count the band nodes of each tile, scan the tile counts, then scatter. Inside a
// tile the rank of a node is its wave-ballot prefix plus the counts of the waves before it,
// so the output is in increasing linear index with no atomics.
#include <cmath>

#include "pb_internal.hpp"
#include "stencil.hpp"

#pragma clang fp contract(off)

namespace pb {
namespace {

constexpr int kBlock = 256;
constexpr int kPerThread = 16;
constexpr int64_t kTile = (int64_t)kBlock * kPerThread;

struct GridDev {
  int nx, ny, nz;
  double ox, oy, oz, h;
};

__device__ __forceinline__ bool in_band(double f, double eps) { return f > -eps && f < eps; }

__global__ void __launch_bounds__(kBlock) k_count(const double* __restrict__ phi, int64_t total, double eps,
                                                  int64_t* __restrict__ counts) {
  __shared__ int s[kBlock / 64];
  int64_t base = (int64_t)blockIdx.x * kTile;
  int c = 0;
  for (int r = 0; r < kPerThread; ++r) {
    int64_t id = base + (int64_t)r * kBlock + threadIdx.x;
    if (id < total && in_band(phi[id], eps)) ++c;
  }
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kBlock / 64; ++w) t += s[w];
    counts[blockIdx.x] = t;
  }
}

// (p₋ + p₊)/2 along one axis: WENO5 one-sided derivatives of φ at node id (coordinate c of
// n along the axis, stride st), ghosts by even reflection about the boundary node as in the
// level-set stage. ih = 1/h.
__device__ double weno_average(const double* __restrict__ phi, int64_t id, int64_t c, int64_t n, int64_t st,
                               double ih) {
  double f[7];
  for (int s = -3; s <= 3; ++s) {
    int64_t q = c + s;
    q = q < 0 ? -q : (q > n - 1 ? 2 * (n - 1) - q : q);
    f[s + 3] = phi[id + (q - c) * st];
  }
  double D[6];
  for (int m = 0; m < 6; ++m) D[m] = (f[m + 1] - f[m]) * ih;
  const double a = weno5(D[0], D[1], D[2], D[3], D[4]);
  const double b = weno5(D[5], D[4], D[3], D[2], D[1]);
  return (a + b) * 0.5;
}

// tr(H) and nᵀ adj(H) n at an interior node, H the central-difference Hessian of φ (mixed
// terms from the four diagonal neighbours), adj(H) the adjugate of the symmetric H.
__device__ void hessian_terms(const double* __restrict__ phi, int64_t id, int64_t si, int64_t sj, double h, double f,
                              double nx, double ny, double nz, double* tr, double* q) {
  const double ih2 = 1.0 / (h * h), iq = 0.25 * ih2;
  const double hxx = (phi[id + si] - 2.0 * f + phi[id - si]) * ih2;
  const double hyy = (phi[id + sj] - 2.0 * f + phi[id - sj]) * ih2;
  const double hzz = (phi[id + 1] - 2.0 * f + phi[id - 1]) * ih2;
  const double hxy = (phi[id + si + sj] - phi[id + si - sj] - phi[id - si + sj] + phi[id - si - sj]) * iq;
  const double hxz = (phi[id + si + 1] - phi[id + si - 1] - phi[id - si + 1] + phi[id - si - 1]) * iq;
  const double hyz = (phi[id + sj + 1] - phi[id + sj - 1] - phi[id - sj + 1] + phi[id - sj - 1]) * iq;
  const double axx = hyy * hzz - hyz * hyz, ayy = hxx * hzz - hxz * hxz, azz = hxx * hyy - hxy * hxy;
  const double axy = hxz * hyz - hxy * hzz, axz = hxy * hyz - hxz * hyy, ayz = hxy * hxz - hxx * hyz;
  *q = axx * nx * nx + ayy * ny * ny + azz * nz * nz + 2.0 * (axy * nx * ny + axz * nx * nz + ayz * ny * nz);
  *tr = hxx + hyy + hzz;
}

__global__ void __launch_bounds__(kBlock) k_scatter(GridDev g, const double* __restrict__ phi, double eps,
                                                    int grad_scheme, int full_jacobian,
                                                    const int64_t* __restrict__ offsets, int64_t capacity,
                                                    pb_band band, int* __restrict__ bad) {
  __shared__ int wave_cnt[kBlock / 64];
  int64_t total = (int64_t)g.nx * g.ny * g.nz;
  int64_t base = (int64_t)blockIdx.x * kTile;
  int64_t run = offsets[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = 0; r < kPerThread; ++r) {
    int64_t id = base + (int64_t)r * kBlock + threadIdx.x;
    double f = id < total ? phi[id] : 0.0;
    bool sel = id < total && in_band(f, eps);
    uint64_t mask = __ballot(sel);
    int before = __popcll(mask & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
    if (lane == 0) wave_cnt[wave] = __popcll(mask);
    __syncthreads();
    int64_t pos = run + before;
    for (int w = 0; w < wave; ++w) pos += wave_cnt[w];
    int64_t round_total = 0;
    for (int w = 0; w < kBlock / 64; ++w) round_total += wave_cnt[w];
    __syncthreads();
    run += round_total;
    if (!sel || pos >= capacity) continue;
    int64_t k = id % g.nz, j = (id / g.nz) % g.ny, i = id / ((int64_t)g.ny * g.nz);
    if (i == 0 || j == 0 || k == 0 || i == g.nx - 1 || j == g.ny - 1 || k == g.nz - 1) {
      atomicOr(bad, 1);
      continue;
    }
    const int64_t si = (int64_t)g.ny * g.nz, sj = g.nz;
    double gx, gy, gz;
    if (grad_scheme == PB_GRAD_WENO) {
      const double ih = 1.0 / g.h;
      gx = weno_average(phi, id, i, g.nx, si, ih);
      gy = weno_average(phi, id, j, g.ny, sj, ih);
      gz = weno_average(phi, id, k, g.nz, 1, ih);
    } else {
      gx = (phi[id + si] - phi[id - si]) / (2.0 * g.h);
      gy = (phi[id + sj] - phi[id - sj]) / (2.0 * g.h);
      gz = (phi[id + 1] - phi[id - 1]) / (2.0 * g.h);
    }
    double gn = sqrt((gx * gx + gy * gy) + gz * gz);
    if (!(gn > 0.0)) {
      atomicOr(bad, 2);
      continue;
    }
    double nx = gx / gn, ny = gy / gn, nz = gz / gn;
    band.px[pos] = g.ox + g.h * (double)i - f * nx;
    band.py[pos] = g.oy + g.h * (double)j - f * ny;
    band.pz[pos] = g.oz + g.h * (double)k - f * nz;
    band.nx[pos] = nx;
    band.ny[pos] = ny;
    band.nz[pos] = nz;
    band.phi[pos] = f;
    double w = (1.0 + cos(kPi * f / eps)) / (2.0 * eps);
    if (full_jacobian || band.curv) {
      // J = 1 − φ tr(H) + φ² nᵀadj(H)n; the level set through the node has curvature sum tr(H)
      // and product nᵀadj(H)n, and moving back by φ gives κ1 + κ2 = (tr(H) − 2φ nᵀadj(H)n)/J at x*
      double tr, q;
      hessian_terms(phi, id, si, sj, g.h, f, nx, ny, nz, &tr, &q);
      const double J = 1.0 - f * tr + f * f * q;
      if (full_jacobian) w *= J;
      if (band.curv) band.curv[pos] = (tr - 2.0 * f * q) / J;
    }
    band.w[pos] = w;
    if (band.gidx) band.gidx[pos] = id;
  }
}

}  // namespace
}  // namespace pb

extern "C" pb_status pb_narrowband_compact(pb_ctx* ctx, const pb_grid* grid, const double* phi, const pb_params* prm,
                                           pb_band* band) {
  using namespace pb;
  if (!ctx) return PB_EINVAL;
  PB_TRY(check_params(ctx, prm));
  if (!grid || !phi || !band) return ctx->fail(PB_EINVAL, "pb_narrowband_compact: NULL argument");
  if (band->capacity < 0) return ctx->fail(PB_EINVAL, "pb_narrowband_compact: negative capacity");
  if (band->capacity > 0 && (!band->px || !band->py || !band->pz || !band->nx || !band->ny || !band->nz ||
                             !band->phi || !band->w))
    return ctx->fail(PB_EINVAL, "pb_narrowband_compact: band arrays must be non-NULL");
  if (grid->nx < 3 || grid->ny < 3 || grid->nz < 3) return ctx->fail(PB_EINVAL, "grid too small");
  PB_HIP(ctx, hipSetDevice(ctx->device));
  GridDev g{grid->nx, grid->ny, grid->nz, grid->origin[0], grid->origin[1], grid->origin[2], grid->h};
  int64_t total = (int64_t)g.nx * g.ny * g.nz;
  int64_t nb = (total + kTile - 1) / kTile;
  const double eps = prm->band_k * prm->h;
  int64_t* counts = (int64_t*)workspace(ctx, "band_counts", sizeof(int64_t) * (size_t)nb);
  int* bad = (int*)workspace(ctx, "band_bad", sizeof(int));
  if (!counts || !bad) return PB_ENOMEM;
  {
    Scope t(ctx, "band");
    k_count<<<(unsigned)nb, kBlock, 0, ctx->stream>>>(phi, total, eps, counts);
  }
  PB_TRY(launch_ok(ctx, "band count"));
  int64_t n = 0;
  PB_TRY(exclusive_scan_i64(ctx, counts, nb, &n));
  if (n > band->capacity) {
    band->n = n;
    return ctx->fail(PB_ECAPACITY, "band needs %lld nodes, capacity %lld", (long long)n, (long long)band->capacity);
  }
  PB_HIP(ctx, hipMemsetAsync(bad, 0, sizeof(int), ctx->stream));
  {
    Scope t(ctx, "band");
    k_scatter<<<(unsigned)nb, kBlock, 0, ctx->stream>>>(g, phi, eps, prm->grad_scheme, prm->jacobian, counts,
                                                        band->capacity, *band, bad);
  }
  PB_TRY(launch_ok(ctx, "band scatter"));
  int badh = 0;
  PB_HIP(ctx, hipMemcpyAsync(&badh, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  PB_TRY(sync(ctx, "pb_narrowband_compact"));
  band->n = n;
  if (badh & 1) return ctx->fail(PB_EGEOM, "a band node lies on the grid edge; enlarge the grid margin");
  if (badh & 2) return ctx->fail(PB_EGEOM, "zero level-set gradient at a band node");
  if (n == 0) return ctx->fail(PB_EGEOM, "the band is empty");
  return PB_OK;
}
