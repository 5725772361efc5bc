// The IBIM operator y = Λp + KWp (eq. final-lin-sys) between the band nodes of one molecule.
//
// FP64 path: one target per lane, sources staged through LDS in tiles of 256, the source
// range split into chunks so that small bands still fill the 256 CUs; chunk partial sums are
// reduced in a fixed order (no atomics, bitwise reproducible).
//
// Mixed path: the FP32 far field (k_p2p_f32, rsq and exp2 on the transcendental unit, 32 B
// source records in LDS, FP32 partials per tile flushed to FP64) plus the FP64 near field, a
// CSR matrix of 2×2 blocks for every pair closer than r_c (≥ 2τ, so every regularized pair).
// Both sides decide "near" with the same FP32 function of the same FP32 records, so each pair
// is counted exactly once. The near matrix depends only on the geometry and is built once per
// band; each application is then an SpMV. The far kernel's tile shape (sources per LDS tile,
// targets per lane) is chosen per band size by timing the candidates once (autotuner); the
// symmetric kernel (each unordered pair once, both directions) is one of the candidates.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "pair_kernels.hpp"
#include "sym64_kernels.hpp"
#include "sym_kernels.hpp"

namespace pb {
namespace {

struct FarCfg {
  int tile, tpl;
};
constexpr FarCfg kFarCfgs[] = {{256, 1}, {512, 1}, {256, 2}, {512, 2}};
constexpr int kNumTiled = sizeof(kFarCfgs) / sizeof(kFarCfgs[0]);
constexpr int kSymCfg = kNumTiled;  // the symmetric kernel
constexpr int kNumFarCfgs = kNumTiled + 1;

// Work items (Ic, Jc), Ic ≤ Jc, of the symmetric kernel for a band of n nodes: off-diagonal
// chunk pairs first (they cost the most), the diagonal ones last.
std::vector<int2> sym_items(int n) {
  const int nc = sym_chunks(n);
  std::vector<int2> v;
  v.reserve((size_t)nc * (nc + 1) / 2);
  for (int i = 0; i < nc; ++i)
    for (int j = i + 1; j < nc; ++j) v.push_back(make_int2(i, j));
  for (int i = 0; i < nc; ++i) v.push_back(make_int2(i, i));
  return v;
}

// The item list on the device for a band of n nodes (rebuilt when n changes).
const int2* sym_items_dev(pb_ctx* ctx, int n, int* n_items) {
  const std::vector<int2> v = sym_items(n);
  int2* d = (int2*)workspace(ctx, "sym_items", sizeof(int2) * v.size());
  if (!d) return nullptr;
  if (ctx->sym_items_n != n) {
    if (hipMemcpyAsync(d, v.data(), sizeof(int2) * v.size(), hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
      return nullptr;
    ctx->sym_items_n = n;
    ctx->sym_n_items = (int)v.size();
  }
  *n_items = ctx->sym_n_items;
  return d;
}

// Source chunks for a launch: at least ~8 blocks per CU, chunks a multiple of the tile.
int far_chunks(pb_ctx* ctx, int n, int targets_per_block, int tile, int* chunk) {
  int tb = (n + targets_per_block - 1) / targets_per_block;
  int want = (8 * ctx->n_cu + tb - 1) / tb;
  int max_chunks = (n + tile - 1) / tile;
  int s = std::max(1, std::min(want, max_chunks));
  int c = (n + s - 1) / s;
  c = (c + tile - 1) / tile * tile;
  *chunk = c;
  return (n + c - 1) / c;
}

template <int TILE, int TPL>
int launch_far_t(pb_ctx* ctx, bool screened, const float4* A, const float4* M, const float4* N, const float4* box,
                 int n, const F32Params& fp, double sig1, double sig2, double* partial, const int* skip) {
  int chunk = 0;
  const int S = far_chunks(ctx, n, kBlock * TPL, TILE, &chunk);
  dim3 grid((unsigned)((n + kBlock * TPL - 1) / (kBlock * TPL)), (unsigned)S);
  if (screened)
    k_p2p_f32<TILE, TPL, true><<<grid, kBlock, 0, ctx->stream>>>(A, M, N, box, n, chunk, fp, sig1, sig2, partial, skip);
  else
    k_p2p_f32<TILE, TPL, false><<<grid, kBlock, 0, ctx->stream>>>(A, M, N, box, n, chunk, fp, sig1, sig2, partial, skip);
  return S;
}

int launch_far(pb_ctx* ctx, int cfg, bool screened, const float4* A, const float4* M, const float4* N,
               const float4* box, int n, const F32Params& fp, double sig1, double sig2, double* partial,
               const int* skip) {
  if (cfg == kSymCfg) {
    int n_items = 0;
    const int2* items = sym_items_dev(ctx, n, &n_items);
    if (!items) return -1;
    if (screened)
      k_p2p_f32_sym<true><<<(unsigned)n_items, kBlock, 0, ctx->stream>>>(A, N, box, n, sym_nsub(n), items,
                                                                          n_items, fp, sig1, sig2, partial, skip);
    else
      k_p2p_f32_sym<false><<<(unsigned)n_items, kBlock, 0, ctx->stream>>>(A, N, box, n, sym_nsub(n), items,
                                                                           n_items, fp, sig1, sig2, partial, skip);
    return sym_chunks(n);
  }
  switch (cfg) {
    case 0: return launch_far_t<256, 1>(ctx, screened, A, M, N, box, n, fp, sig1, sig2, partial, skip);
    case 1: return launch_far_t<512, 1>(ctx, screened, A, M, N, box, n, fp, sig1, sig2, partial, skip);
    case 2: return launch_far_t<256, 2>(ctx, screened, A, M, N, box, n, fp, sig1, sig2, partial, skip);
    default: return launch_far_t<512, 2>(ctx, screened, A, M, N, box, n, fp, sig1, sig2, partial, skip);
  }
}

int far_max_chunks(pb_ctx* ctx, int n) {
  int m = sym_chunks(n), c = 0;
  for (int k = 0; k < kNumTiled; ++k)
    m = std::max(m, far_chunks(ctx, n, kBlock * kFarCfgs[k].tpl, kFarCfgs[k].tile, &c));
  return m;
}

}  // namespace

// Bands from this size on take the symmetric kernels without timing: they were the faster
// ones at every band size timed (3281 to 638,391 nodes; 1.7× for FP32 and 1.8× for FP64 at
// the largest), and one timed one-directional launch costs seconds at millions of nodes.
constexpr int kTuneMaxN = 1 << 18;

// Picks the far-field tile shape for a band of n nodes by timing each candidate once on the
// packed records (after one warm-up launch); the choice is cached per n on the context.
// PB_FAR_CFG=<index> in the environment fixes the choice instead.
pb_status far_autotune(pb_ctx* ctx, int n, bool screened, const float4* A, const float4* M, const float4* N,
                       const float4* box, const F32Params& fp, double* partial, int* cfg_out) {
  auto it = ctx->far_cfg.find(n);
  if (it != ctx->far_cfg.end()) {
    *cfg_out = it->second;
    return PB_OK;
  }
  if (const char* env = std::getenv("PB_FAR_CFG")) {
    int c = std::atoi(env);
    if (c >= 0 && c < kNumFarCfgs) {
      ctx->far_cfg[n] = c;
      *cfg_out = c;
      return PB_OK;
    }
  }
  if (n >= kTuneMaxN) {
    ctx->far_cfg[n] = kSymCfg;
    *cfg_out = kSymCfg;
    return PB_OK;
  }
  hipEvent_t e0, e1;
  PB_HIP(ctx, hipEventCreate(&e0));
  PB_HIP(ctx, hipEventCreate(&e1));
  int best = 0;
  float best_ms = 1e30f;
  for (int c = 0; c < kNumFarCfgs; ++c) {
    if (launch_far(ctx, c, screened, A, M, N, box, n, fp, 1.0, 1.0, partial, nullptr) < 0)
      return ctx->fail(PB_ENOMEM, "far-field work list");
    PB_HIP(ctx, hipEventRecord(e0, ctx->stream));
    launch_far(ctx, c, screened, A, M, N, box, n, fp, 1.0, 1.0, partial, nullptr);
    PB_HIP(ctx, hipEventRecord(e1, ctx->stream));
    PB_TRY(launch_ok(ctx, "far autotune"));
    PB_HIP(ctx, hipEventSynchronize(e1));
    float ms = 0.f;
    PB_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->far_cfg[n] = best;
  *cfg_out = best;
  return PB_OK;
}

namespace {

// FP64 operator kernel: 0 = one target per lane over source chunks, 1 = symmetric.
int launch_f64(pb_ctx* ctx, int cfg, const pb_band* band, const double* wpsi, const double* wpsn, const KParams& kp,
               double* partial, const int* skip) {
  const int n = (int)band->n;
  if (cfg == 1) {
    int n_items = 0;
    const int2* items = sym_items_dev(ctx, n, &n_items);
    if (!items) return -1;
    k_p2p_f64_sym<<<(unsigned)n_items, kBlock, 0, ctx->stream>>>(band_dev(band), wpsi, wpsn, n, sym_nsub(n), items,
                                                                 n_items, kp, kp.kappa * kp.kappa, partial, skip);
    return sym_chunks(n);
  }
  int chunk = 0;
  const int S = far_chunks(ctx, n, kBlock, kBlock, &chunk);
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  k_p2p_f64<<<dim3(nb, S), kBlock, 0, ctx->stream>>>(band_dev(band, kp.curved), wpsi, wpsn, n, chunk, partial, kp,
                                                                     skip);
  return S;
}

// The FP64 kernel for bands of n nodes: timed once per n (PB_F64_CFG=<0|1> fixes it).
pb_status f64_autotune(pb_ctx* ctx, const pb_band* band, const double* wpsi, const double* wpsn, const KParams& kp,
                       double* partial, int* cfg_out) {
  const int n = (int)band->n;
  auto it = ctx->f64_cfg.find(n);
  if (it != ctx->f64_cfg.end()) {
    *cfg_out = it->second;
    return PB_OK;
  }
  if (const char* env = std::getenv("PB_F64_CFG")) {
    const int c = std::atoi(env);
    if (c == 0 || c == 1) {
      ctx->f64_cfg[n] = c;
      *cfg_out = c;
      return PB_OK;
    }
  }
  if (n >= kTuneMaxN) {
    ctx->f64_cfg[n] = 1;
    *cfg_out = 1;
    return PB_OK;
  }
  hipEvent_t e0, e1;
  PB_HIP(ctx, hipEventCreate(&e0));
  PB_HIP(ctx, hipEventCreate(&e1));
  int best = 0;
  float best_ms = 1e30f;
  for (int c = 0; c < 2; ++c) {
    PB_HIP(ctx, hipEventRecord(e0, ctx->stream));
    if (launch_f64(ctx, c, band, wpsi, wpsn, kp, partial, nullptr) < 0)
      return ctx->fail(PB_ENOMEM, "FP64 work list");
    PB_HIP(ctx, hipEventRecord(e1, ctx->stream));
    PB_TRY(launch_ok(ctx, "f64 autotune"));
    PB_HIP(ctx, hipEventSynchronize(e1));
    float ms = 0.f;
    PB_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->f64_cfg[n] = best;
  *cfg_out = best;
  return PB_OK;
}

}  // namespace

pb_status matvec_fp64(pb_ctx* ctx, const pb_band* band, const Derived& d, const double* p, double* y) {
  const int n = (int)band->n;
  int chunk = 0;
  const int S64 = std::max(far_chunks(ctx, n, kBlock, kBlock, &chunk), sym_chunks(n));
  double* wpsi = (double*)workspace(ctx, "mv_wpsi", sizeof(double) * n);
  double* wpsn = (double*)workspace(ctx, "mv_wpsn", sizeof(double) * n);
  double* partial = (double*)workspace(ctx, "mv_partial64", sizeof(double) * 2 * (size_t)n * S64);
  if (!wpsi || !wpsn || !partial) return PB_ENOMEM;
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  k_weights_f64<<<nb, kBlock, 0, ctx->stream>>>(n, band->w, p, d.h3 / (4.0 * kPi), wpsi, wpsn);
  const KParams kp = kparams(d);
  int cfg = 0;  // the symmetric kernel takes the paper's disc averages only
  if (!d.curved) PB_TRY(f64_autotune(ctx, band, wpsi, wpsn, kp, partial, &cfg));
  int S = 0;
  {
    Scope t(ctx, "p2p_f64");
    S = launch_f64(ctx, cfg, band, wpsi, wpsn, kp, partial, ctx->skip);
  }
  if (S < 0) return ctx->fail(PB_ENOMEM, "FP64 work list");
  {
    Scope t(ctx, "reduce");
    k_reduce<<<(unsigned)((2 * n + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(n, S, partial, nullptr, p, d.lam1,
                                                                                    d.lam2, y);
  }
  return launch_ok(ctx, "matvec_fp64");
}

F32Params f32params(const Derived& d, double sigma) {
  const double rcs = sigma * d.rc;
  return F32Params{(float)d.th1, (float)d.th2, (float)(-1.4426950408889634), (float)(rcs * rcs),
                   (float)(rcs * rcs * 1.001)};
}

// Geometry of the mixed operator for one band: centre and scale of the FP32 records, the
// cell list and the FP64 near-field CSR matrix. Buffers are named `<pfx>...` in the context
// workspace; the plan receives the sizes and pointers.
pb_status near_build(pb_ctx* ctx, const pb_band* band, const Derived& d, const char* pfx, MixedPlan& P,
                     bool cells_only) {
  const int n = (int)band->n;
  auto name = [&](const char* s) {
    static thread_local char buf[64];
    snprintf(buf, sizeof(buf), "%s%s", pfx, s);
    return (const char*)buf;
  };
  const int nbb = 256;
  double* bb = (double*)workspace(ctx, name("bbox"), sizeof(double) * 6 * nbb);
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
  P.band_key = band->px;
  P.n = n;
  P.cx = 0.5 * (lo[0] + hi[0]);
  P.cy = 0.5 * (lo[1] + hi[1]);
  P.cz = 0.5 * (lo[2] + hi[2]);
  P.sigma = d.kappa > 0.0 ? d.kappa : 1.0;
  P.rc = d.rc;
  P.rc2f = f32params(d, P.sigma).rc2;
  // cells at least r_c wide (margin for the FP32 rounding of the coordinates), at most 2^26 cells
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
  int64_t* start = (int64_t*)workspace(ctx, name("cell_start"), sizeof(int64_t) * (size_t)(ncell + 1));
  int* cursor = (int*)workspace(ctx, name("cell_cursor"), sizeof(int) * (size_t)ncell);
  int* nodes = (int*)workspace(ctx, name("cell_nodes"), sizeof(int) * (size_t)n);
  int* cell_of = (int*)workspace(ctx, name("cell_of"), sizeof(int) * (size_t)n);
  float4* A = (float4*)workspace(ctx, name("A"), sizeof(float4) * n);
  float4* M = (float4*)workspace(ctx, name("M"), sizeof(float4) * n);
  float4* N = (float4*)workspace(ctx, name("N"), sizeof(float4) * n);
  const int ngroup = (n + kGroup - 1) / kGroup;
  float4* box = (float4*)workspace(ctx, name("box"), sizeof(float4) * 2 * (size_t)ngroup);
  int64_t* row = (int64_t*)workspace(ctx, name("near_row"), sizeof(int64_t) * (size_t)(n + 1));
  if (!start || !cursor || !nodes || !cell_of || !A || !M || !N || !box || !row) return PB_ENOMEM;
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
  if (cells_only) return PB_OK;
  // FP32 records (weights zero) for the near predicate, then the near-field block matrix
  k_pack_f32<<<nb, kBlock, 0, ctx->stream>>>(n, band_dev(band), band->w, nullptr, 0.0, P.cx, P.cy, P.cz, P.sigma, A,
                                             M, N);
  k_group_box<<<(unsigned)ngroup, kGroup, 0, ctx->stream>>>(n, A, box);
  const CellsDev cells{start, nodes, cell_of, P.ncx, P.ncy, P.ncz};
  PB_HIP(ctx, hipMemsetAsync(row + n, 0, sizeof(int64_t), ctx->stream));
  const unsigned nbw = (unsigned)((n + kNearWaves - 1) / kNearWaves);
  k_near_count<<<nbw, kBlock, 0, ctx->stream>>>(n, A, cells, P.rc2f, row);
  PB_TRY(launch_ok(ctx, "near count"));
  int64_t nnz = 0;
  PB_TRY(exclusive_scan_i64(ctx, row, n + 1, &nnz));
  P.nnz = nnz;
  int* col = (int*)workspace(ctx, name("near_col"), sizeof(int) * (size_t)std::max<int64_t>(nnz, 1));
  double4* coef = (double4*)workspace(ctx, name("near_coef"), sizeof(double4) * (size_t)std::max<int64_t>(nnz, 1));
  if (!col || !coef) return PB_ENOMEM;
  k_near_fill<<<nbw, kBlock, 0, ctx->stream>>>(n, band_dev(band, d.curved), band->w, d.h3 / (4.0 * kPi), A, cells,
                                               P.rc2f, kparams(d), row, col, coef);
  PB_TRY(launch_ok(ctx, "near fill"));
  P.A = A;
  P.M = M;
  P.N = N;
  P.box = box;
  P.row = row;
  P.col = col;
  P.coef = coef;
  return PB_OK;
}

pb_status mixed_prepare(pb_ctx* ctx, const pb_band* band, const Derived& d) {
  PB_TRY(near_build(ctx, band, d, "mx_", ctx->mixed));
  const int n = (int)band->n;
  MixedPlan& P = ctx->mixed;
  double* partial = (double*)workspace(ctx, "mv_partial", sizeof(double) * 2 * (size_t)n * far_max_chunks(ctx, n));
  if (!partial) return PB_ENOMEM;
  return far_autotune(ctx, n, d.kappa > 0.0, P.A, P.M, P.N, P.box, f32params(d, P.sigma), partial, &P.far_cfg);
}

pb_status matvec_mixed(pb_ctx* ctx, const pb_band* band, const Derived& d, const double* p, double* y) {
  const int n = (int)band->n;
  const MixedPlan& P = ctx->mixed;
  if (P.band_key != band->px || P.n != n || P.rc != d.rc)
    return ctx->fail(PB_EINVAL, "mixed operator used before its geometry was prepared");
  double* partial = (double*)workspace(ctx, "mv_partial", sizeof(double) * 2 * (size_t)n * far_max_chunks(ctx, n));
  double* near = (double*)workspace(ctx, "mx_near", sizeof(double) * 2 * (size_t)n);
  if (!partial || !near) return PB_ENOMEM;
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  k_pack_f32<<<nb, kBlock, 0, ctx->stream>>>(n, band_dev(band), band->w, p, d.h3 / (4.0 * kPi), P.cx, P.cy, P.cz,
                                             P.sigma, P.A, P.M, P.N);
  int S;
  {
    Scope t(ctx, "p2p_f32");
    S = launch_far(ctx, P.far_cfg, d.kappa > 0.0, P.A, P.M, P.N, P.box, n, f32params(d, P.sigma), P.sigma,
                   P.sigma * P.sigma, partial, ctx->skip);
  }
  if (S < 0) return ctx->fail(PB_ENOMEM, "far-field work list");
  {
    Scope t(ctx, "near_f64");
    k_near_spmv<<<(unsigned)(((int64_t)n * kRowLanes + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(
        n, P.row, P.col, P.coef, p, near);
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
  if (precision != PB_FP64 && precision != PB_MIXED && precision != PB_TREE)
    return ctx->fail(PB_EINVAL, "unknown precision %d", precision);
  if (precision != PB_FP64 && prm->reg_metric == PB_REG_TANGENT)
    return ctx->fail(PB_EINVAL, "the mixed path needs a bounded regularization radius (guarded or Euclidean metric)");
  PB_TRY(check_curv(ctx, band, prm));
  PB_HIP(ctx, hipSetDevice(ctx->device));
  Derived d = derive(*prm);
  if (precision == PB_FP64) {
    PB_TRY(matvec_fp64(ctx, band, d, p, y));
  } else if (precision == PB_MIXED) {
    PB_TRY(mixed_prepare(ctx, band, d));
    PB_TRY(matvec_mixed(ctx, band, d, p, y));
  } else {
    PB_TRY(tree_prepare(ctx, band, d, prm->tree_degree, prm->tree_theta, ctx->tree, "tc_"));
    PB_TRY(matvec_tree(ctx, band, d, p, y, ctx->tree));
  }
  return sync(ctx, "pb_ibim_matvec");
}
