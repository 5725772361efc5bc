// Context, parameters, validation, workspace, timing and the shared scan.
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "pb_internal.hpp"

pb_status pb_ctx::fail(pb_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  err = buf;
  return s;
}

namespace pb {

Derived derive(const pb_params& p) {
  Derived d{};
  d.h = p.h;
  d.h3 = p.h * p.h * p.h;
  d.eps = p.band_k * p.h;
  d.tau = p.tau_k * p.h;
  d.tau2 = d.tau * d.tau;
  d.four_tau2 = 4.0 * d.tau * d.tau;
  d.th1 = p.eps_out / p.eps_in;
  d.th2 = p.eps_in / p.eps_out;
  d.lam1 = 0.5 * (1.0 + d.th1);
  d.lam2 = 0.5 * (1.0 + d.th2);
  d.kappa = p.kappa;
  d.eps_in = p.eps_in;
  // mean of (1 − e^{−κρ})/(4πρ) over the tangent disc of radius τ (eq. reg-kernel-a)
  d.k12bar = p.kappa == 0.0 ? 0.0 : (std::exp(-p.kappa * d.tau) - 1.0 + p.kappa * d.tau) /
                                        (2.0 * kPi * p.kappa * d.tau * d.tau);
  // near-field radius; the margin keeps every pair with r < 2τ inside it after FP32 rounding
  d.rc = std::fmax(p.near_k * p.h, 2.0 * d.tau) * (1.0 + 1e-4);
  d.metric = p.reg_metric;
  // curvature-corrected disc averages (PB_AVG_CURVED), times 4π as the kernels use them:
  // 4πK̄11 = k11c·c, 4πK̄22 = k22c·c (c = κ1 + κ2 at the target), 4πK̄21 = k21bar4pi
  d.curved = p.reg_avg == PB_AVG_CURVED;
  if (d.curved) {
    const double kt = p.kappa * d.tau;
    const double abar = p.kappa == 0.0 ? 1.0 : (2.0 - (2.0 + kt) * std::exp(-kt)) / kt;
    d.k11c = -(1.0 - d.th1 * abar) / (2.0 * d.tau);
    d.k22c = -(1.0 - d.th2 * abar) / (2.0 * d.tau);
    d.k21bar4pi = 2.0 * (std::exp(-kt) - 1.0 + kt) / (d.tau * d.tau * d.tau);
  }
  return d;
}

void* workspace(pb_ctx* ctx, const char* name, size_t bytes) {
  DevBuf& b = ctx->bufs[name];
  if (b.bytes >= bytes && b.ptr) return b.ptr;
  if (b.ptr) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
  }
  size_t want = bytes < 256 ? 256 : bytes;
  if (hipMalloc(&b.ptr, want) != hipSuccess) {
    b.ptr = nullptr;
    ctx->fail(PB_ENOMEM, "workspace '%s': cannot allocate %zu bytes", name, want);
    return nullptr;
  }
  b.bytes = want;
  return b.ptr;
}

static hipEvent_t get_event(pb_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e{};
  (void)hipEventCreate(&e);
  return e;
}

// The far-field families: what timing level 2 measures (events around every other launch
// would add their own gaps to a timed run).
static bool far_family(const char* n) {
  return !std::strcmp(n, "p2p_f32") || !std::strcmp(n, "p2p_f64") || !std::strcmp(n, "tree_f32") ||
         !std::strcmp(n, "tree_fine_f32");
}

Scope::Scope(pb_ctx* c, const char* n)
    : ctx(c), name(n), on(c->timing == 1 || (c->timing == 2 && far_family(n))) {
  if (!on) return;
  a = get_event(ctx);
  b = get_event(ctx);
  (void)hipEventRecord(a, ctx->stream);
}

Scope::~Scope() {
  if (!on) return;
  (void)hipEventRecord(b, ctx->stream);
  ctx->pending.emplace_back(a, b);
  ctx->pending_name.emplace_back(name);
  if (ctx->pending.size() > 32768) {
    (void)hipStreamSynchronize(ctx->stream);
    flush_timers(ctx);
  }
}

void flush_timers(pb_ctx* ctx) {
  for (size_t i = 0; i < ctx->pending.size(); ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->pending[i].first, ctx->pending[i].second) == hipSuccess) {
      Timer& t = ctx->timers[ctx->pending_name[i]];
      t.ms += ms;
      t.launches += 1;
    }
    ctx->event_pool.push_back(ctx->pending[i].first);
    ctx->event_pool.push_back(ctx->pending[i].second);
  }
  ctx->pending.clear();
  ctx->pending_name.clear();
}

void drop_timers(pb_ctx* ctx, size_t mark) {
  for (size_t i = mark; i < ctx->pending.size(); ++i) {
    ctx->event_pool.push_back(ctx->pending[i].first);
    ctx->event_pool.push_back(ctx->pending[i].second);
  }
  if (mark < ctx->pending.size()) {
    ctx->pending.resize(mark);
    ctx->pending_name.resize(mark);
  }
}

pb_status sync(pb_ctx* ctx, const char* where) {
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return ctx->fail(PB_EDEVICE, "%s: stream synchronize: %s", where, hipGetErrorString(e));
  if (ctx->timing) flush_timers(ctx);
  return PB_OK;
}

pb_status launch_ok(pb_ctx* ctx, const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ctx->fail(PB_EDEVICE, "%s: launch failed: %s", where, hipGetErrorString(e));
  return PB_OK;
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

pb_status check_params(pb_ctx* ctx, const pb_params* p) {
  if (!p) return ctx->fail(PB_EINVAL, "params is NULL");
  if (!finite_pos(p->eps_in) || !finite_pos(p->eps_out))
    return ctx->fail(PB_EINVAL, "dielectric constants must be finite and positive");
  if (!std::isfinite(p->kappa) || p->kappa < 0.0) return ctx->fail(PB_EINVAL, "kappa must be finite and >= 0");
  if (!finite_pos(p->h) || !finite_pos(p->band_k) || !finite_pos(p->tau_k))
    return ctx->fail(PB_EINVAL, "h, band_k and tau_k must be finite and positive");
  if (!finite_pos(p->cfl) || p->cfl > 0.5) return ctx->fail(PB_EINVAL, "cfl must be in (0, 0.5]");
  if (!std::isfinite(p->probe) || p->probe < 0.0) return ctx->fail(PB_EINVAL, "probe radius must be >= 0");
  if (!std::isfinite(p->near_k) || p->near_k < 0.0) return ctx->fail(PB_EINVAL, "near_k must be >= 0");
  if (p->reg_metric < 0 || p->reg_metric > 2) return ctx->fail(PB_EINVAL, "unknown reg_metric %d", p->reg_metric);
  if (p->ls_mode < 0 || p->ls_mode > 1) return ctx->fail(PB_EINVAL, "unknown ls_mode %d", p->ls_mode);
  if (p->reinit_steps < 0) return ctx->fail(PB_EINVAL, "reinit_steps must be >= 0");
  if (p->grad_scheme < 0 || p->grad_scheme > 1) return ctx->fail(PB_EINVAL, "unknown grad_scheme %d", p->grad_scheme);
  if (p->jacobian < 0 || p->jacobian > 1) return ctx->fail(PB_EINVAL, "unknown jacobian %d", p->jacobian);
  if (!(p->tree_theta > 0.0 && p->tree_theta < 1.0)) return ctx->fail(PB_EINVAL, "tree_theta must be in (0, 1)");
  if (p->tree_degree < 2 || p->tree_degree > kTreeMaxDegree)
    return ctx->fail(PB_EINVAL, "tree_degree must be in [2, %d]", kTreeMaxDegree);
  if (p->reg_avg < 0 || p->reg_avg > 1) return ctx->fail(PB_EINVAL, "unknown reg_avg %d", p->reg_avg);
  return PB_OK;
}

pb_status check_curv(pb_ctx* ctx, const pb_band* b, const pb_params* p) {
  if (p->reg_avg == PB_AVG_CURVED && !b->curv)
    return ctx->fail(PB_EINVAL, "reg_avg PB_AVG_CURVED needs band->curv (written by pb_narrowband_compact)");
  return PB_OK;
}

pb_status check_band(pb_ctx* ctx, const pb_band* b) {
  if (!b) return ctx->fail(PB_EINVAL, "band is NULL");
  if (b->n <= 0) return ctx->fail(PB_EGEOM, "band is empty");
  if (b->n > b->capacity) return ctx->fail(PB_EINVAL, "band n exceeds capacity");
  if (!b->px || !b->py || !b->pz || !b->nx || !b->ny || !b->nz || !b->w)
    return ctx->fail(PB_EINVAL, "band arrays must be non-NULL");
  if (b->n > (int64_t)1 << 31) return ctx->fail(PB_EINVAL, "band larger than 2^31 nodes");
  return PB_OK;
}

// ---------------------------------------------------------------- scan

constexpr int kScanBlock = 256;

// Per-block inclusive scan of a segment; writes the block total to sums.
__global__ void __launch_bounds__(kScanBlock) k_scan_blocks(int64_t* data, int64_t n, int64_t* sums) {
  __shared__ int64_t s[kScanBlock];
  int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  int64_t v = i < n ? data[i] : 0;
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int64_t t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < n) data[i] = s[threadIdx.x] - v;  // exclusive within block
  if (threadIdx.x == kScanBlock - 1) sums[blockIdx.x] = s[threadIdx.x];
}

__global__ void __launch_bounds__(kScanBlock) k_scan_add(int64_t* data, int64_t n, const int64_t* offs) {
  int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  if (i < n) data[i] += offs[blockIdx.x];
}

// Recursive exclusive scan; total = sum of all inputs.
static pb_status scan_rec(pb_ctx* ctx, int64_t* data, int64_t n, int64_t* total_dev, int depth) {
  int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  char name[32];
  snprintf(name, sizeof(name), "scan_sums%d", depth);
  int64_t* sums = (int64_t*)workspace(ctx, name, sizeof(int64_t) * (size_t)(nb + 1));
  if (!sums) return PB_ENOMEM;
  k_scan_blocks<<<(unsigned)nb, kScanBlock, 0, ctx->stream>>>(data, n, sums);
  PB_TRY(launch_ok(ctx, "scan"));
  if (nb == 1) {
    PB_HIP(ctx, hipMemcpyAsync(total_dev, sums, sizeof(int64_t), hipMemcpyDeviceToDevice, ctx->stream));
    return PB_OK;
  }
  PB_TRY(scan_rec(ctx, sums, nb, total_dev, depth + 1));
  k_scan_add<<<(unsigned)nb, kScanBlock, 0, ctx->stream>>>(data, n, sums);
  return launch_ok(ctx, "scan_add");
}

pb_status exclusive_scan_i64(pb_ctx* ctx, int64_t* data, int64_t n, int64_t* total_host) {
  int64_t* tot = (int64_t*)workspace(ctx, "scan_total", sizeof(int64_t));
  if (!tot) return PB_ENOMEM;
  PB_TRY(scan_rec(ctx, data, n, tot, 0));
  if (total_host) {
    PB_HIP(ctx, hipMemcpyAsync(total_host, tot, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    PB_TRY(sync(ctx, "scan"));
  }
  return PB_OK;
}

}  // namespace pb

// ---------------------------------------------------------------- C-ABI

extern "C" {

pb_status pb_create(pb_ctx** out, int device, void* hip_stream) {
  if (!out) return PB_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return PB_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return PB_EDEVICE;
  pb_ctx* c = new pb_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
  if (pb::noalloc_init(c) != PB_OK) {
    delete c;
    return PB_EDEVICE;
  }
  *out = c;
  return PB_OK;
}

void pb_destroy(pb_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& kv : ctx->bufs)
    if (kv.second.ptr) (void)hipFree(kv.second.ptr);
  for (auto& e : ctx->pending) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
  if (ctx->host_state) (void)hipHostFree(ctx->host_state);
  if (ctx->batch_stream) {
    (void)hipStreamSynchronize(ctx->batch_stream);
    (void)hipStreamDestroy(ctx->batch_stream);
  }
  delete ctx;
}

const char* pb_last_error(const pb_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

void pb_default_params(pb_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->eps_in = 1.0;
  p->eps_out = 80.0;
  p->kappa = 0.1257;
  p->probe = 1.4;
  p->h = 0.5;
  p->band_k = 2.0;
  p->tau_k = 1.0;
  p->cfl = 0.3;
  p->near_k = 2.0;
  p->reg_metric = PB_REG_TANGENT_GUARDED;
  p->grad_scheme = PB_GRAD_WENO;
  p->jacobian = PB_JAC_ONE;
  p->tree_theta = 0.6;
  p->tree_degree = 4;
  p->reg_avg = PB_AVG_FLAT;
  p->ls_mode = PB_LS_SES;
  p->reinit_steps = 0;
}

void pb_default_solve_opts(pb_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-6;
  o->max_iter = 500;
  o->restart = 100;
  o->precision = PB_FP64;
  o->x0 = PB_X0_DIAG;
  o->precond = PB_PRECOND_NONE;
  o->max_outer = 5;
  o->nn = nullptr;
}

pb_status pb_grid_for_atoms(const double* atoms, int n_atoms, const pb_params* prm, pb_grid* grid) {
  if (!atoms || n_atoms <= 0 || !prm || !grid) return PB_EINVAL;
  if (!std::isfinite(prm->h) || prm->h <= 0) return PB_EINVAL;
  double rmax = 0.0;
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) lo[a] = hi[a] = atoms[a];
  for (int k = 0; k < n_atoms; ++k) {
    for (int a = 0; a < 5; ++a)
      if (!std::isfinite(atoms[5 * k + a])) return PB_EINVAL;
    if (atoms[5 * k + 3] < 0) return PB_EINVAL;
    rmax = std::fmax(rmax, atoms[5 * k + 3]);
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::fmin(lo[a], atoms[5 * k + a]);
      hi[a] = std::fmax(hi[a], atoms[5 * k + a]);
    }
  }
  double h = prm->h;
  double margin = rmax + (prm->ls_mode == PB_LS_SES ? prm->probe : 0.0) + prm->band_k * h + 4.0 * h + 1.0;
  for (int a = 0; a < 3; ++a) {
    long ilo = (long)std::floor((lo[a] - margin) / h);
    long ihi = (long)std::ceil((hi[a] + margin) / h);
    grid->origin[a] = (double)ilo * h;
    if (ihi - ilo + 1 > 4096) return PB_EINVAL;  // the level set takes axes of at most 4096 nodes
    int n = (int)(ihi - ilo + 1);
    if (a == 0) grid->nx = n;
    if (a == 1) grid->ny = n;
    if (a == 2) grid->nz = n;
  }
  grid->h = h;
  return PB_OK;
}

pb_status pb_set_timing(pb_ctx* ctx, int enable) {
  if (!ctx) return PB_EINVAL;
  PB_TRY(pb::sync(ctx, "pb_set_timing"));
  if (enable < 0 || enable > 2) return ctx->fail(PB_EINVAL, "timing level %d", enable);
  ctx->timing = enable;
  ctx->timers.clear();
  return PB_OK;
}

pb_status pb_far_kernel(pb_ctx* ctx, int64_t n, int* cfg) {
  if (!ctx || !cfg) return PB_EINVAL;
  auto it = ctx->far_cfg.find((int)n);
  if (n < 1 || n > INT32_MAX || it == ctx->far_cfg.end())
    return ctx->fail(PB_EINVAL, "no far-field kernel chosen for bands of %lld nodes", (long long)n);
  *cfg = it->second;
  return PB_OK;
}

pb_status pb_tree_info(pb_ctx* ctx, int64_t info[6]) {
  if (!ctx || !info) return PB_EINVAL;
  const pb::TreePlan& T = ctx->tree;
  if (!T.band_key) return ctx->fail(PB_EINVAL, "no treecode operator prepared on this context");
  info[0] = T.n_batch;
  info[1] = T.n_cl;
  info[2] = T.n_items;
  info[3] = T.n_dir_pairs;
  info[4] = T.n_app_pairs;
  info[5] = T.near.nnz;
  return PB_OK;
}

pb_status pb_kernel_time(pb_ctx* ctx, const char* name, double* total_ms, int64_t* launches) {
  if (!ctx || !name) return PB_EINVAL;
  PB_TRY(pb::sync(ctx, "pb_kernel_time"));
  auto it = ctx->timers.find(name);
  if (total_ms) *total_ms = it == ctx->timers.end() ? 0.0 : it->second.ms;
  if (launches) *launches = it == ctx->timers.end() ? 0 : it->second.launches;
  return PB_OK;
}

}  // extern "C"
