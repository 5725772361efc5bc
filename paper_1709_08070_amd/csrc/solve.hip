// Stage 3: GMRES on Λp + KWp = g (section "Fast linear solvers").
//
// Restarted GMRES with classical Gram–Schmidt applied twice (CGS2). The Krylov basis, every
// vector operation and the Givens rotations with the residual estimate live in FP64 device
// memory; the host reads one step's convergence flag while the next step runs and solves the
// small triangular system once per cycle. Dot products are two-stage fixed-order reductions.
//
// Initial guess: Λ⁻¹g by default, the paper's "solution of the diagonal part" with D = 0.
// Mixed precision: GMRES on A_mixed x = g from the initial guess, then iterative refinement:
// form the true FP64 residual r = g − A₆₄x and, while it misses tol, solve A_mixed d = r and
// set x ← x + d. Each inner solve stops at max(½·tol·‖g‖, η·‖r₀‖), r₀ its initial residual
// and η = kInnerEta. Its last cycle ends on the Arnoldi residual estimate: the inner operator
// is not applied to the result again, since the refinement forms the better residual next.
#include <chrono>
#include <cmath>
#include <functional>
#include <vector>

#include "pb_internal.hpp"

namespace pb {
namespace {

constexpr int kBlock = 256;
constexpr int kDotBlocks = 1024;
constexpr int kGroup = 8;
constexpr int kMaxRestart = 2000;  // the largest restart length pb_ibim_solve accepts

// Arguments of the Givens step that ends an Arnoldi step (see givens_step).
struct GivensArgs {
  int k, m;
  const double* hcol;  // [pass 1 (m+1) | pass 2 (m+1) | ‖w‖]
  double *H, *cs, *sn, *s;
  double tol_abs;
  int* state;
  int* host_out;  // the step's slot in pinned host memory: state after the step
};

// Arnoldi column k into the QR factor of the Hessenberg matrix (row-major, (m+1) × m):
// H(i,k) = sum of the two Gram–Schmidt passes' coefficients (i ≤ k), H(k+1,k) = ‖w‖; the
// earlier rotations are applied, a new one (cs[k], sn[k]) zeroes H(k+1,k), and s is rotated
// so that |s[k+1]| is the residual estimate. state[0] is set once that estimate is at most
// tol_abs or ‖w‖ is not positive (breakdown); state[1] counts the steps taken. Once state[0]
// is set, later steps leave everything as it is. One thread.
__device__ void givens_step(const GivensArgs& g) {
  const int k = g.k, m = g.m;
  double* __restrict__ H = g.H;
  const double* __restrict__ hc = g.hcol;
  const double* __restrict__ cs = g.cs;
  const double* __restrict__ sn = g.sn;
  if (g.state[0]) {  // a step after the test was met: report the state unchanged
    g.host_out[0] = g.state[0];
    g.host_out[1] = g.state[1];
    return;
  }
  const double hn = hc[2 * (m + 1)];
  // rotation i acts on rows i (already rotated by the earlier ones: `a`) and i + 1 (still
  // the raw coefficient); the loads do not depend on the chain and run ahead of it
  double a = hc[0] + hc[m + 1];
#pragma unroll 4
  for (int i = 0; i < k; ++i) {
    const double b = hc[i + 1] + hc[(m + 1) + i + 1];
    const double c = cs[i], s = sn[i];
    H[(size_t)i * m + k] = c * a + s * b;
    a = -s * a + c * b;
  }
  const double den = sqrt(a * a + hn * hn);
  const double c = den > 0.0 ? a / den : 1.0, sg = den > 0.0 ? hn / den : 0.0;
  g.cs[k] = c;
  g.sn[k] = sg;
  H[(size_t)k * m + k] = den;
  H[(size_t)(k + 1) * m + k] = 0.0;
  const double sk = g.s[k];
  g.s[k + 1] = -sg * sk;
  g.s[k] = c * sk;
  const int done = fabs(g.s[k + 1]) <= g.tol_abs || !(hn > 0.0);
  g.state[1] = k + 1;
  if (done) g.state[0] = 1;
  g.host_out[0] = done;
  g.host_out[1] = k + 1;
}

// Whether the vectors can be read as pairs of doubles: an even length and leading dimension
// and 16-byte aligned bases (the solver's vectors always are: length 2N, workspace bases).
__device__ __forceinline__ bool pairs_ok(int64_t M, int64_t ldv, const void* V, const void* w) {
  return ((M | ldv) & 1) == 0 && (((uintptr_t)V | (uintptr_t)w) & 15) == 0;
}

// partial[q·nb + block] = Σ_{e in the block's share} w[e]·V[q][e], q < k, in groups of 8
// vectors so that w is read once per group. The block's share is the pairs (2p, 2p + 1) with
// p = block·kBlock + tid + i·nb·kBlock, read as 16-byte loads, or, when pairs_ok fails, the
// single elements e at the same positions (pairs = false).
__device__ __forceinline__ void block_dots(int64_t M, const double* __restrict__ V, int64_t ldv, int k,
                                           const double* __restrict__ w, bool pairs,
                                           double* __restrict__ partial, double (*red)[kBlock]) {
  const int64_t P = pairs ? M >> 1 : M, step = (int64_t)gridDim.x * kBlock;
  for (int q0 = 0; q0 < k; q0 += kGroup) {
    double acc[kGroup];
#pragma unroll
    for (int g = 0; g < kGroup; ++g) acc[g] = 0.0;
    const int nq = min(kGroup, k - q0);
    if (pairs) {
      const double2* __restrict__ w2 = reinterpret_cast<const double2*>(w);
      for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < P; p += step) {
        const double2 we = w2[p];
#pragma unroll
        for (int g = 0; g < kGroup; ++g)
          if (g < nq) {
            const double2 v = reinterpret_cast<const double2*>(V + (int64_t)(q0 + g) * ldv)[p];
            acc[g] = fma(we.y, v.y, fma(we.x, v.x, acc[g]));
          }
      }
    } else {
      for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < P; e += step) {
        const double we = w[e];
#pragma unroll
        for (int g = 0; g < kGroup; ++g)
          if (g < nq) acc[g] = fma(we, V[(int64_t)(q0 + g) * ldv + e], acc[g]);
      }
    }
#pragma unroll
    for (int g = 0; g < kGroup; ++g) red[g][threadIdx.x] = acc[g];
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off)
#pragma unroll
        for (int g = 0; g < kGroup; ++g) red[g][threadIdx.x] += red[g][threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x < nq) partial[(int64_t)(q0 + threadIdx.x) * gridDim.x + blockIdx.x] = red[threadIdx.x][0];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kBlock) k_dots(int64_t M, const double* __restrict__ V, int64_t ldv, int k,
                                                 const double* __restrict__ w, double* __restrict__ partial) {
  __shared__ double red[kGroup][kBlock];
  block_dots(M, V, ldv, k, w, pairs_ok(M, ldv, V, w), partial, red);
}

// One Gram–Schmidt update and the next reduction in one launch: w[e] −= Σ_q c[q]·V[q][e]
// (q < k) over the block's share (as in block_dots), then the partial sums of w·V[q] (q < k;
// kd = k) or of w·w (kd = 1, V = w, ldv = 0). Both phases split the elements the same way (pairs
// or single elements, decided once), so each thread reads back only the elements it wrote
// itself and no grid-wide synchronization is needed between them.
__global__ void __launch_bounds__(kBlock) k_axpy_dots(int64_t M, const double* __restrict__ V, int64_t ldv, int k,
                                                      const double* __restrict__ c, double* __restrict__ w,
                                                      int norm_only, double* __restrict__ partial) {
  __shared__ double red[kGroup][kBlock];
  const int64_t step = (int64_t)gridDim.x * kBlock;
  const bool pairs = pairs_ok(M, ldv, V, w);
  if (pairs) {
    double2* __restrict__ w2 = reinterpret_cast<double2*>(w);
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < (M >> 1); p += step) {
      double sx = 0.0, sy = 0.0;
      for (int q = 0; q < k; ++q) {
        const double2 v = reinterpret_cast<const double2*>(V + (int64_t)q * ldv)[p];
        sx = fma(c[q], v.x, sx);
        sy = fma(c[q], v.y, sy);
      }
      double2 x = w2[p];
      x.x -= sx;
      x.y -= sy;
      w2[p] = x;
    }
  } else {
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < M; e += step) {
      double s = 0.0;
      for (int q = 0; q < k; ++q) s = fma(c[q], V[(int64_t)q * ldv + e], s);
      w[e] -= s;
    }
  }
  if (norm_only) block_dots(M, w, 0, 1, w, pairs, partial, red);
  else block_dots(M, V, ldv, k, w, pairs, partial, red);
}

// out[q] = Σ_b partial[q·nb + b] (one block per q, fixed tree); if sqrt_out, out[q] =
// sqrt(out[q]). With do_givens (a single block, the norm that ends an Arnoldi step) the
// Givens step follows.
__global__ void __launch_bounds__(kBlock) k_dots_finish(const double* __restrict__ partial, int nb,
                                                        double* __restrict__ out, int sqrt_out, int do_givens,
                                                        GivensArgs ga) {
  __shared__ double red[kBlock];
  const int q = blockIdx.x;
  double a = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) a += partial[(int64_t)q * nb + b];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[q] = sqrt_out ? sqrt(red[0]) : red[0];
    if (do_givens) givens_step(ga);
  }
}

// w[e] += sign · Σ_q c[q] V[q][e]
__global__ void __launch_bounds__(kBlock) k_axpy_multi(int64_t M, const double* __restrict__ V, int64_t ldv, int k,
                                                       const double* __restrict__ c, double sign,
                                                       double* __restrict__ w) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < M; e += (int64_t)gridDim.x * kBlock) {
    double s = 0.0;
    for (int q = 0; q < k; ++q) s += c[q] * V[(int64_t)q * ldv + e];
    w[e] += sign * s;
  }
}

// out = in / *nrm
__global__ void __launch_bounds__(kBlock) k_scale(int64_t M, const double* __restrict__ in,
                                                  const double* __restrict__ nrm, double* __restrict__ out) {
  const double s = 1.0 / *nrm;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < M; e += (int64_t)gridDim.x * kBlock)
    out[e] = in[e] * s;
}

// r = b − r
__global__ void __launch_bounds__(kBlock) k_residual(int64_t M, const double* __restrict__ b, double* __restrict__ r) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < M; e += (int64_t)gridDim.x * kBlock)
    r[e] = b[e] - r[e];
}

// x = Λ⁻¹ g
__global__ void __launch_bounds__(kBlock) k_diag_solve(int64_t n, const double* __restrict__ g, double lam1, double lam2,
                                                       double* __restrict__ x) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < 2 * n; e += (int64_t)gridDim.x * kBlock)
    x[e] = g[e] / (e < n ? lam1 : lam2);
}

__global__ void __launch_bounds__(kBlock) k_add(int64_t M, const double* __restrict__ d, double* __restrict__ x) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < M; e += (int64_t)gridDim.x * kBlock) x[e] += d[e];
}

__global__ void __launch_bounds__(kBlock) k_zero(int64_t M, double* __restrict__ x) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < M; e += (int64_t)gridDim.x * kBlock) x[e] = 0.0;
}

// w = w / *nrm when *nrm > 0 (after a breakdown w is left as it is).
__global__ void __launch_bounds__(kBlock) k_scale_pos(int64_t M, const double* __restrict__ nrm,
                                                      double* __restrict__ w) {
  const double v = *nrm;
  if (!(v > 0.0)) return;
  const double s = 1.0 / v;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < M; e += (int64_t)gridDim.x * kBlock) w[e] *= s;
}

// A new restart cycle: clears the step state and sets s = (β, 0, ...).
__global__ void k_cycle_start(int* __restrict__ state, double* __restrict__ s, double beta) {
  if (threadIdx.x != 0) return;
  state[0] = 0;
  state[1] = 0;
  s[0] = beta;
}

unsigned vec_blocks(int64_t M) { return (unsigned)std::min<int64_t>(2048, (M + kBlock - 1) / kBlock); }
unsigned dot_blocks(int64_t M) { return (unsigned)std::min<int64_t>(kDotBlocks, (M + kBlock - 1) / kBlock); }

using OpFn = std::function<pb_status(const double*, double*)>;

struct Krylov {
  pb_ctx* ctx;
  int64_t M;
  double* partial;  // kDotBlocks × (m+1)
  double* hcol;     // device: [pass1 (m+1) | pass2 (m+1) | norm]
  int m;
};

// ‖v‖₂ to host
pb_status norm2(pb_ctx* ctx, Krylov& K, const double* v, double* out) {
  const unsigned db = dot_blocks(K.M);
  k_dots<<<db, kBlock, 0, ctx->stream>>>(K.M, v, 0, 1, v, K.partial);
  k_dots_finish<<<1, kBlock, 0, ctx->stream>>>(K.partial, (int)db, K.hcol + 2 * (K.m + 1), 1, 0, GivensArgs{});
  PB_TRY(launch_ok(ctx, "norm"));
  PB_HIP(ctx, hipMemcpyAsync(out, K.hcol + 2 * (K.m + 1), sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  return sync(ctx, "norm");
}

// Sets up the pinned host slots through which GMRES reads each step's state.
pb_status step_sync_init(pb_ctx* ctx) {
  if (!ctx->host_state) {
    void* h = nullptr;
    // coherent and mapped: the Givens step writes each step's state straight into it
    PB_HIP(ctx, hipHostMalloc(&h, sizeof(int) * 2 * kMaxRestart, hipHostMallocCoherent | hipHostMallocMapped));
    ctx->host_state = (int*)h;
    void* d = nullptr;
    PB_HIP(ctx, hipHostGetDevicePointer(&d, h, 0));
    ctx->host_state_dev = (int*)d;
  }
  return PB_OK;
}

// Waits until the Givens step of Arnoldi step k has written its slot (the host set it to −1
// before enqueuing the step). Polling the pinned memory puts no marker into the stream (an
// event record costs a few microseconds of idle GPU per step); the stream is queried now and
// then so that a device error, or a stream that drained without writing, ends the wait.
pb_status wait_slot(pb_ctx* ctx, const volatile int* hs, int k) {
  for (unsigned spin = 1; hs[2 * k] < 0; ++spin) {
    if ((spin & 255u) == 0u) {
      const hipError_t e = hipStreamQuery(ctx->stream);
      if (e == hipSuccess) {
        if (hs[2 * k] >= 0) break;
        return ctx->fail(PB_EDEVICE, "GMRES: step %d ended without reporting its state", k);
      }
      if (e != hipErrorNotReady) return ctx->fail(PB_EDEVICE, "GMRES step %d: %s", k, hipGetErrorString(e));
    }
    __builtin_ia32_pause();
  }
  return PB_OK;
}

// Clears the operator's skip flag when a cycle ends, also on an error return.
struct SkipGuard {
  pb_ctx* ctx;
  ~SkipGuard() { ctx->skip = nullptr; }
};

// Restarted GMRES(m) for A x = b from the given x until ‖b − Ax‖ ≤ max(tol_abs, rel·‖b − Ax₀‖)
// (estimate, then confirmed with the operator at each restart) or max_iter operator
// applications. With rel > 0 the solve is the inner solve of a refinement whose caller forms
// a more accurate residual of the result next: a cycle that stops on its estimate ends the
// solve without the confirming application, and *res_out is that estimate. With x_zero the
// caller guarantees x = 0 on entry, and the first residual is b itself (no application).
// With prec (flexible GMRES, right preconditioning): z_k = prec(v_k), w = A z_k, and the
// update is x += Z y; the preconditioner may change from step to step (it may be nonlinear).
//
// The Givens rotations and the convergence test run on the device (givens_step, after the
// norm that ends each step), and the host enqueues step k before it reads the test of step
// k − 1, so the GPU never waits for the host inside a cycle. A step enqueued after the test
// was met finds the operator's skip flag set: its heavy kernels return at once and the step
// is not counted (*skipped counts them).
pb_status gmres(pb_ctx* ctx, Krylov& K, const OpFn& op, const OpFn* prec, const double* b, double* x, double tol_abs,
                double rel, int max_iter, int* iters, double* res_out, int* skipped, bool x_zero = false) {
  const int64_t M = K.M;
  const int m = K.m;
  double* V = (double*)workspace(ctx, "kr_V", sizeof(double) * (size_t)M * (m + 1));
  double* Z = prec ? (double*)workspace(ctx, "kr_Z", sizeof(double) * (size_t)M * m) : nullptr;
  double* r = (double*)workspace(ctx, "kr_r", sizeof(double) * (size_t)M);
  double* ydev = (double*)workspace(ctx, "kr_y", sizeof(double) * (size_t)(m + 1));
  double* Hd = (double*)workspace(ctx, "kr_H", sizeof(double) * (size_t)(m + 1) * m);
  double* gv = (double*)workspace(ctx, "kr_rot", sizeof(double) * (size_t)(3 * m + 1));  // cs | sn | s
  int* state = (int*)workspace(ctx, "kr_state", 2 * sizeof(int));
  if (!V || !r || !ydev || !Hd || !gv || !state || (prec && !Z)) return PB_ENOMEM;
  PB_TRY(step_sync_init(ctx));
  double *cs = gv, *sn = gv + m, *sd = gv + 2 * m;
  volatile int* hs = ctx->host_state;  // step slots, written by the device (k_dots_finish)
  const unsigned vb = vec_blocks(M), db = dot_blocks(M);
  std::vector<double> H((size_t)(m + 1) * m, 0.0), s(m + 1), y(m);
  if (x_zero) k_zero<<<vb, kBlock, 0, ctx->stream>>>(M, r);  // A·0
  else PB_TRY(op(x, r));
  k_residual<<<vb, kBlock, 0, ctx->stream>>>(M, b, r);
  double beta = 0.0;
  PB_TRY(norm2(ctx, K, r, &beta));
  tol_abs = std::fmax(tol_abs, rel * beta);
  int it = 0;
  for (;;) {
    if (!(beta > tol_abs) || it >= max_iter) break;
    {
      Scope t(ctx, "gmres");
      k_cycle_start<<<1, 64, 0, ctx->stream>>>(state, sd, beta);
      k_scale<<<vb, kBlock, 0, ctx->stream>>>(M, r, K.hcol + 2 * (m + 1), V);  // norm2 left ‖r‖ there
    }
    const int steps = std::min(m, max_iter - it);
    int enq = 0;
    size_t mark = 0;  // timers pending before the last enqueued step
    {
      SkipGuard guard{ctx};
      ctx->skip = state;
      for (int k = 0; k < steps; ++k) {
        mark = ctx->pending.size();
        hs[2 * k] = -1;
        double* w = V + (size_t)(k + 1) * M;
        if (prec) {
          PB_TRY((*prec)(V + (size_t)k * M, Z + (size_t)k * M));
          PB_TRY(op(Z + (size_t)k * M, w));
        } else {
          PB_TRY(op(V + (size_t)k * M, w));
        }
        ++enq;
        {
          Scope t(ctx, "gmres");
          // CGS2: h1 = Vᵀw, w −= V h1, h2 = Vᵀw, w −= V h2, ‖w‖; each update is fused with
          // the reduction that follows it
          double *h1 = K.hcol, *h2 = K.hcol + (m + 1);
          k_dots<<<db, kBlock, 0, ctx->stream>>>(M, V, M, k + 1, w, K.partial);
          k_dots_finish<<<k + 1, kBlock, 0, ctx->stream>>>(K.partial, (int)db, h1, 0, 0, GivensArgs{});
          k_axpy_dots<<<db, kBlock, 0, ctx->stream>>>(M, V, M, k + 1, h1, w, 0, K.partial);
          k_dots_finish<<<k + 1, kBlock, 0, ctx->stream>>>(K.partial, (int)db, h2, 0, 0, GivensArgs{});
          k_axpy_dots<<<db, kBlock, 0, ctx->stream>>>(M, V, M, k + 1, h2, w, 1, K.partial);
          const GivensArgs ga{k, m, K.hcol, Hd, cs, sn, sd, tol_abs, state, ctx->host_state_dev + 2 * k};
          k_dots_finish<<<1, kBlock, 0, ctx->stream>>>(K.partial, (int)db, K.hcol + 2 * (m + 1), 1, 1, ga);
          k_scale_pos<<<vb, kBlock, 0, ctx->stream>>>(M, K.hcol + 2 * (m + 1), w);
        }
        PB_TRY(launch_ok(ctx, "arnoldi"));
        if (k >= 1) {
          PB_TRY(wait_slot(ctx, hs, k - 1));
          if (hs[2 * (k - 1)]) break;  // step k − 1 met the test; step k did nothing
        }
      }
    }
    PB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const int kd = hs[2 * (enq - 1) + 1];  // steps taken
    const bool early = hs[2 * (enq - 1)] != 0;  // the cycle ended on its residual estimate
    if (kd < 1 || kd > enq) return ctx->fail(PB_EDEVICE, "GMRES: inconsistent step count %d of %d", kd, enq);
    if (enq > kd) drop_timers(ctx, mark);  // the last step was skipped
    *skipped += enq - kd;
    it += kd;
    PB_HIP(ctx, hipMemcpyAsync(H.data(), Hd, sizeof(double) * (size_t)kd * m, hipMemcpyDeviceToHost, ctx->stream));
    PB_HIP(ctx, hipMemcpyAsync(s.data(), sd, sizeof(double) * (size_t)(kd + 1), hipMemcpyDeviceToHost, ctx->stream));
    PB_TRY(sync(ctx, "arnoldi"));
    for (int i = kd - 1; i >= 0; --i) {
      double acc = s[i];
      for (int j = i + 1; j < kd; ++j) acc -= H[(size_t)i * m + j] * y[j];
      y[i] = acc / H[(size_t)i * m + i];
    }
    PB_HIP(ctx, hipMemcpyAsync(ydev, y.data(), sizeof(double) * kd, hipMemcpyHostToDevice, ctx->stream));
    k_axpy_multi<<<vb, kBlock, 0, ctx->stream>>>(M, prec ? Z : V, M, kd, ydev, 1.0, x);
    PB_TRY(launch_ok(ctx, "update"));
    if (rel > 0.0 && early) {
      beta = std::fabs(s[kd]);
      break;
    }
    PB_TRY(op(x, r));
    k_residual<<<vb, kBlock, 0, ctx->stream>>>(M, b, r);
    PB_TRY(norm2(ctx, K, r, &beta));
  }
  *iters = it;
  *res_out = beta;
  return PB_OK;
}

}  // namespace
}  // namespace pb

extern "C" pb_status pb_ibim_solve(pb_ctx* ctx, const pb_band* band, const double* atoms, int n_atoms,
                                   const pb_params* prm, const pb_solve_opts* opts_in, double* p,
                                   pb_solve_stats* stats) {
  using namespace pb;
  auto t0 = std::chrono::steady_clock::now();
  if (!ctx) return PB_EINVAL;
  PB_TRY(check_params(ctx, prm));
  PB_TRY(check_band(ctx, band));
  PB_TRY(check_curv(ctx, band, prm));
  pb_solve_opts opts;
  if (opts_in) opts = *opts_in;
  else pb_default_solve_opts(&opts);
  if (!atoms || n_atoms <= 0 || !p) return ctx->fail(PB_EINVAL, "pb_ibim_solve: NULL or empty input");
  if (!(opts.tol > 0.0) || !std::isfinite(opts.tol)) return ctx->fail(PB_EINVAL, "tolerance must be positive");
  if (opts.max_iter < 1 || opts.restart < 1 || opts.restart > kMaxRestart) return ctx->fail(PB_EINVAL, "bad iteration limits");
  if (opts.precision != PB_FP64 && opts.precision != PB_MIXED && opts.precision != PB_TREE)
    return ctx->fail(PB_EINVAL, "unknown precision");
  if (opts.precision != PB_FP64 && prm->reg_metric == PB_REG_TANGENT)
    return ctx->fail(PB_EINVAL, "the mixed path needs a bounded regularization radius");
  if (opts.x0 < PB_X0_ZERO || opts.x0 > PB_X0_LEARNED) return ctx->fail(PB_EINVAL, "unknown x0 mode %d", opts.x0);
  if (opts.precond != PB_PRECOND_NONE && opts.precond != PB_PRECOND_LEARNED)
    return ctx->fail(PB_EINVAL, "unknown preconditioner %d", opts.precond);
  const bool learned = opts.x0 == PB_X0_LEARNED || opts.precond == PB_PRECOND_LEARNED;
  if (learned && !opts.nn) return ctx->fail(PB_EINVAL, "the learned path needs opts->nn");
  if (learned && !band->phi) return ctx->fail(PB_EINVAL, "the learned path needs band->phi");
  const pb_nn* net = (const pb_nn*)opts.nn;
  PB_HIP(ctx, hipSetDevice(ctx->device));
  PB_TRY(sync(ctx, "pb_ibim_solve"));
  auto matvec_ms = [&]() {
    double tm = 0.0;
    for (const char* nm : {"p2p_f64", "p2p_f32", "tree_f32", "tree_fine_f32", "near_f64", "reduce"}) {
      auto itt = ctx->timers.find(nm);
      if (itt != ctx->timers.end()) tm += itt->second.ms;
    }
    return tm;
  };
  const double tm0 = matvec_ms();
  const Derived d = derive(*prm);
  const int64_t n = band->n, M = 2 * n;
  const int m = opts.restart;
  Krylov K{ctx, M, (double*)workspace(ctx, "kr_partial", sizeof(double) * kDotBlocks * (size_t)(m + 1)),
           (double*)workspace(ctx, "kr_hcol", sizeof(double) * (size_t)(2 * (m + 1) + 1)), m};
  double* g = (double*)workspace(ctx, "sv_g", sizeof(double) * M);
  double* r = (double*)workspace(ctx, "sv_r", sizeof(double) * M);
  double* dx = (double*)workspace(ctx, "sv_d", sizeof(double) * M);
  if (!K.partial || !K.hcol || !g || !r || !dx) return PB_ENOMEM;
  const unsigned vb = vec_blocks(M);

  PB_TRY(rhs(ctx, band, atoms, n_atoms, d, g));
  double gnorm = 0.0;
  PB_TRY(norm2(ctx, K, g, &gnorm));
  if (!std::isfinite(gnorm)) return ctx->fail(PB_EINVAL, "non-finite right-hand side");
  if (gnorm == 0.0) gnorm = 1.0;
  if (learned) PB_TRY(nn_prepare(ctx, band, d));
  if (opts.x0 == PB_X0_DIAG) k_diag_solve<<<vb, kBlock, 0, ctx->stream>>>(n, g, d.lam1, d.lam2, p);
  else if (opts.x0 == PB_X0_ZERO) k_zero<<<vb, kBlock, 0, ctx->stream>>>(M, p);
  else if (opts.x0 == PB_X0_LEARNED) PB_TRY(nn_apply(ctx, net, band, d, g, p));
  PB_TRY(launch_ok(ctx, "x0"));

  const bool fine_tree = opts.precision == PB_TREE && n >= kTreeFineMin;
  if (opts.precision == PB_MIXED || (opts.precision == PB_TREE && !fine_tree)) PB_TRY(mixed_prepare(ctx, band, d));
  if (opts.precision == PB_TREE) {
    std::shared_ptr<TreeHost> host;  // one octree for both plans
    PB_TRY(tree_prepare(ctx, band, d, prm->tree_degree, prm->tree_theta, ctx->tree, "tc_", nullptr, &host));
    if (fine_tree)
      PB_TRY(tree_prepare(ctx, band, d, kTreeFineDegree, kTreeFineTheta, ctx->tree_fine, "tf_", &ctx->tree.near,
                          &host));
  }
  int n64 = 0, nmx = 0, nmid = 0, nnn = 0;
  OpFn op64 = [&](const double* in, double* out) {
    ++n64;
    return matvec_fp64(ctx, band, d, in, out);
  };
  OpFn opmx = [&](const double* in, double* out) {
    ++nmx;
    return opts.precision == PB_TREE ? matvec_tree(ctx, band, d, in, out, ctx->tree)
                                     : matvec_mixed(ctx, band, d, in, out);
  };
  // PB_TREE: the refinement's residuals come from an operator about 1e-7 from the FP64 one,
  // far below the inner treecode's ~1e-5 (the dense mixed operator, or on large bands the
  // fine treecode at the same FP32 rounding level), until they meet half the tolerance; the
  // FP64 operator then certifies the result once
  OpFn opmid = [&](const double* in, double* out) {
    ++nmid;
    return fine_tree ? matvec_tree(ctx, band, d, in, out, ctx->tree_fine) : matvec_mixed(ctx, band, d, in, out);
  };
  OpFn opnn = [&](const double* in, double* out) {
    ++nnn;
    return nn_apply(ctx, net, band, d, in, out);
  };
  int iters = 0, outer = 0;
  double relres = 0.0;
  bool p_zero = opts.x0 == PB_X0_ZERO;  // p = 0 on entry to the first pass
  // one solve from the current p; prec = learned right preconditioner or none
  auto run = [&](const OpFn* prec, int iter_budget) -> pb_status {
    const bool from_zero = p_zero;
    p_zero = false;
    if (opts.precision == PB_FP64) {
      double res = 0.0;
      int it = 0;
      int sk = 0;
      PB_TRY(gmres(ctx, K, op64, prec, g, p, opts.tol * gnorm, 0.0, iter_budget, &it, &res, &sk, from_zero));
      n64 -= sk;
      if (prec) nnn -= sk;
      iters += it;
      relres = res / gnorm;
      outer += 1;
      return PB_OK;
    }
    int used = 0, steps = 0;
    {
      // first pass straight on the inner operator from the initial guess (A_mixed p = g, or
      // the treecode's); the residual below then decides whether a correction step is needed
      int it = 0;
      double res = 0.0;
      int sk = 0;
      PB_TRY(gmres(ctx, K, opmx, prec, g, p, 0.5 * opts.tol * gnorm, kInnerEta, iter_budget, &it, &res, &sk,
                   from_zero));
      nmx -= sk;
      if (prec) nnn -= sk;
      used += it;
      ++steps;
    }
    // below about 1e-7 the dense mixed operator is too far from the FP64 one to steer the
    // refinement, so tighter tolerances use the FP64 residual from the start
    bool certify = opts.precision != PB_TREE || opts.tol < 1e-7;
    for (;;) {
      PB_TRY(certify ? op64(p, r) : opmid(p, r));
      k_residual<<<vb, kBlock, 0, ctx->stream>>>(M, g, r);
      double rn = 0.0;
      PB_TRY(norm2(ctx, K, r, &rn));
      if (!certify) {
        if (!(rn / gnorm > 0.5 * opts.tol) || steps >= opts.max_outer || used >= iter_budget) certify = true;
        if (certify) continue;  // the FP64 residual of the same iterate decides
      } else {
        relres = rn / gnorm;
        if (!(relres > opts.tol) || steps >= opts.max_outer || used >= iter_budget) break;
      }
      k_zero<<<vb, kBlock, 0, ctx->stream>>>(M, dx);
      int it = 0;
      double res = 0.0;
      int sk = 0;
      PB_TRY(gmres(ctx, K, opmx, prec, r, dx, 0.5 * opts.tol * gnorm, kInnerEta, iter_budget - used, &it, &res,
                   &sk, true));
      nmx -= sk;
      if (prec) nnn -= sk;
      used += it;
      k_add<<<vb, kBlock, 0, ctx->stream>>>(M, dx, p);
      PB_TRY(launch_ok(ctx, "refine"));
      ++steps;
    }
    iters += used;
    outer += steps;
    return PB_OK;
  };
  bool fallback = false;
  // the preconditioned pass gets at most half of the iteration budget, so that plain GMRES
  // keeps at least the other half should the network fail
  const bool use_prec = opts.precond == PB_PRECOND_LEARNED;
  PB_TRY(run(use_prec ? &opnn : nullptr, use_prec ? opts.max_iter - opts.max_iter / 2 : opts.max_iter));
  if (learned && (!std::isfinite(relres) || relres > opts.tol)) {
    // plain GMRES judges the learned path (x0 = M(g) and/or the preconditioner M): restart
    // without the network from the last iterate, or from Λ⁻¹g if that iterate is not finite,
    // with what is left of the iteration budget (with none left, the residual of that
    // iterate is still formed and reported)
    fallback = true;
    if (!std::isfinite(relres)) k_diag_solve<<<vb, kBlock, 0, ctx->stream>>>(n, g, d.lam1, d.lam2, p);
    PB_TRY(launch_ok(ctx, "fallback x0"));
    PB_TRY(run(nullptr, std::max(opts.max_iter - iters, 0)));
  }
  PB_TRY(sync(ctx, "pb_ibim_solve"));
  if (stats) {
    stats->iters = iters;
    stats->outer = outer;
    stats->converged = relres <= opts.tol;
    stats->fallback_used = fallback;
    stats->matvecs_fp64 = n64;
    stats->matvecs_mixed = nmx + nmid;
    stats->true_relres = relres;
    const double per_mx = opts.precision == PB_TREE
                              ? (double)(ctx->tree.n_dir_pairs + ctx->tree.n_app_pairs + ctx->tree.near.nnz)
                              : (double)n * (double)n;
    const double per_mid = fine_tree ? (double)(ctx->tree_fine.n_dir_pairs + ctx->tree_fine.n_app_pairs +
                                                ctx->tree_fine.near.nnz)
                                     : (double)n * (double)n;
    stats->pairs = (double)n64 * (double)n * (double)n + (double)nmid * per_mid + (double)nmx * per_mx;
    stats->t_matvec_s = (matvec_ms() - tm0) * 1e-3;
    stats->t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (!std::isfinite(relres)) return ctx->fail(PB_ENOCONV, "solver produced a non-finite residual");
  if (relres > opts.tol) return ctx->fail(PB_ENOCONV, "GMRES stopped at relative residual %.3e", relres);
  return PB_OK;
}
