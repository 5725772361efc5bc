// Stage 1: level set of the solvent excluded surface on the Cartesian grid.
//
// vdW union F (eq. vdW-levelset-fn), SAS = F − ρ0, inward eikonal flow φ_t = |∇φ| to
// t = ρ0, cavity removal by flood fill from the grid boundary, and reinitialization
// φ_t + sgn_h(φ0)(|∇φ| − 1) = 0 (eqs. reinit, signum). Time stepping is third-order TVD
// Runge–Kutta; |∇φ| is the Godunov Hamiltonian on fifth-order WENO one-sided derivatives.
//
// Layout: φ is one FP64 array, k fastest. Each stencil kernel maps one thread to one node;
// consecutive threads are consecutive k, so the ±k neighbours are coalesced and the ±i/±j
// neighbours are served from L2. Products and sums are rounded as written (no FMA
// contraction) except in the Godunov Hamiltonian of the stage kernel, where the compiler
// fuses them into FMAs; either way the grid values are the same to the last bit from run
// to run.
#include <cmath>
#include <utility>

#include "pb_internal.hpp"
#include "stencil.hpp"

#pragma clang fp contract(off)

namespace pb {
namespace {

constexpr int kBlock = 256;

struct GridDev {
  int nx, ny, nz;
  double ox, oy, oz, h;
};

__device__ __forceinline__ int64_t lin(const GridDev& g, int64_t i, int64_t j, int64_t k) {
  return (i * g.ny + j) * g.nz + k;
}

__device__ __forceinline__ double sq(double a) { return a * a; }

// F(x) − shift, F = min over atoms of |x − z| − r, on tiles of kTI × kTJ × kTK nodes (one block
// each, k fastest inside the tile). The tile's nodes lie within R of its centre c, so for every
// node F ≤ U + R with U = min_k(|c − z_k| − r_k), and an atom can attain the minimum at a node of
// the tile only if |c − z_k| ≤ U + 2R + r_k. The block keeps those atoms (with a margin far
// above the rounding of both sides) in LDS and takes the minimum over them, with the same
// per-atom arithmetic as a scan over all atoms, so F is the same to the last bit; a tile that
// keeps more than kVdwList atoms scans them all.
constexpr int kTI = 4, kTJ = 8, kTK = 8;  // kTI·kTJ·kTK = kBlock
constexpr int kVdwList = 512;
static_assert(kTI * kTJ * kTK == kBlock, "one node per thread");

// One atom's candidate for F at x, with the skip of atoms that cannot lower best (their
// distance exceeds best + r by a relative margin far above the rounding of both sides).
__device__ __forceinline__ void vdw_update(double x, double y, double z, const double4& at, double& best) {
  const double d2 = (sq(x - at.x) + sq(y - at.y)) + sq(z - at.z);
  const double lim = best + at.w;
  if (lim > 0.0 && d2 < lim * lim * (1.0 + 1e-12)) {
    const double dist = sqrt(d2) - at.w;
    best = dist < best ? dist : best;
  }
}

__global__ void __launch_bounds__(kBlock) k_vdw(GridDev g, const double* __restrict__ atoms, int n_atoms,
                                                double shift, double* __restrict__ phi) {
  __shared__ double4 list[kVdwList];
  __shared__ double red[kBlock];
  __shared__ int count;
  const int ntk = (g.nz + kTK - 1) / kTK, ntj = (g.ny + kTJ - 1) / kTJ;
  const int tile = blockIdx.x;
  const int bk = tile % ntk, bj = (tile / ntk) % ntj, bi = tile / (ntk * ntj);
  const int t = threadIdx.x;
  const int i = bi * kTI + t / (kTJ * kTK), j = bj * kTJ + (t / kTK) % kTJ, k = bk * kTK + t % kTK;
  const bool live = i < g.nx && j < g.ny && k < g.nz;
  const double x = g.ox + g.h * (double)i, y = g.oy + g.h * (double)j, z = g.oz + g.h * (double)k;
  // centre and radius of the full tile
  const double cx = g.ox + g.h * (bi * kTI + 0.5 * (kTI - 1)), cy = g.oy + g.h * (bj * kTJ + 0.5 * (kTJ - 1)),
               cz = g.oz + g.h * (bk * kTK + 0.5 * (kTK - 1));
  const double R = g.h * 0.5 * sqrt((double)((kTI - 1) * (kTI - 1) + (kTJ - 1) * (kTJ - 1) + (kTK - 1) * (kTK - 1)));
  if (t == 0) count = 0;
  // U = min over atoms of |c − z| − r
  double u = INFINITY;
  for (int a = t; a < n_atoms; a += kBlock) {
    const double ax = atoms[5 * a], ay = atoms[5 * a + 1], az = atoms[5 * a + 2], ar = atoms[5 * a + 3];
    const double dc = sqrt((sq(cx - ax) + sq(cy - ay)) + sq(cz - az)) - ar;
    u = dc < u ? dc : u;
  }
  red[t] = u;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (t < off) red[t] = red[t + off] < red[t] ? red[t + off] : red[t];
    __syncthreads();
  }
  const double reach = red[0] + 2.0 * R;  // an atom matters only within reach + r of c
  for (int a = t; a < n_atoms; a += kBlock) {
    const double ax = atoms[5 * a], ay = atoms[5 * a + 1], az = atoms[5 * a + 2], ar = atoms[5 * a + 3];
    const double lim = (reach + ar) * (1.0 + 1e-9) + 1e-9 * (1.0 + g.h);
    if (lim > 0.0 && (sq(cx - ax) + sq(cy - ay)) + sq(cz - az) <= lim * lim) {
      const int q = atomicAdd(&count, 1);
      if (q < kVdwList) list[q] = make_double4(ax, ay, az, ar);
    }
  }
  __syncthreads();
  const int m = count;
  double best = INFINITY;
  if (m <= kVdwList) {
    for (int q = 0; q < m; ++q) vdw_update(x, y, z, list[q], best);
  } else {
    for (int a = 0; a < n_atoms; ++a)
      vdw_update(x, y, z, make_double4(atoms[5 * a], atoms[5 * a + 1], atoms[5 * a + 2], atoms[5 * a + 3]), best);
  }
  if (live) phi[((int64_t)i * g.ny + j) * g.nz + k] = best - shift;
}

// One axis of the Godunov Hamiltonian sg·|∇φ| (sg = ±1) from the seven values f[0..6] centred
// on the node: the WENO5 one-sided derivatives a (differences d0..d4) and b (d5..d1), then
// max((a⁺)², (b⁻)²) for sg > 0 and max((a⁻)², (b⁺)²) for sg < 0. It works on the differences
// d = h·D instead of the divided differences D: the smoothness indicators are taken ×12h²
// (so ε enters as e = 12h²ε, the same weights), the weights ×10 and the candidate stencils ×6h,
// so the value returned is (6h)² times the axis's term; both one-sided derivatives share their
// common second differences, and the larger of the two quotients is chosen by cross
// multiplication (their denominators are positive), one division instead of two.
struct Frac {
  double n, d;
};

__device__ __forceinline__ Frac weno_frac(double b1, double b2, double b3, double e, double p1, double p2,
                                          double p3) {
#pragma clang fp contract(fast)
  const double q1 = sq(b1 + e), q2 = sq(b2 + e), q3 = sq(b3 + e);
  const double w1 = q2 * q3, w2 = 6.0 * (q1 * q3), w3 = 3.0 * (q1 * q2);
  return {w1 * p1 + w2 * p2 + w3 * p3, (w1 + w2) + w3};
}

__device__ __forceinline__ double godunov_axis(const double f[7], double e, double sg) {
#pragma clang fp contract(fast)
  const double d0 = f[1] - f[0], d1 = f[2] - f[1], d2 = f[3] - f[2], d3 = f[4] - f[3], d4 = f[5] - f[4],
               d5 = f[6] - f[5];
  const double t0 = (d0 - 2.0 * d1) + d2, t1 = (d1 - 2.0 * d2) + d3, t2 = (d2 - 2.0 * d3) + d4,
               t3 = (d3 - 2.0 * d4) + d5;
  const double s1 = 13.0 * sq(t1), s2 = 13.0 * sq(t2);
  const Frac a = weno_frac(13.0 * sq(t0) + 3.0 * sq((d0 - 4.0 * d1) + 3.0 * d2), s1 + 3.0 * sq(d1 - d3),
                           s2 + 3.0 * sq((3.0 * d2 - 4.0 * d3) + d4), e, (2.0 * d0 - 7.0 * d1) + 11.0 * d2,
                           (5.0 * d2 - d1) + 2.0 * d3, (2.0 * d2 + 5.0 * d3) - d4);
  const Frac b = weno_frac(13.0 * sq(t3) + 3.0 * sq((d5 - 4.0 * d4) + 3.0 * d3), s2 + 3.0 * sq(d4 - d2),
                           s1 + 3.0 * sq((3.0 * d3 - 4.0 * d2) + d1), e, (2.0 * d5 - 7.0 * d4) + 11.0 * d3,
                           (5.0 * d3 - d4) + 2.0 * d2, (2.0 * d3 + 5.0 * d2) - d1);
  const double A = fmax(sg * a.n, 0.0), B = fmax(-sg * b.n, 0.0);
  const double x = A * b.d >= B * a.d ? A / a.d : B / b.d;
  return x * x;
}

// One TVD-RK3 stage: L = L(φ_in), then
//   stage 0: out = φ_in + dt·L
//   stage 1: out = 0.75 φ_n + 0.25 (φ_in + dt·L)
//   stage 2: out = φ_n / 3 + (2/3)(φ_in + dt·L)
// MODE 0: eikonal flow (L = |∇φ| with Hamiltonian −|∇φ|); MODE 1: reinit (L = −S(|∇φ| − 1)).
// |∇φ| is the Godunov Hamiltonian with zero-Neumann ghosts (even reflection about the boundary
// node, −m ↦ m and n−1+m ↦ n−1−m), taken only by nodes within three of a face; e = 12h²ε and
// c = 1/(6h) undo the scaling of godunov_axis. 32-bit node indexing (grids hold fewer than 2^31
// nodes).
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_rk_stage(GridDev g, const double* __restrict__ phi_in,
                                                     const double* __restrict__ phi_n, const double* __restrict__ S,
                                                     double* __restrict__ out, int stage, double dt, double e,
                                                     double c) {
  const unsigned total = (unsigned)g.nx * (unsigned)g.ny * (unsigned)g.nz;
  const unsigned uid = blockIdx.x * kBlock + threadIdx.x;
  if (uid >= total) return;
  const unsigned t = uid / (unsigned)g.nz;
  const int k = (int)(uid - t * (unsigned)g.nz), j = (int)(t % (unsigned)g.ny), i = (int)(t / (unsigned)g.ny);
  const double* __restrict__ p = phi_in + uid;
  const int n3[3] = {g.nx, g.ny, g.nz};
  const int c3[3] = {i, j, k};
  const int stride[3] = {g.ny * g.nz, g.nz, 1};
  double s = -1.0;
  if (MODE == 1) s = S[uid];
  const double sg = s >= 0.0 ? 1.0 : -1.0;
  double acc = 0.0, f[7];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    if ((unsigned)(c3[ax] - 3) <= (unsigned)(n3[ax] - 7)) {
#pragma unroll
      for (int m = 0; m < 7; ++m) f[m] = p[(m - 3) * stride[ax]];
    } else {
#pragma unroll
      for (int m = 0; m < 7; ++m) {
        int q = c3[ax] + m - 3;
        q = q < 0 ? -q : (q > n3[ax] - 1 ? 2 * (n3[ax] - 1) - q : q);
        f[m] = p[(q - c3[ax]) * stride[ax]];
      }
    }
    acc += godunov_axis(f, e, sg);
  }
  const double G = sqrt(acc) * c;
  const double L = MODE == 0 ? G : -s * (G - 1.0);
  const double v0 = p[0] + dt * L;
  double v;
  if (stage == 0) v = v0;
  else if (stage == 1) v = 0.75 * phi_n[uid] + 0.25 * v0;
  else v = phi_n[uid] * (1.0 / 3.0) + (2.0 / 3.0) * v0;
  out[uid] = v;
}

__global__ void __launch_bounds__(kBlock) k_sign(int64_t total, const double* __restrict__ phi, double h,
                                                 double* __restrict__ S) {
  int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id < total) S[id] = phi[id] / sqrt(phi[id] * phi[id] + h * h);
}

// ---- cavity removal

__global__ void __launch_bounds__(kBlock) k_cav_init(GridDev g, const double* __restrict__ phi,
                                                     uint8_t* __restrict__ outside) {
  int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int64_t total = (int64_t)g.nx * g.ny * g.nz;
  if (id >= total) return;
  int64_t k = id % g.nz, j = (id / g.nz) % g.ny, i = id / ((int64_t)g.ny * g.nz);
  bool edge = i == 0 || j == 0 || k == 0 || i == g.nx - 1 || j == g.ny - 1 || k == g.nz - 1;
  outside[id] = (edge && phi[id] > 0.0) ? 1 : 0;
}

constexpr int kLineChunks = 64;  // the wave-per-line sweep handles lines of up to 64·64 nodes
constexpr int kMaxAxis = 64 * kLineChunks;
constexpr int kLineWaves = kBlock / 64;

// Bits t of F (< 64) that some seed s ≤ t reaches through set bits of P: a doubling scan
// on a 64-node chunk (Kogge–Stone over the ballot masks; bits shifted in are 0).
__device__ __forceinline__ uint64_t reach_up(uint64_t S, uint64_t P) {
  uint64_t F = S, A = P;
  for (int d = 1; d < 64; d <<= 1) {
    F |= (F << d) & A;
    A &= A << d;
  }
  return F;
}
__device__ __forceinline__ uint64_t reach_down(uint64_t S, uint64_t P) {
  uint64_t F = S, A = P;
  for (int d = 1; d < 64; d <<= 1) {
    F |= (F >> d) & A;
    A &= A >> d;
  }
  return F;
}

// One sweep of the flood fill along `axis`, one wave per grid line (lines of at most
// 64·kLineChunks nodes). A node joins the exterior if φ > 0 and a node reachable from it
// through φ > 0 along the line is exterior or has an exterior neighbour across the line.
// The lanes take 64 consecutive nodes of the line at a time; ballots give P (φ > 0), the
// exterior nodes O and the seeds S (P-nodes exterior already or with an exterior neighbour
// across the line); doubling scans per chunk, carries between chunks (forward pass, then
// backward). Labels only go 0 → 1, so reads of neighbours being updated by other lines are
// harmless; repeated sweeps over the three axes reach the unique fixed point, the
// 6-connected component of {φ > 0} that touches the grid boundary.
__global__ void __launch_bounds__(kBlock) k_cav_line(GridDev g, const double* __restrict__ phi, uint8_t* outside,
                                                     int axis, int* changed) {
  __shared__ uint64_t sP[kLineWaves][kLineChunks], sO[kLineWaves][kLineChunks], sF[kLineWaves][kLineChunks];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t line = (int64_t)blockIdx.x * kLineWaves + wave;
  const int64_t n3[3] = {g.nx, g.ny, g.nz};
  const int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
  if (line >= n3[a1] * n3[a2]) return;  // the whole wave
  const int64_t L = n3[axis];
  const int nch = (int)((L + 63) / 64);
  int64_t c[3];
  c[a1] = line / n3[a2];
  c[a2] = line % n3[a2];
  uint64_t carry = 0;  // the last node of the previous chunk was reached
  for (int ch = 0; ch < nch; ++ch) {
    const int64_t t = (int64_t)ch * 64 + lane;
    bool pos = false, out = false, seed = false;
    if (t < L) {
      c[axis] = t;
      const int64_t id = lin(g, c[0], c[1], c[2]);
      pos = phi[id] > 0.0;
      out = outside[id] != 0;
      seed = pos && out;
      if (pos && !out)
        for (int ax = 0; ax < 3 && !seed; ++ax) {
          if (ax == axis) continue;
          for (int s = -1; s <= 1 && !seed; s += 2) {
            int64_t q[3] = {c[0], c[1], c[2]};
            q[ax] += s;
            if (q[ax] < 0 || q[ax] >= n3[ax]) continue;
            if (outside[lin(g, q[0], q[1], q[2])]) seed = true;
          }
        }
    }
    const uint64_t P = __ballot(pos), O = __ballot(out);
    const uint64_t S = __ballot(seed) | (carry & P & 1ull);
    const uint64_t F = reach_up(S, P);
    carry = F >> 63;
    if (lane == 0) {
      sP[wave][ch] = P;
      sO[wave][ch] = O;
      sF[wave][ch] = F;
    }
  }
  // lane 0's masks are read by every lane of the same wave below
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  carry = 0;  // the first node of the next chunk was reached
  bool any = false;
  for (int ch = nch - 1; ch >= 0; --ch) {
    const uint64_t P = sP[wave][ch], O = sO[wave][ch], Ff = sF[wave][ch];
    // seeds of the backward scan: everything the forward scan reached (it holds the seeds)
    const uint64_t B = reach_down(Ff | ((carry << 63) & P), P);
    carry = B & 1ull;
    const uint64_t add = (Ff | B) & P & ~O;
    if (add) {
      any = true;
      if ((add >> lane) & 1ull) {
        c[axis] = (int64_t)ch * 64 + lane;
        outside[lin(g, c[0], c[1], c[2])] = 1;
      }
    }
  }
  if (any && lane == 0) *changed = 1;
}

// Unreached nodes within (ε + h) of a cavity node (unreached, φ > 0) get −ε.
__global__ void __launch_bounds__(kBlock) k_cav_dilate(GridDev g, const double* __restrict__ phi,
                                                       const uint8_t* __restrict__ outside, double eps, int m,
                                                       double rr2, double* __restrict__ out, int* n_set) {
  int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int64_t total = (int64_t)g.nx * g.ny * g.nz;
  if (id >= total) return;
  double v = phi[id];
  if (!outside[id]) {
    int64_t k = id % g.nz, j = (id / g.nz) % g.ny, i = id / ((int64_t)g.ny * g.nz);
    bool hit = v > 0.0;
    for (int a = -m; a <= m && !hit; ++a)
      for (int b = -m; b <= m && !hit; ++b)
        for (int c = -m; c <= m && !hit; ++c) {
          if ((double)(a * a + b * b + c * c) > rr2) continue;
          int64_t ii = i + a, jj = j + b, kk = k + c;
          if (ii < 0 || jj < 0 || kk < 0 || ii >= g.nx || jj >= g.ny || kk >= g.nz) continue;
          int64_t q = lin(g, ii, jj, kk);
          if (!outside[q] && phi[q] > 0.0) hit = true;
        }
    if (hit) {
      v = -eps;
      atomicAdd(n_set, 1);
    }
  }
  out[id] = v;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Three-stage TVD-RK3 for `steps` steps of size dt; φ is updated in place. The step's result
// goes to the buffer its first stage used, which then holds φ (the two swap every step);
// after an odd number of steps it is copied back into phi.
pb_status tvd_rk3(pb_ctx* ctx, const GridDev& g, double* phi, double* p1, double* p2, const double* S, int mode,
                  int steps, double dt) {
  int64_t total = (int64_t)g.nx * g.ny * g.nz;
  unsigned nb = blocks_for(total);
  const double e = 12.0 * g.h * g.h * kWenoEps, c = 1.0 / (6.0 * g.h);
  double *cur = phi, *spare = p1;
  for (int s = 0; s < steps; ++s) {
    Scope t(ctx, "levelset");
    auto stage = mode == 0 ? k_rk_stage<0> : k_rk_stage<1>;
    stage<<<nb, kBlock, 0, ctx->stream>>>(g, cur, cur, S, spare, 0, dt, e, c);
    stage<<<nb, kBlock, 0, ctx->stream>>>(g, spare, cur, S, p2, 1, dt, e, c);
    stage<<<nb, kBlock, 0, ctx->stream>>>(g, p2, cur, S, spare, 2, dt, e, c);
    std::swap(cur, spare);
  }
  if (cur != phi) PB_HIP(ctx, hipMemcpyAsync(phi, cur, sizeof(double) * total, hipMemcpyDeviceToDevice, ctx->stream));
  return launch_ok(ctx, "levelset rk3");
}

}  // namespace
}  // namespace pb

extern "C" pb_status pb_build_levelset(pb_ctx* ctx, const double* atoms, int n_atoms, const pb_params* prm,
                                       const pb_grid* grid, double* phi, size_t cap, size_t* needed) {
  using namespace pb;
  if (!ctx) return PB_EINVAL;
  PB_TRY(check_params(ctx, prm));
  if (!grid) return ctx->fail(PB_EINVAL, "pb_build_levelset: NULL grid");
  if (grid->nx < 7 || grid->ny < 7 || grid->nz < 7)
    return ctx->fail(PB_EINVAL, "pb_build_levelset: grid must be at least 7 nodes per axis");
  if (grid->nx > kMaxAxis || grid->ny > kMaxAxis || grid->nz > kMaxAxis)
    return ctx->fail(PB_EINVAL, "pb_build_levelset: grid axes hold at most %d nodes", kMaxAxis);
  if (!std::isfinite(grid->origin[0]) || !std::isfinite(grid->origin[1]) || !std::isfinite(grid->origin[2]))
    return ctx->fail(PB_EINVAL, "pb_build_levelset: non-finite grid origin");
  if (std::fabs(grid->h - prm->h) > 1e-12 * prm->h)
    return ctx->fail(PB_EINVAL, "pb_build_levelset: grid spacing differs from params.h");
  const size_t count = (size_t)grid->nx * (size_t)grid->ny * (size_t)grid->nz;
  if (count >= ((size_t)1 << 31)) return ctx->fail(PB_EINVAL, "pb_build_levelset: grid of 2^31 nodes or more");
  if (needed) *needed = count;
  if (!phi) return PB_OK;  // size query
  if (cap < count)
    return ctx->fail(PB_ECAPACITY, "pb_build_levelset: phi holds %zu doubles, the grid needs %zu", cap, count);
  if (!atoms || n_atoms <= 0) return ctx->fail(PB_EINVAL, "pb_build_levelset: NULL or empty atoms");
  PB_HIP(ctx, hipSetDevice(ctx->device));
  GridDev g{grid->nx, grid->ny, grid->nz, grid->origin[0], grid->origin[1], grid->origin[2], grid->h};
  int64_t total = (int64_t)g.nx * g.ny * g.nz;
  unsigned nb = blocks_for(total);
  const double h = prm->h;
  const bool ses = prm->ls_mode == PB_LS_SES;
  {
    Scope t(ctx, "levelset");
    const unsigned tiles = (unsigned)(((g.nx + kTI - 1) / kTI) * (int64_t)((g.ny + kTJ - 1) / kTJ) *
                                      ((g.nz + kTK - 1) / kTK));
    k_vdw<<<tiles, kBlock, 0, ctx->stream>>>(g, atoms, n_atoms, ses ? prm->probe : 0.0, phi);
  }
  PB_TRY(launch_ok(ctx, "vdw"));
  if (!ses) return sync(ctx, "pb_build_levelset");

  double* p1 = (double*)workspace(ctx, "ls_p1", sizeof(double) * total);
  double* p2 = (double*)workspace(ctx, "ls_p2", sizeof(double) * total);
  double* S = (double*)workspace(ctx, "ls_S", sizeof(double) * total);
  uint8_t* outside = (uint8_t*)workspace(ctx, "ls_outside", (size_t)total);
  int* flags = (int*)workspace(ctx, "ls_flags", 4 * sizeof(int));
  if (!p1 || !p2 || !S || !outside || !flags) return PB_ENOMEM;

  // inward eikonal flow to t = ρ0 in equal steps no longer than cfl·h
  if (prm->probe > 0.0) {
    int n_e = (int)std::ceil(prm->probe / (prm->cfl * h) - 1e-9);
    PB_TRY(tvd_rk3(ctx, g, phi, p1, p2, nullptr, 0, n_e, prm->probe / n_e));
  }

  // cavity removal
  {
    Scope t(ctx, "levelset");
    k_cav_init<<<nb, kBlock, 0, ctx->stream>>>(g, phi, outside);
  }
  PB_TRY(launch_ok(ctx, "cavity init"));
  int64_t n3[3] = {g.nx, g.ny, g.nz};
  int it = 0;
  for (;; ++it) {
    if (it > 100000) return ctx->fail(PB_EDEVICE, "cavity flood fill did not converge");
    PB_HIP(ctx, hipMemsetAsync(flags, 0, sizeof(int), ctx->stream));
    for (int ax = 0; ax < 3; ++ax) {
      int a1 = ax == 0 ? 1 : 0, a2 = ax == 2 ? 1 : 2;
      Scope t(ctx, "levelset");
      const int64_t lines = n3[a1] * n3[a2];
      k_cav_line<<<(unsigned)((lines + kLineWaves - 1) / kLineWaves), kBlock, 0, ctx->stream>>>(g, phi, outside, ax,
                                                                                               flags);
    }
    PB_TRY(launch_ok(ctx, "cavity sweep"));
    int changed = 0;
    PB_HIP(ctx, hipMemcpyAsync(&changed, flags, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    PB_TRY(sync(ctx, "cavity sweep"));
    if (!changed) break;
  }
  const double eps = prm->band_k * h;
  const double rr = (eps + h) / h;
  PB_HIP(ctx, hipMemsetAsync(flags + 1, 0, sizeof(int), ctx->stream));
  {
    Scope t(ctx, "levelset");
    k_cav_dilate<<<nb, kBlock, 0, ctx->stream>>>(g, phi, outside, eps, (int)std::floor(rr), rr * rr, p1, flags + 1);
  }
  PB_TRY(launch_ok(ctx, "cavity dilate"));
  PB_HIP(ctx, hipMemcpyAsync(phi, p1, sizeof(double) * total, hipMemcpyDeviceToDevice, ctx->stream));

  // reinitialization with the frozen smoothed sign of the post-removal φ
  int steps = prm->reinit_steps > 0 ? prm->reinit_steps
                                    : 2 * (int)std::ceil((prm->band_k + 4.0) / prm->cfl - 1e-9);
  {
    Scope t(ctx, "levelset");
    k_sign<<<nb, kBlock, 0, ctx->stream>>>(total, phi, h, S);
  }
  PB_TRY(launch_ok(ctx, "sign"));
  PB_TRY(tvd_rk3(ctx, g, phi, p1, p2, S, 1, steps, prm->cfl * h));
  return sync(ctx, "pb_build_levelset");
}
