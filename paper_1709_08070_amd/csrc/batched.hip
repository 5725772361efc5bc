// Batched solve: many molecules of uneven band size in one set of launches.
//
// Operator: one persistent launch covers the far field of every molecule. The work list
// holds (molecule, target block, source chunk) items of about equal cost, ordered largest
// first (LPT); each block strides through it, so molecules of very different n share the
// CUs evenly. Items of molecules that have converged are skipped. The FP64 near field of
// each molecule is its own CSR block matrix; one SpMV launch and one reduce launch cover all
// molecules. The far-field kernel (one of the tile shapes of the one-directional kernel, or
// the symmetric kernel over (molecule, chunk, chunk) items) is picked per batch by the
// autotuner (each candidate timed once).
//
// Krylov: every molecule runs its own GMRES (FP64 Arnoldi with CGS2, Givens rotations on the
// device, one thread per molecule). The vectors of all molecules are concatenated, molecule m
// owning [2·off_m, 2·off_m + 2·n_m) as [ψ̄ | ψ̄_n]. One Arnoldi step of the whole batch —
// pack, far field, near field, reduce, two Gram–Schmidt passes, norm, Givens, scaling — is
// captured once as a hipGraph and replayed; the step index lives in device memory, so the
// same graph serves every step. The host polls the number of active molecules every few
// replays.
//
// Mixed precision as in the single solve: each outer step forms the FP64 residual with the
// persistent FP64 operator and solves the correction with the mixed operator, to
// max(½·tol·‖g‖, η·‖r‖). A molecule whose cycle ends on its residual estimate leaves the
// inner solve without a further mixed application: its FP64 residual follows.
//
// Learned path: the network runs over all molecules at once (their nodes concatenated,
// neighbour lists offset to global indices). As right preconditioner it is applied inside
// the captured Arnoldi step (flexible GMRES: z_k = M(v_k), w = A z_k, x += Z y); as initial
// guess x0 = M(g). Molecules that miss the tolerance on the learned path are solved again
// from their last iterate (from Λ⁻¹g if it is not finite) without the network.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

#include "pair_kernels.hpp"
#include "sym64_kernels.hpp"
#include "sym_kernels.hpp"

namespace pb {
namespace {

constexpr int kSeg = 4096;  // vector elements per block in the batched reductions

struct MolDev {
  int off;          // first node in the concatenated node index
  int n;            // band nodes
  int S32, S64;     // source chunks of the FP32 / FP64 far field
  int Ssym, nsub;   // chunks and sub-blocks per chunk of the symmetric FP32 far field
  int64_t poff32;   // offset of the molecule's FP32-path partial sums (doubles)
  int64_t poff64;   // offset of the FP64-path partial sums
  int64_t poffsym;  // offset of the symmetric-kernel partial sums
  double cx, cy, cz;
  BandDev band;
  const double* w;
  float4* A;  // FP32 records (σ(x − c), ψn weight), σ·(ψ weight)·n, (n, σ·ψ weight)
  float4* M;
  float4* N;
  const float4* box;  // bounding boxes of groups of 256 records
  const int64_t* row;
  const int* col;
  const double4* coef;
};

struct Item {
  int mol, tb, ch;
};

// Krylov state of one molecule.
struct KState {
  double tol_abs;  // stop when the residual estimate is at or below this
  double beta;     // ‖r0‖ of the current cycle
  int active;      // still iterating in this cycle
  int k_used;      // Arnoldi steps taken in this cycle
  int iters;       // total steps
  int early;       // the cycle ended on its residual estimate (not on the restart length)
  unsigned long long t_inner;  // device clock when its last restart cycle ended
  unsigned long long t_done;   // the same, for the cycle whose result met the tolerance
};

// ---------------------------------------------------------------- operator kernels

static __global__ void __launch_bounds__(kBlock) k_pack_batch(int ntot, const int* __restrict__ mol_of,
                                                              const MolDev* __restrict__ mols,
                                                              const double* __restrict__ x, const int* __restrict__ kptr,
                                                              int kmax, int64_t ldv, double scale, double sigma) {
  const int g = blockIdx.x * kBlock + threadIdx.x;
  if (g >= ntot) return;
  if (kptr && *kptr >= kmax) return;
  const MolDev& m = mols[mol_of[g]];
  const double* v = x + (kptr ? (int64_t)(*kptr) * ldv : 0);
  const int l = g - m.off;
  const double s = scale * m.w[l];
  const double w1 = sigma * s * v[2 * (int64_t)m.off + l], w2 = s * v[2 * (int64_t)m.off + m.n + l];
  m.A[l] = make_float4((float)(sigma * (m.band.px[l] - m.cx)), (float)(sigma * (m.band.py[l] - m.cy)),
                       (float)(sigma * (m.band.pz[l] - m.cz)), (float)w2);
  m.M[l] = make_float4((float)(w1 * m.band.nx[l]), (float)(w1 * m.band.ny[l]), (float)(w1 * m.band.nz[l]), 0.f);
  m.N[l] = make_float4((float)m.band.nx[l], (float)m.band.ny[l], (float)m.band.nz[l], (float)w1);
}

template <int TILE, int TPL, bool kScreened>
static __global__ void __launch_bounds__(kBlock) k_far32_batch(const Item* __restrict__ items, int n_items,
                                                               const MolDev* __restrict__ mols, int chunk,
                                                               const int* __restrict__ active, F32Params fp, double sig1,
                                                               double sig2, double* __restrict__ partial) {
  __shared__ float4 sA[TILE], sM[TILE];
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const Item w = items[it];
    if (!active[w.mol]) continue;
    const MolDev& m = mols[w.mol];
    const int t0 = w.tb * kBlock * TPL;
    const int j0 = w.ch * chunk;
    const int j1 = min(m.n, j0 + chunk);
    double* out = partial + m.poff32 + (int64_t)w.ch * 2 * m.n;
    far_tile_loop<kBlock, TILE, TPL, kScreened>(m.A, m.M, m.N, m.box, t0, m.n, j0, j1, fp, sig1, sig2, sA, sM,
                                                out + t0, out + m.n + t0);
  }
}

// Symmetric far field of every active molecule: items (molecule, Ic, Jc), persistent.
template <bool kScreened>
static __global__ void __launch_bounds__(kBlock) k_far32_sym_batch(const Item* __restrict__ items, int n_items,
                                                                   const MolDev* __restrict__ mols,
                                                                   const int* __restrict__ active, F32Params fp,
                                                                   double sig1, double sig2,
                                                                   double* __restrict__ partial) {
  __shared__ SymShared sh;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const Item w = items[it];
    if (!active[w.mol]) continue;
    const MolDev& m = mols[w.mol];
    sym_item<kScreened>(m.A, m.N, m.box, m.n, w.tb, w.ch, m.nsub, fp, sig1, sig2, partial + m.poffsym, sh);
  }
}

// Symmetric FP64 operator of every selected molecule: items (molecule, Ic, Jc), persistent.
// k2 = κ².
static __global__ void __launch_bounds__(kBlock) k_far64_sym_batch(const Item* __restrict__ items, int n_items,
                                                                   const MolDev* __restrict__ mols,
                                                                   const int* __restrict__ active,
                                                                   const double* __restrict__ wpsi,
                                                                   const double* __restrict__ wpsn, KParams kp,
                                                                   double k2, double* __restrict__ partial) {
  __shared__ Sym64Shared sh;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const Item w = items[it];
    if (!active[w.mol]) continue;
    const MolDev& m = mols[w.mol];
    sym64_item(m.band, wpsi + m.off, wpsn + m.off, m.n, w.tb, w.ch, m.nsub, kp, k2, partial + m.poffsym, sh);
  }
}

static __global__ void __launch_bounds__(kBlock) k_weights_batch(int ntot, const int* __restrict__ mol_of,
                                                                 const MolDev* __restrict__ mols,
                                                                 const double* __restrict__ x, double scale,
                                                                 double* __restrict__ wpsi, double* __restrict__ wpsn) {
  const int g = blockIdx.x * kBlock + threadIdx.x;
  if (g >= ntot) return;
  const MolDev& m = mols[mol_of[g]];
  const int l = g - m.off;
  const double s = scale * m.w[l];
  wpsi[g] = s * x[2 * (int64_t)m.off + l];
  wpsn[g] = s * x[2 * (int64_t)m.off + m.n + l];
}

static __global__ void __launch_bounds__(kBlock) k_far64_batch(const Item* __restrict__ items, int n_items,
                                                               const MolDev* __restrict__ mols, int chunk,
                                                               const int* __restrict__ active,
                                                               const double* __restrict__ wpsi,
                                                               const double* __restrict__ wpsn, KParams kp,
                                                               double* __restrict__ partial) {
  __shared__ double smem[8 * kBlock];
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const Item w = items[it];
    if (!active[w.mol]) continue;
    const MolDev& m = mols[w.mol];
    const int t0 = w.tb * kBlock;
    const int j0 = w.ch * chunk;
    const int j1 = min(m.n, j0 + chunk);
    double* out = partial + m.poff64 + (int64_t)w.ch * 2 * m.n;
    far64_tile_loop<kBlock>(m.band, wpsi + m.off, wpsn + m.off, t0, m.n, j0, j1, kp, smem, out + t0,
                            out + m.n + t0);
  }
}

// Layout of the far-field partial sums read by k_reduce_batch.
constexpr int kModeTiled = 0, kModeF64 = 1, kModeSym = 2, kModeF64Sym = 3;

// y = Λx + Σ chunks (+ near), per molecule; x and y at step *kptr / *kptr + 1 of a basis
// when kptr is given. kRowLanes lanes share a node: lane t sums the chunk rows t, t + 16, …
// and the near-field pairs row[l] + t, row[l] + t + 16, … (coalesced across the lanes), then a
// fixed-order lane reduction; thread g·kRowLanes + t. The lanes of a node sit in one wave and
// take the same branches.
static __global__ void __launch_bounds__(kBlock) k_reduce_batch(int ntot, const int* __restrict__ mol_of,
                                                                const MolDev* __restrict__ mols,
                                                                const int* __restrict__ active, int mode,
                                                                const double* __restrict__ partial,
                                                                const double* __restrict__ x, double* __restrict__ y,
                                                                const int* __restrict__ kptr, int kmax, int64_t ldv,
                                                                double lam1, double lam2) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int g = (int)(t / kRowLanes), lane = (int)(t % kRowLanes);
  if (g >= ntot) return;
  const int mi = mol_of[g];
  if (!active[mi]) return;
  if (kptr && *kptr >= kmax) return;
  const MolDev& m = mols[mi];
  const int64_t k = kptr ? *kptr : 0;
  const double* xv = x + k * ldv;
  double* yv = y + (kptr ? (k + 1) * ldv : 0);
  const int l = g - m.off;
  const bool use64 = mode == kModeF64 || mode == kModeF64Sym;  // the FP64 operator has no near field
  const bool sym = mode == kModeSym || mode == kModeF64Sym;
  const int S = sym ? m.Ssym : use64 ? m.S64 : m.S32;
  const double* part = partial + (sym ? m.poffsym : use64 ? m.poff64 : m.poff32);
  double s1 = 0.0, s2 = 0.0;
  for (int c = lane; c < S; c += kRowLanes) {
    s1 += part[(int64_t)c * 2 * m.n + l];
    s2 += part[(int64_t)c * 2 * m.n + m.n + l];
  }
  if (!use64) {  // FP64 near field
    const int64_t e = m.row[l + 1];
    for (int64_t q = m.row[l] + lane; q < e; q += kRowLanes) {
      const int j = m.col[q];
      const double4 cf = m.coef[q];
      const double ps = xv[2 * (int64_t)m.off + j], pn = xv[2 * (int64_t)m.off + m.n + j];
      s1 += cf.x * ps + cf.y * pn;
      s2 += cf.z * ps + cf.w * pn;
    }
  }
  for (int off = kRowLanes / 2; off > 0; off >>= 1) {
    s1 += __shfl_down(s1, off, kRowLanes);
    s2 += __shfl_down(s2, off, kRowLanes);
  }
  if (lane == 0) {
    const int64_t e1 = 2 * (int64_t)m.off + l, e2 = e1 + m.n;
    yv[e1] = lam1 * xv[e1] + s1;
    yv[e2] = lam2 * xv[e2] + s2;
  }
}

// ---------------------------------------------------------------- Krylov kernels

// Blocks of kSeg elements, each inside one molecule's segment: seg_mol[b], seg_lo[b], seg_hi[b].
struct Segs {
  const int* mol;
  const int64_t* lo;
  const int64_t* hi;
  const int* first;  // first block of each molecule (n_mol + 1 entries)
};

// partial[b·(m+1) + q] = Σ_{e in block b} w[e]·V[q][e] for q ≤ k (k = *kptr, or kfix when kptr
// is null), w = V[k+1] (or wfix).
static __global__ void __launch_bounds__(kBlock) k_dots_batch(int nseg, Segs sg, const int* __restrict__ active,
                                                              const double* __restrict__ V, int64_t ldv,
                                                              const int* __restrict__ kptr, int kmax, int nq_fixed,
                                                              const double* __restrict__ wfix, int mstride,
                                                              double* __restrict__ partial) {
  __shared__ double red[kBlock];
  const int b = blockIdx.x;
  if (b >= nseg || !active[sg.mol[b]]) return;
  if (kptr && *kptr >= kmax) return;
  const int nq = kptr ? *kptr + 1 : nq_fixed;
  const double* w = wfix ? wfix : V + (int64_t)nq * ldv;
  for (int q = 0; q < nq; ++q) {
    const double* vq = V + (int64_t)q * ldv;
    double a = 0.0;
    for (int64_t e = sg.lo[b] + threadIdx.x; e < sg.hi[b]; e += kBlock) a += w[e] * vq[e];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)b * mstride + q] = red[0];
    __syncthreads();
  }
}

// out[mol·ostride + q] = Σ_{blocks of mol} partial[b·mstride + q]; sqrt if asked.
static __global__ void __launch_bounds__(64) k_dots_finish_batch(int n_mol, Segs sg, const int* __restrict__ active,
                                                                 const double* __restrict__ partial, int mstride,
                                                                 const int* __restrict__ kptr, int kmax, int nq_fixed,
                                                                 double* __restrict__ out, int ostride, int sqrt_out) {
  const int mol = blockIdx.x;
  const int q = blockIdx.y;
  if (mol >= n_mol || !active[mol]) return;
  if (kptr && *kptr >= kmax) return;
  const int nq = kptr ? *kptr + 1 : nq_fixed;
  if (q >= nq) return;
  __shared__ double red[64];
  double a = 0.0;
  for (int b = sg.first[mol] + threadIdx.x; b < sg.first[mol + 1]; b += 64) a += partial[(int64_t)b * mstride + q];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int off = 32; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(int64_t)mol * ostride + q] = sqrt_out ? sqrt(red[0]) : red[0];
}

// w[e] += sign·Σ_{q<nq} c[mol][q] V[q][e] over each active molecule's elements.
static __global__ void __launch_bounds__(kBlock) k_axpy_batch(int nseg, Segs sg, const int* __restrict__ active,
                                                              const double* __restrict__ V, int64_t ldv,
                                                              const int* __restrict__ kptr, int kmax,
                                                              const int* __restrict__ nq_mol,
                                                              const double* __restrict__ c, int cstride, double sign,
                                                              double* __restrict__ wfix) {
  const int b = blockIdx.x;
  if (b >= nseg) return;
  const int mol = sg.mol[b];
  if (!active[mol]) return;
  if (kptr && *kptr >= kmax) return;
  const int nq = kptr ? *kptr + 1 : nq_mol[mol];
  double* w = wfix ? wfix : const_cast<double*>(V) + (int64_t)nq * ldv;
  const double* cm = c + (int64_t)mol * cstride;
  for (int64_t e = sg.lo[b] + threadIdx.x; e < sg.hi[b]; e += kBlock) {
    double s = 0.0;
    for (int q = 0; q < nq; ++q) s += cm[q] * V[(int64_t)q * ldv + e];
    w[e] += sign * s;
  }
}

// dst[e] = src[e] / nrm[mol] over each active molecule's elements (dst, src at basis steps
// given by kptr offsets: src = V[*kptr + ks], dst = V[*kptr + kd]; or fixed pointers).
static __global__ void __launch_bounds__(kBlock) k_scale_batch(int nseg, Segs sg, const int* __restrict__ active,
                                                               double* __restrict__ V, int64_t ldv,
                                                               const int* __restrict__ kptr, int kmax, int ks, int kd,
                                                               const double* __restrict__ src_fix,
                                                               const double* __restrict__ nrm, int nstride) {
  const int b = blockIdx.x;
  if (b >= nseg) return;
  const int mol = sg.mol[b];
  if (!active[mol]) return;
  if (kptr && *kptr >= kmax) return;
  const int64_t k = kptr ? *kptr : 0;
  const double* src = src_fix ? src_fix : V + (k + ks) * ldv;
  double* dst = V + (k + kd) * ldv;
  const double s = 1.0 / nrm[(int64_t)mol * nstride];
  for (int64_t e = sg.lo[b] + threadIdx.x; e < sg.hi[b]; e += kBlock) dst[e] = src[e] * s;
}

// One thread per molecule: the new Hessenberg column from the two Gram–Schmidt passes and
// the norm, the previous rotations, a new rotation, the residual estimate and the stop test.
static __global__ void k_givens_batch(int n_mol, int m, const int* __restrict__ kptr, const double* __restrict__ h,
                                      int hstride, double* __restrict__ H, double* __restrict__ cs,
                                      double* __restrict__ sn, double* __restrict__ s, KState* __restrict__ st,
                                      int* __restrict__ active, int* __restrict__ n_active) {
  const int mol = blockIdx.x * blockDim.x + threadIdx.x;
  if (mol >= n_mol || !active[mol]) return;
  const int k = *kptr;
  if (k >= m) return;
  const double* hm = h + (int64_t)mol * hstride;  // [pass1 (m+1) | pass2 (m+1) | norm]
  double* Hm = H + (int64_t)mol * (m + 1) * m;
  double* csm = cs + (int64_t)mol * m;
  double* snm = sn + (int64_t)mol * m;
  double* sm = s + (int64_t)mol * (m + 1);
  const double hn = hm[2 * (m + 1)];
  for (int i = 0; i <= k; ++i) Hm[(int64_t)i * m + k] = hm[i] + hm[(m + 1) + i];
  Hm[(int64_t)(k + 1) * m + k] = hn;
  for (int i = 0; i < k; ++i) {
    const double a = Hm[(int64_t)i * m + k], b = Hm[(int64_t)(i + 1) * m + k];
    Hm[(int64_t)i * m + k] = csm[i] * a + snm[i] * b;
    Hm[(int64_t)(i + 1) * m + k] = -snm[i] * a + csm[i] * b;
  }
  const double a = Hm[(int64_t)k * m + k], b = Hm[(int64_t)(k + 1) * m + k];
  const double den = sqrt(a * a + b * b);
  csm[k] = den > 0 ? a / den : 1.0;
  snm[k] = den > 0 ? b / den : 0.0;
  Hm[(int64_t)k * m + k] = den;
  Hm[(int64_t)(k + 1) * m + k] = 0.0;
  sm[k + 1] = -snm[k] * sm[k];
  sm[k] = csm[k] * sm[k];
  st[mol].k_used = k + 1;
  st[mol].iters += 1;
  const bool reached = fabs(sm[k + 1]) <= st[mol].tol_abs || !(hn > 0.0);
  if (reached || k + 1 >= m) {
    st[mol].early = reached;
    st[mol].t_inner = wall_clock64();
    active[mol] = 0;
    atomicSub(n_active, 1);
  }
}

// partial[b] = Σ_{e in block b} w[e]² with w = V[*kptr + 1].
static __global__ void __launch_bounds__(kBlock) k_wnorm_batch(int nseg, Segs sg, const int* __restrict__ active,
                                                               const double* __restrict__ V, int64_t ldv,
                                                               const int* __restrict__ kptr, int kmax,
                                                               double* __restrict__ partial) {
  __shared__ double red[kBlock];
  const int b = blockIdx.x;
  if (b >= nseg || !active[sg.mol[b]]) return;
  if (*kptr >= kmax) return;
  const double* w = V + (int64_t)(*kptr + 1) * ldv;
  double a = 0.0;
  for (int64_t e = sg.lo[b] + threadIdx.x; e < sg.hi[b]; e += kBlock) a += w[e] * w[e];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[b] = red[0];
}

static __global__ void k_advance(int* kptr, int kmax) {
  if (*kptr < kmax) *kptr += 1;
}

// One thread per molecule: y = H⁻¹ s over the k_used steps (upper triangular).
static __global__ void k_trisolve_batch(int n_mol, int m, const int* __restrict__ cycle_active,
                                        const double* __restrict__ H, const double* __restrict__ s,
                                        const KState* __restrict__ st, double* __restrict__ y, int* __restrict__ nq) {
  const int mol = blockIdx.x * blockDim.x + threadIdx.x;
  if (mol >= n_mol) return;
  const int k = cycle_active[mol] ? st[mol].k_used : 0;
  nq[mol] = k;
  const double* Hm = H + (int64_t)mol * (m + 1) * m;
  const double* sm = s + (int64_t)mol * (m + 1);
  double* ym = y + (int64_t)mol * m;
  for (int i = k - 1; i >= 0; --i) {
    double acc = sm[i];
    for (int j = i + 1; j < k; ++j) acc -= Hm[(int64_t)i * m + j] * ym[j];
    ym[i] = acc / Hm[(int64_t)i * m + i];
  }
}

// Start of a cycle: s = [β, 0, …], active, tolerance; one thread per molecule.
static __global__ void k_cycle_init(int n_mol, int m, const double* __restrict__ beta,
                                    const double* __restrict__ tol_abs, const int* __restrict__ want,
                                    double* __restrict__ s, KState* __restrict__ st, int* __restrict__ active,
                                    int* __restrict__ n_active, int* __restrict__ kptr) {
  const int mol = blockIdx.x * blockDim.x + threadIdx.x;
  if (mol == 0) *kptr = 0;
  if (mol >= n_mol) return;
  double* sm = s + (int64_t)mol * (m + 1);
  for (int i = 0; i <= m; ++i) sm[i] = 0.0;
  sm[0] = beta[mol];
  st[mol].beta = beta[mol];
  st[mol].tol_abs = tol_abs[mol];
  st[mol].k_used = 0;
  st[mol].early = 0;
  const int a = want[mol] && beta[mol] > tol_abs[mol];
  active[mol] = a;
  if (a) atomicAdd(n_active, 1);
}

// End of a cycle: a molecule whose cycle ended on its residual estimate leaves the inner
// solve (the refinement forms its FP64 residual next); the others restart. One thread per
// molecule.
static __global__ void k_drop_early(int n_mol, const KState* __restrict__ st, int* __restrict__ cycle) {
  const int mol = blockIdx.x * blockDim.x + threadIdx.x;
  if (mol < n_mol && st[mol].early) cycle[mol] = 0;
}

static __global__ void __launch_bounds__(kBlock) k_fill_mol(int* mol_of, int off, int n, int m) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) mol_of[off + i] = m;
}

static __global__ void __launch_bounds__(kBlock) k_copy(int64_t M, const double* __restrict__ a, double* __restrict__ b) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < M; e += (int64_t)gridDim.x * kBlock) b[e] = a[e];
}

static __global__ void __launch_bounds__(kBlock) k_zero_vec(int64_t M, double* __restrict__ x) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < M; e += (int64_t)gridDim.x * kBlock) x[e] = 0.0;
}

// r = b − r over the molecules in sel.
static __global__ void __launch_bounds__(kBlock) k_resid_keep(int ntot, const int* __restrict__ mol_of,
                                                              const MolDev* __restrict__ mols,
                                                              const int* __restrict__ sel, const double* __restrict__ b,
                                                              double* __restrict__ r) {
  const int gi = blockIdx.x * kBlock + threadIdx.x;
  if (gi >= ntot) return;
  const int mi = mol_of[gi];
  if (!sel[mi]) return;
  const MolDev& m = mols[mi];
  const int64_t e1 = 2 * (int64_t)m.off + (gi - m.off), e2 = e1 + m.n;
  r[e1] = b[e1] - r[e1];
  r[e2] = b[e2] - r[e2];
}

// r = g − r and d = 0 for molecules in `sel`; x = Λ⁻¹g when diag is set.
static __global__ void __launch_bounds__(kBlock) k_resid_batch(int ntot, const int* __restrict__ mol_of,
                                                               const MolDev* __restrict__ mols,
                                                               const int* __restrict__ sel, const double* __restrict__ g,
                                                               double* __restrict__ r, double* __restrict__ d) {
  const int gi = blockIdx.x * kBlock + threadIdx.x;
  if (gi >= ntot) return;
  const int mi = mol_of[gi];
  if (!sel[mi]) return;
  const MolDev& m = mols[mi];
  const int64_t e1 = 2 * (int64_t)m.off + (gi - m.off), e2 = e1 + m.n;
  r[e1] = g[e1] - r[e1];
  r[e2] = g[e2] - r[e2];
  d[e1] = 0.0;
  d[e2] = 0.0;
}

static __global__ void __launch_bounds__(kBlock) k_diag_batch(int ntot, const int* __restrict__ mol_of,
                                                              const MolDev* __restrict__ mols,
                                                              const double* __restrict__ g, double lam1, double lam2,
                                                              double* __restrict__ x) {
  const int gi = blockIdx.x * kBlock + threadIdx.x;
  if (gi >= ntot) return;
  const MolDev& m = mols[mol_of[gi]];
  const int64_t e1 = 2 * (int64_t)m.off + (gi - m.off), e2 = e1 + m.n;
  x[e1] = g[e1] / lam1;
  x[e2] = g[e2] / lam2;
}

// x = Λ⁻¹g over molecules whose last residual is not finite (before the plain-GMRES rerun).
static __global__ void __launch_bounds__(kBlock) k_reset_nonfinite(int ntot, const int* __restrict__ mol_of,
                                                                   const MolDev* __restrict__ mols,
                                                                   const double* __restrict__ relres,
                                                                   const double* __restrict__ g, double lam1,
                                                                   double lam2, double* __restrict__ x) {
  const int gi = blockIdx.x * kBlock + threadIdx.x;
  if (gi >= ntot) return;
  const int mi = mol_of[gi];
  if (isfinite(relres[mi])) return;
  const MolDev& m = mols[mi];
  const int64_t e1 = 2 * (int64_t)m.off + (gi - m.off), e2 = e1 + m.n;
  x[e1] = g[e1] / lam1;
  x[e2] = g[e2] / lam2;
}

// x += d over molecules in sel
static __global__ void __launch_bounds__(kBlock) k_add_batch(int nseg, Segs sg, const int* __restrict__ sel,
                                                             const double* __restrict__ d, double* __restrict__ x) {
  const int b = blockIdx.x;
  if (b >= nseg || !sel[sg.mol[b]]) return;
  for (int64_t e = sg.lo[b] + threadIdx.x; e < sg.hi[b]; e += kBlock) x[e] += d[e];
}

// relres per molecule and the outer-loop selection: sel[m] = relres > tol (done otherwise;
// its time to solution is when its last restart cycle ended, or now if it ran none); the next
// inner solve's target max(½·tol·‖g‖, η·‖r‖).
static __global__ void k_outer_check(int n_mol, const double* __restrict__ rn, const double* __restrict__ gn,
                                     double tol, double eta, int* __restrict__ sel, double* __restrict__ relres,
                                     double* __restrict__ tol_abs, KState* __restrict__ st, int* __restrict__ n_sel) {
  const int mol = blockIdx.x * blockDim.x + threadIdx.x;
  if (mol >= n_mol || !sel[mol]) return;
  const double rr = rn[mol] / gn[mol];
  relres[mol] = rr;
  tol_abs[mol] = fmax(0.5 * tol * gn[mol], eta * rn[mol]);
  if (rr <= tol) {  // a non-finite residual stays selected
    sel[mol] = 0;
    st[mol].t_done = st[mol].t_inner ? st[mol].t_inner : wall_clock64();
  } else {
    atomicAdd(n_sel, 1);
  }
}

// Target of the first inner pass of the selected molecules, whose residual comes from the
// mixed operator: the same max(½·tol·‖g‖, η·‖r‖) as after an FP64 residual, no convergence
// decision.
static __global__ void k_first_target(int n_mol, const double* __restrict__ rn, const double* __restrict__ gn,
                                      double tol, double eta, const int* __restrict__ sel,
                                      double* __restrict__ tol_abs) {
  const int mol = blockIdx.x * blockDim.x + threadIdx.x;
  if (mol >= n_mol || !sel[mol]) return;
  tol_abs[mol] = fmax(0.5 * tol * gn[mol], eta * rn[mol]);
}

static __global__ void k_stamp(unsigned long long* t) { *t = wall_clock64(); }

}  // namespace


// ---------------------------------------------------------------- host side

namespace {

constexpr int kNumTiledB = 4;           // tile shapes of the one-directional kernel
constexpr int kSymB = kNumTiledB;        // the symmetric kernel
constexpr int kNumCfgB = kNumTiledB + 1;
constexpr int kChunk32 = 4096, kChunk64 = 2048;

struct Batch {
  pb_ctx* ctx = nullptr;
  hipStream_t st = nullptr;
  int n_mol = 0, ntot = 0, m = 0, hstride = 0, nseg = 0, cfg = 0;
  int64_t M = 0;
  Derived d{};
  double sigma = 1.0;
  std::vector<MolDev> mols_h;
  MolDev* mols = nullptr;
  int* mol_of = nullptr;
  Segs segs{};
  Item* items32[kNumCfgB] = {};
  int n_items32[kNumCfgB] = {}, grid32[kNumCfgB] = {};
  Item* items64 = nullptr;
  int n_items64 = 0, grid64 = 0;
  int grid64sym = 0;
  int cfg64 = 0;  // FP64 operator kernel: 0 tiled, 1 symmetric (over items32[kSymB])
  double* partial = nullptr;  // far-field chunk sums of either path
  double* wpsi = nullptr;
  double* wpsn = nullptr;
  double* dpart = nullptr;  // per-block partial dots, nseg × (m+1)
  // Krylov
  double* V = nullptr;
  double* Z = nullptr;  // preconditioned basis (flexible GMRES), learned path only
  const NNBatch* nb = nullptr;
  const pb_nn* net = nullptr;
  double* H = nullptr;
  double* cs = nullptr;
  double* sn = nullptr;
  double* s = nullptr;
  double* hbuf = nullptr;
  double* ybuf = nullptr;
  int* nq = nullptr;
  KState* kst = nullptr;
  int* active = nullptr;  // iterating in the current Arnoldi cycle
  int* cycle = nullptr;   // took part in the current cycle
  int* n_active = nullptr;
  int* kptr = nullptr;
};

template <int TILE, int TPL>
void launch_far32_t(Batch& B, int c, const int* active, const F32Params& fp, double sig1, double sig2) {
  if (B.d.kappa > 0.0)
    k_far32_batch<TILE, TPL, true><<<B.grid32[c], kBlock, 0, B.st>>>(B.items32[c], B.n_items32[c], B.mols, kChunk32,
                                                                      active, fp, sig1, sig2, B.partial);
  else
    k_far32_batch<TILE, TPL, false><<<B.grid32[c], kBlock, 0, B.st>>>(B.items32[c], B.n_items32[c], B.mols, kChunk32,
                                                                       active, fp, sig1, sig2, B.partial);
}

constexpr int kCfgTile[kNumCfgB] = {256, 512, 256, 512, kSymSub};
constexpr int kCfgTpl[kNumCfgB] = {1, 1, 2, 2, 2};

void launch_far32(Batch& B, int c, const int* active, const F32Params& fp, double sig1, double sig2) {
  if (c == kSymB) {
    if (B.d.kappa > 0.0)
      k_far32_sym_batch<true><<<B.grid32[c], kBlock, 0, B.st>>>(B.items32[c], B.n_items32[c], B.mols, active, fp,
                                                                 sig1, sig2, B.partial);
    else
      k_far32_sym_batch<false><<<B.grid32[c], kBlock, 0, B.st>>>(B.items32[c], B.n_items32[c], B.mols, active, fp,
                                                                  sig1, sig2, B.partial);
    return;
  }
  switch (c) {
    case 0: launch_far32_t<256, 1>(B, c, active, fp, sig1, sig2); break;
    case 1: launch_far32_t<512, 1>(B, c, active, fp, sig1, sig2); break;
    case 2: launch_far32_t<256, 2>(B, c, active, fp, sig1, sig2); break;
    default: launch_far32_t<512, 2>(B, c, active, fp, sig1, sig2); break;
  }
}

template <int TILE, int TPL>
int grid_for_t(pb_ctx* ctx, bool screened) {
  int per_cu = 0;
  const void* kern = screened ? (const void*)k_far32_batch<TILE, TPL, true> : (const void*)k_far32_batch<TILE, TPL, false>;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, 0) != hipSuccess || per_cu < 1) per_cu = 2;
  return per_cu * ctx->n_cu;
}

int grid_for(pb_ctx* ctx, int c, bool screened) {
  if (c == kSymB) {
    int per_cu = 0;
    const void* kern = screened ? (const void*)k_far32_sym_batch<true> : (const void*)k_far32_sym_batch<false>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, 0) != hipSuccess || per_cu < 1) per_cu = 2;
    return per_cu * ctx->n_cu;
  }
  switch (c) {
    case 0: return grid_for_t<256, 1>(ctx, screened);
    case 1: return grid_for_t<512, 1>(ctx, screened);
    case 2: return grid_for_t<256, 2>(ctx, screened);
    default: return grid_for_t<512, 2>(ctx, screened);
  }
}

// Work items of about equal size — (molecule, target block of kBlock·tpl, source chunk) —
// ordered by cost, largest first.
std::vector<Item> make_items(const std::vector<MolDev>& mols, int tpl, int chunk) {
  std::vector<std::pair<int64_t, Item>> v;
  for (int mi = 0; mi < (int)mols.size(); ++mi) {
    const int n = mols[mi].n, tb = (n + kBlock * tpl - 1) / (kBlock * tpl), S = (n + chunk - 1) / chunk;
    for (int t = 0; t < tb; ++t)
      for (int c = 0; c < S; ++c) {
        const int64_t nt = std::min(kBlock * tpl, n - t * kBlock * tpl), ns = std::min(chunk, n - c * chunk);
        v.push_back({nt * ns, Item{mi, t, c}});
      }
  }
  std::stable_sort(v.begin(), v.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  std::vector<Item> out(v.size());
  for (size_t i = 0; i < v.size(); ++i) out[i] = v[i].second;
  return out;
}

// Work items (molecule, Ic, Jc) of the symmetric kernel, ordered by cost (a diagonal chunk
// pair costs about half an off-diagonal one), largest first.
std::vector<Item> make_sym_items(const std::vector<MolDev>& mols) {
  std::vector<std::pair<int64_t, Item>> v;
  for (int mi = 0; mi < (int)mols.size(); ++mi) {
    const int n = mols[mi].n, C = mols[mi].nsub * kSymSub, nc = mols[mi].Ssym;
    for (int i = 0; i < nc; ++i)
      for (int j = i; j < nc; ++j) {
        const int64_t ni = std::min(C, n - i * C), nj = std::min(C, n - j * C);
        v.push_back({i == j ? ni * nj / 2 : ni * nj, Item{mi, i, j}});
      }
  }
  std::stable_sort(v.begin(), v.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  std::vector<Item> out(v.size());
  for (size_t i = 0; i < v.size(); ++i) out[i] = v[i].second;
  return out;
}

// FP64 far sums of the molecules in sel, with kernel cfg (0 tiled, 1 symmetric).
void far64(Batch& B, int cfg, const int* sel) {
  if (cfg == 1)
    k_far64_sym_batch<<<B.grid64sym, kBlock, 0, B.st>>>(B.items32[kSymB], B.n_items32[kSymB], B.mols, sel, B.wpsi,
                                                        B.wpsn, kparams(B.d), B.d.kappa * B.d.kappa, B.partial);
  else
    k_far64_batch<<<B.grid64, kBlock, 0, B.st>>>(B.items64, B.n_items64, B.mols, kChunk64, sel, B.wpsi, B.wpsn,
                                                 kparams(B.d), B.partial);
}

// Blocks of k_reduce_batch: kRowLanes threads per node.
unsigned reduce_blocks(const Batch& B) { return (unsigned)(((int64_t)B.ntot * kRowLanes + kBlock - 1) / kBlock); }

// Molecules selected by `sel` get y = A x with the FP64 operator (persistent launch).
void op64(Batch& B, const double* x, double* y, const int* sel) {
  const unsigned nbn = (unsigned)((B.ntot + kBlock - 1) / kBlock);
  k_weights_batch<<<nbn, kBlock, 0, B.st>>>(B.ntot, B.mol_of, B.mols, x, B.d.h3 / (4.0 * kPi), B.wpsi, B.wpsn);
  far64(B, B.cfg64, sel);
  k_reduce_batch<<<reduce_blocks(B), kBlock, 0, B.st>>>(B.ntot, B.mol_of, B.mols, sel,
                                                        B.cfg64 ? kModeF64Sym : kModeF64, B.partial, x, y, nullptr,
                                                        0, 0, B.d.lam1, B.d.lam2);
}

// Mixed operator: y = A x for molecules in `act`; with kptr, x = V[*kptr] and y = V[*kptr+1].
void op_mixed(Batch& B, const double* x, double* y, const int* kptr, int64_t ldv, const int* act) {
  const unsigned nbn = (unsigned)((B.ntot + kBlock - 1) / kBlock);
  k_pack_batch<<<nbn, kBlock, 0, B.st>>>(B.ntot, B.mol_of, B.mols, x, kptr, B.m, ldv, B.d.h3 / (4.0 * kPi), B.sigma);
  launch_far32(B, B.cfg, act, f32params(B.d, B.sigma), B.sigma, B.sigma * B.sigma);
  k_reduce_batch<<<reduce_blocks(B), kBlock, 0, B.st>>>(B.ntot, B.mol_of, B.mols, act,
                                                        B.cfg == kSymB ? kModeSym : kModeTiled, B.partial, x, y,
                                                        kptr, B.m, ldv, B.d.lam1, B.d.lam2);
}

// Per-molecule 2-norms of v over the molecules in sel, into out[mol].
void norms(Batch& B, const double* v, const int* sel, double* out) {
  k_dots_batch<<<B.nseg, kBlock, 0, B.st>>>(B.nseg, B.segs, sel, v, 0, nullptr, 0, 1, v, 1, B.dpart);
  k_dots_finish_batch<<<dim3(B.n_mol, 1), 64, 0, B.st>>>(B.n_mol, B.segs, sel, B.dpart, 1, nullptr, 0, 1, out, 1, 1);
}

// One Arnoldi step of every active molecule (the graph body): w = A V[k] (with prec:
// Z[k] = M(V[k]), w = A Z[k]), two classical Gram–Schmidt passes, the norm, Givens,
// scaling, k += 1.
void arnoldi_step(Batch& B, bool prec) {
  const int m = B.m, hs = B.hstride;
  if (prec) {
    nn_batch_apply(B.st, B.net, *B.nb, B.V, B.Z, B.M, B.kptr, m, B.d.lam1, B.d.lam2);
    op_mixed(B, B.Z, B.V, B.kptr, B.M, B.active);
  } else {
    op_mixed(B, B.V, B.V, B.kptr, B.M, B.active);
  }
  for (int pass = 0; pass < 2; ++pass) {
    double* hv = B.hbuf + pass * (m + 1);
    k_dots_batch<<<B.nseg, kBlock, 0, B.st>>>(B.nseg, B.segs, B.active, B.V, B.M, B.kptr, m, 0, nullptr, m + 1,
                                              B.dpart);
    k_dots_finish_batch<<<dim3(B.n_mol, m), 64, 0, B.st>>>(B.n_mol, B.segs, B.active, B.dpart, m + 1, B.kptr, m, 0, hv,
                                                           hs, 0);
    k_axpy_batch<<<B.nseg, kBlock, 0, B.st>>>(B.nseg, B.segs, B.active, B.V, B.M, B.kptr, m, nullptr, hv, hs, -1.0,
                                              nullptr);
  }
  k_wnorm_batch<<<B.nseg, kBlock, 0, B.st>>>(B.nseg, B.segs, B.active, B.V, B.M, B.kptr, m, B.dpart);
  k_dots_finish_batch<<<dim3(B.n_mol, 1), 64, 0, B.st>>>(B.n_mol, B.segs, B.active, B.dpart, 1, nullptr, 0, 1,
                                                         B.hbuf + 2 * (m + 1), hs, 1);
  k_givens_batch<<<(B.n_mol + 63) / 64, 64, 0, B.st>>>(B.n_mol, m, B.kptr, B.hbuf, hs, B.H, B.cs, B.sn, B.s, B.kst,
                                                       B.active, B.n_active);
  k_scale_batch<<<B.nseg, kBlock, 0, B.st>>>(B.nseg, B.segs, B.active, B.V, B.M, B.kptr, m, 1, 1, nullptr,
                                             B.hbuf + 2 * (m + 1), hs);
  k_advance<<<1, 1, 0, B.st>>>(B.kptr, m);
}

}  // namespace
}  // namespace pb

extern "C" pb_status pb_ibim_solve_batched(pb_ctx* ctx, int n_mol, const pb_band* bands, const double* const* atoms,
                                           const int* n_atoms, const pb_params* prm, const pb_solve_opts* opts_in,
                                           double* const* p, pb_solve_stats* stats, pb_batch_stats* bstats) {
  using namespace pb;
  auto t_start = std::chrono::steady_clock::now();
  if (!ctx) return PB_EINVAL;
  PB_TRY(check_params(ctx, prm));
  if (n_mol < 1 || !bands || !atoms || !n_atoms || !p) return ctx->fail(PB_EINVAL, "pb_ibim_solve_batched: bad batch");
  pb_solve_opts opts;
  if (opts_in) opts = *opts_in;
  else pb_default_solve_opts(&opts);
  if (!(opts.tol > 0.0) || opts.max_iter < 1 || opts.restart < 1 || opts.restart > 1000)
    return ctx->fail(PB_EINVAL, "bad tolerance or iteration limits");
  if (opts.precision != PB_FP64 && opts.precision != PB_MIXED) return ctx->fail(PB_EINVAL, "unknown precision");
  if (prm->reg_metric == PB_REG_TANGENT)
    return ctx->fail(PB_EINVAL, "the batched path needs a bounded regularization radius (guarded or Euclidean)");
  if (opts.x0 < PB_X0_ZERO || opts.x0 > PB_X0_LEARNED) return ctx->fail(PB_EINVAL, "unknown x0 mode %d", opts.x0);
  if (opts.precond != PB_PRECOND_NONE && opts.precond != PB_PRECOND_LEARNED)
    return ctx->fail(PB_EINVAL, "unknown preconditioner %d", opts.precond);
  const bool learned_x0 = opts.x0 == PB_X0_LEARNED, prec = opts.precond == PB_PRECOND_LEARNED;
  if ((learned_x0 || prec) && !opts.nn) return ctx->fail(PB_EINVAL, "the learned path needs opts->nn");
  int64_t ntot64 = 0;
  for (int i = 0; i < n_mol; ++i) {
    PB_TRY(check_band(ctx, &bands[i]));
    if (!atoms[i] || n_atoms[i] <= 0 || !p[i]) return ctx->fail(PB_EINVAL, "molecule %d: NULL input", i);
    ntot64 += bands[i].n;
  }
  if (ntot64 > (int64_t)1 << 30) return ctx->fail(PB_EINVAL, "batch larger than 2^30 nodes");
  PB_HIP(ctx, hipSetDevice(ctx->device));
  if (!ctx->batch_stream) PB_HIP(ctx, hipStreamCreateWithFlags(&ctx->batch_stream, hipStreamNonBlocking));

  Batch B;
  B.ctx = ctx;
  B.st = ctx->batch_stream;
  B.n_mol = n_mol;
  B.ntot = (int)ntot64;
  B.M = 2 * ntot64;
  B.m = opts.restart;
  B.hstride = 2 * (B.m + 1) + 1;
  B.d = derive(*prm);
  B.sigma = B.d.kappa > 0.0 ? B.d.kappa : 1.0;
  const int m = B.m;

  // per-molecule geometry: FP32 records and near-field CSR on the context stream
  B.mols_h.resize(n_mol);
  int64_t off = 0, p32 = 0, p64 = 0, psym = 0;
  for (int i = 0; i < n_mol; ++i) {
    char pfx[32];
    snprintf(pfx, sizeof(pfx), "bt%d_", i);
    MixedPlan P;
    PB_TRY(near_build(ctx, &bands[i], B.d, pfx, P));
    MolDev& md = B.mols_h[i];
    md.off = (int)off;
    md.n = (int)bands[i].n;
    md.S32 = (md.n + kChunk32 - 1) / kChunk32;
    md.S64 = (md.n + kChunk64 - 1) / kChunk64;
    md.Ssym = sym_chunks(md.n);
    md.nsub = sym_nsub(md.n);
    md.poff32 = p32;
    md.poff64 = p64;
    md.poffsym = psym;
    md.cx = P.cx;
    md.cy = P.cy;
    md.cz = P.cz;
    md.band = band_dev(&bands[i]);
    md.w = bands[i].w;
    md.A = P.A;
    md.M = P.M;
    md.N = P.N;
    md.box = P.box;
    md.row = P.row;
    md.col = P.col;
    md.coef = P.coef;
    off += md.n;
    p32 += (int64_t)md.S32 * 2 * md.n;
    p64 += (int64_t)md.S64 * 2 * md.n;
    psym += (int64_t)md.Ssym * 2 * md.n;
  }
  // segments of kSeg vector elements within each molecule
  std::vector<int> seg_mol, first(n_mol + 1);
  std::vector<int64_t> seg_lo, seg_hi;
  for (int i = 0; i < n_mol; ++i) {
    first[i] = (int)seg_mol.size();
    const int64_t lo = 2 * (int64_t)B.mols_h[i].off, hi = lo + 2 * (int64_t)B.mols_h[i].n;
    for (int64_t e = lo; e < hi; e += kSeg) {
      seg_mol.push_back(i);
      seg_lo.push_back(e);
      seg_hi.push_back(std::min(hi, e + kSeg));
    }
  }
  first[n_mol] = (int)seg_mol.size();
  B.nseg = (int)seg_mol.size();

  auto ws = [&](const char* name, size_t bytes) { return workspace(ctx, name, bytes); };
  B.mols = (MolDev*)ws("bt_mols", sizeof(MolDev) * n_mol);
  B.mol_of = (int*)ws("bt_mol_of", sizeof(int) * B.ntot);
  int* sm = (int*)ws("bt_seg_mol", sizeof(int) * B.nseg);
  int64_t* slo = (int64_t*)ws("bt_seg_lo", sizeof(int64_t) * B.nseg);
  int64_t* shi = (int64_t*)ws("bt_seg_hi", sizeof(int64_t) * B.nseg);
  int* sfirst = (int*)ws("bt_seg_first", sizeof(int) * (n_mol + 1));
  B.partial = (double*)ws("bt_partial", sizeof(double) * (size_t)std::max(std::max(p32, p64), psym));
  B.wpsi = (double*)ws("bt_wpsi", sizeof(double) * B.ntot);
  B.wpsn = (double*)ws("bt_wpsn", sizeof(double) * B.ntot);
  B.dpart = (double*)ws("bt_dpart", sizeof(double) * (size_t)B.nseg * (m + 1));
  B.V = (double*)ws("bt_V", sizeof(double) * (size_t)B.M * (m + 1));
  if (prec) {
    B.Z = (double*)ws("bt_Z", sizeof(double) * (size_t)B.M * m);
    if (!B.Z) return PB_ENOMEM;
  }
  B.H = (double*)ws("bt_H", sizeof(double) * (size_t)n_mol * (m + 1) * m);
  B.cs = (double*)ws("bt_cs", sizeof(double) * (size_t)n_mol * m);
  B.sn = (double*)ws("bt_sn", sizeof(double) * (size_t)n_mol * m);
  B.s = (double*)ws("bt_s", sizeof(double) * (size_t)n_mol * (m + 1));
  B.hbuf = (double*)ws("bt_hbuf", sizeof(double) * (size_t)n_mol * B.hstride);
  B.ybuf = (double*)ws("bt_y", sizeof(double) * (size_t)n_mol * m);
  B.nq = (int*)ws("bt_nq", sizeof(int) * n_mol);
  B.kst = (KState*)ws("bt_kst", sizeof(KState) * n_mol);
  B.active = (int*)ws("bt_active", sizeof(int) * n_mol);
  B.cycle = (int*)ws("bt_cycle", sizeof(int) * n_mol);
  B.n_active = (int*)ws("bt_nact", sizeof(int) * 4);
  B.kptr = B.n_active + 1;
  int* n_sel = B.n_active + 2;
  int* sel = (int*)ws("bt_sel", sizeof(int) * n_mol);
  int* all_on = (int*)ws("bt_all", sizeof(int) * n_mol);
  double* g = (double*)ws("bt_g", sizeof(double) * B.M);
  double* x = (double*)ws("bt_x", sizeof(double) * B.M);
  double* r = (double*)ws("bt_r", sizeof(double) * B.M);
  double* dvec = (double*)ws("bt_d", sizeof(double) * B.M);
  double* gn = (double*)ws("bt_gn", sizeof(double) * n_mol);
  double* rn = (double*)ws("bt_rn", sizeof(double) * n_mol);
  double* tolabs = (double*)ws("bt_tolabs", sizeof(double) * n_mol);
  double* relres = (double*)ws("bt_relres", sizeof(double) * n_mol);
  unsigned long long* t0dev = (unsigned long long*)ws("bt_t0", sizeof(unsigned long long));
  if (!B.mols || !B.mol_of || !sm || !slo || !shi || !sfirst || !B.partial || !B.wpsi || !B.wpsn || !B.dpart || !B.V ||
      !B.H || !B.cs || !B.sn || !B.s || !B.hbuf || !B.ybuf || !B.nq || !B.kst || !B.active || !B.cycle || !B.n_active ||
      !sel || !all_on || !g || !x || !r || !dvec || !gn || !rn || !tolabs || !relres || !t0dev)
    return PB_ENOMEM;
  B.segs = Segs{sm, slo, shi, sfirst};
  // work lists
  std::vector<Item> it64 = make_items(B.mols_h, 1, kChunk64);
  Item* items_all[kNumCfgB + 1];
  std::vector<std::vector<Item>> lists;
  for (int c = 0; c < kNumTiledB; ++c) lists.push_back(make_items(B.mols_h, kCfgTpl[c], kChunk32));
  lists.push_back(make_sym_items(B.mols_h));
  lists.push_back(it64);
  for (int c = 0; c <= kNumCfgB; ++c) {
    char nm[32];
    snprintf(nm, sizeof(nm), "bt_items%d", c);
    items_all[c] = (Item*)ws(nm, sizeof(Item) * std::max<size_t>(lists[c].size(), 1));
    if (!items_all[c]) return PB_ENOMEM;
  }
  // host tables → device (on the context stream, then hand over to the batch stream)
  std::vector<int> ones(n_mol, 1);
  PB_HIP(ctx, hipMemcpyAsync(B.mols, B.mols_h.data(), sizeof(MolDev) * n_mol, hipMemcpyHostToDevice, ctx->stream));
  PB_HIP(ctx, hipMemcpyAsync(sm, seg_mol.data(), sizeof(int) * B.nseg, hipMemcpyHostToDevice, ctx->stream));
  PB_HIP(ctx, hipMemcpyAsync(slo, seg_lo.data(), sizeof(int64_t) * B.nseg, hipMemcpyHostToDevice, ctx->stream));
  PB_HIP(ctx, hipMemcpyAsync(shi, seg_hi.data(), sizeof(int64_t) * B.nseg, hipMemcpyHostToDevice, ctx->stream));
  PB_HIP(ctx, hipMemcpyAsync(sfirst, first.data(), sizeof(int) * (n_mol + 1), hipMemcpyHostToDevice, ctx->stream));
  PB_HIP(ctx, hipMemcpyAsync(all_on, ones.data(), sizeof(int) * n_mol, hipMemcpyHostToDevice, ctx->stream));
  for (int c = 0; c <= kNumCfgB; ++c)
    PB_HIP(ctx, hipMemcpyAsync(items_all[c], lists[c].data(), sizeof(Item) * lists[c].size(), hipMemcpyHostToDevice,
                               ctx->stream));
  for (int c = 0; c < kNumCfgB; ++c) {
    B.items32[c] = items_all[c];
    B.n_items32[c] = (int)lists[c].size();
    B.grid32[c] = std::min(B.n_items32[c], grid_for(ctx, c, B.d.kappa > 0.0));
  }
  B.items64 = items_all[kNumCfgB];
  B.n_items64 = (int)it64.size();
  {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_far64_batch, kBlock, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 2;
    B.grid64 = std::min(B.n_items64, per_cu * ctx->n_cu);
    per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_far64_sym_batch, kBlock, 0) !=
            hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    B.grid64sym = std::min(B.n_items32[kSymB], per_cu * ctx->n_cu);
  }
  for (int i = 0; i < n_mol; ++i) {
    const MolDev& md = B.mols_h[i];
    k_fill_mol<<<(unsigned)((md.n + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(B.mol_of, md.off, md.n, i);
    PB_TRY(rhs(ctx, &bands[i], atoms[i], n_atoms[i], B.d, g + 2 * (int64_t)md.off));
    if (opts.x0 == PB_X0_USER)
      PB_HIP(ctx, hipMemcpyAsync(x + 2 * (int64_t)md.off, p[i], sizeof(double) * 2 * md.n, hipMemcpyDeviceToDevice,
                                 ctx->stream));
  }
  NNBatch nb;
  if (learned_x0 || prec) {
    std::vector<int> off_h(n_mol);
    for (int i = 0; i < n_mol; ++i) off_h[i] = B.mols_h[i].off;
    PB_TRY(nn_batch_prepare(ctx, n_mol, bands, off_h.data(), B.mol_of, B.d, nb));
    B.nb = &nb;
    B.net = (const pb_nn*)opts.nn;
  }
  PB_TRY(launch_ok(ctx, "batch setup"));
  PB_TRY(sync(ctx, "batch setup"));

  const unsigned nbn = (unsigned)((B.ntot + kBlock - 1) / kBlock);
  const unsigned vb = (unsigned)std::min<int64_t>(4096, (B.M + kBlock - 1) / kBlock);
  PB_HIP(ctx, hipMemsetAsync(B.kst, 0, sizeof(KState) * n_mol, B.st));
  k_stamp<<<1, 1, 0, B.st>>>(t0dev);
  if (opts.x0 == PB_X0_DIAG) k_diag_batch<<<nbn, kBlock, 0, B.st>>>(B.ntot, B.mol_of, B.mols, g, B.d.lam1, B.d.lam2, x);
  else if (opts.x0 == PB_X0_ZERO) k_zero_vec<<<vb, kBlock, 0, B.st>>>(B.M, x);
  else if (learned_x0) nn_batch_apply(B.st, B.net, nb, g, x, 0, nullptr, 0, B.d.lam1, B.d.lam2);
  norms(B, g, all_on, gn);
  PB_TRY(launch_ok(ctx, "batch x0"));
  std::vector<double> gn_h(n_mol);
  PB_HIP(ctx, hipMemcpyAsync(gn_h.data(), gn, sizeof(double) * n_mol, hipMemcpyDeviceToHost, B.st));
  PB_HIP(ctx, hipStreamSynchronize(B.st));
  for (double& v : gn_h)
    if (!(v > 0.0)) v = 1.0;
  PB_HIP(ctx, hipMemcpyAsync(gn, gn_h.data(), sizeof(double) * n_mol, hipMemcpyHostToDevice, B.st));

  // far-field tile shape: autotuned once per batch shape
  {
    const int64_t key = (int64_t)B.ntot * 4096 + n_mol;
    auto itc = ctx->batch_cfg.find(key);
    const char* env = std::getenv("PB_FAR_CFG");
    if (itc != ctx->batch_cfg.end()) {
      B.cfg = itc->second;
    } else if (env && std::atoi(env) >= 0 && std::atoi(env) < kNumCfgB) {
      B.cfg = std::atoi(env);
      ctx->batch_cfg[key] = B.cfg;
    } else {
      k_pack_batch<<<nbn, kBlock, 0, B.st>>>(B.ntot, B.mol_of, B.mols, x, nullptr, 0, 0, B.d.h3 / (4.0 * kPi), B.sigma);
      hipEvent_t e0, e1;
      PB_HIP(ctx, hipEventCreate(&e0));
      PB_HIP(ctx, hipEventCreate(&e1));
      float best = 1e30f;
      for (int c = 0; c < kNumCfgB; ++c) {
        launch_far32(B, c, all_on, f32params(B.d, B.sigma), B.sigma, B.sigma * B.sigma);
        PB_HIP(ctx, hipEventRecord(e0, B.st));
        launch_far32(B, c, all_on, f32params(B.d, B.sigma), B.sigma, B.sigma * B.sigma);
        PB_HIP(ctx, hipEventRecord(e1, B.st));
        PB_TRY(launch_ok(ctx, "batch autotune"));
        PB_HIP(ctx, hipEventSynchronize(e1));
        float ms = 0.f;
        PB_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
          best = ms;
          B.cfg = c;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      ctx->batch_cfg[key] = B.cfg;
    }
    // the FP64 operator's kernel, the same way (PB_F64_CFG=<0|1> fixes it)
    auto it64 = ctx->batch_cfg64.find(key);
    const char* env64 = std::getenv("PB_F64_CFG");
    if (it64 != ctx->batch_cfg64.end()) {
      B.cfg64 = it64->second;
    } else if (env64 && (std::atoi(env64) == 0 || std::atoi(env64) == 1)) {
      B.cfg64 = std::atoi(env64);
      ctx->batch_cfg64[key] = B.cfg64;
    } else {
      k_weights_batch<<<nbn, kBlock, 0, B.st>>>(B.ntot, B.mol_of, B.mols, x, B.d.h3 / (4.0 * kPi), B.wpsi, B.wpsn);
      hipEvent_t e0, e1;
      PB_HIP(ctx, hipEventCreate(&e0));
      PB_HIP(ctx, hipEventCreate(&e1));
      float best = 1e30f;
      for (int c = 0; c < 2; ++c) {
        PB_HIP(ctx, hipEventRecord(e0, B.st));
        far64(B, c, all_on);
        PB_HIP(ctx, hipEventRecord(e1, B.st));
        PB_TRY(launch_ok(ctx, "batch autotune"));
        PB_HIP(ctx, hipEventSynchronize(e1));
        float ms = 0.f;
        PB_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
          best = ms;
          B.cfg64 = c;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      ctx->batch_cfg64[key] = B.cfg64;
    }
  }

  // the graph of one Arnoldi step of the batch, captured on first use (with or without
  // the learned preconditioner)
  struct GraphPair {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    ~GraphPair() {
      if (e) (void)hipGraphExecDestroy(e);
      if (g) (void)hipGraphDestroy(g);
    }
  } graphs[2];
  auto graph_for = [&](bool with_prec, hipGraphExec_t* out) -> pb_status {
    GraphPair& gp = graphs[with_prec ? 1 : 0];
    if (!gp.e) {
      PB_HIP(ctx, hipStreamSynchronize(B.st));
      PB_HIP(ctx, hipStreamBeginCapture(B.st, hipStreamCaptureModeThreadLocal));
      arnoldi_step(B, with_prec);
      hipError_t cap = hipStreamEndCapture(B.st, &gp.g);
      if (cap != hipSuccess) return ctx->fail(PB_EDEVICE, "graph capture failed: %s", hipGetErrorString(cap));
      if (hipGraphInstantiate(&gp.e, gp.g, nullptr, nullptr, 0) != hipSuccess)
        return ctx->fail(PB_EDEVICE, "graph instantiation failed");
    }
    *out = gp.e;
    return PB_OK;
  };

  int replays = 0, outer = 0, outer_run = 0, iters_total = 0;
  // iteration budget of the current pass: the learned-preconditioned pass gets at most half of
  // max_iter, so that the plain fallback keeps at least the other half
  int iter_cap = prec ? opts.max_iter - opts.max_iter / 2 : opts.max_iter;
  std::vector<int> mv64(n_mol, 0), mvmx(n_mol, 0), cyc_h(n_mol), sel_h(n_mol);
  PB_HIP(ctx, hipMemcpyAsync(sel, all_on, sizeof(int) * n_mol, hipMemcpyDeviceToDevice, B.st));

  // Inner GMRES on the mixed operator for the molecules in `want`, from d = 0 with residual r.
  double* rr = (double*)ws("bt_rr", sizeof(double) * B.M);
  if (!rr) return PB_ENOMEM;
  auto inner = [&](const int* want, const double* rhs_vec, double* sol, bool with_prec) -> pb_status {
    hipGraphExec_t exec = nullptr;
    PB_TRY(graph_for(with_prec, &exec));
    // sol = 0, so the first residual is the right-hand side itself
    k_copy<<<vb, kBlock, 0, B.st>>>(B.M, rhs_vec, rr);
    norms(B, rr, want, rn);
    for (;;) {
      PB_HIP(ctx, hipMemsetAsync(B.n_active, 0, sizeof(int), B.st));
      k_cycle_init<<<(n_mol + 63) / 64, 64, 0, B.st>>>(n_mol, m, rn, tolabs, want, B.s, B.kst, B.active,
                                                      B.n_active, B.kptr);
      PB_HIP(ctx, hipMemcpyAsync(B.cycle, B.active, sizeof(int) * n_mol, hipMemcpyDeviceToDevice, B.st));
      int nact = 0;
      PB_HIP(ctx, hipMemcpyAsync(&nact, B.n_active, sizeof(int), hipMemcpyDeviceToHost, B.st));
      PB_HIP(ctx, hipStreamSynchronize(B.st));
      if (nact == 0 || iters_total >= iter_cap) break;
      PB_HIP(ctx, hipMemcpyAsync(cyc_h.data(), B.cycle, sizeof(int) * n_mol, hipMemcpyDeviceToHost, B.st));
      // V0 = r0/‖r0‖ (rhs_vec holds r0 when sol = 0, otherwise the refreshed residual in r)
      k_scale_batch<<<B.nseg, kBlock, 0, B.st>>>(B.nseg, B.segs, B.active, B.V, B.M, nullptr, m, 0, 0, rr, rn, 1);
      int steps = 0;
      while (steps < m) {
        const int burst = std::min(4, m - steps);
        for (int q = 0; q < burst; ++q) PB_HIP(ctx, hipGraphLaunch(exec, B.st));
        steps += burst;
        replays += burst;
        PB_HIP(ctx, hipMemcpyAsync(&nact, B.n_active, sizeof(int), hipMemcpyDeviceToHost, B.st));
        PB_HIP(ctx, hipStreamSynchronize(B.st));
        if (nact == 0) break;
      }
      // iterations actually taken this cycle per molecule
      std::vector<KState> ks(n_mol);
      PB_HIP(ctx, hipMemcpyAsync(ks.data(), B.kst, sizeof(KState) * n_mol, hipMemcpyDeviceToHost, B.st));
      k_trisolve_batch<<<(n_mol + 63) / 64, 64, 0, B.st>>>(n_mol, m, B.cycle, B.H, B.s, B.kst, B.ybuf, B.nq);
      k_axpy_batch<<<B.nseg, kBlock, 0, B.st>>>(B.nseg, B.segs, B.cycle, with_prec ? B.Z : B.V, B.M, nullptr, m, B.nq,
                                                B.ybuf, m, 1.0, sol);
      PB_HIP(ctx, hipStreamSynchronize(B.st));
      int maxk = 0;
      for (int i = 0; i < n_mol; ++i)
        if (cyc_h[i]) {
          mvmx[i] += ks[i].k_used;
          maxk = std::max(maxk, ks[i].k_used);
        }
      iters_total += maxk;
      // molecules that restart: the true residual of the correction equation with the mixed
      // operator, r = rhs − A sol
      int nrestart = 0;
      for (int i = 0; i < n_mol; ++i)
        if (cyc_h[i] && !ks[i].early) {
          mvmx[i] += 1;
          ++nrestart;
        }
      if (nrestart == 0) break;
      k_drop_early<<<(n_mol + 63) / 64, 64, 0, B.st>>>(n_mol, B.kst, B.cycle);
      op_mixed(B, sol, rr, nullptr, 0, B.cycle);
      k_resid_keep<<<nbn, kBlock, 0, B.st>>>(B.ntot, B.mol_of, B.mols, B.cycle, rhs_vec, rr);
      norms(B, rr, B.cycle, rn);
      PB_TRY(launch_ok(ctx, "batch cycle"));
      want = B.cycle;
    }
    return PB_OK;
  };

  if (opts.precision != PB_MIXED)
    return ctx->fail(PB_EINVAL, "the batched solve runs the mixed path (precision PB_MIXED)");
  if (prm->reg_avg != PB_AVG_FLAT)
    return ctx->fail(PB_EINVAL, "the batched solve takes the paper's disc averages (reg_avg PB_AVG_FLAT)");
  // refinement over the molecules in sel: FP64 residual, inner solve, update. With
  // mixed_first the first pass runs straight on the mixed operator from the initial guess, as
  // the single solve does: its residual comes from the mixed operator (none from a zero
  // start), and only the FP64 residuals after it decide convergence.
  auto outer_loop = [&](bool with_prec, bool mixed_first) -> pb_status {
    if (mixed_first) {
      if (opts.x0 == PB_X0_ZERO) {
        k_copy<<<vb, kBlock, 0, B.st>>>(B.M, g, r);
        k_zero_vec<<<vb, kBlock, 0, B.st>>>(B.M, dvec);
      } else {
        op_mixed(B, x, r, nullptr, 0, sel);
        k_resid_batch<<<nbn, kBlock, 0, B.st>>>(B.ntot, B.mol_of, B.mols, sel, g, r, dvec);
        for (int i = 0; i < n_mol; ++i) mvmx[i] += 1;  // every molecule is selected on entry
      }
      norms(B, r, sel, rn);
      k_first_target<<<(n_mol + 63) / 64, 64, 0, B.st>>>(n_mol, rn, gn, opts.tol, kInnerEta, sel, tolabs);
      PB_TRY(launch_ok(ctx, "first pass"));
      PB_TRY(inner(sel, r, dvec, with_prec));
      k_add_batch<<<B.nseg, kBlock, 0, B.st>>>(B.nseg, B.segs, sel, dvec, x);
      ++outer;
      ++outer_run;
    }
    for (;;) {
      op64(B, x, r, sel);
      k_resid_batch<<<nbn, kBlock, 0, B.st>>>(B.ntot, B.mol_of, B.mols, sel, g, r, dvec);
      norms(B, r, sel, rn);
      PB_HIP(ctx, hipMemsetAsync(n_sel, 0, sizeof(int), B.st));
      PB_HIP(ctx, hipMemcpyAsync(sel_h.data(), sel, sizeof(int) * n_mol, hipMemcpyDeviceToHost, B.st));
      k_outer_check<<<(n_mol + 63) / 64, 64, 0, B.st>>>(n_mol, rn, gn, opts.tol, kInnerEta, sel, relres, tolabs,
                                                        B.kst, n_sel);
      PB_TRY(launch_ok(ctx, "outer check"));
      int nsel = 0;
      PB_HIP(ctx, hipMemcpyAsync(&nsel, n_sel, sizeof(int), hipMemcpyDeviceToHost, B.st));
      PB_HIP(ctx, hipStreamSynchronize(B.st));
      for (int i = 0; i < n_mol; ++i) mv64[i] += sel_h[i];
      if (nsel == 0 || outer_run >= opts.max_outer || iters_total >= iter_cap) return PB_OK;
      PB_TRY(inner(sel, r, dvec, with_prec));
      k_add_batch<<<B.nseg, kBlock, 0, B.st>>>(B.nseg, B.segs, sel, dvec, x);
      ++outer;
      ++outer_run;
    }
  };
  std::vector<int> fallback(n_mol, 0);
  PB_TRY(outer_loop(prec, true));
  if (learned_x0 || prec) {
    // plain GMRES judges the learned path (x0 = M(g) and/or the preconditioner): molecules
    // still selected missed the tolerance; they continue without the network, from Λ⁻¹g where
    // their iterate is not finite, with what is left of the iteration budget
    PB_HIP(ctx, hipMemcpyAsync(sel_h.data(), sel, sizeof(int) * n_mol, hipMemcpyDeviceToHost, B.st));
    PB_HIP(ctx, hipStreamSynchronize(B.st));
    bool any = false;
    for (int i = 0; i < n_mol; ++i) {
      fallback[i] = sel_h[i];
      any = any || fallback[i];
    }
    if (any) {
      k_reset_nonfinite<<<nbn, kBlock, 0, B.st>>>(B.ntot, B.mol_of, B.mols, relres, g, B.d.lam1, B.d.lam2, x);
      outer_run = 0;
      iter_cap = opts.max_iter;
      PB_TRY(outer_loop(false, false));
    }
  }

  // results
  for (int i = 0; i < n_mol; ++i)
    PB_HIP(ctx, hipMemcpyAsync(p[i], x + 2 * (int64_t)B.mols_h[i].off, sizeof(double) * 2 * B.mols_h[i].n,
                               hipMemcpyDeviceToDevice, B.st));
  std::vector<double> rel_h(n_mol);
  std::vector<KState> ks(n_mol);
  unsigned long long t0h = 0;
  PB_HIP(ctx, hipMemcpyAsync(rel_h.data(), relres, sizeof(double) * n_mol, hipMemcpyDeviceToHost, B.st));
  PB_HIP(ctx, hipMemcpyAsync(ks.data(), B.kst, sizeof(KState) * n_mol, hipMemcpyDeviceToHost, B.st));
  PB_HIP(ctx, hipMemcpyAsync(&t0h, t0dev, sizeof(t0h), hipMemcpyDeviceToHost, B.st));
  PB_HIP(ctx, hipStreamSynchronize(B.st));
  int rate_khz = 0;
  if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess || rate_khz <= 0)
    rate_khz = 100000;
  std::vector<double> tsolve;
  double pairs = 0.0;
  bool all_ok = true;
  for (int i = 0; i < n_mol; ++i) {
    const double n2 = (double)B.mols_h[i].n * (double)B.mols_h[i].n;
    pairs += n2 * (mv64[i] + mvmx[i]);
    const bool ok = rel_h[i] <= opts.tol;
    all_ok = all_ok && ok;
    if (stats) {
      stats[i].iters = ks[i].iters;
      stats[i].outer = outer;
      stats[i].converged = ok;
      stats[i].fallback_used = fallback[i];
      stats[i].matvecs_fp64 = mv64[i];
      stats[i].matvecs_mixed = mvmx[i];
      stats[i].true_relres = rel_h[i];
      stats[i].t_total_s = ok && ks[i].t_done > t0h ? (double)(ks[i].t_done - t0h) / (rate_khz * 1e3) : -1.0;
      stats[i].t_matvec_s = 0.0;
      stats[i].pairs = n2 * (mv64[i] + mvmx[i]);
    }
    if (ok && ks[i].t_done > t0h) tsolve.push_back((double)(ks[i].t_done - t0h) / (rate_khz * 1e3));
  }
  std::sort(tsolve.begin(), tsolve.end());
  auto pct = [&](double q) {
    if (tsolve.empty()) return -1.0;
    size_t idx = (size_t)std::ceil(q * tsolve.size()) - 1;
    return tsolve[std::min(idx, tsolve.size() - 1)];
  };
  if (bstats) {
    bstats->t_total_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    bstats->t_p50_s = pct(0.50);
    bstats->t_p99_s = pct(0.99);
    bstats->pairs = pairs;
    bstats->graph_replays = replays;
    bstats->far_tile = kCfgTile[B.cfg];
    bstats->far_tpl = kCfgTpl[B.cfg];
    bstats->n_items = B.n_items32[B.cfg];
    bstats->outer = outer;
    bstats->far_symmetric = B.cfg == kSymB;
  }
  if (!all_ok) return ctx->fail(PB_ENOCONV, "some molecules did not reach the tolerance");
  return PB_OK;
}
