// Treecode far field of the mixed operator: the paper accelerates the operator with a
// kernel-independent fast multipole method (section "Fast linear solvers"); this is the
// cluster–particle form of the same idea, built for the GPU.
//
// Sources are clustered by an octree over the FP32 (scaled) coordinates, nodes renumbered in
// Morton order so that every tree node owns a contiguous range. A source cluster C far from
// a target batch is replaced by (p+1)³ proxy points ŷ_k, the tensor-product Chebyshev points
// of the second kind on C's bounding box, carrying the interpolation weights of its sources.
// With L_k the Lagrange basis of those points, interpolating the kernels in the source
// variable and differentiating the interpolant for the source normal derivatives gives
//   Q_k = Σ_j σw̃_j (n_j · ∇L_k(y_j)),   M_k = Σ_j w̃n_j L_k(y_j),
// and, for a target x with normal n_x, d = x − ŷ_k, r = |d| (scaled by σ = κ), E = e^{−r},
// a = E(1 + r):
//   S1 += [(1 − θ1 E) Q_k − (1 − E) M_k] / r
//   S2 += −(d · n_x)[(1 − a) Q_k − (1 − θ2 a) M_k] / r³,
// which are the four kernels of eq. IBIM-PBE (K11 and K21 as source-normal derivatives of
// G0 − θ1Gκ and G0 − Gκ, K12 = G0 − Gκ, K22 as the target-normal derivative of G0 − θ2Gκ)
// applied to the interpolated density. y1 = σS1 and y2 = σ²S2 as for the dense FP32 kernel.
//
// Target batches are runs of consecutive leaves in Morton order of at most kBatch nodes whose
// union box has a radius of at most kPackRadius times that of their largest leaf: a run that
// straddles a jump of the curve would have a wide box and interpolate almost nothing, while
// neighbouring leaves of different parents fill the wave's lanes (a batch costs one wave
// whatever its size). On bands too small to give every compute unit kMinWavesPerCU such
// batches, runs of sibling leaves (smaller, more waves) are used instead. For each batch the host walks the tree once: a cluster with more than
// (p+1)³ sources goes to the batch's proxy list when (r_B + r_C) < θ·dist and the two balls are at least 1.01·r_c apart (so it
// holds no near pair); leaves that fail the test go to the direct list, evaluated with the
// dense FP32 pair function (near pairs excluded by the shared FP32 predicate, the FP64 near
// field supplies them). Lists, ranges and boxes are built once per band; each application
// packs the records, computes the proxy weights and runs one fused far-field kernel. Fixed
// orders throughout: the operator is bitwise reproducible.
//
// Local coordinates. The FP32 records hold σ(x − c) relative to the band's centre; their
// rounding, about 6e-8·|σ(x − c)|, is a relative error of |x − c|/r in the difference d of a
// pair at distance r, and the double-layer kernel amplifies it into the residual (at 2.57M
// band nodes it puts the FP32 operator about 1.2e-6·‖g‖ from the FP64 one, nearly all of it
// from pairs closer than 1 Å). The treecode therefore forms every difference from FP32
// coordinates local to an FP64 origin near the pair: a source of a direct range is stored
// as its offset from the centre of its aligned group of kAnchor tree-order nodes (a compact
// patch in Morton order) and the target is converted to the same origin, once per group, from
// its FP64 position; a proxy is stored as its offset from its cluster's FP64 centre, and the
// target converted to that centre once per cluster. The error in d is then about 6e-8 times
// the pair's own scale. Which pairs are near stays the shared FP32 predicate on the global
// records, evaluated on the direct ranges that can hold a near pair (the host marks them);
// the other ranges skip it.
#include <algorithm>
#include <memory>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "pair_kernels.hpp"

namespace pb {
namespace {

constexpr int kBatch = 64;        // targets per batch = lanes of the far-field wave
constexpr double kPackRadius = 4.0;  // batch box radius / largest leaf radius in the batch
constexpr int kMinWavesPerCU = 16;   // packed batches per compute unit below which siblings are used
constexpr int kLeaf = 64;         // source leaves hold at most this many nodes
static_assert(kLeaf <= kBatch, "a leaf fits one target batch");
constexpr int kProxyChunk = 2048; // sources per proxy work item
constexpr int kProxyBlock = 256;
constexpr int kProxyTile = 64;
constexpr int kAnchor = 16;       // tree-order nodes per local-coordinate group of direct sources

// 1D Chebyshev points of the second kind on [−1, 1], u_a = cos(πa/p), for degree p.
struct ChebNodes {
  float u[kTreeMaxDegree + 1];
};

// ℓ_a(u) and ℓ'_a(u) of the degree-(P1 − 1) Lagrange basis on the nodes u (product form).
template <int P1>
__device__ __forceinline__ void lagrange(float x, const ChebNodes& cn, float* L, float* dL) {
#pragma unroll
  for (int a = 0; a < P1; ++a) {
    float l = 1.f, dl = 0.f;
#pragma unroll
    for (int b = 0; b < P1; ++b) {
      if (b == a) continue;
      const float inv = 1.f / (cn.u[a] - cn.u[b]);
      const float f = (x - cn.u[b]) * inv;
      dl = dl * f + l * inv;
      l *= f;
    }
    L[a] = l;
    dL[a] = dl;
  }
}

// Tree-order records gathered from the band-order ones: At = (offset from the node's group
// anchor, w̃n ψn), Mt and Nt as in band order, and Gt = the FP32 global coordinates (the same
// bits the near-field predicate was evaluated on).
__global__ void __launch_bounds__(kBlock) k_tree_gather(int n, const int* __restrict__ perm,
                                                        const float4* __restrict__ A, const float4* __restrict__ M,
                                                        const float4* __restrict__ N, const double* __restrict__ St,
                                                        const double* __restrict__ anc, float4* __restrict__ At,
                                                        float4* __restrict__ Mt, float4* __restrict__ Nt,
                                                        float4* __restrict__ Gt) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  const int j = perm[t];
  const float4 a = A[j];
  const double* o = anc + 3 * (size_t)(t / kAnchor);
  const double* x = St + 3 * (size_t)t;
  At[t] = make_float4((float)(x[0] - o[0]), (float)(x[1] - o[1]), (float)(x[2] - o[2]), a.w);
  Mt[t] = M[j];
  Nt[t] = N[j];
  Gt[t] = make_float4(a.x, a.y, a.z, 0.f);
}

// Exact scaled coordinates in tree order, St[t] = σ(x − c) of band node perm[t] in FP64.
__global__ void __launch_bounds__(kBlock) k_tree_coords(int n, const int* __restrict__ perm, BandDev b, double cx,
                                                        double cy, double cz, double sigma, double* __restrict__ St) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  const int j = perm[t];
  St[3 * (size_t)t] = sigma * (b.px[j] - cx);
  St[3 * (size_t)t + 1] = sigma * (b.py[j] - cy);
  St[3 * (size_t)t + 2] = sigma * (b.pz[j] - cz);
}

// Anchor of each aligned group of kAnchor tree-order nodes: the centre of its bounding box.
__global__ void __launch_bounds__(kBlock) k_tree_anchor(int n, const double* __restrict__ St,
                                                        double* __restrict__ anc) {
  const int g = blockIdx.x * kBlock + threadIdx.x;
  if ((int64_t)g * kAnchor >= n) return;
  const int e = min(n, (g + 1) * kAnchor);
  for (int a = 0; a < 3; ++a) {
    double lo = INFINITY, hi = -INFINITY;
    for (int t = g * kAnchor; t < e; ++t) {
      lo = fmin(lo, St[3 * (size_t)t + a]);
      hi = fmax(hi, St[3 * (size_t)t + a]);
    }
    anc[3 * (size_t)g + a] = 0.5 * (lo + hi);
  }
}

// Partial proxy weights of one work item (cluster c, sources [b, e)): part[item][k] =
// (Q_k, M_k) summed over the item's sources in FP64. Cluster box: FP64 centre ccen[c],
// half-widths half[c]; the basis variable is u = (y − centre)/half per axis, formed in FP64
// from the exact coordinates St. Block of kProxyBlock threads; a tile of kProxyTile sources
// has its 1D bases evaluated once (three axes) and shared through LDS.
template <int P1>
__global__ void __launch_bounds__(kProxyBlock) k_proxy(const int4* __restrict__ items, const double* __restrict__ ccen,
                                                       const float4* __restrict__ half, const double* __restrict__ St,
                                                       const float4* __restrict__ At, const float4* __restrict__ Nt,
                                                       ChebNodes cn, double2* __restrict__ part,
                                                       const int* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int P3 = P1 * P1 * P1;
  constexpr int kPer = (P3 + kProxyBlock - 1) / kProxyBlock;
  __shared__ float sL[kProxyTile][3][P1], sD[kProxyTile][3][P1];
  __shared__ float4 sN[kProxyTile];
  __shared__ float sW[kProxyTile];
  const int4 it = items[blockIdx.x];  // (cluster, begin, end, unused)
  const float4 hw = half[it.x];
  const double* mid = ccen + 3 * (size_t)it.x;
  int ka[kPer], kb[kPer], kc[kPer];
  double q[kPer], m[kPer];
#pragma unroll
  for (int s = 0; s < kPer; ++s) {
    const int k = threadIdx.x + s * kProxyBlock;
    ka[s] = k / (P1 * P1);
    kb[s] = (k / P1) % P1;
    kc[s] = k % P1;
    q[s] = m[s] = 0.0;
  }
  for (int base = it.y; base < it.z; base += kProxyTile) {
    const int cnt = min(kProxyTile, it.z - base);
    if (threadIdx.x < 3 * kProxyTile) {
      const int j = threadIdx.x / 3, ax = threadIdx.x % 3;
      float L[P1], dL[P1];
      if (j < cnt) {
        const double ihd = 1.0 / (double)(ax == 0 ? hw.x : (ax == 1 ? hw.y : hw.z));
        const float s = (float)ihd;
        lagrange<P1>((float)((St[3 * (size_t)(base + j) + ax] - mid[ax]) * ihd), cn, L, dL);
#pragma unroll
        for (int b = 0; b < P1; ++b) dL[b] *= s;
      } else {
#pragma unroll
        for (int b = 0; b < P1; ++b) L[b] = dL[b] = 0.f;
      }
#pragma unroll
      for (int b = 0; b < P1; ++b) {
        sL[j][ax][b] = L[b];
        sD[j][ax][b] = dL[b];
      }
    }
    if (threadIdx.x < kProxyTile) {
      const int j = threadIdx.x;
      sN[j] = j < cnt ? Nt[base + j] : make_float4(0.f, 0.f, 0.f, 0.f);
      sW[j] = j < cnt ? At[base + j].w : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kPer; ++s) {
      if (threadIdx.x + s * kProxyBlock >= P3) continue;
      float qf = 0.f, mf = 0.f;
      for (int j = 0; j < cnt; ++j) {
        const float lx = sL[j][0][ka[s]], ly = sL[j][1][kb[s]], lz = sL[j][2][kc[s]];
        const float dx = sD[j][0][ka[s]], dy = sD[j][1][kb[s]], dz = sD[j][2][kc[s]];
        const float4 nw = sN[j];
        const float lyz = ly * lz;
        const float g = nw.x * dx * lyz + lx * (nw.y * dy * lz + nw.z * ly * dz);
        qf = fmaf(nw.w, g, qf);
        mf = fmaf(sW[j], lx * lyz, mf);
      }
      q[s] += (double)qf;
      m[s] += (double)mf;
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < kPer; ++s) {
    const int k = threadIdx.x + s * kProxyBlock;
    if (k < P3) part[(size_t)blockIdx.x * P3 + k] = make_double2(q[s], m[s]);
  }
}

// Proxies of cluster c: position ŷ_k = centre + half·(u_a, u_b, u_c) and the weights Q_k, M_k,
// the sum of the cluster's item partials in item order. PX[k] = (ŷ_k − centre, Q_k) (the
// offset from the FP64 centre), PM[k] = M_k.
__global__ void __launch_bounds__(kBlock) k_proxy_sum(int n_cl, int P1, const int* __restrict__ item_ptr,
                                                      const double2* __restrict__ part, const float4* __restrict__ half,
                                                      ChebNodes cn, float4* __restrict__ PX, float* __restrict__ PM) {
  const int P3 = P1 * P1 * P1;
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= (int64_t)n_cl * P3) return;
  const int c = (int)(g / P3), k = (int)(g % P3);
  double q = 0.0, m = 0.0;
  for (int it = item_ptr[c]; it < item_ptr[c + 1]; ++it) {
    const double2 v = part[(size_t)it * P3 + k];
    q += v.x;
    m += v.y;
  }
  const float4 hw = half[c];
  const int a = k / (P1 * P1), b = (k / P1) % P1, cc = k % P1;
  PX[g] = make_float4(hw.x * cn.u[a], hw.y * cn.u[b], hw.z * cn.u[cc], (float)q);
  PM[g] = (float)m;
}

// One target–proxy interaction (scaled coordinates, no near pair possible).
template <bool kScreened>
__device__ __forceinline__ void proxy_f32(const float4& ta, const float4& tn, const float4& sp, float sm,
                                          const F32Params& fp, float& a1, float& a2) {
  const float dx = ta.x - sp.x, dy = ta.y - sp.y, dz = ta.z - sp.z;
  const float r2 = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx));
  const float rinv = __builtin_amdgcn_rsqf(r2);
  float E = 1.f, a = 1.f;
  if (kScreened) {
    const float z = r2 * rinv;
    E = __builtin_amdgcn_exp2f(fp.mlog2e * z);
    a = __fmaf_rn(E, z, E);
  }
  const float dn = __fmaf_rn(dz, tn.z, __fmaf_rn(dy, tn.y, dx * tn.x));
  // [(1 − θ1E)Q − (1 − E)M]/r and −dn[(1 − a)Q − (1 − θ2 a)M]/r³
  const float t1 = __fmaf_rn(__fmaf_rn(-fp.th1, E, 1.f), sp.w, -__fmaf_rn(-E, sm, sm));
  const float t2 = __fmaf_rn(-a, sp.w, sp.w) - __fmaf_rn(-fp.th2 * a, sm, sm);
  a1 = __fmaf_rn(t1, rinv, a1);
  a2 = __fmaf_rn(-dn * t2, rinv * rinv * rinv, a2);
}

// A direct pair in local coordinates (tl − sl = d) on a range that may hold near pairs: the
// shared FP32 predicate on the global coordinates tg, sg decides, and a near pair is replaced
// by a far stand-in with zero weights, which contributes exactly zero.
template <bool kScreened>
__device__ __forceinline__ void pair_local_checked(const float4& tl, const float4& tn, const float4& sl,
                                                   const float4& sm, const float4& tg, const float4& sg,
                                                   const F32Params& fp, float& a1, float& a2) {
  const bool near = r2_f32(tg.x, tg.y, tg.z, sg.x, sg.y, sg.z) < fp.rc2;
  const float4 s = near ? make_float4(tl.x + 1.f, tl.y, tl.z, 0.f) : sl;
  const float4 m = near ? make_float4(0.f, 0.f, 0.f, 0.f) : sm;
  pair_f32<kScreened, false>(tl, tn, s, m, fp, a1, a2);
}

// Far field of one target batch per wave: its direct source ranges with the dense pair
// function, then its proxy clusters. Every lane reads the same source or proxy at the same
// time (wave-uniform addresses, no LDS staging and no barriers). Differences are formed in
// local coordinates: per anchor group of a direct range and per proxy cluster, each lane
// converts its target's FP64 position to that origin. A range whose end carries the sign bit
// may hold near pairs and runs the predicate. FP32 sums per range and per cluster, flushed
// into FP64. Output in band order (through perm), scaled by σ and σ².
template <bool kScreened>
__global__ void __launch_bounds__(kBatch) k_tree_far(const int2* __restrict__ batch, const int* __restrict__ dir_ptr,
                                                     const int2* __restrict__ dir_rng, const int* __restrict__ app_ptr,
                                                     const int* __restrict__ app_cl, int P3,
                                                     const float4* __restrict__ PX, const float* __restrict__ PM,
                                                     const double* __restrict__ ccen, const float4* __restrict__ At,
                                                     const float4* __restrict__ Mt, const float4* __restrict__ Nt,
                                                     const float4* __restrict__ Gt, const double* __restrict__ St,
                                                     const double* __restrict__ anc, const int* __restrict__ perm,
                                                     F32Params fp, int n, double sig1, double sig2,
                                                     double* __restrict__ out, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int2 bt = batch[blockIdx.x];
  const int t = bt.x + (int)threadIdx.x;
  const bool live = t < bt.y;
  const int tt = live ? t : bt.x;  // idle lanes shadow the batch's first target (results unused)
  const double tx = St[3 * (size_t)tt], ty = St[3 * (size_t)tt + 1], tz = St[3 * (size_t)tt + 2];
  const float4 tn = Nt[tt];
  double acc1 = 0.0, acc2 = 0.0;
  const int r1 = dir_ptr[blockIdx.x + 1];
  for (int r = dir_ptr[blockIdx.x]; r < r1; ++r) {
    const int2 rg = dir_rng[r];
    const bool check = rg.y < 0;
    const int end = rg.y & 0x7fffffff;
    float f1 = 0.f, f2 = 0.f;
    for (int j = rg.x; j < end;) {
      const int je = min(end, (j / kAnchor + 1) * kAnchor);
      const double* o = anc + 3 * (size_t)(j / kAnchor);
      const float4 tl = make_float4((float)(tx - o[0]), (float)(ty - o[1]), (float)(tz - o[2]), 0.f);
      if (check) {
        const float4 tg = Gt[tt];
        for (; j < je; ++j) pair_local_checked<kScreened>(tl, tn, At[j], Mt[j], tg, Gt[j], fp, f1, f2);
      } else {
        for (; j + 4 <= je; j += 4) {
#pragma unroll
          for (int u = 0; u < 4; ++u) pair_f32<kScreened, false>(tl, tn, At[j + u], Mt[j + u], fp, f1, f2);
        }
        for (; j < je; ++j) pair_f32<kScreened, false>(tl, tn, At[j], Mt[j], fp, f1, f2);
      }
    }
    acc1 += (double)f1;
    acc2 += (double)f2;
  }
  const int c1 = app_ptr[blockIdx.x + 1];
  for (int r = app_ptr[blockIdx.x]; r < c1; ++r) {
    const int cl = app_cl[r];
    const size_t base = (size_t)cl * P3;
    const float4* __restrict__ px = PX + base;
    const float* __restrict__ pm = PM + base;
    const double* o = ccen + 3 * (size_t)cl;
    const float4 tl = make_float4((float)(tx - o[0]), (float)(ty - o[1]), (float)(tz - o[2]), 0.f);
    float f1 = 0.f, f2 = 0.f;
    int k = 0;
    for (; k + 4 <= P3; k += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) proxy_f32<kScreened>(tl, tn, px[k + u], pm[k + u], fp, f1, f2);
    }
    for (; k < P3; ++k) proxy_f32<kScreened>(tl, tn, px[k], pm[k], fp, f1, f2);
    acc1 += (double)f1;
    acc2 += (double)f2;
  }
  if (live) {
    const int i = perm[t];
    out[i] = sig1 * acc1;
    out[n + i] = sig2 * acc2;
  }
}

// ------------------------------------------------------------------ host: tree and lists

struct HNode {
  int b, e;           // tree-order range
  int first_kid, n_kids;
  double lo[3], hi[3];
  double c[3], r;     // centre and radius of the tight box
};

uint64_t spread3(uint64_t v) {  // 21 bits → every third bit
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}

void tight_box(const std::vector<double>& s, int b, int e, double lo[3], double hi[3], double c[3], double* r) {
  for (int a = 0; a < 3; ++a) {
    lo[a] = INFINITY;
    hi[a] = -INFINITY;
  }
  for (int t = b; t < e; ++t)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], s[3 * (size_t)t + a]);
      hi[a] = std::max(hi[a], s[3 * (size_t)t + a]);
    }
  double r2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    c[a] = 0.5 * (lo[a] + hi[a]);
    r2 += 0.25 * (hi[a] - lo[a]) * (hi[a] - lo[a]);
  }
  *r = std::sqrt(r2);
}

}  // namespace

// Morton order, octree and target batches of one band (host). Shared by the plans that one
// solve builds for the same band (they differ in degree and θ only).
struct TreeHost {
  int n = 0;
  std::vector<int> perm;
  std::vector<double> s;  // scaled coordinates in tree order
  std::vector<HNode> nodes;
  std::vector<int2> batch;
};

namespace {

pb_status build_host_tree(pb_ctx* ctx, const pb_band* band, const MixedPlan& P, TreeHost& H) {
  const int n = (int)band->n;
  H.n = n;
  // scaled coordinates on the host, exactly as the FP32 records hold them (rounded to FP32)
  std::vector<double> px(n), py(n), pz(n);
  PB_HIP(ctx, hipMemcpyAsync(px.data(), band->px, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
  PB_HIP(ctx, hipMemcpyAsync(py.data(), band->py, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
  PB_HIP(ctx, hipMemcpyAsync(pz.data(), band->pz, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
  PB_TRY(sync(ctx, "tree coordinates"));
  std::vector<double> s0(3 * (size_t)n);
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int j = 0; j < n; ++j) {
    const double v[3] = {(double)(float)(P.sigma * (px[j] - P.cx)), (double)(float)(P.sigma * (py[j] - P.cy)),
                         (double)(float)(P.sigma * (pz[j] - P.cz))};
    for (int a = 0; a < 3; ++a) {
      s0[3 * (size_t)j + a] = v[a];
      lo[a] = std::min(lo[a], v[a]);
      hi[a] = std::max(hi[a], v[a]);
    }
  }
  const double size = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-12}) * (1.0 + 1e-9);
  std::vector<uint64_t> code(n);
  for (int j = 0; j < n; ++j) {
    uint64_t m = 0;
    for (int a = 0; a < 3; ++a) {
      double f = (s0[3 * (size_t)j + a] - lo[a]) / size * 2097152.0;
      uint64_t q = (uint64_t)std::min(std::max(f, 0.0), 2097151.0);
      m |= spread3(q) << (2 - a);
    }
    code[j] = m;
  }
  // sort by code, ties by index: a stable LSD radix sort of the indices, 16 bits per pass
  std::vector<int>& perm = H.perm;
  perm.resize(n);
  {
    std::vector<int> tmp(n);
    std::iota(perm.begin(), perm.end(), 0);
    std::vector<int> count(65537);
    for (int pass = 0; pass < 4; ++pass) {
      const int shift = 16 * pass;
      std::fill(count.begin(), count.end(), 0);
      for (int j = 0; j < n; ++j) ++count[((code[j] >> shift) & 0xffff) + 1];
      for (int v = 0; v < 65536; ++v) count[v + 1] += count[v];
      for (int t = 0; t < n; ++t) {
        const int j = perm[t];
        tmp[count[(code[j] >> shift) & 0xffff]++] = j;
      }
      perm.swap(tmp);
    }
  }
  std::vector<double>& s = H.s;
  s.resize(3 * (size_t)n);
  std::vector<uint64_t> cs(n);
  for (int t = 0; t < n; ++t) {
    for (int a = 0; a < 3; ++a) s[3 * (size_t)t + a] = s0[3 * (size_t)perm[t] + a];
    cs[t] = code[perm[t]];
  }
  // octree over the sorted codes: children in octant order, leaves of at most kLeaf nodes
  std::vector<HNode>& nodes = H.nodes;
  nodes.clear();
  nodes.reserve(4 * (size_t)n / kLeaf + 64);
  struct Todo {
    int idx, level;
  };
  nodes.push_back(HNode{0, n, -1, 0, {}, {}, {}, 0.0});
  std::vector<Todo> todo{{0, 0}};
  while (!todo.empty()) {
    Todo td = todo.back();
    todo.pop_back();
    const HNode& nd = nodes[td.idx];
    if (nd.e - nd.b <= kLeaf || td.level >= 21) continue;
    const int shift = 3 * (20 - td.level);
    const int b = nd.b, e = nd.e;
    const int first = (int)nodes.size();
    int nk = 0;
    for (int o = 0, t = b; o < 8 && t < e; ++o) {
      int u = t;
      while (u < e && (int)((cs[u] >> shift) & 7) == o) ++u;
      if (u > t) {
        nodes.push_back(HNode{t, u, -1, 0, {}, {}, {}, 0.0});
        ++nk;
      }
      t = u;
    }
    nodes[td.idx].first_kid = first;
    nodes[td.idx].n_kids = nk;
    for (int k = nk - 1; k >= 0; --k) todo.push_back(Todo{first + k, td.level + 1});
  }
  // tight boxes bottom up (children are created after their parent): leaves scan their
  // nodes, a parent takes the union of its children's boxes
  for (int k = (int)nodes.size() - 1; k >= 0; --k) {
    HNode& nd = nodes[k];
    if (nd.n_kids == 0) {
      tight_box(s, nd.b, nd.e, nd.lo, nd.hi, nd.c, &nd.r);
      continue;
    }
    double r2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      nd.lo[a] = INFINITY;
      nd.hi[a] = -INFINITY;
      for (int q = 0; q < nd.n_kids; ++q) {
        nd.lo[a] = std::min(nd.lo[a], nodes[nd.first_kid + q].lo[a]);
        nd.hi[a] = std::max(nd.hi[a], nodes[nd.first_kid + q].hi[a]);
      }
      nd.c[a] = 0.5 * (nd.lo[a] + nd.hi[a]);
      r2 += 0.25 * (nd.hi[a] - nd.lo[a]) * (nd.hi[a] - nd.lo[a]);
    }
    nd.r = std::sqrt(r2);
  }
  // target batches: the leaves in Morton order (depth first, children in octant order),
  // packed greedily into runs of at most kBatch nodes whose union box stays within
  // kPackRadius times the radius of the run's largest leaf. Packing trades waves for fuller
  // waves; when it would leave fewer than kMinWavesPerCU batches per compute unit, the
  // batches are the runs of sibling leaves instead (more, smaller waves fill the GPU better).
  std::vector<int2>& batch = H.batch;
  batch.clear();
  {
    int cb = -1, ce = -1;
    double blo[3] = {}, bhi[3] = {}, maxr = 0.0;
    std::vector<int> st{0};
    while (!st.empty()) {
      const HNode& nd = nodes[st.back()];
      st.pop_back();
      if (nd.n_kids > 0) {
        for (int q = nd.n_kids - 1; q >= 0; --q) st.push_back(nd.first_kid + q);
        continue;
      }
      if (cb >= 0 && nd.e - cb <= kBatch) {
        double ulo[3], uhi[3], r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
          ulo[a] = std::min(blo[a], nd.lo[a]);
          uhi[a] = std::max(bhi[a], nd.hi[a]);
          r2 += 0.25 * (uhi[a] - ulo[a]) * (uhi[a] - ulo[a]);
        }
        const double mr = std::max(maxr, nd.r);
        if (std::sqrt(r2) <= kPackRadius * mr) {
          ce = nd.e;
          std::copy(ulo, ulo + 3, blo);
          std::copy(uhi, uhi + 3, bhi);
          maxr = mr;
          continue;
        }
      }
      if (cb >= 0) batch.push_back(make_int2(cb, ce));
      cb = nd.b;
      ce = nd.e;
      std::copy(nd.lo, nd.lo + 3, blo);
      std::copy(nd.hi, nd.hi + 3, bhi);
      maxr = nd.r;
    }
    if (cb >= 0) batch.push_back(make_int2(cb, ce));
  }
  if ((int64_t)batch.size() < (int64_t)kMinWavesPerCU * ctx->n_cu) {  // sibling runs
    batch.clear();
    if (nodes[0].n_kids == 0) batch.push_back(make_int2(0, n));
    std::vector<int> st{0};
    while (!st.empty()) {
      const HNode nd = nodes[st.back()];
      st.pop_back();
      if (nd.n_kids == 0) continue;
      int cb = -1, ce = -1;
      for (int q = 0; q < nd.n_kids; ++q) {
        const HNode& ch = nodes[nd.first_kid + q];
        if (ch.n_kids == 0 && cb >= 0 && ce == ch.b && ch.e - cb <= kBatch) {
          ce = ch.e;
          continue;
        }
        if (cb >= 0) batch.push_back(make_int2(cb, ce));
        cb = ce = -1;
        if (ch.n_kids == 0) {
          cb = ch.b;
          ce = ch.e;
        } else {
          st.push_back(nd.first_kid + q);
        }
      }
      if (cb >= 0) batch.push_back(make_int2(cb, ce));
    }
  }
  {  // a leaf can exceed kBatch only at the depth limit (coincident codes): split it
    std::vector<int2> split;
    for (const int2& bt : batch)
      for (int b = bt.x; b < bt.y; b += kBatch) split.push_back(make_int2(b, std::min(bt.y, b + kBatch)));
    batch.swap(split);
  }
  return PB_OK;
}

}  // namespace

pb_status tree_prepare(pb_ctx* ctx, const pb_band* band, const Derived& d, int degree, double theta, TreePlan& T,
                       const char* pfx, const MixedPlan* near, std::shared_ptr<TreeHost>* host) {
  const int n = (int)band->n;
  const std::string px_ = pfx;
  if (near) T.near = *near;  // the near field depends on the geometry only: shared between plans
  else PB_TRY(near_build(ctx, band, d, (px_ + "n_").c_str(), T.near));
  const MixedPlan& P = T.near;
  const int P1 = degree + 1, P3 = P1 * P1 * P1;
  std::shared_ptr<TreeHost> hp = host && *host && (*host)->n == n ? *host : nullptr;
  if (!hp) {
    hp = std::make_shared<TreeHost>();
    PB_TRY(build_host_tree(ctx, band, P, *hp));
    if (host) *host = hp;
  }
  const std::vector<int>& perm = hp->perm;
  const std::vector<double>& s = hp->s;
  const std::vector<HNode>& nodes = hp->nodes;
  std::vector<int2> batch = hp->batch;
  const int n_batch = (int)batch.size();
  // interaction lists per batch, then batches ordered by decreasing work (the longest waves
  // start first)
  const double rcs = P.sigma * P.rc * 1.01;
  // a direct leaf whose box is at least this far (squared) from the batch's box holds no pair
  // that the FP32 predicate calls near (its rounding is far below the margin)
  const double clear2 = (double)P.rc2f * (1.0 + 1e-3);
  std::vector<std::vector<int2>> dirs(n_batch);
  std::vector<std::vector<int>> apps(n_batch);
  std::vector<int64_t> work(n_batch, 0);
  // the walks of the batches are independent: host threads over contiguous slices
  auto walk = [&](int b0, int b1) {
    std::vector<int> stack;
    for (int bi = b0; bi < b1; ++bi) {
      const int b = batch[bi].x, e = batch[bi].y;
      double blo[3], bhi[3], bc[3], br;
      tight_box(s, b, e, blo, bhi, bc, &br);
      std::vector<int2>& dl = dirs[bi];
      stack.assign(1, 0);
      while (!stack.empty()) {
        const int k = stack.back();
        stack.pop_back();
        const HNode& nd = nodes[k];
        const double dist = std::sqrt((bc[0] - nd.c[0]) * (bc[0] - nd.c[0]) + (bc[1] - nd.c[1]) * (bc[1] - nd.c[1]) +
                                      (bc[2] - nd.c[2]) * (bc[2] - nd.c[2]));
        if (nd.e - nd.b > P3 && br + nd.r < theta * dist && dist - br - nd.r > rcs) {
          apps[bi].push_back(k);
          work[bi] += P3;
        } else if (nd.n_kids == 0) {
          // ranges of consecutive leaves with the same predicate flag (sign bit of the end)
          double gap2 = 0.0;
          for (int a = 0; a < 3; ++a) {
            const double g = std::max(0.0, std::max(nd.lo[a] - bhi[a], blo[a] - nd.hi[a]));
            gap2 += g * g;
          }
          const int flag = gap2 >= clear2 ? 0 : (int)0x80000000u;
          if (!dl.empty() && (dl.back().y & 0x7fffffff) == nd.b && (dl.back().y & (int)0x80000000u) == flag)
            dl.back().y = nd.e | flag;
          else
            dl.push_back(make_int2(nd.b, nd.e | flag));
          work[bi] += 2 * (nd.e - nd.b);  // a direct pair costs about twice a proxy interaction
        } else {
          for (int q = nd.n_kids - 1; q >= 0; --q) stack.push_back(nd.first_kid + q);
        }
      }
    }
  };
  {
    const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
    const int n_thr = std::max(1, std::min({hw, 16, n_batch / 256}));
    std::vector<std::thread> pool;
    for (int q = 1; q < n_thr; ++q)
      pool.emplace_back(walk, (int)((int64_t)n_batch * q / n_thr), (int)((int64_t)n_batch * (q + 1) / n_thr));
    walk(0, (int)((int64_t)n_batch / n_thr));
    for (std::thread& th : pool) th.join();
  }
  int64_t n_dir_pairs = 0, n_app_pairs = 0;
  for (int bi = 0; bi < n_batch; ++bi) {
    const int64_t cnt = batch[bi].y - batch[bi].x;
    for (const int2& r : dirs[bi]) n_dir_pairs += cnt * ((r.y & 0x7fffffff) - r.x);
    n_app_pairs += cnt * P3 * (int64_t)apps[bi].size();
  }
  std::vector<int> order(n_batch);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
  std::vector<int2> batch_sorted(n_batch);
  std::vector<int> dir_ptr(n_batch + 1, 0), app_ptr(n_batch + 1, 0);
  std::vector<int2> dir_rng;
  std::vector<int> app_node;
  for (int q = 0; q < n_batch; ++q) {
    const int bi = order[q];
    batch_sorted[q] = batch[bi];
    dir_rng.insert(dir_rng.end(), dirs[bi].begin(), dirs[bi].end());
    app_node.insert(app_node.end(), apps[bi].begin(), apps[bi].end());
    dir_ptr[q + 1] = (int)dir_rng.size();
    app_ptr[q + 1] = (int)app_node.size();
  }
  batch.swap(batch_sorted);
  // proxy clusters: the tree nodes that some list uses, numbered in tree-node order
  std::vector<char> used(nodes.size(), 0);
  for (int k : app_node) used[k] = 1;
  std::vector<float4> half;
  std::vector<double> ccen;
  std::vector<int> item_ptr{0};
  std::vector<int4> items;
  int n_cl = 0;
  std::vector<int> cl_of(nodes.size(), -1);
  for (size_t k = 0; k < nodes.size(); ++k) {
    if (!used[k]) continue;
    const HNode& nd = nodes[k];
    const int cl = cl_of[k] = n_cl++;
    double hw[3], ext = 0.0;
    for (int a = 0; a < 3; ++a) ext = std::max(ext, nd.hi[a] - nd.lo[a]);
    for (int a = 0; a < 3; ++a) hw[a] = std::max(0.5 * (nd.hi[a] - nd.lo[a]), std::max(1e-3 * ext, 1e-6));
    half.push_back(make_float4((float)hw[0], (float)hw[1], (float)hw[2], 0.f));
    ccen.insert(ccen.end(), nd.c, nd.c + 3);
    for (int t = nd.b; t < nd.e; t += kProxyChunk) items.push_back(make_int4(cl, t, std::min(nd.e, t + kProxyChunk), 0));
    item_ptr.push_back((int)items.size());
  }
  std::vector<int> app_cl(app_node.size());
  for (size_t q = 0; q < app_node.size(); ++q) app_cl[q] = cl_of[app_node[q]];
  // upload
  auto up = [&](const char* nm, const void* src, size_t bytes, void** dst) -> pb_status {
    *dst = workspace(ctx, nm, std::max<size_t>(bytes, 16));
    if (!*dst) return PB_ENOMEM;
    if (bytes) PB_HIP(ctx, hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, ctx->stream));
    return PB_OK;
  };
  PB_TRY(up((px_ + "perm").c_str(), perm.data(), sizeof(int) * n, (void**)&T.perm));
  PB_TRY(up((px_ + "batch").c_str(), batch.data(), sizeof(int2) * n_batch, (void**)&T.batch));
  PB_TRY(up((px_ + "dir_ptr").c_str(), dir_ptr.data(), sizeof(int) * (n_batch + 1), (void**)&T.dir_ptr));
  PB_TRY(up((px_ + "dir_rng").c_str(), dir_rng.data(), sizeof(int2) * dir_rng.size(), (void**)&T.dir_rng));
  PB_TRY(up((px_ + "app_ptr").c_str(), app_ptr.data(), sizeof(int) * (n_batch + 1), (void**)&T.app_ptr));
  PB_TRY(up((px_ + "app_cl").c_str(), app_cl.data(), sizeof(int) * app_cl.size(), (void**)&T.app_cl));
  PB_TRY(up((px_ + "half").c_str(), half.data(), sizeof(float4) * half.size(), (void**)&T.half));
  PB_TRY(up((px_ + "ccen").c_str(), ccen.data(), sizeof(double) * ccen.size(), (void**)&T.ccen));
  PB_TRY(up((px_ + "items").c_str(), items.data(), sizeof(int4) * items.size(), (void**)&T.items));
  PB_TRY(up((px_ + "item_ptr").c_str(), item_ptr.data(), sizeof(int) * item_ptr.size(), (void**)&T.item_ptr));
  T.At = (float4*)workspace(ctx, (px_ + "At").c_str(), sizeof(float4) * n);
  T.Mt = (float4*)workspace(ctx, (px_ + "Mt").c_str(), sizeof(float4) * n);
  T.Nt = (float4*)workspace(ctx, (px_ + "Nt").c_str(), sizeof(float4) * n);
  T.PX = (float4*)workspace(ctx, (px_ + "PX").c_str(), sizeof(float4) * std::max<size_t>((size_t)n_cl * P3, 1));
  T.PM = (float*)workspace(ctx, (px_ + "PM").c_str(), sizeof(float) * std::max<size_t>((size_t)n_cl * P3, 1));
  T.part = (double2*)workspace(ctx, (px_ + "part").c_str(), sizeof(double2) * std::max<size_t>(items.size() * P3, 1));
  T.far = (double*)workspace(ctx, (px_ + "far").c_str(), sizeof(double) * 2 * (size_t)n);
  T.Gt = (float4*)workspace(ctx, (px_ + "Gt").c_str(), sizeof(float4) * n);
  T.St = (double*)workspace(ctx, (px_ + "St").c_str(), sizeof(double) * 3 * (size_t)n);
  const int n_anc = (n + kAnchor - 1) / kAnchor;
  T.anc = (double*)workspace(ctx, (px_ + "anc").c_str(), sizeof(double) * 3 * (size_t)std::max(n_anc, 1));
  if (!T.At || !T.Mt || !T.Nt || !T.PX || !T.PM || !T.part || !T.far || !T.Gt || !T.St || !T.anc) return PB_ENOMEM;
  // exact scaled coordinates in tree order and the anchors of the direct sources' groups
  k_tree_coords<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(n, T.perm, band_dev(band), P.cx,
                                                                                    P.cy, P.cz, P.sigma, T.St);
  k_tree_anchor<<<(unsigned)((n_anc + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(n, T.St, T.anc);
  PB_TRY(launch_ok(ctx, "tree coordinates"));
  T.band_key = band->px;
  T.n = n;
  T.rc = d.rc;
  T.theta = theta;
  T.degree = degree;
  T.n_batch = n_batch;
  T.n_cl = n_cl;
  T.n_items = (int)items.size();
  T.n_dir_pairs = n_dir_pairs;
  T.n_app_pairs = n_app_pairs;
  for (int a = 0; a <= degree; ++a) T.u[a] = (float)std::cos(kPi * a / degree);
  return sync(ctx, "tree_prepare");
}

namespace {

template <int P1>
void launch_proxy(pb_ctx* ctx, const TreePlan& T, const ChebNodes& cn) {
  k_proxy<P1><<<(unsigned)T.n_items, kProxyBlock, 0, ctx->stream>>>(T.items, T.ccen, T.half, T.St, T.At, T.Nt, cn,
                                                                        T.part, ctx->skip);
}

void launch_tree(pb_ctx* ctx, const TreePlan& T, bool screened, const F32Params& fp, double sig1, double sig2) {
  ChebNodes cn{};
  const int P1 = T.degree + 1, P3 = P1 * P1 * P1;
  for (int a = 0; a < P1; ++a) cn.u[a] = T.u[a];
  if (T.n_items > 0) {
    switch (P1) {
      case 3: launch_proxy<3>(ctx, T, cn); break;
      case 4: launch_proxy<4>(ctx, T, cn); break;
      case 5: launch_proxy<5>(ctx, T, cn); break;
      case 6: launch_proxy<6>(ctx, T, cn); break;
      case 7: launch_proxy<7>(ctx, T, cn); break;
      case 8: launch_proxy<8>(ctx, T, cn); break;
      default: launch_proxy<9>(ctx, T, cn); break;
    }
    k_proxy_sum<<<(unsigned)(((int64_t)T.n_cl * P3 + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(
        T.n_cl, P1, T.item_ptr, T.part, T.half, cn, T.PX, T.PM);
  }
  auto far = screened ? k_tree_far<true> : k_tree_far<false>;
  far<<<(unsigned)T.n_batch, kBatch, 0, ctx->stream>>>(T.batch, T.dir_ptr, T.dir_rng, T.app_ptr, T.app_cl, P3, T.PX,
                                                        T.PM, T.ccen, T.At, T.Mt, T.Nt, T.Gt, T.St, T.anc, T.perm, fp,
                                                        (int)T.n, sig1, sig2, T.far, ctx->skip);
}

}  // namespace

pb_status matvec_tree(pb_ctx* ctx, const pb_band* band, const Derived& d, const double* p, double* y,
                      const TreePlan& T) {
  const MixedPlan& P = T.near;
  const int n = (int)band->n;
  if (T.band_key != band->px || T.n != n || T.rc != d.rc)
    return ctx->fail(PB_EINVAL, "treecode operator used before its tree was prepared");
  double* near = (double*)workspace(ctx, "tc_near", sizeof(double) * 2 * (size_t)n);
  if (!near) return PB_ENOMEM;
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  k_pack_f32<<<nb, kBlock, 0, ctx->stream>>>(n, band_dev(band), band->w, p, d.h3 / (4.0 * kPi), P.cx, P.cy, P.cz,
                                             P.sigma, P.A, P.M, P.N);
  k_tree_gather<<<nb, kBlock, 0, ctx->stream>>>(n, T.perm, P.A, P.M, P.N, T.St, T.anc, T.At, T.Mt, T.Nt, T.Gt);
  const F32Params fp = f32params(d, P.sigma);
  const bool screened = d.kappa > 0.0;
  {
    Scope t(ctx, &T == &ctx->tree_fine ? "tree_fine_f32" : "tree_f32");
    launch_tree(ctx, T, screened, fp, P.sigma, P.sigma * P.sigma);
  }
  {
    Scope t(ctx, "near_f64");
    k_near_spmv<<<(unsigned)(((int64_t)n * kRowLanes + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(
        n, P.row, P.col, P.coef, p, near);
  }
  {
    Scope t(ctx, "reduce");
    k_reduce<<<(unsigned)((2 * n + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(n, 1, T.far, near, p, d.lam1,
                                                                                    d.lam2, y);
  }
  return launch_ok(ctx, "matvec_tree");
}

}  // namespace pb
