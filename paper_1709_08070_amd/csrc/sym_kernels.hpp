// Symmetric FP32 far field: every unordered pair {i, j} is evaluated once and contributes to
// both i and j.
//
// The four kernels of the IBIM operator (eq. IBIM-PBE with the regularized kernels of the
// section "Regularization of the singular kernels") depend on the pair through d = x_i − x_j,
// the two normals and the two weights. With the scalar weights W = σ·w̃ (ψ) and V = w̃n (ψn),
// in κ-scaled coordinates (r' = κr, E = e^{−r'}, a = E(1 + r'), c1,2 = 1 − θ1,2 a,
// g = E r'² − 3(1 − a)) the contributions of the pair are
//   to i:  a1 += (c1/r'³)(d·n_j) W_j − ((1 − E)/r') V_j,
//          a2 += [W_j Q + c2 (d·n_i) V_j]/r'³,
//   to j:  a1 += −(c1/r'³)(d·n_i) W_i − ((1 − E)/r') V_i,
//          a2 += [W_i Q − c2 (d·n_j) V_i]/r'³,
// with Q = (1 − a)(n_i·n_j) + (d·n_i)(d·n_j) g/r'² the weight-free K21 core, symmetric in
// (i, j); it is evaluated with g/r'² = E − 3(1 − a)/r'² and a = E(1 + r') as one FMA each.
// Everything but the last products is shared: 42 FP32 operations and 2 transcendentals per
// unordered pair, 21 + 1 per ordered pair (34 + 2 for one direction at a time); the factor
// 1/r'³ enters once through a/r'³, c2/r'³ and Q/r'³. Records: A = (σ(x − c), V) and
// N = (n, W), two float4 per node.
//
// Work decomposition. The band is cut into chunks of C = 512·nsub nodes (nC chunks). One
// work item is a chunk pair (Ic, Jc) with Ic ≤ Jc; the partial sums keep the chunked layout
// of the one-directional kernel, partial[c][e] = contributions to vector entry e from the
// sources of chunk c. Item (Ic, Jc), Ic < Jc, owns the slots (Jc, i ∈ Ic) (forward) and
// (Ic, j ∈ Jc) (reverse); the diagonal item (Ic, Ic) owns (Ic, i ∈ Ic). Every slot belongs to
// exactly one item, which accumulates into it in FP64 in a fixed order, so the result is
// bitwise reproducible and needs no atomics in global memory. The forward sums of a target
// sub-block stay in registers over all the item's source sub-blocks and are stored once; the
// reverse sums of a source sub-block are stored after its first target sub-block and added
// to after each later one (a slot's first writer stores, the later ones add: no zeroing pass).
//
// Inside an item the block (256 threads, 4 waves) walks sub-blocks of 512 nodes: targets T
// (2 per thread), sources S staged in LDS. For T ≠ S, lane l of a wave pairs its targets with
// source g·64 + ((l + s) mod 64) at step s, so the 64 lanes touch 64 different sources. The
// reverse sums travel with their source: after each step every lane passes its running sums
// to lane l − 1 (ds_bpermute), which takes that source at the next step; after 64 steps lane
// l holds the sums of source g·64 + l, accumulated in a fixed order. For T = S (only in
// diagonal items; it holds the self pair and the nearest pairs) the one-directional loop with
// the near-pair predicate runs.
// Sub-block pairs whose bounding boxes are farther apart than r_c (with the margin of
// F32Params::far2) skip the predicate.
#pragma once

#include "pair_kernels.hpp"

namespace pb {

constexpr int kSymSub = 512;  // nodes per sub-block
constexpr int kSymWaves = kBlock / 64;

struct SymShared {
  float4 sA[kSymSub], sN[kSymSub];
  float racc[kSymWaves][2][kSymSub];
};

// Radial and pair terms shared by both directions (see the header), 1/r' being 0 for a near
// pair when kCheck: P1 = c1/r'³, C2 = c2/r'³, f0r = (1 − E)/r', Qr = Q/r'³; dnx = d·n_i,
// dny = d·n_j.
struct PairTerms {
  float P1, C2, f0r, Qr, dnx, dny;
};

template <bool kScreened, bool kCheck>
__device__ __forceinline__ PairTerms pair_terms(const float4& ta, const float4& tn, const float4& sa,
                                                const float4& sn, const F32Params& fp) {
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
  const float ri2 = rinv * rinv;
  const float r3 = ri2 * rinv;
  const float ar3 = a * r3;
  PairTerms t;
  t.dnx = __fmaf_rn(dz, tn.z, __fmaf_rn(dy, tn.y, dx * tn.x));
  t.dny = __fmaf_rn(dz, sn.z, __fmaf_rn(dy, sn.y, dx * sn.x));
  t.P1 = __fmaf_rn(-fp.th1, ar3, r3);
  t.C2 = __fmaf_rn(-fp.th2, ar3, r3);
  if (kScreened) {
    const float nn = __fmaf_rn(tn.z, sn.z, __fmaf_rn(tn.y, sn.y, tn.x * sn.x));
    const float gr = __fmaf_rn(__fmaf_rn(3.f, a, -3.f), ri2, E);  // g/r'² = E − 3(1 − a)/r'²
    t.f0r = __fmaf_rn(-E, rinv, rinv);
    t.Qr = __fmaf_rn(t.dnx * t.dny, gr, __fmaf_rn(-a, nn, nn)) * r3;
  } else {  // κ = 0: E = a = 1 and z = 0, so 1 − E = 0 and Q = 0
    t.f0r = 0.f;
    t.Qr = 0.f;
  }
  return t;
}

// Both directions of one pair. Target side (i): ta = (x_i, V_i), tn = (n_i, W_i); source side
// (j): sa, sn. fa1/fa2 accumulate the contributions to i, ra1/ra2 those to j.
template <bool kScreened, bool kCheck>
__device__ __forceinline__ void pair_sym(const float4& ta, const float4& tn, const float4& sa, const float4& sn,
                                         const F32Params& fp, float& fa1, float& fa2, float& ra1, float& ra2) {
  const PairTerms t = pair_terms<kScreened, kCheck>(ta, tn, sa, sn, fp);
  fa1 = __fmaf_rn(t.P1 * t.dny, sn.w, fa1);
  ra1 = __fmaf_rn(-(t.P1 * t.dnx), tn.w, ra1);
  fa2 = __fmaf_rn(t.C2 * t.dnx, sa.w, __fmaf_rn(t.Qr, sn.w, fa2));
  ra2 = __fmaf_rn(-(t.C2 * t.dny), ta.w, __fmaf_rn(t.Qr, tn.w, ra2));
  if (kScreened) {
    fa1 = __fmaf_rn(-t.f0r, sa.w, fa1);
    ra1 = __fmaf_rn(-t.f0r, ta.w, ra1);
  }
}

// One direction (i ← j) of the same formula, for the diagonal sub-blocks.
template <bool kScreened>
__device__ __forceinline__ void pair_fwd(const float4& ta, const float4& tn, const float4& sa, const float4& sn,
                                         const F32Params& fp, float& fa1, float& fa2) {
  const PairTerms t = pair_terms<kScreened, true>(ta, tn, sa, sn, fp);
  fa1 = __fmaf_rn(t.P1 * t.dny, sn.w, fa1);
  fa2 = __fmaf_rn(t.C2 * t.dnx, sa.w, __fmaf_rn(t.Qr, sn.w, fa2));
  if (kScreened) fa1 = __fmaf_rn(-t.f0r, sa.w, fa1);
}

// Targets [t0, t0 + 512) (full, 2 per thread: t0 + 128w + l and 64 further) against sources
// [s0, s0 + 512) of the same records, s0 ≠ t0, both directions. Adds the unscaled forward sums
// S1, S2 of the thread's two targets into f (a1, a2 of the first, then of the second); stores
// σ·S1, σ²·S2 of the sources into rev (index j − s0), or adds them when rev_acc. Every thread
// of the block calls it (it synchronizes).
template <bool kScreened, bool kCheck>
__device__ __forceinline__ void sym_block(const float4* __restrict__ A, const float4* __restrict__ N, int n, int t0,
                                          int s0, const F32Params& fp, double sig1, double sig2, SymShared& sh,
                                          double (&f)[4], double* rev1, double* rev2, bool rev_acc) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int q = tid; q < kSymSub; q += kBlock) {
    const int j = s0 + q;
    if (j < n) {
      sh.sA[q] = A[j];
      sh.sN[q] = N[j];
    } else {  // padding: zero weights and normals (such tiles run with the predicate)
      sh.sA[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      sh.sN[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  const int ia = t0 + w * 128 + lane, ib = ia + 64;
  const float4 taa = A[ia], tna = N[ia];
  const float4 tab = A[ib], tnb = N[ib];
  __syncthreads();
  const int next = ((lane + 1) & 63) << 2;  // byte address of lane l + 1 for ds_bpermute
  for (int g = 0; g < kSymSub; g += 64) {
    float fa1 = 0.f, fa2 = 0.f, fb1 = 0.f, fb2 = 0.f;
    float ra1 = 0.f, ra2 = 0.f;  // at step s: the reverse sums of source g + ((lane + s) mod 64)
#pragma unroll 2
    for (int s = 0; s < 64; ++s) {
      const int q = g + ((lane + s) & 63);
      const float4 sa = sh.sA[q], sn = sh.sN[q];
      pair_sym<kScreened, kCheck>(taa, tna, sa, sn, fp, fa1, fa2, ra1, ra2);
      pair_sym<kScreened, kCheck>(tab, tnb, sa, sn, fp, fb1, fb2, ra1, ra2);
      ra1 = __int_as_float(__builtin_amdgcn_ds_bpermute(next, __float_as_int(ra1)));
      ra2 = __int_as_float(__builtin_amdgcn_ds_bpermute(next, __float_as_int(ra2)));
    }
    sh.racc[w][0][g + lane] = ra1;  // 64 rotations: lane l holds source g + l
    sh.racc[w][1][g + lane] = ra2;
    f[0] += (double)fa1;
    f[1] += (double)fa2;
    f[2] += (double)fb1;
    f[3] += (double)fb2;
  }
  __syncthreads();
  for (int q = tid; q < kSymSub; q += kBlock) {
    if (s0 + q < n) {
      double x1 = 0.0, x2 = 0.0;
      for (int v = 0; v < kSymWaves; ++v) {
        x1 += (double)sh.racc[v][0][q];
        x2 += (double)sh.racc[v][1][q];
      }
      rev1[q] = sig1 * x1 + (rev_acc ? rev1[q] : 0.0);
      rev2[q] = sig2 * x2 + (rev_acc ? rev2[q] : 0.0);
    }
  }
  __syncthreads();
}

// Targets [t0, t0 + 512) (the same two per thread as sym_block) against the sources of the
// same sub-block, one direction, with the near-pair predicate (the self pair and the nearest
// pairs are here). Adds the unscaled sums into f.
template <bool kScreened>
__device__ __forceinline__ void diag_block(const float4* __restrict__ A, const float4* __restrict__ N, int n, int t0,
                                           const F32Params& fp, SymShared& sh, double (&f)[4]) {
  const int tid = threadIdx.x;
  for (int q = tid; q < kSymSub; q += kBlock) {
    const int j = t0 + q;
    if (j < n) {
      sh.sA[q] = A[j];
      sh.sN[q] = N[j];
    } else {
      sh.sA[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      sh.sN[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  const int ia = t0 + (tid >> 6) * 128 + (tid & 63), ib = ia + 64;
  const float4 taa = ia < n ? A[ia] : make_float4(0.f, 0.f, 0.f, 0.f);
  const float4 tna = ia < n ? N[ia] : make_float4(0.f, 0.f, 1.f, 0.f);  // dead targets: results unused
  const float4 tab = ib < n ? A[ib] : make_float4(0.f, 0.f, 0.f, 0.f);
  const float4 tnb = ib < n ? N[ib] : make_float4(0.f, 0.f, 1.f, 0.f);
  __syncthreads();
  for (int g = 0; g < kSymSub; g += 64) {
    float fa1 = 0.f, fa2 = 0.f, fb1 = 0.f, fb2 = 0.f;
#pragma unroll 4
    for (int q = g; q < g + 64; ++q) {
      const float4 sa = sh.sA[q], sn = sh.sN[q];
      pair_fwd<kScreened>(taa, tna, sa, sn, fp, fa1, fa2);
      pair_fwd<kScreened>(tab, tnb, sa, sn, fp, fb1, fb2);
    }
    f[0] += (double)fa1;
    f[1] += (double)fa2;
    f[2] += (double)fb1;
    f[3] += (double)fb2;
  }
  __syncthreads();
}

// One work item (Ic, Jc), Ic ≤ Jc, of a band of n records with chunks of nsub sub-blocks.
// partial: the band's chunked partial sums (slot (c, e) at partial[c·2n + e]).
template <bool kScreened>
__device__ __forceinline__ void sym_item(const float4* __restrict__ A, const float4* __restrict__ N,
                                         const float4* __restrict__ box, int n, int Ic, int Jc, int nsub,
                                         const F32Params& fp, double sig1, double sig2, double* __restrict__ partial,
                                         SymShared& sh) {
  const int C = nsub * kSymSub;
  const int i0 = Ic * C, i1 = min(n, i0 + C), j0 = Jc * C, j1 = min(n, j0 + C);
  double* rowF = partial + (int64_t)Jc * 2 * n;  // slots (Jc, i): contributions of chunk Jc
  double* rowR = partial + (int64_t)Ic * 2 * n;  // slots (Ic, j): contributions of chunk Ic
  const bool diag = Ic == Jc;
  const int tid = threadIdx.x;
  for (int T = i0; T < i1; T += kSymSub) {
    float4 tlo, thi;
    box_union(box, T / kGroup, min(T + kSymSub, n + kGroup - 1) / kGroup, tlo, thi);
    double f[4] = {0.0, 0.0, 0.0, 0.0};
    // reverse slots of the item's source sub-blocks: stored at the first target sub-block,
    // added to at the later ones (in a diagonal item a sub-block's slots then also take its
    // own forward sums, after every reverse contribution, since targets go in increasing order)
    const bool rev_acc = T != i0;
    for (int S = (diag ? T : j0); S < j1; S += kSymSub) {
      if (S == T) {
        diag_block<kScreened>(A, N, n, T, fp, sh, f);
        continue;
      }
      int clear = 0;
      if (S + kSymSub <= n) {
        float4 slo, shi;
        box_union(box, S / kGroup, (S + kSymSub) / kGroup, slo, shi);
        clear = box_gap2(tlo, thi, slo, shi) >= fp.far2;
      }
      clear = __builtin_amdgcn_readfirstlane(clear);
      if (clear)
        sym_block<kScreened, false>(A, N, n, T, S, fp, sig1, sig2, sh, f, rowR + S, rowR + n + S, rev_acc);
      else
        sym_block<kScreened, true>(A, N, n, T, S, fp, sig1, sig2, sh, f, rowR + S, rowR + n + S, rev_acc);
    }
    // forward sums of the two targets of this thread, once per target sub-block; in a
    // diagonal item the earlier target sub-blocks' reverse sums are already in these slots
    const bool fwd_acc = diag && T != i0;
    const int ia = T + (tid >> 6) * 128 + (tid & 63), ib = ia + 64;
    if (ia < n) {
      rowF[ia] = sig1 * f[0] + (fwd_acc ? rowF[ia] : 0.0);
      rowF[n + ia] = sig2 * f[1] + (fwd_acc ? rowF[n + ia] : 0.0);
    }
    if (ib < n) {
      rowF[ib] = sig1 * f[2] + (fwd_acc ? rowF[ib] : 0.0);
      rowF[n + ib] = sig2 * f[3] + (fwd_acc ? rowF[n + ib] : 0.0);
    }
    __syncthreads();
  }
}

// Symmetric FP32 far field of one band: one block per work item (items: (Ic, Jc) pairs).
template <bool kScreened>
static __global__ void __attribute__((unused)) __launch_bounds__(kBlock)
    k_p2p_f32_sym(const float4* __restrict__ A, const float4* __restrict__ N,
                  const float4* __restrict__ box, int n, int nsub, const int2* __restrict__ items, int n_items,
                  F32Params fp, double sig1, double sig2, double* __restrict__ partial,
                  const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ SymShared sh;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int2 w = items[it];
    sym_item<kScreened>(A, N, box, n, w.x, w.y, nsub, fp, sig1, sig2, partial, sh);
  }
}

// Chunking of a band of n nodes for the symmetric kernel: about 100 chunks (≈5000 items)
// for large bands, chunks of one sub-block for small ones.
inline int sym_nsub(int n) { return std::max(1, (n + 100 * kSymSub - 1) / (100 * kSymSub)); }
inline int sym_chunks(int n) {
  const int C = sym_nsub(n) * kSymSub;
  return (n + C - 1) / C;
}

}  // namespace pb
