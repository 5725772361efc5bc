// Learned initial guess and right preconditioner for the IBIM system (not part of the
// paper's method): a point-convolution network over the band nodes, served and trained with
// BF16 MFMA kernels (FP32 accumulation, FP32 master weights, Adam).
//
// Network. Each node has 16 neighbour slots: itself and its 15 nearest band nodes by
// projection distance |x_i* − x_j*| (ties by index). Layer l maps the gathered slot features
// [16 × C_l] of a node to C_{l+1} channels: Z = G·W_l + b_l, X = leaky-ReLU(Z) (slope 0.01),
// with widths 16 → 64 → 64 → 64 → 16 (outputs 0 and 1 used). Layer-1 slot features of
// neighbour j seen from node i (10 used of 16): φ_j/ε, n_j, H_j·ε (H: mean curvature from the
// normals of the neighbours), v1_j/s1, v2_j/s2, (x_j* − x_i*)/ε, where v is the vector the
// network is applied to and s1, s2 the RMS of its two halves.
//
// Map. M(v) = Λ⁻¹ (v + s ⊙ O(v)) per node (s = (s1, s2)), i.e. the paper's diagonal solve
// plus a learned correction; a zero network is exactly Λ⁻¹. M is positively homogeneous
// (M(αv) = αM(v), α > 0). Served as x0 = M(g) and as a right preconditioner inside FGMRES.
//
// Training target for a pair (v, u = A⁻¹v): T = (Λu − v)/s per node; the loss is
// Σ|O − T|² / Σ|T|² over the band.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <type_traits>
#include <vector>

#include "pair_kernels.hpp"

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;
typedef short short8_t __attribute__((ext_vector_type(8)));

struct pb_nn {
  int device = 0;
  int64_t n_params = 0;
  float* params = nullptr;  // FP32 master: per layer W[K][Cout] (k-major) then b[Cout]
  float* grads = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  uint16_t* wt = nullptr;   // BF16 W^T per layer: [Cout][K]
  uint16_t* wk = nullptr;   // BF16 W per layer: [K][Cout]
  int64_t step = 0;
};

namespace pb {
namespace nnk {

constexpr int kSlots = 16;
constexpr int kLayers = 4;
constexpr int kCin[kLayers] = {16, 64, 64, 64};
constexpr int kCout[kLayers] = {64, 64, 64, 16};
constexpr float kSlope = 0.01f;

constexpr int kdim(int l) { return kSlots * kCin[l]; }

// parameter offsets (floats) of W_l and b_l in the flat buffer, and of the BF16 copies
inline int64_t w_off(int l) {
  int64_t o = 0;
  for (int q = 0; q < l; ++q) o += (int64_t)kdim(q) * kCout[q] + kCout[q];
  return o;
}
inline int64_t b_off(int l) { return w_off(l) + (int64_t)kdim(l) * kCout[l]; }
inline int64_t wbf_off(int l) {
  int64_t o = 0;
  for (int q = 0; q < l; ++q) o += (int64_t)kdim(q) * kCout[q];
  return o;
}
inline int64_t n_params() { return w_off(kLayers); }
inline int64_t n_wbf() { return wbf_off(kLayers); }

// FP32 → BF16 bits, round to nearest even (NaN kept quiet).
__host__ __device__ __forceinline__ uint16_t bf16_bits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8_t pack8(const float* v) {
  short8_t s;
#pragma unroll
  for (int r = 0; r < 8; ++r) s[r] = (short)bf16_bits(v[r]);
  return __builtin_bit_cast(bf16x8_t, s);
}

__device__ __forceinline__ bf16x8_t load8_bf16(const uint16_t* p) {
  short8_t s = *reinterpret_cast<const short8_t*>(p);
  return __builtin_bit_cast(bf16x8_t, s);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

__device__ __forceinline__ float act(float z) { return z > 0.f ? z : kSlope * z; }
__device__ __forceinline__ float dact(float x) { return x > 0.f ? 1.f : kSlope; }

// ---------------------------------------------------------------- geometry

// 16 nearest band nodes by projection distance (self first), from the near-field cell list.
__global__ void __launch_bounds__(kBlock) k_knn(int n, BandDev b, CellsDev cells, int* __restrict__ nbr) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double bd[kSlots];
  int bi[kSlots];
  for (int s = 0; s < kSlots; ++s) {
    bd[s] = INFINITY;
    bi[s] = i;
  }
  const double xi = b.px[i], yi = b.py[i], zi = b.pz[i];
  const int c = cells.cell_of[i];
  const int cz = c % cells.ncz, cy = (c / cells.ncz) % cells.ncy, cx = c / (cells.ncz * cells.ncy);
  for (int ax = max(cx - 1, 0); ax <= min(cx + 1, cells.ncx - 1); ++ax)
    for (int ay = max(cy - 1, 0); ay <= min(cy + 1, cells.ncy - 1); ++ay)
      for (int az = max(cz - 1, 0); az <= min(cz + 1, cells.ncz - 1); ++az) {
        const int cc = (ax * cells.ncy + ay) * cells.ncz + az;
        for (int64_t q = cells.start[cc]; q < cells.start[cc + 1]; ++q) {
          const int j = cells.nodes[q];
          const double dx = xi - b.px[j], dy = yi - b.py[j], dz = zi - b.pz[j];
          const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
          if (d2 > bd[kSlots - 1] || (d2 == bd[kSlots - 1] && j >= bi[kSlots - 1])) continue;
          int s = kSlots - 1;
          while (s > 0 && (bd[s - 1] > d2 || (bd[s - 1] == d2 && bi[s - 1] > j))) {
            bd[s] = bd[s - 1];
            bi[s] = bi[s - 1];
            --s;
          }
          bd[s] = d2;
          bi[s] = j;
        }
      }
  for (int s = 0; s < kSlots; ++s) nbr[(int64_t)i * kSlots + s] = bd[s] < INFINITY ? bi[s] : i;
}

// Per-node geometry features: φ/ε, n (3), H·ε with H = (2/m) Σ_{j≠i} (n_j − n_i)·(x_j − x_i)/|x_j − x_i|².
__global__ void __launch_bounds__(kBlock) k_geom(int n, BandDev b, const double* __restrict__ phi, double eps,
                                                 const int* __restrict__ nbr, float* __restrict__ feat) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double H = 0.0;
  int m = 0;
  for (int s = 0; s < kSlots; ++s) {
    const int j = nbr[(int64_t)i * kSlots + s];
    const double dx = b.px[j] - b.px[i], dy = b.py[j] - b.py[i], dz = b.pz[j] - b.pz[i];
    const double d2 = dx * dx + dy * dy + dz * dz;
    if (j == i || d2 < 1e-12 * eps * eps) continue;
    H += ((b.nx[j] - b.nx[i]) * dx + (b.ny[j] - b.ny[i]) * dy + (b.nz[j] - b.nz[i]) * dz) / d2;
    ++m;
  }
  H = m ? 2.0 * H / m : 0.0;
  float* f = feat + (int64_t)i * 5;
  f[0] = (float)(phi[i] / eps);
  f[1] = (float)b.nx[i];
  f[2] = (float)b.ny[i];
  f[3] = (float)b.nz[i];
  f[4] = (float)(H * eps);
}

// s[0..1] = RMS of the two halves of v (1 when zero); partial sums per block, then one block.
__global__ void __launch_bounds__(kBlock) k_rms_partial(int n, const double* __restrict__ v, double* __restrict__ part) {
  __shared__ double r1[kBlock], r2[kBlock];
  double a = 0.0, c = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    a += v[i] * v[i];
    c += v[n + i] * v[n + i];
  }
  r1[threadIdx.x] = a;
  r2[threadIdx.x] = c;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      r1[threadIdx.x] += r1[threadIdx.x + off];
      r2[threadIdx.x] += r2[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r1[0];
    part[2 * blockIdx.x + 1] = r2[0];
  }
}

// One block: strided partial sums per thread, then a fixed tree over the block.
__global__ void __launch_bounds__(kBlock) k_rms_finish(int n, int nb, const double* __restrict__ part,
                                                       double* __restrict__ s) {
  __shared__ double r1[kBlock], r2[kBlock];
  double a = 0.0, c = 0.0;
  for (int q = threadIdx.x; q < nb; q += kBlock) {
    a += part[2 * q];
    c += part[2 * q + 1];
  }
  r1[threadIdx.x] = a;
  r2[threadIdx.x] = c;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      r1[threadIdx.x] += r1[threadIdx.x + off];
      r2[threadIdx.x] += r2[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a = sqrt(r1[0] / n);
    c = sqrt(r2[0] / n);
    s[0] = a > 0.0 ? a : 1.0;
    s[1] = c > 0.0 ? c : 1.0;
  }
}

// Layer-1 input rows G1[i] = 16 slots × 16 features (BF16).
__global__ void __launch_bounds__(kBlock) k_build_g1(int n, BandDev b, const int* __restrict__ nbr,
                                                     const float* __restrict__ feat, const double* __restrict__ v,
                                                     const double* __restrict__ s, double eps,
                                                     uint16_t* __restrict__ G1) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n * kSlots) return;
  const int i = t / kSlots, slot = t % kSlots;
  const int j = nbr[(int64_t)i * kSlots + slot];
  const float* fj = feat + (int64_t)j * 5;
  float f[16];
  f[0] = fj[0];
  f[1] = fj[1];
  f[2] = fj[2];
  f[3] = fj[3];
  f[4] = fj[4];
  f[5] = (float)(v[j] / s[0]);
  f[6] = (float)(v[n + j] / s[1]);
  f[7] = (float)((b.px[j] - b.px[i]) / eps);
  f[8] = (float)((b.py[j] - b.py[i]) / eps);
  f[9] = (float)((b.pz[j] - b.pz[i]) / eps);
  for (int q = 10; q < 16; ++q) f[q] = 0.f;
  uint16_t* out = G1 + (int64_t)t * 16;
  for (int q = 0; q < 16; ++q) out[q] = bf16_bits(f[q]);
}

// ---------------------------------------------------------------- forward

// Z = A·W + b for 16-node wave tiles; A rows are G1 (dense, BF16, K = 256) or the gathered
// BF16 activations of the 16 neighbour slots (8 channels, one 16-byte load per lane and
// step). kAct (hidden layers) applies the leaky ReLU and stores BF16, rounded to nearest even
// once here (the rounding every consumer applies: the next layer's MFMA operand and the
// weight gradient's); the output layer stores FP32. Block = 4 waves = 64 nodes. The BF16 weights are staged in LDS in chunks of
// kWChunk columns and shared by the block's four waves (each wave would otherwise stream the
// whole matrix from the caches); rows are padded by 8 elements so that the 16 rows a wave
// reads at one column offset fall on different banks.
constexpr int kWChunk = 256;
constexpr int kWPad = 8;
constexpr int kFwdWaves = 8;  // 128 nodes per block: each staged weight chunk serves twice as many nodes
constexpr int kFwdNodes = 16 * kFwdWaves;

template <bool kDense, int CIN, int COUT, bool kAct>
__global__ void __launch_bounds__(64 * kFwdWaves) k_layer_fwd(int n, const uint16_t* __restrict__ G1,
                                                   const uint16_t* __restrict__ X, const int* __restrict__ nbr,
                                                   const uint16_t* __restrict__ Wt, const float* __restrict__ bias,
                                                   std::conditional_t<kAct, uint16_t, float>* __restrict__ Y,
                                                   const int* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int K = kSlots * CIN;
  constexpr int NT = COUT / 16;
  constexpr int KC = K < kWChunk ? K : kWChunk;
  static_assert(K % KC == 0 && KC % 32 == 0, "whole chunks of 32-column steps");
  __shared__ uint16_t sW[COUT][KC + kWPad];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int node0 = (blockIdx.x * kFwdWaves + wave) * 16;
  const int node = node0 + (lane & 15);
  const bool live = node < n;
  const int kq = 8 * (lane >> 4);
  f32x4_t acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  // the node's neighbour rows, looked up once (the gathered layers read every slot)
  int rows[kSlots];
#pragma unroll
  for (int q = 0; q < kSlots; ++q) rows[q] = 0;
  if (!kDense && live) {
#pragma unroll
    for (int q = 0; q < kSlots; q += 4) {
      const int4 v = *reinterpret_cast<const int4*>(nbr + (int64_t)node * kSlots + q);
      rows[q] = v.x, rows[q + 1] = v.y, rows[q + 2] = v.z, rows[q + 3] = v.w;
    }
  }
  for (int k0 = 0; k0 < K; k0 += KC) {
    // this chunk's A operands, loaded before the weights are staged so that the gathers'
    // latency overlaps the staging
    bf16x8_t a[KC / 32];
#pragma unroll
    for (int u = 0; u < KC / 32; ++u) {
      const int kk = k0 + u * 32 + kq;
      if (!live) {
        a[u] = __builtin_bit_cast(bf16x8_t, short8_t{0, 0, 0, 0, 0, 0, 0, 0});
      } else if (kDense) {
        a[u] = load8_bf16(G1 + (int64_t)node * K + kk);
      } else {
        a[u] = load8_bf16(X + (int64_t)rows[kk / CIN] * CIN + kk % CIN);
      }
    }
    __syncthreads();  // the previous chunk is no longer read
    for (int e = threadIdx.x; e < COUT * KC / 8; e += 64 * kFwdWaves) {
      const int row = e / (KC / 8), col = (e % (KC / 8)) * 8;
      *reinterpret_cast<short8_t*>(&sW[row][col]) =
          *reinterpret_cast<const short8_t*>(Wt + (int64_t)row * K + k0 + col);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < KC / 32; ++u) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const bf16x8_t bw = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const short8_t*>(
                                                             &sW[t * 16 + (lane & 15)][u * 32 + kq]));
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u], bw, acc[t], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = t * 16 + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int nd = node0 + 4 * (lane >> 4) + r;
      if (nd < n) {
        const float z = acc[t][r] + bias[j];
        if constexpr (kAct)
          Y[(int64_t)nd * COUT + j] = bf16_bits(act(z));
        else
          Y[(int64_t)nd * COUT + j] = z;
      }
    }
  }
}

// p = Λ⁻¹(v + s ⊙ O[:, 0:2])
__global__ void __launch_bounds__(kBlock) k_apply_out(int n, const double* __restrict__ v, const float* __restrict__ O,
                                                      const double* __restrict__ s, double lam1, double lam2,
                                                      double* __restrict__ p) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  p[i] = (v[i] + s[0] * (double)O[(int64_t)i * 16]) / lam1;
  p[n + i] = (v[n + i] + s[1] * (double)O[(int64_t)i * 16 + 1]) / lam2;
}

// ---------------------------------------------------------------- loss and backward

// T = (Λu − v)/s, partial Σ|T|² per block.
__global__ void __launch_bounds__(kBlock) k_target(int n, const double* __restrict__ v, const double* __restrict__ u,
                                                   const double* __restrict__ s, double lam1, double lam2,
                                                   float* __restrict__ T, double* __restrict__ part) {
  __shared__ double red[kBlock];
  double a = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const double t1 = (lam1 * u[i] - v[i]) / s[0], t2 = (lam2 * u[n + i] - v[n + i]) / s[1];
    T[2 * (int64_t)i] = (float)t1;
    T[2 * (int64_t)i + 1] = (float)t2;
    a += t1 * t1 + t2 * t2;
  }
  red[threadIdx.x] = a;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// dO = 2(O − T)/Σ|T|² on the two used channels (0 elsewhere); partial Σ|O − T|².
__global__ void __launch_bounds__(kBlock) k_loss(int n, const float* __restrict__ O, const float* __restrict__ T,
                                                 const double* __restrict__ tpart, int ntp, float* __restrict__ dO,
                                                 double* __restrict__ part) {
  __shared__ double red[kBlock];
  __shared__ double denom;
  if (threadIdx.x == 0) {
    double d = 0.0;
    for (int q = 0; q < ntp; ++q) d += tpart[q];
    denom = d > 0.0 ? d : 1.0;
  }
  __syncthreads();
  double a = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    for (int c = 0; c < 16; ++c) {
      float g = 0.f;
      if (c < 2) {
        const double e = (double)O[(int64_t)i * 16 + c] - (double)T[2 * (int64_t)i + c];
        a += e * e;
        g = (float)(2.0 * e / denom);
      }
      dO[(int64_t)i * 16 + c] = g;
    }
  }
  red[threadIdx.x] = a / denom;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// dZ = dY ⊙ act'(Y) (hidden layers; Y the stored BF16 activation, whose sign is that of the
// pre-activation) or dY (output layer), as an FP32 array.
template <bool kAct>
__global__ void __launch_bounds__(kBlock) k_dz(int64_t total, const float* __restrict__ dY,
                                               const uint16_t* __restrict__ Y, float* __restrict__ dZ) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += (int64_t)gridDim.x * kBlock)
    dZ[e] = kAct ? dY[e] * dact(bf16_to_f32(Y[e])) : dY[e];
}

// Weight gradient partials over a chunk of nodes: dW_part[blk][k][j] = Σ_nodes A[node][k]·dZ[node][j],
// db_part[blk][j] = Σ_nodes dZ[node][j]. MFMA with the nodes as the inner dimension: one
// wave per 16×16 (k, j) tile, tiles strided over the block's waves.
template <bool kDense, int CIN, int COUT>
__global__ void __launch_bounds__(256) k_wgrad(int n, int chunk, const uint16_t* __restrict__ G1,
                                               const uint16_t* __restrict__ X, const int* __restrict__ nbr,
                                               const float* __restrict__ dZ, float* __restrict__ dWp,
                                               float* __restrict__ dbp) {
  constexpr int K = kSlots * CIN;
  constexpr int KT = K / 16, JT = COUT / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n0 = blockIdx.x * chunk, n1 = min(n, n0 + chunk);
  const int nq = 8 * (lane >> 4);
  for (int tile = wave; tile < KT * JT; tile += 4) {
    const int kt = tile / JT, jt = tile % JT;
    const int krow = kt * 16 + (lane & 15);
    const int jcol = jt * 16 + (lane & 15);
    const int slot = krow / CIN, c = krow % CIN;
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    for (int nb = n0; nb < n1; nb += 32) {
      short8_t as;
      float bv[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int nd = nb + nq + r;
        if (nd < n1) {
          as[r] = (short)(kDense ? G1[(int64_t)nd * K + krow] : X[(int64_t)nbr[(int64_t)nd * kSlots + slot] * CIN + c]);
          bv[r] = dZ[(int64_t)nd * COUT + jcol];
        } else {
          as[r] = 0;
          bv[r] = 0.f;
        }
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, as), pack8(bv), acc, 0, 0, 0);
    }
    // lane holds D[k = kt·16 + 4·(lane/16) + r][j = jt·16 + lane%16]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = kt * 16 + 4 * (lane >> 4) + r;
      dWp[(int64_t)blockIdx.x * K * COUT + (int64_t)k * COUT + jcol] = acc[r];
    }
  }
  // bias partials (FP32, fixed order)
  for (int j = threadIdx.x; j < COUT; j += 256) {
    float sacc = 0.f;
    for (int nd = n0; nd < n1; ++nd) sacc += dZ[(int64_t)nd * COUT + j];
    dbp[(int64_t)blockIdx.x * COUT + j] = sacc;
  }
}

// grads[off + e] = Σ_blocks part[blk·count + e] (fixed order)
__global__ void __launch_bounds__(kBlock) k_sum_parts(int64_t count, int nblk, const float* __restrict__ part,
                                                      float* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < count; e += (int64_t)gridDim.x * kBlock) {
    float s = 0.f;
    for (int q = 0; q < nblk; ++q) s += part[(int64_t)q * count + e];
    out[e] = s;
  }
}

// dA = dZ · Wᵀ for 16-node wave tiles: dA[node][k] = Σ_j dZ[node][j]·W[k][j].
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_dgrad(int n, const float* __restrict__ dZ, const uint16_t* __restrict__ Wk,
                                               float* __restrict__ dA) {
  constexpr int K = kSlots * CIN;
  constexpr int JSTEPS = (COUT + 31) / 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int node0 = (blockIdx.x * 4 + wave) * 16;
  const int node = node0 + (lane & 15);
  const bool live = node < n;
  const int jq = 8 * (lane >> 4);
  bf16x8_t a[JSTEPS];
#pragma unroll
  for (int s = 0; s < JSTEPS; ++s) {
    float vals[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int j = s * 32 + jq + r;
      vals[r] = (live && j < COUT) ? dZ[(int64_t)node * COUT + j] : 0.f;
    }
    a[s] = pack8(vals);
  }
  for (int kt = 0; kt < K / 16; ++kt) {
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    const int kcol = kt * 16 + (lane & 15);
#pragma unroll
    for (int s = 0; s < JSTEPS; ++s) {
      float wv[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int j = s * 32 + jq + r;
        if (j < COUT) {
          const uint32_t bits = (uint32_t)Wk[(int64_t)kcol * COUT + j] << 16;
          memcpy(&wv[r], &bits, 4);
        } else {
          wv[r] = 0.f;
        }
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[s], pack8(wv), acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int nd = node0 + 4 * (lane >> 4) + r;
      if (nd < n) dA[(int64_t)nd * K + kcol] = acc[r];
    }
  }
}

// dX[j][c] = Σ_{(i, slot) with nbr[i][slot] = j} dA[i][slot·C + c], over the reverse lists
// (sorted, so the sum order is fixed).
template <int CIN>
__global__ void __launch_bounds__(kBlock) k_scatter_back(int n, const int64_t* __restrict__ rrow,
                                                         const int* __restrict__ rent, const float* __restrict__ dA,
                                                         float* __restrict__ dX) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (int64_t)n * CIN) return;
  const int j = (int)(t / CIN), c = (int)(t % CIN);
  float s = 0.f;
  for (int64_t q = rrow[j]; q < rrow[j + 1]; ++q) {
    const int e = rent[q];  // i·16 + slot
    s += dA[(int64_t)(e / kSlots) * kSlots * CIN + (int64_t)(e % kSlots) * CIN + c];
  }
  dX[t] = s;
}

__global__ void __launch_bounds__(kBlock) k_rev_count(int64_t ne, const int* __restrict__ nbr,
                                                      int64_t* __restrict__ cnt) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < ne) atomicAdd((unsigned long long*)&cnt[nbr[e]], 1ull);
}

__global__ void __launch_bounds__(kBlock) k_rev_fill(int64_t ne, const int* __restrict__ nbr,
                                                     const int64_t* __restrict__ row, int* __restrict__ cursor,
                                                     int* __restrict__ ent) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= ne) return;
  const int j = nbr[e];
  const int slot = atomicAdd(&cursor[j], 1);
  ent[row[j] + slot] = (int)e;
}

__global__ void __launch_bounds__(kBlock) k_rev_sort(int n, const int64_t* __restrict__ row, int* __restrict__ ent) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  for (int64_t q = row[j] + 1; q < row[j + 1]; ++q) {
    const int v = ent[q];
    int64_t t = q - 1;
    while (t >= row[j] && ent[t] > v) {
      ent[t + 1] = ent[t];
      --t;
    }
    ent[t + 1] = v;
  }
}

// Adam on the FP32 master parameters (bias-corrected), then the BF16 copies of the weights.
__global__ void __launch_bounds__(kBlock) k_adam(int64_t np, float* __restrict__ w, const float* __restrict__ g,
                                                 float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                                 float b2, float eps, float c1, float c2) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < np; e += (int64_t)gridDim.x * kBlock) {
    const float ge = g[e];
    const float me = b1 * m[e] + (1.f - b1) * ge;
    const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    w[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
  }
}

__global__ void __launch_bounds__(kBlock) k_cast(int K, int COUT, const float* __restrict__ W, uint16_t* __restrict__ wt,
                                                 uint16_t* __restrict__ wk) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= K * COUT) return;
  const int k = e / COUT, j = e % COUT;
  const uint16_t b = bf16_bits(W[e]);
  wk[e] = b;
  wt[(int64_t)j * K + k] = b;
}

}  // namespace nnk
}  // namespace pb

// ---------------------------------------------------------------- host side

namespace pb {
namespace {

using namespace nnk;

struct NNBufs {
  int* nbr;
  float* feat;
  int64_t* rrow;
  int* rent;
  double* s;
  double* spart;
  uint16_t* G1;
  uint16_t* X[kLayers];  // BF16; X[0] unused (layer 0 reads G1); X[l] = input of layer l
  float* T;
  float* dY;
  float* dZ;
  float* dA;
  float* dWp;
  double* lpart;
};

constexpr int kRedBlocks = 256;
constexpr int kWgradChunk = 2048;

pb_status bufs(pb_ctx* ctx, int n, NNBufs& B) {
  auto ws = [&](const char* name, size_t bytes) { return workspace(ctx, name, bytes); };
  B.nbr = (int*)ws("nn_nbr", sizeof(int) * (size_t)n * kSlots);
  B.feat = (float*)ws("nn_feat", sizeof(float) * (size_t)n * 5);
  B.rrow = (int64_t*)ws("nn_rrow", sizeof(int64_t) * (size_t)(n + 1));
  B.rent = (int*)ws("nn_rent", sizeof(int) * (size_t)n * kSlots);
  B.s = (double*)ws("nn_s", sizeof(double) * 2);
  B.spart = (double*)ws("nn_spart", sizeof(double) * 2 * kRedBlocks);
  B.G1 = (uint16_t*)ws("nn_G1", sizeof(uint16_t) * (size_t)n * kdim(0));
  B.X[0] = nullptr;
  B.X[1] = (uint16_t*)ws("nn_X1", sizeof(uint16_t) * (size_t)n * 64);
  B.X[2] = (uint16_t*)ws("nn_X2", sizeof(uint16_t) * (size_t)n * 64);
  B.X[3] = (uint16_t*)ws("nn_X3", sizeof(uint16_t) * (size_t)n * 64);
  B.T = (float*)ws("nn_T", sizeof(float) * (size_t)n * 2);
  B.dY = (float*)ws("nn_dY", sizeof(float) * (size_t)n * 64);
  B.dZ = (float*)ws("nn_dZ", sizeof(float) * (size_t)n * 64);
  B.dA = (float*)ws("nn_dA", sizeof(float) * (size_t)n * 1024);
  const int nblk = (n + kWgradChunk - 1) / kWgradChunk;
  B.dWp = (float*)ws("nn_dWp", sizeof(float) * (size_t)nblk * (1024 * 64 + 64));
  B.lpart = (double*)ws("nn_lpart", sizeof(double) * 2 * kRedBlocks);
  if (!B.nbr || !B.feat || !B.rrow || !B.rent || !B.s || !B.spart || !B.G1 || !B.X[1] || !B.X[2] || !B.X[3] || !B.T ||
      !B.dY || !B.dZ || !B.dA || !B.dWp || !B.lpart)
    return PB_ENOMEM;
  return PB_OK;
}

float* out_buf(pb_ctx* ctx, int n) { return (float*)workspace(ctx, "nn_O", sizeof(float) * (size_t)n * 16); }

}  // namespace

// Neighbour lists, geometry features and reverse lists of a band, cached on the context for
// the band last prepared.
pb_status nn_prepare(pb_ctx* ctx, const pb_band* band, const Derived& d) {
  const int n = (int)band->n;
  NNBufs B;
  PB_TRY(bufs(ctx, n, B));
  if (!band->phi) return ctx->fail(PB_EINVAL, "the learned path needs the band's phi array");
  MixedPlan P;
  PB_TRY(near_build(ctx, band, d, "nn_", P, true));
  const CellsDev cells{(const int64_t*)ctx->bufs["nn_cell_start"].ptr, (const int*)ctx->bufs["nn_cell_nodes"].ptr,
                       (const int*)ctx->bufs["nn_cell_of"].ptr, P.ncx, P.ncy, P.ncz};
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  k_knn<<<nb, kBlock, 0, ctx->stream>>>(n, band_dev(band), cells, B.nbr);
  k_geom<<<nb, kBlock, 0, ctx->stream>>>(n, band_dev(band), band->phi, d.eps, B.nbr, B.feat);
  // reverse lists of (node, slot) per neighbour
  const int64_t ne = (int64_t)n * kSlots;
  int* cursor = (int*)workspace(ctx, "nn_cursor", sizeof(int) * (size_t)n);
  if (!cursor) return PB_ENOMEM;
  PB_HIP(ctx, hipMemsetAsync(B.rrow, 0, sizeof(int64_t) * (size_t)(n + 1), ctx->stream));
  PB_HIP(ctx, hipMemsetAsync(cursor, 0, sizeof(int) * (size_t)n, ctx->stream));
  const unsigned nbe = (unsigned)((ne + kBlock - 1) / kBlock);
  k_rev_count<<<nbe, kBlock, 0, ctx->stream>>>(ne, B.nbr, B.rrow);
  PB_TRY(launch_ok(ctx, "nn reverse count"));
  PB_TRY(exclusive_scan_i64(ctx, B.rrow, n + 1, nullptr));
  k_rev_fill<<<nbe, kBlock, 0, ctx->stream>>>(ne, B.nbr, B.rrow, cursor, B.rent);
  k_rev_sort<<<nb, kBlock, 0, ctx->stream>>>(n, B.rrow, B.rent);
  PB_TRY(launch_ok(ctx, "nn prepare"));
  ctx->nn_key = band->px;
  ctx->nn_n = n;
  return PB_OK;
}

static pb_status nn_check_prepared(pb_ctx* ctx, const pb_band* band) {
  if (ctx->nn_key != band->px || ctx->nn_n != band->n)
    return ctx->fail(PB_EINVAL, "the learned path was not prepared for this band");
  return PB_OK;
}

// p = M(v); keeps the activations of this application in the workspace.
pb_status nn_apply(pb_ctx* ctx, const pb_nn* net, const pb_band* band, const Derived& d, const double* v, double* p) {
  PB_TRY(nn_check_prepared(ctx, band));
  const int n = (int)band->n;
  NNBufs B;
  PB_TRY(bufs(ctx, n, B));
  float* O = out_buf(ctx, n);
  if (!O) return PB_ENOMEM;
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  const unsigned nbf = (unsigned)((n + kFwdNodes - 1) / kFwdNodes);
  Scope t(ctx, "nn");
  k_rms_partial<<<kRedBlocks, kBlock, 0, ctx->stream>>>(n, v, B.spart);
  k_rms_finish<<<1, kBlock, 0, ctx->stream>>>(n, kRedBlocks, B.spart, B.s);
  k_build_g1<<<(unsigned)(((int64_t)n * kSlots + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(
      n, band_dev(band), B.nbr, B.feat, v, B.s, d.eps, B.G1);
  const uint16_t* wt = net->wt;
  const float* prm = net->params;
  k_layer_fwd<true, 16, 64, true><<<nbf, 64 * kFwdWaves, 0, ctx->stream>>>(n, B.G1, nullptr, B.nbr, wt + wbf_off(0),
                                                                 prm + b_off(0), B.X[1], ctx->skip);
  k_layer_fwd<false, 64, 64, true><<<nbf, 64 * kFwdWaves, 0, ctx->stream>>>(n, nullptr, B.X[1], B.nbr, wt + wbf_off(1),
                                                                  prm + b_off(1), B.X[2], ctx->skip);
  k_layer_fwd<false, 64, 64, true><<<nbf, 64 * kFwdWaves, 0, ctx->stream>>>(n, nullptr, B.X[2], B.nbr, wt + wbf_off(2),
                                                                  prm + b_off(2), B.X[3], ctx->skip);
  k_layer_fwd<false, 64, 16, false><<<nbf, 64 * kFwdWaves, 0, ctx->stream>>>(n, nullptr, B.X[3], B.nbr, wt + wbf_off(3),
                                                                   prm + b_off(3), O, ctx->skip);
  k_apply_out<<<nb, kBlock, 0, ctx->stream>>>(n, v, O, B.s, d.lam1, d.lam2, p);
  return launch_ok(ctx, "nn apply");
}

// Loss and gradients (into net->grads) of the pair (v, u = A⁻¹v); loss to host.
pb_status nn_grads(pb_ctx* ctx, pb_nn* net, const pb_band* band, const Derived& d, const double* v, const double* u,
                   double* loss) {
  const int n = (int)band->n;
  double* ptmp = (double*)workspace(ctx, "nn_ptmp", sizeof(double) * 2 * (size_t)n);
  if (!ptmp) return PB_ENOMEM;
  PB_TRY(nn_apply(ctx, net, band, d, v, ptmp));
  NNBufs B;
  PB_TRY(bufs(ctx, n, B));
  float* O = out_buf(ctx, n);
  const unsigned nbl = (unsigned)((n + 63) / 64);
  const unsigned ew = 2048;
  Scope t(ctx, "nn");
  k_target<<<kRedBlocks, kBlock, 0, ctx->stream>>>(n, v, u, B.s, d.lam1, d.lam2, B.T, B.lpart);
  float* dO = B.dY;  // n × 16 fits in the n × 64 buffer
  k_loss<<<kRedBlocks, kBlock, 0, ctx->stream>>>(n, O, B.T, B.lpart, kRedBlocks, dO, B.lpart + kRedBlocks);
  const int nblk = (n + kWgradChunk - 1) / kWgradChunk;
  float* g = net->grads;
  const int64_t n64 = n;
  // layer 3 (output): dZ = dO
  k_dz<false><<<ew, kBlock, 0, ctx->stream>>>(n64 * 16, dO, nullptr, B.dZ);
  k_wgrad<false, 64, 16><<<nblk, 256, 0, ctx->stream>>>(n, kWgradChunk, nullptr, B.X[3], B.nbr, B.dZ, B.dWp,
                                                        B.dWp + (int64_t)nblk * 1024 * 16);
  k_sum_parts<<<ew, kBlock, 0, ctx->stream>>>(1024 * 16, nblk, B.dWp, g + w_off(3));
  k_sum_parts<<<1, kBlock, 0, ctx->stream>>>(16, nblk, B.dWp + (int64_t)nblk * 1024 * 16, g + b_off(3));
  k_dgrad<64, 16><<<nbl, 256, 0, ctx->stream>>>(n, B.dZ, net->wk + wbf_off(3), B.dA);
  k_scatter_back<64><<<(unsigned)((n64 * 64 + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(n, B.rrow, B.rent,
                                                                                              B.dA, B.dY);
  // layers 2, 1: dZ = dX_{l+1} ⊙ act'(X_{l+1}); input of layer l is X[l]
  for (int l = 2; l >= 1; --l) {
    k_dz<true><<<ew, kBlock, 0, ctx->stream>>>(n64 * 64, B.dY, B.X[l + 1], B.dZ);
    k_wgrad<false, 64, 64><<<nblk, 256, 0, ctx->stream>>>(n, kWgradChunk, nullptr, B.X[l], B.nbr, B.dZ, B.dWp,
                                                          B.dWp + (int64_t)nblk * 1024 * 64);
    k_sum_parts<<<ew, kBlock, 0, ctx->stream>>>(1024 * 64, nblk, B.dWp, g + w_off(l));
    k_sum_parts<<<1, kBlock, 0, ctx->stream>>>(64, nblk, B.dWp + (int64_t)nblk * 1024 * 64, g + b_off(l));
    k_dgrad<64, 64><<<nbl, 256, 0, ctx->stream>>>(n, B.dZ, net->wk + wbf_off(l), B.dA);
    k_scatter_back<64><<<(unsigned)((n64 * 64 + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(n, B.rrow, B.rent,
                                                                                                B.dA, B.dY);
  }
  // layer 0: input G1 (dense), no input gradient
  k_dz<true><<<ew, kBlock, 0, ctx->stream>>>(n64 * 64, B.dY, B.X[1], B.dZ);
  k_wgrad<true, 16, 64><<<nblk, 256, 0, ctx->stream>>>(n, kWgradChunk, B.G1, nullptr, B.nbr, B.dZ, B.dWp,
                                                       B.dWp + (int64_t)nblk * 256 * 64);
  k_sum_parts<<<ew, kBlock, 0, ctx->stream>>>(256 * 64, nblk, B.dWp, g + w_off(0));
  k_sum_parts<<<1, kBlock, 0, ctx->stream>>>(64, nblk, B.dWp + (int64_t)nblk * 256 * 64, g + b_off(0));
  PB_TRY(launch_ok(ctx, "nn backward"));
  if (loss) {
    std::vector<double> lp(kRedBlocks);
    PB_HIP(ctx, hipMemcpyAsync(lp.data(), B.lpart + kRedBlocks, sizeof(double) * kRedBlocks, hipMemcpyDeviceToHost,
                               ctx->stream));
    PB_TRY(sync(ctx, "nn loss"));
    double s = 0.0;
    for (double x : lp) s += x;
    *loss = s;
  }
  return PB_OK;
}

pb_status nn_cast(pb_ctx* ctx, pb_nn* net) {
  for (int l = 0; l < kLayers; ++l) {
    const int K = kdim(l), C = kCout[l];
    k_cast<<<(unsigned)((K * C + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(
        K, C, net->params + w_off(l), net->wt + wbf_off(l), net->wk + wbf_off(l));
  }
  return launch_ok(ctx, "nn cast");
}

// ---------------------------------------------------------------- batch of bands

namespace {

// Per molecule: s[2m], s[2m + 1] = RMS of the two halves of its segment of v (1 when zero).
// One block per molecule, fixed summation order.
__global__ void __launch_bounds__(kBlock) k_rms_batch(int n_mol, const int* __restrict__ off, const int* __restrict__ cnt,
                                                      const double* __restrict__ V, int64_t ldv,
                                                      const int* __restrict__ kptr, int kmax, double* __restrict__ s) {
  __shared__ double r1[kBlock], r2[kBlock];
  const int m = blockIdx.x;
  if (m >= n_mol) return;
  if (kptr && *kptr >= kmax) return;
  const double* v = V + (kptr ? (int64_t)(*kptr) * ldv : 0) + 2 * (int64_t)off[m];
  const int n = cnt[m];
  double a = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) {
    a += v[i] * v[i];
    c += v[n + i] * v[n + i];
  }
  r1[threadIdx.x] = a;
  r2[threadIdx.x] = c;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      r1[threadIdx.x] += r1[threadIdx.x + o];
      r2[threadIdx.x] += r2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double q1 = sqrt(r1[0] / n), q2 = sqrt(r2[0] / n);
    s[2 * m] = q1 > 0.0 ? q1 : 1.0;
    s[2 * m + 1] = q2 > 0.0 ? q2 : 1.0;
  }
}

// Layer-1 input rows of every node of the batch (as k_build_g1, per molecule).
__global__ void __launch_bounds__(kBlock) k_build_g1_batch(int ntot, const int* __restrict__ mol_of,
                                                           const int* __restrict__ off, const int* __restrict__ cnt,
                                                           const double* __restrict__ pos, const int* __restrict__ nbr,
                                                           const float* __restrict__ feat,
                                                           const double* __restrict__ V, int64_t ldv,
                                                           const int* __restrict__ kptr, int kmax,
                                                           const double* __restrict__ s, double eps,
                                                           uint16_t* __restrict__ G1) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (int64_t)ntot * kSlots) return;
  if (kptr && *kptr >= kmax) return;
  const int i = (int)(t / kSlots), slot = (int)(t % kSlots);
  const int j = nbr[(int64_t)i * kSlots + slot];
  const int m = mol_of[i];
  const int n = cnt[m];
  const double* v = V + (kptr ? (int64_t)(*kptr) * ldv : 0) + 2 * (int64_t)off[m];
  const int lj = j - off[m];
  const float* fj = feat + (int64_t)j * 5;
  float f[16];
  f[0] = fj[0];
  f[1] = fj[1];
  f[2] = fj[2];
  f[3] = fj[3];
  f[4] = fj[4];
  f[5] = (float)(v[lj] / s[2 * m]);
  f[6] = (float)(v[n + lj] / s[2 * m + 1]);
  f[7] = (float)((pos[3 * (int64_t)j] - pos[3 * (int64_t)i]) / eps);
  f[8] = (float)((pos[3 * (int64_t)j + 1] - pos[3 * (int64_t)i + 1]) / eps);
  f[9] = (float)((pos[3 * (int64_t)j + 2] - pos[3 * (int64_t)i + 2]) / eps);
  for (int q = 10; q < 16; ++q) f[q] = 0.f;
  uint16_t* out = G1 + t * 16;
  for (int q = 0; q < 16; ++q) out[q] = bf16_bits(f[q]);
}

// p = Λ⁻¹(v + s_m ⊙ O[:, 0:2]) over every molecule's segment.
__global__ void __launch_bounds__(kBlock) k_apply_out_batch(int ntot, const int* __restrict__ mol_of,
                                                            const int* __restrict__ off, const int* __restrict__ cnt,
                                                            const double* __restrict__ V, double* __restrict__ Z,
                                                            int64_t ldv, const int* __restrict__ kptr, int kmax,
                                                            const float* __restrict__ O, const double* __restrict__ s,
                                                            double lam1, double lam2) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= ntot) return;
  if (kptr && *kptr >= kmax) return;
  const int m = mol_of[i];
  const int n = cnt[m], l = i - off[m];
  const int64_t base = (kptr ? (int64_t)(*kptr) * ldv : 0) + 2 * (int64_t)off[m];
  Z[base + l] = (V[base + l] + s[2 * m] * (double)O[(int64_t)i * 16]) / lam1;
  Z[base + n + l] = (V[base + n + l] + s[2 * m + 1] * (double)O[(int64_t)i * 16 + 1]) / lam2;
}

// Local neighbour indices of one molecule → global node indices; positions into the batch table.
__global__ void __launch_bounds__(kBlock) k_batch_geometry(int n, int off, BandDev b, int* __restrict__ nbr,
                                                           double* __restrict__ pos) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  for (int q = 0; q < kSlots; ++q) nbr[(int64_t)i * kSlots + q] += off;
  pos[3 * (int64_t)i] = b.px[i];
  pos[3 * (int64_t)i + 1] = b.py[i];
  pos[3 * (int64_t)i + 2] = b.pz[i];
}

}  // namespace

pb_status nn_batch_prepare(pb_ctx* ctx, int n_mol, const pb_band* bands, const int* off_host, const int* mol_of,
                           const Derived& d, NNBatch& nb) {
  int64_t ntot64 = 0;
  std::vector<int> cnt_host(n_mol);
  for (int m = 0; m < n_mol; ++m) {
    if (!bands[m].phi) return ctx->fail(PB_EINVAL, "the learned path needs each band's phi array (molecule %d)", m);
    cnt_host[m] = (int)bands[m].n;
    ntot64 += bands[m].n;
  }
  const int ntot = (int)ntot64;
  auto ws = [&](const char* name, size_t bytes) { return workspace(ctx, name, bytes); };
  nb.n_mol = n_mol;
  nb.ntot = ntot;
  nb.eps = d.eps;
  nb.mol_of = mol_of;
  nb.off = (int*)ws("nnb_off", sizeof(int) * n_mol);
  nb.cnt = (int*)ws("nnb_cnt", sizeof(int) * n_mol);
  nb.pos = (double*)ws("nnb_pos", sizeof(double) * 3 * (size_t)ntot);
  nb.nbr = (int*)ws("nnb_nbr", sizeof(int) * kSlots * (size_t)ntot);
  nb.feat = (float*)ws("nnb_feat", sizeof(float) * 5 * (size_t)ntot);
  nb.s = (double*)ws("nnb_s", sizeof(double) * 2 * n_mol);
  nb.G1 = (uint16_t*)ws("nnb_G1", sizeof(uint16_t) * (size_t)ntot * kdim(0));
  nb.X[0] = nullptr;
  nb.X[1] = (uint16_t*)ws("nnb_X1", sizeof(uint16_t) * 64 * (size_t)ntot);
  nb.X[2] = (uint16_t*)ws("nnb_X2", sizeof(uint16_t) * 64 * (size_t)ntot);
  nb.X[3] = (uint16_t*)ws("nnb_X3", sizeof(uint16_t) * 64 * (size_t)ntot);
  nb.O = (float*)ws("nnb_O", sizeof(float) * 16 * (size_t)ntot);
  if (!nb.off || !nb.cnt || !nb.pos || !nb.nbr || !nb.feat || !nb.s || !nb.G1 || !nb.X[1] || !nb.X[2] || !nb.X[3] ||
      !nb.O)
    return PB_ENOMEM;
  PB_HIP(ctx, hipMemcpyAsync(nb.off, off_host, sizeof(int) * n_mol, hipMemcpyHostToDevice, ctx->stream));
  PB_HIP(ctx, hipMemcpyAsync(nb.cnt, cnt_host.data(), sizeof(int) * n_mol, hipMemcpyHostToDevice, ctx->stream));
  for (int m = 0; m < n_mol; ++m) {
    const pb_band* band = &bands[m];
    const int n = (int)band->n, o = off_host[m];
    MixedPlan P;
    PB_TRY(near_build(ctx, band, d, "nnb_", P, true));
    const CellsDev cells{(const int64_t*)ctx->bufs["nnb_cell_start"].ptr, (const int*)ctx->bufs["nnb_cell_nodes"].ptr,
                         (const int*)ctx->bufs["nnb_cell_of"].ptr, P.ncx, P.ncy, P.ncz};
    const unsigned nbk = (unsigned)((n + kBlock - 1) / kBlock);
    int* nbr_m = nb.nbr + (int64_t)o * kSlots;
    k_knn<<<nbk, kBlock, 0, ctx->stream>>>(n, band_dev(band), cells, nbr_m);
    k_geom<<<nbk, kBlock, 0, ctx->stream>>>(n, band_dev(band), band->phi, d.eps, nbr_m, nb.feat + (int64_t)o * 5);
    k_batch_geometry<<<nbk, kBlock, 0, ctx->stream>>>(n, o, band_dev(band), nbr_m, nb.pos + 3 * (int64_t)o);
    PB_TRY(launch_ok(ctx, "nn batch prepare"));
  }
  return PB_OK;
}

void nn_batch_apply(hipStream_t stream, const pb_nn* net, const NNBatch& nb, const double* V, double* Z, int64_t ldv,
                    const int* kptr, int kmax, double lam1, double lam2) {
  const int ntot = nb.ntot;
  k_rms_batch<<<nb.n_mol, kBlock, 0, stream>>>(nb.n_mol, nb.off, nb.cnt, V, ldv, kptr, kmax, nb.s);
  k_build_g1_batch<<<(unsigned)(((int64_t)ntot * kSlots + kBlock - 1) / kBlock), kBlock, 0, stream>>>(
      ntot, nb.mol_of, nb.off, nb.cnt, nb.pos, nb.nbr, nb.feat, V, ldv, kptr, kmax, nb.s, nb.eps, nb.G1);
  const unsigned nbf = (unsigned)((ntot + kFwdNodes - 1) / kFwdNodes);
  const uint16_t* wt = net->wt;
  const float* prm = net->params;
  k_layer_fwd<true, 16, 64, true><<<nbf, 64 * kFwdWaves, 0, stream>>>(ntot, nb.G1, nullptr, nb.nbr, wt + wbf_off(0),
                                                          prm + b_off(0), nb.X[1], nullptr);
  k_layer_fwd<false, 64, 64, true><<<nbf, 64 * kFwdWaves, 0, stream>>>(ntot, nullptr, nb.X[1], nb.nbr, wt + wbf_off(1),
                                                           prm + b_off(1), nb.X[2], nullptr);
  k_layer_fwd<false, 64, 64, true><<<nbf, 64 * kFwdWaves, 0, stream>>>(ntot, nullptr, nb.X[2], nb.nbr, wt + wbf_off(2),
                                                           prm + b_off(2), nb.X[3], nullptr);
  k_layer_fwd<false, 64, 16, false><<<nbf, 64 * kFwdWaves, 0, stream>>>(ntot, nullptr, nb.X[3], nb.nbr, wt + wbf_off(3),
                                                            prm + b_off(3), nb.O, nullptr);
  k_apply_out_batch<<<(unsigned)((ntot + kBlock - 1) / kBlock), kBlock, 0, stream>>>(
      ntot, nb.mol_of, nb.off, nb.cnt, V, Z, ldv, kptr, kmax, nb.O, nb.s, lam1, lam2);
}

}  // namespace pb

// ---------------------------------------------------------------- C-ABI

extern "C" {

pb_status pb_nn_create(pb_ctx* ctx, uint64_t seed, pb_nn** out) {
  using namespace pb;
  using namespace pb::nnk;
  if (!ctx || !out) return PB_EINVAL;
  PB_HIP(ctx, hipSetDevice(ctx->device));
  pb_nn* net = new pb_nn();
  net->device = ctx->device;
  net->n_params = n_params();
  const size_t pb = sizeof(float) * (size_t)net->n_params;
  if (hipMalloc(&net->params, pb) != hipSuccess || hipMalloc(&net->grads, pb) != hipSuccess ||
      hipMalloc(&net->adam_m, pb) != hipSuccess || hipMalloc(&net->adam_v, pb) != hipSuccess ||
      hipMalloc(&net->wt, sizeof(uint16_t) * (size_t)n_wbf()) != hipSuccess ||
      hipMalloc(&net->wk, sizeof(uint16_t) * (size_t)n_wbf()) != hipSuccess) {
    pb_nn_destroy(net);
    return ctx->fail(PB_ENOMEM, "pb_nn_create: allocation failed");
  }
  // He-uniform weights from a SplitMix64 stream; biases zero; the output layer starts at zero
  // so an untrained network is exactly the diagonal solve Λ⁻¹.
  std::vector<float> h((size_t)net->n_params, 0.f);
  uint64_t st = seed;
  auto next = [&]() {
    uint64_t z = (st += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  };
  for (int l = 0; l < kLayers - 1; ++l) {
    const double a = std::sqrt(6.0 / kdim(l));
    for (int64_t e = 0; e < (int64_t)kdim(l) * kCout[l]; ++e) h[w_off(l) + e] = (float)((2.0 * next() - 1.0) * a);
  }
  PB_HIP(ctx, hipMemcpy(net->params, h.data(), pb, hipMemcpyHostToDevice));
  PB_HIP(ctx, hipMemset(net->adam_m, 0, pb));
  PB_HIP(ctx, hipMemset(net->adam_v, 0, pb));
  PB_HIP(ctx, hipMemset(net->grads, 0, pb));
  PB_TRY(nn_cast(ctx, net));
  PB_TRY(sync(ctx, "pb_nn_create"));
  *out = net;
  return PB_OK;
}

void pb_nn_destroy(pb_nn* net) {
  if (!net) return;
  (void)hipSetDevice(net->device);
  for (void* p : {(void*)net->params, (void*)net->grads, (void*)net->adam_m, (void*)net->adam_v, (void*)net->wt,
                  (void*)net->wk})
    if (p) (void)hipFree(p);
  delete net;
}

int64_t pb_nn_param_count(void) { return pb::nnk::n_params(); }

pb_status pb_nn_get_params(pb_ctx* ctx, const pb_nn* net, float* host, float* grads_host) {
  if (!ctx || !net || (!host && !grads_host)) return PB_EINVAL;
  PB_HIP(ctx, hipSetDevice(ctx->device));
  PB_TRY(pb::sync(ctx, "pb_nn_get_params"));
  const size_t bytes = sizeof(float) * (size_t)net->n_params;
  if (host) PB_HIP(ctx, hipMemcpy(host, net->params, bytes, hipMemcpyDeviceToHost));
  if (grads_host) PB_HIP(ctx, hipMemcpy(grads_host, net->grads, bytes, hipMemcpyDeviceToHost));
  return PB_OK;
}

pb_status pb_nn_set_params(pb_ctx* ctx, pb_nn* net, const float* host) {
  if (!ctx || !net || !host) return PB_EINVAL;
  for (int64_t e = 0; e < net->n_params; ++e)
    if (!std::isfinite(host[e])) return ctx->fail(PB_EINVAL, "pb_nn_set_params: non-finite parameter %lld", (long long)e);
  PB_HIP(ctx, hipSetDevice(ctx->device));
  PB_HIP(ctx, hipMemcpy(net->params, host, sizeof(float) * (size_t)net->n_params, hipMemcpyHostToDevice));
  PB_TRY(pb::nn_cast(ctx, net));
  return pb::sync(ctx, "pb_nn_set_params");
}

pb_status pb_nn_prepare(pb_ctx* ctx, const pb_band* band, const pb_params* prm) {
  using namespace pb;
  if (!ctx) return PB_EINVAL;
  PB_TRY(check_params(ctx, prm));
  PB_TRY(check_band(ctx, band));
  PB_HIP(ctx, hipSetDevice(ctx->device));
  PB_TRY(nn_prepare(ctx, band, derive(*prm)));
  return sync(ctx, "pb_nn_prepare");
}

pb_status pb_nn_apply(pb_ctx* ctx, const pb_nn* net, const pb_band* band, const pb_params* prm, const double* v,
                      double* p) {
  using namespace pb;
  if (!ctx || !net || !v || !p) return PB_EINVAL;
  PB_TRY(check_params(ctx, prm));
  PB_TRY(check_band(ctx, band));
  PB_HIP(ctx, hipSetDevice(ctx->device));
  PB_TRY(nn_apply(ctx, net, band, derive(*prm), v, p));
  return sync(ctx, "pb_nn_apply");
}

pb_status pb_nn_train_step(pb_ctx* ctx, pb_nn* net, const pb_band* band, const pb_params* prm, const double* v,
                           const double* u, float lr, double* loss) {
  using namespace pb;
  if (!ctx || !net || !v || !u || !(lr >= 0.f)) return PB_EINVAL;
  PB_TRY(check_params(ctx, prm));
  PB_TRY(check_band(ctx, band));
  PB_HIP(ctx, hipSetDevice(ctx->device));
  PB_TRY(nn_grads(ctx, net, band, derive(*prm), v, u, loss));
  if (lr > 0.f) {
    net->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)net->step), c2 = 1.f - std::pow(b2, (float)net->step);
    k_adam<<<1024, kBlock, 0, ctx->stream>>>(net->n_params, net->params, net->grads, net->adam_m, net->adam_v, lr, b1,
                                             b2, 1e-8f, c1, c2);
    PB_TRY(nn_cast(ctx, net));
  }
  return sync(ctx, "pb_nn_train_step");
}

pb_status pb_nn_geometry(pb_ctx* ctx, const pb_band* band, int* nbr_host, float* feat_host) {
  if (!ctx || !band) return PB_EINVAL;
  PB_TRY(pb::nn_check_prepared(ctx, band));
  PB_TRY(pb::sync(ctx, "pb_nn_geometry"));
  const size_t n = (size_t)band->n;
  if (nbr_host)
    PB_HIP(ctx, hipMemcpy(nbr_host, ctx->bufs["nn_nbr"].ptr, sizeof(int) * n * pb::nnk::kSlots, hipMemcpyDeviceToHost));
  if (feat_host) PB_HIP(ctx, hipMemcpy(feat_host, ctx->bufs["nn_feat"].ptr, sizeof(float) * n * 5, hipMemcpyDeviceToHost));
  return PB_OK;
}

}  // extern "C"
