// Right-hand side at the projections and Stage 4 (area and polarization energy).
//
// RHS (eq. IBIM-PBE): g1_i = Σ_k q_k/ε_I G0(x_i*, z_k),
//                     g2_i = Σ_k q_k/ε_I ∂G0(x_i*, z_k)/∂n(x_i*) = −Σ_k q_k (x_i*−z_k)·n_i/(4π ε_I |x_i*−z_k|³).
// Energy (eq. G pol): ψ_rxn(z_k) = h³ Σ_j ω_j [(θ1 ∂Gκ/∂n(y) − ∂G0/∂n(y)) ψ̄_j + (G0 − Gκ) ψ̄n_j]
//   at y = y_j*, with ρ = |z − y|, s = (z − y)·n_j: ∂G0/∂n(y) = s/(4πρ³),
//   ∂Gκ/∂n(y) = e^{−κρ}(1+κρ) s/(4πρ³). G_pol = ½ Σ_k q_k ψ_rxn(z_k); area = h³ Σ_j ω_j.
// All FP64. Reductions are fixed-order block trees (bitwise reproducible).
//
// pb_solvation_energy_noalloc runs the same kernels with no device allocation: ψ_rxn goes to
// the caller's array or to the file-scope `scratch` array below, and the three results to a
// caller-owned device array.
#include <cmath>
#include <mutex>

#include "fp64_math.hpp"
#include "pb_internal.hpp"

// ψ_rxn per atom for pb_solvation_energy_noalloc when the caller passes no array: 1 MiB
// per device, held until the process ends. Host code never names it in a launch or copy;
// it uses the address from hipGetSymbolAddress (pb::scratch_dev below).
constexpr int kNoallocMaxAtoms = 1 << 17;
static __device__ __align__(256) double scratch[kNoallocMaxAtoms];

namespace pb {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxDevices = 64;
double* scratch_dev[kMaxDevices];  // device address of `scratch` per device ordinal
std::mutex scratch_mu;

__global__ void __launch_bounds__(kBlock) k_rhs(int n, const double* __restrict__ px, const double* __restrict__ py,
                                                const double* __restrict__ pz, const double* __restrict__ nx,
                                                const double* __restrict__ ny, const double* __restrict__ nz,
                                                const double* __restrict__ atoms, int n_atoms, double eps_in,
                                                double* __restrict__ g) {
  __shared__ double4 tile[kBlock];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool live = i < n;
  double x = 0, y = 0, z = 0, a = 0, b = 0, c = 1;
  if (live) {
    x = px[i]; y = py[i]; z = pz[i];
    a = nx[i]; b = ny[i]; c = nz[i];
  }
  double s1 = 0.0, s2 = 0.0;
  const double c4 = 1.0 / (4.0 * kPi);
  for (int base = 0; base < n_atoms; base += kBlock) {
    int k = base + threadIdx.x;
    // the charge enters as q/ε_I/(4π), formed once per atom (the same operations, hoisted)
    if (k < n_atoms)
      tile[threadIdx.x] = make_double4(atoms[5 * k], atoms[5 * k + 1], atoms[5 * k + 2], atoms[5 * k + 4] / eps_in * c4);
    __syncthreads();
    int m = min(kBlock, n_atoms - base);
    if (live)
      for (int q = 0; q < m; ++q) {
        const double4 at = tile[q];
        double dx = x - at.x, dy = y - at.y, dz = z - at.z;
        double r2 = dx * dx + dy * dy + dz * dz;
        double rinv = rsqrt_f64(r2);
        double dn = dx * a + dy * b + dz * c;
        double qe = at.w;
        s1 += qe * rinv;
        s2 -= qe * dn * rinv * rinv * rinv;
      }
    __syncthreads();
  }
  if (live) {
    g[i] = s1;
    g[n + i] = s2;
  }
}

constexpr int kPsiAtoms = 8;    // atoms per block of k_psi_rxn
constexpr int kPsiBlock = 512;  // its threads: few blocks (n_atoms / 8), so wide ones

// ψ_rxn of kPsiAtoms atoms per block: every thread reads the data of each of its nodes once
// and adds that node's term to the sums of all the block's atoms, then one fixed-order block
// reduction per atom. 1/ρ is rsqrt_f64 and e^{−κρ} exp_neg_f64 (fp64_math.hpp). Per pair, times
// 4π: s(θ1 E(1 + κρ) − 1)/ρ³ · ψ̄_j + (1 − E)/ρ · ψ̄n_j, with the weight h³ω_j/4π.
__global__ void __launch_bounds__(kPsiBlock) k_psi_rxn(int n, const double* __restrict__ px, const double* __restrict__ py,
                                                    const double* __restrict__ pz, const double* __restrict__ nx,
                                                    const double* __restrict__ ny, const double* __restrict__ nz,
                                                    const double* __restrict__ w, const double* __restrict__ p,
                                                    const double* __restrict__ atoms, int n_atoms, double th1,
                                                    double kappa, double h3, double* __restrict__ psi) {
  __shared__ double red[kPsiBlock];
  __shared__ double za[kPsiAtoms][3];
  const int k0 = blockIdx.x * kPsiAtoms;
  if (threadIdx.x < 3 * kPsiAtoms) {
    const int a = threadIdx.x / 3, c = threadIdx.x % 3;
    za[a][c] = k0 + a < n_atoms ? atoms[5 * (k0 + a) + c] : 0.0;  // a missing atom's sum is not stored
  }
  __syncthreads();
  const double c4 = h3 / (4.0 * kPi);
  double acc[kPsiAtoms];
#pragma unroll
  for (int a = 0; a < kPsiAtoms; ++a) acc[a] = 0.0;
  for (int j = threadIdx.x; j < n; j += kPsiBlock) {
    const double yx = px[j], yy = py[j], yz = pz[j], nxj = nx[j], nyj = ny[j], nzj = nz[j];
    const double ww = c4 * w[j];
    const double w1 = ww * p[j], w2 = ww * p[n + j];
#pragma unroll
    for (int a = 0; a < kPsiAtoms; ++a) {
      const double dx = za[a][0] - yx, dy = za[a][1] - yy, dz = za[a][2] - yz;
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double rinv = rsqrt_f64(r2);
      const double z = kappa * (r2 * rinv);
      const double E = exp_neg_f64(z);
      const double s = dx * nxj + dy * nyj + dz * nzj;
      const double r3 = rinv * rinv * rinv;
      acc[a] += w1 * (s * r3 * (th1 * fma(E, z, E) - 1.0)) + w2 * ((1.0 - E) * rinv);
    }
  }
#pragma unroll
  for (int a = 0; a < kPsiAtoms; ++a) {
    red[threadIdx.x] = acc[a];
    __syncthreads();
    for (int off = kPsiBlock / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0 && k0 + a < n_atoms) psi[k0 + a] = red[0];
    __syncthreads();
  }
}

// The fields of pb_energy in order: out[0] = G_pol = ½ Σ_k q_k ψ_k, out[1] = G_pol in kcal/mol,
// out[2] = area = h³ Σ_j ω_j (one block, fixed order).
__global__ void __launch_bounds__(kBlock) k_finish(int n_atoms, const double* __restrict__ atoms,
                                                   const double* __restrict__ psi, int n, const double* __restrict__ w,
                                                   double h3, double* __restrict__ out) {
  __shared__ double r1[kBlock], r2[kBlock];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < n_atoms; k += kBlock) a += atoms[5 * k + 4] * psi[k];
  for (int j = threadIdx.x; j < n; j += kBlock) b += w[j];
  r1[threadIdx.x] = a;
  r2[threadIdx.x] = b;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      r1[threadIdx.x] += r1[threadIdx.x + off];
      r2[threadIdx.x] += r2[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double gpol = 0.5 * r1[0];
    out[0] = gpol;
    out[1] = gpol * 4.0 * kPi * 332.0637;
    out[2] = h3 * r2[0];
  }
}

// ψ_rxn at every atom and the energy and area into out (3 doubles, device), on ctx->stream.
void energy_launch(pb_ctx* ctx, const pb_band* band, const double* atoms, int n_atoms, const Derived& d,
                   const double* p, double* psi, double* out) {
  const int n = (int)band->n;
  k_psi_rxn<<<(n_atoms + kPsiAtoms - 1) / kPsiAtoms, kPsiBlock, 0, ctx->stream>>>(
      n, band->px, band->py, band->pz, band->nx, band->ny, band->nz, band->w, p, atoms, n_atoms, d.th1, d.kappa, d.h3,
      psi);
  k_finish<<<1, kBlock, 0, ctx->stream>>>(n_atoms, atoms, psi, n, band->w, d.h3, out);
}

}  // namespace

pb_status noalloc_init(pb_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return ctx->fail(PB_EDEVICE, "device ordinal %d beyond %d", ctx->device, kMaxDevices);
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_dev[ctx->device]) return PB_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return ctx->fail(PB_EDEVICE, "address of the energy scratch array on device %d: %s", ctx->device,
                     hipGetErrorString(e));
  scratch_dev[ctx->device] = (double*)ptr;
  return PB_OK;
}

pb_status rhs(pb_ctx* ctx, const pb_band* band, const double* atoms, int n_atoms, const Derived& d, double* g) {
  const int n = (int)band->n;
  Scope t(ctx, "rhs");
  k_rhs<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(n, band->px, band->py, band->pz, band->nx,
                                                                          band->ny, band->nz, atoms, n_atoms,
                                                                          d.eps_in, g);
  return launch_ok(ctx, "rhs");
}

}  // namespace pb

extern "C" pb_status pb_ibim_rhs(pb_ctx* ctx, const pb_band* band, const double* atoms, int n_atoms,
                                 const pb_params* prm, double* g) {
  using namespace pb;
  if (!ctx) return PB_EINVAL;
  PB_TRY(check_params(ctx, prm));
  PB_TRY(check_band(ctx, band));
  if (!atoms || n_atoms <= 0 || !g) return ctx->fail(PB_EINVAL, "pb_ibim_rhs: NULL or empty input");
  PB_HIP(ctx, hipSetDevice(ctx->device));
  PB_TRY(rhs(ctx, band, atoms, n_atoms, derive(*prm), g));
  return sync(ctx, "pb_ibim_rhs");
}

extern "C" pb_status pb_solvation_energy(pb_ctx* ctx, const pb_band* band, const double* atoms, int n_atoms,
                                         const pb_params* prm, const double* p, pb_energy* out, double* psi_rxn) {
  using namespace pb;
  if (!ctx) return PB_EINVAL;
  PB_TRY(check_params(ctx, prm));
  PB_TRY(check_band(ctx, band));
  if (!atoms || n_atoms <= 0 || !p || !out) return ctx->fail(PB_EINVAL, "pb_solvation_energy: NULL or empty input");
  PB_HIP(ctx, hipSetDevice(ctx->device));
  Derived d = derive(*prm);
  double* psi = psi_rxn ? psi_rxn : (double*)workspace(ctx, "en_psi", sizeof(double) * n_atoms);
  double* res = (double*)workspace(ctx, "en_out", 3 * sizeof(double));
  if (!psi || !res) return PB_ENOMEM;
  {
    Scope t(ctx, "energy");
    energy_launch(ctx, band, atoms, n_atoms, d, p, psi, res);
  }
  PB_TRY(launch_ok(ctx, "energy"));
  double h[3];
  PB_HIP(ctx, hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  PB_TRY(sync(ctx, "pb_solvation_energy"));
  out->g_pol = h[0];
  out->g_pol_kcal = h[1];
  out->area = h[2];
  return PB_OK;
}

extern "C" pb_status pb_solvation_energy_noalloc(pb_ctx* ctx, const pb_band* band, const double* atoms, int n_atoms,
                                                 const pb_params* prm, const double* p, double* out,
                                                 double* psi_rxn) {
  using namespace pb;
  if (!ctx) return PB_EINVAL;
  PB_TRY(check_params(ctx, prm));
  PB_TRY(check_band(ctx, band));
  if (!atoms || n_atoms <= 0 || !p || !out)
    return ctx->fail(PB_EINVAL, "pb_solvation_energy_noalloc: NULL or empty input");
  if (!psi_rxn && n_atoms > kNoallocMaxAtoms)
    return ctx->fail(PB_EINVAL,
                     "pb_solvation_energy_noalloc: %d atoms exceed the scratch array (%d); pass psi_rxn",
                     n_atoms, kNoallocMaxAtoms);
  double* psi = psi_rxn;
  if (!psi) {
    // set at pb_create for this device
    psi = ctx->device >= 0 && ctx->device < kMaxDevices ? scratch_dev[ctx->device] : nullptr;
    if (!psi) return ctx->fail(PB_EDEVICE, "pb_solvation_energy_noalloc: no scratch address for device %d",
                               ctx->device);
  }
  PB_HIP(ctx, hipSetDevice(ctx->device));
  energy_launch(ctx, band, atoms, n_atoms, derive(*prm), p, psi, out);
  return launch_ok(ctx, "pb_solvation_energy_noalloc");
}
