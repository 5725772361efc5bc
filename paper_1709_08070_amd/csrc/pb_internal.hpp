// Internal declarations of the MI355X IBIM library (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/pb.h"

namespace pb {

constexpr double kPi = 3.14159265358979323846;
// Mixed-precision refinement: an inner solve on the FP32-far-field operator is asked for no
// more than this reduction of its own right-hand side. Below about 1e-9 relative, the FP32
// rounding of the far field dominates the residual and GMRES stops making progress; the
// outer step with the FP64 residual supplies the remaining accuracy.
constexpr double kInnerEta = 1e-7;

// Parameters derived once per call from pb_params, in the form the kernels consume.
struct Derived {
  double h, h3, eps, tau, tau2, four_tau2;
  double th1, th2;        // ε_E/ε_I, ε_I/ε_E
  double lam1, lam2;      // ½(1+ε_E/ε_I), ½(1+ε_I/ε_E)
  double kappa;
  double eps_in;
  double k12bar;          // disc average of G0 − Gκ over radius τ
  double rc;              // mixed path: near-field radius
  int metric;
  bool curved;            // curvature-corrected disc averages
  double k11c, k22c, k21bar4pi;
};

Derived derive(const pb_params& p);

// Growable device buffer owned by the context.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// Geometry of the mixed-precision operator for one band: centre of the FP32 coordinates
// and the cell list of the near field.
struct MixedPlan {
  const void* band_key = nullptr;
  int64_t n = 0;
  double cx = 0, cy = 0, cz = 0;  // centre of the FP32 coordinates
  double sigma = 1;               // FP32 coordinates are scaled by σ (= κ when κ > 0)
  double rc = 0;                  // near-field radius (unscaled)
  float rc2f = 0;                 // (σ r_c)² in FP32
  double cell = 0;
  int ncx = 0, ncy = 0, ncz = 0;
  int64_t nnz = 0;                // near-field pairs
  float4* A = nullptr;            // FP32 records: (σ(x − c), ψn weight)
  float4* M = nullptr;            //               σ·(ψ weight)·n
  float4* N = nullptr;            //               n (the target side's normal)
  float4* box = nullptr;          // bounding boxes of groups of 256 records (lo, hi)
  int64_t* row = nullptr;         // near-field CSR
  int* col = nullptr;
  double4* coef = nullptr;
  int far_cfg = 0;                // far-field tile shape chosen by the autotuner
};

// Treecode far field of the mixed operator for one band (tree.hip): octree over the FP32
// coordinates in Morton order, target batches with their direct source ranges and proxy
// clusters, and the buffers of one application. Built once per band.
constexpr int kTreeMaxDegree = 8;
struct TreePlan {
  const void* band_key = nullptr;
  int64_t n = 0;
  double rc = 0, theta = 0;
  int degree = 0;
  float u[kTreeMaxDegree + 1] = {};  // Chebyshev points of the second kind, cos(πa/p)
  MixedPlan near;                    // FP32 records (band order) and the FP64 near field
  int n_batch = 0, n_cl = 0, n_items = 0;
  int64_t n_dir_pairs = 0, n_app_pairs = 0;  // target–source and target–proxy interactions
  int* perm = nullptr;               // tree position → band index
  int2* batch = nullptr;             // target batches (tree-order ranges)
  int* dir_ptr = nullptr;            // per batch: direct source ranges
  int2* dir_rng = nullptr;
  int* app_ptr = nullptr;            // per batch: proxy clusters
  int* app_cl = nullptr;
  float4* half = nullptr;            // per cluster: half-widths of its box (scaled coordinates)
  double* ccen = nullptr;            // per cluster: FP64 centre of its box (3 doubles)
  int4* items = nullptr;             // proxy work items (cluster, begin, end, ·)
  int* item_ptr = nullptr;           // per cluster: its items
  float4 *At = nullptr, *Mt = nullptr, *Nt = nullptr;  // records in tree order (At: group-local offsets)
  float4* Gt = nullptr;              // FP32 global coordinates in tree order (the near predicate's)
  double* St = nullptr;              // exact scaled coordinates in tree order (3 per node)
  double* anc = nullptr;             // per aligned group of tree-order nodes: FP64 local origin
  float4* PX = nullptr;              // proxies: offset from the cluster centre, and Q
  float* PM = nullptr;               // proxies: M
  double2* part = nullptr;           // per item partial proxy weights
  double* far = nullptr;             // far field, band order, 2n
};

// Per-kernel-family event timing.
struct Timer {
  double ms = 0.0;
  int64_t launches = 0;
};

}  // namespace pb

struct pb_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::map<std::string, pb::DevBuf> bufs;
  int timing = 0;  // 0 off, 1 every kernel family, 2 the far-field families only
  std::map<std::string, pb::Timer> timers;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;  // per launch, resolved at sync
  std::vector<std::string> pending_name;
  std::vector<hipEvent_t> event_pool;
  int n_cu = 256;
  pb::MixedPlan mixed;
  pb::TreePlan tree;       // PB_TREE operator (and the inner operator of PB_TREE solves)
  pb::TreePlan tree_fine;  // residual operator of PB_TREE solves on large bands
  std::map<int, int> far_cfg;          // autotuned far-field tile shape per band size
  std::map<int, int> f64_cfg;          // FP64 operator kernel per band size (0 tiled, 1 symmetric)
  int sym_items_n = -1;                // band size the symmetric kernel's item list was built for
  int sym_n_items = 0;
  std::map<int64_t, int> batch_cfg;    // the same for batches, per (nodes, molecules)
  std::map<int64_t, int> batch_cfg64;  // FP64 operator kernel for batches (0 tiled, 1 symmetric)
  hipStream_t batch_stream = nullptr;  // capture stream of the batched solve
  const void* nn_key = nullptr;        // band prepared for the learned preconditioner
  int64_t nn_n = 0;
  // Device flag read by the operator's heavy kernels (far field, FP64 pairs, treecode,
  // network layers): while GMRES runs one Arnoldi step ahead of its convergence test, a
  // step enqueued after the test has been met finds the flag set and does no work.
  // nullptr outside such a cycle.
  const int* skip = nullptr;
  int* host_state = nullptr;      // pinned host slots of the per-step GMRES state (2 ints per step)
  int* host_state_dev = nullptr;  // the same memory as the device addresses it
  // status of the last allocation/launch
  pb_status fail(pb_status s, const char* fmt, ...);
};

namespace pb {

// Returns a device buffer of at least `bytes` under `name` (reallocated if smaller).
void* workspace(pb_ctx* ctx, const char* name, size_t bytes);

// Event timing around kernel launches on the context stream.
struct Scope {
  pb_ctx* ctx;
  const char* name;
  bool on;
  hipEvent_t a{}, b{};
  Scope(pb_ctx* c, const char* n);
  ~Scope();
};
void flush_timers(pb_ctx* ctx);  // after a stream synchronize
// Forgets the timings recorded since pending.size() was `mark` (launches that did no work).
void drop_timers(pb_ctx* ctx, size_t mark);

pb_status check_params(pb_ctx* ctx, const pb_params* p);
// Looks up, once per device (the context's device current), the address of the energy scratch
// array that pb_solvation_energy_noalloc uses; called by pb_create.
pb_status noalloc_init(pb_ctx* ctx);
pb_status check_band(pb_ctx* ctx, const pb_band* b);
// PB_AVG_CURVED needs the band's curvature array.
pb_status check_curv(pb_ctx* ctx, const pb_band* b, const pb_params* p);
pb_status sync(pb_ctx* ctx, const char* where);
pb_status launch_ok(pb_ctx* ctx, const char* where);

// Scans and reductions shared by the stages.
// Exclusive scan of n int64 values in place on the context stream; returns the total on host.
pb_status exclusive_scan_i64(pb_ctx* ctx, int64_t* data, int64_t n, int64_t* total_host);

// Operator internals used by the solver.
pb_status matvec_fp64(pb_ctx* ctx, const pb_band* band, const Derived& d, const double* p, double* y);
pb_status mixed_prepare(pb_ctx* ctx, const pb_band* band, const Derived& d);
pb_status near_build(pb_ctx* ctx, const pb_band* band, const Derived& d, const char* pfx, MixedPlan& P,
                     bool cells_only = false);
struct F32Params;
F32Params f32params(const Derived& d, double sigma);
// learned preconditioner (nn.hip)
pb_status nn_prepare(pb_ctx* ctx, const pb_band* band, const Derived& d);
pb_status nn_apply(pb_ctx* ctx, const pb_nn* net, const pb_band* band, const Derived& d, const double* v, double* p);
// The same network over a batch of bands whose nodes are concatenated: molecule m owns nodes
// [off[m], off[m] + cnt[m]) and vector entries [2·off[m], 2·off[m] + 2·cnt[m]) as [ψ | ψn].
struct NNBatch {
  int n_mol = 0, ntot = 0;
  double eps = 0.0;
  const int* mol_of = nullptr;  // node → molecule (caller-owned)
  int* off = nullptr;           // per molecule, device
  int* cnt = nullptr;
  double* pos = nullptr;        // ntot × 3 projections
  int* nbr = nullptr;           // ntot × 16 neighbour slots, global node indices
  float* feat = nullptr;        // ntot × 5 node features
  double* s = nullptr;          // per molecule: RMS of the two halves of the input
  uint16_t* G1 = nullptr;
  uint16_t* X[4] = {};  // hidden activations, BF16
  float* O = nullptr;
};
pb_status nn_batch_prepare(pb_ctx* ctx, int n_mol, const pb_band* bands, const int* off_host, const int* mol_of,
                           const Derived& d, NNBatch& nb);
// Z[k] = M(V[k]) for every molecule, k = *kptr (or k = 0 with kptr null); launches only, on
// `stream` (it may be under graph capture). Kernels return early once *kptr ≥ kmax.
void nn_batch_apply(hipStream_t stream, const pb_nn* net, const NNBatch& nb, const double* V, double* Z, int64_t ldv,
                    const int* kptr, int kmax, double lam1, double lam2);
pb_status matvec_mixed(pb_ctx* ctx, const pb_band* band, const Derived& d, const double* p, double* y);
// Treecode far field (tree.hip): degree of the Chebyshev proxies and the acceptance ratio θ;
// buffers named `<pfx>...`; near: an existing near field of the same band to share (else built).
// host: in/out, the Morton order, octree and batches of the band, built by the first plan of a
// solve and reused by the second (null: built and dropped).
struct TreeHost;
pb_status tree_prepare(pb_ctx* ctx, const pb_band* band, const Derived& d, int degree, double theta, TreePlan& T,
                       const char* pfx, const MixedPlan* near = nullptr, std::shared_ptr<TreeHost>* host = nullptr);
pb_status matvec_tree(pb_ctx* ctx, const pb_band* band, const Derived& d, const double* p, double* y,
                      const TreePlan& T);
// PB_TREE solves: the refinement's residuals on bands of at least kTreeFineMin nodes come from a
// finer treecode (degree 7, θ = 0.5: at the FP32 rounding level of the dense mixed operator,
// and about 5× cheaper than it at 6e5 nodes), below that from the dense mixed operator.
constexpr int kTreeFineDegree = 7;
constexpr double kTreeFineTheta = 0.5;
constexpr int64_t kTreeFineMin = 150000;
pb_status rhs(pb_ctx* ctx, const pb_band* band, const double* atoms, int n_atoms, const Derived& d, double* g);

}  // namespace pb

#define PB_HIP(ctx, call)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return (ctx)->fail(PB_EDEVICE, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                         __FILE__, __LINE__);                                               \
  } while (0)

#define PB_TRY(expr)              \
  do {                            \
    pb_status s_ = (expr);        \
    if (s_ != PB_OK) return s_;   \
  } while (0)
