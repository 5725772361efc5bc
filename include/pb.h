/*
 * pb.h — C-ABI of the MI355X implicit boundary integral method (IBIM) library for the
 * linearized Poisson–Boltzmann equation (Zhong, Ren, Tsai, arXiv:1709.08070).
 *
 * Conventions shared by every call
 * --------------------------------
 * Units: lengths in Å, charges in e. Potentials and energies are in the paper's units,
 *   in which G0 = 1/(4πr) and charges enter as q/ε (energy unit e²/(ε0·Å));
 *   pb_energy.g_pol_kcal multiplies by 4π·332.0637 to give kcal/mol.
 * Memory: pointers documented as "device" are HIP device memory owned by the caller
 *   (for example torch tensors); the library never frees them and never keeps them
 *   after a call returns. "host" pointers are ordinary CPU memory. The library owns
 *   its own workspace (allocated on demand, released by pb_destroy).
 * Layouts:
 *   atoms  — n_atoms × 5 doubles, row-major (x, y, z, radius, charge).
 *   grid   — node (i, j, k) sits at origin + h·(i, j, k); linear index (i·ny + j)·nz + k.
 *   band   — structure of arrays, one entry per band node, nodes in increasing linear
 *            grid index (lexicographic order).
 *   p, y, g — 2n doubles [ψ̄(band order); ψ̄_n(band order)].
 * Streams: every kernel runs on the stream given to pb_create (0 = the null stream).
 *   Calls that return host values (counts, statistics, energies) synchronize that stream.
 * Errors: every call returns a pb_status; nothing throws across the ABI. pb_last_error
 *   gives a message for the last failing call on a context. Inputs are validated
 *   (PB_EINVAL) before any kernel is launched.
 * Threads: a context is not thread-safe; use one context per host thread.
 */
#ifndef PB_H_
#define PB_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PB_OK = 0,
  PB_EINVAL = -1,    /* invalid argument (non-finite, non-positive, NULL, unsupported mode) */
  PB_ENOMEM = -2,    /* device workspace allocation failed */
  PB_EDEVICE = -3,   /* a HIP runtime call failed */
  PB_ECAPACITY = -4, /* output buffer too small; the required size is reported */
  PB_ENOCONV = -5,   /* solver stopped before the tolerance; best iterate and statistics written */
  PB_EGEOM = -6      /* degenerate geometry: empty band, band touching the grid edge, zero gradient */
} pb_status;

/* Regularization predicate ‖x* − y*‖_P < τ of the kernel regularization (eq. reg-kernel):
   tangent-plane distance at x* with the guard |x* − y*| < 2τ (default), the literal
   tangent-plane distance, or the Euclidean distance. */
enum { PB_REG_TANGENT_GUARDED = 0, PB_REG_TANGENT = 1, PB_REG_EUCLIDEAN = 2 };
/* Level set: van der Waals union F(x) = min_k(|x − z_k| − r_k) (exact signed distance for a
   single atom), or the solvent excluded surface of Stage 1. */
enum { PB_LS_VDW = 0, PB_LS_SES = 1 };
/* Arithmetic of the operator: FP64 everywhere; FP32 pair kernels with FP64 near field,
   FP64 accumulation and FP64 iterative refinement; or the same with the far field from a
   treecode (Chebyshev proxies of degree tree_degree on octree source clusters accepted at
   ratio tree_theta; the cluster-particle form of the fast multipole acceleration of section
   "Fast linear solvers"). In a solve, PB_TREE is the inner operator of the refinement; the
   refinement's residuals come from the dense PB_MIXED operator until they meet tol/2, and
   the exact FP64 operator then certifies the result, so the solution meets tol for the
   exact discrete system. */
enum { PB_FP64 = 0, PB_MIXED = 1, PB_TREE = 2 };
/* GMRES initial guess: zero, Λ⁻¹g (the paper's diagonal preconditioner), caller's p, learned. */
enum { PB_X0_ZERO = 0, PB_X0_DIAG = 1, PB_X0_USER = 2, PB_X0_LEARNED = 3 };
enum { PB_PRECOND_NONE = 0, PB_PRECOND_LEARNED = 1 };
/* ∇φ at band nodes (section "Projections and weights"): the average (p₋ + p₊)/2 of the two
   fifth-order WENO one-sided derivatives per axis (the section's choice for its simulations;
   the default), or second-order central differences. */
enum { PB_GRAD_CENTRAL = 0, PB_GRAD_WENO = 1 };
/* Jacobian in the band weight: J ≡ 1 (every experiment of the paper), or the explicit
   J = 1 − φΔφ + φ²⟨n, adj(∇²φ) n⟩ of section "Implicit boundary integral methods" (read
   with the adjugate of the Hessian; second-order central differences). */
enum { PB_JAC_ONE = 0, PB_JAC_FULL = 1 };
/* Values of the regularized pairs (eq. reg-kernel-a, reg-kernel-b): the paper's disc
   averages (0, K̄12, 0, 0), or with the leading curvature term of the double-layer averages
   and the exact flat-disc average of K21:
     K̄11 = −(1 − θ1ā)·c/(8πτ),  K̄22 = −(1 − θ2ā)·c/(8πτ),  K̄21 = (e^{−κτ} − 1 + κτ)/(2πτ³),
   c = κ1 + κ2 of the surface at the target's projection (pb_band.curv), ā = (2 − (2 + κτ)e^{−κτ})/(κτ)
   the disc mean of e^{−κr}(1 + κr). PB_AVG_CURVED needs band->curv; the batched solve and the
   symmetric FP64 kernel take the paper's averages only. */
enum { PB_AVG_FLAT = 0, PB_AVG_CURVED = 1 };

typedef struct pb_ctx pb_ctx;

typedef struct {
  double eps_in;     /* ε_I, dielectric constant inside the molecule (experiments: 1) */
  double eps_out;    /* ε_E, dielectric constant of the solvent (experiments: 80) */
  double kappa;      /* κ in Gκ = e^{−κr}/(4πr), Å⁻¹ (experiments: 0.1257) */
  double probe;      /* ρ0, probe radius of the SES, Å (1.4) */
  double h;          /* grid spacing, Å */
  double band_k;     /* band half-width ε = band_k·h (experiments: 2) */
  double tau_k;      /* regularization radius τ = tau_k·h (experiments: 1 or 0.5) */
  double cfl;        /* level-set time step Δt = cfl·h (0.3) */
  double near_k;     /* mixed path: pairs closer than max(near_k·h, 2τ) use the FP64 near field (2) */
  double tree_theta; /* PB_TREE: a source cluster is interpolated when (r_B + r_C) < θ·distance (0.6) */
  int reg_metric;    /* PB_REG_* */
  int ls_mode;       /* PB_LS_* */
  int reinit_steps;  /* reinitialization steps; 0 = 2·ceil((band_k + 4)/cfl) */
  int grad_scheme;   /* PB_GRAD_* (default the WENO average) */
  int jacobian;      /* PB_JAC_* (default J ≡ 1) */
  int tree_degree;   /* PB_TREE: degree p of the Chebyshev proxies per axis, 2..8 (4) */
  int reg_avg;       /* PB_AVG_* (default the paper's flat disc averages) */
} pb_params;

typedef struct {
  int nx, ny, nz;
  double origin[3];
  double h;
} pb_grid;

typedef struct {
  int64_t n;          /* out: band node count (on PB_ECAPACITY: the required count) */
  int64_t capacity;   /* in: entries available in every array below */
  double *px, *py, *pz;   /* device: closest-point projection x* = x − φ n */
  double *nx, *ny, *nz;   /* device: unit normal ∇φ/|∇φ|, ∇φ by pb_params.grad_scheme */
  double *phi;            /* device: level-set value at the node */
  double *w;              /* device: ω = J·δ_ε(φ), J per pb_params.jacobian (h³ is applied by the operator) */
  int64_t *gidx;          /* device: linear grid index of the node */
  double *curv;           /* device, optional: κ1 + κ2 of Γ at x* from the central-difference Hessian
                             of φ, written when non-NULL; needed by PB_AVG_CURVED */
} pb_band;

typedef struct {
  double tol;        /* stop when ‖g − Ap‖₂/‖g‖₂ ≤ tol (true FP64 residual) */
  int max_iter;      /* total Krylov iterations allowed (all restarts and refinement steps) */
  int restart;       /* GMRES restart length m (basis of m+1 vectors of 2n doubles) */
  int precision;     /* PB_FP64 or PB_MIXED */
  int x0;            /* PB_X0_* */
  int precond;       /* PB_PRECOND_* */
  int max_outer;     /* mixed path: refinement steps (each one FP64 residual) */
  const void* nn;    /* learned preconditioner weights (pb_nn handle) or NULL */
} pb_solve_opts;

typedef struct {
  int iters;            /* Krylov iterations (operator applications inside Arnoldi) */
  int outer;            /* refinement steps taken (1 for the FP64 path) */
  int converged;        /* 1 if the true residual met tol */
  int fallback_used;    /* 1 if the learned path was abandoned for plain GMRES */
  int matvecs_fp64;     /* FP64 operator applications */
  int matvecs_mixed;    /* mixed-precision (or treecode) operator applications: one per Arnoldi
                           step, one per restart that ends on the restart length, one for a
                           non-zero starting vector; a cycle that ends on its residual
                           estimate takes none (the FP64 or fine residual of the refinement
                           follows), nor does a solve from zero */
  double true_relres;   /* ‖g − Ap‖₂/‖g‖₂ with the FP64 operator, at exit */
  double t_total_s;     /* wall time of the call */
  double t_matvec_s;    /* device time inside the operator kernels */
  double pairs;         /* pair-interactions evaluated: n² per dense operator application; for
                           PB_TREE applications the direct, proxy and near-field interactions */
} pb_solve_stats;

typedef struct {
  double g_pol;       /* polarization energy ½ Σ q_k ψ_rxn(z_k), paper units */
  double g_pol_kcal;  /* the same in kcal/mol */
  double area;        /* surface area h³ Σ ω_j, Å² */
} pb_energy;

/* Context on one device and one stream. device: HIP ordinal; hip_stream: a hipStream_t
   or NULL. Returns PB_EDEVICE if the device cannot be used. */
pb_status pb_create(pb_ctx** out, int device, void* hip_stream);
void pb_destroy(pb_ctx* ctx);
const char* pb_last_error(const pb_ctx* ctx);
/* Parameters of the paper's experiments ("Numerical experiments": ε_I = 1, ε_E = 80,
   κ = 0.1257, ε = 2h, τ = h; normals from the WENO average and J ≡ 1 as in section
   "Projections and weights") with ρ0 = 1.4, h = 0.5, cfl = 0.3, near_k = 2. */
void pb_default_params(pb_params* out);
void pb_default_solve_opts(pb_solve_opts* out);

/* Grid on hℤ³ covering the atoms (host, n_atoms × 5) with a margin of
   r_max + ρ0 (SES only) + ε + 4h + 1 Å. Host-only; no device work. PB_EINVAL for non-finite
   atoms, negative radii, h ≤ 0, or an axis of more than 4096 nodes. */
pb_status pb_grid_for_atoms(const double* atoms_host, int n_atoms, const pb_params* prm, pb_grid* grid);

/* Stage 1 (section "Creating a signed distance function to the solvent accessible
   surface" and its subsections): φ on the grid.
   PB_LS_VDW: φ = F(x) = min_k(|x − z_k| − r_k) (eq. vdW-levelset-fn).
   PB_LS_SES: φ_SAS = F − ρ0, inward eikonal flow φ_t = |∇φ| to t = ρ0 (TVD-RK3, Godunov
   Hamiltonian, WENO5, zero-Neumann ghosts), cavity removal (flood fill from the grid
   boundary through φ > 0; unreached nodes within ε + h of a cavity set to −ε), then
   reinitialization φ_t + sgn_h(φ0)(|∇φ| − 1) = 0 (eqs. reinit, signum).
   grid: as from pb_grid_for_atoms (grid->h must equal prm->h). atoms: device, n_atoms × 5.
   phi: device, cap doubles, caller-owned; on success its first nx·ny·nz entries hold φ in
   the grid's linear order. Two-call size protocol: with phi == NULL the call only validates
   and writes the element count nx·ny·nz to *needed (atoms may then be NULL); with
   cap < nx·ny·nz it returns PB_ECAPACITY with *needed set, before any device work, and
   writes nothing. needed may be NULL. PB_EINVAL if an axis has fewer than 7 or more than 4096
   nodes, grid->h differs from prm->h, the grid has 2^31 nodes or more, or atoms is NULL or
   empty in a call that builds φ. */
pb_status pb_build_levelset(pb_ctx* ctx, const double* atoms, int n_atoms, const pb_params* prm,
                            const pb_grid* grid, double* phi, size_t cap, size_t* needed);

/* Stage 2 (section "Projections and weights"): band nodes −ε < φ < ε in lexicographic
   order, n = ∇φ/|∇φ| with ∇φ by prm->grad_scheme, x* = x − φ n, ω = δ_ε(φ)·J
   (eq. cosine-kernel; J by prm->jacobian, WENO ghosts by even reflection at the grid
   boundary as in Stage 1). phi: device. band: caller fills capacity and the device arrays; on return n holds
   the node count. PB_ECAPACITY if capacity < count (n = count, arrays untouched beyond
   capacity); PB_EGEOM if a band node lies on the grid edge or has zero gradient. */
pb_status pb_narrowband_compact(pb_ctx* ctx, const pb_grid* grid, const double* phi, const pb_params* prm,
                                pb_band* band);

/* The right-hand side g at the projections (eq. IBIM-PBE): g1 = Σ_k q_k/ε_I G0(x*, z_k),
   g2 = Σ_k q_k/ε_I ∂G0(x*, z_k)/∂n(x*). atoms: device; g: device, 2n. */
pb_status pb_ibim_rhs(pb_ctx* ctx, const pb_band* band, const double* atoms, int n_atoms, const pb_params* prm,
                      double* g);

/* y = Λp + KWp (eq. final-lin-sys), the four regularized kernels of eq. IBIM-PBE and the
   regularization subsection, h³ and ω folded in. precision PB_FP64 or PB_MIXED.
   p, y: device, 2n; they must not overlap.
   PB_MIXED: FP32 far field + FP64 near field (every pair closer than r_c, the regularized
   ones included). The far-field kernel is chosen once per band size (per batch shape in
   pb_ibim_solve_batched) by timing the candidates (bands of 262,144 nodes or more take the
   symmetric kernel without timing); the environment variable PB_FAR_CFG=k
   fixes it instead: k = 0..3 the one-directional kernel with (sources per LDS tile, targets
   per lane) = (256, 1), (512, 1), (256, 2), (512, 2); k = 4 the symmetric kernel (each
   unordered pair evaluated once for both directions). All give the same operator up to
   FP32 rounding; each is bitwise reproducible from run to run.
   PB_FP64: the same choice between the one-directional kernel (PB_F64_CFG=0) and the
   symmetric one (PB_F64_CFG=1), which evaluates the regularization test per direction and
   skips it on sub-block pairs too far apart for any pair to be regularized. */
pb_status pb_ibim_matvec(pb_ctx* ctx, const pb_band* band, const pb_params* prm, int precision, const double* p,
                         double* y);

/* Solve Λp + KWp = g by GMRES (section "Fast linear solvers"; x0 = Λ⁻¹g by default).
   Computes g from the atoms (device). p: device, 2n; input when opts->x0 == PB_X0_USER,
   output always (best iterate on PB_ENOCONV). stats: host, may be NULL. */
pb_status pb_ibim_solve(pb_ctx* ctx, const pb_band* band, const double* atoms, int n_atoms, const pb_params* prm,
                        const pb_solve_opts* opts, double* p, pb_solve_stats* stats);

/* Stage 4 (sections "Computing surface area", "Computing the polarization energy"):
   area = h³ Σ ω_j and G_pol = ½ Σ_k q_k ψ_rxn(z_k) with ψ_rxn by the IBIM sum. atoms and p:
   device. out: host. psi_rxn: device, n_atoms doubles, or NULL. */
pb_status pb_solvation_energy(pb_ctx* ctx, const pb_band* band, const double* atoms, int n_atoms,
                              const pb_params* prm, const double* p, pb_energy* out, double* psi_rxn);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
   serving loops, harnesses that forbid allocation): pb_solvation_energy that allocates
   nothing and does not synchronize. It launches the same kernels on the context stream and
   writes the fields of pb_energy, in order (g_pol, g_pol_kcal, area), to out: device, 3
   doubles, caller-owned, valid once the stream has reached the call. psi_rxn: device,
   n_atoms doubles, or NULL, in which case ψ_rxn goes to a scratch array of the library's
   (131072 doubles per device, one per GPU for the life of the process; located at pb_create).
   PB_EINVAL beyond 131072 atoms with psi_rxn == NULL. Every call on one GPU that passes
   psi_rxn == NULL shares that GPU's scratch array: such calls must not overlap in time
   (different streams or host threads race on it); each call overwrites the entries it
   uses before reading them. Results equal pb_solvation_energy's bit for bit. */
pb_status pb_solvation_energy_noalloc(pb_ctx* ctx, const pb_band* band, const double* atoms, int n_atoms,
                                      const pb_params* prm, const double* p, double* out, double* psi_rxn);

/* Batched solve statistics (host). */
typedef struct {
  double t_total_s;    /* wall time of the call, set-up included */
  double t_p50_s;      /* median per-molecule time to solution, from the start of the solve to
                          the end of the molecule's last restart cycle (device clock); the
                          FP64 residual that confirms it is formed at the batch's next outer
                          step */
  double t_p99_s;      /* 99th percentile of the same */
  double pairs;        /* pair-interactions evaluated over the whole batch */
  int graph_replays;   /* replays of the captured Arnoldi-step graph */
  int far_tile;        /* far-field sources per LDS tile chosen by the autotuner */
  int far_tpl;         /* far-field targets per lane chosen by the autotuner */
  int n_items;         /* work items of the persistent far-field launch */
  int outer;           /* refinement steps */
  int far_symmetric;   /* 1 if the autotuner chose the symmetric far-field kernel (each
                          unordered pair once, both directions; far_tile/far_tpl then give
                          its 512-node sub-block and 2 targets per lane) */
} pb_batch_stats;

/* Solves n_mol independent molecules (section "Fast linear solvers" for each) in one batch,
   mixed precision (opts->precision must be PB_MIXED): every operator application of the
   batch is one persistent far-field launch over a largest-first list of equal-cost
   (molecule, target block, source chunk) items plus one near-field/reduce launch; one
   Arnoldi step of all molecules is a captured hipGraph replayed until every molecule has
   converged. bands: host array of n_mol bands (device arrays inside). atoms: host array of
   n_mol device pointers (n_atoms[m] × 5). p: host array of n_mol device pointers (2n_m
   doubles each), input when opts->x0 == PB_X0_USER, output always. stats: host, n_mol
   entries, may be NULL; bstats: host, may be NULL. PB_ENOCONV if any molecule misses the
   tolerance (all results still written). The refinement is pb_ibim_solve's: a first pass on
   the mixed operator from the initial guess, then FP64 residuals (stats[m].matvecs_fp64, one
   per pass of molecule m) decide convergence and drive the correction solves.
   Learned path (opts->x0 == PB_X0_LEARNED and/or opts->precond == PB_PRECOND_LEARNED,
   opts->nn set, every band's phi present): the network runs over all molecules at once;
   as right preconditioner inside the captured step (flexible GMRES), as x0 = M(g). A
   molecule that misses the tolerance on the learned path is solved again without the
   network from its last iterate (from Λ⁻¹g if that is not finite) with what is left of
   opts->max_iter (the preconditioned pass takes at most half of it); stats[m].fallback_used
   reports it. PB_EINVAL: precision other than PB_MIXED, the literal tangent metric, an
   unknown x0 or preconditioner mode, a learned mode without opts->nn or a band's phi. */
pb_status pb_ibim_solve_batched(pb_ctx* ctx, int n_mol, const pb_band* bands, const double* const* atoms,
                                const int* n_atoms, const pb_params* prm, const pb_solve_opts* opts,
                                double* const* p, pb_solve_stats* stats, pb_batch_stats* bstats);

/* ---- Learned initial guess / right preconditioner (not part of the paper's method).
   A point-convolution network over the band nodes (16 neighbour slots: the node and its 15
   nearest band nodes by projection distance; widths 16 → 64 → 64 → 64 → 2; leaky ReLU),
   BF16 weights and MFMA products with FP32 accumulation. Applied to a vector v it returns
   M(v) = Λ⁻¹(v + s ⊙ O(v)), s = per-half RMS of v: the paper's diagonal solve plus a learned
   correction (an untrained network is exactly Λ⁻¹). pb_ibim_solve uses it as x0 = M(g)
   (PB_X0_LEARNED) and as a right preconditioner inside FGMRES (PB_PRECOND_LEARNED), with plain
   GMRES as the fallback: a learned solve that misses the tolerance (or whose iterate is not
   finite) continues without the network from its last iterate (from Λ⁻¹g if that is not
   finite) and reports fallback_used. Both passes share opts->max_iter; the preconditioned
   pass takes at most half of it. */
typedef struct pb_nn pb_nn;
/* Network with He-uniform weights from a SplitMix64 stream of `seed`, last layer zero. */
pb_status pb_nn_create(pb_ctx* ctx, uint64_t seed, pb_nn** out);
void pb_nn_destroy(pb_nn* net);
/* Number of FP32 parameters (per layer W[K][Cout] row-major, then b[Cout]). */
int64_t pb_nn_param_count(void);
/* Host copies of the FP32 master parameters and/or the last gradients (either may be NULL). */
pb_status pb_nn_get_params(pb_ctx* ctx, const pb_nn* net, float* params_host, float* grads_host);
pb_status pb_nn_set_params(pb_ctx* ctx, pb_nn* net, const float* params_host);
/* Neighbour lists and geometry features of a band (needs band->phi); required before
   pb_nn_apply / pb_nn_train_step on that band (the solve does it itself). */
pb_status pb_nn_prepare(pb_ctx* ctx, const pb_band* band, const pb_params* prm);
/* p = M(v); v, p: device, 2n. */
pb_status pb_nn_apply(pb_ctx* ctx, const pb_nn* net, const pb_band* band, const pb_params* prm, const double* v,
                      double* p);
/* One Adam step (lr > 0; lr = 0 only computes gradients) on the pair (v, u = A⁻¹v): loss
   Σ|O − T|²/Σ|T|² with T = (Λu − v)/s. v, u: device, 2n. loss: host, may be NULL. */
pb_status pb_nn_train_step(pb_ctx* ctx, pb_nn* net, const pb_band* band, const pb_params* prm, const double* v,
                           const double* u, float lr, double* loss);
/* Host copies of the prepared neighbour lists (n × 16 int) and node features (n × 5 float:
   φ/ε, n, H·ε); either may be NULL. */
pb_status pb_nn_geometry(pb_ctx* ctx, const pb_band* band, int* nbr_host, float* feat_host);

/* Device time (ms) and launch count of one kernel family since the last reset, measured
   with HIP events around each launch on the context stream when timing is enabled.
   name: "p2p_f32", "p2p_f64", "tree_f32" (the treecode far field: proxies and k_tree_far),
   "tree_fine_f32" (the same for the fine residual treecode of PB_TREE solves on large bands),
   "near_f64", "reduce", "gmres", "levelset", "band", "rhs", "energy", "nn". pb_set_timing:
   enable = 0 off, 1 every family, 2 the far-field families only ("p2p_f32", "p2p_f64",
   "tree_f32", "tree_fine_f32"; each event pair adds a few microseconds
   between launches, so a timed run measures only what it reports). It synchronizes the
   context stream and resets the counters; other values give PB_EINVAL. The launches of a
   GMRES step enqueued after the solve's convergence test was met (they return at once)
   are not counted, so the counts equal the operator applications the solve reports. */
pb_status pb_set_timing(pb_ctx* ctx, int enable);
pb_status pb_kernel_time(pb_ctx* ctx, const char* name, double* total_ms, int64_t* launches);

/* The far-field kernel the mixed operator uses for bands of n nodes on this context (the
   autotuner's choice or PB_FAR_CFG; see pb_ibim_matvec): *cfg = 0..3 the one-directional
   kernel, 4 the symmetric one. PB_EINVAL if no mixed operator was applied to a band of that
   size yet. */
pb_status pb_far_kernel(pb_ctx* ctx, int64_t n, int* cfg);

/* Sizes of the treecode last prepared on this context (PB_TREE operator or solve), host
   array of 6: target batches, proxy clusters, proxy work items, target–source pairs of the
   direct lists (near pairs included, they contribute zero there), target–proxy
   interactions, and the FP64 near-field pairs. PB_EINVAL if none was prepared. */
pb_status pb_tree_info(pb_ctx* ctx, int64_t info[6]);

#ifdef __cplusplus
}
#endif
#endif
