/*
 * pbo.h — plain FP64 CPU oracle of the implicit boundary integral method (IBIM)
 * for the linearized Poisson–Boltzmann equation (Zhong, Ren, Tsai, arXiv:1709.08070).
 *
 * TEST INFRASTRUCTURE ONLY. This library exists to check the GPU library against
 * the paper. Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it; the product path never does. It shares no code with the GPU
 * library: its own layouts, its own parameter vector, its own loops.
 *
 * Layouts (all host memory, FP64):
 *   atoms : n × 5 rows (x, y, z, radius, charge), Å and e.
 *   grid  : dims[3] = (nx, ny, nz), origin[3], spacing h; node (i,j,k) sits at
 *           origin + h·(i,j,k) and has linear index (i·ny + j)·nz + k.
 *   nodes : band node table, n × 8 rows (x*, y*, z*, n_x, n_y, n_z, φ, ω), where
 *           x* is the closest-point projection, n the unit normal, φ the level-set
 *           value and ω = δ_ε(φ)·J (J ≡ 1 unless the explicit J is asked for). h³ is
 *           applied inside the sums.
 *   prm   : parameter vector, PBO_NPRM doubles, indices below.
 *   p     : 2n vector [ψ̄(nodes in band order); ψ̄_n(same order)].
 */
#ifndef PBO_ORACLE_H_
#define PBO_ORACLE_H_
#ifdef __cplusplus
extern "C" {
#endif

enum {
  PBO_EPS_IN = 0,   /* ε_I */
  PBO_EPS_OUT = 1,  /* ε_E */
  PBO_KAPPA = 2,    /* κ (Å⁻¹) */
  PBO_H = 3,        /* grid spacing h */
  PBO_BAND = 4,     /* band half-width ε */
  PBO_TAU = 5,      /* regularization radius τ */
  PBO_METRIC = 6,   /* 0 tangent-plane distance with r < 2τ guard, 1 tangent literal, 2 Euclidean */
  PBO_PROBE = 7,    /* probe radius ρ0 */
  PBO_CFL = 8,      /* Δt / h for level-set time stepping */
  PBO_REINIT = 9,   /* reinitialization steps (0 → 2·ceil((ε/h + 4)/cfl)) */
  PBO_AVG = 10,     /* disc averages of regularized pairs: 0 the paper's (0, K̄12, 0, 0), 1 curvature-corrected */
  PBO_NPRM = 11
};

/* Grid that covers the atoms with the given margin, nodes on hℤ³. */
void pbo_grid(const double* atoms, int n_atoms, double h, double margin, int* dims, double* origin);

/* Stage 1 — level set. */
void pbo_vdw(const int* dims, const double* origin, double h, const double* atoms, int n_atoms, double* phi);
void pbo_eikonal(const int* dims, double h, double* phi, double t_end, double cfl);
long pbo_cavity(const int* dims, double h, double* phi, double eps, unsigned char* outside);
void pbo_reinit(const int* dims, double h, double* phi, int steps, double cfl);
long pbo_ses(const int* dims, const double* origin, const double* atoms, int n_atoms, const double* prm, double* phi);
void pbo_weno_grad(const int* dims, double h, const double* phi, long node, double* minus3, double* plus3);

/* Stage 2 — band selection, projection, weights. Returns the node count;
   nodes/gidx may be NULL to count only. Returns -1 if a band node touches the grid edge.
   grad_scheme: 0 central differences, 1 WENO5 average (p₋ + p₊)/2. jacobian: 0 J ≡ 1,
   1 the explicit J (pbo_jacobian). */
long pbo_band(const int* dims, const double* origin, double h, const double* phi, double eps, int grad_scheme,
              int jacobian, double* nodes, long* gidx);
/* J = 1 − φΔφ + φ²⟨n, adj(∇²φ) n⟩ at an interior grid node with unit normal n (3 doubles). */
double pbo_jacobian(const int* dims, double h, const double* phi, long node, const double* n);
/* κ1 + κ2 of Γ at the node's projection (from the same Hessian). */
double pbo_curvature(const int* dims, double h, const double* phi, long node, const double* n);
double pbo_delta(double eta, double eps);

/* Stage 3 — kernels, operator, right-hand side, GMRES. curv: per node κ1 + κ2 at the
   projection (pbo_curvature), used by the curvature-corrected disc averages; NULL = 0. */
void pbo_pair(const double* x, const double* nx, const double* y, const double* ny, const double* prm, double curv,
              double* K);
void pbo_matvec(long n, const double* nodes, const double* prm, const double* curv, const double* p, double* y);
void pbo_matvec_rows(long n, const double* nodes, const double* prm, const double* curv, const double* p,
                     const long* rows, long n_rows, double* y1, double* y2);
void pbo_dense(long n, const double* nodes, const double* prm, const double* curv, double* A);
void pbo_rhs(long n, const double* nodes, const double* atoms, int n_atoms, const double* prm, double* g);
int pbo_gmres(long n, const double* nodes, const double* prm, const double* curv, const double* g, double* x,
              double tol, int max_iter, int restart, int* iters, double* relres);

/* Stage 4 — area and polarization energy (paper units, G0 = 1/(4πr)). */
double pbo_area(long n, const double* nodes, double h);
double pbo_energy(long n, const double* nodes, const double* atoms, int n_atoms, const double* prm,
                  const double* p, double* psi_rxn);

#ifdef __cplusplus
}
#endif
#endif
