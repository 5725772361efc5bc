/*
 * pbo.c — plain FP64 CPU oracle of the implicit boundary integral method (IBIM)
 * for the linearized Poisson–Boltzmann equation (Zhong, Ren, Tsai, arXiv:1709.08070).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU-baseline
 * leg of the benchmark, never by the product path. It shares no code with the GPU
 * library. Every routine is a direct loop over the definition it cites; OpenMP only
 * splits independent target rows (each row's sum runs in plain j order).
 *
 * Built with -ffp-contract=off so that every product and sum is rounded as written.
 *
 * Pins (see tests/test_oracle_*.py): kernel values against high-precision finite
 * differences of G0 and Gκ; kernel symmetries; ∫δ_ε = 1 and its second moment;
 * lattice node counts by brute force; the band area of a sphere; Gauss's lemma;
 * the continuum l = 0 operator identities on a sphere; the Kirkwood solvation
 * energy (closed form of the single-ion section) with a first-order error that
 * decreases with h; GMRES against dense LU; the single-atom level set against the
 * exact distance; two-atom SES signs against a brute-force probe rolling; a closed
 * cavity removed.
 */
#include "pbo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

static double sq(double a) { return a * a; }
static long lin(const int* d, long i, long j, long k) { return (i * d[1] + j) * d[2] + k; }

/* ------------------------------------------------------------------ grid */

void pbo_grid(const double* atoms, int n_atoms, double h, double margin, int* dims, double* origin) {
  for (int a = 0; a < 3; ++a) {
    double lo = atoms[a], hi = atoms[a];
    for (int k = 1; k < n_atoms; ++k) {
      if (atoms[5 * k + a] < lo) lo = atoms[5 * k + a];
      if (atoms[5 * k + a] > hi) hi = atoms[5 * k + a];
    }
    long ilo = (long)floor((lo - margin) / h);
    long ihi = (long)ceil((hi + margin) / h);
    origin[a] = (double)ilo * h;
    dims[a] = (int)(ihi - ilo + 1);
  }
}

/* ---------------------------------------------------- Stage 1: level set */

/* van der Waals level set F(x) = min_k (|x − z_k| − r_k) (section "Creating a
   signed distance function to the solvent accessible surface", eq. vdW-levelset-fn). */
void pbo_vdw(const int* dims, const double* origin, double h, const double* atoms, int n_atoms, double* phi) {
#pragma omp parallel for schedule(static)
  for (long i = 0; i < dims[0]; ++i)
    for (long j = 0; j < dims[1]; ++j)
      for (long k = 0; k < dims[2]; ++k) {
        double x = origin[0] + h * (double)i, y = origin[1] + h * (double)j, z = origin[2] + h * (double)k;
        double best = INFINITY;
        for (int a = 0; a < n_atoms; ++a) {
          const double* at = atoms + 5 * a;
          double dist = sqrt((sq(x - at[0]) + sq(y - at[1])) + sq(z - at[2])) - at[3];
          if (dist < best) best = dist;
        }
        phi[lin(dims, i, j, k)] = best;
      }
}

/* Zero-Neumann boundary by even reflection about the boundary node: index −m ↦ m,
   n−1+m ↦ n−1−m (reading of "zero Neumann boundary conditions" for the eikonal flow). */
static long refl(long i, long n) {
  if (i < 0) return -i;
  if (i > n - 1) return 2 * (n - 1) - i;
  return i;
}

/* Fifth-order WENO one-sided derivative (Jiang & Peng) from five consecutive first
   differences v1..v5, ordered from the far upwind side towards the node. */
static double weno5(double v1, double v2, double v3, double v4, double v5) {
  const double e = 1e-6;
  double s1 = 13.0 / 12.0 * sq(v1 - 2.0 * v2 + v3) + 0.25 * sq(v1 - 4.0 * v2 + 3.0 * v3);
  double s2 = 13.0 / 12.0 * sq(v2 - 2.0 * v3 + v4) + 0.25 * sq(v2 - v4);
  double s3 = 13.0 / 12.0 * sq(v3 - 2.0 * v4 + v5) + 0.25 * sq(3.0 * v3 - 4.0 * v4 + v5);
  double a1 = 0.1 / sq(s1 + e), a2 = 0.6 / sq(s2 + e), a3 = 0.3 / sq(s3 + e);
  double p1 = v1 / 3.0 - 7.0 * v2 / 6.0 + 11.0 * v3 / 6.0;
  double p2 = -v2 / 6.0 + 5.0 * v3 / 6.0 + v4 / 3.0;
  double p3 = v3 / 3.0 + 5.0 * v4 / 6.0 - v5 / 6.0;
  return (a1 * p1 + a2 * p2 + a3 * p3) / (a1 + a2 + a3);
}

/* phi value at (i,j,k) shifted by s along axis ax, with reflected ghosts. */
static double at_shift(const int* d, const double* phi, long i, long j, long k, int ax, long s) {
  if (ax == 0) i = refl(i + s, d[0]);
  else if (ax == 1) j = refl(j + s, d[1]);
  else k = refl(k + s, d[2]);
  return phi[lin(d, i, j, k)];
}

/* Backward (dm) and forward (dp) WENO5 derivatives along one axis. */
static void weno_axis(const int* d, const double* phi, double h, long i, long j, long k, int ax,
                      double* dm, double* dp) {
  double f[7];
  for (long s = -3; s <= 3; ++s) f[s + 3] = at_shift(d, phi, i, j, k, ax, s);
  /* f[m] is phi at offset m−3; D[m] = (f[m+1] − f[m]) / h is the difference between offsets m−3 and m−2. */
  double D[6];
  for (int m = 0; m < 6; ++m) D[m] = (f[m + 1] - f[m]) / h;
  *dm = weno5(D[0], D[1], D[2], D[3], D[4]);
  *dp = weno5(D[5], D[4], D[3], D[2], D[1]);
}

void pbo_weno_grad(const int* dims, double h, const double* phi, long node, double* minus3, double* plus3) {
  long k = node % dims[2], j = (node / dims[2]) % dims[1], i = node / ((long)dims[1] * dims[2]);
  for (int ax = 0; ax < 3; ++ax) weno_axis(dims, phi, h, i, j, k, ax, minus3 + ax, plus3 + ax);
}

/* Godunov approximation of |∇φ| for the Hamiltonian s·|∇φ| (Rouy–Tourin form):
   s ≥ 0 takes max(a⁺², b⁻²), s < 0 takes max(a⁻², b⁺²) per axis, with a the
   backward and b the forward WENO derivative. */
static double godunov_norm(const int* d, const double* phi, double h, long i, long j, long k, double s) {
  double g = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    double a, b;
    weno_axis(d, phi, h, i, j, k, ax, &a, &b);
    if (s >= 0.0) g += fmax(sq(fmax(a, 0.0)), sq(fmin(b, 0.0)));
    else g += fmax(sq(fmin(a, 0.0)), sq(fmax(b, 0.0)));
  }
  return sqrt(g);
}

/* Right-hand side L(φ) of φ_t = L(φ).
   mode 0: inward eikonal flow φ_t − |∇φ| = 0, i.e. L = |∇φ| with Hamiltonian −|∇φ|.
   mode 1: reinitialization φ_t + S(|∇φ| − 1) = 0 with frozen S = sgn_h(φ_0). */
static void ls_rhs(const int* d, double h, const double* phi, const double* S, int mode, double* L) {
#pragma omp parallel for schedule(static)
  for (long i = 0; i < d[0]; ++i)
    for (long j = 0; j < d[1]; ++j)
      for (long k = 0; k < d[2]; ++k) {
        long id = lin(d, i, j, k);
        if (mode == 0) {
          L[id] = godunov_norm(d, phi, h, i, j, k, -1.0);
        } else {
          double s = S[id];
          L[id] = -s * (godunov_norm(d, phi, h, i, j, k, s) - 1.0);
        }
      }
}

/* Third-order TVD Runge–Kutta (Shu–Osher) for φ_t = L(φ), nsteps of size dt. */
static void tvd_rk3(const int* d, double h, double* phi, const double* S, int mode, int nsteps, double dt) {
  long n = (long)d[0] * d[1] * d[2];
  double* p1 = malloc(sizeof(double) * n);
  double* p2 = malloc(sizeof(double) * n);
  double* L = malloc(sizeof(double) * n);
  for (int step = 0; step < nsteps; ++step) {
    ls_rhs(d, h, phi, S, mode, L);
    for (long q = 0; q < n; ++q) p1[q] = phi[q] + dt * L[q];
    ls_rhs(d, h, p1, S, mode, L);
    for (long q = 0; q < n; ++q) p2[q] = 0.75 * phi[q] + 0.25 * (p1[q] + dt * L[q]);
    ls_rhs(d, h, p2, S, mode, L);
    for (long q = 0; q < n; ++q) phi[q] = phi[q] / 3.0 + (2.0 / 3.0) * (p2[q] + dt * L[q]);
  }
  free(p1);
  free(p2);
  free(L);
}

/* Inward eikonal flow to t = t_end in equal steps no longer than cfl·h. */
void pbo_eikonal(const int* dims, double h, double* phi, double t_end, double cfl) {
  int nsteps = (int)ceil(t_end / (cfl * h) - 1e-9);
  if (nsteps < 1) return;
  tvd_rk3(dims, h, phi, NULL, 0, nsteps, t_end / nsteps);
}

/* Cavity removal ("Cavities removal" subsection): breadth-first search from the grid
   boundary through the 6-connected nodes with φ > 0 marks the exterior solvent. The
   unreached nodes with φ > 0 are cavities; every unreached node within ε + h of a
   cavity node forms C_ε and gets φ = −ε. Returns the number of nodes set.
   outside (optional) receives 1 for reached nodes. */
long pbo_cavity(const int* dims, double h, double* phi, double eps, unsigned char* outside) {
  long nx = dims[0], ny = dims[1], nz = dims[2], n = nx * ny * nz;
  unsigned char* seen = calloc((size_t)n, 1);
  long* queue = malloc(sizeof(long) * n);
  long head = 0, tail = 0;
  for (long i = 0; i < nx; ++i)
    for (long j = 0; j < ny; ++j)
      for (long k = 0; k < nz; ++k) {
        if (!(i == 0 || j == 0 || k == 0 || i == nx - 1 || j == ny - 1 || k == nz - 1)) continue;
        long id = lin(dims, i, j, k);
        if (phi[id] > 0.0 && !seen[id]) { seen[id] = 1; queue[tail++] = id; }
      }
  while (head < tail) {
    long id = queue[head++];
    long k = id % nz, j = (id / nz) % ny, i = id / (ny * nz);
    long nb[6][3] = {{i - 1, j, k}, {i + 1, j, k}, {i, j - 1, k}, {i, j + 1, k}, {i, j, k - 1}, {i, j, k + 1}};
    for (int q = 0; q < 6; ++q) {
      long a = nb[q][0], b = nb[q][1], c = nb[q][2];
      if (a < 0 || b < 0 || c < 0 || a >= nx || b >= ny || c >= nz) continue;
      long t = lin(dims, a, b, c);
      if (!seen[t] && phi[t] > 0.0) { seen[t] = 1; queue[tail++] = t; }
    }
  }
  /* Dilate the cavity set by ε + h (Euclidean, on the lattice), never into the exterior. */
  double rr = (eps + h) / h;
  double rr2 = rr * rr;
  long m = (long)floor(rr);
  unsigned char* cav = calloc((size_t)n, 1);
  for (long id = 0; id < n; ++id) cav[id] = (!seen[id] && phi[id] > 0.0);
  long changed = 0;
  double* out = malloc(sizeof(double) * n);
  memcpy(out, phi, sizeof(double) * n);
  for (long i = 0; i < nx; ++i)
    for (long j = 0; j < ny; ++j)
      for (long k = 0; k < nz; ++k) {
        long id = lin(dims, i, j, k);
        if (seen[id]) continue;
        int hit = cav[id];
        for (long a = -m; a <= m && !hit; ++a)
          for (long b = -m; b <= m && !hit; ++b)
            for (long c = -m; c <= m && !hit; ++c) {
              if ((double)(a * a + b * b + c * c) > rr2) continue;
              long ii = i + a, jj = j + b, kk = k + c;
              if (ii < 0 || jj < 0 || kk < 0 || ii >= nx || jj >= ny || kk >= nz) continue;
              if (cav[lin(dims, ii, jj, kk)]) hit = 1;
            }
        if (hit) { out[id] = -eps; ++changed; }
      }
  memcpy(phi, out, sizeof(double) * n);
  if (outside) memcpy(outside, seen, (size_t)n);
  free(out);
  free(cav);
  free(queue);
  free(seen);
  return changed;
}

/* Reinitialization φ_t + sgn_h(φ_0)(|∇φ| − 1) = 0, sgn_h(φ) = φ/√(φ² + h²)
   (eqs. reinit and signum), Δt = cfl·h. */
void pbo_reinit(const int* dims, double h, double* phi, int steps, double cfl) {
  long n = (long)dims[0] * dims[1] * dims[2];
  double* S = malloc(sizeof(double) * n);
  for (long q = 0; q < n; ++q) S[q] = phi[q] / sqrt(phi[q] * phi[q] + h * h);
  tvd_rk3(dims, h, phi, S, 1, steps, cfl * h);
  free(S);
}

/* Whole Stage 1: F − ρ0, eikonal flow to t = ρ0, cavity removal, reinitialization.
   Returns the number of nodes set by cavity removal. */
long pbo_ses(const int* dims, const double* origin, const double* atoms, int n_atoms, const double* prm, double* phi) {
  double h = prm[PBO_H], rho = prm[PBO_PROBE], cfl = prm[PBO_CFL], eps = prm[PBO_BAND];
  long n = (long)dims[0] * dims[1] * dims[2];
  pbo_vdw(dims, origin, h, atoms, n_atoms, phi);
  for (long q = 0; q < n; ++q) phi[q] -= rho;
  pbo_eikonal(dims, h, phi, rho, cfl);
  long cav = pbo_cavity(dims, h, phi, eps, NULL);
  int steps = (int)prm[PBO_REINIT];
  if (steps <= 0) steps = 2 * (int)ceil((eps / h + 4.0) / cfl - 1e-9);
  pbo_reinit(dims, h, phi, steps, cfl);
  return cav;
}

/* ------------------------------------- Stage 2: band, projection, weights */

/* Cosine weight δ_ε(η) = (1 + cos(πη/ε)) / (2ε) on |η| < ε, 0 otherwise (eq. cosine-kernel). */
double pbo_delta(double eta, double eps) {
  if (fabs(eta) >= eps) return 0.0;
  return (1.0 + cos(PI * eta / eps)) / (2.0 * eps);
}

/* Jacobian between Γ and the level set of φ through node (i,j,k) (section "Implicit
   boundary integral methods", the explicit J):
     J = 1 − φ Δφ + φ² ⟨n, adj(∇²φ) n⟩,
   with the Hessian ∇²φ by second-order central differences (the mixed derivatives from the
   four diagonal neighbours), adj its adjugate (transposed cofactor matrix) and n the unit
   normal of the node. Reading: the printed last term has the Hessian itself, which vanishes
   on ∇φ for a distance function; with the adjugate, J = (1 − φκ1)(1 − φκ2) for the principal
   curvatures κ1, κ2 of the level set through the node, the area ratio of the projection. */
static void hessian_terms(const int* dims, double h, const double* phi, long node, const double* n, double* trace,
                          double* q_adj) {
  long k = node % dims[2], j = (node / dims[2]) % dims[1], i = node / ((long)dims[1] * dims[2]);
  double c = phi[node], h2 = h * h;
  double H[3][3];
  H[0][0] = (phi[lin(dims, i + 1, j, k)] - 2.0 * c + phi[lin(dims, i - 1, j, k)]) / h2;
  H[1][1] = (phi[lin(dims, i, j + 1, k)] - 2.0 * c + phi[lin(dims, i, j - 1, k)]) / h2;
  H[2][2] = (phi[lin(dims, i, j, k + 1)] - 2.0 * c + phi[lin(dims, i, j, k - 1)]) / h2;
  H[0][1] = H[1][0] = (phi[lin(dims, i + 1, j + 1, k)] - phi[lin(dims, i + 1, j - 1, k)] -
                       phi[lin(dims, i - 1, j + 1, k)] + phi[lin(dims, i - 1, j - 1, k)]) / (4.0 * h2);
  H[0][2] = H[2][0] = (phi[lin(dims, i + 1, j, k + 1)] - phi[lin(dims, i + 1, j, k - 1)] -
                       phi[lin(dims, i - 1, j, k + 1)] + phi[lin(dims, i - 1, j, k - 1)]) / (4.0 * h2);
  H[1][2] = H[2][1] = (phi[lin(dims, i, j + 1, k + 1)] - phi[lin(dims, i, j + 1, k - 1)] -
                       phi[lin(dims, i, j - 1, k + 1)] + phi[lin(dims, i, j - 1, k - 1)]) / (4.0 * h2);
  /* adj(H)[a][b] = cofactor of H[b][a]: the signed 2×2 minor left after deleting row b, column a */
  double A[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      int r0 = (b + 1) % 3, r1 = (b + 2) % 3, c0 = (a + 1) % 3, c1 = (a + 2) % 3;
      A[a][b] = H[r0][c0] * H[r1][c1] - H[r0][c1] * H[r1][c0];
    }
  double q = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) q += n[a] * A[a][b] * n[b];
  *trace = H[0][0] + H[1][1] + H[2][2];
  *q_adj = q;
}

double pbo_jacobian(const int* dims, double h, const double* phi, long node, const double* n) {
  double tr, q, c = phi[node];
  hessian_terms(dims, h, phi, node, n, &tr, &q);
  return 1.0 - c * tr + c * c * q;
}

/* Sum of the principal curvatures of Γ at the projection x* of node (κ1 + κ2 > 0 on a convex
   surface with outward normals). The level set of φ through the node has curvatures k1, k2 with
   k1 + k2 = Δφ and k1·k2 = ⟨n, adj(∇²φ) n⟩; moving a distance φ back along the normal gives
   κ = k/(1 − φk) for each, so κ1 + κ2 = (k1 + k2 − 2φ k1k2)/J with the J above. */
double pbo_curvature(const int* dims, double h, const double* phi, long node, const double* n) {
  double tr, q, c = phi[node];
  hessian_terms(dims, h, phi, node, n, &tr, &q);
  return (tr - 2.0 * c * q) / (1.0 - c * tr + c * c * q);
}

/* Nodes with −ε < φ < ε in lexicographic order ("Projections and weights"):
   ∇φ by central differences (grad_scheme 0) or the average (p₋ + p₊)/2 of the two WENO5
   one-sided derivatives per axis (grad_scheme 1); n = ∇φ/|∇φ|; x* = x − φ n;
   ω = δ_ε(φ)·J with J ≡ 1 (jacobian 0, the paper's experiments) or the explicit J of
   pbo_jacobian (jacobian 1). */
long pbo_band(const int* dims, const double* origin, double h, const double* phi, double eps, int grad_scheme,
              int jacobian, double* nodes, long* gidx) {
  long cnt = 0;
  for (long i = 0; i < dims[0]; ++i)
    for (long j = 0; j < dims[1]; ++j)
      for (long k = 0; k < dims[2]; ++k) {
        long id = lin(dims, i, j, k);
        double f = phi[id];
        if (!(f > -eps && f < eps)) continue;
        if (i == 0 || j == 0 || k == 0 || i == dims[0] - 1 || j == dims[1] - 1 || k == dims[2] - 1) return -1;
        if (nodes) {
          double g[3];
          if (grad_scheme == 1) {
            double m[3], p[3];
            pbo_weno_grad(dims, h, phi, id, m, p);
            for (int a = 0; a < 3; ++a) g[a] = (m[a] + p[a]) / 2.0;
          } else {
            g[0] = (phi[lin(dims, i + 1, j, k)] - phi[lin(dims, i - 1, j, k)]) / (2.0 * h);
            g[1] = (phi[lin(dims, i, j + 1, k)] - phi[lin(dims, i, j - 1, k)]) / (2.0 * h);
            g[2] = (phi[lin(dims, i, j, k + 1)] - phi[lin(dims, i, j, k - 1)]) / (2.0 * h);
          }
          double gn = sqrt((g[0] * g[0] + g[1] * g[1]) + g[2] * g[2]);
          double nv[3] = {g[0] / gn, g[1] / gn, g[2] / gn};
          double* o = nodes + 8 * cnt;
          o[0] = origin[0] + h * (double)i - f * nv[0];
          o[1] = origin[1] + h * (double)j - f * nv[1];
          o[2] = origin[2] + h * (double)k - f * nv[2];
          o[3] = nv[0];
          o[4] = nv[1];
          o[5] = nv[2];
          o[6] = f;
          o[7] = pbo_delta(f, eps);
          if (jacobian) o[7] *= pbo_jacobian(dims, h, phi, id, nv);
        }
        if (gidx) gidx[cnt] = id;
        ++cnt;
      }
  return cnt;
}

/* ---------------------------------- Stage 3: kernels, operator, GMRES */

/* Is the pair regularized? t² = r² − (d·n_x)² is the squared distance between the
   projections of x* and y* on the tangent plane at x* (eq. reg-kernel). */
static int regularized(double r2, double t2, double tau, int metric) {
  if (metric == 2) return r2 < tau * tau;
  if (metric == 1) return t2 < tau * tau;
  return t2 < tau * tau && r2 < 4.0 * tau * tau;
}

/* Disc average of G0 − Gκ over radius τ (eq. reg-kernel-a). */
static double k12_bar(double kappa, double tau) {
  if (kappa == 0.0) return 0.0;
  return (exp(-kappa * tau) - 1.0 + kappa * tau) / (2.0 * PI * kappa * tau * tau);
}

/* Disc averages of K11, K21, K22 over the regularization disc of radius τ at x*, whose
   surface has curvature sum curv = κ1 + κ2 there. avg = 0 is the paper's choice, all three 0.
   avg = 1 keeps the leading term of each (reading of the paper's remark that the
   regularization can be improved):
   - on the surface, in tangent coordinates (u, v) of y about x, (x − y)·n_y = −½(κ1u² + κ2v²)
     and (x − y)·n_x = +½(κ1u² + κ2v²) to second order, so K11 = −(κ1u² + κ2v²)(1 − θ1a)/(8πr³)
     and K22 = −(κ1u² + κ2v²)(1 − θ2a)/(8πr³); over the disc the angular mean of κ1u² + κ2v²
     is ½(κ1 + κ2)r², which gives the integrals −(κ1 + κ2)τ(1 − θ ā)/8, ā = (1/τ)∫₀^τ a dr
     = (2 − (2 + κτ)e^{−κτ})/(κτ) (1 at κ = 0), and the averages (÷ πτ²)
       K̄11 = −(1 − θ1ā)·curv/(8πτ),   K̄22 = −(1 − θ2ā)·curv/(8πτ);
   - K21 on the flat disc (n_x = n_y, d·n = 0) is (1 − e^{−κr}(1 + κr))/(4πr³), the
     r-derivative of (e^{−κr} − 1)/r over 4πr: its integral is (e^{−κτ} − 1 + κτ)/(2τ) and
       K̄21 = (e^{−κτ} − 1 + κτ)/(2πτ³). */
static void disc_averages(const double* prm, double curv, double* K) {
  double kappa = prm[PBO_KAPPA], tau = prm[PBO_TAU];
  double th1 = prm[PBO_EPS_OUT] / prm[PBO_EPS_IN], th2 = prm[PBO_EPS_IN] / prm[PBO_EPS_OUT];
  K[1] = k12_bar(kappa, tau);
  if ((int)prm[PBO_AVG] == 0) {
    K[0] = K[2] = K[3] = 0.0;
    return;
  }
  double kt = kappa * tau;
  double abar = kappa == 0.0 ? 1.0 : (2.0 - (2.0 + kt) * exp(-kt)) / kt;
  K[0] = -(1.0 - th1 * abar) * curv / (8.0 * PI * tau);
  K[2] = (exp(-kt) - 1.0 + kt) / (2.0 * PI * tau * tau * tau);
  K[3] = -(1.0 - th2 * abar) * curv / (8.0 * PI * tau);
}

/* The four regularized kernels between target x (normal nx) and source y (normal ny)
   (eq. IBIM-PBE and the regularization subsection):
     K11 = ∂G0/∂n(y) − θ1 ∂Gκ/∂n(y),  θ1 = ε_E/ε_I
     K12 = G0 − Gκ
     K21 = ∂²G0/∂n(x)∂n(y) − ∂²Gκ/∂n(x)∂n(y)
     K22 = ∂G0/∂n(x) − θ2 ∂Gκ/∂n(x),  θ2 = ε_I/ε_E
   with G0 = 1/(4πr), Gκ = e^{−κr}/(4πr). Written out for d = x − y, r = |d|, E = e^{−κr}:
     ∂G0/∂n(y) = (d·n_y)/(4πr³),      ∂Gκ/∂n(y) = E(1+κr)(d·n_y)/(4πr³)
     ∂G0/∂n(x) = −(d·n_x)/(4πr³),     ∂Gκ/∂n(x) = −E(1+κr)(d·n_x)/(4πr³)
     ∂²G0/∂n(x)∂n(y) = (n_x·n_y)/(4πr³) − 3(d·n_x)(d·n_y)/(4πr⁵)
     ∂²Gκ/∂n(x)∂n(y) = E(1+κr)(n_x·n_y)/(4πr³) − E(3+3κr+κ²r²)(d·n_x)(d·n_y)/(4πr⁵)
   Regularized pairs take the disc averages (disc_averages; curv: κ1 + κ2 at x). */
void pbo_pair(const double* x, const double* nx, const double* y, const double* ny, const double* prm, double curv,
              double* K) {
  double th1 = prm[PBO_EPS_OUT] / prm[PBO_EPS_IN], th2 = prm[PBO_EPS_IN] / prm[PBO_EPS_OUT];
  double kappa = prm[PBO_KAPPA], tau = prm[PBO_TAU];
  double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
  double r2 = (dx * dx + dy * dy) + dz * dz;
  double dnx = (dx * nx[0] + dy * nx[1]) + dz * nx[2];
  double t2 = r2 - dnx * dnx;
  if (regularized(r2, t2, tau, (int)prm[PBO_METRIC])) {
    disc_averages(prm, curv, K);
    return;
  }
  double dny = (dx * ny[0] + dy * ny[1]) + dz * ny[2];
  double nn = (nx[0] * ny[0] + nx[1] * ny[1]) + nx[2] * ny[2];
  double r = sqrt(r2);
  double E = exp(-kappa * r);
  double a = E * (1.0 + kappa * r);
  double b = E * (3.0 + 3.0 * kappa * r + kappa * kappa * r2);
  double c = 1.0 / (4.0 * PI);
  double dG0_ny = c * dny / (r2 * r), dGk_ny = c * a * dny / (r2 * r);
  double dG0_nx = -c * dnx / (r2 * r), dGk_nx = -c * a * dnx / (r2 * r);
  double d2G0 = c * nn / (r2 * r) - 3.0 * c * dnx * dny / (r2 * r2 * r);
  double d2Gk = c * a * nn / (r2 * r) - c * b * dnx * dny / (r2 * r2 * r);
  K[0] = dG0_ny - th1 * dGk_ny;
  K[1] = c / r - c * E / r;
  K[2] = d2G0 - d2Gk;
  K[3] = dG0_nx - th2 * dGk_nx;
}

/* One row of Λp + KWp (eq. final-lin-sys): Λ = diag(½(1+ε_E/ε_I), ½(1+ε_I/ε_E)),
   W = diag(ω) and the sums carry h³ (eq. IBIM-PBE). */
static void row(long n, const double* nodes, const double* prm, const double* curv, const double* p, long i, double* y1,
                double* y2) {
  double h3 = prm[PBO_H] * prm[PBO_H] * prm[PBO_H];
  double lam1 = 0.5 * (1.0 + prm[PBO_EPS_OUT] / prm[PBO_EPS_IN]);
  double lam2 = 0.5 * (1.0 + prm[PBO_EPS_IN] / prm[PBO_EPS_OUT]);
  const double* xi = nodes + 8 * i;
  double s1 = 0.0, s2 = 0.0, K[4];
  for (long j = 0; j < n; ++j) {
    const double* yj = nodes + 8 * j;
    pbo_pair(xi, xi + 3, yj, yj + 3, prm, curv ? curv[i] : 0.0, K);
    double wpsi = h3 * yj[7] * p[j], wpsn = h3 * yj[7] * p[n + j];
    s1 += K[0] * wpsi - K[1] * wpsn;
    s2 += K[2] * wpsi - K[3] * wpsn;
  }
  *y1 = lam1 * p[i] + s1;
  *y2 = lam2 * p[n + i] + s2;
}

void pbo_matvec(long n, const double* nodes, const double* prm, const double* curv, const double* p, double* y) {
#pragma omp parallel for schedule(dynamic, 16)
  for (long i = 0; i < n; ++i) row(n, nodes, prm, curv, p, i, y + i, y + n + i);
}

void pbo_matvec_rows(long n, const double* nodes, const double* prm, const double* curv, const double* p,
                     const long* rows, long n_rows, double* y1, double* y2) {
#pragma omp parallel for schedule(dynamic, 4)
  for (long q = 0; q < n_rows; ++q) row(n, nodes, prm, curv, p, rows[q], y1 + q, y2 + q);
}

/* Dense 2n × 2n matrix Λ + KW, row-major. */
void pbo_dense(long n, const double* nodes, const double* prm, const double* curv, double* A) {
  double h3 = prm[PBO_H] * prm[PBO_H] * prm[PBO_H];
  double lam1 = 0.5 * (1.0 + prm[PBO_EPS_OUT] / prm[PBO_EPS_IN]);
  double lam2 = 0.5 * (1.0 + prm[PBO_EPS_IN] / prm[PBO_EPS_OUT]);
  long m = 2 * n;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < n; ++i) {
    const double* xi = nodes + 8 * i;
    double K[4];
    for (long j = 0; j < n; ++j) {
      const double* yj = nodes + 8 * j;
      pbo_pair(xi, xi + 3, yj, yj + 3, prm, curv ? curv[i] : 0.0, K);
      double w = h3 * yj[7];
      A[i * m + j] = K[0] * w;
      A[i * m + n + j] = -K[1] * w;
      A[(n + i) * m + j] = K[2] * w;
      A[(n + i) * m + n + j] = -K[3] * w;
    }
    A[i * m + i] += lam1;
    A[(n + i) * m + n + i] += lam2;
  }
}

/* Right-hand side at the projections x_i*: g1 = Σ_k q_k/ε_I G0(x*, z_k),
   g2 = Σ_k q_k/ε_I ∂G0(x*, z_k)/∂n(x*) with ∂G0/∂n(x) = −(x−z)·n/(4π|x−z|³). */
void pbo_rhs(long n, const double* nodes, const double* atoms, int n_atoms, const double* prm, double* g) {
  double epsi = prm[PBO_EPS_IN];
#pragma omp parallel for schedule(static)
  for (long i = 0; i < n; ++i) {
    const double* x = nodes + 8 * i;
    double s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < n_atoms; ++k) {
      const double* z = atoms + 5 * k;
      double dx = x[0] - z[0], dy = x[1] - z[1], dz = x[2] - z[2];
      double rho = sqrt((dx * dx + dy * dy) + dz * dz);
      double dn = (dx * x[3] + dy * x[4]) + dz * x[5];
      s1 += z[4] / epsi / (4.0 * PI * rho);
      s2 += z[4] / epsi * (-dn / (4.0 * PI * rho * rho * rho));
    }
    g[i] = s1;
    g[n + i] = s2;
  }
}

static double dot(long m, const double* a, const double* b) {
  double s = 0.0;
  for (long q = 0; q < m; ++q) s += a[q] * b[q];
  return s;
}

/* Restarted GMRES (Saad–Schultz) with modified Gram–Schmidt and Givens rotations,
   stopping when ‖g − Ax‖₂/‖g‖₂ ≤ tol (section "Fast linear solvers"). x holds the
   initial guess on entry. iters counts operator applications inside Arnoldi; relres
   is the true relative residual at exit. Returns 1 if converged. */
int pbo_gmres(long n, const double* nodes, const double* prm, const double* curv, const double* g, double* x,
              double tol, int max_iter, int restart, int* iters, double* relres) {
  long m2 = 2 * n;
  int mr = restart;
  double* V = malloc(sizeof(double) * m2 * (size_t)(mr + 1));
  double* H = calloc((size_t)(mr + 1) * mr, sizeof(double));
  double* cs = malloc(sizeof(double) * mr);
  double* sn = malloc(sizeof(double) * mr);
  double* s = malloc(sizeof(double) * (mr + 1));
  double* yv = malloc(sizeof(double) * mr);
  double* r = malloc(sizeof(double) * m2);
  double gnorm = sqrt(dot(m2, g, g));
  int it = 0, converged = 0;
  if (gnorm == 0.0) gnorm = 1.0;
  while (!converged) {
    pbo_matvec(n, nodes, prm, curv, x, r);
    for (long q = 0; q < m2; ++q) r[q] = g[q] - r[q];
    double beta = sqrt(dot(m2, r, r));
    if (beta / gnorm <= tol) { converged = 1; break; }
    if (it >= max_iter) break;
    for (long q = 0; q < m2; ++q) V[q] = r[q] / beta;
    memset(s, 0, sizeof(double) * (mr + 1));
    s[0] = beta;
    int k = 0;
    for (; k < mr && it < max_iter; ++k) {
      double* w = V + (size_t)(k + 1) * m2;
      pbo_matvec(n, nodes, prm, curv, V + (size_t)k * m2, w);
      ++it;
      for (int i = 0; i <= k; ++i) {
        double hik = dot(m2, w, V + (size_t)i * m2);
        H[i * mr + k] = hik;
        for (long q = 0; q < m2; ++q) w[q] -= hik * V[(size_t)i * m2 + q];
      }
      double hn = sqrt(dot(m2, w, w));
      H[(k + 1) * mr + k] = hn;
      if (hn > 0.0)
        for (long q = 0; q < m2; ++q) w[q] /= hn;
      for (int i = 0; i < k; ++i) {
        double a = H[i * mr + k], b = H[(i + 1) * mr + k];
        H[i * mr + k] = cs[i] * a + sn[i] * b;
        H[(i + 1) * mr + k] = -sn[i] * a + cs[i] * b;
      }
      double a = H[k * mr + k], b = H[(k + 1) * mr + k];
      double den = sqrt(a * a + b * b);
      cs[k] = a / den;
      sn[k] = b / den;
      H[k * mr + k] = den;
      H[(k + 1) * mr + k] = 0.0;
      s[k + 1] = -sn[k] * s[k];
      s[k] = cs[k] * s[k];
      if (fabs(s[k + 1]) / gnorm <= tol || hn == 0.0) { ++k; break; }
    }
    for (int i = k - 1; i >= 0; --i) {
      double acc = s[i];
      for (int j = i + 1; j < k; ++j) acc -= H[i * mr + j] * yv[j];
      yv[i] = acc / H[i * mr + i];
    }
    for (int i = 0; i < k; ++i)
      for (long q = 0; q < m2; ++q) x[q] += yv[i] * V[(size_t)i * m2 + q];
  }
  pbo_matvec(n, nodes, prm, curv, x, r);
  for (long q = 0; q < m2; ++q) r[q] = g[q] - r[q];
  double rr = sqrt(dot(m2, r, r)) / gnorm;
  *relres = rr;
  *iters = it;
  free(V); free(H); free(cs); free(sn); free(s); free(yv); free(r);
  return rr <= tol;
}

/* ------------------------------------------- Stage 4: area and energy */

/* Surface area S_h[1] = h³ Σ ω_j ("Computing surface area", eq. IBIM sum with f ≡ 1). */
double pbo_area(long n, const double* nodes, double h) {
  double s = 0.0;
  for (long j = 0; j < n; ++j) s += nodes[8 * j + 7];
  return h * h * h * s;
}

/* Polarization energy G_pol = ½ Σ_k q_k ψ_rxn(z_k) (eq. G pol), ψ_rxn by the IBIM sum of
     (θ1 ∂Gκ(z,y)/∂n(y) − ∂G0(z,y)/∂n(y)) ψ̄ + (G0(z,y) − Gκ(z,y)) ψ̄_n
   at the projections y*. With ρ = |z − y*| and s = (z − y*)·n_y:
     ∂G0/∂n(y) = s/(4πρ³), ∂Gκ/∂n(y) = e^{−κρ}(1+κρ) s/(4πρ³). */
double pbo_energy(long n, const double* nodes, const double* atoms, int n_atoms, const double* prm,
                  const double* p, double* psi_rxn) {
  double th1 = prm[PBO_EPS_OUT] / prm[PBO_EPS_IN], kappa = prm[PBO_KAPPA];
  double h3 = prm[PBO_H] * prm[PBO_H] * prm[PBO_H];
  double c = 1.0 / (4.0 * PI);
  double* psi = malloc(sizeof(double) * (size_t)n_atoms);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < n_atoms; ++k) {
    const double* z = atoms + 5 * k;
    double acc = 0.0;
    for (long j = 0; j < n; ++j) {
      const double* y = nodes + 8 * j;
      double dx = z[0] - y[0], dy = z[1] - y[1], dz = z[2] - y[2];
      double rho = sqrt((dx * dx + dy * dy) + dz * dz);
      double sdn = (dx * y[3] + dy * y[4]) + dz * y[5];
      double E = exp(-kappa * rho);
      double dG0 = c * sdn / (rho * rho * rho);
      double dGk = c * E * (1.0 + kappa * rho) * sdn / (rho * rho * rho);
      double G0mGk = c / rho - c * E / rho;
      acc += h3 * y[7] * ((th1 * dGk - dG0) * p[j] + G0mGk * p[n + j]);
    }
    psi[k] = acc;
  }
  double G = 0.0;
  for (int k = 0; k < n_atoms; ++k) G += atoms[5 * k + 4] * psi[k];
  if (psi_rxn) memcpy(psi_rxn, psi, sizeof(double) * (size_t)n_atoms);
  free(psi);
  return 0.5 * G;
}
