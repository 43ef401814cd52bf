// Plain FP64 CPU oracle for the Augmented Lagrangian TFW orbital-free DFT method
// (Suryanarayana & Phanish, "Augmented Lagrangian formulation of Orbital-Free
// Density Functional Theory", arXiv:1405.6456).
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library.  The GPU library never
// links, loads or calls it, and it shares no code with the GPU library.
//
// Every routine is written for a reader holding the paper: plain loops over the
// unpadded grid (index i + n1*(j + n2*k)), ghost values read through a bounds
// check that returns zero (the zero-Dirichlet convention of Sec. 4), and every
// sum in double precision.  OpenMP only splits outer loops.
//
// Readings of the paper that this file takes (the paper is silent or uses other
// inputs there) are marked "reading:" at the place they apply.
//
// Build: g++ -O2 -fopenmp -ffp-contract=off -shared -fPIC oracle.cpp -o liboracle.so

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

// ---------------------------------------------------------------- data types
typedef struct {
  int n[3];          // nodes per axis
  double h;          // grid spacing (Bohr)
  double origin[3];  // position of node (0,0,0)
} OrGrid;

typedef struct {
  OrGrid grid;
  int M;            // number of atoms
  const double* R;  // 3M positions (Bohr)
  const double* Z;  // M valence charges
  double N;         // number of electrons
} OrSystem;

typedef struct {
  int fd_n;             // FD half-width n (order 2n)
  double lambda;        // von Weizsaecker weight
  int xc;               // 0 = none, 1 = LDA Ceperley-Alder / Perdew-Zunger
  double gauss_s;       // width s of the Gaussian pseudocharge
  double r_cut;         // support radius of b_J
  int method;           // 0 = augmented Lagrangian, 1 = penalty, 2 = Lagrange multiplier
  double eta0, mu0, kappa;
  double tol_constraint;  // |C_h|/N
  double tol_grad;        // (h^3 sum g^2)^(1/2)
  double tol_poisson;     // ||rhs - A phi||_2 / ||rhs||_2
  int bc;                 // 0 = zero Dirichlet phi, 1 = multipole (monopole+dipole+quadrupole)
  int max_al, max_nlcg, max_cg;
  double sigma0;        // secant probe step
  int max_secant;       // secant steps per line search
  double secant_rel;    // stop the line search once |slope| <= secant_rel*|slope at start|
  int restart_every;    // NLCG restart period
  int tf_on;            // test switch: Thomas-Fermi term
  int hartree_on;       // test switch: electrostatics (pseudocharge + Hartree)
  const double* vext;   // test switch: fixed external potential on the grid (nullable)
  int verbose;
  int al_stop;          // outer stopping rule: 0 = |C_h|/N < tol_constraint, 1 = |E_q - E_(q-1)|/M < tol_energy
  double tol_energy;    // Ha per atom (rule 1)
  int pseudo;           // pseudocharge: 0 = Gaussian b_J, 1 = -(1/4 pi) Delta_h V_J at the nodes
  int domain;           // 0 = the box of nodes; 1 = the ellipsoid inscribed in it (Sec. 5.1): u and
                        // phi are zero (Dirichlet) at every node outside it; needs bc = 0
} OrParams;

typedef struct {
  double E_total, E_TF, E_vW, E_xc, E_es, E_self, E_c, E_ext, L;
  double eta, C, gnorm, dE_last, poisson_relres;
  long al_iters, nlcg_iters, grad_evals, poisson_solves, cg_iters, matvecs;
  int status;  // 0 converged, 1 iteration cap reached, -4 non-finite value, -5 ellipsoid with bc != 0
} OrResult;

typedef struct {
  double E_TF, E_vW, E_xc, E_es, E_ext, C, L, E_self, E_c, E_total;
} OrEnergies;

// ---------------------------------------------------------------- grid helpers
static inline long npts(const OrGrid* g) { return (long)g->n[0] * g->n[1] * g->n[2]; }
static inline long lin(const OrGrid* g, int i, int j, int k) {
  return i + (long)g->n[0] * (j + (long)g->n[1] * k);
}
// Zero Dirichlet ghosts: any index outside the grid reads 0 (Sec. 4).
static inline double at(const OrGrid* g, const double* f, int i, int j, int k) {
  if (i < 0 || j < 0 || k < 0 || i >= g->n[0] || j >= g->n[1] || k >= g->n[2]) return 0.0;
  return f[lin(g, i, j, k)];
}
static inline void pos(const OrGrid* g, int i, int j, int k, double x[3]) {
  x[0] = g->origin[0] + i * g->h;
  x[1] = g->origin[1] + j * g->h;
  x[2] = g->origin[2] + k * g->h;
}
static inline void centre(const OrGrid* g, double c[3]) {
  for (int a = 0; a < 3; ++a) c[a] = g->origin[a] + 0.5 * (g->n[a] - 1) * g->h;
}
// Sec. 5.1 (remark on the efficiency of the calculations): the Dirichlet conditions on u and
// phi imposed on an ellipsoid inside the box instead of on the box.  reading: the ellipsoid
// inscribed in the box of nodes, centre and semi-axes (n_a - 1) h / 2 per axis; a node on or
// inside it is a free node, every other node a Dirichlet node with u = phi = 0.
int or_domain_inside(const OrGrid* g, int i, int j, int k) {
  const int idx[3] = {i, j, k};
  double q = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double c = 0.5 * (g->n[a] - 1);
    if (c > 0) q += ((idx[a] - c) / c) * ((idx[a] - c) / c);
  }
  return q <= 1.0 + 1e-12 ? 1 : 0;
}

void or_domain_mask(const OrGrid* g, unsigned char* mask) {
  for (int k = 0; k < g->n[2]; ++k)
    for (int j = 0; j < g->n[1]; ++j)
      for (int i = 0; i < g->n[0]; ++i) mask[lin(g, i, j, k)] = (unsigned char)or_domain_inside(g, i, j, k);
}

static double dot(long n, const double* a, const double* b) {
  double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (long i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

void or_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}
int or_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// ---------------------------------------------------------------- FD weights
// (n!)^2 / ((n-p)! (n+p)!) as a product of p ratios.
static double fact_ratio(int n, int p) {
  double r = 1.0;
  for (int q = 1; q <= p; ++q) r *= double(n - q + 1) / double(n + q);
  return r;
}

// Laplacian weights w_0..w_n of the order-2n central difference (Sec. 4,
// weights of Eq. FD:Laplacian).
void or_fd_weights(int n, double h, double* w) {
  double s = 0.0;
  for (int q = 1; q <= n; ++q) s += 1.0 / double(q * q);
  w[0] = -s / (h * h);
  for (int p = 1; p <= n; ++p) {
    double sgn = (p % 2 == 1) ? 1.0 : -1.0;  // (-1)^(p+1)
    w[p] = 2.0 * sgn / (h * h * p * p) * fact_ratio(n, p);
  }
}

// Gradient weights w~_1..w~_n (Sec. 4, FD gradient used for the forces);
// wt[0] is set to 0.
void or_fd_grad_weights(int n, double h, double* wt) {
  wt[0] = 0.0;
  for (int p = 1; p <= n; ++p) {
    double sgn = (p % 2 == 1) ? 1.0 : -1.0;
    wt[p] = sgn / (h * p) * fact_ratio(n, p);
  }
}

// ---------------------------------------------------------------- stencil
// out = Delta_h f with zero ghosts (Sec. 4, Eq. FD:Laplacian).  The sum runs from
// p = 0 exactly as printed, so the centre value enters six times with w_0.
void or_laplacian(const OrGrid* g, int n, const double* f, double* out) {
  std::vector<double> w(n + 1);
  or_fd_weights(n, g->h, w.data());
#pragma omp parallel for schedule(static)
  for (int k = 0; k < g->n[2]; ++k)
    for (int j = 0; j < g->n[1]; ++j)
      for (int i = 0; i < g->n[0]; ++i) {
        double acc = 0.0;
        for (int p = 0; p <= n; ++p)
          acc += w[p] * (at(g, f, i + p, j, k) + at(g, f, i - p, j, k) + at(g, f, i, j + p, k) +
                         at(g, f, i, j - p, k) + at(g, f, i, j, k + p) + at(g, f, i, j, k - p));
        out[lin(g, i, j, k)] = acc;
      }
}

// ---------------------------------------------------------------- LDA XC
// Exchange and Ceperley-Alder correlation in the Perdew-Zunger form, energy per
// particle eps_xc and potential V_xc = d(rho eps_xc)/d rho (Sec. 2 and Sec. 3).
// reading: below rho = 1e-30 both are set to their r_s -> infinity limit 0.
void or_xc_point(double u, double* eps, double* v) {
  const double g1 = -0.1423, b1 = 1.0529, b2 = 0.3334;
  const double A1 = 0.0311, B1 = -0.048, C1 = 0.002, D1 = -0.0116;
  double au = std::fabs(u);
  double rho = au * au;
  if (rho < 1e-30) {
    *eps = 0.0;
    *v = 0.0;
    return;
  }
  double c3pi = std::cbrt(3.0 / M_PI);
  double u23 = std::pow(au, 2.0 / 3.0);
  double ex = -0.75 * c3pi * u23;
  double vx = -c3pi * u23;
  double rs = std::cbrt(3.0 / (4.0 * M_PI * rho));
  double ec, vc;
  if (rs >= 1.0) {
    double sq = std::sqrt(rs);
    double den = 1.0 + b1 * sq + b2 * rs;
    ec = g1 / den;
    vc = (g1 + (7.0 / 6.0) * g1 * b1 * sq + (4.0 / 3.0) * g1 * b2 * rs) / (den * den);
  } else {
    double lr = std::log(rs);
    ec = A1 * lr + B1 + C1 * rs * lr + D1 * rs;
    vc = (A1 + (2.0 / 3.0) * C1 * rs) * lr + (B1 - A1 / 3.0) + (1.0 / 3.0) * (2.0 * D1 - C1) * rs;
  }
  *eps = ex + ec;
  *v = vx + vc;
}

// Thomas-Fermi constant C_F = (3/10)(3 pi^2)^(2/3) (Sec. 2, Eq. KineticEnergy).
double or_CF(void) { return 0.3 * std::pow(3.0 * M_PI * M_PI, 2.0 / 3.0); }

// ---------------------------------------------------------------- nuclei
// reading: the pseudocharge of nucleus J is -Z_J times a normalised Gaussian of
// width s, cut at r_cut; its potential is V_J = -Z_J erf(r/s)/r, which satisfies
// b_J = -(1/4 pi) Laplacian V_J (Sec. 2, Eq. b:Pseudopotential).
double or_bJ(double Z, double s, double rcut, double r) {
  if (r > rcut) return 0.0;
  return -Z * std::pow(M_PI, -1.5) / (s * s * s) * std::exp(-(r * r) / (s * s));
}
double or_VJ(double Z, double s, double r) {
  if (r == 0.0) return -2.0 * Z / (s * std::sqrt(M_PI));
  return -Z * std::erf(r / s) / r;
}

// reading: the paper builds b_J = -(1/4 pi) Delta_h V_J from the pseudopotential on
// the nodes of the ball (Sec. 4, the b_J formula after Eq. FD:Laplacian); here V_J is the
// Gaussian potential above, and b_J is taken on the same ball |x - R_J| <= r_cut (beyond it
// V_J is the Coulomb potential to 1e-21 and its discrete Laplacian only the truncation
// error of the stencil).  (dx, dy, dz) = x - R_J.
double or_bJ_fd(double Z, double s, double rcut, double h, int n, double dx, double dy, double dz) {
  if (dx * dx + dy * dy + dz * dz > rcut * rcut) return 0.0;
  std::vector<double> w(n + 1);
  or_fd_weights(n, h, w.data());
  auto V = [&](double x, double y, double z) { return or_VJ(Z, s, std::sqrt(x * x + y * y + z * z)); };
  double lap = 0.0;
  for (int p = 0; p <= n; ++p) {
    double ph = p * h;
    lap += w[p] * (V(dx + ph, dy, dz) + V(dx - ph, dy, dz) + V(dx, dy + ph, dz) + V(dx, dy - ph, dz) +
                   V(dx, dy, dz + ph) + V(dx, dy, dz - ph));
  }
  return -lap / (4.0 * M_PI);
}

// b_J at offset (dx, dy, dz) from its nucleus for pseudocharge mode 0 (Gaussian) or 1
// (discrete Laplacian of V_J).
static double bJ_mode(int mode, int n, double h, double Z, double s, double rcut, double dx, double dy, double dz) {
  if (mode == 1) return or_bJ_fd(Z, s, rcut, h, n, dx, dy, dz);
  return or_bJ(Z, s, rcut, std::sqrt(dx * dx + dy * dy + dz * dz));
}

// Index box of the nodes that can lie within distance rad of point x.
static void ball_box(const OrGrid* g, const double* x, double rad, int lo[3], int hi[3]) {
  for (int a = 0; a < 3; ++a) {
    lo[a] = (int)std::floor((x[a] - rad - g->origin[a]) / g->h) - 1;
    hi[a] = (int)std::ceil((x[a] + rad - g->origin[a]) / g->h) + 1;
    lo[a] = std::max(lo[a], 0);
    hi[a] = std::min(hi[a], g->n[a] - 1);
  }
}

// b = sum_J b_J on the grid, visiting each atom's ball (Sec. 4, construction of b).
void or_pseudocharge(const OrGrid* g, int M, const double* R, const double* Z, double s, double rcut, int mode,
                     int n, double* b) {
  std::memset(b, 0, sizeof(double) * npts(g));
  for (int J = 0; J < M; ++J) {
    int lo[3], hi[3];
    ball_box(g, R + 3 * J, rcut, lo, hi);
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          double x[3];
          pos(g, i, j, k, x);
          double dx = x[0] - R[3 * J], dy = x[1] - R[3 * J + 1], dz = x[2] - R[3 * J + 2];
          double r = std::sqrt(dx * dx + dy * dy + dz * dz);
          if (r <= rcut) b[lin(g, i, j, k)] += bJ_mode(mode, n, g->h, Z[J], s, rcut, dx, dy, dz);
        }
  }
}

// b at one node, summing over all atoms (used for sampled checks on large grids).
double or_pseudocharge_at(const OrGrid* g, int M, const double* R, const double* Z, double s,
                          double rcut, int mode, int n, int i, int j, int k) {
  double x[3], acc = 0.0;
  pos(g, i, j, k, x);
  for (int J = 0; J < M; ++J) {
    double dx = x[0] - R[3 * J], dy = x[1] - R[3 * J + 1], dz = x[2] - R[3 * J + 2];
    double r = std::sqrt(dx * dx + dy * dy + dz * dz);
    if (r <= rcut) acc += bJ_mode(mode, n, g->h, Z[J], s, rcut, dx, dy, dz);
  }
  return acc;
}

// Self energy 1/2 sum_J int b_J V_J with the nodal quadrature (Sec. 2, last term
// of Eq. ElectroststaticReformulation; Sec. 4 quadrature).
double or_self_energy(const OrGrid* g, int M, const double* R, const double* Z, double s, double rcut, int mode,
                      int n) {
  double h3 = g->h * g->h * g->h, tot = 0.0;
  for (int J = 0; J < M; ++J) {
    int lo[3], hi[3];
    ball_box(g, R + 3 * J, rcut, lo, hi);
    double acc = 0.0;
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          double x[3];
          pos(g, i, j, k, x);
          double dx = x[0] - R[3 * J], dy = x[1] - R[3 * J + 1], dz = x[2] - R[3 * J + 2];
          double r = std::sqrt(dx * dx + dy * dy + dz * dz);
          if (r <= rcut) acc += bJ_mode(mode, n, g->h, Z[J], s, rcut, dx, dy, dz) * or_VJ(Z[J], s, r);
        }
    tot += 0.5 * h3 * acc;
  }
  return tot;
}

// Initial guess (Sec. 4: a superposition of isolated-atom densities).  reading: each
// atom contributes a Gaussian density of Z_J electrons, rho_J = Z_J (pi w^2)^(-3/2)
// exp(-r^2/w^2) cut at r = 5w, and a uniform floor of floor_frac N/V keeps u > 0 in the
// vacuum; the sum is scaled to h^3 sum rho = N and u0 = sqrt(rho).
void or_atomic_guess(const OrGrid* g, int M, const double* R, const double* Z, double N, double w,
                     double floor_frac, double* u) {
  const long n = npts(g);
  const double h3 = g->h * g->h * g->h, rc = 5.0 * w, norm = std::pow(M_PI * w * w, -1.5);
  std::vector<double> rho(n, 0.0);
  for (int J = 0; J < M; ++J) {
    int lo[3], hi[3];
    ball_box(g, R + 3 * J, rc, lo, hi);
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          double x[3];
          pos(g, i, j, k, x);
          double dx = x[0] - R[3 * J], dy = x[1] - R[3 * J + 1], dz = x[2] - R[3 * J + 2];
          double r2 = dx * dx + dy * dy + dz * dz;
          if (r2 <= rc * rc) rho[lin(g, i, j, k)] += Z[J] * norm * std::exp(-r2 / (w * w));
        }
  }
  double tot = 0.0;
  const double fl = floor_frac * N / (n * h3);
  for (long i = 0; i < n; ++i) {
    rho[i] += fl;
    tot += rho[i];
  }
  const double scale = N / (h3 * tot);
  for (long i = 0; i < n; ++i) u[i] = std::sqrt(rho[i] * scale);
}

// Overlap correction (Appendix A).  reading: for Gaussian pseudocharges the
// reference charges of the appendix can be taken as point charges, and the
// correction becomes the point-charge repulsion minus the Gaussian-Gaussian
// repulsion, 1/2 sum_{I!=J} Z_I Z_J erfc(R_IJ/(sqrt2 s))/R_IJ.  fc (nullable)
// receives f^c_J = -dE_c/dR_J.
double or_overlap_correction(int M, const double* R, const double* Z, double s, double* fc) {
  double a = std::sqrt(2.0) * s, E = 0.0;
  if (fc) std::memset(fc, 0, sizeof(double) * 3 * M);
  for (int I = 0; I < M; ++I)
    for (int J = 0; J < M; ++J) {
      if (I == J) continue;
      double d[3] = {R[3 * J] - R[3 * I], R[3 * J + 1] - R[3 * I + 1], R[3 * J + 2] - R[3 * I + 2]};
      double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      E += 0.5 * Z[I] * Z[J] * std::erfc(r / a) / r;
      if (fc) {
        // dF/dr for F(r) = erfc(r/a)/r
        double dF = -std::erfc(r / a) / (r * r) - 2.0 / (a * std::sqrt(M_PI)) * std::exp(-r * r / (a * a)) / r;
        for (int c = 0; c < 3; ++c) fc[3 * J + c] -= Z[I] * Z[J] * dF * d[c] / r;
      }
    }
  return E;
}

// ---------------------------------------------------------------- electrostatics
// Multipole moments of rho about the box centre: Q, P_a, and the traceless
// Theta_ab = h^3 sum rho (3 d_a d_b - |d|^2 delta_ab), stored as
// [Q, Px, Py, Pz, Txx, Tyy, Tzz, Txy, Txz, Tyz].
// reading: the paper suggests a multipole boundary condition for phi (Sec. 5.1);
// the expansion is taken to quadrupole order about the box centre.
void or_moments(const OrGrid* g, const double* rho, double mom[10]) {
  double c[3];
  centre(g, c);
  double h3 = g->h * g->h * g->h;
  double m[10] = {0};
  for (int k = 0; k < g->n[2]; ++k)
    for (int j = 0; j < g->n[1]; ++j)
      for (int i = 0; i < g->n[0]; ++i) {
        double x[3];
        pos(g, i, j, k, x);
        double d[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
        double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double q = rho[lin(g, i, j, k)];
        m[0] += q;
        m[1] += q * d[0];
        m[2] += q * d[1];
        m[3] += q * d[2];
        m[4] += q * (3 * d[0] * d[0] - d2);
        m[5] += q * (3 * d[1] * d[1] - d2);
        m[6] += q * (3 * d[2] * d[2] - d2);
        m[7] += q * 3 * d[0] * d[1];
        m[8] += q * 3 * d[0] * d[2];
        m[9] += q * 3 * d[1] * d[2];
      }
  for (int a = 0; a < 10; ++a) mom[a] = h3 * m[a];
}

// phi_mp(y) = Q/r + P.D/r^3 + 1/2 sum_ab Theta_ab D_a D_b / r^5, D = y - centre.
double or_phi_multipole(const double mom[10], const double c[3], const double y[3]) {
  double D[3] = {y[0] - c[0], y[1] - c[1], y[2] - c[2]};
  double r2 = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
  double r = std::sqrt(r2);
  double r3 = r2 * r, r5 = r3 * r2;
  double dip = mom[1] * D[0] + mom[2] * D[1] + mom[3] * D[2];
  double quad = mom[4] * D[0] * D[0] + mom[5] * D[1] * D[1] + mom[6] * D[2] * D[2] +
                2.0 * (mom[7] * D[0] * D[1] + mom[8] * D[0] * D[2] + mom[9] * D[1] * D[2]);
  return mom[0] / r + dip / r3 + 0.5 * quad / r5;
}

// Right-hand side of the discrete Poisson problem (Sec. 4, Eq. Poisson:Discretized):
// rhs = rho plus, for bc = 1, the known ghost values moved to the right:
// rhs_i += (1/4 pi) sum over the stencil taps that leave the grid of w_p phi_mp(ghost).
void or_poisson_rhs(const OrGrid* g, int n, int bc, const double* rho, double* rhs) {
  long N = npts(g);
  for (long i = 0; i < N; ++i) rhs[i] = rho[i];
  if (bc == 0) return;
  std::vector<double> w(n + 1);
  or_fd_weights(n, g->h, w.data());
  double mom[10], c[3];
  or_moments(g, rho, mom);
  centre(g, c);
  const int dirs[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
  for (int k = 0; k < g->n[2]; ++k)
    for (int j = 0; j < g->n[1]; ++j)
      for (int i = 0; i < g->n[0]; ++i) {
        double add = 0.0;
        for (int d = 0; d < 6; ++d)
          for (int p = 1; p <= n; ++p) {
            int ii = i + p * dirs[d][0], jj = j + p * dirs[d][1], kk = k + p * dirs[d][2];
            bool inside = ii >= 0 && jj >= 0 && kk >= 0 && ii < g->n[0] && jj < g->n[1] && kk < g->n[2];
            if (inside) continue;
            double y[3];
            pos(g, ii, jj, kk, y);
            add += w[p] * or_phi_multipole(mom, c, y);
          }
        rhs[lin(g, i, j, k)] += add / (4.0 * M_PI);
      }
}

// A f = -(1/4 pi) Delta_h f with zero ghosts.
static void apply_A(const OrGrid* g, int n, const double* f, double* out) {
  or_laplacian(g, n, f, out);
  long N = npts(g);
  for (long i = 0; i < N; ++i) out[i] *= -1.0 / (4.0 * M_PI);
}

// Conjugate gradients on A phi = rhs from the given phi (warm start, Sec. 4),
// stopping at ||rhs - A phi||_2 < tol ||rhs||_2.
// reading: the paper solves this symmetric positive definite system with GMRES;
// CG reaches the same solution to the same tolerance.
// With a mask (the active domain), the unknowns are the masked nodes only: phi is zero at
// every other node, and the equations there are dropped (A restricted to the domain, which is
// again symmetric positive definite).
// Returns 0 on convergence, 1 at the iteration cap.  *iters = iterations taken.
int or_poisson_cg_masked(const OrGrid* g, int n, const unsigned char* mask, const double* rhs, double* phi,
                         double tol, int maxit, int* iters, double* relres) {
  long N = npts(g);
  std::vector<double> r(N), p(N), Ap(N), b(rhs, rhs + N);
  auto restrict_to = [&](double* f) {
    if (mask)
      for (long i = 0; i < N; ++i)
        if (!mask[i]) f[i] = 0.0;
  };
  restrict_to(b.data());
  restrict_to(phi);
  double bnorm = std::sqrt(dot(N, b.data(), b.data()));
  if (iters) *iters = 0;
  if (bnorm == 0.0) {
    std::fill(phi, phi + N, 0.0);
    if (relres) *relres = 0.0;
    return 0;
  }
  apply_A(g, n, phi, Ap.data());
  restrict_to(Ap.data());
  for (long i = 0; i < N; ++i) r[i] = b[i] - Ap[i];
  p = r;
  double rr = dot(N, r.data(), r.data());
  int it = 0;
  while (std::sqrt(rr) >= tol * bnorm && it < maxit) {
    apply_A(g, n, p.data(), Ap.data());
    restrict_to(Ap.data());
    double alpha = rr / dot(N, p.data(), Ap.data());
    for (long i = 0; i < N; ++i) {
      phi[i] += alpha * p[i];
      r[i] -= alpha * Ap[i];
    }
    double rr_new = dot(N, r.data(), r.data());
    double beta = rr_new / rr;
    rr = rr_new;
    for (long i = 0; i < N; ++i) p[i] = r[i] + beta * p[i];
    ++it;
  }
  if (iters) *iters = it;
  if (relres) *relres = std::sqrt(rr) / bnorm;
  return std::sqrt(rr) < tol * bnorm ? 0 : 1;
}

int or_poisson_cg(const OrGrid* g, int n, const double* rhs, double* phi, double tol, int maxit, int* iters,
                  double* relres) {
  return or_poisson_cg_masked(g, n, nullptr, rhs, phi, tol, maxit, iters, relres);
}

// ---------------------------------------------------------------- energy and gradient
struct Work {
  const OrSystem* sys;
  const OrParams* prm;
  long N;
  double h3;
  std::vector<double> b, phi, lap, rho, rhs, jac;
  std::vector<unsigned char> mask;  // active domain (empty: the whole box)
  double E_self, E_c;
  long grad_evals, poisson_solves, cg_iters, matvecs;
  double last_relres;
  int poisson_capped;
};

static void work_init(Work& W, const OrSystem* sys, const OrParams* prm) {
  W.sys = sys;
  W.prm = prm;
  W.N = npts(&sys->grid);
  W.h3 = sys->grid.h * sys->grid.h * sys->grid.h;
  W.b.assign(W.N, 0.0);
  W.phi.assign(W.N, 0.0);
  W.lap.assign(W.N, 0.0);
  W.rho.assign(W.N, 0.0);
  W.rhs.assign(W.N, 0.0);
  W.jac.assign(W.N, 0.0);
  W.E_self = 0.0;
  W.E_c = 0.0;
  W.mask.clear();
  if (prm->domain == 1) {
    W.mask.assign(W.N, 0);
    or_domain_mask(&sys->grid, W.mask.data());
  }
  if (prm->hartree_on) {
    or_pseudocharge(&sys->grid, sys->M, sys->R, sys->Z, prm->gauss_s, prm->r_cut, prm->pseudo, prm->fd_n,
                    W.b.data());
    W.E_self = or_self_energy(&sys->grid, sys->M, sys->R, sys->Z, prm->gauss_s, prm->r_cut, prm->pseudo,
                              prm->fd_n);
    W.E_c = or_overlap_correction(sys->M, sys->R, sys->Z, prm->gauss_s, nullptr);
  }
  W.grad_evals = W.poisson_solves = W.cg_iters = W.matvecs = 0;
  W.last_relres = 0.0;
  W.poisson_capped = 0;
}

// Solve for phi of the density u^2 + b, warm-started from W.phi (Sec. 4: phi is
// re-solved for every update of u).
static void solve_phi(Work& W, const double* u) {
  const OrSystem* S = W.sys;
  const OrParams* P = W.prm;
  for (long i = 0; i < W.N; ++i) W.rho[i] = u[i] * u[i] + W.b[i];
  or_poisson_rhs(&S->grid, P->fd_n, P->bc, W.rho.data(), W.rhs.data());
  int it = 0;
  double rel = 0.0;
  int st = or_poisson_cg_masked(&S->grid, P->fd_n, W.mask.empty() ? nullptr : W.mask.data(), W.rhs.data(),
                                W.phi.data(), P->tol_poisson, P->max_cg, &it, &rel);
  if (st != 0) W.poisson_capped++;
  W.poisson_solves++;
  W.cg_iters += it;
  W.matvecs += it + 1;  // CG matvecs plus the initial residual
  W.last_relres = rel;
}

// Energies of u (Sec. 2, Eq. F with the quadrature of Sec. 4) and, if g != null,
// the discrete Euler-Lagrange residual (Sec. 4, Eq. EulerLagrangeDiscretized):
// g = -(lambda/2) Delta_h u + (V_K + V_xc + phi [+ V_ext]) u + (-eta + C_h/mu) u.
// reading: the residual is half the derivative of L with respect to u_i/h^3.
// W.phi must already hold the potential of u.
static void energy_gradient(Work& W, const double* u, double eta, double mu, double* g, OrEnergies* e) {
  const OrSystem* S = W.sys;
  const OrParams* P = W.prm;
  const OrGrid* G = &S->grid;
  long N = W.N;
  double CF = or_CF();
  or_laplacian(G, P->fd_n, u, W.lap.data());
  W.matvecs += 1;
  double sum_u2 = 0, sTF = 0, svW = 0, sxc = 0, ses = 0, sext = 0;
#pragma omp parallel for reduction(+ : sum_u2, sTF, svW, sxc, ses, sext) schedule(static)
  for (long i = 0; i < N; ++i) {
    double ui = u[i], au = std::fabs(ui);
    sum_u2 += ui * ui;
    if (P->tf_on) sTF += std::pow(au, 10.0 / 3.0);
    svW += ui * W.lap[i];
    if (P->xc) {
      double eps, v;
      or_xc_point(ui, &eps, &v);
      sxc += eps * ui * ui;
    }
    if (P->hartree_on) ses += (ui * ui + W.b[i]) * W.phi[i];
    if (P->vext) sext += P->vext[i] * ui * ui;
  }
  double C = W.h3 * sum_u2 - S->N;
  OrEnergies en;
  en.E_TF = CF * W.h3 * sTF;
  en.E_vW = -0.5 * P->lambda * W.h3 * svW;
  en.E_xc = W.h3 * sxc;
  en.E_es = P->hartree_on ? 0.5 * W.h3 * ses - W.E_self : 0.0;
  en.E_ext = W.h3 * sext;
  en.E_self = W.E_self;
  en.E_c = W.E_c;
  en.E_total = en.E_TF + en.E_vW + en.E_xc + en.E_es + en.E_ext + en.E_c;
  en.C = C;
  en.L = en.E_total - eta * C + (mu > 0 ? C * C / (2.0 * mu) : 0.0);
  if (e) *e = en;
  if (!g) return;
  double shift = -eta + (mu > 0 ? C / mu : 0.0);
  std::vector<double> w(P->fd_n + 1);
  or_fd_weights(P->fd_n, G->h, w.data());
  const double vw_diag = -3.0 * P->lambda * w[0];
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    double ui = u[i], au = std::fabs(ui);
    double veff = 0.0;
    if (P->tf_on) veff += (5.0 / 3.0) * CF * std::pow(au, 4.0 / 3.0);
    if (P->xc) {
      double eps, v;
      or_xc_point(ui, &eps, &v);
      veff += v;
    }
    double vk = P->tf_on ? (5.0 / 3.0) * CF * std::pow(au, 4.0 / 3.0) : 0.0;
    if (P->hartree_on) veff += W.phi[i];
    if (P->vext) veff += P->vext[i];
    g[i] = -0.5 * P->lambda * W.lap[i] + veff * ui + shift * ui;
    if (!W.mask.empty() && !W.mask[i]) g[i] = 0.0;  // u is fixed (zero) outside the domain
    // local diagonal of the residual's Jacobian (Jacobi preconditioner), with the
    // non-vW part clipped at zero: -3 lambda w_0 + max(0, (4/3)V_K + V_eff + shift)
    W.jac[i] = vw_diag + std::max(0.0, (4.0 / 3.0) * vk + veff + shift);
  }
  W.grad_evals++;
}

// Full evaluation at u: phi re-solved, then energies and residual.
static void evaluate(Work& W, const double* u, double eta, double mu, double* g, OrEnergies* e) {
  if (W.prm->hartree_on) solve_phi(W, u);
  energy_gradient(W, u, eta, mu, g, e);
}

// Exported single evaluation (phi_inout is the warm start and receives the solution).
int or_evaluate(const OrSystem* sys, const OrParams* prm, const double* u, double eta, double mu,
                double* phi_inout, double* g, OrEnergies* e, long* cg_iters) {
  Work W;
  work_init(W, sys, prm);
  if (phi_inout) std::memcpy(W.phi.data(), phi_inout, sizeof(double) * W.N);
  std::vector<double> um(u, u + W.N);  // u is zero outside the active domain
  for (long i = 0; i < (long)W.mask.size(); ++i)
    if (!W.mask[i]) um[i] = 0.0;
  evaluate(W, um.data(), eta, mu, g, e);
  if (phi_inout) std::memcpy(phi_inout, W.phi.data(), sizeof(double) * W.N);
  if (cg_iters) *cg_iters = W.cg_iters;
  return W.poisson_capped ? 1 : 0;
}

static double hnorm(const Work& W, const double* g) { return std::sqrt(W.h3 * dot(W.N, g, g)); }

static bool finite_all(long n, const double* a) {
  for (long i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

// ---------------------------------------------------------------- inner minimiser
// Minimise L(u; eta, mu) over u >= 0 with the Polak-Ribiere nonlinear conjugate
// gradient method, a secant line search and a Jacobi preconditioner (Sec. 4),
// every trial point being made non-negative.
// reading: the Jacobi preconditioner is the local diagonal of the residual's
// Jacobian, -3 lambda w_0 + (4/3)V_K + V_eff - eta + C/mu, with everything but
// the von Weizsaecker part clipped at zero so that it stays positive.
// reading: each line search runs Shewchuk's secant iteration on the derivative
// of t -> L(|u + t d|) from the start point u (trial points |u + t d|; the
// derivative is sum_i g_i sign(u_i + t d_i) d_i), kept inside a bracket [a, b] of slopes
// (negative at a, positive at b): a secant proposal outside the bracket is
// replaced by bisection, or by doubling while no positive slope has been seen.
// It stops once |slope| <= secant_rel |slope at t = 0| or after max_secant
// steps.  The probe step is sigma0.
// Returns 0 when ||g|| < tol_grad, 1 at the iteration cap, -4 on a non-finite value.
static int nlcg(Work& W, double* u, double eta, double mu, OrEnergies* e_out, double* gnorm_out,
                long* iters_out) {
  const OrParams* P = W.prm;
  long N = W.N;
  std::vector<double> g(N), s(N), s_old(N), d(N), u_start(N);
  OrEnergies e;
  evaluate(W, u, eta, mu, g.data(), &e);
  double gn = hnorm(W, g.data());
  long it = 0;
  int status = 1;
  auto precondition = [&]() {  // s = M^-1 r with r = -g
    for (long i = 0; i < N; ++i) s[i] = -g[i] / W.jac[i];
  };
  precondition();
  d = s;
  double delta_new = -dot(N, g.data(), s.data());  // r.s
  s_old = s;
  int since_restart = 0;
  // Trial point u = |u_start + t d|; returns the derivative of t -> L(|u_start + t d|),
  // sum_i g_i sign(u_start_i + t d_i) d_i.
  auto trial = [&](double t) {
    double slope = 0.0;
    for (long i = 0; i < N; ++i) u[i] = std::fabs(u_start[i] + t * d[i]);
    evaluate(W, u, eta, mu, g.data(), &e);
    for (long i = 0; i < N; ++i) {
      double v = u_start[i] + t * d[i];
      slope += g[i] * (v < 0.0 ? -d[i] : d[i]);
    }
    return slope;
  };
  while (true) {
    if (!std::isfinite(gn)) { status = -4; break; }
    if (gn < P->tol_grad) { status = 0; break; }
    if (it >= P->max_nlcg) { status = 1; break; }
    double slope0 = dot(N, g.data(), d.data());
    if (!(slope0 < 0.0)) {  // not a descent direction: restart along s
      d = s;
      since_restart = 0;
      slope0 = dot(N, g.data(), d.data());
    }
    std::copy(u, u + N, u_start.begin());
    // line search on the directional derivative from u_start along d; false when no
    // finite point was found (the last trial overshot to a non-finite value)
    double t_cur = P->sigma0;
    double s_cur = 0.0;
    auto bad = [&]() { return !std::isfinite(s_cur) || !std::isfinite(e.L); };
    auto search = [&](double slope0) {
      double a = 0.0, b = INFINITY;
      double t_prev = 0.0, s_prev = slope0;
      t_cur = P->sigma0;
      s_cur = trial(t_cur);
      // a trial with a non-finite slope or L overshot: it closes the bracket from above
      if (s_cur > 0.0 || bad()) b = t_cur; else a = t_cur;
      for (int j = 0; j < P->max_secant || bad(); ++j) {
        if (bad()) {
          if (j > 60) break;
          t_prev = a;
          s_prev = slope0;
          t_cur = 0.5 * (a + b);
          s_cur = trial(t_cur);
          if (s_cur > 0.0 || bad()) b = t_cur; else a = t_cur;
          continue;
        }
        if (std::fabs(s_cur) <= P->secant_rel * std::fabs(slope0)) break;
        double curv = (s_cur - s_prev) / (t_cur - t_prev);
        double t_new = (curv > 0.0) ? t_cur - s_cur / curv : NAN;
        double hi = std::isfinite(b) ? b : 4.0 * std::max(a, t_cur);
        if (!(t_new > a && t_new < hi)) t_new = std::isfinite(b) ? 0.5 * (a + b) : 2.0 * std::max(a, t_cur);
        t_prev = t_cur;
        s_prev = s_cur;
        t_cur = t_new;
        s_cur = trial(t_cur);
        if (P->verbose > 2)
          std::printf("      secant j=%d t=%.4e slope=%.4e slope0=%.4e [a=%.3e b=%.3e]\n", j, t_cur, s_cur, slope0, a, b);
        if (s_cur > 0.0 || bad()) b = std::min(b, t_cur); else a = std::max(a, t_cur);
      }
      return !bad();
    };
    bool ok = search(slope0);
    if (!ok && since_restart > 0) {
      // no finite point along the conjugate direction: search again from the same
      // point along the preconditioned steepest-descent direction s
      d = s;
      since_restart = 0;
      ok = search(-delta_new);
    }
    if (!ok) {  // no finite point found along d
      status = -4;
      break;
    }
    gn = hnorm(W, g.data());
    // Polak-Ribiere update with s = M^-1 r, r = -g
    precondition();
    double delta_old = delta_new;
    double delta_mid = -dot(N, g.data(), s_old.data());
    delta_new = -dot(N, g.data(), s.data());
    double beta = (delta_new - delta_mid) / delta_old;
    ++since_restart;
    // restart also when successive residuals have lost orthogonality (Powell's test,
    // |r_new . s_old| >= 0.2 r_new . s_new), before the direction can run away
    if (since_restart >= P->restart_every || beta <= 0.0 || std::fabs(delta_mid) >= 0.2 * delta_new) {
      d = s;
      since_restart = 0;
    } else {
      for (long i = 0; i < N; ++i) d[i] = s[i] + beta * d[i];
    }
    s_old = s;
    ++it;
    if (P->verbose > 1) std::printf("    nlcg %ld |g|=%.3e L=%.12f t=%.3e beta=%.3f\n", it, gn, e.L, t_cur, beta);
  }
  if (e_out) *e_out = e;
  if (gnorm_out) *gnorm_out = gn;
  if (iters_out) *iters_out += it;
  return status;
}

// ---------------------------------------------------------------- Lagrange multiplier variant
// Energy at |u(theta)| with u(theta) = u cos(theta) + sqrt(N) dhat sin(theta).
static double lm_energy_at(Work& W, const double* u, const double* dhat, double theta, double* ut) {
  double sN = std::sqrt(W.sys->N);
  double c = std::cos(theta), s = std::sin(theta);
  for (long i = 0; i < W.N; ++i) ut[i] = std::fabs(u[i] * c + sN * dhat[i] * s);
  OrEnergies e;
  evaluate(W, ut, 0.0, 0.0, nullptr, &e);
  return e.E_total;
}

// Brent's minimisation of f on [a, c] around b (f(b) < f(a), f(b) < f(c)).
static double brent_min(const std::function<double(double)>& f, double a, double b, double c, double fb, double tol, int maxit) {
  const double cg = 0.3819660112501051;
  double lo = std::min(a, c), hi = std::max(a, c);
  double x = b, wv = b, v = b, fx = fb, fw = fb, fv = fb;
  double dstep = 0.0, e = 0.0;
  for (int it = 0; it < maxit; ++it) {
    double xm = 0.5 * (lo + hi);
    double tol1 = tol * std::fabs(x) + 1e-12, tol2 = 2.0 * tol1;
    if (std::fabs(x - xm) <= tol2 - 0.5 * (hi - lo)) break;
    bool golden = true;
    if (std::fabs(e) > tol1) {
      double r = (x - wv) * (fx - fv), q = (x - v) * (fx - fw);
      double pp = (x - v) * q - (x - wv) * r;
      q = 2.0 * (q - r);
      if (q > 0.0) pp = -pp;
      q = std::fabs(q);
      double etemp = e;
      e = dstep;
      if (!(std::fabs(pp) >= std::fabs(0.5 * q * etemp) || pp <= q * (lo - x) || pp >= q * (hi - x))) {
        dstep = pp / q;
        double uu = x + dstep;
        if (uu - lo < tol2 || hi - uu < tol2) dstep = (xm - x >= 0 ? tol1 : -tol1);
        golden = false;
      }
    }
    if (golden) {
      e = (x >= xm) ? lo - x : hi - x;
      dstep = cg * e;
    }
    double uu = (std::fabs(dstep) >= tol1) ? x + dstep : x + (dstep >= 0 ? tol1 : -tol1);
    double fu = f(uu);
    if (fu <= fx) {
      if (uu >= x) lo = x; else hi = x;
      v = wv; fv = fw; wv = x; fw = fx; x = uu; fx = fu;
    } else {
      if (uu < x) lo = uu; else hi = uu;
      if (fu <= fw || wv == x) { v = wv; fv = fw; wv = uu; fw = fu; }
      else if (fu <= fv || v == x || v == wv) { v = uu; fv = fu; }
    }
  }
  return x;
}

// Lagrange multiplier method (Sec. 5.3.2): u stays on h^3 sum u^2 = N; the
// multiplier is the Rayleigh quotient; Polak-Ribiere directions projected
// orthogonal to u; a Brent line search on the energy along the great circle.
static int lagrange_solve(Work& W, double* u, OrResult* res, OrEnergies* e_out, double* gnorm_out) {
  const OrParams* P = W.prm;
  long N = W.N;
  double h3 = W.h3, Ne = W.sys->N;
  std::vector<double> w(P->fd_n + 1);
  or_fd_weights(P->fd_n, W.sys->grid.h, w.data());
  const double Mjac = -3.0 * P->lambda * w[0];
  // start on the constraint surface
  double nrm = h3 * dot(N, u, u);
  for (long i = 0; i < N; ++i) u[i] = std::fabs(u[i]) * std::sqrt(Ne / nrm);
  std::vector<double> g(N), gp(N), gp_old(N, 0.0), d(N, 0.0), dhat(N), ut(N);
  OrEnergies e;
  double eta = 0.0, gn = 0.0, delta_new = 1.0;
  long it = 0;
  int status = 1, since_restart = 0;
  while (true) {
    evaluate(W, u, 0.0, 0.0, g.data(), &e);  // g = H u (no multiplier terms)
    eta = h3 * dot(N, u, g.data()) / Ne;      // Rayleigh quotient
    for (long i = 0; i < N; ++i) gp[i] = g[i] - eta * u[i];
    gn = hnorm(W, gp.data());
    if (!std::isfinite(gn)) { status = -4; break; }
    if (gn < P->tol_grad) { status = 0; break; }
    if (it >= P->max_nlcg) { status = 1; break; }
    double delta_old = delta_new;
    double delta_mid = dot(N, gp.data(), gp_old.data()) / Mjac;
    delta_new = dot(N, gp.data(), gp.data()) / Mjac;
    double beta = (it == 0) ? 0.0 : (delta_new - delta_mid) / delta_old;
    ++since_restart;
    if (it == 0 || beta <= 0.0 || since_restart >= P->restart_every) {
      beta = 0.0;
      since_restart = 0;
    }
    for (long i = 0; i < N; ++i) d[i] = -gp[i] / Mjac + beta * d[i];
    // project orthogonal to u and normalise to h^3 sum dhat^2 = 1
    double ud = h3 * dot(N, u, d.data()) / Ne;
    for (long i = 0; i < N; ++i) d[i] -= ud * u[i];
    if (h3 * dot(N, g.data(), d.data()) >= 0.0) {  // not descent: steepest
      for (long i = 0; i < N; ++i) d[i] = -gp[i] / Mjac;
      ud = h3 * dot(N, u, d.data()) / Ne;
      for (long i = 0; i < N; ++i) d[i] -= ud * u[i];
      since_restart = 0;
    }
    double dn = std::sqrt(h3 * dot(N, d.data(), d.data()));
    for (long i = 0; i < N; ++i) dhat[i] = d[i] / dn;
    // bracket a minimum of E(theta) starting from theta = 0
    double E0 = e.E_total;
    double slope = 2.0 * h3 * std::sqrt(Ne) * dot(N, g.data(), dhat.data());  // dE/dtheta at 0
    double curv_guess = 2.0 * Mjac;  // rough curvature scale
    double t1 = std::min(0.5, std::fabs(slope) / (curv_guess * Ne) + 1e-6);
    double f1 = lm_energy_at(W, u, dhat.data(), t1, ut.data());
    double ta = 0.0, fa = E0, tb = t1, fb = f1, tc, fc;
    if (fb > fa) {  // shrink until below E0
      tc = tb; fc = fb;
      int guard = 0;
      do {
        tb = 0.5 * tb;
        fb = lm_energy_at(W, u, dhat.data(), tb, ut.data());
        if (fb > fa) { tc = tb; fc = fb; }
      } while (fb > fa && ++guard < 40);
      if (fb > fa) { status = 1; break; }
    } else {
      tc = 2.0 * tb;
      fc = lm_energy_at(W, u, dhat.data(), tc, ut.data());
      int guard = 0;
      while (fc < fb && ++guard < 40) {
        ta = tb; fa = fb; tb = tc; fb = fc;
        tc = 2.0 * tc;
        fc = lm_energy_at(W, u, dhat.data(), tc, ut.data());
      }
    }
    (void)fa; (void)fc;
    double theta = brent_min([&](double t) { return lm_energy_at(W, u, dhat.data(), t, ut.data()); },
                             ta, tb, tc, fb, 1e-8, 60);
    double sN = std::sqrt(Ne), cth = std::cos(theta), sth = std::sin(theta);
    for (long i = 0; i < N; ++i) u[i] = std::fabs(u[i] * cth + sN * dhat[i] * sth);
    gp_old = gp;
    ++it;
    if (P->verbose > 1) std::printf("    lm %ld |g|=%.3e E=%.12f eta=%.8f\n", it, gn, e.E_total, eta);
  }
  res->nlcg_iters += it;
  res->eta = eta;
  if (e_out) *e_out = e;
  if (gnorm_out) *gnorm_out = gn;
  return status;
}

// ---------------------------------------------------------------- forces
// Hellmann-Feynman forces (Sec. 2, Eq. Force:Nuclei, with the FD gradient of
// Sec. 4): f_J = h^3 sum_{|x_i - R_J| <= r_cut} (grad_h b_J)_i (phi_i - V_J(x_i)),
// plus the overlap correction of Appendix A (closed form for Gaussians).
// grad_h b_J uses b_J evaluated at the neighbouring node positions.
void or_forces(const OrSystem* sys, const OrParams* prm, const double* phi, double* f) {
  const OrGrid* g = &sys->grid;
  int n = prm->fd_n;
  double h = g->h, h3 = h * h * h, s = prm->gauss_s, rc = prm->r_cut;
  std::vector<double> wt(n + 1);
  or_fd_grad_weights(n, h, wt.data());
  std::vector<double> fc(3 * sys->M);
  or_overlap_correction(sys->M, sys->R, sys->Z, s, fc.data());
#pragma omp parallel for schedule(dynamic)
  for (int J = 0; J < sys->M; ++J) {
    const double* RJ = sys->R + 3 * J;
    double ZJ = sys->Z[J];
    auto bJ_at = [&](int i, int j, int k) {
      double x[3];
      pos(g, i, j, k, x);
      double dx = x[0] - RJ[0], dy = x[1] - RJ[1], dz = x[2] - RJ[2];
      return bJ_mode(prm->pseudo, n, h, ZJ, s, rc, dx, dy, dz);
    };
    int lo[3], hi[3];
    ball_box(g, RJ, rc, lo, hi);
    double acc[3] = {0, 0, 0};
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          double x[3];
          pos(g, i, j, k, x);
          double dx = x[0] - RJ[0], dy = x[1] - RJ[1], dz = x[2] - RJ[2];
          double r = std::sqrt(dx * dx + dy * dy + dz * dz);
          if (r > rc) continue;
          double grad[3] = {0, 0, 0};
          for (int p = 1; p <= n; ++p) {
            grad[0] += wt[p] * (bJ_at(i + p, j, k) - bJ_at(i - p, j, k));
            grad[1] += wt[p] * (bJ_at(i, j + p, k) - bJ_at(i, j - p, k));
            grad[2] += wt[p] * (bJ_at(i, j, k + p) - bJ_at(i, j, k - p));
          }
          double pot = phi[lin(g, i, j, k)] - or_VJ(ZJ, s, r);
          for (int a = 0; a < 3; ++a) acc[a] += grad[a] * pot;
        }
    for (int a = 0; a < 3; ++a) f[3 * J + a] = h3 * acc[a] + fc[3 * J + a];
  }
}

// ---------------------------------------------------------------- driver
void or_default_params(OrParams* p) {
  std::memset(p, 0, sizeof(*p));
  p->fd_n = 6;
  p->lambda = 0.2;
  p->xc = 1;
  p->gauss_s = 1.0;
  p->r_cut = 7.0;
  p->method = 0;
  p->eta0 = -0.2;
  p->mu0 = 1.0;
  p->kappa = 0.1;
  p->tol_constraint = 1e-8;
  p->tol_grad = 1e-6;
  p->tol_poisson = 1e-10;
  p->bc = 1;
  p->max_al = 30;
  p->max_nlcg = 20000;
  p->max_cg = 100000;
  p->sigma0 = 0.5;
  p->max_secant = 4;
  p->secant_rel = 0.1;
  p->restart_every = 50;
  p->tf_on = 1;
  p->hartree_on = 1;
  p->vext = nullptr;
  p->verbose = 0;
  p->al_stop = 0;
  p->tol_energy = 3.6749e-6;  // 1e-4 eV per atom (Sec. 5.3.1), in Hartree
  p->pseudo = 0;
  p->domain = 0;
}

// Ground state for fixed nuclei (Sec. 3, Algorithm AugLag, and Sec. 5.3.2 for
// the penalty and Lagrange multiplier variants).
// reading: the outer loop stops once |C_h|/N < tol_constraint (|Delta E| is
// reported); every inner problem is solved to ||g|| < tol_grad.
int or_solve(const OrSystem* sys, const OrParams* prm, const double* u0, double* u_out, double* phi_out,
             double* forces_out, OrResult* res) {
  std::memset(res, 0, sizeof(*res));
  Work W;
  work_init(W, sys, prm);
  long N = W.N;
  std::vector<double> u(u0, u0 + N);
  for (long i = 0; i < N; ++i) u[i] = std::fabs(u[i]);
  if (!finite_all(N, u.data())) {
    res->status = -4;
    return -4;
  }
  if (prm->domain == 1 && prm->bc != 0) {  // the ellipsoid takes zero Dirichlet values for phi
    res->status = -5;
    return -5;
  }
  for (long i = 0; i < (long)W.mask.size(); ++i)
    if (!W.mask[i]) u[i] = 0.0;
  OrEnergies e;
  std::memset(&e, 0, sizeof(e));
  double gn = 0.0;
  int status = 1;
  if (prm->method == 2) {
    status = lagrange_solve(W, u.data(), res, &e, &gn);
    res->al_iters = 1;
    res->dE_last = 0.0;
  } else {
    double eta = (prm->method == 1) ? 0.0 : prm->eta0;
    double mu = prm->mu0, E_prev = 0.0;
    for (int q = 0; q < prm->max_al; ++q) {
      long its = 0;
      int st = nlcg(W, u.data(), eta, mu, &e, &gn, &its);
      res->nlcg_iters += its;
      res->al_iters = q + 1;
      if (st == -4) { status = -4; break; }
      double C = e.C;
      double eta_next = eta - C / mu;  // Algorithm AugLag multiplier update
      res->dE_last = (q == 0) ? 0.0 : e.E_total - E_prev;
      E_prev = e.E_total;
      if (prm->verbose)
        std::printf("  AL q=%d eta=%.10f mu=%.3e C/N=%.3e E=%.12f nlcg=%ld |g|=%.2e\n", q, eta, mu,
                    C / sys->N, e.E_total, its, gn);
      res->eta = eta_next;
      // Algorithm AugLag stops on the change of the energy between outer steps; the
      // workloads' rule is the constraint (both need a converged inner problem)
      const bool stop = prm->al_stop == 1 ? (q > 0 && std::fabs(res->dE_last) / sys->M < prm->tol_energy)
                                          : std::fabs(C) / sys->N < prm->tol_constraint;
      if (stop && st == 0) {
        status = 0;
        break;
      }
      eta = (prm->method == 1) ? 0.0 : eta_next;
      mu *= prm->kappa;
    }
  }
  // energies of the last evaluation of the returned u (phi solved to tol_poisson there)
  res->E_total = e.E_total;
  res->E_TF = e.E_TF;
  res->E_vW = e.E_vW;
  res->E_xc = e.E_xc;
  res->E_es = e.E_es;
  res->E_self = W.E_self;
  res->E_c = W.E_c;
  res->E_ext = e.E_ext;
  res->L = e.L;
  res->C = e.C;
  res->gnorm = gn;
  res->poisson_relres = W.last_relres;
  res->grad_evals = W.grad_evals;
  res->poisson_solves = W.poisson_solves;
  res->cg_iters = W.cg_iters;
  res->matvecs = W.matvecs;
  res->status = status;
  if (u_out) std::memcpy(u_out, u.data(), sizeof(double) * N);
  if (phi_out) std::memcpy(phi_out, W.phi.data(), sizeof(double) * N);
  if (forces_out && prm->hartree_on) or_forces(sys, prm, W.phi.data(), forces_out);
  return status;
}

}  // extern "C"
