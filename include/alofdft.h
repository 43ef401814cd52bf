/*
 * alofdft.h -- C ABI of the MI355X (gfx950) implementation of the augmented
 * Lagrangian orbital-free DFT ground-state solve of Suryanarayana & Phanish,
 * "Augmented Lagrangian formulation of Orbital-Free Density Functional Theory"
 * (arXiv:1405.6456).
 *
 * Problem statement (Sec. 2 and Sec. 4): M nuclei with positions R and valence
 * charges Z on a uniform grid of spacing h; the electron density is u^2 with
 * u >= 0, and the energy is the TFW kinetic energy (Eq. KineticEnergy), LDA
 * exchange-correlation, and the electrostatics rewritten through the potential
 * phi of the charge u^2 + b (Eq. ElectroststaticReformulation).  The ground state
 * minimises the energy subject to h^3 sum u^2 = N (the constraint C_h of Sec. 4),
 * solved by the augmented Lagrangian iteration (Sec. 3, Algorithm AugLag) around a
 * Polak-Ribiere nonlinear CG inner solver (Sec. 4); phi is re-solved for every
 * update of u (Eq. Poisson:Discretized, here by conjugate gradients).  Forces are
 * the Hellmann-Feynman expression of Eq. Force:Nuclei with the order-2n FD
 * gradient, plus the overlap correction of Appendix A.
 *
 * Conventions for every call:
 *   - Atomic units (Hartree, Bohr).
 *   - Grid arrays are dense n[0]*n[1]*n[2] doubles, node (i,j,k) at
 *     origin + h*(i,j,k), flat index i + n[0]*(j + n[1]*k) (x fastest).
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *     memory on the context's device (for example a torch tensor's data_ptr()).
 *   - The caller owns every input and output buffer; the library owns only the
 *     context (and server) workspace.  Outputs are complete when a call returns.
 *   - Every call returns an int status: ALOFDFT_OK (0), ALOFDFT_NOT_CONVERGED (1,
 *     outputs hold the last iterate), ALOFDFT_PENDING (2) or a negative error.
 *     No exception or exit crosses the ABI; alofdft_last_error() gives detail.
 *   - A context is used by one host thread at a time.
 */
#ifndef ALOFDFT_H
#define ALOFDFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ALOFDFT_OK 0
#define ALOFDFT_NOT_CONVERGED 1
#define ALOFDFT_PENDING 2
#define ALOFDFT_INVALID_ARGUMENT (-1)
#define ALOFDFT_OUT_OF_MEMORY (-2)
#define ALOFDFT_DEVICE_ERROR (-3)
#define ALOFDFT_NUMERICAL (-4)
#define ALOFDFT_REJECTED (-5)
#define ALOFDFT_CANCELLED (-6)

/* constraint methods (Sec. 3; Sec. 5.3.2 for the two comparison methods) */
#define ALOFDFT_METHOD_AUGMENTED_LAGRANGIAN 0
#define ALOFDFT_METHOD_PENALTY 1
#define ALOFDFT_METHOD_LAGRANGE 2

/* pseudocharge of a nucleus: the Gaussian -Z pi^-3/2 s^-3 exp(-r^2/s^2), or the
 * construction of Sec. 4, b_J = -(1/4 pi) Delta_h V_J on the nodes (order-2n stencil
 * applied to V_J = -Z erf(r/s)/r); both on the ball r <= r_cut */
#define ALOFDFT_PSEUDO_GAUSSIAN 0
#define ALOFDFT_PSEUDO_FD_LAPLACIAN 1

/* initial guess used when no u0 is passed: sqrt(N/V)(1 + 0.05 xi) (uniform with
 * seeded noise), or the superposition of atomic densities of Sec. 4 */
#define ALOFDFT_GUESS_UNIFORM 0
#define ALOFDFT_GUESS_ATOMIC 1

/* stopping rule of the outer loop: |C_h|/N < tol_constraint, or Algorithm AugLag's
 * energy change |E_q - E_(q-1)| / M < tol_energy (Sec. 3); both require the inner
 * problem solved to tol_grad */
#define ALOFDFT_STOP_CONSTRAINT 0
#define ALOFDFT_STOP_ENERGY_CHANGE 1

/* computational domain: the box of nodes, or the ellipsoid inscribed in it (Sec. 5.1:
 * Dirichlet conditions for u and phi on an ellipsoid inside the box): every node outside
 * the ellipsoid (centre and semi-axes (n_a - 1) h / 2 per axis, nodes on its surface
 * inside) is a Dirichlet node with u = phi = 0; the ellipsoid takes zero boundary values
 * for phi (phi_bc = ALOFDFT_BC_ZERO) */
#define ALOFDFT_DOMAIN_BOX 0
#define ALOFDFT_DOMAIN_ELLIPSOID 1

/* boundary values of phi: zero Dirichlet (Sec. 4) or the multipole expansion
 * (monopole + dipole + traceless quadrupole of u^2 + b about the box centre)
 * suggested in Sec. 5.1 */
#define ALOFDFT_BC_ZERO 0
#define ALOFDFT_BC_MULTIPOLE 1

/* arithmetic of the Poisson solve: all FP64, or FP32 stencil and CG vectors
 * inside an FP64 iterative-refinement loop (FP64 residual, dots, phi) */
#define ALOFDFT_FP64 0
#define ALOFDFT_FP32_REFINED 1

#define ALOFDFT_XC_NONE 0
#define ALOFDFT_XC_LDA_PZ 1

typedef struct alofdft_ctx alofdft_ctx;

typedef struct {
  int fd_half_width;      /* n of the order-2n stencils, 1..8 (default 6: order 12) */
  double lambda;          /* von Weizsaecker weight (default 0.2, Sec. 5) */
  int xc;                 /* ALOFDFT_XC_* (default LDA_PZ, Sec. 2) */
  double gauss_width;     /* s of b_J = -Z pi^-3/2 s^-3 exp(-r^2/s^2) (default 1.0) */
  double r_cut;           /* support radius of b_J (default 7.0) */
  int method;             /* ALOFDFT_METHOD_* (default augmented Lagrangian); LAGRANGE keeps
                             h^3 sum u^2 = N exactly, eta the Rayleigh quotient, Polak-Ribiere
                             directions projected orthogonal to u and a Brent search of the
                             energy along u cos(t) + sqrt(N) d sin(t) (Sec. 5.3.2; eta0, mu0,
                             kappa, tol_constraint and al_stop unused) */
  double eta0, mu0, kappa; /* Algorithm AugLag inputs (defaults -0.2, 1.0, 0.1, Sec. 5.3.1) */
  double tol_constraint;  /* stop the outer loop at |C_h|/N below this (1e-8) */
  double tol_grad;        /* inner stop: (h^3 sum g^2)^1/2 below this (1e-6) */
  double tol_poisson;     /* ||rhs - A phi||_2 / ||rhs||_2 below this (1e-10) */
  int phi_bc;             /* ALOFDFT_BC_* (default multipole) */
  int precision;          /* ALOFDFT_FP64 or ALOFDFT_FP32_REFINED */
  int max_outer;          /* outer (multiplier) iterations (30) */
  int max_inner;          /* nonlinear CG iterations per outer step (20000) */
  int max_cg;             /* CG iterations per Poisson solve (100000) */
  double sigma0;          /* secant probe step (0.5) */
  int max_secant;         /* secant steps per line search (4) */
  double secant_rel;      /* line-search slope reduction (0.1) */
  int restart_every;      /* nonlinear CG restart period (50) */
  int cg_check_every;     /* most CG iterations between host convergence checks (32); the
                             checks are timed by the observed residual reduction */
  uint64_t seed;          /* seed of the default initial guess (6456) */
  int pseudocharge;       /* ALOFDFT_PSEUDO_* (default Gaussian) */
  int initial_guess;      /* ALOFDFT_GUESS_* (default uniform) */
  double guess_width;     /* atomic guess: Gaussian width w of each atom's Z electrons, cut at 5w (1.5) */
  double guess_floor;     /* atomic guess: uniform floor as a fraction of N/V (1e-3) */
  int al_stop;            /* ALOFDFT_STOP_* (default constraint) */
  double tol_energy;      /* energy-change rule, Ha per atom (3.6749e-6 = 1e-4 eV, Sec. 5.3.1) */
  int domain;             /* ALOFDFT_DOMAIN_* (default box); ELLIPSOID needs phi_bc ZERO */
} alofdft_params;

typedef struct {
  int M;                  /* number of atoms, >= 1 */
  const double* R;        /* host, 3*M positions */
  const double* Z;        /* host, M charges */
  double N_elec;          /* number of electrons, > 0 */
  int n[3];               /* nodes per axis, each >= 2*fd_half_width+1 */
  double h;               /* grid spacing, > 0 */
  double origin[3];       /* position of node (0,0,0) */
} alofdft_system;

typedef struct {
  long long outer, inner, grad_evals, poisson_solves, cg_iters;
  long long matvec_fp64, matvec_fp32; /* stencil applications per precision */
  long long refinements;              /* FP64 outer residuals of the refined solve */
} alofdft_counts;

typedef struct {
  double E_total, E_TF, E_vW, E_xc, E_es, E_self, E_corr; /* Hartree */
  double eta_star;        /* Lagrange multiplier estimate (Algorithm AugLag output) */
  double C_h;             /* h^3 sum u^2 - N at the returned u */
  double grad_norm;       /* (h^3 sum g^2)^1/2 at the returned u */
  double poisson_relres;  /* relative residual of the last Poisson solve */
  double dE_last;         /* energy change of the last outer step */
  alofdft_counts counts;
  double time_total_ms, time_poisson_ms, time_grad_ms, time_setup_ms;
  int status;
} alofdft_result;

typedef struct {
  double E_TF, E_vW, E_xc, E_es, E_self, E_corr, E_total; /* Hartree */
  double C_h;             /* h^3 sum u^2 - N */
  double L;               /* E - eta C_h + C_h^2/(2 mu) */
  double grad_norm;       /* (h^3 sum g^2)^1/2 */
  long long cg_iters;
} alofdft_energy;

/* Status text for a return code. */
const char* alofdft_strerror(int status);

/* Detail of the last error on this context (never NULL). */
const char* alofdft_last_error(const alofdft_ctx* ctx);

/* Fills *p with the defaults listed above.  Returns ALOFDFT_OK or INVALID_ARGUMENT. */
int alofdft_default_params(alofdft_params* p);

/* Asks the call running on ctx (a solve, relaxation, Poisson solve or energy
 * evaluation) to stop: it returns ALOFDFT_CANCELLED at its next check (every host read
 * of a conjugate-gradient state, at most cg_check_every iterations apart, and every
 * nonlinear CG step), with its outputs not written.  If no call is running, the next
 * one on ctx stops at its first check.  The only call on a context that may be made
 * from another thread while it is in use.  INVALID_ARGUMENT for NULL. */
int alofdft_cancel(alofdft_ctx* ctx);

/* Creates a context on HIP device `hip_device` that enqueues all work on
 * `hip_stream` (a hipStream_t, borrowed, may be NULL for the null stream).  The
 * context allocates its device workspace lazily and owns it until destroy.  With
 * the environment variable ALOFDFT_PROGRESS set at creation, its solves write one
 * line to stderr per 100 nonlinear-CG steps and per augmented-Lagrangian step; with
 * ALOFDFT_TRACE=path, one line per Poisson solve is appended to that file (counts,
 * verdicts and exact hashes of the right-hand side and of phi before and after, which
 * copies three grid arrays to the host per solve: a diagnostic, slow). */
int alofdft_create(alofdft_ctx** out, int hip_device, void* hip_stream);
void alofdft_destroy(alofdft_ctx* ctx);

/* Ground state for fixed nuclei (Sec. 3, Algorithm AugLag; method = penalty
 * runs the same loop with eta fixed at 0, Sec. 5.3.2).
 *   u0         host, grid array, nullable: NULL uses sqrt(N/V)(1 + 0.05 xi),
 *              xi uniform in [-1,1) from SplitMix64(seed XOR node index).
 *   u_out, phi_out  host grid arrays, nullable.
 *   forces_out host 3*M, nullable: Hellmann-Feynman forces (Eq. Force:Nuclei,
 *              FD gradient of Sec. 4) plus the Appendix-A overlap correction.
 *   res        required.
 * Errors: INVALID_ARGUMENT for h <= 0, fd_half_width outside 1..8, n < 2n+1,
 * a grid whose padded FP64 array would reach 4 GiB (the kernels address arrays
 * with 32-bit byte offsets: cubes up to 768^3 nodes at n = 6), M < 1, N <= 0, an
 * atom whose r_cut ball leaves the box, non-finite input;
 * OUT_OF_MEMORY; DEVICE_ERROR; NUMERICAL when a non-finite value appears. */
int alofdft_solve(alofdft_ctx* ctx, const alofdft_system* sys, const alofdft_params* prm, const double* u0,
                  double* u_out, double* phi_out, double* forces_out, alofdft_result* res);

/* Same as alofdft_solve with device grid arrays (u0_dev nullable, u_out_dev and
 * phi_out_dev nullable) and host forces; all device work is ordered on the
 * context stream and complete on return. */
int alofdft_solve_device(alofdft_ctx* ctx, const alofdft_system* sys, const alofdft_params* prm,
                         const double* u0_dev, double* u_out_dev, double* phi_out_dev, double* forces_out,
                         alofdft_result* res);

/* Relaxation of the nuclei to the ground-state configuration (Sec. 4: Polak-Ribiere
 * nonlinear CG with a secant line search over the 3M positions).  The objective is
 * the ground-state energy E(R) of alofdft_solve, its gradient minus the forces;
 * every evaluation is a full solve at that geometry, warm-started from the previous
 * evaluation's u and phi.  One line-search step: a probe of length `probe` (largest
 * atom displacement, Bohr), then secant steps on the directional derivative
 * -F . d until |F . d| <= secant_rel |F0 . d| or max_secant evaluations; the last
 * evaluated point is accepted.  No step moves an atom more than max_move, nor its
 * r_cut ball out of the box.  Stops when every atom's |F| < ftol (Ha/Bohr). */
typedef struct {
  double ftol;       /* force threshold, Ha/Bohr (default 1e-3) */
  double max_move;   /* largest displacement of one atom per step, Bohr (0.3) */
  double probe;      /* largest displacement of the first trial of a line, Bohr (0.05) */
  int max_steps;     /* nonlinear CG steps (50) */
  int max_secant;    /* solves per line search (3) */
  double secant_rel; /* directional-derivative reduction that ends a line search (0.1) */
} alofdft_relax_params;

typedef struct {
  int status;        /* OK (converged), NOT_CONVERGED (step cap or an atom at the box edge), or an error */
  int steps;         /* nonlinear CG steps taken */
  int solves;        /* ground-state solves */
  double fmax;       /* largest |F| of an atom at R_out */
  double E_total;    /* energy at R_out */
} alofdft_relax_info;

/* Fills *p with the defaults above.  INVALID_ARGUMENT for NULL. */
int alofdft_default_relax_params(alofdft_relax_params* p);

/*   sys        the starting geometry (its R is not modified); prm as for alofdft_solve.
 *   u0         host grid array, nullable (as for alofdft_solve), guess of the first solve.
 *   R_out      host 3*M, required: relaxed positions.
 *   forces_out host 3*M, nullable: forces at R_out.
 *   res        required: the result of the solve at R_out.  info required.
 * Returns info->status.  Errors: those of alofdft_solve (from any evaluation);
 * INVALID_ARGUMENT for a null pointer or parameters out of range (ftol, max_move,
 * probe > 0; max_steps, max_secant >= 1; 0 < secant_rel < 1). */
int alofdft_relax(alofdft_ctx* ctx, const alofdft_system* sys, const alofdft_params* prm,
                  const alofdft_relax_params* rp, const double* u0, double* R_out, double* forces_out,
                  alofdft_result* res, alofdft_relax_info* info);

/* y = Delta_h x, the order-2*fd_half_width stencil of Eq. FD:Laplacian with zero
 * ghosts.  x_dev, y_dev: device grid arrays of n[0]*n[1]*n[2] elements of type
 * dtype (0 = double, 1 = float).  Returns INVALID_ARGUMENT for bad sizes. */
int alofdft_apply_laplacian(alofdft_ctx* ctx, const int n[3], double h, int fd_half_width, int dtype,
                            const void* x_dev, void* y_dev);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): alofdft_apply_laplacian without any
 * allocation.  Same arguments and result; the padded copies of x and y live in a
 * fixed 64 MiB device array of the library (held on every device the library runs on
 * until the process ends) instead of context workspace.  The work is enqueued on the
 * context stream and NOT waited for: y is complete when that stream reaches this point.
 * Every call on a device shares that device's array, so calls that overlap on one device
 * (other contexts or streams) race; the array keeps the last call's contents (the halo
 * is cleared by each call).  INVALID_ARGUMENT for bad sizes and for a grid whose two
 * padded arrays need more than 64 MiB (for example beyond about 110^3 in FP64). */
int alofdft_apply_laplacian_noalloc(alofdft_ctx* ctx, const int n[3], double h, int fd_half_width, int dtype,
                                    const void* x_dev, void* y_dev);

/* Discrete Poisson problem -(1/4pi) Delta_h phi = rho (Eq. Poisson:Discretized)
 * with boundary values `bc` (ALOFDFT_BC_*), solved by conjugate gradients in
 * `precision` (ALOFDFT_FP64 / FP32_REFINED) from the guess in phi_dev to
 * ||rhs - A phi||_2 < tol ||rhs||_2.  rho_dev, phi_dev: device grid arrays.
 * *iters (nullable) receives the CG iterations; *relres (nullable) the final
 * relative residual.  NOT_CONVERGED at max_cg.  INVALID_ARGUMENT for bad
 * arguments and for grids beyond the 4 GiB array limit of alofdft_solve. */
int alofdft_poisson(alofdft_ctx* ctx, const int n[3], double h, const double origin[3], int fd_half_width,
                    int bc, int precision, const double* rho_dev, double* phi_dev, double tol, int max_cg,
                    long long* iters, double* relres);

/* One energy and residual evaluation at u (Sec. 2 Eq. F with the quadrature of
 * Sec. 4; residual of Eq. EulerLagrangeDiscretized):
 *   g = -(lambda/2) Delta_h u + (V_K + V_xc + phi) u + (-eta + C_h/mu) u
 * (mu <= 0 drops the C_h/mu term).  phi_dev is the warm start on entry and the
 * potential of u on return.  u_dev, phi_dev, g_dev (nullable): device grid
 * arrays.  e: required. */
int alofdft_energy_gradient(alofdft_ctx* ctx, const alofdft_system* sys, const alofdft_params* prm,
                            const double* u_dev, double eta, double mu, double* phi_dev, double* g_dev,
                            alofdft_energy* e);

/* The initial guess a solve takes when no u0 is passed (prm->initial_guess): the
 * uniform guess sqrt(N/V)(1 + 0.05 xi) with xi from SplitMix64(seed XOR node), or the
 * superposition of atomic densities of Sec. 4 (each atom a Gaussian of Z_J electrons of
 * width guess_width cut at 5 widths, plus guess_floor N/V, scaled to h^3 sum u^2 = N).
 * u0_dev: device grid array (written).  Errors as alofdft_solve's validation. */
int alofdft_initial_guess(alofdft_ctx* ctx, const alofdft_system* sys, const alofdft_params* prm, double* u0_dev);

/* Nuclear pseudocharge b = sum_J b_J on the grid (Sec. 4 construction; Gaussian b_J or
 * the discrete Laplacian of V_J, prm->pseudocharge, support r_cut).  b_dev: device grid
 * array.  *self_energy (nullable) receives 1/2 sum_J h^3 sum b_J V_J. */
int alofdft_pseudocharge(alofdft_ctx* ctx, const alofdft_system* sys, const alofdft_params* prm, double* b_dev,
                         double* self_energy);

/* Forces for a given potential (Eq. Force:Nuclei with the order-2n FD gradient
 * of b_J, plus the Appendix-A correction).  phi_dev: device grid array;
 * forces_out: host 3*M. */
int alofdft_forces(alofdft_ctx* ctx, const alofdft_system* sys, const alofdft_params* prm, const double* phi_dev,
                   double* forces_out);

/* Stencil throughput measurement: applies Delta_h `reps` times over a rotation
 * of `nbuf` distinct (x, y) padded array pairs of n^3 elements (dtype 0/1) and
 * returns the mean kernel time per application in *ms_per_apply (HIP events on
 * the context stream).  Inputs are filled with a fixed pattern. */
int alofdft_bench_stencil(alofdft_ctx* ctx, const int n[3], int fd_half_width, int dtype, int reps, int nbuf,
                          double* ms_per_apply);

/* Launch tuning of a context.  stencil_variant selects the schedule of the
 * stencil passes (the residual pass of the energy gradient always uses the
 * register-addressed 64x4 kernel):
 *   -1  automatic, by op, precision and grid (all measured on MI355X): the plain
 *       Laplacian over (waves, rows per wave, planes ahead) = (4,2,1) below 150^3
 *       nodes; FP64 (16,1,1) from 150^3 and the forward-accumulating kernel (4,4,2)
 *       from 250^3; FP32 (16,2,1) from 250^3.  The CG first half (schedule 1)
 *       (8,1,1); the pipelined iteration (8,2,1).  Radii other than 6 take the same
 *       shapes.
 *   0..4  register-addressed kernels (order 12): 0: 64x8 nodes, two rows per
 *       thread, one plane ahead; 1: 64x4, one row, three ahead; 2: 64x8, one row,
 *       one ahead; 3: 64x8, one row, three ahead; 4: 64x4, one row, one ahead.
 *   5..10, 17..19  buffer-addressed streaming kernel (order 12), (waves, rows per
 *       wave, planes ahead): 5 (4,2,1), 6 (4,4,1), 7 (4,2,3), 8 (4,4,3), 9 (8,2,1),
 *       10 (2,8,1), 17 (8,1,1), 18 (16,1,1), 19 (16,2,1).
 *   11..16  forward-accumulating kernel (order 12): 11 (4,2,1), 12 (4,4,1),
 *       13 (4,2,2), 14 (8,2,1), 15 (4,4,2), 16 (8,4,1).
 *   100 + v  variant v with every z chunk swept upwards (v in 5..19; by default
 *       odd chunks are swept downwards).
 * The stencil launches of the CG iterations (schedules 1 and 2 of
 * alofdft_set_cg_schedule) take variants 5, 6, 7, 9, 10, 17, 18, 19 as above and
 * 11..16 as the forward-accumulating (4,2,1); every other value selects their
 * automatic shape.
 * target_blocks is the number of stencil workgroups to aim for (it sets the z
 * chunk length); 0 fills one round of the workgroups the device holds at once.
 * inner_tol_exp is the FP32 inner-solve residual reduction 10^-inner_tol_exp of
 * the refined Poisson solve (1..7).  Defaults -1, 0, 6.  INVALID_ARGUMENT outside
 * those ranges.  Every variant computes the same stencil; they differ in speed. */
int alofdft_set_tuning(alofdft_ctx* ctx, int stencil_variant, int target_blocks, int inner_tol_exp);

/* Schedule of the conjugate-gradient iterations of every Poisson solve of the
 * context (Sec. 4: the discrete Poisson problem solved by CG).  Schedules 0 and 1
 * take two launches per iteration; the second is x += alpha p, r -= alpha A p and
 * r.r.  The first:
 *   0  p = r + beta p formed on load (the stencil input is r and p over every
 *      tile's halo), A p by the stencil, p.Ap;
 *   1  A r by the stencil (one input array), then p = r + beta p and
 *      A p = A r + beta A p updated in place at each node, p.Ap.  In FP64 this
 *      launch also makes x += alpha p of the previous iteration (p is loaded there
 *      anyway) and the second launch updates only r; the launch that finds the
 *      solve converged makes the last x update.  In FP32 p and A p are kept as one
 *      array of (p, A p) pairs, one 8-byte access per node in both launches.
 *   2  one launch and one reduction per iteration, pipelined form (Chronopoulos-
 *      Gear scalars, Ghysels-Vanroose recurrences): w = A r, s = A p and z = A s
 *      are kept as vectors, the stencil is applied to the stored w (m = A w), then
 *      z = m + beta z, s = w + beta s, p = r + beta p, x += alpha p, r -= alpha s,
 *      w -= alpha z, with r.r and w.r reduced together; alpha = r.r / (w.r -
 *      beta r.r / alpha_prev).  FP64 solves only (the FP32 inner solves of the
 *      refined path use 1: in FP32 these recurrences stall near 1e-4).  r is a
 *      recurrence here, so a converged solve is restarted once from its true
 *      residual, which stops at once when the tolerance holds.
 *  -1  (default) automatic: 2 for FP64 solves on grids of at most 1.5e6 nodes
 *      (latency-bound iterations, where one launch instead of two pays), else 1.
 * All stop on the same relative residual; their iterates differ by rounding.
 * INVALID_ARGUMENT for a null context or another value. */
int alofdft_set_cg_schedule(alofdft_ctx* ctx, int schedule);

/* Measurement of the dominant kernels.  With sample_every > 0, every
 * sample_every-th conjugate-gradient iteration has each of its launches (schedules
 * 0 and 1: the stencil launch -- A r, p, A p and p.Ap with schedule 1 (and the
 * previous x += alpha p in FP64); p = r + beta p, A p and p.Ap with schedule 0 -- and
 * the update x += alpha p (not in FP64 with schedule 1), r -= alpha A p, r.r;
 * schedule 2: the single pipelined launch) carry a pair of HIP events that the
 * runtime stamps with the start and end of the kernel itself (hipExtLaunchKernel),
 * so the means are the kernel durations a kernel trace reports; iterations launched
 * after a solve has converged (which exit at once) are not counted.  sample_every = 0
 * stops sampling.  Calling it resets the statistics.  INVALID_ARGUMENT for a null
 * context or a negative value. */
int alofdft_profile_cg_kernel(alofdft_ctx* ctx, int sample_every);

/* Statistics of the sampled iterations for dtype 0 (FP64 CG) or 1 (FP32 inner CG of
 * the refined solve): number of timed iterations, mean kernel time of one iteration
 * in ms (all its launches), the grid points (n[0]*n[1]*n[2]) of the last timed one,
 * and, for the non-null optional pointers, the CG schedule (0..2, see
 * alofdft_set_cg_schedule; -1 if none) and the mean durations of the iteration's
 * first (stencil) and second (update; 0 for schedule 2) launch.  The first three
 * pointers required. */
int alofdft_cg_kernel_stats(alofdft_ctx* ctx, int dtype, long long* launches, double* mean_ms, long long* points,
                            int* schedule, double* first_ms, double* second_ms);

/* ------------------------------------------------------------------ serving
 * A request loop that solves independent ground-state requests (systems of any
 * grid size) concurrently on one GPU: up to max_slots requests are on the device
 * at once, each on its own HIP stream with its own resident work arrays, so their
 * kernels overlap; a queued request is admitted as soon as a slot is free and the
 * HBM footprint of the admitted requests stays within hbm_budget_bytes (continuous
 * batching).  A request's result does not depend on what else is running (every
 * reduction has a fixed order per request).  submit and poll are thread safe. */
typedef struct alofdft_server alofdft_server;

typedef struct {
  long long submitted, admitted, completed, rejected;
  int queued, running;
  double p50_ms, p99_ms, mean_ms; /* submit-to-finish latency of completed requests */
  double solves_per_s;            /* completed / (last finish - first submit) */
  double hbm_reserved_bytes;      /* footprints of running requests + arrays cached by the slots */
  long long cancelled;            /* requests ended by alofdft_server_cancel or destroy */
} alofdft_server_stats;

/* Device memory (bytes) one request of this system reserves while it runs: the
 * padded work arrays of the solve in both precisions plus the dense I/O arrays.
 * Returns 0 for an invalid system. */
size_t alofdft_footprint_bytes(const alofdft_system* sys, const alofdft_params* prm);

/* Starts max_slots (1..16) worker slots on HIP device `hip_device`.  OUT_OF_MEMORY
 * or DEVICE_ERROR if the streams cannot be created. */
int alofdft_server_create(alofdft_server** out, int hip_device, size_t hbm_budget_bytes, int max_slots);

/* Queues a request; the system (atoms copied) and params are copied before return.
 * *ticket identifies it.  REJECTED if its footprint exceeds the whole budget;
 * INVALID_ARGUMENT for an invalid system (same checks as alofdft_solve). */
int alofdft_server_submit(alofdft_server* srv, const alofdft_system* sys, const alofdft_params* prm,
                          uint64_t* ticket);

/* PENDING while the request is queued or running; otherwise its final status with
 * *res filled (and, when not NULL, u_out: host grid array, forces_out: host 3*M).
 * A finished request is released by the first poll that returns its status;
 * INVALID_ARGUMENT for an unknown ticket. */
int alofdft_server_poll(alofdft_server* srv, uint64_t ticket, alofdft_result* res, double* u_out,
                        double* forces_out);

int alofdft_server_get_stats(alofdft_server* srv, alofdft_server_stats* st);

/* Cancels a request: a queued one is removed at once, a running one stops at its
 * solve's next check (see alofdft_cancel); poll then returns ALOFDFT_CANCELLED.  A
 * request that has finished keeps its result.  INVALID_ARGUMENT for an unknown ticket. */
int alofdft_server_cancel(alofdft_server* srv, uint64_t ticket);

/* Workgroups per stencil launch of every slot (alofdft_set_tuning's target_blocks; 0 is
 * one round of resident workgroups).  Default ALOFDFT_SERVER_SLOT_BLOCKS: launches smaller
 * than a round leave the device room to run the slots' kernels side by side (measured on
 * the fcc1-3 stream with 4 slots at twice the sequential FP64 capacity: 0.93 solves/s and
 * p50/p99 7.0/15.1 s against 0.86 and 10.6/20.2 s at one round).  The shape of a launch
 * changes the order of its partial sums, so results depend on it (within the solver's
 * tolerance) but never on the other requests: a served result equals a context's solve with
 * the same target_blocks.  INVALID_ARGUMENT while any request is queued or running. */
#define ALOFDFT_SERVER_SLOT_BLOCKS 256
int alofdft_server_set_tuning(alofdft_server* srv, int target_blocks);

/* Stops the server: queued requests are cancelled, running ones stop at their next
 * check, then the workers exit and every slot's device memory is freed. */
void alofdft_server_destroy(alofdft_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* ALOFDFT_H */
