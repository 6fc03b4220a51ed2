/*
 * biofilm.h -- C ABI of the MI355X (gfx950) solver for the per-step linear
 * systems of the 2D modified Cahn-Hilliard / Flory-Huggins biofilm-flow model
 * (McClanahan, Stegmeier, Sundermann, Doom, Kimn: "Parallel Simulations of
 * Biofilm Flow using the Modified Cahn-Hilliard Equation", arXiv:1811.11842).
 *
 * The paper discretises the model on a uniform vertex grid (Sec. 4: nodes
 * (i*dx, j*dy)), periodic in x and no-flux in y with two ghost layers given by
 * even reflection (Sec. 4, eq. discreteBC), which yields a sequence of sparse
 * systems A x = b solved by a preconditioned Krylov method (Sec. 4.1).  This
 * library holds the grid, applies the operators matrix-free and solves those
 * systems on one GPU.
 *
 * Conventions shared by every entry point
 *  - Grid: n intervals per side (n a power of two, 4 <= n <= 32768), h = 1/n.
 *    A field is a contiguous row-major float64 array of (n+1) rows by n
 *    columns, element (j, i) at offset j*n + i: row j = y-node j (0..n),
 *    column i = x-node i (0..n-1; node n is the periodic image of node 0).
 *  - Field pointers are DEVICE pointers owned by the caller.  The library never
 *    frees them and keeps no reference after a call returns.  Inputs and
 *    outputs must not alias unless an argument is documented as in/out.
 *  - All work is enqueued on the stream given at grid creation.  bf_apply,
 *    bf_ch_rhs, bf_pressure_rhs, bf_velocity_correct, bf_vcycle, bf_restrict
 *    and bf_prolong_add are asynchronous; the solves and bf_step return after
 *    the device work has finished (they read convergence scalars).
 *  - Inner products, norms and means use the trapezoid weights w_j = 1/2 on
 *    the wall rows j = 0 and j = n, 1 elsewhere; the reflected operators are
 *    self-adjoint in that inner product.
 *  - Return value: BF_OK (0); a positive "soft" status (outputs hold the best
 *    iterate, stats are filled); or a negative error (outputs unspecified,
 *    bf_last_error() describes it).  A grid handle is not thread-safe.
 */
#ifndef BIOFILM_H
#define BIOFILM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bf_grid bf_grid;

enum bf_status {
  BF_OK = 0,
  BF_NOT_CONVERGED = 1,   /* maxit reached before the tolerance            */
  BF_AT_FLOOR = 2,        /* recursive residual met rtol; the true one is  */
                          /* at the float64 representation floor of the    */
                          /* iterate (above rtol): its rounding noise      */
  BF_EINVAL = -1,         /* bad argument (null pointer, n, option value)  */
  BF_ENOMEM = -2,         /* device allocation failed                      */
  BF_EHIP = -3,           /* HIP runtime error                             */
  BF_ENONFINITE = -4,     /* NaN/Inf met in a residual norm                */
  BF_EUNSUPPORTED = -5    /* entry point or option not available           */
};

enum { BF_F64 = 0 };
enum { BF_OP_LAP = 0, BF_OP_CH = 1, BF_OP_HELM = 2 };
enum { BF_KSP_CG = 0, BF_KSP_GMRES = 1 };
enum { BF_PC_NONE = 0, BF_PC_JACOBI = 1, BF_PC_MG = 2 };
enum { BF_SMOOTH_CHEBYSHEV = 0, BF_SMOOTH_JACOBI = 1 };
enum { BF_MG_F64 = 0, BF_MG_F32 = 1 };

/* Grid description (the paper's DMDA object of Sec. 4.1, Listing "Initializing
 * a 2D DMDA object": periodic x, reflected y, stencil width 2, one dof). */
typedef struct {
  int32_t n;        /* intervals per side, power of two, 4..32768          */
  int32_t dtype;    /* BF_F64                                              */
  void*   stream;   /* hipStream_t all work is enqueued on (0 = default)    */
} bf_grid_desc;

/* Krylov / preconditioner choice (Sec. 4.1, Listing "Creating PETSc KSP and
 * PC objects": GMRES + Jacobi in the paper; CG + multigrid by default here). */
typedef struct {
  int32_t ksp;          /* BF_KSP_CG or BF_KSP_GMRES                        */
  int32_t pc;           /* BF_PC_NONE, BF_PC_JACOBI or BF_PC_MG             */
  int32_t maxit;        /* iteration limit (>= 1)                           */
  int32_t restart;      /* GMRES restart length m (1..64)                   */
  int32_t smoother;     /* BF_SMOOTH_CHEBYSHEV or BF_SMOOTH_JACOBI          */
  int32_t degree;       /* smoothing sweeps before and after the coarse     */
                        /* correction (1..8); 0 = operator default (CH 3, P 2) */
  int32_t check_every;  /* read the residual norm on the host every k iters */
  int32_t max_restarts; /* residual replacements before declaring a floor   */
  double  rtol;         /* relative weighted residual ||b-Ax||/||b||        */
  double  ratio;        /* Chebyshev interval lmax/lmin; 0 = default        */
                        /* (CH 16, P 4)                                     */
  double  omega;        /* damped-Jacobi weight; 0 = default                */
  int32_t mg_precision; /* BF_MG_F64, or BF_MG_F32: the multigrid V-cycle   */
                        /* (smoothing, residuals, transfers, coarse tail)   */
                        /* runs on float32 fields while the Krylov method,  */
                        /* its residual and the iterate stay float64 (CG    */
                        /* keeps the plain beta: the float32 V-cycle is     */
                        /* symmetric up to rounding).                       */
                        /* The float32 hierarchy is allocated on first use. */
  int32_t reserved;     /* 0                                                */
} bf_solver_opts;

typedef struct {
  int32_t status;        /* same value as the call's return code           */
  int32_t iters;         /* Krylov iterations performed                     */
  int32_t restarts;      /* residual replacements performed                 */
  int32_t clamped;       /* bf_step: points where phi was clamped for mu    */
  double  rel_res;       /* recursively updated relative residual at exit   */
  double  rel_res_true;  /* ||b - A x||_W / ||b||_W recomputed at exit      */
  double  ms;            /* device time of the call (HIP events)            */
  double  floor_est;     /* expected rel_res_true of x rounded to float64:   */
                         /* sqrt(sum_W ulp(x)^2/12 * sum_j A_jk^2)/||b||_W;  */
                         /* BF_AT_FLOOR: rel_res_true <= 1.5 sqrt(k+1)       */
                         /* floor_est for an iterate built by k rounded      */
                         /* updates (CG iterations, GMRES cycles, constant-  */
                         /* mode corrections; twice that after a refinement  */
                         /* restart that stopped improving)                  */
} bf_solve_stats;

/* Parameters of the reduced semi-implicit step (dimensionless). */
typedef struct {
  double dt, M, kappa;   /* time step, mobility, gradient-energy coefficient */
  double Npoly, chi;     /* Flory-Huggins N and chi (Sec. 5 parameter table) */
  double phi_lo, phi_hi; /* clamp of phi inside the logarithms               */
} bf_params;

/* Fill *o with the defaults for operator op (BF_OP_CH or BF_OP_LAP):
 * CG + multigrid, Chebyshev smoothing, rtol 1e-10, maxit 200. */
void bf_solver_opts_default(int32_t op, bf_solver_opts* o);

/* Allocate a grid and its multigrid hierarchy and Krylov workspaces on the
 * current HIP device (the grid's workspaces belong to the handle).
 * Errors: BF_EINVAL (n not a power of two in range, null out), BF_ENOMEM. */
int bf_grid_create(const bf_grid_desc* desc, bf_grid** out);
int bf_grid_destroy(bf_grid* g);
int bf_grid_shape(const bf_grid* g, int64_t* rows, int64_t* cols);

/* y = L x (op = BF_OP_LAP, 5-point Laplacian: the paper's matrix row 4, -1,
 * -1, -1, -1 of Sec. 4.1 scaled by -1/h^2) or y = x + c * L^2 x (op =
 * BF_OP_CH, the 13-point Cahn-Hilliard operator; c = dt*M*kappa, Sec. 2.2
 * eq. modCH), ghosts by eq. discreteBC, periodic x; or y = x - c * L_D x
 * (op = BF_OP_HELM, the momentum predictor's Helmholtz operator: interior rows
 * 1..n-1 read the wall rows 0 and n as Dirichlet values, the wall rows are
 * identity rows, y = x there).  Asynchronous. */
int bf_apply(bf_grid* g, int32_t op, double c, const double* x, double* y);

/* Solve (I + c L^2) x = b (Sec. 4.1: KSPSolve).  x: in = initial guess,
 * out = solution.  b = 0 gives x = 0.  c >= 0. */
int bf_solve_ch(bf_grid* g, double c, const double* b, double* x,
                const bf_solver_opts* o, bf_solve_stats* st);

/* Solve the Neumann pressure Poisson problem L p = rhs (Sec. 4, eq.
 * pressuresolve).  The weighted mean is removed from a copy of rhs (the null
 * space of constants, Sec. 4.1 Listing "Removing a nullspace"); rhs is not
 * modified.  p: in = initial guess, out = solution with zero weighted mean. */
int bf_solve_pressure(bf_grid* g, const double* rhs, double* p,
                      const bf_solver_opts* o, bf_solve_stats* st);

/* Solve the Helmholtz problem of the momentum predictor (Sec. 4, eq.
 * nopressmomentum with the viscous term implicit):
 *   x - beta * L_D x = b on the interior rows 1..n-1,  x = b on rows 0 and n,
 * i.e. Dirichlet walls whose values are given in the wall rows of b; L_D is
 * the 5-point Laplacian (row values of Sec. 4.1 times -1/h^2) reading the wall
 * rows as boundary values, periodic in x.  x: in = initial guess (its wall
 * rows are replaced by b's), out = solution.  beta >= 0.  MG-preconditioned
 * CG by default; the multigrid keeps every correction zero on the wall rows.
 * Synchronous; errors as bf_solve_ch. */
int bf_solve_helmholtz(bf_grid* g, double beta, const double* b, double* x,
                       const bf_solver_opts* o, bf_solve_stats* st);

/* Cahn-Hilliard operator with a variable mobility (the phi-dependent
 * mobility of the modified equation, Sec. 2.2 eq. modCH):
 *   y = x + c * L_m L x,  L_m f = div_h(m grad_h f)
 *     = n^2 sum over the four faces of m_face (f_nb - f), m_face = (m + m_nb)/2,
 * L the 5-point Laplacian; x, f and m reflected evenly across the walls
 * (eq. discreteBC), periodic x.  m: device field of node mobilities (> 0).
 * Evaluated in double-double, rounded once.  Asynchronous. */
int bf_apply_mob(bf_grid* g, double c, const double* m, const double* x, double* y);

/* Solve (I + c L_m L) x = b (the operator of bf_apply_mob).  L_m L is not
 * symmetric: the solve is GMRES (o->ksp must be BF_KSP_GMRES; o == NULL gives
 * GMRES(10) + multigrid, rtol 1e-10) right-preconditioned by a V-cycle
 * that rediscretises the operator with the node mobilities on every level
 * above 64 x 64 (m injected level to level) and uses I + c mbar L^2 below,
 * mbar the weighted mean of m rounded to 6 significant bits (with a Jacobi
 * or no preconditioner, that of I + c mbar L^2).  Residuals in double-double; the constant
 * mode is corrected as in bf_solve_ch (L_m conserves the weighted sum).
 * x: in = initial guess, out = solution.  Synchronous. */
int bf_solve_ch_mob(bf_grid* g, double c, const double* m, const double* b, double* x,
                    const bf_solver_opts* o, bf_solve_stats* st);

/* One Cahn-Hilliard step with the phi-dependent mobility m = M clamp(phi^n):
 *   b = phi + dt L_m mu_FH(clamp(phi)),
 *   (I + dt*kappa*L_m L) phi' = b,  solved in place (bf_solve_ch_mob) from
 * gamma phi, the least-squares multiple of phi for this operator (zero when
 * no positive gamma helps).  Synchronous; stats (may be NULL) receives the solve's
 * statistics and the clamp count. */
int bf_step_ch_mob(bf_grid* g, const bf_params* prm, double* phi, const bf_solver_opts* o,
                   bf_solve_stats* stats);

/* Momentum predictor of the projection method (Sec. 4, eq. nopressmomentum),
 * without the stress term R, viscosity nu = 1/(rho Re_a) constant:
 *   (I - theta*dt*nu*L_D) u* = u - dt*(u u_x + v u_y) + (1-theta)*dt*nu*L_D u
 *   (I - theta*dt*nu*L_D) v* = v - dt*(u v_x + v v_y) + (1-theta)*dt*nu*L_D v
 * on the interior rows (2h central differences; theta = 1/2 is the paper's
 * Crank-Nicolson, 1 backward Euler), with u* = 0 on the bottom wall, u* = U
 * on the top wall and v* = 0 on both.  u, v: the velocity v^n (device
 * fields); u*, v*: out (u may alias ustar and v may alias vstar, no other
 * aliasing); the solves start from u, v.  The two component solves run
 * concurrently on a second stream (as the two solves of bf_step).
 * stats[0] = x component, stats[1] = y component (may be NULL).
 * Synchronous.  dt > 0, nu >= 0, 0 <= theta <= 1. */
int bf_momentum_predict(bf_grid* g, double dt, double nu, double theta, double U,
                        const double* u, const double* v, double* ustar, double* vstar,
                        const bf_solver_opts* o, bf_solve_stats stats[2]);

/* b = phi + dt*M*L mu_FH(clamp(phi)), mu_FH(f) = ln(f)/N + 1/N - ln(1-f) - 1
 * + chi*(1-2f), clamp to [phi_lo, phi_hi] (phi itself untouched).  If
 * clamped != NULL it receives (device int32) the number of clamped points. */
int bf_ch_rhs(bf_grid* g, const bf_params* prm, const double* phi, double* b,
              int32_t* clamped_dev);

/* rhs = div_h(u, v) / dt with 2h central differences, v odd across the walls
 * (Sec. 4: v.n = 0), u periodic.  Asynchronous. */
int bf_pressure_rhs(bf_grid* g, double dt, const double* u, const double* v,
                    double* rhs);

/* u = ustar - dt * dp/dx, v = vstar - dt * dp/dy (central, p even across the
 * walls): the velocity update of Sec. 4, eq. velocityupdate, in the sign
 * convention L p = div(u*)/dt.  u may alias ustar and v may alias vstar. */
int bf_velocity_correct(bf_grid* g, double dt, const double* p,
                        const double* ustar, const double* vstar,
                        double* u, double* v);

/* One time step of the reduced biofilm-flow model:
 *   Cahn-Hilliard (Sec. 2.2, eq. modCH, constant mobility, the bulk
 *   Flory-Huggins potential explicit and the gradient-energy term implicit):
 *     b = phi + dt*M*L mu_FH(clamp(phi)),  (I + dt*M*kappa*L^2) phi' = b,
 *   then the projection of Sec. 4 (eqs. pressuresolve and velocityupdate):
 *     L p = div_h(u*, v*)/dt (weighted mean removed),  (u, v) = (u*, v*) -
 *     dt grad_h p.
 * phi: in phi^n, out phi^{n+1} (the solve starts from gamma phi^n, gamma
 * minimising the initial residual, or from zero when no gamma helps --
 * nothing is carried over between calls); p: out (zero initial guess); u, v:
 * out (both may be NULL to skip the velocity correction; u may alias u*
 * and v may alias v*, neither may alias phi).  stats[0] = Cahn-Hilliard solve, stats[1] =
 * pressure solve (may be NULL).  ch / pr may be NULL for the defaults.  The
 * parameters and both options are checked before anything is written: a
 * BF_EINVAL return leaves phi, p, u and v as they were.  The two solves are
 * independent and run concurrently (the pressure half on a second stream).
 * Synchronous. */
int bf_step(bf_grid* g, const bf_params* prm, double* phi, const double* ustar,
            const double* vstar, double* p, double* u, double* v,
            const bf_solver_opts* ch, const bf_solver_opts* pr,
            bf_solve_stats stats[2]);

/* One Cahn-Hilliard step with explicit advection (the flux div(phi v) of
 * Sec. 2.2, eq. modCH):
 *   b = phi + dt*M*L mu_FH(clamp(phi)) - dt*D(phi; u, v),
 *   D(phi; u, v) = div_h(phi*u, phi*v)  (2h central, phi even and v odd
 *   across the walls),
 *   (I + dt*M*kappa*L^2) phi' = b, solved in place from gamma phi (the
 *   least-squares multiple of phi for this b, zero when no positive gamma
 *   helps, as in bf_step).
 * u, v: device fields of the advecting velocity (both NULL: no advection,
 * the Cahn-Hilliard half of bf_step); they must not alias phi.  Synchronous;
 * stats (may be NULL) receives the solve's statistics and the clamp count. */
int bf_step_ch(bf_grid* g, const bf_params* prm, double* phi, const double* u,
               const double* v, const bf_solver_opts* o, bf_solve_stats* stats);

/* One Crank-Nicolson Cahn-Hilliard step with extrapolated chemical potential
 * (the paper's second-order time scheme, Sec. 4):
 *   (I + c/2 L^2) phi^{n+1} = (I - c/2 L^2) phi^n + dt*M*L mu_FH(clamp(phi*)),
 *   phi* = (3 phi^n - phi^{n-1}) / 2,  c = dt*M*kappa,
 * solved from gamma phi^n (as in bf_step_ch).  phi: in phi^n, out phi^{n+1}; phi_prev: in
 * phi^{n-1} (ignored when first != 0, then phi* = phi^n), out phi^n.  They
 * must not alias.  Synchronous; stats as in bf_step_ch. */
int bf_step_ch_cn(bf_grid* g, const bf_params* prm, double* phi, double* phi_prev,
                  int32_t first, const bf_solver_opts* o, bf_solve_stats* stats);

/* Reverse (adjoint) of one bf_step_ch, for gradients of a functional J of a
 * later state (the rollout's checkpointing is the caller's; the adjoint of a
 * rollout calls this once per step in reverse order).  With the plain
 * (Euclidean) transpose and lambda_in = dJ/dphi',
 *   eta = A^{-T} lambda_in = W A^{-1} W^{-1} lambda_in  (A = I + c L^2 is
 *         self-adjoint in the trapezoid inner product W; the transpose solve
 *         is the forward solve between two diagonal scalings),
 *   lambda_out = dJ/dphi_n = eta + dt*M*mu_FH'(phi_n) (L^T eta) - dt*D^T eta
 *         (mu_FH' = 1/(N phi) + 1/(1 - phi) - 2 chi, 0 where the clamp is
 *         active; L^T = W L W^{-1}; D^T the transpose of phi -> D(phi; u, v)),
 *   grads[0] += dt*M * sum (L^T eta)(1 - 2 clamp(phi_n))      (dJ/dchi),
 *   grads[1] += -dt * sum eta D(phi_n; du, dv)               (dJ/dU, where
 *         (du, dv) = d(u, v)/dU; both NULL: grads[1] unchanged).
 * phi_n is the state the forward step started from; u, v as in bf_step_ch
 * (both NULL: no advection).  lambda_out may alias lambda_in, not phi_n, u, v,
 * du or dv.  grads is a host array (may be NULL).  o / stats: options and
 * statistics of the transpose solve.  Synchronous.  Returns the solve's
 * status (BF_OK, BF_AT_FLOOR, BF_NOT_CONVERGED) or a negative error. */
int bf_adjoint_step(bf_grid* g, const bf_params* prm, const double* phi_n,
                    const double* u, const double* v, const double* du,
                    const double* dv, const double* lambda_in, double* lambda_out,
                    double grads[2], const bf_solver_opts* o, bf_solve_stats* stats);

/* ------------------------------------------------------------ ensemble
 * Many independent instances of bf_step, of uneven sizes and with their own
 * parameters (the batched-ensemble configuration: seeded sizes in
 * {128, 256, 512, 1024}, per-instance chi, dt, protrusion radius and noise).
 * Instances of equal size form a class; every operation on a class is one
 * launch over all its instances with per-instance coefficients and
 * convergence masks; classes run concurrently on streams of their own.  */
typedef struct bf_ensemble bf_ensemble;

/* n[count]: intervals per side of each instance, powers of two in
 * [128, 8192].  stream: hipStream_t the caller orders work on (0 = default).
 * Allocates all workspaces (per class: fields, multigrid hierarchy, Krylov
 * vectors) and tunes the stencil tile height per class by timing. */
int bf_ensemble_create(const int32_t* n, int32_t count, void* stream, bf_ensemble** out);
int bf_ensemble_destroy(bf_ensemble* e);

/* Packed field layout: every field of the ensemble (phi, u*, v*, p, u, v) is
 * one caller-owned device array of *total doubles; instance i occupies the
 * (n_i+1) x n_i row-major block starting at offsets[i] (host arrays). */
int bf_ensemble_layout(const bf_ensemble* e, int64_t* offsets, int64_t* total);

/* Size classes: their sizes, instance counts and tuned tile heights (host
 * arrays of at least as many entries as classes, each may be NULL). */
int bf_ensemble_info(const bf_ensemble* e, int32_t* nclasses, int32_t* class_n,
                     int32_t* class_count, int32_t* class_rpw);

/* One step of every instance (bf_step semantics: phi in/out, p out, u, v out
 * or both NULL; each instance's Cahn-Hilliard solve starts from its own
 * least-squares multiple of phi, its pressure solve from zero; nothing is
 * carried over between calls) with the parameters prm[i].  ch / pr: only rtol and maxit may
 * differ from the defaults (float64 CG with the default multigrid; others
 * return BF_EUNSUPPORTED); no refinement restarts.  stats[2 i] / stats[2 i + 1]
 * receive the Cahn-Hilliard / pressure solve of instance i.  ms (host, may be
 * NULL) receives the device time of the step in milliseconds: HIP events on
 * the caller's stream, from the marker every size class waits for before its
 * first kernel to the marker that waits for every class's last one.
 * Synchronous.  Returns the worst soft status or a negative error. */
int bf_ensemble_step(bf_ensemble* e, const bf_params* prm, double* phi, const double* ustar,
                     const double* vstar, double* p, double* u, double* v,
                     const bf_solver_opts* ch, const bf_solver_opts* pr, bf_solve_stats* stats,
                     double* ms);

/* z = V(r): one multigrid V-cycle (the preconditioner of the solves) of the
 * operator op with the options o (smoother, degree, ratio, omega), from a
 * zero initial guess.  Asynchronous.  Used to check the cycle itself. */
int bf_vcycle(bf_grid* g, int32_t op, double c, const bf_solver_opts* o,
              const double* r, double* z);

/* Grid-transfer operators between a fine grid of nf intervals and the coarse
 * grid of nf/2 (nf a power of two, 8 <= nf <= the grid's n):
 *   coarse = R fine       (R = 1/4 W_c^-1 P^T W_f, 7x7 stencil),
 *   fine  += P coarse     (tensor-product cubic interpolation).
 * Asynchronous. */
int bf_restrict(bf_grid* g, int32_t nf, const double* fine, double* coarse);
int bf_prolong_add(bf_grid* g, int32_t nf, const double* coarse, double* fine);

/* r = b - A x for op (BF_OP_LAP, BF_OP_CH or BF_OP_HELM with coefficient c).  accurate
 * != 0 evaluates the stencil sum in double-double (r correct to a few ulps
 * of r itself, whatever c/h^4); accurate == 0 uses plain float64.  If
 * rel_norm (host) is given it receives ||r||_W / ||b||_W; if floor_est (host)
 * is given (accurate only) it receives the expected value of that ratio for
 * the exact solution rounded to float64.  Synchronous when a host output is
 * requested, asynchronous otherwise.  r must not alias x. */
int bf_residual(bf_grid* g, int32_t op, double c, const double* b, const double* x,
                double* r, int32_t accurate, double* rel_norm, double* floor_est);

/* Allocation-free variant of bf_residual (accurate), for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  It takes no grid handle, allocates
 * nothing (no hipMalloc, hipFree or allocating library call) and never
 * synchronises:
 *   r = b - A x  for op (BF_OP_LAP, BF_OP_CH or BF_OP_HELM with coefficient
 *   c, as in bf_apply) on a grid of n intervals (power of two, 4 <= n <=
 *   32768; larger n returns BF_EINVAL), evaluated with the double-double
 *   stencil sum, and the device array norms[3] (caller-owned, 8-byte
 *   aligned): norms[0] = ||r||_W / ||b||_W, norms[1] = the float64 floor
 *   estimate of bf_residual's floor_est, norms[2] = ||b||_W (b = 0: the
 *   ratios divide by 1).
 * b, x, r: device fields of the (n+1) x n layout; r must not alias x or b.
 * stream: hipStream_t the work is enqueued on (0 = default).  Asynchronous.
 * Its reductions use a fixed device array of 264 KB per GPU that the library
 * holds until the process ends; calls on one GPU share it, so calls that
 * overlap on one GPU (other streams, other host threads) race. */
int bf_residual_noalloc(int32_t n, int32_t op, double c, const double* b, const double* x,
                        double* r, double* norms, void* stream);

/* One smoothing sweep of the multigrid preconditioner (the paper's Jacobi
 * preconditioner of Sec. 4.1, listing "Creating PETSc KSP and PC objects",
 * in the three-term Chebyshev form):
 *   xout = x + a D^{-1} (b - A x) + gcoef (x - xprev),
 * D = diag(A) (1 + 20 s, or 1 + 21 s on rows 1 and n-1, for the CH operator;
 * -4 n^2 for the Laplacian; 1 + 4 c n^2 for the Helmholtz operator, whose
 * wall rows the sweep leaves unchanged).  xprev may be NULL (taken as 0) and may alias
 * xout; xout must not alias x or b.  gcoef = 0, a = omega is damped Jacobi.
 * Asynchronous. */
int bf_smooth(bf_grid* g, int32_t op, double c, const double* x, const double* xprev,
              const double* b, double* xout, double a, double gcoef);

/* y = x for one field (16-byte aligned pointers), with the memory access
 * pattern of the stencil kernels (16 bytes per lane, coalesced rows): a
 * streaming kernel of known traffic (8 (n+1) n bytes each way), used to
 * calibrate hardware byte counters.  Asynchronous. */
int bf_copy(bf_grid* g, const double* x, double* y);

/* *out (host) = <x, y>_W.  Synchronises the grid's stream. */
int bf_wdot(bf_grid* g, const double* x, const double* y, double* out);

/* Device time of the Cahn-Hilliard CG step kernel (p' = z + beta p, q = A p',
 * the partials of <p', q>_W and, where the step does it, the deferred
 * x += alpha p), for measuring it inside a timed run.  enable > 0 clears the
 * record and starts recording a pair of HIP events on the grid's stream
 * around every enable-th launch of the kernel in the grid's Cahn-Hilliard
 * solves (bf_solve_ch, the Cahn-Hilliard half of bf_step, ...): 1 times
 * every launch; a larger period lowers the cost of the events (each leaves
 * the stream idle for a few microseconds).  enable == 0 stops; enable < 0 is
 * BF_EINVAL.  bf_grid_cg_timing_read synchronises the grid's stream and
 * returns the summed duration in ms of the recorded launches, their number,
 * and how many of them were the first step of a Krylov cycle (no beta p term,
 * no x update); it then clears the record.  Outputs may be NULL. */
int bf_grid_cg_timing(bf_grid* g, int32_t enable);
int bf_grid_cg_timing_read(bf_grid* g, double* total_ms, int64_t* launches,
                           int64_t* first_launches);
/* The same for the residual update of the same iterations (r -= alpha q,
 * the partials of ||r||_W^2 and, with the float32 V-cycle, the float32 copy
 * of r), recorded while bf_grid_cg_timing is on: synchronises the grid's
 * stream, returns the summed duration in ms and the number of recorded
 * launches, and clears that record.  Outputs may be NULL.  Each record (two
 * pooled events per recorded launch) grows until its read function, or
 * bf_grid_cg_timing with enable > 0, clears it. */
int bf_grid_rupdate_timing_read(bf_grid* g, double* total_ms, int64_t* launches);

/* Message of the last failure on this thread ("" if none). */
const char* bf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BIOFILM_H */
