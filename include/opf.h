/* opf.h -- C ABI of the MI355X pipe-flow time-step library.
 *
 * The library advances the incompressible Navier-Stokes equations in a
 * periodic pipe, discretised as in Section 2 of Willis, "The Openpipeflow
 * Navier-Stokes solver" (SoftwareX 6, 2017):
 *   A(r,theta,z) = sum_{|k|<K} sum_{|m|<M} A_km(r_n) exp(i(alpha k z + mp m theta))   (Eq. 1)
 * with finite differences on N radial points (9-point stencils), 3/2
 * dealiasing on a 3K x 3M grid, pseudospectral nonlinear terms, a
 * pressure-Poisson equation with an influence-matrix boundary correction,
 * banded LU per Fourier mode for the implicit viscous terms and a
 * second-order predictor-corrector time step.
 *
 * Units: pipe radius R = 1, laminar centre-line speed U_cl = 1; Re = U_cl R / nu
 * (equal to the bulk-velocity / diameter Reynolds number of the paper).
 *
 * Conventions common to every call
 *  - Return value: opf_status, 0 (OPF_OK) on success.  No call aborts or throws.
 *  - Device pointers ("_dev") are HIP device memory owned by the caller; the
 *    library never frees them and keeps no pointer to them after the call,
 *    except the workspace given to opf_create, which it uses until
 *    opf_destroy.  Host pointers ("_host") are read or written synchronously.
 *  - Work is enqueued on the HIP stream given to opf_create and is
 *    asynchronous unless a call returns host values (stated per call).
 *  - External spectral layout of a vector field (state, nonlinear term,
 *    right-hand side): complex128, interleaved (re, im), shape
 *    [3][M][2K-1][N], components (u_r, u_theta, u_z), azimuthal index
 *    m = 0..M-1 (wavenumber mp*m), axial index k = -(K-1)..K-1 stored at
 *    position k+K-1, radial node n = 0..N-1 ascending (r[N-1] = 1).  Negative m
 *    follow from reality, A(-m,-k) = conj(A(m,k)).  A scalar field (pressure)
 *    has shape [M][2K-1][N].
 */
#ifndef OPF_H
#define OPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OPF_OK = 0,
    OPF_E_INVALID = -1,     /* bad argument or parameter set                      */
    OPF_E_NOMEM = -2,       /* workspace too small                                */
    OPF_E_HIP = -3,         /* a HIP runtime call failed (message: opf_last_error) */
    OPF_E_UNSUPPORTED = -4, /* size or option not implemented                      */
    OPF_E_NUMERIC = -5,     /* non-finite values, or an unstable factorisation     */
    OPF_E_STATE = -6        /* called before opf_set_state                         */
} opf_status;

enum { OPF_FP64 = 0, OPF_MIXED = 1 };
enum { OPF_SOLVE_PRED = 0, OPF_SOLVE_CORR = 1, OPF_SOLVE_RAW = 2 };

/* Problem definition (Section 2: domain [0,1] x [0,2pi/mp) x [0,2pi/alpha),
 * N radial points, |m| < M, |k| < K).
 *  N        radial points, 12 <= N <= 64
 *  M, K     Fourier modes |m| < M, |k| < K; 3M and 3K must factor into 2s and
 *           3s (the dealiased grid is 3K x 3M), 2 <= M <= 64, 2 <= K <= 64
 *  mp       azimuthal periodicity (rotational symmetry order), >= 1
 *  stencil  finite-difference points, must be 9
 *  alpha    axial wavenumber (pipe length 2pi/alpha), > 0
 *  Re       Reynolds number, > 0
 *  dt       time step, > 0
 *  c        implicitness of the viscous terms, 0.5 gives second order
 *  n_corr   corrector iterations per step, >= 1
 *  fixed_flux  1: hold the flux at its laminar value 1/4 (pressure gradient
 *           4(1+beta)/Re adjusts); 0: fixed pressure gradient 4/Re
 *  precision OPF_FP64, or OPF_MIXED (transforms and products in FP32, radial
 *           solves and influence correction in FP64)
 *  nonlinear 1; 0 drops u x omega (linear Stokes step, for tests)
 *  r_nodes  host array of N increasing nodes in (0,1] with r[N-1] = 1, or NULL
 *           for the default Chebyshev points r_n = cos(pi (N-n)/(2N-1)), n=1..N
 *           (read during opf_create only). */
typedef struct {
    int32_t N, M, K, mp, stencil;
    double alpha, Re, dt, c;
    int32_t n_corr, fixed_flux, precision, nonlinear;
    const double* r_nodes;
} opf_params;

/* Global diagnostics (Section 3.2: kinetic energy E, energy input from the
 * driving pressure gradient I, dissipation D; laminar values for
 * normalisation), plus wall shear tau_w = -du_z/dr of the mean flow at r = 1,
 * flux = int_0^1 u_z,00 r dr and the pressure-gradient excess beta.
 * g_norm: largest boundary-condition residual over all modes of the state,
 * max |g_i| of g = (u+(1), u-(1), u_z(1), div u(1)) (Section 2: the influence
 * matrix drives it to round-off).  div_max: largest |div u| over all modes
 * and interior nodes (finite-difference divergence).  cfl: dt times the
 * largest |u_r|/dr_n + |u_theta|/(r_n dtheta) + |u_z|/dz over the dealiased
 * physical grid, dtheta = 2 pi/(mp 3M), dz = 2 pi/(alpha 3K), dr_n the
 * distance from r_n to its nearer radial neighbour (-r_0 for n = 0). */
typedef struct {
    double E, I, D, tau_w, flux, beta;
    double E_lam, I_lam, D_lam;
    double g_norm, div_max, cfl;
} opf_diag;

typedef struct opf_ctx opf_ctx;

/* Fill *p with the tiny test case defaults (N=24, M=K=8, mp=1, alpha=1.25,
 * Re=2400, dt=0.01, c=0.5, n_corr=1, fixed flux, FP64, nonlinear). */
opf_status opf_default_params(opf_params* p);

/* Create-time radial tables computed on the host only (no device needed):
 * nodes r[N], quadrature weights quad[N] of int_0^1 g(r) r dr for g even in
 * r, folded 9-point first / second derivative weights d1, d2 [2][N][9]
 * (index 0: even axis parity, 1: odd) acting on columns s0[n]..s0[n]+8.
 * Any output pointer may be NULL.  Section 2: radial finite differences on a
 * 9-point stencil, nodes bunched towards the wall. */
opf_status opf_tables(const opf_params* p, double* r, double* quad, double* d1, double* d2,
                      int32_t* s0);

/* Bytes of device workspace opf_create needs for *p (tables, state, buffers). */
opf_status opf_workspace_size(const opf_params* p, size_t* bytes);

/* Build grid, finite-difference weights, quadrature, banded LU factors of every
 * radial operator, influence-matrix data and FFT tables, upload them into the
 * caller's workspace (>= opf_workspace_size bytes, 256-byte aligned) on
 * `hip_stream` (a hipStream_t; NULL = default stream).  Synchronises.
 * Returns OPF_E_NUMERIC if an LU factor shows element growth (unstable without
 * pivoting).  *out is valid until opf_destroy. */
opf_status opf_create(const opf_params* p, void* dev_workspace, size_t bytes,
                      void* hip_stream, opf_ctx** out);
opf_status opf_destroy(opf_ctx* ctx);

/* Radial nodes in use (host array of N doubles). */
opf_status opf_get_nodes(const opf_ctx* ctx, double* r_host);

/* Copy a state (external layout, complex128) into / out of the context. */
opf_status opf_set_state(opf_ctx* ctx, const void* u_dev);
opf_status opf_get_state(opf_ctx* ctx, void* u_dev);

/* Advance the state by nsteps predictor-corrector steps (Section 2):
 * N^n = (u x omega)(u^n); u^p = S(R0); N^p = (u x omega)(u^p); u^{n+1} = S(R1),
 * R0 = [1/dt + (1-c)L/Re] u^n + N^n + f, R1 = [..] u^n + c N^p + (1-c) N^n + f.
 * The steps run as captured hipGraphs: one launch per 8 steps, then one per
 * remaining step; changing dt, the wall velocity or the rotation drops them.
 * Asynchronous on the context's stream. */
opf_status opf_step(opf_ctx* ctx, int32_t nsteps);

/* Dealiased nonlinear term N = u x omega, omega = curl u (Section 2.2:
 * pseudospectral, 3/2 rule).  u_dev, n_dev: external layout, complex128.
 * Uses the context's scratch buffers; the state is not changed. */
opf_status opf_nonlinear(opf_ctx* ctx, const void* u_dev, void* n_dev);

/* omega = curl u by the radial finite differences (external layout). */
opf_status opf_vorticity(opf_ctx* ctx, const void* u_dev, void* w_dev);

/* One substep solve S (Section 2.2: pressure-Poisson equation, banded LU per
 * Fourier mode, influence-matrix correction so that g = 0; fixed flux on the
 * (0,0) mode; m = 0 made Hermitian).
 *  kind OPF_SOLVE_RAW : rhs_dev = R (3 fields, external layout); u = S(R)
 *  kind OPF_SOLVE_PRED: rhs_dev = N^n; R = [1/dt + (1-c)L/Re] u^n + N^n + f
 *                       with u^n the context's state
 *  kind OPF_SOLVE_CORR: rhs_dev = [N^n ; N^p] (6 fields);
 *                       R = [..] u^n + c N^p + (1-c) N^n + f
 * u_out_dev: 3 fields (external layout); p_out_dev: pressure head
 * [M][2K-1][N] complex128 or NULL.  The state is not changed. */
opf_status opf_radial_solve(opf_ctx* ctx, int32_t kind, const void* rhs_dev,
                            void* u_out_dev, void* p_out_dev);

/* Travelling-wave residual (Section 2: Newton-Krylov for invariant solutions;
 * a travelling wave is an equilibrium in a frame moving at its phase speed):
 *   F(x) = shift(Phi_T(x), -s) - x,
 * Phi_T = round(T/dt) steps, shift(A, s)_k = A_k exp(-i alpha k s) moves the
 * pattern downstream by s.  x_dev, F_dev: external layout; the context's
 * state is overwritten.  *norm_out (host, synchronises): energy norm of F,
 * sqrt(sum_k sum_{m>=0} c_m sum_n w_n |F_mk(r_n)|^2), c_0 = 1, c_m = 2. */
opf_status opf_newton_residual(opf_ctx* ctx, const void* x_dev, double T,
                               double shift, void* F_dev, double* norm_out);

/* Advance nsteps steps like opf_step but with every kernel launched on its
 * own (for measurement), through hipExtLaunchKernel with a start and a stop
 * event tied to that kernel's dispatch, so the times exclude the gaps
 * between launches.  ms[5] / launches[5]
 * receive the summed device time and launch count of the z-inverse
 * transform, theta transform + product, z-forward transform, predictor solve
 * and corrector solve kernels.  Synchronises. */
opf_status opf_profile_steps(opf_ctx* ctx, int32_t nsteps, double* ms, int32_t* launches);

/* Energy inner product of two external-layout fields (host result,
 * synchronises): sum_k sum_{m>=0} c_m sum_n w_n Re(a conj b), c_0 = 1,
 * c_m = 2, w_n the radial quadrature weights of int_0^1 f r dr. */
opf_status opf_vec_dot(opf_ctx* ctx, const void* a_dev, const void* b_dev, double* out_host);

/* y = a x + b y over a whole external-layout field (complex128, real a, b);
 * b = 0 overwrites y without reading it. */
opf_status opf_vec_axpby(opf_ctx* ctx, double a, const void* x_dev, double b, void* y_dev);

/* Learned preconditioner network (declared below). */
typedef struct opf_mlp opf_mlp;

/* Newton-Krylov search for a travelling wave (Section 2: Newton solver for
 * invariant solutions; Section 3.2: a travelling wave is an equilibrium in a
 * frame moving with its phase speed c_w): solves
 *   F(x, c_w) = shift(Phi_T(x), -c_w T) - x = 0
 * by Newton steps, each with restarted GMRES(gmres_m) on the linearised
 * system (J v by the forward difference (F(X + eps V) - F(X)) / eps,
 * eps = fd_eps max(||X||, 1) / ||V||), and a backtracking line search on
 * ||F||.  x_dev (in/out, external layout) holds the guess and receives the
 * solution; *cw_inout (host) is the phase speed, in and out.  krylov_dev is
 * caller device memory of at least opf_nk_workspace_size bytes.  The
 * context's state is overwritten.  Synchronises.
 *
 * free_speed = 0: c_w stays as given (shift s = c_w T fixed).
 * free_speed != 0: c_w is an unknown too.  The unknowns are X = (x, c_w)
 * with the phase condition <d_z x, dx> = 0 on the update as the extra
 * equation (d_z = i alpha k; it removes the axial-shift direction, along
 * which shifted copies of a travelling wave are travelling waves too); the
 * inner product of extended vectors is the energy inner product plus the
 * product of the speed entries, and ||X|| includes c_w.  Where
 * ||d_z x|| <= speed_freeze ||x|| (default 1e-6; laminar flow is a
 * travelling wave of every speed, so the speed direction is null there) a
 * Newton step keeps c_w and solves for x alone (report.frozen_steps).
 *
 * precond: NULL for plain GMRES; otherwise flexible GMRES with right
 * preconditioning (Saad 1993), z_j = P(v_j) with P = opf_precondition of
 * that network (created for this context's grid; a speed entry passes
 * unchanged), one cycle of at most gmres_m products per Newton step.  Plain
 * GMRES is the fallback (unless no_fallback): a step whose preconditioned
 * cycle misses gmres_tol, or whose line search does not lower ||F||, is
 * solved again by restarted plain GMRES (report.fallbacks).
 * record_dev: NULL, or device memory for record_capacity pairs of
 * external-layout vectors; each product J z with a zero speed entry is
 * stored as pair i = (z at vector 2i, J z at vector 2i+1) until the
 * capacity is reached (training data for the network).
 * max_jvps caps the products of one Newton step.
 *
 * hookstep != 0 replaces restarts and the line search by the Krylov
 * trust-region step of the paper's Newton solver (Section 2, after
 * Viswanath 2007): one Arnoldi cycle from v_1 = -F/||F|| (up to gmres_m
 * products, stopping at the gmres_tol least-squares residual) gives
 * J V_k = V_{k+1} Hb; dX = V_k y with y from opf_hookstep_solve for the
 * current radius Delta.  rho = (||F||^2 - ||F(X+dX)||^2) / (||F||^2 - r^2)
 * (r the model residual): rho < 0.1 rejects the step and retries with
 * Delta = ||dX||/2 on the same basis (at most max_hook tries, then the
 * search stops unconverged); an accepted step doubles Delta (up to
 * tr_delta_max) if rho > 0.75 and ||dX|| >= 0.99 Delta, and sets
 * Delta = ||dX||/2 if rho < 0.25.  Not combined with precond (returns
 * OPF_E_UNSUPPORTED).
 * Errors: OPF_E_INVALID for null pointers, gmres_m or max_jvps < 1, a
 * non-finite *cw_inout or a negative record capacity; OPF_E_NOMEM for a
 * short krylov_dev; OPF_E_NUMERIC for a non-finite preconditioned vector,
 * a non-finite residual at x, or a line search whose shortest trial
 * (step/1024) still has one.  A trial point whose residual is not finite
 * (its trajectory left the range the explicit terms can follow) counts as
 * rejected: the line search halves the step, the hookstep halves Delta. */
typedef struct {
    int32_t gmres_m;     /* Krylov dimension per restart, e.g. 40             */
    int32_t max_newton;  /* Newton iterations                                  */
    int32_t max_jvps;    /* cap on Jacobian-vector products per Newton step    */
    double tol;          /* stop when ||F|| / ||x|| <= tol (e.g. 1e-8)        */
    double gmres_tol;    /* relative GMRES tolerance per Newton step           */
    double fd_eps;       /* relative finite-difference step, e.g. 1e-7        */
    opf_mlp* precond;
    void* record_dev;
    int32_t record_capacity;
    int32_t hookstep;      /* 0: restarted GMRES + line search; 1: hookstep  */
    double tr_delta0;      /* first trust radius (energy norm); <= 0: the
                              length of the first unconstrained step        */
    double tr_delta_max;   /* largest radius; <= 0: unbounded                */
    int32_t max_hook;      /* tries per Newton step; <= 0: 12                */
    int32_t free_speed;    /* 0: c_w fixed; 1: c_w solved for (phase condition) */
    int32_t no_fallback;   /* 1: no plain-GMRES fallback for precond           */
    double speed_freeze;   /* ||d_z x|| / ||x|| below which c_w is held; <= 0: 1e-6 */
} opf_nk_opts;

typedef struct {
    int32_t newton_iterations, gmres_iterations, jvps, converged;
    double residual;               /* final ||F|| / ||x||                    */
    double residual_history[32];   /* ||F|| / ||x|| after each Newton step   */
    int32_t recorded;              /* pairs written to record_dev            */
    int32_t precond_applies;       /* applications of the preconditioner     */
    int32_t residual_evals;        /* evaluations of F (each T/dt steps), JVPs excluded */
    int32_t hook_trials;           /* hookstep candidates evaluated          */
    int32_t stalled;               /* hookstep: max_hook tries all rejected  */
    double tr_delta;               /* hookstep: trust radius on return       */
    double speed;                  /* c_w on return (= *cw_inout)            */
    int32_t frozen_steps;          /* free_speed: steps taken at fixed c_w   */
    int32_t fallbacks;             /* precond: steps solved again plainly    */
} opf_nk_report;

/* The hookstep subproblem (host only, no device): y minimising
 * ||beta e_1 - Hb y|| subject to ||y|| <= delta, for the (k+1) x k matrix Hb
 * (host, row-major; k >= 1).  Through the SVD Hb = U S W^T (one-sided Jacobi)
 * with p = beta U^T e_1: y = W z, z_j = p_j s_j / (s_j^2 + mu) (z_j = 0 for
 * s_j <= 1e-14 max s), mu = 0 if that fits, else the mu > 0 with ||z|| =
 * delta (safeguarded Newton on 1/||z||).  Outputs: y_host[k], *mu_host and
 * *resid_host = ||beta e_1 - Hb y||.  delta may be +infinity. */
opf_status opf_hookstep_solve(const double* hb_host, int32_t k, double beta, double delta,
                              double* y_host, double* mu_host, double* resid_host);

/* Device bytes for opf_nk_solve: (gmres_m + 6) vectors, plus gmres_m more
 * (the preconditioned directions) when preconditioned != 0. */
opf_status opf_nk_workspace_size(const opf_ctx* ctx, int32_t gmres_m, int32_t preconditioned,
                                 size_t* bytes);
opf_status opf_nk_solve(opf_ctx* ctx, void* x_dev, double T, double* cw_inout, const opf_nk_opts* opts,
                        void* krylov_dev, size_t krylov_bytes, opf_nk_report* report);

/* ---- Relative periodic orbits by multiple shooting -------------------------
 * Section 2: the Newton solver has a multiple-shooting option (an orbit split
 * into sections) and uses the Krylov trust-region step.  Unknowns
 * X = (x_1 .. x_S, T, s): S states (external layout, contiguous in x_dev),
 * the period T and the axial shift s.  Each section runs n steps of
 * dt = T / (S n) (opf_set_dt is applied as T changes; the context's dt is
 * restored on return).  Residual G_i = Phi_{T/S}(x_i) - x_{i+1} (i < S),
 * G_S = shift(Phi_{T/S}(x_S), -s) - x_1.  free_T / free_s add the phase
 * conditions <xdot_1, dx_1> = 0 (xdot_1 = (Phi_dt(x_1) - x_1) / dt) and
 * <d_z x_1, dx_1> = 0 (d_z = i alpha k) on the update.  Inner product: the
 * energy inner product summed over sections plus the products of the T and s
 * entries.  J V is the forward difference of the whole residual,
 * eps = fd_eps max(||X||, 1) / ||V||, plus the phase rows.  The Newton step
 * is the hookstep of opf_nk_solve (one Arnoldi cycle of at most gmres_m
 * products, opf_hookstep_solve, the same trust-region rule).  Stops when
 * ||G|| / ||X|| <= tol.  x_dev, *T_inout, *shift_inout: guess in, solution
 * out.  The context's state is overwritten.  Synchronises. */
typedef struct {
    int32_t sections;      /* S >= 1                                            */
    int32_t steps;         /* n >= 1 steps per section                          */
    int32_t free_T, free_s;
    int32_t gmres_m, max_newton;
    double tol, gmres_tol, fd_eps;
    double tr_delta0;      /* <= 0: the first unconstrained step length          */
    double tr_delta_max;   /* <= 0: unbounded                                     */
    int32_t max_hook;      /* <= 0: 12                                            */
} opf_shoot_opts;

typedef struct {
    int32_t newton_iterations, products, residual_evals, hook_trials, converged, stalled;
    double residual;               /* final ||G|| / ||X||                    */
    double residual_history[32];
    double T, shift, tr_delta;
} opf_shoot_report;

/* Device bytes for opf_shoot_solve: (gmres_m + 6) S + 3 fields. */
opf_status opf_shoot_workspace_size(const opf_ctx* ctx, int32_t sections, int32_t gmres_m, size_t* bytes);
opf_status opf_shoot_solve(opf_ctx* ctx, void* x_dev, double* T_inout, double* shift_inout,
                           const opf_shoot_opts* opts, void* work_dev, size_t work_bytes,
                           opf_shoot_report* report);

/* ---- Stability: Arnoldi iteration on the linearised time-T map -------------
 * Floquet multipliers of an invariant solution x (Section 3: the leading
 * eigenvalue of a travelling wave): eigenvalues mu of
 * J = d shift(Phi_T(x), -s)/dx, growth rate log|mu| / T.  J v is the forward
 * difference (P(x + eps v) - P(x)) / eps, P(x) = shift(Phi_T(x), -s),
 * eps = fd_eps max(||x||, 1) / ||v||.  Arnoldi with modified Gram-Schmidt in
 * the energy inner product from v0 (normalised, any nonzero field), without
 * restart; every check_every products, at breakdown and after m products the
 * Ritz values (eigenvalues of the leading k x k Hessenberg block,
 * opf_hessenberg_eigvals) are ordered by decreasing modulus, then decreasing
 * imaginary part, and the search stops when the leading nev moved by at most
 * tol |mu_1| since the previous check.  work_dev: opf_arnoldi_workspace_size
 * bytes.  ritz_re/ritz_im (host, nev each) receive the leading Ritz values;
 * hess_host ((m+1) x m row-major, or NULL) the Hessenberg matrix.  The
 * context's state is overwritten.  Synchronises. */
typedef struct {
    int32_t products;    /* Jacobian products (each T/dt steps + one residual) */
    int32_t converged;   /* 1 if the tol test passed or the space is invariant */
    int32_t checks;      /* Ritz-value checks made                              */
} opf_arnoldi_report;
opf_status opf_arnoldi_workspace_size(const opf_ctx* ctx, int32_t m, size_t* bytes);
opf_status opf_arnoldi(opf_ctx* ctx, const void* x_dev, double T, double shift, const void* v0_dev, int32_t m,
                       int32_t nev, double tol, int32_t check_every, double fd_eps, void* work_dev,
                       size_t work_bytes, double* ritz_re_host, double* ritz_im_host, double* hess_host,
                       opf_arnoldi_report* report);

/* Eigenvalues of a k x k upper Hessenberg matrix (host only, no device):
 * Francis double-shift QR iteration with deflation at subdiagonal entries
 * below 2^-52 times the neighbouring diagonal, 2 x 2 blocks solved in closed
 * form.  h_host: row-major, entries below the subdiagonal ignored.  re/im
 * (host, k each) receive the eigenvalues in the order above (modulus, then
 * imaginary part, decreasing).  OPF_E_NUMERIC if the iteration does not
 * converge in 60 k double steps. */
opf_status opf_hessenberg_eigvals(const double* h_host, int32_t k, double* re_host, double* im_host);

/* Jacobian probes of the travelling-wave residual at x_dev (training data
 * for the learned preconditioner, in the layout opf_nk_solve records):
 * pair i = (z_i, J z_i) at vectors 2i, 2i+1 of pairs_dev.  z_i: independent
 * unit normals in every real and imaginary part (SplitMix64 of (seed, i) and
 * the element counter, Box-Muller), made the spectrum of a real field
 * (m = 0: A(0,-k) = conj A(0,k), A(0,0) real) and scaled to unit energy norm;
 * J z = (F(x + eps z) - F(x)) / eps, eps = fd_eps max(||x||, 1).
 * work_dev: 3 vectors of scratch.  The context's state is overwritten.
 * Synchronises. */
opf_status opf_probe_pairs(opf_ctx* ctx, const void* x_dev, double T, double shift, int32_t n,
                           uint64_t seed, double fd_eps, void* pairs_dev, void* work_dev);
/* opf_probe_pairs for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same pairs, bitwise, with no work_dev argument.  Its three work
 * vectors live in a file-scope device array of 16 MiB (3 fields of the
 * grid must fit: OPF_E_INVALID otherwise, before any device work), which
 * each device holds from the first call on it until the process ends; the
 * steps are launched kernel by kernel (no step graph is captured).  It
 * calls no hipMalloc, hipFree or allocating library routine.  Every call on
 * one device shares that device's array: calls that overlap on one device
 * (other threads or streams) race.  Synchronises. */
opf_status opf_probe_pairs_noalloc(opf_ctx* ctx, const void* x_dev, double T, double shift, int32_t n,
                                   uint64_t seed, double fd_eps, void* pairs_dev);

/* ---- Learned preconditioner (not part of the paper) ----------------------
 * A residual MLP, shared by every Fourier mode (m, k) of one grid and fed
 * only the mode's features, models the Newton-Krylov Jacobian on each mode
 * as -I plus a rank-R term,
 *   J_mk ~ -I + U_mk V_mk^H,   U_mk, V_mk: 3N x R complex,
 * acting on the mode's radial profile (element e = c N + n for component
 * c = u_r, u_theta, u_z and node n).  Near laminar flow the Jacobian couples
 * no two modes and differs from -I by a few slow, non-normal directions per
 * mode, which the rank-R term holds.  The preconditioner is the exact
 * inverse of that model (Sherman-Morrison-Woodbury, FP64):
 *   P(v)_mk = -v_mk - U (I_R - V^H U)^{-1} V^H v_mk = -v_mk + A_mk (B_mk^H v_mk).
 * Learning J rather than J^{-1} keeps the fit well conditioned: the
 * network's bfloat16-limited errors are not multiplied by the large gains
 * J^{-1} has along nearly neutral directions.  P is linear on every mode,
 * so flexible GMRES with it keeps the minimal-residual property of GMRES.
 * (m = 0, k < 0) is the conjugate of (0, -k) and (0, 0) keeps its real
 * part, so P maps real fields to real fields.
 *   Network (L residual layers of width H), one row per mode:
 *     h_0 = W_in x + b_in;  h_l = h_{l-1} + relu(W_l h_{l-1} + b_l);
 *     y = W_out h_L + b_out.
 *   x = 32 features of (mu, kappa) = (mp m, alpha k): 1, mu/48, kappa/40,
 *   |kappa|/40, sign kappa, (mu/48)^2, (kappa/40)^2, mu |kappa|/1920,
 *   one-hot of m for m < 8, one-hot of k for |k| <= 7, [|k| > 7].
 *   y = (U, V): U[e][j] at 2(e R + j) (+1 imaginary part), V likewise from
 *   6 N R on; dout = 12 N R rounded up to a multiple of 32.
 *   Dense layers run on the matrix cores: weights, x, h and back-propagated
 *   gradients enter each product rounded to bfloat16 (nearest even) and
 *   products accumulate in FP32; master weights, biases, activations,
 *   gradients, the Adam moments and U, V are FP32.
 *   Training pairs (z, J z) (as opf_nk_solve records them or
 *   opf_probe_pairs makes them): for mode q and pair p with s the RMS of the
 *   z_q profile (pairs with s = 0 skip), r = -z_q/s + U (V^H z_q/s) - (J z)_q/s;
 *   loss = mean over modes and pairs of |r|^2. */
typedef struct {
    int32_t width;      /* H: multiple of 32 in [32, 512] (256)              */
    int32_t layers;     /* L: 1..8 (4)                                       */
    int32_t rank;       /* R: 1..32 with 3 N R <= 3072 (8)                   */
    int32_t max_rows;   /* rows of the plain row calls (>= mode count used)  */
    uint64_t seed;      /* initial weights (SplitMix64 uniforms)             */
    float lr, beta1, beta2, adam_eps;  /* Adam (1e-3, 0.9, 0.999, 1e-8)      */
    float lr_final;     /* opf_mlp_train_pairs: cosine decay from lr to this
                           over the steps of one call (1e-3: constant)      */
} opf_mlp_config;

opf_status opf_mlp_default_config(opf_mlp_config* cfg);
/* Device bytes a network of this configuration needs for this context's grid. */
opf_status opf_mlp_workspace_size(const opf_ctx* ctx, const opf_mlp_config* cfg, size_t* bytes);
/* Create a network for ctx's grid (N, M, K, mp, alpha) in caller device
 * memory (256-byte aligned); work goes to ctx's stream and the context must
 * outlive the network.  Weights: U(-a, a), a = 1/sqrt(fan_in) (0.01 of that
 * for the output layer), biases 0, so P starts near -I.  Synchronises. */
opf_status opf_mlp_create(opf_ctx* ctx, const opf_mlp_config* cfg, void* dev_workspace, size_t bytes,
                          opf_mlp** out);
opf_status opf_mlp_destroy(opf_mlp* net);
opf_status opf_mlp_dims(const opf_mlp* net, int32_t* din, int32_t* dout, int64_t* n_params);
/* Parameters as one FP32 host array: W_in [H][din], b_in [H], then per
 * layer W_l [H][H], b_l [H], then W_out [dout][H], b_out [dout].  Setting
 * them clears the Adam state.  Synchronise. */
opf_status opf_mlp_set_params(opf_mlp* net, const float* host, int64_t n);
opf_status opf_mlp_get_params(opf_mlp* net, float* host, int64_t n);
/* The plain network on rows: y_dev [rows][dout] = net(x_dev [rows][din])
 * (FP32 device rows, rows <= max(max_rows, M(2K-1))). */
opf_status opf_mlp_forward(opf_mlp* net, const float* x_dev, int32_t rows, float* y_dev);
/* Squared-error loss sum_r w_r sum_j (y_rj - t_rj)^2 / sum_r w_r of one
 * batch of rows (w_dev NULL: w = 1) and its parameter gradient (host FP32,
 * parameter order); no update.  Synchronises. */
opf_status opf_mlp_gradient(opf_mlp* net, const float* x_dev, const float* t_dev, const float* w_dev,
                            int32_t rows, double* loss_host, float* grad_host);
/* Adam on that loss over consecutive batches of `batch` rows, `epochs`
 * passes in an order shuffled per pass; loss_host[epochs] (or NULL) gets
 * the mean batch loss of each pass; batches * epochs <= 65536.  Synchronises. */
opf_status opf_mlp_train(opf_mlp* net, const float* x_dev, const float* t_dev, const float* w_dev,
                         int32_t rows, int32_t batch, int32_t epochs, uint64_t shuffle_seed, float* loss_host);
/* Pair loss of the pairs idx_host[0..batch) of pairs_dev (npairs pairs,
 * opf_nk_opts.record_dev layout) and its parameter gradient (host FP32);
 * no update.  Synchronises. */
opf_status opf_mlp_pair_gradient(opf_ctx* ctx, opf_mlp* net, const void* pairs_dev, int32_t npairs,
                                 const int32_t* idx_host, int32_t batch, double* loss_host, float* grad_host);
/* Adam on the pair loss: `steps` steps of `batch` pairs, taken in order from
 * per-epoch shuffles (seed) of the npairs pairs; loss_host[steps] (or NULL)
 * gets each step's loss.  steps <= 65536, batch * steps <= 2^20.  Synchronises. */
opf_status opf_mlp_train_pairs(opf_ctx* ctx, opf_mlp* net, const void* pairs_dev, int32_t npairs, int32_t batch,
                               int32_t steps, uint64_t seed, float* loss_host);
/* The preconditioner's factor rows (A, B) for the grid's modes (host FP32
 * [M(2K-1)][dout], same layout as (U, V); host may be NULL) and the number
 * of modes whose I - V^H U is singular (those get P = -I).  Synchronises. */
opf_status opf_mlp_factors(opf_mlp* net, float* host, int64_t n, int32_t* singular_modes);
/* z_dev = P(v_dev) (external layout, complex128), on ctx's stream. */
opf_status opf_precondition(opf_ctx* ctx, opf_mlp* net, const void* v_dev, void* z_dev);
const char* opf_mlp_last_error(const opf_mlp* net);

/* Diagnostics of the current state (host struct; synchronises).  Returns
 * OPF_E_NUMERIC, with *out filled, when a value is not finite or cfl > 1. */
opf_status opf_diagnostics(opf_ctx* ctx, opf_diag* out);

/* ---- Forcing: Coriolis force ---------------------------------------------
 * Section 3.1: the Earth's rotation is modelled by adding the Coriolis force
 * to the nonlinear terms just after they are evaluated.  With the rotation
 * vector Omega = (ox, oy, oz) in Cartesian components (z the pipe axis,
 * theta measured from x), units U_cl / R, every later nonlinear term (steps,
 * opf_nonlinear, Newton residuals) is u x omega - 2 Omega x u, formed at the
 * points of the dealiased grid and truncated with it.  An Ekman number
 * E = nu / (2 Omega D^2) gives |Omega| = 1 / (8 E Re).  (0, 0, 0) switches
 * the force off (the default).  OPF_E_UNSUPPORTED for a transverse axis
 * (ox or oy nonzero) with mp != 1 (the force couples m to m +- 1), for
 * nonlinear = 0 and for an ensemble member.  The step graph is captured
 * again at the next opf_step. */
opf_status opf_set_rotation(opf_ctx* ctx, double ox, double oy, double oz);

/* ---- Boundary conditions through the influence-matrix vector g -------------
 * Section 2: the boundary conditions enter through the vector g, which the
 * influence matrix drives to its target.  A prescribed wall velocity b (the
 * target of u(1)) replaces no slip: b_host is host complex128 [3][M][2K-1]
 * (components r, theta, z; the external mode layout) or NULL for no slip.
 * For every mode other than (0,0) the correction solves A a = -(g(u_b) - g_b)
 * with g_b = (b_r + i b_theta, b_r - i b_theta, b_z, 0); mode (0,0) takes
 * b_theta and b_z as the Dirichlet values of its Helmholtz solves (the
 * fixed-flux correction keeps the flux).  m = 0, k < 0 values are replaced
 * by the conjugates of k > 0 and the (0,0) imaginary parts are dropped (a
 * real field); a nonzero (0,0) radial entry (net flux through the wall) is
 * OPF_E_INVALID.  Applies to steps, opf_radial_solve and everything built on
 * them; opf_diagnostics reports g_norm against b.  OPF_E_UNSUPPORTED for an
 * ensemble member.  Synchronises; the step graph is captured again. */
opf_status opf_set_wall_velocity(opf_ctx* ctx, const double* b_host);

/* ---- Automatic time-step control ------------------------------------------
 * Section 2: the predictor-corrector scheme runs with automatic time-step
 * control.  The paper gives no rule; the one implemented here:
 *  - Courant limit: with U = cfl / dt (cfl as in opf_diag), dt_c = C / U;
 *  - corrector limit: the last correction delta = ||u^{n+1} - u^p|| (energy
 *    norm of opf_vec_dot; u^p the iterate before the last corrector) is
 *    O(dt^2), so dt_e = dt sqrt(tau / delta);
 *  - every check_every steps: lim = min(dt_c, dt_e),
 *    new = min(dt_max, lim / (1 + h)); dt shrinks to new when dt > lim and
 *    grows to new when new > dt and (new >= (1 + h) dt or new == dt_max);
 *    new < dt_min is OPF_E_NUMERIC.  A new dt applies from the next step
 *    on; no step is repeated. */

/* Rebuild every dt-dependent table (Helmholtz factors, homogeneous
 * solutions, influence matrices, flux Green's function) for a new step size
 * dt > 0 and upload them on the context's stream (synchronises); the step
 * graph is captured again at the next opf_step.  The state is kept.
 * OPF_E_NUMERIC (context unchanged) if a factor fails; OPF_E_UNSUPPORTED for
 * an ensemble member (its step runs in the class graph). */
opf_status opf_set_dt(opf_ctx* ctx, double dt);

/* delta = ||u^{n+1} - u^p|| of the last step taken by opf_step (host result,
 * synchronises).  In mixed precision u^p is the FP32 iterate.  OPF_E_STATE if
 * no step was taken since opf_set_state or the buffer was reused since. */
opf_status opf_pc_difference(opf_ctx* ctx, double* out_host);

typedef struct {
    double courant;       /* C > 0: the CFL number to aim for (0.5)            */
    double pc_tol;        /* tau >= 0: limit on delta; 0 switches it off       */
    double dt_min;        /* > 0                                               */
    double dt_max;        /* >= dt_min; the context's dt must lie in between   */
    double grow;          /* h >= 0: headroom and growth threshold (0.1)       */
    int32_t check_every;  /* >= 1 steps between checks (10)                    */
} opf_dt_control;

typedef struct {
    int32_t steps, checks, changes;
    double t;             /* simulated time of the steps taken                 */
    double dt;            /* step size in force on return                      */
    double cfl, pc_diff;  /* at the last check                                 */
    double rebuild_ms;    /* host time spent in opf_set_dt                     */
} opf_dt_report;

/* nsteps steps under the control above (graph launches between checks; each
 * check synchronises).  dt_trace (host, nsteps doubles, or NULL) receives the
 * step size of every step.  *report is filled also on error.
 * OPF_E_UNSUPPORTED for an ensemble member. */
opf_status opf_step_adaptive(opf_ctx* ctx, int32_t nsteps, const opf_dt_control* ctl,
                             double* dt_trace_host, opf_dt_report* report);

/* ---- Ensembles of independent trajectories -------------------------------
 * Members with equal (N, M, K, mp, precision) form a class; every kernel of
 * the step runs once per class over all its members, and one step of every
 * class is a single captured graph launch.  Members may differ in Re, alpha,
 * dt, c and initial state.  Workspace: caller device memory of at least
 * opf_ensemble_workspace_size bytes (256-byte aligned); each member gets
 * its own slice. */
typedef struct opf_ensemble opf_ensemble;
opf_status opf_ensemble_workspace_size(const opf_params* members, int32_t count, size_t* bytes);

/* Tile shapes of one class of equal (N, M, K, mp, precision): gm consecutive
 * m per radial-solve workgroup (1, 2 or 4 with mp (gm - 1) + 3 <= 6), tz
 * axial points per theta-stage workgroup (2, 4 or 8) and ztile radial lines
 * per z-transform workgroup (4, 8 or 16), each while the longer radix pass
 * of the transform length fits the workgroup (tz r <= 64; ztile r <= 256,
 * with 256-thread z workgroups when ztile r > 128; r the larger radix of the
 * length's two-pass split: 16 for 192, 12 for 144 ... 3 for 6).  Results
 * never depend on the tiles, only the speed.  members and us_per_step are
 * informative. */
typedef struct {
    int32_t N, M, K, mp, precision;
    int32_t members;
    int32_t gm, tz, ztile;
    double us_per_step;
} opf_tiles;

/* tune_cache_json: NULL (default tiles), or the path of a tile cache written
 * by opf_autotune, opf_tile_cache_write or saved from opf_ensemble_tune:
 * classes found in it take its tiles.  A file that cannot be read or
 * parsed, or that holds inadmissible tiles, gives OPF_E_INVALID. */
opf_status opf_ensemble_create(const opf_params* members, int32_t count, void* dev_workspace,
                               size_t bytes, void* hip_stream, const char* tune_cache_json, opf_ensemble** out);
opf_status opf_ensemble_destroy(opf_ensemble* ens);
/* The context of member i (set/get state, diagnostics through the single-
 * trajectory calls; do not destroy it). */
opf_status opf_ensemble_member(opf_ensemble* ens, int32_t i, opf_ctx** out);
/* nsteps predictor-corrector steps of every member; one graph launch per step. */
opf_status opf_ensemble_step(opf_ensemble* ens, int32_t nsteps);
/* Autotuner (the batched step of an ensemble, one graph launch per step;
 * not in the paper): for each class, time nsteps batched steps of the class
 * over the admissible values of each tile dimension in turn (gm, then tz,
 * then ztile, each from the best so far), keep the fastest, and write the
 * choice as a tile cache (JSON, the format opf_ensemble_create reads, with
 * every timed candidate) into `report` (host, may be NULL).  Members that
 * have a state advance by the timed steps (the cost is data-independent);
 * members without one run on laminar flow and have no state afterwards.
 * Synchronises. */
opf_status opf_ensemble_tune(opf_ensemble* ens, int32_t nsteps, char* report, size_t report_bytes);
/* The current tiles of each class (in order of first member): *nclasses
 * classes, the first `capacity` written to out (host). */
opf_status opf_ensemble_tiles(const opf_ensemble* ens, opf_tiles* out, int32_t capacity, int32_t* nclasses);
/* Offline tuning: times each of the ncls classes as a batch of 8 equal
 * members (opf_ensemble_tune, 5 steps per candidate) and writes the tile
 * cache to the file cache_json_out.  This call allocates: one device
 * workspace (opf_ensemble_workspace_size of the 8 ncls members) and one
 * stream on the current device, freed before it returns.  Synchronises. */
opf_status opf_autotune(const opf_params* cls, int32_t ncls, const char* cache_json_out);
/* Tile cache files (host only): write n entries (OPF_E_INVALID for
 * inadmissible tiles or an unwritable path); read one back, *n entries,
 * the first `capacity` into out. */
opf_status opf_tile_cache_write(const opf_tiles* tiles, int32_t n, const char* path);
opf_status opf_tile_cache_read(const char* path, opf_tiles* out, int32_t capacity, int32_t* n);
const char* opf_ensemble_last_error(const opf_ensemble* ens);
/* opf_probe_pairs with the probes' trajectories run as ensemble members:
 * every member must have the same parameters (one class, equal nodes); the
 * B members advance B probes per batch of graph launches (idle members of
 * the last batch run x).  The pairs equal those of opf_probe_pairs with the
 * same seed bitwise.  Uses the first member as the context; the members'
 * states are overwritten.  work_dev: 3 vectors.  Synchronises. */
opf_status opf_probe_pairs_ensemble(opf_ensemble* ens, const void* x_dev, double T, double shift, int32_t n,
                                    uint64_t seed, double fd_eps, void* pairs_dev, void* work_dev);

const char* opf_status_string(opf_status s);
const char* opf_last_error(const opf_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* OPF_H */
