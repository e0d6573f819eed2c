/*
 * maxent.h -- C-ABI of the MI355X solver for the explicit finite-volume step of the
 * 5-moment (1D1V) and 14-moment (3V) maximum-entropy moment systems with the interpolative
 * closure (Boccelli, Kaufmann, Magin & McDonald, arXiv 2401.15233).
 *
 * One time step (Section 3 of the paper): primitive recovery, interface reconstruction
 * with one common limiter (Section 3.2), the sigma-limited interpolative closure
 * (Sections 2.3-2.4, Appendix A), approximate wave speeds (Section 5.1, Appendix B), the
 * HLL or Rusanov interface flux (Section 3.1), the BGK relaxation source (Sections
 * 2.3-2.4), ghost-cell boundary conditions (Section 6) and an explicit Runge-Kutta update
 * with the CFL time step (Sections 3 and 4.3).
 *
 * Conventions for every function below
 *   - extern "C", never throws, never aborts; returns MAXENT_OK (0) or a negative
 *     maxent_status.  maxent_last_error() then describes the failure.
 *   - Field arrays are float64, component-major, unpadded: value (v, j, i) at
 *     src[(v * ny + j) * nx + i], x fastest.  Component orders:
 *       14 primitives  [rho, u_x, u_y, u_z, P_xx, P_xy, P_xz, P_yy, P_yz, P_zz, q_x, q_y, q_z, R]
 *       14 conserved   [rho, rho u_i (3), E_ij = rho u_i u_j + P_ij (6, as P), F_i (3), G]
 *        5 primitives  [rho, u, P, q, r];  5 conserved [rho, rho u, rho u^2 + P, ...]
 *     with q_i = Q_ijj (twice the fluid heat flux) and R = R_iijj, gas constant 1.
 *   - Ownership: the library owns all device state (allocated in maxent_create, freed in
 *     maxent_destroy).  Caller buffers are only accessed during the call.
 *   - Streams: all device work is ordered on the stream given to maxent_create (NULL =
 *     the default stream).  A handle is not thread-safe.
 */
#ifndef MAXENT_H
#define MAXENT_H

#ifdef __cplusplus
extern "C" {
#endif

#define MAXENT_ABI_VERSION 4

typedef struct maxent_solver maxent_solver;

typedef enum {
  MAXENT_OK = 0,
  MAXENT_E_INVAL = -1,         /* bad argument; the solver state is unchanged            */
  MAXENT_E_NOMEM = -2,         /* device allocation failed                               */
  MAXENT_E_DEVICE = -3,        /* a HIP runtime call failed                              */
  MAXENT_E_NONFINITE = -4,     /* a cell centre became non-finite (info.fail_step)       */
  MAXENT_E_UNREALIZABLE = -5,  /* rho <= 0 or P not positive definite (info.fail_step)   */
  MAXENT_E_STATE = -6          /* call out of order (e.g. step before init_state)        */
} maxent_status;

enum { MAXENT_BC_TRANSMISSIVE = 0, MAXENT_BC_PERIODIC = 1, MAXENT_BC_REFLECTIVE = 2,
       MAXENT_BC_JET = 3 };
enum { MAXENT_FP64 = 0, MAXENT_FP32 = 1, MAXENT_MIXED = 2 };
enum { MAXENT_MINMOD = 0, MAXENT_VANALBADA = 1 };
enum { MAXENT_HLL = 0, MAXENT_RUSANOV = 1 };
enum { MAXENT_FE = 0, MAXENT_SSPRK2 = 1, MAXENT_MIDPOINT = 2 };
enum { MAXENT_TAU_LOCAL = 0, MAXENT_TAU_CONST = 1 };
enum { MAXENT_PRIMITIVE = 0, MAXENT_CONSERVED = 1, MAXENT_SIGMA = 2, MAXENT_CLOSING = 3 };
/* components per cell of a MAXENT_CLOSING read-back of the 14-moment system */
#define MAXENT_CLOSING_COMPONENTS_14 19

/* Problem definition.
 *   system        5 (1D1V, requires dim = 1) or 14.
 *   dim, nx, ny   1 or 2; ny = 1 when dim = 1.  nx, ny >= 4.
 *   x0..y1        domain; uniform cells dx = (x1-x0)/nx, dy = (y1-y0)/ny.
 *   bc[4]         XLO, XHI, YLO, YHI boundary kinds (MAXENT_BC_*).  PERIODIC must be set on
 *                 both sides of an axis.  JET (2D, 14 moments; Section 6): on a JET side,
 *                 the ghost cells of the boundary rows (x sides) or columns (y sides) whose
 *                 centre lies in [c - w/2, c + w/2] of a jet on that side hold the jet
 *                 Maxwellian; the others are transmissive.  Every JET side needs a jet.
 *   jets          up to 4: centre c along its wall (y on the x sides, x on the y sides),
 *                 width w, angle in degrees from +x toward +y, and jet_wall[k] (0 XLO,
 *                 1 XHI, 2 YLO, 3 YHI; that side must be JET).  The paper's crossed jets are
 *                 a jet on XLO at angle 0 and one on YLO at angle 90, both of width L/7.
 *   jet_mach, jet_rho, jet_T   the jet Maxwellian: |u| = M sqrt(5/3 T), P = rho T I,
 *                 q = 0, R = 15 p^2 / rho.
 *   tau_mode      LOCAL: tau = tau_ref (rho_ref/rho) sqrt(T_ref/T) at each cell centre, the
 *                 scaling of tau = (n sigma v_th)^-1 of Section 4; CONST: tau = tau_ref.   */
typedef struct {
  int system;
  int dim;
  int nx, ny;
  double x0, x1, y0, y1;
  int bc[4];
  int n_jets;
  double jet_yc[4], jet_width[4], jet_angle_deg[4];
  double jet_mach, jet_rho, jet_T;
  int tau_mode;
  double rho_ref, T_ref;
  int jet_wall[4];
} maxent_problem;

/* Numerics.
 *   precision     MAXENT_FP64; MAXENT_MIXED: state, primitive recovery, reconstruction,
 *                 HLL dissipation and update in FP64; closure, wave speeds and physical
 *                 fluxes of each face state in FP32 (the dimensionless closure is robust in
 *                 single precision, Section 3.3), re-evaluated in FP64 near the Junk
 *                 subspace (A < -1e-3, sigma < 1e-2) and the realizability boundary
 *                 (sigma > 0.999); MAXENT_FP32: every face-state evaluation (closure, wave
 *                 speeds, physical fluxes, the HLL / Rusanov combination) in FP32 with no
 *                 FP64 re-evaluation, state, primitive recovery, reconstruction, source and
 *                 update in FP64 (single solvers only; the batch takes FP64 or MIXED).
 *   order         1 (first order, cell states at faces) or 2 (MUSCL on primitives with one
 *                 common, most stringent limiter factor, Section 3.2).
 *   limiter       MINMOD or VANALBADA (the paper's choice).
 *   flux          HLL or RUSANOV (Section 3.1).
 *   integrator    FE, SSPRK2 (Heun) or MIDPOINT (Section 3).
 *   cfl           Courant number; dt = cfl dx / max Lambda (1D), cfl / max(Lambda_x/dx +
 *                 Lambda_y/dy) (2D), Lambda = max |lambda_min|, |lambda_max| at cell centres.
 *   sigma_lim     lower bound of the parabolic-mapping parameter (Appendix A), e.g. 1e-4.
 *   k_ws          wave-speed inflation factor k >= 1 (Section 5.1).
 *   positivity_fallback  1: a cell whose reconstructed face states along a direction have
 *                 rho <= 0 or a non-positive-definite P is reconstructed at first order.
 *   source_implicit  0: explicit BGK source.  1 (FE integrator only): point-implicit BGK
 *                 relaxation, the remedy the paper names for stiff collisions (Section 4.3,
 *                 Kn below about 1e-4): the transported state U_t = U + dt (fluxes) relaxes
 *                 by backward Euler, U_new = (U_t + h U_eq) / (1 + h), h = dt / tau, where
 *                 U_eq is the local Maxwellian of U_t and tau is evaluated from U_t (the
 *                 source keeps rho, rho u and the energy, so this is exact backward Euler for
 *                 the source).  Not available with the adjoint. */
typedef struct {
  int precision;
  int order;
  int limiter;
  int flux;
  int integrator;
  double cfl, sigma_lim, k_ws;
  int positivity_fallback;
  int source_implicit;
} maxent_numerics;

/* Per-call report of maxent_step. */
typedef struct {
  double t;                 /* simulated time after the call                         */
  double dt_last;           /* last time step taken                                  */
  long long steps;          /* steps taken since init_state                          */
  long long n_fallback;     /* positivity fallbacks since init_state                 */
  int fail_step;            /* first failing step index (1-based), 0 if none         */
  int fail_code;            /* bit 1: non-finite, bit 2: rho <= 0 / P not SPD        */
  long long n_fp64_states;  /* MIXED: face states re-evaluated in FP64 since init    */
  long long n_face_states;  /* MIXED, FP32: face states evaluated since init          */
  long long n_sigma_limited; /* cells of the current state whose unlimited sigma is
                                below sigma_lim (Appendix A: the closure then uses
                                sigma_lim); counted by maxent_get_info, -1 from
                                maxent_step                                          */
  double fp64_fraction;     /* share of face-state evaluations done in FP64: 1 for FP64,
                               n_fp64_states / n_face_states for MIXED, 0 for FP32      */
  int reduced;              /* the stage kernels carry only the moments the state's
                               symmetry leaves non-zero (maxent_set_reduced): 0 no,
                               1 planar (2D, ten moments), 2 axial (1D, seven moments)  */
  int reserved;
} maxent_info;

/* Allocate a solver.  `stream` is a hipStream_t (NULL for the default stream).
 * Errors: INVAL for an inconsistent problem/numerics (nothing allocated), NOMEM, DEVICE. */
int maxent_create(const maxent_problem* problem, const maxent_numerics* numerics,
                  void* stream, maxent_solver** out);

/* Set the state.  repr = MAXENT_PRIMITIVE or MAXENT_CONSERVED; src is a field array as
 * described above, on the host (src_on_device = 0) or the device (1).  Primitives are
 * converted to conserved moments on the device (the time-derivative terms of the moment
 * equations, Sections 2.3-2.4).  Sets t = t0, resets step and fallback counters and
 * computes the first CFL rate.  Errors: INVAL (null src, bad repr), UNREALIZABLE (a cell
 * with rho <= 0 or P not SPD; the state is loaded anyway), DEVICE. */
int maxent_init_state(maxent_solver* s, int repr, const double* src, int src_on_device,
                      double t0);

/* Advance n >= 0 steps.
 *   dt > 0        fixed time step;  dt <= 0: CFL time step from the cell-centre states.
 *   tau_ref       BGK reference collision time; tau_ref <= 0 switches the source off
 *                 (collisionless flow).
 *   t_end > 0     clip the last step so that t does not pass t_end; steps requested after
 *                 t_end is reached are no-ops.  t_end <= 0: no end time.
 * Work is enqueued on the solver's stream; the call synchronises once at the end to read
 * the status word.  On failure (NONFINITE / UNREALIZABLE) info->fail_step names the first
 * failing step, later steps of the call do nothing, and the state is the one after the
 * failing step.  info may be NULL. */
int maxent_step(maxent_solver* s, int n, double dt, double tau_ref, double t_end,
                maxent_info* info);

/* Copy out a field.  repr = PRIMITIVE or CONSERVED (nv x ny x nx doubles), SIGMA (the
 * unlimited parabolic-mapping parameter, ny x nx) or CLOSING: the closing moments of each
 * cell state, dimensional, at sigma_bar = max(sigma, sigma_lim) (eqs.
 * closure-14mom-Qijk-approx, -Rijkk-approx, -Sijjkk-approx; eq. closure-1D1V-s-approx):
 * 14 moments: MAXENT_CLOSING_COMPONENTS_14 x ny x nx doubles, in the order
 *   Q_ijk  xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz (10),
 *   R_ijkk xx xy xz yy yz zz (6), S_ijjkk x y z (3);
 * 5 moments: s (ny x nx).  dst is host (dst_on_device = 0) or device memory owned by the
 * caller.  Synchronises the solver's stream. */
int maxent_get_moments(maxent_solver* s, int repr, double* dst, int dst_on_device);

/* Number of components (5 or 14); time, step count and counters of a solver (also counts
 * the sigma-limited cells of the current state: one pass over the field).  Synchronises the
 * solver's stream. */
int maxent_num_vars(const maxent_solver* s);
int maxent_get_info(maxent_solver* s, maxent_info* info);

/* ------------------------------------------------------------------ batched 1D tubes
 * Many independent 1D 14-moment problems of uneven length advance together: each instance
 * has its own grid, collision time, end time and CFL time step.  The common settings come
 * from `common` (bc[0], bc[1], tau_mode, rho_ref, T_ref; other fields ignored) and
 * `numerics` (order 2, SSPRK2 or MIDPOINT, FP64 or MIXED).  The state is the concatenation
 * of the instances' fields: init_state / get_moments take [14][total cells] with instance
 * i occupying cells [sum_{k<i} n_k, sum_{k<=i} n_k).  tau_ref <= 0 makes an instance
 * collisionless. */
typedef struct {
  double x0, x1;            /* the instance's domain                                  */
  double tau_ref;           /* BGK reference collision time (<= 0: collisionless)     */
  double t_end;             /* > 0: the instance stops there                          */
  int n_cells;              /* >= 4                                                   */
  int pad;
} maxent_instance;

typedef struct {
  double t, dt_last;
  long long steps;
  int fail_step;            /* first failing step of this instance, 0 if none         */
  int fail_code;
} maxent_instance_info;

typedef struct {
  long long max_steps;      /* steps of the longest-running instance so far           */
  long long cell_updates;   /* sum over instances of cells x steps                    */
  long long n_active;       /* instances that have not reached t_end                  */
  long long n_fallback, n_fp64_states, n_face_states;
  int fail_step, fail_code;
} maxent_batch_info;

/* Errors: INVAL (system != 14, order != 2, FE integrator, an instance with < 4 cells, x1 <= x0,
 * t_end <= 0), NOMEM, DEVICE. */
int maxent_create_batch(const maxent_problem* common, const maxent_numerics* numerics,
                        int n_inst, const maxent_instance* instances, void* stream,
                        maxent_solver** out);

/* Advance every instance until it reaches its t_end, or for at most max_steps steps rounded
 * up to whole chunks (ceil(max_steps / chunk) * chunk).
 * The instances form a queue ordered by estimated work (cells x steps to t_end from the
 * CFL rate of the state given to init_state, largest first; ties by index).  Each step
 * compacts the instances that still advance, in queue order, into a list of tiles that the
 * stage launches split evenly over their workgroups, so finished instances cost nothing.
 * Steps are replayed in chunks of `chunk` steps captured once as a HIP graph (on an internal
 * stream of default priority, ordered after earlier work on the solver's stream); after each
 * chunk one word is read to see whether any instance is still active.  per_inst may be NULL
 * or hold n_inst records.  A failing instance stops (later steps are no-ops for it). */
int maxent_step_batch(maxent_solver* s, int max_steps, int chunk, maxent_batch_info* info,
                      maxent_instance_info* per_inst);

/* Launch shape of the batched stage kernels: threads per workgroup (64, 128 or 256), cells
 * per thread (1, 2 or 4, with threads x cells per thread <= 256; a tile holds
 * threads x cells per thread - 4 cells, so that the tile and its two-cell halos fill whole
 * rounds over the threads) and workgroups per compute unit (1..32).  INVAL for other values. */
int maxent_set_batch_launch(maxent_solver* s, int threads, int cells_per_thread, int wg_per_cu);
int maxent_get_batch_launch(maxent_solver* s, int* threads, int* cells_per_thread, int* wg_per_cu);

/* Autotuner: time trial_steps steps of each launch shape (threads x cells per thread in
 * 64x1, 64x2, 64x4, 128x1, 128x2, 256x1, times workgroups per CU 2/4/8/16) from the current
 * state, restoring the state after every trial, and keep the fastest.  Outputs may be NULL.
 * Errors: STATE before init_state, INVAL for trial_steps outside 1..10000, NOMEM for the
 * snapshot of the state, DEVICE if a trial fails (the launch shape is then the one before the
 * call, and the state should be loaded again with init_state). */
int maxent_autotune_batch(maxent_solver* s, int trial_steps, int* threads, int* cells_per_thread,
                          int* wg_per_cu, double* best_cell_updates_per_s);

/* ------------------------------------------------------------------ discrete adjoint
 * Reverse-mode derivatives of a scalar J(U_final) through the recorded steps: the hand-written
 * adjoint of every piece of the step (the conserved map and primitive recovery, the limited
 * reconstruction of Section 3.2, the closure of Section 2.4 / Appendix A with its sigma
 * mapping and sigma limit, the wave speeds of Section 5.1, the HLL / Rusanov flux of
 * Section 3.1, the BGK source with its local relaxation time, the boundary conditions and the
 * Runge-Kutta stages).  Conventions:
 *   - 14-moment system, FP64 precision, not a batch solver.
 *   - The time steps are frozen: the reverse replays the dt sequence the forward run used and
 *     does not differentiate the CFL maximum.
 *   - At non-smooth points the branch the forward evaluation took is differentiated: the
 *     limiter's selected variable and regime (a factor of 0 or 1 is constant), the
 *     positivity fallback, max(sigma, sigma_lim) (no derivative through sigma when the limit
 *     is active), min(sigma, 1) in the wave speeds, the clamped square roots, the HLL case.
 *   - Parameters: the jet Mach number and jet density of the JET boundary, and tau_ref (the
 *     derivative with respect to one tau_ref shared by all recorded steps, each step's source
 *     scaling as 1/tau_ref). */

/* Start recording a tape at the current state (checkpoint_every >= 1), or stop and free it
 * (checkpoint_every = 0).  While recording, maxent_step keeps each step's time step on the
 * device and its tau_ref on the host, and a copy of the state every checkpoint_every steps;
 * at most max_steps steps can be recorded (a maxent_step call that would exceed it fails with
 * INVAL before doing anything).  Device memory: (max_steps / checkpoint_every + 1) states for
 * the checkpoints; the adjoint adds 2 checkpoint_every + 3 states plus face and cell
 * workspaces (about 6 states in 2D).  maxent_init_state and maxent_destroy end the tape.
 * Errors: INVAL (sizes), STATE (no valid state, batch solver), NOMEM. */
int maxent_record(maxent_solver* s, int checkpoint_every, int max_steps);

/* Jet inflow Mach number and density of the JET boundary (both > 0).  Not allowed while a
 * tape holds recorded steps (STATE). */
int maxent_set_inflow(maxent_solver* s, double mach, double rho);

/* Steps recorded on the tape, and (dt != NULL) their time steps: dt must hold n_steps
 * doubles (host).  Replaying them as fixed time steps reproduces the recorded run bit for
 * bit.  Errors: STATE (no tape), DEVICE. */
int maxent_tape_info(maxent_solver* s, long long* n_steps, double* dt);

/* What the reverse pass differentiates (default EXACT).
 *   MAXENT_ADJ_EXACT           the exact derivative of the discrete step (branch replayed).
 *   MAXENT_ADJ_FROZEN_LIMITER  the same with each cell's common limiter factor held at its
 *                              forward value (no derivative through the limiter's selection).
 * Over long horizons the exact derivative of the common-limiter scheme grows without bound:
 * one variable's jumps set the factor applied to all fourteen slopes, and these cross-variable
 * gains compound from stage to stage, so J becomes rough on scales far below any practical
 * perturbation (the exact derivative, while correct, no longer predicts finite differences).
 * The frozen-limiter derivative stays bounded.  Errors: INVAL (unknown mode). */
enum { MAXENT_ADJ_EXACT = 0, MAXENT_ADJ_FROZEN_LIMITER = 1 };
int maxent_set_adjoint_mode(maxent_solver* s, int mode);

/* Reverse all recorded steps.
 *   dJ_dU       dJ/dU at the final state: conserved field array (14 x ny x nx), host or device.
 *   dJ_dU0      optional output (NULL: skipped): dJ/dU at the tape's start, same layout.
 *   dJ_dparams  optional host output of 3 doubles: dJ/d(jet Mach), dJ/d(jet rho), dJ/d tau_ref
 *               (0 for a parameter that does not enter, e.g. no JET boundary, tau_ref <= 0).
 * Segment by segment, newest first, the steps between two checkpoints are recomputed from the
 * checkpoint with the recorded time steps (bitwise the forward states) and reversed stage by
 * stage.  The solver's state, time and counters are not changed; the tape stays valid, so the
 * call may be repeated for another dJ_dU.  Errors: INVAL (null dJ_dU), STATE (no tape, or
 * the recorded run failed), NOMEM, DEVICE. */
int maxent_step_adjoint(maxent_solver* s, const double* dJ_dU, int dJ_on_device, double* dJ_dU0,
                        int dU0_on_device, double* dJ_dparams);

/* ------------------------------------------------------------------ no-allocation stepping
 * For callers that cannot allocate device memory (tight serving loops, harnesses that forbid
 * allocation): the work of maxent_create + maxent_init_state(CONSERVED) + maxent_step with
 * no handle and no allocation of any kind.  The intermediate stage state and the control block
 * live in a fixed device array of MAXENT_NOALLOC_SCRATCH_BYTES inside the library (one per
 * device, held until the process ends), so a problem fits when
 *   256 + 8 * nv * nx * ny <= MAXENT_NOALLOC_SCRATCH_BYTES
 * (at most 599 184 cells with 14 moments, e.g. 768 x 768; 1 677 715 cells with 5); larger
 * problems are rejected with INVAL before any device work.  A symmetric 14-moment state runs
 * the reduced stage kernel (maxent_set_reduced's default); the call then synchronises the
 * stream once more, after checking the input.
 *   U        the caller's device state, conserved, [nv][ny][nx] unpadded (the field-array
 *            layout above); read as the state at t0, overwritten with the state after the
 *            steps.  Checked first: a non-finite or unrealizable input returns NONFINITE /
 *            UNREALIZABLE with fail_step = 0 and no step taken.
 *   n, dt, tau_ref, t_end   as for maxent_step; t0 the time of the input state.
 *   stream   hipStream_t (NULL: default stream); the call synchronises it once at the end.
 *   info     optional report as for maxent_step (n_sigma_limited = -1).
 * The results equal those of maxent_create / maxent_init_state / maxent_step on the same
 * state (the same kernels).  Every call on one device shares that device's scratch: calls
 * that overlap on one device (other host threads, other streams) race and must be
 * serialised by the caller.  Errors (message in maxent_last_error(NULL)): INVAL (bad
 * arguments, problem too large), NONFINITE, UNREALIZABLE (info->fail_step), DEVICE. */
#define MAXENT_NOALLOC_SCRATCH_BYTES (64ull << 20)
int maxent_step_noalloc(const maxent_problem* problem, const maxent_numerics* numerics,
                        double* U, int n, double dt, double tau_ref, double t_end, double t0,
                        void* stream, maxent_info* info);

/* Symmetry-reduced kernels of the 14-moment system (Section 2.4 equations).
 *   2D planar: a state whose distribution is even in the z velocity has u_z = P_xz = P_yz =
 *     q_z = 0 in every cell, and the step keeps these four moments exactly zero (each of
 *     their fluxes, closing moments and source terms carries a z-odd factor; jet inflow
 *     states lie in the plane); the stage kernels then carry the ten other moments.
 *   1D axial (single solvers and batched tubes): a state also even in the y velocity has, in
 *     addition, u_y = P_xy = q_y = 0, kept zero by the x-direction step; the stage kernels
 *     then carry seven moments (rho, u_x, P_xx, P_yy, P_zz, q_x, R).
 * maxent_init_state checks the loaded state; with the mode on (enable = 1, the default) a
 * symmetric state runs the reduced kernel: the same step up to the rounding order of the
 * terms that remain, with 35 % (planar) or more (axial) fewer operations and bytes.
 * enable = 0 always runs the full 14-moment kernels.  The mode applies from the next step;
 * maxent_info.reduced reports which kernel runs.  Errors: INVAL (null handle), STATE (a tape
 * is recorded: the recorded run and its recomputation must use one kernel). */
int maxent_set_reduced(maxent_solver* s, int enable);

/* Optional timing of the fused stage kernels: when enabled, every stage-kernel launch of
 * maxent_step is bracketed by HIP events on the solver's stream and the elapsed times are
 * accumulated (read at the end of each maxent_step call).  Enabling resets the totals. */
int maxent_set_profiling(maxent_solver* s, int enable);
int maxent_get_profile(maxent_solver* s, double* stage_ms_total, long long* stage_launches);

void maxent_destroy(maxent_solver* s);

/* Last error message of this handle (or of the last failed maxent_create when s is NULL).
 * The pointer stays valid until the next call on the same handle. */
const char* maxent_last_error(const maxent_solver* s);

int maxent_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MAXENT_H */
