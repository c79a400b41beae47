/*
 * edf.h — C-ABI of the Elder density-driven-flow solver for AMD Instinct MI355X (gfx950).
 *
 * The library advances many realisations ("samples") of the 3D Elder box problem
 * by implicit-Euler time steps.  What one step computes is fixed by the paper
 * (Litvinenko, Logashenko, Tempone, Wittum, Keyes, "Solution of the 3D density-driven
 * groundwater flow problem with uncertain porosity and permeability", arXiv 1906.01632):
 *
 *   - the model: liquid mass conservation (eq. e_cont_eq), salt transport
 *     (eq. e_tran_eq), Darcy's law (eq. e_Darcy_vel), isotropic K (eq. e_scalar_perm),
 *     linear density (eq. e_lin_density), D = phi D_m (eq. e_mol_diff), Table 1;
 *   - boundary conditions of the box (Section 2.1): c = 1 on the closed top patch,
 *     c = 0 on the bottom, zero flux elsewhere, p = 0 at the four top corners;
 *   - vertex-centred finite volumes with (p, c) at the grid nodes, implicit Euler,
 *     Newton with a line search, BiCGStab preconditioned by a geometric multigrid
 *     V-cycle whose coarse matrices are the Jacobians re-assembled on every grid
 *     (Section 2.3 and Section 5.1 "Solving the deterministic problem");
 *   - porosity/permeability samples and their statistics: mean (eq. pdestat),
 *     variance (eq. numer_var), exceedance probability (Section 3.2).
 *
 * Conventions (all entry points):
 *   - Units are SI; z is depth (k = 0 is the top face) and gravity points along +z.
 *   - A grid has nx*ny*nz vertices, vertex v = i + nx*(j + ny*k).  A state or residual
 *     is a double array [N][2] with (p, c) interleaved per vertex.
 *   - Samples are numbered 0..S_total-1 across groups in the order the groups were
 *     given to edf_create_problem.
 *   - The library owns all device memory it allocates and frees it in edf_destroy.
 *     Host arrays passed in are read before the call returns.  Device pointers
 *     (is_device_ptr = 1) are borrowed for the duration of the call only.
 *   - All device work is enqueued on the HIP stream given at creation.  Calls that
 *     return values in host memory synchronise that stream before returning.
 *   - A non-zero return is an error; edf_last_error gives its text.  Argument errors
 *     (EDF_ERR_ARG) leave the problem unchanged.  Per-sample numerical failures are
 *     reported in edf_step_stats.status and are not call failures unless every
 *     sample failed (EDF_ERR_NO_CONVERGENCE).
 *   - One problem must not be used from two host threads at once.
 */
#ifndef EDF_H
#define EDF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct edf_problem edf_problem; /* opaque, library-owned */
typedef int32_t edf_status;

enum {
  EDF_OK = 0,
  EDF_ERR_ARG = 1,            /* invalid argument; nothing changed                  */
  EDF_ERR_OOM = 2,            /* device or host allocation failed                   */
  EDF_ERR_HIP = 3,            /* a HIP runtime call failed                          */
  EDF_ERR_STATE = 4,          /* call out of order (e.g. step before set_parameters)*/
  EDF_ERR_NO_CONVERGENCE = 5, /* every sample failed to converge in this call       */
  EDF_ERR_NONFINITE = 6       /* a non-finite value was met                         */
};

/* per-sample status in edf_step_stats.status */
enum {
  EDF_SAMPLE_OK = 0,
  EDF_SAMPLE_NEWTON_FAIL = 1, /* Newton reached its iteration limit                 */
  EDF_SAMPLE_LINEAR_FAIL = 2, /* BiCGStab did not reach its tolerance               */
  EDF_SAMPLE_NONFINITE = 3,   /* the residual became NaN or Inf                     */
  EDF_SAMPLE_INADMISSIBLE = 4 /* Newton converged to a state with c outside [0, 1]  */
};

/* porosity/permeability field models (hex-centroid values, Section 2.2):
 *  0 constant:  phi = phi_mean, K = K_mean
 *  1 one mode:  phi = phi_mean (1 + 0.2 xi1 cos(pi x/lx) cos(pi y/ly)), K = KC(phi)
 *  2 four modes: phi = phi_mean (1 + 0.2 xi1 cos cos + 0.2 xi2 sin(pi x/lx) sin(pi y/ly)),
 *               ln K = ln KC(phi) + 0.5 xi3 cos(pi z/lz) + 0.5 xi4 sin(pi x/lx) cos(pi z/lz)
 *  3 the paper's box field (eq. poro-paral3RVS):
 *               phi = phi_mean + 0.01 (xi1 sx + xi2 sy + xi3 sz + xi1 sx sy + xi2 sx sz),
 *               s* = sin(pi *_coord / l*), K = KC(phi)
 * with KC(phi) = K_mean (phi/phi_mean)^3 ((1 - phi_mean)/(1 - phi))^2 (eq. e_perm_Kozeny_Carman,
 * normalised so that KC(phi_mean) = K_mean). */
enum { EDF_FIELD_CONST = 0, EDF_FIELD_COS1 = 1, EDF_FIELD_MODES4 = 2, EDF_FIELD_PAPER3 = 3 };

enum { EDF_PREC_F64 = 0,       /* V-cycle in FP64                                   */
       EDF_PREC_MIXED = 1,     /* V-cycle in FP32 inside FP64 Newton/BiCGStab       */
       EDF_PREC_MIXED_F16 = 2  /* as EDF_PREC_MIXED, with the finest level's matrix */
                               /* stored in FP16, scaled by its diagonal-block      */
                               /* inverse (unit diagonal blocks, O(1) entries)      */ };

/* One resolution group: n_samples realisations on an nx*ny*nz vertex grid with an
 * n_levels-grid multigrid hierarchy (each coarser grid keeps every other vertex, so
 * (n-1) must be divisible by 2^(n_levels-1) in every direction). */
typedef struct {
  int32_t nx, ny, nz, n_levels, n_samples;
} edf_group_desc;

/* Physical constants (Table 1) and the top patch [patch[0],patch[1]] x [patch[2],patch[3]]. */
typedef struct {
  double lx, ly, lz;
  double rho0, rho1, mu, g, Dm;
  double phi_mean, K_mean;
  double patch[4];
  int32_t field_model, n_xi;
} edf_physics;

/* Solver options.  Residual norms are of the scaled residual: finite-volume rows
 * times dt/(rho0 phi_mean hx hy hz), salt-Dirichlet rows as is, pinned-pressure
 * rows divided by rho0*max(g,1)*lz.  Newton stops at ||F~|| <= max(newton_rtol
 * ||F~_0||, newton_atol), or when the root-mean-square Newton update of the scaled
 * unknowns (p / p_unit, c) is below 1e-14 (rounding level); BiCGStab stops at
 * ||r|| <= lin_rtol ||b||. */
typedef struct {
  double newton_rtol, newton_atol, lin_rtol;
  int32_t newton_max_it;   /* e.g. 20                                              */
  int32_t ls_max_halvings; /* line search halvings, e.g. 5                         */
  int32_t lin_max_it;      /* BiCGStab iterations per Newton step, e.g. 200        */
  int32_t nu_pre, nu_post; /* block Gauss-Seidel sweeps before/after coarse grid   */
  int32_t precision;       /* EDF_PREC_*                                           */
  int32_t check_every;     /* BiCGStab iterations between host convergence checks  */
  int32_t dt_max_halvings; /* a sample whose step fails is redone as 2^h equal      */
                           /* sub-steps, h = 1..dt_max_halvings (0: no retry)       */
  int32_t forcing;         /* 0: every Newton system solved to lin_rtol; 1: to the  */
                           /* Eisenstat-Walker forcing term (choice 2, gamma 0.9,   */
                           /* 0.5 at the first iteration and at most 0.5, at least  */
                           /* lin_rtol)                                             */
  int32_t concurrent_groups; /* 0: edf_step advances the groups one after the other; */
                           /* 1: at the same time, one host thread and stream each  */
                           /* (kernels of different groups then share the GPU, which */
                           /* lengthens each one's measured duration); 2: one host  */
                           /* thread each on one shared stream, and the V-cycles of */
                           /* the groups inside BiCGStab run together: every level  */
                           /* that groups share (same grid, same role in the cycle, */
                           /* the groups' samples side by side in one allocation)   */
                           /* is swept by one launch over all their listed samples, */
                           /* and groups whose fused bottoms cover the same grids   */
                           /* share its launch (bitwise the results of 0; Section 4 */
                           /* runs the scenarios independently, here they also      */
                           /* share launches).  graph_vcycle is not used in mode 2  */
  int32_t graph_vcycle;    /* 1: each V-cycle launch configuration is captured once  */
                           /* as a HIP graph and replayed (same kernels, same order, */
                           /* bitwise the same results; not while edf_profile is     */
                           /* on, which times single launches); 0: launched one by  */
                           /* one                                                   */
  int32_t substep_memory;  /* 0: every step first tries the full step length (so a  */
                           /* step that converges is exactly one implicit-Euler     */
                           /* step); 1: a sample starts a step with the number of   */
                           /* sub-steps that worked for it in its previous step     */
                           /* (fewer failed attempts, but the result then depends  */
                           /* on the sample's history; see edf_step)                */
  int32_t smoother;        /* the multigrid smoother on the levels swept by their   */
                           /* own launches: 0 point-block Gauss-Seidel in 8 colours */
                           /* (i%2, j%2, k%2); 1 vertical-line block Gauss-Seidel:  */
                           /* every z-column's block tridiagonal system solved      */
                           /* exactly, columns in 4 colours (i%2, j%2), the other  */
                           /* couplings lagged (the levels of the fused bottom are  */
                           /* swept the same way inside its launch; an FP16-stored  */
                           /* finest level by lines of its scaled matrix D^-1 A)    */
  int32_t matrix_free;     /* the outer BiCGStab's products J x: 0 with the exact    */
                           /* FP64 Jacobian assembled as a 27-point stencil of 2x2  */
                           /* blocks (864 bytes per vertex); 1 matrix-free, the     */
                           /* directional derivative of the defect computed from    */
                           /* the state, the coefficients and x (the same operator, */
                           /* no exact finest-level stencil stored; the adjoint's   */
                           /* transposed products stay assembled)                   */
  int32_t predictor;       /* Newton's starting point of a step: 0 the state at the */
                           /* start of the step; 1 also the linear extrapolation    */
                           /* 2 u^n - u^{n-1} of the sample's last two states when  */
                           /* its previous step was one implicit-Euler step of the  */
                           /* same length, taken when its scaled defect is the      */
                           /* smaller.  The stopping test stays relative to the     */
                           /* defect at the start of the step, so the step reaches  */
                           /* the same tolerance with fewer Newton iterations.      */
                           /* Not used while edf_solve records a trajectory (the    */
                           /* adjoint recomputes those steps from checkpoints)      */
  int32_t lag_preconditioner; /* 0: the V-cycle's matrices (every level) and their    */
                           /* block inverses, line factors and coarse inverse are   */
                           /* re-assembled at every Newton iteration (Section 5.1);  */
                           /* 1: only at the first Newton iteration of each attempt */
                           /* of a (sub-)step, then kept (the outer products stay    */
                           /* the exact Jacobian at the current iterate, so Newton  */
                           /* and its result are unchanged; only the preconditioner */
                           /* lags)                                                  */
} edf_solver_opts;

/* Per-sample result of a step.  Counters named *_total run over every step since the
 * sample was created or last given a state with edf_set_state. */
typedef struct {
  int32_t status;       /* EDF_SAMPLE_* of this step.  A sample whose step failed keeps */
                        /* that status and its last good state in every later step: */
                        /* it is not advanced again and is left out of the           */
                        /* statistics until edf_set_state gives it a new state       */
  int32_t newton_its;   /* Newton iterations of this step (all attempts)            */
  int32_t lin_its;      /* BiCGStab iterations summed over those Newton iterations  */
  int32_t ls_halvings;  /* line-search halvings summed over them                    */
  int32_t substeps;     /* this step was taken as this many equal sub-steps (2^h)   */
  int32_t retries;      /* attempts of this step that failed and were restarted     */
                        /* with twice as many sub-steps                              */
  int32_t steps_total;    /* steps completed                                        */
  int32_t split_total;    /* of those, steps taken as more than one sub-step        */
  int32_t substeps_total; /* implicit-Euler sub-steps completed                     */
  int32_t retries_total;  /* failed and restarted attempts                          */
  int32_t failed_step;    /* steps_total + 1 at the step that failed; 0: none       */
  int32_t predicted;      /* 1: Newton started this step from the extrapolation     */
                          /* 2 u^n - u^{n-1} (opts.predictor)                       */
  double defect0;       /* ||F~|| at the start of the step (full step length)      */
  double defect;        /* ||F~|| at the end of the last sub-step                  */
  /* Global conservation over this step, computed in FP64 on the device from the     */
  /* states and the boundary rows (eqs. e_cont_eq and e_tran_eq summed over all      */
  /* control volumes: interior face fluxes cancel in pairs and no-flow faces carry   */
  /* none, so the change of the mass in the box equals what the Dirichlet vertices   */
  /* exchange).  Salt: dM = sum_v m_v [rho(c) c - rho(c_old) c_old] over all          */
  /* vertices and sub-steps, B = sum over sub-steps of dt_sub * (finite-volume salt   */
  /* row at the c-Dirichlet vertices); liquid: dM = sum_v m_v [rho(c) - rho(c_old)], */
  /* B = dt_sub * (finite-volume liquid row at the p-pinned vertices).  The error is  */
  /* |dM - B| / (sum_v |m_v [..] change| + |B|) (0 when both are 0): the residual  */
  /* left in the solved rows, relative to the mass moved.  0 for a failed step.      */
  double salt_balance_err;
  double liquid_balance_err;
} edf_step_stats;

/* Quantity of interest of the adjoint (kind 0, the only kind): the salt mass in the
 * box [box[0],box[1]] x [box[2],box[3]] x [box[4],box[5]] (SI units, z = depth) at the
 * final time.  rtol: relative residual tolerance of the adjoint BiCGStab solves (0: the
 * default 1e-12).  The gradient is a sum of products lambda^T dR/dxi that largely cancel,
 * so it is much more sensitive to the adjoint solves than the states are to the forward
 * ones: on the 65x65x17 lattice batch a tolerance of 1e-10 left relative gradient errors
 * of ~3e-5, 1e-6 errors of order one, 1e-12 ~3e-8. */
typedef struct {
  double box[6];
  double rtol;
  int32_t kind;
  int32_t reserved;
} edf_qoi;

/* Creates a problem.  groups[n_groups] describe the resolution groups; every sample
 * starts from the initial state (pure water, p = rho0 g z, c = 1 on the patch).
 * hip_stream is a hipStream_t (NULL = the default stream).
 * Errors: EDF_ERR_ARG for an inconsistent description, EDF_ERR_OOM, EDF_ERR_HIP. */
edf_status edf_create_problem(const edf_physics* phys, const edf_group_desc* groups,
                              int32_t n_groups, const edf_solver_opts* opts,
                              void* hip_stream, edf_problem** out);

/* Sets the porosity/permeability parameters of every sample: xi is a host array
 * [S_total][phys.n_xi], row-major.  Computes phi and K on every grid level
 * (Section 2.2).  EDF_ERR_ARG if some |xi| > 1 or a resulting phi is not in (0,1)
 * or K is not finite and positive; the fields are checked on every level before any
 * is written, so the problem keeps its previous parameters then.  Clears every
 * sample's sub-step history (opts.substep_memory), and any trajectory that
 * edf_solve recorded for edf_adjoint. */
edf_status edf_set_parameters(edf_problem* pb, const double* xi);

/* Copies a state [N][2] (p, c) of one sample in or out; the array is in host memory
 * (is_device_ptr = 0) or device memory (1).  set_state also sets the previous-step
 * state to the same values, and resets the sample: a failure of an earlier step is
 * cleared (the sample is advanced again and counted in the statistics), its
 * sub-step history and its *_total counters start afresh, and any recorded trajectory
 * is dropped. */
edf_status edf_set_state(edf_problem* pb, int32_t sample, const double* pc, int32_t is_device_ptr);
edf_status edf_get_state(edf_problem* pb, int32_t sample, double* pc, int32_t is_device_ptr);

/* One time step of length dt [s] for every sample that has not failed (Section 2.3).
 * With opts.substep_memory = 0 the step is one implicit-Euler step whenever Newton
 * converges at the full length; only a sample whose attempt fails (iteration limit,
 * no 100-fold residual reduction after 8 iterations, a non-finite or 1e4-fold grown
 * residual, a converged state with c outside [-0.05, 1.05], or, while h <
 * opts.dt_max_halvings, a Newton system whose BiCGStab residual ended above twice its
 * tolerance) restarts the step from its state at the start of the call as 2^h equal
 * implicit-Euler sub-steps of dt / 2^h with h raised by one (stats.substeps = 2^h,
 * stats.retries counts the restarts), up to opts.dt_max_halvings.  With
 * opts.substep_memory = 1, h starts at the value that worked for the sample in its
 * previous step (lowered by one after w steps without a restart, where w = 3 and
 * doubles, up to 64, whenever such a lowered start fails).  A sample that still fails
 * at h = dt_max_halvings keeps its state from the start of the call and is marked
 * failed: later steps leave it alone (stats.status keeps the failure) until
 * edf_set_state resets it.  stats, if not NULL, is a host array [S_total], including
 * the FP64 mass-balance errors of the step.  EDF_ERR_NO_CONVERGENCE when no sample is
 * left that has not failed.  Synchronises. */
edf_status edf_step(edf_problem* pb, double dt, edf_step_stats* stats);

/* n_steps steps of length dt, as edf_step; stats (host [S_total] or NULL) describe the
 * last step.  checkpoint_every = k > 0 records the trajectory for edf_adjoint: every
 * sample's state at steps 0, k, 2k, ... (before each segment of k steps) and the
 * sub-step count of every step, in library-owned device memory of
 * (ceil(n_steps / k) + 1) + (k + 1) states per sample (the second part holds the
 * states of one segment while the adjoint recomputes it).  checkpoint_every = 0
 * records nothing.  EDF_ERR_ARG for n_steps < 0 or checkpoint_every < 0. */
edf_status edf_solve(edf_problem* pb, double dt, int32_t n_steps, int32_t checkpoint_every,
                     edf_step_stats* stats);

/* Weighted statistics of c over the samples (eqs. pdestat, numer_var; Section 3.2):
 * mean = sum w_i c_i, var = sum w_i (c_i - mean)^2, exceed = sum w_i [c_i > threshold].
 * Every group is injected to the common vertex set (cx, cy, cz), which must be nested
 * in every group's grid.  weights: host [S_total] or NULL for 1/S_total; they are divided
 * by their sum, which must be positive, and may be signed (a multilevel estimator gives
 * the coarse partners of a level negative weights: var is then sum w c^2 - mean^2 and
 * may dip below zero).  Samples that have failed (edf_step) are left out and the weights
 * of the others renormalised.
 * mean, var, exceed: host arrays [cx*cy*cz].  Synchronises. */
edf_status edf_moments(edf_problem* pb, int32_t cx, int32_t cy, int32_t cz, double threshold,
                       const double* weights, double* mean, double* var, double* exceed);

/* The statistics of edf_moments over the samples of one resolution group at that group's
 * own resolution (every vertex of its grid, no injection): the per-group estimates of
 * eqs. pdestat and numer_var, e.g. the 129^3 group's mean and variance at 129^3 in a
 * problem that also holds coarser groups.  weights: host [S of the group] (in the group's
 * sample order) or NULL for equal weights; normalised and masked for failed samples as in
 * edf_moments.  mean, var, exceed: host arrays [nz][ny][nx] of the group's grid.
 * EDF_ERR_ARG for a group index out of range.  Synchronises. */
edf_status edf_group_moments(edf_problem* pb, int32_t group, double threshold,
                             const double* weights, double* mean, double* var, double* exceed);

/* edf_moments for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same statistics,
 * bitwise, with no hipMalloc, hipFree or other allocating call.  Its working memory
 * (weights, failure flags, the three output fields and the injected c fields of as
 * many samples at a time as fit) lives in a fixed 16 MiB device array of the library,
 * one per GPU, held until the process ends; the samples are taken in chunks in sample
 * order, so the sums are those of edf_moments.  Limit: 2^21 doubles, i.e.
 * 3 cx cy cz + cx cy cz + S_total (+ alignment) must fit: EDF_ERR_ARG beyond that (use
 * edf_moments).  Every call on a GPU shares that GPU's array: calls that overlap on one
 * GPU (two host threads, or two streams) race and must be serialised by the caller.
 * Arguments, outputs and errors as edf_moments.  Synchronises. */
edf_status edf_moments_noalloc(edf_problem* pb, int32_t cx, int32_t cy, int32_t cz,
                               double threshold, const double* weights, double* mean,
                               double* var, double* exceed);

/* Polynomial chaos surrogate of c from the samples of group `group` (Section 3.1,
 * eqs. PCEdecom2, PCEcoef, PCEcoef2, var; appendix).  The samples are the quadrature
 * nodes: theta_i = xi_i (the parameters of edf_set_parameters, M = n_xi in [1, 4]), with
 * probability weights `weights` (host [S_group], e.g. tensor Gauss-Legendre weights
 * times 2^-M).  Basis Psi_beta(theta) = prod_j psi_{beta_j}(theta_j), psi_n the Legendre
 * polynomials of the appendix's recursion; multi-indices with total degree <= degree
 * (truncation 0) or every degree <= degree (truncation 1), degree <= 8, at most 128 of
 * them, ordered by total degree and then decreasingly lexicographic (M = 2: (0,0), (1,0),
 * (0,1), (2,0), (1,1), (0,2), ...).  The c field of every sample is injected to the
 * common vertex set (cx, cy, cz), which must be nested in the group's grid, and
 *   c_beta(x) = sum_i w_i Psi_beta(theta_i) c(x, theta_i) / Q_beta,
 *   Q_beta = prod_j 1/(2 beta_j + 1);  mean = c_0;  var = sum_{beta != 0} Q_beta c_beta^2.
 * Outputs: *n_coef; coef (host [n_coef][cz][cy][cx] or NULL); mean, var (host
 * [cz][cy][cx]); kernel_ms (or NULL): duration of the projection kernel.  The
 * coefficients stay in the problem for edf_gpc_exceed.  Samples that have failed
 * (edf_step) are left out and the weights of the others renormalised to their sum.
 * Synchronises. */
edf_status edf_gpc_project(edf_problem* pb, int32_t group, int32_t cx, int32_t cy, int32_t cz,
                           int32_t degree, int32_t truncation, const double* weights,
                           int32_t* n_coef, double* coef, double* mean, double* var,
                           double* kernel_ms);

/* Exceedance probability of the last edf_gpc_project surrogate (eq. PCEpoint and the
 * count under it, Section 3.2): at every common-grid vertex,
 *   P(c > threshold) ~ #{s : sum_beta c_beta Psi_beta(theta_s) > threshold} / n_points
 * over the points theta (host [n_points][M] in [-1,1]^M; the caller draws them).  The
 * surrogate is evaluated in FP64.  prob: host [cz][cy][cx]; kernel_ms (or NULL): the
 * duration of the evaluation on the device (the basis tables of the points, built about
 * 2^20 points at a time, and the surrogate products and counts), from events around it.
 * EDF_ERR_STATE without a projection.  Synchronises. */
edf_status edf_gpc_exceed(edf_problem* pb, int32_t n_points, const double* theta, double threshold,
                          double* prob, double* kernel_ms);

/* Discrete adjoint (the gradient of a quantity of interest with respect to the field
 * parameters xi) of the trajectory recorded by the last edf_solve with
 * checkpoint_every = k > 0.  The adjoint equations run backwards through the steps:
 * per implicit-Euler sub-step one BiCGStab solve with the transposed Jacobian,
 * preconditioned by the multigrid V-cycle of the transposed (frozen-flux) matrices.
 * The states inside each segment of k steps are recomputed from the segment's
 * checkpoint (the forward kernels give the same states bitwise; the recorded sub-step
 * counts are replayed), one segment at a time from the last.  The quantity (edf_qoi,
 * kind 0) is the salt mass in the box at the final time,
 *   J = sum_v sum_{e adjacent to v} phi_e |octant(e, v) ∩ box| rho(c_v) c_v,
 * the mass density phi rho c of eq. e_tran_eq integrated over the box with the
 * control volumes of the scheme.  Outputs (host): J[S_total], dJ_dxi[S_total][n_xi]
 * (NaN for a sample that failed during the recorded steps).  The states stay at the
 * final time.  Needs a field model with parameters.  EDF_ERR_STATE without a recorded
 * trajectory (or after edf_step, edf_set_state or edf_set_parameters changed the
 * states or parameters since); EDF_ERR_NO_CONVERGENCE if an adjoint solve fails.
 * The adjoint solves run to qoi->rtol.  Synchronises. */
edf_status edf_adjoint(edf_problem* pb, const edf_qoi* qoi, double* J, double* dJ_dxi);

/* Inspection entry points used by the parity tests. */

/* Scaled residual F~(u; u_old) of one sample for dt, written to F [N][2] (same
 * memory kind as u).  u, u_old, F: [N][2]; is_device_ptr applies to all three. */
edf_status edf_residual(edf_problem* pb, int32_t sample, const double* u, const double* u_old,
                        double dt, double* F, int32_t is_device_ptr);

/* Assembles the scaled Jacobian of one sample at state u (host [N][2]) on grid level
 * `level` (0 = finest; coarser levels use u injected) and copies it to host
 * out[27][2][2][N_level]: entry (o, eq, var, v) = dF~_(v,eq) / du~_(v+o,var), where the
 * neighbour offset o = (dx+1) + 3(dy+1) + 9(dz+1) and u~ = (p / p_unit, c).  Entries
 * that point outside the grid are zero. */
edf_status edf_get_jacobian(edf_problem* pb, int32_t sample, const double* u, double dt,
                            int32_t level, double* out);

/* Assembles the matrices of every level of group `group` at the group's current
 * states for step length dt and applies one multigrid V-cycle y = M^{-1} x, where
 * x and y are host arrays [S_group][N][2] of scaled unknowns (p / p_unit, c).
 * The V-cycle is the preconditioner of the Newton systems (Section 2.3). */
edf_status edf_apply_vcycle(edf_problem* pb, int32_t group, double dt, const double* x,
                            double* y);

/* y = J~ x with the exact finest-level Jacobian of group `group`: the stencil of the last
 * assembly (edf_apply_vcycle or a Newton iteration), or with opts.matrix_free the
 * matrix-free product at the group's current states and the last assembly's step
 * length; x, y host [S_group][N][2]. */
edf_status edf_apply_jacobian(edf_problem* pb, int32_t group, const double* x, double* y);

/* Timing of the multigrid preconditioner with HIP events on the groups' streams.
 * edf_profile(pb, 1, out) starts: every 13th smoother launch (the dominant kernel,
 * block Gauss-Seidel over one colour; the stride runs through colours, levels and
 * sweeps alike) and every whole V-cycle is bracketed by events; edf_profile(pb, 0,
 * out) stops.  Both fill out (if not NULL, host double[16]) with totals since the last
 * start: out[0..2] = timed smoother launches, their summed kernel time [ms] and
 * algorithmic bytes; out[3..5] = V-cycles, summed time [ms], algorithmic bytes;
 * out[6..7] = all smoother launches and their algorithmic bytes; out[8..10] = the timed
 * smoother launches of more than 256 MiB of algorithmic bytes (working sets beyond the
 * last-level cache, whose bandwidth is HBM bandwidth), their time and bytes;
 * out[11..12] = all such launches and their bytes; out[13..15] = the V-cycles of more than
 * 256 MiB of algorithmic bytes, their time and bytes.  With the vertical-line smoother the
 * smoother launches are its column sweeps: per vertex of the swept columns and active
 * sample 24 stencil blocks towards the other columns (the first sweep from zero: 0, 6,
 * 18, 24 for column colours 0..3) and the block above, 8 factor values, b, and x written,
 * read and written again.
 * Smoother bytes per vertex of the swept colour and per active sample: 108 stencil +
 * 4 block-inverse entries + 2 right-hand side + 4 own-unknown reads and writes, times
 * the V-cycle precision; the first forward sweep of a level starts from x = 0 and reads
 * only the 4 n_c stencil values towards the colours already swept (n_c = 0, 2, 6, 8, 18,
 * 20, 24, 26 for colours 0..7; colour 0 is done by the kernel that writes b, not by a
 * smoother launch), the block inverse and b, and writes x.  V-cycle bytes per active
 * sample: on every smoothed level its nu_pre + nu_post sweeps (the first from zero),
 * the residual (108 stencil values, b, x in, r out; after a single pre-smoothing sweep
 * only the 4 (26 - n_c) values towards the later colours and r out), r into the
 * restriction and x in and out for the correction, plus the dense coarse inverse.
 * Launches run over the samples still active in their BiCGStab.  Synchronises the
 * streams. */
edf_status edf_profile(edf_problem* pb, int32_t enable, double* out);

/* Autotuning of the V-cycle (an implementation choice, not part of the method): the
 * coarse levels of every group can run in one launch with one workgroup per sample
 * (the fused bottom), which saves launches but walks the levels one after the other,
 * and the vertical-line sweep of each level swept by its own launches has a tile shape
 * (8, 16 or 32 columns per 256-thread workgroup: LDS per workgroup against rows gathered
 * per wave).  This call assembles the Newton matrices at the current states with time
 * step dt, times three V-cycles per group for every admissible first fused level, twice
 * over, and keeps the fastest (the better of its two timings counts for each); with
 * concurrent_groups = 2 (merged V-cycles) the number of fused levels is chosen for all
 * groups together (the least summed time), so that their bottoms share one launch; then,
 * level by level from the finest, every tile shape the level's LDS allows in the same way.
 * States are not changed.  Without it (or edf_set_tuning) a group of >= 64 samples fuses
 * all levels of <= 4096 vertices, a smaller group only the coarse solve, and line sweeps
 * take 16 columns per workgroup.  EDF_ERR_STATE before edf_set_parameters, EDF_ERR_ARG
 * for dt <= 0. */
edf_status edf_autotune(edf_problem* pb, double dt);

/* The V-cycle configuration of group `group`: *fuse_from = first level run in the
 * fused bottom launch; ms (host double[n_levels] or NULL) = the autotuned V-cycle
 * time per candidate first level in milliseconds (-1 where not measured). */
edf_status edf_get_tuning(edf_problem* pb, int32_t group, int32_t* fuse_from, double* ms);

/* Fix the first level of the fused bottom of group `group` (e.g. a tuning saved from
 * an earlier run; a later autotuning step keeps it).  EDF_ERR_ARG unless every level
 * from fuse_from on has at most 4096 vertices, at most 6 levels are fused, and
 * fuse_from <= n_levels - 1 (the coarsest level alone is always allowed). */
edf_status edf_set_tuning(edf_problem* pb, int32_t group, int32_t fuse_from);

/* Tile shapes of the vertical-line sweeps of group `group` (see edf_autotune):
 * cols (host int32_t[n_levels]) = columns per workgroup of each level's k_line_sweep, 0
 * for a level without line smoothing (the coarsest, the point smoother).
 * edf_set_line_tiles fixes them (e.g. from a saved tuning); EDF_ERR_ARG, with nothing
 * changed, unless every entry is 0 exactly where the level has no line smoothing and
 * otherwise 8, 16 or 32 with 10 x nz x cols values in at most 64 KiB of LDS.  Tile shapes
 * do not change results (each column is computed the same way). */
edf_status edf_get_line_tiles(edf_problem* pb, int32_t group, int32_t* cols);
edf_status edf_set_line_tiles(edf_problem* pb, int32_t group, const int32_t* cols);

const char* edf_last_error(const edf_problem* pb);
void edf_destroy(edf_problem* pb); /* NULL is allowed */

#ifdef __cplusplus
}
#endif
#endif /* EDF_H */
