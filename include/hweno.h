/* hweno.h -- C ABI of the MI355X (gfx950) implementation of the fifth-order hybrid
 * Hermite WENO scheme with artificial linear weights of Zhao & Qiu (arXiv 2002.08816).
 *
 * The library advances the zeroth and first moments of 1D and 2D conservation laws
 * (scalar linear advection, Burgers, Euler with a gamma law) on uniform Cartesian meshes
 * with the paper's semi-discrete operator (eq. odeH in 1D, eq. ode2 in 2D) and the
 * third-order TVD Runge-Kutta method (eq. RK).  Everything runs in FP64 on the GPU.
 *
 * Conventions
 *  - Every call returns an hw_status; nothing aborts or throws across the ABI.  After a
 *    failure, hw_last_error(handle) gives a message (NULL handle: the last global error).
 *  - State arrays are structure-of-arrays, x fastest:
 *        1D: avg[ncomp][n], mx[ncomp][n]
 *        2D: avg[ncomp][ny][nx], mx[ncomp][ny][nx], my[ncomp][ny][nx]
 *    where avg are the cell averages, mx and my the first moments
 *        (1/|I|) int_I u (x - x_i)/dx,   (1/|I|) int_I u (y - y_j)/dy
 *    (definitions below eq. odeH and eq. ode2), and ncomp = 1 for scalar laws, 3 (1D)
 *    or 4 (2D) for Euler with components (rho, rho*u[, rho*v], E).
 *  - Host pointers are copied; the caller keeps ownership.  Device pointers (*_device
 *    calls) are used in stream order on the handle's stream and are neither freed nor
 *    retained.  The handle owns all device memory it allocates.
 *  - Handles are not thread-safe; calls on one handle must not overlap.
 */
#ifndef HWENO_H
#define HWENO_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hw_solver hw_solver;

typedef enum {
  HW_OK = 0,
  HW_EINVAL = 1,      /* invalid argument or configuration */
  HW_ENOMEM = 2,      /* device allocation failed */
  HW_EDEVICE = 3,     /* HIP runtime error */
  HW_ENONFINITE = 4,  /* a stage produced a non-finite value, or rho <= 0 or p <= 0 */
  HW_ESTATE = 5       /* call not valid in the handle's current state */
} hw_status;

typedef enum { HW_ADVECTION = 0, HW_BURGERS = 1, HW_EULER = 2 } hw_eq;
/* boundary conditions: periodic; transmissive (ghost cells are even mirror images of the
 * cells they face: averages copied, normal first moments negated); reflective wall (the
 * blast problem of Section 3.2: the transmissive mirror with the normal momentum reversed,
 * i.e. all of that component's values negated on top of the mirror; Euler, 1D and 2D).
 * At transmissive and reflective boundaries a ghost is the mirror image of the cell it
 * faces in every respect: troubled flag, limited moments and edge values as well. */
/* HW_BC_DMR (2D Euler; set as both bc_x and bc_y): the boundaries of the double Mach
 * reflection problem (Example 3.10): a Mach 10 shock at 60 degrees to a wall that runs
 * along y = y0 from x = 1/6.  Cells beyond the left side (x < x0), the top side (y > y1)
 * and the bottom side left of x = 1/6 hold the exact solution's moments at the time of
 * each stage input (post-shock state behind the line x = 1/6 + (y + 20 t)/sqrt(3), gas
 * at rest with rho = 1.4, p = 1 ahead of it); they are never troubled, and their trace on
 * the boundary face is the exact state at its Gauss points.  The bottom side from
 * x = 1/6 is a reflective wall, the right side an outflow (transmissive) boundary.  The
 * handle's time (hw_set_state sets it to 0) is the time of the state. */
/* HW_BC_STEP (2D Euler; set as both bc_x and bc_y): the forward-facing step (Example 3.11):
 * an obstacle inside the rectangular mesh, the cells with x > step_x and y < step_y (the
 * step's corner must lie on cell faces, with 3 <= sj, 2 sj <= ny and sj <= si < nx for
 * its cell indices si, sj).  Those cells are solid: they keep the values they were given
 * and report no flags.  The left side is an inflow of the state `inflow`, the right side
 * an outflow (transmissive), the top and bottom sides and the step's two faces reflective
 * walls.  Reading: stencil data at a position outside the fluid come from one fluid cell
 * (the mirror across the boundary or step face it lies closer to, a point reflection
 * through the corner on the step's diagonal, the prescribed inflow state beyond the left
 * side) with its flag and limited moments; the trace of the non-fluid side of a face is
 * the fluid cell's own trace there, with the normal momentum reversed at a wall. */
typedef enum { HW_BC_PERIODIC = 0, HW_BC_TRANSMISSIVE = 1, HW_BC_REFLECTIVE = 2, HW_BC_DMR = 3,
               HW_BC_STEP = 4 } hw_bc;
/* troubled-cell mode: KXRCF indicator (Step 1 / Step 4), no troubled cell (the linear
 * scheme), or every cell troubled (the "New HWENO" variant of Section 3) */
typedef enum { HW_TC_KXRCF = 0, HW_TC_NONE = 1, HW_TC_ALL = 2 } hw_tc_mode;

typedef struct {
  int dim;             /* 1 or 2 */
  int nx, ny;          /* cells; ny = 1 when dim = 1; nx, ny >= 7 */
  double x0, x1, y0, y1;   /* domain; 2D cells must be square (dx = dy) */
  int eq;              /* hw_eq */
  double adv[2];       /* advection speeds (HW_ADVECTION) */
  double gamma_gas;    /* ratio of specific heats (HW_EULER), 1.4 in the paper */
  int bc_x, bc_y;      /* hw_bc */
  int ng_edge;         /* 2D edge Gauss points: 3 (Section 2.2) or 2 */
  double lim_w[3];     /* limiter linear weights: positive, sum 1 (Step 1) */
  double rec_w[5];     /* reconstruction linear weights: 3 used in 1D (Step 2.1), 5 in 2D (Step 5.1) */
  double eps;          /* epsilon of the nonlinear weights, 1e-6 */
  double cfl;          /* CFL number, 0.6 (Section 3) */
  int tc_mode;         /* hw_tc_mode */
  double step_x, step_y;   /* HW_BC_STEP: the step's corner (0.6, 0.2 in Example 3.11) */
  double inflow[4];    /* HW_BC_STEP: inflow rho, u, v, p (1.4, 3, 0, 1: Mach 3) */
} hw_config;

/* Fills the paper's defaults for dimension dim (1 or 2): linear weights 0.01 for every
 * low-degree polynomial and the rest for the high-degree one (Section 3.2), eps = 1e-6,
 * CFL 0.6, gamma 1.4, 3-point edge Gauss rule, KXRCF, periodic boundaries, Euler, the
 * unit interval / square, and the step and inflow of Example 3.11.  nx (and ny in 2D)
 * are left 0 for the caller to set. */
void hw_config_default(hw_config* cfg, int dim);

/* Creates a solver for one mesh (the problem of eq. EQ / EQ2 on a uniform mesh, Sections
 * 2.1-2.2; handle management, the paper has no counterpart).  stream: a hipStream_t to run
 * on, or NULL to let the library create its own.  Rejects invalid configurations with
 * HW_EINVAL, failed device allocations with HW_ENOMEM (nothing is left allocated). */
hw_status hw_create(const hw_config* cfg, void* stream, hw_solver** out);

/* Creates a batched 1D solver: n independent instances of the 1D configuration `base`,
 * instance b with nx[b] cells on [x0[b], x1[b]] (x0/x1 may be NULL: base domain).  The
 * state of a batch is the concatenation of the instances' arrays, instance by instance,
 * inside each component: avg[ncomp][sum nx], mx[ncomp][sum nx].  Each instance has its
 * own Lax-Friedrichs speed, CFL time step and time. */
hw_status hw_batch_create(const hw_config* base, int n, const int* nx, const double* x0,
                          const double* x1, void* stream, hw_solver** out);

/* Frees the handle and all device memory it owns (and its stream, if the library created
 * it); a null handle is accepted (HW_OK).  Handle management: no passage of the paper. */
hw_status hw_destroy(hw_solver* h);

/* Number of cells per component plane (nx*ny, or sum of nx for a batch), components (1, or
 * 4 for 2D Euler / 3 for 1D Euler) and moments per component (2 in 1D: average and first
 * moment, Section 2.1; 3 in 2D, Section 2.2). */
hw_status hw_get_sizes(const hw_solver* h, long* cells, int* ncomp, int* nmoments);

/* Sets the state from host arrays (layout above; my = NULL in 1D) and the time to 0. */
hw_status hw_set_state(hw_solver* h, const double* avg, const double* mx, const double* my);
/* Copies the state to host arrays; t (may be NULL) receives the time (batch: instance 0). */
hw_status hw_get_state(hw_solver* h, double* avg, double* mx, double* my, double* t);
/* Device variants: one contiguous device array [nmoments][ncomp][cells], stream-ordered. */
hw_status hw_set_state_device(hw_solver* h, const double* d_state);
hw_status hw_get_state_device(hw_solver* h, double* d_state);

/* One TVD-RK3 step (eq. RK).  dt > 0: that step; dt <= 0: dt = cfl dx / alpha (1D) or
 * cfl / (alpha/dx + beta/dy) (2D) from the current state.  Transactional: on
 * HW_ENONFINITE the state is left at its value before the step.  Synchronises. */
hw_status hw_step(hw_solver* h, double dt);

/* nsteps steps of fixed dt (> 0) or CFL dt (<= 0), enqueued without synchronising and
 * without the transactional copy.  For a batch, dt <= 0 gives every instance its own
 * CFL step.  The non-finite check is reported by the next synchronising call. */
hw_status hw_steps(hw_solver* h, int nsteps, double dt);

/* Advances to time T with CFL steps, the last one clipped to reach T exactly; at most
 * max_steps steps.  steps and t_reached (may be NULL) receive the totals. */
hw_status hw_run(hw_solver* h, double T, long max_steps, long* steps, double* t_reached);

/* Semi-discrete operator only: d_L = L(d_in) (eq. odeH / ode2) with the Lax-Friedrichs
 * speed of d_in; d_limited (may be NULL) receives d_in with the Step-1/Step-4 modified
 * first moments.  Arrays as in hw_set_state_device.  The flags of this evaluation are
 * available through hw_get_flags(h, 0, ...) when flag export is on. */
hw_status hw_apply_operator(hw_solver* h, const double* d_in, double* d_L, double* d_limited);

/* Replaces the linear weights (e.g. random positive weights every step, Section 3.1). */
hw_status hw_set_linear_weights(hw_solver* h, const double* lim_w, const double* rec_w);

/* Flag export: when on, every stage writes its troubled flags T and hybrid mask H.
 * hw_get_flags copies those of stage s (0, 1, 2) of the last step (or of the last
 * operator call, s = 0) into host arrays of `cells` bytes. */
hw_status hw_set_flag_export(hw_solver* h, int on);
hw_status hw_get_flags(hw_solver* h, int stage, unsigned char* T, unsigned char* H);

/* Time (per instance for a batch: times[n]) and completed step count. */
hw_status hw_get_time(hw_solver* h, double* times, long* steps);
/* Sets the time of the current state (every instance of a batch); hw_set_state sets it to
 * 0.  Only time-dependent boundary data (HW_BC_DMR) and hw_run's final time read it. */
hw_status hw_set_time(hw_solver* h, double t);

/* A one-dimensional handle on meshes of cells of different sizes (Section 2.1: every
 * polynomial of Steps 1-2 is defined by moment conditions on the cells of its stencil, and
 * the artificial linear weights do not depend on the geometry; the Introduction names this
 * independence as the point of the method).  faces: host array of nx + 1 finite, strictly
 * increasing face coordinates (copied); for a batch, instance after instance, n_b + 1 per
 * instance (sum of sizes + number of instances in all); cell i is
 * [faces[i], faces[i+1]], its first moment is (1/dx_i) int u (x - x_i)/dx_i dx.  The
 * library solves the polynomials' conditions once per cell on the device; the stage
 * kernel then evaluates them with the cell's own size (KXRCF with h = dx_i / 2, eq. odeH
 * with dx_i), and the CFL step uses the smallest cell (of each instance).  Periodic meshes wrap the
 * neighbour sizes; a mirrored ghost at a transmissive or reflective boundary has the size
 * of the cell it mirrors.  faces = NULL returns to the configuration's uniform meshes.  2D
 * handles get HW_EINVAL, and so do faces that are not strictly increasing.  Fixes the
 * launch form (256-cell tiles, one workgroup per tile: hw_batch_tune and hw_batch_set_form
 * then return HW_EINVAL); captured step graphs are rebuilt.  Tables of 112 doubles per
 * cell are kept on the device. */
hw_status hw_set_mesh_1d(hw_solver* h, const double* faces);

/* Run statistics.  alpha (may be NULL) receives the Lax-Friedrichs speed of the current
 * state per direction (1 value in 1D, 2 in 2D; the maximum of the spectral radius at the
 * cell averages, Section 2.1 Step 3 / Section 2.2 Step 6, over all cells and, for a batch,
 * all instances).  flagged and hybrid (may be NULL) receive 3 counts each: the troubled
 * cells (Steps 1 / 4) and the cells reconstructed by HWENO (Steps 2 / 5) in stages 1, 2, 3
 * of the last step (stage 1 only after an operator call).  2D handles always keep them;
 * 1D handles count them from exported flags (hw_set_flag_export), and report -1 while
 * export is off.  Without troubled-cell detection the counts are 0. */
hw_status hw_get_stats(hw_solver* h, double* alpha, long* flagged, long* hybrid);

/* Times nsteps steps (fixed dt > 0 or CFL dt) with HIP events around every stage and
 * between its launches on the handle's stream; ms_stage receives the mean duration of one
 * stage (in 2D its four launches), ms_step the mean wall time of one step, and ms_kernels
 * (4 doubles, may be NULL) the mean duration of each launch of a stage: 2D flags,
 * limiter, HWENO, stage kernel (the first three 0 without troubled-cell detection); 1D:
 * 0, 0, 0, stage kernel.  Any pointer may be NULL. */
hw_status hw_profile_steps(hw_solver* h, int nsteps, double dt, double* ms_stage, double* ms_step,
                           double* ms_kernels);

/* Batched form: runs nsteps CFL steps of every instance through a captured HIP graph of
 * the step's launches; persistent = 1 runs each stage as one persistent grid over the
 * (instance, tile) work list, 0 as one workgroup per work item, -1 the form picked by
 * hw_batch_tune (one workgroup per work item until it has run). */
hw_status hw_batch_steps(hw_solver* h, int nsteps, int persistent);

/* Autotuner of the batched stage: times one captured step (3 replays after a warm-up)
 * on the handle's own workload for every tile width (64, 128, 256, 512 cells = 1, 2, 4, 8
 * waves per workgroup) and launch form (one workgroup per tile; persistent grids of
 * 1, 2, 4, 8 workgroups per compute unit), keeps the fastest for later calls, and leaves
 * the state, times and step counts as they were.  choice (may be NULL) receives three
 * ints: tile width, persistent (0/1), persistent grid size (0 when not persistent).  The
 * halo is fixed at three cells by the stencil. */
hw_status hw_batch_tune(hw_solver* h, int* choice);

/* Sets the batched launch form directly (e.g. a choice hw_batch_tune made earlier for the
 * same workload and kept by the caller): tile width 64, 128, 256 or 512 cells, persistent
 * 0 or 1, and for a persistent form the grid size (>= 1 workgroups).  Every form computes
 * the same values; only the launch changes.  HW_EINVAL for other values or a 2D handle. */
hw_status hw_batch_set_form(hw_solver* h, int tile, int persistent, int grid);

/* ---- Reverse mode (Section 2.2 operator and eq. RK, differentiated).  Two-dimensional
 * handles: advection and Burgers on meshes whose sides are periodic or transmissive; Euler
 * (the characteristic limiter and HWENO reconstruction of Remark 4 differentiated
 * including the eigenvectors' dependence on the cell average) on meshes whose sides are
 * periodic, transmissive or reflective, each ghost cell being the mirror image of the cell
 * beside the side as in the forward operator, on the forward step (HW_BC_STEP: the
 * position and face rules above, the prescribed inflow state carrying no dependence on the
 * state; solid cells are never updated, so their rows of the operator are zero and a step
 * maps them to themselves) and on the double Mach reflection (HW_BC_DMR, with troubled-cell
 * detection: its prescribed ghosts and exact face states depend on time only; the wall and
 * outflow ghosts mirror as above); other handles (1D, batched, the double Mach reflection
 * without detection) get HW_EINVAL.
 * Troubled-cell flags, hybrid masks and Lax-Friedrichs speeds are those of the forward
 * evaluation and are held fixed (they are piecewise constant in the state); inside tau the
 * absolute value is differentiated as sign(x), sign(0) = 0.  Cotangents are device arrays
 * laid out like the state ([3][ncomp][ny][nx]) and are inner products in the plain
 * Euclidean sense over all stored numbers.  Work is enqueued on the handle's stream.  The
 * Euler reverse keeps about 1 KB of work arrays per cell (allocated on first use). */

/* d_out = (d L(d_in) / d d_in)^T d_lambda, with L the operator of hw_apply_operator (the
 * limiter included).  d_out must not alias d_in or d_lambda. */
hw_status hw_apply_operator_adjoint(hw_solver* h, const double* d_in, const double* d_lambda,
                                    double* d_out);

/* Advances the current state by nsteps TVD-RK3 steps of fixed dt > 0 (the same kernels
 * as hw_steps) and keeps a device checkpoint of the state every k steps for hw_adjoint
 * (ceil(nsteps / k) states, plus 3k + 1 states of segment workspace; Euler with
 * troubled-cell detection also keeps, for each of the segment's 3k stages, the flags,
 * hybrid masks, limited moments, HWENO edge values and work lists of its replay: about
 * (74 + 128 NG) bytes per cell and stage; the double Mach reflection also each stage's
 * table of prescribed ghosts and each step's time, so that the replay sees the boundary
 * data of the recorded run).  On a non-finite result returns HW_ENONFINITE
 * and no run is recorded. */
hw_status hw_forward_ckpt(hw_solver* h, int nsteps, double dt, int k);

/* Gradient of the recorded run: d_grad_U0 = (d U(T) / d U(0))^T d_lambda_T, U(0) being
 * the state at the start of the last hw_forward_ckpt and U(T) the state after it.  Each
 * k-step segment is recomputed from its checkpoint (bit for bit the recorded run) and
 * then reversed stage by stage.  Needs a recorded run (else HW_ESTATE); leaves the state
 * unchanged and may be called again with another d_lambda_T. */
hw_status hw_adjoint(hw_solver* h, const double* d_lambda_T, double* d_grad_U0);

/* ---- For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  The same operator as hw_apply_operator
 * (the same kernels and results) for a two-dimensional configuration, without a handle:
 * d_L = L(d_in) and, if d_limited is not NULL, d_in with the limited first moments; arrays
 * [3][ncomp][ny][nx] in device memory, owned by the caller.  stream: a hipStream_t of the
 * current device, or NULL for the null stream; the work is enqueued there and the call
 * does not synchronise.  cfg is validated as by hw_create (dim must be 2).
 *
 * Nothing is allocated: the speeds, list counters, flags, hybrid masks, work lists,
 * limited moments and HWENO edge values live in one static device array of
 * HW_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends.  A mesh whose buffers
 * need more (about 330 bytes per cell for Euler with ng_edge = 2, 460 with ng_edge = 3;
 * 90 and 122 for scalar laws; nothing beyond a 2 KiB header without troubled-cell
 * detection) is rejected with HW_EINVAL.  Every call on one GPU uses that GPU's array
 * and clears what must start at zero; calls that overlap on one GPU (concurrent streams,
 * threads) race and give wrong results. */
#define HW_NOALLOC_SCRATCH_BYTES (64u << 20)
hw_status hw_apply_operator_noalloc(const hw_config* cfg, const double* d_in, double* d_L,
                                    double* d_limited, void* stream);

const char* hw_last_error(const hw_solver* h);
const char* hw_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* HWENO_H */
