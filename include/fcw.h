/*
 * fcw.h - C ABI of the explicit / semi-explicit immersed-boundary spectral-cell
 * wave solver for AMD Instinct MI355X (gfx950).
 *
 * The library advances the semi-discrete system  M u'' + K u = F  (paper eq. semi)
 * that the finite/spectral cell method builds on a Cartesian grid of GLL-Lagrange
 * cells (Sec. 2.2) over a box from which a union of balls (voids) is removed.  Cells
 * inside a void are dropped; cells that meet no void share one reference stiffness;
 * each cut cell carries its own stiffness and mass, integrated by a space tree with
 * the indicator alpha^FCM (Sec. 2.2, eq. weak_form_extended), eigenvalue-stabilised
 * (Sec. 2.6) and HRZ-lumped (Sec. 2.4).  Time stepping is the central difference
 * method (Sec. 2.3, eq. cdm) with the Newmark beta = 0 start-up (Alg. newmark).
 *
 * Conventions
 *  - Every function returns an fcw_status; nothing throws or aborts across the ABI.
 *    fcw_last_error() gives a thread-local message for the last non-OK status.
 *  - Call order: fcw_assemble_cells -> fcw_stabilize_cut_cells -> fcw_critical_dt
 *    (optional before stepping when dt is given) -> fcw_step_explicit / fcw_run.
 *    A call out of order returns FCW_E_STATE and leaves the context unchanged.
 *  - Host arrays in descriptors are copied during the call; the context owns every
 *    device allocation it makes until fcw_destroy.  State vectors are caller-owned
 *    device buffers, borrowed for the duration of the call.
 *  - Work is enqueued on the context's stream (desc.stream, a hipStream_t; NULL means
 *    the default stream).  Only calls that return host values synchronise.
 *  - DOF layout: node-lexicographic over the full structured node grid
 *    (n_k = ncells_k * p + 1 nodes per direction, x fastest), components stored one
 *    after another (dof = comp * nnodes + node), right-hand sides one after another
 *    (index = rhs * ndof + dof).  Nodes of no active cell have zero mass and stay 0.
 *  - State precision: FCW_FP64 stores u, d as double; FCW_FP32 and FCW_BF16 store
 *    them as float (FCW_BF16 only changes the operands of the stiffness product).
 *  - A context is not thread-safe; distinct contexts are.
 */
#ifndef FCW_H
#define FCW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fcw_ctx fcw_ctx;
typedef int32_t fcw_status;

enum {
  FCW_OK = 0,
  FCW_E_ARG = -1,         /* invalid argument (shape, range, source in a void, ...) */
  FCW_E_NOMEM = -2,       /* device allocation failed */
  FCW_E_DEVICE = -3,      /* HIP runtime error; the context is poisoned */
  FCW_E_STATE = -4,       /* call out of order */
  FCW_E_NOCONV = -5,      /* an iterative eigen-solve did not converge */
  FCW_E_UNSTABLE = -6,    /* dt above the critical step (detected growth) */
  FCW_E_UNSUPPORTED = -7  /* configuration not built into this library */
};

enum { FCW_FP64 = 0, FCW_FP32 = 1, FCW_BF16 = 2 };

/* Problem description (Sec. 2.1-2.2).  dim 2 or 3; ncomp 1 (scalar wave, eq.
 * scalar_wave_equation: rho u'' - div(rho c^2 grad u) = rho f) or 3 (isotropic
 * linear elasticity with E, nu, rho; dim must be 3).  Cells are cubes of edge
 * (hi-lo)/ncells, equal in every direction.  Voids: nvoids balls (centre [dim],
 * radius); a point is fictitious iff |x-c|^2 < r^2 for some void (or, with a cube,
 * iff it lies outside the cube).  alpha is the
 * indicator value in the fictitious domain.  The outer box boundary and the void
 * surfaces carry homogeneous Neumann conditions (natural).  tree_depth: depth of the
 * space tree in cut cells (leaf edge h / 2^depth).  precision: FCW_FP64 / FCW_FP32 /
 * FCW_BF16 for the per-step stiffness product; all setup runs in FP64. */
typedef struct {
  int32_t dim, ncomp;
  int32_t ncells[3];
  double lo[3], hi[3];
  int32_t p, tree_depth;
  int32_t nvoids;
  const double* void_center; /* host, [nvoids][dim], copied */
  const double* void_radius; /* host, [nvoids], copied */
  double alpha, rho, c, E, nu;
  int32_t precision;
  void* stream;              /* hipStream_t or NULL */
  /* Optional rotated cube (Sec. 3.1): with cube_half > 0 the physical domain is the cube
   * {x : |sum_k (x_k - cube_center_k) cube_rot[3k + j]| <= cube_half for every axis j}
   * minus the voids; cube_rot is row-major [3][3] (the top-left dim x dim block is used),
   * a rotation whose column j is the cube's axis j.  Cells entirely outside the cube are
   * dropped like cells inside a void.  cube_half = 0: no cube. */
  double cube_center[3];
  double cube_half;
  double cube_rot[9];
} fcw_problem_desc;

/* Source with Ricker time function f_t (eq. source_time, t_s = 2 sqrt(6)/(pi f0)).
 * sigma = 0: point source, F(t) = f_t(t) * amp * rho * N(x) * dir_c on component c (dir
 * ignored for scalar problems).
 * sigma > 0: volumetric Gaussian source of Sec. 3.1, f(y, t) = f_t(t) * amp *
 * exp(-|y - x|^2 / (2 sigma^2)), so F_i(t) = f_t(t) * int alpha^FCM rho amp exp(...) N_i dy
 * (times dir_c), integrated once per call that changes the sources: over the active cells
 * within 8 sigma of x, each split into m^dim boxes (m = ceil(h / sigma), at most 64) with
 * a Gauss-Legendre rule of p + 3 points per direction and the pointwise indicator.  Its
 * load enters the increment before each step (one small launch per step).  Volumetric
 * sources are taken by fcw_step_explicit and fcw_run; the other stepping calls return
 * FCW_E_UNSUPPORTED for them. */
typedef struct {
  double x[3], dir[3], f0, amp;
  double sigma;
} fcw_source;

typedef struct {
  int64_t ndof, nnodes, ncells, n_cut, n_uncut, n_out;
  int32_t n_loc, precision;
  int64_t footprint_bytes; /* device bytes held by the context */
  double dt_crit;          /* 0 until fcw_critical_dt has run */
  double min_evs_margin;   /* min over cut cells of |lambda_i/lambda_max - f_lambda| */
} fcw_info;

/* Classify cells, build the reference element and integrate every cut cell with the
 * space tree (Sec. 2.2).  Allocates the context. */
fcw_status fcw_assemble_cells(const fcw_problem_desc* desc, fcw_ctx** out);

/* Eigenvalue-stabilise (Sec. 2.6: M^s from the eigenvectors of M^o whose eigenvalues
 * are below f_lambda * lambda_max, scaled to max(M^f)) and lump (Sec. 2.4, HRZ) the
 * cut-cell masses: diag = HRZ(M^o) + eps * diag(M^s); assemble the global diagonal
 * mass and prepare the per-step operands in the context precision.  Returns
 * FCW_E_NOCONV if a cut-cell eigen-solve does not converge. */
fcw_status fcw_stabilize_cut_cells(fcw_ctx* ctx, double eps, double f_lambda);

/* Critical step dt_crit = 2 / sqrt(lambda_max(K, M)) (Sec. 2.3) by FP64 Lanczos on
 * M^{-1/2} K M^{-1/2} from a fixed pseudo-random start vector.  Every 20 iterations the
 * largest Ritz value theta and the residual norm r = beta_k |s_k| of its Ritz pair are
 * computed; the iteration stops once r <= rtol * theta, and lambda_max is taken as
 * theta + r (Ritz values rise toward lambda_max from below, so the step errs on the safe
 * side).  Returns FCW_E_NOCONV, leaving *dt_crit untouched, when max_iter iterations do
 * not reach the tolerance.  Synchronises; writes *dt_crit. */
fcw_status fcw_critical_dt(fcw_ctx* ctx, int32_t max_iter, double rtol, double* dt_crit);

/* Advance nrhs independent right-hand sides by nsteps central-difference steps
 * (eq. cdm in increment form: d_{k+1} = d_k + dt^2 M^{-1}(F_k - K u_k),
 * u_{k+1} = u_k + d_{k+1}, where d_k = u_k - u_{k-1}).
 *   u, d : device, [nrhs][ndof] in the state precision, in/out.
 *   src  : host, [nrhs] one point source per right-hand side (may be NULL: F = 0).
 *   t0   : time of the first step of this call; step j uses F at t0 + j*dt.
 *   start: nonzero on the first call of a run; d then holds dt * v_0 and the first
 *          step is the Newmark beta = 0 start-up u_1 = u_0 + dt v_0 + dt^2/2 a_0.
 * Returns FCW_E_ARG for a source outside the box or inside a void. */
fcw_status fcw_step_explicit(fcw_ctx* ctx, int32_t nrhs, void* u, void* d,
                             const fcw_source* src, double t0, double dt,
                             int32_t nsteps, int32_t start);

/* Size in bytes of the fixed device work array of fcw_step_explicit_noalloc (64 MiB; each
 * device the library runs on holds one until the process ends). */
#define FCW_NOALLOC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory during the call (tight serving loops,
 * harnesses that forbid hipMalloc): fcw_step_explicit with
 * the same arguments, results and errors, whose work areas (load vectors, cut-cell
 * products, the ping-pong partner of u) live in one fixed per-device array of
 * FCW_NOALLOC_SCRATCH_BYTES instead of buffers the context allocates.  It calls no
 * hipMalloc / hipFree.  Needs about nrhs * ndof * state bytes + nrhs * n_cut * n_loc *
 * state bytes + 136 KiB; larger calls return FCW_E_ARG (fcw_step_explicit serves them).
 * Every call on one device shares that device's array: calls that overlap on one device
 * (from other threads or on other streams) race; calls in sequence on one stream do not.
 * With sources the call synchronises its stream once while it stages their load vectors. */
fcw_status fcw_step_explicit_noalloc(fcw_ctx* ctx, int32_t nrhs, void* u, void* d,
                                     const fcw_source* src, double t0, double dt,
                                     int32_t nsteps, int32_t start);

/* Outcome of one problem of a batched run (fcw_run), written when the call returns. */
typedef struct {
  int32_t status;      /* FCW_OK, or FCW_E_UNSTABLE when growth was detected (see fcw_run) */
  int32_t steps_done;  /* steps taken; below nsteps when the problem was stopped early */
  double dt_used;      /* the step size of the run (after the dt <= 0 rule) */
  double growth;       /* last ratio of the mass-free increment norms sum d_i^2 between two
                          checks (0 before the second check or without checks) */
} fcw_run_result;

/* Largest number of receivers of one problem in a run. */
#define FCW_MAX_RECEIVERS 64

/* One problem's share of a batched run (fcw_run). */
typedef struct {
  fcw_ctx* ctx;
  int32_t nrhs;
  void* u;                /* device [nrhs][ndof], in/out */
  void* d;                /* device [nrhs][ndof], in/out (dt * v_0 on a start call) */
  const fcw_source* src;  /* host [nrhs] or NULL */
  double t0;              /* time of the first step of this call */
  double dt;              /* step; <= 0 selects the rule of Sec. 3.3,
                             dt = min(0.9 dt_crit, dt_max) (fcw_critical_dt must have run) */
  double dt_max;          /* cap of that rule; <= 0 means none */
  int32_t nsteps;         /* steps of this problem (problems may differ) */
  int32_t start;          /* nonzero on the first call of a run (Newmark beta = 0 start-up) */
  /* Observers (Sec. 3.2, observer traces): nrec points (host [nrec][3], copied; 0 <= nrec
   * <= FCW_MAX_RECEIVERS; each inside the box; points on or beyond an immersed boundary
   * read the field that the fictitious-domain discretisation defines there).  The field
   * u_h(x_r) = sum_a N_a(x_r) u_a of the cell holding x_r (the same cell rule as for
   * sources) is written for the state before the first step and after every step:
   * traces is device double [nrhs][nsteps + 1][nrec][ncomp]; row k holds u_k of this call
   * (row 0 = the state passed in).  NULL / 0: no traces. */
  int32_t nrec;
  const double* rec_x;
  double* traces;
  /* Growth detection (Sec. 2.3 stability limit): every check_every steps the library
   * computes s = sum_i d_i^2 per right-hand side (FP64) and synchronises.  The problem is
   * stopped with FCW_E_UNSTABLE when s is not finite or when s grew by more than 1e6 over
   * each of three consecutive check intervals (a Ricker onset from rest can do neither:
   * its amplitude grows by at most e^24 in total, concentrated at the start; a step
   * above dt_crit amplifies the highest mode by a factor above one per step).  0: no
   * checks.  Items that check must share one check_every. */
  int32_t check_every;
  fcw_run_result* result; /* host, may be NULL */
  double* energy;         /* host [nrhs] or NULL: discrete energy after the last step,
                             E = 1/2 v^T M v + 1/2 u_{k+1}^T K u_k with v = d / dt */
} fcw_run_item;

enum { FCW_RUN_GRAPH = 1 };

/* Advance several problems, each by its own nsteps central-difference steps.  Problems
 * of the first problem's kind (2-D scalar with the same p and precision, or 3-D with the
 * same p, components and precision) are advanced together: one cut-cell launch and one
 * step launch per step cover every problem, right-hand side and tile of the group (3-D:
 * the first problem's step configuration for all, its resident blocks shared out by
 * tiles), and problems that have finished their steps drop out of later launches.  Other
 * problems run one after another.  All work goes on the stream of the first problem's context.  With
 * FCW_RUN_GRAPH the launches of a group are captured once into a HIP graph and replayed
 * (the graph is cached and reused while the group's shape is unchanged); a group with
 * receivers or growth checks runs without a graph.  Sources, state layout and errors as
 * in fcw_step_explicit.  The call synchronises when an item checks growth, asks for the
 * energy or has a result to fill; an unstable problem stops at the check that found it
 * (its state is that of the check) while the others go on, and the call then returns
 * FCW_E_UNSTABLE (every result says which problems). */
fcw_status fcw_run(const fcw_run_item* items, int32_t n, int32_t flags);

/* Autotuner of the step kernel: times every compiled tile configuration for this
 * problem kind on scratch state (nrhs right-hand sides, nsteps steps each, F = 0) and
 * keeps the fastest for later fcw_step_explicit calls.  *chosen (may be NULL)
 * receives its index.  Synchronises; the caller's state is not touched. */
fcw_status fcw_autotune(fcw_ctx* ctx, int32_t nrhs, int32_t nsteps, int32_t* chosen);

/* Tile configuration i of this problem kind: cells per tile (x, y, z) and its time per
 * step in microseconds from the last fcw_autotune (0 if not timed); *count receives the
 * number of configurations.  FCW_E_ARG when i is out of range (count still set). */
fcw_status fcw_tile_config(const fcw_ctx* ctx, int32_t i, int32_t tile[3], double* us_per_step,
                           int32_t* count);

/* Name of the step kernel of tile configuration i, as a profiler prints it (for
 * example "fcw::step2d_kernel<float, 4, 16, true>"), zero-terminated into buf of cap
 * bytes.  FCW_E_ARG when i is out of range or buf is too small. */
fcw_status fcw_tile_name(const fcw_ctx* ctx, int32_t i, char* buf, int32_t cap);

/* Use tile configuration i (as listed by fcw_tile_config) for later steps. */
fcw_status fcw_select_tile(fcw_ctx* ctx, int32_t i);

/* Queue the context's later work on another stream (a hipStream_t; NULL means the
 * default stream), for instance to set a problem up on one stream and step it on
 * another.  Synchronises the old stream first, so nothing queued there is still
 * running when work arrives on the new one. */
fcw_status fcw_set_stream(fcw_ctx* ctx, void* stream);

/* Average duration in microseconds of one launch of the step's main kernel (*main_us:
 * the tile or 2-D kernel of the selected configuration) and of the cut-cell product
 * kernel (*cut_us; 0 without cut cells), each timed over nsteps launches back to back,
 * captured into a HIP graph and replayed between HIP events on the context's stream (so
 * host launch gaps between short kernels are not counted), on scratch state with nrhs
 * right-hand sides.  For measurement; the caller's state is not touched.  Synchronises. */
fcw_status fcw_kernel_times(fcw_ctx* ctx, int32_t nrhs, int32_t nsteps, double* main_us,
                            double* cut_us);

/* Largest block of coupled implicit DOFs of the IMEX step (each block's matrices are
 * held dense; the implicit set as a whole has no such limit). */
#define FCW_IMEX_MAX_NC 16384

/* Set up the semi-explicit (IMEX) scheme of Sec. 2.5 (Alg. imex) for step size dt:
 * the implicit DOFs are those of the nodes of the cut cells (every component), the
 * rest of the active DOFs are explicit.  Assembles M^cc (the consistent cut-cell masses
 * M^o_e without stabilisation plus the GLL diagonals of the uncut cells on implicit
 * DOFs) and S = M^cc + dt^2/4 K^cc.  Both are block diagonal over the blocks of implicit
 * nodes linked through shared active cells; each block is assembled dense and factored
 * by Cholesky on the device (FP64).  The steps use the blocks of S^{-1} and (M^cc)^{-1}
 * (kept as the packed 32 x 32 tiles of their upper triangles) and the rows of K at the
 * implicit DOFs (kept as padded sparse rows).
 * *n_c receives the number of implicit DOFs, whose global indices
 * FCW_ARR_IMEX_DOFS exports (ascending: component-major, then node).
 * FP64 contexts only (FCW_E_UNSUPPORTED otherwise, when a block holds more than
 * FCW_IMEX_MAX_NC DOFs and when ndof >= 2^31);
 * FCW_E_NOCONV if a matrix is not positive definite.  Requires the stabilised state.
 * fcw_step_imex calls it itself when dt changes. */
fcw_status fcw_imex_prepare(fcw_ctx* ctx, double dt, int64_t* n_c);

/* Layout of the prepared implicit set (Sec. 2.5: S and M^cc are block diagonal over the
 * blocks of implicit nodes linked through shared active cells): *n_blocks blocks, the
 * largest with *largest DOFs, and *solve_bytes, the bytes of the packed upper tiles of
 * the blocks of S^{-1} (the same for (M^cc)^{-1}): what one step's implicit solve reads
 * per call.  Any output pointer may be NULL.  FCW_E_ARG before fcw_imex_prepare. */
fcw_status fcw_imex_layout(fcw_ctx* ctx, int32_t* n_blocks, int64_t* largest,
                           int64_t* solve_bytes);

/* nsteps semi-explicit steps (Alg. imex, beta = 1/4, gamma = 1/2): central differences on
 * the explicit DOFs (the step of fcw_step_explicit, in increment form), the trapezoidal
 * Newmark rule on the implicit DOFs with S of fcw_imex_prepare.
 *   u, d  device double [nrhs][ndof]: state and increment d = u_k - u_{k-1} (the
 *         increment is used on the explicit DOFs);
 *   v_c, a_c  device double [nrhs][n_c]: velocity and acceleration of the implicit DOFs
 *         in the FCW_ARR_IMEX_DOFS order (may be NULL when n_c = 0);
 *   src, t0: as for fcw_step_explicit; the load of the implicit step is taken at t_{k+1};
 *   start = 1: the call starts from rest (d = 0, v_c = 0): the explicit DOFs take the
 *         Newmark start-up (beta = 0) and a_c is computed from M^cc a_0 = F_0 - (K u_0).
 * FP64 contexts only.  Arrays are caller-owned; the call queues on the context's stream. */
fcw_status fcw_step_imex(fcw_ctx* ctx, int32_t nrhs, void* u, void* d, void* v_c, void* a_c,
                         const fcw_source* src, double t0, double dt, int32_t nsteps,
                         int32_t start);

/* nsteps central-difference steps (eq. cdm, Newmark beta = 0 start-up) with the block mass
 * M = diag(M^dd, M^cc) of the IMEX split: the consistent cut-DOF mass M^cc of
 * fcw_imex_prepare is inverted each step (a dense product with (M^cc)^{-1}), the other
 * DOFs keep their GLL diagonal (the consistent-mass spectral cell method).  Stable below
 * 2 / sqrt(lambda_max(M^{-1} K)) of that block mass, which the caller supplies through dt
 * (fcw_critical_dt covers the lumped mass only).  u, d, src, t0, start as for
 * fcw_step_explicit; FP64 contexts only; sets the scheme up for dt when needed. */
fcw_status fcw_step_consistent(fcw_ctx* ctx, int32_t nrhs, void* u, void* d,
                               const fcw_source* src, double t0, double dt, int32_t nsteps,
                               int32_t start);

/* Stiffness action r = K u (eq. semi, element by element, same kernels as the step):
 * u, r device [nrhs][ndof] in the state precision. */
fcw_status fcw_apply_stiffness(fcw_ctx* ctx, int32_t nrhs, const void* u, void* r);

/* Problem sizes and state; synchronises. */
fcw_status fcw_query(const fcw_ctx* ctx, fcw_info* info);

/* Copy an internal array to host memory (synchronous) for inspection:
 * which = FCW_ARR_*; *count receives the number of elements; dst may be NULL to
 * query the count; capacity is in elements. */
enum {
  FCW_ARR_CELL_CLASS = 0, /* int8 [ncells]: 0 OUT, 1 UNCUT, 2 CUT (after reclassification) */
  FCW_ARR_CUT_CELLS = 1,  /* int32 [n_cut_candidates] cell of each cut candidate (dropped ones are OUT in FCW_ARR_CELL_CLASS) */
  FCW_ARR_K_REF = 2,      /* double [n_loc*n_loc] uncut stiffness, row-major */
  FCW_ARR_K_CUT = 3,      /* double [n_cut_candidates*n_loc*n_loc] cut-cell stiffness */
  FCW_ARR_M_CUT = 4,      /* double [n_cut_candidates*n_s*n_s] cut-cell scalar consistent mass */
  FCW_ARR_LUMPED_CUT = 5, /* double [n_cut_candidates*n_s] stabilised lumped diagonal */
  FCW_ARR_MASS = 6,       /* double [nnodes] assembled lumped mass */
  FCW_ARR_EVS_MARGIN = 7, /* double [n_cut_candidates] */
  FCW_ARR_IMEX_DOFS = 8   /* int64 [n_c] implicit DOFs of the prepared IMEX scheme */
};
fcw_status fcw_export(const fcw_ctx* ctx, int32_t which, void* dst, int64_t capacity,
                      int64_t* count);

/* Accuracy measure of Sec. 3.2 (eq. error): the average over n_obs observers of the
 * relative L2 error of a trace over n_s time samples,
 *   e = 1/n_obs sum_i ||Psi_i - Psi_i,ref||_2 / ||Psi_i,ref||_2,
 * with Psi_i = (Psi(x_i, t_1), ..., Psi(x_i, t_ns)).  Host arrays laid out as fcw_run
 * writes traces of one right-hand side and component ([rows][n_obs], row 0 the initial
 * state): sample s = 1..n_s is row s * sim_stride of sim and row s * ref_stride of ref
 * (so a reference run with a finer step is sampled at the same times).  Host only; no
 * context needed.  FCW_E_ARG when an observer's reference trace is zero. */
fcw_status fcw_trace_error(const double* sim, int64_t sim_stride, const double* ref,
                           int64_t ref_stride, int32_t n_samples, int32_t n_obs, double* e);

/* Release every device allocation of the context. */
void fcw_destroy(fcw_ctx* ctx);

/* ---- IGA-FCM: B-spline discretisation of the same immersed problem ----------------------
 * (Sec. 2.2: B-spline shape functions, the isogeometric variant of the finite cell method;
 * Sec. 2.4: row-sum lumping; Table methods: IGA-FCM, alpha stabilisation, epsilon = 0,
 * central differences).  Degree p, maximum continuity, open uniform knot vectors: n cells
 * of a direction carry n + p functions, cell c supports functions c .. c + p, DOF
 * i0 + nb0 (i1 + nb1 i2) with nb_k = n_k + p.  The mass is row-sum lumped,
 * m_i = int alpha rho N_i (positive on every DOF supported by a kept cell; the others are
 * inactive, with zero mass, and stay zero).  Scalar wave equation only; 2-D p = 2..4,
 * 3-D p = 2..3; FP64 or FP32 steps (the precision of the cells' context); at least
 * 2p + 1 cells per direction. */
typedef struct fcw_iga fcw_iga;
typedef struct {
  int64_t ndof;           /* prod nbasis */
  int32_t nbasis[3];      /* n_k + p (1 beyond dim) */
  int32_t n_s, precision; /* (p+1)^dim functions per cell; FCW_FP64 or FCW_FP32 */
  int64_t n_cut, n_uncut, n_out;
  double dt_crit;         /* 0 until fcw_iga_critical_dt has run */
  int64_t footprint_bytes;
} fcw_iga_info;

/* Build the B-spline problem from a context whose cells are assembled
 * (fcw_assemble_cells; no stabilisation needed): its classification and the tree
 * quadrature of its cut cells are reused, each element matrix transformed to the B-spline
 * basis of the same polynomial space.  The IGA object holds its own copies afterwards
 * (the cells' context may be destroyed).  Synchronises.  FCW_E_UNSUPPORTED for vector
 * problems, other degrees or BF16; FCW_E_ARG for fewer than 2p + 1 cells. */
fcw_status fcw_iga_create(fcw_ctx* cells, fcw_iga** out);

/* dt_crit = 2 / sqrt(lambda_max(M^{-1} K)) with the lumped mass (Sec. 2.3), by the FP64
 * Lanczos iteration of fcw_critical_dt (same rtol, max_iter and FCW_E_NOCONV rule). */
fcw_status fcw_iga_critical_dt(fcw_iga* iga, int32_t max_iter, double rtol, double* dt_crit);

/* nsteps steps of eq. cdm in increment form with the lumped mass, as fcw_step_explicit:
 * u, d device [nrhs][ndof] in the step precision (d = u_k - u_{k-1}; on a start call
 * d = dt v_0 and the first step is the Newmark beta = 0 start-up); src host [nrhs] point
 * sources (x, f0, amp; dir and sigma unused, sigma > 0 gives FCW_E_UNSUPPORTED), the load
 * of right-hand side r being f_t(t) rho amp N_i(x_s) with the Ricker f_t of eq.
 * source_time at t = t0 + k dt.  Asynchronous on the cells' stream; nrhs <= 64.
 * FCW_E_ARG for a source outside the box. */
fcw_status fcw_iga_step(fcw_iga* iga, int32_t nrhs, void* u, void* d, const fcw_source* src,
                        double t0, double dt, int32_t nsteps, int32_t start);

/* r = K u (the step kernel's stiffness action), device [nrhs][ndof], step precision. */
fcw_status fcw_iga_apply_stiffness(fcw_iga* iga, int32_t nrhs, const void* u, void* r);

fcw_status fcw_iga_query(const fcw_iga* iga, fcw_iga_info* info);

/* Copy an FP64 array to host memory (synchronous); as fcw_export. */
enum {
  FCW_IGA_ARR_MASS = 0,    /* double [ndof] row-sum lumped mass */
  FCW_IGA_ARR_K_CLASS = 1, /* double [(2p+1)^dim][n_s*n_s] stiffness of an uncut cell of
                              each position class q_0 + (2p+1)(q_1 + (2p+1) q_2), where
                              along a direction cell c of n has class c (c < p), p (inside)
                              or 2p - (n - 1 - c) (c > n - 1 - p); row-major */
  FCW_IGA_ARR_K_CUT = 2    /* double [n_cut_candidates][n_s*n_s] stiffness of each cut cell
                              in the order of FCW_ARR_CUT_CELLS (zero for dropped ones) */
};
fcw_status fcw_iga_export(const fcw_iga* iga, int32_t which, void* dst, int64_t capacity,
                          int64_t* count);

void fcw_iga_destroy(fcw_iga* iga);

/* Thread-local message of the last failing call ("" if none). */
const char* fcw_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FCW_H */
