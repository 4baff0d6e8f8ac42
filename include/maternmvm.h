/*
 * maternmvm.h - C ABI of the exact fast Matern kernel matrix-vector product
 * on AMD Instinct MI355X (gfx950), with the conjugate-gradient GP solve, the
 * linear fixed-effects (GLS) estimate and the posterior-mean predictor built
 * on it.
 *
 * Method (Langrene, Warin, Gruet et al., "Fast Gaussian process inference by
 * exact Matern kernel decomposition", arXiv 2508.01864):
 *   - the kernel sum  y_j = sum_i K(x_j, x_i) v_i  (Section 2, eq. Ky / kde)
 *     is split over the 2^d sign orthants into weighted empirical CDFs
 *     (eq. ECDFdelta; Proposition 1 for the L1 kernel, eq. L1_decomposition;
 *     Proposition 2 for the product kernel, eq. product_decomposition),
 *   - those CDFs are evaluated for every point at once by sorting (d = 1,
 *     Section 2.1, fast sum updating) or by divide and conquer on presorted
 *     coordinates (d >= 2, Section 2.2; the sorted subsets are computed once
 *     and stored, then reused by every product).
 * The result is exact up to floating-point rounding; it is not an
 * approximation.
 *
 * Conventions common to every call
 *   - All arithmetic is IEEE binary64.
 *   - Pointers documented as "device" must point to memory of the device that
 *     was current when the plan was created; "host" pointers are ordinary CPU
 *     memory.  The library never frees caller memory.
 *   - Matrices are column-major: element (i, c) of an n x k array with leading
 *     dimension ld is at index c*ld + i.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls enqueue work on it and return without waiting, unless the
 *     description says "synchronises".
 *   - Every call returns an mm_status.  On error the outputs are unspecified,
 *     no caller memory is freed, and mm_last_error() returns a message for the
 *     calling thread.
 *   - Point indices in inputs and outputs are the caller's order.
 *   - A plan must not be used from two streams at the same time.
 */
#ifndef MATERNMVM_H
#define MATERNMVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mm_plan_s *mm_plan;

typedef enum {
    MM_OK = 0,
    MM_ERR_ARG = 1,        /* invalid argument (size, pointer, NaN, unsupported nu/d/form) */
    MM_ERR_NOMEM = 2,      /* device allocation failed */
    MM_ERR_HIP = 3,        /* a HIP runtime call failed */
    MM_ERR_NOTPD = 4,      /* solve requested with a kernel form that is not positive definite */
    MM_ERR_BREAKDOWN = 5,  /* conjugate gradients met p^T A p <= 0 */
    MM_ERR_NOCONV = 6      /* conjugate gradients hit maxit before the tolerance */
} mm_status;

/* Multivariate kernel form (Section 2.2): L1 form k(||u||_1) (eq. L1_kernel)
 * or product form prod_k k(|u_k|) (eq. product_kernel).  They coincide for
 * nu = 1/2 (remark after eq. matern_l1_12) and for d = 1. */
typedef enum { MM_FORM_L1 = 0, MM_FORM_PRODUCT = 1 } mm_form;

/* Scaled Matern kernel  outputscale2 * k_nu(r / lengthscale)  (eq. scaled_kernel,
 * Appendix C eq. matern_1_2 / matern_3_2 / matern_5_2) with nu = two_nu / 2.
 *   two_nu        1, 3 or 5
 *   form          MM_FORM_L1 or MM_FORM_PRODUCT
 *   lengthscale   ell > 0, finite
 *   outputscale2  varsigma^2 > 0, finite                                      */
typedef struct {
    int32_t two_nu;
    int32_t form;
    double lengthscale;
    double outputscale2;
} mm_kernel;

/* Outcome of a conjugate-gradient solve. */
typedef struct {
    int32_t iters;           /* iterations performed (matrix-vector products of the loop) */
    double relres_max;       /* max over columns of ||r_c|| / ||b_c|| at exit: the recurrence
                                residual, or the recomputed one after a final check */
    int32_t converged_cols;  /* columns whose relative residual reached rtol */
    double true_relres;      /* the residual recomputed with a fresh product at exit:
                                ||y - H beta - (K + sigma2 I) alpha|| / ||y|| with fixed
                                effects, else max_c ||b_c - (K + sigma2 I) x_c|| / ||b_c||;
                                -1 when not computed (breakdown, calls without a check) */
} mm_solve_info;

/* Library version string. */
const char *mm_version(void);

/* Human-readable name of a status code. */
const char *mm_status_str(mm_status st);

/* Detail message of the last error raised on the calling thread ("" if none). */
const char *mm_last_error(void);

/*
 * Device memory of the library.  Every device buffer the library allocates
 * (plans, solvers, batches, preconditioners, temporaries) comes from
 * alloc(bytes, stream, ctx), which returns device memory of the current device
 * or NULL (the call then fails with MM_ERR_NOMEM), and goes back through
 * free(ptr, stream, ctx) of the allocator that provided it.  stream is passed
 * as NULL: the library synchronises the device before it releases a buffer,
 * so a stream-ordered caching allocator (torch's) may reuse it at once.
 * Both NULL restores hipMalloc / hipFree; exactly one NULL is MM_ERR_ARG.
 * Process-wide: set it while no other library call is running.  Pinned host
 * staging buffers are not affected.
 */
typedef void *(*mm_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*mm_free_fn)(void *ptr, void *stream, void *ctx);
mm_status mm_set_allocator(mm_alloc_fn alloc, mm_free_fn free, void *ctx);

/*
 * Upper bound of the device memory a plan for n points in dimension d needs,
 * including work buffers for products with up to nrhs right-hand sides.  Host
 * only; intended for admission control.  Returns 0 for invalid arguments.
 */
size_t mm_plan_footprint_bytes(int64_t n, int32_t d, int32_t nrhs, const mm_kernel *kernel);

/*
 * Build the stored sorting outputs for a point set (Section 2.2: the sorted
 * subsets for each coordinate are computed once and reused by every product).
 *   x       device, n x d column-major with leading dimension ldx >= n
 *   n       number of points, 1 <= n <= 2^30
 *   d       dimension, 1, 2 or 3
 *   kernel  host, the kernel (validated, copied)
 *   stream  stream for the build kernels
 *   out     host, receives the plan handle
 * The plan keeps its own copy of the (reordered) coordinates, so x may be
 * freed once the call's work on `stream` has completed.  Fails with
 * MM_ERR_ARG if any coordinate is NaN or infinite (synchronises to check).
 */
mm_status mm_plan_create(const double *x, int64_t n, int32_t d, int64_t ldx,
                         const mm_kernel *kernel, void *stream, mm_plan *out);

/*
 * Scan schedule of the plan's products at one padded width (the number of
 * right-hand sides rounded up to the column block: 1, 2, 4, multiples of 4
 * below 32, multiples of 32): columns per wavefront `wb`, positions per lane
 * run `e` (tiles of 64 / wb * e positions, 128 to 1024), and whether the
 * tile-aggregate pre-pass stores every run's within-tile carry for the main
 * launch (`runex`; d <= 2).  Every product of the plan at
 * that width uses it: matern_mvm, solvers and batches (a problem gives the
 * same bits alone and batched whenever their schedules agree).  The
 * schedules are an implementation choice of the divide-and-conquer sweeps
 * (Section 2.2) and never change the exact result beyond rounding; the
 * autotuner picks them by measurement.  Available: (wb, e) = (1, 4), (2, 8),
 * (4, 16), (4, 32), (32, 128) for every kernel, and also (1, 8), (1, 16),
 * (4, 8), (8, 16), (8, 32), (16, 32), (16, 64), (32, 64) for the product form
 * with nu = 3/2 in d = 2 and nu = 5/2 in d = 3; e = 0 selects the default run
 * length of the block.  MM_ERR_ARG for other values, a width that wb does not
 * divide, or while solvers or batches of the plan are alive.
 * mm_plan_set_kernel clears the plan's schedules.  Host only.
 */
mm_status mm_plan_set_schedule(mm_plan plan, int32_t width, int32_t wb, int32_t e, int32_t runex);

/* The schedule in effect at a width (set, or the default of that width). */
mm_status mm_plan_get_schedule(mm_plan plan, int32_t width, int32_t *wb, int32_t *e, int32_t *runex);

/* Replace the kernel (nu, form, lengthscale, outputscale) of a plan; the
 * stored sorting outputs are kept.  Later products on `stream` use the new
 * kernel; the lengthscale factors are evaluated on chip by every product, so
 * nothing is recomputed here and no work is enqueued.  MM_ERR_ARG while
 * solvers or batches of the plan are alive. */
mm_status mm_plan_set_kernel(mm_plan plan, const mm_kernel *kernel, void *stream);

/* Point count and dimension of a plan (host). */
mm_status mm_plan_info(mm_plan plan, int64_t *n, int32_t *d, mm_kernel *kernel);

/* Release a plan and every device buffer it owns (synchronises the device
 * with the plan's last stream).  NULL is accepted. */
mm_status mm_plan_destroy(mm_plan plan);

/*
 * Exact kernel matrix-vector product with nrhs right-hand sides
 * (Section 2, eq. Ky, evaluated by Prop. 1 or Prop. 2):
 *     y = (K + diag_shift * I) v
 * where K_ij = outputscale2 * k_nu(dist(x_i, x_j) / lengthscale).
 *   v      device, n x nrhs column-major, leading dimension ldv >= n
 *   y      device, n x nrhs column-major, leading dimension ldy >= n;
 *          must not overlap v
 *   nrhs   1 <= nrhs <= 256
 *   diag_shift  added times v (e.g. the noise variance sigma^2); may be 0
 */
mm_status matern_mvm(mm_plan plan, const double *v, int64_t ldv, double *y, int64_t ldy,
                     int32_t nrhs, double diag_shift, void *stream);

/*
 * matern_mvm without device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, hosts that forbid
 * allocation.  Same arguments, layouts, errors and results (bitwise) as
 * matern_mvm; the plan must have been created beforehand.  Its work buffers
 * (canonical input and sum, tile aggregates and carries, per-pass partial
 * slabs) come from one fixed scratch array of MM_NOALLOC_SCRATCH_MIB MiB in
 * device memory, which each device the library runs on holds until the
 * process ends.  Sizes whose work buffers exceed it are refused with
 * MM_ERR_ARG (the headline d = 2, n = 100,000 fits up to 4 right-hand sides;
 * use matern_mvm beyond).  Every call on a device shares that device's array:
 * calls that overlap on one device (concurrent streams or threads) race and
 * must be serialised by the caller.  Nothing in the array needs to start at
 * zero: every buffer is written before it is read.
 */
#define MM_NOALLOC_SCRATCH_MIB 256
mm_status matern_mvm_noalloc(mm_plan plan, const double *v, int64_t ldv, double *y, int64_t ldy,
                             int32_t nrhs, double diag_shift, void *stream);

/*
 * Exact product with the lengthscale derivative of the kernel matrix (the
 * gradients of the Section 2.3 examples, for every nu and both forms):
 *     y = (dK/d lengthscale) v.
 * With t = sqrt(2 nu) r / lengthscale the profile derivative is
 * -t k'(t) / lengthscale, a profile with one more channel in the basis of the
 * decomposition; the product form sums over the coordinates the products with
 * one factor differentiated.  The diagonal of K does not depend on the
 * lengthscale.  Arguments, layouts and errors as matern_mvm (no diag_shift).
 */
mm_status matern_mvm_dlengthscale(mm_plan plan, const double *v, int64_t ldv, double *y, int64_t ldy,
                                  int32_t nrhs, void *stream);

/*
 * Gaussian-process solve by conjugate gradients (Appendix A, Algorithm 2 with
 * the identity preconditioner and a null initial guess), each iteration one
 * product of the fast MVM:
 *     alpha = (K + sigma2 I)^{-1} (y - H beta)
 * With fixed_effects != 0 the mean is affine, m(x) = beta_0 + beta^T x
 * (eq. BetaLin), H = [1, x_1, ..., x_d], and beta is the generalised least
 * squares estimate of Section 3.2,
 *     beta = (H^T A^{-1} H)^{-1} H^T A^{-1} y,   A = K + sigma2 I,
 * obtained from one multi-column CG over [y, H]; otherwise beta = 0.
 *   y        device, n targets (caller order)
 *   sigma2   noise variance > 0
 *   rtol     tolerance of the returned solution: the residual recomputed with
 *            a fresh product, ||y - H beta - A alpha|| <= rtol ||y|| (with fixed
 *            effects) or ||y - A alpha|| <= rtol ||y||.  Each column stops when its
 *            recurrence residual reaches its tolerance (rtol at first); then the
 *            residual is recomputed, and if it misses rtol the column tolerances
 *            shrink and the iteration restarts from the recomputed residual
 *            (residual replacement; at most 8 checks)
 *   maxit    iteration limit >= 1
 *   alpha    device, n outputs (caller order)
 *   beta     host, d+1 outputs, or NULL when fixed_effects == 0
 *   info     host, may be NULL (info->true_relres: the recomputed residual)
 * The L1 form with nu >= 3/2 and d >= 2 is not positive definite and is
 * refused with MM_ERR_NOTPD (the product form is; Appendix B).  Returns
 * MM_ERR_NOCONV when maxit iterations end before the recomputed residual
 * meets rtol, and MM_ERR_BREAKDOWN on a non-positive curvature p^T A p; both
 * still write the last iterate and info.  Synchronises.
 */
mm_status gp_cg_solve(mm_plan plan, const double *y, double sigma2, int32_t fixed_effects,
                      double rtol, int32_t maxit, double *alpha, double *beta,
                      mm_solve_info *info, void *stream);

/*
 * Multi-column conjugate gradients (Appendix A, Algorithm 2, identity
 * preconditioner, null initial guess): X = (K + sigma2 I)^{-1} B.
 *   B     device, n x nrhs column-major, leading dimension ldb >= n
 *   X     device, n x nrhs column-major, leading dimension ldx >= n
 *   nrhs  1 <= nrhs <= 64
 * Columns are stopped independently; each must end with its recomputed
 * residual ||b_c - A x_c|| <= rtol ||b_c|| (same checks and restarts, status
 * rules and synchronisation as gp_cg_solve).
 */
mm_status gp_cg_solve_multi(mm_plan plan, const double *B, int64_t ldb, int32_t nrhs,
                            double sigma2, double rtol, int32_t maxit, double *X, int64_t ldx,
                            mm_solve_info *info, void *stream);

/*
 * Posterior mean at m new points (eq. gp_mean, eq. gp_mean_2):
 *     mean(z) = sum_i alpha_i K(z, x_i) + h(z)^T beta,  h(z) = [1, z_1..z_d]
 * computed exactly by the same decomposition on the union of the training
 * and prediction points with zero weights on the latter.
 *   alpha  device, n weights (caller order of the plan's points)
 *   beta   host, d+1 coefficients, or NULL for a zero mean function
 *   z      device, m x d column-major, leading dimension ldz >= m
 *   mean   device, m outputs
 * Synchronises (it builds and releases a temporary plan).
 */
mm_status gp_predict(mm_plan plan, const double *alpha, const double *beta, const double *z,
                     int64_t m, int64_t ldz, double *mean, void *stream);

/*
 * Posterior variance at m new points (eq. gp_variance):
 *     var(z) = K(z, z) - k_z^T (K + sigma2 I)^{-1} k_z,   K(z, z) = outputscale2,
 * the variance of the latent function (add sigma2 for a new observation).
 * k_z = K(X, z) comes from exact products on the union of the training and
 * prediction points with unit weights on the latter; the solves run by
 * multi-column conjugate gradients, 32 points at a time, each column to
 * ||r|| <= rtol ||k_z||.
 *   z      device, m x d column-major, leading dimension ldz >= m
 *   rtol   > 0; maxit >= 1 per block of points
 *   var    device, m outputs
 *   info   host (may be NULL): the largest iteration count and residual over
 *          the blocks, and the number of converged columns
 * Same status rules as gp_cg_solve (outputs written).  Synchronises.
 */
mm_status gp_variance(mm_plan plan, double sigma2, const double *z, int64_t m, int64_t ldz, double rtol,
                      int32_t maxit, double *var, mm_solve_info *info, void *stream);

/*
 * Rank-k pivoted Cholesky preconditioner (Appendix A, "Preconditioning"):
 * P = L L^T + sigma2 I with L L^T the pivoted Cholesky decomposition of K,
 * applied in conjugate gradients through the Woodbury identity
 *     P^{-1} r = r / sigma2 - L (I_k + L^T L / sigma2)^{-1} L^T r / sigma2^2.
 * The factorisation is greedy on the residual diagonal diag(K - L L^T): each
 * column takes the largest residual (smallest caller index among equal
 * values).  It stops after max_rank columns, when the pivot's residual is not
 * positive, or when the residual trace is at most tol * trace(K).  It does not
 * depend on sigma2, so one preconditioner serves solves with any noise level.
 *   max_rank  1 .. MM_PRECOND_MAX_RANK (capped at n)
 *   tol       >= 0 (0: always max_rank columns unless the residual vanishes)
 * Synchronises.  The preconditioner pins its plan (see the solver objects) and
 * must outlive the solvers that use it (mm_precond_destroy fails otherwise).
 */
#define MM_PRECOND_MAX_RANK 256
typedef struct mm_precond_s *mm_precond;

mm_status mm_precond_create(mm_plan plan, int32_t max_rank, double tol, void *stream, mm_precond *out);

/* Computed rank, residual trace sum(diag(K - L L^T)) and trace(K) (host). */
mm_status mm_precond_info(mm_precond pc, int32_t *rank, double *trace_residual, double *trace_k);

/* Copy L to device memory (n x rank column-major, leading dimension ldl >= n,
 * rows in the caller's point order; may be NULL) and the pivots to host
 * memory (rank caller indices in column order; may be NULL). */
mm_status mm_precond_factor(mm_precond pc, double *L, int64_t ldl, int32_t *pivots, void *stream);

/* Release a preconditioner (synchronises the device).  NULL is accepted. */
mm_status mm_precond_destroy(mm_precond pc);

/*
 * Solver objects: the conjugate-gradient solve of gp_cg_solve (Appendix A,
 * Algorithm 2, identity preconditioner, null initial guess; with fixed
 * effects the GLS of Section 3.2) split into steps, so that a caller can
 * advance many independent GP problems together.  A solver keeps its state on
 * the device; gp_cg_solve itself is create + iterate until done + finish +
 * destroy, and every path runs the same kernels, so a problem's iterates do
 * not depend on which other solvers share its batch (bitwise).
 * The solver reads the plan's stored orders and the kernel it had at
 * creation: while solvers of a plan are alive, mm_plan_set_kernel and
 * mm_plan_destroy on it fail with MM_ERR_ARG.  Several solvers may share one
 * plan.
 */
typedef struct mm_solver_s *mm_solver;
typedef struct mm_solver_batch_s *mm_solver_batch;

/* Upper bound of the device memory of one solver (its CG state, sweep
 * workspaces and the work tables of a batch it joins), excluding the plan;
 * host only, for admission control.  0 for invalid arguments. */
size_t mm_solver_footprint_bytes(int64_t n, int32_t d, int32_t fixed_effects, const mm_kernel *kernel);

/* Create a solver for (K + sigma2 I) alpha = y - H beta with the arguments of
 * gp_cg_solve (y: device, n targets in caller order; it is copied) and run
 * its initialisation on `stream`; *out receives the handle. */
mm_status mm_solver_create(mm_plan plan, const double *y, double sigma2, int32_t fixed_effects,
                           double rtol, void *stream, mm_solver *out);

/* As mm_solver_create, preconditioned by pc (Algorithm 2 with the solve
 * s_P of the pivoted Cholesky preconditioner; pc may be NULL for none).  The
 * Woodbury factors for this sigma2 are formed at creation.  Fixed effects
 * (at most 8 columns) are supported; the stop test stays on the residual
 * ||r_c|| <= rtol ||b_c||. */
mm_status mm_solver_create_pc(mm_plan plan, const double *y, double sigma2, int32_t fixed_effects,
                              double rtol, mm_precond pc, void *stream, mm_solver *out);

/* gp_cg_solve with the preconditioner pc (may be NULL). */
mm_status gp_pcg_solve(mm_plan plan, const double *y, double sigma2, int32_t fixed_effects, double rtol,
                       int32_t maxit, mm_precond pc, double *alpha, double *beta, mm_solve_info *info,
                       void *stream);

/* Enqueue `iters` further iterations (columns that reached rtol stay frozen;
 * iterating a solved problem changes nothing). */
mm_status mm_solver_iterate(mm_solver solver, int32_t iters, void *stream);

/* Columns still above rtol, whether a breakdown (p^T A p <= 0) occurred, and
 * the convergence summary so far (any output may be NULL).  Synchronises. */
mm_status mm_solver_poll(mm_solver solver, int32_t *active_cols, int32_t *breakdown,
                         mm_solve_info *info, void *stream);

/* Residual check of gp_cg_solve on the current iterate (Appendix A,
 * Algorithm 2; with fixed effects the Section 3.2 combination): the residual
 * recomputed with one fresh product, ||y - H beta - A alpha|| / ||y|| (fixed
 * effects) or max_c ||b_c - A x_c|| / ||b_c||, into *true_relres.  The solver
 * restarts from it (R = B - A X; the next direction is the residual, or its
 * preconditioned image).  *passed = 1 when it meets rtol: every column is
 * then frozen and further iterations change nothing.  Otherwise, when tighten
 * is nonzero and every column had converged by the recurrence, the column
 * tolerances shrink by 0.5 rtol / true_relres (clamped to [0.05, 0.5]) and
 * the missing columns (all columns with fixed effects) continue under
 * mm_solver_iterate.  The iterate X itself is unchanged.  Outputs may be NULL.
 * Synchronises. */
mm_status mm_solver_check(mm_solver solver, int32_t tighten, int32_t *passed, double *true_relres,
                          void *stream);

/* Write alpha (device, n, caller order) and beta (host, d+1, fixed effects
 * only) from the current iterate, with the status rules of gp_cg_solve
 * (MM_ERR_NOCONV / MM_ERR_BREAKDOWN still write the outputs).  Unless the
 * iterate was checked since its last iteration, the residual is recomputed
 * first as by mm_solver_check without tightening (info->true_relres).
 * Synchronises. */
mm_status mm_solver_finish(mm_solver solver, double *alpha, double *beta, mm_solve_info *info,
                           void *stream);

/* Release a solver (synchronises the device).  NULL is accepted. */
mm_status mm_solver_destroy(mm_solver solver);

/* Group `count` solvers (host array of handles; any mix of n, d, nu, forms and
 * column counts) for joint iteration: every iteration runs all their products
 * in one launch per kernel configuration, column width and phase, and all
 * their vector updates in one launch per step.  With use_graph != 0
 * the iterations are captured once into a HIP graph and replayed on a
 * private stream ordered after `stream`.  A solver whose per-pass partial
 * sums (passes x n x columns doubles) exceed 16 GiB cannot join a batch of
 * two or more (MM_ERR_ARG).  A solver may belong to several batches but must not be
 * iterated by two at the same time.  The solvers must outlive the batch. */
mm_status mm_solver_batch_create(mm_solver *solvers, int32_t count, int32_t use_graph,
                                 mm_solver_batch *out);

/* Launch schedule of a batch: workgroups per compute unit of the persistent
 * carry-scan grids (>= 1; the sweep launches run one workgroup per work item)
 * and the grid of the vector-update kernels (>= 1).  Results do not depend
 * on it. */
mm_status mm_solver_batch_set_schedule(mm_solver_batch batch, int32_t sweep_wg_per_cu,
                                       int32_t cg_grid);

/* Enqueue `iters` iterations of every solver of the batch. */
mm_status mm_solver_batch_iterate(mm_solver_batch batch, int32_t iters, void *stream);

/* Host array of count entries: columns still active per solver after the
 * last batch iteration, or -1 after a breakdown.  Synchronises. */
mm_status mm_solver_batch_poll(mm_solver_batch batch, int32_t *active, void *stream);

/* Release a batch (not its solvers).  NULL is accepted. */
mm_status mm_solver_batch_destroy(mm_solver_batch batch);

/*
 * Stochastic log-determinant of K + sigma2 I (Appendix A: Hutchinson's
 * estimator with partial Lanczos decompositions taken from conjugate
 * gradients, Algorithm 2 and eq. approximationLogDet):
 *     log det(K + sigma2 I) ~ (1/l) sum_i ||z_i||^2 e_1^T log(T_i) e_1,
 * where T_i is the Lanczos matrix of CG started from probe z_i with a null
 * initial guess (for Rademacher probes ||z_i||^2 = n, the paper's form).
 *   Z       device, n x nprobes column-major probes (caller order; the caller
 *           draws them, e.g. Rademacher or standard normal)
 *   nprobes 1..64
 *   steps   maximal CG (Lanczos) steps per probe
 *   rtol    a probe stops early when ||r|| <= rtol ||z|| (0: run all steps)
 *   logdet  host, the estimate
 *   quad    host, nprobes per-probe terms ||z_i||^2 e_1^T log(T_i) e_1 (may be NULL)
 *   lanczos_steps host, nprobes sizes of the T_i (may be NULL)
 * No preconditioner (gp_logdet_pc draws its probes from the preconditioner's
 * distribution).  Synchronises.
 */
mm_status gp_logdet(mm_plan plan, double sigma2, const double *Z, int64_t ldz, int32_t nprobes,
                    int32_t steps, double rtol, double *logdet, double *quad, int32_t *lanczos_steps,
                    void *stream);

/*
 * Preconditioned stochastic log-determinant (Appendix A, the preconditioned
 * log-determinant with the pivoted Cholesky preconditioner P = L L^T + sigma2 I):
 *     log det A = log det P + log det(P^{-1/2} A P^{-1/2}),
 *     log det P = n log sigma2 + log det(I_k + L^T L / sigma2)   (Sylvester),
 * the second term by Lanczos quadrature from preconditioned CG (Algorithm 2
 * with s_P = P^{-1}): probes z_i = L g1_i + sqrt(sigma2) g2_i are N(0, P)
 * draws, so P^{-1/2} z_i ~ N(0, I) and each (z_i^T P^{-1} z_i) e_1^T log(T_i) e_1
 * is an unbiased term (T_i the Lanczos matrix of P^{-1/2} A P^{-1/2} from the
 * PCG coefficients).  The caller draws the standard normal numbers:
 *   pc      preconditioner of this plan (mm_precond_create), rank k = its rank
 *   G1      device, k x nprobes column-major, leading dimension ldg1 >= k
 *           (may be NULL when k = 0)
 *   G2      device, n x nprobes column-major (caller order), ldg2 >= n
 *   nprobes 1..64 (solved in blocks of 8); steps, rtol as gp_logdet
 *   logdet  host, the estimate (log det P included)
 *   quad    host, nprobes per-probe terms (without log det P; may be NULL)
 *   lanczos_steps host, nprobes sizes of the T_i (may be NULL)
 *   logdet_precond host, log det P (may be NULL)
 * Synchronises.
 */
mm_status gp_logdet_pc(mm_plan plan, double sigma2, mm_precond pc, const double *G1, int64_t ldg1,
                       const double *G2, int64_t ldg2, int32_t nprobes, int32_t steps, double rtol,
                       double *logdet, double *quad, int32_t *lanczos_steps, double *logdet_precond,
                       void *stream);

/*
 * Log marginal likelihood and its gradient (eq. gp_log_likelihood and eq.
 * gp_log_likelihood_derivative; Appendix A), zero mean, A = K + sigma2 I:
 *     L = -1/2 y^T A^{-1} y - 1/2 log det A - n/2 log(2 pi),
 *     dL/dtheta = 1/2 alpha^T (dA/dtheta) alpha - 1/2 tr(A^{-1} dA/dtheta),
 * alpha = A^{-1} y.  One multi-column CG solves [y, z_1 .. z_l] together
 * (null start, each column to rtol) and records the Lanczos coefficients of
 * the probe columns.  Then
 *   log det A          ~ (1/l) sum_i ||z_i||^2 e_1^T log(T_i) e_1
 *                        (eq. approximationLogDet),
 *   tr(A^{-1} dK/dl)   ~ (1/l) sum_i (A^{-1} z_i)^T (dK/dl z_i)
 *                        (Hutchinson; one derivative product of the probes),
 *   tr(A^{-1})         ~ (1/l) sum_i z_i^T A^{-1} z_i,
 * and for the output scale tr(A^{-1} dK/d outputscale2) = (n - sigma2
 * tr(A^{-1})) / outputscale2 with the same probes.
 *   y        device, n targets (caller order)
 *   Z        device, n x nprobes column-major probes (caller order),
 *            leading dimension ldz >= n; 1 <= nprobes <= 63 (nprobes = 31
 *            fills a 32-column sweep)
 *   maxit    iteration limit >= 1 (also the largest Lanczos matrix)
 *   rtol     per-column stop test ||r_c|| <= rtol ||b_c|| (> 0)
 *   info     host, the estimates
 *   alpha    device, n outputs A^{-1} y (caller order), or NULL
 * Returns MM_ERR_NOCONV (info still written) when a column did not reach
 * rtol within maxit, MM_ERR_NOTPD for the L1 form with nu >= 3/2, d >= 2.
 * Synchronises.
 */
typedef struct {
    double lml;                  /* the log marginal likelihood estimate */
    double quad;                 /* y^T A^{-1} y */
    double logdet;               /* stochastic log det A */
    double dlml_dlengthscale;
    double dlml_dsigma2;
    double dlml_doutputscale2;
    double trace_dk_dlengthscale; /* estimate of tr(A^{-1} dK/dl) */
    double trace_inv;            /* estimate of tr(A^{-1}) */
    double relres_max;           /* largest final relative residual over the columns */
    int32_t iters;               /* CG iterations */
    int32_t converged;           /* 1 when every column reached rtol */
} mm_lml_info;

mm_status gp_lml(mm_plan plan, const double *y, double sigma2, const double *Z, int64_t ldz,
                 int32_t nprobes, int32_t maxit, double rtol, mm_lml_info *info, double *alpha,
                 void *stream);

/* Host only: e_1^T log(T) e_1 for the m x m Lanczos matrix built from CG
 * coefficients alpha[0..m-1], beta[0..m-2] (Algorithm 2): T[k][k] = 1/alpha_k +
 * beta_{k-1}/alpha_{k-1}, T[k][k+1] = sqrt(beta_k)/alpha_k.  MM_ERR_BREAKDOWN if
 * the spectrum is not positive. */
mm_status mm_lanczos_logquad(const double *alpha, const double *beta, int32_t m, double *out);

/*
 * Batched products over independent point sets: y_k = (K_k + diag_shift I) v_k
 * for every plan k of the batch (Section 2, eq. Ky, per problem), with one
 * gather launch, one launch per kernel configuration and sweep phase, and one
 * scatter launch for the whole batch.  Each problem's result is bitwise the
 * result of matern_mvm on its plan alone.  The batch owns its work buffers
 * and pins its plans (mm_plan_set_kernel / mm_plan_destroy fail while it
 * lives).  A problem whose per-pass partial sums (passes x n x columns
 * doubles) exceed 16 GiB cannot be batched (MM_ERR_ARG).
 *   plans     host array of count plan handles (count >= 1; any mix of n, d, nu, form)
 *   nrhs      right-hand sides of every problem, 1..256
 *   use_graph != 0: the launches are captured once into a HIP graph and
 *             replayed on a private stream ordered after the caller's stream
 */
typedef struct mm_mvm_batch_s *mm_mvm_batch;

mm_status mm_mvm_batch_create(const mm_plan *plans, int32_t count, int32_t nrhs, int32_t use_graph,
                              mm_mvm_batch *out);

/* Launch schedule: workgroups per compute unit of the persistent carry-scan
 * grids (the sweep launches run one workgroup per work item) and the grid of
 * the gather/scatter kernels (both >= 1; results do not depend on them). */
mm_status mm_mvm_batch_set_schedule(mm_mvm_batch batch, int32_t sweep_wg_per_cu, int32_t grid);

/* Run the batch.  v, y: host arrays of count device pointers (n_k x nrhs
 * column-major, caller order); ldv, ldy: host arrays of leading dimensions
 * (>= n_k).  The pointer tables are copied before the call returns (it waits
 * for the previous call's copy only). */
mm_status mm_mvm_batch_run(mm_mvm_batch batch, const double *const *v, const int64_t *ldv,
                           double *const *y, const int64_t *ldy, double diag_shift, void *stream);

/* Release a batch and its work buffers (synchronises the device); NULL is accepted. */
mm_status mm_mvm_batch_destroy(mm_mvm_batch batch);

/*
 * Kernel-time accounting for measurement: when enabled, every launch of the
 * divide-and-conquer sweep kernel of this plan (one launch covers a group of
 * passes) is bracketed by HIP events on its stream.  mm_plan_profile_read()
 * returns, since the last reset, the summed elapsed milliseconds, the number
 * of bracketed launches and the number of passes they covered (any output
 * pointer may be NULL; synchronises with the recorded events).
 */
mm_status mm_plan_profile_enable(mm_plan plan, int32_t enable);
mm_status mm_plan_profile_read(mm_plan plan, double *sweep_ms, int64_t *sweep_launches,
                               int64_t *sweep_passes, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* MATERNMVM_H */
