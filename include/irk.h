/*
 * irk.h -- C ABI of libirk, the gfx950 (MI355X) solver for the transformed
 * s-stage Radau IIA Newton system
 *
 *     B W = R,    B = A^{-1} (x) M  -  dt diag(J_1, ..., J_s)
 *
 * (Pazner & Persson, "Stage-parallel fully implicit Runge-Kutta solvers for
 * discontinuous Galerkin fluid simulations", Sec. 4.3, Eq. big-irk) with
 * restarted, right-preconditioned GMRES and a block ILU(0) preconditioner,
 * either stage-coupled (Sec. 4.3.1) or stage-uncoupled with shifts
 * (Sec. 4.3.2).
 *
 * Layout conventions shared by every entry point
 *   - T elements, m unknowns per element, s stages, n = T*m.
 *   - Vectors (rhs, solution) are stage-major [s][T][m], FP64, on the device.
 *   - J is a T x T block matrix of dense m x m blocks in BSR form (Sec. 2.1):
 *     row_ptr[T+1], col_idx[nnzb] with ascending columns per row and the
 *     diagonal block present; values J[nJ][nnzb][m][m], each block
 *     row-major.  nJ = 1 shares one Jacobian between all stages (I (x) J);
 *     nJ = s gives stage Jacobians J_k (Sec. 4.1).
 *   - M is block diagonal, M[T][m][m], each block row-major.
 *   - The pattern must be structurally symmetric and triangle-free (no two
 *     neighbours of an element are neighbours of each other, Sec. 4.2.1,
 *     Alg. 2); irk_setup rejects patterns that are not.
 *   - Element numbering is the elimination order of the ILU(0): the library
 *     factors in the caller's numbering, stage-major for the coupled form.
 *
 * Errors: every call returns an irk_status and never aborts.  Arguments are
 * checked on the host before anything is enqueued.  Conditions found on the
 * device (singular pivot block, non-finite values, breakdown) are returned
 * by the call that synchronizes (irk_factor_ilu, irk_gmres_solve).
 *
 * Threading: one host thread at a time per handle.  All device work goes to
 * the stream given to irk_setup.
 */
#ifndef IRK_H
#define IRK_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IRK_OK = 0,
    IRK_ERR_ARG = 1,         /* invalid argument or unsupported shape            */
    IRK_ERR_NOMEM = 2,       /* workspace smaller than irk_workspace_size        */
    IRK_ERR_SINGULAR = 3,    /* a pivot block of the ILU(0) is singular          */
    IRK_ERR_NOCONV = 4,      /* max_iters reached; x holds the last iterate      */
    IRK_ERR_BREAKDOWN = 5,   /* Arnoldi breakdown without convergence            */
    IRK_ERR_NONFINITE = 6,   /* NaN or Inf in the input or the iteration         */
    IRK_ERR_DEVICE = 7,      /* a HIP runtime call failed                        */
    IRK_ERR_STATE = 8,       /* call out of order (e.g. solve before factor)     */
    IRK_ERR_INTERNAL = 9     /* an internal consistency check failed (a bug)     */
} irk_status;

typedef enum {
    IRK_PC_COUPLED = 0,            /* stage-coupled block ILU(0), Sec. 4.3.1    */
    IRK_PC_UNCOUPLED_SHIFTED = 1,  /* per-stage ILU(0) of (A^-1_kk + alpha_k)M - dt J_k, Sec. 4.3.2 */
    IRK_PC_UNCOUPLED = 2,          /* the same with alpha = 0                   */
    IRK_PC_NONE = 3                /* no preconditioner                         */
} irk_pc;

typedef enum {
    IRK_FP64 = 0,
    IRK_FP32 = 1,
    IRK_BF16 = 2,            /* factor storage only                              */
    IRK_FP16_SCALED = 3      /* factor storage only: FP16 with a power-of-two scale per block */
} irk_prec;

typedef struct {
    int s;                   /* stages, 1..5                                      */
    const double *A;         /* HOST, s*s row-major Butcher matrix (invertible)   */
    int T, m, nnzb;          /* elements, block size (1..160), stored J blocks    */
    const int32_t *row_ptr;  /* HOST, T+1                                         */
    const int32_t *col_idx;  /* HOST, nnzb                                        */
    const double *J;         /* DEVICE, nJ*nnzb*m*m                               */
    int nJ;                  /* 1 or s                                            */
    const double *M;         /* DEVICE, T*m*m                                     */
    double dt;               /* time step, > 0                                    */
} irk_problem;

typedef struct {
    irk_pc pc;
    int shift_rule;          /* 0: alpha_k = sum_{j!=k} |A^-1_jk| (Sec. 4.3.2);
                                1: alpha = 0;  2: alpha taken from `alpha`       */
    const double *alpha;     /* HOST, s values, read when shift_rule == 2         */
    irk_prec matvec_prec;    /* IRK_FP64, or IRK_FP32 for the inner iteration    */
    irk_prec factor_prec;    /* factor storage read by the inner sweeps; with
                                FP64 the whole solve is FP64; any other value
                                selects the mixed-precision scheme (FP32 or BF16
                                or FP16-scaled factors, FP32 matvec and sweeps,
                                FP64 Arnoldi, FP64 refinement outer loop)         */
    int restart;             /* Krylov dimension per cycle, 1..64                 */
    int max_iters;           /* cap on Arnoldi steps (summed over all cycles)     */
    int max_outer;           /* cap on refinement steps (mixed precision)         */
    double rtol;             /* stop when ||R - B W||_2 / ||R||_2 <= rtol (FP64)  */
    double inner_rtol;       /* inner relative tolerance (mixed precision)        */
} irk_options;

typedef struct {
    int converged;           /* 1 if the FP64 true relative residual <= rtol      */
    int iters;               /* Arnoldi steps (matvecs with B), all cycles        */
    int outer_iters;         /* refinement steps (1 for the FP64 path)            */
    int restarts;            /* GMRES cycles started after the first              */
    int equiv_mults;         /* iters * s: n x n products, the paper's count      */
    double rel_res_true;     /* ||R - B W|| / ||R|| computed in FP64 at the end   */
    double rel_res_est;      /* last GMRES estimate |g_{j+1}| / ||r0||            */
    int bad_element;         /* element of a singular pivot, else -1              */
    float ms_factor;         /* device time of the last irk_factor_ilu            */
    float ms_solve;          /* device time of this solve                         */
} irk_solve_info;

typedef struct irk_handle irk_handle;

/* Fill *o with defaults: coupled, column-sum shifts, FP64, restart 30,
 * max_iters 3000, max_outer 20, rtol 1e-10, inner_rtol 1e-4. */
irk_status irk_default_options(irk_options *o);

/* Device bytes the caller must provide to irk_setup for this problem and
 * these options.  Pure host computation. */
irk_status irk_workspace_size(const irk_problem *p, const irk_options *o, size_t *bytes);

/* The level schedule that the factorization and both sweeps follow (Sec.
 * 4.2.1, Alg. 2: on a triangle-free mesh an element's pivot and sweep
 * values need only its lower neighbours in the forward direction and its
 * upper neighbours in the backward one).  Forward level of element i:
 * 1 + the largest forward level of its lower neighbours (0 without any);
 * backward level: the same over its upper neighbours.  lvl_fwd, lvl_bwd
 * (HOST, T): the elements by ascending level, ascending element number
 * within a level; off_fwd, off_bwd (HOST, T + 1): level l is
 * lvl[off[l] .. off[l+1]); *nlev_fwd, *nlev_bwd: the level counts.  The
 * pattern (row_ptr[T+1], col_idx[nnzb], HOST) is checked as irk_setup
 * checks it: IRK_ERR_ARG for a malformed row pointer, a column out of
 * range or out of order, a missing diagonal, an asymmetric pattern or a
 * triangle; IRK_ERR_INTERNAL if the schedule fails its own check (every
 * element listed once, after the neighbours it reads).  Host only; the
 * caller owns every array. */
irk_status irk_level_schedule(int T, int nnzb, const int32_t *row_ptr, const int32_t *col_idx,
                              int *lvl_fwd, int *off_fwd, int *nlev_fwd, int *lvl_bwd, int *off_bwd,
                              int *nlev_bwd);

/* Set up the solver of the transformed Newton system B W = R (Sec. 4.1,
 * Eq. modified-IRK, written as Eq. big-irk in Sec. 4.3; the tableau A of Sec. 3, the block Jacobians of Sec. 2.1 and
 * the block-diagonal mass matrix M).  Validates the problem, computes A^{-1}
 * and the shifts of Sec. 4.3.2, builds the level schedule of the block
 * ILU(0) sweeps on the host, and copies J and M into the caller-owned device
 * workspace (re-laid for the kernels).  The caller may free J and M
 * afterwards.  The handle keeps host memory only; it never allocates device
 * memory.  `workspace` must stay valid and untouched until irk_destroy.
 * Work goes to `stream`; returns after the copies are done.  Errors:
 * IRK_ERR_ARG (invalid shape, pattern not structurally symmetric or not
 * triangle-free, malformed row_ptr), IRK_ERR_NOMEM (ws_bytes below
 * irk_workspace_size), IRK_ERR_DEVICE. */
irk_status irk_setup(const irk_problem *p, const irk_options *o, void *workspace,
                     size_t ws_bytes, hipStream_t stream, irk_handle **out);

/* Replace J, M and dt (same pattern, same nJ): a new Newton iteration or
 * time step re-evaluates the Jacobians (Sec. 4.1) and must refactor
 * (Sec. 4.4: the preconditioner is computed once per linear solve).  J, M:
 * DEVICE, same layout as in irk_problem; read by kernels on the handle's
 * stream (the caller keeps them valid until that stream has passed this
 * call, e.g. until the next solve returns).  The factors are stale until the
 * next factorization.  IRK_ERR_ARG for null pointers or dt <= 0. */
irk_status irk_update_values(irk_handle *h, const double *J, const double *M, double dt);

/* Block ILU(0) factorization chosen by the options (Sec. 4.2.1 Alg. 2,
 * Sec. 4.3.1 Alg. 3 in its standard ILU(0) reading, Sec. 4.3.2).  Computed
 * in FP64 level by level (the uncoupled forms, and the stage-coupled form
 * with m <= 64: every wavefront in one launch, each task waiting only for the tasks whose
 * blocks it reads, with the same arithmetic; variable IRK_FACTOR_FLOW=0 at
 * set-up keeps one launch per wavefront); then quantized when factor_prec
 * is not FP64.  Synchronizes; IRK_ERR_SINGULAR names the element in
 * irk_last_bad_element. */
irk_status irk_factor_ilu(irk_handle *h);

/* The same factorization without waiting for it: returns once its launches
 * are enqueued, so the host prepares the next calls while it runs (the
 * uncoupled forms, and the stage-coupled form with m <= 64, in up to three
 * dependency-driven launches, cut at the points named below).  It
 * starts at the current point of the handle's stream and runs on a second
 * stream of the handle (on the handle's stream itself while profiling is
 * on); the handle's stream goes on when the factorization reaches its first
 * wavefront with fewer tasks than the device has compute units, so work the
 * caller enqueues next (a solve's initial residual, which needs no factors)
 * runs beside its latency-bound last wavefronts.  Every call of this
 * library that reads or writes the factors, or writes J, M or dt, makes the
 * handle's stream wait for the factorization first, except that
 * irk_gmres_solve starts its first forward sweep's first launch group
 * (the first level, or the first run of chained levels) once the
 * wavefront that makes those levels' factors final has ended.  A singular pivot is reported by the next call that uses the factors:
 * irk_gmres_solve (which reads the flag with the first state read that
 * follows the factorization), irk_apply_preconditioner(_inner),
 * irk_export_factors, irk_autotune and irk_batch_admit (which wait for it
 * first) return IRK_ERR_SINGULAR, irk_last_bad_element names the element,
 * and the handle is not factored. */
irk_status irk_factor_ilu_async(irk_handle *h);

/* Solve B x = rhs (Sec. 4.3, Eq. big-irk) by restarted GMRES, right-
 * preconditioned with the factored block ILU(0) (Sec. 4.2-4.3), to
 * ||rhs - B x||_2 <= rtol ||rhs||_2 with the FP64 operator (the true
 * residual, recomputed at the end of every restart cycle).  rhs, x: DEVICE
 * [s][T][m]; x is the initial guess on entry (zero-fill it for x0 = 0) and
 * the solution on return (updated in place during the solve).  info (HOST,
 * may be NULL) is filled.  The device decides when a cycle ends; the host
 * reads the convergence state at the end of each cycle and at a few steps
 * inside it, placed where the residual estimate is about to meet the
 * tolerance, and waits for the stream before returning.  Returns
 * IRK_ERR_STATE before irk_factor_ilu, IRK_ERR_NOCONV (x holds the last
 * iterate), IRK_ERR_BREAKDOWN or IRK_ERR_NONFINITE with info filled. */
irk_status irk_gmres_solve(irk_handle *h, const double *rhs, double *x, irk_solve_info *info);

/* ---- batches: many independent systems in the same kernel launches ----
 * A batch runs the GMRES iteration of all its members together: every
 * launch of a step (sweep levels, operator, orthogonalization) covers all
 * members that are still iterating, so small systems fill the GPU together.
 * Members must share the preconditioner kind, the precision scheme and the
 * Jacobian sharing mode; they may differ in T, m, s, dt and restart.  Each
 * member keeps using its own handle's workspace.  A batch never allocates
 * device memory. */
typedef struct irk_batch irk_batch;

/* Device bytes of a batch of at most `capacity` members whose element
 * counts add up to at most `max_elements`. */
irk_status irk_batch_workspace_size(int capacity, long long max_elements, size_t *bytes);

/* Create a batch working on `stream` in a caller-owned device workspace. */
irk_status irk_batch_create(int capacity, long long max_elements, void *workspace,
                            size_t ws_bytes, hipStream_t stream, irk_batch **out);

/* Queue a factored handle with its right-hand side and its initial guess /
 * solution vector (DEVICE [s][T][m] each; both must stay valid until the
 * member is retired).  It starts at the next irk_batch_advance.  The batch's
 * stream first waits for the end of the handle's last set-up, value update
 * or factorization (not for other work enqueued on the handle's stream
 * since), so new systems can be set up and factored on another stream while
 * the batch iterates; rhs and x must be ready in the batch stream's order.
 * IRK_ERR_NOMEM: no free slot or element budget. */
irk_status irk_batch_admit(irk_batch *b, irk_handle *h, const double *rhs, double *x,
                           long long tag);

/* Run up to `cycles` GMRES cycles (restart periods) for every member;
 * newly admitted members first get their initial residual.  Members that
 * converge or fail leave the batch and wait to be retired.  Synchronizes at
 * every step boundary where it checks convergence. */
irk_status irk_batch_advance(irk_batch *b, int cycles);

/* Pop up to `cap` retired members: their tags, statuses and infos (HOST
 * arrays, any may be NULL).  *count receives the number popped. */
irk_status irk_batch_retire(irk_batch *b, long long *tags, irk_status *status,
                            irk_solve_info *info, int cap, int *count);

/* Members queued or still iterating. */
int irk_batch_pending(const irk_batch *b);

irk_status irk_batch_destroy(irk_batch *b);

/* Solve `count` independent systems B_q x_q = rhs_q (Sec. 4.3, Eq.
 * big-irk, each with its own factored block ILU(0), Sec. 4.2-4.3) in the
 * batch: admit the handles (tags 0..count-1), advance until all have left,
 * retire them.  rhs[q], x[q]: DEVICE [s_q][T_q][m_q] (x[q] is the initial
 * guess on entry and the solution on return; both ready in the order of the
 * batch's stream).  info (HOST, may be NULL) receives one entry per handle.
 * The batch must be empty (IRK_ERR_STATE otherwise).  Returns the first
 * non-OK member status. */
irk_status irk_solve_batched(irk_batch *b, irk_handle *const *h, const double *const *rhs,
                             double *const *x, int count, irk_solve_info *info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc):
 * irk_solve_batched without a batch object.  The batch's device scratch
 * (system table, gathered convergence states, merged work items) is a
 * library-owned static device array of about 19 MB per GPU, taken at the
 * first call on a device (the current device) and held until the process
 * ends; the call allocates no device memory.  Limits: count <= 64 and at
 * most 32768 elements over all handles, else IRK_ERR_ARG before any work.
 * Handles, rhs, x, info and the result as for irk_solve_batched; all work
 * goes to `stream`, and the call returns after it has finished.  Every call
 * on one GPU shares the array: calls from several host threads are
 * serialized by the library; the array's contents are rewritten by each
 * call before they are read. */
irk_status irk_solve_batched_noalloc(irk_handle *const *h, const double *const *rhs,
                                     double *const *x, int count, hipStream_t stream,
                                     irk_solve_info *info);

/* Block ILU(0) factorization of `count` handles together (the same
 * factorization as irk_factor_ilu, Sec. 4.2-4.3): level l of every handle
 * runs in the same launches (one per level and kernel class), so many small
 * systems pay one chain of level launches instead of one chain each.  The
 * batch b (no members allowed) lends its device table and item buffer; the
 * handles may differ in every shape and option.  Runs on the batch's stream
 * after the work already enqueued on each handle's stream and returns when
 * the factors are complete.  status (HOST, may be NULL): one entry per
 * handle, IRK_OK or IRK_ERR_SINGULAR (irk_last_bad_element names the
 * element).  Returns IRK_ERR_SINGULAR if any handle has a singular pivot,
 * IRK_ERR_STATE if the batch has members, IRK_ERR_ARG for a null or
 * repeated handle.  Handles are processed in groups that fit the batch's
 * capacity and item buffer. */
irk_status irk_factor_batched(irk_batch *b, irk_handle *const *h, int count, irk_status *status);

/* y = B x with the FP64 operator (Eq. big-irk); DEVICE vectors. */
irk_status irk_apply_operator(irk_handle *h, const double *x, double *y);

/* z = P^{-1} v with the FP64 factors (Sec. 4.2.1, forward and backward
 * block-triangular sweeps); DEVICE vectors; requires irk_factor_ilu. */
irk_status irk_apply_preconditioner(irk_handle *h, const double *v, double *z);

/* y = (I (x) M - dt [a_kl J_k]_{kl}) x: the untransformed Newton operator of
 * Sec. 4.1 (Eq. newton-system-2) for the same problem, the operator that the
 * transformation W = (A (x) I) K replaces by B (kept as the baseline that
 * Table 2 compares against).  form 0: block by block, one pass over J_k for
 * each of the s^2 blocks (k, l) of the s x s block matrix (the
 * s^2 (r+1) m^2 T multiply-adds Table 2 counts); form 1: fused, each
 * element's Jacobian row streamed once and applied to the combinations
 * sum_l a_kl x_l.  FP64; x, y DEVICE [s][T][m]; IRK_ERR_ARG for another
 * form.  Timed as `untr` while profiling is on. */
irk_status irk_apply_operator_untransformed(irk_handle *h, int form, const double *x, double *y);

/* The inner-iteration kernels of a mixed-precision handle, the ones its
 * GMRES cycles run: y = B x (Eq. big-irk) with the FP32 copies of J and M
 * and FP32 arithmetic, x rounded to FP32 first; z = P^{-1} v (Sec. 4.2.1)
 * with the stored FP32 / BF16 / FP16-scaled factors and FP32 sweeps.
 * Vectors are FP64 on the DEVICE.  For an FP64 handle these are
 * irk_apply_operator and irk_apply_preconditioner.  The preconditioner
 * needs irk_factor_ilu (IRK_ERR_STATE otherwise); both overwrite the
 * handle's work vectors and its per-solve state (not x, rhs or factors). */
irk_status irk_apply_operator_inner(irk_handle *h, const double *x, double *y);
irk_status irk_apply_preconditioner_inner(irk_handle *h, const double *v, double *z);

/* Copy the FP64 inverse pivot blocks P_{k,i}^{-1} to pinv (DEVICE,
 * [s][T][m][m] row-major) and, for the coupled form, the cross-stage blocks
 * C_{kl,i} (k != l) to cross (DEVICE, [s][s][T][m][m] row-major, diagonal
 * slots left untouched; may be NULL). */
irk_status irk_export_factors(irk_handle *h, double *pinv, double *cross);

/* Kernel timing for benchmarks.  While enabled, the library records HIP
 * events on the handle's stream around every operator launch (FP64 and
 * FP32), every preconditioner application (all sweep levels of one apply),
 * every Arnoldi orthogonalization (CGS2 + Givens) and every factorization.
 * irk_profile_read waits for the stream, adds up the recorded intervals and
 * clears them.  Up to 4096 intervals are kept between reads; later ones are
 * counted in `dropped`. */
typedef struct {
    int matvec_count;  double matvec_ms;   /* FP64 operator launches            */
    int matvec32_count; double matvec32_ms;/* FP32 operator launches            */
    int pc_count;      double pc_ms;       /* preconditioner applications       */
    int orth_count;    double orth_ms;     /* CGS2 + Givens steps               */
    int factor_count;  double factor_ms;   /* factorizations (incl. quantize)   */
    int dropped;
    int untr_count;    double untr_ms;     /* untransformed operator products   */
} irk_profile_stats;

irk_status irk_profile_enable(irk_handle *h, int on);
irk_status irk_profile_read(irk_handle *h, irk_profile_stats *out);

/* Launch shapes chosen by irk_autotune. */
typedef struct {
    int matvec_teams;    /* block rows per 256-thread workgroup of the inner-precision matvec */
    int sweep_big_min;   /* levels of at least this many elements use the large-level sweep form
                            (the smaller ones the prefetching form) */
    int sweep_teams;     /* elements per 512-thread workgroup in the streaming form */
    int from_cache;      /* 1: shapes taken from the process-wide table, nothing timed */
    float matvec_us;     /* timed cost of one matvec / one preconditioner application with */
    float sweep_us;      /* the chosen shapes (0 when from_cache)                          */
    int sweep_big_form;  /* large-level form: 0 streaming, 2 prefetching without the first
                            Jacobian columns (one element per workgroup) */
    int sweep_flow;      /* 0: one launch per level; 1 + form: every level of a sweep in one
                            launch, each element waiting only for the neighbours it reads
                            (form 0 streaming, 1 prefetching, 2 prefetching without the
                            Jacobian columns) */
    int sweep_chain_max; /* (sweep_flow 0) levels of fewer elements run chained: each run of
                            consecutive such levels of one form in one launch; 0 none */
    int sweep_split;     /* (sweep_flow 0, streaming large levels) levels of fewer elements
                            take sweep_teams / 2 elements per workgroup; 0 none */
} irk_tune_info;

/* Choose the launch shapes of a handle's matvec and preconditioner sweeps
 * by timing the candidates on the handle's own data (the multi-stage BSR
 * product and the level-scheduled sweeps of Sec. 4.3; the shapes change
 * only how the work is spread over workgroups).  Candidates: 1, 2, 4 or 8
 * block rows per matvec workgroup; for the sweeps, the level size from which
 * the large-level form replaces the prefetching one (1, 64, 128, 256, 512,
 * never) and that form: streaming with half, the default or twice the
 * default elements per workgroup, or prefetching without the Jacobian
 * columns; then, on top of the best of these, the level size below which
 * consecutive levels run chained in one launch (32 to 1024, or every level),
 * each element waiting only for the neighbours it reads (variable
 * IRK_SWEEP_CHAIN fixes it), then the level size (256 to 1024) below which
 * streaming levels take half the elements per workgroup (variable
 * IRK_SWEEP_SPLIT fixes it); or every level of a direction in one launch in
 * one form (variable IRK_SWEEP_FLOW: 0 never, 1 always, 10 + form that form;
 * any value fixes this choice).  Each candidate is run once and timed over three runs on the
 * handle's stream; the fastest is kept.  The result is stored in a
 * process-wide table keyed by (m, s, preconditioner, precision, shared J,
 * row length, log2 T), and later calls for the same key (from any handle)
 * apply it without timing unless retime != 0.  The sweep results do not
 * depend on the form or the chaining (each accumulates in the same order);
 * the elements per workgroup of a level (the column groups of a team) and
 * the matvec's shape change the order in which partial sums combine, so
 * results may differ in the last bits.
 * h must be factored (IRK_ERR_STATE otherwise; any handle with pc NONE).
 * The handle's work vectors (not x, rhs or factors) are overwritten.
 * info may be NULL.  Synchronizes the handle's stream. */
irk_status irk_autotune(irk_handle *h, int retime, irk_tune_info *info);

/* Quantize nblk blocks of m*m FP64 values with the library's factor
 * quantizer (the kernel irk_factor_ilu uses for reduced-precision factors):
 *   IRK_FP32: float, round to nearest even;
 *   IRK_BF16: bfloat16 of the FP32 value, round to nearest even;
 *   IRK_FP16_SCALED: per block, e = 14 - E where max|x| lies in
 *     [2^(E-1), 2^E) (e clamped to [-100, 100], 0 for a zero block), stored
 *     value fp16(fp32(x * 2^e)), round to nearest even.
 * src: DEVICE nblk*m*m doubles; dst: DEVICE nblk*m*m elements of 4 (FP32)
 * or 2 bytes, same element order; exps: DEVICE nblk ints (FP16_SCALED,
 * else may be NULL).  Enqueued on `stream` and waited for. */
irk_status irk_quantize_blocks(const double *src, long long nblk, int m, irk_prec prec,
                               void *dst, int *exps, hipStream_t stream);

/* ---- one implicit Runge-Kutta time step by Newton's method ----
 * The ODE is M u' = f(t, u) (Sec. 3) with the right-hand side
 *     f(t, u) = J u + cos(omega t) g - eps u^3     (u^3 component-wise),
 * J and M being the problem given to irk_setup / irk_update_values (with
 * nJ = s the stage Jacobians given there must all equal J) and dt its time
 * step.  The step solves the stage equations in the variables
 * W = (A (x) I) K, Eq. modified-IRK of Sec. 4.1,
 *     (A^{-1} (x) M) W = F(t0 + dt c, U0 + dt W),   c_k = sum_l a_kl,
 * by Newton's method: every iteration solves the Eq. big-irk system with
 * the stage Jacobians J_k = J - 3 eps diag(U_k^2), U_k = u0 + dt w_k
 * (re-evaluated and refactored per iteration, Sec. 4.4; with eps = 0 the
 * matrix is the handle's own and an existing factorization is reused), by
 * the handle's preconditioned GMRES to its rtol.  It stops when the update
 * has ||delta W||_inf <= newton_tol (the Newton test of Sec. 5.1.1) and
 * returns u1 = u0 + dt (b^T A^{-1} (x) I) W, which is u0 + dt w_s for the
 * stiffly accurate Radau IIA methods. */
typedef struct {
    const double *g;       /* DEVICE [T][m] forcing direction, or NULL (none)   */
    double omega;          /* forcing frequency                                 */
    double eps;            /* cubic term; 0 makes f linear                      */
} irk_rhs;

typedef struct {
    int converged;         /* ||delta W||_inf <= newton_tol reached             */
    int newton_iters;      /* Newton iterations (linear solves)                 */
    int gmres_iters;       /* Arnoldi steps summed over them                    */
    int equiv_mults;       /* n x n operator products of those steps: the
                              paper's equivalent multiplications (Sec. 5.1.1),
                              gmres_iters * s for a Radau step, gmres_iters
                              for a DIRK step                                   */
    int factorizations;    /* block ILU(0) factorizations done by the step      */
    double update_norm;    /* ||delta W||_inf of the last iteration             */
    float ms;              /* device time of the step                           */
} irk_step_info;

/* Device bytes of the `work` buffer irk_radau_step needs for this handle. */
irk_status irk_step_workspace_size(const irk_handle *h, size_t *bytes);

/* One step from (t0, u0) to u1 (DEVICE [T][m] each; u1 may not alias u0).
 * b: HOST s weights, or NULL for a stiffly accurate tableau (b^T A^{-1} =
 * e_s).  work: DEVICE, irk_step_workspace_size bytes, caller-owned, scratch.
 * The handle's work vectors are overwritten; with eps != 0 its Jacobians are
 * restored on return and its factors are left stale (the next solve must
 * factor).  FP64 handles only (IRK_ERR_ARG for mixed precision, and for
 * eps != 0 unless nJ = s).  Returns IRK_ERR_NOCONV when max_newton
 * iterations do not meet newton_tol (u1 is then not written), or the first
 * error of a factorization or linear solve.  Synchronizes. */
irk_status irk_radau_step(irk_handle *h, const irk_rhs *f, const double *b, double t0,
                          const double *u0, double *u1, double newton_tol, int max_newton,
                          void *work, size_t work_bytes, irk_step_info *info);

/* Tableaux of the diagonally implicit comparison methods (App. A):
 * IRK_DIRK33 (3 stages, order 3) and IRK_ESDIRK65 (6 stages, order 5, first
 * stage explicit).  A: HOST, room for 8 x 8 doubles, filled row-major
 * stages x stages; b, c: HOST, room for 8 (b = last row of A, c = row
 * sums).  IRK_ERR_ARG for another `which`. */
enum { IRK_DIRK33 = 0, IRK_ESDIRK65 = 1 };
irk_status irk_dirk_tableau(int which, int *stages, double *A, double *b, double *c);

/* The diagonally implicit comparison methods (Sec. 3; DIRK33, ESDIRK65 of
 * App. A): `stages` (1..8) stages of a lower-triangular tableau A (HOST,
 * row-major stages x stages) whose implicit diagonal entries all equal the
 * handle's own one-stage tableau entry a (irk_setup with s = 1, A = [[a]],
 * so the handle's matrix is (1/a) M - dt J, Eq. big-irk at s = 1); only a
 * first stage with a zero row may be explicit, and the method must be
 * stiffly accurate (b = last row of A, c = row sums).  Stage i solves
 *     M (U_i - u0) = dt sum_{j<i} a_ij F_j + dt a_ii f(t_i, U_i),
 * F_j = f(t_j, U_j), by Newton in W = (U_i - u0)/dt with the handle's block
 * ILU(0) and GMRES, one n x n system per stage in sequence; u1 = U_s.  f,
 * newton_tol, max_newton, info and errors as for irk_radau_step
 * (IRK_ERR_ARG for another tableau shape or a handle with s != 1).  work:
 * DEVICE scratch of irk_dirk_workspace_size(h, stages) bytes. */
irk_status irk_dirk_workspace_size(const irk_handle *h, int stages, size_t *bytes);
irk_status irk_dirk_step(irk_handle *h, const irk_rhs *f, int stages, const double *A, double t0,
                         const double *u0, double *u1, double newton_tol, int max_newton,
                         void *work, size_t work_bytes, irk_step_info *info);

/* Element of the last singular pivot, or -1. */
int irk_last_bad_element(const irk_handle *h);

/* Release host state.  The workspace stays the caller's. */
irk_status irk_destroy(irk_handle *h);

const char *irk_status_str(irk_status st);

/* s-stage Radau IIA tableau (A s*s row-major, b, c; HOST), 1 <= s <= 12:
 * collocation at the zeros of P_s(2x-1) - P_{s-1}(2x-1) (App. A). */
irk_status irk_radau_iia(int s, double *A, double *b, double *c);

#ifdef __cplusplus
}
#endif
#endif /* IRK_H */
