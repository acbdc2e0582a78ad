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
    IRK_ERR_STATE = 8        /* call out of order (e.g. solve before factor)     */
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

/* Validate the problem, build the ILU level schedule on the host, and copy
 * J and M into the caller-owned device workspace (re-laid for the kernels).
 * The caller may free J and M afterwards.  The handle keeps host memory
 * only; it never allocates device memory.  `workspace` must stay valid and
 * untouched until irk_destroy.  Work goes to `stream`; returns after the
 * copies are done. */
irk_status irk_setup(const irk_problem *p, const irk_options *o, void *workspace,
                     size_t ws_bytes, hipStream_t stream, irk_handle **out);

/* Replace J, M and dt (same pattern, same nJ); the factors become stale
 * until the next irk_factor_ilu. */
irk_status irk_update_values(irk_handle *h, const double *J, const double *M, double dt);

/* Block ILU(0) factorization chosen by the options (Sec. 4.2.1 Alg. 2,
 * Sec. 4.3.1 Alg. 3 in its standard ILU(0) reading, Sec. 4.3.2).  Computed
 * in FP64 level by level; then quantized when factor_prec is not FP64.
 * Synchronizes; IRK_ERR_SINGULAR names the element in irk_last_bad_element. */
irk_status irk_factor_ilu(irk_handle *h);

/* Solve B x = rhs to the options' tolerance.  rhs, x: DEVICE [s][T][m];
 * x is the initial guess on entry (zero-fill it for x0 = 0) and the
 * solution on return (updated in place during the solve).  info (HOST, may
 * be NULL) is filled.  Synchronizes once per GMRES step to test
 * convergence and once per restart cycle. */
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
 * stream first waits for the work already enqueued on the handle's stream,
 * so a new system can be set up and factored on another stream while the
 * batch iterates.  IRK_ERR_NOMEM: no free slot or element budget. */
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

/* Admit `count` handles (tags 0..count-1), advance until all have left,
 * retire them; info (HOST, may be NULL) receives one entry per handle.
 * The batch must be empty.  Returns the first non-OK member status. */
irk_status irk_solve_batched(irk_batch *b, irk_handle *const *h, const double *const *rhs,
                             double *const *x, int count, irk_solve_info *info);

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
} irk_profile_stats;

irk_status irk_profile_enable(irk_handle *h, int on);
irk_status irk_profile_read(irk_handle *h, irk_profile_stats *out);

/* Launch shapes chosen by irk_autotune. */
typedef struct {
    int matvec_teams;    /* block rows per 256-thread workgroup of the inner-precision matvec */
    int sweep_big_min;   /* levels of at least this many elements use the streaming sweep form
                            (the smaller ones the prefetching form) */
    int sweep_teams;     /* elements per 512-thread workgroup in the streaming form */
    int from_cache;      /* 1: shapes taken from the process-wide table, nothing timed */
    float matvec_us;     /* timed cost of one matvec / one preconditioner application with */
    float sweep_us;      /* the chosen shapes (0 when from_cache)                          */
} irk_tune_info;

/* Choose the launch shapes of a handle's matvec and preconditioner sweeps
 * by timing the candidates on the handle's own data (the multi-stage BSR
 * product and the level-scheduled sweeps of Sec. 4.3; the shapes change
 * only how the work is spread over workgroups).  Candidates: 1, 2, 4 or 8
 * block rows per matvec workgroup; for the sweeps, the level size from which
 * the streaming form replaces the prefetching one (1, 64, 128, 256, 512,
 * never) and half, the default or twice the default elements per streaming
 * workgroup.  Each candidate is run once and timed over three runs on the
 * handle's stream; the fastest is kept.  The result is stored in a
 * process-wide table keyed by (m, s, preconditioner, precision, shared J,
 * row length, log2 T), and later calls for the same key (from any handle)
 * apply it without timing unless retime != 0.  The sweep results are
 * unchanged by the choice (both forms accumulate in the same order); the
 * matvec's partial sums are combined in a different order, so results may
 * differ in the last bits.
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
