// irk_internal.h -- shared declarations of the gfx950 library (host + device).
//
// Device data of one system lives in a SysDesc in device memory.  Kernels that
// work element by element (matvec rows, ILU levels, factor tasks) take the
// SysDesc table plus a list of work items, so one launch can cover any number
// of systems; vectors are addressed by slot (see Slot) so the launch arguments
// stay small and graph-capturable.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace irk {

constexpr int SMAX = 5;          // most stages handled
constexpr int MMAX = 160;        // largest block size
constexpr int RESTART_MAX = 64;  // largest Krylov dimension
constexpr int NTHREADS = 256;    // threads per workgroup of the element kernels
constexpr int SW_THREADS = 512;  // threads per workgroup of the sweep kernels
constexpr int RED_BLOCKS = 1024; // rows of reduction partials (two banks)
constexpr int RED_BANK = RED_BLOCKS / 2;   // workgroups of a vector reduction kernel (max)

enum Slot : int {
    SL_V = 0,   // Krylov basis, index j selects v_j            (FP64)
    SL_W,       // Arnoldi work vector                          (FP64)
    SL_Z,       // preconditioned vector z = P^{-1} v          (compute type)
    SL_YH,      // sweep scratch: y^ (forward), z (backward)    (compute type)
    SL_R,       // residual                                     (FP64)
    SL_X,       // solution / iterate                           (FP64)
    SL_B,       // right-hand side                              (FP64)
    SL_D,       // inner correction of the refinement loop      (FP64)
    SL_U,       // combination Z y at cycle end                 (FP64)
    SL_EXT0,    // caller vectors for the kernel-level entry points
    SL_EXT1,
    SL_ZB,      // preconditioned basis z_j = P^{-1} v_j, index j    (FP64)
    NSLOT
};

enum FactorType : int { FT_F64 = 0, FT_F32 = 1, FT_BF16 = 2, FT_F16S = 3 };

struct DevState {
    double bnorm;      // ||b|| of the current GMRES solve
    double beta;       // ||r0|| of the current cycle
    double est;        // last |g_{j+1}|
    double rnorm2;     // scratch for a norm reduction
    int j;             // index of the last Arnoldi step done in the cycle (-1 none)
    int done;          // cycle finished: converged estimate or breakdown
    int breakdown;
    int singular;      // 1 + element of the first singular pivot, 0 if none
    int nonfinite;
    int iters;          // Arnoldi steps of the current solve
    double tol_abs;     // cycle ends when |g_{j+1}| <= tol_abs
    // the finished cycle's breakdown flag and last estimate, kept by the
    // start of the next cycle (so the host reads both in one copy)
    int prev_breakdown;
    double prev_est;
};

struct SysDesc {
    // shape
    int s, T, m, nJ, nnzb;
    int ld;        // leading dimension of FP64 blocks
    int ld32;      // FP32 blocks
    int ld16;      // 16-bit blocks
    int maxrow;    // most blocks in one block row
    int pc;        // irk_pc
    int ftype;     // FactorType of the sweep factors
    int restart;
    int max_iters;
    int mixed;     // 1: FP32 inner iteration inside FP64 refinement
    long long N;   // s*T*m
    double dt;
    double rtol, inner_rtol;
    double Ainv[SMAX * SMAX];
    double A[SMAX * SMAX];  // the tableau itself (untransformed operator)
    double dcoef[SMAX];     // diagonal mass coefficient of each stage's pivot
    // structure (device)
    const int *row_ptr, *col_idx, *diag_pos, *tpos;
    const int *lvl_fwd, *lvl_bwd;   // elements sorted by forward / backward level
    // operator values
    const double *Jc;  const double *Mc;      // col-major blocks, ld
    const float *Jc32; const float *Mc32;     // col-major blocks, ld32
    // factors: pivots [T][s] blocks (inverted); cross blocks C_{lq} with
    // l, q >= 1, l != q: [T][s-1][s-2] blocks, group q - 1 holding C_{lq} in
    // ascending l (the ones in stage row or column 0 are A^{-1}_lq M)
    double *P64; double *C64;                 // ld
    float *P32;  float *C32;                  // ld32
    uint16_t *P16; uint16_t *C16;             // ld16
    int *P16e; int *C16e;                     // per-block exponents (FP16S)
    double *Fscr;                             // per-element factor scratch [T][s] blocks (ld)
    unsigned long long *flow;                 // [T] epoch of the last single-launch sweep that
                                              // published the element's result
    // vectors
    void *vec[NSLOT];
    // Krylov state
    double *H;       // [(restart+1) * restart], row-major, H[r*restart + c]
    double *g;       // [restart+1]
    double *cs, *sn; // [restart]
    double *y;       // [restart]
    double *hbuf;    // [2 * (restart+1)] h1 and h2 of CGS2
    double *part;    // [RED_BLOCKS * (restart+2)] reduction partials
    DevState *st;
};

// one workgroup's work: system, first task, task count, aux
struct Item { int sys, first, count, aux; };

// One element of a sweep level: system, element, position of the first
// off-diagonal block of its row in the sweep's direction (lower blocks in the
// forward sweep, upper ones in the backward sweep), their count, and the
// columns of the first SW_NB of them (more are read from col_idx).  Stored
// in the item array, three Items per record.
constexpr int SW_NB = 8;
struct SwItem { int sys, i, pa, nb; int col[SW_NB]; };
static_assert(sizeof(SwItem) == 3 * sizeof(Item), "SwItem spans three Items");

// LDS elements (of the compute type) one team needs; host and device must agree.
__host__ __device__ inline int round_up(int a, int b) { return (a + b - 1) / b * b; }
__host__ __device__ inline int imax(int a, int b) { return a > b ? a : b; }
// matvec: gather of (maxrow+1)*m columns for S stages, or the [G][S][ld] partials
__host__ __device__ inline int matvec_region(int S, int m, int maxrow, int ld, int V, int team) {
    const int G = team / (ld / V);
    return imax(S * (maxrow + 1) * m, G * S * ld);
}
// sweep: gather of the neighbours' stage vectors [S][maxrow*m], reused for
// the [G][S][ld] partial sums of the Jacobian and factor products, then the
// y and u vectors [S][round_up(m, 8)] of one element and one more vector
// (the stage-0 combination of the coupled backward sweep)
__host__ __device__ inline int sweep_region(int S, int m, int maxrow, int team, int ldJ, int VJ,
                                            int ldF, int VF) {
    const int GJ = team / (ldJ / VJ), GF = team / (ldF / VF);
    const int r = imax(S * maxrow * m, imax(GJ * S * ldJ, GF * S * ldF));
    return r + (2 * S + 1) * round_up(m, 8);
}

// ---------------------------------------------------------------------------
// launchers (defined in the .hip files; all enqueue on `stream`)
// ---------------------------------------------------------------------------

// src: row-major FP64 blocks; dst: col-major with leading dimension ld, in
// the requested type (0 double, 1 float).  nblk blocks of m x m.
void launch_relayout(const double *src, void *dst, int dst_type, long long nblk, int m,
                     int ld, hipStream_t st);

// y_slot = B x_slot   (mode 0)   or   y_slot = b_slot - B x_slot   (mode 1)
// prec 0: FP64 (Jc, Mc); 1: FP32 copies (x read as compute type of slot).
// skip_done: systems whose GMRES cycle has ended (st->done) do nothing.
void launch_matvec(const SysDesc *dsys, const Item *items, int nitems, int s_max,
                   int prec, bool sharedJ, int x_slot, int y_slot, int b_slot, int mode,
                   int skip_done, size_t shmem, hipStream_t st);

// Untransformed operator y = (I (x) M - dt [a_kl J_k]) x (FP64): fused (one
// launch, each Jacobian row streamed once for all stages) or block by block
// (s^2 launches, block (k, l) streams J_k).  Items and LDS as the FP64 matvec.
void launch_untransformed(const SysDesc *dsys, const Item *items, int nitems, int s, bool fused,
                          int x_slot, int y_slot, size_t shmem, hipStream_t st);

// ---- one Newton time step (k_step.hip); raw device pointers ----
void launch_save_diag(const SysDesc *dsys, const SysDesc &hsys, double *Dbase, hipStream_t st);
void launch_stage_jac(const SysDesc *dsys, const SysDesc &hsys, const double *Dbase, const double *u0,
                      const double *W, double dt, double eps, hipStream_t st);
void launch_jac_u0(const SysDesc *dsys, const SysDesc &hsys, const double *Dbase, const double *u0,
                   double *y, hipStream_t st);
void launch_stage_rhs(int s, long long n, const double *Ju0, const double *g, const double *u0,
                      const double *W, double dt, double eps, const double *gam, const double *hist,
                      double *out, hipStream_t st);
constexpr int DIRK_STAGES_MAX = 8;
void launch_combine(int cnt, long long n, const double *coef, const double *F, double *out,
                    hipStream_t st);
void launch_stage_state(long long n, const double *u0, const double *W, double dt, double *U,
                        hipStream_t st);
void launch_rhs_eval(long long n, const double *JU, const double *U, const double *g, double gam,
                     double eps, double *F, hipStream_t st);
void launch_newton_update(long long N, double *W, const double *delta, double *part, double *out,
                          hipStream_t st);
void launch_step_finish(int s, long long n, const double *u0, const double *W, double dt,
                        const double *dcoef, double *u1, hipStream_t st);

// One level of the forward sweep (L~ y = v, then y^ = P^{-1} y per element),
// or of the backward sweep (z = y^ + P^{-1} (dt J_upper z - C z)).
//   recs: nrec SwItem records of the level; tps elements per workgroup
//   (SW_THREADS / tps threads each), region LDS elements per team.
//   fp64: FP64 factors/values with double vectors; otherwise FP32 values
//   and factors of type ftype with float vectors.
//   v_slot/v_index: input of the forward sweep (FP64); result in SL_YH;
//   acc_slot >= 0 adds the backward result to that FP64 slot (x += z).
//   form: 0 streaming; 1 prefetching (factor blocks, mass block, first
//   Jacobian columns); 2 prefetching without the Jacobian columns (k_sweep.hip);
//   a prefetching form whose blocks exceed the register budget runs streaming.
//   epoch != 0: publish each element's flag (a later launch of the same
//   sweep chains levels, see launch_sweep_flow).
void launch_sweep(bool forward, const SysDesc *dsys, const SwItem *recs, int nrec, int tps,
                  int region, int s_max, bool fp64, int ftype, bool coupled, bool sharedJ,
                  int v_slot, int v_index, int acc_slot, int skip_done, size_t shmem,
                  hipStream_t st, int form, unsigned long long epoch = 0);

// Consecutive levels of one sweep in a single launch (k_sweep_flow.hip):
// workgroups take the entries of the table items[tab .. tab + nblk) (first
// record's item offset, records per workgroup; levels in sweep order) in
// claim order (ticket counter, back at zero when the launch ends); each
// element waits for the flags of the neighbours it reads, then publishes
// its own flag = epoch.  A workgroup's records belong to one system and one
// level (i = -1 pads).  region: LDS elements per workgroup; a workgroup of
// tps records gives each team region / tps (at least what any entry
// needs).  epoch: the same for every launch of one sweep, larger than
// any epoch an earlier sweep used on these flags.
void launch_sweep_flow(bool forward, const SysDesc *dsys, const Item *items, int tab, int nblk,
                       int region, int s_max, bool fp64, int ftype, bool coupled, bool sharedJ,
                       int v_slot, int v_index, int acc_slot, int skip_done, size_t shmem,
                       hipStream_t st, int form, unsigned *ticket, unsigned long long epoch);

// One wavefront of the factorization: tasks (stage k = aux, element =
// first) build P_{k,i} from the neighbour terms, invert it, and (coupled)
// run the stage round on the element's later stages (k_factor.hip).  The
// kernels are chosen by the block order m (all systems of one launch share
// its class, factor_class(m)): four-wave workgroups for m <= 64, eight-wave
// ones above.
void launch_factor(const SysDesc *dsys, const Item *items, int nitems, bool coupled, bool sharedJ, int m,
                   size_t shmem, hipStream_t st);
int factor_class(int m);

// Quantize nblk column-major blocks (leading dimensions ld in, ldq out).
void quantize_blocks(const double *src, void *dst, int *ex, long long nblk, int m, int ld,
                     int ldq, int ftype, hipStream_t st);
// Quantize the FP64 factors to ftype (FP32 / BF16 / FP16 scaled).
void launch_quantize(const SysDesc *dsys, const SysDesc &hsys, int ftype, hipStream_t st);
// The same for several systems of one factor type in one launch: item =
// (system, first block, block count, 0 pivots / 1 cross blocks).
void launch_quantize_sys(const SysDesc *dsys, const Item *items, int nitems, int ftype, hipStream_t st);

// ---- Krylov (FP64; vec items: (sys, chunk, chunks); fin items: one per system) ----
// one Arnoldi step j: CGS2 passes, Givens update, v_{j+1} = w / ||w||
void launch_arnoldi(const SysDesc *dsys, const Item *vec, int nvec, const Item *fin, int nfin, int j,
                    hipStream_t st);
// y = H^{-1} g over the cycle's steps, u = B y with B the basis in
// basis_slot (SL_ZB: the preconditioned vectors, so x + u is the right-
// preconditioned update; SL_V without a preconditioner)
void launch_cycle_end(const SysDesc *dsys, const Item *vec, int nvec, int restart, int basis_slot,
                      hipStream_t st);
// ||slot||: which 0 -> st->bnorm; which 1 -> start of a cycle (beta, g, tolerance, flags)
void launch_norm(const SysDesc *dsys, const Item *vec, int nvec, const Item *fin, int nfin, int slot,
                 int which, hipStream_t st);
// start a cycle from the residual in src_slot: beta = ||r||, v_0 = r / beta
void launch_start_cycle(const SysDesc *dsys, const Item *vec, int nvec, const Item *fin, int nfin,
                        int src_slot, hipStream_t st);
void launch_axpy(const SysDesc *dsys, const Item *vec, int nvec, int dst_slot, int src_slot,
                 hipStream_t st);
// SL_ZB[j] = SL_YH (the preconditioned vector just applied), as FP64
void launch_store_z(const SysDesc *dsys, const Item *vec, int nvec, bool fp64, int j, hipStream_t st);
// SL_YH = src_slot[src_index] in the compute type
void launch_copy_to_yh(const SysDesc *dsys, const Item *vec, int nvec, bool fp64, int src_slot,
                       int src_index, int skip_done, hipStream_t st);
void launch_fill_zero_slot(const SysDesc *dsys, const Item *vec, int nvec, int slot, hipStream_t st);
// DevState of every system of fin into out[0..nfin)
void launch_gather_state(const SysDesc *dsys, const Item *fin, int nfin, DevState *out, hipStream_t st);
// per-solve counters and flags to zero
void launch_reset_state(const SysDesc *dsys, const Item *fin, int nfin, hipStream_t st);
// the factorization's flags (singular pivot, non-finite value) to zero
void launch_reset_factor_flags(const SysDesc *dsys, const Item *fin, int nfin, hipStream_t st);
// export FP64 factors to the caller's row-major stage-major layout
void launch_export(const SysDesc *dsys, const SysDesc &hsys, double *pinv, double *cross, bool coupled,
                   hipStream_t st);
void factor_set_lds_limit(size_t bytes);
// Tasks items[off .. off + n) (consecutive wavefronts of one system's
// factorization: m <= 64, or any m uncoupled) in one launch, each waiting only for the tasks it
// reads (flags fflag[T][s] = epoch; ticket counter at zero on entry and on
// exit); k_factor.hip.
void launch_factor_flow(const SysDesc *dsys, const Item *items, int off, int n, bool coupled, bool sharedJ,
                        int m, size_t shmem, unsigned long long *fflag, unsigned *ticket,
                        unsigned long long epoch, hipStream_t st);

}  // namespace irk
