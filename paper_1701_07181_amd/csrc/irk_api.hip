// irk_api.hip -- host side of libirk: validation, ILU level schedule,
// workspace plan, and the factor / GMRES drivers that enqueue the kernels.
#include "irk.h"
#include "irk_internal.h"
#include "dense64.h"
#include "schedule.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

using namespace irk;

namespace {

struct Launch { int off, n; };
// sweep launch: n SwItem records starting at item `off`, tps elements per
// workgroup, form (0 streaming, 1 prefetching, 2 prefetching without the
// Jacobian columns)
// One sweep level (or, in a merged work set, the members of a level that
// share a launch shape): records at item offset off, n records, tps per
// workgroup.  chain: the level may run chained with its neighbours; group:
// the chain (SwChain) it runs in, -1 for a launch of its own.
struct SwLaunch { int off, n, tps; int form; int region; int chain; int group = -1; };
// A run of consecutive chained levels of one form in one launch
// (k_sweep_flow.hip): workgroup table at item offset tab (one Item per
// workgroup: first record's item offset, records), nblk workgroups; region:
// LDS elements per workgroup (the largest records-per-workgroup times team
// region product of its levels; a workgroup of tps records gives each team
// region / tps).
struct SwChain { int tab, nblk, form, region; };

constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ---------------------------------------------------------------------------
// small dense helpers (host)
// ---------------------------------------------------------------------------

// Gauss-Jordan inverse with row pivoting, n <= 12.  Returns false if singular.
bool host_inverse(int n, const double *a, double *out)
{
    double w[12][24];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j) w[i][j] = (j < n) ? a[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(w[r][c]) > std::fabs(w[p][c])) p = r;
        if (!(std::fabs(w[p][c]) > 0.0) || !std::isfinite(w[p][c])) return false;
        if (p != c)
            for (int j = 0; j < 2 * n; ++j) std::swap(w[c][j], w[p][j]);
        const double inv = 1.0 / w[c][c];
        for (int j = 0; j < 2 * n; ++j) w[c][j] *= inv;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = w[r][c];
            if (f != 0.0)
                for (int j = 0; j < 2 * n; ++j) w[r][j] -= f * w[c][j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) out[i * n + j] = w[i][n + j];
    return true;
}

// Solve the n x n system a x = b (Gaussian elimination with partial pivoting).
bool host_solve(int n, std::vector<double> a, std::vector<double> &b)
{
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(a[r * n + c]) > std::fabs(a[p * n + c])) p = r;
        if (!(std::fabs(a[p * n + c]) > 0.0)) return false;
        if (p != c) {
            for (int j = 0; j < n; ++j) std::swap(a[c * n + j], a[p * n + j]);
            std::swap(b[c], b[p]);
        }
        for (int r = c + 1; r < n; ++r) {
            const double f = a[r * n + c] / a[c * n + c];
            for (int j = c; j < n; ++j) a[r * n + j] -= f * a[c * n + j];
            b[r] -= f * b[c];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double t = b[i];
        for (int j = i + 1; j < n; ++j) t -= a[i * n + j] * b[j];
        b[i] = t / a[i * n + i];
    }
    return true;
}

// P_n(t), P_n'(t) by the recurrences (n+1)P_{n+1} = (2n+1)tP_n - nP_{n-1},
// P'_{n+1} = (n+1)P_n + tP'_n.
void legendre_pd(int n, double t, double &p, double &dp)
{
    double p0 = 1.0, d0 = 0.0;
    if (n == 0) { p = 1.0; dp = 0.0; return; }
    double p1 = t, d1 = 1.0;
    for (int k = 1; k < n; ++k) {
        const double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
        const double d2 = (k + 1.0) * p1 + t * d1;
        p0 = p1; d0 = d1; p1 = p2; d1 = d2;
    }
    (void)d0;
    p = p1; dp = d1;
}

// ---------------------------------------------------------------------------
// problem checks and the level schedule (schedule.h)
// ---------------------------------------------------------------------------
irk_status analyze(const irk_problem *p, Schedule &sc)
{
    const int st = analyze_pattern(p->T, p->nnzb, p->row_ptr, p->col_idx, sc);
    return st == SCHED_OK ? IRK_OK : st == SCHED_BAD_PATTERN ? IRK_ERR_ARG : IRK_ERR_INTERNAL;
}

bool is_mixed(const irk_options *o) { return o->factor_prec != IRK_FP64 || o->matvec_prec != IRK_FP64; }

int factor_type(const irk_options *o)
{
    switch (o->factor_prec) {
    case IRK_FP32: return FT_F32;
    case IRK_BF16: return FT_BF16;
    case IRK_FP16_SCALED: return FT_F16S;
    default: return is_mixed(o) ? FT_F32 : FT_F64;
    }
}

irk_status check_args(const irk_problem *p, const irk_options *o)
{
    if (!p || !o) return IRK_ERR_ARG;
    if (p->s < 1 || p->s > SMAX || !p->A) return IRK_ERR_ARG;
    if (p->T < 1 || p->m < 1 || p->m > MMAX || p->nnzb < p->T) return IRK_ERR_ARG;
    if (!p->row_ptr || !p->col_idx || !p->J || !p->M) return IRK_ERR_ARG;
    if (!(p->nJ == 1 || p->nJ == p->s)) return IRK_ERR_ARG;
    if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return IRK_ERR_ARG;
    if (o->pc < IRK_PC_COUPLED || o->pc > IRK_PC_NONE) return IRK_ERR_ARG;
    if (o->restart < 1 || o->restart > RESTART_MAX) return IRK_ERR_ARG;
    if (o->max_iters < 1 || o->max_outer < 1) return IRK_ERR_ARG;
    if (!(o->rtol > 0.0) || !(o->inner_rtol > 0.0)) return IRK_ERR_ARG;
    if (o->matvec_prec != IRK_FP64 && o->matvec_prec != IRK_FP32) return IRK_ERR_ARG;
    if (o->factor_prec < IRK_FP64 || o->factor_prec > IRK_FP16_SCALED) return IRK_ERR_ARG;
    if (is_mixed(o) && o->pc == IRK_PC_NONE) return IRK_ERR_ARG;
    if (o->shift_rule < 0 || o->shift_rule > 2) return IRK_ERR_ARG;
    if (o->shift_rule == 2 && !o->alpha) return IRK_ERR_ARG;
    if ((long long)p->T * p->m * p->s > (1LL << 31) / 2) return IRK_ERR_ARG;
    for (int k = 0; k < p->s * p->s; ++k)
        if (!std::isfinite(p->A[k])) return IRK_ERR_NONFINITE;
    return IRK_OK;
}

// team count per workgroup for the element kernels: one row / element per
// team, with at least 8 column groups per team where possible
int pick_tpw(int ld, int V)
{
    const int R = ld / V;
    int tpw = 1;
    while (tpw < 8 && (NTHREADS / (tpw * 2)) >= R * 8) tpw *= 2;
    return tpw;
}

// Register budget of the prefetching sweep: the pivot blocks (and, coupled,
// the stored cross blocks one sweep reads and the mass block) of an element
// plus the first Jacobian columns, 8 compute-type values per thread and
// block (VGPRs of 32 bits).
bool sweep_prefetch_fits(int S, bool coupled, int VJ, int VF, bool jac_cols = true)
{
    const int blocks = S + (coupled && S > 1 ? (S - 1) * (S - 2) / 2 + 1 : 0);
    const int per_block = (VF == 2) ? 16 : 8;        // FP64: 8 doubles; float: 8 floats
    const int jac = !jac_cols ? 0 : (VJ == 2) ? 64 : 32;   // 16 FP64 or 8 FP32 column loads
    return blocks * per_block + jac <= 176;
}

// Shape of the sweep launches of one system.  Small levels are latency
// bound: one element per workgroup of SW_THREADS threads in the prefetching
// form when its register budget allows (the most elements per workgroup,
// up to 16, for which each thread covers at most 8 / VF columns of a factor
// block).  Levels of at least big_min elements use big_form: the streaming
// form (0) with teams of at least 8 column groups, which keeps several
// elements in flight per compute unit, or the prefetching form without the
// Jacobian columns (2), which holds fewer registers than the full one.
// Streaming levels of fewer than st_split elements take half tps_st elements
// per workgroup (twice the threads per element), so that a level that does
// not fill the compute units still spreads over them.
struct SweepShape {
    int tps_pf; bool pf; int tps_st; int big_min; int big_form; bool pf_lite;
    bool flow;       // every level in one launch per direction (k_sweep_flow.hip)
    int flow_form;   // its form: 0 streaming (tps_st), 1 prefetching, 2 prefetching
                     // without the Jacobian columns (tps_pf)
    int chain_max;   // otherwise: levels of fewer elements run chained (0: none)
    int st_split;    // 0: none
};

// elements per workgroup of the streaming levels below st_split (0: none)
inline int st_small_tps(const SweepShape &sh) { return (sh.st_split > 0 && sh.tps_st >= 2) ? sh.tps_st / 2 : 0; }

SweepShape pick_sweep(int m, int ldJ, int VJ, int ldF, int VF, int s, bool coupled)
{
    SweepShape sh{0, false, 1, 0, 0, false, false, 0, 0, 0};
    const int RF = ldF / VF, RJ = ldJ / VJ, NQ = 8 / VF;
    for (int tpw = 1; tpw <= 16; tpw *= 2) {
        const int team = SW_THREADS / tpw;
        if (team < RF || team < RJ) break;
        const int G = team / RF;
        if ((m + G - 1) / G <= NQ) sh.tps_pf = tpw;
    }
    sh.pf = sh.tps_pf > 0 && sweep_prefetch_fits(s, coupled, VJ, VF);
    sh.pf_lite = sh.tps_pf > 0 && sweep_prefetch_fits(s, coupled, VJ, VF, false);
    const int R = std::max(RF, RJ);
    while (sh.tps_st < 8 && SW_THREADS / (sh.tps_st * 2) >= R * 8) sh.tps_st *= 2;
    sh.big_min = 256;
    if (const char *e = std::getenv("IRK_SWEEP_BIG")) sh.big_min = std::max(1, std::atoi(e));
    if (const char *e = std::getenv("IRK_SWEEP_BIG_FORM")) sh.big_form = (std::atoi(e) == 2) ? 2 : 0;
    if (!sh.pf) { sh.tps_pf = sh.tps_st; sh.big_min = 1; }
    sh.flow_form = sh.pf ? 1 : 0;
    if (const char *e = std::getenv("IRK_SWEEP_FLOW")) {
        const int f = std::atoi(e);            // 1: single launch, default form; 10 + form: that form
        sh.flow = f > 0;
        if (f >= 10) sh.flow_form = (f - 10 == 1 && sh.pf) ? 1 : (f - 10 == 2 && sh.pf_lite) ? 2 : 0;
    }
    if (const char *e = std::getenv("IRK_SWEEP_CHAIN")) sh.chain_max = std::max(0, std::atoi(e));
    if (const char *e = std::getenv("IRK_SWEEP_SPLIT")) sh.st_split = std::max(0, std::atoi(e));
    return sh;
}

struct Plan {
    size_t o_dsys, o_dsys2, o_st, o_ints, o_items, o_J, o_M, o_J32, o_M32, o_P64, o_C64, o_P32, o_C32,
        o_P16, o_C16, o_P16e, o_C16e, o_Fscr, o_vec[NSLOT], o_H, o_g, o_cs, o_sn, o_y,
        o_hbuf, o_part, o_gather, o_flow, o_ticket, o_fflag, o_fticket, total;
    int ld, ld32, ld16, nitems_max;
};

Plan make_plan(const irk_problem *p, const irk_options *o)
{
    Plan P;
    std::memset(&P, 0, sizeof(P));
    const int s = p->s, T = p->T, m = p->m, R = o->restart;
    P.ld = round_up(m, 2);
    P.ld32 = round_up(m, 4);
    P.ld16 = round_up(m, 8);
    const bool mixed = is_mixed(o);
    const bool coupled = (o->pc == IRK_PC_COUPLED) && s > 1;
    const int ft = factor_type(o);
    const long long N = (long long)s * T * m;
    // cross blocks C_{lq} with l, q >= 1 (those in stage row or column 0 stay
    // multiples of M and are not stored)
    const long long nblkP = (long long)T * s, nblkC = coupled ? (long long)T * (s - 1) * (s - 2) : 0;
    // sweep records (four lists; chained levels padded to whole workgroups of
    // up to 16), chain workgroup tables, padded factor tasks
    P.nitems_max = T * (24 + 10 * s + 4 * 3 * 15 + 8) + 2 * RED_BLOCKS + 64;
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o2 = off; off = align256(off + bytes); return o2; };
    P.o_dsys = take(sizeof(SysDesc));
    P.o_dsys2 = take(sizeof(SysDesc));
    P.o_st = take(sizeof(DevState));
    P.o_ints = take(sizeof(int) * ((size_t)(T + 1) + 2 * (size_t)p->nnzb + 3 * (size_t)T));
    P.o_items = take(sizeof(Item) * (size_t)P.nitems_max);
    P.o_J = take(sizeof(double) * (size_t)p->nJ * p->nnzb * m * P.ld);
    P.o_M = take(sizeof(double) * (size_t)T * m * P.ld);
    if (mixed) {
        P.o_J32 = take(sizeof(float) * (size_t)p->nJ * p->nnzb * m * P.ld32);
        P.o_M32 = take(sizeof(float) * (size_t)T * m * P.ld32);
    }
    if (o->pc != IRK_PC_NONE) {
        P.o_P64 = take(sizeof(double) * (size_t)nblkP * m * P.ld);
        if (nblkC) P.o_C64 = take(sizeof(double) * (size_t)nblkC * m * P.ld);
        // product scratch of the factorization for m > 64 (smaller blocks
        // keep their intermediate products in registers and LDS)
        if (m > 64) P.o_Fscr = take(sizeof(double) * (size_t)nblkP * m * P.ld);
        if (mixed && ft == FT_F32) {
            P.o_P32 = take(sizeof(float) * (size_t)nblkP * m * P.ld32);
            if (nblkC) P.o_C32 = take(sizeof(float) * (size_t)nblkC * m * P.ld32);
        } else if (mixed) {
            P.o_P16 = take(sizeof(uint16_t) * (size_t)nblkP * m * P.ld16);
            P.o_P16e = take(sizeof(int) * (size_t)nblkP);
            if (nblkC) {
                P.o_C16 = take(sizeof(uint16_t) * (size_t)nblkC * m * P.ld16);
                P.o_C16e = take(sizeof(int) * (size_t)nblkC);
            }
        }
    }
    for (int sl = 0; sl < NSLOT; ++sl) {
        if (sl == SL_D) { P.o_vec[sl] = (size_t)-1; continue; }
        if (sl == SL_ZB && o->pc == IRK_PC_NONE) { P.o_vec[sl] = (size_t)-1; continue; }
        const size_t n = (sl == SL_V) ? (size_t)(R + 1) * N : (sl == SL_ZB) ? (size_t)R * N : (size_t)N;
        P.o_vec[sl] = take(sizeof(double) * n);
    }
    P.o_H = take(sizeof(double) * (size_t)(R + 1) * R);
    P.o_g = take(sizeof(double) * (size_t)(R + 1));
    P.o_cs = take(sizeof(double) * (size_t)R);
    P.o_sn = take(sizeof(double) * (size_t)R);
    P.o_y = take(sizeof(double) * (size_t)R);
    P.o_hbuf = take(sizeof(double) * 2 * (RESTART_MAX + 1));
    P.o_part = take(sizeof(double) * (size_t)RED_BLOCKS * (RESTART_MAX + 2));
    P.o_gather = take(sizeof(DevState));
    if (o->pc != IRK_PC_NONE) {
        P.o_flow = take(sizeof(unsigned long long) * (size_t)T);   // single-launch sweep flags
        P.o_ticket = take(sizeof(unsigned));                        // its ticket counter
        P.o_fflag = take(sizeof(unsigned long long) * (size_t)T * s);   // factorization task flags
        P.o_fticket = take(sizeof(unsigned));                             // their ticket counter
    }
    P.total = off;
    return P;
}

#define HIPCHK(x)                                   \
    do {                                            \
        if ((x) != hipSuccess) return IRK_ERR_DEVICE; \
    } while (0)

}  // namespace

// ---------------------------------------------------------------------------
// work sets: the merged work items of one or more systems
// ---------------------------------------------------------------------------
namespace {

struct WorkSet {
    const SysDesc *dsys = nullptr;   // device table the items index into
    Item *ditems = nullptr;          // device copy of `items`
    std::vector<Item> items;
    Launch mv64{0, 0}, mv32{0, 0}, vec{0, 0}, fin{0, 0};
    std::vector<SwLaunch> fwd64, bwd64, fwd32, bwd32;   // one or more per level
    int smax = 1, restart = 1, nsys = 0;
    bool mixed = false, coupled = false, sharedJ = true, has_pc = true;
    int ftype = FT_F64;
    size_t shm_mv64 = 0, shm_mv32 = 0, shm_sw64 = 0, shm_sw32 = 0;
    // runs of chained levels of each sweep, and the ticket counter their
    // launches claim workgroups from
    std::vector<SwChain> cf64, cb64, cf32, cb32;
    unsigned *dticket = nullptr;
};

}  // namespace

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
struct irk_handle {
    int s, T, m, nnzb, nJ;
    double dt;
    double A[SMAX * SMAX], Ainv[SMAX * SMAX], alpha[SMAX];
    irk_options opt;
    hipStream_t stream;
    char *ws;
    size_t ws_bytes;
    Plan plan;
    SysDesc hsys;
    SysDesc *dsys;
    Item *ditems;
    DevState *dst;
    DevState *dgather;   // one gathered DevState (device)
    DevState *hst;       // pinned host mirror
    Schedule sc;
    std::vector<int> ints;
    // per-system work lists (sys = 0) and factorization tasks
    WorkSet W;
    int tpw64, tpw32, nblk;
    SweepShape sw64, sw32;   // sweep launch shapes (FP64, mixed inner)
    std::vector<Launch> fa;    // factor tasks, one launch per wavefront
    std::vector<Item> fitems;
    size_t shm_fac;
    bool mixed, coupled, sharedJ, factored;
    bool factor_pending = false;   // an asynchronous factorization's flags not read yet
    int ftype;
    int bad_element;
    float ms_factor;
    hipEvent_t ev0, ev1, ev_ready;
    hipEvent_t ev_done = nullptr;   // end of the last set-up, value update or factorization
    hipEvent_t ev_s0 = nullptr, ev_s1 = nullptr;   // span of a time step
    hipEvent_t ev_f0 = nullptr, ev_f1 = nullptr;   // span of the last factorization
    SysDesc solve_desc;  // descriptor with the caller's rhs / x (staging for the copy)
    SysDesc *dsys_solve = nullptr;   // its device copy (the work set's descriptor during a solve)
    // An asynchronous factorization runs on sstream (ev_pre: the point of
    // the handle's stream it starts from; ev_factored: its end), so that what
    // the caller enqueues next on the handle's stream (a solve's initial
    // residual) runs beside it.  factor_side: the handle's stream has not
    // waited for it yet (join_factor).
    hipStream_t sstream = nullptr;
    hipEvent_t ev_pre = nullptr, ev_factored = nullptr, ev_tail = nullptr;
    hipEvent_t ev_read = nullptr;   // end of an in-cycle state copy (run_cycle)
    // part_levels > 0: ev_part marks the end of the wavefront after which the
    // factors of the first part_levels forward levels are final (those of
    // the forward sweep's first launch group)
    hipEvent_t ev_part = nullptr;
    int part_levels = 0;
    // dependency-driven factorization (k_factor_flow): its task flags and
    // ticket counter
    bool factor_flow = false;
    unsigned long long *dfflag = nullptr;
    unsigned *dfticket = nullptr;
    bool factor_side = false;
    int ncu = 0;         // compute units of the device
    // profiling: event pool and recorded intervals (kind, event index)
    bool prof;
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<int, int>> spans;
    int dropped;
};

struct irk_batch {
    int capacity;
    long long max_elements;
    hipStream_t stream;
    char *ws;
    size_t ws_bytes;
    SysDesc *dtab;               // device table [capacity]
    DevState *dgather;           // [capacity]
    Item *ditems;
    unsigned *dticket;           // ticket counter of the single-launch sweeps
    size_t max_items;
    std::vector<SysDesc> htab;   // host copy of the table
    DevState *hgather;           // [capacity]: pinned (own_host) or the caller's host array
    bool own_host = true;
    std::vector<hipEvent_t> slot_ev;   // start of the member in each slot
    struct Member {
        irk_handle *h;
        int slot;
        long long tag;
        double *x;
        int phase;               // 0 queued, 1 iterating, 2 finished
        double bn, rel, est;
        int cycles, stall;
        irk_status status;
        irk_solve_info info;
        hipEvent_t t0;
    };
    std::vector<Member> members;   // queued and iterating
    std::vector<Member> retired;
    std::vector<int> free_slots;
    hipEvent_t ev_end;
    hipEvent_t ev_f0 = nullptr, ev_f1 = nullptr;   // span of a batched factorization
    hipEvent_t ev_read = nullptr;                  // end of an in-cycle state copy (run_cycle)
};

namespace {
enum ProfKind { PK_MV64 = 0, PK_MV32, PK_PC, PK_ORTH, PK_FACTOR, PK_UNTR, PK_N };

// Start an interval; returns its pool index or -1.
// The handle's stream waits for an asynchronous factorization running on
// the side stream (before anything that reads or writes the factors, or
// writes what the factorization reads).
irk_status join_factor(irk_handle *h)
{
    if (!h->factor_side) return IRK_OK;
    h->factor_side = false;
    return hipStreamWaitEvent(h->stream, h->ev_factored, 0) == hipSuccess ? IRK_OK : IRK_ERR_DEVICE;
}

int prof_begin(irk_handle *h)
{
    if (!h || !h->prof) return -1;
    const int idx = 2 * (int)h->spans.size();
    if (idx + 1 >= (int)h->pool.size()) { h->dropped++; return -1; }
    hipEventRecord(h->pool[idx], h->stream);
    return idx;
}
void prof_end(irk_handle *h, int idx, int kind)
{
    if (idx < 0) return;
    hipEventRecord(h->pool[idx + 1], h->stream);
    h->spans.push_back({kind, idx});
}

// Launch context: where the items live, which stream, optional profiling.
struct Ctx {
    WorkSet *W;
    hipStream_t st;
    irk_handle *prof;      // handle whose event pool records intervals (or null)
    hipEvent_t ev_read = nullptr;   // end of a state copy the host reads later (or null)
    // the next forward sweep waits for ev_rest before its launches of
    // levels >= rest_level (the end of a factorization whose earlier
    // wavefronts it already waited for); cleared once that wait is enqueued
    hipEvent_t ev_rest = nullptr;
    int rest_level = 0;
};

// Sweep records of every level (in level order) of one system, one launch
// per level; region = LDS elements of one team (region_st2: of a streaming
// team at st_small_tps elements per workgroup).
void add_level_records(std::vector<Item> &items, const Schedule &sc, const int32_t *rp,
                       const int32_t *ci, bool fwd, const SweepShape &sh, int region_pf,
                       int region_st, int region_st2, std::vector<SwLaunch> &out)
{
    out.clear();
    const std::vector<int> &off = fwd ? sc.off_fwd : sc.off_bwd;
    const std::vector<int> &lst = fwd ? sc.lvl_fwd : sc.lvl_bwd;
    for (size_t l = 0; l + 1 < off.size(); ++l) {
        const bool big = off[l + 1] - off[l] >= sh.big_min;
        const bool lite = big && sh.big_form == 2 && sh.pf_lite;
        SwLaunch L{(int)items.size(), 0, (big && !lite) ? sh.tps_st : sh.tps_pf,
                   lite ? 2 : (sh.pf && !big ? 1 : 0), (big && !lite) ? region_st : region_pf};
        if (big && !lite && st_small_tps(sh) && off[l + 1] - off[l] < sh.st_split) {
            L.tps = st_small_tps(sh);
            L.region = region_st2;
        }
        if (sh.flow) {
            // one form for every level
            L.tps = sh.flow_form == 0 ? sh.tps_st : sh.tps_pf;
            L.form = sh.flow_form;
            L.region = sh.flow_form == 0 ? region_st : region_pf;
        }
        // chained levels hold whole workgroups
        L.chain = (sh.flow || off[l + 1] - off[l] < sh.chain_max) ? 1 : 0;
        for (int a = off[l]; a < off[l + 1]; ++a) {
            const int i = lst[a];
            SwItem r;
            std::memset(&r, 0, sizeof(r));
            r.sys = 0;
            r.i = i;
            r.pa = fwd ? rp[i] : sc.diag[i] + 1;
            r.nb = fwd ? sc.diag[i] - rp[i] : rp[i + 1] - sc.diag[i] - 1;
            for (int b = 0; b < r.nb && b < SW_NB; ++b) r.col[b] = ci[r.pa + b];
            Item it[3];
            std::memcpy(it, &r, sizeof(r));
            items.insert(items.end(), it, it + 3);
            L.n++;
        }
        while (L.chain && L.n % L.tps) {
            SwItem r;
            std::memset(&r, 0, sizeof(r));
            r.i = -1;
            Item it[3];
            std::memcpy(it, &r, sizeof(r));
            items.insert(items.end(), it, it + 3);
            L.n++;
        }
        if (L.n) out.push_back(L);
    }
}

// Runs of consecutive chained levels of one form (whole workgroups, within
// the LDS limit) become chains: their workgroup tables are appended to
// items and the levels point at their chain.  A run of one level stays a
// launch of its own.
void make_chains(std::vector<Item> &items, std::vector<SwLaunch> &L, size_t w, std::vector<SwChain> &out)
{
    out.clear();
    for (SwLaunch &x : L) x.group = -1;
    auto fits = [&](const SwLaunch &x) { return x.chain && x.n % x.tps == 0; };
    size_t a = 0;
    while (a < L.size()) {
        if (!fits(L[a])) { ++a; continue; }
        int region = L[a].tps * L[a].region;
        size_t b = a + 1;
        while (b < L.size() && fits(L[b]) && L[b].form == L[a].form) {
            const int r2 = std::max(region, L[b].tps * L[b].region);
            if (w * (size_t)r2 + 64 > 160 * 1024) break;
            region = r2;
            ++b;
        }
        if (b - a >= 2 && w * (size_t)region + 64 <= 160 * 1024) {
            SwChain c{(int)items.size(), 0, L[a].form, region};
            for (size_t q = a; q < b; ++q) {
                for (int r = 0; r < L[q].n; r += L[q].tps) {
                    items.push_back(Item{0, L[q].off + 3 * r, L[q].tps, 0});
                    c.nblk++;
                }
                L[q].group = (int)out.size();
            }
            out.push_back(c);
        }
        a = b;
    }
}

// Epochs of the sweeps that chain levels: one per sweep, increasing over
// the process, so a flag from an earlier sweep never equals the current one.
std::atomic<unsigned long long> g_flow_epoch{0};

int reduction_chunks(long long N)
{
    const long long nb = (N + NTHREADS * 4 - 1) / (NTHREADS * 4);
    return (int)std::max(1LL, std::min<long long>(nb, RED_BANK));
}

size_t lds_matvec(int S, int m, int maxrow, int ld, int V, int tpw, size_t w)
{
    return w * (size_t)tpw * matvec_region(S, m, maxrow, ld, V, NTHREADS / tpw);
}
// LDS elements of one sweep team (FP64 sweep, or the mixed inner sweep with
// FP32 Jacobian and factors of type ftype)
int sw_region(int S, int m, int maxrow, const Plan &P, bool fp64, int ftype, int tps)
{
    const int team = SW_THREADS / tps;
    if (fp64) return sweep_region(S, m, maxrow, team, P.ld, 2, P.ld, 2);
    const int ldF = (ftype == FT_F32) ? P.ld32 : P.ld16, VF = (ftype == FT_F32) ? 4 : 8;
    return sweep_region(S, m, maxrow, team, P.ld32, 4, ldF, VF);
}

// Work lists of several systems merged: every list of member q is copied
// with sys = q; level l of the merged sweep holds level l of every member.
void build_merged(WorkSet &M, const std::vector<std::pair<irk_handle *, int>> &mem)
{
    M.items.clear();
    M.fwd64.clear(); M.bwd64.clear(); M.fwd32.clear(); M.bwd32.clear();
    M.cf64.clear(); M.cb64.clear(); M.cf32.clear(); M.cb32.clear();
    M.nsys = (int)mem.size();
    if (mem.empty()) return;
    const irk_handle *h0 = mem[0].first;
    M.mixed = h0->mixed; M.coupled = h0->coupled; M.sharedJ = h0->sharedJ;
    M.has_pc = h0->opt.pc != IRK_PC_NONE; M.ftype = h0->ftype;
    M.smax = 1; M.restart = 1;
    for (auto &pr : mem) {
        M.smax = std::max(M.smax, pr.first->s);
        M.restart = std::max(M.restart, pr.first->opt.restart);
    }
    auto copy_list = [&](const Launch &L, const irk_handle *h, int sys) {
        for (int a = 0; a < L.n; ++a) {
            Item it = h->W.items[L.off + a];
            it.sys = sys;
            M.items.push_back(it);
        }
    };
    auto merge = [&](Launch WorkSet::*f, Launch &out) {
        out.off = (int)M.items.size();
        for (auto &pr : mem) copy_list(pr.first->W.*f, pr.first, pr.second);
        out.n = (int)M.items.size() - out.off;
    };
    // Sweep levels: level l of every member; members with the same elements
    // per workgroup share a launch.  Records are copied with their system
    // index; the team region is the largest one of the launch (S = smax).
    auto merge_sweeps = [&](std::vector<SwLaunch> WorkSet::*f, bool fp64, std::vector<SwLaunch> &out) {
        size_t L = 0;
        for (auto &pr : mem) L = std::max(L, (pr.first->W.*f).size());
        for (size_t l = 0; l < L; ++l) {
            std::vector<int> seen;
            for (auto &pr0 : mem) {
                const auto &lv0 = pr0.first->W.*f;
                if (l >= lv0.size()) continue;
                const int tps = lv0[l].tps;
                if (std::find(seen.begin(), seen.end(), tps) != seen.end()) continue;
                seen.push_back(tps);
                SwLaunch o{(int)M.items.size(), 0, tps, -1, 0, 1};
                for (auto &pr : mem) {
                    const irk_handle *h = pr.first;
                    const auto &lv = h->W.*f;
                    if (l >= lv.size() || lv[l].tps != tps) continue;
                    const SwLaunch &src = lv[l];
                    const int padded = (src.n + tps - 1) / tps * tps;   // whole workgroups per system
                    for (int a = 0; a < padded; ++a) {
                        SwItem r;
                        if (a < src.n) {
                            std::memcpy(&r, &h->W.items[src.off + 3 * a], sizeof(r));
                        } else {
                            std::memset(&r, 0, sizeof(r));
                            r.i = -1;
                        }
                        r.sys = pr.second;
                        Item it[3];
                        std::memcpy(it, &r, sizeof(r));
                        M.items.insert(M.items.end(), it, it + 3);
                    }
                    o.n += padded;
                    const int VF = fp64 ? 2 : ((h->ftype == FT_F32) ? 4 : 8);
                    // one form per launch: the members' common one if it fits
                    // every member at S = smax, else the streaming form
                    const bool fits = src.form == 0 ||
                                      sweep_prefetch_fits(M.smax, M.coupled, fp64 ? 2 : 4, VF, src.form == 1);
                    o.form = (o.form == -1 || o.form == src.form) && fits ? src.form : 0;
                    o.region = std::max(o.region, sw_region(M.smax, h->m, h->sc.maxrow, h->plan, fp64,
                                                            h->ftype, tps));
                    o.chain = o.chain && src.chain;
                }
                if (o.n) out.push_back(o);
            }
        }
    };
    merge(&WorkSet::mv64, M.mv64);
    if (M.mixed) merge(&WorkSet::mv32, M.mv32);
    merge(&WorkSet::vec, M.vec);
    merge(&WorkSet::fin, M.fin);
    if (M.has_pc) {
        merge_sweeps(&WorkSet::fwd64, true, M.fwd64);
        merge_sweeps(&WorkSet::bwd64, true, M.bwd64);
        if (M.mixed) {
            merge_sweeps(&WorkSet::fwd32, false, M.fwd32);
            merge_sweeps(&WorkSet::bwd32, false, M.bwd32);
        }
        make_chains(M.items, M.fwd64, sizeof(double), M.cf64);
        make_chains(M.items, M.bwd64, sizeof(double), M.cb64);
        make_chains(M.items, M.fwd32, sizeof(float), M.cf32);
        make_chains(M.items, M.bwd32, sizeof(float), M.cb32);
    }

    // LDS for the merged launches (template S = smax for every member)
    M.shm_mv64 = M.shm_mv32 = M.shm_sw64 = M.shm_sw32 = 0;
    for (auto &pr : mem) {
        const irk_handle *h = pr.first;
        const Plan &P = h->plan;
        const int mr = h->sc.maxrow;
        M.shm_mv64 = std::max(M.shm_mv64, lds_matvec(M.smax, h->m, mr, P.ld, 2, h->tpw64, sizeof(double)));
        for (int tps : {h->sw64.tps_pf, h->sw64.tps_st, st_small_tps(h->sw64)})
            if (tps)
                M.shm_sw64 = std::max(M.shm_sw64, sizeof(double) * tps * (size_t)sw_region(M.smax, h->m, mr, P, true, h->ftype, tps));
        if (M.mixed) {
            M.shm_mv32 = std::max(M.shm_mv32, lds_matvec(M.smax, h->m, mr, P.ld32, 4, h->tpw32, sizeof(float)));
            for (int tps : {h->sw32.tps_pf, h->sw32.tps_st, st_small_tps(h->sw32)})
                if (tps)
                    M.shm_sw32 = std::max(M.shm_sw32, sizeof(float) * tps * (size_t)sw_region(M.smax, h->m, mr, P, false, h->ftype, tps));
        }
    }
}

// z = P^{-1} v into SL_YH; acc_slot >= 0 also adds it to that FP64 slot
void enqueue_pc(Ctx &C, bool fp64, int v_slot, int v_index, int acc_slot, int skip_done)
{
    WorkSet &W = *C.W;
    const int pi = prof_begin(C.prof);
    const std::vector<SwLaunch> &F = fp64 ? W.fwd64 : W.fwd32;
    const std::vector<SwLaunch> &B = fp64 ? W.bwd64 : W.bwd32;
    const int ft = fp64 ? FT_F64 : W.ftype;
    const size_t w = fp64 ? sizeof(double) : sizeof(float);
    // Levels in a chain run in its one launch (k_sweep_flow.hip); every
    // launch of a sweep with chains publishes its elements' flags with the
    // sweep's epoch, which the chained launches wait for.
    const std::vector<SwChain> &CF = fp64 ? W.cf64 : W.cf32;
    const std::vector<SwChain> &CB = fp64 ? W.cb64 : W.cb32;
    auto run = [&](const std::vector<SwLaunch> &L, const std::vector<SwChain> &CH, bool fwd, int acc) {
        const unsigned long long ep = (!CH.empty() && W.dticket) ? ++g_flow_epoch : 0;
        size_t a = 0;
        while (a < L.size()) {
            if (C.ev_rest && (!fwd || (int)a >= C.rest_level)) {
                // (a failure shows in the caller's hipGetLastError check)
                (void)hipStreamWaitEvent(C.st, C.ev_rest, 0);
                C.ev_rest = nullptr;
            }
            const SwLaunch &A = L[a];
            if (ep && A.group >= 0) {
                const SwChain &c = CH[A.group];
                launch_sweep_flow(fwd, W.dsys, W.ditems, c.tab, c.nblk, c.region, W.smax, fp64, ft, W.coupled,
                                  W.sharedJ, v_slot, v_index, acc, skip_done, w * c.region, C.st,
                                  c.form, W.dticket, ep);
                while (a < L.size() && L[a].group == A.group) ++a;
                continue;
            }
            launch_sweep(fwd, W.dsys, reinterpret_cast<const SwItem *>(W.ditems + A.off), A.n, A.tps,
                         A.region, W.smax, fp64, ft, W.coupled, W.sharedJ, v_slot, v_index, acc, skip_done,
                         w * A.tps * A.region, C.st, A.form, ep);
            ++a;
        }
    };
    run(F, CF, true, -1);
    run(B, CB, false, acc_slot);
    prof_end(C.prof, pi, PK_PC);
}

void enqueue_matvec(Ctx &C, bool fp64, int x_slot, int y_slot, int b_slot, int mode, int skip_done)
{
    WorkSet &W = *C.W;
    const Launch &L = fp64 ? W.mv64 : W.mv32;
    const int pi = prof_begin(C.prof);
    launch_matvec(W.dsys, W.ditems + L.off, L.n, W.smax, fp64 ? 0 : 1, W.sharedJ, x_slot, y_slot,
                  b_slot, mode, skip_done, fp64 ? W.shm_mv64 : W.shm_mv32, C.st);
    prof_end(C.prof, pi, fp64 ? PK_MV64 : PK_MV32);
}

irk_status sync_states(Ctx &C, DevState *dgather, DevState *hgather)
{
    WorkSet &W = *C.W;
    launch_gather_state(W.dsys, W.ditems + W.fin.off, W.fin.n, dgather, C.st);
    HIPCHK(hipMemcpyAsync(hgather, dgather, sizeof(DevState) * W.fin.n, hipMemcpyDeviceToHost, C.st));
    HIPCHK(hipStreamSynchronize(C.st));
    return IRK_OK;
}

// A system being solved: its handle, its position in the work set, progress.
struct Solve {
    irk_handle *h;
    double *x = nullptr;     // the solution vector the solve updates
    double bn = 0, rel = 0, est = 0;
    int cycles = 0, stall = 0;
    bool finished = false;
    irk_status status = IRK_OK;
    irk_solve_info info{};
};

void finish(Solve &S, const DevState &st, irk_status status)
{
    S.finished = true;
    S.status = status;
    S.info.iters = st.iters;
    S.info.outer_iters = std::max(S.cycles, 1);
    S.info.restarts = std::max(S.cycles - 1, 0);
    S.info.rel_res_true = S.rel;
    S.info.rel_res_est = S.est;
    S.info.equiv_mults = st.iters * S.h->s;
    S.info.converged = (S.rel <= S.h->opt.rtol) ? 1 : 0;
    S.info.bad_element = -1;
    S.info.ms_factor = S.h->ms_factor;
}

// Initial residual of every system of the work set: ||b||, r = b - B x,
// first cycle start.  Systems already converged (or with b = 0 or
// non-finite data) are finished here.
irk_status init_systems(Ctx &C, std::vector<Solve *> &sv, DevState *dg, DevState *hg)
{
    WorkSet &W = *C.W;
    const Item *vec = W.ditems + W.vec.off, *fin = W.ditems + W.fin.off;
    launch_reset_state(W.dsys, fin, W.fin.n, C.st);
    launch_norm(W.dsys, vec, W.vec.n, fin, W.fin.n, SL_B, 0, C.st);
    enqueue_matvec(C, true, SL_X, SL_R, SL_B, 1, 0);
    launch_start_cycle(W.dsys, vec, W.vec.n, fin, W.fin.n, SL_R, C.st);
    HIPCHK(hipGetLastError());
    irk_status st = sync_states(C, dg, hg);
    if (st != IRK_OK) return st;
    for (size_t q = 0; q < sv.size(); ++q) {
        Solve &S = *sv[q];
        const DevState &d = hg[q];
        S.bn = d.bnorm;
        if (d.nonfinite || !std::isfinite(S.bn)) { S.rel = NAN; finish(S, d, IRK_ERR_NONFINITE); continue; }
        if (S.bn == 0.0) {
            // x = 0 solves B x = 0 exactly
            HIPCHK(hipMemsetAsync(S.x, 0, sizeof(double) * S.h->hsys.N, C.st));
            S.rel = 0.0;
            finish(S, d, IRK_OK);
            continue;
        }
        S.rel = d.beta / S.bn;
        S.est = S.rel;
        if (!std::isfinite(S.rel)) { finish(S, d, IRK_ERR_NONFINITE); continue; }
        if (S.rel <= S.h->opt.rtol) finish(S, d, IRK_OK);
    }
    return IRK_OK;
}

// One GMRES cycle for every system of the work set (all unfinished):
// up to `restart` Arnoldi steps (systems drop out when their estimate meets
// the cycle tolerance), x += Z y (z_j = P^{-1} v_j kept from the steps),
// FP64 true residual, next cycle start.
irk_status run_cycle(Ctx &C, std::vector<Solve *> &sv, DevState *dg, DevState *hg)
{
    WorkSet &W = *C.W;
    const Item *vec = W.ditems + W.vec.off, *fin = W.ditems + W.fin.off;
    const bool fp64 = !W.mixed;
    // The host reads the systems' state only at some steps (the device ends
    // a system's cycle by itself: steps after its convergence do nothing).
    // Several systems: every second step.  One system: first after two
    // steps, then one step before the step at which the estimate, shrinking
    // at the rate observed since the previous read (the cycle's starting
    // residual for the first), would meet the tolerance.
    const int check_every = (W.nsys == 1) ? 1 : 2;
    int next_check = (W.nsys == 1) ? std::min(1, W.restart - 1) : check_every - 1;
    double prev_est = (W.nsys == 1) ? hg[0].beta : -1.0;
    int prev_j = -1;
    // A read expected not to end the cycle overlaps the next step: its copy
    // is issued after step j, the next step is enqueued, and only then does
    // the host wait for the copy (the device runs that step meanwhile; if
    // the read shows the cycle ended, the step's kernels skip the ended
    // systems).  The last step of a cycle, and a single system's steps from
    // the one at which its estimate is predicted to meet the tolerance on,
    // are read at once.
    int pend_j = -1;          // step whose state copy is in flight
    int last_pred = -1;       // one system: step predicted to end the cycle
    auto consume = [&](int rj) -> bool {
        bool all_done = true;
        for (int q = 0; q < W.nsys; ++q) all_done = all_done && hg[q].done;
        if (all_done) return true;
        next_check = rj + check_every;
        if (W.nsys == 1) {
            const double est = hg[0].est, tol = hg[0].tol_abs;
            if (prev_est > 0.0 && est > 0.0 && est < prev_est && tol > 0.0 && tol < est) {
                // steps still needed at the per-step rate since the last read
                const double steps = std::log(tol / est) * (rj - prev_j) / std::log(est / prev_est);
                if (steps > 2.0 && steps < 1e6) next_check = rj + (int)steps - 1;
                if (steps > 0.0 && steps < 1e6) last_pred = rj + std::max(1, (int)steps);
            }
            prev_est = est;
            prev_j = rj;
        }
        return false;
    };
    for (int j = 0; j < W.restart; ++j) {
        if (W.has_pc) {
            enqueue_pc(C, fp64, SL_V, j, -1, 1);
            launch_store_z(W.dsys, vec, W.vec.n, fp64, j, C.st);
        } else {
            launch_copy_to_yh(W.dsys, vec, W.vec.n, true, SL_V, j, 1, C.st);
        }
        enqueue_matvec(C, fp64, SL_YH, SL_W, -1, 0, 1);
        const int po = prof_begin(C.prof);
        launch_arnoldi(W.dsys, vec, W.vec.n, fin, W.fin.n, j, C.st);
        prof_end(C.prof, po, PK_ORTH);
        if (pend_j >= 0) {
            HIPCHK(hipEventSynchronize(C.ev_read));
            const int rj = pend_j;
            pend_j = -1;
            if (consume(rj)) break;
        }
        if (j >= next_check || j + 1 == W.restart) {
            const bool at_once = !C.ev_read || j + 1 == W.restart ||
                                 (W.nsys == 1 && last_pred >= 0 && j >= last_pred);
            if (at_once) {
                irk_status st = sync_states(C, dg, hg);
                if (st != IRK_OK) return st;
                if (consume(j)) break;
            } else {
                launch_gather_state(W.dsys, fin, W.fin.n, dg, C.st);
                HIPCHK(hipMemcpyAsync(hg, dg, sizeof(DevState) * W.fin.n, hipMemcpyDeviceToHost, C.st));
                HIPCHK(hipEventRecord(C.ev_read, C.st));
                pend_j = j;
            }
        }
    }
    // (a copy still in flight is that of a step whose successor was the
    // last: it ended with a read at once)
    if (pend_j >= 0) HIPCHK(hipEventSynchronize(C.ev_read));
    // x += Z y with the stored z_j = P^{-1} v_j (equal to P^{-1} V y, without
    // one more preconditioner application)
    launch_cycle_end(W.dsys, vec, W.vec.n, W.restart, W.has_pc ? SL_ZB : SL_V, C.st);
    launch_axpy(W.dsys, vec, W.vec.n, SL_X, SL_U, C.st);
    // FP64 true residual and the next cycle (whose start keeps the finished
    // cycle's breakdown flag and estimate: one read for both)
    enqueue_matvec(C, true, SL_X, SL_R, SL_B, 1, 0);
    launch_start_cycle(W.dsys, vec, W.vec.n, fin, W.fin.n, SL_R, C.st);
    HIPCHK(hipGetLastError());
    irk_status st = sync_states(C, dg, hg);
    if (st != IRK_OK) return st;
    for (int q = 0; q < W.nsys; ++q) {
        Solve &S = *sv[q];
        const DevState &d = hg[q];
        const irk_options &o = S.h->opt;
        const double newrel = d.beta / S.bn;
        S.est = d.prev_est / std::max(S.bn, 1e-300);
        S.cycles++;
        if (d.nonfinite || !std::isfinite(newrel)) { S.rel = newrel; finish(S, d, IRK_ERR_NONFINITE); continue; }
        if (newrel <= o.rtol) { S.rel = newrel; finish(S, d, IRK_OK); continue; }
        if (d.prev_breakdown && !(newrel < 0.5 * S.rel)) {
            if (++S.stall >= 2) { S.rel = newrel; finish(S, d, IRK_ERR_BREAKDOWN); continue; }
        }
        S.rel = newrel;
        if (d.iters >= o.max_iters || (S.h->mixed && S.cycles >= o.max_outer)) {
            finish(S, d, IRK_ERR_NOCONV);
            continue;
        }
    }
    return IRK_OK;
}

}  // namespace

extern "C" {

const char *irk_status_str(irk_status st)
{
    switch (st) {
    case IRK_OK: return "ok";
    case IRK_ERR_ARG: return "invalid argument";
    case IRK_ERR_NOMEM: return "workspace too small";
    case IRK_ERR_SINGULAR: return "singular pivot block";
    case IRK_ERR_NOCONV: return "not converged within max_iters";
    case IRK_ERR_BREAKDOWN: return "Krylov breakdown";
    case IRK_ERR_NONFINITE: return "non-finite value";
    case IRK_ERR_DEVICE: return "HIP runtime error";
    case IRK_ERR_STATE: return "call out of order";
    case IRK_ERR_INTERNAL: return "internal consistency check failed";
    }
    return "unknown status";
}

irk_status irk_default_options(irk_options *o)
{
    if (!o) return IRK_ERR_ARG;
    o->pc = IRK_PC_COUPLED;
    o->shift_rule = 0;
    o->alpha = nullptr;
    o->matvec_prec = IRK_FP64;
    o->factor_prec = IRK_FP64;
    o->restart = 30;
    o->max_iters = 3000;
    o->max_outer = 20;
    o->rtol = 1e-10;
    o->inner_rtol = 1e-4;
    return IRK_OK;
}

irk_status irk_level_schedule(int T, int nnzb, const int32_t *row_ptr, const int32_t *col_idx,
                              int *lvl_fwd, int *off_fwd, int *nlev_fwd, int *lvl_bwd, int *off_bwd,
                              int *nlev_bwd)
{
    if (!lvl_fwd || !off_fwd || !nlev_fwd || !lvl_bwd || !off_bwd || !nlev_bwd) return IRK_ERR_ARG;
    Schedule sc;
    const int st = analyze_pattern(T, nnzb, row_ptr, col_idx, sc);
    if (st != SCHED_OK) return st == SCHED_BAD_PATTERN ? IRK_ERR_ARG : IRK_ERR_INTERNAL;
    std::copy(sc.lvl_fwd.begin(), sc.lvl_fwd.end(), lvl_fwd);
    std::copy(sc.off_fwd.begin(), sc.off_fwd.end(), off_fwd);
    std::copy(sc.lvl_bwd.begin(), sc.lvl_bwd.end(), lvl_bwd);
    std::copy(sc.off_bwd.begin(), sc.off_bwd.end(), off_bwd);
    *nlev_fwd = (int)sc.off_fwd.size() - 1;
    *nlev_bwd = (int)sc.off_bwd.size() - 1;
    return IRK_OK;
}

irk_status irk_workspace_size(const irk_problem *p, const irk_options *o, size_t *bytes)
{
    if (!bytes) return IRK_ERR_ARG;
    irk_status st = check_args(p, o);
    if (st != IRK_OK) return st;
    *bytes = make_plan(p, o).total;
    return IRK_OK;
}

irk_status irk_radau_iia(int s, double *A, double *b, double *c)
{
    if (s < 1 || s > 12 || !A || !b || !c) return IRK_ERR_ARG;
    // abscissae: zeros of Q(x) = P_s(2x-1) - P_{s-1}(2x-1); x = 1 is one.
    // The others by Newton with Maehly deflation started left of all zeros,
    // which converges monotonically to the smallest remaining zero.
    std::vector<double> roots;
    roots.push_back(1.0);
    for (int r = 0; r < s - 1; ++r) {
        double x = -0.05;
        for (int it = 0; it < 200; ++it) {
            double ps, dps, pm, dpm;
            legendre_pd(s, 2 * x - 1, ps, dps);
            legendre_pd(s - 1, 2 * x - 1, pm, dpm);
            const double q = ps - pm, dq = 2.0 * (dps - dpm);
            double sdef = 0.0;
            for (double z : roots) sdef += 1.0 / (x - z);
            const double step = q / (dq - q * sdef);
            x -= step;
            if (std::fabs(step) <= 1e-17 * std::max(1.0, std::fabs(x))) break;
        }
        roots.push_back(x);
    }
    std::sort(roots.begin(), roots.end());
    for (int i = 0; i < s; ++i) c[i] = roots[i];
    // A from the collocation conditions: the quadrature with nodes c on
    // [0, c_i] integrates every polynomial of degree < s exactly.  Written in
    // the shifted Legendre basis phi_q(x) = P_q(2x-1) (better conditioned than
    // monomials):  sum_j a_ij phi_q(c_j) = int_0^{c_i} phi_q, with
    // int_0^c phi_q = (P_{q+1}(2c-1) - P_{q-1}(2c-1)) / (2(2q+1)) for q >= 1.
    auto Pq = [](int q, double t) { double p, dp; legendre_pd(q, t, p, dp); return p; };
    std::vector<double> Vm(s * s);
    for (int q = 0; q < s; ++q)
        for (int j = 0; j < s; ++j) Vm[q * s + j] = Pq(q, 2 * c[j] - 1);
    for (int i = 0; i < s; ++i) {
        std::vector<double> rhs(s);
        const double t = 2 * c[i] - 1;
        rhs[0] = c[i];
        for (int q = 1; q < s; ++q) rhs[q] = (Pq(q + 1, t) - Pq(q - 1, t)) / (2.0 * (2 * q + 1));
        if (!host_solve(s, Vm, rhs)) return IRK_ERR_ARG;
        for (int j = 0; j < s; ++j) A[i * s + j] = rhs[j];
    }
    std::vector<double> rb(s, 0.0);
    rb[0] = 1.0;
    if (!host_solve(s, Vm, rb)) return IRK_ERR_ARG;
    for (int j = 0; j < s; ++j) b[j] = rb[j];
    return IRK_OK;
}

irk_status irk_dirk_tableau(int which, int *stages, double *A, double *b, double *c)
{
    if (!stages || !A || !b || !c) return IRK_ERR_ARG;
    if (which == IRK_DIRK33) {
        // L-stable three-stage SDIRK of order 3: the diagonal is the root of
        // 6 a^3 - 18 a^2 + 9 a - 1 in (1/3, 1/2), in the trigonometric form
        const double th = std::atan(std::sqrt(2.0) / 4.0) / 3.0;
        const double a = 1.0 + std::sqrt(6.0) / 2.0 * std::sin(th) - std::sqrt(2.0) / 2.0 * std::cos(th);
        const double t2 = 0.5 * (1.0 + a);
        const double b1 = -(6.0 * a * a - 16.0 * a + 1.0) / 4.0, b2 = (6.0 * a * a - 20.0 * a + 5.0) / 4.0;
        const double T[9] = {a, 0.0, 0.0, t2 - a, a, 0.0, b1, b2, a};
        *stages = 3;
        std::memcpy(A, T, sizeof(T));
        b[0] = b1; b[1] = b2; b[2] = a;
        c[0] = a; c[1] = t2; c[2] = 1.0;
        return IRK_OK;
    }
    if (which == IRK_ESDIRK65) {
        // six stages, explicit first stage, common implicit diagonal
        static const double T[36] = {
            0.0, 0.0, 0.0, 0.0, 0.0, 0.0,
            0.2780538411364465, 0.2780538411364465, 0.0, 0.0, 0.0, 0.0,
            0.3137405401502951, 0.4363327154020044, 0.2780538411364465, 0.0, 0.0, 0.0,
            0.2741986534107860, -0.0164268277321164, 0.0048197082596452, 0.2780538411364465, 0.0, 0.0,
            -0.2441776975175844, -3.3203529439447852, 0.0477747285706825, 3.2974431145814931,
            0.2780538411364465, 0.0,
            -0.2786732780227907, 1.8929947094010862, -0.1280948204262490, -1.3574693381380240,
            0.5931888860495311, 0.2780538411364465};
        *stages = 6;
        std::memcpy(A, T, sizeof(T));
        for (int i = 0; i < 6; ++i) {
            b[i] = T[30 + i];
            double r = 0.0;
            for (int j = 0; j < 6; ++j) r += T[6 * i + j];
            c[i] = r;
        }
        return IRK_OK;
    }
    return IRK_ERR_ARG;
}

// Work items of a handle (matvec rows, reduction chunks, sweep records per
// level, factor tasks) and the LDS sizes of its launches, from the launch
// shapes in the handle (tpw64/32, sw64/32) and the host copy of the
// pattern.  Used by irk_setup and again by irk_autotune for each candidate.
static irk_status build_items(irk_handle *h)
{
    const Plan &P = h->plan;
    const irk_options *o = &h->opt;
    const int s = h->s, T = h->T, m = h->m;
    const int32_t *rp = h->ints.data(), *ci = h->ints.data() + T + 1;
    // ---- work items ----
    WorkSet &W = h->W;
    W.items.clear();
    W.fwd64.clear(); W.bwd64.clear(); W.fwd32.clear(); W.bwd32.clear();
    W.cf64.clear(); W.cb64.clear(); W.cf32.clear(); W.cb32.clear();
    auto row_items = [&](int tpw, Launch &L) {
        L.off = (int)W.items.size();
        L.n = 0;
        for (int a = 0; a < T; a += tpw) { W.items.push_back(Item{0, a, std::min(tpw, T - a), tpw}); L.n++; }
    };
    row_items(h->tpw64, W.mv64);
    if (h->mixed) row_items(h->tpw32, W.mv32);
    h->nblk = reduction_chunks((long long)s * T * m);
    W.vec.off = (int)W.items.size();
    for (int c = 0; c < h->nblk; ++c) W.items.push_back(Item{0, c, h->nblk, 0});
    W.vec.n = h->nblk;
    W.fin.off = (int)W.items.size();
    W.items.push_back(Item{0, 0, h->nblk, 0});
    W.fin.n = 1;
    if (o->pc != IRK_PC_NONE) {
        const int mr = h->sc.maxrow;
        const SweepShape &a = h->sw64, &b = h->sw32;
        const int pa = sw_region(s, m, mr, P, true, h->ftype, a.tps_pf);
        const int sa = sw_region(s, m, mr, P, true, h->ftype, a.tps_st);
        const int sa2 = st_small_tps(a) ? sw_region(s, m, mr, P, true, h->ftype, st_small_tps(a)) : 0;
        add_level_records(W.items, h->sc, rp, ci, true, a, pa, sa, sa2, W.fwd64);
        add_level_records(W.items, h->sc, rp, ci, false, a, pa, sa, sa2, W.bwd64);
        if (h->mixed) {
            const int pb = sw_region(s, m, mr, P, false, h->ftype, b.tps_pf);
            const int sb = sw_region(s, m, mr, P, false, h->ftype, b.tps_st);
            const int sb2 = st_small_tps(b) ? sw_region(s, m, mr, P, false, h->ftype, st_small_tps(b)) : 0;
            add_level_records(W.items, h->sc, rp, ci, true, b, pb, sb, sb2, W.fwd32);
            add_level_records(W.items, h->sc, rp, ci, false, b, pb, sb, sb2, W.bwd32);
        }
        make_chains(W.items, W.fwd64, sizeof(double), W.cf64);
        make_chains(W.items, W.bwd64, sizeof(double), W.cb64);
        make_chains(W.items, W.fwd32, sizeof(float), W.cf32);
        make_chains(W.items, W.bwd32, sizeof(float), W.cb32);
    }
    // factor tasks, one launch per wavefront (stored after the work set's
    // items).  Uncoupled: wavefront = forward level; with the level's
    // elements listed by lower-neighbour count, most first (the longest
    // tasks start first), workgroup w takes stage k = (w / 8) % s of element
    // 8 (w / (8 s)) + w % 8 of that list, so the s tasks of an element run on
    // one XCD (workgroups go to the XCDs round-robin) and share its L2 for
    // the blocks common to all stages; first = -1 pads the last group of
    // eight.  Coupled: task (k, i) belongs to wavefront level(i) + k (its own
    // earlier stages and the lower neighbours' same stage are done by then).
    h->fa.clear();
    h->fitems.clear();
    if (o->pc != IRK_PC_NONE) {
        const int L = (int)h->sc.off_fwd.size() - 1;
        const int nw = h->coupled ? L + s - 1 : L;
        for (int wf = 0; wf < nw; ++wf) {
            Launch A{(int)(W.items.size() + h->fitems.size()), 0};
            if (h->coupled) {
                // the longest tasks first, so the wavefront does not end on
                // one of them: block products per task = 2 per lower
                // neighbour + the stage round's (k = 0: two and an
                // element-wise pass, counted as three; 0 < k < s - 1: one L
                // product and s - 1 - k updates per later stage)
                std::vector<std::pair<int, Item>> tk;
                for (int k = 0; k < s; ++k) {
                    const int l = wf - k;
                    if (l < 0 || l >= L) continue;
                    const int later = s - 1 - k;
                    const int round = (k == 0 && s > 1) ? 3 : later * (1 + later);
                    for (int a = h->sc.off_fwd[l]; a < h->sc.off_fwd[l + 1]; ++a) {
                        const int e = h->sc.lvl_fwd[a];
                        tk.push_back({2 * (h->sc.diag[e] - rp[e]) + round, Item{0, e, 1, k}});
                    }
                }
                std::stable_sort(tk.begin(), tk.end(),
                                 [](const std::pair<int, Item> &x, const std::pair<int, Item> &y) {
                                     return x.first > y.first;
                                 });
                for (const auto &t : tk) {
                    h->fitems.push_back(t.second);
                    A.n++;
                }
            } else {
                // elements with the most lower neighbours (the longest tasks) first
                std::vector<int> el(h->sc.lvl_fwd.begin() + h->sc.off_fwd[wf],
                                    h->sc.lvl_fwd.begin() + h->sc.off_fwd[wf + 1]);
                std::stable_sort(el.begin(), el.end(), [&](int x, int y) {
                    return h->sc.diag[x] - rp[x] > h->sc.diag[y] - rp[y];
                });
                const int ne = (int)el.size();
                for (int g = 0; g < (ne + 7) / 8; ++g)
                    for (int k = 0; k < s; ++k)
                        for (int r = 0; r < 8; ++r) {
                            const int e = 8 * g + r;
                            h->fitems.push_back(Item{0, e < ne ? el[e] : -1, 1, k});
                            A.n++;
                        }
            }
            h->fa.push_back(A);
        }
    }
    if ((int)(W.items.size() + h->fitems.size()) > P.nitems_max) return IRK_ERR_ARG;
    W.smax = s;
    W.restart = o->restart;
    W.nsys = 1;
    W.mixed = h->mixed; W.coupled = h->coupled; W.sharedJ = h->sharedJ;
    W.has_pc = o->pc != IRK_PC_NONE; W.ftype = h->ftype;

    // ---- LDS sizes ----
    const int maxrow = h->sc.maxrow;
    W.shm_mv64 = lds_matvec(s, m, maxrow, P.ld, 2, h->tpw64, sizeof(double));
    W.shm_mv32 = lds_matvec(s, m, maxrow, P.ld32, 4, h->tpw32, sizeof(float));
    W.shm_sw64 = W.shm_sw32 = 0;
    for (int tps : {h->sw64.tps_pf, h->sw64.tps_st, st_small_tps(h->sw64)})
        if (tps) W.shm_sw64 = std::max(W.shm_sw64, sizeof(double) * tps * (size_t)sw_region(s, m, maxrow, P, true, h->ftype, tps));
    for (int tps : {h->sw32.tps_pf, h->sw32.tps_st, st_small_tps(h->sw32)})
        if (tps) W.shm_sw32 = std::max(W.shm_sw32, sizeof(float) * tps * (size_t)sw_region(s, m, maxrow, P, false, h->ftype, tps));
    // factorization: matrix-core products and register Gauss-Jordan, four
    // waves for m <= 64, eight above
    h->shm_fac = sizeof(double) * (size_t)((m <= 64) ? D64_LDS_DOUBLES : std::max(DM_LDS_DOUBLES, DMI_LDS_DOUBLES));
    const size_t lds_max = 160 * 1024;
    if (h->shm_fac > lds_max || W.shm_mv64 > lds_max || W.shm_sw64 > lds_max ||
        (h->mixed && (W.shm_sw32 > lds_max || W.shm_mv32 > lds_max)))
        return IRK_ERR_ARG;
    return IRK_OK;
}

irk_status irk_setup(const irk_problem *p, const irk_options *o, void *workspace, size_t ws_bytes,
                     hipStream_t stream, irk_handle **out)
{
    if (!out) return IRK_ERR_ARG;
    *out = nullptr;
    irk_status st = check_args(p, o);
    if (st != IRK_OK) return st;
    if (!workspace) return IRK_ERR_ARG;
    irk_handle *h = new (std::nothrow) irk_handle();
    if (!h) return IRK_ERR_ARG;
    h->s = p->s; h->T = p->T; h->m = p->m; h->nnzb = p->nnzb; h->nJ = p->nJ; h->dt = p->dt;
    h->opt = *o;
    h->opt.alpha = nullptr;
    h->stream = stream;
    h->ws = (char *)workspace;
    h->ws_bytes = ws_bytes;
    h->bad_element = -1;
    h->ms_factor = 0.0f;
    h->factored = false;
    const int s = p->s, T = p->T, m = p->m;
    std::memcpy(h->A, p->A, sizeof(double) * s * s);
    double Ainv[SMAX * SMAX];
    if (!host_inverse(s, p->A, Ainv)) { delete h; return IRK_ERR_ARG; }
    std::memcpy(h->Ainv, Ainv, sizeof(Ainv));
    for (int k = 0; k < s; ++k) {
        double a = 0.0;
        if (o->shift_rule == 0)
            for (int j = 0; j < s; ++j) a += (j == k) ? 0.0 : std::fabs(Ainv[j * s + k]);
        else if (o->shift_rule == 2)
            a = o->alpha[k];
        h->alpha[k] = a;
    }
    st = analyze(p, h->sc);
    if (st != IRK_OK) { delete h; return st; }
    h->plan = make_plan(p, o);
    if (ws_bytes < h->plan.total) { delete h; return IRK_ERR_NOMEM; }
    const Plan &P = h->plan;
    h->mixed = is_mixed(o);
    h->coupled = (o->pc == IRK_PC_COUPLED) && s > 1;
    h->sharedJ = (p->nJ == 1);
    h->ftype = factor_type(o);

    h->tpw64 = pick_tpw(P.ld, 2);
    h->tpw32 = pick_tpw(P.ld32, 4);
    {
        const int ldF = (h->ftype == FT_F32) ? P.ld32 : P.ld16;
        const int VF = (h->ftype == FT_F32) ? 4 : 8;
        h->sw64 = pick_sweep(m, P.ld, 2, P.ld, 2, s, h->coupled);
        h->sw32 = pick_sweep(m, P.ld32, 4, ldF, VF, s, h->coupled);
    }
    h->ints.assign((size_t)(T + 1) + 2 * (size_t)p->nnzb + 3 * (size_t)T, 0);
    std::memcpy(h->ints.data(), p->row_ptr, sizeof(int) * (T + 1));
    std::memcpy(h->ints.data() + T + 1, p->col_idx, sizeof(int) * p->nnzb);
    st = build_items(h);
    if (st != IRK_OK) { delete h; return st; }
    WorkSet &W = h->W;
    const int maxrow = h->sc.maxrow;
    // the largest any factor kernel takes, whatever this handle's m: the
    // attribute is per kernel and process-wide, and handles of other block
    // orders (a batched factorization mixes them) launch the same kernels
    factor_set_lds_limit(sizeof(double) * (size_t)std::max(D64_LDS_DOUBLES, std::max(DM_LDS_DOUBLES, DMI_LDS_DOUBLES)));
    // ---- device pointers ----
    char *ws = h->ws;
    SysDesc &d = h->hsys;
    std::memset(&d, 0, sizeof(d));
    d.s = s; d.T = T; d.m = m; d.nJ = p->nJ; d.nnzb = p->nnzb;
    d.ld = P.ld; d.ld32 = P.ld32; d.ld16 = P.ld16;
    d.maxrow = maxrow;
    d.pc = o->pc;
    d.ftype = h->ftype;
    d.restart = o->restart;
    d.max_iters = o->max_iters;
    d.mixed = h->mixed ? 1 : 0;
    d.rtol = o->rtol;
    d.inner_rtol = o->inner_rtol;
    d.N = (long long)s * T * m;
    d.dt = p->dt;
    for (int k = 0; k < s; ++k) {
        for (int l = 0; l < s; ++l) {
            d.Ainv[k * SMAX + l] = Ainv[k * s + l];
            d.A[k * SMAX + l] = p->A[k * s + l];
        }
        d.dcoef[k] = Ainv[k * s + k] + ((o->pc == IRK_PC_UNCOUPLED_SHIFTED) ? h->alpha[k] : 0.0);
    }
    int *ip = (int *)(ws + P.o_ints);
    d.row_ptr = ip;
    d.col_idx = ip + (T + 1);
    d.tpos = ip + (T + 1) + p->nnzb;
    d.diag_pos = ip + (T + 1) + 2 * p->nnzb;
    d.lvl_fwd = d.diag_pos + T;
    d.lvl_bwd = d.lvl_fwd + T;
    d.Jc = (const double *)(ws + P.o_J);
    d.Mc = (const double *)(ws + P.o_M);
    if (h->mixed) { d.Jc32 = (const float *)(ws + P.o_J32); d.Mc32 = (const float *)(ws + P.o_M32); }
    if (o->pc != IRK_PC_NONE) {
        d.P64 = (double *)(ws + P.o_P64);
        d.Fscr = P.o_Fscr ? (double *)(ws + P.o_Fscr) : nullptr;
        if (P.o_C64) d.C64 = (double *)(ws + P.o_C64);
        if (P.o_P32) d.P32 = (float *)(ws + P.o_P32);
        if (P.o_C32) d.C32 = (float *)(ws + P.o_C32);
        if (P.o_P16) { d.P16 = (uint16_t *)(ws + P.o_P16); d.P16e = (int *)(ws + P.o_P16e); }
        if (P.o_C16) { d.C16 = (uint16_t *)(ws + P.o_C16); d.C16e = (int *)(ws + P.o_C16e); }
    }
    for (int sl = 0; sl < NSLOT; ++sl) d.vec[sl] = (P.o_vec[sl] == (size_t)-1) ? nullptr : (void *)(ws + P.o_vec[sl]);
    d.H = (double *)(ws + P.o_H);
    d.g = (double *)(ws + P.o_g);
    d.cs = (double *)(ws + P.o_cs);
    d.sn = (double *)(ws + P.o_sn);
    d.y = (double *)(ws + P.o_y);
    d.hbuf = (double *)(ws + P.o_hbuf);
    d.part = (double *)(ws + P.o_part);
    d.st = (DevState *)(ws + P.o_st);
    h->dsys = (SysDesc *)(ws + P.o_dsys);
    h->dsys_solve = (SysDesc *)(ws + P.o_dsys2);
    h->ditems = (Item *)(ws + P.o_items);
    h->dst = d.st;
    h->dgather = (DevState *)(ws + P.o_gather);
    if (o->pc != IRK_PC_NONE) {
        d.flow = (unsigned long long *)(ws + P.o_flow);
        W.dticket = (unsigned *)(ws + P.o_ticket);
        h->dfflag = (unsigned long long *)(ws + P.o_fflag);
        h->dfticket = (unsigned *)(ws + P.o_fticket);
    }
    W.dsys = h->dsys;
    W.ditems = h->ditems;

    // ---- uploads ----
    // (row_ptr and col_idx are already in h->ints)
    std::memcpy(h->ints.data() + T + 1 + p->nnzb, h->sc.tpos.data(), sizeof(int) * p->nnzb);
    std::memcpy(h->ints.data() + T + 1 + 2 * p->nnzb, h->sc.diag.data(), sizeof(int) * T);
    std::memcpy(h->ints.data() + T + 1 + 2 * p->nnzb + T, h->sc.lvl_fwd.data(), sizeof(int) * T);
    std::memcpy(h->ints.data() + T + 1 + 2 * p->nnzb + 2 * T, h->sc.lvl_bwd.data(), sizeof(int) * T);
    if (hipHostMalloc((void **)&h->hst, sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
        delete h;
        return IRK_ERR_DEVICE;
    }
    std::memset(h->hst, 0, sizeof(DevState));
    {
        // (irk_destroy releases whatever was created before a failure)
        hipEvent_t *timed[] = {&h->ev0, &h->ev1, &h->ev_s0, &h->ev_s1, &h->ev_f0, &h->ev_f1};
        hipEvent_t *plain[] = {&h->ev_ready, &h->ev_done, &h->ev_pre, &h->ev_factored,
                               &h->ev_tail, &h->ev_read, &h->ev_part};
        bool ok = true;
        for (hipEvent_t *e : timed) ok = ok && hipEventCreate(e) == hipSuccess;
        for (hipEvent_t *e : plain) ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            irk_destroy(h);
            return IRK_ERR_DEVICE;
        }
    }
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&h->ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            h->ncu = 0;
    }
    // (non-blocking: no implicit ordering with a legacy default stream)
    if (hipStreamCreateWithFlags(&h->sstream, hipStreamNonBlocking) != hipSuccess) h->sstream = nullptr;
    // the dependency-driven factorization: the uncoupled forms, and the
    // coupled form with m <= 64 (variable IRK_FACTOR_FLOW=0 turns it off)
    {
        const char *e = std::getenv("IRK_FACTOR_FLOW");
        h->factor_flow = (m <= 64 || !h->coupled) && o->pc != IRK_PC_NONE && !(e && std::atoi(e) == 0);
    }
    std::vector<Item> all(W.items);
    all.insert(all.end(), h->fitems.begin(), h->fitems.end());
    bool ok = true;
    ok &= hipMemcpyAsync(ip, h->ints.data(), sizeof(int) * h->ints.size(), hipMemcpyHostToDevice, stream) == hipSuccess;
    ok &= hipMemcpyAsync(h->ditems, all.data(), sizeof(Item) * all.size(), hipMemcpyHostToDevice, stream) == hipSuccess;
    ok &= hipMemcpyAsync(h->dsys, &h->hsys, sizeof(SysDesc), hipMemcpyHostToDevice, stream) == hipSuccess;
    ok &= hipMemcpyAsync(h->dst, h->hst, sizeof(DevState), hipMemcpyHostToDevice, stream) == hipSuccess;
    if (o->pc != IRK_PC_NONE) {
        // sweep flags at epoch 0 (every sweep uses a larger one), ticket counter at 0
        ok &= hipMemsetAsync(d.flow, 0, sizeof(unsigned long long) * (size_t)T, stream) == hipSuccess;
        ok &= hipMemsetAsync(h->dfflag, 0, sizeof(unsigned long long) * (size_t)T * s, stream) == hipSuccess;
        ok &= hipMemsetAsync(h->dfticket, 0, sizeof(unsigned), stream) == hipSuccess;
        ok &= hipMemsetAsync(W.dticket, 0, sizeof(unsigned), stream) == hipSuccess;
    }
    if (!ok) { irk_destroy(h); return IRK_ERR_DEVICE; }
    *out = h;
    st = irk_update_values(h, p->J, p->M, p->dt);
    if (st != IRK_OK) { irk_destroy(h); *out = nullptr; return st; }
    if (hipStreamSynchronize(stream) != hipSuccess) { irk_destroy(h); *out = nullptr; return IRK_ERR_DEVICE; }
    return IRK_OK;
}

irk_status irk_update_values(irk_handle *h, const double *J, const double *M, double dt)
{
    if (!h || !J || !M || !(dt > 0.0) || !std::isfinite(dt)) return IRK_ERR_ARG;
    if (irk_status js = join_factor(h); js != IRK_OK) return js;
    const SysDesc &d = h->hsys;
    const long long nJb = (long long)h->nJ * h->nnzb;
    launch_relayout(J, (void *)d.Jc, 0, nJb, h->m, d.ld, h->stream);
    launch_relayout(M, (void *)d.Mc, 0, h->T, h->m, d.ld, h->stream);
    if (h->mixed) {
        launch_relayout(J, (void *)d.Jc32, 1, nJb, h->m, d.ld32, h->stream);
        launch_relayout(M, (void *)d.Mc32, 1, h->T, h->m, d.ld32, h->stream);
    }
    if (dt != h->dt) {
        h->dt = dt;
        h->hsys.dt = dt;
        HIPCHK(hipMemcpyAsync(h->dsys, &h->hsys, sizeof(SysDesc), hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    h->factored = false;
    h->factor_pending = false;
    if (h->ev_done) HIPCHK(hipEventRecord(h->ev_done, h->stream));
    return hipGetLastError() == hipSuccess ? IRK_OK : IRK_ERR_DEVICE;
}

irk_status irk_factor_ilu(irk_handle *h)
{
    if (!h) return IRK_ERR_ARG;
    if (h->opt.pc == IRK_PC_NONE) { h->factored = true; return IRK_OK; }
    if (irk_status js = join_factor(h); js != IRK_OK) return js;
    h->factor_pending = false;
    h->hst->singular = 0;
    h->hst->nonfinite = 0;
    HIPCHK(hipMemcpyAsync(h->dst, h->hst, sizeof(DevState), hipMemcpyHostToDevice, h->stream));
    hipEventRecord(h->ev_f0, h->stream);
    const int pf = prof_begin(h);
    if (h->factor_flow && !h->fa.empty()) {
        // every wavefront in one dependency-driven launch (k_factor_flow)
        int n = 0;
        for (const Launch &F : h->fa) n += F.n;
        launch_factor_flow(h->dsys, h->ditems, h->fa[0].off, n, h->coupled, h->sharedJ, h->m, h->shm_fac, h->dfflag, h->dfticket,
                           ++g_flow_epoch, h->stream);
    } else {
        for (const Launch &F : h->fa)
            launch_factor(h->dsys, h->ditems + F.off, F.n, h->coupled, h->sharedJ, h->m, h->shm_fac, h->stream);
    }
    if (h->mixed) launch_quantize(h->dsys, h->hsys, h->ftype, h->stream);
    prof_end(h, pf, PK_FACTOR);
    hipEventRecord(h->ev_f1, h->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(h->hst, h->dst, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    hipEventElapsedTime(&h->ms_factor, h->ev_f0, h->ev_f1);
    HIPCHK(hipEventRecord(h->ev_done, h->stream));
    if (h->hst->singular) {
        h->bad_element = h->hst->singular - 1;
        h->factored = false;
        return IRK_ERR_SINGULAR;
    }
    h->bad_element = -1;
    h->factored = true;
    return IRK_OK;
}

irk_status irk_factor_ilu_async(irk_handle *h)
{
    if (!h) return IRK_ERR_ARG;
    if (h->opt.pc == IRK_PC_NONE) { h->factored = true; return IRK_OK; }
    if (irk_status js = join_factor(h); js != IRK_OK) return js;
    // flags cleared by a kernel (the pinned host copy may be in use), in the
    // handle's stream order
    launch_reset_factor_flags(h->dsys, h->ditems + h->W.fin.off, 1, h->stream);
    // the factorization itself on the side stream (unless profiled: the
    // profile's events are on the handle's stream), from this point on
    const bool side = h->sstream && !h->prof;
    hipStream_t fs = side ? h->sstream : h->stream;
    if (side) {
        HIPCHK(hipEventRecord(h->ev_pre, h->stream));
        HIPCHK(hipStreamWaitEvent(fs, h->ev_pre, 0));
    }
    hipEventRecord(h->ev_f0, fs);
    const int pf = prof_begin(h);
    // the forward sweep's first launch group (levels 0 .. a-1) reads only
    // the factors of its own elements, final after wavefront a - 1 (+ s - 1
    // when coupled: task (k, i) is in wavefront level(i) + k)
    int a = 0;
    const std::vector<SwLaunch> &F0 = h->W.fwd64;
    if (!F0.empty()) {
        a = 1;
        if (F0[0].group >= 0)
            while (a < (int)F0.size() && F0[a].group == F0[0].group) ++a;
    }
    const int wpart = (side && !h->mixed && a > 0) ? (h->coupled ? a - 1 + h->s - 1 : a - 1) : -1;
    h->part_levels = 0;
    const int nw = (int)h->fa.size();
    if (h->factor_flow) {
        // runs of consecutive wavefronts in one launch each (k_factor_flow),
        // cut (on the side stream) where the handle's stream goes on and
        // where the first forward launch group's factors are final
        int wtail = -1;
        for (int w = 0; w < nw && wtail < 0 && side; ++w)
            if (h->fa[w].n < h->ncu) wtail = w;
        std::vector<int> cuts{0, nw};
        if (wtail > 0) cuts.push_back(wtail);
        if (wpart >= 0 && wpart + 1 < nw) cuts.push_back(wpart + 1);
        std::sort(cuts.begin(), cuts.end());
        cuts.erase(std::unique(cuts.begin(), cuts.end()), cuts.end());
        const unsigned long long ep = ++g_flow_epoch;
        for (size_t c = 0; c + 1 < cuts.size(); ++c) {
            const int w0 = cuts[c], w1 = cuts[c + 1];
            if (w0 == wtail) {
                HIPCHK(hipEventRecord(h->ev_tail, fs));
                HIPCHK(hipStreamWaitEvent(h->stream, h->ev_tail, 0));
            }
            int n = 0;
            for (int w = w0; w < w1; ++w) n += h->fa[w].n;
            launch_factor_flow(h->dsys, h->ditems, h->fa[w0].off, n, h->coupled, h->sharedJ, h->m, h->shm_fac, h->dfflag,
                               h->dfticket, ep, fs);
            if (w1 == wpart + 1 && w1 < nw) {
                HIPCHK(hipEventRecord(h->ev_part, fs));
                h->part_levels = a;
            }
        }
    } else {
        bool tail = false;
        for (int w = 0; w < nw; ++w) {
            const Launch &F = h->fa[w];
            // the handle's stream goes on (a solve's initial residual) when
            // the first wavefront with fewer tasks than compute units starts:
            // the earlier ones fill the device, the later ones leave most of
            // it idle
            if (side && !tail && F.n < h->ncu) {
                HIPCHK(hipEventRecord(h->ev_tail, fs));
                HIPCHK(hipStreamWaitEvent(h->stream, h->ev_tail, 0));
                tail = true;
            }
            launch_factor(h->dsys, h->ditems + F.off, F.n, h->coupled, h->sharedJ, h->m, h->shm_fac, fs);
            if (w == wpart && w + 1 < nw) {
                HIPCHK(hipEventRecord(h->ev_part, fs));
                h->part_levels = a;
            }
        }
    }
    if (h->mixed) launch_quantize(h->dsys, h->hsys, h->ftype, fs);
    prof_end(h, pf, PK_FACTOR);
    hipEventRecord(h->ev_f1, fs);
    HIPCHK(hipEventRecord(h->ev_done, fs));
    if (side) {
        HIPCHK(hipEventRecord(h->ev_factored, fs));
        h->factor_side = true;
    }
    HIPCHK(hipGetLastError());
    h->bad_element = -1;
    h->factored = true;
    h->factor_pending = true;
    return IRK_OK;
}

int irk_last_bad_element(const irk_handle *h) { return h ? h->bad_element : -1; }

irk_status irk_quantize_blocks(const double *src, long long nblk, int m, irk_prec prec, void *dst,
                               int *exps, hipStream_t stream)
{
    if (!src || !dst || nblk < 0 || m < 1 || m > MMAX) return IRK_ERR_ARG;
    if (prec != IRK_FP32 && prec != IRK_BF16 && prec != IRK_FP16_SCALED) return IRK_ERR_ARG;
    if (prec == IRK_FP16_SCALED && !exps) return IRK_ERR_ARG;
    const int ft = prec == IRK_FP32 ? FT_F32 : (prec == IRK_BF16 ? FT_BF16 : FT_F16S);
    // the element-wise quantizer does not depend on the block's layout: an
    // m x m row-major block is passed as a column-major one with ld = m
    quantize_blocks(src, dst, exps, nblk, m, m, m, ft, stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    return IRK_OK;
}

}  // extern "C"

namespace {
// The flags of an asynchronous factorization, once h->hst holds the state
// copied after it: its time, and a singular pivot (the handle is then not
// factored).
irk_status settle_factor(irk_handle *h)
{
    if (!h->factor_pending) return IRK_OK;
    h->factor_pending = false;
    hipEventElapsedTime(&h->ms_factor, h->ev_f0, h->ev_f1);
    if (h->hst->singular) {
        h->bad_element = h->hst->singular - 1;
        h->factored = false;
        return IRK_ERR_SINGULAR;
    }
    return IRK_OK;
}

// The same for a call that has not read the state: waits for the stream.
irk_status settle_factor_sync(irk_handle *h)
{
    if (irk_status js = join_factor(h); js != IRK_OK) return js;
    if (!h->factor_pending) return IRK_OK;
    HIPCHK(hipMemcpyAsync(h->hst, h->dst, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return settle_factor(h);
}
}  // namespace

extern "C" {

irk_status irk_apply_operator(irk_handle *h, const double *x, double *y)
{
    if (!h || !x || !y) return IRK_ERR_ARG;
    const size_t bytes = sizeof(double) * (size_t)h->hsys.N;
    HIPCHK(hipMemcpyAsync(h->hsys.vec[SL_EXT0], x, bytes, hipMemcpyDeviceToDevice, h->stream));
    Ctx C{&h->W, h->stream, h};
    enqueue_matvec(C, true, SL_EXT0, SL_EXT1, -1, 0, 0);
    HIPCHK(hipMemcpyAsync(y, h->hsys.vec[SL_EXT1], bytes, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return IRK_OK;
}

irk_status irk_apply_preconditioner(irk_handle *h, const double *v, double *z)
{
    if (!h || !v || !z) return IRK_ERR_ARG;
    if (!h->factored) return IRK_ERR_STATE;
    if (irk_status fs = settle_factor_sync(h); fs != IRK_OK) return fs;
    const size_t bytes = sizeof(double) * (size_t)h->hsys.N;
    if (h->opt.pc == IRK_PC_NONE) {
        HIPCHK(hipMemcpyAsync(z, v, bytes, hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        return IRK_OK;
    }
    HIPCHK(hipMemcpyAsync(h->hsys.vec[SL_EXT0], v, bytes, hipMemcpyDeviceToDevice, h->stream));
    Ctx C{&h->W, h->stream, h};
    enqueue_pc(C, true, SL_EXT0, 0, -1, 0);
    HIPCHK(hipMemcpyAsync(z, h->hsys.vec[SL_YH], bytes, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return IRK_OK;
}

irk_status irk_apply_operator_untransformed(irk_handle *h, int form, const double *x, double *y)
{
    if (!h || !x || !y || (form != 0 && form != 1)) return IRK_ERR_ARG;
    const size_t bytes = sizeof(double) * (size_t)h->hsys.N;
    HIPCHK(hipMemcpyAsync(h->hsys.vec[SL_EXT0], x, bytes, hipMemcpyDeviceToDevice, h->stream));
    const int pi = prof_begin(h);
    launch_untransformed(h->dsys, h->W.ditems + h->W.mv64.off, h->W.mv64.n, h->s, form == 1,
                         SL_EXT0, SL_EXT1, h->W.shm_mv64, h->stream);
    prof_end(h, pi, PK_UNTR);
    HIPCHK(hipMemcpyAsync(y, h->hsys.vec[SL_EXT1], bytes, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
    return IRK_OK;
}

irk_status irk_apply_operator_inner(irk_handle *h, const double *x, double *y)
{
    if (!h || !x || !y) return IRK_ERR_ARG;
    if (!h->mixed) return irk_apply_operator(h, x, y);
    const size_t bytes = sizeof(double) * (size_t)h->hsys.N;
    const Item *vec = h->W.ditems + h->W.vec.off;
    HIPCHK(hipMemcpyAsync(h->hsys.vec[SL_EXT0], x, bytes, hipMemcpyDeviceToDevice, h->stream));
    // the FP32 operator reads its input in the compute type from SL_YH
    launch_copy_to_yh(h->dsys, vec, h->W.vec.n, false, SL_EXT0, 0, 0, h->stream);
    Ctx C{&h->W, h->stream, h};
    enqueue_matvec(C, false, SL_YH, SL_EXT1, -1, 0, 0);
    HIPCHK(hipMemcpyAsync(y, h->hsys.vec[SL_EXT1], bytes, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
    return IRK_OK;
}

irk_status irk_apply_preconditioner_inner(irk_handle *h, const double *v, double *z)
{
    if (!h || !v || !z) return IRK_ERR_ARG;
    if (!h->factored) return IRK_ERR_STATE;
    if (irk_status fs = settle_factor_sync(h); fs != IRK_OK) return fs;
    if (!h->mixed || h->opt.pc == IRK_PC_NONE) return irk_apply_preconditioner(h, v, z);
    const size_t bytes = sizeof(double) * (size_t)h->hsys.N;
    const Item *vec = h->W.ditems + h->W.vec.off;
    HIPCHK(hipMemcpyAsync(h->hsys.vec[SL_EXT0], v, bytes, hipMemcpyDeviceToDevice, h->stream));
    Ctx C{&h->W, h->stream, h};
    enqueue_pc(C, false, SL_EXT0, 0, -1, 0);
    // SL_ZB[0] = (double) SL_YH; the copy kernel runs only while the
    // system's cycle flag is clear, so the per-solve state is reset first
    launch_reset_state(h->dsys, h->W.ditems + h->W.fin.off, h->W.fin.n, h->stream);
    launch_store_z(h->dsys, vec, h->W.vec.n, false, 0, h->stream);
    HIPCHK(hipMemcpyAsync(z, h->hsys.vec[SL_ZB], bytes, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
    return IRK_OK;
}

irk_status irk_export_factors(irk_handle *h, double *pinv, double *cross)
{
    if (!h) return IRK_ERR_ARG;
    if (!h->factored || h->opt.pc == IRK_PC_NONE) return IRK_ERR_STATE;
    if (irk_status fs = settle_factor_sync(h); fs != IRK_OK) return fs;
    launch_export(h->dsys, h->hsys, pinv, cross, h->coupled, h->stream);
    HIPCHK(hipStreamSynchronize(h->stream));
    return IRK_OK;
}

irk_status irk_gmres_solve(irk_handle *h, const double *rhs, double *x, irk_solve_info *info)
{
    if (!h || !rhs || !x) return IRK_ERR_ARG;
    if (!h->factored) return IRK_ERR_STATE;
    // the solve's descriptor (caller's rhs and x) is the work set's during
    // the solve; the workspace's own descriptor stays as it is
    h->solve_desc = h->hsys;
    h->solve_desc.vec[SL_B] = const_cast<double *>(rhs);
    h->solve_desc.vec[SL_X] = x;
    hipEventRecord(h->ev0, h->stream);
    HIPCHK(hipMemcpyAsync(h->dsys_solve, &h->solve_desc, sizeof(SysDesc), hipMemcpyHostToDevice, h->stream));
    const SysDesc *const dsys_ws = h->W.dsys;
    h->W.dsys = h->dsys_solve;
    Ctx C{&h->W, h->stream, h, h->ev_read};
    Solve S;
    S.h = h;
    S.x = x;
    std::vector<Solve *> sv{&S};
    // The initial residual needs no factors: after an asynchronous
    // factorization on the side stream it runs beside it, and the Arnoldi
    // steps wait for it.  Its flags are read with the first state read that
    // follows it: the initial one if it ran on this stream, else the end of
    // the first cycle (or a wait at the end).
    const bool side = h->factor_side;
    irk_status st = init_systems(C, sv, h->dgather, h->hst);
    if (st == IRK_OK && h->factor_side && h->part_levels > 0) {
        // the first forward launch group runs once its levels' factors are
        // final (beside the factorization's last wavefronts); the later
        // launches wait for the whole factorization (C.ev_rest)
        HIPCHK(hipStreamWaitEvent(h->stream, h->ev_part, 0));
        C.ev_rest = h->ev_factored;
        C.rest_level = h->part_levels;
        h->factor_side = false;
    } else if (st == IRK_OK) {
        st = join_factor(h);
    }
    bool settled = !h->factor_pending;
    if (st == IRK_OK && !settled && !side) {
        settled = true;
        st = settle_factor(h);
    }
    while (st == IRK_OK && !S.finished) {
        st = run_cycle(C, sv, h->dgather, h->hst);
        if (st == IRK_OK && !settled) {
            settled = true;
            st = settle_factor(h);
        }
    }
    if (C.ev_rest) {
        // (no preconditioner application ran)
        HIPCHK(hipStreamWaitEvent(h->stream, C.ev_rest, 0));
        C.ev_rest = nullptr;
    }
    if (st == IRK_OK && !settled) st = settle_factor_sync(h);
    S.info.ms_factor = h->ms_factor;
    h->W.dsys = dsys_ws;
    hipEventRecord(h->ev1, h->stream);
    HIPCHK(hipStreamSynchronize(h->stream));
    if (st != IRK_OK) return st;
    hipEventElapsedTime(&S.info.ms_solve, h->ev0, h->ev1);
    if (info) *info = S.info;
    return S.status;
}

// ---------------------------------------------------------------------------
// one time step by Newton's method (Sec. 4.1, Eq. modified-IRK)
// ---------------------------------------------------------------------------
namespace {
struct StepPlan { size_t o_dbase, o_ju0, o_w, o_delta, o_part, o_res, o_f, o_hist, o_u, total; };

// Scratch of one step: the linear part's diagonal blocks, J u0, the Newton
// iterate W and update (s vectors for a Radau step, one for a DIRK stage),
// the max-reduction partials; a DIRK step (dirk_stages > 0) adds the stage
// right-hand sides F_j, the history term and the stage state.
StepPlan step_plan(const irk_handle *h, int dirk_stages)
{
    StepPlan P{};
    const size_t n = (size_t)h->T * h->m, N = (size_t)h->s * n;
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o2 = off; off = align256(off + bytes); return o2; };
    P.o_dbase = take(sizeof(double) * (size_t)h->T * h->m * h->plan.ld);
    P.o_ju0 = take(sizeof(double) * n);
    P.o_w = take(sizeof(double) * N);
    P.o_delta = take(sizeof(double) * N);
    P.o_part = take(sizeof(double) * 1024);
    P.o_res = take(sizeof(double));
    P.o_f = P.o_hist = P.o_u = (size_t)-1;
    if (dirk_stages > 0) {
        P.o_f = take(sizeof(double) * n * (size_t)dirk_stages);
        P.o_hist = take(sizeof(double) * n);
        P.o_u = take(sizeof(double) * n);
    }
    P.total = off;
    return P;
}
}  // namespace

irk_status irk_step_workspace_size(const irk_handle *h, size_t *bytes)
{
    if (!h || !bytes) return IRK_ERR_ARG;
    *bytes = step_plan(h, 0).total;
    return IRK_OK;
}

namespace {
// Pointers into a step's scratch (see step_plan).
struct StepBufs { double *Dbase, *Ju0, *W, *delta, *part, *res, *F, *hist, *U; };

StepBufs step_bufs(const StepPlan &P, void *work)
{
    char *wk = (char *)work;
    auto at = [&](size_t o) { return o == (size_t)-1 ? nullptr : (double *)(wk + o); };
    return StepBufs{at(P.o_dbase), at(P.o_ju0), at(P.o_w), at(P.o_delta), at(P.o_part),
                    at(P.o_res), at(P.o_f), at(P.o_hist), at(P.o_u)};
}

bool rhs_ok(const irk_rhs *f)
{
    return f && std::isfinite(f->omega) && std::isfinite(f->eps);
}

// Newton's method on the handle's stage equations (s = h->s stages, stage
// times entering through the forcing factors gam[k]): W (DEVICE, s n) holds
// the initial guess and receives the iterate; hist (DEVICE n or null) is the
// constant history term of a diagonally implicit stage.  Every iteration:
// stage Jacobians from u0 + dt W (nonlinear f), refactor when stale, the
// Newton residual b' - B_N W, GMRES on B_N delta = residual, W += delta,
// ||delta||_inf read back.
irk_status newton_solve(irk_handle *h, const irk_rhs *f, const double *gam, const double *u0,
                        const StepBufs &B, const double *hist, double newton_tol, int max_newton,
                        irk_step_info &inf, bool &converged)
{
    const int s = h->s;
    const long long n = (long long)h->T * h->m, N = (long long)s * n;
    const double dt = h->dt;
    double *bp = (double *)h->hsys.vec[SL_EXT1];   // b', then the Newton residual
    double *Wslot = (double *)h->hsys.vec[SL_EXT0];
    const bool nonlin = f->eps != 0.0;
    converged = false;
    for (int it = 0; it < max_newton; ++it) {
        if (nonlin) {
            launch_stage_jac(h->dsys, h->hsys, B.Dbase, u0, B.W, dt, f->eps, h->stream);
            h->factored = false;
        }
        if (!h->factored) {
            const irk_status st = irk_factor_ilu(h);
            if (st != IRK_OK) return st;
            inf.factorizations++;
        }
        launch_stage_rhs(s, n, B.Ju0, f->g, u0, B.W, dt, f->eps, gam, hist, bp, h->stream);
        HIPCHK(hipMemcpyAsync(Wslot, B.W, sizeof(double) * N, hipMemcpyDeviceToDevice, h->stream));
        {
            Ctx C{&h->W, h->stream, h};
            enqueue_matvec(C, true, SL_EXT0, SL_EXT1, SL_EXT1, 1, 0);
        }
        HIPCHK(hipMemsetAsync(B.delta, 0, sizeof(double) * N, h->stream));
        irk_solve_info si{};
        const irk_status st = irk_gmres_solve(h, bp, B.delta, &si);
        inf.gmres_iters += si.iters;
        if (st != IRK_OK) return st;
        launch_newton_update(N, B.W, B.delta, B.part, B.res, h->stream);
        HIPCHK(hipGetLastError());
        double nrm = 0.0;
        HIPCHK(hipMemcpyAsync(&nrm, B.res, sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        inf.newton_iters++;
        inf.update_norm = nrm;
        if (!std::isfinite(nrm)) return IRK_ERR_NONFINITE;
        if (nrm <= newton_tol) { converged = true; return IRK_OK; }
    }
    return IRK_OK;
}
}  // namespace

irk_status irk_radau_step(irk_handle *h, const irk_rhs *f, const double *b, double t0,
                          const double *u0, double *u1, double newton_tol, int max_newton,
                          void *work, size_t work_bytes, irk_step_info *info)
{
    if (!h || !rhs_ok(f) || !u0 || !u1 || !work) return IRK_ERR_ARG;
    if (!(newton_tol > 0.0) || max_newton < 1 || !std::isfinite(t0)) return IRK_ERR_ARG;
    if (h->mixed) return IRK_ERR_ARG;                       // the FP64 solve only
    if (f->eps != 0.0 && h->nJ != h->s) return IRK_ERR_ARG; // stage Jacobians differ
    const StepPlan SP = step_plan(h, 0);
    if (work_bytes < SP.total) return IRK_ERR_NOMEM;
    if (irk_status js = join_factor(h); js != IRK_OK) return js;
    const StepBufs B = step_bufs(SP, work);
    const int s = h->s;
    const long long n = (long long)h->T * h->m, N = (long long)s * n;
    const double dt = h->dt;
    // stage times c_k = sum_l a_kl, forcing factors, output weights d = b^T A^{-1}
    double gam[SMAX], dco[SMAX];
    for (int k = 0; k < s; ++k) {
        double c = 0.0;
        for (int l = 0; l < s; ++l) c += h->A[k * s + l];
        gam[k] = std::cos(f->omega * (t0 + c * dt));
        dco[k] = 0.0;
    }
    if (b) {
        for (int k = 0; k < s; ++k)
            for (int l = 0; l < s; ++l) dco[k] += b[l] * h->Ainv[l * s + k];
    } else {
        dco[s - 1] = 1.0;     // stiffly accurate: b^T A^{-1} = e_s
    }
    irk_step_info inf{};
    hipEventRecord(h->ev_s0, h->stream);
    // the linear part's diagonal blocks (restored at the end), J u0, W = 0
    launch_save_diag(h->dsys, h->hsys, B.Dbase, h->stream);
    launch_jac_u0(h->dsys, h->hsys, B.Dbase, u0, B.Ju0, h->stream);
    HIPCHK(hipMemsetAsync(B.W, 0, sizeof(double) * N, h->stream));
    HIPCHK(hipGetLastError());
    bool conv = false;
    irk_status st = newton_solve(h, f, gam, u0, B, nullptr, newton_tol, max_newton, inf, conv);
    inf.converged = conv ? 1 : 0;
    inf.equiv_mults = inf.gmres_iters * s;
    if (st == IRK_OK && conv) launch_step_finish(s, n, u0, B.W, dt, dco, u1, h->stream);
    if (f->eps != 0.0) {
        // leave the handle's Jacobians as they were given; its factors are
        // those of the last Newton matrix, so they are stale
        launch_stage_jac(h->dsys, h->hsys, B.Dbase, u0, B.W, dt, 0.0, h->stream);
        h->factored = false;
    }
    hipEventRecord(h->ev_s1, h->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
    hipEventElapsedTime(&inf.ms, h->ev_s0, h->ev_s1);
    if (info) *info = inf;
    if (st != IRK_OK) return st;
    return conv ? IRK_OK : IRK_ERR_NOCONV;
}

irk_status irk_dirk_workspace_size(const irk_handle *h, int stages, size_t *bytes)
{
    if (!h || !bytes || stages < 1 || stages > DIRK_STAGES_MAX) return IRK_ERR_ARG;
    *bytes = step_plan(h, stages).total;
    return IRK_OK;
}

irk_status irk_dirk_step(irk_handle *h, const irk_rhs *f, int stages, const double *A, double t0,
                         const double *u0, double *u1, double newton_tol, int max_newton,
                         void *work, size_t work_bytes, irk_step_info *info)
{
    if (!h || !rhs_ok(f) || !A || !u0 || !u1 || !work) return IRK_ERR_ARG;
    if (stages < 1 || stages > DIRK_STAGES_MAX) return IRK_ERR_ARG;
    if (!(newton_tol > 0.0) || max_newton < 1 || !std::isfinite(t0)) return IRK_ERR_ARG;
    if (h->s != 1 || h->mixed) return IRK_ERR_ARG;
    // a lower-triangular tableau whose implicit diagonal is the handle's a_11;
    // only a first stage with a zero row may be explicit
    const double diag = h->A[0];
    for (int i = 0; i < stages; ++i) {
        for (int j = 0; j < stages; ++j)
            if (!std::isfinite(A[i * stages + j]) || (j > i && A[i * stages + j] != 0.0)) return IRK_ERR_ARG;
        const double aii = A[i * stages + i];
        if (aii == 0.0) {
            if (i != 0) return IRK_ERR_ARG;
            for (int j = 0; j < stages; ++j)
                if (A[j] != 0.0) return IRK_ERR_ARG;
        } else if (aii != diag) {
            return IRK_ERR_ARG;
        }
    }
    const StepPlan SP = step_plan(h, stages);
    if (work_bytes < SP.total) return IRK_ERR_NOMEM;
    if (irk_status js = join_factor(h); js != IRK_OK) return js;
    const StepBufs B = step_bufs(SP, work);
    const long long n = (long long)h->T * h->m;
    const double dt = h->dt;
    irk_step_info inf{};
    hipEventRecord(h->ev_s0, h->stream);
    launch_save_diag(h->dsys, h->hsys, B.Dbase, h->stream);
    launch_jac_u0(h->dsys, h->hsys, B.Dbase, u0, B.Ju0, h->stream);
    HIPCHK(hipGetLastError());
    irk_status st = IRK_OK;
    bool all_conv = true;
    for (int i = 0; i < stages && st == IRK_OK && all_conv; ++i) {
        double ci = 0.0;
        for (int j = 0; j < stages; ++j) ci += A[i * stages + j];
        const double gam = std::cos(f->omega * (t0 + ci * dt));
        const double aii = A[i * stages + i];
        double *Fi = B.F + (long long)i * n;
        if (aii == 0.0) {
            // explicit first stage: U_1 = u0, F_1 = f(t0, u0)
            launch_rhs_eval(n, B.Ju0, u0, f->g, gam, f->eps, Fi, h->stream);
            continue;
        }
        // history term h_i = (1/a_ii) sum_{j<i} a_ij F_j; Newton from W = 0
        if (i > 0) {
            double coef[DIRK_STAGES_MAX];
            for (int j = 0; j < i; ++j) coef[j] = A[i * stages + j] / aii;
            launch_combine(i, n, coef, B.F, B.hist, h->stream);
        }
        HIPCHK(hipMemsetAsync(B.W, 0, sizeof(double) * n, h->stream));
        bool conv = false;
        st = newton_solve(h, f, &gam, u0, B, i > 0 ? B.hist : nullptr, newton_tol, max_newton, inf, conv);
        all_conv = all_conv && conv;
        if (st != IRK_OK || !conv) break;
        // F_i = f(t_i, U_i) with U_i = u0 + dt W (the linear part's Jacobian)
        launch_stage_state(n, u0, B.W, dt, B.U, h->stream);
        launch_jac_u0(h->dsys, h->hsys, B.Dbase, B.U, B.hist, h->stream);
        launch_rhs_eval(n, B.hist, B.U, f->g, gam, f->eps, Fi, h->stream);
    }
    inf.converged = (st == IRK_OK && all_conv) ? 1 : 0;
    inf.equiv_mults = inf.gmres_iters;          // each Arnoldi step is one n x n product
    // stiffly accurate: u1 = U_s (the last stage is implicit here unless s = 1
    // and explicit, which the checks above exclude for a one-stage tableau
    // only through a zero diagonal: then u1 = u0)
    if (inf.converged) {
        if (A[(stages - 1) * stages + stages - 1] == 0.0)
            HIPCHK(hipMemcpyAsync(u1, u0, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
        else
            launch_stage_state(n, u0, B.W, dt, u1, h->stream);
    }
    if (f->eps != 0.0) {
        launch_stage_jac(h->dsys, h->hsys, B.Dbase, u0, B.W, dt, 0.0, h->stream);
        h->factored = false;
    }
    hipEventRecord(h->ev_s1, h->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
    hipEventElapsedTime(&inf.ms, h->ev_s0, h->ev_s1);
    if (info) *info = inf;
    if (st != IRK_OK) return st;
    return inf.converged ? IRK_OK : IRK_ERR_NOCONV;
}

irk_status irk_profile_enable(irk_handle *h, int on)
{
    if (!h) return IRK_ERR_ARG;
    if (on && h->pool.empty()) {
        h->pool.resize(8192);
        for (auto &e : h->pool)
            if (hipEventCreate(&e) != hipSuccess) return IRK_ERR_DEVICE;
    }
    h->prof = on != 0;
    h->spans.clear();
    h->dropped = 0;
    return IRK_OK;
}

irk_status irk_profile_read(irk_handle *h, irk_profile_stats *out)
{
    if (!h || !out) return IRK_ERR_ARG;
    std::memset(out, 0, sizeof(*out));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (const auto &sp : h->spans) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, h->pool[sp.second], h->pool[sp.second + 1]) != hipSuccess) continue;
        switch (sp.first) {
        case PK_MV64: out->matvec_count++; out->matvec_ms += ms; break;
        case PK_MV32: out->matvec32_count++; out->matvec32_ms += ms; break;
        case PK_PC: out->pc_count++; out->pc_ms += ms; break;
        case PK_ORTH: out->orth_count++; out->orth_ms += ms; break;
        case PK_UNTR: out->untr_count++; out->untr_ms += ms; break;
        default: out->factor_count++; out->factor_ms += ms; break;
        }
    }
    out->dropped = h->dropped;
    h->spans.clear();
    h->dropped = 0;
    return IRK_OK;
}

irk_status irk_destroy(irk_handle *h)
{
    if (!h) return IRK_ERR_ARG;
    for (auto &e : h->pool) hipEventDestroy(e);
    if (h->hst) hipHostFree(h->hst);
    if (h->ev0) hipEventDestroy(h->ev0);
    if (h->ev1) hipEventDestroy(h->ev1);
    if (h->ev_ready) hipEventDestroy(h->ev_ready);
    if (h->ev_done) hipEventDestroy(h->ev_done);
    if (h->ev_s0) hipEventDestroy(h->ev_s0);
    if (h->ev_s1) hipEventDestroy(h->ev_s1);
    if (h->ev_f0) hipEventDestroy(h->ev_f0);
    if (h->ev_f1) hipEventDestroy(h->ev_f1);
    if (h->sstream) hipStreamSynchronize(h->sstream);
    if (h->ev_pre) hipEventDestroy(h->ev_pre);
    if (h->ev_factored) hipEventDestroy(h->ev_factored);
    if (h->ev_tail) hipEventDestroy(h->ev_tail);
    if (h->ev_read) hipEventDestroy(h->ev_read);
    if (h->ev_part) hipEventDestroy(h->ev_part);
    if (h->sstream) hipStreamDestroy(h->sstream);
    delete h;
    return IRK_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
static constexpr size_t batch_items_bound(int capacity, long long max_elements)
{
    return (size_t)(32 * max_elements) + (size_t)capacity * (2 * RED_BLOCKS + 8);
}

static constexpr size_t batch_ws_bytes(int capacity, long long max_elements)
{
    size_t off = 0;
    off = align256(off + sizeof(SysDesc) * (size_t)capacity);
    off = align256(off + sizeof(DevState) * (size_t)capacity);
    off = align256(off + sizeof(Item) * batch_items_bound(capacity, max_elements));
    off = align256(off + sizeof(unsigned));   // ticket counter of the single-launch sweeps
    return off;
}

irk_status irk_batch_workspace_size(int capacity, long long max_elements, size_t *bytes)
{
    if (!bytes || capacity < 1 || max_elements < 1) return IRK_ERR_ARG;
    *bytes = batch_ws_bytes(capacity, max_elements);
    return IRK_OK;
}

}  // extern "C"

// Lay out a batch over `workspace` (device table, gathered states, merged
// items) and create its events; hgather is the host array the states are
// read into.
static irk_status batch_init(irk_batch *b, int capacity, long long max_elements, void *workspace,
                             size_t ws_bytes, hipStream_t stream, DevState *hgather, bool own_host)
{
    b->capacity = capacity;
    b->max_elements = max_elements;
    b->stream = stream;
    b->ws = (char *)workspace;
    b->ws_bytes = ws_bytes;
    size_t off = 0;
    b->dtab = (SysDesc *)(b->ws + off);
    off = align256(off + sizeof(SysDesc) * (size_t)capacity);
    b->dgather = (DevState *)(b->ws + off);
    off = align256(off + sizeof(DevState) * (size_t)capacity);
    b->ditems = (Item *)(b->ws + off);
    off = align256(off + sizeof(Item) * batch_items_bound(capacity, max_elements));
    b->dticket = (unsigned *)(b->ws + off);
    HIPCHK(hipMemsetAsync(b->dticket, 0, sizeof(unsigned), stream));
    b->max_items = batch_items_bound(capacity, max_elements);
    b->htab.assign(capacity, SysDesc());
    b->hgather = hgather;
    b->own_host = own_host;
    b->free_slots.clear();
    for (int q = capacity - 1; q >= 0; --q) b->free_slots.push_back(q);
    b->slot_ev.assign(capacity, nullptr);
    for (auto &e : b->slot_ev) HIPCHK(hipEventCreate(&e));
    HIPCHK(hipEventCreate(&b->ev_end));
    HIPCHK(hipEventCreate(&b->ev_f0));
    HIPCHK(hipEventCreate(&b->ev_f1));
    HIPCHK(hipEventCreateWithFlags(&b->ev_read, hipEventDisableTiming));
    return IRK_OK;
}

extern "C" {

irk_status irk_batch_create(int capacity, long long max_elements, void *workspace, size_t ws_bytes,
                            hipStream_t stream, irk_batch **out)
{
    if (!out || !workspace || capacity < 1 || max_elements < 1) return IRK_ERR_ARG;
    *out = nullptr;
    if (ws_bytes < batch_ws_bytes(capacity, max_elements)) return IRK_ERR_NOMEM;
    irk_batch *b = new (std::nothrow) irk_batch();
    if (!b) return IRK_ERR_ARG;
    DevState *hg = nullptr;
    if (hipHostMalloc((void **)&hg, sizeof(DevState) * capacity, hipHostMallocDefault) != hipSuccess) {
        delete b;
        return IRK_ERR_DEVICE;
    }
    const irk_status st = batch_init(b, capacity, max_elements, workspace, ws_bytes, stream, hg, true);
    if (st != IRK_OK) {
        irk_batch_destroy(b);
        return st;
    }
    *out = b;
    return IRK_OK;
}

irk_status irk_batch_admit(irk_batch *b, irk_handle *h, const double *rhs, double *x, long long tag)
{
    if (!b || !h || !rhs || !x) return IRK_ERR_ARG;
    if (!h->factored) return IRK_ERR_STATE;
    if (irk_status fs = settle_factor_sync(h); fs != IRK_OK) return fs;
    if (b->free_slots.empty()) return IRK_ERR_NOMEM;
    long long elems = h->T;
    for (auto &m : b->members) elems += m.h->T;
    if (elems > b->max_elements) return IRK_ERR_NOMEM;
    for (auto &m : b->members)
        if (m.h == h) return IRK_ERR_ARG;   // a handle can be in a batch once
    if (!b->members.empty()) {
        const irk_handle *h0 = b->members[0].h;
        if (h0->mixed != h->mixed || h0->coupled != h->coupled || h0->sharedJ != h->sharedJ ||
            h0->ftype != h->ftype || (h0->opt.pc == IRK_PC_NONE) != (h->opt.pc == IRK_PC_NONE))
            return IRK_ERR_ARG;
    }
    irk_batch::Member m{};
    m.h = h;
    m.slot = b->free_slots.back();
    b->free_slots.pop_back();
    m.tag = tag;
    m.x = x;
    m.phase = 0;
    // table entry: the handle's descriptor with rhs and x in place of its own slots
    SysDesc d = h->hsys;
    d.vec[SL_B] = const_cast<double *>(rhs);
    d.vec[SL_X] = x;
    b->htab[m.slot] = d;
    // the batch stream waits for the handle's own last set-up, value update
    // or factorization only, not for later work on the handle's stream (a
    // server prepares other systems there meanwhile)
    if (h->ev_done) HIPCHK(hipStreamWaitEvent(b->stream, h->ev_done, 0));
    m.t0 = b->slot_ev[m.slot];
    HIPCHK(hipEventRecord(m.t0, b->stream));
    b->members.push_back(m);
    return IRK_OK;
}

int irk_batch_pending(const irk_batch *b) { return b ? (int)b->members.size() : 0; }

// Merged work set of the given members (phase filter), items uploaded.
static irk_status batch_workset(irk_batch *b, int phase, WorkSet &W, std::vector<int> &idx)
{
    std::vector<std::pair<irk_handle *, int>> mem;
    idx.clear();
    for (size_t q = 0; q < b->members.size(); ++q)
        if (b->members[q].phase == phase) {
            mem.push_back({b->members[q].h, b->members[q].slot});
            idx.push_back((int)q);
        }
    build_merged(W, mem);
    if (W.items.size() > b->max_items) return IRK_ERR_NOMEM;
    if (W.shm_sw64 > 160 * 1024 || W.shm_sw32 > 160 * 1024) return IRK_ERR_ARG;
    W.dsys = b->dtab;
    W.ditems = b->ditems;
    W.dticket = b->dticket;
    if (!W.items.empty())
        HIPCHK(hipMemcpyAsync(b->ditems, W.items.data(), sizeof(Item) * W.items.size(),
                              hipMemcpyHostToDevice, b->stream));
    return IRK_OK;
}

static void batch_retire_finished(irk_batch *b, std::vector<Solve> &sol, const std::vector<int> &idx)
{
    for (size_t q = 0; q < idx.size(); ++q) {
        irk_batch::Member &m = b->members[idx[q]];
        const Solve &S = sol[q];
        m.bn = S.bn; m.rel = S.rel; m.est = S.est; m.cycles = S.cycles; m.stall = S.stall;
        m.info = S.info;
        if (S.finished) {
            m.phase = 2;
            m.status = S.status;
        } else {
            m.phase = 1;
        }
    }
    std::vector<irk_batch::Member> keep;
    for (auto &m : b->members) {
        if (m.phase == 2) {
            hipEventRecord(b->ev_end, b->stream);
            hipEventSynchronize(b->ev_end);
            float ms = 0.0f;
            hipEventElapsedTime(&ms, m.t0, b->ev_end);
            m.info.ms_solve = ms;
            b->free_slots.push_back(m.slot);
            b->retired.push_back(m);
        } else {
            keep.push_back(m);
        }
    }
    b->members.swap(keep);
}

irk_status irk_batch_advance(irk_batch *b, int cycles)
{
    if (!b || cycles < 1) return IRK_ERR_ARG;
    if (b->members.empty()) return IRK_OK;
    HIPCHK(hipMemcpyAsync(b->dtab, b->htab.data(), sizeof(SysDesc) * b->capacity,
                          hipMemcpyHostToDevice, b->stream));
    WorkSet W;
    std::vector<int> idx;
    // newly admitted members: initial residual and first cycle start
    irk_status st = batch_workset(b, 0, W, idx);
    if (st != IRK_OK) return st;
    if (!idx.empty()) {
        std::vector<Solve> sol(idx.size());
        std::vector<Solve *> sv;
        for (size_t q = 0; q < idx.size(); ++q) {
            sol[q].h = b->members[idx[q]].h;
            sol[q].x = b->members[idx[q]].x;
            sv.push_back(&sol[q]);
        }
        Ctx C{&W, b->stream, nullptr};
        st = init_systems(C, sv, b->dgather, b->hgather);
        if (st != IRK_OK) return st;
        batch_retire_finished(b, sol, idx);
    }
    for (int c = 0; c < cycles; ++c) {
        st = batch_workset(b, 1, W, idx);
        if (st != IRK_OK) return st;
        if (idx.empty()) break;
        std::vector<Solve> sol(idx.size());
        std::vector<Solve *> sv;
        for (size_t q = 0; q < idx.size(); ++q) {
            const irk_batch::Member &m = b->members[idx[q]];
            sol[q].h = m.h; sol[q].x = m.x; sol[q].bn = m.bn; sol[q].rel = m.rel; sol[q].est = m.est;
            sol[q].cycles = m.cycles; sol[q].stall = m.stall;
            sv.push_back(&sol[q]);
        }
        Ctx C{&W, b->stream, nullptr, b->ev_read};
        st = run_cycle(C, sv, b->dgather, b->hgather);
        if (st != IRK_OK) return st;
        batch_retire_finished(b, sol, idx);
    }
    return IRK_OK;
}

irk_status irk_batch_retire(irk_batch *b, long long *tags, irk_status *status, irk_solve_info *info,
                            int cap, int *count)
{
    if (!b || !count || cap < 0) return IRK_ERR_ARG;
    const int n = std::min<int>(cap, (int)b->retired.size());
    for (int q = 0; q < n; ++q) {
        if (tags) tags[q] = b->retired[q].tag;
        if (status) status[q] = b->retired[q].status;
        if (info) info[q] = b->retired[q].info;
    }
    b->retired.erase(b->retired.begin(), b->retired.begin() + n);
    *count = n;
    return IRK_OK;
}

}  // extern "C"

namespace {

// One group of handles for irk_factor_batched: the batch's table holds their
// descriptors; the items are one per handle (flags), then, wavefront by
// wavefront and for each launch class (coupled, shared J, factor class of
// m), the wavefront's factor tasks of every handle of that class.  Each
// uncoupled handle's tasks come in whole groups of eight, so every task
// keeps its XCD.
irk_status factor_group(irk_batch *b, const std::vector<irk_handle *> &hs, irk_status *status)
{
    const int n = (int)hs.size();
    for (irk_handle *h : hs) {
        if (irk_status js = join_factor(h); js != IRK_OK) return js;
        if (h->stream != b->stream) {
            HIPCHK(hipEventRecord(h->ev_ready, h->stream));
            HIPCHK(hipStreamWaitEvent(b->stream, h->ev_ready, 0));
        }
    }
    for (int q = 0; q < n; ++q) b->htab[q] = hs[q]->hsys;
    struct FL { int off, n; bool coupled, sharedJ; int m; size_t shm; };
    std::vector<Item> items;
    std::vector<FL> launches;
    for (int q = 0; q < n; ++q) items.push_back(Item{q, 0, 1, 0});
    size_t waves = 0;
    for (irk_handle *h : hs) waves = std::max(waves, h->fa.size());
    std::vector<char> taken(n);
    // wavefront l of every handle, one launch per kernel class
    for (size_t l = 0; l < waves; ++l) {
        std::fill(taken.begin(), taken.end(), 0);
        for (int q = 0; q < n; ++q) {
            const irk_handle *h = hs[q];
            if (taken[q] || l >= h->fa.size()) continue;
            FL F{(int)items.size(), 0, h->coupled, h->sharedJ, h->m, h->shm_fac};
            for (int r = q; r < n; ++r) {
                const irk_handle *g = hs[r];
                if (taken[r] || l >= g->fa.size() || g->coupled != h->coupled ||
                    g->sharedJ != h->sharedJ || factor_class(g->m) != factor_class(h->m))
                    continue;
                taken[r] = 1;
                const Launch &L = g->fa[l];
                const size_t base = (size_t)L.off - g->W.items.size();
                for (int t = 0; t < L.n; ++t) {
                    Item it = g->fitems[base + t];
                    it.sys = r;
                    items.push_back(it);
                }
                F.n += L.n;
                F.shm = std::max(F.shm, g->shm_fac);
            }
            if (F.n) launches.push_back(F);
        }
    }
    // quantization of the mixed members' factors: one launch per factor
    // type, chunks of 16 blocks
    int q_off[4] = {0, 0, 0, 0}, q_n[4] = {0, 0, 0, 0};
    for (int ft = FT_F32; ft <= FT_F16S; ++ft) {
        q_off[ft] = (int)items.size();
        for (int q = 0; q < n; ++q) {
            const irk_handle *h = hs[q];
            if (!h->mixed || h->opt.pc == IRK_PC_NONE || h->ftype != ft) continue;
            const long long np = (long long)h->T * h->s;
            const long long nc = h->coupled ? (long long)h->T * (h->s - 1) * (h->s - 2) : 0;
            for (int kind = 0; kind < 2; ++kind)
                for (long long b0 = 0; b0 < (kind ? nc : np); b0 += 16)
                    items.push_back(Item{q, (int)b0, (int)std::min<long long>(16, (kind ? nc : np) - b0), kind});
        }
        q_n[ft] = (int)items.size() - q_off[ft];
    }
    if (items.size() > b->max_items) return IRK_ERR_NOMEM;
    HIPCHK(hipMemcpyAsync(b->dtab, b->htab.data(), sizeof(SysDesc) * n, hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipMemcpyAsync(b->ditems, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice,
                          b->stream));
    launch_reset_factor_flags(b->dtab, b->ditems, n, b->stream);
    HIPCHK(hipEventRecord(b->ev_f0, b->stream));
    for (const FL &F : launches)
        launch_factor(b->dtab, b->ditems + F.off, F.n, F.coupled, F.sharedJ, F.m, F.shm, b->stream);
    for (int ft = FT_F32; ft <= FT_F16S; ++ft)
        if (q_n[ft] > 0) launch_quantize_sys(b->dtab, b->ditems + q_off[ft], q_n[ft], ft, b->stream);
    HIPCHK(hipEventRecord(b->ev_f1, b->stream));
    for (irk_handle *h : hs) HIPCHK(hipEventRecord(h->ev_done, b->stream));
    HIPCHK(hipGetLastError());
    launch_gather_state(b->dtab, b->ditems, n, b->dgather, b->stream);
    HIPCHK(hipMemcpyAsync(b->hgather, b->dgather, sizeof(DevState) * n, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    float ms = 0.0f;
    hipEventElapsedTime(&ms, b->ev_f0, b->ev_f1);
    irk_status worst = IRK_OK;
    for (int q = 0; q < n; ++q) {
        irk_handle *h = hs[q];
        *h->hst = b->hgather[q];
        h->ms_factor = ms;             // the whole group's time
        h->factor_pending = false;
        irk_status st = IRK_OK;
        if (h->opt.pc != IRK_PC_NONE && h->hst->singular) {
            h->bad_element = h->hst->singular - 1;
            h->factored = false;
            st = worst = IRK_ERR_SINGULAR;
        } else {
            h->bad_element = -1;
            h->factored = true;
        }
        if (status) status[q] = st;
    }
    return worst;
}

}  // namespace

extern "C" {

irk_status irk_factor_batched(irk_batch *b, irk_handle *const *h, int count, irk_status *status)
{
    if (!b || count < 0 || (count > 0 && !h)) return IRK_ERR_ARG;
    if (!b->members.empty()) return IRK_ERR_STATE;
    for (int q = 0; q < count; ++q) {
        if (!h[q]) return IRK_ERR_ARG;
        for (int r = 0; r < q; ++r)
            if (h[r] == h[q]) return IRK_ERR_ARG;
    }
    irk_status worst = IRK_OK;
    for (int q0 = 0; q0 < count;) {
        std::vector<irk_handle *> grp;
        size_t nit = 0;
        int q1 = q0;
        while (q1 < count && (int)grp.size() < b->capacity) {
            const size_t need = h[q1]->fitems.size() + 1;
            if (need > b->max_items) return IRK_ERR_NOMEM;
            if (nit + need > b->max_items) break;
            grp.push_back(h[q1]);
            nit += need;
            ++q1;
        }
        const irk_status st = factor_group(b, grp, status ? status + q0 : nullptr);
        if (st != IRK_OK && st != IRK_ERR_SINGULAR) return st;
        if (st != IRK_OK) worst = st;
        q0 = q1;
    }
    return worst;
}

irk_status irk_solve_batched(irk_batch *b, irk_handle *const *h, const double *const *rhs,
                             double *const *x, int count, irk_solve_info *info)
{
    if (!b || !h || !rhs || !x || count < 0) return IRK_ERR_ARG;
    if (!b->members.empty() || !b->retired.empty()) return IRK_ERR_STATE;
    for (int q = 0; q < count; ++q) {
        irk_status st = irk_batch_admit(b, h[q], rhs[q], x[q], q);
        if (st != IRK_OK) return st;
    }
    while (!b->members.empty()) {
        irk_status st = irk_batch_advance(b, 1000000);
        if (st != IRK_OK) return st;
    }
    HIPCHK(hipStreamSynchronize(b->stream));
    irk_status worst = IRK_OK;
    for (auto &m : b->retired) {
        if (info && m.tag >= 0 && m.tag < count) info[m.tag] = m.info;
        if (m.status != IRK_OK && worst == IRK_OK) worst = m.status;
    }
    b->retired.clear();
    return worst;
}

// ---------------------------------------------------------------------------
// batched solve without device allocation: the batch's device table,
// gathered states and merged work items live in a library-owned array
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {
constexpr int NA_CAPACITY = 64;                 // members per call
constexpr long long NA_ELEMENTS = 1LL << 15;    // elements of all members together
constexpr size_t NA_BYTES = batch_ws_bytes(NA_CAPACITY, NA_ELEMENTS);
constexpr int NA_MAX_DEVICES = 64;

// One batch per device over that device's copy of `scratch`; created at the
// first call on the device and kept until the process ends.
struct NoAllocCtx {
    std::mutex mu;
    bool ready = false;
    irk_batch b;
    DevState hgather[NA_CAPACITY];
};
NoAllocCtx g_noalloc[NA_MAX_DEVICES];
}  // namespace

// Device memory of irk_solve_batched_noalloc (each GPU holds its own copy).
// Host code reaches it only through the address hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

extern "C" irk_status irk_solve_batched_noalloc(irk_handle *const *h, const double *const *rhs,
                                                double *const *x, int count, hipStream_t stream,
                                                irk_solve_info *info)
{
    if (!h || !rhs || !x || count < 0) return IRK_ERR_ARG;
    if (count > NA_CAPACITY) return IRK_ERR_ARG;
    long long elems = 0;
    for (int q = 0; q < count; ++q) {
        if (!h[q]) return IRK_ERR_ARG;
        elems += h[q]->T;
    }
    if (elems > NA_ELEMENTS) return IRK_ERR_ARG;
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NA_MAX_DEVICES) return IRK_ERR_ARG;
    NoAllocCtx &c = g_noalloc[dev];
    std::lock_guard<std::mutex> lk(c.mu);
    if (!c.ready) {
        // once per device, with that device current
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return IRK_ERR_DEVICE;
        const irk_status st = batch_init(&c.b, NA_CAPACITY, NA_ELEMENTS, ptr, NA_BYTES, stream, c.hgather,
                                         false);
        if (st != IRK_OK) return st;
        c.ready = true;
    }
    // a call that failed part-way may have left members behind: every call
    // starts from an empty batch (the array's contents are rewritten before
    // any kernel reads them)
    c.b.members.clear();
    c.b.retired.clear();
    c.b.free_slots.clear();
    for (int q = NA_CAPACITY - 1; q >= 0; --q) c.b.free_slots.push_back(q);
    c.b.stream = stream;
    return irk_solve_batched(&c.b, h, rhs, x, count, info);
}

extern "C" {

irk_status irk_batch_destroy(irk_batch *b)
{
    if (!b) return IRK_ERR_ARG;
    for (auto &e : b->slot_ev)
        if (e) hipEventDestroy(e);
    if (b->hgather && b->own_host) hipHostFree(b->hgather);
    if (b->ev_end) hipEventDestroy(b->ev_end);
    if (b->ev_f0) hipEventDestroy(b->ev_f0);
    if (b->ev_f1) hipEventDestroy(b->ev_f1);
    if (b->ev_read) hipEventDestroy(b->ev_read);
    delete b;
    return IRK_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// autotuning of the launch shapes
// ---------------------------------------------------------------------------
namespace {

// Items to the device (work set + factor tasks); synchronous, so the host
// vector may go out of scope.
irk_status upload_items(irk_handle *h)
{
    std::vector<Item> all(h->W.items);
    all.insert(all.end(), h->fitems.begin(), h->fitems.end());
    HIPCHK(hipMemcpyAsync(h->ditems, all.data(), sizeof(Item) * all.size(), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return IRK_OK;
}

struct TuneVal {
    int tpw64, tpw32;
    SweepShape sw64, sw32;
    float matvec_us, sweep_us;
};

std::mutex g_tune_mu;
std::map<std::vector<long long>, TuneVal> g_tune;   // process-wide: one timing per problem class

std::vector<long long> tune_key(const irk_handle *h)
{
    int lg = 0;
    while ((1LL << lg) < h->T) ++lg;
    return {h->m, h->s, h->coupled, h->mixed, h->ftype, h->sharedJ, h->sc.maxrow, (long long)h->opt.pc, lg};
}

// Average time of reps calls of f on the handle's stream (after one warm-up).
template <typename F>
float time_us(irk_handle *h, F f, int reps)
{
    f();
    hipEventRecord(h->ev0, h->stream);
    for (int r = 0; r < reps; ++r) f();
    hipEventRecord(h->ev1, h->stream);
    float ms = 0.0f;
    // (a failed candidate never wins)
    if (hipEventSynchronize(h->ev1) != hipSuccess || hipEventElapsedTime(&ms, h->ev0, h->ev1) != hipSuccess)
        return 1e30f;
    return ms * 1e3f / reps;
}

}  // namespace

extern "C" irk_status irk_autotune(irk_handle *h, int retime, irk_tune_info *info)
{
    if (!h) return IRK_ERR_ARG;
    if (h->opt.pc != IRK_PC_NONE && !h->factored) return IRK_ERR_STATE;
    if (irk_status fs = settle_factor_sync(h); fs != IRK_OK) return fs;
    const std::vector<long long> key = tune_key(h);
    TuneVal best{h->tpw64, h->tpw32, h->sw64, h->sw32, 0.0f, 0.0f};
    bool cached = false;
    if (!retime) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) { best = it->second; cached = true; }
    }
    if (!cached) {
        HIPCHK(hipStreamSynchronize(h->stream));
        Ctx C{&h->W, h->stream, nullptr};
        const bool fp64 = !h->mixed;        // the precision of the inner iteration
        const Plan &P = h->plan;
        // matvec: block rows per workgroup
        {
            const int ld = fp64 ? P.ld : P.ld32, V = fp64 ? 2 : 4;
            int &tpw = fp64 ? h->tpw64 : h->tpw32;
            float tbest = 0.0f;
            int cbest = tpw;
            for (int cand = 1; cand <= 8; cand *= 2) {
                if (NTHREADS / cand < ld / V) break;
                tpw = cand;
                if (build_items(h) != IRK_OK) continue;
                irk_status st = upload_items(h);
                if (st != IRK_OK) return st;
                const float t = time_us(h, [&] { enqueue_matvec(C, fp64, SL_YH, SL_W, -1, 0, 0); }, 3);
                if (tbest == 0.0f || t < tbest) { tbest = t; cbest = cand; }
            }
            tpw = cbest;
            best.matvec_us = tbest;
            best.tpw64 = h->tpw64;
            best.tpw32 = h->tpw32;
        }
        // sweeps: streaming-form threshold and elements per streaming workgroup
        if (h->opt.pc != IRK_PC_NONE) {
            SweepShape &sh = fp64 ? h->sw64 : h->sw32;
            const SweepShape base = sh;
            const int ldF = fp64 ? P.ld : ((h->ftype == FT_F32) ? P.ld32 : P.ld16);
            const int VF = fp64 ? 2 : ((h->ftype == FT_F32) ? 4 : 8);
            const int R = std::max(ldF / VF, fp64 ? P.ld / 2 : P.ld32 / 4);
            const int bigs[] = {1, 64, 128, 256, 512, 1 << 30};
            float tbest = 0.0f;
            SweepShape cbest = base;
            // candidates: the level size from which the large-level form
            // replaces the prefetching one, that form (streaming with half,
            // the default or twice the default elements per workgroup, or
            // prefetching without the Jacobian columns)
            // (IRK_SWEEP_FLOW / IRK_SWEEP_CHAIN in the environment fix the
            // single-launch / chaining choice)
            const bool flow_fixed = std::getenv("IRK_SWEEP_FLOW") != nullptr;
            const bool chain_fixed = std::getenv("IRK_SWEEP_CHAIN") != nullptr;
            const bool split_fixed = std::getenv("IRK_SWEEP_SPLIT") != nullptr;
            auto time_shape = [&](const SweepShape &cand) -> irk_status {
                sh = cand;
                if (build_items(h) != IRK_OK) return IRK_OK;
                irk_status st = upload_items(h);
                if (st != IRK_OK) return st;
                const float t = time_us(h, [&] { enqueue_pc(C, fp64, SL_EXT0, 0, -1, 0); }, 3);
                if (tbest == 0.0f || t < tbest) { tbest = t; cbest = sh; }
                return IRK_OK;
            };
            if (flow_fixed && base.flow) {
                irk_status st = time_shape(base);
                if (st != IRK_OK) return st;
            } else {
                for (int tps : {base.tps_st / 2, base.tps_st, base.tps_st * 2, 0}) {
                    const bool lite = tps == 0;
                    if (lite && !base.pf_lite) continue;
                    if (!lite && (tps < 1 || tps > 16 || SW_THREADS / tps < 4 * R)) continue;
                    for (int bm : bigs) {
                        if (!base.pf && bm != 1) continue;
                        if (lite && bm == (1 << 30)) continue;     // no large levels: same as above
                        SweepShape c = base;
                        c.flow = false;
                        if (!chain_fixed) c.chain_max = 0;
                        c.tps_st = lite ? base.tps_st : tps;
                        c.big_form = lite ? 2 : 0;
                        c.big_min = bm;
                        irk_status st = time_shape(c);
                        if (st != IRK_OK) return st;
                    }
                }
                // the best shape with its levels below a size chained into one
                // launch per run of equal forms
                const SweepShape per_level = cbest;
                for (int cm : {32, 64, 128, 256, 512, 1024, 1 << 30}) {
                    if (chain_fixed) break;
                    SweepShape c = per_level;
                    c.chain_max = cm;
                    irk_status st = time_shape(c);
                    if (st != IRK_OK) return st;
                }
                // streaming levels below a size at half the elements per workgroup
                const SweepShape chained = cbest;
                if (!split_fixed && chained.tps_st >= 2 && chained.big_form == 0 && chained.big_min < (1 << 30)) {
                    for (int sp : {256, 384, 512, 768, 1024}) {
                        if (sp <= chained.big_min) continue;
                        SweepShape c = chained;
                        c.st_split = sp;
                        irk_status st = time_shape(c);
                        if (st != IRK_OK) return st;
                    }
                }
                // every level of a direction in one launch, in each form that fits
                for (int ff = 0; ff < 3 && !flow_fixed; ++ff) {
                    if ((ff == 1 && !base.pf) || (ff == 2 && !base.pf_lite)) continue;
                    SweepShape c = base;
                    c.flow = true;
                    c.flow_form = ff;
                    irk_status st = time_shape(c);
                    if (st != IRK_OK) return st;
                }
            }
            sh = cbest;
            best.sweep_us = tbest;
            best.sw64 = h->sw64;
            best.sw32 = h->sw32;
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = best;
    }
    h->tpw64 = best.tpw64; h->tpw32 = best.tpw32;
    h->sw64 = best.sw64; h->sw32 = best.sw32;
    irk_status st = build_items(h);
    if (st != IRK_OK) return st;
    st = upload_items(h);
    if (st != IRK_OK) return st;
    if (info) {
        const SweepShape &sh = h->mixed ? h->sw32 : h->sw64;
        info->matvec_teams = h->mixed ? h->tpw32 : h->tpw64;
        info->sweep_big_min = sh.big_min;
        info->sweep_teams = sh.tps_st;
        info->sweep_big_form = sh.big_form;
        info->sweep_flow = sh.flow ? 1 + sh.flow_form : 0;
        info->sweep_chain_max = sh.flow ? 0 : sh.chain_max;
        info->sweep_split = st_small_tps(sh) ? sh.st_split : 0;
        info->from_cache = cached ? 1 : 0;
        info->matvec_us = best.matvec_us;
        info->sweep_us = best.sweep_us;
    }
    return IRK_OK;
}
