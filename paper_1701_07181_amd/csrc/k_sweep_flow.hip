// k_sweep_flow.hip -- all levels of one block ILU(0) sweep in a single launch
//
// The level schedule only says which elements may run together; what an
// element really needs is the result of the neighbours it reads (its lower
// neighbours in the forward sweep, its upper ones in the backward sweep,
// Sec. 4.2.1).  Here every element of every level is one task of one
// launch.  A task first issues the loads that depend on nothing computed in
// this sweep (its own input, and in the prefetching forms its pivot, cross
// and mass blocks and the first Jacobian columns), then waits for the flags
// of its neighbours, then runs the same arithmetic, in the same order, as
// the level-per-launch kernel, and finally publishes its own flag.  The
// factor traffic of the next level's elements thus overlaps the dependent
// chain of the current one, and a sweep costs one launch instead of one per
// level.
//
// Progress without co-residency assumptions: workgroups take entries of a
// workgroup table (first record, records per workgroup) in the order they
// claim a ticket (one atomic increment), and the table is in level order,
// so a task only waits for tasks with smaller tickets, which belong to
// workgroups that are already running.  The last claimant sets the counter
// back to zero, so every launch finds it at zero.  Entries may differ in
// their records per workgroup (the members of a batch do, and so may the
// levels of one system), not in form; the LDS of a workgroup is split
// evenly among its teams.
//
// Flags hold the epoch of the sweep that published them (a 64-bit number
// that grows with every sweep of the process that chains levels), so they
// are never reset.  The L2 caches of the XCDs are not coherent with each
// other, and release / acquire fences at device scope write back or
// invalidate a whole L2 (measured: they made the launch several times
// slower than one launch per level).  So the values exchanged inside the
// launch bypass them instead: results are stored, and neighbour values
// loaded, with device-scope relaxed atomic accesses.  Publication: every
// thread waits for its stores to complete, the workgroup synchronizes, the
// team's first thread stores the flag; a waiting thread polls the flag and
// loads the neighbour values only after it has seen the epoch.  A wait that
// exceeds its poll budget marks the system's state non-finite and writes NaN
// for its element, so a failure shows up as an error, never as a hang.
//
// A sweep may also chain only some levels (the small ones): the launches of
// single levels before a chain publish their flags too, with the same epoch.
#include "sweep_item.h"

namespace irk {

template <int S, typename TJ, typename TF, typename TC, bool COUPLED, bool SHJ, bool FWD, int PFM>
__global__ __launch_bounds__(SW_THREADS) void k_sweep_flow(const SysDesc *__restrict__ sysv,
                                                           const Item *__restrict__ items, int tab,
                                                           int nblk, int region, int v_slot,
                                                           int v_index, int acc_slot, int skip_done,
                                                           unsigned *ticket, unsigned long long epoch)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_blk, s_late;
    if (threadIdx.x == 0) {
        const unsigned t = atomicAdd(ticket, 1u);
        if (t == (unsigned)nblk - 1u) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_blk = (int)t;
        s_late = 0;
    }
    __syncthreads();
    const int blk = s_blk;
    if (blk >= nblk) return;   // (the counter was not at zero: no record to read)
    const Item wg = items[tab + blk];
    const int tps = __builtin_amdgcn_readfirstlane(wg.count);
    const SwItem *recs = reinterpret_cast<const SwItem *>(items + __builtin_amdgcn_readfirstlane(wg.first));
    // every record of a workgroup belongs to one system and one level
    const int sys = __builtin_amdgcn_readfirstlane(recs[0].sys);
    const SysDesc &d = sysv[sys];
    // a finished system: none of its tasks runs, and no task of another
    // system waits for them
    if (skip_done && d.st->done) return;
    const int team = SW_THREADS / tps;
    const int tid = threadIdx.x % team;
    const SwItem rec = recs[threadIdx.x / team];
    const bool has = rec.i >= 0;
    sweep_item<S, TJ, TF, TC, COUPLED, SHJ, FWD, PFM, true>(d, rec, has, tps, region / tps, v_slot, v_index,
                                                           acc_slot, smem_raw, epoch, &s_late);
    __syncthreads();
    if (s_late) {
        // a neighbour never published: this element's result is undefined
        if (has) {
            GAS TC *yh = gp(reinterpret_cast<TC *>(d.vec[SL_YH]));
            const long long n = (long long)d.T * d.m;
            for (int q = tid; q < d.s * d.m; q += team)
                __hip_atomic_store((TC *)&yh[(q / d.m) * n + (long long)rec.i * d.m + q % d.m],
                                   (TC)__builtin_nan(""), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (tid == 0) d.st->nonfinite = 1;
        }
    }
    __builtin_amdgcn_s_waitcnt(0);   // this thread's result stores have completed
    __syncthreads();
    if (has && tid == 0)
        __hip_atomic_store(d.flow + rec.i, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int S, typename TJ, typename TF, typename TC, int PFM>
static void launch_flow_t(bool forward, const SysDesc *dsys, const Item *items, int tab, int nblk,
                          int region, bool coupled, bool sharedJ, int v_slot, int v_index,
                          int acc_slot, int skip_done, size_t shmem, hipStream_t st, unsigned *ticket,
                          unsigned long long epoch)
{
    dim3 grid(nblk), block(SW_THREADS);
#define SWF(C, SH, F)                                                                                   \
    hipLaunchKernelGGL((k_sweep_flow<S, TJ, TF, TC, C, SH, F, pf_form(PFM, S, C, sizeof(TC) == 8)>),   \
                       grid, block, shmem, st, dsys, items, tab, nblk, region, v_slot, v_index,        \
                       acc_slot, skip_done, ticket, epoch)
    if (forward) {
        if (coupled) { if (sharedJ) SWF(true, true, true); else SWF(true, false, true); }
        else { if (sharedJ) SWF(false, true, true); else SWF(false, false, true); }
    } else {
        if (coupled) { if (sharedJ) SWF(true, true, false); else SWF(true, false, false); }
        else { if (sharedJ) SWF(false, true, false); else SWF(false, false, false); }
    }
#undef SWF
}

template <int S, int PFM>
static void launch_flow_p(bool forward, const SysDesc *dsys, const Item *items, int tab, int nblk,
                          int region, bool fp64, int ftype, bool coupled, bool sharedJ, int v_slot,
                          int v_index, int acc_slot, int skip_done, size_t shmem, hipStream_t st,
                          unsigned *ticket, unsigned long long epoch)
{
#define SWP(TJ, TF, TC)                                                                                \
    launch_flow_t<S, TJ, TF, TC, PFM>(forward, dsys, items, tab, nblk, region, coupled, sharedJ, v_slot, \
                                     v_index, acc_slot, skip_done, shmem, st, ticket, epoch)
    if (fp64) SWP(double, double, double);
    else if (ftype == FT_F32) SWP(float, float, float);
    else if (ftype == FT_BF16) SWP(float, bf16s, float);
    else SWP(float, f16s, float);
#undef SWP
}

void launch_sweep_flow(bool forward, const SysDesc *dsys, const Item *items, int tab, int nblk,
                       int region, int s_max, bool fp64, int ftype, bool coupled, bool sharedJ,
                       int v_slot, int v_index, int acc_slot, int skip_done, size_t shmem,
                       hipStream_t st, int form, unsigned *ticket, unsigned long long epoch)
{
    if (nblk <= 0) return;
#define SWF(SS, FM)                                                                                  \
    launch_flow_p<SS, FM>(forward, dsys, items, tab, nblk, region, fp64, ftype, coupled, sharedJ,     \
                          v_slot, v_index, acc_slot, skip_done, shmem, st, ticket, epoch)
#define SWS(SS)                                                                                      \
    do {                                                                                             \
        if (form == 1) SWF(SS, 1);                                                                   \
        else if (form == 2) SWF(SS, 2);                                                              \
        else SWF(SS, 0);                                                                             \
    } while (0)
    switch (s_max) {
    case 1: SWS(1); break;
    case 2: SWS(2); break;
    case 3: SWS(3); break;
    case 4: SWS(4); break;
    default: SWS(5); break;
    }
#undef SWS
#undef SWF
}

}  // namespace irk
