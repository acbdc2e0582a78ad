// k_sweep.hip -- block ILU(0) preconditioner application, one level per launch
//
// On a triangle-free mesh the ILU(0) factors of the (stage-coupled or
// stage-uncoupled) matrix keep every off-diagonal Jacobian block unchanged
// (Sec. 4.2.1, Alg. 2): the lower factor is B_ji P_i^{-1}, the upper factor is
// B_ij, and only the pivot blocks P_{k,i} (stored inverted) and, for the
// coupled form, the element-local cross-stage blocks C_{kl,i} (Sec. 4.3.1)
// are new.  With y^ = P^{-1} y, the two triangular solves become
//
//   forward  (ascending level):
//       y_{k,i} = v_{k,i} + dt sum_{j<i} J_ij y^_{k,j} - sum_{l<k} C_{kl,i} y^_{l,i}
//       y^_{k,i} = P_{k,i}^{-1} y_{k,i}
//   backward (descending level):
//       z_{k,i} = y^_{k,i} + P_{k,i}^{-1} ( dt sum_{j>i} J_ij z_{k,j}
//                                           - sum_{l>k} C_{kl,i} z_{l,i} )
//
// Pivot (0, i) is eliminated first, so the cross blocks in stage row or
// column 0 keep their starting value A^{-1}_kl M_i and are not stored: the
// forward round of stage 0 applies M_i once (t = M_i y^_0, y_l -= A^{-1}_l0 t
// for every l >= 1), and the backward sweep gathers the stage-0 couplings
// into a = sum_{l>=1} A^{-1}_0l z_l and applies M_i once before the stage-0
// pivot.  The stored cross blocks are the C_{lk,i} with l, k >= 1.
//
// Elements of one level are independent; a team of threads handles one
// element and all s stages of it: the shared Jacobian blocks of the
// element's row are streamed once and applied to the s stage vectors, then
// the stage-local pivot (and cross-stage) products follow.  The element-major
// order reaches every unknown after its dependencies in the stage-major
// elimination order, so the coupled form needs the same number of levels as
// the uncoupled one.  The backward sweep overwrites y^ with z in place.
//
// A level holds roughly one element per compute unit, so the time of a level
// is the latency of one element's chain of dependent products.  Each element
// starts from one record (system, element, row position, block count and
// columns) rather than a chain of index loads.  When the
// blocks are small enough (prefetching form, PF), every thread issues the
// loads of all its pivot and cross-block pieces and of the first columns of
// the Jacobian row before anything else, so the element pays about one
// memory latency; the products then run from registers and LDS.  Larger
// blocks stream each product's matrix in its turn.  Both forms accumulate in
// the same order, so they give identical results.
#include "sweep_item.h"

namespace irk {

// One level per launch: workgroup b handles records b*tps .. b*tps+tps-1.
// epoch != 0: a later launch of the same sweep chains levels and waits for
// the flags of these elements (k_sweep_flow.hip), so they are published.
template <int S, typename TJ, typename TF, typename TC, bool COUPLED, bool SHJ, bool FWD, int PFM>
__global__ __launch_bounds__(SW_THREADS) void k_sweep(const SysDesc *__restrict__ sysv,
                                                      const SwItem *__restrict__ recs, int nrec,
                                                      int tps, int region, int v_slot, int v_index,
                                                      int acc_slot, int skip_done,
                                                      unsigned long long epoch)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // every record of a workgroup belongs to one system (the host pads each
    // system's records to whole workgroups), so the descriptor is uniform
    const int sys = __builtin_amdgcn_readfirstlane(recs[blockIdx.x * tps].sys);
    const SysDesc &d = sysv[sys];
    if (skip_done && d.st->done) return;
    const int team = SW_THREADS / tps;
    const int idx = blockIdx.x * tps + threadIdx.x / team;
    const SwItem rec = recs[min(idx, nrec - 1)];
    const bool has = idx < nrec && rec.i >= 0;
    sweep_item<S, TJ, TF, TC, COUPLED, SHJ, FWD, PFM>(d, rec, has, tps, region, v_slot, v_index,
                                                     acc_slot, smem_raw);
    // (the end of the launch makes the results visible to later launches)
    if (epoch && has && threadIdx.x % team == 0) d.flow[rec.i] = epoch;
}

template <int S, typename TJ, typename TF, typename TC, int PFM>
static void launch_sweep_t(bool forward, const SysDesc *dsys, const SwItem *recs, int nrec, int tps,
                           int region, bool coupled, bool sharedJ, int v_slot, int v_index,
                           int acc_slot, int skip_done, size_t shmem, hipStream_t st,
                           unsigned long long epoch)
{
    dim3 grid((nrec + tps - 1) / tps), block(SW_THREADS);
#define SW(C, SH, F)                                                                                   \
    hipLaunchKernelGGL((k_sweep<S, TJ, TF, TC, C, SH, F, pf_form(PFM, S, C, sizeof(TC) == 8)>), grid, \
                       block, shmem, st, dsys, recs, nrec, tps, region, v_slot, v_index, acc_slot,   \
                       skip_done, epoch)
    if (forward) {
        if (coupled) { if (sharedJ) SW(true, true, true); else SW(true, false, true); }
        else { if (sharedJ) SW(false, true, true); else SW(false, false, true); }
    } else {
        if (coupled) { if (sharedJ) SW(true, true, false); else SW(true, false, false); }
        else { if (sharedJ) SW(false, true, false); else SW(false, false, false); }
    }
#undef SW
}

template <int S, int PFM>
static void launch_sweep_p(bool forward, const SysDesc *dsys, const SwItem *recs, int nrec, int tps,
                           int region, bool fp64, int ftype, bool coupled, bool sharedJ, int v_slot,
                           int v_index, int acc_slot, int skip_done, size_t shmem, hipStream_t st,
                           unsigned long long epoch)
{
#define SWP(TJ, TF, TC)                                                                             \
    launch_sweep_t<S, TJ, TF, TC, PFM>(forward, dsys, recs, nrec, tps, region, coupled, sharedJ, v_slot, \
                                      v_index, acc_slot, skip_done, shmem, st, epoch)
    if (fp64) SWP(double, double, double);
    else if (ftype == FT_F32) SWP(float, float, float);
    else if (ftype == FT_BF16) SWP(float, bf16s, float);
    else SWP(float, f16s, float);
#undef SWP
}

void launch_sweep(bool forward, const SysDesc *dsys, const SwItem *recs, int nrec, int tps,
                  int region, int s_max, bool fp64, int ftype, bool coupled, bool sharedJ,
                  int v_slot, int v_index, int acc_slot, int skip_done, size_t shmem, hipStream_t st,
                  int form, unsigned long long epoch)
{
    if (nrec <= 0) return;
#define SWF(SS, FM)                                                                                 \
    launch_sweep_p<SS, FM>(forward, dsys, recs, nrec, tps, region, fp64, ftype, coupled, sharedJ,   \
                           v_slot, v_index, acc_slot, skip_done, shmem, st, epoch)
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
