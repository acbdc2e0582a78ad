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
// Elements of one level are independent; each team handles one element and
// all s stages of it: the shared Jacobian blocks of the element's row are
// streamed once and applied to the s stage vectors, then the stage-local
// pivot (and cross-stage) products follow.  The element-major order reaches
// every unknown after its dependencies in the stage-major elimination order,
// so the coupled form needs the same number of levels as the uncoupled one.
// The backward sweep overwrites y^ with z in place.
#include "irk_device.h"

namespace irk {

// Reduce team partials red[g][S][ldr] over g for stage k, row r.
template <typename TC, int S>
__device__ __forceinline__ TC sum_groups(const TC *red, int G, int k, int ldr, int r) {
    TC a = 0;
    for (int g = 0; g < G; ++g) a += red[(g * S + k) * ldr + r];
    return a;
}

template <int S, typename TJ, typename TF, typename TC, bool COUPLED, bool SHJ, bool FWD>
__device__ __forceinline__ void sweep_item(const SysDesc &d, const Item it, int v_slot, int v_index,
                                           int acc_slot, unsigned char *smem_raw)
{
    const int s = d.s, m = d.m, T = d.T;
    constexpr int VJ = Vec16<TJ>::V, VF = Vec16<TF>::V;
    const int ldJ = ld_of<TJ>(d), ldF = ld_of<TF>(d);
    const int ldv = round_up(m, 8);
    const int tpw = it.aux;
    const int team = NTHREADS / tpw;
    const int tm = threadIdx.x / team, tid = threadIdx.x - tm * team;
    const int RJ = ldJ / VJ, GJ = team / RJ;
    const int gJ = tid / RJ, sJ = tid - gJ * RJ;
    const int RF = ldF / VF, GF = team / RF;
    const int gF = tid / RF, sF = tid - gF * RF;
    const int maxg = d.maxrow * m;
    const int region = sweep_region(S, m, d.maxrow, ldJ, VJ, ldF, VF, team);
    TC *base_lds = reinterpret_cast<TC *>(smem_raw) + (size_t)tm * region;
    TC *xg = base_lds;                       // gather, then partials
    TC *yv = base_lds + (region - 2 * S * ldv);   // [S][ldv]
    TC *uv = yv + S * ldv;                   // [S][ldv]

    const bool has = tm < it.count;
    const long long n = (long long)T * m;
    const GAS int *lvl = gp(FWD ? d.lvl_fwd : d.lvl_bwd);
    const GAS int *row_ptr = gp(d.row_ptr);
    const GAS int *col_idx = gp(d.col_idx);
    const GAS int *diag_pos = gp(d.diag_pos);
    const int i = has ? lvl[it.first + tm] : 0;
    GAS TC *yh = gp(reinterpret_cast<TC *>(d.vec[SL_YH]));
    const TC dt = (TC)d.dt;

    int pa = 0, ncol = 0;
    if (has) {
        const int p0 = row_ptr[i], p1 = row_ptr[i + 1], pd = diag_pos[i];
        pa = FWD ? p0 : pd + 1;
        ncol = (FWD ? (pd - p0) : (p1 - pd - 1)) * m;
        for (int q = tid; q < ncol; q += team) {
            const int b = q / m, c = q - b * m;
            const long long j = col_idx[pa + b];
#pragma unroll
            for (int k = 0; k < S; ++k)
                if (k < s) xg[k * maxg + q] = yh[k * n + j * m + c];
        }
        if (FWD) {
            const GAS double *v = gp(reinterpret_cast<const double *>(d.vec[v_slot])) + (long long)v_index * d.N;
            for (int q = tid; q < s * m; q += team) {
                const int k = q / m, r = q - k * m;
                yv[k * ldv + r] = (TC)v[k * n + (long long)i * m + r];
            }
        } else {
            for (int q = tid; q < s * m; q += team) {
                const int k = q / m, r = q - k * m;
                yv[k * ldv + r] = yh[k * n + (long long)i * m + r];
            }
        }
    }
    __syncthreads();

    // ---- Jacobian part: dt * sum_j J_ij w_{k,j} for all stages ----
    {
        TC aj[S][VJ];
#pragma unroll
        for (int k = 0; k < S; ++k)
#pragma unroll
            for (int v = 0; v < VJ; ++v) aj[k][v] = 0;
        if (has && gJ < GJ && ncol > 0) {
            const auto Jb = jac_of<TJ>(d);
            if (SHJ) {
                const auto base = Jb + (size_t)pa * m * ldJ + sJ * VJ;
#pragma unroll 4
                for (int cg = gJ; cg < ncol; cg += GJ) {
                    TC a[VJ];
                    Vec16<TJ>::load(base + (size_t)cg * ldJ, a);
#pragma unroll
                    for (int k = 0; k < S; ++k) {
                        if (k >= s) continue;
                        const TC xv = xg[k * maxg + cg];
#pragma unroll
                        for (int v = 0; v < VJ; ++v) aj[k][v] += a[v] * xv;
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < S; ++k) {
                    if (k >= s) continue;
                    const auto base =
                        Jb + ((size_t)k * d.nnzb + pa) * m * ldJ + sJ * VJ;
#pragma unroll 4
                    for (int cg = gJ; cg < ncol; cg += GJ) {
                        TC a[VJ];
                        Vec16<TJ>::load(base + (size_t)cg * ldJ, a);
                        const TC xv = xg[k * maxg + cg];
#pragma unroll
                        for (int v = 0; v < VJ; ++v) aj[k][v] += a[v] * xv;
                    }
                }
            }
        }
        __syncthreads();
        if (has && gJ < GJ) {
#pragma unroll
            for (int k = 0; k < S; ++k) {
                if (k >= s) continue;
#pragma unroll
                for (int v = 0; v < VJ; ++v) xg[(gJ * S + k) * ldJ + sJ * VJ + v] = aj[k][v];
            }
        }
        __syncthreads();
        if (has) {
            for (int q = tid; q < s * m; q += team) {
                const int k = q / m, r = q - k * m;
                const TC u = dt * sum_groups<TC, S>(xg, GJ, k, ldJ, r);
                if (FWD) yv[k * ldv + r] += u;
                else uv[k * ldv + r] = u;
            }
        }
        __syncthreads();
    }

    const auto Pb = piv_of<TF>(d);
    const long long bsF = (long long)m * ldF;
    TC *red = xg;

    if (!COUPLED) {
        // all stages at once: out_k = P_k^{-1} in_k
        const TC *in = FWD ? yv : uv;
        TC ap[S][VF];
#pragma unroll
        for (int k = 0; k < S; ++k)
#pragma unroll
            for (int v = 0; v < VF; ++v) ap[k][v] = 0;
        if (has && gF < GF) {
#pragma unroll
            for (int k = 0; k < S; ++k) {
                if (k >= s) continue;
                const auto pb = Pb + ((long long)i * s + k) * bsF + sF * VF;
#pragma unroll 4
                for (int c = gF; c < m; c += GF) {
                    TC a[VF];
                    Vec16<TF>::load(pb + (size_t)c * ldF, a);
                    const TC xv = in[k * ldv + c];
#pragma unroll
                    for (int v = 0; v < VF; ++v) ap[k][v] += a[v] * xv;
                }
            }
#pragma unroll
            for (int k = 0; k < S; ++k) {
                if (k >= s) continue;
#pragma unroll
                for (int v = 0; v < VF; ++v) red[(gF * S + k) * ldF + sF * VF + v] = ap[k][v];
            }
        }
        __syncthreads();
        if (has) {
            GAS double *acc = acc_slot >= 0 ? gp(reinterpret_cast<double *>(d.vec[acc_slot])) : nullptr;
            for (int q = tid; q < s * m; q += team) {
                const int k = q / m, r = q - k * m;
                const TC sc = block_scale<TF, TC>(d.P16e, (long long)i * s + k);
                TC o = sc * sum_groups<TC, S>(red, GF, k, ldF, r);
                const long long gi = k * n + (long long)i * m + r;
                if (!FWD) o += yv[k * ldv + r];
                yh[gi] = o;
                if (!FWD && acc) acc[gi] += (double)o;
            }
        }
        return;
    }

    // ---- coupled: stage rounds inside the element ----
    const auto Cb = cross_of<TF>(d);
    const int sm1 = s - 1;
    GAS double *acc = acc_slot >= 0 ? gp(reinterpret_cast<double *>(d.vec[acc_slot])) : nullptr;
#pragma unroll 1
    for (int kk = 0; kk < S; ++kk) {
        const int k = FWD ? kk : (S - 1 - kk);
        const bool act = has && k < s;
        // (a) pivot product of stage k
        {
            const TC *in = FWD ? yv : uv;
            TC ap[VF];
#pragma unroll
            for (int v = 0; v < VF; ++v) ap[v] = 0;
            if (act && gF < GF) {
                const auto pb = Pb + ((long long)i * s + k) * bsF + sF * VF;
#pragma unroll 4
                for (int c = gF; c < m; c += GF) {
                    TC a[VF];
                    Vec16<TF>::load(pb + (size_t)c * ldF, a);
                    const TC xv = in[k * ldv + c];
#pragma unroll
                    for (int v = 0; v < VF; ++v) ap[v] += a[v] * xv;
                }
#pragma unroll
                for (int v = 0; v < VF; ++v) red[gF * ldF + sF * VF + v] = ap[v];
            }
            __syncthreads();
            if (act) {
                const TC sc = block_scale<TF, TC>(d.P16e, (long long)i * s + k);
                for (int r = tid; r < m; r += team) {
                    TC o = 0;
                    for (int g = 0; g < GF; ++g) o += red[g * ldF + r];
                    o *= sc;
                    const long long gi = k * n + (long long)i * m + r;
                    if (!FWD) o += yv[k * ldv + r];
                    yh[gi] = o;
                    if (!FWD && acc) acc[gi] += (double)o;
                    yv[k * ldv + r] = o;   // y^_k (forward) or z_k (backward) for the cross terms
                }
            }
            __syncthreads();
        }
        // (b) cross-stage update of the stages not yet done:
        //     forward: y_l -= C_{lk} y^_k (l > k);  backward: u_l -= C_{lk} z_k (l < k)
        {
            TC ac[S][VF];
#pragma unroll
            for (int l = 0; l < S; ++l)
#pragma unroll
                for (int v = 0; v < VF; ++v) ac[l][v] = 0;
            if (act && gF < GF) {
#pragma unroll
                for (int l = 0; l < S; ++l) {
                    if (l >= s || l == k || (FWD ? (l < k) : (l > k))) continue;
                    const int idx = l < k ? l : l - 1;
                    const auto cb =
                        Cb + (((long long)i * s + k) * sm1 + idx) * bsF + sF * VF;
#pragma unroll 2
                    for (int c = gF; c < m; c += GF) {
                        TC a[VF];
                        Vec16<TF>::load(cb + (size_t)c * ldF, a);
                        const TC xv = yv[k * ldv + c];
#pragma unroll
                        for (int v = 0; v < VF; ++v) ac[l][v] += a[v] * xv;
                    }
#pragma unroll
                    for (int v = 0; v < VF; ++v) red[(gF * S + l) * ldF + sF * VF + v] = ac[l][v];
                }
            }
            __syncthreads();
            if (act) {
                for (int q = tid; q < s * m; q += team) {
                    const int l = q / m, r = q - l * m;
                    if (l == k || (FWD ? (l < k) : (l > k))) continue;
                    const int idx = l < k ? l : l - 1;
                    const TC sc = block_scale<TF, TC>(d.C16e, ((long long)i * s + k) * sm1 + idx);
                    const TC cv = sc * sum_groups<TC, S>(red, GF, l, ldF, r);
                    if (FWD) yv[l * ldv + r] -= cv;
                    else uv[l * ldv + r] -= cv;
                }
            }
            __syncthreads();
        }
    }
}

// One level per launch: workgroup b handles items[b].
template <int S, typename TJ, typename TF, typename TC, bool COUPLED, bool SHJ, bool FWD>
__global__ __launch_bounds__(NTHREADS) void k_sweep(const SysDesc *__restrict__ sysv,
                                                    const Item *__restrict__ items,
                                                    int v_slot, int v_index, int acc_slot,
                                                    int skip_done)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Item it = items[blockIdx.x];
    if (skip_done && sysv[it.sys].st->done) return;
    sweep_item<S, TJ, TF, TC, COUPLED, SHJ, FWD>(sysv[it.sys], it, v_slot, v_index, acc_slot, smem_raw);
}

// Whole sweep in one launch.  Workgroups take the items of all levels in
// level order from an atomic ticket; before an item runs, one thread per
// team waits until every dependency of its element (lower neighbours in the
// forward sweep, upper ones in the backward sweep) has published its flag
// for this sweep (`epoch`).  Every dependency sits at an earlier level, so
// its ticket was taken earlier by a workgroup that is already running and
// only waits on still earlier tickets: the smallest unfinished ticket can
// always proceed, and the grid drains.  A bounded spin turns a lost flag
// into an error flag instead of a hang.  Results are written, then made
// visible device-wide (release fence) before the flag is set; the waiting
// side acquires before reading them.
template <int S, typename TJ, typename TF, typename TC, bool COUPLED, bool SHJ, bool FWD>
__global__ __launch_bounds__(NTHREADS) void k_sweep_persist(const SysDesc *__restrict__ sysv,
                                                            const Item *__restrict__ items,
                                                            int nitems, int v_slot, int v_index,
                                                            int acc_slot, int skip_done,
                                                            unsigned epoch)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int tk;
    const SysDesc &d = sysv[items[0].sys];
    unsigned *ticket = &d.st->tickets[FWD ? 4 : 5];
    unsigned *flags = d.dep_flags;
    const GAS int *lvl = gp(FWD ? d.lvl_fwd : d.lvl_bwd);
    const GAS int *row_ptr = gp(d.row_ptr);
    const GAS int *col_idx = gp(d.col_idx);
    const GAS int *diag_pos = gp(d.diag_pos);
    for (;;) {
        if (threadIdx.x == 0) tk = (int)atomicAdd(ticket, 1u);
        __syncthreads();
        const int t = tk;
        if (t >= nitems) {
            // the last workgroup to leave resets the ticket for the next launch
            if (threadIdx.x == 0 && t == nitems + (int)gridDim.x - 1) *ticket = 0u;
            return;
        }
        const Item it = items[t];
        if (skip_done && d.st->done) {   // uniform: one system per launch
            __syncthreads();             // everybody has read tk before it changes
            continue;
        }
        const int team = NTHREADS / it.aux;
        const int tm = threadIdx.x / team, tid = threadIdx.x - tm * team;
        if (tid == 0 && tm < it.count) {
            const int i = lvl[it.first + tm];
            const int p0 = FWD ? row_ptr[i] : diag_pos[i] + 1;
            const int p1 = FWD ? diag_pos[i] : row_ptr[i + 1];
            for (int q = p0; q < p1; ++q) {
                const int j = col_idx[q];
                long long spins = 0;
                while (__hip_atomic_load(&flags[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > (1LL << 22)) { d.st->spin_timeout = 1; break; }
                }
            }
            __atomic_thread_fence(__ATOMIC_ACQUIRE);
        }
        __syncthreads();
        sweep_item<S, TJ, TF, TC, COUPLED, SHJ, FWD>(d, it, v_slot, v_index, acc_slot, smem_raw);
        __syncthreads();
        if (tid == 0 && tm < it.count) {
            const int i = lvl[it.first + tm];
            __hip_atomic_store(&flags[i], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int S, typename TJ, typename TF, typename TC>
static void launch_sweep_t(bool forward, const SysDesc *dsys, const Item *items, int nitems,
                           bool coupled, bool sharedJ, int v_slot, int v_index, int acc_slot,
                           int skip_done, size_t shmem, hipStream_t st, int pgrid, unsigned epoch)
{
    dim3 grid(pgrid > 0 ? pgrid : nitems), block(NTHREADS);
#define SW(C, SH, F)                                                                             \
    do {                                                                                         \
        if (pgrid > 0)                                                                           \
            hipLaunchKernelGGL((k_sweep_persist<S, TJ, TF, TC, C, SH, F>), grid, block, shmem, st, \
                               dsys, items, nitems, v_slot, v_index, acc_slot, skip_done, epoch); \
        else                                                                                     \
            hipLaunchKernelGGL((k_sweep<S, TJ, TF, TC, C, SH, F>), grid, block, shmem, st, dsys,   \
                               items, v_slot, v_index, acc_slot, skip_done);                     \
    } while (0)
    if (forward) {
        if (coupled) { if (sharedJ) SW(true, true, true); else SW(true, false, true); }
        else { if (sharedJ) SW(false, true, true); else SW(false, false, true); }
    } else {
        if (coupled) { if (sharedJ) SW(true, true, false); else SW(true, false, false); }
        else { if (sharedJ) SW(false, true, false); else SW(false, false, false); }
    }
#undef SW
}

template <int S>
static void launch_sweep_s(bool forward, const SysDesc *dsys, const Item *items, int nitems,
                           bool fp64, int ftype, bool coupled, bool sharedJ, int v_slot,
                           int v_index, int acc_slot, int skip_done, size_t shmem, hipStream_t st,
                           int pgrid, unsigned epoch)
{
    if (fp64) {
        launch_sweep_t<S, double, double, double>(forward, dsys, items, nitems, coupled, sharedJ,
                                                  v_slot, v_index, acc_slot, skip_done, shmem, st, pgrid, epoch);
    } else if (ftype == FT_F32) {
        launch_sweep_t<S, float, float, float>(forward, dsys, items, nitems, coupled, sharedJ,
                                               v_slot, v_index, acc_slot, skip_done, shmem, st, pgrid, epoch);
    } else if (ftype == FT_BF16) {
        launch_sweep_t<S, float, bf16s, float>(forward, dsys, items, nitems, coupled, sharedJ,
                                               v_slot, v_index, acc_slot, skip_done, shmem, st, pgrid, epoch);
    } else {
        launch_sweep_t<S, float, f16s, float>(forward, dsys, items, nitems, coupled, sharedJ,
                                              v_slot, v_index, acc_slot, skip_done, shmem, st, pgrid, epoch);
    }
}

void launch_sweep(bool forward, const SysDesc *dsys, const Item *items, int nitems, int s_max,
                  bool fp64, int ftype, bool coupled, bool sharedJ, int v_slot, int v_index,
                  int acc_slot, int skip_done, size_t shmem, hipStream_t st, int pgrid,
                  unsigned epoch)
{
    if (nitems <= 0) return;
    switch (s_max) {
    case 1: launch_sweep_s<1>(forward, dsys, items, nitems, fp64, ftype, coupled, sharedJ, v_slot, v_index, acc_slot, skip_done, shmem, st, pgrid, epoch); break;
    case 2: launch_sweep_s<2>(forward, dsys, items, nitems, fp64, ftype, coupled, sharedJ, v_slot, v_index, acc_slot, skip_done, shmem, st, pgrid, epoch); break;
    case 3: launch_sweep_s<3>(forward, dsys, items, nitems, fp64, ftype, coupled, sharedJ, v_slot, v_index, acc_slot, skip_done, shmem, st, pgrid, epoch); break;
    case 4: launch_sweep_s<4>(forward, dsys, items, nitems, fp64, ftype, coupled, sharedJ, v_slot, v_index, acc_slot, skip_done, shmem, st, pgrid, epoch); break;
    default: launch_sweep_s<5>(forward, dsys, items, nitems, fp64, ftype, coupled, sharedJ, v_slot, v_index, acc_slot, skip_done, shmem, st, pgrid, epoch); break;
    }
}

}  // namespace irk
