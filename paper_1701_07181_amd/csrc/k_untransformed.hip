// k_untransformed.hip -- the untransformed Newton operator (Sec. 4.1,
// Eq. newton-system-2), the baseline that the transformation to Eq. big-irk
// improves on:
//
//   y_k = M x_k  -  dt J_k sum_l a_kl x_l
//
// Two forms:
//  * per block: the s x s block matrix of Eq. newton-system-2 applied one
//    block at a time, one launch per block (k, l) = delta_kl M - dt a_kl J_k,
//    each streaming J_k (and M when k == l) and adding its product with x_l
//    to y_k.  A product costs s^2 streams of a Jacobian: the s^2 (r+1) m^2 T
//    count of Table 2 for the untransformed matrix.
//  * fused: one launch; each element's Jacobian row is streamed once and
//    applied to the stage combinations sum_l a_kl x_l, which the team
//    gathers into LDS first.
// Both follow the team layout of the transformed product (one team per block
// row, thread = V consecutive rows of one block column per step, column
// partials combined through LDS); FP64 only.
#include "irk_device.h"

namespace irk {

template <int S, bool FUSED>
__global__ __launch_bounds__(NTHREADS) void k_untransformed(const SysDesc *__restrict__ sysv,
                                                            const Item *__restrict__ items,
                                                            int x_slot, int y_slot, int kb, int lb,
                                                            int accumulate)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Item it = items[blockIdx.x];
    const SysDesc &d = sysv[it.sys];
    const int s = d.s, m = d.m, T = d.T;
    constexpr int V = 2;
    const int ld = d.ld;
    const int tpw = it.aux;
    const int team = NTHREADS / tpw;
    const int tm = threadIdx.x / team, tid = threadIdx.x - tm * team;
    const int R = ld / V;
    const int G = team / R;
    const int grp = tid / R, slot = tid - grp * R;
    const int maxcols = (d.maxrow + 1) * m;
    const int region = max(S * maxcols, G * S * ld);
    double *xg = reinterpret_cast<double *>(smem_raw) + (size_t)tm * region;

    const int row = it.first + tm;
    const bool has = tm < it.count;
    const long long n = (long long)T * m;
    const GAS double *x = gp(reinterpret_cast<const double *>(d.vec[x_slot]));
    GAS double *y = gp(reinterpret_cast<double *>(d.vec[y_slot]));
    const GAS int *row_ptr = gp(d.row_ptr);
    const GAS int *col_idx = gp(d.col_idx);
    // stages this launch writes: all s (fused, LDS entry k) or kb (entry 0)
    const int nk = FUSED ? s : 1;
    int p0 = 0, ncol = 0;
    if (has) {
        p0 = row_ptr[row];
        ncol = (row_ptr[row + 1] - p0) * m;
    }
    // ---- gather: the Jacobian's inputs for every column of the row, then
    //      the mass block's input (this element's own stage vectors) ----
    if (has) {
        for (int q = tid; q < ncol; q += team) {
            const int b = q / m, c = q - b * m;
            const long long j = col_idx[p0 + b];
            if (FUSED) {
                double xl[S];
#pragma unroll
                for (int l = 0; l < S; ++l) xl[l] = (l < s) ? x[l * n + j * m + c] : 0.0;
#pragma unroll
                for (int k = 0; k < S; ++k) {
                    if (k >= s) continue;
                    double a = 0.0;
#pragma unroll
                    for (int l = 0; l < S; ++l)
                        if (l < s) a += d.A[k * SMAX + l] * xl[l];
                    xg[k * maxcols + q] = a;
                }
            } else {
                xg[q] = x[lb * n + j * m + c];
            }
        }
        for (int c = tid; c < m; c += team) {
            if (FUSED) {
#pragma unroll
                for (int k = 0; k < S; ++k)
                    if (k < s) xg[k * maxcols + ncol + c] = x[k * n + (long long)row * m + c];
            } else {
                xg[ncol + c] = x[lb * n + (long long)row * m + c];
            }
        }
    }
    __syncthreads();

    double aj[S][V], am[S][V];
#pragma unroll
    for (int k = 0; k < S; ++k)
#pragma unroll
        for (int v = 0; v < V; ++v) { aj[k][v] = 0.0; am[k][v] = 0.0; }
    const bool with_mass = FUSED || kb == lb;
    if (has && grp < G) {
        const GAS double *Jb = jac_of<double>(d);
        if (FUSED && d.nJ == 1) {
            // one stream of the shared Jacobian row feeds every stage
            const GAS double *jrow = Jb + (size_t)p0 * m * ld + slot * V;
#pragma unroll 4
            for (int cg = grp; cg < ncol; cg += G) {
                double a[V];
                Vec16<double>::load(jrow + (size_t)cg * ld, a);
#pragma unroll
                for (int k = 0; k < S; ++k) {
                    if (k >= s) continue;
                    const double xv = xg[k * maxcols + cg];
#pragma unroll
                    for (int v = 0; v < V; ++v) aj[k][v] += a[v] * xv;
                }
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < S; ++kk) {
                if (kk >= nk) continue;
                const int kj = (d.nJ == 1) ? 0 : (FUSED ? kk : kb);
                const GAS double *base = Jb + ((size_t)kj * d.nnzb + p0) * m * ld + slot * V;
#pragma unroll 4
                for (int cg = grp; cg < ncol; cg += G) {
                    double a[V];
                    Vec16<double>::load(base + (size_t)cg * ld, a);
                    const double xv = xg[kk * maxcols + cg];
#pragma unroll
                    for (int v = 0; v < V; ++v) aj[kk][v] += a[v] * xv;
                }
            }
        }
        if (with_mass) {
            const GAS double *mb = mass_of<double>(d) + (size_t)row * m * ld + slot * V;
#pragma unroll 2
            for (int c = grp; c < m; c += G) {
                double a[V];
                Vec16<double>::load(mb + (size_t)c * ld, a);
#pragma unroll
                for (int k = 0; k < S; ++k) {
                    if (k >= nk) continue;
                    const double xv = xg[k * maxcols + ncol + c];
#pragma unroll
                    for (int v = 0; v < V; ++v) am[k][v] += a[v] * xv;
                }
            }
        }
    }
    __syncthreads();
    double *red = xg;   // [G][S][ld] partials, reusing the gather buffer
    if (has && grp < G) {
        const double cj = FUSED ? d.dt : d.dt * d.A[kb * SMAX + lb];
#pragma unroll
        for (int k = 0; k < S; ++k) {
            if (k >= nk) continue;
#pragma unroll
            for (int v = 0; v < V; ++v) red[(grp * S + k) * ld + slot * V + v] = am[k][v] - cj * aj[k][v];
        }
    }
    __syncthreads();
    if (has) {
        for (int q = tid; q < nk * m; q += team) {
            const int k = q / m, r = q - k * m;
            double sum = 0.0;
            for (int g2 = 0; g2 < G; ++g2) sum += red[(g2 * S + k) * ld + r];
            const long long o = (FUSED ? k : kb) * n + (long long)row * m + r;
            y[o] = accumulate ? y[o] + sum : sum;
        }
    }
}

template <int S>
static void launch_untr_fused(const SysDesc *dsys, const Item *items, int nitems, int x_slot,
                              int y_slot, size_t shmem, hipStream_t st)
{
    hipLaunchKernelGGL((k_untransformed<S, true>), dim3(nitems), dim3(NTHREADS), shmem, st, dsys,
                       items, x_slot, y_slot, 0, 0, 0);
}

void launch_untransformed(const SysDesc *dsys, const Item *items, int nitems, int s, bool fused,
                          int x_slot, int y_slot, size_t shmem, hipStream_t st)
{
    if (nitems <= 0) return;
    if (fused) {
        switch (s) {
        case 1: launch_untr_fused<1>(dsys, items, nitems, x_slot, y_slot, shmem, st); break;
        case 2: launch_untr_fused<2>(dsys, items, nitems, x_slot, y_slot, shmem, st); break;
        case 3: launch_untr_fused<3>(dsys, items, nitems, x_slot, y_slot, shmem, st); break;
        case 4: launch_untr_fused<4>(dsys, items, nitems, x_slot, y_slot, shmem, st); break;
        default: launch_untr_fused<5>(dsys, items, nitems, x_slot, y_slot, shmem, st); break;
        }
        return;
    }
    // block (k, l) of the s x s block matrix, in ascending l for each k: the
    // first block of a block row writes y_k, the others add to it
    for (int k = 0; k < s; ++k)
        for (int l = 0; l < s; ++l)
            hipLaunchKernelGGL((k_untransformed<1, false>), dim3(nitems), dim3(NTHREADS), shmem, st, dsys,
                               items, x_slot, y_slot, k, l, l > 0 ? 1 : 0);
}

}  // namespace irk
