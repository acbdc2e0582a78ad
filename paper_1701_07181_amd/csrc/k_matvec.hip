// k_matvec.hip -- multi-stage BSR product with the transformed operator
//
//   y_k = sum_l A^{-1}_kl M x_l  -  dt J_k x_k          (Sec. 4.1, Eq. big-irk)
//
// One team of threads owns one block row i.  The team first gathers, into
// LDS, the stage vectors x_{k,j} of every column j of row i and the mass
// combination xhat_k = sum_l A^{-1}_kl x_{l,i}.  It then streams the row's
// blocks -- the (r+1) Jacobian blocks, contiguous in the workspace, then M_i
// -- exactly once, column by column: every thread owns V consecutive rows of
// one block column per step (one aligned 16-byte load) and updates s
// accumulators per row, so a shared Jacobian block feeds all stages from a
// single HBM read.  Partial sums of the column groups are combined through
// LDS at the end.  Blocks are stored column-major (leading dimension ld), so
// consecutive threads read consecutive rows of a column: fully coalesced.
// Block loads are nontemporal (each block is read once per product), and the
// first columns of a shared Jacobian row are requested before the gather.
#include "irk_device.h"

namespace irk {

template <int S, typename TM, typename TC, bool SHJ, int MODE, typename TX>
__global__ __launch_bounds__(NTHREADS) void k_matvec(const SysDesc *__restrict__ sysv,
                                                     const Item *__restrict__ items,
                                                     int x_slot, int y_slot, int b_slot,
                                                     int skip_done)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Item it = items[blockIdx.x];
    const SysDesc &d = sysv[it.sys];
    if (skip_done && d.st->done) return;
    const int s = d.s, m = d.m, T = d.T;
    constexpr int V = Vec16<TM>::V;
    const int ld = ld_of<TM>(d);
    const int tpw = it.aux;
    const int team = NTHREADS / tpw;
    const int tm = threadIdx.x / team, tid = threadIdx.x - tm * team;
    const int R = ld / V;
    const int G = team / R;
    const int grp = tid / R, slot = tid - grp * R;
    const int maxcols = (d.maxrow + 1) * m;
    const int region = max(S * maxcols, G * S * ld);
    TC *xg = reinterpret_cast<TC *>(smem_raw) + (size_t)tm * region;

    const int row = it.first + tm;
    const bool has = tm < it.count;
    const long long n = (long long)T * m;
    const GAS TX *x = gp(reinterpret_cast<const TX *>(d.vec[x_slot]));
    const GAS int *row_ptr = gp(d.row_ptr);
    const GAS int *col_idx = gp(d.col_idx);
    int p0 = 0, p1 = 0, ncol = 0;
    if (has) {
        p0 = row_ptr[row];
        p1 = row_ptr[row + 1];
        ncol = (p1 - p0) * m;
    }
    // The first PFU column loads of the shared Jacobian row go out before the
    // gather (addresses clamped into the row; a team without a row reads
    // block 0), so the stream starts while the gather waits on x.
    constexpr int PFU = SHJ ? 8 : 1;
    TC pre[PFU][V];
    const auto Jb = jac_of<TM>(d);
    const auto jrow = Jb + (size_t)p0 * m * ld + slot * V;
    if (SHJ) {
#pragma unroll
        for (int u = 0; u < PFU; ++u) Vec16<TM>::load(jrow + (size_t)min(grp + G * u, max(ncol - 1, 0)) * ld, pre[u]);
    }
    if (has) {
        for (int q = tid; q < ncol; q += team) {
            const int b = q / m, c = q - b * m;
            const long long j = col_idx[p0 + b];
#pragma unroll
            for (int k = 0; k < S; ++k)
                if (k < s) xg[k * maxcols + q] = (TC)x[k * n + j * m + c];
        }
        for (int c = tid; c < m; c += team) {
            TC xv[S];
#pragma unroll
            for (int l = 0; l < S; ++l) xv[l] = (l < s) ? (TC)x[l * n + (long long)row * m + c] : (TC)0;
#pragma unroll
            for (int k = 0; k < S; ++k) {
                if (k >= s) continue;
                TC a = 0;
#pragma unroll
                for (int l = 0; l < S; ++l)
                    if (l < s) a += (TC)d.Ainv[k * SMAX + l] * xv[l];
                xg[k * maxcols + ncol + c] = a;
            }
        }
    }
    __syncthreads();

    TC aj[S][V], am[S][V];
#pragma unroll
    for (int k = 0; k < S; ++k)
#pragma unroll
        for (int v = 0; v < V; ++v) { aj[k][v] = 0; am[k][v] = 0; }

    if (has && grp < G) {
        const auto Mb = mass_of<TM>(d);
        if (SHJ) {
#pragma unroll
            for (int u = 0; u < PFU; ++u) {
                const int cg = grp + G * u;
                if (cg < ncol) {
#pragma unroll
                    for (int k = 0; k < S; ++k) {
                        if (k >= s) continue;
                        const TC xv = xg[k * maxcols + cg];
#pragma unroll
                        for (int v = 0; v < V; ++v) aj[k][v] += pre[u][v] * xv;
                    }
                }
            }
#pragma unroll 4
            for (int cg = grp + G * PFU; cg < ncol; cg += G) {
                TC a[V];
                Vec16<TM>::load(jrow + (size_t)cg * ld, a);
#pragma unroll
                for (int k = 0; k < S; ++k) {
                    if (k >= s) continue;
                    const TC xv = xg[k * maxcols + cg];
#pragma unroll
                    for (int v = 0; v < V; ++v) aj[k][v] += a[v] * xv;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < S; ++k) {
                if (k >= s) continue;
                const auto base =
                    Jb + ((size_t)k * d.nnzb + p0) * m * ld + slot * V;
#pragma unroll 4
                for (int cg = grp; cg < ncol; cg += G) {
                    TC a[V];
                    Vec16<TM>::load(base + (size_t)cg * ld, a);
                    const TC xv = xg[k * maxcols + cg];
#pragma unroll
                    for (int v = 0; v < V; ++v) aj[k][v] += a[v] * xv;
                }
            }
        }
        const auto mb = Mb + (size_t)row * m * ld + slot * V;
#pragma unroll 2
        for (int c = grp; c < m; c += G) {
            TC a[V];
            Vec16<TM>::load(mb + (size_t)c * ld, a);
#pragma unroll
            for (int k = 0; k < S; ++k) {
                if (k >= s) continue;
                const TC xv = xg[k * maxcols + ncol + c];
#pragma unroll
                for (int v = 0; v < V; ++v) am[k][v] += a[v] * xv;
            }
        }
    }
    __syncthreads();
    TC *red = xg;   // [G][S][ld], reuses the gather buffer
    if (has && grp < G) {
        const TC dt = (TC)d.dt;
#pragma unroll
        for (int k = 0; k < S; ++k) {
            if (k >= s) continue;
#pragma unroll
            for (int v = 0; v < V; ++v) red[(grp * S + k) * ld + slot * V + v] = am[k][v] - dt * aj[k][v];
        }
    }
    __syncthreads();
    if (has) {
        for (int q = tid; q < s * m; q += team) {
            const int k = q / m, r = q - k * m;
            TC sum = 0;
            for (int g2 = 0; g2 < G; ++g2) sum += red[(g2 * S + k) * ld + r];
            const long long o = k * n + (long long)row * m + r;
            if (MODE == 0) {
                gp(reinterpret_cast<double *>(d.vec[y_slot]))[o] = (double)sum;
            } else {
                const GAS double *b = gp(reinterpret_cast<const double *>(d.vec[b_slot]));
                gp(reinterpret_cast<double *>(d.vec[y_slot]))[o] = b[o] - (double)sum;
            }
        }
    }
}

template <int S>
static void dispatch_matvec(const SysDesc *dsys, const Item *items, int nitems, int prec,
                            bool sharedJ, int x_slot, int y_slot, int b_slot, int mode,
                            int skip_done, size_t shmem, hipStream_t st)
{
    dim3 grid(nitems), block(NTHREADS);
#define MV_LAUNCH(TM, TC, SH, MD, TX) \
    hipLaunchKernelGGL((k_matvec<S, TM, TC, SH, MD, TX>), grid, block, shmem, st, dsys, items, \
                       x_slot, y_slot, b_slot, skip_done)
    if (prec == 0) {
        if (sharedJ) { if (mode == 0) MV_LAUNCH(double, double, true, 0, double); else MV_LAUNCH(double, double, true, 1, double); }
        else { if (mode == 0) MV_LAUNCH(double, double, false, 0, double); else MV_LAUNCH(double, double, false, 1, double); }
    } else {
        // FP32 operator; input is the compute-type (float) vector, output FP64
        if (sharedJ) MV_LAUNCH(float, float, true, 0, float);
        else MV_LAUNCH(float, float, false, 0, float);
    }
#undef MV_LAUNCH
}

void launch_matvec(const SysDesc *dsys, const Item *items, int nitems, int s_max, int prec,
                   bool sharedJ, int x_slot, int y_slot, int b_slot, int mode, int skip_done,
                   size_t shmem, hipStream_t st)
{
    if (nitems <= 0) return;
    switch (s_max) {
    case 1: dispatch_matvec<1>(dsys, items, nitems, prec, sharedJ, x_slot, y_slot, b_slot, mode, skip_done, shmem, st); break;
    case 2: dispatch_matvec<2>(dsys, items, nitems, prec, sharedJ, x_slot, y_slot, b_slot, mode, skip_done, shmem, st); break;
    case 3: dispatch_matvec<3>(dsys, items, nitems, prec, sharedJ, x_slot, y_slot, b_slot, mode, skip_done, shmem, st); break;
    case 4: dispatch_matvec<4>(dsys, items, nitems, prec, sharedJ, x_slot, y_slot, b_slot, mode, skip_done, shmem, st); break;
    default: dispatch_matvec<5>(dsys, items, nitems, prec, sharedJ, x_slot, y_slot, b_slot, mode, skip_done, shmem, st); break;
    }
}

}  // namespace irk
