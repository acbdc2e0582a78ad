// k_step.hip -- the element-wise and small kernels of one implicit Runge-
// Kutta time step by Newton's method (Sec. 4.1): the ODE M u' = f(t, u) with
//
//   f(t, u) = J u + cos(omega t) g - eps u^3          (u^3 component-wise)
//
// whose Jacobian J - 3 eps diag(u^2) differs from J only on the diagonal of
// the diagonal blocks.  The stage equations in W = (A (x) I) K (Eq.
// modified-IRK) are solved by Newton with the matrix of Eq. big-irk and the
// per-stage Jacobians J_k = J - 3 eps diag(U_k^2), U_k = u0 + dt w_k.  The
// linear solves run the library's GMRES; these kernels build their inputs:
//
//   k_save_diag      the diagonal blocks of the linear part's Jacobian
//   k_stage_jac      J_k's diagonal blocks in the workspace (or J's, to restore)
//   k_jac_u0         J u0 (the part of every stage's f that W does not change)
//   k_stage_rhs      b'_k = J u0 + cos(omega t_k) g - eps U_k^3 + 3 eps dt U_k^2 w_k
//                    (+ h, the history term of a diagonally implicit stage),
//                    so that the Newton residual -G(W) = b' - B_N W with B_N
//                    the Newton matrix
//   k_combine        h = sum_j coef_j F_j (the earlier stages of a DIRK step)
//   k_rhs_eval       F = J U + cos(omega t) g - eps U^3 given J U, and U = u0 + dt W
//   k_newton_update  W += delta and the per-workgroup max |delta|
//   k_max_finish     max over the workgroups
//   k_step_finish    u1 = u0 + dt sum_k d_k w_k  (d = b^T A^{-1})
#include "irk_device.h"

namespace irk {

constexpr int STEP_RED = 1024;   // workgroups of the max reduction

// Dbase[i] = diagonal block of element i of J (slot 0), column-major m x ld
__global__ __launch_bounds__(NTHREADS) void k_save_diag(const SysDesc *__restrict__ dsys,
                                                        double *__restrict__ Dbase)
{
    const SysDesc &d = *dsys;
    const long long bs = (long long)d.m * d.ld;
    const long long total = (long long)d.T * bs;
    for (long long e = (long long)blockIdx.x * NTHREADS + threadIdx.x; e < total;
         e += (long long)gridDim.x * NTHREADS) {
        const long long i = e / bs, o = e - i * bs;
        Dbase[e] = d.Jc[(long long)d.diag_pos[i] * bs + o];
    }
}

// Diagonal block of element i of J_k = Dbase[i] - 3 eps diag(U_k,i^2) for
// every stage k (restore: eps = 0, plain copies of Dbase)
__global__ __launch_bounds__(NTHREADS) void k_stage_jac(const SysDesc *__restrict__ dsys,
                                                        const double *__restrict__ Dbase,
                                                        const double *__restrict__ u0,
                                                        const double *__restrict__ W, double dt,
                                                        double eps)
{
    const SysDesc &d = *dsys;
    const int m = d.m, ld = d.ld;
    const long long bs = (long long)m * ld;
    const long long per = (long long)d.T * bs;
    const long long total = (long long)d.nJ * per;
    const long long n = (long long)d.T * m;
    double *Jc = const_cast<double *>(d.Jc);
    for (long long e = (long long)blockIdx.x * NTHREADS + threadIdx.x; e < total;
         e += (long long)gridDim.x * NTHREADS) {
        const long long k = e / per, r0 = e - k * per;
        const long long i = r0 / bs, o = r0 - i * bs;
        const int c = (int)(o / ld), r = (int)(o - (long long)c * ld);
        double v = Dbase[r0];
        if (eps != 0.0 && r == c && r < m) {
            const long long q = i * m + r;
            const double U = u0[q] + dt * W[k * n + q];
            v -= 3.0 * eps * U * U;
        }
        Jc[((long long)k * d.nnzb + d.diag_pos[i]) * bs + o] = v;
    }
}

// y = J u0: one workgroup per block row, thread r owns output row r; the
// diagonal block comes from Dbase (the linear part's Jacobian)
__global__ __launch_bounds__(NTHREADS) void k_jac_u0(const SysDesc *__restrict__ dsys,
                                                     const double *__restrict__ Dbase,
                                                     const double *__restrict__ u0,
                                                     double *__restrict__ y)
{
    const SysDesc &d = *dsys;
    const int i = blockIdx.x, m = d.m, ld = d.ld;
    const long long bs = (long long)m * ld;
    for (int r = threadIdx.x; r < m; r += NTHREADS) {
        double acc = 0.0;
        for (int q = d.row_ptr[i]; q < d.row_ptr[i + 1]; ++q) {
            const int j = d.col_idx[q];
            const double *blk = (j == i) ? Dbase + (long long)i * bs : d.Jc + (long long)q * bs;
            const double *uj = u0 + (long long)j * m;
            for (int c = 0; c < m; ++c) acc += blk[(long long)c * ld + r] * uj[c];
        }
        y[(long long)i * m + r] = acc;
    }
}

struct StageCoef { double gam[SMAX]; };

__global__ __launch_bounds__(NTHREADS) void k_stage_rhs(int s, long long n, const double *__restrict__ Ju0,
                                                        const double *__restrict__ g,
                                                        const double *__restrict__ u0,
                                                        const double *__restrict__ W, double dt,
                                                        double eps, StageCoef sc,
                                                        const double *__restrict__ hist,
                                                        double *__restrict__ out)
{
    const long long total = (long long)s * n;
    for (long long e = (long long)blockIdx.x * NTHREADS + threadIdx.x; e < total;
         e += (long long)gridDim.x * NTHREADS) {
        const int k = (int)(e / n);
        const long long q = e - (long long)k * n;
        const double w = W[e];
        const double U = u0[q] + dt * w;
        double v = Ju0[q];
        if (g) v += sc.gam[k] * g[q];
        if (eps != 0.0) v += eps * U * U * (3.0 * dt * w - U);
        if (hist) v += hist[q];
        out[e] = v;
    }
}

constexpr int DIRK_SMAX = 8;   // most stages of a diagonally implicit step
struct CombCoef { double c[DIRK_SMAX]; };

__global__ __launch_bounds__(NTHREADS) void k_combine(int cnt, long long n, CombCoef cf,
                                                      const double *__restrict__ F,
                                                      double *__restrict__ out)
{
    for (long long q = (long long)blockIdx.x * NTHREADS + threadIdx.x; q < n;
         q += (long long)gridDim.x * NTHREADS) {
        double acc = 0.0;
        for (int j = 0; j < cnt; ++j) acc += cf.c[j] * F[(long long)j * n + q];
        out[q] = acc;
    }
}

// U = u0 + dt W
__global__ __launch_bounds__(NTHREADS) void k_stage_state(long long n, const double *__restrict__ u0,
                                                          const double *__restrict__ W, double dt,
                                                          double *__restrict__ U)
{
    for (long long q = (long long)blockIdx.x * NTHREADS + threadIdx.x; q < n;
         q += (long long)gridDim.x * NTHREADS)
        U[q] = u0[q] + dt * W[q];
}

__global__ __launch_bounds__(NTHREADS) void k_rhs_eval(long long n, const double *__restrict__ JU,
                                                       const double *__restrict__ U,
                                                       const double *__restrict__ g, double gam,
                                                       double eps, double *__restrict__ F)
{
    for (long long q = (long long)blockIdx.x * NTHREADS + threadIdx.x; q < n;
         q += (long long)gridDim.x * NTHREADS) {
        double v = JU[q];
        if (g) v += gam * g[q];
        if (eps != 0.0) { const double u = U[q]; v -= eps * u * u * u; }
        F[q] = v;
    }
}

__global__ __launch_bounds__(NTHREADS) void k_newton_update(long long N, double *__restrict__ W,
                                                            const double *__restrict__ delta,
                                                            double *__restrict__ part)
{
    __shared__ double red[NTHREADS / 64];
    double mx = 0.0;
    for (long long e = (long long)blockIdx.x * NTHREADS + threadIdx.x; e < N;
         e += (long long)gridDim.x * NTHREADS) {
        const double dl = delta[e];
        W[e] += dl;
        // NaN propagates: fmax would drop it
        const double a = fabs(dl);
        mx = (a > mx || a != a) ? a : mx;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double t = __shfl_xor(mx, o, 64);
        mx = (t > mx || t != t) ? t : mx;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = red[0];
        for (int w = 1; w < NTHREADS / 64; ++w) t = (red[w] > t || red[w] != red[w]) ? red[w] : t;
        part[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(64) void k_max_finish(int nb, const double *__restrict__ part,
                                                   double *__restrict__ out)
{
    double mx = 0.0;
    for (int b = threadIdx.x; b < nb; b += 64) mx = (part[b] > mx || part[b] != part[b]) ? part[b] : mx;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double t = __shfl_xor(mx, o, 64);
        mx = (t > mx || t != t) ? t : mx;
    }
    if (threadIdx.x == 0) *out = mx;
}

__global__ __launch_bounds__(NTHREADS) void k_step_finish(int s, long long n, const double *__restrict__ u0,
                                                          const double *__restrict__ W, double dt,
                                                          StageCoef dc, double *__restrict__ u1)
{
    for (long long q = (long long)blockIdx.x * NTHREADS + threadIdx.x; q < n;
         q += (long long)gridDim.x * NTHREADS) {
        double acc = 0.0;
        for (int k = 0; k < s; ++k) acc += dc.gam[k] * W[(long long)k * n + q];
        u1[q] = u0[q] + dt * acc;
    }
}

static int grid_for(long long total)
{
    const long long g = (total + NTHREADS - 1) / NTHREADS;
    return (int)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}

void launch_save_diag(const SysDesc *dsys, const SysDesc &h, double *Dbase, hipStream_t st)
{
    hipLaunchKernelGGL(k_save_diag, dim3(grid_for((long long)h.T * h.m * h.ld)), dim3(NTHREADS), 0, st,
                       dsys, Dbase);
}

void launch_stage_jac(const SysDesc *dsys, const SysDesc &h, const double *Dbase, const double *u0,
                      const double *W, double dt, double eps, hipStream_t st)
{
    hipLaunchKernelGGL(k_stage_jac, dim3(grid_for((long long)h.nJ * h.T * h.m * h.ld)), dim3(NTHREADS), 0,
                       st, dsys, Dbase, u0, W, dt, eps);
}

void launch_jac_u0(const SysDesc *dsys, const SysDesc &h, const double *Dbase, const double *u0,
                   double *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_jac_u0, dim3(h.T), dim3(NTHREADS), 0, st, dsys, Dbase, u0, y);
}

void launch_stage_rhs(int s, long long n, const double *Ju0, const double *g, const double *u0,
                      const double *W, double dt, double eps, const double *gam, const double *hist,
                      double *out, hipStream_t st)
{
    StageCoef sc{};
    for (int k = 0; k < s && k < SMAX; ++k) sc.gam[k] = gam[k];
    hipLaunchKernelGGL(k_stage_rhs, dim3(grid_for((long long)s * n)), dim3(NTHREADS), 0, st, s, n, Ju0,
                       g, u0, W, dt, eps, sc, hist, out);
}

void launch_combine(int cnt, long long n, const double *coef, const double *F, double *out,
                    hipStream_t st)
{
    CombCoef cf{};
    for (int j = 0; j < cnt && j < DIRK_SMAX; ++j) cf.c[j] = coef[j];
    hipLaunchKernelGGL(k_combine, dim3(grid_for(n)), dim3(NTHREADS), 0, st, cnt, n, cf, F, out);
}

void launch_stage_state(long long n, const double *u0, const double *W, double dt, double *U,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_stage_state, dim3(grid_for(n)), dim3(NTHREADS), 0, st, n, u0, W, dt, U);
}

void launch_rhs_eval(long long n, const double *JU, const double *U, const double *g, double gam,
                     double eps, double *F, hipStream_t st)
{
    hipLaunchKernelGGL(k_rhs_eval, dim3(grid_for(n)), dim3(NTHREADS), 0, st, n, JU, U, g, gam, eps, F);
}

void launch_newton_update(long long N, double *W, const double *delta, double *part, double *out,
                          hipStream_t st)
{
    const long long g = (N + NTHREADS - 1) / NTHREADS;
    const int nb = (int)(g < 1 ? 1 : (g > STEP_RED ? STEP_RED : g));
    hipLaunchKernelGGL(k_newton_update, dim3(nb), dim3(NTHREADS), 0, st, N, W, delta, part);
    hipLaunchKernelGGL(k_max_finish, dim3(1), dim3(64), 0, st, nb, part, out);
}

void launch_step_finish(int s, long long n, const double *u0, const double *W, double dt,
                        const double *dcoef, double *u1, hipStream_t st)
{
    StageCoef dc{};
    for (int k = 0; k < s && k < SMAX; ++k) dc.gam[k] = dcoef[k];
    hipLaunchKernelGGL(k_step_finish, dim3(grid_for(n)), dim3(NTHREADS), 0, st, s, n, u0, W, dt, dc, u1);
}

}  // namespace irk
