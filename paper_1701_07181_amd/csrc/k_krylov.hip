// k_krylov.hip -- FP64 Arnoldi (classical Gram-Schmidt with one
// re-orthogonalization, CGS2), Givens least squares and cycle bookkeeping of
// restarted right-preconditioned GMRES, all on the device.
//
// Each pass streams the basis once: pass 0 forms h1 = V^T w; pass 1 updates
// w -= V h1 and, with the same loaded basis entries, forms h2 = V^T w; pass 2
// updates w -= V h2 and forms ||w||^2.  Partial sums go to a per-workgroup
// buffer; the last workgroup to finish (atomic ticket) adds them in a fixed
// order, so every reduction is deterministic.  The last workgroup of pass 2
// also applies the Givens rotations to the new Hessenberg column and updates
// the residual estimate |g_{j+1}| and the cycle flags.
#include "irk_device.h"

namespace irk {

// sum NV values of every thread over the workgroup; result in out[0..NV) of
// thread 0's view (written to lds_out)
template <int NV>
__device__ __forceinline__ void wg_sum(double (&v)[NV], int nv, double *lds /*[4][NV]*/) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int p = 0; p < NV; ++p) {
        if (p < nv) {
            const double x = wave_sum(v[p]);
            if (lane == 0) lds[w * NV + p] = x;
        }
    }
    __syncthreads();
}

// Reduction of the partials part[b][p] (b < nblk, p < nv) into out[p] by one
// workgroup: every thread adds the blocks b = t, t + 256, ... for all p
// (independent loads, all in flight), then the per-thread sums go through
// the fixed wave/LDS tree: deterministic.  Runs in a separate kernel after
// the pass that wrote the partials, so the kernel boundary orders them.
template <int NVMAX>
__device__ void reduce_partials(const SysDesc &d, int nblk, int nv, double *out) {
    __shared__ double red[4 * NVMAX];
    const int stride = RESTART_MAX + 2;
    double a[NVMAX];
#pragma unroll
    for (int p = 0; p < NVMAX; ++p) a[p] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += NTHREADS) {
        const GAS double *row = gp(d.part) + (size_t)b * stride;
#pragma unroll
        for (int p = 0; p < NVMAX; ++p)
            if (p < nv) a[p] += row[p];
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int p = 0; p < NVMAX; ++p) {
        if (p < nv) {
            const double x = wave_sum(a[p]);
            if (lane == 0) red[w * NVMAX + p] = x;
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < nv; p += NTHREADS)
        out[p] = (red[p] + red[NVMAX + p]) + (red[2 * NVMAX + p] + red[3 * NVMAX + p]);
    __syncthreads();
}

template <int NVMAX, int PASS>
__global__ __launch_bounds__(NTHREADS) void k_cgs(const SysDesc *__restrict__ sysv, int sys, int j,
                                                  double tol_abs)
{
    __shared__ double lds[4 * NVMAX];
    __shared__ double cf[NVMAX];
    const SysDesc &d = sysv[sys];
    const long long N = d.N;
    const int nv = j + 1;
    const GAS double *V = gp(reinterpret_cast<const double *>(d.vec[SL_V]));
    GAS double *w = gp(reinterpret_cast<double *>(d.vec[SL_W]));
    const int off2 = RESTART_MAX + 1;
    for (int p = threadIdx.x; p < NVMAX; p += NTHREADS)
        cf[p] = (PASS == 1) ? ((p < nv) ? d.hbuf[p] : 0.0)
              : (PASS == 2) ? ((p < nv) ? d.hbuf[off2 + p] : 0.0) : 0.0;
    __syncthreads();
    constexpr int NACC = (PASS == 2) ? 1 : NVMAX;
    double acc[NACC];
#pragma unroll
    for (int p = 0; p < NACC; ++p) acc[p] = 0.0;
    const long long stride = (long long)gridDim.x * NTHREADS;
    for (long long e = (long long)blockIdx.x * NTHREADS + threadIdx.x; e < N; e += stride) {
        double wv = w[e];
        if (PASS == 0) {
#pragma unroll
            for (int p = 0; p < NVMAX; ++p)
                if (p < nv) acc[p] += V[p * N + e] * wv;
        } else if (PASS == 1) {
            double vp[NVMAX];
#pragma unroll
            for (int p = 0; p < NVMAX; ++p) vp[p] = (p < nv) ? V[p * N + e] : 0.0;
#pragma unroll
            for (int p = 0; p < NVMAX; ++p) wv -= cf[p] * vp[p];
#pragma unroll
            for (int p = 0; p < NVMAX; ++p) acc[p] += vp[p] * wv;
            w[e] = wv;
        } else {
#pragma unroll
            for (int p = 0; p < NVMAX; ++p)
                if (p < nv) wv -= cf[p] * V[p * N + e];
            acc[0] += wv * wv;
            w[e] = wv;
        }
    }
    const int nred = (PASS == 2) ? 1 : nv;
    wg_sum<NACC>(acc, nred, lds);
    const int pstride = RESTART_MAX + 2;
    for (int p = threadIdx.x; p < nred; p += NTHREADS) {
        double a = 0.0;
        for (int w2 = 0; w2 < NTHREADS / 64; ++w2) a += lds[w2 * NACC + p];
        gp(d.part)[(size_t)blockIdx.x * pstride + p] = a;
    }
}

template <int NVMAX, int PASS>
__global__ __launch_bounds__(NTHREADS) void k_cgs_finish(const SysDesc *__restrict__ sysv, int sys,
                                                         int j, int nblk, double tol_abs)
{
    __shared__ double outv[NVMAX];
    const SysDesc &d = sysv[sys];
    const int nv = j + 1;
    const int off2 = RESTART_MAX + 1;
    constexpr int NACC = (PASS == 2) ? 1 : NVMAX;
    reduce_partials<NACC>(d, nblk, (PASS == 2) ? 1 : nv, outv);
    if (PASS == 0) {
        for (int p = threadIdx.x; p < nv; p += NTHREADS) d.hbuf[p] = outv[p];
        return;
    }
    if (PASS == 1) {
        for (int p = threadIdx.x; p < nv; p += NTHREADS) d.hbuf[off2 + p] = outv[p];
        return;
    }
    // Hessenberg column j, Givens rotation, estimate, flags
    if (threadIdx.x == 0) {
        const int R = d.restart;
        double *H = d.H;
        DevState *st = d.st;
        const double hn = sqrt(outv[0]);
        for (int p = 0; p <= j; ++p) H[p * R + j] = d.hbuf[p] + d.hbuf[off2 + p];
        H[(j + 1) * R + j] = hn;
        for (int q = 0; q < j; ++q) {
            const double a = H[q * R + j], b = H[(q + 1) * R + j];
            H[q * R + j] = d.cs[q] * a + d.sn[q] * b;
            H[(q + 1) * R + j] = -d.sn[q] * a + d.cs[q] * b;
        }
        const double a = H[j * R + j], b = H[(j + 1) * R + j];
        const double r = hypot(a, b);
        const double c = (r == 0.0) ? 1.0 : a / r, s = (r == 0.0) ? 0.0 : b / r;
        d.cs[j] = c;
        d.sn[j] = s;
        H[j * R + j] = r;
        H[(j + 1) * R + j] = 0.0;
        const double gj = d.g[j];
        d.g[j + 1] = -s * gj;
        d.g[j] = c * gj;
        st->est = fabs(d.g[j + 1]);
        st->j = j;
        st->rnorm2 = hn;
        if (!isfinite(hn) || !isfinite(r)) { st->nonfinite = 1; st->done = 1; }
        if (!(hn > 0.0)) { st->breakdown = 1; st->done = 1; }
        if (st->est <= tol_abs) st->done = 1;
    }
}

// dst = src / *div  (div from device memory; a zero divisor writes zeros)
__global__ __launch_bounds__(NTHREADS) void k_scale(const SysDesc *__restrict__ sysv, int sys,
                                                    int dst_slot, int dst_index, int src_slot,
                                                    int use_norm)
{
    const SysDesc &d = sysv[sys];
    const long long N = d.N;
    GAS double *dst = gp(reinterpret_cast<double *>(d.vec[dst_slot])) + (long long)dst_index * N;
    const GAS double *src = gp(reinterpret_cast<const double *>(d.vec[src_slot]));
    const double dv = d.st->rnorm2;
    const double inv = (dv > 0.0 && use_norm) ? 1.0 / dv : 0.0;
    for (long long e = (long long)blockIdx.x * NTHREADS + threadIdx.x; e < N;
         e += (long long)gridDim.x * NTHREADS)
        dst[e] = src[e] * inv;
}

// partial sums of ||slot||^2
__global__ __launch_bounds__(NTHREADS) void k_norm(const SysDesc *__restrict__ sysv, int sys,
                                                   int slot)
{
    __shared__ double lds[4];
    const SysDesc &d = sysv[sys];
    const long long N = d.N;
    const GAS double *x = gp(reinterpret_cast<const double *>(d.vec[slot]));
    double a[1] = {0.0};
    for (long long e = (long long)blockIdx.x * NTHREADS + threadIdx.x; e < N;
         e += (long long)gridDim.x * NTHREADS)
        a[0] += x[e] * x[e];
    wg_sum<1>(a, 1, lds);
    if (threadIdx.x == 0)
        gp(d.part)[(size_t)blockIdx.x * (RESTART_MAX + 2)] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

// which = 0: bnorm;  which = 1: start of a cycle (beta, g, flags)
__global__ __launch_bounds__(NTHREADS) void k_norm_finish(const SysDesc *__restrict__ sysv, int sys,
                                                          int which, int nblk)
{
    __shared__ double outv[1];
    const SysDesc &d = sysv[sys];
    reduce_partials<1>(d, nblk, 1, outv);
    if (threadIdx.x == 0) {
        const double nrm = sqrt(outv[0]);
        DevState *st = d.st;
        if (!isfinite(nrm)) st->nonfinite = 1;
        if (which == 0) {
            st->bnorm = nrm;
        } else {
            st->beta = nrm;
            st->rnorm2 = nrm;
            st->j = -1;
            st->done = 0;
            st->breakdown = 0;
            st->est = nrm;
            d.g[0] = nrm;
            for (int q = 1; q <= d.restart; ++q) d.g[q] = 0.0;
        }
    }
}

// y = H^{-1} g over nv steps (every workgroup solves the small system), u = V y
template <int NVMAX>
__global__ __launch_bounds__(NTHREADS) void k_cycle_end(const SysDesc *__restrict__ sysv, int sys,
                                                        int nv)
{
    __shared__ double ys[NVMAX];
    const SysDesc &d = sysv[sys];
    const long long N = d.N;
    const int R = d.restart;
    if (threadIdx.x == 0) {
        for (int i = nv - 1; i >= 0; --i) {
            double t = d.g[i];
            for (int k = i + 1; k < nv; ++k) t -= d.H[i * R + k] * ys[k];
            ys[i] = t / d.H[i * R + i];
        }
        if (blockIdx.x == 0)
            for (int i = 0; i < nv; ++i) d.y[i] = ys[i];
    }
    __syncthreads();
    const GAS double *V = gp(reinterpret_cast<const double *>(d.vec[SL_V]));
    GAS double *u = gp(reinterpret_cast<double *>(d.vec[SL_U]));
    for (long long e = (long long)blockIdx.x * NTHREADS + threadIdx.x; e < N;
         e += (long long)gridDim.x * NTHREADS) {
        double a = 0.0;
#pragma unroll
        for (int p = 0; p < NVMAX; ++p)
            if (p < nv) a += ys[p] * V[p * N + e];
        u[e] = a;
    }
}

__global__ __launch_bounds__(NTHREADS) void k_copy(const SysDesc *__restrict__ sysv, int sys,
                                                   int dst_slot, int src_slot, double scale)
{
    const SysDesc &d = sysv[sys];
    const long long N = d.N;
    GAS double *dst = gp(reinterpret_cast<double *>(d.vec[dst_slot]));
    const GAS double *src = gp(reinterpret_cast<const double *>(d.vec[src_slot]));
    for (long long e = (long long)blockIdx.x * NTHREADS + threadIdx.x; e < N;
         e += (long long)gridDim.x * NTHREADS)
        dst[e] = scale * src[e];
}

__global__ __launch_bounds__(NTHREADS) void k_axpy(const SysDesc *__restrict__ sysv, int sys,
                                                   int dst_slot, int src_slot)
{
    const SysDesc &d = sysv[sys];
    const long long N = d.N;
    GAS double *dst = gp(reinterpret_cast<double *>(d.vec[dst_slot]));
    const GAS double *src = gp(reinterpret_cast<const double *>(d.vec[src_slot]));
    for (long long e = (long long)blockIdx.x * NTHREADS + threadIdx.x; e < N;
         e += (long long)gridDim.x * NTHREADS)
        dst[e] += src[e];
}

__global__ __launch_bounds__(NTHREADS) void k_fill_zero(double *pp, long long n)
{
    GAS double *p = gp(pp);
    for (long long e = (long long)blockIdx.x * NTHREADS + threadIdx.x; e < n;
         e += (long long)gridDim.x * NTHREADS)
        p[e] = 0.0;
}

// ---------------------------------------------------------------------------
template <int PASS>
static void cgs_dispatch(const SysDesc *dsys, int j, int nblk, double tol, hipStream_t st) {
    const int nv = j + 1;
    dim3 g(nblk), b(NTHREADS), one(1);
#define CGS(NV)                                                                              \
    do {                                                                                     \
        hipLaunchKernelGGL((k_cgs<NV, PASS>), g, b, 0, st, dsys, 0, j, tol);                \
        hipLaunchKernelGGL((k_cgs_finish<NV, PASS>), one, b, 0, st, dsys, 0, j, nblk, tol); \
    } while (0)
    if (nv <= 8) CGS(8);
    else if (nv <= 16) CGS(16);
    else if (nv <= 32) CGS(32);
    else CGS(64);
#undef CGS
}

void launch_cgs(int pass, const SysDesc *dsys, const SysDesc &hsys, int j, int nblk, hipStream_t st)
{
    (void)hsys;
    if (pass == 0) cgs_dispatch<0>(dsys, j, nblk, 0.0, st);
    else if (pass == 1) cgs_dispatch<1>(dsys, j, nblk, 0.0, st);
}

void launch_givens(const SysDesc *dsys, const SysDesc &hsys, int j, double tol_abs, int nblk,
                   hipStream_t st)
{
    cgs_dispatch<2>(dsys, j, nblk, tol_abs, st);
    // v_{j+1} = w / ||w||
    hipLaunchKernelGGL(k_scale, dim3(nblk), dim3(NTHREADS), 0, st, dsys, 0, (int)SL_V, j + 1,
                       (int)SL_W, 1);
    (void)hsys;
}

void launch_cycle_end_n(const SysDesc *dsys, int nv, int nblk, hipStream_t st)
{
    dim3 g(nblk), b(NTHREADS);
    if (nv <= 8) hipLaunchKernelGGL((k_cycle_end<8>), g, b, 0, st, dsys, 0, nv);
    else if (nv <= 16) hipLaunchKernelGGL((k_cycle_end<16>), g, b, 0, st, dsys, 0, nv);
    else if (nv <= 32) hipLaunchKernelGGL((k_cycle_end<32>), g, b, 0, st, dsys, 0, nv);
    else hipLaunchKernelGGL((k_cycle_end<64>), g, b, 0, st, dsys, 0, nv);
}

void launch_norm(const SysDesc *dsys, const SysDesc &hsys, int slot, int which, int nblk,
                 hipStream_t st)
{
    (void)hsys;
    hipLaunchKernelGGL(k_norm, dim3(nblk), dim3(NTHREADS), 0, st, dsys, 0, slot);
    hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(NTHREADS), 0, st, dsys, 0, which, nblk);
}

void launch_start_cycle(const SysDesc *dsys, const SysDesc &hsys, int src_slot, int nblk,
                        hipStream_t st)
{
    (void)hsys;
    hipLaunchKernelGGL(k_norm, dim3(nblk), dim3(NTHREADS), 0, st, dsys, 0, src_slot);
    hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(NTHREADS), 0, st, dsys, 0, 1, nblk);
    hipLaunchKernelGGL(k_scale, dim3(nblk), dim3(NTHREADS), 0, st, dsys, 0, (int)SL_V, 0, src_slot, 1);
}

void launch_axpy(const SysDesc *dsys, const SysDesc &hsys, int dst_slot, int src_slot, int nblk,
                 hipStream_t st)
{
    (void)hsys;
    hipLaunchKernelGGL(k_axpy, dim3(nblk), dim3(NTHREADS), 0, st, dsys, 0, dst_slot, src_slot);
}

void launch_copy(const SysDesc *dsys, const SysDesc &hsys, int dst_slot, int src_slot,
                 double scale, int nblk, hipStream_t st)
{
    (void)hsys;
    hipLaunchKernelGGL(k_copy, dim3(nblk), dim3(NTHREADS), 0, st, dsys, 0, dst_slot, src_slot, scale);
}

void launch_fill_zero(double *p, long long n, hipStream_t st)
{
    if (n <= 0) return;
    long long nb = (n + NTHREADS - 1) / NTHREADS;
    if (nb > 2048) nb = 2048;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)nb), dim3(NTHREADS), 0, st, p, n);
}

}  // namespace irk
