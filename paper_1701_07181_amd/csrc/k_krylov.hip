// k_krylov.hip -- FP64 Arnoldi (classical Gram-Schmidt with one
// re-orthogonalization, CGS2), Givens least squares and cycle bookkeeping of
// restarted right-preconditioned GMRES, on the device, for any number of
// systems per launch.
//
// Work items: a vector kernel gets one item per (system, chunk); chunk c of
// a system with nc chunks covers the elements c*256 + t, stepping nc*256.
// Reductions write one partial per chunk; the next kernel adds them in a
// fixed order (deterministic, and the kernel boundary orders the partials
// without device-wide fences): a finish kernel with one workgroup per
// system, or, for coefficients the next pass needs, every workgroup of that
// pass (the same sums in each).
//
// One Arnoldi step j (the same j for every system of a launch; systems whose
// cycle already ended, st->done, skip):
//   pass 0: partials of h1 = V_{0..j}^T w
//   pass 1: h1 from them; w -= V h1 and, with the same loaded basis
//           entries, partials of h2 = V^T w
//   pass 2: h2 from them; w -= V h2 and partials of ||w||^2; its finish
//           kernel forms the Hessenberg column h1 + h2, applies the Givens
//           rotations, updates the residual estimate |g_{j+1}| and sets done
//           when it drops below the system's cycle tolerance (or on
//           breakdown / non-finite values)
//   scale:  v_{j+1} = w / ||w||
#include "irk_device.h"

namespace irk {

// Sum NV values of every thread over the workgroup into lds[w*NV + p].
template <int NV>
__device__ __forceinline__ void wg_sum(double (&v)[NV], int nv, double *lds) {
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

// Partials are kept in two banks of RED_BANK rows (a pass reads the bank
// the previous pass wrote while it writes the other).
// Add the partials part[bank][b][p] (b < nblk, p < nv) in a fixed order:
// every thread sums the blocks b = t, t + 256, ... for all p, then the
// fixed wave/LDS tree.  Any workgroup that runs it gets the same sums.
template <int NVMAX>
__device__ void reduce_partials(const SysDesc &d, int nblk, int nv, double *out, int bank = 0) {
    __shared__ double red[4 * NVMAX];
    const int stride = RESTART_MAX + 2;
    double a[NVMAX];
#pragma unroll
    for (int p = 0; p < NVMAX; ++p) a[p] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += NTHREADS) {
        const GAS double *row = gp(d.part) + (size_t)(b + bank * RED_BANK) * stride;
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

__device__ __forceinline__ void store_partials(const SysDesc &d, int chunk, const double *lds,
                                               int nv, int nvmax, int bank = 0) {
    for (int p = threadIdx.x; p < nv; p += NTHREADS) {
        double a = 0.0;
        for (int w2 = 0; w2 < NTHREADS / 64; ++w2) a += lds[w2 * nvmax + p];
        gp(d.part)[(size_t)(chunk + bank * RED_BANK) * (RESTART_MAX + 2) + p] = a;
    }
}

template <int NVMAX, int PASS>
__global__ __launch_bounds__(NTHREADS) void k_cgs(const SysDesc *__restrict__ sysv,
                                                  const Item *__restrict__ items, int j)
{
    __shared__ double lds[4 * NVMAX];
    __shared__ double cf[NVMAX];
    const Item it = items[blockIdx.x];
    const SysDesc &d = sysv[it.sys];
    if (d.st->done) return;
    const long long N = d.N;
    const int nv = j + 1;
    const GAS double *V = gp(reinterpret_cast<const double *>(d.vec[SL_V]));
    GAS double *w = gp(reinterpret_cast<double *>(d.vec[SL_W]));
    const int off2 = RESTART_MAX + 1;
    for (int p = threadIdx.x; p < NVMAX; p += NTHREADS) cf[p] = 0.0;
    constexpr int NACC = (PASS == 2) ? 1 : NVMAX;
    double acc[NACC];
#pragma unroll
    for (int p = 0; p < NACC; ++p) acc[p] = 0.0;
    const long long stride = (long long)it.count * NTHREADS;
    // one element: the basis entries vp (zero past nv) and w's entry wv
    auto element = [&](long long e, const double (&vp)[NVMAX], double wv) {
        if (PASS == 0) {
#pragma unroll
            for (int p = 0; p < NVMAX; ++p)
                if (p < nv) acc[p] += vp[p] * wv;
        } else if (PASS == 1) {
#pragma unroll
            for (int p = 0; p < NVMAX; ++p) wv -= cf[p] * vp[p];
#pragma unroll
            for (int p = 0; p < NVMAX; ++p) acc[p] += vp[p] * wv;
            w[e] = wv;
        } else {
#pragma unroll
            for (int p = 0; p < NVMAX; ++p)
                if (p < nv) wv -= cf[p] * vp[p];
            acc[0] += wv * wv;
            w[e] = wv;
        }
    };
    // U elements of this thread (e, e + stride, ...) at a time: all their
    // loads are issued before the arithmetic, which then runs element by
    // element in the order of the one-at-a-time tail loop
    constexpr int U = (NVMAX <= 8) ? 4 : (NVMAX <= 16) ? 2 : 1;
    long long e = (long long)it.first * NTHREADS + threadIdx.x;
    double wv[U], vp[U][NVMAX];
    auto load = [&]() {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            wv[u] = w[e + u * stride];
#pragma unroll
            for (int p = 0; p < NVMAX; ++p) vp[u][p] = (p < nv) ? V[p * N + e + u * stride] : 0.0;
        }
    };
    // the first group's loads are in flight while the coefficients of the
    // previous pass are formed: h1 (pass 1) or h2 (pass 2) from that pass's
    // partials, the same sums in every workgroup; chunk 0 keeps them for
    // the Hessenberg column
    if (e + (U - 1) * stride < N) load();
    if (PASS >= 1) {
        reduce_partials<NVMAX>(d, it.count, nv, cf, PASS == 1 ? 0 : 1);
        if (it.first == 0)
            for (int p = threadIdx.x; p < nv; p += NTHREADS) d.hbuf[(PASS == 1 ? 0 : off2) + p] = cf[p];
    }
    for (; e + (U - 1) * stride < N; e += U * stride) {
        if (e != (long long)it.first * NTHREADS + threadIdx.x) load();
#pragma unroll
        for (int u = 0; u < U; ++u) element(e + u * stride, vp[u], wv[u]);
    }
    for (; e < N; e += stride) {
        double vp[NVMAX];
#pragma unroll
        for (int p = 0; p < NVMAX; ++p) vp[p] = (p < nv) ? V[p * N + e] : 0.0;
        element(e, vp, w[e]);
    }
    const int nred = (PASS == 2) ? 1 : nv;
    wg_sum<NACC>(acc, nred, lds);
    store_partials(d, it.first, lds, nred, NACC, PASS == 1 ? 1 : 0);
}

// End of step j, one workgroup per system (item = (sys, 0, number of
// chunks)): ||w|| from pass 2's partials; Hessenberg column j = h1 + h2
// (kept by passes 1 and 2) with ||w|| below, the earlier Givens rotations
// and a new one applied to it (in LDS, by one thread); estimate and flags.
template <int NVMAX>
__global__ __launch_bounds__(NTHREADS) void k_cgs_finish(const SysDesc *__restrict__ sysv,
                                                         const Item *__restrict__ items, int j)
{
    __shared__ double outv[1], hc[NVMAX + 1], csl[NVMAX], snl[NVMAX];
    const Item it = items[blockIdx.x];
    const SysDesc &d = sysv[it.sys];
    if (d.st->done) return;
    const int off2 = RESTART_MAX + 1;
    const int R = d.restart;
    for (int p = threadIdx.x; p <= j; p += NTHREADS) hc[p] = d.hbuf[p] + d.hbuf[off2 + p];
    for (int q = threadIdx.x; q < j; q += NTHREADS) { csl[q] = d.cs[q]; snl[q] = d.sn[q]; }
    reduce_partials<1>(d, it.count, 1, outv);      // (its barriers cover the loads above)
    if (threadIdx.x == 0) {
        DevState *st = d.st;
        const double hn = sqrt(outv[0]);
        hc[j + 1] = hn;
        for (int q = 0; q < j; ++q) {
            const double a = hc[q], b = hc[q + 1];
            hc[q] = csl[q] * a + snl[q] * b;
            hc[q + 1] = -snl[q] * a + csl[q] * b;
        }
        const double a = hc[j], b = hc[j + 1];
        const double r = hypot(a, b);
        const double c = (r == 0.0) ? 1.0 : a / r, s = (r == 0.0) ? 0.0 : b / r;
        d.cs[j] = c;
        d.sn[j] = s;
        hc[j] = r;
        hc[j + 1] = 0.0;
        const double gj = d.g[j];
        d.g[j + 1] = -s * gj;
        d.g[j] = c * gj;
        st->est = fabs(d.g[j + 1]);
        st->j = j;
        st->rnorm2 = hn;
        st->iters += 1;
        if (!isfinite(hn) || !isfinite(r)) { st->nonfinite = 1; st->done = 1; }
        if (!(hn > 0.0)) { st->breakdown = 1; st->done = 1; }
        if (st->est <= st->tol_abs || j + 1 >= d.restart || st->iters >= d.max_iters) st->done = 1;
    }
    __syncthreads();
    for (int p = threadIdx.x; p <= j + 1; p += NTHREADS) d.H[p * R + j] = hc[p];
}

// dst = src / st->rnorm2 (zeros if that is not positive); skip_done: the
// system's cycle has ended (the next basis vector is not needed)
__global__ __launch_bounds__(NTHREADS) void k_scale(const SysDesc *__restrict__ sysv,
                                                    const Item *__restrict__ items, int dst_slot,
                                                    int dst_index, int src_slot, int skip_done)
{
    const Item it = items[blockIdx.x];
    const SysDesc &d = sysv[it.sys];
    if (skip_done && d.st->done) return;
    const long long N = d.N;
    GAS double *dst = gp(reinterpret_cast<double *>(d.vec[dst_slot])) + (long long)dst_index * N;
    const GAS double *src = gp(reinterpret_cast<const double *>(d.vec[src_slot]));
    const double dv = d.st->rnorm2;
    const double inv = (dv > 0.0) ? 1.0 / dv : 0.0;
    const long long stride = (long long)it.count * NTHREADS;
    long long e = (long long)it.first * NTHREADS + threadIdx.x;
    for (; e + 3 * stride < N; e += 4 * stride) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = src[e + u * stride];
#pragma unroll
        for (int u = 0; u < 4; ++u) dst[e + u * stride] = v[u] * inv;
    }
    for (; e < N; e += stride) dst[e] = src[e] * inv;
}

// partial sums of ||slot||^2
__global__ __launch_bounds__(NTHREADS) void k_norm(const SysDesc *__restrict__ sysv,
                                                   const Item *__restrict__ items, int slot)
{
    __shared__ double lds[4];
    const Item it = items[blockIdx.x];
    const SysDesc &d = sysv[it.sys];
    const long long N = d.N;
    const GAS double *x = gp(reinterpret_cast<const double *>(d.vec[slot]));
    double a[1] = {0.0};
    const long long stride = (long long)it.count * NTHREADS;
    long long e = (long long)it.first * NTHREADS + threadIdx.x;
    for (; e + 3 * stride < N; e += 4 * stride) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = x[e + u * stride];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[0] += v[u] * v[u];
    }
    for (; e < N; e += stride) a[0] += x[e] * x[e];
    wg_sum<1>(a, 1, lds);
    store_partials(d, it.first, lds, 1, 1);
}

// which = 0: ||b|| into st->bnorm;  which = 1: start of a cycle from the
// residual norm: beta, g = (beta, 0, ...), step counter and flags reset, and
// the cycle tolerance |g_{j+1}| <= tol_abs (FP64: rtol ||b||; refinement
// inner cycles: max(inner_rtol beta, rtol ||b||))
__global__ __launch_bounds__(NTHREADS) void k_norm_finish(const SysDesc *__restrict__ sysv,
                                                          const Item *__restrict__ items, int which)
{
    __shared__ double outv[1];
    const Item it = items[blockIdx.x];
    const SysDesc &d = sysv[it.sys];
    reduce_partials<1>(d, it.count, 1, outv);
    if (threadIdx.x == 0) {
        const double nrm = sqrt(outv[0]);
        DevState *st = d.st;
        if (!isfinite(nrm)) st->nonfinite = 1;
        if (which == 0) {
            st->bnorm = nrm;
        } else {
            st->prev_breakdown = st->breakdown;
            st->prev_est = st->est;
            st->beta = nrm;
            st->rnorm2 = nrm;
            st->j = -1;
            st->done = 0;
            st->breakdown = 0;
            st->est = nrm;
            const double t0 = d.rtol * st->bnorm;
            st->tol_abs = d.mixed ? fmax(d.inner_rtol * nrm, t0) : t0;
            d.g[0] = nrm;
            for (int q = 1; q <= d.restart; ++q) d.g[q] = 0.0;
        }
    }
}

// y = H^{-1} g over the nv = st->j + 1 steps of the cycle (every workgroup
// solves the small triangular system), u = B y for the basis B in basis_slot
template <int NVMAX>
__global__ __launch_bounds__(NTHREADS) void k_cycle_end(const SysDesc *__restrict__ sysv,
                                                        const Item *__restrict__ items, int basis_slot)
{
    __shared__ double ys[NVMAX], gs[NVMAX], Hs[NVMAX * NVMAX];
    const Item it = items[blockIdx.x];
    const SysDesc &d = sysv[it.sys];
    const long long N = d.N;
    const int R = d.restart;
    const int nv = d.st->j + 1;
    // the triangle of H and g into LDS (one load per thread), then the
    // back substitution by one thread
    for (int q = threadIdx.x; q < nv * nv; q += NTHREADS) {
        const int i = q / nv, k = q - i * nv;
        if (k >= i) Hs[i * NVMAX + k] = d.H[i * R + k];
    }
    for (int q = threadIdx.x; q < nv; q += NTHREADS) gs[q] = d.g[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = nv - 1; i >= 0; --i) {
            double t = gs[i];
            for (int k = i + 1; k < nv; ++k) t -= Hs[i * NVMAX + k] * ys[k];
            ys[i] = t / Hs[i * NVMAX + i];
        }
    }
    __syncthreads();
    if (it.first == 0)
        for (int q = threadIdx.x; q < nv; q += NTHREADS) d.y[q] = ys[q];
    const GAS double *V = gp(reinterpret_cast<const double *>(d.vec[basis_slot]));
    GAS double *u = gp(reinterpret_cast<double *>(d.vec[SL_U]));
    const long long stride = (long long)it.count * NTHREADS;
    constexpr int U = (NVMAX <= 8) ? 4 : (NVMAX <= 16) ? 2 : 1;
    long long e = (long long)it.first * NTHREADS + threadIdx.x;
    for (; e + (U - 1) * stride < N; e += U * stride) {
        double vp[U][NVMAX];
#pragma unroll
        for (int q = 0; q < U; ++q)
#pragma unroll
            for (int p = 0; p < NVMAX; ++p) vp[q][p] = (p < nv) ? V[p * N + e + q * stride] : 0.0;
#pragma unroll
        for (int q = 0; q < U; ++q) {
            double a = 0.0;
#pragma unroll
            for (int p = 0; p < NVMAX; ++p)
                if (p < nv) a += ys[p] * vp[q][p];
            u[e + q * stride] = a;
        }
    }
    for (; e < N; e += stride) {
        double a = 0.0;
#pragma unroll
        for (int p = 0; p < NVMAX; ++p)
            if (p < nv) a += ys[p] * V[p * N + e];
        u[e] = a;
    }
}

// dst_slot (FP64) += src_slot (FP64)
__global__ __launch_bounds__(NTHREADS) void k_axpy(const SysDesc *__restrict__ sysv,
                                                   const Item *__restrict__ items, int dst_slot,
                                                   int src_slot)
{
    const Item it = items[blockIdx.x];
    const SysDesc &d = sysv[it.sys];
    const long long N = d.N;
    GAS double *dst = gp(reinterpret_cast<double *>(d.vec[dst_slot]));
    const GAS double *src = gp(reinterpret_cast<const double *>(d.vec[src_slot]));
    const long long stride = (long long)it.count * NTHREADS;
    long long e = (long long)it.first * NTHREADS + threadIdx.x;
    for (; e + 3 * stride < N; e += 4 * stride) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) { a[u] = dst[e + u * stride]; b[u] = src[e + u * stride]; }
#pragma unroll
        for (int u = 0; u < 4; ++u) dst[e + u * stride] = a[u] + b[u];
    }
    for (; e < N; e += stride) dst[e] += src[e];
}

// SL_YH (compute type TD) = src_slot[src_index] (FP64)
template <typename TD>
__global__ __launch_bounds__(NTHREADS) void k_copy_yh(const SysDesc *__restrict__ sysv,
                                                      const Item *__restrict__ items, int src_slot,
                                                      int src_index, int skip_done)
{
    const Item it = items[blockIdx.x];
    const SysDesc &d = sysv[it.sys];
    if (skip_done && d.st->done) return;
    const long long N = d.N;
    GAS TD *dst = gp(reinterpret_cast<TD *>(d.vec[SL_YH]));
    const GAS double *src = gp(reinterpret_cast<const double *>(d.vec[src_slot])) + (long long)src_index * N;
    for (long long e = (long long)it.first * NTHREADS + threadIdx.x; e < N;
         e += (long long)it.count * NTHREADS)
        dst[e] = (TD)src[e];
}

// SL_ZB[j] = (double) SL_YH (skipped for systems whose cycle has ended)
template <typename TS>
__global__ __launch_bounds__(NTHREADS) void k_store_z(const SysDesc *__restrict__ sysv,
                                                      const Item *__restrict__ items, int j)
{
    const Item it = items[blockIdx.x];
    const SysDesc &d = sysv[it.sys];
    if (d.st->done) return;
    const long long N = d.N;
    const GAS TS *src = gp(reinterpret_cast<const TS *>(d.vec[SL_YH]));
    GAS double *dst = gp(reinterpret_cast<double *>(d.vec[SL_ZB])) + (long long)j * N;
    const long long stride = (long long)it.count * NTHREADS;
    long long e = (long long)it.first * NTHREADS + threadIdx.x;
    for (; e + 3 * stride < N; e += 4 * stride) {
        TS v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = src[e + u * stride];
#pragma unroll
        for (int u = 0; u < 4; ++u) dst[e + u * stride] = (double)v[u];
    }
    for (; e < N; e += stride) dst[e] = (double)src[e];
}

__global__ __launch_bounds__(NTHREADS) void k_fill_zero_slot(const SysDesc *__restrict__ sysv,
                                                             const Item *__restrict__ items, int slot)
{
    const Item it = items[blockIdx.x];
    const SysDesc &d = sysv[it.sys];
    const long long N = d.N;
    GAS double *p = gp(reinterpret_cast<double *>(d.vec[slot]));
    for (long long e = (long long)it.first * NTHREADS + threadIdx.x; e < N;
         e += (long long)it.count * NTHREADS)
        p[e] = 0.0;
}

// copy every system's DevState into one contiguous array (items: one per system)
__global__ void k_gather_state(const SysDesc *__restrict__ sysv, const Item *__restrict__ items,
                               int n, DevState *out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const SysDesc &d = sysv[items[q].sys];
    const int *src = reinterpret_cast<const int *>(d.st);
    int *dst = reinterpret_cast<int *>(out + q);
    for (int w = 0; w < (int)(sizeof(DevState) / sizeof(int)); ++w) dst[w] = src[w];
}

// reset the per-solve counters of every system (items: one per system)
__global__ void k_reset_state(const SysDesc *__restrict__ sysv, const Item *__restrict__ items, int n)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    DevState *st = sysv[items[q].sys].st;
    st->iters = 0;
    st->nonfinite = 0;
    st->breakdown = 0;
    st->done = 0;
    st->j = -1;
}

// clear the factorization flags of every system (items: one per system)
__global__ void k_reset_factor_flags(const SysDesc *__restrict__ sysv, const Item *__restrict__ items, int n)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    DevState *st = sysv[items[q].sys].st;
    st->singular = 0;
    st->nonfinite = 0;
}

// ---------------------------------------------------------------------------
template <int PASS>
static void cgs_dispatch(const SysDesc *dsys, const Item *vec, int nvec, const Item *fin, int nfin,
                         int j, hipStream_t st) {
    const int nv = j + 1;
    dim3 b(NTHREADS);
#define CGS(NV)                                                                              \
    do {                                                                                     \
        hipLaunchKernelGGL((k_cgs<NV, PASS>), dim3(nvec), b, 0, st, dsys, vec, j);          \
        if (PASS == 2)                                                                       \
            hipLaunchKernelGGL((k_cgs_finish<NV>), dim3(nfin), b, 0, st, dsys, fin, j);      \
    } while (0)
    if (nv <= 8) CGS(8);
    else if (nv <= 16) CGS(16);
    else if (nv <= 32) CGS(32);
    else CGS(64);
#undef CGS
}

void launch_arnoldi(const SysDesc *dsys, const Item *vec, int nvec, const Item *fin, int nfin, int j,
                    hipStream_t st)
{
    cgs_dispatch<0>(dsys, vec, nvec, fin, nfin, j, st);
    cgs_dispatch<1>(dsys, vec, nvec, fin, nfin, j, st);
    cgs_dispatch<2>(dsys, vec, nvec, fin, nfin, j, st);
    // v_{j+1} = w / ||w||
    hipLaunchKernelGGL(k_scale, dim3(nvec), dim3(NTHREADS), 0, st, dsys, vec, (int)SL_V, j + 1,
                       (int)SL_W, 1);
}

void launch_cycle_end(const SysDesc *dsys, const Item *vec, int nvec, int restart, int basis_slot,
                      hipStream_t st)
{
    dim3 g(nvec), b(NTHREADS);
    if (restart <= 8) hipLaunchKernelGGL((k_cycle_end<8>), g, b, 0, st, dsys, vec, basis_slot);
    else if (restart <= 16) hipLaunchKernelGGL((k_cycle_end<16>), g, b, 0, st, dsys, vec, basis_slot);
    else if (restart <= 32) hipLaunchKernelGGL((k_cycle_end<32>), g, b, 0, st, dsys, vec, basis_slot);
    else hipLaunchKernelGGL((k_cycle_end<64>), g, b, 0, st, dsys, vec, basis_slot);
}

void launch_norm(const SysDesc *dsys, const Item *vec, int nvec, const Item *fin, int nfin, int slot,
                 int which, hipStream_t st)
{
    hipLaunchKernelGGL(k_norm, dim3(nvec), dim3(NTHREADS), 0, st, dsys, vec, slot);
    hipLaunchKernelGGL(k_norm_finish, dim3(nfin), dim3(NTHREADS), 0, st, dsys, fin, which);
}

void launch_start_cycle(const SysDesc *dsys, const Item *vec, int nvec, const Item *fin, int nfin,
                        int src_slot, hipStream_t st)
{
    launch_norm(dsys, vec, nvec, fin, nfin, src_slot, 1, st);
    hipLaunchKernelGGL(k_scale, dim3(nvec), dim3(NTHREADS), 0, st, dsys, vec, (int)SL_V, 0, src_slot, 0);
}

void launch_axpy(const SysDesc *dsys, const Item *vec, int nvec, int dst_slot, int src_slot,
                 hipStream_t st)
{
    hipLaunchKernelGGL(k_axpy, dim3(nvec), dim3(NTHREADS), 0, st, dsys, vec, dst_slot, src_slot);
}

void launch_copy_to_yh(const SysDesc *dsys, const Item *vec, int nvec, bool fp64, int src_slot,
                       int src_index, int skip_done, hipStream_t st)
{
    if (fp64)
        hipLaunchKernelGGL(k_copy_yh<double>, dim3(nvec), dim3(NTHREADS), 0, st, dsys, vec, src_slot,
                           src_index, skip_done);
    else
        hipLaunchKernelGGL(k_copy_yh<float>, dim3(nvec), dim3(NTHREADS), 0, st, dsys, vec, src_slot,
                           src_index, skip_done);
}

void launch_store_z(const SysDesc *dsys, const Item *vec, int nvec, bool fp64, int j, hipStream_t st)
{
    if (fp64) hipLaunchKernelGGL(k_store_z<double>, dim3(nvec), dim3(NTHREADS), 0, st, dsys, vec, j);
    else hipLaunchKernelGGL(k_store_z<float>, dim3(nvec), dim3(NTHREADS), 0, st, dsys, vec, j);
}

void launch_fill_zero_slot(const SysDesc *dsys, const Item *vec, int nvec, int slot, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_zero_slot, dim3(nvec), dim3(NTHREADS), 0, st, dsys, vec, slot);
}

void launch_gather_state(const SysDesc *dsys, const Item *fin, int nfin, DevState *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather_state, dim3((nfin + 63) / 64), dim3(64), 0, st, dsys, fin, nfin, out);
}

void launch_reset_state(const SysDesc *dsys, const Item *fin, int nfin, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset_state, dim3((nfin + 63) / 64), dim3(64), 0, st, dsys, fin, nfin);
}

void launch_reset_factor_flags(const SysDesc *dsys, const Item *fin, int nfin, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset_factor_flags, dim3((nfin + 63) / 64), dim3(64), 0, st, dsys, fin, nfin);
}

}  // namespace irk
