// k_factor.hip -- level-scheduled block ILU(0) factorization in FP64
//
// Triangle-free meshes (Sec. 4.2.1, Alg. 2): only pivot blocks change.
// For stage k of element i (all lower neighbours j < i already final):
//
//     P_{k,i} = d_k M_i - dt J_{k,ii} - dt^2 sum_{j<i, j~i} J_{k,ij} P_{k,j}^{-1} J_{k,ji}
//
// with d_k = A^{-1}_kk (+ alpha_k for the shifted uncoupled form, Sec. 4.3.2).
// The stage-coupled form (Sec. 4.3.1) is the ILU(0) of the full s*n matrix
// in stage-major order; its extra fill is element-local: at pivot (k, i),
// for every later stage l,
//
//     L = C_{lk,i} P_{k,i}^{-1};   P_{l,i} -= L C_{kl,i};   C_{lq,i} -= L C_{kq,i} (q > k, q != l)
//
// with C_{kl,i} starting at A^{-1}_kl M_i.  Element-major processing (all
// stages of an element inside one task, elements level by level) reaches
// every pivot after its dependencies, so both forms use the same level
// schedule.  Pivots are stored inverted (Gauss-Jordan with partial pivoting)
// because the sweeps apply them as matrix-vector products.
//
// Tasks: phase 0 -- one workgroup per (stage k, element i): builds P_{k,i}
// (and inverts it for the uncoupled forms; sets the cross blocks of stage
// column k for the coupled form).  Phase 1 (coupled only) -- one workgroup
// per element: the stage rounds above.
#include "irk_device.h"
#include "dense64.h"

namespace irk {

// ---------------------------------------------------------------------------
// C = (acc ? C : 0) + alpha * A * B for m x m column-major blocks (leading
// dimension ld), computed by the whole workgroup with a 4 x 4 register tile
// per thread (16 x 16 threads cover a 64 x 64 output tile).
//   m <= 64: both operands are staged in LDS at once (one round of loads in
//            flight, no panel barriers);
//   m >  64: 64 x 64 output tiles, K panels of 16, the next panel prefetched
//            into registers while the current one is multiplied.
// LDS: 2 * 64 * 64 doubles.
// ---------------------------------------------------------------------------
constexpr int GT = 64, GK = 16;

__device__ __forceinline__ void tile_fma(const double *As, const double *Bs, int kn, int tx, int ty,
                                         double (&c)[4][4])
{
#pragma unroll 4
    for (int kk = 0; kk < kn; ++kk) {
        const double2 a01 = *reinterpret_cast<const double2 *>(&As[kk * GT + tx * 4]);
        const double2 a23 = *reinterpret_cast<const double2 *>(&As[kk * GT + tx * 4 + 2]);
        const double2 b01 = *reinterpret_cast<const double2 *>(&Bs[kk * GT + ty * 4]);
        const double2 b23 = *reinterpret_cast<const double2 *>(&Bs[kk * GT + ty * 4 + 2]);
        const double av[4] = {a01.x, a01.y, a23.x, a23.y};
        const double bv[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) c[a][b] += av[a] * bv[b];
    }
}

__device__ __forceinline__ void tile_store(int m, int ld, double alpha, bool acc, GAS double *C, int i0,
                                           int j0, int tx, int ty, const double (&c)[4][4])
{
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int gj = j0 + ty * 4 + b;
        if (gj >= m) continue;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int gi = i0 + tx * 4 + a;
            if (gi >= m) continue;
            GAS double *cp = C + (size_t)gj * ld + gi;
            *cp = (acc ? *cp : 0.0) + alpha * c[a][b];
        }
    }
}

__device__ __forceinline__ void wg_gemm(int m, int ld, double alpha, const double *__restrict__ Ap,
                        const double *__restrict__ Bp, bool acc, double *Cp, double *lds)
{
    const GAS double *A = gp(Ap);
    const GAS double *B = gp(Bp);
    GAS double *C = gp(Cp);
    double *As = lds;               // [k][64]
    double *Bs = lds + GT * GT;     // [k][64]
    const int t = threadIdx.x;
    const int tx = t & 15, ty = t >> 4;
    if (m <= GT) {
        // whole operands: As[k][i] = A(i,k), Bs[k][j] = B(k,j)
        for (int e = t; e < GT * GT; e += NTHREADS) {
            const int i = e & 63, k = e >> 6;
            As[k * GT + i] = (i < m && k < m) ? A[(size_t)k * ld + i] : 0.0;
            const int kb = e & 63, j = e >> 6;
            Bs[kb * GT + j] = (kb < m && j < m) ? B[(size_t)j * ld + kb] : 0.0;
        }
        __syncthreads();
        double c[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) c[a][b] = 0.0;
        tile_fma(As, Bs, m, tx, ty, c);
        tile_store(m, ld, alpha, acc, C, 0, 0, tx, ty, c);
        __syncthreads();
        return;
    }
    for (int i0 = 0; i0 < m; i0 += GT) {
        for (int j0 = 0; j0 < m; j0 += GT) {
            double c[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) c[a][b] = 0.0;
            double ra[4], rb[4];
            auto load_panel = [&](int k0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = t + q * NTHREADS;         // 0..1023
                    const int ii = e & 63, kk = e >> 6;
                    const int gi = i0 + ii, gk = k0 + kk;
                    ra[q] = (gi < m && gk < m) ? A[(size_t)gk * ld + gi] : 0.0;
                    const int kb = e & 15, jj = e >> 4;
                    const int gkb = k0 + kb, gj = j0 + jj;
                    rb[q] = (gkb < m && gj < m) ? B[(size_t)gj * ld + gkb] : 0.0;
                }
            };
            load_panel(0);
            for (int k0 = 0; k0 < m; k0 += GK) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = t + q * NTHREADS;
                    As[(e >> 6) * GT + (e & 63)] = ra[q];
                    Bs[(e & 15) * GT + (e >> 4)] = rb[q];
                }
                __syncthreads();
                if (k0 + GK < m) load_panel(k0 + GK);
                tile_fma(As, Bs, GK, tx, ty, c);
                __syncthreads();
            }
            tile_store(m, ld, alpha, acc, C, i0, j0, tx, ty, c);
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// In-place inverse of an m x m block by Gauss-Jordan elimination with
// partial pivoting, in LDS.  The block's memory image is handled as the
// row-major matrix Q = P^T (row stride ld); inverting Q and writing it back
// the same way leaves P^{-1} in column-major order.  Returns nonzero (in
// every thread) if a pivot column is zero or not finite.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wg_invert(double *gptr, int m, int ld, double *lds)
{
    GAS double *g = gp(gptr);
    const int lda = m + 1;
    double *a = lds;                              // [m][lda]
    double *colc = a + m * lda;                   // [m]
    int *perm = reinterpret_cast<int *>(colc + m);   // [m]
    int *sh = perm + m;                           // [2]: pivot row, bad flag
    const int t = threadIdx.x;
    // 2D mapping: thread owns column tc (+64, +128) and rows tr, tr+4, ...
    const int tc = t & 63, tr = t >> 6;
    for (int c0 = tc; c0 < m; c0 += 64)
        for (int r = tr; r < m; r += NTHREADS / 64) a[r * lda + c0] = g[(size_t)r * ld + c0];
    if (t == 0) sh[1] = 0;
    __syncthreads();
    for (int c = 0; c < m; ++c) {
        if (t < 64) {
            double best = -1.0;
            int bi = c;
            for (int r = c + t; r < m; r += 64) {
                const double v = fabs(a[r * lda + c]);
                if (v > best) { best = v; bi = r; }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const double ob = __shfl_xor(best, o, 64);
                const int oi = __shfl_xor(bi, o, 64);
                if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
            }
            if (t == 0) {
                sh[0] = bi;
                perm[c] = bi;
                if (!(best > 0.0) || !isfinite(best)) sh[1] = 1;
            }
        }
        __syncthreads();
        const int p = sh[0];
        if (p != c) {
            for (int j = t; j < m; j += NTHREADS) {
                const double tmp = a[c * lda + j];
                a[c * lda + j] = a[p * lda + j];
                a[p * lda + j] = tmp;
            }
            __syncthreads();
        }
        const double pinv = 1.0 / a[c * lda + c];
        // pivot row scaled; every thread keeps the entries of its columns
        // (read before the barrier: row c is rewritten after it)
        double prow[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int j = tc + 64 * q;
            prow[q] = (j < m) ? ((j == c) ? pinv : a[c * lda + j] * pinv) : 0.0;
        }
        for (int r = t; r < m; r += NTHREADS) colc[r] = a[r * lda + c];
        __syncthreads();
        for (int r = tr; r < m; r += NTHREADS / 64) {
            const double f = colc[r];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int j = tc + 64 * q;
                if (j >= m) continue;
                double v;
                if (r == c) v = prow[q];
                else if (j == c) v = -f * pinv;
                else v = a[r * lda + j] - f * prow[q];
                a[r * lda + j] = v;
            }
        }
        __syncthreads();
    }
    for (int c = m - 1; c >= 0; --c) {
        const int p = perm[c];
        if (p != c) {
            for (int r = t; r < m; r += NTHREADS) {
                const double tmp = a[r * lda + c];
                a[r * lda + c] = a[r * lda + p];
                a[r * lda + p] = tmp;
            }
            __syncthreads();
        }
    }
    for (int c0 = tc; c0 < m; c0 += 64)
        for (int r = tr; r < m; r += NTHREADS / 64) g[(size_t)r * ld + c0] = a[r * lda + c0];
    const int bad = sh[1];
    __syncthreads();
    return bad;
}

// Block product and inverse: the matrix-core path and the register
// Gauss-Jordan for m <= 64 (SMALL), the LDS-tiled ones above otherwise.  The
// kernels are compiled separately for the two classes so that each carries
// only its own register demand.
template <bool SMALL>
__device__ __forceinline__ void blk_gemm(int m, int ld, double alpha, const double *A, const double *B,
                                         bool acc, double *C, double *lds)
{
    if (SMALL) d64_gemm(m, ld, alpha, A, B, acc, C, lds);
    else wg_gemm(m, ld, alpha, A, B, acc, C, lds);
}

template <bool SMALL>
__device__ __forceinline__ int wg_inverse(double *g, int m, int ld, double *lds)
{
    return SMALL ? d64_invert(g, m, ld, lds) : wg_invert(g, m, ld, lds);
}

__device__ __forceinline__ void flag_singular(const SysDesc &d, int elem) {
    if (threadIdx.x == 0) atomicCAS(&d.st->singular, 0, elem + 1);
}

template <bool COUPLED, bool SHJ, bool SMALL>
__device__ __forceinline__ void factor_a_body(const SysDesc *__restrict__ sysv,
                                              const Item *__restrict__ items, double *lds)
{
    const Item it = items[blockIdx.x];
    const SysDesc &d = sysv[it.sys];
    const int s = d.s, m = d.m, ld = d.ld;
    const int i = it.first, k = it.aux;
    const long long bs = (long long)m * ld;
    double *Pk = d.P64 + ((long long)i * s + k) * bs;
    const double *Jk = d.Jc + (SHJ ? 0 : (long long)k * d.nnzb * bs);
    const double *Mi = d.Mc + (long long)i * bs;
    const GAS int *diag_pos = gp(d.diag_pos), *row_ptr = gp(d.row_ptr), *col_idx = gp(d.col_idx),
                  *tpos = gp(d.tpos);
    const double *Jd = Jk + (long long)diag_pos[i] * bs;
    const double dk = d.dcoef[k], dt = d.dt;
    for (long long e = threadIdx.x; e < bs; e += NTHREADS) gp(Pk)[e] = dk * gp(Mi)[e] - dt * gp(Jd)[e];
    if (COUPLED) {
        // column k of the cross blocks: C_{lk,i} = A^{-1}_lk M_i (l != k)
        for (int l = 0; l < s; ++l) {
            if (l == k) continue;
            const int idx = l < k ? l : l - 1;
            double *Cl = d.C64 + (((long long)i * s + k) * (s - 1) + idx) * bs;
            const double al = d.Ainv[l * SMAX + k];
            for (long long e = threadIdx.x; e < bs; e += NTHREADS) gp(Cl)[e] = al * gp(Mi)[e];
        }
    }
    __syncthreads();
    double *X = d.Fscr + ((long long)i * s + k) * bs;
    const int p0 = row_ptr[i], pd = diag_pos[i];
    for (int p = p0; p < pd; ++p) {
        const long long j = col_idx[p];
        const double *Pinv_j = d.P64 + (j * s + k) * bs;
        blk_gemm<SMALL>(m, ld, 1.0, Pinv_j, Jk + (long long)tpos[p] * bs, false, X, lds);   // P_j^{-1} J_ji
        blk_gemm<SMALL>(m, ld, -dt * dt, Jk + (long long)p * bs, X, true, Pk, lds);           // -= dt^2 J_ij X
    }
    if (!COUPLED) {
        if (wg_inverse<SMALL>(Pk, m, ld, lds)) flag_singular(d, i);
    }
}

template <bool SHJ, bool SMALL>
__device__ __forceinline__ void factor_b_body(const SysDesc *__restrict__ sysv,
                                              const Item *__restrict__ items, double *lds)
{
    const Item it = items[blockIdx.x];
    const SysDesc &d = sysv[it.sys];
    const int s = d.s, m = d.m, ld = d.ld, sm1 = s - 1;
    const int i = it.first;
    const long long bs = (long long)m * ld;
    auto P = [&](int k) { return d.P64 + ((long long)i * s + k) * bs; };
    // C_{row,col}: column group col, index of row within it
    auto C = [&](int row, int col) {
        const int idx = row < col ? row : row - 1;
        return d.C64 + (((long long)i * s + col) * sm1 + idx) * bs;
    };
    double *L = d.Fscr + ((long long)i * s) * bs;
    double *X = d.Fscr + ((long long)i * s + 1) * bs;
    const double *Mi = d.Mc + (long long)i * bs;
    for (int k = 0; k < s; ++k) {
        if (wg_inverse<SMALL>(P(k), m, ld, lds)) flag_singular(d, i);
        if (k == 0) {
            // every cross block is still A^{-1}_kl M_i: with X = M_i P_0^{-1} M_i,
            //   P_l  -= A^{-1}_l0 A^{-1}_0l X,   C_lq -= A^{-1}_l0 A^{-1}_0q X
            blk_gemm<SMALL>(m, ld, 1.0, Mi, P(0), false, L, lds);
            blk_gemm<SMALL>(m, ld, 1.0, L, Mi, false, X, lds);
            for (int l = 1; l < s; ++l)
                for (int q = 1; q < s; ++q) {
                    double *D = (q == l) ? P(l) : C(l, q);
                    const double f = d.Ainv[l * SMAX + 0] * d.Ainv[0 * SMAX + q];
                    for (long long e = threadIdx.x; e < bs; e += NTHREADS) gp(D)[e] -= f * gp(X)[e];
                }
            __syncthreads();
            continue;
        }
        for (int l = k + 1; l < s; ++l) {
            blk_gemm<SMALL>(m, ld, 1.0, C(l, k), P(k), false, L, lds);          // L = C_lk P_k^{-1}
            blk_gemm<SMALL>(m, ld, -1.0, L, C(k, l), true, P(l), lds);          // P_l -= L C_kl
            for (int q = k + 1; q < s; ++q) {
                if (q == l) continue;
                blk_gemm<SMALL>(m, ld, -1.0, L, C(k, q), true, C(l, q), lds);   // C_lq -= L C_kq
            }
        }
    }
}

// Kernels: blocks of order <= 64 ask for four waves per SIMD (the products
// run out of line, so the bodies fit 128 VGPRs); larger blocks keep the
// default budget of the LDS-tiled routines.
template <bool COUPLED, bool SHJ>
__global__ __launch_bounds__(NTHREADS, 4) void k_factor_a64(const SysDesc *__restrict__ sysv,
                                                          const Item *__restrict__ items)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    factor_a_body<COUPLED, SHJ, true>(sysv, items, reinterpret_cast<double *>(smem_raw));
}
template <bool COUPLED, bool SHJ>
__global__ __launch_bounds__(NTHREADS) void k_factor_a(const SysDesc *__restrict__ sysv,
                                                       const Item *__restrict__ items)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    factor_a_body<COUPLED, SHJ, false>(sysv, items, reinterpret_cast<double *>(smem_raw));
}
template <bool SHJ>
__global__ __launch_bounds__(NTHREADS, 4) void k_factor_b64(const SysDesc *__restrict__ sysv,
                                                          const Item *__restrict__ items)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    factor_b_body<SHJ, true>(sysv, items, reinterpret_cast<double *>(smem_raw));
}
template <bool SHJ>
__global__ __launch_bounds__(NTHREADS) void k_factor_b(const SysDesc *__restrict__ sysv,
                                                       const Item *__restrict__ items)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    factor_b_body<SHJ, false>(sysv, items, reinterpret_cast<double *>(smem_raw));
}

template <bool SMALL>
static void launch_factor_t(int phase, const SysDesc *dsys, const Item *items, int nitems, bool coupled,
                            bool sharedJ, size_t shmem, hipStream_t st)
{
    dim3 grid(nitems), block(NTHREADS);
#define FA(C, SH)                                                                                 \
    do {                                                                                          \
        if (SMALL) hipLaunchKernelGGL((k_factor_a64<C, SH>), grid, block, shmem, st, dsys, items); \
        else hipLaunchKernelGGL((k_factor_a<C, SH>), grid, block, shmem, st, dsys, items);        \
    } while (0)
#define FB(SH)                                                                                    \
    do {                                                                                          \
        if (SMALL) hipLaunchKernelGGL((k_factor_b64<SH>), grid, block, shmem, st, dsys, items);    \
        else hipLaunchKernelGGL((k_factor_b<SH>), grid, block, shmem, st, dsys, items);           \
    } while (0)
    if (phase == 0) {
        if (coupled) { if (sharedJ) FA(true, true); else FA(true, false); }
        else { if (sharedJ) FA(false, true); else FA(false, false); }
    } else {
        if (sharedJ) FB(true); else FB(false);
    }
#undef FA
#undef FB
}

void launch_factor(int phase, const SysDesc *dsys, const Item *items, int nitems, bool coupled,
                   bool sharedJ, bool small, size_t shmem, hipStream_t st)
{
    if (small) launch_factor_t<true>(phase, dsys, items, nitems, coupled, sharedJ, shmem, st);
    else launch_factor_t<false>(phase, dsys, items, nitems, coupled, sharedJ, shmem, st);
}

// Allow the factor kernels the LDS they need for m up to MMAX.
void factor_set_lds_limit(size_t bytes)
{
    const int b = (int)bytes;
    const void *k[] = {
        (const void *)k_factor_a<true, true>, (const void *)k_factor_a<true, false>,
        (const void *)k_factor_a<false, true>, (const void *)k_factor_a<false, false>,
        (const void *)k_factor_a64<true, true>, (const void *)k_factor_a64<true, false>,
        (const void *)k_factor_a64<false, true>, (const void *)k_factor_a64<false, false>,
        (const void *)k_factor_b<true>, (const void *)k_factor_b<false>,
        (const void *)k_factor_b64<true>, (const void *)k_factor_b64<false>};
    for (const void *f : k) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, b);
}

// ---------------------------------------------------------------------------
// relayout: row-major FP64 blocks -> column-major blocks (leading dimension
// ld, zero padding rows) in FP64 or FP32.  One workgroup per block, 32 x 32
// tiles through LDS so both the read and the write are coalesced.
// ---------------------------------------------------------------------------
template <typename TO>
__global__ __launch_bounds__(NTHREADS) void k_relayout(const double *__restrict__ src,
                                                       TO *__restrict__ dst, int m, int ld)
{
    __shared__ double tile[32][33];
    const long long b = blockIdx.x;
    const double *S = src + b * (long long)m * m;
    TO *D = dst + b * (long long)m * ld;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int r0 = 0; r0 < ld; r0 += 32) {
        for (int c0 = 0; c0 < m; c0 += 32) {
            for (int q = ty; q < 32; q += 8) {
                const int r = r0 + q, c = c0 + tx;
                tile[q][tx] = (r < m && c < m) ? S[(long long)r * m + c] : 0.0;
            }
            __syncthreads();
            for (int q = ty; q < 32; q += 8) {
                const int c = c0 + q, r = r0 + tx;
                if (c < m && r < ld) D[(long long)c * ld + r] = (TO)tile[tx][q];
            }
            __syncthreads();
        }
    }
}

void launch_relayout(const double *src, void *dst, int dst_type, long long nblk, int m, int ld,
                     hipStream_t st)
{
    if (nblk <= 0) return;
    dim3 grid((unsigned)nblk), block(NTHREADS);
    if (dst_type == 0)
        hipLaunchKernelGGL(k_relayout<double>, grid, block, 0, st, src, (double *)dst, m, ld);
    else
        hipLaunchKernelGGL(k_relayout<float>, grid, block, 0, st, src, (float *)dst, m, ld);
}

// ---------------------------------------------------------------------------
// quantization of the FP64 factor blocks (column-major, ld) into the sweep
// format.  FP16S: per-block exponent e with |x|_max in [2^(E-1), 2^E) and
// e = 14 - E (clamped to [-100, 100]); stored value fp16(fp32(x * 2^e)).
// ---------------------------------------------------------------------------
template <int FT>
__global__ __launch_bounds__(NTHREADS) void k_quantize(const double *__restrict__ src,
                                                       void *__restrict__ dst, int *__restrict__ ex,
                                                       int m, int ld, int ldq)
{
    __shared__ double red[NTHREADS / 64];
    const long long b = blockIdx.x;
    const double *S = src + b * (long long)m * ld;
    int e = 0;
    if (FT == FT_F16S) {
        double amax = 0.0;
        for (int q = threadIdx.x; q < m * m; q += NTHREADS) {
            const int c = q / m, r = q - c * m;
            amax = fmax(amax, fabs(S[(long long)c * ld + r]));
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = amax;
        __syncthreads();
        amax = red[0];
        for (int w = 1; w < NTHREADS / 64; ++w) amax = fmax(amax, red[w]);
        if (amax > 0.0 && isfinite(amax)) {
            int E;
            frexp(amax, &E);
            e = 14 - E;
            e = e < -100 ? -100 : (e > 100 ? 100 : e);
        }
        if (threadIdx.x == 0) ex[b] = e;
    }
    for (int q = threadIdx.x; q < m * ldq; q += NTHREADS) {
        const int c = q / ldq, r = q - c * ldq;
        const double x = (r < m) ? S[(long long)c * ld + r] : 0.0;
        const long long o = b * (long long)m * ldq + q;
        if (FT == FT_F32) reinterpret_cast<float *>(dst)[o] = (float)x;
        else if (FT == FT_BF16) reinterpret_cast<uint16_t *>(dst)[o] = f32_to_bf16_rne((float)x);
        else reinterpret_cast<uint16_t *>(dst)[o] = f32_to_f16_rne((float)ldexp(x, e));
    }
}

void quantize_blocks(const double *src, void *dst, int *ex, long long nblk, int m, int ld,
                     int ldq, int ftype, hipStream_t st)
{
    if (nblk <= 0) return;
    dim3 grid((unsigned)nblk), block(NTHREADS);
    if (ftype == FT_F32) hipLaunchKernelGGL(k_quantize<FT_F32>, grid, block, 0, st, src, dst, ex, m, ld, ldq);
    else if (ftype == FT_BF16) hipLaunchKernelGGL(k_quantize<FT_BF16>, grid, block, 0, st, src, dst, ex, m, ld, ldq);
    else hipLaunchKernelGGL(k_quantize<FT_F16S>, grid, block, 0, st, src, dst, ex, m, ld, ldq);
}

void launch_quantize(const SysDesc *dsys, const SysDesc &h, int ftype, hipStream_t st)
{
    (void)dsys;
    const long long np = (long long)h.T * h.s;
    const long long nc = (h.C64 != nullptr) ? (long long)h.T * h.s * (h.s - 1) : 0;
    if (ftype == FT_F32) {
        quantize_blocks(h.P64, h.P32, nullptr, np, h.m, h.ld, h.ld32, ftype, st);
        if (nc) quantize_blocks(h.C64, h.C32, nullptr, nc, h.m, h.ld, h.ld32, ftype, st);
    } else {
        quantize_blocks(h.P64, h.P16, h.P16e, np, h.m, h.ld, h.ld16, ftype, st);
        if (nc) quantize_blocks(h.C64, h.C16, h.C16e, nc, h.m, h.ld, h.ld16, ftype, st);
    }
}

// ---------------------------------------------------------------------------
// export of the FP64 factors to the caller's layout (row-major blocks):
// pinv [s][T][m][m], cross [s][s][T][m][m] (C_{kl,i} at (k, l, i)).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NTHREADS) void k_export(const double *__restrict__ src, double *dst,
                                                     int s, int T, int m, int ld, int cross)
{
    const long long b = blockIdx.x;   // source block index
    long long o;
    if (!cross) {
        const long long i = b / s, k = b - i * s;
        o = (k * T + i) * (long long)m * m;
    } else {
        const int sm1 = s - 1;
        const long long ik = b / sm1;
        const int idx = (int)(b - ik * sm1);
        const long long i = ik / s;
        const int col = (int)(ik - i * s);
        const int row = idx < col ? idx : idx + 1;
        o = (((long long)row * s + col) * T + i) * (long long)m * m;
    }
    const double *S = src + b * (long long)m * ld;
    for (int e = threadIdx.x; e < m * m; e += NTHREADS) {
        const int r = e / m, c = e - r * m;
        dst[o + e] = S[(long long)c * ld + r];
    }
}

void launch_export(const SysDesc &h, double *pinv, double *cross, hipStream_t st)
{
    if (pinv)
        hipLaunchKernelGGL(k_export, dim3((unsigned)((long long)h.T * h.s)), dim3(NTHREADS), 0, st,
                           (const double *)h.P64, pinv, h.s, h.T, h.m, h.ld, 0);
    if (cross && h.C64 && h.s > 1)
        hipLaunchKernelGGL(k_export, dim3((unsigned)((long long)h.T * h.s * (h.s - 1))), dim3(NTHREADS),
                           0, st, (const double *)h.C64, cross, h.s, h.T, h.m, h.ld, 1);
}

}  // namespace irk
