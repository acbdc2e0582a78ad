// dense64.h -- dense FP64 block kernels for blocks of order m <= 64, run by
// one 256-thread workgroup (four waves):
//
//   * d64_gemm: C = alpha A B (+ C) for column-major blocks on the FP64
//     matrix cores (v_mfma_f64_16x16x4f64).  Both operands are staged in
//     LDS; each wave owns a 32 x 32 quadrant of the 64 x 64 output (2 x 2
//     tiles of 16 x 16), so a K step costs every wave two A and two B
//     fragment loads for four matrix instructions.
//   * d64_invert: in-place Gauss-Jordan inversion with partial pivoting.
//     Lane r of wave w keeps row r, columns 16w .. 16w+15 in registers.  The
//     wave that owns the pivot column compares every unused row against the
//     first unused one with a single wave vote and searches the column only
//     when some row is larger, so the chosen pivot is the largest entry
//     (first of equals) as in ordinary partial pivoting.  Rows are never
//     moved; the row and column permutations are undone when the inverse is
//     written back.
#pragma once
#include "irk_device.h"

namespace irk {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int D64_LDA = 64;                 // As[k * 64 + i] = A(i, k)
constexpr int D64_LDB = 65;                 // Bs[j * 65 + k] = B(k, j): odd stride, conflict-free
constexpr int D64_LDS_DOUBLES = 64 * D64_LDA + 64 * D64_LDB;

// Fragment layouts of v_mfma_f64_16x16x4f64 (checked on gfx950): lane l
// supplies A(l % 16, l / 16) and B(l / 16, l % 16); element r of the result
// in lane l is D(4 r + l / 16, l % 16).
__device__ __forceinline__ int d64_frag_row(int lane, int r) { return 4 * r + (lane >> 4); }
__device__ __forceinline__ int d64_frag_col(int lane) { return lane & 15; }

// A (m x m, column-major, leading dimension ld) -> As, zero outside m x m.
// All eight 16-byte loads of a thread are issued before the first LDS write
// (addresses are clamped into the block, values outside m masked).
__device__ __forceinline__ void d64_stage_a(double *As, const double *gA, int m, int ld)
{
    const GAS double *A = gp(gA);
    dbl2 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int e = threadIdx.x + q * NTHREADS;
        const int k = e >> 5, i = (e & 31) * 2;
        v[q] = *reinterpret_cast<const GAS dbl2 *>(A + (size_t)min(k, m - 1) * ld + min(i, ld - 2));
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int e = threadIdx.x + q * NTHREADS;
        const int k = e >> 5, i = (e & 31) * 2;
        dbl2 x = v[q];
        if (k >= m || i >= m) x.x = 0.0;
        if (k >= m || i + 1 >= m) x.y = 0.0;
        *reinterpret_cast<dbl2 *>(As + k * D64_LDA + i) = x;
    }
}

// B (m x m, column-major) -> Bs, zero outside m x m.
__device__ __forceinline__ void d64_stage_b(double *Bs, const double *gB, int m, int ld)
{
    const GAS double *B = gp(gB);
    dbl2 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int e = threadIdx.x + q * NTHREADS;
        const int j = e >> 5, k = (e & 31) * 2;
        v[q] = *reinterpret_cast<const GAS dbl2 *>(B + (size_t)min(j, m - 1) * ld + min(k, ld - 2));
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int e = threadIdx.x + q * NTHREADS;
        const int j = e >> 5, k = (e & 31) * 2;
        const double x0 = (j < m && k < m) ? v[q].x : 0.0;
        const double x1 = (j < m && k + 1 < m) ? v[q].y : 0.0;
        Bs[j * D64_LDB + k] = x0;
        Bs[j * D64_LDB + k + 1] = x1;
    }
}

// acc += this wave's quadrant of As * Bs over k < m (rounded up to 4).  The
// fragments of the next K step are loaded while the current one multiplies.
__device__ __forceinline__ void d64_mma(const double *As, const double *Bs, int m, dbl4 (&acc)[2][2])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int qi = w & 1, qj = w >> 1;
    const int r = lane & 15, kq = lane >> 4;
    const double *ap = As + kq * D64_LDA + 32 * qi + r;
    const double *bp = Bs + (32 * qj + r) * D64_LDB + kq;
    const int nk = (m + 3) >> 2;
    double a0 = ap[0], a1 = ap[16], b0 = bp[0], b1 = bp[16 * D64_LDB];
    for (int kc = 0; kc < nk; ++kc) {
        const int kn = min(kc + 1, nk - 1);
        const double na0 = ap[kn * 4 * D64_LDA], na1 = ap[kn * 4 * D64_LDA + 16];
        const double nb0 = bp[kn * 4], nb1 = bp[kn * 4 + 16 * D64_LDB];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        a0 = na0; a1 = na1; b0 = nb0; b1 = nb1;
    }
}

__device__ __forceinline__ void d64_zero(dbl4 (&acc)[2][2])
{
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
}

// C = alpha acc (+ C when add) for rows and columns below m.  The old
// values are all loaded before the first store.
__device__ __forceinline__ void d64_store(double *gC, int m, int ld, double alpha, bool add,
                                          const dbl4 (&acc)[2][2])
{
    GAS double *C = gp(gC);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int qi = w & 1, qj = w >> 1;
    double old[2][2][4];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = 32 * qj + 16 * y + d64_frag_col(lane);
                const int i = 32 * qi + 16 * x + d64_frag_row(lane, r);
                old[x][y][r] = 0.0;
                if (add && i < m && j < m) old[x][y][r] = C[(size_t)j * ld + i];
            }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = 32 * qj + 16 * y + d64_frag_col(lane);
                const int i = 32 * qi + 16 * x + d64_frag_row(lane, r);
                if (i < m && j < m) C[(size_t)j * ld + i] = fma(alpha, acc[x][y][r], old[x][y][r]);
            }
}

// C = alpha A B (+ C when add); blocks m x m column-major with leading
// dimension ld; C must not overlap A or B.  LDS: D64_LDS_DOUBLES doubles.
__device__ __forceinline__ void d64_gemm(int m, int ld, double alpha, const double *A, const double *B,
                                         bool add, double *C, double *lds)
{
    double *As = lds, *Bs = lds + 64 * D64_LDA;
    d64_stage_a(As, A, m, ld);
    d64_stage_b(Bs, B, m, ld);
    __syncthreads();
    dbl4 acc[2][2];
    d64_zero(acc);
    d64_mma(As, Bs, m, acc);
    d64_store(C, m, ld, alpha, add, acc);
    __syncthreads();
}

__device__ __forceinline__ double d64_readlane(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// In-place inverse of the m x m block at gptr.  The memory image is handled
// as the row-major matrix Q = P^T (row stride ld); writing Q^{-1} back the
// same way leaves P^{-1} in column-major order.  Returns nonzero (in every
// thread) when a pivot is zero or a pivot column holds a non-finite value.
//
// Pivot rows are not scaled when they are used: a row that served as pivot
// with value piv is stored as piv times its Gauss-Jordan value (the update
// of every other row is the same either way), and the scale is removed when
// the result is written back.  Step c: the wave owning column c picks the
// pivot row p and publishes the column, p and 1/piv through LDS; after one
// barrier every wave updates its 16 columns from row p (read with
// v_readlane) and the column multipliers.
// LDS: 2 * 64 + 2 + 64 * 64 doubles + 132 ints.
__device__ __forceinline__ int d64_invert(double *gptr, int m, int ld, double *lds)
{
    GAS double *g = gp(gptr);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double *colbuf = lds;                                          // [2][64] pivot columns
    double *pinvbuf = lds + 128;                                   // [2] 1 / pivot
    double *stage = lds + 130;                                     // [64][64] permuted result
    int *pbuf = reinterpret_cast<int *>(lds + 130 + 64 * 64);      // [2] pivot row (+ flag)
    int *step_of_row = pbuf + 2;                                   // [64]
    int *row_of_step = pbuf + 66;                                  // [64]
    double a[16];
    {
        const GAS double *src = g + (size_t)lane * ld + 16 * w;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int c = 16 * w + j;
            a[j] = (lane < m && c < m) ? src[j] : (lane == c ? 1.0 : 0.0);
        }
    }
    unsigned long long unused = (m >= 64) ? ~0ull : ((1ull << m) - 1ull);
    double myscale = 1.0;           // pivot value of this lane's row once it has been used
    int bad = 0;
    for (int wc = 0; wc < 4; ++wc) {
        if (16 * wc >= m) break;
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) {
            const int c = 16 * wc + cc;
            if (c >= m) continue;           // uniform: every thread skips the same steps
            const int par = c & 1;
            if (w == wc) {
                const double v = a[cc];
                const int n = __builtin_ctzll(unused);
                const double vn = d64_readlane(v, n);
                const bool mine = (unused >> lane) & 1ull;
                const bool big = __any(mine && fabs(v) > fabs(vn));
                const bool nonfin = __any(mine && !isfinite(v));
                int p = n;
                double piv = vn;
                if (big) {
                    double best = mine ? fabs(v) : -1.0;
                    int bi = mine ? lane : 64;
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) {
                        const double ob = __shfl_xor(best, o);
                        const int oi = __shfl_xor(bi, o);
                        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
                    }
                    p = __builtin_amdgcn_readfirstlane(bi);
                    if (p < 0 || p >= 64 || !((unused >> p) & 1ull)) p = n;
                    piv = d64_readlane(v, p);
                }
                colbuf[par * 64 + lane] = v;
                if (lane == 0) {
                    pbuf[par] = p | ((nonfin || !(fabs(piv) > 0.0) || !isfinite(piv)) ? 0x100 : 0);
                    pinvbuf[par] = 1.0 / piv;
                }
            }
            __syncthreads();
            const int pw = __builtin_amdgcn_readfirstlane(pbuf[par]);
            const double pinv = pinvbuf[par];
            const double f = colbuf[par * 64 + lane];
            const int p = pw & 0xff;
            bad |= pw >> 8;
            const bool isp = (lane == p);
            const double gm = isp ? 0.0 : f * pinv;
            if (isp) myscale = f;
#pragma unroll
            for (int j = 0; j < 16; ++j) a[j] = fma(-gm, d64_readlane(a[j], p), a[j]);
            if (w == wc) a[cc] = isp ? 1.0 : -gm;
            unused &= ~(1ull << p);
            if (threadIdx.x == 0) { step_of_row[p] = c; row_of_step[c] = p; }
        }
    }
    __syncthreads();
    // element (r, c) of the result is Q^{-1}(step(r), row(c)) times the scale of row r
    if (lane < m) {
        const int row = step_of_row[lane];
        const double sc = 1.0 / myscale;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int c = 16 * w + j;
            if (c < m) stage[row * 64 + row_of_step[c]] = a[j] * sc;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m * 64; e += NTHREADS) {
        const int r = e >> 6, c = e & 63;
        if (c < m) g[(size_t)r * ld + c] = stage[e];
    }
    __syncthreads();
    return bad;
}

}  // namespace irk
