// dense64.h -- dense FP64 block kernels for blocks of order m <= 64, run by
// one 256-thread workgroup (four waves):
//
//   * d64_gemm: C = alpha A B (+ C) for column-major blocks on the FP64
//     matrix cores (v_mfma_f64_16x16x4f64).  Each wave owns a 32 x 32
//     quadrant of the 64 x 64 output (2 x 2 tiles of 16 x 16); the operands
//     pass through LDS in K panels of 32, so a K step costs every wave two A
//     and two B fragment loads for four matrix instructions.
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

constexpr int D64_LDS_DOUBLES = 4352;       // the larger of the inversion (4291) and product (4160) needs

// Fragment layouts of v_mfma_f64_16x16x4f64 (checked on gfx950): lane l
// supplies A(l % 16, l / 16) and B(l / 16, l % 16); element r of the result
// in lane l is D(4 r + l / 16, l % 16).
__device__ __forceinline__ int d64_frag_row(int lane, int r) { return 4 * r + (lane >> 4); }
__device__ __forceinline__ int d64_frag_col(int lane) { return lane & 15; }


// K panels of 32: A(:, k0:k0+32) -> As[kk * 64 + i] and B(k0:k0+32, :) ->
// Bs[j * 33 + kk] (odd stride: conflict-free fragment reads), zero outside
// m.  Each thread moves four 16-byte pieces of each operand per panel, all
// loads issued before the first LDS write.
constexpr int D64_KP = 32;
constexpr int D64_LDB = 33;

__device__ __forceinline__ void d64_stage_panel(double *As, double *Bs, const GAS double *A,
                                                const GAS double *B, int m, int ld, int k0)
{
    dbl2 ra[4], rb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + q * NTHREADS;        // 0 .. 1023
        const int kk = e >> 5, i = (e & 31) * 2;         // A: column k0+kk, rows i, i+1
        ra[q] = *reinterpret_cast<const GAS dbl2 *>(A + (size_t)min(k0 + kk, m - 1) * ld + min(i, ld - 2));
        const int j = e >> 4, kb = (e & 15) * 2;         // B: column j, rows k0+kb, +1
        rb[q] = *reinterpret_cast<const GAS dbl2 *>(B + (size_t)min(j, m - 1) * ld + min(k0 + kb, ld - 2));
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + q * NTHREADS;
        const int kk = e >> 5, i = (e & 31) * 2;
        dbl2 x = ra[q];
        if (k0 + kk >= m || i >= m) x.x = 0.0;
        if (k0 + kk >= m || i + 1 >= m) x.y = 0.0;
        *reinterpret_cast<dbl2 *>(As + kk * 64 + i) = x;
        const int j = e >> 4, kb = (e & 15) * 2;
        Bs[j * D64_LDB + kb] = (j < m && k0 + kb < m) ? rb[q].x : 0.0;
        Bs[j * D64_LDB + kb + 1] = (j < m && k0 + kb + 1 < m) ? rb[q].y : 0.0;
    }
}

// acc += this wave's quadrant of one K panel (nkc steps of 4).
__device__ __forceinline__ void d64_mma_panel(const double *As, const double *Bs, int nkc, dbl4 (&acc)[2][2])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int qi = w & 1, qj = w >> 1;
    const int r = lane & 15, kq = lane >> 4;
    const double *ap = As + kq * 64 + 32 * qi + r;
    const double *bp = Bs + (32 * qj + r) * D64_LDB + kq;
#pragma unroll 2
    for (int kc = 0; kc < nkc; ++kc) {
        const double a0 = ap[kc * 4 * 64], a1 = ap[kc * 4 * 64 + 16];
        const double b0 = bp[kc * 4], b1 = bp[kc * 4 + 16 * D64_LDB];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
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
// dimension ld; C must not overlap A or B.  The operands pass through LDS in
// K panels of 32 (33 KB).  Not inlined: one body serves every call site of a
// kernel, which keeps the kernels' register demand (and so their occupancy)
// at the level of the product itself.
__device__ __noinline__ void d64_gemm(int m, int ld, double alpha, const double *gA, const double *gB,
                                      bool add, double *C, double *lds)
{
    const GAS double *A = gp(gA);
    const GAS double *B = gp(gB);
    double *As = lds, *Bs = lds + 64 * D64_KP;
    dbl4 acc[2][2];
    d64_zero(acc);
    for (int k0 = 0; k0 < m; k0 += D64_KP) {
        d64_stage_panel(As, Bs, A, B, m, ld, k0);
        __syncthreads();
        d64_mma_panel(As, Bs, (min(m - k0, D64_KP) + 3) >> 2, acc);
        __syncthreads();
    }
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

// ---------------------------------------------------------------------------
// C = alpha A B (+ C when add) for column-major blocks of order 64 < m <= 160
// on the FP64 matrix cores.  The 16 x 16 output tiles (NT = ceil(m/16) per
// side) are split into four quadrants, one per wave (at most 5 x 5 tiles, 25
// accumulators of four doubles).  K runs in panels of 16: A(:, panel) ->
// Am[kk][i] (row stride 160) and B(panel, :) -> Bm[j][kk] (stride 17, odd:
// conflict-free fragment reads); the next panel's loads are issued before the
// current panel is multiplied.  LDS: 16 * 160 + 160 * 17 doubles.
// ---------------------------------------------------------------------------
constexpr int DM_AP = 160, DM_BP = 17, DM_KP = 16;
constexpr int DM_LDS_DOUBLES = DM_KP * DM_AP + DM_AP * DM_BP;

__device__ __forceinline__ void dm_load_panel(const GAS double *A, const GAS double *B, int m, int ld,
                                              int k0, dbl2 (&ra)[5], dbl2 (&rb)[5])
{
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int e = threadIdx.x + q * NTHREADS;        // 0 .. 1279
        const int kk = e / 80, i = (e - kk * 80) * 2;     // A: column k0+kk, rows i, i+1
        ra[q] = *reinterpret_cast<const GAS dbl2 *>(A + (size_t)min(k0 + kk, m - 1) * ld + min(i, ld - 2));
        const int j = e >> 3, kb = (e & 7) * 2;           // B: column j, rows k0+kb, +1
        rb[q] = *reinterpret_cast<const GAS dbl2 *>(B + (size_t)min(j, m - 1) * ld + min(k0 + kb, ld - 2));
    }
}

__device__ __forceinline__ void dm_put_panel(double *Am, double *Bm, int m, int k0, const dbl2 (&ra)[5],
                                             const dbl2 (&rb)[5])
{
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int e = threadIdx.x + q * NTHREADS;
        const int kk = e / 80, i = (e - kk * 80) * 2;
        Am[kk * DM_AP + i] = (k0 + kk < m && i < m) ? ra[q].x : 0.0;
        Am[kk * DM_AP + i + 1] = (k0 + kk < m && i + 1 < m) ? ra[q].y : 0.0;
        const int j = e >> 3, kb = (e & 7) * 2;
        Bm[j * DM_BP + kb] = (j < m && k0 + kb < m) ? rb[q].x : 0.0;
        Bm[j * DM_BP + kb + 1] = (j < m && k0 + kb + 1 < m) ? rb[q].y : 0.0;
    }
}

__device__ __forceinline__ void dm_gemm(int m, int ld, double alpha, const double *gA, const double *gB,
                                     bool add, double *gC, double *lds)
{
    const GAS double *A = gp(gA);
    const GAS double *B = gp(gB);
    GAS double *C = gp(gC);
    double *Am = lds, *Bm = lds + DM_KP * DM_AP;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, kq = lane >> 4;
    const int NT = (m + 15) >> 4, H = (NT + 1) >> 1;
    const int ti0 = (w & 1) * H, tj0 = (w >> 1) * H;
    const int TI = min(H, NT - ti0), TJ = min(H, NT - tj0);
    dbl4 acc[5][5];
#pragma unroll
    for (int x = 0; x < 5; ++x)
#pragma unroll
        for (int y = 0; y < 5; ++y) acc[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
    dbl2 ra[5], rb[5];
    dm_load_panel(A, B, m, ld, 0, ra, rb);
    for (int k0 = 0; k0 < m; k0 += DM_KP) {
        __syncthreads();                                  // previous panel fully read
        dm_put_panel(Am, Bm, m, k0, ra, rb);
        if (k0 + DM_KP < m) dm_load_panel(A, B, m, ld, k0 + DM_KP, ra, rb);
        __syncthreads();
#pragma unroll
        for (int kc = 0; kc < DM_KP / 4; ++kc) {
            double a[5], b[5];
#pragma unroll
            for (int x = 0; x < 5; ++x) a[x] = Am[(4 * kc + kq) * DM_AP + 16 * (ti0 + min(x, TI - 1)) + r];
#pragma unroll
            for (int y = 0; y < 5; ++y) b[y] = Bm[(16 * (tj0 + min(y, TJ - 1)) + r) * DM_BP + 4 * kc + kq];
#pragma unroll
            for (int x = 0; x < 5; ++x)
#pragma unroll
                for (int y = 0; y < 5; ++y)
                    if (x < TI && y < TJ)
                        acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
        }
    }
    // store (old values first when accumulating)
#pragma unroll
    for (int x = 0; x < 5; ++x)
#pragma unroll
        for (int y = 0; y < 5; ++y) {
            if (x >= TI || y >= TJ) continue;
            const int j = 16 * (tj0 + y) + d64_frag_col(lane);
            double o[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 16 * (ti0 + x) + d64_frag_row(lane, q);
                o[q] = (add && i < m && j < m) ? C[(size_t)j * ld + i] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 16 * (ti0 + x) + d64_frag_row(lane, q);
                if (i < m && j < m) C[(size_t)j * ld + i] = fma(alpha, acc[x][y][q], o[q]);
            }
        }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// In-place inverse for 64 < m <= 160 (same contract as d64_invert): lane l of
// wave w keeps rows l, l + 64, l + 128 and columns 40w .. 40w + 39 in
// registers (120 values).  Step c: the owner wave of column c picks the
// pivot (wave vote against the first unused row, full search only when a
// larger entry exists), publishes the column, p and 1/piv through LDS; after
// one barrier every wave takes the pivot row's values for its own columns
// from the lane that holds them (through a wave-private LDS row, no barrier)
// and updates its columns.  Pivot rows keep a deferred scale.  The result is
// written straight to global memory with the row and column permutations
// undone.  LDS: 2 * 160 + 2 + 4 * 40 doubles and 2 + 2 * 160 ints.
// ---------------------------------------------------------------------------
constexpr int DMI_LDS_DOUBLES = 2 * 160 + 2 + 4 * 40 + 162;

__device__ __forceinline__ double dm_pick3(const double (&v)[3], int g)
{
    return g == 0 ? v[0] : (g == 1 ? v[1] : v[2]);
}

__device__ __forceinline__ int dm_invert(double *gptr, int m, int ld, double *lds)
{
    GAS double *gm_ = gp(gptr);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double *colbuf = lds;                                   // [2][160]
    double *pinvbuf = lds + 320;                            // [2]
    double *rowbuf = lds + 322 + 40 * w;                    // [40] this wave's pivot-row values
    int *pbuf = reinterpret_cast<int *>(lds + 322 + 160);   // [2]
    int *step_of_row = pbuf + 2;                            // [160]
    int *row_of_step = pbuf + 162;                          // [160]
    double a[3][40];
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        const int row = lane + 64 * g;
#pragma unroll
        for (int j = 0; j < 40; ++j) {
            const int c = 40 * w + j;
            a[g][j] = (row < m && c < m) ? gm_[(size_t)row * ld + c] : (row == c ? 1.0 : 0.0);
        }
    }
    unsigned long long un[3];
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        const int lo = 64 * g;
        un[g] = (m <= lo) ? 0ull : (m - lo >= 64 ? ~0ull : ((1ull << (m - lo)) - 1ull));
    }
    double myscale[3] = {1.0, 1.0, 1.0};
    int bad = 0;
    for (int wc = 0; wc < 4; ++wc) {
        if (40 * wc >= m) break;
#pragma unroll
        for (int cc = 0; cc < 40; ++cc) {
            const int c = 40 * wc + cc;
            if (c >= m) continue;
            const int par = c & 1;
            if (w == wc) {
                const double v[3] = {a[0][cc], a[1][cc], a[2][cc]};
                bool mine[3];
#pragma unroll
                for (int g = 0; g < 3; ++g) mine[g] = (un[g] >> lane) & 1ull;
                const int ng = un[0] ? 0 : (un[1] ? 1 : 2);
                const int n = 64 * ng + __builtin_ctzll(un[ng]);
                const double vn = d64_readlane(dm_pick3(v, ng), n & 63);
                bool big = false, nonfin = false;
#pragma unroll
                for (int g = 0; g < 3; ++g) {
                    big |= mine[g] && fabs(v[g]) > fabs(vn);
                    nonfin |= mine[g] && !isfinite(v[g]);
                }
                const bool anybig = __any(big), anynf = __any(nonfin);
                int p = n;
                if (anybig) {
                    double best = -1.0;
                    int bi = 1 << 20;
#pragma unroll
                    for (int g = 0; g < 3; ++g)
                        if (mine[g] && fabs(v[g]) > best) { best = fabs(v[g]); bi = lane + 64 * g; }
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) {
                        const double ob = __shfl_xor(best, o);
                        const int oi = __shfl_xor(bi, o);
                        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
                    }
                    p = __builtin_amdgcn_readfirstlane(bi);
                    if (p < 0 || p >= m || !((un[p >> 6] >> (p & 63)) & 1ull)) p = n;
                }
                const double piv = d64_readlane(dm_pick3(v, p >> 6), p & 63);
#pragma unroll
                for (int g = 0; g < 3; ++g)
                    if (lane + 64 * g < 160) colbuf[par * 160 + lane + 64 * g] = v[g];
                if (lane == 0) {
                    pbuf[par] = p | ((anynf || !(fabs(piv) > 0.0) || !isfinite(piv)) ? 0x1000 : 0);
                    pinvbuf[par] = 1.0 / piv;
                }
            }
            __syncthreads();
            const int pw = __builtin_amdgcn_readfirstlane(pbuf[par]);
            const int p = pw & 0xfff;
            if (pw & 0x1000) bad = 1;
            const double pinv = pinvbuf[par];
            const int pg = p >> 6, pl = p & 63;
            // the pivot row's values of this wave's columns, from lane pl
            if (lane == pl) {
#pragma unroll
                for (int j = 0; j < 40; ++j) rowbuf[j] = pg == 0 ? a[0][j] : (pg == 1 ? a[1][j] : a[2][j]);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            double gmul[3];
#pragma unroll
            for (int g = 0; g < 3; ++g) {
                const int row = lane + 64 * g;
                const double f = (row < 160) ? colbuf[par * 160 + row] : 0.0;
                const bool isp = (row == p);
                gmul[g] = isp ? 0.0 : f * pinv;
                if (isp) myscale[g] = f;
            }
#pragma unroll
            for (int j = 0; j < 40; ++j) {
                const double pr = rowbuf[j];
#pragma unroll
                for (int g = 0; g < 3; ++g) a[g][j] = fma(-gmul[g], pr, a[g][j]);
            }
            if (w == wc) {
#pragma unroll
                for (int g = 0; g < 3; ++g) a[g][cc] = (lane + 64 * g == p) ? 1.0 : -gmul[g];
            }
            un[pg] &= ~(1ull << pl);
            if (threadIdx.x == 0) { step_of_row[p] = c; row_of_step[c] = p; }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();   // rowbuf is rewritten next step
        }
    }
    __syncthreads();
    // element (r, c) of the result is Q^{-1}(step(r), row(c)) times the scale of row r
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        const int row = lane + 64 * g;
        if (row >= m) continue;
        const int st = step_of_row[row];
        const double sc = 1.0 / myscale[g];
#pragma unroll
        for (int j = 0; j < 40; ++j) {
            const int c = 40 * w + j;
            if (c < m) gm_[(size_t)st * ld + row_of_step[c]] = a[g][j] * sc;
        }
    }
    __syncthreads();
    return bad;
}

}  // namespace irk
