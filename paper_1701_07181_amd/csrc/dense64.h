// dense64.h -- dense FP64 block kernels (product on the matrix cores,
// Gauss-Jordan inverse in registers).  Blocks of order m <= 64 are run by one
// 256-thread workgroup (four waves):
//
//   * d64_gemm: C = alpha A B (+ C) for column-major blocks on the FP64
//     matrix cores (v_mfma_f64_16x16x4f64).  Each wave owns a 32 x 32
//     quadrant of the 64 x 64 output (2 x 2 tiles of 16 x 16) and loads its
//     operands from global memory directly (no LDS, no barrier inside).
//   * d64_invert: in-place Gauss-Jordan inversion with partial pivoting.
//     Lane r of wave w keeps row r, columns 16w .. 16w+15 in registers.  The
//     wave that owns the pivot column finds the largest candidate with a
//     DPP maximum of a 32-bit key (pivot_key) and one ballot.  Rows are never
//     moved; the row and column permutations are undone when the inverse is
//     written back.
//
// Blocks of order 64 < m <= 160 use the same two methods, sized for
// 512-thread workgroups (dm_gemm, dm_invert).
#pragma once
#include "irk_device.h"

namespace irk {

typedef double dbl4 __attribute__((ext_vector_type(4)));


// Fragment layouts of v_mfma_f64_16x16x4f64 (checked on gfx950): lane l
// supplies A(l % 16, l / 16) and B(l / 16, l % 16); element r of the result
// in lane l is D(4 r + l / 16, l % 16).
__device__ __forceinline__ int d64_frag_row(int lane, int r) { return 4 * r + (lane >> 4); }
__device__ __forceinline__ int d64_frag_col(int lane) { return lane & 15; }

// index of the calling wave in its workgroup, as a scalar (uniform) value
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }


// C = alpha A B (+ C when add) for column-major m x m blocks (m <= 64,
// leading dimension ld) on the FP64 matrix cores, without LDS: wave w owns
// the 32 x 32 quadrant (w & 1, w >> 1) of C (up to 2 x 2 tiles of 16 x 16,
// tiles wholly outside m skipped) and loads its matrix-core operands
// straight from global memory.  K is taken in blocks of 8; inside block t
// lane (r, kq) of step u supplies k = 8 t + 2 kq + u, so its two B values of
// a block are one 16-byte load and its A values are 16 consecutive doubles
// of a column per lane group.  Two blocks are in flight while one is
// multiplied.  With add the accumulators start from alpha * C, which
// requires alpha = 1 or -1 (then C + alpha A B is alpha * (alpha C + A B),
// exactly).  C must not overlap A or B.  Ends with a workgroup barrier, so
// the result can be read by every wave of the workgroup afterwards.
struct D64Ops {
    double a[2][2];     // A(i, k) of tiles x = 0, 1 for the two steps of a block
    dbl2 b[2];          // B(k, j) of tiles y = 0, 1 for the two steps
};

// Loads of block t; every address is clamped into the block, so the loads
// are unconditional (K padding is zeroed when the values are used).  B comes
// from global memory (leading dimension ld) or, with BLDS, from LDS
// (leading dimension D64_LDX).
constexpr int D64_LDX = 66;
// LDS of the inversion: pivot columns and reciprocals (130 doubles), the
// inverse (64 columns of D64_LDX doubles, where it stays after the call),
// the permutation (130 ints).  The products take their LDS operand with the
// same leading dimension.
constexpr int D64_STAGE = 130;
constexpr int D64_LDS_DOUBLES = D64_STAGE + 64 * D64_LDX + 65;

// Loads and stores coherent across the XCDs' L2 caches (device-scope
// relaxed atomics): for blocks that other workgroups of the same launch
// write or read (the dependency-driven factorization, k_factor.hip).
__device__ __forceinline__ double ld_coh(const GAS double *p)
{
    return __hip_atomic_load((double *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh(GAS double *p, double v)
{
    __hip_atomic_store((double *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// COH: bit 0 -- A, bit 1 -- B read from memory with coherent loads.
template <bool BLDS, bool ALDS = false, int COH = 0>
__device__ __forceinline__ void d64_load_ops(D64Ops &o, const GAS double *A, const GAS double *B, const double *Bs,
                                             int m, int ld, int i0, int j0, int kq, int t,
                                             const double *As = nullptr)
{
    const int kb = 8 * t + 2 * kq;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (ALDS) o.a[x][u] = As[min(kb + u, 63) * D64_LDX + i0 + 16 * x];
            else if (COH & 1) o.a[x][u] = ld_coh(A + (size_t)min(kb + u, m - 1) * ld + min(i0 + 16 * x, ld - 1));
            else o.a[x][u] = A[(size_t)min(kb + u, m - 1) * ld + min(i0 + 16 * x, ld - 1)];
        }
#pragma unroll
    for (int y = 0; y < 2; ++y) {
        if (BLDS) {
            o.b[y] = *reinterpret_cast<const dbl2 *>(Bs + (j0 + 16 * y) * D64_LDX + min(kb, 62));
        } else if (COH & 2) {
            const GAS double *q = B + (size_t)min(j0 + 16 * y, m - 1) * ld + min(kb, ld - 2);
            o.b[y].x = ld_coh(q);
            o.b[y].y = ld_coh(q + 1);
        } else {
            o.b[y] = *reinterpret_cast<const GAS dbl2 *>(B + (size_t)min(j0 + 16 * y, m - 1) * ld + min(kb, ld - 2));
        }
    }
}

template <bool FULL>
__device__ __forceinline__ void d64_mma_ops(const D64Ops &o, int m, int kq, int t, int nx, int ny,
                                            dbl4 (&acc)[2][2])
{
    const int kb = 8 * t + 2 * kq;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const bool kin = kb + u < m;
        double av[2], bv[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) av[x] = kin ? o.a[x][u] : 0.0;
#pragma unroll
        for (int y = 0; y < 2; ++y) bv[y] = kin ? (u ? o.b[y].y : o.b[y].x) : 0.0;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                if (!FULL && (x >= nx || y >= ny)) continue;
                acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
            }
    }
}

// acc += A B over K = m for this wave's tiles (quadrant (w & 1, w >> 1)).
// FULL (m > 56: all 2 x 2 tiles, eight K blocks): straight-line code, so the
// waits before each block's products leave the two later blocks' loads in
// flight; otherwise blocks past the last one are skipped.
// DEPTH operand buffers: DEPTH - 1 blocks in flight while one is multiplied.
// With BLDS / ALDS the operand comes from LDS (column-major, leading
// dimension D64_LDX): entries outside the m x m block may hold anything
// (those of K are zeroed, the others only reach result rows or columns
// >= m).
template <bool FULL, bool BLDS, int DEPTH = 3, bool ALDS = false, int COH = 0>
__device__ __forceinline__ void d64_accum(dbl4 (&acc)[2][2], int m, int ld, const GAS double *A,
                                          const GAS double *B, const double *Bs, int nx, int ny,
                                          const double *As = nullptr)
{
    const int lane = threadIdx.x & 63, w = wave_id();
    const int r = lane & 15, kq = lane >> 4;
    const int i0 = 32 * (w & 1) + r, j0 = 32 * (w >> 1) + r;
    const int nb = FULL ? 8 : (m + 7) >> 3;
    D64Ops o[DEPTH];
#pragma unroll
    for (int t = 0; t < DEPTH - 1; ++t)
        if (FULL || t < nb) d64_load_ops<BLDS, ALDS, COH>(o[t], A, B, Bs, m, ld, i0, j0, kq, t, As);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        if (!FULL && t >= nb) continue;
        const int tn = t + DEPTH - 1;
        if (FULL ? (tn < 8) : (tn < nb)) d64_load_ops<BLDS, ALDS, COH>(o[tn % DEPTH], A, B, Bs, m, ld, i0, j0, kq, tn, As);
        d64_mma_ops<FULL>(o[t % DEPTH], m, kq, t, nx, ny, acc);
    }
}

// Row and column of element q of tile (x, y) of this wave's quadrant.
__device__ __forceinline__ int d64_tile_row(int lane, int w, int x, int q) { return 32 * (w & 1) + 16 * x + d64_frag_row(lane, q); }
__device__ __forceinline__ int d64_tile_col(int lane, int w, int y) { return 32 * (w >> 1) + 16 * y + d64_frag_col(lane); }

template <bool FULL>
__device__ __forceinline__ void d64_gemm_tiles(int m, int ld, double alpha, const GAS double *A,
                                               const GAS double *B, bool add, GAS double *C, int nx, int ny)
{
    const int lane = threadIdx.x & 63, w = wave_id();
    dbl4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = d64_tile_row(lane, w, x, q), j = d64_tile_col(lane, w, y);
                const double old = C[(size_t)min(j, m - 1) * ld + min(i, m - 1)];
                acc[x][y][q] = (add && i < m && j < m) ? alpha * old : 0.0;
            }
    d64_accum<FULL, false>(acc, m, ld, A, B, nullptr, nx, ny);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            if (!FULL && (x >= nx || y >= ny)) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = d64_tile_row(lane, w, x, q), j = d64_tile_col(lane, w, y);
                if (i < m && j < m) C[(size_t)j * ld + i] = alpha * acc[x][y][q];
            }
        }
}

// Tiles (of 16 x 16) of wave w's quadrant that hold rows / columns below m.
__device__ __forceinline__ int d64_ntiles(int m, int q) { return min(2, max(0, (m - 32 * q + 15) >> 4)); }

__device__ __forceinline__ void d64_gemm(int m, int ld, double alpha, const double *gA, const double *gB,
                                         bool add, double *gC)
{
    // opaque copies of the sizes: keeps the per-lane operand offsets inside
    // each call instead of letting them be hoisted (and held in registers)
    // across a caller's loop of products
    asm volatile("" : "+s"(m), "+s"(ld));
    const int w = wave_id();
    const int nx = d64_ntiles(m, w & 1), ny = d64_ntiles(m, w >> 1);
    if (m > 56) d64_gemm_tiles<true>(m, ld, alpha, gp(gA), gp(gB), add, gp(gC), 2, 2);
    else if (nx > 0 && ny > 0) d64_gemm_tiles<false>(m, ld, alpha, gp(gA), gp(gB), add, gp(gC), nx, ny);
    __syncthreads();
}

__device__ __forceinline__ double d64_readlane(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Maximum of x over the 64 lanes of a wave (every lane active), as a scalar:
// DPP exchanges inside each row of 16 lanes (quad swaps, half-row and row
// mirrors), then the four row results.
__device__ __forceinline__ int wave_max_i32(int x)
{
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false));    // quad_perm 1,0,3,2
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false));    // quad_perm 2,3,0,1
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false));   // row_half_mirror
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false));   // row_mirror
    const int r0 = __builtin_amdgcn_readlane(x, 0), r1 = __builtin_amdgcn_readlane(x, 16);
    const int r2 = __builtin_amdgcn_readlane(x, 32), r3 = __builtin_amdgcn_readlane(x, 48);
    return max(max(r0, r1), max(r2, r3));
}

// Pivot key of a candidate entry: the high word of |v| (sign cleared), which
// orders non-negative doubles like their values up to the top 20 mantissa
// bits; -1 for rows already used.  The pivot is the first unused row whose
// key equals the column maximum, so its magnitude is within a factor
// 1 - 2^-20 of the largest one (partial pivoting).
__device__ __forceinline__ int pivot_key(double v, bool unused_row)
{
    return unused_row ? (__double2hiint(v) & 0x7fffffff) : -1;
}

// 1 / x from the hardware reciprocal and one Newton step (three dependent
// operations instead of a full division; a few ulp at most for normal x).
__device__ __forceinline__ double fast_recip(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

// Pivot choice for the column v (one value per lane = row) among the rows
// marked in unused, by the owner wave (every lane active): publishes the
// column, the pivot row (with 0x100 set when the pivot is zero or the column
// holds a non-finite value) and 1 / pivot.
__device__ __forceinline__ void d64_publish(double v, unsigned long long unused, int lane, double *col, int *pw,
                                            double *pinv)
{
    const bool mine = (unused >> lane) & 1ull;
    const int key = pivot_key(v, mine);
    const int K = wave_max_i32(key);
    const bool nonfin = __any(mine && !isfinite(v));
    const int p = __builtin_ctzll(__ballot(key == K));
    const double piv = d64_readlane(v, p);
    col[lane] = v;
    if (lane == 0) {
        *pw = p | ((nonfin || K <= 0 || !isfinite(piv)) ? 0x100 : 0);
        *pinv = fast_recip(piv);
    }
}

// In-place inverse of the column-major m x m block P at gptr.  Returns
// nonzero (in every thread) when a pivot is zero or a pivot column holds a
// non-finite value.
//
// Lane r of wave w keeps row r of P, columns 16w .. 16w+15, in registers
// (consecutive lanes read consecutive doubles of a column: coalesced).
//
// Pivot rows are not scaled when they are used: a row that served as pivot
// with value piv is stored as piv times its Gauss-Jordan value (the update
// of every other row is the same either way), and the scale is removed when
// the result is written back.  Step c, after one barrier: every wave reads
// the published column c, pivot row p and 1/piv, takes row p of its columns
// with v_readlane and updates them.  The owner of column c+1 updates that
// column first and publishes its pivot choice (look-ahead), so the search
// overlaps the other updates and each step costs one barrier.
// LDS: D64_LDS_DOUBLES; the inverse is left at lds + D64_STAGE (column c at
// c * D64_LDX) for the caller's next product.  FROM_LDS: P is read from that
// same place (the caller stored it there) instead of from gptr.  COH: the
// inverse is written to gptr with coherent stores.
template <bool FROM_LDS = false, bool COH = false>
__device__ __forceinline__ int d64_invert(double *gptr, int m, int ld, double *lds)
{
    GAS double *g = gp(gptr);
    asm volatile("" : "+s"(m), "+s"(ld));      // nothing of a call hoisted into a caller's loop
    const int lane = threadIdx.x & 63, w = wave_id();
    double *colbuf = lds;                                          // [2][64] pivot columns
    double *pinvbuf = lds + 128;                                   // [2] 1 / pivot
    double *stage = lds + D64_STAGE;                               // [64][D64_LDX] permuted result
    int *pbuf = reinterpret_cast<int *>(lds + D64_STAGE + 64 * D64_LDX);   // [2] pivot row (+ flag)
    int *step_of_row = pbuf + 2;                                   // [64]
    int *row_of_step = pbuf + 66;                                  // [64]
    double a[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int c = 16 * w + j;
        a[j] = (lane < m && c < m) ? (FROM_LDS ? stage[c * D64_LDX + lane] : g[(size_t)c * ld + lane])
                                   : (lane == c ? 1.0 : 0.0);
    }
    unsigned long long unused = (m >= 64) ? ~0ull : ((1ull << m) - 1ull);
    double myscale = 1.0;           // pivot value of this lane's row once it has been used
    int bad = 0;
    if (w == 0) d64_publish(a[0], unused, lane, colbuf, pbuf, pinvbuf);
    for (int wc = 0; wc < 4; ++wc) {
        if (16 * wc >= m) break;
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) {
            const int c = 16 * wc + cc;
            if (c >= m) continue;           // uniform: every thread skips the same steps
            const int par = c & 1;
            __syncthreads();
            const int pw = __builtin_amdgcn_readfirstlane(pbuf[par]);
            const double pinv = pinvbuf[par];
            const double f = colbuf[par * 64 + lane];
            const int p = pw & 0xff;
            bad |= pw >> 8;
            const bool isp = (lane == p);
            const double gm = isp ? 0.0 : f * pinv;
            if (isp) myscale = f;
            unused &= ~(1ull << p);
            // row p of this wave's columns
            double prow[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) prow[j] = d64_readlane(a[j], p);
            // column c + 1 (index cn of wave wn): updated and searched first
            const int cn = (cc + 1) & 15;        // a constant once the loop is unrolled
            const int wn = (cc == 15) ? wc + 1 : wc;
            const bool ahead = (c + 1 < m) && (w == wn);
            if (ahead) {
                a[cn] = fma(-gm, prow[cn], a[cn]);
                d64_publish(a[cn], unused, lane, colbuf + (par ^ 1) * 64, pbuf + (par ^ 1), pinvbuf + (par ^ 1));
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if (j == cn && ahead) continue;
                a[j] = fma(-gm, prow[j], a[j]);
            }
            if (w == wc) a[cc] = isp ? 1.0 : -gm;
            if (threadIdx.x == 0) { step_of_row[p] = c; row_of_step[c] = p; }
        }
    }
    __syncthreads();
    // the value kept for (row r, column c) is P^{-1}(step(r), row(c)) times
    // the pivot of row r; stage[col * D64_LDX + row] is written one column per
    // instruction (conflict-free), then copied out column by column
    if (lane < m) {
        const int row = step_of_row[lane];
        const double sc = 1.0 / myscale;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int c = 16 * w + j;
            if (c < m) stage[row_of_step[c] * D64_LDX + row] = a[j] * sc;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m * 64; e += NTHREADS) {
        const int c = e >> 6, r = e & 63;
        if (r < m) {
            if (COH) st_coh(g + (size_t)c * ld + r, stage[c * D64_LDX + r]);
            else g[(size_t)c * ld + r] = stage[c * D64_LDX + r];
        }
    }
    __syncthreads();
    return bad;
}

// ---------------------------------------------------------------------------
// Blocks of order 64 < m <= 160 are processed by 512-thread workgroups
// (eight waves, two per SIMD).
// ---------------------------------------------------------------------------
constexpr int DM_TEAM = 512;

// C = alpha A B (+ C when add) for column-major blocks on the FP64 matrix
// cores.  The NT x NT grid of 16 x 16 output tiles (NT = ceil(m / 16) <= 10)
// is split in two tile-row halves and four tile-column quarters, one part
// per wave (at most 5 x 3 tiles, 15 accumulators of four doubles).  K runs
// in panels of 16: A(:, panel) -> Am[kk * 160 + i] and B(panel, :) ->
// Bm[j * 17 + kk] (odd stride: conflict-free fragment reads); the next
// panel's loads are issued before the current panel is multiplied.
constexpr int DM_AP = 160, DM_BP = 17, DM_KP = 16;
constexpr int DM_PIECES = DM_KP * DM_AP / 2;           // 16-byte pieces of either panel (1280)
constexpr int DM_Q = (DM_PIECES + DM_TEAM - 1) / DM_TEAM;
constexpr int DM_LDS_DOUBLES = DM_KP * DM_AP + DM_AP * DM_BP;

// coh_a: A read with coherent loads (see ld_coh)
__device__ __forceinline__ void dm_load_panel(const GAS double *A, const GAS double *B, int m, int ld,
                                              int k0, dbl2 (&ra)[DM_Q], dbl2 (&rb)[DM_Q], bool coh_a = false)
{
#pragma unroll
    for (int q = 0; q < DM_Q; ++q) {
        const int e = min((int)threadIdx.x + q * DM_TEAM, DM_PIECES - 1);
        const int kk = e / 80, i = (e - kk * 80) * 2;     // A: column k0+kk, rows i, i+1
        const GAS double *pa = A + (size_t)min(k0 + kk, m - 1) * ld + min(i, ld - 2);
        if (coh_a) {
            ra[q].x = ld_coh(pa);
            ra[q].y = ld_coh(pa + 1);
        } else {
            ra[q] = *reinterpret_cast<const GAS dbl2 *>(pa);
        }
        const int j = e >> 3, kb = (e & 7) * 2;           // B: column j, rows k0+kb, +1
        rb[q] = *reinterpret_cast<const GAS dbl2 *>(B + (size_t)min(j, m - 1) * ld + min(k0 + kb, ld - 2));
    }
}

__device__ __forceinline__ void dm_put_panel(double *Am, double *Bm, int m, int k0, const dbl2 (&ra)[DM_Q],
                                             const dbl2 (&rb)[DM_Q])
{
#pragma unroll
    for (int q = 0; q < DM_Q; ++q) {
        const int e = (int)threadIdx.x + q * DM_TEAM;
        if (e >= DM_PIECES) continue;
        const int kk = e / 80, i = (e - kk * 80) * 2;
        Am[kk * DM_AP + i] = (k0 + kk < m && i < m) ? ra[q].x : 0.0;
        Am[kk * DM_AP + i + 1] = (k0 + kk < m && i + 1 < m) ? ra[q].y : 0.0;
        const int j = e >> 3, kb = (e & 7) * 2;
        Bm[j * DM_BP + kb] = (j < m && k0 + kb < m) ? rb[q].x : 0.0;
        Bm[j * DM_BP + kb + 1] = (j < m && k0 + kb + 1 < m) ? rb[q].y : 0.0;
    }
}

__device__ __forceinline__ void dm_gemm(int m, int ld, double alpha, const double *gA, const double *gB,
                                        bool add, double *gC, double *lds, bool coh_a = false)
{
    const GAS double *A = gp(gA);
    const GAS double *B = gp(gB);
    GAS double *C = gp(gC);
    double *Am = lds, *Bm = lds + DM_KP * DM_AP;
    const int lane = threadIdx.x & 63, w = wave_id();
    const int r = lane & 15, kq = lane >> 4;
    const int NT = (m + 15) >> 4;
    const int rh = w & 1, cq = w >> 1;
    const int ti0 = rh * NT / 2, TI = (rh + 1) * NT / 2 - ti0;      // <= 5
    const int tj0 = cq * NT / 4, TJ = (cq + 1) * NT / 4 - tj0;      // <= 3
    dbl4 acc[5][3];
#pragma unroll
    for (int x = 0; x < 5; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) acc[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
    dbl2 ra[DM_Q], rb[DM_Q];
    dm_load_panel(A, B, m, ld, 0, ra, rb, coh_a);
    for (int k0 = 0; k0 < m; k0 += DM_KP) {
        __syncthreads();                                  // previous panel fully read
        dm_put_panel(Am, Bm, m, k0, ra, rb);
        if (k0 + DM_KP < m) dm_load_panel(A, B, m, ld, k0 + DM_KP, ra, rb, coh_a);
        __syncthreads();
        const int nkc = (min(m - k0, DM_KP) + 3) >> 2;
#pragma unroll
        for (int kc = 0; kc < DM_KP / 4; ++kc) {
            if (kc >= nkc) continue;
            double a[5], b[3];
#pragma unroll
            for (int x = 0; x < 5; ++x) a[x] = Am[(4 * kc + kq) * DM_AP + 16 * (ti0 + min(x, TI - 1)) + r];
#pragma unroll
            for (int y = 0; y < 3; ++y) b[y] = Bm[(16 * (tj0 + min(y, TJ - 1)) + r) * DM_BP + 4 * kc + kq];
#pragma unroll
            for (int x = 0; x < 5; ++x)
#pragma unroll
                for (int y = 0; y < 3; ++y)
                    if (x < TI && y < TJ)
                        acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
        }
    }
    // store (old values first when accumulating)
#pragma unroll
    for (int x = 0; x < 5; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) {
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

// In-place inverse for 64 < m <= 160 (same contract as d64_invert).  Lane l
// of wave w keeps rows l + 64 g (g < RG, RG = 2 for m <= 128, else 3) and
// columns 20w .. 20w + 19 in registers.  The owner wave of column c picks
// the pivot row p (pivot_key maximum) and publishes the column with its entry
// p set to zero, p, the pivot and its reciprocal through LDS.  Step c, after
// one barrier: every wave reads row p's values of its own columns from the
// lane that holds them (v_readlane) and updates its columns
// with multipliers column(r) / pivot (zero for row p itself, which keeps a
// deferred scale); the owner of column c + 1 updates that column first and
// publishes its pivot choice (look-ahead).  The result is written straight to
// global memory with the row and column permutations undone (one column per
// store instruction).
constexpr int DMI_CW = 20;
constexpr int DMI_LDS_DOUBLES = 2 * DM_AP + 2 + DM_AP + (2 + 2 * DM_AP) / 2;

// (x0, x1, x2)[g] for a uniform g, from scalars: arrays selected this way can
// be turned into indexed (scratch) loads by the compiler
template <typename T>
__device__ __forceinline__ T dm_sel(int g, T x0, T x1, T x2)
{
    return g == 0 ? x0 : (g == 1 ? x1 : x2);
}

// Pivot choice for the column (v0, v1, v2) of row groups 0..2 among the rows
// marked in un0..un2, by the owner wave (every lane active): publishes the
// column with its pivot entry set to zero, the pivot row (0x1000 set when
// the pivot is zero or the column holds a non-finite value), the pivot and
// its reciprocal.
template <int RG>
__device__ __forceinline__ void dm_publish(double v0, double v1, double v2, unsigned long long un0,
                                           unsigned long long un1, unsigned long long un2, int lane,
                                           double *col, int *pw, double *pinv, double *pivc)
{
    const bool m0 = (un0 >> lane) & 1ull, m1 = (un1 >> lane) & 1ull, m2 = (un2 >> lane) & 1ull;
    const int k0 = pivot_key(v0, m0), k1 = pivot_key(v1, m1), k2 = pivot_key(v2, m2);
    const int K = wave_max_i32(max(k0, max(k1, k2)));
    const bool anynf = __any((m0 && !isfinite(v0)) || (m1 && !isfinite(v1)) || (m2 && !isfinite(v2)));
    const unsigned long long b0 = __ballot(k0 == K), b1 = __ballot(k1 == K), b2 = __ballot(k2 == K);
    const int p = b0 ? __builtin_ctzll(b0) : (b1 ? 64 + __builtin_ctzll(b1) : 128 + __builtin_ctzll(b2));
    const double piv = d64_readlane(dm_sel(p >> 6, v0, v1, v2), p & 63);
    col[lane] = (lane == p) ? 0.0 : v0;
    col[lane + 64] = (lane + 64 == p) ? 0.0 : v1;
    if (RG > 2 && lane + 128 < DM_AP) col[lane + 128] = (lane + 128 == p) ? 0.0 : v2;
    if (lane == 0) {
        *pw = p | ((anynf || K <= 0 || !isfinite(piv)) ? 0x1000 : 0);
        *pinv = fast_recip(piv);
        *pivc = piv;
    }
}

template <int RG, bool COH = false>
__device__ __forceinline__ int dm_invert_rg(double *gptr, int m, int ld, double *lds)
{
    GAS double *G = gp(gptr);
    asm volatile("" : "+s"(m), "+s"(ld));      // nothing of a call hoisted into a caller's loop
    const int lane = threadIdx.x & 63, w = wave_id();
    double *colbuf = lds;                                           // [2][160] pivot columns
    double *pinvbuf = lds + 2 * DM_AP;                              // [2] 1 / pivot
    double *pivval = lds + 2 * DM_AP + 2;                           // [160] pivot of step c
    int *pbuf = reinterpret_cast<int *>(lds + 3 * DM_AP + 2);      // [2]
    int *step_of_row = pbuf + 2;                                    // [160]
    int *row_of_step = pbuf + 2 + DM_AP;                            // [160]
    double a[RG][DMI_CW];
#pragma unroll
    for (int g = 0; g < RG; ++g) {
        const int row = lane + 64 * g;
#pragma unroll
        for (int j = 0; j < DMI_CW; ++j) {
            const int c = DMI_CW * w + j;
            a[g][j] = (row < m && c < m) ? G[(size_t)c * ld + row] : (row == c ? 1.0 : 0.0);
        }
    }
    // unused rows of the three row groups (groups >= RG stay empty)
    auto group_mask = [m](int g) {
        const int lo = 64 * g;
        return (m <= lo) ? 0ull : (m - lo >= 64 ? ~0ull : ((1ull << (m - lo)) - 1ull));
    };
    unsigned long long un0 = group_mask(0), un1 = group_mask(1), un2 = (RG > 2) ? group_mask(2) : 0ull;
    int bad = 0;
    if (w == 0)
        dm_publish<RG>(a[0][0], a[1][0], a[RG - 1][0], un0, un1, un2, lane, colbuf, pbuf, pinvbuf, pivval);
    for (int wc = 0; wc < DM_TEAM / 64; ++wc) {
        if (DMI_CW * wc >= m) break;
#pragma unroll
        for (int cc = 0; cc < DMI_CW; ++cc) {
            const int c = DMI_CW * wc + cc;
            if (c >= m) continue;                     // uniform
            const int par = c & 1;
            __syncthreads();
            const int pw = __builtin_amdgcn_readfirstlane(pbuf[par]);
            const int p = pw & 0xfff;
            if (pw & 0x1000) bad = 1;
            const double pinv = pinvbuf[par];
            const int pg = p >> 6, pl = p & 63;
            // the pivot row's values of this wave's columns, read from lane pl
            double prow[DMI_CW];
            if (pg == 0) {
#pragma unroll
                for (int j = 0; j < DMI_CW; ++j) prow[j] = d64_readlane(a[0][j], pl);
            } else if (RG == 2 || pg == 1) {
#pragma unroll
                for (int j = 0; j < DMI_CW; ++j) prow[j] = d64_readlane(a[1][j], pl);
            } else {
#pragma unroll
                for (int j = 0; j < DMI_CW; ++j) prow[j] = d64_readlane(a[RG - 1][j], pl);
            }
            double gmul[RG];
#pragma unroll
            for (int g = 0; g < RG; ++g) {
                const int row = lane + 64 * g;
                gmul[g] = (row < DM_AP) ? colbuf[par * DM_AP + row] * pinv : 0.0;
            }
            if (pg == 0) un0 &= ~(1ull << pl);
            else if (pg == 1) un1 &= ~(1ull << pl);
            else un2 &= ~(1ull << pl);
            // column c + 1 (index cn of wave wn): updated and published first
            const int cn = (cc + 1) % DMI_CW;         // a constant once the loop is unrolled
            const int wn = (cc == DMI_CW - 1) ? wc + 1 : wc;
            const bool ahead = (c + 1 < m) && (w == wn);
            if (ahead) {
#pragma unroll
                for (int g = 0; g < RG; ++g) a[g][cn] = fma(-gmul[g], prow[cn], a[g][cn]);
                dm_publish<RG>(a[0][cn], a[1][cn], a[RG - 1][cn], un0, un1, un2, lane, colbuf + (par ^ 1) * DM_AP,
                               pbuf + (par ^ 1), pinvbuf + (par ^ 1), pivval + c + 1);
            }
#pragma unroll
            for (int j = 0; j < DMI_CW; ++j) {
                if (j == cn && ahead) continue;
#pragma unroll
                for (int g = 0; g < RG; ++g) a[g][j] = fma(-gmul[g], prow[j], a[g][j]);
            }
            if (w == wc) {
#pragma unroll
                for (int g = 0; g < RG; ++g) a[g][cc] = (lane + 64 * g == p) ? 1.0 : -gmul[g];
            }
            if (threadIdx.x == 0) { step_of_row[p] = c; row_of_step[c] = p; }
        }
    }
    __syncthreads();
    // the value kept for (row r, column c) is P^{-1}(step(r), row(c)) times
    // the pivot of row r
#pragma unroll
    for (int g = 0; g < RG; ++g) {
        const int row = lane + 64 * g;
        if (row >= m) continue;
        const int st = step_of_row[row];
        const double sc = 1.0 / pivval[st];
#pragma unroll
        for (int j = 0; j < DMI_CW; ++j) {
            const int c = DMI_CW * w + j;
            if (c < m) {
                if (COH) st_coh(G + (size_t)row_of_step[c] * ld + st, a[g][j] * sc);
                else G[(size_t)row_of_step[c] * ld + st] = a[g][j] * sc;
            }
        }
    }
    __syncthreads();
    return bad;
}

__device__ __forceinline__ int dm_invert(double *gptr, int m, int ld, double *lds)
{
    return (m <= 128) ? dm_invert_rg<2>(gptr, m, ld, lds) : dm_invert_rg<3>(gptr, m, ld, lds);
}

}  // namespace irk
