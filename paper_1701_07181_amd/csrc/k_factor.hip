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

// Block-size classes: 0 -- m <= 64, four-wave routines (the bodies fit 128
// VGPRs: four waves per SIMD);
// 2 / 3 -- 64 < m <= 128 / 128 < m <= 160, eight-wave routines holding two /
// three row groups per lane in the inverse.  Each body has one call site of
// the product and one of the inverse, so each kernel carries one copy.  The
// product accumulates (acc) only with alpha = 1 or -1.
template <int CLS>
__device__ __forceinline__ void blk_gemm(int m, int ld, double alpha, const double *A, const double *B,
                                         bool acc, double *C, double *lds)
{
    if (CLS == 0) d64_gemm(m, ld, alpha, A, B, acc, C);
    else dm_gemm(m, ld, alpha, A, B, acc, C, lds);
}

template <int CLS>
__device__ __forceinline__ int blk_inverse(double *g, int m, int ld, double *lds)
{
    if (CLS == 0) return d64_invert(g, m, ld, lds);
    return dm_invert_rg<(CLS == 0 ? 2 : CLS)>(g, m, ld, lds);
}

template <int CLS> constexpr int team_of() { return CLS == 0 ? NTHREADS : DM_TEAM; }

__device__ __forceinline__ void flag_singular(const SysDesc &d, int elem) {
    if (threadIdx.x == 0) atomicCAS(&d.st->singular, 0, elem + 1);
}

// Phase 0 for m <= 64 with the products fused: the accumulators of P_{k,i}
// stay in registers from d_k M_i - dt J_ii through every lower neighbour j,
// and X = -dt^2 P_j^{-1} J_ji passes through LDS (64 x 66 doubles) into
// P_{k,i} += J_ij X; P_{k,i} is written once.
template <bool FULL>
__device__ __forceinline__ void factor_a_small_products(const SysDesc &d, int i, int k, const double *Jk,
                                                        double *Pk, double *Xs)
{
    const int s = d.s, lane = threadIdx.x & 63, w = wave_id();
    int m = d.m, ld = d.ld;
    const long long bs = (long long)m * ld;
    const GAS int *diag_pos = gp(d.diag_pos), *row_ptr = gp(d.row_ptr), *col_idx = gp(d.col_idx),
                  *tpos = gp(d.tpos);
    const double dk = d.dcoef[k], dt = d.dt;
    const int nx = FULL ? 2 : d64_ntiles(m, w & 1), ny = FULL ? 2 : d64_ntiles(m, w >> 1);
    const bool act = nx > 0 && ny > 0;
    const GAS double *Mi = gp(d.Mc + (long long)i * bs);
    const GAS double *Jd = gp(Jk + (long long)diag_pos[i] * bs);
    dbl4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = d64_tile_row(lane, w, x, q), c = d64_tile_col(lane, w, y);
                const size_t e = (size_t)min(c, m - 1) * ld + min(r, m - 1);
                acc[x][y][q] = dk * Mi[e] - dt * Jd[e];
            }
    const int p0 = row_ptr[i], pd = diag_pos[i];
    for (int p = p0; p < pd; ++p) {
        asm volatile("" : "+s"(m), "+s"(ld));   // per-lane offsets recomputed inside the loop
        const long long j = col_idx[p];
        dbl4 ax[2][2];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) ax[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
        if (act)
            d64_accum<FULL, false, 2>(ax, m, ld, gp(d.P64 + (j * s + k) * bs), gp(Jk + (long long)tpos[p] * bs),
                                      nullptr, nx, ny);
        __syncthreads();                          // the previous neighbour's X is consumed
        if (act) {
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    if (!FULL && (x >= nx || y >= ny)) continue;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        Xs[d64_tile_col(lane, w, y) * D64_LDX + d64_tile_row(lane, w, x, q)] = -dt * dt * ax[x][y][q];
                }
        }
        __syncthreads();
        if (act) d64_accum<FULL, true, 2>(acc, m, ld, gp(Jk + (long long)p * bs), nullptr, Xs, nx, ny);
    }
    if (act) {
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                if (!FULL && (x >= nx || y >= ny)) continue;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = d64_tile_row(lane, w, x, q), c = d64_tile_col(lane, w, y);
                    if (r < m && c < m) gp(Pk)[(size_t)c * ld + r] = acc[x][y][q];
                }
            }
    }
    __syncthreads();
}

template <bool COUPLED, bool SHJ, int CLS>
__device__ __forceinline__ void factor_a_body(const SysDesc *__restrict__ sysv,
                                              const Item *__restrict__ items, double *lds)
{
    constexpr int TEAM = team_of<CLS>();
    const Item it = items[blockIdx.x];
    if (it.first < 0) return;                     // padding task (whole workgroup)
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
    if (CLS != 0)
        for (long long e = threadIdx.x; e < bs; e += TEAM) gp(Pk)[e] = dk * gp(Mi)[e] - dt * gp(Jd)[e];
    if (COUPLED) {
        // column k of the cross blocks: C_{lk,i} = A^{-1}_lk M_i (l != k)
        for (int l = 0; l < s; ++l) {
            if (l == k) continue;
            const int idx = l < k ? l : l - 1;
            double *Cl = d.C64 + (((long long)i * s + k) * (s - 1) + idx) * bs;
            const double al = d.Ainv[l * SMAX + k];
            for (long long e = threadIdx.x; e < bs; e += TEAM) gp(Cl)[e] = al * gp(Mi)[e];
        }
    }
    if (CLS == 0) {
        if (m > 56) factor_a_small_products<true>(d, i, k, Jk, Pk, lds);
        else factor_a_small_products<false>(d, i, k, Jk, Pk, lds);
        if (!COUPLED) {
            if (blk_inverse<CLS>(Pk, m, ld, lds)) flag_singular(d, i);
        }
        return;
    }
    __syncthreads();
    double *X = d.Fscr + ((long long)i * s + k) * bs;
    const int p0 = row_ptr[i], pd = diag_pos[i];
    // per lower neighbour j: X = -dt^2 P_j^{-1} J_ji, then P_k += J_ij X
    for (int t = 2 * p0; t < 2 * pd; ++t) {
        const int p = t >> 1;
        const bool second = t & 1;
        const long long j = col_idx[p];
        const double *A = second ? Jk + (long long)p * bs : d.P64 + (j * s + k) * bs;
        const double *B = second ? X : Jk + (long long)tpos[p] * bs;
        blk_gemm<CLS>(m, ld, second ? 1.0 : -dt * dt, A, B, second, second ? Pk : X, lds);
    }
    if (!COUPLED) {
        if (blk_inverse<CLS>(Pk, m, ld, lds)) flag_singular(d, i);
    }
}

template <bool SHJ, int CLS>
__device__ __forceinline__ void factor_b_body(const SysDesc *__restrict__ sysv,
                                              const Item *__restrict__ items, double *lds)
{
    constexpr int TEAM = team_of<CLS>();
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
        if (blk_inverse<CLS>(P(k), m, ld, lds)) flag_singular(d, i);
        // k = 0: every cross block is still A^{-1}_kl M_i; with
        //   L = M_i P_0^{-1},  X = L M_i:
        //   P_l -= A^{-1}_l0 A^{-1}_0l X,   C_lq -= A^{-1}_l0 A^{-1}_0q X.
        // k > 0, for every later stage l (q runs over k, k+1, .., s-1):
        //   q = k:  L = C_lk P_k^{-1};  q = l:  P_l -= L C_kl;  else  C_lq -= L C_kq
        const int w = s - k;
        const int nops = (k == 0) ? 2 : (s - 1 - k) * w;
        for (int t = 0; t < nops; ++t) {
            const double *A, *B;
            double *D;
            double al;
            bool add;
            if (k == 0) {
                A = t ? L : Mi;
                B = t ? Mi : P(0);
                D = t ? X : L;
                al = 1.0;
                add = false;
            } else {
                const int l = k + 1 + t / w, q = k + t % w;
                if (q == k) { A = C(l, k); B = P(k); D = L; al = 1.0; add = false; }
                else { A = L; B = C(k, q); D = (q == l) ? P(l) : C(l, q); al = -1.0; add = true; }
            }
            blk_gemm<CLS>(m, ld, al, A, B, add, D, lds);
        }
        if (k == 0) {
            for (int l = 1; l < s; ++l)
                for (int q = 1; q < s; ++q) {
                    double *D = (q == l) ? P(l) : C(l, q);
                    const double f = d.Ainv[l * SMAX + 0] * d.Ainv[0 * SMAX + q];
                    for (long long e = threadIdx.x; e < bs; e += TEAM) gp(D)[e] -= f * gp(X)[e];
                }
            __syncthreads();
        }
    }
}

template <bool COUPLED, bool SHJ, int CLS>
__global__ __launch_bounds__(team_of<CLS>(), CLS == 0 ? 4 : 1) void k_factor_a(const SysDesc *__restrict__ sysv,
                                                                          const Item *__restrict__ items)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    factor_a_body<COUPLED, SHJ, CLS>(sysv, items, reinterpret_cast<double *>(smem_raw));
}
template <bool SHJ, int CLS>
__global__ __launch_bounds__(team_of<CLS>(), CLS == 0 ? 4 : 1) void k_factor_b(const SysDesc *__restrict__ sysv,
                                                                          const Item *__restrict__ items)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    factor_b_body<SHJ, CLS>(sysv, items, reinterpret_cast<double *>(smem_raw));
}

template <int CLS>
static void launch_factor_t(int phase, const SysDesc *dsys, const Item *items, int nitems, bool coupled,
                            bool sharedJ, size_t shmem, hipStream_t st)
{
    dim3 grid(nitems), block(team_of<CLS>());
    if (phase == 0) {
        if (coupled) {
            if (sharedJ) hipLaunchKernelGGL((k_factor_a<true, true, CLS>), grid, block, shmem, st, dsys, items);
            else hipLaunchKernelGGL((k_factor_a<true, false, CLS>), grid, block, shmem, st, dsys, items);
        } else {
            if (sharedJ) hipLaunchKernelGGL((k_factor_a<false, true, CLS>), grid, block, shmem, st, dsys, items);
            else hipLaunchKernelGGL((k_factor_a<false, false, CLS>), grid, block, shmem, st, dsys, items);
        }
    } else {
        if (sharedJ) hipLaunchKernelGGL((k_factor_b<true, CLS>), grid, block, shmem, st, dsys, items);
        else hipLaunchKernelGGL((k_factor_b<false, CLS>), grid, block, shmem, st, dsys, items);
    }
}

int factor_class(int m) { return m <= 64 ? 0 : (m <= 128 ? 2 : 3); }

void launch_factor(int phase, const SysDesc *dsys, const Item *items, int nitems, bool coupled,
                   bool sharedJ, int m, size_t shmem, hipStream_t st)
{
    switch (factor_class(m)) {
    case 0: launch_factor_t<0>(phase, dsys, items, nitems, coupled, sharedJ, shmem, st); break;
    case 2: launch_factor_t<2>(phase, dsys, items, nitems, coupled, sharedJ, shmem, st); break;
    default: launch_factor_t<3>(phase, dsys, items, nitems, coupled, sharedJ, shmem, st); break;
    }
}

template <int CLS>
static void set_lds_limit_t(int b)
{
    const void *k[] = {(const void *)k_factor_a<true, true, CLS>, (const void *)k_factor_a<true, false, CLS>,
                       (const void *)k_factor_a<false, true, CLS>, (const void *)k_factor_a<false, false, CLS>,
                       (const void *)k_factor_b<true, CLS>, (const void *)k_factor_b<false, CLS>};
    for (const void *f : k) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, b);
}

// Allow the factor kernels the LDS they need for m up to MMAX.
void factor_set_lds_limit(size_t bytes)
{
    set_lds_limit_t<0>((int)bytes);
    set_lds_limit_t<2>((int)bytes);
    set_lds_limit_t<3>((int)bytes);
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
