// k_factor.hip -- block ILU(0) factorization in FP64, stage by stage and
// level by level
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
// with C_{kl,i} starting at A^{-1}_kl M_i.  Pivot (0, i) is eliminated first,
// so every cross block in stage row 0 or stage column 0 keeps its starting
// value A^{-1}_kl M_i: those are never stored (the sweeps apply M_i and the
// scalar), and the first round collapses to one product X = M_i P_0^{-1} M_i:
//
//     P_{l,i} = d_l M_i - dt J_{l,ii} - A^{-1}_l0 A^{-1}_0l X,
//     C_{lq,i} = A^{-1}_lq M_i - A^{-1}_l0 A^{-1}_0q X        (l, q >= 1).
//
// Schedule.  A task is (stage k, element i).  Its pivot needs the same stage
// of the lower neighbours (earlier levels) and the earlier stages of its own
// element, so task (k, i) runs in wavefront level(i) + k: L + s - 1 launches
// for L levels (the uncoupled forms need none of the stage order: wavefront
// = level).  A task adds the neighbour terms to P_{k,i} (stage 0 and the
// uncoupled forms start it from d_k M_i - dt J_{k,ii}; later coupled stages
// from the value the earlier rounds left), inverts it in place (pivots are
// stored inverted because the sweeps apply them as matrix-vector products),
// and runs its stage round on the later stages of the element.
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
                                         bool acc, double *C, double *lds, bool coh_a = false)
{
    if (CLS == 0) d64_gemm(m, ld, alpha, A, B, acc, C);
    else dm_gemm(m, ld, alpha, A, B, acc, C, lds, coh_a);
}

template <int CLS, bool COH = false>
__device__ __forceinline__ int blk_inverse(double *g, int m, int ld, double *lds)
{
    if (CLS == 0) return d64_invert(g, m, ld, lds);
    return dm_invert_rg<(CLS == 0 ? 2 : CLS), COH>(g, m, ld, lds);
}

template <int CLS> constexpr int team_of() { return CLS == 0 ? NTHREADS : DM_TEAM; }

constexpr int FACTOR_SPIN_MAX = 1 << 22;

__device__ __forceinline__ void flag_singular(const SysDesc &d, int elem) {
    if (threadIdx.x == 0) atomicCAS(&d.st->singular, 0, elem + 1);
}

// Dependency-driven factorization: the workgroup waits until flag f holds
// the launch's epoch (the task it names has published its blocks); a wait
// beyond the poll budget marks the system's state non-finite (never a hang).
__device__ __forceinline__ void flow_wait(const SysDesc &d, unsigned long long *fflag, long long f,
                                          unsigned long long epoch)
{
    if (threadIdx.x == 0) {
        int spins = 0;
        while (__hip_atomic_load(fflag + f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > FACTOR_SPIN_MAX) { d.st->nonfinite = 1; break; }
        }
    }
    __syncthreads();
}

// Neighbour terms for m <= 64 with the products fused: the accumulators of
// P_{k,i} stay in registers from their starting value (d_k M_i - dt J_ii;
// zero when from_p, the stored P_{k,i} being added after the last
// neighbour) through every lower neighbour j, and
// X = -dt^2 P_j^{-1} J_ji passes through LDS (64 x 66 doubles) into
// P_{k,i} += J_ij X; P_{k,i} is left in LDS where the inverse reads it
// (lds + D64_STAGE, leading dimension D64_LDX).
template <bool FULL, bool FLOW = false>
__device__ __forceinline__ void factor_small_products(const SysDesc &d, int i, int k, const double *Jk,
                                                      double *Pk, bool from_p, double *Xs,
                                                      unsigned long long *fflag, unsigned long long epoch)
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
    const GAS double *Ps = gp(Pk);
    dbl4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = d64_tile_row(lane, w, x, q), c = d64_tile_col(lane, w, y);
                const size_t e = (size_t)min(c, m - 1) * ld + min(r, m - 1);
                acc[x][y][q] = from_p ? 0.0 : dk * Mi[e] - dt * Jd[e];
            }
    const int p0 = row_ptr[i], pd = diag_pos[i];
    for (int p = p0; p < pd; ++p) {
        asm volatile("" : "+s"(m), "+s"(ld));   // per-lane offsets recomputed inside the loop
        const long long j = col_idx[p];
        if (FLOW) flow_wait(d, fflag, j * s + k, epoch);   // P_{k,j}^{-1} is published
        dbl4 ax[2][2];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) ax[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
        if (act)
            d64_accum<FULL, false, 2, false, FLOW ? 1 : 0>(ax, m, ld, gp(d.P64 + (j * s + k) * bs),
                                                           gp(Jk + (long long)tpos[p] * bs), nullptr, nx, ny);
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
    if (from_p) {
        // the stored P_{k,i} last, so the neighbour terms need not wait for
        // the earlier stage round that leaves it
        if (FLOW) flow_wait(d, fflag, (long long)i * s + k - 1, epoch);
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = d64_tile_row(lane, w, x, q), c = d64_tile_col(lane, w, y);
                    const size_t e = (size_t)min(c, m - 1) * ld + min(r, m - 1);
                    acc[x][y][q] += FLOW ? ld_coh(Ps + e) : Ps[e];
                }
    }
    __syncthreads();                              // every wave is done with X in LDS
    if (act) {
        double *Pst = Xs + D64_STAGE;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                if (!FULL && (x >= nx || y >= ny)) continue;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = d64_tile_row(lane, w, x, q), c = d64_tile_col(lane, w, y);
                    if (r < m && c < m) Pst[c * D64_LDX + r] = acc[x][y][q];
                }
            }
    }
    __syncthreads();
}

// Stored cross block C_{lq,i} (l, q >= 1, l != q): group q, entry l.
__device__ __forceinline__ double *cross_blk(const SysDesc &d, long long i, int l, int q)
{
    const int s = d.s;
    const long long bs = (long long)d.m * d.ld;
    const int e = (q - 1) * (s - 2) + (l < q ? l - 1 : l - 2);
    return d.C64 + (i * (s - 1) * (s - 2) + e) * bs;
}

// This wave's accumulators (tiles of its quadrant) into an LDS block with
// leading dimension D64_LDX.
template <bool FULL>
__device__ __forceinline__ void d64_put_lds(const dbl4 (&acc)[2][2], double *Ls, int nx, int ny)
{
    const int lane = threadIdx.x & 63, w = wave_id();
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            if (!FULL && (x >= nx || y >= ny)) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                Ls[d64_tile_col(lane, w, y) * D64_LDX + d64_tile_row(lane, w, x, q)] = acc[x][y][q];
        }
}

// Stage round of task (k, i) for m <= 64, right after the inverse, which
// leaves P_k^{-1} in LDS.  L = (k = 0: M_i; else C_lk) P_k^{-1} is kept in
// LDS (in place of P_k^{-1}) for the products that consume it, so neither L
// nor X goes through memory:
//   k = 0: X = L M_i in registers; the later stages' pivots and stored
//          cross blocks are written from X directly;
//   k >= 1: for every later stage l, P_l -= L C_kl and C_lq -= L C_kq.
// P_k^{-1} is read from LDS by the first L product when that is the only
// one (k = 0 or k = s - 2), else from memory (the inverse has written it).
// The products and their order are those of the file comment; the results
// are those of the same products through memory.
template <bool FULL, bool SHJ, bool FLOW = false>
__device__ __forceinline__ void factor_round_small(const SysDesc &d, int i, int k, double *lds)
{
    const int s = d.s, lane = threadIdx.x & 63, w = wave_id();
    int m = d.m, ld = d.ld;
    asm volatile("" : "+s"(m), "+s"(ld));
    const long long bs = (long long)m * ld;
    const int nx = FULL ? 2 : d64_ntiles(m, w & 1), ny = FULL ? 2 : d64_ntiles(m, w >> 1);
    const bool act = nx > 0 && ny > 0;
    double *Ls = lds + D64_STAGE;
    const GAS double *Mi = gp(d.Mc + (long long)i * bs);
    dbl4 acc[2][2];
    auto clear = [&]() {
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) acc[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
    };
    const bool one_l = (k == 0) || (k == s - 2);
    for (int l = k + 1; l < s; ++l) {
        // L = A P_k^{-1}
        const GAS double *A = k == 0 ? Mi : gp(cross_blk(d, i, l, k));
        clear();
        if (act) {
            // (with FLOW, blocks written by other tasks of the launch are
            // read coherently: the cross blocks, and P_k^{-1} from memory)
            if (one_l) d64_accum<FULL, true, 3, false, FLOW ? 1 : 0>(acc, m, ld, A, nullptr, Ls, nx, ny);
            else d64_accum<FULL, false, 3, false, FLOW ? 3 : 0>(acc, m, ld, A, gp(d.P64 + ((long long)i * s + k) * bs),
                                                                nullptr, nx, ny);
        }
        __syncthreads();                          // P_k^{-1} / the previous L is consumed
        if (act) d64_put_lds<FULL>(acc, Ls, nx, ny);
        __syncthreads();
        if (k == 0) break;
        // P_l -= L C_kl, C_lq -= L C_kq (q > k, q != l), q in order
        for (int q = k + 1; q < s; ++q) {
            GAS double *D = gp(q == l ? d.P64 + ((long long)i * s + l) * bs : cross_blk(d, i, l, q));
            const GAS double *B = gp(cross_blk(d, i, k, q));
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int r = d64_tile_row(lane, w, x, e), c = d64_tile_col(lane, w, y);
                        const GAS double *po = D + (size_t)min(c, m - 1) * ld + min(r, m - 1);
                        const double old = FLOW ? ld_coh(po) : *po;
                        acc[x][y][e] = (r < m && c < m) ? -old : 0.0;
                    }
            if (act) d64_accum<FULL, false, 3, true, FLOW ? 2 : 0>(acc, m, ld, nullptr, B, nullptr, nx, ny, Ls);
            if (act) {
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y) {
                        if (!FULL && (x >= nx || y >= ny)) continue;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int r = d64_tile_row(lane, w, x, e), c = d64_tile_col(lane, w, y);
                            if (r < m && c < m) {
                                if (FLOW) st_coh(D + (size_t)c * ld + r, -acc[x][y][e]);
                                else D[(size_t)c * ld + r] = -acc[x][y][e];
                            }
                        }
                    }
            }
        }
        __syncthreads();                          // L is consumed before the next one is stored
    }
    if (k != 0) return;
    // X = L M_i, then for every later stage l:
    //   P_l = d_l M_i - dt J_l,ii - A^{-1}_l0 A^{-1}_0l X,  C_lq = A^{-1}_lq M_i - A^{-1}_l0 A^{-1}_0q X
    clear();
    if (act) d64_accum<FULL, false, 3, true>(acc, m, ld, nullptr, Mi, nullptr, nx, ny, Ls);
    const double dt = d.dt;
    const long long dp = gp(d.diag_pos)[i];
    double mv[2][2][4];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = d64_tile_row(lane, w, x, e), c = d64_tile_col(lane, w, y);
                mv[x][y][e] = Mi[(size_t)min(c, m - 1) * ld + min(r, m - 1)];
            }
    for (int l = 1; l < s; ++l) {
        const GAS double *Jd = gp(d.Jc + (SHJ ? 0 : (long long)l * d.nnzb * bs) + dp * bs);
        const double dl = d.dcoef[l], fl = d.Ainv[l * SMAX] * d.Ainv[l];
        GAS double *Pl = gp(d.P64 + ((long long)i * s + l) * bs);
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = d64_tile_row(lane, w, x, e), c = d64_tile_col(lane, w, y);
                    if (c >= m || r >= ld) continue;
                    const size_t o = (size_t)c * ld + r;
                    // (padding rows r >= m of a block stay zero)
                    const double v = r < m ? dl * mv[x][y][e] - dt * Jd[o] - fl * acc[x][y][e] : 0.0;
                    if (FLOW) st_coh(Pl + o, v);
                    else Pl[o] = v;
                }
        for (int q = 1; q < s; ++q) {
            if (q == l) continue;
            GAS double *Cq = gp(cross_blk(d, i, l, q));
            const double a = d.Ainv[l * SMAX + q], f = d.Ainv[l * SMAX] * d.Ainv[q];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int r = d64_tile_row(lane, w, x, e), c = d64_tile_col(lane, w, y);
                        if (c >= m || r >= ld) continue;
                        const double v = r < m ? a * mv[x][y][e] - f * acc[x][y][e] : 0.0;
                        if (FLOW) st_coh(Cq + (size_t)c * ld + r, v);
                        else Cq[(size_t)c * ld + r] = v;
                    }
        }
    }
}

// One task: stage k of element i (see the file comment).  The products of a
// task are one operation list (the neighbour products for m > 64, then the
// stage round), so a kernel holds one inlined copy of the product and one of
// the inverse.
// (FLOW: fflag / epoch of the launch; each lower neighbour's flag is awaited
// right before its first product, so the task's own set-up and its earlier
// neighbours' products overlap the later neighbours' tasks)
template <bool COUPLED, bool SHJ, int CLS, bool FLOW = false>
__device__ __forceinline__ void factor_task_body(const SysDesc *__restrict__ sysv, const Item it, double *lds,
                                                 unsigned long long *fflag = nullptr,
                                                 unsigned long long epoch = 0)
{
    constexpr int TEAM = team_of<CLS>();
    if (it.first < 0) return;                     // padding task (whole workgroup)
    const SysDesc &d = sysv[it.sys];
    const int s = d.s, m = d.m, ld = d.ld;
    const int i = it.first, k = it.aux;
    const long long bs = (long long)m * ld;
    auto P = [&](int q) { return d.P64 + ((long long)i * s + q) * bs; };
    auto Jst = [&](int q) { return d.Jc + (SHJ ? 0 : (long long)q * d.nnzb * bs); };
    double *Pk = P(k);
    const double *Jk = Jst(k);
    const double *Mi = d.Mc + (long long)i * bs;
    const GAS int *diag_pos = gp(d.diag_pos), *row_ptr = gp(d.row_ptr), *col_idx = gp(d.col_idx),
                  *tpos = gp(d.tpos);
    const double dt = d.dt;
    // later coupled stages start from what the earlier rounds left in P_{k,i}
    const bool from_p = COUPLED && k > 0;
    const int p0 = row_ptr[i], pd = diag_pos[i];
    const int nnb = (CLS == 0) ? 0 : 2 * (pd - p0);   // neighbour products (m > 64)
    if (CLS == 0) {
        if (m > 56) factor_small_products<true, FLOW>(d, i, k, Jk, Pk, from_p, lds, fflag, epoch);
        else factor_small_products<false, FLOW>(d, i, k, Jk, Pk, from_p, lds, fflag, epoch);
        if (d64_invert<true, FLOW>(Pk, m, ld, lds)) flag_singular(d, i);
        if (COUPLED && k + 1 < s) {
            if (m > 56) factor_round_small<true, SHJ, FLOW>(d, i, k, lds);
            else factor_round_small<false, SHJ, FLOW>(d, i, k, lds);
        }
        return;
    }
    if (!from_p) {
        const double *Jd = Jk + (long long)diag_pos[i] * bs;
        const double dk = d.dcoef[k];
        for (long long e = threadIdx.x; e < bs; e += TEAM) gp(Pk)[e] = dk * gp(Mi)[e] - dt * gp(Jd)[e];
        __syncthreads();
    }
    // stage round: k = 0 -> L = M P_0^{-1}, X = L M; k >= 1 -> for every
    // later stage l: L = C_lk P_k^{-1}, P_l -= L C_kl, C_lq -= L C_kq
    const bool round = COUPLED && k + 1 < s;
    const int w = s - k;
    const int nround = !round ? 0 : (k == 0 ? 2 : (s - 1 - k) * w);
    double *L = d.Fscr + ((long long)i * s + k) * bs;
    double *X = d.Fscr + ((long long)i * s + (k + 1) % s) * bs;
    const int ntot = nnb + nround;
    for (int t = 0; t <= ntot; ++t) {
        // every neighbour term is in: invert the pivot block in place
        if (t == nnb && blk_inverse<CLS, FLOW>(Pk, m, ld, lds)) flag_singular(d, i);
        if (t == ntot) break;
        const double *A, *B;
        double *D;
        double al;
        bool add;
        if (t < nnb) {
            // per lower neighbour j: X = -dt^2 P_j^{-1} J_ji, then P_k += J_ij X
            const int p = p0 + (t >> 1);
            const bool second = t & 1;
            const long long j = col_idx[p];
            if (FLOW && !second) flow_wait(d, fflag, j * s + k, epoch);   // P_{k,j}^{-1} is published
            A = second ? Jk + (long long)p * bs : d.P64 + (j * s + k) * bs;
            B = second ? X : Jk + (long long)tpos[p] * bs;
            D = second ? Pk : X;
            al = second ? 1.0 : -dt * dt;
            add = second;
        } else if (k == 0) {
            const int u = t - nnb;
            A = u ? L : Mi;
            B = u ? Mi : Pk;
            D = u ? X : L;
            al = 1.0;
            add = false;
        } else {
            // w operations per later stage l, q = k .. s-1: q = k -> L = C_lk P_k^{-1};
            // q = l -> P_l -= L C_kl; other q -> C_lq -= L C_kq
            const int u = t - nnb;
            const int l = k + 1 + u / w, q = k + u % w;
            if (q == k) { A = cross_blk(d, i, l, k); B = Pk; D = L; al = 1.0; add = false; }
            else if (q == l) { A = L; B = cross_blk(d, i, k, l); D = P(l); al = -1.0; add = true; }
            else { A = L; B = cross_blk(d, i, k, q); D = cross_blk(d, i, l, q); al = -1.0; add = true; }
        }
        // (FLOW, uncoupled only: the lower neighbours' inverses come from
        // other tasks of the launch)
        blk_gemm<CLS>(m, ld, al, A, B, add, D, lds, FLOW && t < nnb && !(t & 1));
    }
    if (round && k == 0) {
        // later stages' pivots and the stored cross blocks from X = M P_0^{-1} M
        for (int l = 1; l < s; ++l) {
            const double *Jd = Jst(l) + (long long)diag_pos[i] * bs;
            const double dl = d.dcoef[l], fl = d.Ainv[l * SMAX] * d.Ainv[l];
            double *Pl = P(l);
            // (padding rows r >= m of a block stay zero: X holds only rows < m)
            for (long long e = threadIdx.x; e < bs; e += TEAM)
                gp(Pl)[e] = (e % ld < m) ? dl * gp(Mi)[e] - dt * gp(Jd)[e] - fl * gp(X)[e] : 0.0;
            for (int q = 1; q < s; ++q) {
                if (q == l) continue;
                double *Cq = cross_blk(d, i, l, q);
                const double a = d.Ainv[l * SMAX + q], f = d.Ainv[l * SMAX] * d.Ainv[q];
                for (long long e = threadIdx.x; e < bs; e += TEAM)
                    gp(Cq)[e] = (e % ld < m) ? a * gp(Mi)[e] - f * gp(X)[e] : 0.0;
            }
        }
        __syncthreads();
    }
}

template <bool COUPLED, bool SHJ, int CLS>
__global__ __launch_bounds__(team_of<CLS>(), CLS == 0 ? 4 : 1) void k_factor_task(const SysDesc *__restrict__ sysv,
                                                                             const Item *__restrict__ items)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    factor_task_body<COUPLED, SHJ, CLS>(sysv, items[blockIdx.x], reinterpret_cast<double *>(smem_raw));
}

// Consecutive wavefronts of the factorization (one system: the uncoupled
// forms, and the coupled form with m <= 64) in one launch, each task waiting only for the tasks it reads: (k, j) for the
// lower neighbours j (their pivot inverses) and, coupled, (k - 1, i) (the
// stage round that left P_{k,i} and the cross blocks).  The scheme of the chained
// sweeps (k_sweep_flow.hip): workgroups take the tasks items[off ..
// off + n) (wavefront order) in the order they claim a ticket, so a task
// only waits for tasks of workgroups already running, and the last claimant
// sets the counter back to zero; a task's flag (element-major, [T][s])
// holds the epoch of the factorization that published it.  Blocks written
// by one task and read by another go through coherent (device-scope)
// loads and stores; a task publishes after its stores have completed.  A
// wait beyond its poll budget marks the system's state non-finite (never
// a hang).
template <bool COUPLED, bool SHJ, int CLS>
__global__ __launch_bounds__(team_of<CLS>(), CLS == 0 ? 4 : 1) void k_factor_flow(const SysDesc *__restrict__ sysv,
                                                             const Item *__restrict__ items, int off, int n,
                                                             unsigned long long *fflag, unsigned *ticket,
                                                             unsigned long long epoch)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_t;
    if (threadIdx.x == 0) {
        const unsigned t = atomicAdd(ticket, 1u);
        if (t == (unsigned)n - 1u) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_t = (int)t;
    }
    __syncthreads();
    const int t = s_t;
    if (t >= n) return;   // (the counter was not at zero: no task to read)
    const Item it = items[off + t];
    if (it.first < 0) return;   // padding task: no flag, nothing waits for it
    const SysDesc &d = sysv[it.sys];
    const int s = d.s, i = it.first, k = it.aux;
    // (every wait is in the task body: each lower neighbour right before its
    // first product, coupled k > 0 the earlier stage round right before
    // P_{k,i} is read)
    factor_task_body<COUPLED, SHJ, CLS, true>(sysv, it, reinterpret_cast<double *>(smem_raw), fflag, epoch);
    __builtin_amdgcn_s_waitcnt(0);   // this thread's block stores have completed
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(fflag + (long long)i * s + k, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

void launch_factor_flow(const SysDesc *dsys, const Item *items, int off, int n, bool coupled, bool sharedJ,
                        int m, size_t shmem, unsigned long long *fflag, unsigned *ticket,
                        unsigned long long epoch, hipStream_t st)
{
    if (n <= 0) return;
    const int cls = factor_class(m);
    dim3 grid(n), block(cls == 0 ? NTHREADS : DM_TEAM);
#define FF(C, SH, K) hipLaunchKernelGGL((k_factor_flow<C, SH, K>), grid, block, shmem, st, dsys, items, off, n, fflag, ticket, epoch)
    // (m > 64: the uncoupled forms only)
    if (cls == 0) {
        if (coupled) { if (sharedJ) FF(true, true, 0); else FF(true, false, 0); }
        else { if (sharedJ) FF(false, true, 0); else FF(false, false, 0); }
    } else if (cls == 2) {
        if (sharedJ) FF(false, true, 2); else FF(false, false, 2);
    } else {
        if (sharedJ) FF(false, true, 3); else FF(false, false, 3);
    }
#undef FF
}

template <int CLS>
static void launch_factor_t(const SysDesc *dsys, const Item *items, int nitems, bool coupled, bool sharedJ,
                            size_t shmem, hipStream_t st)
{
    dim3 grid(nitems), block(team_of<CLS>());
    if (coupled) {
        if (sharedJ) hipLaunchKernelGGL((k_factor_task<true, true, CLS>), grid, block, shmem, st, dsys, items);
        else hipLaunchKernelGGL((k_factor_task<true, false, CLS>), grid, block, shmem, st, dsys, items);
    } else {
        if (sharedJ) hipLaunchKernelGGL((k_factor_task<false, true, CLS>), grid, block, shmem, st, dsys, items);
        else hipLaunchKernelGGL((k_factor_task<false, false, CLS>), grid, block, shmem, st, dsys, items);
    }
}

int factor_class(int m) { return m <= 64 ? 0 : (m <= 128 ? 2 : 3); }

void launch_factor(const SysDesc *dsys, const Item *items, int nitems, bool coupled, bool sharedJ, int m,
                   size_t shmem, hipStream_t st)
{
    if (nitems <= 0) return;
    switch (factor_class(m)) {
    case 0: launch_factor_t<0>(dsys, items, nitems, coupled, sharedJ, shmem, st); break;
    case 2: launch_factor_t<2>(dsys, items, nitems, coupled, sharedJ, shmem, st); break;
    default: launch_factor_t<3>(dsys, items, nitems, coupled, sharedJ, shmem, st); break;
    }
}

template <int CLS>
static void set_lds_limit_t(int b)
{
    const void *k[] = {(const void *)k_factor_task<true, true, CLS>, (const void *)k_factor_task<true, false, CLS>,
                       (const void *)k_factor_task<false, true, CLS>, (const void *)k_factor_task<false, false, CLS>};
    for (const void *f : k) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, b);
}

// Allow the factor kernels the LDS they need for m up to MMAX.
void factor_set_lds_limit(size_t bytes)
{
    set_lds_limit_t<0>((int)bytes);
    const void *ff[] = {(const void *)k_factor_flow<true, true, 0>, (const void *)k_factor_flow<true, false, 0>,
                        (const void *)k_factor_flow<false, true, 0>, (const void *)k_factor_flow<false, false, 0>,
                        (const void *)k_factor_flow<false, true, 2>, (const void *)k_factor_flow<false, false, 2>,
                        (const void *)k_factor_flow<false, true, 3>, (const void *)k_factor_flow<false, false, 3>};
    for (const void *f : ff) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
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
__device__ __forceinline__ void quantize_block(const double *__restrict__ src, void *__restrict__ dst,
                                               int *__restrict__ ex, int m, int ld, int ldq,
                                               long long b, double *red)
{
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

template <int FT>
__global__ __launch_bounds__(NTHREADS) void k_quantize(const double *__restrict__ src,
                                                       void *__restrict__ dst, int *__restrict__ ex,
                                                       int m, int ld, int ldq)
{
    __shared__ double red[NTHREADS / 64];
    quantize_block<FT>(src, dst, ex, m, ld, ldq, blockIdx.x, red);
}

// The factors of several systems in one launch: item = (system, first
// block, block count, 0 pivots / 1 cross blocks).
template <int FT>
__global__ __launch_bounds__(NTHREADS) void k_quantize_sys(const SysDesc *__restrict__ sysv,
                                                           const Item *__restrict__ items)
{
    __shared__ double red[NTHREADS / 64];
    const Item it = items[blockIdx.x];
    const SysDesc &d = sysv[it.sys];
    const bool cross = it.aux != 0;
    const double *src = cross ? d.C64 : d.P64;
    void *dst = (FT == FT_F32) ? (void *)(cross ? d.C32 : d.P32) : (void *)(cross ? d.C16 : d.P16);
    int *ex = cross ? d.C16e : d.P16e;
    const int ldq = (FT == FT_F32) ? d.ld32 : d.ld16;
    for (int b = it.first; b < it.first + it.count; ++b) {
        quantize_block<FT>(src, dst, ex, d.m, d.ld, ldq, b, red);
        __syncthreads();   // red is reused by the next block
    }
}

void launch_quantize_sys(const SysDesc *dsys, const Item *items, int nitems, int ftype, hipStream_t st)
{
    if (nitems <= 0) return;
    dim3 grid((unsigned)nitems), block(NTHREADS);
    if (ftype == FT_F32) hipLaunchKernelGGL(k_quantize_sys<FT_F32>, grid, block, 0, st, dsys, items);
    else if (ftype == FT_BF16) hipLaunchKernelGGL(k_quantize_sys<FT_BF16>, grid, block, 0, st, dsys, items);
    else hipLaunchKernelGGL(k_quantize_sys<FT_F16S>, grid, block, 0, st, dsys, items);
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
    const long long nc = (h.C64 != nullptr) ? (long long)h.T * (h.s - 1) * (h.s - 2) : 0;
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
// pinv [s][T][m][m], cross [s][s][T][m][m] (C_{kl,i} at (k, l, i); those in
// stage row or column 0 are A^{-1}_kl M_i, the others the stored blocks).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NTHREADS) void k_export_pivots(const double *__restrict__ src, double *dst,
                                                            int s, int T, int m, int ld)
{
    const long long b = blockIdx.x;   // source block (element i, stage k)
    const long long i = b / s, k = b - i * s;
    const long long o = (k * T + i) * (long long)m * m;
    const double *S = src + b * (long long)m * ld;
    for (int e = threadIdx.x; e < m * m; e += NTHREADS) {
        const int r = e / m, c = e - r * m;
        dst[o + e] = S[(long long)c * ld + r];
    }
}

// one workgroup per (element i, stage pair k != l)
__global__ __launch_bounds__(NTHREADS) void k_export_cross(const SysDesc *__restrict__ dsys, double *dst)
{
    const SysDesc &d = *dsys;
    const int s = d.s, T = d.T, m = d.m, ld = d.ld;
    const long long b = blockIdx.x;
    const long long i = b / (s * (s - 1));
    const int pr = (int)(b - i * s * (s - 1));
    const int k = pr / (s - 1), lr = pr - k * (s - 1), l = lr < k ? lr : lr + 1;
    const long long o = (((long long)k * s + l) * T + i) * (long long)m * m;
    const long long bs = (long long)m * ld;
    const bool mass = (k == 0 || l == 0);
    const double a = d.Ainv[k * SMAX + l];
    const double *S = mass ? d.Mc + i * bs
                           : d.C64 + (i * (s - 1) * (s - 2) + (l - 1) * (s - 2) + (k < l ? k - 1 : k - 2)) * bs;
    for (int e = threadIdx.x; e < m * m; e += NTHREADS) {
        const int r = e / m, c = e - r * m;
        const double v = S[(long long)c * ld + r];
        dst[o + e] = mass ? a * v : v;
    }
}

void launch_export(const SysDesc *dsys, const SysDesc &h, double *pinv, double *cross, bool coupled,
                   hipStream_t st)
{
    if (pinv)
        hipLaunchKernelGGL(k_export_pivots, dim3((unsigned)((long long)h.T * h.s)), dim3(NTHREADS), 0, st,
                           (const double *)h.P64, pinv, h.s, h.T, h.m, h.ld);
    if (cross && coupled && h.s > 1)
        hipLaunchKernelGGL(k_export_cross, dim3((unsigned)((long long)h.T * h.s * (h.s - 1))), dim3(NTHREADS),
                           0, st, dsys, cross);
}

}  // namespace irk
