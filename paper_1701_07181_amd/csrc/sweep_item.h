// sweep_item.h -- one element of a block ILU(0) sweep (forward or backward),
// shared by the level-per-launch kernel (k_sweep.hip) and the single-launch
// dependency-driven kernel (k_sweep_flow.hip).  The arithmetic and its order
// are the same in both, so they give identical results.
#pragma once
#include "irk_device.h"

namespace irk {

// Reduce team partials red[g][S][ldr] over g for stage k, row r.
// Four running sums over g = 0, 4, 8, ... (+1, +2, +3) keep four LDS loads in
// flight; they are combined as (a0 + a1) + (a2 + a3), a fixed order.
template <typename TC>
__device__ __forceinline__ TC sum_strided(const TC *p, int G, int stride) {
    TC a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int g = 0;
    for (; g + 4 <= G; g += 4) {
        a0 += p[g * stride];
        a1 += p[(g + 1) * stride];
        a2 += p[(g + 2) * stride];
        a3 += p[(g + 3) * stride];
    }
    if (g < G) a0 += p[g * stride];
    if (g + 1 < G) a1 += p[(g + 1) * stride];
    if (g + 2 < G) a2 += p[(g + 2) * stride];
    return (a0 + a1) + (a2 + a3);
}

template <typename TC, int S>
__device__ __forceinline__ TC sum_groups(const TC *red, int G, int k, int ldr, int r) {
    return sum_strided(red + k * ldr + r, G, S * ldr);
}

// acc[v] += column c of a block (rows slot*V .. slot*V+V-1) times x, for the
// columns c = g, g + G, ... of this thread; the first NQ come from registers
// (prefetching form), the rest are loaded here.
template <typename TF, typename TC, int NQ, bool PF>
__device__ __forceinline__ void col_product(const GAS typename Vec16<TF>::st *blk, int ld, int m,
                                            int g, int G, const TC (&pre)[NQ][Vec16<TF>::V],
                                            const TC *x, TC (&acc)[Vec16<TF>::V])
{
    constexpr int V = Vec16<TF>::V;
    int c0 = g;
    if (PF) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int c = g + G * q;
            if (c < m) {
                const TC xv = x[c];
#pragma unroll
                for (int v = 0; v < V; ++v) acc[v] += pre[q][v] * xv;
            }
        }
        c0 = g + G * NQ;
    }
    // chunks of U columns: the loads of a chunk are unconditional (clamped
    // addresses), so they are all in flight before the first product
    constexpr int U = (V <= 4) ? 8 : 4;
    for (int cb = c0; cb < m; cb += U * G) {
        TC a[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) Vec16<TF>::load(blk + (size_t)min(cb + u * G, m - 1) * ld, a[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = cb + u * G;
            if (c < m) {
                const TC xv = x[c];
#pragma unroll
                for (int v = 0; v < V; ++v) acc[v] += a[u][v] * xv;
            }
        }
    }
}

template <typename TF, typename TC, int NQ>
__device__ __forceinline__ void prefetch_block(const GAS typename Vec16<TF>::st *blk, int ld, int m,
                                               int g, int G, TC (&pre)[NQ][Vec16<TF>::V])
{
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int c = g + G * q;
        Vec16<TF>::load(blk + (size_t)min(c, m - 1) * ld, pre[q]);
    }
}

// The record's first SW_NB (= 8) columns as separate register values: a
// select over them picks block b's column.  (Selects over loads of an array
// are folded into one indexed load, which places the array in private
// memory; scalars produced by an empty asm statement stay in registers.)
struct RecCols {
    int c0, c1, c2, c3, c4, c5, c6, c7;
    __device__ __forceinline__ explicit RecCols(const SwItem &rec)
        : c0(rec.col[0]), c1(rec.col[1]), c2(rec.col[2]), c3(rec.col[3]),
          c4(rec.col[4]), c5(rec.col[5]), c6(rec.col[6]), c7(rec.col[7])
    {
        asm volatile("" : "+v"(c0), "+v"(c1), "+v"(c2), "+v"(c3), "+v"(c4), "+v"(c5), "+v"(c6), "+v"(c7));
    }
    __device__ __forceinline__ int operator()(int b) const
    {
        return b == 0 ? c0 : b == 1 ? c1 : b == 2 ? c2 : b == 3 ? c3 : b == 4 ? c4 : b == 5 ? c5 : b == 6 ? c6 : c7;
    }
};
static_assert(SW_NB == 8, "RecCols holds eight columns");

// PFM: 0 streaming form; 1 prefetching form (factor blocks, the mass block
// and the first Jacobian columns); 2 prefetching form without the Jacobian
// columns (fewer registers: more elements in flight on the large levels).
//
// FLOW: the element waits, after issuing its prefetch, until every
// neighbour it reads has published this sweep's result (flag = epoch, see
// k_sweep_flow.hip); a wait longer than FLOW_SPIN_MAX polls sets *late.
// The neighbours' values are then read, and this element's results
// written, with device-scope (relaxed atomic) accesses, which are coherent
// across the XCDs' L2 caches.
constexpr int FLOW_SPIN_MAX = 1 << 21;

template <int S, typename TJ, typename TF, typename TC, bool COUPLED, bool SHJ, bool FWD, int PFM,
          bool FLOW = false>
__device__ __forceinline__ void sweep_item(const SysDesc &d, const SwItem &rec, bool has, int tps,
                                           int region, int v_slot, int v_index, int acc_slot,
                                           unsigned char *smem_raw, unsigned long long epoch = 0,
                                           int *late = nullptr)
{
    constexpr bool PF = PFM > 0;
    const int s = d.s, m = d.m, T = d.T;
    constexpr int VJ = Vec16<TJ>::V, VF = Vec16<TF>::V;
    constexpr int NQ = 8 / VF;        // prefetched loads per thread and factor block
    constexpr int QJ = (PFM == 1) ? 32 / VJ : 0;   // prefetched loads per thread of the Jacobian row
    const int ldJ = ld_of<TJ>(d), ldF = ld_of<TF>(d);
    const int ldv = round_up(m, 8);
    const int team = SW_THREADS / tps;
    const int tm = threadIdx.x / team, tid = threadIdx.x - tm * team;
    const int RJ = ldJ / VJ, GJ = team / RJ;
    const int gJ = tid / RJ, sJ = tid - gJ * RJ;
    const int RF = ldF / VF, GF = team / RF;
    const int gF = tid / RF, sF = tid - gF * RF;
    const int maxg = d.maxrow * m;
    TC *base_lds = reinterpret_cast<TC *>(smem_raw) + (size_t)tm * region;
    TC *xg = base_lds;                       // gather, then partials
    TC *yv = base_lds + (region - (2 * S + 1) * ldv);   // [S][ldv]
    TC *uv = yv + S * ldv;                   // [S][ldv]
    TC *av = uv + S * ldv;                   // [ldv]: backward stage-0 combination

    const long long n = (long long)T * m;
    const int i = rec.i;
    GAS TC *yh = gp(reinterpret_cast<TC *>(d.vec[SL_YH]));
    const TC dt = (TC)d.dt;
    const auto Jb = jac_of<TJ>(d);
    const auto Pb = piv_of<TF>(d);
    const auto Cb = cross_of<TF>(d);
    const long long bsF = (long long)m * ldF;
    const bool fact = has && gF < GF;

    const int pa = rec.pa, ncol = rec.nb * m;
    const auto jrow = Jb + (size_t)pa * m * ldJ + sJ * VJ;

    // Every load below (first gather pass, prefetch) is unconditional, with
    // indices clamped into the arrays (padding teams read element 0), so all
    // of them are in flight together and the first pass's stores wait only
    // for its own loads.
    // ---- gather, first pass (loads): this element's input and the
    //      neighbours' vectors ----
    const int nown = s * m;
    const long long ic = max(i, 0);
    const RecCols cols(rec);
    const GAS double *vin = gp(reinterpret_cast<const double *>(d.vec[v_slot])) + (long long)v_index * d.N;
    // entry q: this element's input (q < s m) and, for q < ncol, block b row
    // c of the neighbours' vectors (every stage); blocks b >= SW_NB (rows of
    // more than SW_NB blocks) are redone below with the index array
    TC own0, nv0[S];
    // values of other elements written in this launch (FLOW) / results
    auto ldn = [&](GAS TC *p) -> TC {
        if (FLOW) return __hip_atomic_load((TC *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return *p;
    };
    auto sty = [&](GAS TC *p, TC v) {
        if (FLOW) __hip_atomic_store((TC *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else *p = v;
    };
    auto load_neighbours = [&]() {
        const int qn = min(tid, max(ncol - 1, 0)), b = qn / m, c = qn - b * m;
        const long long j = (ncol == 0) ? ic : cols(b);
#pragma unroll
        for (int k = 0; k < S; ++k) nv0[k] = ldn(yh + (min(k, s - 1) * n + j * m + c));
    };
    {
        const int q = tid;
        const int qo = min(q, nown - 1), ko = qo / m, ro = qo - ko * m;
        const long long go = ko * n + ic * m + ro;
        own0 = FWD ? (TC)vin[go] : yh[go];
        if (!FLOW) load_neighbours();
    }
    __builtin_amdgcn_sched_barrier(0);   // keep these loads ahead of the prefetch

    // ---- prefetch: Jacobian row (first QJ column loads), pivots, cross blocks ----
    TC rJ[QJ > 0 ? QJ : 1][VJ];
    TC rP[S][NQ][VF];
    TC rC[S][S][NQ][VF];   // [k][l]: stored block C_{lk} (l, k >= 1) used by round k
    constexpr int NQJ = 8 / VJ;                     // prefetched column pieces of M_i
    TC rM[NQJ][VJ];
    const auto Mb = mass_of<TJ>(d) + (size_t)ic * m * ldJ + sJ * VJ;
    // stored cross block C_{lk,i} (l, k >= 1): group k - 1, entry l
    auto cross_idx = [&](long long e, int l, int k) {
        return e * (s - 1) * (s - 2) + (long long)(k - 1) * (s - 2) + (l < k ? l - 1 : l - 2);
    };
    if (PF) {
        if (SHJ) {
            const auto jrow_c = Jb + (size_t)min(pa, d.nnzb - 1) * m * ldJ + sJ * VJ;
#pragma unroll
            for (int q = 0; q < QJ; ++q) {
                const int cg = gJ + GJ * q;
                Vec16<TJ>::load(jrow_c + (size_t)min(cg, max(ncol - 1, 0)) * ldJ, rJ[q]);
            }
        }
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const int kc = min(k, s - 1);
            prefetch_block<TF, TC, NQ>(Pb + (ic * s + kc) * bsF + sF * VF, ldF, m, gF, GF, rP[k]);
            if (COUPLED && S > 2 && s > 2) {
#pragma unroll
                for (int l = 1; l < S; ++l) {
                    if (l == k || k == 0 || (FWD ? (l < k) : (l > k))) continue;
                    // clamped into this system's stored blocks (s may be below S)
                    const int lc = min(l, s - 1), kk2 = max(1, min(k, s - 1));
                    const long long ci = (s > 2 && lc != kk2) ? cross_idx(ic, lc, kk2) : 0;
                    prefetch_block<TF, TC, NQ>(Cb + ci * bsF + sF * VF, ldF, m, gF, GF, rC[k][l]);
                }
            }
        }
        if (COUPLED) prefetch_block<TJ, TC, NQJ>(Mb, ldJ, m, gJ, GJ, rM);
    }

    if (FLOW) {
        __builtin_amdgcn_sched_barrier(0);   // the prefetch stays ahead of the wait
        // wait until every neighbour this element reads is published
        if (has) {
            for (int b = tid; b < rec.nb; b += team) {
                const long long j = (b < SW_NB) ? cols(b) : gp(d.col_idx)[pa + b];
                int spins = 0;
                while (__hip_atomic_load(d.flow + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
                    __builtin_amdgcn_s_sleep(4);
                    if (++spins > FLOW_SPIN_MAX) { *late = 1; break; }
                }
            }
        }
        __syncthreads();
        load_neighbours();
    }

    // ---- gather: first pass stores, entries beyond it (more than a team's
    //      worth, or blocks past SW_NB) ----
    if (has) {
        if (tid < nown) yv[(tid / m) * ldv + tid % m] = own0;
        if (tid < ncol) {
#pragma unroll
            for (int k = 0; k < S; ++k)
                if (k < s) xg[k * maxg + tid] = nv0[k];
        }
        for (int q = tid; q < max(ncol, nown); q += team) {
            const bool far = q < ncol && q / m >= SW_NB;
            if (q == tid && !far) continue;           // done by the first pass
            if (q < nown && q != tid) {
                const int ko = q / m, ro = q - ko * m;
                const long long go = ko * n + (long long)i * m + ro;
                yv[ko * ldv + ro] = FWD ? (TC)vin[go] : yh[go];
            }
            if (q < ncol) {
                const int b = q / m, c = q - b * m;
                const long long j = (b < SW_NB) ? cols(b) : gp(d.col_idx)[pa + b];
#pragma unroll
                for (int k = 0; k < S; ++k)
                    if (k < s) xg[k * maxg + q] = ldn(yh + (k * n + j * m + c));
            }
        }
    }
    __syncthreads();

    // ---- Jacobian part: dt * sum_j J_ij w_{k,j} for all stages ----
    {
        TC aj[S][VJ];
#pragma unroll
        for (int k = 0; k < S; ++k)
#pragma unroll
            for (int v = 0; v < VJ; ++v) aj[k][v] = 0;
        if (has && gJ < GJ && ncol > 0) {
            if (SHJ) {
                int c0 = gJ;
                if (PF) {
#pragma unroll
                    for (int q = 0; q < QJ; ++q) {
                        const int cg = gJ + GJ * q;
                        if (cg < ncol) {
#pragma unroll
                            for (int k = 0; k < S; ++k) {
                                if (k >= s) continue;
                                const TC xv = xg[k * maxg + cg];
#pragma unroll
                                for (int v = 0; v < VJ; ++v) aj[k][v] += rJ[q][v] * xv;
                            }
                        }
                    }
                    c0 = gJ + GJ * QJ;
                }
                constexpr int UJ = (VJ <= 4) ? 8 : 4;   // columns per chunk, loads all in flight
                for (int cb = c0; cb < ncol; cb += UJ * GJ) {
                    TC a[UJ][VJ];
#pragma unroll
                    for (int u = 0; u < UJ; ++u) Vec16<TJ>::load(jrow + (size_t)min(cb + u * GJ, ncol - 1) * ldJ, a[u]);
#pragma unroll
                    for (int u = 0; u < UJ; ++u) {
                        const int cg = cb + u * GJ;
                        if (cg >= ncol) continue;
#pragma unroll
                        for (int k = 0; k < S; ++k) {
                            if (k >= s) continue;
                            const TC xv = xg[k * maxg + cg];
#pragma unroll
                            for (int v = 0; v < VJ; ++v) aj[k][v] += a[u][v] * xv;
                        }
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < S; ++k) {
                    if (k >= s) continue;
                    const auto base = Jb + ((size_t)k * d.nnzb + pa) * m * ldJ + sJ * VJ;
                    constexpr int UJ = (VJ <= 4) ? 8 : 4;
                    for (int cb = gJ; cb < ncol; cb += UJ * GJ) {
                        TC a[UJ][VJ];
#pragma unroll
                        for (int u = 0; u < UJ; ++u) Vec16<TJ>::load(base + (size_t)min(cb + u * GJ, ncol - 1) * ldJ, a[u]);
#pragma unroll
                        for (int u = 0; u < UJ; ++u) {
                            const int cg = cb + u * GJ;
                            if (cg >= ncol) continue;
                            const TC xv = xg[k * maxg + cg];
#pragma unroll
                            for (int v = 0; v < VJ; ++v) aj[k][v] += a[u][v] * xv;
                        }
                    }
                }
            }
        }
        __syncthreads();
        if (has && gJ < GJ) {
#pragma unroll
            for (int k = 0; k < S; ++k) {
                if (k >= s) continue;
#pragma unroll
                for (int v = 0; v < VJ; ++v) xg[(gJ * S + k) * ldJ + sJ * VJ + v] = aj[k][v];
            }
        }
        __syncthreads();
        if (has) {
            for (int q = tid; q < s * m; q += team) {
                const int k = q / m, r = q - k * m;
                const TC u = dt * sum_groups<TC, S>(xg, GJ, k, ldJ, r);
                if (FWD) yv[k * ldv + r] += u;
                else uv[k * ldv + r] = u;
            }
        }
        __syncthreads();
    }

    TC *red = xg;
    GAS double *acc = acc_slot >= 0 ? gp(reinterpret_cast<double *>(d.vec[acc_slot])) : nullptr;

    if (!COUPLED) {
        // all stages at once: out_k = P_k^{-1} in_k
        const TC *in = FWD ? yv : uv;
        if (fact) {
#pragma unroll
            for (int k = 0; k < S; ++k) {
                if (k >= s) continue;
                TC ap[VF];
#pragma unroll
                for (int v = 0; v < VF; ++v) ap[v] = 0;
                col_product<TF, TC, NQ, PF>(Pb + ((long long)i * s + k) * bsF + sF * VF, ldF, m, gF, GF,
                                            rP[k], in + k * ldv, ap);
#pragma unroll
                for (int v = 0; v < VF; ++v) red[(gF * S + k) * ldF + sF * VF + v] = ap[v];
            }
        }
        __syncthreads();
        if (has) {
            for (int q = tid; q < s * m; q += team) {
                const int k = q / m, r = q - k * m;
                const TC sc = block_scale<TF, TC>(d.P16e, (long long)i * s + k);
                TC o = sc * sum_groups<TC, S>(red, GF, k, ldF, r);
                const long long gi = k * n + (long long)i * m + r;
                if (!FWD) o += yv[k * ldv + r];
                sty(yh + gi, o);
                if (!FWD && acc) acc[gi] += (double)o;
            }
        }
        return;
    }

    // ---- coupled: stage rounds inside the element ----
    // mass step (Jacobian-block layout): t = M_i vin; forward: y_l -= A^{-1}_l0 t
    // for every later stage; backward: u_0 -= t
    auto mass_step = [&](const TC *vin, bool act) {
        TC am[VJ];
#pragma unroll
        for (int v = 0; v < VJ; ++v) am[v] = 0;
        if (act && gJ < GJ) {
            col_product<TJ, TC, NQJ, PF>(Mb, ldJ, m, gJ, GJ, rM, vin, am);
#pragma unroll
            for (int v = 0; v < VJ; ++v) red[gJ * ldJ + sJ * VJ + v] = am[v];
        }
        __syncthreads();
        if (act) {
            for (int r = tid; r < m; r += team) {
                const TC t = sum_strided(red + r, GJ, ldJ);
                if (FWD) {
#pragma unroll
                    for (int l = 1; l < S; ++l)
                        if (l < s) yv[l * ldv + r] -= (TC)d.Ainv[l * SMAX] * t;
                } else {
                    uv[r] -= t;
                }
            }
        }
        __syncthreads();
    };
#pragma unroll
    for (int kk = 0; kk < S; ++kk) {
        const int k = FWD ? kk : (S - 1 - kk);
        const bool act = has && k < s;
        // backward, stage 0: the stage-0 couplings u_0 -= M_i sum_{l>=1} A^{-1}_0l z_l
        if (!FWD && k == 0 && S > 1) mass_step(av, has && s > 1);
        // (a) pivot product of stage k
        {
            const TC *in = FWD ? yv : uv;
            TC ap[VF];
#pragma unroll
            for (int v = 0; v < VF; ++v) ap[v] = 0;
            if (act && gF < GF) {
                col_product<TF, TC, NQ, PF>(Pb + ((long long)i * s + k) * bsF + sF * VF, ldF, m, gF, GF,
                                            rP[k], in + k * ldv, ap);
#pragma unroll
                for (int v = 0; v < VF; ++v) red[gF * ldF + sF * VF + v] = ap[v];
            }
            __syncthreads();
            if (act) {
                const TC sc = block_scale<TF, TC>(d.P16e, (long long)i * s + k);
                const TC a0k = (TC)d.Ainv[k];
                for (int r = tid; r < m; r += team) {
                    TC o = sum_strided(red + r, GF, ldF);
                    o *= sc;
                    const long long gi = k * n + (long long)i * m + r;
                    if (!FWD) o += yv[k * ldv + r];
                    sty(yh + gi, o);
                    if (!FWD && acc) acc[gi] += (double)o;
                    yv[k * ldv + r] = o;   // y^_k (forward) or z_k (backward) for the cross terms
                    // backward: a = sum over the stages done so far of A^{-1}_0k z_k
                    if (!FWD && k > 0) av[r] = (k == s - 1) ? a0k * o : av[r] + a0k * o;
                }
            }
            __syncthreads();
        }
        // (b) cross-stage update of the stages not yet done:
        //     forward: y_l -= C_{lk} y^_k (l > k);  backward: u_l -= C_{lk} z_k (1 <= l < k)
        if (FWD && k == 0 && S > 1) {
            mass_step(yv, has && s > 1);
        } else if (S > 2 && k >= 1 && (FWD ? k + 1 < S : k > 1)) {
            const bool cact = act && s > 2;
            if (cact && gF < GF) {
#pragma unroll
                for (int l = 1; l < S; ++l) {
                    if (l >= s || l == k || (FWD ? (l < k) : (l > k))) continue;
                    TC ac[VF];
#pragma unroll
                    for (int v = 0; v < VF; ++v) ac[v] = 0;
                    col_product<TF, TC, NQ, PF>(Cb + cross_idx(i, l, k) * bsF + sF * VF,
                                                ldF, m, gF, GF, rC[k][l], yv + k * ldv, ac);
#pragma unroll
                    for (int v = 0; v < VF; ++v) red[(gF * S + l) * ldF + sF * VF + v] = ac[v];
                }
            }
            __syncthreads();
            if (cact) {
                for (int q = tid; q < s * m; q += team) {
                    const int l = q / m, r = q - l * m;
                    if (l == 0 || l == k || (FWD ? (l < k) : (l > k))) continue;
                    const TC sc = block_scale<TF, TC>(d.C16e, cross_idx(i, l, k));
                    const TC cv = sc * sum_groups<TC, S>(red, GF, l, ldF, r);
                    if (FWD) yv[l * ldv + r] -= cv;
                    else uv[l * ldv + r] -= cv;
                }
            }
            __syncthreads();
        }
    }
}

// Same register budget as the host's choice of form: variants beyond it are
// never selected and are not instantiated.
constexpr int pf_form(int PFM, int S, bool coupled, bool fp64)
{
    return (PFM == 0) ? 0 :
           ((S + (coupled && S > 1 ? (S - 1) * (S - 2) / 2 + 1 : 0)) * (fp64 ? 16 : 8) +
            (PFM == 1 ? (fp64 ? 64 : 32) : 0) <= 176) ? PFM : 0;
}

}  // namespace irk
