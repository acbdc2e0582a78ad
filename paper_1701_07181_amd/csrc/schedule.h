// schedule.h -- pattern checks and the level schedule (host only, no HIP).
//
// The block ILU(0) factorization and both sweeps visit elements level by
// level (Sec. 4.2.1): the forward level of element i is 1 + the largest
// forward level of its lower neighbours (0 without any), the backward level
// 1 + the largest backward level of its upper neighbours.  Elements of one
// level are independent in the factorization and in the forward (backward)
// sweep.  The method needs a structurally symmetric pattern with the
// diagonal stored and no triangles (no two neighbours of an element are
// neighbours of each other, Sec. 4.2.1), which is checked here too.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <vector>

namespace irk {

struct Schedule {
    std::vector<int> diag, tpos, lvl_fwd, lvl_bwd, off_fwd, off_bwd;
    int maxrow = 0;
};

enum SchedStatus { SCHED_OK = 0, SCHED_BAD_PATTERN = 1, SCHED_INCONSISTENT = 2 };

// Pattern (T block rows, nnzb blocks, row_ptr[T+1], col_idx[nnzb], columns
// ascending per row) -> diagonal and transpose positions, row length bound
// and the two level schedules.  SCHED_BAD_PATTERN: malformed row pointer,
// column out of range or unsorted, missing diagonal, asymmetric pattern or
// a triangle.  SCHED_INCONSISTENT: the finished schedule fails its own
// check (every element after the neighbours it reads, every element listed
// once), which would be a bug here.
inline int analyze_pattern(int T, int nnzb, const int32_t *rp, const int32_t *ci, Schedule &sc)
{
    if (T < 1 || nnzb < T || !rp || !ci) return SCHED_BAD_PATTERN;
    // the whole row pointer first: every later read of col_idx stays inside
    // [0, nnzb) only if rp starts at 0, never decreases and ends at nnzb
    if (rp[0] != 0 || rp[T] != nnzb) return SCHED_BAD_PATTERN;
    for (int i = 0; i < T; ++i)
        if (rp[i + 1] < rp[i] || rp[i + 1] > nnzb) return SCHED_BAD_PATTERN;
    sc.diag.assign(T, -1);
    sc.tpos.assign(nnzb, -1);
    sc.maxrow = 0;
    for (int i = 0; i < T; ++i) {
        sc.maxrow = std::max(sc.maxrow, rp[i + 1] - rp[i]);
        for (int q = rp[i]; q < rp[i + 1]; ++q) {
            if (ci[q] < 0 || ci[q] >= T) return SCHED_BAD_PATTERN;
            if (q > rp[i] && ci[q] <= ci[q - 1]) return SCHED_BAD_PATTERN;   // ascending, no repeats
            if (ci[q] == i) sc.diag[i] = q;
        }
        if (sc.diag[i] < 0) return SCHED_BAD_PATTERN;
    }
    auto find = [&](int row, int col) -> int {
        const int32_t *b = ci + rp[row], *e = ci + rp[row + 1];
        const int32_t *f = std::lower_bound(b, e, col);
        return (f != e && *f == col) ? int(f - ci) : -1;
    };
    // structural symmetry, transpose positions, triangle-freeness
    for (int i = 0; i < T; ++i)
        for (int q = rp[i]; q < rp[i + 1]; ++q) {
            const int j = ci[q];
            const int t = find(j, i);
            if (t < 0) return SCHED_BAD_PATTERN;
            sc.tpos[q] = t;
            if (j == i) continue;
            for (int q2 = q + 1; q2 < rp[i + 1]; ++q2) {
                const int k = ci[q2];
                if (k == i) continue;
                if (find(j, k) >= 0) return SCHED_BAD_PATTERN;   // j, k both neighbours of i and of each other
            }
        }
    // forward levels: lev(i) = 1 + max over lower neighbours
    std::vector<int> lf(T, 0), lb(T, 0);
    int Lf = 0, Lb = 0;
    for (int i = 0; i < T; ++i) {
        int l = 0;
        for (int q = rp[i]; q < sc.diag[i]; ++q) l = std::max(l, lf[ci[q]] + 1);
        lf[i] = l;
        Lf = std::max(Lf, l + 1);
    }
    for (int i = T - 1; i >= 0; --i) {
        int l = 0;
        for (int q = sc.diag[i] + 1; q < rp[i + 1]; ++q) l = std::max(l, lb[ci[q]] + 1);
        lb[i] = l;
        Lb = std::max(Lb, l + 1);
    }
    auto bucket = [&](const std::vector<int> &lev, int L, std::vector<int> &list, std::vector<int> &off) {
        off.assign(L + 1, 0);
        for (int i = 0; i < T; ++i) off[lev[i] + 1]++;
        for (int l = 0; l < L; ++l) off[l + 1] += off[l];
        list.assign(T, 0);
        std::vector<int> pos(off.begin(), off.end() - 1);
        for (int i = 0; i < T; ++i) list[pos[lev[i]]++] = i;
    };
    bucket(lf, Lf, sc.lvl_fwd, sc.off_fwd);
    bucket(lb, Lb, sc.lvl_bwd, sc.off_bwd);
    // self-check: each element listed once, at its level, after every
    // neighbour it reads (lower ones forward, upper ones backward)
    std::vector<int> seen_f(T, 0), seen_b(T, 0);
    for (int l = 0; l < Lf; ++l)
        for (int a = sc.off_fwd[l]; a < sc.off_fwd[l + 1]; ++a) {
            const int i = sc.lvl_fwd[a];
            if (i < 0 || i >= T || seen_f[i]++ || lf[i] != l) return SCHED_INCONSISTENT;
            for (int q = rp[i]; q < sc.diag[i]; ++q)
                if (lf[ci[q]] >= l) return SCHED_INCONSISTENT;
        }
    for (int l = 0; l < Lb; ++l)
        for (int a = sc.off_bwd[l]; a < sc.off_bwd[l + 1]; ++a) {
            const int i = sc.lvl_bwd[a];
            if (i < 0 || i >= T || seen_b[i]++ || lb[i] != l) return SCHED_INCONSISTENT;
            for (int q = sc.diag[i] + 1; q < rp[i + 1]; ++q)
                if (lb[ci[q]] >= l) return SCHED_INCONSISTENT;
        }
    if (sc.off_fwd[Lf] != T || sc.off_bwd[Lb] != T) return SCHED_INCONSISTENT;
    return SCHED_OK;
}

}  // namespace irk
