/*
 * oracle.c -- plain, slow FP64 reference for the transformed Radau IIA linear
 * solve (Pazner & Persson, "Stage-parallel fully implicit Runge-Kutta solvers
 * for discontinuous Galerkin fluid simulations").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the solver library links, includes or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header, table or constant with
 * the HIP path.
 *
 * Conventions (the caller's layout):
 *   blocks are m x m, row-major;  vectors are stage-major [s][T][m];
 *   the Jacobian is BSR: row_ptr[T+1], col_idx[nnzb] (ascending, diagonal
 *   present), J[nJ][nnzb][m][m];  nJ = 1 means one Jacobian for all stages,
 *   nJ = s means J_k per stage;  the mass matrix is M[T][m][m].
 *
 * Everything is written as plain loops in FP64 with no blocking, no BLAS and
 * no reordering beyond what the cited definition states.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* small dense helpers                                                        */
/* ------------------------------------------------------------------------- */

/* C[n x n] = A[n x n] * B[n x n]  (row-major). */
static void mm(int n, const double *A, const double *B, double *C)
{
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) C[i * n + j] = 0.0;
        for (int k = 0; k < n; ++k) {
            double a = A[i * n + k];
            for (int j = 0; j < n; ++j) C[i * n + j] += a * B[k * n + j];
        }
    }
}

/* C -= A * B */
static void mm_sub(int n, const double *A, const double *B, double *C)
{
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            double a = A[i * n + k];
            for (int j = 0; j < n; ++j) C[i * n + j] -= a * B[k * n + j];
        }
}

/* y += alpha * A x */
static void mv_add(int n, double alpha, const double *A, const double *x, double *y)
{
    for (int i = 0; i < n; ++i) {
        double t = 0.0;
        for (int j = 0; j < n; ++j) t += A[i * n + j] * x[j];
        y[i] += alpha * t;
    }
}

/* LU factorization with partial (row) pivoting, in place:  P A = L U with L
 * unit lower.  piv[k] is the row swapped with row k at step k.
 * Returns 0, or k+1 if the pivot column k is exactly zero (or not finite). */
int orc_lu(int n, double *a, int *piv)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(a[k * n + k]);
        for (int r = k + 1; r < n; ++r)
            if (fabs(a[r * n + k]) > best) { best = fabs(a[r * n + k]); p = r; }
        if (!(best > 0.0) || !isfinite(best)) return k + 1;
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < n; ++j) {
                double t = a[k * n + j]; a[k * n + j] = a[p * n + j]; a[p * n + j] = t;
            }
        for (int r = k + 1; r < n; ++r) {
            double l = a[r * n + k] / a[k * n + k];
            a[r * n + k] = l;
            for (int j = k + 1; j < n; ++j) a[r * n + j] -= l * a[k * n + j];
        }
    }
    return 0;
}

/* Solve A x = b in place with the factors from orc_lu. */
void orc_lu_solve(int n, const double *lu, const int *piv, double *b)
{
    for (int k = 0; k < n; ++k)
        if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) b[i] -= lu[i * n + j] * b[j];
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) b[i] -= lu[i * n + j] * b[j];
        b[i] /= lu[i * n + i];
    }
}

/* Inverse through LU with partial pivoting and n column solves.
 * Returns 0 or the orc_lu failure code. */
int orc_inverse(int n, const double *a, double *ainv)
{
    double *lu = malloc(sizeof(double) * n * n);
    int *piv = malloc(sizeof(int) * n);
    double *col = malloc(sizeof(double) * n);
    memcpy(lu, a, sizeof(double) * n * n);
    int rc = orc_lu(n, lu, piv);
    if (rc == 0) {
        for (int j = 0; j < n; ++j) {
            for (int i = 0; i < n; ++i) col[i] = (i == j) ? 1.0 : 0.0;
            orc_lu_solve(n, lu, piv, col);
            for (int i = 0; i < n; ++i) ainv[i * n + j] = col[i];
        }
    }
    free(lu); free(piv); free(col);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Radau IIA tableau: construction of App. A (Axelsson's derivation).         */
/*   c_k  = zeros of Q_s(x) = P_s(2x-1) - P_{s-1}(2x-1), ascending;           */
/*   l_k  = Lagrange basis on the c's (equal to Q_s/((x-c_k) Q_s'(c_k)));     */
/*   a_ik = integral of l_k over [0, c_i];  b = last row of A (c_s = 1).      */
/* ------------------------------------------------------------------------- */

/* Legendre P_n(t) by the three-term recurrence (n+1)P_{n+1} = (2n+1)tP_n - nP_{n-1}. */
static double legendre(int n, double t)
{
    if (n == 0) return 1.0;
    double p0 = 1.0, p1 = t;
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
        p0 = p1; p1 = p2;
    }
    return p1;
}

static double radau_q(int s, double x) { return legendre(s, 2.0 * x - 1.0) - legendre(s - 1, 2.0 * x - 1.0); }
static double legendre_s(int s, double x) { return legendre(s, x); }

/* All roots of f(s, .) in [lo, hi]: sign changes on a uniform grid of nseg
 * segments, each refined by bisection to the last bit; exact grid zeros are
 * taken as they are.  Returns the number of roots found (ascending). */
static int grid_roots(double (*f)(int, double), int s, double lo, double hi,
                      int nseg, double *out, int cap)
{
    int cnt = 0;
    double xa = lo, fa = f(s, lo);
    if (fa == 0.0 && cnt < cap) out[cnt++] = lo;
    for (int q = 1; q <= nseg; ++q) {
        double xb = lo + (hi - lo) * (double)q / (double)nseg;
        double fb = f(s, xb);
        if (fb == 0.0) {
            if (cnt < cap) out[cnt++] = xb;
        } else if (fa != 0.0 && ((fa < 0.0) != (fb < 0.0))) {
            double a = xa, b = xb, fla = fa;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (a + b);
                if (mid <= a || mid >= b) break;
                double fm = f(s, mid);
                if (fm == 0.0) { a = b = mid; break; }
                if ((fm < 0.0) == (fla < 0.0)) { a = mid; fla = fm; } else b = mid;
            }
            if (cnt < cap) out[cnt++] = 0.5 * (a + b);
        }
        xa = xb; fa = fb;
    }
    return cnt;
}

/* Lagrange basis polynomial l_k on nodes c[0..s-1] at x. */
static double lagrange(int s, const double *c, int k, double x)
{
    double v = 1.0;
    for (int j = 0; j < s; ++j)
        if (j != k) v *= (x - c[j]) / (c[k] - c[j]);
    return v;
}

/* s-stage Radau IIA tableau (App. A).  A is s x s row-major.  Returns 0 on
 * success, -1 if the root count is wrong (s outside 1..20). */
int orc_radau_iia(int s, double *A, double *b, double *c)
{
    if (s < 1 || s > 20) return -1;
    double roots[64], gl[64], w[64];
    int nr = grid_roots(radau_q, s, 0.0, 1.0, 200000, roots, 64);
    if (nr != s) return -1;
    for (int i = 0; i < s; ++i) c[i] = roots[i];
    /* s-point Gauss-Legendre rule on [-1,1]: nodes = zeros of P_s,
     * weights 2 / ((1 - t^2) P_s'(t)^2), P_s'(t) = s (t P_s - P_{s-1}) / (t^2 - 1). */
    int ng = grid_roots(legendre_s, s, -1.0, 1.0, 200000, gl, 64);
    if (ng != s) return -1;
    for (int q = 0; q < s; ++q) {
        double t = gl[q];
        double dp = s * (t * legendre(s, t) - legendre(s - 1, t)) / (t * t - 1.0);
        w[q] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
    for (int i = 0; i < s; ++i)
        for (int k = 0; k < s; ++k) {
            double acc = 0.0;
            for (int q = 0; q < s; ++q) {
                double x = 0.5 * c[i] * (gl[q] + 1.0);
                acc += w[q] * lagrange(s, c, k, x);
            }
            A[i * s + k] = 0.5 * c[i] * acc;
        }
    for (int k = 0; k < s; ++k) b[k] = A[(s - 1) * s + k];
    return 0;
}

/* Shifts of the stage-uncoupled preconditioner (Sec. 4.3.2):
 *   rule 0: alpha_k = sum_{j != k} |Ainv[j][k]|   (the paper's choice)
 *   rule 1: alpha_k = 0                            (unshifted)
 *   rule 2: alpha_k = sum_{j != k} |Ainv[k][j]|   (row-sum variant)            */
void orc_shifts(int s, const double *Ainv, int rule, double *alpha)
{
    for (int k = 0; k < s; ++k) {
        double a = 0.0;
        for (int j = 0; j < s; ++j) {
            if (j == k) continue;
            if (rule == 0) a += fabs(Ainv[j * s + k]);
            else if (rule == 2) a += fabs(Ainv[k * s + j]);
        }
        alpha[k] = a;
    }
}

/* ------------------------------------------------------------------------- */
/* Operators                                                                  */
/* ------------------------------------------------------------------------- */

typedef struct {
    int s, T, m, nJ;
    const int32_t *row_ptr, *col_idx;
    const double *J;   /* [nJ][nnzb][m][m] */
    const double *M;   /* [T][m][m]        */
    double dt;
} orc_problem;

static const double *jblk(const orc_problem *p, int k, int pos)
{
    int kk = (p->nJ == 1) ? 0 : k;
    size_t nnzb = (size_t)p->row_ptr[p->T];
    return p->J + ((size_t)kk * nnzb + (size_t)pos) * p->m * p->m;
}

/* Transformed operator (Sec. 4.1, Eq. big-irk):
 *   y_k = sum_l Ainv[k][l] M x_l  -  dt J_k x_k. */
void orc_matvec_transformed(const orc_problem *p, const double *Ainv,
                            const double *x, double *y)
{
    int s = p->s, T = p->T, m = p->m;
    size_t n = (size_t)T * m;
#ifdef _OPENMP
#pragma omp parallel for collapse(2) schedule(static)
#endif
    for (int k = 0; k < s; ++k)
        for (int i = 0; i < T; ++i) {
            double *mx = malloc(sizeof(double) * m);
            double *yk = y + k * n + (size_t)i * m;
            for (int r = 0; r < m; ++r) yk[r] = 0.0;
            const double *Mi = p->M + (size_t)i * m * m;
            for (int l = 0; l < s; ++l) {
                for (int r = 0; r < m; ++r) mx[r] = 0.0;
                mv_add(m, 1.0, Mi, x + l * n + (size_t)i * m, mx);
                for (int r = 0; r < m; ++r) yk[r] += Ainv[k * s + l] * mx[r];
            }
            for (int q = p->row_ptr[i]; q < p->row_ptr[i + 1]; ++q) {
                int j = p->col_idx[q];
                mv_add(m, -p->dt, jblk(p, k, q), x + k * n + (size_t)j * m, yk);
            }
            free(mx);
        }
}

/* Untransformed Newton operator (Sec. 4.1, Eq. newton-system-2):
 *   y_k = M x_k  -  dt J_k sum_l a_kl x_l. */
void orc_matvec_untransformed(const orc_problem *p, const double *A,
                              const double *x, double *y)
{
    int s = p->s, T = p->T, m = p->m;
    size_t n = (size_t)T * m;
    double *comb = malloc(sizeof(double) * n);
    for (int k = 0; k < s; ++k) {
        for (size_t e = 0; e < n; ++e) {
            double t = 0.0;
            for (int l = 0; l < s; ++l) t += A[k * s + l] * x[l * n + e];
            comb[e] = t;
        }
        for (int i = 0; i < T; ++i) {
            double *yk = y + k * n + (size_t)i * m;
            for (int r = 0; r < m; ++r) yk[r] = 0.0;
            mv_add(m, 1.0, p->M + (size_t)i * m * m, x + k * n + (size_t)i * m, yk);
            for (int q = p->row_ptr[i]; q < p->row_ptr[i + 1]; ++q)
                mv_add(m, -p->dt, jblk(p, k, q), comb + (size_t)p->col_idx[q] * m, yk);
        }
    }
    free(comb);
}

/* ------------------------------------------------------------------------- */
/* Generic block sparse matrices and block ILU(0) (Sec. 4.2.1, Alg. 1)         */
/* ------------------------------------------------------------------------- */

/* Binary search of column c in the sorted row segment; -1 if absent. */
static long find_block(const int32_t *ptr, const int32_t *col, int row, int c)
{
    int lo = ptr[row], hi = ptr[row + 1] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (col[mid] == c) return mid;
        if (col[mid] < c) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Number of blocks of the stage-coupled matrix B (Sec. 4.3, Eq. big-irk) on
 * s*T block rows: the Jacobian pattern in every diagonal stage block plus one
 * element-diagonal mass block in every off-diagonal stage block. */
long orc_coupled_nnzb(int s, int T, const int32_t *row_ptr)
{
    return (long)s * row_ptr[T] + (long)s * (s - 1) * T;
}

/* Assemble B with block row/column (k, i) -> k*T + i (stage-major):
 *   B_{kl,ij} = Ainv[k][l] M_i delta_ij - delta_kl dt J_{k,ij}. */
void orc_build_coupled(const orc_problem *p, const double *Ainv,
                       int32_t *bptr, int32_t *bcol, double *bval)
{
    int s = p->s, T = p->T, m = p->m;
    size_t bs = (size_t)m * m;
    long pos = 0;
    bptr[0] = 0;
    for (int k = 0; k < s; ++k)
        for (int i = 0; i < T; ++i) {
            const double *Mi = p->M + (size_t)i * bs;
            for (int l = 0; l < k; ++l) {            /* earlier stages: mass only */
                bcol[pos] = l * T + i;
                for (size_t e = 0; e < bs; ++e) bval[pos * bs + e] = Ainv[k * s + l] * Mi[e];
                ++pos;
            }
            for (int q = p->row_ptr[i]; q < p->row_ptr[i + 1]; ++q) {
                int j = p->col_idx[q];
                const double *Jb = jblk(p, k, q);
                bcol[pos] = k * T + j;
                for (size_t e = 0; e < bs; ++e) {
                    double v = -p->dt * Jb[e];
                    if (j == i) v += Ainv[k * s + k] * Mi[e];
                    bval[pos * bs + e] = v;
                }
                ++pos;
            }
            for (int l = k + 1; l < s; ++l) {        /* later stages: mass only */
                bcol[pos] = l * T + i;
                for (size_t e = 0; e < bs; ++e) bval[pos * bs + e] = Ainv[k * s + l] * Mi[e];
                ++pos;
            }
            bptr[k * T + i + 1] = (int32_t)pos;
        }
}

/* One stage block of the uncoupled preconditioner (Sec. 4.3.2):
 *   (diag_coeff) M - dt J_k,   on the Jacobian pattern. */
void orc_build_stage(const orc_problem *p, int k, double diag_coeff,
                     int32_t *bptr, int32_t *bcol, double *bval)
{
    int T = p->T, m = p->m;
    size_t bs = (size_t)m * m;
    for (int i = 0; i <= T; ++i) bptr[i] = p->row_ptr[i];
    for (int i = 0; i < T; ++i)
        for (int q = p->row_ptr[i]; q < p->row_ptr[i + 1]; ++q) {
            int j = p->col_idx[q];
            const double *Jb = jblk(p, k, q);
            bcol[q] = j;
            for (size_t e = 0; e < bs; ++e) {
                double v = -p->dt * Jb[e];
                if (j == i) v += diag_coeff * p->M[(size_t)i * bs + e];
                bval[(size_t)q * bs + e] = v;
            }
        }
}

/* Block ILU(0) in place (Sec. 4.2.1, Alg. 1), in the matrix's own index
 * order, right-looking, with every update that stays inside the pattern:
 *   for each pivot p:
 *     for each q > p with (q,p) in the pattern:
 *        F_qp <- F_qp F_pp^{-1}
 *        for each t > p with (p,t) and (q,t) in the pattern:
 *           F_qt <- F_qt - F_qp F_pt
 * (the paper's line restricting t to t > q is read as every t > p; the set is
 * empty on triangle-free meshes).  F_pp^{-1} comes from LU with partial
 * pivoting.  On return, the strict block lower part holds L~ (unit block
 * diagonal implied) and the rest holds U~.  dlu/dpiv receive the LU factors
 * of every final diagonal block (nb*m*m and nb*m).  The pattern must be
 * structurally symmetric and hold every diagonal block.
 * Returns 0, or 1 + the block row whose pivot block is singular. */
int orc_ilu0(int nb, int m, const int32_t *ptr, const int32_t *col, double *val,
             double *dlu, int *dpiv)
{
    size_t bs = (size_t)m * m;
    double *inv = malloc(sizeof(double) * bs);
    int rc = 0;
    for (int pv = 0; pv < nb && rc == 0; ++pv) {
        long dpp = find_block(ptr, col, pv, pv);
        if (dpp < 0) { rc = 1 + pv; break; }
        memcpy(dlu + (size_t)pv * bs, val + dpp * bs, sizeof(double) * bs);
        if (orc_lu(m, dlu + (size_t)pv * bs, dpiv + (size_t)pv * m) != 0) { rc = 1 + pv; break; }
        if (orc_inverse(m, val + dpp * bs, inv) != 0) { rc = 1 + pv; break; }
        /* column pv below the pivot: rows q in row pv's pattern with q > pv
         * (pattern symmetric); each row q only touches its own blocks */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic)
#endif
        for (int a = ptr[pv]; a < ptr[pv + 1]; ++a) {
            int q = col[a];
            if (q <= pv) continue;
            long qp = find_block(ptr, col, q, pv);
            if (qp < 0) continue;
            double *tmp = malloc(sizeof(double) * bs);
            mm(m, val + qp * bs, inv, tmp);
            memcpy(val + qp * bs, tmp, sizeof(double) * bs);
            free(tmp);
            for (int b2 = ptr[pv]; b2 < ptr[pv + 1]; ++b2) {
                int t = col[b2];
                if (t <= pv) continue;
                long qt = find_block(ptr, col, q, t);
                if (qt < 0) continue;
                mm_sub(m, val + qp * bs, val + (long)b2 * bs, val + qt * bs);
            }
        }
    }
    free(inv);
    return rc;
}

/* Apply the ILU(0) preconditioner: solve L~ U~ z = v.
 *   forward  L~ y = v:  y_p = v_p - sum_{t<p} F_pt y_t         (ascending p)
 *   backward U~ z = y:  z_p = F_pp^{-1} (y_p - sum_{t>p} F_pt z_t)  (descending) */
void orc_ilu0_apply(int nb, int m, const int32_t *ptr, const int32_t *col,
                    const double *val, const double *dlu, const int *dpiv,
                    const double *v, double *z)
{
    size_t bs = (size_t)m * m;
    double *y = malloc(sizeof(double) * (size_t)nb * m);
    for (int pv = 0; pv < nb; ++pv) {
        double *yp = y + (size_t)pv * m;
        for (int r = 0; r < m; ++r) yp[r] = v[(size_t)pv * m + r];
        for (int a = ptr[pv]; a < ptr[pv + 1]; ++a) {
            int t = col[a];
            if (t >= pv) continue;
            mv_add(m, -1.0, val + (size_t)a * bs, y + (size_t)t * m, yp);
        }
    }
    for (int pv = nb - 1; pv >= 0; --pv) {
        double *zp = z + (size_t)pv * m;
        for (int r = 0; r < m; ++r) zp[r] = y[(size_t)pv * m + r];
        for (int a = ptr[pv]; a < ptr[pv + 1]; ++a) {
            int t = col[a];
            if (t <= pv) continue;
            mv_add(m, -1.0, val + (size_t)a * bs, z + (size_t)t * m, zp);
        }
        orc_lu_solve(m, dlu + (size_t)pv * bs, dpiv + (size_t)pv * m, zp);
    }
    free(y);
}

/* y = B x for a generic block matrix. */
void orc_bsr_matvec(int nb, int m, const int32_t *ptr, const int32_t *col,
                    const double *val, const double *x, double *y)
{
    size_t bs = (size_t)m * m;
    for (int i = 0; i < nb; ++i) {
        double *yi = y + (size_t)i * m;
        for (int r = 0; r < m; ++r) yi[r] = 0.0;
        for (int a = ptr[i]; a < ptr[i + 1]; ++a)
            mv_add(m, 1.0, val + (size_t)a * bs, x + (size_t)col[a] * m, yi);
    }
}

/* ------------------------------------------------------------------------- */
/* Stage-coupled ILU(0), explicit form on triangle-free meshes (Sec. 4.3.1,   */
/* Alg. 3 with its B_kk,ii factor read as B_kl,ii and with the cross-stage    */
/* updates of standard block ILU(0) for s >= 3).  A second, independent way   */
/* of computing what orc_ilu0 gives on the coupled matrix.                    */
/*   P[s][T][m][m]   pivot blocks (not inverted)                              */
/*   C[s][s][T][m][m] cross-stage blocks C_{kl,i}, k != l, as left by the      */
/*                    factorization (diagonal slots unused)                   */
/* ------------------------------------------------------------------------- */
int orc_coupled_explicit(const orc_problem *p, const double *Ainv, double *P, double *C)
{
    int s = p->s, T = p->T, m = p->m;
    size_t bs = (size_t)m * m;
    double *inv = malloc(sizeof(double) * bs);
    double *L = malloc(sizeof(double) * bs);
    double *t1 = malloc(sizeof(double) * bs);
#define PB(k, i) (P + ((size_t)(k) * T + (i)) * bs)
#define CB(k, l, i) (C + (((size_t)(k) * s + (l)) * T + (i)) * bs)
    for (int k = 0; k < s; ++k)
        for (int i = 0; i < T; ++i) {
            const double *Mi = p->M + (size_t)i * bs;
            long d = find_block(p->row_ptr, p->col_idx, i, i);
            const double *Jd = jblk(p, k, (int)d);
            for (size_t e = 0; e < bs; ++e) PB(k, i)[e] = Ainv[k * s + k] * Mi[e] - p->dt * Jd[e];
            for (int l = 0; l < s; ++l)
                if (l != k)
                    for (size_t e = 0; e < bs; ++e) CB(k, l, i)[e] = Ainv[k * s + l] * Mi[e];
        }
    int rc = 0;
    for (int k = 0; k < s && rc == 0; ++k)
        for (int i = 0; i < T; ++i) {
            if (orc_inverse(m, PB(k, i), inv) != 0) { rc = 1 + k * T + i; break; }
            /* same-stage neighbours j > i:  P_{k,j} -= (-dt J_ji) P^{-1} (-dt J_ij) */
            for (int q = p->row_ptr[i]; q < p->row_ptr[i + 1]; ++q) {
                int j = p->col_idx[q];
                if (j <= i) continue;
                long ji = find_block(p->row_ptr, p->col_idx, j, i);
                const double *Jji = jblk(p, k, (int)ji), *Jij = jblk(p, k, q);
                mm(m, Jji, inv, L);                  /* J_ji P^{-1} */
                for (size_t e = 0; e < bs; ++e) L[e] *= p->dt * p->dt;
                mm_sub(m, L, Jij, PB(k, j));
            }
            /* later stages at the same element */
            for (int l = k + 1; l < s; ++l) {
                mm(m, CB(l, k, i), inv, L);           /* L = C_{lk} P^{-1} */
                mm_sub(m, L, CB(k, l, i), PB(l, i));
                for (int q2 = k + 1; q2 < s; ++q2) {
                    if (q2 == l) continue;
                    mm(m, L, CB(k, q2, i), t1);
                    for (size_t e = 0; e < bs; ++e) CB(l, q2, i)[e] -= t1[e];
                }
            }
        }
#undef PB
#undef CB
    free(inv); free(L); free(t1);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Preconditioners and restarted GMRES                                         */
/* ------------------------------------------------------------------------- */

enum { ORC_PC_COUPLED = 0, ORC_PC_SHIFTED = 1, ORC_PC_UNSHIFTED = 2, ORC_PC_NONE = 3 };

typedef struct {
    int kind, s, T, m;
    int nfac;                 /* 1 (coupled) or s (uncoupled) */
    int nb[8];
    int32_t *ptr[8], *col[8];
    double *val[8], *dlu[8];
    int *dpiv[8];
} orc_pc;

typedef struct {
    const orc_problem *p;
    const double *Ainv;
} mv_ctx;

static void op_transformed(void *ctx, const double *x, double *y)
{
    mv_ctx *c = ctx;
    orc_matvec_transformed(c->p, c->Ainv, x, y);
}

static void op_pc(void *ctx, const double *v, double *z)
{
    orc_pc *pc = ctx;
    size_t n = (size_t)pc->T * pc->m;
    if (pc->kind == ORC_PC_NONE) { memcpy(z, v, sizeof(double) * pc->s * n); return; }
    if (pc->nfac == 1) {
        orc_ilu0_apply(pc->nb[0], pc->m, pc->ptr[0], pc->col[0], pc->val[0],
                       pc->dlu[0], pc->dpiv[0], v, z);
        return;
    }
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int k = 0; k < pc->s; ++k)
        orc_ilu0_apply(pc->nb[k], pc->m, pc->ptr[k], pc->col[k], pc->val[k],
                       pc->dlu[k], pc->dpiv[k], v + k * n, z + k * n);
}

static void pc_free(orc_pc *pc)
{
    for (int f = 0; f < pc->nfac; ++f) {
        free(pc->ptr[f]); free(pc->col[f]); free(pc->val[f]);
        free(pc->dlu[f]); free(pc->dpiv[f]);
    }
}

/* Build and factor the preconditioner.  Returns 0 or 1 + failing block row. */
static int pc_setup(orc_pc *pc, const orc_problem *p, const double *Ainv, int kind,
                    const double *alpha)
{
    memset(pc, 0, sizeof(*pc));
    pc->kind = kind; pc->s = p->s; pc->T = p->T; pc->m = p->m;
    size_t bs = (size_t)p->m * p->m;
    if (kind == ORC_PC_NONE) { pc->nfac = 0; return 0; }
    if (kind == ORC_PC_COUPLED) {
        pc->nfac = 1;
        long nnz = orc_coupled_nnzb(p->s, p->T, p->row_ptr);
        int nb = p->s * p->T;
        pc->nb[0] = nb;
        pc->ptr[0] = malloc(sizeof(int32_t) * (nb + 1));
        pc->col[0] = malloc(sizeof(int32_t) * nnz);
        pc->val[0] = malloc(sizeof(double) * nnz * bs);
        pc->dlu[0] = malloc(sizeof(double) * (size_t)nb * bs);
        pc->dpiv[0] = malloc(sizeof(int) * (size_t)nb * p->m);
        orc_build_coupled(p, Ainv, pc->ptr[0], pc->col[0], pc->val[0]);
        return orc_ilu0(nb, p->m, pc->ptr[0], pc->col[0], pc->val[0], pc->dlu[0], pc->dpiv[0]);
    }
    pc->nfac = p->s;
    long nnz = p->row_ptr[p->T];
    int bad = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int k = 0; k < p->s; ++k) {
        double dcoef = Ainv[k * p->s + k] + ((kind == ORC_PC_SHIFTED) ? alpha[k] : 0.0);
        pc->nb[k] = p->T;
        pc->ptr[k] = malloc(sizeof(int32_t) * (p->T + 1));
        pc->col[k] = malloc(sizeof(int32_t) * nnz);
        pc->val[k] = malloc(sizeof(double) * nnz * bs);
        pc->dlu[k] = malloc(sizeof(double) * (size_t)p->T * bs);
        pc->dpiv[k] = malloc(sizeof(int) * (size_t)p->T * p->m);
        orc_build_stage(p, k, dcoef, pc->ptr[k], pc->col[k], pc->val[k]);
        int rc = orc_ilu0(p->T, p->m, pc->ptr[k], pc->col[k], pc->val[k], pc->dlu[k], pc->dpiv[k]);
        if (rc) {
#ifdef _OPENMP
#pragma omp critical
#endif
            if (!bad || 1 + k * p->T + (rc - 1) < bad) bad = 1 + k * p->T + (rc - 1);
        }
    }
    return bad;
}

typedef void (*orc_op)(void *ctx, const double *in, double *out);

typedef struct {
    int converged, iters, restarts, status;
    double rel_res_true, rel_res_est;
} orc_info;

static double dot(size_t n, const double *a, const double *b)
{
    double t = 0.0;
#ifdef _OPENMP
#pragma omp parallel for reduction(+:t) schedule(static)
#endif
    for (size_t e = 0; e < n; ++e) t += a[e] * b[e];
    return t;
}

/* Restarted GMRES, right-preconditioned (Saad & Schultz), Givens rotations.
 *   A z and Minv v are the caller's operators;  x holds x0 on entry.
 *   orth = 0: modified Gram-Schmidt;  orth = 1: classical Gram-Schmidt with
 *   one re-orthogonalization pass (CGS2).
 *   A cycle ends when |g_{j+1}| <= rtol ||b|| (estimate), on happy breakdown
 *   or when maxit Arnoldi steps are spent; the update x += Minv V y follows,
 *   and convergence is only declared on the true residual ||b - A x|| / ||b||.
 *   hist (optional, maxit+1 entries) receives the estimate after each step.
 * Returns 0 converged, 4 not converged within maxit. */
int orc_gmres(size_t n, orc_op Aop, void *actx, orc_op Mop, void *mctx,
              const double *b, double *x, int restart, int maxit, double rtol,
              int orth, orc_info *info, double *hist)
{
    double *V = malloc(sizeof(double) * n * (restart + 1));
    double *H = calloc((size_t)(restart + 1) * restart, sizeof(double));
    double *cs = malloc(sizeof(double) * restart), *sn = malloc(sizeof(double) * restart);
    double *g = malloc(sizeof(double) * (restart + 1)), *yv = malloc(sizeof(double) * restart);
    double *w = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *h1 = malloc(sizeof(double) * (restart + 1));
    double bnorm = sqrt(dot(n, b, b));
    int iters = 0, restarts = 0, status = 4;
    double est = 0.0, truer = 0.0;
    if (bnorm == 0.0) {
        for (size_t e = 0; e < n; ++e) x[e] = 0.0;
        status = 0; truer = 0.0;
        goto done;
    }
    for (;;) {
        Aop(actx, x, w);
        for (size_t e = 0; e < n; ++e) w[e] = b[e] - w[e];
        double beta = sqrt(dot(n, w, w));
        truer = beta / bnorm;
        if (truer <= rtol) { status = 0; break; }
        if (iters >= maxit) { status = 4; break; }
        if (iters > 0) ++restarts;
        for (size_t e = 0; e < n; ++e) V[e] = w[e] / beta;
        for (int q = 0; q <= restart; ++q) g[q] = 0.0;
        g[0] = beta;
        int jl = -1;
        for (int j = 0; j < restart; ++j) {
            double *vj = V + (size_t)j * n, *vn = V + (size_t)(j + 1) * n;
            Mop(mctx, vj, z);
            Aop(actx, z, w);
            ++iters;
            double *Hj = H + (size_t)j;            /* column j, stride restart */
#define HH(r) H[(size_t)(r) * restart + j]
            if (orth == 0) {
                for (int i = 0; i <= j; ++i) {
                    double h = dot(n, V + (size_t)i * n, w);
                    HH(i) = h;
                    for (size_t e = 0; e < n; ++e) w[e] -= h * V[(size_t)i * n + e];
                }
            } else {
                for (int i = 0; i <= j; ++i) h1[i] = dot(n, V + (size_t)i * n, w);
                for (int i = 0; i <= j; ++i)
                    for (size_t e = 0; e < n; ++e) w[e] -= h1[i] * V[(size_t)i * n + e];
                for (int i = 0; i <= j; ++i) HH(i) = h1[i];
                for (int i = 0; i <= j; ++i) h1[i] = dot(n, V + (size_t)i * n, w);
                for (int i = 0; i <= j; ++i)
                    for (size_t e = 0; e < n; ++e) w[e] -= h1[i] * V[(size_t)i * n + e];
                for (int i = 0; i <= j; ++i) HH(i) += h1[i];
            }
            double hn = sqrt(dot(n, w, w));
            HH(j + 1) = hn;
            (void)Hj;
            for (int i = 0; i < j; ++i) {
                double a = HH(i), bb = HH(i + 1);
                HH(i) = cs[i] * a + sn[i] * bb;
                HH(i + 1) = -sn[i] * a + cs[i] * bb;
            }
            double a = HH(j), bb = HH(j + 1);
            double r = hypot(a, bb);
            if (r == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
            else { cs[j] = a / r; sn[j] = bb / r; }
            HH(j) = r; HH(j + 1) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
#undef HH
            est = fabs(g[j + 1]) / bnorm;
            if (hist) hist[iters - 1] = est;
            jl = j;
            if (hn == 0.0) break;                             /* happy breakdown */
            for (size_t e = 0; e < n; ++e) vn[e] = w[e] / hn;
            if (est <= rtol || iters >= maxit) break;
        }
        /* y = H^{-1} g (upper triangular, (jl+1) x (jl+1)) */
        for (int i = jl; i >= 0; --i) {
            double t = g[i];
            for (int k = i + 1; k <= jl; ++k) t -= H[(size_t)i * restart + k] * yv[k];
            yv[i] = t / H[(size_t)i * restart + i];
        }
        for (size_t e = 0; e < n; ++e) {
            double t = 0.0;
            for (int i = 0; i <= jl; ++i) t += yv[i] * V[(size_t)i * n + e];
            w[e] = t;
        }
        Mop(mctx, w, z);
        for (size_t e = 0; e < n; ++e) x[e] += z[e];
    }
done:
    if (info) {
        info->converged = (status == 0);
        info->iters = iters; info->restarts = restarts; info->status = status;
        info->rel_res_true = truer; info->rel_res_est = est;
    }
    free(V); free(H); free(cs); free(sn); free(g); free(yv); free(w); free(z); free(h1);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Full solve of B W = R (Sec. 4.3, Eq. big-irk) with GMRES + the chosen      */
/* block ILU(0) preconditioner.                                               */
/* ------------------------------------------------------------------------- */

typedef struct {
    int pc;          /* ORC_PC_* */
    int shift_rule;  /* 0 paper column sums, 1 none, 2 row sums */
    int restart, maxit, orth;
    double rtol;
} orc_opts;

/* A is the s x s Butcher matrix.  x holds x0 on entry.  Returns the GMRES
 * status, or 3 (singular pivot) / 1 (bad tableau). */
int orc_solve(const orc_problem *p, const double *A, const orc_opts *o,
              const double *rhs, double *x, orc_info *info, double *hist)
{
    int s = p->s;
    double Ainv[64], alpha[8];
    if (s < 1 || s > 8 || orc_inverse(s, A, Ainv) != 0) return 1;
    orc_shifts(s, Ainv, o->shift_rule, alpha);
    orc_pc pc;
    int rc = pc_setup(&pc, p, Ainv, o->pc, alpha);
    if (rc) { pc_free(&pc); if (info) { info->status = 3; info->converged = 0; } return 3; }
    mv_ctx mc = { p, Ainv };
    size_t N = (size_t)s * p->T * p->m;
    rc = orc_gmres(N, op_transformed, &mc, op_pc, &pc, rhs, x, o->restart, o->maxit,
                   o->rtol, o->orth, info, hist);
    pc_free(&pc);
    return rc;
}

/* Preconditioner apply on its own (for kernel-level parity): factor, then
 * z = P^{-1} v for each of nvec vectors.  Returns 0 or 3. */
int orc_pc_apply(const orc_problem *p, const double *A, int kind, int shift_rule,
                 int nvec, const double *v, double *z)
{
    int s = p->s;
    double Ainv[64], alpha[8];
    if (s < 1 || s > 8 || orc_inverse(s, A, Ainv) != 0) return 1;
    orc_shifts(s, Ainv, shift_rule, alpha);
    orc_pc pc;
    int rc = pc_setup(&pc, p, Ainv, kind, alpha);
    if (rc) { pc_free(&pc); return 3; }
    size_t N = (size_t)s * p->T * p->m;
    for (int q = 0; q < nvec; ++q) op_pc(&pc, v + q * N, z + q * N);
    pc_free(&pc);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Reduced-precision quantizers (pure functions of their input bits).         */
/* ------------------------------------------------------------------------- */

static uint32_t f32_bits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }

/* FP32 -> BF16, round to nearest even; NaN stays a quiet NaN. */
uint16_t orc_bf16_from_f32(float f)
{
    uint32_t u = f32_bits(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return (uint16_t)((u >> 16) | 0x0040u);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

/* FP32 -> IEEE binary16, round to nearest even, with subnormals, overflow to
 * infinity, NaN kept quiet. */
uint16_t orc_f16_from_f32(float f)
{
    uint32_t u = f32_bits(f);
    uint32_t sign = (u >> 16) & 0x8000u;
    uint32_t ex = (u >> 23) & 0xffu;
    uint32_t man = u & 0x007fffffu;
    if (ex == 0xffu) return (uint16_t)(sign | 0x7c00u | (man ? 0x0200u : 0u));
    int e = (int)ex - 127 + 15;                   /* biased half exponent */
    if (e >= 0x1f) return (uint16_t)(sign | 0x7c00u);
    if (e <= 0) {                                 /* half subnormal or zero */
        if (e < -10) return (uint16_t)sign;
        uint32_t mant = man | 0x00800000u;        /* 24 significant bits */
        int shift = 14 - e;                       /* 13 + (1 - e) */
        uint32_t q = mant >> shift;
        uint32_t rem = mant & ((1u << shift) - 1u);
        uint32_t half = 1u << (shift - 1);
        if (rem > half || (rem == half && (q & 1u))) ++q;
        return (uint16_t)(sign | q);
    }
    uint32_t q = ((uint32_t)e << 10) | (man >> 13);
    uint32_t rem = man & 0x1fffu;
    if (rem > 0x1000u || (rem == 0x1000u && (q & 1u))) ++q;   /* may carry into exponent */
    return (uint16_t)(sign | q);
}

/* Per-block power-of-two scale for the FP16 factor store: with |x|_max in
 * [2^(E-1), 2^E), the block is stored as x * 2^e, e = 14 - E, so every scaled
 * entry is below 2^14; e is clamped to [-100, 100]; a zero block gets e = 0. */
int orc_f16_block_exponent(size_t n, const double *x)
{
    double amax = 0.0;
    for (size_t q = 0; q < n; ++q) if (fabs(x[q]) > amax) amax = fabs(x[q]);
    if (!(amax > 0.0) || !isfinite(amax)) return 0;
    int E;
    frexp(amax, &E);
    int e = 14 - E;
    if (e < -100) e = -100;
    if (e > 100) e = 100;
    return e;
}

void orc_quantize_bf16(size_t n, const double *x, uint16_t *q)
{
    for (size_t i = 0; i < n; ++i) q[i] = orc_bf16_from_f32((float)x[i]);
}

void orc_quantize_f16_scaled(size_t n, const double *x, int e, uint16_t *q)
{
    for (size_t i = 0; i < n; ++i) q[i] = orc_f16_from_f32((float)ldexp(x[i], e));
}
