/*
 * FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Liu & Chen, arXiv 1701.05913.  Each function names the passage it
 * follows.  Nothing here is blocked, fused or reordered beyond what the
 * definition states; loops run in row order, sums in column order.
 * Compile without -ffast-math and without FMA contraction.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ======================================================================
 * Small dense helpers for bs x bs blocks (row-major)
 * ====================================================================== */

/* y -= A x */
static void blk_sub_mv(int bs, const double *A, const double *x, double *y)
{
    for (int r = 0; r < bs; r++) {
        double s = 0.0;
        for (int c = 0; c < bs; c++) s += A[r * bs + c] * x[c];
        y[r] -= s;
    }
}

/* C = A B */
static void blk_mm(int bs, const double *A, const double *B, double *C)
{
    for (int r = 0; r < bs; r++)
        for (int c = 0; c < bs; c++) {
            double s = 0.0;
            for (int k = 0; k < bs; k++) s += A[r * bs + k] * B[k * bs + c];
            C[r * bs + c] = s;
        }
}

static double blk_norm_inf(int bs, const double *A)
{
    double m = 0.0;
    for (int r = 0; r < bs; r++) {
        double s = 0.0;
        for (int c = 0; c < bs; c++) s += fabs(A[r * bs + c]);
        if (s > m) m = s;
    }
    return m;
}

/* Solve A X = B for X (bs x nrhs, row-major, nrhs columns) by Gaussian
 * elimination with partial pivoting (first maximal pivot on ties).
 * Zero pivot: |pivot| < 1e-14 ||A||_inf for bs > 1, |a| < 1e-300 for
 * bs = 1, or a non-finite pivot.  Returns 0 or OR_ERR_ZERO_PIVOT. */
static int blk_solve(int bs, const double *A, double *X, int nrhs)
{
    double M[64], R[64 * 64];
    double anorm = blk_norm_inf(bs, A);
    memcpy(M, A, sizeof(double) * bs * bs);
    memcpy(R, X, sizeof(double) * bs * nrhs);
    for (int k = 0; k < bs; k++) {
        int piv = k;
        double best = fabs(M[k * bs + k]);
        for (int r = k + 1; r < bs; r++)
            if (fabs(M[r * bs + k]) > best) { best = fabs(M[r * bs + k]); piv = r; }
        if (!isfinite(best)) return OR_ERR_ZERO_PIVOT;
        if (bs == 1 ? best < 1e-300 : best < 1e-14 * anorm) return OR_ERR_ZERO_PIVOT;
        if (piv != k) {
            for (int c = 0; c < bs; c++) {
                double t = M[k * bs + c]; M[k * bs + c] = M[piv * bs + c]; M[piv * bs + c] = t;
            }
            for (int c = 0; c < nrhs; c++) {
                double t = R[k * nrhs + c]; R[k * nrhs + c] = R[piv * nrhs + c]; R[piv * nrhs + c] = t;
            }
        }
        for (int r = k + 1; r < bs; r++) {
            double f = M[r * bs + k] / M[k * bs + k];
            for (int c = k; c < bs; c++) M[r * bs + c] -= f * M[k * bs + c];
            for (int c = 0; c < nrhs; c++) R[r * nrhs + c] -= f * R[k * nrhs + c];
        }
    }
    for (int k = bs - 1; k >= 0; k--)
        for (int c = 0; c < nrhs; c++) {
            double s = R[k * nrhs + c];
            for (int j = k + 1; j < bs; j++) s -= M[k * bs + j] * R[j * nrhs + c];
            R[k * nrhs + c] = s / M[k * bs + k];
        }
    memcpy(X, R, sizeof(double) * bs * nrhs);
    return 0;
}

static int blk_inverse(int bs, const double *A, double *Ainv)
{
    for (int r = 0; r < bs; r++)
        for (int c = 0; c < bs; c++) Ainv[r * bs + c] = (r == c) ? 1.0 : 0.0;
    return blk_solve(bs, A, Ainv, bs);
}

static double dot(int n, const double *x, const double *y)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int i = 0; i < n; i++) s += x[i] * y[i];
    return s;
}

static double nrm2(int n, const double *x) { return sqrt(dot(n, x, x)); }

static int diag_pos(const int *rp, const int *ci, int i)
{
    for (int p = rp[i]; p < rp[i + 1]; p++)
        if (ci[p] == i) return p;
    return -1;
}

/* ======================================================================
 * Precision emulation
 * ====================================================================== */
float or_bf16_round(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) {          /* inf / nan */
        if (u & 0x007fffffu) u |= 0x00400000u;
        u &= 0xffff0000u;
    } else {
        u += 0x7fffu + ((u >> 16) & 1u);              /* nearest, ties to even */
        u &= 0xffff0000u;
    }
    memcpy(&f, &u, 4);
    return f;
}

static double bf16d(double x) { return (double)or_bf16_round((float)x); }

/* The SpMV row loops, dot products and the vector loops of GMRES carry
 * OpenMP pragmas, as the paper's kernels carry USE_OMP loops; a plain
 * build (no -fopenmp, the correctness reference) ignores them.  The
 * triangular sweeps and the factorization stay serial.
 * ======================================================================
 * C1. SpMV -- Figures 20 and 21: y_i = sum_j a_ij x_j row by row.
 * ====================================================================== */
void or_bsr_spmv(int nb, int bs, const int *rp, const int *ci,
                 const double *a, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nb; i++) {
        for (int r = 0; r < bs; r++) {
            double t = 0.0;
            for (int p = rp[i]; p < rp[i + 1]; p++) {
                const double *blk = a + (size_t)p * bs * bs;
                const double *xj = x + (size_t)ci[p] * bs;
                for (int c = 0; c < bs; c++) t += blk[r * bs + c] * xj[c];
            }
            y[(size_t)i * bs + r] = t;
        }
    }
}

/* y = alpha A x + beta y  (Figure 21) */
void or_bsr_amxpby(int nb, int bs, const int *rp, const int *ci,
                   const double *a, double alpha, const double *x,
                   double beta, double *y)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nb; i++) {
        for (int r = 0; r < bs; r++) {
            double t = 0.0;
            for (int p = rp[i]; p < rp[i + 1]; p++) {
                const double *blk = a + (size_t)p * bs * bs;
                const double *xj = x + (size_t)ci[p] * bs;
                for (int c = 0; c < bs; c++) t += blk[r * bs + c] * xj[c];
            }
            y[(size_t)i * bs + r] = alpha * t + beta * y[(size_t)i * bs + r];
        }
    }
}

/* ======================================================================
 * C2/C3. ILU(0) and block ILU(0): incomplete LU restricted to the pattern
 * of A, row-oriented (IKJ) elimination, no pivoting across rows.
 *   for each row i, for each k < i in row i (ascending):
 *       a_ik <- a_ik * a_kk^{-1}
 *       for each j > k in row k with (i, j) in the pattern:
 *           a_ij <- a_ij - a_ik * a_kj
 * Output lu: strictly-lower blocks hold L (unit block diagonal implied),
 * diagonal and upper blocks hold U.
 * ====================================================================== */
int or_bilu0(int nb, int bs, const int *rp, const int *ci,
             const double *a, double *lu)
{
    const int b2 = bs * bs;
    memcpy(lu, a, sizeof(double) * (size_t)rp[nb] * b2);
    double inv[64], tmp[64];
    for (int i = 0; i < nb; i++) {
        int di = diag_pos(rp, ci, i);
        if (di < 0) return OR_ERR_ARG;
        for (int p = rp[i]; p < rp[i + 1]; p++) {
            int k = ci[p];
            if (k >= i) break;
            int dk = diag_pos(rp, ci, k);
            if (blk_inverse(bs, lu + (size_t)dk * b2, inv)) return OR_ERR_ZERO_PIVOT;
            blk_mm(bs, lu + (size_t)p * b2, inv, tmp);
            memcpy(lu + (size_t)p * b2, tmp, sizeof(double) * b2);
            for (int q = dk + 1; q < rp[k + 1]; q++) {
                int j = ci[q];
                for (int s = rp[i]; s < rp[i + 1]; s++) {
                    if (ci[s] == j) {
                        blk_mm(bs, lu + (size_t)p * b2, lu + (size_t)q * b2, tmp);
                        for (int e = 0; e < b2; e++) lu[(size_t)s * b2 + e] -= tmp[e];
                        break;
                    }
                }
            }
        }
        if (blk_inverse(bs, lu + (size_t)di * b2, inv)) return OR_ERR_ZERO_PIVOT;
    }
    return OR_OK;
}

/* C4, eq. (3): L y = b row by row (unit lower) */
void or_bilu0_solve_lower(int nb, int bs, const int *rp, const int *ci,
                          const double *lu, const double *b, double *y)
{
    const int b2 = bs * bs;
    for (int i = 0; i < nb; i++) {
        double t[8];
        for (int r = 0; r < bs; r++) t[r] = b[(size_t)i * bs + r];
        for (int p = rp[i]; p < rp[i + 1] && ci[p] < i; p++)
            blk_sub_mv(bs, lu + (size_t)p * b2, y + (size_t)ci[p] * bs, t);
        for (int r = 0; r < bs; r++) y[(size_t)i * bs + r] = t[r];
    }
}

/* C4, eq. (3): U x = y from the last row up; U_ii solved by elimination */
void or_bilu0_solve_upper(int nb, int bs, const int *rp, const int *ci,
                          const double *lu, const double *y, double *x)
{
    const int b2 = bs * bs;
    for (int i = nb - 1; i >= 0; i--) {
        double t[8];
        int di = -1;
        for (int r = 0; r < bs; r++) t[r] = y[(size_t)i * bs + r];
        for (int p = rp[i]; p < rp[i + 1]; p++) {
            if (ci[p] == i) di = p;
            if (ci[p] > i) blk_sub_mv(bs, lu + (size_t)p * b2, x + (size_t)ci[p] * bs, t);
        }
        if (blk_solve(bs, lu + (size_t)di * b2, t, 1)) {
            for (int r = 0; r < bs; r++) t[r] = NAN;
        }
        for (int r = 0; r < bs; r++) x[(size_t)i * bs + r] = t[r];
    }
}

void or_bilu0_solve(int nb, int bs, const int *rp, const int *ci,
                    const double *lu, const double *b, double *x)
{
    double *y = (double *)malloc(sizeof(double) * (size_t)nb * bs);
    or_bilu0_solve_lower(nb, bs, rp, ci, lu, b, y);
    or_bilu0_solve_upper(nb, bs, rp, ci, lu, y, x);
    free(y);
}

/* ----------------------------------------------------------------------
 * Reduced-precision ILU(0) apply (mixed-precision extension).
 * Factor computed in FP64 (or_bilu0), then stored rounded: off-diagonal
 * L and U blocks to float (or to bfloat16 held in a float), the inverse of
 * each diagonal U block computed in FP64 and rounded to float.  The apply
 * is the same two sweeps as eq. (3), in float arithmetic, with the
 * backward step x_i = U_ii^{-1} (y_i - sum_j U_ij x_j).
 * ---------------------------------------------------------------------- */
typedef struct {
    int nb, bs;
    const int *rp, *ci;
    float *f;    /* nnzb*b2: off-diagonal blocks rounded; diagonal -> U_ii^-1 */
    float *y, *x;
} lowp_lu;

static int lowp_init(lowp_lu *L, int nb, int bs, const int *rp,
                     const int *ci, const double *lu, int prec)
{
    const int b2 = bs * bs;
    size_t nnzb = (size_t)rp[nb];
    L->nb = nb; L->bs = bs; L->rp = rp; L->ci = ci;
    L->f = (float *)malloc(sizeof(float) * nnzb * b2);
    L->y = (float *)malloc(sizeof(float) * (size_t)nb * bs);
    L->x = (float *)malloc(sizeof(float) * (size_t)nb * bs);
    double inv[64];
    for (int i = 0; i < nb; i++)
        for (int p = rp[i]; p < rp[i + 1]; p++) {
            if (ci[p] == i) {
                if (blk_inverse(bs, lu + (size_t)p * b2, inv)) return OR_ERR_ZERO_PIVOT;
                for (int e = 0; e < b2; e++) L->f[(size_t)p * b2 + e] = (float)inv[e];
            } else {
                for (int e = 0; e < b2; e++) {
                    float v = (float)lu[(size_t)p * b2 + e];
                    L->f[(size_t)p * b2 + e] = (prec == OR_PREC_BF16) ? or_bf16_round(v) : v;
                }
            }
        }
    return OR_OK;
}

static void lowp_free(lowp_lu *L)
{
    free(L->f); free(L->y); free(L->x);
    memset(L, 0, sizeof(*L));
}

/* x = (LU)^-1 b in float; b and x given as float arrays */
static void lowp_apply(lowp_lu *L, const float *b, float *x)
{
    const int bs = L->bs, b2 = bs * bs;
    const int *rp = L->rp, *ci = L->ci;
    for (int i = 0; i < L->nb; i++) {
        float t[8];
        for (int r = 0; r < bs; r++) t[r] = b[(size_t)i * bs + r];
        for (int p = rp[i]; p < rp[i + 1] && ci[p] < i; p++) {
            const float *blk = L->f + (size_t)p * b2;
            const float *yk = L->y + (size_t)ci[p] * bs;
            for (int r = 0; r < bs; r++) {
                float s = 0.0f;
                for (int c = 0; c < bs; c++) s += blk[r * bs + c] * yk[c];
                t[r] -= s;
            }
        }
        for (int r = 0; r < bs; r++) L->y[(size_t)i * bs + r] = t[r];
    }
    for (int i = L->nb - 1; i >= 0; i--) {
        float t[8], u[8];
        int di = -1;
        for (int r = 0; r < bs; r++) t[r] = L->y[(size_t)i * bs + r];
        for (int p = rp[i]; p < rp[i + 1]; p++) {
            if (ci[p] == i) { di = p; continue; }
            if (ci[p] < i) continue;
            const float *blk = L->f + (size_t)p * b2;
            const float *xj = x + (size_t)ci[p] * bs;
            for (int r = 0; r < bs; r++) {
                float s = 0.0f;
                for (int c = 0; c < bs; c++) s += blk[r * bs + c] * xj[c];
                t[r] -= s;
            }
        }
        const float *dinv = L->f + (size_t)di * b2;
        for (int r = 0; r < bs; r++) {
            float s = 0.0f;
            for (int c = 0; c < bs; c++) s += dinv[r * bs + c] * t[c];
            u[r] = s;
        }
        for (int r = 0; r < bs; r++) x[(size_t)i * bs + r] = u[r];
    }
}

/* ======================================================================
 * C8. CPR with quasi-IMPES decoupling (eqs. (5)-(9), Algorithms 5-8).
 * Block unknown 0 is the pressure; Pi_r picks it, Pi_p injects it.
 * Quasi-IMPES weight of cell i from its diagonal block
 *   D_i = [[d_pp, d_ps^T], [d_sp, D_ss]]:  w_i^T = [1, -d_ps^T D_ss^{-1}],
 * so that w_i^T D_i has zeros in the secondary columns.
 * Pressure matrix: (A_pp)_ij = w_i^T A_ij e_0, on the block pattern of A.
 * ====================================================================== */
int or_cpr_weights(int nb, const int *rp, const int *ci, const double *a,
                   double *w)
{
    for (int i = 0; i < nb; i++) {
        int d = diag_pos(rp, ci, i);
        if (d < 0) return OR_ERR_ARG;
        const double *D = a + (size_t)d * 9;
        /* solve D_ss^T y = d_ps  ->  w_s = -y */
        double Dss_T[4] = { D[4], D[7], D[5], D[8] };
        double y[2] = { D[1], D[2] };
        if (blk_solve(2, Dss_T, y, 1)) return OR_ERR_ZERO_PIVOT;
        w[3 * i + 0] = 1.0;
        w[3 * i + 1] = -y[0];
        w[3 * i + 2] = -y[1];
    }
    return OR_OK;
}

void or_cpr_extract_pressure(int nb, const int *rp, const int *ci,
                             const double *a, const double *w, double *app)
{
    for (int i = 0; i < nb; i++)
        for (int p = rp[i]; p < rp[i + 1]; p++) {
            const double *B = a + (size_t)p * 9;
            app[p] = w[3 * i] * B[0] + w[3 * i + 1] * B[3] + w[3 * i + 2] * B[6];
        }
}

/* ======================================================================
 * Algebraic multigrid (Section 4.2: Algorithms 3 and 4, eq. (4), the
 * defaults of Figure 34).  Classical Ruge-Stueben AMG on a scalar CSR
 * matrix, one level at a time (Algorithm 3):
 *   strength       j is a strong dependency of i when
 *                  -s a_ij >= theta max_{k != i} (-s a_ik), s = sign(a_ii);
 *                  a row with |sum_j a_ij| > max_row_sum |a_ii| has none
 *   coarse points  Ruge-Stueben first pass (the undecided point of largest
 *                  measure becomes C, ties to the smallest index, and the
 *                  undecided points depending on it become F; a measure
 *                  starts at the number of points depending on the point,
 *                  +1 when one of them becomes F that way, -1 when one
 *                  becomes C; a point taken with measure 0 becomes F) and
 *                  second pass (a strong F-F pair shares a C point)
 *   interpolation  classical: an F point interpolates from its strong C
 *                  points; its strong F neighbours are distributed over
 *                  them through their entries of sign opposite to their
 *                  diagonal (the "modified" restriction), weak neighbours
 *                  are lumped into the diagonal; weights below trunc times
 *                  the row's largest are dropped and the row rescaled to
 *                  keep its sum
 *   restriction    R = P^T; coarse matrix A_{l+1} = R A_l P (eq. (4))
 *   smoother       hybrid Gauss-Seidel, forward: Gauss-Seidel inside
 *                  contiguous chunks of gs_chunk rows (all rows when <= 0),
 *                  Jacobi between chunks; num_sweeps sweeps before and
 *                  after the coarse correction
 *   cycle          V-cycle from x = 0 on every level (Algorithm 4), the
 *                  coarsest level solved exactly (dense LU)
 * Rounding order, where it decides a later integer choice: row sums and
 * maxima in ascending column order; (A P)_iJ = sum over the entries of row
 * i of A in ascending order of a_ik P_kJ; (R (A P))_IJ = sum over the
 * entries of row I of R in ascending order of R_Ii (A P)_iJ.
 * ====================================================================== */
void or_amg_defaults(or_amg_opts *o)
{
    o->strength = 0.5;
    o->max_row_sum = 0.9;
    o->trunc = 1e-2;
    o->max_levels = 8;
    o->num_sweeps = 2;
    o->gs_chunk = 0;
    o->coarse_size = 9;
}

typedef struct {
    int n, nc;
    int *rp, *ci; double *a;            /* A_l                          */
    int *cf;                            /* 1 = C point, 0 = F point     */
    int *prp, *pci; double *pv;         /* P_l, n x nc                  */
    int *trp, *tci; double *tv;         /* R_l = P_l^T, nc x n          */
    double *lu; int *piv;               /* coarsest level: dense LU     */
    double *x, *b, *r, *t;
} amg_level;

struct or_amg {
    or_amg_opts o;
    int nlev;
    amg_level *lev;
};

/* strong dependencies S_i of every row, ascending; sci holds rp[n] ints */
int or_amg_strength(int n, const int *rp, const int *ci, const double *a,
                    double theta, double max_row_sum, int *srp, int *sci)
{
    int m = 0;
    srp[0] = 0;
    for (int i = 0; i < n; i++) {
        double diag = 0.0, rsum = 0.0, mx = 0.0;
        for (int q = rp[i]; q < rp[i + 1]; q++) {
            if (ci[q] == i) diag = a[q];
            rsum += a[q];
        }
        const double s = diag < 0.0 ? -1.0 : 1.0;
        for (int q = rp[i]; q < rp[i + 1]; q++)
            if (ci[q] != i && -s * a[q] > mx) mx = -s * a[q];
        const int dependent = !(max_row_sum < 1.0 && fabs(rsum) > max_row_sum * fabs(diag));
        if (dependent && mx > 0.0)
            for (int q = rp[i]; q < rp[i + 1]; q++)
                if (ci[q] != i && -s * a[q] >= theta * mx) sci[m++] = ci[q];
        srp[i + 1] = m;
    }
    return m;
}

/* transpose of a pattern (rows of the result ascending) */
static void pattern_transpose(int n, int m, const int *rp, const int *ci, int *trp, int *tci,
                              const double *v, double *tv)
{
    for (int j = 0; j <= m; j++) trp[j] = 0;
    for (int q = 0; q < rp[n]; q++) trp[ci[q] + 1]++;
    for (int j = 0; j < m; j++) trp[j + 1] += trp[j];
    int *fill = (int *)malloc(sizeof(int) * (size_t)(m + 1));
    memcpy(fill, trp, sizeof(int) * (size_t)(m + 1));
    for (int i = 0; i < n; i++)
        for (int q = rp[i]; q < rp[i + 1]; q++) {
            const int p = fill[ci[q]]++;
            tci[p] = i;
            if (v) tv[p] = v[q];
        }
    free(fill);
}

/* binary max-heap on (measure, -index) */
typedef struct { int lam, i; } amg_hent;
typedef struct { amg_hent *h; int n, cap; } amg_heap;

static int hfirst(amg_hent a, amg_hent b) { return a.lam > b.lam || (a.lam == b.lam && a.i < b.i); }

static void heap_push(amg_heap *H, int lam, int i)
{
    if (H->n == H->cap) {
        H->cap = H->cap ? 2 * H->cap : 64;
        H->h = (amg_hent *)realloc(H->h, sizeof(amg_hent) * (size_t)H->cap);
    }
    int c = H->n++;
    H->h[c].lam = lam; H->h[c].i = i;
    while (c > 0) {
        int p = (c - 1) / 2;
        if (!hfirst(H->h[c], H->h[p])) break;
        amg_hent t = H->h[c]; H->h[c] = H->h[p]; H->h[p] = t;
        c = p;
    }
}

static amg_hent heap_pop(amg_heap *H)
{
    amg_hent top = H->h[0];
    H->h[0] = H->h[--H->n];
    int c = 0;
    for (;;) {
        int l = 2 * c + 1, r = l + 1, b = c;
        if (l < H->n && hfirst(H->h[l], H->h[b])) b = l;
        if (r < H->n && hfirst(H->h[r], H->h[b])) b = r;
        if (b == c) break;
        amg_hent t = H->h[c]; H->h[c] = H->h[b]; H->h[b] = t;
        c = b;
    }
    return top;
}

/* C/F splitting: cf[i] = 1 (C) or 0 (F) */
static void amg_coarsen(int n, const int *srp, const int *sci, const int *trp,
                        const int *tci, int *cf)
{
    enum { UND = -1, FPT = 0, CPT = 1 };
    int *lam = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    amg_heap H = { NULL, 0, 0 };
    for (int i = 0; i < n; i++) {
        lam[i] = trp[i + 1] - trp[i];               /* points depending on i */
        cf[i] = (srp[i + 1] == srp[i] && lam[i] == 0) ? FPT : UND;
        if (cf[i] == UND) heap_push(&H, lam[i], i);
    }
    /* first pass */
    while (H.n > 0) {
        const amg_hent e = heap_pop(&H);
        const int i = e.i;
        if (cf[i] != UND || e.lam != lam[i]) continue;   /* stale entry */
        if (lam[i] == 0) { cf[i] = FPT; continue; }
        cf[i] = CPT;
        for (int q = trp[i]; q < trp[i + 1]; q++) {      /* j depends on i */
            const int j = tci[q];
            if (cf[j] != UND) continue;
            cf[j] = FPT;
            for (int p = srp[j]; p < srp[j + 1]; p++) {  /* j depends on k */
                const int k = sci[p];
                if (cf[k] == UND) { lam[k]++; heap_push(&H, lam[k], k); }
            }
        }
        for (int q = srp[i]; q < srp[i + 1]; q++) {      /* i depends on j */
            const int j = sci[q];
            if (cf[j] == UND) { lam[j]--; heap_push(&H, lam[j], j); }
        }
    }
    free(H.h);
    /* second pass: every strong F neighbour j of an F point i must depend
     * strongly on a C point of i; one offender becomes C, a second one
     * makes i itself C instead */
    int *mark = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    for (int i = 0; i < n; i++) mark[i] = -1;
    for (int i = 0; i < n; i++) {
        if (cf[i] != FPT) continue;
        for (int q = srp[i]; q < srp[i + 1]; q++)
            if (cf[sci[q]] == CPT) mark[sci[q]] = i;
        int tent = -1;
        for (int q = srp[i]; q < srp[i + 1] && cf[i] == FPT; q++) {
            const int j = sci[q];
            if (cf[j] != FPT || j == tent) continue;
            int common = 0;
            for (int p = srp[j]; p < srp[j + 1] && !common; p++)
                common = mark[sci[p]] == i;
            if (common) continue;
            if (tent >= 0) cf[i] = CPT;
            else { tent = j; mark[j] = i; }
        }
        if (cf[i] == FPT && tent >= 0) cf[tent] = CPT;
    }
    free(mark);
    free(lam);
}

static int opposite(double akk, double akm)
{
    return (akk > 0.0 && akm < 0.0) || (akk < 0.0 && akm > 0.0);
}

/* classical interpolation with truncation; P rows: C point -> its coarse
 * number with weight 1, F point -> its strong C points */
static int amg_interp(int n, const int *rp, const int *ci, const double *a, const int *srp,
                      const int *sci, const int *cf, double trunc, int *nc_out,
                      int **prp_o, int **pci_o, double **pv_o)
{
    int *cmap = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    int nc = 0;
    for (int i = 0; i < n; i++) cmap[i] = cf[i] ? nc++ : -1;
    int *prp = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    int cap = srp[n] + n + 1;
    int *pci = (int *)malloc(sizeof(int) * (size_t)cap);
    double *pv = (double *)malloc(sizeof(double) * (size_t)cap);
    int *sm = (int *)malloc(sizeof(int) * (size_t)(n + 1));   /* strong stamp */
    int *pos = (int *)malloc(sizeof(int) * (size_t)(n + 1));  /* place in C_i */
    int *cl = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    double *num = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    for (int i = 0; i < n; i++) { sm[i] = -1; pos[i] = -1; }
    int m = 0, e = OR_OK;
    prp[0] = 0;
    for (int i = 0; i < n && !e; i++) {
        if (cf[i]) {
            pci[m] = cmap[i]; pv[m] = 1.0; m++;
            prp[i + 1] = m;
            continue;
        }
        int nci = 0;
        for (int q = srp[i]; q < srp[i + 1]; q++) {
            const int j = sci[q];
            sm[j] = i;
            if (cf[j]) { pos[j] = nci; cl[nci] = j; num[nci] = 0.0; nci++; }
        }
        if (nci == 0) { prp[i + 1] = m; continue; }
        double diag = 0.0;
        for (int q = rp[i]; q < rp[i + 1]; q++) if (ci[q] == i) diag = a[q];
        for (int q = rp[i]; q < rp[i + 1]; q++) {
            const int j = ci[q];
            if (j == i) continue;
            const int strong = sm[j] == i;
            if (strong && cf[j]) {
                num[pos[j]] += a[q];
            } else if (strong) {                 /* strong F neighbour k = j */
                double akk = 0.0, den = 0.0;
                for (int p = rp[j]; p < rp[j + 1]; p++) if (ci[p] == j) akk = a[p];
                for (int p = rp[j]; p < rp[j + 1]; p++) {
                    const int mm = ci[p];
                    if (sm[mm] == i && cf[mm] && pos[mm] >= 0 && opposite(akk, a[p])) den += a[p];
                }
                if (den == 0.0) {
                    diag += a[q];
                } else {
                    for (int p = rp[j]; p < rp[j + 1]; p++) {
                        const int mm = ci[p];
                        if (sm[mm] == i && cf[mm] && opposite(akk, a[p]))
                            num[pos[mm]] += a[q] * a[p] / den;
                    }
                }
            } else {
                diag += a[q];                    /* weak: lumped */
            }
        }
        if (diag == 0.0) { e = OR_ERR_ZERO_PIVOT; break; }
        double mx = 0.0, sum_all = 0.0, sum_kept = 0.0;
        for (int t = 0; t < nci; t++) {
            num[t] = -num[t] / diag;
            if (fabs(num[t]) > mx) mx = fabs(num[t]);
            sum_all += num[t];
        }
        for (int t = 0; t < nci; t++)
            if (fabs(num[t]) >= trunc * mx) sum_kept += num[t];
        const double scale = sum_kept != 0.0 ? sum_all / sum_kept : 1.0;
        for (int t = 0; t < nci; t++)
            if (fabs(num[t]) >= trunc * mx) {
                pci[m] = cmap[cl[t]];
                pv[m] = num[t] * scale;
                m++;
            }
        for (int t = 0; t < nci; t++) pos[cl[t]] = -1;
        prp[i + 1] = m;
    }
    free(sm); free(pos); free(cl); free(num); free(cmap);
    if (e) { free(prp); free(pci); free(pv); return e; }
    *nc_out = nc; *prp_o = prp; *pci_o = pci; *pv_o = pv;
    return OR_OK;
}

static int cmp_int(const void *x, const void *y)
{
    const int a = *(const int *)x, b = *(const int *)y;
    return (a > b) - (a < b);
}

/* C = A B (row-wise, contributions in ascending order of A's entries);
 * columns of every row ascending; returns the allocated product */
static void csr_mult(int n, int k, int m, const int *arp, const int *aci, const double *av,
                     const int *brp, const int *bci, const double *bv,
                     int **crp_o, int **cci_o, double **cv_o)
{
    (void)k;
    int *crp = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    int *stamp = (int *)malloc(sizeof(int) * (size_t)(m + 1));
    int *list = (int *)malloc(sizeof(int) * (size_t)(m + 1));
    double *acc = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    for (int j = 0; j < m; j++) stamp[j] = -1;
    size_t cap = 1024, nnz = 0;
    int *cci = (int *)malloc(sizeof(int) * cap);
    double *cv = (double *)malloc(sizeof(double) * cap);
    crp[0] = 0;
    for (int i = 0; i < n; i++) {
        int len = 0;
        for (int q = arp[i]; q < arp[i + 1]; q++) {
            const int kk = aci[q];
            for (int p = brp[kk]; p < brp[kk + 1]; p++) {
                const int j = bci[p];
                if (stamp[j] != i) { stamp[j] = i; acc[j] = 0.0; list[len++] = j; }
                acc[j] += av[q] * bv[p];
            }
        }
        qsort(list, (size_t)len, sizeof(int), cmp_int);
        if (nnz + (size_t)len > cap) {
            while (nnz + (size_t)len > cap) cap *= 2;
            cci = (int *)realloc(cci, sizeof(int) * cap);
            cv = (double *)realloc(cv, sizeof(double) * cap);
        }
        for (int t = 0; t < len; t++) { cci[nnz] = list[t]; cv[nnz] = acc[list[t]]; nnz++; }
        crp[i + 1] = (int)nnz;
    }
    free(stamp); free(list); free(acc);
    *crp_o = crp; *cci_o = cci; *cv_o = cv;
}

/* dense LU with partial pivoting (first largest pivot) */
static int dense_lu(int n, double *M, int *piv)
{
    for (int k = 0; k < n; k++) {
        int p = k;
        for (int i = k + 1; i < n; i++)
            if (fabs(M[(size_t)i * n + k]) > fabs(M[(size_t)p * n + k])) p = i;
        piv[k] = p;
        if (M[(size_t)p * n + k] == 0.0) return OR_ERR_ZERO_PIVOT;
        if (p != k)
            for (int j = 0; j < n; j++) {
                double t = M[(size_t)k * n + j];
                M[(size_t)k * n + j] = M[(size_t)p * n + j];
                M[(size_t)p * n + j] = t;
            }
        for (int i = k + 1; i < n; i++) {
            const double l = M[(size_t)i * n + k] / M[(size_t)k * n + k];
            M[(size_t)i * n + k] = l;
            for (int j = k + 1; j < n; j++) M[(size_t)i * n + j] -= l * M[(size_t)k * n + j];
        }
    }
    return OR_OK;
}

static void dense_lu_solve(int n, const double *M, const int *piv, double *x)
{
    for (int k = 0; k < n; k++)
        if (piv[k] != k) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < i; j++) x[i] -= M[(size_t)i * n + j] * x[j];
    for (int i = n - 1; i >= 0; i--) {
        for (int j = i + 1; j < n; j++) x[i] -= M[(size_t)i * n + j] * x[j];
        x[i] /= M[(size_t)i * n + i];
    }
}

static void amg_level_free(amg_level *L)
{
    free(L->rp); free(L->ci); free(L->a); free(L->cf);
    free(L->prp); free(L->pci); free(L->pv);
    free(L->trp); free(L->tci); free(L->tv);
    free(L->lu); free(L->piv);
    free(L->x); free(L->b); free(L->r); free(L->t);
}

void or_amg_destroy(or_amg *M)
{
    if (!M) return;
    for (int l = 0; l < M->nlev; l++) amg_level_free(&M->lev[l]);
    free(M->lev);
    free(M);
}

or_amg *or_amg_create(int n, const int *rp, const int *ci, const double *a,
                      const or_amg_opts *opts, int *err)
{
    or_amg_opts o;
    if (opts) o = *opts; else or_amg_defaults(&o);
    int e = OR_OK;
    if (n < 1 || o.max_levels < 1 || o.num_sweeps < 0) e = OR_ERR_ARG;
    if (e) { if (err) *err = e; return NULL; }
    or_amg *M = (or_amg *)calloc(1, sizeof(or_amg));
    M->o = o;
    M->lev = (amg_level *)calloc((size_t)o.max_levels, sizeof(amg_level));
    amg_level *L = &M->lev[0];
    L->n = n;
    L->rp = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    L->ci = (int *)malloc(sizeof(int) * (size_t)(rp[n] + 1));
    L->a = (double *)malloc(sizeof(double) * (size_t)(rp[n] + 1));
    memcpy(L->rp, rp, sizeof(int) * (size_t)(n + 1));
    memcpy(L->ci, ci, sizeof(int) * (size_t)rp[n]);
    memcpy(L->a, a, sizeof(double) * (size_t)rp[n]);
    M->nlev = 1;
    for (int l = 0; !e; l++) {
        L = &M->lev[l];
        const int nl = L->n;
        L->x = (double *)calloc((size_t)nl + 1, sizeof(double));
        L->b = (double *)calloc((size_t)nl + 1, sizeof(double));
        L->r = (double *)calloc((size_t)nl + 1, sizeof(double));
        L->t = (double *)calloc((size_t)nl + 1, sizeof(double));
        int coarsest = l == o.max_levels - 1 || nl <= o.coarse_size;
        if (!coarsest) {
            const int nnz = L->rp[nl];
            int *srp = (int *)malloc(sizeof(int) * (size_t)(nl + 1));
            int *sci = (int *)malloc(sizeof(int) * (size_t)(nnz + 1));
            or_amg_strength(nl, L->rp, L->ci, L->a, o.strength, o.max_row_sum, srp, sci);
            int *trp = (int *)malloc(sizeof(int) * (size_t)(nl + 1));
            int *tci = (int *)malloc(sizeof(int) * (size_t)(srp[nl] + 1));
            pattern_transpose(nl, nl, srp, sci, trp, tci, NULL, NULL);
            L->cf = (int *)malloc(sizeof(int) * (size_t)(nl + 1));
            amg_coarsen(nl, srp, sci, trp, tci, L->cf);
            free(trp); free(tci);
            e = amg_interp(nl, L->rp, L->ci, L->a, srp, sci, L->cf, o.trunc, &L->nc,
                           &L->prp, &L->pci, &L->pv);
            free(srp); free(sci);
            if (e) break;
            if (L->nc == 0 || L->nc == nl) {           /* no coarsening */
                free(L->cf); free(L->prp); free(L->pci); free(L->pv);
                L->cf = NULL; L->prp = NULL; L->pci = NULL; L->pv = NULL;
                L->nc = 0;
                coarsest = 1;
            }
        }
        if (coarsest) {
            L->lu = (double *)calloc((size_t)nl * nl, sizeof(double));
            L->piv = (int *)malloc(sizeof(int) * (size_t)nl);
            for (int i = 0; i < nl; i++)
                for (int q = L->rp[i]; q < L->rp[i + 1]; q++)
                    L->lu[(size_t)i * nl + L->ci[q]] = L->a[q];
            e = dense_lu(nl, L->lu, L->piv);
            break;
        }
        /* R = P^T, A_{l+1} = R (A P) */
        const int nc = L->nc;
        L->trp = (int *)malloc(sizeof(int) * (size_t)(nc + 1));
        L->tci = (int *)malloc(sizeof(int) * (size_t)(L->prp[nl] + 1));
        L->tv = (double *)malloc(sizeof(double) * (size_t)(L->prp[nl] + 1));
        pattern_transpose(nl, nc, L->prp, L->pci, L->trp, L->tci, L->pv, L->tv);
        int *aprp, *apci;
        double *apv;
        csr_mult(nl, nl, nc, L->rp, L->ci, L->a, L->prp, L->pci, L->pv, &aprp, &apci, &apv);
        amg_level *Lc = &M->lev[l + 1];
        Lc->n = nc;
        csr_mult(nc, nl, nc, L->trp, L->tci, L->tv, aprp, apci, apv, &Lc->rp, &Lc->ci, &Lc->a);
        free(aprp); free(apci); free(apv);
        M->nlev = l + 2;
    }
    if (err) *err = e;
    if (e) { or_amg_destroy(M); return NULL; }
    return M;
}

/* one hybrid Gauss-Seidel sweep: xn from xo */
static void amg_hgs(const amg_level *L, int chunk, const double *b, const double *xo, double *xn)
{
    const int n = L->n, c = chunk > 0 ? chunk : n;
    for (int i = 0; i < n; i++) {
        const int c0 = i / c * c;
        double s = b[i], d = 0.0;
        for (int q = L->rp[i]; q < L->rp[i + 1]; q++) {
            const int j = L->ci[q];
            if (j == i) d = L->a[q];
            else if (j >= c0 && j < i) s -= L->a[q] * xn[j];
            else s -= L->a[q] * xo[j];
        }
        xn[i] = s / d;
    }
}

static void amg_smooth(const or_amg *M, amg_level *L)
{
    for (int s = 0; s < M->o.num_sweeps; s++) {
        amg_hgs(L, M->o.gs_chunk, L->b, L->x, L->t);
        memcpy(L->x, L->t, sizeof(double) * (size_t)L->n);
    }
}

static void amg_cycle(or_amg *M, int l)
{
    amg_level *L = &M->lev[l];
    const int n = L->n;
    if (l == M->nlev - 1) {
        memcpy(L->x, L->b, sizeof(double) * (size_t)n);
        dense_lu_solve(n, L->lu, L->piv, L->x);
        return;
    }
    amg_level *Lc = &M->lev[l + 1];
    for (int i = 0; i < n; i++) L->x[i] = 0.0;
    amg_smooth(M, L);                                     /* x = S(x, A, b) */
    for (int i = 0; i < n; i++) {                         /* r = b - A x    */
        double s = L->b[i];
        for (int q = L->rp[i]; q < L->rp[i + 1]; q++) s -= L->a[q] * L->x[L->ci[q]];
        L->r[i] = s;
    }
    for (int I = 0; I < L->nc; I++) {                     /* b_c = R r      */
        double s = 0.0;
        for (int q = L->trp[I]; q < L->trp[I + 1]; q++) s += L->tv[q] * L->r[L->tci[q]];
        Lc->b[I] = s;
    }
    amg_cycle(M, l + 1);
    for (int i = 0; i < n; i++) {                         /* x += P x_c     */
        double s = 0.0;
        for (int q = L->prp[i]; q < L->prp[i + 1]; q++) s += L->pv[q] * Lc->x[L->pci[q]];
        L->x[i] += s;
    }
    amg_smooth(M, L);                                     /* x = T(x, A, b) */
}

void or_amg_vcycle(or_amg *M, const double *b, double *x)
{
    memcpy(M->lev[0].b, b, sizeof(double) * (size_t)M->lev[0].n);
    amg_cycle(M, 0);
    memcpy(x, M->lev[0].x, sizeof(double) * (size_t)M->lev[0].n);
}

int or_amg_nlevels(const or_amg *M) { return M->nlev; }

/* sizes of level l: rows, entries of A_l, coarse rows and entries of P_l
 * (0 on the coarsest level) */
void or_amg_level_size(const or_amg *M, int l, int *n, int *nnz, int *nc, int *pnnz)
{
    const amg_level *L = &M->lev[l];
    *n = L->n;
    *nnz = L->rp[L->n];
    *nc = l < M->nlev - 1 ? L->nc : 0;
    *pnnz = l < M->nlev - 1 ? L->prp[L->n] : 0;
}

void or_amg_level_get(const or_amg *M, int l, int *rp, int *ci, double *a, int *cf,
                      int *prp, int *pci, double *pv)
{
    const amg_level *L = &M->lev[l];
    const int n = L->n;
    memcpy(rp, L->rp, sizeof(int) * (size_t)(n + 1));
    memcpy(ci, L->ci, sizeof(int) * (size_t)L->rp[n]);
    memcpy(a, L->a, sizeof(double) * (size_t)L->rp[n]);
    if (l < M->nlev - 1) {
        memcpy(cf, L->cf, sizeof(int) * (size_t)n);
        memcpy(prp, L->prp, sizeof(int) * (size_t)(n + 1));
        memcpy(pci, L->pci, sizeof(int) * (size_t)L->prp[n]);
        memcpy(pv, L->pv, sizeof(double) * (size_t)L->prp[n]);
    }
}

/* ======================================================================
 * Preconditioner objects (Figure 29)
 * ====================================================================== */
/* one subdomain of RAS: its number s (it owns the rows r with part[r] =
 * s), the overlapped set idx[0..nidx) (ascending global block rows), the
 * principal submatrix of A on it in local numbering and its block ILU(0)
 * factor */
typedef struct {
    int s, nidx;
    int *idx, *rp, *ci;
    double *a, *lu;
} ras_sub;

struct or_pc {
    int kind, nb, bs, prec, p_sweeps;
    int nsub;
    ras_sub *subs;              /* RAS */
    int *part;                  /* RAS: owner subdomain of each block row */
    const int *rp, *ci;
    const double *a;
    double *lu;                 /* FP64 (block) ILU(0) factor of A        */
    lowp_lu lp;                 /* rounded copy for F32 / BF16            */
    /* CPR */
    double *w, *app, *applu;
    lowp_lu lpp;                /* rounded pressure factor                */
    float *appf, *af;           /* rounded A_pp values, rounded A values  */
    or_amg *amg;                /* AMG, or CPR's AMG pressure stage       */
    or_pc *full;                /* CPR's full-system stage when not BILU(0) */
    /* learned stage */
    or_pc *base;
    int nx, ny, nz, bf16;
    double *params, *lnk;
    long applies, fallbacks;
};

or_pc *or_pc_create(int kind, int nb, int bs, const int *rp, const int *ci,
                    const double *a, int prec, int p_sweeps, int *err)
{
    or_pc *pc = (or_pc *)calloc(1, sizeof(or_pc));
    size_t nnzb = (size_t)rp[nb];
    int b2 = bs * bs, e = OR_OK;
    pc->kind = kind; pc->nb = nb; pc->bs = bs; pc->prec = prec;
    pc->p_sweeps = p_sweeps; pc->rp = rp; pc->ci = ci; pc->a = a;
    const int is_cpr = kind == OR_PC_CPR_PF || kind == OR_PC_CPR_FP ||
                       kind == OR_PC_CPR_FPF || kind == OR_PC_CPR_FFPF;
    if (kind == OR_PC_BILU0 || is_cpr) {
        pc->lu = (double *)malloc(sizeof(double) * nnzb * b2);
        e = or_bilu0(nb, bs, rp, ci, a, pc->lu);
        if (!e && prec != OR_PREC_F64) e = lowp_init(&pc->lp, nb, bs, rp, ci, pc->lu, prec);
    }
    if (!e && is_cpr) {
        if (bs != 3) e = OR_ERR_ARG;
        if (!e) {
            pc->w = (double *)malloc(sizeof(double) * 3 * (size_t)nb);
            pc->app = (double *)malloc(sizeof(double) * nnzb);
            pc->applu = (double *)malloc(sizeof(double) * nnzb);
            e = or_cpr_weights(nb, rp, ci, a, pc->w);
        }
        if (!e) {
            or_cpr_extract_pressure(nb, rp, ci, a, pc->w, pc->app);
            e = or_bilu0(nb, 1, rp, ci, pc->app, pc->applu);
        }
        if (!e && prec != OR_PREC_F64) {
            /* the pressure factor is rounded to float in both reduced
             * variants; only the block factor is held in bfloat16 */
            e = lowp_init(&pc->lpp, nb, 1, rp, ci, pc->applu, OR_PREC_F32);
            pc->appf = (float *)malloc(sizeof(float) * nnzb);
            pc->af = (float *)malloc(sizeof(float) * nnzb * 9);
            for (size_t p = 0; p < nnzb; p++) pc->appf[p] = (float)pc->app[p];
            for (size_t p = 0; p < nnzb * 9; p++) pc->af[p] = (float)a[p];
        }
    }
    if (err) *err = e;
    if (e) { or_pc_destroy(pc); return NULL; }
    return pc;
}

or_pc *or_pc_create_learned(or_pc *base, int nx, int ny, int nz,
                            const double *params, const double *lnk,
                            int bf16_emul)
{
    or_pc *pc = (or_pc *)calloc(1, sizeof(or_pc));
    int np = or_conv_nparams();
    size_t cells = (size_t)nx * ny * nz;
    pc->kind = OR_PC_LEARNED;
    pc->base = base;
    pc->nb = base->nb; pc->bs = base->bs; pc->rp = base->rp; pc->ci = base->ci;
    pc->a = base->a;
    pc->nx = nx; pc->ny = ny; pc->nz = nz; pc->bf16 = bf16_emul;
    pc->params = (double *)malloc(sizeof(double) * np);
    memcpy(pc->params, params, sizeof(double) * np);
    pc->lnk = (double *)malloc(sizeof(double) * cells);
    memcpy(pc->lnk, lnk, sizeof(double) * cells);
    return pc;
}

/* ======================================================================
 * C9b. Restricted additive Schwarz (Section 4.1, Cai & Sarkis): block row
 * r is owned by subdomain part[r] (contiguous ranges: or_pc_create_ras);
 * subdomain s grows by `overlap` rounds of graph neighbours (the column
 * indices of its rows), its principal submatrix A_s is factored by block
 * ILU(0), and
 *     M^-1 v = sum_s R0_s^T (L_s U_s)^-1 R_s v,
 * R_s restricting to the overlapped set, R0_s^T writing back only the
 * owned rows (restricted prolongation).
 * ====================================================================== */
/* Subdomain s of RAS: the rows with part[r] == s, grown by `overlap`
 * rounds of graph neighbours, or (sets != NULL) the explicitly given
 * overlapped set sets[s_ptr[s] .. s_ptr[s+1]) of ascending block rows. */
static or_pc *ras_build(int nb, int bs, const int *rp, const int *ci, const double *a,
                        int nsub, const int *part, int overlap, const int *s_ptr,
                        const int *sets, int *err)
{
    int e = OR_OK;
    if (nsub < 1 || overlap < 0) e = OR_ERR_ARG;
    for (int r = 0; !e && r < nb; r++)
        if (part[r] < 0 || part[r] >= nsub) e = OR_ERR_ARG;
    if (e) { if (err) *err = e; return NULL; }
    or_pc *pc = (or_pc *)calloc(1, sizeof(or_pc));
    const int b2 = bs * bs;
    pc->kind = OR_PC_RAS; pc->nb = nb; pc->bs = bs; pc->prec = OR_PREC_F64;
    pc->rp = rp; pc->ci = ci; pc->a = a;
    pc->nsub = nsub;
    pc->subs = (ras_sub *)calloc((size_t)nsub, sizeof(ras_sub));
    pc->part = (int *)malloc(sizeof(int) * (size_t)nb);
    memcpy(pc->part, part, sizeof(int) * (size_t)nb);
    char *in = (char *)malloc((size_t)nb);
    char *add = (char *)malloc((size_t)nb);
    int *loc = (int *)malloc(sizeof(int) * (size_t)nb);
    for (int s = 0; !e && s < nsub; s++) {
        ras_sub *S = &pc->subs[s];
        S->s = s;
        if (sets) {
            for (int r = 0; r < nb; r++) in[r] = 0;
            for (int q = s_ptr[s]; q < s_ptr[s + 1]; q++) {
                if (sets[q] < 0 || sets[q] >= nb) { e = OR_ERR_ARG; break; }
                in[sets[q]] = 1;
            }
            for (int r = 0; !e && r < nb; r++)      /* a set holds its owned rows */
                if (part[r] == s && !in[r]) e = OR_ERR_ARG;
            if (e) break;
        } else {
            for (int r = 0; r < nb; r++) in[r] = (char)(part[r] == s);
            for (int d = 0; d < overlap; d++) {        /* one round of neighbours */
                for (int r = 0; r < nb; r++) add[r] = 0;
                for (int r = 0; r < nb; r++)
                    if (in[r])
                        for (int q = rp[r]; q < rp[r + 1]; q++) add[ci[q]] = 1;
                for (int r = 0; r < nb; r++) in[r] = (char)(in[r] | add[r]);
            }
        }
        S->nidx = 0;
        for (int r = 0; r < nb; r++) S->nidx += in[r];
        if (S->nidx == 0) { e = OR_ERR_ARG; break; }   /* an empty subdomain */
        S->idx = (int *)malloc(sizeof(int) * (size_t)S->nidx);
        for (int r = 0, l = 0; r < nb; r++) {
            loc[r] = in[r] ? l : -1;
            if (in[r]) S->idx[l++] = r;
        }
        /* principal submatrix in local numbering (columns stay ascending) */
        S->rp = (int *)malloc(sizeof(int) * (size_t)(S->nidx + 1));
        S->rp[0] = 0;
        for (int l = 0; l < S->nidx; l++) {
            int g = S->idx[l], c = 0;
            for (int q = rp[g]; q < rp[g + 1]; q++) c += loc[ci[q]] >= 0;
            S->rp[l + 1] = S->rp[l] + c;
        }
        const int nnz = S->rp[S->nidx];
        S->ci = (int *)malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
        S->a = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1) * b2);
        S->lu = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1) * b2);
        for (int l = 0, p = 0; l < S->nidx; l++) {
            int g = S->idx[l];
            for (int q = rp[g]; q < rp[g + 1]; q++)
                if (loc[ci[q]] >= 0) {
                    S->ci[p] = loc[ci[q]];
                    memcpy(S->a + (size_t)p * b2, a + (size_t)q * b2, sizeof(double) * b2);
                    p++;
                }
        }
        e = or_bilu0(S->nidx, bs, S->rp, S->ci, S->a, S->lu);
    }
    free(in); free(add); free(loc);
    if (err) *err = e;
    if (e) { or_pc_destroy(pc); return NULL; }
    return pc;
}

or_pc *or_pc_create_ras_part(int nb, int bs, const int *rp, const int *ci,
                             const double *a, int nsub, const int *part,
                             int overlap, int *err)
{
    return ras_build(nb, bs, rp, ci, a, nsub, part, overlap, NULL, NULL, err);
}

or_pc *or_pc_create_ras_sets(int nb, int bs, const int *rp, const int *ci,
                             const double *a, int nsub, const int *part,
                             const int *set_ptr, const int *sets, int *err)
{
    return ras_build(nb, bs, rp, ci, a, nsub, part, 0, set_ptr, sets, err);
}

/* contiguous owned ranges [starts[s], starts[s+1]) */
or_pc *or_pc_create_ras(int nb, int bs, const int *rp, const int *ci,
                        const double *a, int nsub, const int *starts,
                        int overlap, int *err)
{
    int e = OR_OK;
    if (nsub < 1 || overlap < 0 || starts[0] != 0 || starts[nsub] != nb) e = OR_ERR_ARG;
    for (int s = 0; !e && s < nsub; s++)
        if (starts[s + 1] <= starts[s]) e = OR_ERR_ARG;
    if (e) { if (err) *err = e; return NULL; }
    int *part = (int *)malloc(sizeof(int) * (size_t)(nb > 0 ? nb : 1));
    for (int s = 0; s < nsub; s++)
        for (int r = starts[s]; r < starts[s + 1]; r++) part[r] = s;
    or_pc *pc = or_pc_create_ras_part(nb, bs, rp, ci, a, nsub, part, overlap, err);
    free(part);
    return pc;
}

static void ras_apply(or_pc *pc, const double *v, double *z)
{
    const int bs = pc->bs;
    for (int s = 0; s < pc->nsub; s++) {
        const ras_sub *S = &pc->subs[s];
        const size_t nl = (size_t)S->nidx * bs;
        double *vl = (double *)malloc(sizeof(double) * nl);
        double *xl = (double *)malloc(sizeof(double) * nl);
        for (int l = 0; l < S->nidx; l++)                 /* R_s v */
            memcpy(vl + (size_t)l * bs, v + (size_t)S->idx[l] * bs, sizeof(double) * bs);
        or_bilu0_solve(S->nidx, bs, S->rp, S->ci, S->lu, vl, xl);
        for (int l = 0; l < S->nidx; l++) {               /* owned rows only */
            const int g = S->idx[l];
            if (pc->part[g] == S->s)
                memcpy(z + (size_t)g * bs, xl + (size_t)l * bs, sizeof(double) * bs);
        }
        free(vl); free(xl);
    }
}

void or_pc_destroy(or_pc *pc)
{
    if (!pc) return;
    free(pc->lu); free(pc->w); free(pc->app); free(pc->applu);
    free(pc->appf); free(pc->af);
    if (pc->lp.f) lowp_free(&pc->lp);
    if (pc->lpp.f) lowp_free(&pc->lpp);
    if (pc->base) or_pc_destroy(pc->base);
    free(pc->params); free(pc->lnk);
    for (int s = 0; s < pc->nsub; s++) {
        free(pc->subs[s].idx); free(pc->subs[s].rp); free(pc->subs[s].ci);
        free(pc->subs[s].a); free(pc->subs[s].lu);
    }
    free(pc->subs);
    free(pc->part);
    or_amg_destroy(pc->amg);
    if (pc->full) or_pc_destroy(pc->full);
    free(pc);
}

or_pc *or_pc_create_cpr(int kind, int nb, const int *rp, const int *ci, const double *a,
                        const or_amg_opts *amg, int p_sweeps, or_pc *full, int *err)
{
    const int is_cpr = kind == OR_PC_CPR_PF || kind == OR_PC_CPR_FP ||
                       kind == OR_PC_CPR_FPF || kind == OR_PC_CPR_FFPF;
    int e = is_cpr ? OR_OK : OR_ERR_ARG;
    or_pc *pc = NULL;
    if (!e) pc = amg ? or_pc_create_amg(kind, nb, 3, rp, ci, a, amg, &e)
                     : or_pc_create(kind, nb, 3, rp, ci, a, OR_PREC_F64, p_sweeps, &e);
    if (pc) pc->full = full;
    else if (full) or_pc_destroy(full);
    if (err) *err = e;
    return pc;
}

or_pc *or_pc_create_amg(int kind, int nb, int bs, const int *rp, const int *ci,
                        const double *a, const or_amg_opts *o, int *err)
{
    const int is_cpr = kind == OR_PC_CPR_PF || kind == OR_PC_CPR_FP ||
                       kind == OR_PC_CPR_FPF || kind == OR_PC_CPR_FFPF;
    int e = OR_OK;
    or_pc *pc = NULL;
    if (kind == OR_PC_AMG && bs == 1) {
        pc = (or_pc *)calloc(1, sizeof(or_pc));
        pc->kind = kind; pc->nb = nb; pc->bs = 1; pc->prec = OR_PREC_F64;
        pc->rp = rp; pc->ci = ci; pc->a = a;
        pc->amg = or_amg_create(nb, rp, ci, a, o, &e);
    } else if (is_cpr && bs == 3) {
        pc = or_pc_create(kind, nb, bs, rp, ci, a, OR_PREC_F64, 0, &e);
        if (pc) pc->amg = or_amg_create(nb, rp, ci, pc->app, o, &e);
    } else {
        e = OR_ERR_ARG;
    }
    if (err) *err = e;
    if (e) { or_pc_destroy(pc); return NULL; }
    return pc;
}

void or_pc_learned_stats(const or_pc *pc, long *applies, long *fallbacks)
{
    if (applies) *applies = pc->applies;
    if (fallbacks) *fallbacks = pc->fallbacks;
}

/* FP64 pressure stage: p = 0, then s sweeps p <- p + (LU)^-1 (r_p - A_pp p);
 * with AMG, p = one V-cycle on A_pp */
static void pstage_f64(or_pc *pc, const double *rpv, double *p)
{
    int nb = pc->nb;
    if (pc->amg) {
        or_amg_vcycle(pc->amg, rpv, p);
        return;
    }
    double *res = (double *)malloc(sizeof(double) * nb);
    double *d = (double *)malloc(sizeof(double) * nb);
    for (int i = 0; i < nb; i++) p[i] = 0.0;
    for (int s = 0; s < pc->p_sweeps; s++) {
        memcpy(res, rpv, sizeof(double) * nb);
        or_bsr_amxpby(nb, 1, pc->rp, pc->ci, pc->app, -1.0, p, 1.0, res);
        or_bilu0_solve(nb, 1, pc->rp, pc->ci, pc->applu, res, d);
        for (int i = 0; i < nb; i++) p[i] += d[i];
    }
    free(res); free(d);
}

/* float pressure stage, same steps in float arithmetic */
static void pstage_f32(or_pc *pc, const float *rpv, float *p)
{
    int nb = pc->nb;
    float *res = (float *)malloc(sizeof(float) * nb);
    float *d = (float *)malloc(sizeof(float) * nb);
    for (int i = 0; i < nb; i++) p[i] = 0.0f;
    for (int s = 0; s < pc->p_sweeps; s++) {
        for (int i = 0; i < nb; i++) {
            float t = 0.0f;
            for (int q = pc->rp[i]; q < pc->rp[i + 1]; q++) t += pc->appf[q] * p[pc->ci[q]];
            res[i] = rpv[i] - t;
        }
        lowp_apply(&pc->lpp, res, d);
        for (int i = 0; i < nb; i++) p[i] += d[i];
    }
    free(res); free(d);
}

/* Stages of the multi-stage CPR variants (Algorithms 7 and 8), each acting
 * on the running iterate x: the residual r = f - A x, the full-system stage
 * x <- x + BILU^-1 r, and the pressure stage x <- x + Pi_p P(Pi_r W r). */
static void cpr_resid_f64(or_pc *pc, const double *f, const double *x, double *r)
{
    memcpy(r, f, sizeof(double) * 3 * (size_t)pc->nb);
    or_bsr_amxpby(pc->nb, 3, pc->rp, pc->ci, pc->a, -1.0, x, 1.0, r);
}

/* the full-system solve R(A)^-1 of Algorithms 5-8: block ILU(0), or the
 * preconditioner given as the full stage (RAS) */
static void full_solve_f64(or_pc *pc, const double *r, double *t)
{
    if (pc->full) or_pc_apply(pc->full, r, t);
    else or_bilu0_solve(pc->nb, 3, pc->rp, pc->ci, pc->lu, r, t);
}

static void cpr_full_f64(or_pc *pc, const double *r, double *x)
{
    const size_t n = 3 * (size_t)pc->nb;
    double *t = (double *)malloc(sizeof(double) * n);
    full_solve_f64(pc, r, t);
    for (size_t i = 0; i < n; i++) x[i] += t[i];
    free(t);
}

static void cpr_pressure_f64(or_pc *pc, const double *r, double *x)
{
    const int nb = pc->nb;
    double *rpv = (double *)calloc((size_t)nb + 1, sizeof(double));
    double *p = (double *)calloc((size_t)nb + 1, sizeof(double));
    for (int i = 0; i < nb; i++)
        rpv[i] = pc->w[3 * i] * r[3 * i] + pc->w[3 * i + 1] * r[3 * i + 1]
               + pc->w[3 * i + 2] * r[3 * i + 2];
    pstage_f64(pc, rpv, p);
    for (int i = 0; i < nb; i++) x[3 * i] += p[i];
    free(rpv); free(p);
}

static void cpr_resid_f32(or_pc *pc, const float *f, const float *x, float *r)
{
    for (int i = 0; i < pc->nb; i++)
        for (int rr = 0; rr < 3; rr++) {
            float s = 0.0f;
            for (int q = pc->rp[i]; q < pc->rp[i + 1]; q++) {
                const float *B = pc->af + (size_t)q * 9;
                const float *xj = x + (size_t)pc->ci[q] * 3;
                s += B[rr * 3] * xj[0] + B[rr * 3 + 1] * xj[1] + B[rr * 3 + 2] * xj[2];
            }
            r[3 * i + rr] = f[3 * i + rr] - s;
        }
}

static void cpr_full_f32(or_pc *pc, const float *r, float *x)
{
    const size_t n = 3 * (size_t)pc->nb;
    float *t = (float *)malloc(sizeof(float) * n);
    lowp_apply(&pc->lp, r, t);
    for (size_t i = 0; i < n; i++) x[i] += t[i];
    free(t);
}

static void cpr_pressure_f32(or_pc *pc, const float *r, float *x)
{
    const int nb = pc->nb;
    float *rpv = (float *)calloc((size_t)nb + 1, sizeof(float));
    float *p = (float *)calloc((size_t)nb + 1, sizeof(float));
    for (int i = 0; i < nb; i++)
        rpv[i] = (float)pc->w[3 * i] * r[3 * i] + (float)pc->w[3 * i + 1] * r[3 * i + 1]
               + (float)pc->w[3 * i + 2] * r[3 * i + 2];
    pstage_f32(pc, rpv, p);
    for (int i = 0; i < nb; i++) x[3 * i] += p[i];
    free(rpv); free(p);
}

/* Algorithm 7 (FPF) and Algorithm 8 (FFPF) from x = 0; the first
 * full-system stage sees r = f. */
static void cpr_multistage_f64(or_pc *pc, const double *f, double *x)
{
    const size_t n = 3 * (size_t)pc->nb;
    double *r = (double *)malloc(sizeof(double) * n);
    memset(x, 0, sizeof(double) * n);
    cpr_full_f64(pc, f, x);                       /* x = R^-1 f        */
    if (pc->kind == OR_PC_CPR_FFPF) {
        cpr_resid_f64(pc, f, x, r);               /* r = f - A x       */
        cpr_full_f64(pc, r, x);                   /* x = x + R^-1 r    */
    }
    cpr_resid_f64(pc, f, x, r);                   /* r = f - A x       */
    cpr_pressure_f64(pc, r, x);                   /* x = x + Pi_p(..)  */
    cpr_resid_f64(pc, f, x, r);                   /* r = f - A x       */
    cpr_full_f64(pc, r, x);                       /* x = x + R^-1 r    */
    free(r);
}

static void cpr_multistage_f32(or_pc *pc, const float *f, float *x)
{
    const size_t n = 3 * (size_t)pc->nb;
    float *r = (float *)malloc(sizeof(float) * n);
    memset(x, 0, sizeof(float) * n);
    cpr_full_f32(pc, f, x);
    if (pc->kind == OR_PC_CPR_FFPF) {
        cpr_resid_f32(pc, f, x, r);
        cpr_full_f32(pc, r, x);
    }
    cpr_resid_f32(pc, f, x, r);
    cpr_pressure_f32(pc, r, x);
    cpr_resid_f32(pc, f, x, r);
    cpr_full_f32(pc, r, x);
    free(r);
}

static void conv_apply_learned(or_pc *pc, const double *v, double *z);

void or_pc_apply(or_pc *pc, const double *v, double *z)
{
    const int nb = pc->nb, bs = pc->bs;
    const size_t n = (size_t)nb * bs;
    if (pc->kind == OR_PC_NONE) {
        memcpy(z, v, sizeof(double) * n);
        return;
    }
    if (pc->kind == OR_PC_LEARNED) {
        conv_apply_learned(pc, v, z);
        return;
    }
    if (pc->kind == OR_PC_RAS) {
        ras_apply(pc, v, z);
        return;
    }
    if (pc->kind == OR_PC_AMG) {
        or_amg_vcycle(pc->amg, v, z);
        return;
    }
    if (pc->prec == OR_PREC_F64) {
        if (pc->kind == OR_PC_BILU0) {
            or_bilu0_solve(nb, bs, pc->rp, pc->ci, pc->lu, v, z);
            return;
        }
        if (pc->kind == OR_PC_CPR_FPF || pc->kind == OR_PC_CPR_FFPF) {
            cpr_multistage_f64(pc, v, z);
            return;
        }
        double *rpv = (double *)calloc((size_t)nb + 1, sizeof(double));
        double *p = (double *)malloc(sizeof(double) * nb);
        double *r = (double *)malloc(sizeof(double) * n);
        double *t = (double *)malloc(sizeof(double) * n);
        if (pc->kind == OR_PC_CPR_PF) {
            /* Algorithm 6 read as: z1 = Pi_p(P-stage(Pi_r W v));
             * r = v - A z1; z = z1 + BILU^-1 r */
            for (int i = 0; i < nb; i++)
                rpv[i] = pc->w[3 * i] * v[3 * i] + pc->w[3 * i + 1] * v[3 * i + 1]
                       + pc->w[3 * i + 2] * v[3 * i + 2];
            pstage_f64(pc, rpv, p);
            for (int i = 0; i < nb; i++) { z[3 * i] = p[i]; z[3 * i + 1] = 0.0; z[3 * i + 2] = 0.0; }
            memcpy(r, v, sizeof(double) * n);
            or_bsr_amxpby(nb, 3, pc->rp, pc->ci, pc->a, -1.0, z, 1.0, r);
            full_solve_f64(pc, r, t);
            for (size_t i = 0; i < n; i++) z[i] += t[i];
        } else {
            /* Algorithm 5: z1 = BILU^-1 v; r = v - A z1;
             * z = z1 + Pi_p(P-stage(Pi_r W r)) */
            full_solve_f64(pc, v, z);
            memcpy(r, v, sizeof(double) * n);
            or_bsr_amxpby(nb, 3, pc->rp, pc->ci, pc->a, -1.0, z, 1.0, r);
            for (int i = 0; i < nb; i++)
                rpv[i] = pc->w[3 * i] * r[3 * i] + pc->w[3 * i + 1] * r[3 * i + 1]
                       + pc->w[3 * i + 2] * r[3 * i + 2];
            pstage_f64(pc, rpv, p);
            for (int i = 0; i < nb; i++) z[3 * i] += p[i];
        }
        free(rpv); free(p); free(r); free(t);
        return;
    }
    /* reduced precision: input rounded to float, float arithmetic,
     * output widened to double */
    float *vf = (float *)malloc(sizeof(float) * n);
    float *zf = (float *)malloc(sizeof(float) * n);
    for (size_t i = 0; i < n; i++) vf[i] = (float)v[i];
    if (pc->kind == OR_PC_BILU0) {
        lowp_apply(&pc->lp, vf, zf);
    } else if (pc->kind == OR_PC_CPR_FPF || pc->kind == OR_PC_CPR_FFPF) {
        cpr_multistage_f32(pc, vf, zf);
    } else {
        float *rpv = (float *)calloc((size_t)nb + 1, sizeof(float));
        float *p = (float *)malloc(sizeof(float) * nb);
        float *r = (float *)malloc(sizeof(float) * n);
        float *t = (float *)malloc(sizeof(float) * n);
        if (pc->kind == OR_PC_CPR_PF) {
            for (int i = 0; i < nb; i++)
                rpv[i] = (float)pc->w[3 * i] * vf[3 * i] + (float)pc->w[3 * i + 1] * vf[3 * i + 1]
                       + (float)pc->w[3 * i + 2] * vf[3 * i + 2];
            pstage_f32(pc, rpv, p);
            /* r = v - A Pi_p p: only column 0 of each block meets p */
            for (int i = 0; i < nb; i++)
                for (int rr = 0; rr < 3; rr++) {
                    float s = 0.0f;
                    for (int q = pc->rp[i]; q < pc->rp[i + 1]; q++)
                        s += pc->af[(size_t)q * 9 + rr * 3] * p[pc->ci[q]];
                    r[3 * i + rr] = vf[3 * i + rr] - s;
                }
            lowp_apply(&pc->lp, r, t);
            for (int i = 0; i < nb; i++) {
                zf[3 * i] = p[i] + t[3 * i];
                zf[3 * i + 1] = t[3 * i + 1];
                zf[3 * i + 2] = t[3 * i + 2];
            }
        } else {
            lowp_apply(&pc->lp, vf, zf);
            for (int i = 0; i < nb; i++)
                for (int rr = 0; rr < 3; rr++) {
                    float s = 0.0f;
                    for (int q = pc->rp[i]; q < pc->rp[i + 1]; q++) {
                        const float *B = pc->af + (size_t)q * 9;
                        const float *zj = zf + (size_t)pc->ci[q] * 3;
                        s += B[rr * 3] * zj[0] + B[rr * 3 + 1] * zj[1] + B[rr * 3 + 2] * zj[2];
                    }
                    r[3 * i + rr] = vf[3 * i + rr] - s;
                }
            for (int i = 0; i < nb; i++)
                rpv[i] = (float)pc->w[3 * i] * r[3 * i] + (float)pc->w[3 * i + 1] * r[3 * i + 1]
                       + (float)pc->w[3 * i + 2] * r[3 * i + 2];
            pstage_f32(pc, rpv, p);
            for (int i = 0; i < nb; i++) zf[3 * i] += p[i];
        }
        free(rpv); free(p); free(r); free(t);
    }
    for (size_t i = 0; i < n; i++) z[i] = (double)zf[i];
    free(vf); free(zf);
}

/* ======================================================================
 * C5/C6. Restarted GMRES(m) (Algorithm 1) and FGMRES(m).
 * Default reading: right preconditioning (A M^-1 u = b, x = M^-1 u) so the
 * Arnoldi estimate |g_{j+1}| is the unpreconditioned residual; modified
 * Gram-Schmidt as in the Arnoldi step of Algorithm 1; Givens rotations
 * c = h_jj / r, s = h_{j+1,j} / r, r = hypot(h_jj, h_{j+1,j}); the
 * estimate is checked after every Arnoldi step; the true residual
 * b - A x decides convergence at each restart.  `left` runs Algorithm 1
 * as printed (M r = b - A x0, M w = A v).
 * Converged iff ||b - A x|| <= max(rtol ||b||, atol).
 * ====================================================================== */
int or_gmres(int nb, int bs, const int *rp, const int *ci, const double *a,
             or_pc *pc, const double *b, double *x, const or_krylov_opts *o,
             or_krylov_result *res, double *hist)
{
    const size_t n = (size_t)nb * bs;
    const int m = o->restart;
    if (m < 1 || o->maxit < 0) return OR_ERR_ARG;
    double *V = (double *)malloc(sizeof(double) * n * (m + 1));
    double *Z = o->flexible ? (double *)malloc(sizeof(double) * n * m) : NULL;
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = (double *)malloc(sizeof(double) * m);
    double *sn = (double *)malloc(sizeof(double) * m);
    double *g = (double *)malloc(sizeof(double) * (m + 1));
    double *y = (double *)malloc(sizeof(double) * m);
    double *r = (double *)malloc(sizeof(double) * n);
    double *w = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    const double bnorm = nrm2((int)n, b);
    double ref = bnorm;
    if (o->left) {                 /* tolerance on ||M^-1 b|| */
        or_pc_apply(pc, b, z);
        ref = nrm2((int)n, z);
    }
    const double tol_true = fmax(o->rtol * bnorm, o->atol);
    const double tol_est = fmax(o->rtol * ref, o->atol);
    int nits = 0, cycles = 0, status = OR_NOT_CONVERGED;
    double relres = 0.0;
#define HH(i, j) H[(size_t)(i) * m + (j)]
    for (;;) {
        /* true residual r = b - A x */
        memcpy(r, b, sizeof(double) * n);
        or_bsr_amxpby(nb, bs, rp, ci, a, -1.0, x, 1.0, r);
        double tnorm = nrm2((int)n, r);
        relres = bnorm > 0 ? tnorm / bnorm : tnorm;
        if (hist && nits == 0) hist[0] = tnorm;
        if (!o->fixed_iters && tnorm <= tol_true) { status = OR_OK; break; }
        if (nits >= o->maxit) break;
        if (o->left) { or_pc_apply(pc, r, w); memcpy(r, w, sizeof(double) * n); }
        double beta = nrm2((int)n, r);
        if (beta == 0.0 || !isfinite(beta)) { status = isfinite(beta) ? OR_OK : OR_ERR_BREAKDOWN; break; }
        for (size_t i = 0; i < n; i++) V[i] = r[i] / beta;
        for (int i = 0; i <= m; i++) g[i] = 0.0;
        g[0] = beta;
        int jend = 0;
        cycles++;
        for (int j = 0; j < m; j++) {
            double *vj = V + n * j;
            if (o->left) {
                or_bsr_spmv(nb, bs, rp, ci, a, vj, z);
                or_pc_apply(pc, z, w);
            } else {
                double *zj = o->flexible ? Z + n * j : z;
                or_pc_apply(pc, vj, zj);
                or_bsr_spmv(nb, bs, rp, ci, a, zj, w);
            }
            for (int k = 0; k <= j; k++) {           /* MGS */
                double h = dot((int)n, w, V + n * k);
                HH(k, j) = h;
#pragma omp parallel for schedule(static)
                for (size_t i = 0; i < n; i++) w[i] -= h * V[n * k + i];
            }
            double hn = nrm2((int)n, w);
            HH(j + 1, j) = hn;
            if (hn != 0.0) {
#pragma omp parallel for schedule(static)
                for (size_t i = 0; i < n; i++) V[n * (j + 1) + i] = w[i] / hn;
            }
            for (int k = 0; k < j; k++) {            /* old rotations */
                double t = cs[k] * HH(k, j) + sn[k] * HH(k + 1, j);
                HH(k + 1, j) = -sn[k] * HH(k, j) + cs[k] * HH(k + 1, j);
                HH(k, j) = t;
            }
            double rr = hypot(HH(j, j), HH(j + 1, j));
            if (rr == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
            else { cs[j] = HH(j, j) / rr; sn[j] = HH(j + 1, j) / rr; }
            HH(j, j) = rr;
            HH(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            nits++;
            jend = j + 1;
            if (hist) hist[nits] = fabs(g[j + 1]);
            if (nits >= o->maxit) break;
            if (hn == 0.0) break;                     /* lucky breakdown */
            if (!o->fixed_iters && !o->check_at_cycle_end && fabs(g[j + 1]) <= tol_est) break;
        }
        /* R y = g(0:jend) by back substitution */
        for (int i = jend - 1; i >= 0; i--) {
            double s = g[i];
            for (int k = i + 1; k < jend; k++) s -= HH(i, k) * y[k];
            y[i] = HH(i, i) != 0.0 ? s / HH(i, i) : 0.0;
        }
        if (o->flexible && !o->left) {
            for (int k = 0; k < jend; k++) {
#pragma omp parallel for schedule(static)
                for (size_t i = 0; i < n; i++) x[i] += y[k] * Z[n * k + i];
            }
        } else {
            for (size_t i = 0; i < n; i++) w[i] = 0.0;
            for (int k = 0; k < jend; k++) {
#pragma omp parallel for schedule(static)
                for (size_t i = 0; i < n; i++) w[i] += y[k] * V[n * k + i];
            }
            if (o->left) {
                for (size_t i = 0; i < n; i++) x[i] += w[i];
            } else {
                or_pc_apply(pc, w, z);
                for (size_t i = 0; i < n; i++) x[i] += z[i];
            }
        }
        for (size_t i = 0; i < (size_t)(m + 1) * m; i++) H[i] = 0.0;
    }
#undef HH
    if (o->fixed_iters && nits >= o->maxit) status = relres <= o->rtol ? OR_OK : OR_NOT_CONVERGED;
    if (res) { res->iters = nits; res->true_relres = relres; res->restarts = cycles; }
    free(V); free(Z); free(H); free(cs); free(sn); free(g); free(y);
    free(r); free(w); free(z);
    return status;
}

/* ======================================================================
 * C6b. LGMRES(m, k) (named with its aug_k parameter in Section 3; the
 * algorithm is not printed).  Baker, Jessup & Manteuffel (2005), right
 * preconditioned: every cycle runs m Arnoldi steps on preconditioned
 * directions u_j = M^-1 v_j, then one more step for each stored
 * correction of the previous cycles (newest first, at most k of them,
 * each normalized), with u_j the correction itself.  The new iterate is
 * x + U y, y minimizing ||beta e_1 - H y||; the correction U y of the
 * cycle becomes the newest stored one.  maxit counts Arnoldi steps of
 * both kinds; the tolerance tests follow or_gmres.
 * ====================================================================== */
int or_lgmres(int nb, int bs, const int *rp, const int *ci, const double *a,
              or_pc *pc, const double *b, double *x, const or_krylov_opts *o,
              int aug_k, or_krylov_result *res, double *hist)
{
    const size_t n = (size_t)nb * bs;
    const int m = o->restart, k = aug_k, mt = o->restart + aug_k;
    if (m < 1 || k < 0 || o->maxit < 0) return OR_ERR_ARG;
    double *V = (double *)malloc(sizeof(double) * n * (mt + 1));
    double *U = (double *)malloc(sizeof(double) * n * mt);
    double *Zs = (double *)malloc(sizeof(double) * n * (k > 0 ? k : 1));  /* newest first */
    double *H = (double *)calloc((size_t)(mt + 1) * mt, sizeof(double));
    double *cs = (double *)malloc(sizeof(double) * mt);
    double *sn = (double *)malloc(sizeof(double) * mt);
    double *g = (double *)malloc(sizeof(double) * (mt + 1));
    double *y = (double *)malloc(sizeof(double) * mt);
    double *r = (double *)malloc(sizeof(double) * n);
    double *w = (double *)malloc(sizeof(double) * n);
    double *dx = (double *)malloc(sizeof(double) * n);
    const double bnorm = nrm2((int)n, b);
    const double tol = fmax(o->rtol * bnorm, o->atol);
    int nits = 0, cycles = 0, nstored = 0, status = OR_NOT_CONVERGED;
    double relres = 0.0;
#define HH(i, j) H[(size_t)(i) * mt + (j)]
    for (;;) {
        memcpy(r, b, sizeof(double) * n);
        or_bsr_amxpby(nb, bs, rp, ci, a, -1.0, x, 1.0, r);
        double tnorm = nrm2((int)n, r);
        relres = bnorm > 0 ? tnorm / bnorm : tnorm;
        if (hist && nits == 0) hist[0] = tnorm;
        if (!o->fixed_iters && tnorm <= tol) { status = OR_OK; break; }
        if (nits >= o->maxit) break;
        double beta = tnorm;
        if (beta == 0.0 || !isfinite(beta)) { status = isfinite(beta) ? OR_OK : OR_ERR_BREAKDOWN; break; }
        for (size_t i = 0; i < n; i++) V[i] = r[i] / beta;
        for (int i = 0; i <= mt; i++) g[i] = 0.0;
        g[0] = beta;
        const int steps = m + nstored;
        int jend = 0;
        cycles++;
        for (int j = 0; j < steps; j++) {
            double *uj = U + n * j;
            if (j < m) or_pc_apply(pc, V + n * j, uj);
            else memcpy(uj, Zs + n * (j - m), sizeof(double) * n);
            or_bsr_spmv(nb, bs, rp, ci, a, uj, w);
            for (int q = 0; q <= j; q++) {           /* MGS */
                double h = dot((int)n, w, V + n * q);
                HH(q, j) = h;
                for (size_t i = 0; i < n; i++) w[i] -= h * V[n * q + i];
            }
            double hn = nrm2((int)n, w);
            HH(j + 1, j) = hn;
            if (hn != 0.0)
                for (size_t i = 0; i < n; i++) V[n * (j + 1) + i] = w[i] / hn;
            for (int q = 0; q < j; q++) {            /* old rotations */
                double t = cs[q] * HH(q, j) + sn[q] * HH(q + 1, j);
                HH(q + 1, j) = -sn[q] * HH(q, j) + cs[q] * HH(q + 1, j);
                HH(q, j) = t;
            }
            double rr = hypot(HH(j, j), HH(j + 1, j));
            if (rr == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
            else { cs[j] = HH(j, j) / rr; sn[j] = HH(j + 1, j) / rr; }
            HH(j, j) = rr;
            HH(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            nits++;
            jend = j + 1;
            if (hist) hist[nits] = fabs(g[j + 1]);
            if (nits >= o->maxit) break;
            if (hn == 0.0) break;                     /* lucky breakdown */
            if (!o->fixed_iters && fabs(g[j + 1]) <= tol) break;
        }
        for (int i = jend - 1; i >= 0; i--) {
            double s = g[i];
            for (int q = i + 1; q < jend; q++) s -= HH(i, q) * y[q];
            y[i] = HH(i, i) != 0.0 ? s / HH(i, i) : 0.0;
        }
        for (size_t i = 0; i < n; i++) dx[i] = 0.0;
        for (int q = 0; q < jend; q++)
            for (size_t i = 0; i < n; i++) dx[i] += y[q] * U[n * q + i];
        for (size_t i = 0; i < n; i++) x[i] += dx[i];
        if (k > 0) {                                  /* store the correction, newest first */
            const double dn = nrm2((int)n, dx);
            if (dn > 0.0 && isfinite(dn)) {
                const int keep = nstored < k ? nstored : k - 1;
                memmove(Zs + n, Zs, sizeof(double) * n * keep);
                for (size_t i = 0; i < n; i++) Zs[i] = dx[i] / dn;
                nstored = keep + 1;
            }
        }
        for (size_t i = 0; i < (size_t)(mt + 1) * mt; i++) H[i] = 0.0;
    }
#undef HH
    if (o->fixed_iters && nits >= o->maxit) status = relres <= o->rtol ? OR_OK : OR_NOT_CONVERGED;
    if (res) { res->iters = nits; res->true_relres = relres; res->restarts = cycles; }
    free(V); free(U); free(Zs); free(H); free(cs); free(sn); free(g); free(y);
    free(r); free(w); free(dx);
    return status;
}

/* ======================================================================
 * C6c. Preconditioned conjugate gradients, Algorithm 2, for symmetric
 * positive definite A and M.  The stopping test is on the recursively
 * updated residual, ||r|| <= max(rtol ||b||, atol), as printed; the
 * reported relative residual is the true one at exit.  A curvature
 * (p, A p) <= 0 or a non-finite scalar ends with OR_ERR_BREAKDOWN.
 * ====================================================================== */
int or_pcg(int nb, int bs, const int *rp, const int *ci, const double *a,
           or_pc *pc, const double *b, double *x, const or_krylov_opts *o,
           or_krylov_result *res, double *hist)
{
    const size_t n = (size_t)nb * bs;
    if (o->maxit < 0) return OR_ERR_ARG;
    double *r = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *q = (double *)malloc(sizeof(double) * n);
    const double bnorm = nrm2((int)n, b);
    const double tol = fmax(o->rtol * bnorm, o->atol);
    int nits = 0, status = OR_NOT_CONVERGED;
    memcpy(r, b, sizeof(double) * n);                 /* r = b - A x0 */
    or_bsr_amxpby(nb, bs, rp, ci, a, -1.0, x, 1.0, r);
    double rn = nrm2((int)n, r);
    if (hist) hist[0] = rn;
    double rho_prev = 0.0;
    if (!o->fixed_iters && rn <= tol) status = OR_OK;
    while (status != OR_OK && nits < o->maxit) {
        or_pc_apply(pc, r, z);                        /* M z = r */
        const double rho = dot((int)n, r, z);
        if (nits == 0) memcpy(p, z, sizeof(double) * n);
        else {
            const double beta = rho / rho_prev;
            for (size_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
        }
        or_bsr_spmv(nb, bs, rp, ci, a, p, q);         /* q = A p */
        const double pq = dot((int)n, p, q);
        if (!(pq > 0.0) || !isfinite(rho)) { status = OR_ERR_BREAKDOWN; break; }
        const double alpha = rho / pq;
        for (size_t i = 0; i < n; i++) x[i] += alpha * p[i];
        for (size_t i = 0; i < n; i++) r[i] -= alpha * q[i];
        rho_prev = rho;
        nits++;
        rn = nrm2((int)n, r);
        if (hist) hist[nits] = rn;
        if (!o->fixed_iters && rn <= tol) status = OR_OK;
    }
    memcpy(q, b, sizeof(double) * n);                 /* true residual at exit */
    or_bsr_amxpby(nb, bs, rp, ci, a, -1.0, x, 1.0, q);
    const double relres = bnorm > 0 ? nrm2((int)n, q) / bnorm : nrm2((int)n, q);
    if (o->fixed_iters && status != OR_ERR_BREAKDOWN)
        status = relres <= o->rtol ? OR_OK : OR_NOT_CONVERGED;
    if (res) { res->iters = nits; res->true_relres = relres; res->restarts = 0; }
    free(r); free(z); free(p); free(q);
    return status;
}

/* ======================================================================
 * C7. BiCGSTAB (van der Vorst 1992), right-preconditioned.  The paper
 * names the method (Section 3) without printing it.  Breakdown
 * (|rho| < 1e-300 ||rhat|| ||r||, <rhat, v> = 0, or omega = 0) restarts
 * from the true residual.  Convergence at a half step (||s||) or a full
 * step (||r||) is confirmed with the true residual; if that fails the
 * iteration restarts from it.
 * ====================================================================== */
int or_bicgstab(int nb, int bs, const int *rp, const int *ci,
                const double *a, or_pc *pc, const double *b, double *x,
                const or_krylov_opts *o, or_krylov_result *res, double *hist)
{
    const size_t n = (size_t)nb * bs;
    double *r = (double *)malloc(sizeof(double) * n);
    double *rh = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *v = (double *)malloc(sizeof(double) * n);
    double *ph = (double *)malloc(sizeof(double) * n);
    double *s = (double *)malloc(sizeof(double) * n);
    double *sh = (double *)malloc(sizeof(double) * n);
    double *t = (double *)malloc(sizeof(double) * n);
    const double bnorm = nrm2((int)n, b);
    const double tol = fmax(o->rtol * bnorm, o->atol);
    int nits = 0, restarts = 0, status = OR_NOT_CONVERGED;
    double relres = 0.0, rho0 = 1.0, alpha = 1.0, omega = 1.0;
    int fresh = 1;
    for (;;) {
        if (fresh) {
            memcpy(r, b, sizeof(double) * n);
            or_bsr_amxpby(nb, bs, rp, ci, a, -1.0, x, 1.0, r);
            double tn = nrm2((int)n, r);
            relres = bnorm > 0 ? tn / bnorm : tn;
            if (hist && nits == 0) hist[0] = tn;
            if (!o->fixed_iters && tn <= tol) { status = OR_OK; break; }
            if (!isfinite(tn)) { status = OR_ERR_BREAKDOWN; break; }
            memcpy(rh, r, sizeof(double) * n);
            rho0 = alpha = omega = 1.0;
            for (size_t i = 0; i < n; i++) { v[i] = 0.0; p[i] = 0.0; }
            fresh = 0;
        }
        if (nits >= o->maxit) break;
        double rho = dot((int)n, rh, r);
        if (fabs(rho) < 1e-300 * nrm2((int)n, rh) * nrm2((int)n, r) || rho == 0.0) {
            fresh = 1; restarts++;
            continue;
        }
        double beta = (rho / rho0) * (alpha / omega);
        for (size_t i = 0; i < n; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        or_pc_apply(pc, p, ph);
        or_bsr_spmv(nb, bs, rp, ci, a, ph, v);
        double rv = dot((int)n, rh, v);
        nits++;
        if (rv == 0.0 || !isfinite(rv)) { fresh = 1; restarts++; continue; }
        alpha = rho / rv;
        for (size_t i = 0; i < n; i++) s[i] = r[i] - alpha * v[i];
        double sn = nrm2((int)n, s);
        if (!o->fixed_iters && sn <= tol) {
            for (size_t i = 0; i < n; i++) x[i] += alpha * ph[i];
            if (hist) hist[nits] = sn;
            fresh = 1;                       /* confirm with true residual */
            continue;
        }
        or_pc_apply(pc, s, sh);
        or_bsr_spmv(nb, bs, rp, ci, a, sh, t);
        double tt = dot((int)n, t, t);
        double ts = dot((int)n, t, s);
        omega = tt != 0.0 ? ts / tt : 0.0;
        for (size_t i = 0; i < n; i++) x[i] += alpha * ph[i] + omega * sh[i];
        for (size_t i = 0; i < n; i++) r[i] = s[i] - omega * t[i];
        double rn = nrm2((int)n, r);
        if (hist) hist[nits] = rn;
        rho0 = rho;
        if (!o->fixed_iters && rn <= tol) { fresh = 1; continue; }
        if (omega == 0.0 || !isfinite(rn)) { fresh = 1; restarts++; continue; }
    }
    if (o->fixed_iters) {
        memcpy(r, b, sizeof(double) * n);
        or_bsr_amxpby(nb, bs, rp, ci, a, -1.0, x, 1.0, r);
        double tn = nrm2((int)n, r);
        relres = bnorm > 0 ? tn / bnorm : tn;
        status = relres <= o->rtol ? OR_OK : OR_NOT_CONVERGED;
    }
    if (res) { res->iters = nits; res->true_relres = relres; res->restarts = restarts; }
    free(r); free(rh); free(p); free(v); free(ph); free(s); free(sh); free(t);
    return status;
}

/* ======================================================================
 * C10. Learned stage network: 4 conv layers 4 -> 32 -> 32 -> 32 -> 3,
 * 3x3x3 cross-correlation, stride 1, zero padding 1, bias, exact GELU
 * x * Phi(x) (Phi via erf) after layers 1-3, linear output.
 * bf16_emul rounds every conv operand (activations and weights, and the
 * upstream gradient in the backward pass) to bfloat16; sums stay FP64.
 * ====================================================================== */
static const int CONV_C[5] = { 4, 32, 32, 32, 3 };

int or_conv_nparams(void)
{
    int np = 0;
    for (int l = 0; l < 4; l++) np += CONV_C[l + 1] * CONV_C[l] * 27 + CONV_C[l + 1];
    return np;
}

double or_gelu(double x) { return 0.5 * x * (1.0 + erf(x / sqrt(2.0))); }

static double gelu_grad(double x)
{
    const double pi = 3.14159265358979323846;
    return 0.5 * (1.0 + erf(x / sqrt(2.0))) + x * exp(-0.5 * x * x) / sqrt(2.0 * pi);
}

/* out[co][cell] = b[co] + sum_ci sum_tap W[co][ci][tap] in[ci][cell+tap] */
static void conv3d(int nx, int ny, int nz, int cin, int cout, const double *W,
                   const double *bias, const double *in, double *out)
{
    size_t cells = (size_t)nx * ny * nz;
    for (int co = 0; co < cout; co++)
        for (int k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    double s = bias[co];
                    for (int ci = 0; ci < cin; ci++)
                        for (int dz = -1; dz <= 1; dz++)
                            for (int dy = -1; dy <= 1; dy++)
                                for (int dx = -1; dx <= 1; dx++) {
                                    int kk = k + dz, jj = j + dy, ii = i + dx;
                                    if (kk < 0 || kk >= nz || jj < 0 || jj >= ny || ii < 0 || ii >= nx) continue;
                                    double wv = W[(((size_t)co * cin + ci) * 27) + (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)];
                                    s += wv * in[ci * cells + ((size_t)kk * ny + jj) * nx + ii];
                                }
                    out[co * cells + ((size_t)k * ny + j) * nx + i] = s;
                }
}

static void round_copy(size_t n, const double *src, double *dst, int bf16)
{
    for (size_t i = 0; i < n; i++) dst[i] = bf16 ? bf16d(src[i]) : src[i];
}

/* forward pass keeping pre-activations z_l and operand copies h_l */
static void conv_forward_full(int nx, int ny, int nz, const double *params,
                              const double *in, int bf16, double **h,
                              double **zpre, double *out)
{
    size_t cells = (size_t)nx * ny * nz;
    const double *pp = params;
    round_copy(cells * CONV_C[0], in, h[0], bf16);
    for (int l = 0; l < 4; l++) {
        int cin = CONV_C[l], cout = CONV_C[l + 1];
        size_t nw = (size_t)cout * cin * 27;
        double *W = (double *)malloc(sizeof(double) * nw);
        round_copy(nw, pp, W, bf16);
        conv3d(nx, ny, nz, cin, cout, W, pp + nw, h[l], zpre[l]);
        free(W);
        pp += nw + cout;
        if (l < 3) {
            double *act = (double *)malloc(sizeof(double) * cells * cout);
            for (size_t q = 0; q < cells * cout; q++) act[q] = or_gelu(zpre[l][q]);
            round_copy(cells * cout, act, h[l + 1], bf16);
            free(act);
        } else {
            memcpy(out, zpre[l], sizeof(double) * cells * cout);
        }
    }
}

void or_conv_forward(int nx, int ny, int nz, const double *params,
                     const double *in, double *out, int bf16_emul)
{
    size_t cells = (size_t)nx * ny * nz;
    double *h[4], *zp[4];
    for (int l = 0; l < 4; l++) {
        h[l] = (double *)malloc(sizeof(double) * cells * CONV_C[l]);
        zp[l] = (double *)malloc(sizeof(double) * cells * CONV_C[l + 1]);
    }
    conv_forward_full(nx, ny, nz, params, in, bf16_emul, h, zp, out);
    for (int l = 0; l < 4; l++) { free(h[l]); free(zp[l]); }
}

double or_conv_loss_grad(int nx, int ny, int nz, const double *params,
                         const double *in, const double *target,
                         double *grad, double *dinput, int bf16_emul)
{
    size_t cells = (size_t)nx * ny * nz;
    double *h[4], *zp[4];
    for (int l = 0; l < 4; l++) {
        h[l] = (double *)malloc(sizeof(double) * cells * CONV_C[l]);
        zp[l] = (double *)malloc(sizeof(double) * cells * CONV_C[l + 1]);
    }
    double *out = (double *)malloc(sizeof(double) * cells * 3);
    conv_forward_full(nx, ny, nz, params, in, bf16_emul, h, zp, out);
    size_t nout = cells * 3;
    double loss = 0.0;
    for (size_t q = 0; q < nout; q++) {
        double d = out[q] - target[q];
        loss += d * d;
    }
    loss /= (double)nout;
    /* g = dL/d(out) */
    double *g = (double *)malloc(sizeof(double) * nout);
    for (size_t q = 0; q < nout; q++) g[q] = 2.0 * (out[q] - target[q]) / (double)nout;
    /* parameter offsets */
    size_t off[4], acc = 0;
    for (int l = 0; l < 4; l++) {
        off[l] = acc;
        acc += (size_t)CONV_C[l + 1] * CONV_C[l] * 27 + CONV_C[l + 1];
    }
    for (int l = 3; l >= 0; l--) {
        int cin = CONV_C[l], cout = CONV_C[l + 1];
        size_t nw = (size_t)cout * cin * 27;
        /* dz = g * act'(z) */
        double *dz = (double *)malloc(sizeof(double) * cells * cout);
        for (size_t q = 0; q < cells * cout; q++)
            dz[q] = (l < 3) ? g[q] * gelu_grad(zp[l][q]) : g[q];
        /* bias gradient from the unrounded dz */
        for (int co = 0; co < cout; co++) {
            double s = 0.0;
            for (size_t c = 0; c < cells; c++) s += dz[co * cells + c];
            grad[off[l] + nw + co] = s;
        }
        double *dzr = (double *)malloc(sizeof(double) * cells * cout);
        round_copy(cells * cout, dz, dzr, bf16_emul);
        /* weight gradient: dW[co][ci][tap] = sum_cell dz[co][cell] h[ci][cell+tap] */
        for (int co = 0; co < cout; co++)
            for (int ci = 0; ci < cin; ci++)
                for (int dzz = -1; dzz <= 1; dzz++)
                    for (int dy = -1; dy <= 1; dy++)
                        for (int dx = -1; dx <= 1; dx++) {
                            double s = 0.0;
                            for (int k = 0; k < nz; k++)
                                for (int j = 0; j < ny; j++)
                                    for (int i = 0; i < nx; i++) {
                                        int kk = k + dzz, jj = j + dy, ii = i + dx;
                                        if (kk < 0 || kk >= nz || jj < 0 || jj >= ny || ii < 0 || ii >= nx) continue;
                                        s += dzr[co * cells + ((size_t)k * ny + j) * nx + i]
                                           * h[l][ci * cells + ((size_t)kk * ny + jj) * nx + ii];
                                    }
                            grad[off[l] + (((size_t)co * cin + ci) * 27) + (dzz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] = s;
                        }
        /* input gradient: gin[ci][cell] = sum_co sum_tap W[co][ci][tap] dz[co][cell - tap] */
        if (l > 0 || dinput) {
            double *W = (double *)malloc(sizeof(double) * nw);
            round_copy(nw, params + off[l], W, bf16_emul);
            double *gin = (double *)calloc(cells * cin, sizeof(double));
            for (int ci = 0; ci < cin; ci++)
                for (int k = 0; k < nz; k++)
                    for (int j = 0; j < ny; j++)
                        for (int i = 0; i < nx; i++) {
                            double s = 0.0;
                            for (int co = 0; co < cout; co++)
                                for (int dzz = -1; dzz <= 1; dzz++)
                                    for (int dy = -1; dy <= 1; dy++)
                                        for (int dx = -1; dx <= 1; dx++) {
                                            int kk = k - dzz, jj = j - dy, ii = i - dx;
                                            if (kk < 0 || kk >= nz || jj < 0 || jj >= ny || ii < 0 || ii >= nx) continue;
                                            s += W[(((size_t)co * cin + ci) * 27) + (dzz + 1) * 9 + (dy + 1) * 3 + (dx + 1)]
                                               * dzr[co * cells + ((size_t)kk * ny + jj) * nx + ii];
                                        }
                            gin[ci * cells + ((size_t)k * ny + j) * nx + i] = s;
                        }
            free(W);
            free(g);
            g = gin;
            if (l == 0 && dinput) memcpy(dinput, gin, sizeof(double) * cells * cin);
        }
        free(dz); free(dzr);
    }
    free(g); free(out);
    for (int l = 0; l < 4; l++) { free(h[l]); free(zp[l]); }
    return loss;
}

/* Adam (Kingma & Ba 2015), bias-corrected, step t >= 1 */
void or_adam_step(int n, double *params, const double *grad, double *m,
                  double *v, int t, double lr, double beta1, double beta2,
                  double eps)
{
    double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
    for (int i = 0; i < n; i++) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * grad[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * grad[i] * grad[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        params[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ======================================================================
 * C11. Learned stage apply with fallback:
 *   z1 = M_base^-1 v;  r1 = v - A z1;  s = rms(r1);
 *   e  = s * N([r1 / s, ln k]);  z2 = z1 + e;
 *   z  = z2 if ||v - A z2|| < ||r1||, else z1 (fallback).
 * ====================================================================== */
static void conv_apply_learned(or_pc *pc, const double *v, double *z)
{
    const int nb = pc->nb;
    const size_t n = (size_t)nb * 3, cells = (size_t)nb;
    double *r1 = (double *)malloc(sizeof(double) * n);
    double *z2 = (double *)malloc(sizeof(double) * n);
    double *r2 = (double *)malloc(sizeof(double) * n);
    double *in = (double *)malloc(sizeof(double) * cells * 4);
    double *out = (double *)malloc(sizeof(double) * cells * 3);
    pc->applies++;
    or_pc_apply(pc->base, v, z);
    memcpy(r1, v, sizeof(double) * n);
    or_bsr_amxpby(nb, 3, pc->rp, pc->ci, pc->a, -1.0, z, 1.0, r1);
    double n1 = nrm2((int)n, r1);
    double s = n1 / sqrt((double)n);
    int accept = 0;
    if (s > 0.0 && isfinite(s)) {
        for (size_t c = 0; c < cells; c++) {
            for (int ch = 0; ch < 3; ch++) in[ch * cells + c] = r1[3 * c + ch] / s;
            in[3 * cells + c] = pc->lnk[c];
        }
        or_conv_forward(pc->nx, pc->ny, pc->nz, pc->params, in, out, pc->bf16);
        int finite = 1;
        for (size_t c = 0; c < cells; c++)
            for (int ch = 0; ch < 3; ch++) {
                z2[3 * c + ch] = z[3 * c + ch] + s * out[ch * cells + c];
                if (!isfinite(z2[3 * c + ch])) finite = 0;
            }
        if (finite) {
            memcpy(r2, v, sizeof(double) * n);
            or_bsr_amxpby(nb, 3, pc->rp, pc->ci, pc->a, -1.0, z2, 1.0, r2);
            double n2 = nrm2((int)n, r2);
            if (n2 < n1) accept = 1;
        }
    }
    if (accept) memcpy(z, z2, sizeof(double) * n);
    else pc->fallbacks++;
    free(r1); free(z2); free(r2); free(in); free(out);
}
