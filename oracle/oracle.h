/*
 * FP64 CPU oracle for the preconditioned Krylov solve of Liu & Chen,
 * "Scalable linear solvers for sparse linear systems from large-scale
 * numerical simulations" (arXiv 1701.05913).
 *
 * TEST INFRASTRUCTURE ONLY.  This header and oracle.c are used by the test
 * suite, by the package's smoke check and by the CPU-baseline leg of the
 * benchmark.  The GPU library never includes, links or calls anything here,
 * and nothing here includes or calls the GPU library.
 *
 * Plain, slow, obviously-correct C99 in double precision (the paper's FLOAT
 * is never fixed; double is its most likely meaning).  Single precision and
 * bfloat16 are emulated only where the mixed-precision preconditioner asks
 * for them (float arithmetic, bf16 = round-to-nearest-even of the float bit
 * pattern to its top 16 bits).
 *
 * Matrices are block-CSR with block size bs (bs = 1 is plain CSR), blocks
 * row-major, columns ascending within a row, every row holding its
 * diagonal block.  Vectors of a bs-block system are interleaved per block
 * row: (p, s1, s2) of cell 0, then cell 1, ...
 *
 * Parity status: every function here is pinned by the CPU tests (dense
 * solves, closed forms, invariants, finite differences) except the gain of
 * the learned preconditioner stage, which is measured, not pinned.
 */
#ifndef KRYLOV_ORACLE_H
#define KRYLOV_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_OK = 0, OR_NOT_CONVERGED = 1, OR_ERR_ARG = -1,
       OR_ERR_ZERO_PIVOT = -4, OR_ERR_BREAKDOWN = -5 };

enum { OR_PREC_F64 = 0, OR_PREC_F32 = 1, OR_PREC_BF16 = 2 };

/* ---- sparse matrix-vector products (Figures 20-21) -------------------- */
void or_bsr_spmv(int nb, int bs, const int *rp, const int *ci,
                 const double *a, const double *x, double *y);
void or_bsr_amxpby(int nb, int bs, const int *rp, const int *ci,
                   const double *a, double alpha, const double *x,
                   double beta, double *y);

/* ---- ILU(0) / block ILU(0) (Section 1 "point-wise and block-wise
 *      incomplete factorization", eq. (3) for the solve) ---------------- */
int  or_bilu0(int nb, int bs, const int *rp, const int *ci,
              const double *a, double *lu);
void or_bilu0_solve(int nb, int bs, const int *rp, const int *ci,
                    const double *lu, const double *b, double *x);
void or_bilu0_solve_lower(int nb, int bs, const int *rp, const int *ci,
                          const double *lu, const double *b, double *y);
void or_bilu0_solve_upper(int nb, int bs, const int *rp, const int *ci,
                          const double *lu, const double *y, double *x);

/* ---- algebraic multigrid (Section 4.2, Algorithms 3-4, Figure 34) ------ */
typedef struct {
    double strength;      /* strength threshold theta (0.5)                   */
    double max_row_sum;   /* rows with |row sum| > this * |diagonal| are weak (0.9) */
    double trunc;         /* interpolation truncation factor (1e-2)           */
    int max_levels;       /* levels including the coarsest (8)                */
    int num_sweeps;       /* smoothing sweeps before and after (2)            */
    int gs_chunk;         /* rows per Gauss-Seidel chunk; <= 0: all rows (0)  */
    int coarse_size;      /* a level this small is the coarsest (9)           */
} or_amg_opts;
typedef struct or_amg or_amg;
void or_amg_defaults(or_amg_opts *o);
/* hierarchy of a scalar CSR matrix (Algorithm 3 on every level) */
or_amg *or_amg_create(int n, const int *rp, const int *ci, const double *a,
                      const or_amg_opts *o, int *err);
/* x = one V-cycle (Algorithm 4) applied to b from x = 0 */
void or_amg_vcycle(or_amg *M, const double *b, double *x);
void or_amg_destroy(or_amg *M);
/* strong dependencies of every row into srp[n+1], sci[<= rp[n]]; returns
 * their number */
int or_amg_strength(int n, const int *rp, const int *ci, const double *a,
                    double theta, double max_row_sum, int *srp, int *sci);
int or_amg_nlevels(const or_amg *M);
void or_amg_level_size(const or_amg *M, int l, int *n, int *nnz, int *nc, int *pnnz);
/* A_l, and (not on the coarsest level) the C/F splitting and P_l */
void or_amg_level_get(const or_amg *M, int l, int *rp, int *ci, double *a, int *cf,
                      int *prp, int *pci, double *pv);

/* ---- preconditioner objects (Figure 29: setup / solve / destroy) ------- */
typedef struct or_pc or_pc;
enum { OR_PC_NONE = 0, OR_PC_BILU0 = 1, OR_PC_CPR_PF = 2, OR_PC_CPR_FP = 3,
       OR_PC_LEARNED = 4, OR_PC_CPR_FPF = 5, OR_PC_CPR_FFPF = 6, OR_PC_RAS = 7,
       OR_PC_AMG = 8 };

or_pc *or_pc_create(int kind, int nb, int bs, const int *rp, const int *ci,
                    const double *a, int prec, int p_sweeps, int *err);
/* Learned stage on top of an existing BILU(0)/CPR preconditioner `base`
 * (ownership of base passes to the new object).  w/b are the conv-net
 * parameters (layout of or_conv_forward), lnk per cell, grid nx,ny,nz.
 * bf16_emul != 0 rounds the network's operands to bfloat16. */
or_pc *or_pc_create_learned(or_pc *base, int nx, int ny, int nz,
                            const double *params, const double *lnk,
                            int bf16_emul);
/* RAS with a general partition: block row r owned by subdomain part[r] */
or_pc *or_pc_create_ras_part(int nb, int bs, const int *rp, const int *ci,
                             const double *a, int nsub, const int *part,
                             int overlap, int *err);
/* RAS with explicit overlapped sets: subdomain s solves on the ascending
 * block rows sets[set_ptr[s] .. set_ptr[s+1]), which must hold its owned
 * rows (part[r] == s) */
or_pc *or_pc_create_ras_sets(int nb, int bs, const int *rp, const int *ci,
                             const double *a, int nsub, const int *part,
                             const int *set_ptr, const int *sets, int *err);
/* RAS with block ILU(0) local solves: owned block rows
 * [starts[s], starts[s+1]) for s < nsub, `overlap` rounds of graph
 * neighbours (restricted prolongation) */
or_pc *or_pc_create_ras(int nb, int bs, const int *rp, const int *ci,
                        const double *a, int nsub, const int *starts,
                        int overlap, int *err);
/* AMG preconditioners (FP64): kind OR_PC_AMG, one V-cycle on a scalar
 * matrix (bs = 1); or a CPR kind (bs = 3) whose pressure stage is one
 * V-cycle on A_pp instead of ILU(0) sweeps */
or_pc *or_pc_create_amg(int kind, int nb, int bs, const int *rp, const int *ci,
                        const double *a, const or_amg_opts *o, int *err);
/* FP64 CPR (a CPR kind, bs = 3) with the pressure stage one AMG V-cycle
 * (amg != NULL) or p_sweeps ILU(0) sweeps, and the full-system stage R(A)^-1
 * the preconditioner `full` (e.g. RAS; ownership passes, also on failure)
 * or, when NULL, block ILU(0) */
or_pc *or_pc_create_cpr(int kind, int nb, const int *rp, const int *ci, const double *a,
                        const or_amg_opts *amg, int p_sweeps, or_pc *full, int *err);
void or_pc_apply(or_pc *pc, const double *v, double *z);
void or_pc_destroy(or_pc *pc);
/* counters of the learned stage: applications and fallbacks */
void or_pc_learned_stats(const or_pc *pc, long *applies, long *fallbacks);
/* CPR internals, exposed for pins */
int  or_cpr_weights(int nb, const int *rp, const int *ci, const double *a,
                    double *w /* nb*3 */);
void or_cpr_extract_pressure(int nb, const int *rp, const int *ci,
                             const double *a, const double *w,
                             double *app /* nnzb values, pattern of A */);

/* ---- Krylov solvers (Algorithms 1-2; BiCGSTAB and LGMRES named in Section 3) */
typedef struct {
    int    restart;      /* m of GMRES(m) */
    int    maxit;        /* total iterations (Arnoldi steps / BiCGSTAB its) */
    double rtol, atol;
    int    flexible;     /* FGMRES: store Z = M^-1 V */
    int    left;         /* Algorithm 1 as printed: left preconditioning */
    int    check_at_cycle_end; /* Algorithm 1 literally: test only at cycle end */
    int    fixed_iters;  /* run exactly maxit iterations, ignore tolerance */
} or_krylov_opts;

typedef struct {
    int    iters;
    double true_relres;  /* ||b - A x|| / ||b|| at exit, FP64 */
    int    restarts;     /* GMRES cycles / BiCGSTAB breakdown restarts */
} or_krylov_result;

int or_gmres(int nb, int bs, const int *rp, const int *ci, const double *a,
             or_pc *pc, const double *b, double *x, const or_krylov_opts *o,
             or_krylov_result *res, double *hist /* maxit+1 or NULL */);
/* LGMRES(m = o->restart, k = aug_k): GMRES augmented with up to k stored
 * corrections of earlier cycles (flexible storage; Section 3 names it) */
int or_lgmres(int nb, int bs, const int *rp, const int *ci, const double *a,
              or_pc *pc, const double *b, double *x, const or_krylov_opts *o,
              int aug_k, or_krylov_result *res, double *hist /* maxit+1 or NULL */);
/* preconditioned conjugate gradients (Algorithm 2), SPD A and M */
int or_pcg(int nb, int bs, const int *rp, const int *ci, const double *a,
           or_pc *pc, const double *b, double *x, const or_krylov_opts *o,
           or_krylov_result *res, double *hist /* maxit+1 or NULL */);
int or_bicgstab(int nb, int bs, const int *rp, const int *ci,
                const double *a, or_pc *pc, const double *b, double *x,
                const or_krylov_opts *o, or_krylov_result *res,
                double *hist /* maxit+1 or NULL */);

/* ---- learned stage: 4-layer 3D conv net (4 -> 32 -> 32 -> 32 -> 3) ----
 * params: for each layer l, W_l[co][ci][kz][ky][kx] then b_l[co].
 * Activations channel-major: x[c][k][j][i] (i fastest, cell order).      */
int  or_conv_nparams(void);
void or_conv_forward(int nx, int ny, int nz, const double *params,
                     const double *in /* 4*cells */, double *out /* 3*cells */,
                     int bf16_emul);
/* loss = mean((out - target)^2); returns loss and fills grad (nparams) and
 * optionally dinput (4*cells). */
double or_conv_loss_grad(int nx, int ny, int nz, const double *params,
                         const double *in, const double *target,
                         double *grad, double *dinput, int bf16_emul);
void or_adam_step(int n, double *params, const double *grad, double *m,
                  double *v, int t, double lr, double beta1, double beta2,
                  double eps);
double or_gelu(double x);

/* ---- precision helpers ------------------------------------------------ */
float or_bf16_round(float f);

#ifdef __cplusplus
}
#endif
#endif
