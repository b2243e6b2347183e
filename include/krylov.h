/*
 * krylov.h -- C ABI of the MI355X-native preconditioned Krylov solver.
 *
 * Liu & Chen, "Scalable linear solvers for sparse linear systems from
 * large-scale numerical simulations" (arXiv 1701.05913), re-designed for
 * one gfx950 GPU holding one rank's share of the system.  The object model
 * mirrors the paper's MAP (Section 2.1, Figures 1-5), VEC (Section 2.2,
 * Figures 6-13), MAT (Section 2.3, Figures 15-21), SOLVER (Section 3,
 * Figures 22-28) and preconditioner (Figure 29) interfaces.
 *
 * Conventions
 *  - One rank: a MAP is the trivial row distribution offset = {0, n}
 *    (eq. (1) with N_p = 1); there is no communication.
 *  - Scalars at the boundary are double (the paper's FLOAT); global sizes
 *    int64_t (the paper's INT); matrix index arrays int32_t.
 *  - Every pointer argument marked "device" must point to GPU memory
 *    (hipMalloc, or a PyTorch CUDA tensor); "host" to CPU memory.  The
 *    `where` argument (KRY_HOST / KRY_DEVICE) says which, where both are
 *    accepted.
 *  - Vectors of a block system are interleaved per block row:
 *    (p, s1, s2) of block row 0, then block row 1, ...
 *  - Functions returning int return KRY_OK (0), KRY_NOT_CONVERGED (1) or a
 *    negative error code; functions returning a pointer return NULL on
 *    error.  LastError() describes the most recent error of the calling
 *    thread.
 *  - Work is issued on the solver's stream (SolverSetStream) or, for the
 *    VEC / MAT calls, on the stream set by KrylovSetStream (default: the
 *    null stream).  Calls that return a scalar to the host (VecDot,
 *    VecNorm2, VecGetEntry) synchronize that stream.
 *  - Objects are not thread-safe; distinct objects may be used from
 *    distinct threads.
 */
#ifndef KRYLOV_H
#define KRYLOV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define KRY_OK               0
#define KRY_NOT_CONVERGED    1   /* results (residual, iterations) valid   */
#define KRY_ERR_ARG         -1   /* invalid argument / malformed matrix    */
#define KRY_ERR_DIM         -2   /* size mismatch (the paper's asserts)    */
#define KRY_ERR_ALLOC       -3   /* device or host allocation failed       */
#define KRY_ERR_ZERO_PIVOT  -4   /* ILU pivot block singular              */
#define KRY_ERR_BREAKDOWN   -5   /* Krylov breakdown / non-finite values   */
#define KRY_ERR_HIP         -6   /* HIP runtime error                      */
#define KRY_ERR_UNSUPPORTED -7   /* option not implemented                 */
#define KRY_ERR_STALL       -8   /* a level-scheduled sweep waited longer
                                    than its bound (inconsistent schedule) */

/* ---- enumerations -------------------------------------------------------- */
enum { KRY_HOST = 0, KRY_DEVICE = 1 };
enum { KRY_F64 = 0 };                         /* VEC data type             */
/* GMRES(m) (Algorithm 1, right preconditioned), FGMRES(m), BiCGSTAB, and
 * preconditioned CG (Algorithm 2; A and M symmetric positive definite).
 * GMRES and FGMRES become LGMRES(m, k) with SolverSetAugk(k > 0). */
enum { KRY_GMRES = 0, KRY_FGMRES = 1, KRY_BICGSTAB = 2, KRY_CG = 3 };
enum { KRY_PC_NONE = 0, KRY_PC_ILU0 = 1, KRY_PC_BILU0 = 1, KRY_PC_CPR = 2,
       KRY_PC_CUSTOM = 3,
       /* learned-stage extension: base preconditioner followed by the
        * convolutional correction with its residual-test fallback */
       KRY_PC_BILU0_LEARNED = 4, KRY_PC_CPR_LEARNED = 5,
       /* restricted additive Schwarz with block ILU(0) subdomain solves
        * (Section 4.1): see SolverSetRAS */
       KRY_PC_RAS = 6,
       /* algebraic multigrid, one V-cycle (Section 4.2): see SolverSetAMG */
       KRY_PC_AMG = 7 };
/* precision of the preconditioner apply (mixed-precision extension) */
enum { KRY_PREC_F64 = 0, KRY_PREC_F32 = 1, KRY_PREC_BF16_FACTORS = 2 };
/* CPR stage order (Section 4.2.1): PF = pressure then full (Algorithm 6,
 * read as the two-stage method); FP = full then pressure (Algorithm 5);
 * FPF = full, pressure, full (Algorithm 7); FFPF = full, full, pressure,
 * full (Algorithm 8).  Every stage after the first acts on the residual
 * of the running iterate. */
enum { KRY_CPR_PF = 0, KRY_CPR_FP = 1, KRY_CPR_FPF = 2, KRY_CPR_FFPF = 3 };
/* CPR pressure solver: ILU(0) sweeps (SolverSetCPR's p_sweeps) or one AMG
 * V-cycle on A_pp, the paper's M_g(A_pp)^-1 (Algorithms 5-8) */
enum { KRY_CPR_P_ILU0 = 0, KRY_CPR_P_AMG = 1 };
/* CPR full-system stage R(A)^-1 of Algorithms 5-8: block ILU(0) of A, or
 * RAS with block ILU(0) subdomain solves (the paper's R(A)^-1) on the
 * solver's RAS subdomains (SolverSetRAS / SolverSetRASBoxes) */
enum { KRY_CPR_F_BILU0 = 0, KRY_CPR_F_RAS = 1 };
/* layout of the ILU triangular sweeps: AUTO picks GRID when the matrix is a
 * 7-point stencil on an nx x ny x nz grid (nx, ny, nz >= 2) in natural
 * order, LEVELS otherwise */
enum { KRY_SWEEP_AUTO = 0, KRY_SWEEP_LEVELS = 1, KRY_SWEEP_GRID = 2 };

typedef struct MAP_ MAP;
typedef struct VEC_ VEC;
typedef struct MAT_ MAT;
typedef struct SOLVER_ SOLVER;
typedef struct LEARNED_ LEARNED;

/* ---- MAP: row distribution (Section 2.1, eq. (1)-(2)) --------------------
 * MapCreate requires ilower < iupper (eq. (2)); NULL otherwise.  With one
 * rank the map owns rows [0, iupper - ilower) locally.  MapCreateLocal is
 * the C name of the second creator (Figure 3).  The caller destroys every
 * VEC, MAT and SOLVER built on a map before destroying the map (Figure 4). */
MAP    *MapCreate(int64_t ilower, int64_t iupper);
MAP    *MapCreateLocal(int64_t nlocal);
void    MapDestroy(MAP *map);
int64_t MapGetNlocal(const MAP *map);

/* ---- VEC: device vector (Section 2.2, Figures 6-13) ----------------------
 * VecCreate allocates nlocal doubles on the device (owned, zeroed).
 * VecWrap borrows caller-owned device memory of nlocal doubles; the
 * library never frees it.  VecDestroy frees owned memory and sets *vec to
 * NULL; NULL is a no-op.  Entry access uses local indices and is a slow,
 * synchronous host path meant for tests.  The algebraic calls return
 * KRY_ERR_DIM where the paper asserts equal sizes. */
VEC    *VecCreate(MAP *map, int dtype);
VEC    *VecWrap(MAP *map, void *device_ptr, int dtype);
void    VecDestroy(VEC **vec);
void   *VecGetData(VEC *vec);
int     VecAddEntry(VEC *vec, int64_t idx, double value);    /* Figure 9  */
double  VecGetEntry(VEC *vec, int64_t idx);                  /* Figure 9  */
int     VecSetValue(VEC *x, double v);                       /* Figure 13 */
int     VecAXPBY(double alpha, VEC *x, double beta, VEC *y); /* Figure 10: y = a x + b y */
int     VecAXPBYZ(double alpha, VEC *x, double beta, VEC *y, VEC *z); /* Figure 11 */
double  VecDot(VEC *x, VEC *y);                              /* Figure 12 (NaN on error) */
double  VecNorm2(VEC *x);
/* VecDotNoAlloc: for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Writes <x, y> to result_dev (one double in device memory, caller-owned),
 * asynchronously on the library stream; no allocation, no host sync.  The
 * value equals VecDot's bit for bit (same kernels, same reduction order).
 * The reduction's partial sums live in a static device array of 1024
 * doubles (8 KiB per GPU, held until the process ends); any vector length
 * fits.  All calls on one GPU share that array: calls that overlap on one
 * GPU (other streams, other threads) race.  KRY_ERR_ARG / KRY_ERR_DIM on
 * bad arguments, KRY_ERR_HIP if the array's address cannot be found. */
int     VecDotNoAlloc(VEC *x, VEC *y, double *result_dev);

/* ---- MAT: sparse matrix (Section 2.3, Figures 15-21) ---------------------
 * Built in one call from CSR (bs = 1) or block CSR with bs x bs row-major
 * blocks (bs = 1 or 3).  The arrays are copied into library-owned device
 * storage; `where` says whether they are host or device pointers.
 * Requirements (KRY_ERR_ARG otherwise): rowptr non-decreasing from 0,
 * column indices in [0, n) strictly ascending within a row, every row
 * holding its diagonal.  MatVecMXY: y = A x (Figure 20).  MatVecAMXPBY:
 * y = alpha A x + beta y (Figure 21).  x and y must not alias. */
MAT *MatCreateCSR(MAP *map, int32_t n, const int32_t *rowptr,
                  const int32_t *col, const double *val, int where);
MAT *MatCreateBSR(MAP *map, int32_t nb, int32_t bs, const int32_t *browptr,
                  const int32_t *bcol, const double *bval, int where);
void MatDestroy(MAT **mat);
/* New values for the same pattern (nnzb * bs * bs doubles in the block
 * order of MatCreate*, host or device, copied): a Newton loop's next
 * Jacobian.  A solver holding the matrix refactors at its next
 * SolverAssemble, reusing what depends on the pattern only (the RAS
 * subdomain patterns and tilings). */
int  MatUpdateValues(MAT *A, const double *val, int where);
/* The 7-point grid the pattern was recognised as (MatCreate checks every
 * row against the stencil in natural order cell = i + nx (j + ny k));
 * returns KRY_OK and the sizes, or KRY_ERR_ARG with zeros when the pattern
 * is not such a stencil. */
int  MatGetGrid(const MAT *A, int32_t *nx, int32_t *ny, int32_t *nz);
int  MatVecMXY(MAT *A, VEC *x, VEC *y);
int  MatVecAMXPBY(double alpha, MAT *A, VEC *x, double beta, VEC *y);
int64_t MatGetNnzBlocks(const MAT *A);

/* ---- SOLVER (Section 3, Figures 22-28) -----------------------------------
 * SolverCreate(type, pc_type, map) as in Figure 23.  SolverSetMat borrows
 * the matrix, which must outlive the solver (replaces the entry-adding
 * calls of Figure 27).  SolverAssemble builds the preconditioner
 * (Figure 25): level sets, ILU(0)/block ILU(0) factor, CPR pressure
 * matrix, reduced-precision copies.  SolverSolve(solver, b, x) solves
 * A x = b (Figure 26 plus an explicit right-hand side); x holds the
 * initial guess on entry.  Convergence: ||b - A x||_2 <= max(rtol ||b||_2,
 * atol), judged by the true FP64 residual; btol is stored, unused.
 * Iterations: Arnoldi steps for GMRES/FGMRES, one per BiCGSTAB pass.
 * Returns KRY_OK, KRY_NOT_CONVERGED (maxit reached, results filled) or an
 * error.  SolverPCApply applies the assembled preconditioner once:
 * z = M^-1 v (z and v distinct). */
SOLVER *SolverCreate(int solver_type, int pc_type, MAP *map);
int     SolverDestroy(SOLVER **solver);
int     SolverSetMat(SOLVER *s, MAT *A);
int     SolverAssemble(SOLVER *s);
int     SolverSolve(SOLVER *s, VEC *b, VEC *x);
int     SolverPCApply(SOLVER *s, VEC *v, VEC *z);

void SolverSetDefaultMaxit(int64_t it);
void SolverSetDefaultRtol(double tol);
void SolverSetDefaultAtol(double tol);
void SolverSetDefaultBtol(double tol);
void SolverSetDefaultRestart(int64_t m);
void SolverSetDefaultAugk(int64_t k);
int  SolverSetMaxit(SOLVER *s, int64_t it);
int  SolverSetRtol(SOLVER *s, double tol);
int  SolverSetAtol(SOLVER *s, double tol);
int  SolverSetBtol(SOLVER *s, double tol);
int  SolverSetRestart(SOLVER *s, int64_t m);    /* 1 <= m, m + aug_k <= 63 */
/* aug_k (Section 3, the SOLVER structure): k > 0 turns GMRES/FGMRES into
 * LGMRES(m, k): every cycle adds one Arnoldi step per stored correction
 * x_i - x_{i-1} of the last k cycles (normalized, newest first; Baker,
 * Jessup & Manteuffel), with flexible storage of the directions.  0 <= k,
 * restart + k <= 63, else KRY_ERR_ARG; SolverAssemble rejects k > 0 for
 * BiCGSTAB and CG. */
int  SolverSetAugk(SOLVER *s, int64_t k);

/* Extensions beyond the paper:
 * SolverSetPrecision: precision of the preconditioner apply (FP64, FP32
 *   factors and arithmetic, or BF16-stored off-diagonal factor blocks with
 *   FP32 diagonal inverses and FP32 arithmetic); requires FGMRES for
 *   anything but FP64.  Outer iteration, orthogonalization, Givens and
 *   true residuals stay FP64.
 * SolverSetCPR: stage order (KRY_CPR_*) and number of ILU(0) sweeps of the
 *   pressure stage (default PF, 4); KRY_ERR_ARG for another variant or
 *   p_sweeps < 1.
 * SolverSetStream: HIP stream (hipStream_t) for all work of the solver. */
int SolverSetPrecision(SOLVER *s, int prec);
int SolverSetCPR(SOLVER *s, int variant, int p_sweeps);
/* CPR's pressure solver, KRY_CPR_P_ILU0 (default) or KRY_CPR_P_AMG (FP64
 * only; KRY_ERR_UNSUPPORTED at SolverAssemble otherwise). */
int SolverSetCPRPressure(SOLVER *s, int psolver);
/* CPR's full-system stage, KRY_CPR_F_BILU0 (default) or KRY_CPR_F_RAS (FP64
 * and a 7-point grid matrix; KRY_ERR_UNSUPPORTED at SolverAssemble
 * otherwise). */
int SolverSetCPRFull(SOLVER *s, int fsolver);
/* Algebraic multigrid (Section 4.2: Algorithm 3 setup, Algorithm 4
 * V-cycle; classical Ruge-Stueben strength, coarsening and interpolation
 * with Figure 34's strength 0.5, max row sum 0.9 and truncation 0.01), for
 * KRY_PC_AMG on a scalar (bs = 1) matrix and for CPR's AMG pressure
 * stage.  max_levels (default 8) counts the coarsest level, which is
 * solved exactly through a dense inverse (at most 8192 rows,
 * KRY_ERR_UNSUPPORTED otherwise); num_sweeps (default 2) hybrid
 * Gauss-Seidel sweeps before and after the coarse correction, Gauss-Seidel
 * inside chunks of gs_chunk consecutive rows (1, 2, 4, 8 or 16; default 4)
 * and Jacobi between chunks.  The setup runs on the host at
 * SolverAssemble; the V-cycle runs on the GPU.  FP64 only.  KRY_ERR_ARG
 * for max_levels < 1 or num_sweeps < 1. */
int SolverSetAMG(SOLVER *s, int max_levels, int num_sweeps, int gs_chunk);
/* The AMG hierarchy built by SolverAssemble (KRY_PC_AMG, or CPR with the
 * AMG pressure stage): SolverGetAMGLevels returns the number of levels
 * (KRY_ERR_ARG without a hierarchy).  SolverGetAMGLevel writes the sizes of
 * level l (rows n, entries nnz of A_l, coarse rows nc and entries pnnz of
 * P_l, both 0 on the coarsest level) and, for every non-NULL array, A_l in
 * CSR (rowptr[n+1], col[nnz], val[nnz]), the C/F splitting (cf[n], 1 = C)
 * and P_l in CSR (prowptr[n+1], pcol[pnnz], pval[pnnz]); host memory. */
int SolverGetAMGLevels(const SOLVER *s);
int SolverGetAMGLevel(const SOLVER *s, int l, int *n, int *nnz, int *nc, int *pnnz, int *rowptr,
                      int *col, double *val, int *cf, int *prowptr, int *pcol, double *pval);
/* Restricted additive Schwarz (Section 4.1, the RAS preconditioner, with
 * ILU(0) as the local solver and the paper's default overlap of 1): the
 * matrix must be a 7-point grid stencil in natural order (MatGetGrid); it
 * is cut into nsub z-slabs of nz/nsub layers (owned rows), each grown by
 * `overlap` layers on both sides, factored by block ILU(0) and swept together
 * with the other slabs; the solution is written back on the owned rows only.
 * FP64 only.  Defaults nsub = 4, overlap = 1; KRY_ERR_ARG for nsub < 1 or
 * overlap < 0, and at SolverAssemble for nsub > nz; KRY_ERR_UNSUPPORTED
 * for a matrix that is not a grid stencil or a reduced precision. */
int SolverSetRAS(SOLVER *s, int nsub, int overlap);
/* RAS on boxes: the grid is cut into px x py x pz boxes (sides n/p, the
 * last ones taking the remainder); each box is grown by `overlap` cells in
 * every direction, edges and corners included (for z-slabs, px = py = 1,
 * exactly `overlap` rounds of graph neighbours), factored by block ILU(0)
 * and swept with all other boxes in one launch.  Grown boxes must have
 * sides >= 3 in x and y and >= 2 in z unless px = py = 1 (KRY_ERR_UNSUPPORTED
 * at SolverAssemble).  SolverSetRAS(s, n, o) = SolverSetRASBoxes(s, 1, 1, n, o). */
int SolverSetRASBoxes(SOLVER *s, int px, int py, int pz, int overlap);
/* SolverSetSweepLayout: KRY_SWEEP_AUTO (default), KRY_SWEEP_LEVELS (generic
 * level-scheduled sweeps), or KRY_SWEEP_GRID (grid-tiled sweeps; assembly
 * fails with KRY_ERR_ARG if the matrix is not a 7-point grid stencil).
 * Both layouts apply the same factor. */
int SolverSetSweepLayout(SOLVER *s, int layout);
/* SolverSetOrthog: Gram-Schmidt of the Arnoldi step (Algorithm 1, whose
 * modified Gram-Schmidt both kinds equal in exact arithmetic).
 * KRY_ORTHO_AUTO (default): GMRES with a fixed preconditioner (not custom or
 * learned, no augmentation, restart m <= 31) takes the lagged CGS2 (DCGS2)
 * of Swirydowicz, Langou, Ananthan, Yang and Thomas (2020), two passes over
 * V per step: each step's second projection is applied during the next
 * step, whose residual estimate uses the once-projected column (it differs
 * from the final one by rounding).  Every other solver, and KRY_ORTHO_CGS2,
 * takes CGS2: three passes per step.  KRY_ERR_ARG for another kind. */
enum { KRY_ORTHO_AUTO = 0, KRY_ORTHO_CGS2 = 1 };
int SolverSetOrthog(SOLVER *s, int kind);
int SolverSetStream(SOLVER *s, void *hip_stream);

/* results (Figure 22: residual, nits) */
double SolverGetResidual(const SOLVER *s);   /* final true relative residual */
int    SolverGetIters(const SOLVER *s);
int    SolverGetTimes(const SOLVER *s, double *setup_s, double *solve_s);
/* residual history: entry 0 is ||r0||, entry k the estimate (GMRES) or
 * the recurrence residual norm (BiCGSTAB) after iteration k; returns the
 * number of entries written (at most cap). */
int    SolverGetHistory(const SOLVER *s, double *hist, int cap);
/* Krylov basis of the last Arnoldi cycle (Algorithm 1: the orthonormal
 * v_1 ... v_{m+1} of GMRES / FGMRES / LGMRES): copies columns
 * [first, first + ncols) of V, each n = nb * bs values, into dst (column
 * after column, n apart; dst on `where`).  Column 0 holds the next cycle's
 * unnormalized residual once a solve has ended.  KRY_ERR_ARG if the solver
 * has no basis (BiCGSTAB, CG, no solve yet) or the range exceeds its
 * columns.  Synchronizes the solver's stream. */
int    SolverGetKrylovBasis(const SOLVER *s, int first, int ncols, double *dst, int where);

/* Custom preconditioner (Figure 29): setup(data, A) once in
 * SolverAssemble, solve(data, x, b) computes x = M^-1 b on the solver's
 * stream, destroy(data) in SolverDestroy.  pc_type must be
 * KRY_PC_CUSTOM.  Only FGMRES may use a preconditioner that varies. */
typedef int  (*PC_SETUP)(void *data, MAT *A);
typedef int  (*PC_SOLVE)(void *data, VEC *x, VEC *b);
typedef void (*PC_DESTROY)(void *data);
int SolverSetPC(SOLVER *s, PC_SETUP setup, PC_SOLVE solve,
                PC_DESTROY destroy, void *data);

/* ---- learned preconditioner stage (extension beyond the paper) -------------
 * Network: four 3x3x3 convolutions 4 -> 32 -> 32 -> 32 -> 3 channels with
 * zero padding and bias, exact GELU after the first three, BF16 operands
 * with FP32 accumulation.  Parameters (LearnedNumParams() = 61443 FP32
 * values): for each layer l, W_l[co][ci][tap] with
 * tap = (dz+1)*9 + (dy+1)*3 + (dx+1), then b_l[co].
 *
 * Inside a solver (pc_type KRY_PC_BILU0_LEARNED or KRY_PC_CPR_LEARNED,
 * FGMRES only, a 3x3-block 7-point grid matrix): z1 = M_base^-1 v,
 * r1 = v - A z1, s = ||r1|| / sqrt(n), e = s N([r1 / s, ln k]),
 * z2 = z1 + e; the apply returns z2 if ||v - A z2|| < ||r1|| and z1
 * otherwise (a fallback; also when s is zero or anything is not finite).
 *   SolverSetLearned: parameters from a checkpoint file written by
 *     LearnedSave; ln k per cell (nb values, FP32, device).
 *   SolverSetLearnedParams: parameters from host memory; ln k on `where`.
 *   SolverGetLearnedStats: applications and fallbacks since assembly.
 * Both setters copy their inputs; call them before SolverAssemble. */
int SolverSetLearned(SOLVER *s, const char *weights_path, const float *logk_dev);
int SolverSetLearnedParams(SOLVER *s, const float *params_host, const float *logk,
                           int where);
int SolverGetLearnedStats(SOLVER *s, int64_t *applies, int64_t *fallbacks);

/* Training interface on an nx x ny x nz grid (the network alone).
 * Tensors are channel-major FP32 on the device: input [4][cells]
 * (three residual components, then ln k), output and target [3][cells],
 * cells in natural order (x fastest).
 *   LearnedCreate(training = 0) allocates the forward pass only;
 *     training = 1 adds pre-activations, gradients and Adam moments.
 *   LearnedSetParams / LearnedGetParams copy the FP32 master parameters.
 *   LearnedForward: out = N(in).
 *   LearnedLossGrad: loss = mean((N(in) - target)^2) (returned on the host)
 *     and its gradient (device, LearnedNumParams() values; may be NULL:
 *     kept internally for LearnedAdamStep).
 *   LearnedAdamStep: one bias-corrected Adam step on the last gradient.
 *   LearnedSave / LearnedLoad: checkpoint (parameters, Adam moments and
 *     step count) in a little-endian binary file.
 * All calls synchronize the object's stream (LearnedSetStream). */
/* Training pair of the stage (extension (4) harvest): from the residual
 * r1 = v - A M_base^-1 v and its exact correction d = A^-1 r1 (FP64,
 * interleaved, 3 values per cell, device), writes in = [r1 / s, ln k] and
 * target = d / s, channel-major FP32 on the device, s = ||r1|| / sqrt(n)
 * (returned in *s_host).  Runs on the VEC / MAT stream and synchronizes. */
int LearnedMakePair(int64_t cells, const double *r1, const double *d, const float *logk,
                    float *in, float *target, double *s_host);
LEARNED *LearnedCreate(int nx, int ny, int nz, int training);
int LearnedDestroy(LEARNED **L);
int LearnedNumParams(void);
int LearnedSetStream(LEARNED *L, void *hip_stream);
int LearnedSetParams(LEARNED *L, const float *params, int where);
int LearnedGetParams(LEARNED *L, float *params_host);
int LearnedForward(LEARNED *L, const float *in, float *out);
int LearnedLossGrad(LEARNED *L, const float *in, const float *target, float *loss_host,
                    float *grad);
/* LearnedBackward: parameter gradient of any loss from dout = dL/d(out)
 *   ([3][cells] FP32, device) and the activations of the last
 *   LearnedForward of this (training) object; grad as in LearnedLossGrad.
 * LearnedResidualGrad: the residual loss of the stage,
 *   loss = ||A e - r1/s||^2 / n with e = out (the last output) and r1/s the
 *   first three channels of `in`, and dout = (2/n) A^T (A e - r1/s); At is
 *   the transpose of A as its own MAT (both 3x3-block, one block row per
 *   cell of this object's grid).  The loss is returned on the host. */
int LearnedBackward(LEARNED *L, const float *dout, float *grad);
int LearnedResidualGrad(LEARNED *L, const MAT *A, const MAT *At, const float *in,
                        const float *out, float *dout, double *loss_host);
int LearnedAdamStep(LEARNED *L, float lr, float beta1, float beta2, float eps);
int LearnedSave(LEARNED *L, const char *path);
int LearnedLoad(LEARNED *L, const char *path);

/* ---- per-kernel timing (measurement only) ----------------------------------
 * When enabled, the library brackets every launch of the kernels it times
 * (SpMV, ILU sweeps, Gram-Schmidt passes) with HIP events on the launch
 * stream.
 * KernelTimingQuery synchronizes and returns the launch count and the
 * summed duration in milliseconds of the named kernel family: "spmv_bsr3"
 * and "spmv_csr" (FP64 SpMV), "ilu_fwd_<fmt>_<prec>" and
 * "ilu_bwd_<fmt>_<prec>" (forward / backward sweep, fmt = bsr3 or csr,
 * prec = f64, f32 or bf16 factor storage), "cgs2" (one CGS2
 * orthogonalization step: both Gram-Schmidt passes, the norm and the Givens
 * update), "dcgs2" (one step of the lagged CGS2: its two passes, the
 * finish of the previous Hessenberg column, the norm and the estimate),
 * "learned_stage" (one learned-stage apply after the base preconditioner),
 * "conv_l<k>_fwd" (layer k of the network), "conv_wgrad", "conv_dgrad"
 * (weight and input gradients).  Each event adds a few microseconds
 * between the launches it separates, so a caller that times a whole solve
 * can restrict the events to the families it needs: KernelTimingSelect
 * takes a comma-separated list of the names above (NULL or "" selects
 * every family) and applies to launches issued after the call; the list is
 * copied, the call never fails.  KernelTimingSample(k) brackets only the
 * first of every k launches of each family (k = 1, the default, brackets
 * all; KRY_ERR_ARG for k < 1); it restarts the per-family launch counts,
 * as does KernelTimingReset. */
int KernelTimingEnable(int on);
int KernelTimingSelect(const char *names);
int KernelTimingSample(int every);
int KernelTimingReset(void);
int KernelTimingQuery(const char *name, int64_t *launches, double *total_ms);

/* stream for VEC / MAT calls (hipStream_t; NULL = null stream) */
int KrylovSetStream(void *hip_stream);

const char *LastError(void);

#ifdef __cplusplus
}
#endif
#endif /* KRYLOV_H */
