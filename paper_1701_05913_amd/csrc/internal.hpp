// Internal declarations of the gfx950 Krylov library (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <memory>
#include <utility>
#include <string>
#include <vector>

#include "krylov.h"

namespace kry {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
int set_error(int code, const char *fmt, ...);

#define KRY_HIP(call)                                                          \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess)                                                  \
            return ::kry::set_error(KRY_ERR_HIP, "%s: %s (%s:%d)", #call,      \
                                    hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

#define KRY_TRY(expr)                                                          \
    do {                                                                       \
        int rc_ = (expr);                                                      \
        if (rc_ < 0) return rc_;                                               \
    } while (0)

// ---------------------------------------------------------------------------
// device buffers (library-owned memory)
// ---------------------------------------------------------------------------
template <typename T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }
    int alloc(size_t count) {
        release();
        if (count == 0) count = 1;
        if (hipMalloc(reinterpret_cast<void **>(&p), count * sizeof(T)) != hipSuccess) {
            p = nullptr;
            return set_error(KRY_ERR_ALLOC, "hipMalloc of %zu bytes failed", count * sizeof(T));
        }
        n = count;
        return KRY_OK;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
};

// ---------------------------------------------------------------------------
// sliced ELLPACK with 64-row slices (one wavefront per slice) and
// entry-major value planes: value e of slot t of lane l sits at
// val[(t * b2 + e) * 64 + l].  A slot is one nonzero block position of all
// 64 rows of a slice; col = -1 marks padding.  perm maps slice lanes to
// matrix rows (-1: padding row); empty perm means natural order.
// ---------------------------------------------------------------------------
struct Sell {
    int bs = 1;
    int nslices = 0;
    int64_t nslots = 0;
    int maxw = 0;
    DBuf<int> off;       // nslices + 1
    DBuf<int> col;       // nslots * 64
    DBuf<double> val;    // nslots * b2 * 64
    DBuf<float> valf;    // optional FP32 copy
    DBuf<uint16_t> valh; // optional BF16 copy
    DBuf<int> perm;      // nslices * 64 (optional)
    std::vector<int> h_off;
};

}  // namespace kry

// ---------------------------------------------------------------------------
// C ABI objects
// ---------------------------------------------------------------------------
struct MAP_ {
    int64_t ilower = 0, iupper = 0, nlocal = 0, nglobal = 0;
    int64_t offset[2] = {0, 0};
    int rank = 0, nprocs = 1;
};

struct VEC_ {
    MAP *map = nullptr;
    int64_t n = 0;
    int dtype = KRY_F64;
    double *data = nullptr;
    bool owned = false;
};

struct MAT_ {
    MAP *map = nullptr;
    int nb = 0, bs = 1;
    int64_t nnzb = 0;
    std::vector<int> h_rowptr, h_col, h_diag;   // host copy of the pattern
    kry::DBuf<int> rowptr, col, diag;
    kry::DBuf<double> val;                      // block CSR values (FP64)
    kry::Sell sell;                             // natural-order SpMV layout
    kry::DBuf<float> col0f;                     // FP32 column-0 planes (bs=3)
    int gnx = 0, gny = 0, gnz = 0;              // 7-point grid of the pattern (0: none)
};

namespace kry {

hipStream_t global_stream();

// ---------------------------------------------------------------------------
// kernel timing registry (HIP events around selected launches)
// ---------------------------------------------------------------------------
bool timing_on();
// timing is on and the scope name is among the selected ones (all when
// none are selected)
bool timing_wanted(const char *name);
void timing_begin(const char *name, hipStream_t s);
void timing_end(const char *name, hipStream_t s);

struct TimedScope {
    const char *name;
    hipStream_t s;
    bool on;
    TimedScope(const char *n, hipStream_t st) : name(n), s(st), on(timing_wanted(n)) {
        if (on) timing_begin(name, s);
    }
    ~TimedScope() {
        if (on) timing_end(name, s);
    }
};

// ---------------------------------------------------------------------------
// reductions: fixed-size grids and a fixed summation order, so results
// are bitwise reproducible run to run
// ---------------------------------------------------------------------------
constexpr int RED_BLOCKS = 512;   // partial sums per reduction
constexpr int RED_THREADS = 256;

// vector kernels (vec.hip)
struct Coef {
    const double *p;  // device scalar, or nullptr
    double v;         // host value (p == nullptr) or multiplier of *p
};
inline Coef hc(double v) { return Coef{nullptr, v}; }
inline Coef dc(const double *p, double mul = 1.0) { return Coef{p, mul}; }

int vec_fill(hipStream_t s, int64_t n, double *x, double v);
// z = a x + b y (y may be null when b is a host zero); z may alias x or y
int vec_axpbyz(hipStream_t s, int64_t n, Coef a, const double *x, Coef b,
               const double *y, double *z);
int vec_axpbypcz(hipStream_t s, int64_t n, Coef a, const double *x, Coef b,
                 const double *y, Coef c, double *z);   // z = a x + b y + c z
int vec_scale_copy(hipStream_t s, int64_t n, Coef a, const double *x, double *y);
// partial dots of up to 2 pairs: partial[b*2+k] = sum x_k . y_k
int vec_dot_partial(hipStream_t s, int64_t n, const double *x0, const double *y0,
                    const double *x1, const double *y1, double *partial);
// out[k] = sum_b partial[b*stride + k], k < nk, one block, fixed order
int sum_partials(hipStream_t s, const double *partial, int nparts, int stride,
                 int nk, double *out, int op);
enum { SUM_PLAIN = 0, SUM_SQRT = 1 };
int vec_copy_f64_to_f32(hipStream_t s, int64_t n, const double *x, float *y);

// SpMV (spmv.hip)
int sell_build(hipStream_t s, MAT_ *A);
int sell_build_perm_free(hipStream_t s, int nrows, int bs, const int *d_rowptr,
                         const int *d_col, const double *d_val, Sell &out,
                         const std::vector<int> &h_rowptr);
// y = alpha A x + beta z (z may be y or another vector; beta = 0: z unused)
// ndot fused partial dots of y with u0 / u1 (nullptr = y itself)
int spmv_f64(hipStream_t s, const MAT_ *A, double alpha, const double *x,
             double beta, const double *z, double *y, int ndot,
             const double *u0, const double *u1, double *partial);
// number of partial-sum pairs a fused-dot SpMV of A writes (one per block;
// its partial buffer needs twice this many doubles)
int spmv_partial_blocks(const MAT_ *A);
int spmv_sell_f32(hipStream_t s, const Sell &S, int nrows, float alpha,
                  const float *x, float beta, const float *z, float *y);
int spmv_sell_f64(hipStream_t s, const Sell &S, int nrows, double alpha,
                  const double *x, double beta, const double *z, double *y);
// r = v - A(:, col 0 of each block) p  (bs = 3), in T
int spmv_col0_residual_f32(hipStream_t s, const MAT_ *A, const float *v,
                           const float *p, float *r);
int spmv_col0_residual_f64(hipStream_t s, const MAT_ *A, const double *v,
                           const double *p, double *r);
int ensure_sell_f32(hipStream_t s, Sell &S);
int ensure_col0_f32(hipStream_t s, MAT_ *A);

// ---------------------------------------------------------------------------
// ILU(0) / block ILU(0) factor in level-scheduled layout (ilu.hip)
// ---------------------------------------------------------------------------
// 7-point grid tiling: a tile is TJ x TK x-lines (one lane each) of a
// wavefront; S = nx + TJ + TK - 2 hyperplane steps per tile; order[t] =
// J | (K << 16) lists tiles by increasing J + K.
constexpr int GRID_QUEUES = 8;   // tile queues of the grid sweeps: one per XCD

struct GridTiles {
    int nx = 0, ny = 0, nz = 0;
    int TJ = 0, TK = 0, NJ = 0, NK = 0, ntiles = 0, S = 0;
    int NF = 0;                      // face cells per step: TK (j-face) + TJ (k-face)
    const int *order = nullptr;      // tile T -> J | K << 16, in J + K order
    const int *tidx = nullptr;       // J * NK + K -> tile T
    // tile queues: queue q holds the tiles with J % NQ == q in tile order
    // (qtiles[qoff[q] .. qoff[q + 1])); workgroup b serves queue b % NQ,
    // which the dispatcher places on XCD b % 8
    int NQ = 0, qmax = 0;            // queue count, longest queue
    const int *qtiles = nullptr;
    const int *qoff = nullptr;
};

struct IluFactor {
    int bs = 1, nb = 0;
    // timer names of this factor's sweeps: nullptr = the per-kind names of
    // sweep_timer_name; a subdomain factor reports under its own names
    const char *timer_fwd = nullptr, *timer_bwd = nullptr;
    // grid tiling: tile column J is served by queue (J + qrot) % GRID_QUEUES
    // (workgroups b with b % GRID_QUEUES == queue, i.e. one XCD); several
    // grids in one launch rotate their queues to spread over the XCDs
    int qrot = 0;
    int prec = KRY_PREC_F64;
    int nlev_f = 0, nlev_b = 0;
    Sell L;                 // forward order, strictly lower blocks
    Sell U;                 // backward order, strictly upper blocks
    DBuf<double> dinv;      // U_ii^-1 in U slice layout
    DBuf<float> dinvf;
    DBuf<double> y64;       // forward result (sentinel between sweeps)
    DBuf<float> y32;
    DBuf<int> ctr;          // level sweeps: [0] forward, [1] backward slice counters;
                            // grid sweeps: GRID_QUEUES forward, then backward tile counters
    int grid_waves = 0;     // waves launched per sweep
    // grid-tiled sweeps (7-point stencils in natural order)
    bool grid = false;
    GridTiles G;
    DBuf<int> order, tidx, qtiles, qoff;
    DBuf<double> lt64, ut64, dt64;
    DBuf<float> lt32, ut32, dt32;
    DBuf<uint16_t> lt16, ut16;
    // tile-step-major forward result (overwritten in place by the backward
    // result) and the published face values of both sweeps, in the
    // compute precision
    DBuf<double> yt64, ff64, fb64;
    DBuf<float> yt32, ff32, fb32;
};

// timer name of one sweep kernel: direction, block size, factor storage
// bytes (8, 4, 2) and fused epilogue (add_mode of ilu_apply); each
// distinct kernel instantiation family gets its own name
const char *sweep_timer_name(bool fwd, int bs, int factor_bytes, int add_mode);

// grid-tiled layout and sweeps (ilu_grid.hip)
int ilu_grid_setup(hipStream_t s, const MAT_ *A, const double *lu, const double *uinv,
                   IluFactor &F);
// numeric factorization straight into the grid layout (7-point stencils in
// natural order with nx, ny >= 3, where ILU(0) only changes diagonal blocks)
bool ilu_grid_can_factor(const MAT_ *A);
int ilu_grid_factor_setup(hipStream_t s, const MAT_ *A, const double *d_val, IluFactor &F,
                          int *d_err);
int ilu_grid_apply(hipStream_t s, IluFactor &F, const void *b, int in_type, void *xscr,
                   int out_type, int add_mode, const void *add_in, void *add_out, int *d_err);

// factor A (FP64), pack for prec; err = device int flag; layout one of
// KRY_SWEEP_AUTO / KRY_SWEEP_LEVELS / KRY_SWEEP_GRID
int ilu_setup(hipStream_t s, const MAT_ *A, const double *d_val, IluFactor &F,
              int prec, int *d_err, int layout = KRY_SWEEP_AUTO);
// x = (LU)^-1 b.  in/out element types: 0 = double, 1 = float.
// add_mode 0: out = x; 1: add_out = add_in + x (full vector, out type);
// 2: add_out[i*bs + r] = (r == 0 ? add_in[i] : 0) + x (pressure injection)
// xscr: output of the solve itself (dependency source); when add_mode == 0
// it is the result.
int ilu_apply(hipStream_t s, IluFactor &F, const void *b, int in_type,
              void *xscr, int out_type, int add_mode, const void *add_in,
              void *add_out, int *d_err);

// ---------------------------------------------------------------------------
// CPR two-stage preconditioner (cpr.hip)
// ---------------------------------------------------------------------------
// Classical AMG (Algorithms 3 and 4); Figure 34's defaults, the hybrid
// Gauss-Seidel smoother on chunks of gs_chunk rows.
struct AmgOpts {
    double strength = 0.5, max_row_sum = 0.9, trunc = 1e-2;
    int max_levels = 8, num_sweeps = 2, gs_chunk = 4, coarse_size = 9;
};
// host vectors whose resize leaves new elements uninitialised, so that the
// threads that fill them are the first to touch their pages
template <typename T>
struct NoInitAlloc : std::allocator<T> {
    template <typename U>
    struct rebind {
        using other = NoInitAlloc<U>;
    };
    NoInitAlloc() = default;
    template <typename U>
    NoInitAlloc(const NoInitAlloc<U> &) noexcept {}
    template <typename U>
    void construct(U *p) noexcept {
        ::new (static_cast<void *>(p)) U;
    }
    template <typename U, typename... A>
    void construct(U *p, A &&...a) {
        ::new (static_cast<void *>(p)) U(std::forward<A>(a)...);
    }
};
template <typename T>
using HVec = std::vector<T, NoInitAlloc<T>>;
struct AmgCsr {                 // host CSR, n rows, m columns
    int n = 0, m = 0;
    HVec<int> rp, ci;
    HVec<double> v;
};
struct AmgLevelHost {           // A_l, its C/F splitting and P_l (not on the coarsest)
    AmgCsr A;
    std::vector<int> cf;
    AmgCsr P;
};
struct AmgLevel {
    int n = 0, nc = 0, nch = 0, team = 1;
    int64_t ell_bytes = 0;
    DBuf<int64_t> goff;         // chunk-interleaved rows of A_l, per wavefront group
    DBuf<int> gk, rlen, ecol;
    DBuf<double> eval, low;     // low: each chunk's diagonal and lower block
    DBuf<int> prp, pci, rrp, rci;   // P_l and R_l = P_l^T
    DBuf<double> pv, rv;
    DBuf<double> x, t, r, b;
};
struct AmgPC {
    AmgOpts o;
    std::vector<AmgLevelHost> host;
    std::vector<std::unique_ptr<AmgLevel>> lev;
    DBuf<double> cinv;          // inverse of the coarsest matrix, row-major
};
// hierarchy of the n x n CSR matrix (host pattern, device values)
int amg_setup(hipStream_t s, int n, const int *h_rowptr, const int *h_col, const double *d_val,
              const AmgOpts &o, AmgPC &M, int *d_err);
// x = one V-cycle applied to b (device vectors of n, distinct)
int amg_apply(hipStream_t s, AmgPC &M, const double *b, double *x, int *d_err);

struct RasPC;
struct CprPC {
    int variant = KRY_CPR_PF, sweeps = 4, prec = KRY_PREC_F64;
    int nb = 0;
    DBuf<double> w;         // quasi-IMPES weights nb*3
    MAT_ app;               // pressure matrix (CSR, pattern of A's blocks)
    IluFactor ilu_p;        // ILU(0) of A_pp
    IluFactor ilu_a;        // block ILU(0) of A
    std::unique_ptr<AmgPC> amg;   // pressure stage: one V-cycle instead of ILU(0) sweeps
    AmgOpts amg_opts;
    std::unique_ptr<RasPC> ras;   // full-system stage: RAS instead of block ILU(0)
    int ras_box[4] = {1, 1, 4, 1};   // px, py, pz, overlap
    bool ras_reuse = false;          // ras holds this matrix's subdomains: refactor only
    DBuf<char> work;        // scratch vectors
};
// One grid of a multi-grid sweep launch (the subdomains of RAS, boxes of a
// larger grid): its tiling, FP64 factor planes and work buffers, its tile
// counters (GRID_QUEUES forward, then backward), where its cells sit in the
// caller's vectors (offset of cell (0,0,0) in doubles, strides of j and k in
// cells), the cells it writes back (local i, j, k ranges) and its first
// workgroup in the sweep and untile launches.
struct GridMulti {
    GridTiles G;
    const double *lt, *ut, *dt;
    double *yt, *ff, *fb;
    int *ctr;
    int64_t boff, vsJ, vsK;
    int oi0, oi1, oj0, oj1, ok0, ok1;
    int wg0, ub0;
};
int grid_multi_launch_size(const IluFactor &F, int *wgs, int *untile_blocks);
// own = {i0, i1, j0, j1, k0, k1}: the cells written back, local coordinates
int grid_multi_desc(const IluFactor &F, int64_t boff, int64_t vsJ, int64_t vsK, const int own[6],
                    int wg0, int ub0, GridMulti &d);
// every grid's forward sweep of its cells of v, backward sweep, and untile
// of its owned cells into z, in three launches on s
int grid_multi_apply(hipStream_t s, int bs, const GridMulti *d_desc, int ngrid, int total_wgs,
                     int total_untile, const double *v, double *z, int *err);

// One grid of a multi-grid factor launch: its tiling, matrix, FP64 planes,
// face buffer and tile counter, and its first workgroup.
struct FactorMulti {
    GridTiles G;
    const int *rowptr;
    const double *val;
    double *lt, *ut, *dt, *faces;
    int *ctr;
    int wg0;
};
int grid_factor_prepare(hipStream_t s, const MAT_ *A, IluFactor &F, DBuf<double> &faces,
                        DBuf<int> &fctr);
int grid_factor_rearm(hipStream_t s, IluFactor &F, DBuf<double> &faces, DBuf<int> &fctr);
int grid_factor_desc(const MAT_ *A, const IluFactor &F, DBuf<double> &faces, DBuf<int> &fctr,
                     int wg0, FactorMulti &d, int *wgs);
int grid_factor_multi(hipStream_t s, int bs, const FactorMulti *d_desc, int ngrid, int total_wgs,
                      int *err);

// matrix from device-resident block CSR arrays (pattern validated and grid
// detected as for MatCreate*)
MAT *mat_create_device(MAP *map, int nb, int bs, const int *rowptr, const int *col,
                       const double *val);

// restricted additive Schwarz: z-slab subdomains of a 7-point grid matrix,
// block ILU(0) on each overlapped slab
struct RasSub {
    int lo = 0, hi = 0, o0 = 0, o1 = 0;   // z-slabs: overlapped / owned block rows
    int ob[6] = {0, 0, 0, 0, 0, 0};       // owned box: i0, i1, j0, j1, k0, k1
    int gb[6] = {0, 0, 0, 0, 0, 0};       // overlapped box (grown by `overlap`)
    MAP *map = nullptr;
    MAT *A = nullptr;
    IluFactor F;
    DBuf<int> pos;                        // A's value blocks of the subdomain matrix
    DBuf<double> faces;                   // grid factorization work buffers
    DBuf<int> fctr;
    DBuf<double> x;                       // local solution (level-scheduled slabs)
};
struct RasPC {
    int px = 1, py = 1, pz = 1, overlap = 1, bs = 1, layout = 0;
    const MAT_ *A = nullptr;              // the matrix whose pattern the subdomains hold
    std::vector<std::unique_ptr<RasSub>> subs;
    bool multi = false;                   // all subdomains grid-tiled: one launch per sweep
    DBuf<GridMulti> desc;
    DBuf<FactorMulti> fdesc;
    int wgs = 0, untile_blocks = 0, factor_wgs = 0;
    ~RasPC();
};
int ras_setup(hipStream_t s, MAT_ *A, RasPC &R, int px, int py, int pz, int overlap, int prec,
              int *d_err, int layout);
int ras_refactor(hipStream_t s, const MAT_ *A, RasPC &R, int *d_err);
int ras_apply(hipStream_t s, RasPC &R, const double *v, double *z, int *d_err);

int cpr_setup(hipStream_t s, MAT_ *A, CprPC &C, int variant, int sweeps,
              int prec, int *d_err, int layout);
int cpr_apply(hipStream_t s, MAT_ *A, CprPC &C, const double *v, double *z,
              int *d_err);

}  // namespace kry

// ---------------------------------------------------------------------------
// solver object
// ---------------------------------------------------------------------------
namespace kry {
// learned preconditioner stage (learned.hip)
struct LearnedStage;
void learned_stage_delete(LearnedStage *L);
struct LearnedStageDeleter {
    void operator()(LearnedStage *L) const { learned_stage_delete(L); }
};
int learned_stage_create(hipStream_t s, const MAT_ *A, const float *params_host,
                         const float *lnk, int lnk_where, LearnedStage **out);
// z holds the base preconditioner's result on entry, the stage's on exit
int learned_stage_apply(hipStream_t s, const MAT_ *A, LearnedStage &L, const double *v, double *z);
int learned_stage_stats(hipStream_t s, LearnedStage &L, int64_t *applies, int64_t *fallbacks);
int learned_read_file(const char *path, std::vector<float> &p, std::vector<float> &m,
                      std::vector<float> &v, int &adam_t);
}  // namespace kry

struct SOLVER_ {
    int type = KRY_GMRES, pc_type = KRY_PC_NONE;
    MAP *map = nullptr;
    MAT_ *A = nullptr;
    double rtol = 1e-6, atol = 0.0, btol = 0.0;
    int64_t maxit = 500, augk = 0;
    int restart = 30;
    int prec = KRY_PREC_F64;
    int cpr_variant = KRY_CPR_PF, cpr_sweeps = 4;
    int cpr_psolver = KRY_CPR_P_ILU0, cpr_full = KRY_CPR_F_BILU0;
    kry::AmgOpts amg_opts;
    std::unique_ptr<kry::AmgPC> amg;
    int sweep_layout = KRY_SWEEP_AUTO;
    int ortho = KRY_ORTHO_AUTO;
    hipStream_t stream = nullptr;
    PC_SETUP csetup = nullptr;
    PC_SOLVE csolve = nullptr;
    PC_DESTROY cdestroy = nullptr;
    void *cdata = nullptr;
    std::unique_ptr<kry::IluFactor> ilu;
    std::unique_ptr<kry::CprPC> cpr;
    std::unique_ptr<kry::RasPC> ras;
    int ras_px = 1, ras_py = 1, ras_pz = 4, ras_overlap = 1;
    std::unique_ptr<kry::LearnedStage, kry::LearnedStageDeleter> learned;
    std::vector<float> learned_params;     // host copy until assembly
    kry::DBuf<float> learned_lnk;          // ln k per cell
    bool assembled = false;
    double residual = 0.0;
    int nits = 0;
    double t_setup = 0.0, t_solve = 0.0;
    std::vector<double> hist;
    kry::DBuf<int> err;          // device error flag
    // Krylov workspace
    int64_t ldv = 0;
    kry::DBuf<double> V, Z, wrk, H, small, partial;
    kry::DBuf<double> AUG;       // LGMRES: stored corrections (aug_k columns)
    double *h_pinned = nullptr;  // host-visible readback slots
    hipEvent_t step_ev[2] = {nullptr, nullptr};   // Arnoldi steps' read-backs (slots 8, 16)
};

namespace kry {
int pc_apply(SOLVER_ *S, const double *v, double *z);
int check_device_error(SOLVER_ *S);
}  // namespace kry
