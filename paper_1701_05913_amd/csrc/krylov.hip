// Krylov solvers and the SOLVER object (Section 3, Figures 22-28;
// preconditioner interface of Figure 29).
//
// GMRES(m) follows Algorithm 1 with right preconditioning (the Arnoldi
// estimate is then the true unpreconditioned residual); FGMRES keeps
// Z = [M^-1 v_1 ... M^-1 v_m] so the preconditioner may vary (mixed
// precision, learned stage).  BiCGSTAB is van der Vorst's method, which the
// paper names without printing.
//
// gfx950 design: the Gram-Schmidt of Algorithm 1's Arnoldi step (modified,
// j dependent dot products per step) becomes classical Gram-Schmidt with
// one reorthogonalization (CGS2): two passes of h = V^T w, w -= V h, each a
// tall-skinny GEMV that streams V once.  The second pass also sums ||w||^2,
// so h_{j+1,j} = sqrt(||w||^2 - ||h2||^2) is known before the last update,
// which writes the normalized next basis vector.  When ||h2||^2 is not small
// against ||w||^2 (w nearly in span V, close to a lucky breakdown) that
// difference cancels; the last update then writes w - V h2 unscaled with
// its norm taken explicitly, and a follow-up kernel scales it.  All scalars (Hessenberg column,
// Givens rotations, residual estimate) stay in device memory; the host
// reads back one estimate per step, which is the only per-step sync.
// GMRES with a fixed preconditioner takes the lagged form of CGS2 instead
// (two passes over V per step; see its kernels below).
// Reductions use fixed grids and fixed summation order, so two runs give
// bitwise identical iterates.
#include <cfloat>
#include <chrono>
#include <cmath>

#include "device.hpp"
#include "internal.hpp"

namespace kry {

constexpr int MAXCOL = 64;   // restart length limit (columns of V)
constexpr int DCGS_MAXM = 31; // longest restart of the lagged Gram-Schmidt
static_assert(DCGS_MAXM < 64, "the lagged finish holds one column entry per lane of a wavefront");
static_assert(2 * (DCGS_MAXM + 1) <= MAXCOL, "pass A's sums of a block fit one partial row");

// slots of the small scalar area
enum {
    SC_BETA = 0, SC_INVBETA, SC_HN, SC_INVHN, SC_EST, SC_BREAK,
    SC_RHO, SC_RHO0, SC_ALPHA, SC_OMEGA, SC_BETAB, SC_RV, SC_TT, SC_TS,
    SC_SNORM, SC_RNORM, SC_FLAGS, SC_RHN, SC_NONE, SC_RENORM, SC_WN2,
    SC_ETA, SC_CU, SC_HH, SC_GSAVE, SC_COUNT = 32
};

// H holds the rotated columns (R); the lagged Gram-Schmidt also keeps the
// unrotated final columns (Hu), the provisional column (hp), the update
// coefficients of its second pass (sa, dv) and the sums of its first (ab)
struct SmallLayout {
    int m;
    size_t H, cs, sn, g, y, h1, h2, sc, Hu, hp, sa, dv, ab, total;
    explicit SmallLayout(int m_) : m(m_) {
        H = 0;
        cs = H + (size_t)(m + 1) * m;
        sn = cs + m;
        g = sn + m;
        y = g + (m + 1);
        h1 = y + m;
        h2 = h1 + MAXCOL;
        sc = h2 + MAXCOL;
        Hu = sc + SC_COUNT;
        hp = Hu + (size_t)(m + 1) * m;
        sa = hp + MAXCOL + 1;
        dv = sa + MAXCOL;
        ab = dv + MAXCOL + 1;
        total = ab + 2 * MAXCOL;
    }
};

// ---------------------------------------------------------------------------
// CGS2 kernels.  V is column-major with leading dimension ldv, a multiple of
// 64, so every column (and w, itself a column of V) is 512-byte aligned.
// Each pass writes one partial per workgroup; a one-block kernel sums them
// in block order.  (A last-arriving-block reduction inside the pass would
// need an agent-scope release per block, which writes back and invalidates
// the non-coherent L2 of every XCD, evicting V: slower than a launch.)
// ---------------------------------------------------------------------------
constexpr int CGS_ROWS = 4;      // rows per thread in passes 1 and 3: two 16-byte loads per column
constexpr int CGS_CH = 256;      // rows per LDS tile in pass 2
constexpr int CGS_MAXBLK = 1024; // largest grid of a pass (partials per column)

// Lane l ends with the wavefront total of column l >> (6 - log2 MAXC): each
// butterfly step hands half of the remaining columns to the partner lane,
// so MAXC columns cost MAXC - 1 + (6 - log2 MAXC) shuffles.
template <int MAXC>
__device__ __forceinline__ double wave_transpose_sum(double (&acc)[MAXC]) {
    const int lane = threadIdx.x & 63;
    int off = 32;
#pragma unroll
    for (int half = MAXC / 2; half >= 1; half >>= 1, off >>= 1) {
        const bool upper = (lane & off) != 0;
#pragma unroll
        for (int c = 0; c < half; c++) {
            const double send = upper ? acc[c] : acc[c + half];
            const double keep = upper ? acc[c + half] : acc[c];
            acc[c] = keep + __shfl_xor(send, off, 64);
        }
    }
    double s = acc[0];
    for (; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    return s;
}

template <int MAXC>
constexpr int cgs_shift() {
    return MAXC == 64 ? 0 : MAXC == 32 ? 1 : MAXC == 16 ? 2 : 3;
}

// out[k] = block total of acc[k], k < nc (256 threads; lds >= 4 * MAXC)
template <int MAXC>
__device__ __forceinline__ void block_reduce_cols(double (&acc)[MAXC], int nc, double *lds,
                                                  double *out) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const double s = wave_transpose_sum<MAXC>(acc);
    constexpr int SH = cgs_shift<MAXC>();
    if ((l & ((1 << SH) - 1)) == 0) lds[w * MAXC + (l >> SH)] = s;
    __syncthreads();
    if (threadIdx.x < nc)
        out[threadIdx.x] = lds[threadIdx.x] + lds[MAXC + threadIdx.x] + lds[2 * MAXC + threadIdx.x] +
                           lds[3 * MAXC + threadIdx.x];
}

// out[k] = sum over blocks b of partial[b * MAXCOL + k], k < nc, in one
// block of NT threads: thread t takes column t % MAXC and the blocks
// b = t / MAXC (mod NT / MAXC), four independent loads in flight, then the
// groups are added in order (deterministic)
template <int MAXC, int NT>
__global__ __launch_bounds__(NT) void k_sum_cols(const double *__restrict__ partial, int nblocks,
                                                 int nc, double *__restrict__ out) {
    constexpr int G = NT / MAXC;
    __shared__ double lds[NT];
    const int k = threadIdx.x % MAXC, g = threadIdx.x / MAXC;
    double s = 0.0;
    if (k < nc) {
        int b = g;
        for (; b + 3 * G < nblocks; b += 4 * G) {
            const double a0 = partial[(size_t)b * MAXCOL + k];
            const double a1 = partial[(size_t)(b + G) * MAXCOL + k];
            const double a2 = partial[(size_t)(b + 2 * G) * MAXCOL + k];
            const double a3 = partial[(size_t)(b + 3 * G) * MAXCOL + k];
            s += a0;
            s += a1;
            s += a2;
            s += a3;
        }
        for (; b < nblocks; b += G) s += partial[(size_t)b * MAXCOL + k];
    }
    lds[threadIdx.x] = s;
    __syncthreads();
    if ((int)threadIdx.x < nc) {
        double r = 0.0;
#pragma unroll 8
        for (int q = 0; q < G; q++) r += lds[q * MAXC + threadIdx.x];
        out[threadIdx.x] = r;
    }
}

// pass 1: partials of V^T w
template <int MAXC>
__global__ __launch_bounds__(256) void k_cgs_dots(int n, const double *__restrict__ V, int64_t ldv,
                                                  int nc, const double *__restrict__ w,
                                                  double *__restrict__ partial) {
    __shared__ double lds[256];
    double acc[MAXC];
#pragma unroll
    for (int k = 0; k < MAXC; k++) acc[k] = 0.0;
    const int nq = n / CGS_ROWS;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
        const unsigned off = (unsigned)q * CGS_ROWS;
        const double2 w0 = *reinterpret_cast<const double2 *>(w + off);
        const double2 w1 = *reinterpret_cast<const double2 *>(w + off + 2);
#pragma unroll
        for (int k = 0; k < MAXC; k++)
            if (k < nc) {
                const double2 *col = reinterpret_cast<const double2 *>(V + k * ldv + off);
                const double2 a = col[0], b = col[1];
                acc[k] += a.x * w0.x + a.y * w0.y + b.x * w1.x + b.y * w1.y;
            }
    }
    // ragged tail (n not a multiple of CGS_ROWS)
    if (blockIdx.x == 0 && (int)threadIdx.x < n - nq * CGS_ROWS) {
        const int r = nq * CGS_ROWS + threadIdx.x;
        const double wr = w[r];
#pragma unroll
        for (int k = 0; k < MAXC; k++)
            if (k < nc) acc[k] += V[k * ldv + r] * wr;
    }
    block_reduce_cols<MAXC>(acc, nc, lds, partial + (size_t)blockIdx.x * MAXCOL);
}

// pass 2: w -= V h, then partials of V^T w.  A row's t is final only after all
// nc columns, so each block stages a tile of CGS_CH rows of V in LDS: the
// threads form t row by row, then every wavefront takes MAXC / 4 columns
// of the tile for the dot products.  The next tile's V is loaded into
// registers while the current tile's products run.  With UPD = false the
// same tiling serves pass 1 on many columns: t = w, nothing is written back
// and no norm is formed.
template <int MAXC, bool UPD = true>
__global__ __launch_bounds__(256) void k_cgs_update_dots(int n, const double *__restrict__ V,
                                                         int64_t ldv, int nc, const double *h,
                                                         double *__restrict__ w,
                                                         double *__restrict__ partial) {
    constexpr int CPW = MAXC / 4;
    __shared__ double tile[MAXC][CGS_CH];
    __shared__ double tl[CGS_CH];
    __shared__ double lds[256];
    __shared__ double hs[MAXC];
    __shared__ double nl[4];
    if (threadIdx.x < MAXC) hs[threadIdx.x] = UPD && (int)threadIdx.x < nc ? h[threadIdx.x] : 0.0;
    __syncthreads();
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double nacc = 0.0;   // ||w - V h||^2 of this thread's rows
    double acc[CPW];
#pragma unroll
    for (int c = 0; c < CPW; c++) acc[c] = 0.0;
    double pre[MAXC], wpre = 0.0;
    const int stride = gridDim.x * CGS_CH;
    auto load = [&](int b) {
        const int r = b + threadIdx.x;
        const bool ok = r < n;
        wpre = ok ? w[r] : 0.0;
#pragma unroll
        for (int k = 0; k < MAXC; k++)
            if (k < nc) pre[k] = ok ? V[k * ldv + r] : 0.0;
    };
    int base = blockIdx.x * CGS_CH;
    if (base < n) load(base);
    for (; base < n; base += stride) {
        double t = wpre;
#pragma unroll
        for (int k = 0; k < MAXC; k++)
            if (k < nc) {
                tile[k][threadIdx.x] = pre[k];
                if (UPD) t -= pre[k] * hs[k];
            }
        if (UPD) {
            if (base + (int)threadIdx.x < n) w[base + threadIdx.x] = t;
            nacc += t * t;   // rows past n carry t = 0
        }
        tl[threadIdx.x] = t;
        __syncthreads();
        if (base + stride < n) load(base + stride);
#pragma unroll
        for (int c = 0; c < CPW; c++) {
            const int k = wv * CPW + c;
            if (k < nc) {
#pragma unroll
                for (int q = 0; q < CGS_CH / 64; q++)
                    acc[c] += tile[k][lane + 64 * q] * tl[lane + 64 * q];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < CPW; c++) {
        const double s = wave_sum(acc[c]);
        if (lane == 0) lds[wv * CPW + c] = s;
    }
    if (UPD) {
        nacc = wave_sum(nacc);
        if (lane == 0) nl[wv] = nacc;
    }
    __syncthreads();
    if ((int)threadIdx.x < nc) partial[(size_t)blockIdx.x * MAXCOL + threadIdx.x] = lds[threadIdx.x];
    // column nc (free: nc <= MAXCOL - 1) holds the block's ||w||^2
    if (UPD && threadIdx.x == 0)
        partial[(size_t)blockIdx.x * MAXCOL + nc] = nl[0] + nl[1] + nl[2] + nl[3];
}

// pass 3: w = (w - V h) / h_{j+1,j}, the next basis vector (the scale
// 1/h_{j+1,j} is read from the step's scalars, 0 after a breakdown).  When
// the step's scalars ask for an explicit norm (renorm != 0, scale 1), each
// block also writes its partial of ||w - V h||^2 to partial[block * MAXCOL].
template <int MAXC>
__global__ __launch_bounds__(256) void k_cgs_update_scale(int n, const double *__restrict__ V,
                                                          int64_t ldv, int nc, const double *h,
                                                          const double *inv_hn,
                                                          const double *renorm,
                                                          double *__restrict__ w,
                                                          double *__restrict__ partial) {
    __shared__ double hs[MAXC];
    __shared__ double red[4];
    if (threadIdx.x < MAXC) hs[threadIdx.x] = (int)threadIdx.x < nc ? h[threadIdx.x] : 0.0;
    __syncthreads();
    const double sc = *inv_hn;
    const bool want_norm = *renorm != 0.0;
    double nacc = 0.0;
    const int nq = n / CGS_ROWS;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
        const unsigned off = (unsigned)q * CGS_ROWS;
        double2 t0 = *reinterpret_cast<const double2 *>(w + off);
        double2 t1 = *reinterpret_cast<const double2 *>(w + off + 2);
#pragma unroll
        for (int k = 0; k < MAXC; k++)
            if (k < nc) {
                const double2 *col = reinterpret_cast<const double2 *>(V + k * ldv + off);
                const double2 a = col[0], b = col[1];
                t0.x -= a.x * hs[k];
                t0.y -= a.y * hs[k];
                t1.x -= b.x * hs[k];
                t1.y -= b.y * hs[k];
            }
        if (want_norm) nacc += t0.x * t0.x + t0.y * t0.y + t1.x * t1.x + t1.y * t1.y;
        t0.x *= sc;
        t0.y *= sc;
        t1.x *= sc;
        t1.y *= sc;
        *reinterpret_cast<double2 *>(w + off) = t0;
        *reinterpret_cast<double2 *>(w + off + 2) = t1;
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < n - nq * CGS_ROWS) {
        const int r = nq * CGS_ROWS + threadIdx.x;
        double t = w[r];
#pragma unroll
        for (int k = 0; k < MAXC; k++)
            if (k < nc) t -= V[k * ldv + r] * hs[k];
        if (want_norm) nacc += t * t;
        w[r] = t * sc;
    }
    if (want_norm) {   // uniform across the grid
        nacc = block_sum<256>(nacc, red);
        if (threadIdx.x == 0) partial[(size_t)blockIdx.x * MAXCOL] = nacc;
    }
}

// Hessenberg column j from col[0..j] = h1 + h2 and h_{j+1,j} = hn: apply the
// previous Givens rotations, form rotation j, update g and the residual
// estimate |g_{j+1}| (one thread; cs, sn = the previous rotations, staged
// in LDS by the caller)
__device__ void arnoldi_column(double *small, const SmallLayout &L, int j, int m, double *col,
                               const double *cs, const double *sn, double hn) {
    double *H = small + L.H + (size_t)j * (m + 1), *g = small + L.g, *sc = small + L.sc;
    col[j + 1] = hn;
    sc[SC_HN] = hn;
    sc[SC_INVHN] = hn != 0.0 ? 1.0 / hn : 0.0;
    sc[SC_BREAK] = hn == 0.0 ? 1.0 : 0.0;
    for (int k = 0; k < j; k++) {
        const double t = cs[k] * col[k] + sn[k] * col[k + 1];
        col[k + 1] = -sn[k] * col[k] + cs[k] * col[k + 1];
        col[k] = t;
    }
    const double r = hypot(col[j], col[j + 1]);
    double c = 1.0, sv = 0.0;
    if (r != 0.0) {
        c = col[j] / r;
        sv = col[j + 1] / r;
    }
    small[L.cs + j] = c;
    small[L.sn + j] = sv;
    col[j] = r;
    col[j + 1] = 0.0;
    for (int k = 0; k <= j + 1; k++) H[k] = col[k];
    const double gj = g[j];
    g[j + 1] = -sv * gj;
    g[j] = c * gj;
    sc[SC_EST] = fabs(sv * gj);
}

// After pass 3 of a step that asked for an explicit norm: every block sums
// pass 3's partials in the same order (so all see the same h_{j+1,j}),
// scales its rows of w by 1/h_{j+1,j}, and block 0 finishes the Hessenberg
// column.  Such a step has ||w - V h1|| at the rounding level of the first
// projection, so what the second leaves is either a new direction, kept if
// its norm exceeds the rounding level 8 eps (j + 2) ||w|| of two
// projections, or rounding noise, taken as h_{j+1,j} = 0 (a lucky
// breakdown: w lies in span V).  Exits at once on the usual path.
__global__ __launch_bounds__(256) void k_cgs_renorm(int n, const double *__restrict__ partial,
                                                    int nblocks, double *__restrict__ w, int j,
                                                    int m, double *small, SmallLayout L) {
    __shared__ double red[4];
    __shared__ double hsh;
    __shared__ double col[MAXCOL + 1], cs[MAXCOL], sn[MAXCOL];
    if (small[L.sc + SC_RENORM] == 0.0) return;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += partial[(size_t)b * MAXCOL];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) {
        const double hn = sqrt(s);
        const double floor_ = 8.0 * DBL_EPSILON * (j + 2) * sqrt(small[L.sc + SC_WN2]);
        hsh = hn > floor_ ? hn : 0.0;
    }
    __syncthreads();
    const double hn = hsh;
    const double inv = hn != 0.0 ? 1.0 / hn : 0.0;
    for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) w[r] *= inv;
    if (blockIdx.x != 0) return;
    if ((int)threadIdx.x <= j) col[threadIdx.x] = small[L.h1 + threadIdx.x] + small[L.h2 + threadIdx.x];
    if ((int)threadIdx.x < j) {
        cs[threadIdx.x] = small[L.cs + threadIdx.x];
        sn[threadIdx.x] = small[L.sn + threadIdx.x];
    }
    __syncthreads();
    if (threadIdx.x == 0) arnoldi_column(small, L, j, m, col, cs, sn, hn);
}

// Finish Arnoldi step j in one block: h2 from pass 2's partials (columns
// 0..j, block sums in a fixed order, also stored for pass 3) and ||w||^2
// (column j + 1); column j of H = h1 + h2.  h_{j+1,j} = ||w - V h2|| is
// taken as sqrt(||w||^2 - ||h2||^2) (h2 = V^T w with V orthonormal, so the
// second correction removes exactly ||h2||^2) when ||h2||^2 <= ||w||^2 / 2,
// where the difference keeps all but a few bits; otherwise the step is
// marked for an explicit norm (pass 3 writes w - V h2 unscaled and
// k_cgs_renorm finishes the column).
template <int MAXC>
__global__ __launch_bounds__(1024) void k_arnoldi_finish(const double *__restrict__ partial,
                                                         int nblocks, int j, int m, double *small,
                                                         SmallLayout L) {
    constexpr int NT = 1024, G = NT / MAXC;
    __shared__ double lds[NT];
    __shared__ double red[NT / 64];
    __shared__ double col[MAXCOL + 1], h2s[MAXCOL], cs[MAXCOL], sn[MAXCOL];
    const int nc = j + 1;
    {
        const int k = threadIdx.x % MAXC, gq = threadIdx.x / MAXC;
        double a = 0.0;
        if (k < nc)
            for (int b = gq; b < nblocks; b += G) a += partial[(size_t)b * MAXCOL + k];
        lds[threadIdx.x] = a;
    }
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += NT) s += partial[(size_t)b * MAXCOL + nc];
    if ((int)threadIdx.x < j) {
        cs[threadIdx.x] = small[L.cs + threadIdx.x];
        sn[threadIdx.x] = small[L.sn + threadIdx.x];
    }
    __syncthreads();
    if ((int)threadIdx.x < nc) {
        double r = 0.0;
        for (int q = 0; q < G; q++) r += lds[q * MAXC + threadIdx.x];
        h2s[threadIdx.x] = r;
        small[L.h2 + threadIdx.x] = r;
        col[threadIdx.x] = small[L.h1 + threadIdx.x] + r;
    }
    s = block_sum<NT>(s, red);
    if (threadIdx.x != 0) return;
    double *sc = small + L.sc;
    double h2sq = 0.0;
    for (int k = 0; k <= j; k++) h2sq += h2s[k] * h2s[k];
    if (h2sq <= 0.5 * s) {
        sc[SC_RENORM] = 0.0;
        arnoldi_column(small, L, j, m, col, cs, sn, sqrt(s - h2sq));
    } else {
        // ||w||^2 = ||h1||^2 + ||w - V h1||^2 for the breakdown test
        double h1sq = 0.0;
        for (int k = 0; k <= j; k++) h1sq += small[L.h1 + k] * small[L.h1 + k];
        sc[SC_WN2] = h1sq + s;
        sc[SC_RENORM] = 1.0;
        sc[SC_INVHN] = 1.0;
    }
}

// ---------------------------------------------------------------------------
// Lagged CGS2 for GMRES with a fixed preconditioner (DCGS2 of Swirydowicz,
// Langou, Ananthan, Yang and Thomas, "Low synchronization Gram-Schmidt and
// GMRES algorithms", 2020): the second projection of a step's new vector is
// taken during the next step, in the same pass that projects that step's w,
// so an Arnoldi step streams V twice instead of three times.
//
// Entering step j, columns 0..j-1 of V are final and column j holds u, the
// once-projected vector of step j - 1 (norm eta, not normalized), with the
// provisional Hessenberg column hp (unrotated, rows 0..j-1; h_{j,j-1} =
// eta).  Column j + 1 holds w = A M^-1 u.
//  pass A  a_k = v_k . u and b_k = v_k . w (k < j), u . u and u . w;
//  finish  u / eta = V s + alpha v_j with s = a / eta and alpha^2 =
//          u.u / eta^2 - |s|^2, so column j - 1 of H becomes hp + eta s with
//          h_{j,j-1} = eta alpha (its rotation and g are final from here on).
//          With A M^-1 V = V H over the final columns, the w of v_j is
//          y = (w / eta - V H s) / alpha, and h_k = v_k . y follows from a,
//          b and H alone;
//  pass B  v_j = u / (eta alpha) - V s / alpha into column j and
//          u' = w / (eta alpha) - V d - v_j d_j, d = H s / alpha + h, into
//          column j + 1, row by row (v_j stays in registers), with |u'|^2;
//  norm    eta' = |u'| (0 at the rounding level of the projection: a lucky
//          breakdown); the provisional column h, h_{j+1,j} = eta' (which
//          differs from the final one only by the O(eps) second projection
//          the next step applies) is rotated into H with its Givens rotation,
//          g and the residual estimate, g_j saved for the next finish.
// A cycle's least-squares solve takes its last column in that provisional
// form, and its last basis vector u / eta (normalized, projected once).  A
// step whose alpha^2 keeps less than half of u.u / eta^2 (the
// once-projected vector mostly in span V, which the breakdown floor of the
// norm excludes) ends the cycle as a breakdown: every coefficient of the
// step is zero.
// ---------------------------------------------------------------------------

// pass A: partials of v_k . u and v_k . w for the nc = j + 1 columns
// k = 0..j of V (column j is u), in partial[b * MAXCOL + k] and
// partial[b * MAXCOL + nc + k]; the LDS tiling of pass 2 with u's rows
// staged beside w's
template <int MAXC>
__global__ __launch_bounds__(256) void k_dcgs_dots(int n, const double *__restrict__ V,
                                                   int64_t ldv, int nc,
                                                   const double *__restrict__ w,
                                                   double *__restrict__ partial) {
    constexpr int CPW = MAXC / 4;
    __shared__ double tile[MAXC][CGS_CH];
    __shared__ double tw[CGS_CH];
    __shared__ double lds[2 * MAXC];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ju = nc - 1;
    double au[CPW], aw[CPW];
#pragma unroll
    for (int c = 0; c < CPW; c++) au[c] = aw[c] = 0.0;
    double pre[MAXC], wpre = 0.0;
    const int stride = gridDim.x * CGS_CH;
    auto load = [&](int b) {
        const int r = b + threadIdx.x;
        const bool ok = r < n;
        wpre = ok ? w[r] : 0.0;
#pragma unroll
        for (int k = 0; k < MAXC; k++)
            if (k < nc) pre[k] = ok ? V[k * ldv + r] : 0.0;
    };
    int base = blockIdx.x * CGS_CH;
    if (base < n) load(base);
    for (; base < n; base += stride) {
#pragma unroll
        for (int k = 0; k < MAXC; k++)
            if (k < nc) tile[k][threadIdx.x] = pre[k];
        tw[threadIdx.x] = wpre;
        __syncthreads();
        if (base + stride < n) load(base + stride);
#pragma unroll
        for (int c = 0; c < CPW; c++) {
            const int k = wv * CPW + c;
            if (k < nc) {
#pragma unroll
                for (int q = 0; q < CGS_CH / 64; q++) {
                    const double x = tile[k][lane + 64 * q];
                    au[c] += x * tile[ju][lane + 64 * q];
                    aw[c] += x * tw[lane + 64 * q];
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < CPW; c++) {
        const double su = wave_sum(au[c]);
        const double sw = wave_sum(aw[c]);
        if (lane == 0) {
            lds[wv * CPW + c] = su;
            lds[MAXC + wv * CPW + c] = sw;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nc) {
        partial[(size_t)blockIdx.x * MAXCOL + threadIdx.x] = lds[threadIdx.x];
        partial[(size_t)blockIdx.x * MAXCOL + nc + threadIdx.x] = lds[MAXC + threadIdx.x];
    }
}

// pass B: column j = cu u - V sa and column j + 1 = cu w - V d - v_j d_j,
// with its partial |.|^2 in partial[b * MAXCOL]; sa over the j final
// columns, d over j + 1 values, cu = 1 / (eta alpha)
template <int MAXC>
__global__ __launch_bounds__(256) void k_dcgs_update(int n, double *V, int64_t ldv, int j,
                                                     const double *__restrict__ sa,
                                                     const double *__restrict__ dv,
                                                     const double *__restrict__ cu_p,
                                                     double *__restrict__ partial) {
    __shared__ double ss[MAXC], ds[MAXC];
    __shared__ double red[4];
    if (threadIdx.x < MAXC) {
        ss[threadIdx.x] = (int)threadIdx.x < j ? sa[threadIdx.x] : 0.0;
        ds[threadIdx.x] = (int)threadIdx.x <= j ? dv[threadIdx.x] : 0.0;
    }
    __syncthreads();
    const double cu = *cu_p, dj = ds[j];
    double *u = V + (int64_t)j * ldv;
    double *w = u + ldv;
    double nacc = 0.0;
    const int nq = n / CGS_ROWS;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
        const unsigned off = (unsigned)q * CGS_ROWS;
        double2 v0 = *reinterpret_cast<const double2 *>(u + off);
        double2 v1 = *reinterpret_cast<const double2 *>(u + off + 2);
        double2 t0 = *reinterpret_cast<const double2 *>(w + off);
        double2 t1 = *reinterpret_cast<const double2 *>(w + off + 2);
        v0.x *= cu;
        v0.y *= cu;
        v1.x *= cu;
        v1.y *= cu;
        t0.x *= cu;
        t0.y *= cu;
        t1.x *= cu;
        t1.y *= cu;
#pragma unroll
        for (int k = 0; k < MAXC; k++)
            if (k < j) {
                const double2 *col = reinterpret_cast<const double2 *>(V + k * ldv + off);
                const double2 a = col[0], b = col[1];
                v0.x -= a.x * ss[k];
                v0.y -= a.y * ss[k];
                v1.x -= b.x * ss[k];
                v1.y -= b.y * ss[k];
                t0.x -= a.x * ds[k];
                t0.y -= a.y * ds[k];
                t1.x -= b.x * ds[k];
                t1.y -= b.y * ds[k];
            }
        t0.x -= v0.x * dj;
        t0.y -= v0.y * dj;
        t1.x -= v1.x * dj;
        t1.y -= v1.y * dj;
        *reinterpret_cast<double2 *>(u + off) = v0;
        *reinterpret_cast<double2 *>(u + off + 2) = v1;
        *reinterpret_cast<double2 *>(w + off) = t0;
        *reinterpret_cast<double2 *>(w + off + 2) = t1;
        nacc += t0.x * t0.x + t0.y * t0.y + t1.x * t1.x + t1.y * t1.y;
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < n - nq * CGS_ROWS) {
        const int r = nq * CGS_ROWS + threadIdx.x;
        double v = u[r] * cu, t = w[r] * cu;
#pragma unroll
        for (int k = 0; k < MAXC; k++)
            if (k < j) {
                const double a = V[k * ldv + r];
                v -= a * ss[k];
                t -= a * ds[k];
            }
        t -= v * dj;
        u[r] = v;
        w[r] = t;
        nacc += t * t;
    }
    nacc = block_sum<256>(nacc, red);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * MAXCOL] = nacc;
}

// finish of step j (one wavefront) from pass A's sums ab = [a_0..a_j,
// b_0..b_j]: column j - 1 of H made final (unrotated into Hu, rotated into
// H, with its Givens rotation and g, replacing its provisional form), the
// coefficients sa, cu of v_j, the provisional column j (hp) and d of u'.
// Lane k holds the k-th entries (j <= 31 < 64); the rotations run on lane 0
// over LDS copies.
__global__ __launch_bounds__(64) void k_dcgs_finish(int j, int m, double *small, SmallLayout L) {
    __shared__ double col[MAXCOL + 1], cs[MAXCOL], sn[MAXCOL], sh[MAXCOL];
    const int k = threadIdx.x;
    double *sc = small + L.sc, *Hu = small + L.Hu, *hp = small + L.hp;
    const double *a = small + L.ab, *b = a + (j + 1);
    const double eta = sc[SC_ETA];
    const bool eok = eta > 0.0 && isfinite(eta);
    const double sk = eok && k < j ? a[k] / eta : 0.0;
    const double ss = wave_sum(sk * sk);
    const double sig = eok ? a[j] / (eta * eta) : 0.0;
    const double al2 = sig - ss;
    const bool ok = eok && isfinite(al2) && al2 > 0.5 * sig;
    const double al = ok ? sqrt(al2) : 0.0;
    const double s_k = ok ? sk : 0.0;
    if (k < j) {
        sh[k] = s_k;
        cs[k] = small[L.cs + k];
        sn[k] = small[L.sn + k];
    }
    if (j >= 1) {
        if (k < j) col[k] = hp[k] + (ok ? eta * s_k : 0.0);
        if (k == j) col[j] = ok ? eta * al : 0.0;
        __syncthreads();
        if (k <= j) Hu[(size_t)(j - 1) * (m + 1) + k] = col[k];
        __syncthreads();
        if (k == 0) {
            small[L.g + j - 1] = sc[SC_GSAVE];   // g_{j-1} before the provisional rotation
            arnoldi_column(small, L, j - 1, m, col, cs, sn, col[j]);
        }
    }
    __syncthreads();
    if (k == 0) sc[SC_CU] = ok ? 1.0 / (eta * al) : 0.0;
    if (k < j) small[L.sa + k] = ok ? s_k / al : 0.0;
    if (!ok) {
        if (k <= j) small[L.hp + k] = small[L.dv + k] = 0.0;
        if (k == 0) sc[SC_HH] = 0.0;
        return;
    }
    const double sb = wave_sum(k < j ? s_k * b[k] : 0.0);
    const double bwj = (b[j] / eta - sb) / al;   // v_j . w
    double h = 0.0;
    if (k <= j) {
        double hs = 0.0;   // (H s)_k over the final columns q >= k - 1
        for (int q = k > 0 ? k - 1 : 0; q < j; q++) hs += Hu[(size_t)q * (m + 1) + k] * sh[q];
        h = ((k < j ? b[k] : bwj) / eta - hs) / al;
        small[L.hp + k] = h;
        small[L.dv + k] = hs / al + h;
    }
    const double hh = wave_sum(h * h);
    if (k == 0) sc[SC_HH] = hh;
}

// norm of step j: eta' from pass B's partials (fixed order), then the
// provisional column j rotated into H (rotation j, g, residual estimate,
// h_{j+1,j} and its inverse in the step's scalars), g_j saved first
__global__ __launch_bounds__(256) void k_dcgs_norm(const double *__restrict__ partial, int nblocks,
                                                   int j, int m, double *small, SmallLayout L) {
    __shared__ double red[4];
    __shared__ double col[MAXCOL + 1], cs[MAXCOL], sn[MAXCOL];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += partial[(size_t)b * MAXCOL];
    if ((int)threadIdx.x <= j) col[threadIdx.x] = small[L.hp + threadIdx.x];
    if ((int)threadIdx.x < j) {
        cs[threadIdx.x] = small[L.cs + threadIdx.x];
        sn[threadIdx.x] = small[L.sn + threadIdx.x];
    }
    s = block_sum<256>(s, red);
    if (threadIdx.x != 0) return;
    double *sc = small + L.sc;
    double eta = sqrt(s);
    if (eta <= 8.0 * DBL_EPSILON * (j + 2) * sqrt(sc[SC_HH] + s)) eta = 0.0;
    sc[SC_ETA] = eta;
    sc[SC_GSAVE] = small[L.g + j];
    arnoldi_column(small, L, j, m, col, cs, sn, eta);
}

// g = beta e_1 and the first basis vector scale factor
__global__ void k_cycle_start(double *small, SmallLayout L) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double *g = small + L.g, *sc = small + L.sc;
    const double beta = sc[SC_BETA];
    for (int k = 0; k <= L.m; k++) g[k] = 0.0;
    g[0] = beta;
    sc[SC_INVBETA] = beta != 0.0 ? 1.0 / beta : 0.0;
    sc[SC_ETA] = 1.0;   // the lagged Gram-Schmidt's v_0 = r / beta
}

// R y = g(0:jend) by back substitution
__global__ void k_ls_solve(double *small, SmallLayout L, int jend) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int m = L.m;
    const double *H = small + L.H, *g = small + L.g;
    double *y = small + L.y;
    for (int i = jend - 1; i >= 0; i--) {
        double s = g[i];
        for (int k = i + 1; k < jend; k++) s -= H[(size_t)k * (m + 1) + i] * y[k];
        const double d = H[(size_t)i * (m + 1) + i];
        y[i] = d != 0.0 ? s / d : 0.0;
    }
}

// x = beta x + sum_k Z[k] y[k]
template <int MAXC>
__global__ __launch_bounds__(256) void k_gemvn_acc(int64_t n, const double *__restrict__ Z,
                                                   int64_t ldz, int nc, const double *__restrict__ y,
                                                   double beta, double *x) {
    __shared__ double ys[MAXC];
    if (threadIdx.x < nc) ys[threadIdx.x] = y[threadIdx.x];
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double t = beta != 0.0 ? beta * x[i] : 0.0;
#pragma unroll
        for (int k = 0; k < MAXC; k++)
            if (k < nc) t += Z[k * ldz + i] * ys[k];
        x[i] = t;
    }
}

// ---------------------------------------------------------------------------
// BiCGSTAB fused kernels (scalars in device memory)
// ---------------------------------------------------------------------------
// rho = <rhat, r>; breakdown test; beta = (rho / rho0)(alpha / omega)
__global__ void k_bicg_rho(const double *__restrict__ partial, int nblocks, double *sc) {
    __shared__ double lds[4];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += partial[(size_t)b * 2];
    s = block_sum<256>(s, lds);
    if (threadIdx.x != 0) return;
    const double rho = s;
    sc[SC_RHO] = rho;
    const bool brk = fabs(rho) < 1e-300 * sc[SC_RHN] * sc[SC_RNORM] || rho == 0.0;
    sc[SC_FLAGS] = brk ? 1.0 : 0.0;
    sc[SC_BETAB] = brk ? 0.0 : (rho / sc[SC_RHO0]) * (sc[SC_ALPHA] / sc[SC_OMEGA]);
}

// p = r + beta (p - omega v)
__global__ void k_bicg_p(int64_t n, const double *__restrict__ r, double *__restrict__ p,
                         const double *__restrict__ v, const double *__restrict__ sc) {
    const double beta = sc[SC_BETAB], omega = sc[SC_OMEGA];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

// alpha = rho / <rhat, v>
__global__ void k_bicg_alpha(const double *__restrict__ partial, int nblocks, double *sc) {
    __shared__ double lds[4];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += partial[(size_t)b * 2];
    s = block_sum<256>(s, lds);
    if (threadIdx.x != 0) return;
    sc[SC_RV] = s;
    const bool brk = s == 0.0 || !isfinite(s);
    if (brk) sc[SC_FLAGS] = 2.0;
    sc[SC_ALPHA] = brk ? 0.0 : sc[SC_RHO] / s;
}

// s = r - alpha v, partial ||s||^2
__global__ __launch_bounds__(256) void k_bicg_s(int64_t n, const double *__restrict__ r,
                                                const double *__restrict__ v,
                                                double *__restrict__ s_,
                                                const double *__restrict__ sc,
                                                double *__restrict__ partial) {
    __shared__ double lds[4];
    const double alpha = sc[SC_ALPHA];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double t = r[i] - alpha * v[i];
        s_[i] = t;
        acc += t * t;
    }
    acc = block_sum<256>(acc, lds);
    if (threadIdx.x == 0) partial[blockIdx.x * 2] = acc;
}

// omega = <t, s> / <t, t> from the SpMV's fused partials (tt, ts)
__global__ void k_bicg_omega(const double *__restrict__ partial, int nblocks, double *sc) {
    __shared__ double lds[4];
    double tt = 0.0, ts = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        tt += partial[(size_t)b * 2];
        ts += partial[(size_t)b * 2 + 1];
    }
    tt = block_sum<256>(tt, lds);
    ts = block_sum<256>(ts, lds);
    if (threadIdx.x != 0) return;
    sc[SC_TT] = tt;
    sc[SC_TS] = ts;
    sc[SC_OMEGA] = tt != 0.0 ? ts / tt : 0.0;
}

// x += alpha ph + omega sh; r = s - omega t; partial ||r||^2
__global__ __launch_bounds__(256) void k_bicg_update(int64_t n, double *__restrict__ x,
                                                     const double *__restrict__ ph,
                                                     const double *__restrict__ sh,
                                                     const double *__restrict__ s_,
                                                     const double *__restrict__ t,
                                                     double *__restrict__ r,
                                                     const double *__restrict__ sc,
                                                     double *__restrict__ partial) {
    __shared__ double lds[4];
    const double alpha = sc[SC_ALPHA], omega = sc[SC_OMEGA];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += alpha * ph[i] + omega * sh[i];
        const double ri = s_[i] - omega * t[i];
        r[i] = ri;
        acc += ri * ri;
    }
    acc = block_sum<256>(acc, lds);
    if (threadIdx.x == 0) partial[blockIdx.x * 2] = acc;
}

__global__ void k_bicg_restart_scalars(double *sc) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    sc[SC_RHO0] = 1.0;
    sc[SC_ALPHA] = 1.0;
    sc[SC_OMEGA] = 1.0;
    sc[SC_RHN] = sc[SC_BETA];
    sc[SC_RNORM] = sc[SC_BETA];
    sc[SC_FLAGS] = 0.0;
}

__global__ void k_bicg_next(double *sc) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    sc[SC_RHO0] = sc[SC_RHO];
}

// ---------------------------------------------------------------------------
// preconditioned CG (Algorithm 2): scalars in device memory
// ---------------------------------------------------------------------------
// rho = (r, z); beta = rho / rho_prev (unused on the first step)
__global__ void k_cg_rho(const double *__restrict__ partial, int nblocks, double *sc) {
    __shared__ double lds[4];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += partial[(size_t)b * 2];
    s = block_sum<256>(s, lds);
    if (threadIdx.x != 0) return;
    sc[SC_RHO] = s;
    sc[SC_BETAB] = s / sc[SC_RHO0];
    if (!isfinite(s)) sc[SC_FLAGS] = 1.0;
}

// p = z + beta p
__global__ void k_cg_p(int64_t n, const double *__restrict__ z, double *__restrict__ p,
                       const double *__restrict__ sc) {
    const double beta = sc[SC_BETAB];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z[i] + beta * p[i];
}

// alpha = rho / (p, A p) from the SpMV's fused partials; a curvature that is
// not positive (or not finite) flags a breakdown and zeroes alpha
__global__ void k_cg_alpha(const double *__restrict__ partial, int nblocks, double *sc) {
    __shared__ double lds[4];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += partial[(size_t)b * 2];
    s = block_sum<256>(s, lds);
    if (threadIdx.x != 0) return;
    sc[SC_RV] = s;
    const bool brk = !(s > 0.0) || !isfinite(s) || sc[SC_FLAGS] != 0.0;
    if (brk) sc[SC_FLAGS] = 1.0;
    sc[SC_ALPHA] = brk ? 0.0 : sc[SC_RHO] / s;
}

// x += alpha p; r -= alpha q; partial ||r||^2
__global__ __launch_bounds__(256) void k_cg_update(int64_t n, double *__restrict__ x,
                                                   double *__restrict__ r,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ q,
                                                   const double *__restrict__ sc,
                                                   double *__restrict__ partial) {
    __shared__ double lds[4];
    const double alpha = sc[SC_ALPHA];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc += ri * ri;
    }
    acc = block_sum<256>(acc, lds);
    if (threadIdx.x == 0) partial[blockIdx.x * 2] = acc;
}

__global__ void k_cg_start(double *sc) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    sc[SC_RHO0] = 1.0;
    sc[SC_FLAGS] = 0.0;
}

__global__ void k_zero_int(int *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
static int spmv_blocks(const MAT_ *A) { return spmv_partial_blocks(A); }

// Arnoldi columns per cycle: restart, plus aug_k correction steps (LGMRES)
static int total_cols(const SOLVER_ *S) { return S->restart + static_cast<int>(S->augk); }
static SmallLayout layout_of(const SOLVER_ *S) { return SmallLayout(total_cols(S)); }
// U = [M^-1 v_j ..., corrections] is stored whenever the directions are not
// M^-1 V (flexible preconditioning, or augmentation)
static bool stores_z(const SOLVER_ *S) { return S->type == KRY_FGMRES || S->augk > 0; }

static int ensure_workspace(SOLVER_ *S) {
    const int64_t n = (int64_t)S->A->nb * S->A->bs;
    const int64_t ldv = (n + 63) / 64 * 64;
    const int m = total_cols(S);
    SmallLayout L(m);
    if (S->ldv == ldv && S->V.p && (int64_t)S->V.n >= (m + 1) * ldv &&
        (!stores_z(S) || (int64_t)S->Z.n >= m * ldv) &&
        (S->augk == 0 || (int64_t)S->AUG.n >= S->augk * ldv) && S->small.n >= L.total)
        return KRY_OK;
    S->ldv = ldv;
    KRY_TRY(S->V.alloc((size_t)(m + 1) * ldv));
    if (stores_z(S)) KRY_TRY(S->Z.alloc((size_t)m * ldv));
    if (S->augk > 0) KRY_TRY(S->AUG.alloc((size_t)S->augk * ldv));
    KRY_TRY(S->wrk.alloc((size_t)8 * ldv));
    KRY_TRY(S->small.alloc(L.total));
    const size_t np = std::max<size_t>({(size_t)RED_BLOCKS * MAXCOL, (size_t)CGS_MAXBLK * MAXCOL,
                                        (size_t)spmv_blocks(S->A) * 2});
    KRY_TRY(S->partial.alloc(np));
    if (!S->h_pinned) KRY_HIP(hipHostMalloc(reinterpret_cast<void **>(&S->h_pinned), 64 * sizeof(double)));
    for (auto &ev : S->step_ev)
        if (!ev) KRY_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    KRY_HIP(hipMemsetAsync(S->small.p, 0, S->small.bytes(), S->stream));
    return KRY_OK;
}

// read n scalars from device memory (synchronizes the solver stream)
static int readback(SOLVER_ *S, const double *d, int n, double *h) {
    KRY_HIP(hipMemcpyAsync(S->h_pinned, d, sizeof(double) * n, hipMemcpyDeviceToHost, S->stream));
    KRY_HIP(hipStreamSynchronize(S->stream));
    memcpy(h, S->h_pinned, sizeof(double) * n);
    return KRY_OK;
}

// grids of the three passes (measured at 64^3 x 3 unknowns, 8 to 30
// columns); pass 2 holds MAXC x 256 doubles of LDS per block
template <int MAXC>
static void launch_cgs(hipStream_t st, int n, const double *V, int64_t ldv, int nc, double *w,
                       double *small, SmallLayout L, double *partial, int j, int m) {
    const dim3 b(256);
    const int g2 = MAXC == 64 ? 256 : MAXC == 16 ? 1024 : 512;
    const int g1 = MAXC >= 32 ? g2 : 512;
    const int g3 = 512;
    static_assert(CGS_MAXBLK >= 1024, "partials sized for the largest grid");
    // pass 1: row-parallel dot products up to 16 columns, the LDS tiling of
    // pass 2 beyond
    if constexpr (MAXC >= 32)
        hipLaunchKernelGGL((k_cgs_update_dots<MAXC, false>), dim3(g1), b, 0, st, n, V, ldv, nc,
                           nullptr, w, partial);
    else
        hipLaunchKernelGGL(k_cgs_dots<MAXC>, dim3(g1), b, 0, st, n, V, ldv, nc, w, partial);
    hipLaunchKernelGGL((k_sum_cols<MAXC, 1024>), dim3(1), dim3(1024), 0, st, partial, g1, nc,
                       small + L.h1);
    hipLaunchKernelGGL(k_cgs_update_dots<MAXC>, dim3(g2), b, 0, st, n, V, ldv, nc, small + L.h1, w,
                       partial);
    hipLaunchKernelGGL(k_arnoldi_finish<MAXC>, dim3(1), dim3(1024), 0, st, partial, g2, j, m,
                       small, L);
    hipLaunchKernelGGL(k_cgs_update_scale<MAXC>, dim3(g3), b, 0, st, n, V, ldv, nc, small + L.h2,
                       small + L.sc + SC_INVHN, small + L.sc + SC_RENORM, w, partial);
    hipLaunchKernelGGL(k_cgs_renorm, dim3(256), b, 0, st, n, partial, g3, w, j, m, small, L);
}

static int cgs2_step(SOLVER_ *S, int j, double *w) {
    const int n = S->A->nb * S->A->bs;
    const int nc = j + 1;
    const SmallLayout L = layout_of(S);
    TimedScope ts("cgs2", S->stream);
    double *sm = S->small.p, *pt = S->partial.p;
    if (nc <= 8) launch_cgs<8>(S->stream, n, S->V.p, S->ldv, nc, w, sm, L, pt, j, L.m);
    else if (nc <= 16) launch_cgs<16>(S->stream, n, S->V.p, S->ldv, nc, w, sm, L, pt, j, L.m);
    else if (nc <= 32) launch_cgs<32>(S->stream, n, S->V.p, S->ldv, nc, w, sm, L, pt, j, L.m);
    else launch_cgs<64>(S->stream, n, S->V.p, S->ldv, nc, w, sm, L, pt, j, L.m);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

// one step of the lagged Gram-Schmidt
template <int MAXC>
static void launch_dcgs(hipStream_t st, int n, double *V, int64_t ldv, int j, double *small,
                        SmallLayout L, double *partial, int m) {
    const dim3 b(256);
    const int ga = MAXC == 16 ? 1024 : 512, gb = 512;
    static_assert(2 * MAXC <= MAXCOL, "pass A's sums of a block fit one partial row");
    const int nc = j + 1;
    double *u = V + (int64_t)j * ldv;
    hipLaunchKernelGGL(k_dcgs_dots<MAXC>, dim3(ga), b, 0, st, n, V, ldv, nc, u + ldv, partial);
    hipLaunchKernelGGL((k_sum_cols<2 * MAXC, 1024>), dim3(1), dim3(1024), 0, st, partial, ga,
                       2 * nc, small + L.ab);
    hipLaunchKernelGGL(k_dcgs_finish, dim3(1), dim3(64), 0, st, j, m, small, L);
    hipLaunchKernelGGL(k_dcgs_update<MAXC>, dim3(gb), b, 0, st, n, V, ldv, j,
                       small + L.sa, small + L.dv, small + L.sc + SC_CU, partial);
    hipLaunchKernelGGL(k_dcgs_norm, dim3(1), b, 0, st, partial, gb, j, m, small, L);
}

static int dcgs_step(SOLVER_ *S, int j) {
    const int n = S->A->nb * S->A->bs;
    const SmallLayout L = layout_of(S);
    TimedScope ts("dcgs2", S->stream);
    double *sm = S->small.p, *pt = S->partial.p;
    if (j + 1 <= 8) launch_dcgs<8>(S->stream, n, S->V.p, S->ldv, j, sm, L, pt, L.m);
    else if (j + 1 <= 16) launch_dcgs<16>(S->stream, n, S->V.p, S->ldv, j, sm, L, pt, L.m);
    else launch_dcgs<32>(S->stream, n, S->V.p, S->ldv, j, sm, L, pt, L.m);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

static int gemvn_acc(SOLVER_ *S, const double *Z, int nc, const double *y, double beta, double *x) {
    const int64_t n = (int64_t)S->A->nb * S->A->bs;
    const dim3 g(2048), b(256);
    if (nc <= 8) hipLaunchKernelGGL(k_gemvn_acc<8>, g, b, 0, S->stream, n, Z, S->ldv, nc, y, beta, x);
    else if (nc <= 16) hipLaunchKernelGGL(k_gemvn_acc<16>, g, b, 0, S->stream, n, Z, S->ldv, nc, y, beta, x);
    else if (nc <= 32) hipLaunchKernelGGL(k_gemvn_acc<32>, g, b, 0, S->stream, n, Z, S->ldv, nc, y, beta, x);
    else hipLaunchKernelGGL(k_gemvn_acc<64>, g, b, 0, S->stream, n, Z, S->ldv, nc, y, beta, x);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

// r = b - A x with ||r|| into sc[SC_BETA]; returns it on the host
static int true_residual(SOLVER_ *S, const double *b, const double *x, double *r, double *beta) {
    const SmallLayout L = layout_of(S);
    double *sc = S->small.p + L.sc;
    KRY_TRY(spmv_f64(S->stream, S->A, -1.0, x, 1.0, b, r, 1, nullptr, nullptr, S->partial.p));
    KRY_TRY(sum_partials(S->stream, S->partial.p, spmv_blocks(S->A), 2, 1, sc + SC_BETA, SUM_SQRT));
    return readback(S, sc + SC_BETA, 1, beta);
}

static double host_norm(SOLVER_ *S, const double *b) {
    const int64_t n = (int64_t)S->A->nb * S->A->bs;
    const SmallLayout L = layout_of(S);
    double *sc = S->small.p + L.sc;
    double v = NAN;
    if (vec_dot_partial(S->stream, n, b, b, nullptr, nullptr, S->partial.p) ||
        sum_partials(S->stream, S->partial.p, RED_BLOCKS, 2, 1, sc + SC_NONE, SUM_SQRT) ||
        readback(S, sc + SC_NONE, 1, &v))
        return NAN;
    return v;
}

}  // namespace kry

// ---------------------------------------------------------------------------
// preconditioner dispatch
// ---------------------------------------------------------------------------
namespace kry {

int pc_apply(SOLVER_ *S, const double *v, double *z) {
    const int64_t n = (int64_t)S->A->nb * S->A->bs;
    switch (S->pc_type) {
    case KRY_PC_NONE:
        KRY_HIP(hipMemcpyAsync(z, v, sizeof(double) * n, hipMemcpyDeviceToDevice, S->stream));
        return KRY_OK;
    case KRY_PC_ILU0:
        return ilu_apply(S->stream, *S->ilu, v, 0, z, 0, 0, nullptr, nullptr, S->err.p);
    case KRY_PC_CPR:
        return cpr_apply(S->stream, S->A, *S->cpr, v, z, S->err.p);
    case KRY_PC_BILU0_LEARNED:
        KRY_TRY(ilu_apply(S->stream, *S->ilu, v, 0, z, 0, 0, nullptr, nullptr, S->err.p));
        return learned_stage_apply(S->stream, S->A, *S->learned, v, z);
    case KRY_PC_CPR_LEARNED:
        KRY_TRY(cpr_apply(S->stream, S->A, *S->cpr, v, z, S->err.p));
        return learned_stage_apply(S->stream, S->A, *S->learned, v, z);
    case KRY_PC_RAS:
        return ras_apply(S->stream, *S->ras, v, z, S->err.p);
    case KRY_PC_AMG:
        return amg_apply(S->stream, *S->amg, v, z, S->err.p);
    case KRY_PC_CUSTOM: {
        VEC_ vv, zz;
        vv.map = zz.map = S->map;
        vv.n = zz.n = n;
        vv.data = const_cast<double *>(v);
        zz.data = z;
        const int rc = S->csolve(S->cdata, &zz, &vv);
        return rc < 0 ? set_error(rc, "custom preconditioner solve failed (%d)", rc) : KRY_OK;
    }
    default:
        return set_error(KRY_ERR_ARG, "unknown preconditioner type %d", S->pc_type);
    }
}

int check_device_error(SOLVER_ *S) {
    int e = 0;
    KRY_HIP(hipMemcpyAsync(&e, S->err.p, sizeof(int), hipMemcpyDeviceToHost, S->stream));
    KRY_HIP(hipStreamSynchronize(S->stream));
    if (e == 1) return set_error(KRY_ERR_ZERO_PIVOT, "singular pivot block in the factorization");
    if (e == ERR_STALL_FLAG)
        return set_error(KRY_ERR_STALL, "a level-scheduled sweep exceeded its wait bound");
    if (e != 0) return set_error(KRY_ERR_HIP, "device error flag %d", e);
    return KRY_OK;
}

// ---------------------------------------------------------------------------
// GMRES(m) / FGMRES(m)
// ---------------------------------------------------------------------------
// GMRES(m) / FGMRES(m) (Algorithm 1, right preconditioned), and LGMRES(m, k)
// when aug_k = k > 0 (Baker, Jessup & Manteuffel): every cycle adds one
// Arnoldi step per stored correction of the previous cycles (newest first,
// at most k, each normalized), with the correction itself as the direction;
// the cycle's correction U y becomes the newest stored one.
static int gmres_solve(SOLVER_ *S, const double *b, double *x) {
    const int64_t n = (int64_t)S->A->nb * S->A->bs;
    const int m = S->restart, k = static_cast<int>(S->augk);
    const bool flexible = stores_z(S);
    KRY_TRY(ensure_workspace(S));
    const SmallLayout L = layout_of(S);
    double *small = S->small.p, *sc = small + L.sc;
    double *ztmp = S->wrk.p, *utmp = S->wrk.p + S->ldv;
    const double bnorm = host_norm(S, b);
    if (!std::isfinite(bnorm)) return set_error(KRY_ERR_BREAKDOWN, "non-finite right-hand side");
    const double tol = std::max(S->rtol * bnorm, S->atol);
    int nits = 0;
    S->hist.clear();
    int status = KRY_NOT_CONVERGED;
    double relres = 0.0;
    int nstored = 0, head = 0;   // corrections: the i-th newest in AUG slot (head + i) % k
    // the next Arnoldi step may run ahead of the host's convergence test
    // unless the preconditioner calls back into host code or counts its uses
    const bool speculate = S->pc_type != KRY_PC_CUSTOM && S->pc_type != KRY_PC_BILU0_LEARNED &&
                           S->pc_type != KRY_PC_CPR_LEARNED;
    // the lagged Gram-Schmidt needs A M^-1 to be one linear operator over the
    // cycle: a fixed preconditioner, no stored Z, no augmentation
    const bool lagged = S->ortho != KRY_ORTHO_CGS2 && speculate && !flexible && k == 0 &&
                        m <= DCGS_MAXM;
    for (;;) {
        double beta = 0.0;
        KRY_TRY(true_residual(S, b, x, S->V.p, &beta));
        relres = bnorm > 0 ? beta / bnorm : beta;
        if (nits == 0) S->hist.push_back(beta);
        if (beta <= tol) { status = KRY_OK; break; }
        if (!std::isfinite(beta)) return set_error(KRY_ERR_BREAKDOWN, "non-finite residual");
        if (nits >= S->maxit) break;
        hipLaunchKernelGGL(k_cycle_start, dim3(1), dim3(64), 0, S->stream, small, L);
        KRY_TRY(vec_scale_copy(S->stream, n, dc(sc + SC_INVBETA), S->V.p, S->V.p));
        int jend = 0, last = -1;
        const int steps = m + nstored;
        // step j: z_j = M^-1 v_j (or the stored correction), w = A z_j, CGS2
        // against v_0..v_j with the Hessenberg column and Givens update and
        // w normalized in place into v_{j+1}, then
        // an asynchronous read-back of (h_{j+1,j}, 1/h_{j+1,j}, estimate) into
        // pinned slot j % 2 and an event.  When the preconditioner runs no
        // host code and keeps no counters, step j+1 is issued before step
        // j's estimate is read, so the GPU never waits for the host; if step
        // j ends the cycle, step j+1's results (column j+2 of V, column j+1
        // of H and its rotation) are never used: the least-squares solve
        // takes columns 0..j only.
        auto issue = [&](int j) -> int {
            double *vj = S->V.p + (size_t)j * S->ldv;
            double *zj = flexible ? S->Z.p + (size_t)j * S->ldv : ztmp;
            double *w = S->V.p + (size_t)(j + 1) * S->ldv;
            if (j < m)
                KRY_TRY(pc_apply(S, vj, zj));
            else
                KRY_HIP(hipMemcpyAsync(zj, S->AUG.p + (size_t)((head + j - m) % k) * S->ldv,
                                       sizeof(double) * n, hipMemcpyDeviceToDevice, S->stream));
            KRY_TRY(spmv_f64(S->stream, S->A, 1.0, zj, 0.0, nullptr, w, 0, nullptr, nullptr, nullptr));
            if (lagged) KRY_TRY(dcgs_step(S, j));
            else KRY_TRY(cgs2_step(S, j, w));
            last = j;
            KRY_HIP(hipMemcpyAsync(S->h_pinned + 8 + 8 * (j & 1), sc + SC_HN, 3 * sizeof(double),
                                   hipMemcpyDeviceToHost, S->stream));
            KRY_HIP(hipEventRecord(S->step_ev[j & 1], S->stream));
            return KRY_OK;
        };
        KRY_TRY(issue(0));
        for (int j = 0; j < steps; j++) {
            const bool ahead = speculate && j + 1 < steps;
            if (ahead) KRY_TRY(issue(j + 1));
            KRY_HIP(hipEventSynchronize(S->step_ev[j & 1]));
            const double hn = S->h_pinned[8 + 8 * (j & 1)];        // SC_HN
            const double est = S->h_pinned[8 + 8 * (j & 1) + 2];   // SC_EST
            nits++;
            jend = j + 1;
            S->hist.push_back(est);
            if (nits >= S->maxit) break;
            if (hn == 0.0) break;                         // lucky breakdown
            if (est <= tol) break;
            if (!ahead && j + 1 < steps) KRY_TRY(issue(j + 1));
        }
        // unless step jend was issued ahead, the lagged Gram-Schmidt left
        // column jend - 1 of H provisional (the least-squares solve takes it
        // as it is) and column jend of V once projected: normalize it
        if (lagged && last < jend) {
            double *vj = S->V.p + (size_t)jend * S->ldv;
            KRY_TRY(vec_scale_copy(S->stream, n, dc(sc + SC_INVHN), vj, vj));
        }
        hipLaunchKernelGGL(k_ls_solve, dim3(1), dim3(64), 0, S->stream, small, L, jend);
        if (k > 0) {
            // dx = U y; x += dx; dx / ||dx|| becomes the newest correction
            KRY_TRY(gemvn_acc(S, S->Z.p, jend, small + L.y, 0.0, utmp));
            KRY_TRY(vec_axpbyz(S->stream, n, hc(1.0), utmp, hc(1.0), x, x));
            const double dn = host_norm(S, utmp);
            if (dn > 0.0 && std::isfinite(dn)) {
                head = (head + k - 1) % k;
                KRY_TRY(vec_scale_copy(S->stream, n, hc(1.0 / dn), utmp,
                                       S->AUG.p + (size_t)head * S->ldv));
                nstored = std::min(nstored + 1, k);
            }
        } else if (flexible) {
            KRY_TRY(gemvn_acc(S, S->Z.p, jend, small + L.y, 1.0, x));
        } else {
            KRY_TRY(gemvn_acc(S, S->V.p, jend, small + L.y, 0.0, utmp));
            KRY_TRY(pc_apply(S, utmp, ztmp));
            KRY_TRY(vec_axpbyz(S->stream, n, hc(1.0), ztmp, hc(1.0), x, x));
        }
    }
    S->nits = nits;
    S->residual = relres;
    return status;
}

// ---------------------------------------------------------------------------
// BiCGSTAB
// ---------------------------------------------------------------------------
static int bicgstab_solve(SOLVER_ *S, const double *b, double *x) {
    const int64_t n = (int64_t)S->A->nb * S->A->bs;
    KRY_TRY(ensure_workspace(S));
    const SmallLayout L = layout_of(S);
    double *sc = S->small.p + L.sc;
    const int64_t ld = S->ldv;
    double *r = S->wrk.p, *rh = r + ld, *p = rh + ld, *v = p + ld, *ph = v + ld;
    double *sv = ph + ld, *sh = sv + ld, *t = sh + ld;
    double *part = S->partial.p;
    const int nsb = spmv_blocks(S->A);
    const dim3 gv(2048), bv(256);
    const double bnorm = host_norm(S, b);
    if (!std::isfinite(bnorm)) return set_error(KRY_ERR_BREAKDOWN, "non-finite right-hand side");
    const double tol = std::max(S->rtol * bnorm, S->atol);
    int nits = 0, status = KRY_NOT_CONVERGED;
    double relres = 0.0;
    bool fresh = true;
    S->hist.clear();
    for (;;) {
        if (fresh) {
            double tn = 0.0;
            KRY_TRY(true_residual(S, b, x, r, &tn));
            relres = bnorm > 0 ? tn / bnorm : tn;
            if (nits == 0) S->hist.push_back(tn);
            if (tn <= tol) { status = KRY_OK; break; }
            if (!std::isfinite(tn)) return set_error(KRY_ERR_BREAKDOWN, "non-finite residual");
            KRY_HIP(hipMemcpyAsync(rh, r, sizeof(double) * n, hipMemcpyDeviceToDevice, S->stream));
            KRY_TRY(vec_fill(S->stream, n, v, 0.0));
            KRY_TRY(vec_fill(S->stream, n, p, 0.0));
            hipLaunchKernelGGL(k_bicg_restart_scalars, dim3(1), dim3(64), 0, S->stream, sc);
            fresh = false;
        }
        if (nits >= S->maxit) break;
        // rho, beta, p
        KRY_TRY(vec_dot_partial(S->stream, n, rh, r, nullptr, nullptr, part));
        hipLaunchKernelGGL(k_bicg_rho, dim3(1), dim3(256), 0, S->stream, part, RED_BLOCKS, sc);
        hipLaunchKernelGGL(k_bicg_p, gv, bv, 0, S->stream, n, r, p, v, sc);
        KRY_TRY(pc_apply(S, p, ph));
        KRY_TRY(spmv_f64(S->stream, S->A, 1.0, ph, 0.0, nullptr, v, 1, rh, nullptr, part));
        hipLaunchKernelGGL(k_bicg_alpha, dim3(1), dim3(256), 0, S->stream, part, nsb, sc);
        hipLaunchKernelGGL(k_bicg_s, dim3(RED_BLOCKS), bv, 0, S->stream, n, r, v, sv, sc, part);
        KRY_TRY(sum_partials(S->stream, part, RED_BLOCKS, 2, 1, sc + SC_SNORM, SUM_SQRT));
        double sdata[SC_RHN + 1];
        KRY_TRY(readback(S, sc, SC_RHN + 1, sdata));
        const int flags = static_cast<int>(sdata[SC_FLAGS]);
        if (flags == 1) { fresh = true; continue; }       // rho breakdown: not counted
        nits++;
        if (flags == 2) { fresh = true; continue; }       // <rhat, v> = 0
        const double snorm = sdata[SC_SNORM];
        if (snorm <= tol) {
            KRY_TRY(vec_axpbyz(S->stream, n, dc(sc + SC_ALPHA), ph, hc(1.0), x, x));
            S->hist.push_back(snorm);
            fresh = true;
            continue;
        }
        KRY_TRY(pc_apply(S, sv, sh));
        KRY_TRY(spmv_f64(S->stream, S->A, 1.0, sh, 0.0, nullptr, t, 2, nullptr, sv, part));
        hipLaunchKernelGGL(k_bicg_omega, dim3(1), dim3(256), 0, S->stream, part, nsb, sc);
        hipLaunchKernelGGL(k_bicg_update, dim3(RED_BLOCKS), bv, 0, S->stream, n, x, ph, sh, sv, t, r,
                           sc, part);
        KRY_TRY(sum_partials(S->stream, part, RED_BLOCKS, 2, 1, sc + SC_RNORM, SUM_SQRT));
        hipLaunchKernelGGL(k_bicg_next, dim3(1), dim3(64), 0, S->stream, sc);
        double rv[SC_RNORM + 1];
        KRY_TRY(readback(S, sc, SC_RNORM + 1, rv));
        const double rn = rv[SC_RNORM], omega = rv[SC_OMEGA];
        S->hist.push_back(rn);
        if (rn <= tol) { fresh = true; continue; }
        if (omega == 0.0 || !std::isfinite(rn)) { fresh = true; continue; }
    }
    S->nits = nits;
    S->residual = relres;
    return status;
}

// ---------------------------------------------------------------------------
// preconditioned CG, Algorithm 2: stops on the recursively updated ||r||,
// reports the true residual; negative curvature ends with KRY_ERR_BREAKDOWN
// ---------------------------------------------------------------------------
static int cg_solve(SOLVER_ *S, const double *b, double *x) {
    const int64_t n = (int64_t)S->A->nb * S->A->bs;
    KRY_TRY(ensure_workspace(S));
    const SmallLayout L = layout_of(S);
    double *sc = S->small.p + L.sc;
    const int64_t ld = S->ldv;
    double *r = S->wrk.p, *z = r + ld, *p = z + ld, *q = p + ld;
    double *part = S->partial.p;
    const int nsb = spmv_blocks(S->A);
    const dim3 gv(2048), bv(256);
    const double bnorm = host_norm(S, b);
    if (!std::isfinite(bnorm)) return set_error(KRY_ERR_BREAKDOWN, "non-finite right-hand side");
    const double tol = std::max(S->rtol * bnorm, S->atol);
    S->hist.clear();
    double rn = 0.0;
    KRY_TRY(true_residual(S, b, x, r, &rn));
    S->hist.push_back(rn);
    if (!std::isfinite(rn)) return set_error(KRY_ERR_BREAKDOWN, "non-finite residual");
    int nits = 0, status = rn <= tol ? KRY_OK : KRY_NOT_CONVERGED;
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(64), 0, S->stream, sc);
    while (status != KRY_OK && nits < S->maxit) {
        KRY_TRY(pc_apply(S, r, z));
        KRY_TRY(vec_dot_partial(S->stream, n, r, z, nullptr, nullptr, part));
        hipLaunchKernelGGL(k_cg_rho, dim3(1), dim3(256), 0, S->stream, part, RED_BLOCKS, sc);
        if (nits == 0)
            KRY_HIP(hipMemcpyAsync(p, z, sizeof(double) * n, hipMemcpyDeviceToDevice, S->stream));
        else
            hipLaunchKernelGGL(k_cg_p, gv, bv, 0, S->stream, n, z, p, sc);
        KRY_TRY(spmv_f64(S->stream, S->A, 1.0, p, 0.0, nullptr, q, 1, p, nullptr, part));
        hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(256), 0, S->stream, part, nsb, sc);
        hipLaunchKernelGGL(k_cg_update, dim3(RED_BLOCKS), bv, 0, S->stream, n, x, r, p, q, sc, part);
        KRY_TRY(sum_partials(S->stream, part, RED_BLOCKS, 2, 1, sc + SC_RNORM, SUM_SQRT));
        hipLaunchKernelGGL(k_bicg_next, dim3(1), dim3(64), 0, S->stream, sc);
        static_assert(SC_FLAGS > SC_RNORM, "one readback covers both slots");
        double v[SC_FLAGS + 1];
        KRY_TRY(readback(S, sc, SC_FLAGS + 1, v));
        if (v[SC_FLAGS] != 0.0) {
            status = set_error(KRY_ERR_BREAKDOWN, "CG: curvature (p, A p) not positive");
            break;
        }
        nits++;
        rn = v[SC_RNORM];
        S->hist.push_back(rn);
        if (rn <= tol) status = KRY_OK;
        else if (!std::isfinite(rn)) { status = set_error(KRY_ERR_BREAKDOWN, "CG: non-finite residual"); break; }
    }
    double tn = 0.0;
    KRY_TRY(true_residual(S, b, x, q, &tn));
    S->nits = nits;
    S->residual = bnorm > 0 ? tn / bnorm : tn;
    return status;
}

}  // namespace kry

using namespace kry;

// ===========================================================================
// C ABI: SOLVER
// ===========================================================================
static int64_t g_def_maxit = 500;
static double g_def_rtol = 1e-6, g_def_atol = 0.0, g_def_btol = 0.0;
static int64_t g_def_restart = 30, g_def_augk = 0;

extern "C" void SolverSetDefaultMaxit(int64_t it) { g_def_maxit = it; }
extern "C" void SolverSetDefaultRtol(double tol) { g_def_rtol = tol; }
extern "C" void SolverSetDefaultAtol(double tol) { g_def_atol = tol; }
extern "C" void SolverSetDefaultBtol(double tol) { g_def_btol = tol; }
extern "C" void SolverSetDefaultRestart(int64_t m) { g_def_restart = m; }
extern "C" void SolverSetDefaultAugk(int64_t k) { g_def_augk = k; }

extern "C" SOLVER *SolverCreate(int solver_type, int pc_type, MAP *map) {
    if (!map) { set_error(KRY_ERR_ARG, "SolverCreate: map is NULL"); return nullptr; }
    if (solver_type < KRY_GMRES || solver_type > KRY_CG) {
        set_error(KRY_ERR_UNSUPPORTED, "SolverCreate: solver type %d", solver_type);
        return nullptr;
    }
    if (pc_type < KRY_PC_NONE || pc_type > KRY_PC_AMG) {
        set_error(KRY_ERR_UNSUPPORTED, "SolverCreate: preconditioner type %d", pc_type);
        return nullptr;
    }
    SOLVER *s = new SOLVER_();
    s->type = solver_type;
    s->pc_type = pc_type;
    s->map = map;
    s->maxit = g_def_maxit;
    s->rtol = g_def_rtol;
    s->atol = g_def_atol;
    s->btol = g_def_btol;
    s->restart = static_cast<int>(std::min<int64_t>(std::max<int64_t>(g_def_restart, 1), MAXCOL - 1));
    s->augk = std::max<int64_t>(0, std::min<int64_t>(g_def_augk, MAXCOL - 1 - s->restart));
    return s;
}

extern "C" int SolverDestroy(SOLVER **sp) {
    if (!sp || !*sp) return KRY_OK;
    SOLVER *s = *sp;
    if (s->pc_type == KRY_PC_CUSTOM && s->cdestroy) s->cdestroy(s->cdata);
    if (s->h_pinned) (void)hipHostFree(s->h_pinned);
    for (auto &ev : s->step_ev)
        if (ev) (void)hipEventDestroy(ev);
    delete s;
    *sp = nullptr;
    return KRY_OK;
}

extern "C" int SolverSetMat(SOLVER *s, MAT *A) {
    if (!s || !A) return set_error(KRY_ERR_ARG, "SolverSetMat: NULL argument");
    if ((int64_t)A->nb * A->bs != s->map->nlocal) return set_error(KRY_ERR_DIM, "SolverSetMat: size mismatch");
    s->A = A;
    s->ras.reset();   // subdomain patterns belong to the previous matrix
    s->assembled = false;
    return KRY_OK;
}

extern "C" int SolverSetMaxit(SOLVER *s, int64_t it) {
    if (!s || it < 0) return set_error(KRY_ERR_ARG, "SolverSetMaxit: bad argument");
    s->maxit = it;
    return KRY_OK;
}
extern "C" int SolverSetRtol(SOLVER *s, double t) {
    if (!s || !(t >= 0)) return set_error(KRY_ERR_ARG, "SolverSetRtol: bad argument");
    s->rtol = t;
    return KRY_OK;
}
extern "C" int SolverSetAtol(SOLVER *s, double t) {
    if (!s || !(t >= 0)) return set_error(KRY_ERR_ARG, "SolverSetAtol: bad argument");
    s->atol = t;
    return KRY_OK;
}
extern "C" int SolverSetBtol(SOLVER *s, double t) {
    if (!s || !(t >= 0)) return set_error(KRY_ERR_ARG, "SolverSetBtol: bad argument");
    s->btol = t;
    return KRY_OK;
}
extern "C" int SolverSetRestart(SOLVER *s, int64_t m) {
    if (!s || m < 1 || m + s->augk > MAXCOL - 1)
        return set_error(KRY_ERR_ARG, "SolverSetRestart: need 1 <= m and m + aug_k <= %d", MAXCOL - 1);
    s->restart = static_cast<int>(m);
    s->ldv = 0;
    return KRY_OK;
}
extern "C" int SolverSetAugk(SOLVER *s, int64_t k) {
    if (!s) return set_error(KRY_ERR_ARG, "SolverSetAugk: NULL solver");
    if (k < 0 || s->restart + k > MAXCOL - 1)
        return set_error(KRY_ERR_ARG, "SolverSetAugk: need 0 <= k and restart + k <= %d", MAXCOL - 1);
    s->augk = k;
    s->ldv = 0;
    return KRY_OK;
}
extern "C" int SolverSetPrecision(SOLVER *s, int prec) {
    if (!s || prec < KRY_PREC_F64 || prec > KRY_PREC_BF16_FACTORS)
        return set_error(KRY_ERR_ARG, "SolverSetPrecision: bad argument");
    s->prec = prec;
    s->assembled = false;
    return KRY_OK;
}
extern "C" int SolverSetCPR(SOLVER *s, int variant, int p_sweeps) {
    if (!s || variant < KRY_CPR_PF || variant > KRY_CPR_FFPF || p_sweeps < 1)
        return set_error(KRY_ERR_ARG, "SolverSetCPR: bad argument");
    s->cpr_variant = variant;
    s->cpr_sweeps = p_sweeps;
    s->assembled = false;
    return KRY_OK;
}
extern "C" int SolverSetCPRPressure(SOLVER *s, int psolver) {
    if (!s || (psolver != KRY_CPR_P_ILU0 && psolver != KRY_CPR_P_AMG))
        return set_error(KRY_ERR_ARG, "SolverSetCPRPressure: bad argument");
    s->cpr_psolver = psolver;
    s->assembled = false;
    return KRY_OK;
}
extern "C" int SolverSetCPRFull(SOLVER *s, int fsolver) {
    if (!s || (fsolver != KRY_CPR_F_BILU0 && fsolver != KRY_CPR_F_RAS))
        return set_error(KRY_ERR_ARG, "SolverSetCPRFull: bad argument");
    s->cpr_full = fsolver;
    s->assembled = false;
    return KRY_OK;
}
extern "C" int SolverSetAMG(SOLVER *s, int max_levels, int num_sweeps, int gs_chunk) {
    if (!s || max_levels < 1 || num_sweeps < 1) return set_error(KRY_ERR_ARG, "SolverSetAMG: bad argument");
    s->amg_opts.max_levels = max_levels;
    s->amg_opts.num_sweeps = num_sweeps;
    s->amg_opts.gs_chunk = gs_chunk;
    s->assembled = false;
    return KRY_OK;
}
static const AmgPC *solver_amg(const SOLVER *s) {
    if (!s) return nullptr;
    if (s->amg) return s->amg.get();
    if (s->cpr && s->cpr->amg) return s->cpr->amg.get();
    return nullptr;
}
extern "C" int SolverGetAMGLevels(const SOLVER *s) {
    const AmgPC *M = solver_amg(s);
    if (!M) return set_error(KRY_ERR_ARG, "SolverGetAMGLevels: no AMG hierarchy assembled");
    return (int)M->host.size();
}
extern "C" int SolverGetAMGLevel(const SOLVER *s, int l, int *n, int *nnz, int *nc, int *pnnz,
                                 int *rowptr, int *col, double *val, int *cf, int *prowptr,
                                 int *pcol, double *pval) {
    const AmgPC *M = solver_amg(s);
    if (!M) return set_error(KRY_ERR_ARG, "SolverGetAMGLevel: no AMG hierarchy assembled");
    if (l < 0 || l >= (int)M->host.size()) return set_error(KRY_ERR_ARG, "SolverGetAMGLevel: no level %d", l);
    const AmgLevelHost &H = M->host[l];
    const bool coarsest = l == (int)M->host.size() - 1;
    if (n) *n = H.A.n;
    if (nnz) *nnz = (int)H.A.ci.size();
    if (nc) *nc = coarsest ? 0 : H.P.m;
    if (pnnz) *pnnz = coarsest ? 0 : (int)H.P.ci.size();
    if (rowptr) std::copy(H.A.rp.begin(), H.A.rp.end(), rowptr);
    if (col) std::copy(H.A.ci.begin(), H.A.ci.end(), col);
    if (val) std::copy(H.A.v.begin(), H.A.v.end(), val);
    if (!coarsest) {
        if (cf) std::copy(H.cf.begin(), H.cf.end(), cf);
        if (prowptr) std::copy(H.P.rp.begin(), H.P.rp.end(), prowptr);
        if (pcol) std::copy(H.P.ci.begin(), H.P.ci.end(), pcol);
        if (pval) std::copy(H.P.v.begin(), H.P.v.end(), pval);
    }
    return KRY_OK;
}
extern "C" int SolverSetRASBoxes(SOLVER *s, int px, int py, int pz, int overlap) {
    if (!s || px < 1 || py < 1 || pz < 1 || overlap < 0)
        return set_error(KRY_ERR_ARG, "SolverSetRASBoxes: bad argument");
    s->ras_px = px;
    s->ras_py = py;
    s->ras_pz = pz;
    s->ras_overlap = overlap;
    s->assembled = false;
    return KRY_OK;
}
extern "C" int SolverSetRAS(SOLVER *s, int nsub, int overlap) {
    if (!s || nsub < 1 || overlap < 0) return set_error(KRY_ERR_ARG, "SolverSetRAS: bad argument");
    return SolverSetRASBoxes(s, 1, 1, nsub, overlap);
}
extern "C" int SolverSetSweepLayout(SOLVER *s, int layout) {
    if (!s || layout < KRY_SWEEP_AUTO || layout > KRY_SWEEP_GRID)
        return set_error(KRY_ERR_ARG, "SolverSetSweepLayout: bad argument");
    s->sweep_layout = layout;
    s->assembled = false;
    return KRY_OK;
}

extern "C" int SolverSetOrthog(SOLVER *s, int kind) {
    if (!s || (kind != KRY_ORTHO_AUTO && kind != KRY_ORTHO_CGS2))
        return set_error(KRY_ERR_ARG, "SolverSetOrthog: bad argument");
    s->ortho = kind;
    return KRY_OK;
}

extern "C" int SolverSetStream(SOLVER *s, void *stream) {
    if (!s) return set_error(KRY_ERR_ARG, "SolverSetStream: NULL solver");
    s->stream = static_cast<hipStream_t>(stream);
    return KRY_OK;
}
extern "C" int SolverSetPC(SOLVER *s, PC_SETUP setup, PC_SOLVE solve, PC_DESTROY destroy, void *data) {
    if (!s || !solve) return set_error(KRY_ERR_ARG, "SolverSetPC: NULL solver or solve callback");
    if (s->pc_type != KRY_PC_CUSTOM) return set_error(KRY_ERR_ARG, "SolverSetPC: solver was not created with KRY_PC_CUSTOM");
    s->csetup = setup;
    s->csolve = solve;
    s->cdestroy = destroy;
    s->cdata = data;
    s->assembled = false;
    return KRY_OK;
}

extern "C" int SolverAssemble(SOLVER *s) {
    if (!s || !s->A) return set_error(KRY_ERR_ARG, "SolverAssemble: no matrix");
    if (s->prec != KRY_PREC_F64 && s->type != KRY_FGMRES)
        return set_error(KRY_ERR_ARG, "reduced-precision preconditioning needs FGMRES");
    if (s->augk > 0 && s->type != KRY_GMRES && s->type != KRY_FGMRES)
        return set_error(KRY_ERR_ARG, "aug_k > 0 (LGMRES) applies to GMRES and FGMRES");
    if (s->prec != KRY_PREC_F64 && (s->pc_type == KRY_PC_NONE || s->pc_type == KRY_PC_CUSTOM))
        return set_error(KRY_ERR_ARG, "reduced precision applies to ILU and CPR preconditioners");
    const bool learned = s->pc_type == KRY_PC_BILU0_LEARNED || s->pc_type == KRY_PC_CPR_LEARNED;
    if (learned && s->type != KRY_FGMRES)
        return set_error(KRY_ERR_ARG, "the learned stage varies between applications: it needs FGMRES");
    if (learned && s->learned_params.empty())
        return set_error(KRY_ERR_ARG, "learned stage: call SolverSetLearned before SolverAssemble");
    const auto t0 = std::chrono::steady_clock::now();
    if (!s->err.p) KRY_TRY(s->err.alloc(1));
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s->stream, s->err.p);
    s->ilu.reset();
    // CPR's RAS full stage keeps its subdomain patterns like RAS does
    std::unique_ptr<RasPC> cpr_ras = s->cpr ? std::move(s->cpr->ras) : nullptr;
    s->cpr.reset();
    s->amg.reset();
    // RAS keeps its subdomain patterns when the matrix and options are unchanged
    const bool ras_reuse = s->pc_type == KRY_PC_RAS && s->ras && s->ras->A == s->A &&
                           s->ras->px == s->ras_px && s->ras->py == s->ras_py &&
                           s->ras->pz == s->ras_pz && s->ras->overlap == s->ras_overlap &&
                           s->ras->layout == s->sweep_layout && s->prec == KRY_PREC_F64;
    if (!ras_reuse) s->ras.reset();
    s->learned.reset();
    switch (s->pc_type) {
    case KRY_PC_NONE:
        break;
    case KRY_PC_ILU0:
    case KRY_PC_BILU0_LEARNED:
        s->ilu.reset(new IluFactor());
        KRY_TRY(ilu_setup(s->stream, s->A, s->A->val.p, *s->ilu, s->prec, s->err.p, s->sweep_layout));
        break;
    case KRY_PC_CPR:
    case KRY_PC_CPR_LEARNED:
        s->cpr.reset(new CprPC());
        if (s->cpr_psolver == KRY_CPR_P_AMG) {
            if (s->prec != KRY_PREC_F64)
                return set_error(KRY_ERR_UNSUPPORTED, "CPR with the AMG pressure stage is FP64 only");
            s->cpr->amg.reset(new AmgPC());
            s->cpr->amg_opts = s->amg_opts;
        }
        if (s->cpr_full == KRY_CPR_F_RAS) {
            if (s->prec != KRY_PREC_F64)
                return set_error(KRY_ERR_UNSUPPORTED, "CPR with the RAS full stage is FP64 only");
            const int box[4] = {s->ras_px, s->ras_py, s->ras_pz, s->ras_overlap};
            std::copy(box, box + 4, s->cpr->ras_box);
            const RasPC *R = cpr_ras.get();
            s->cpr->ras_reuse = R && R->A == s->A && R->px == box[0] && R->py == box[1] &&
                                R->pz == box[2] && R->overlap == box[3] &&
                                R->layout == s->sweep_layout;
            if (s->cpr->ras_reuse) s->cpr->ras = std::move(cpr_ras);
            else s->cpr->ras.reset(new RasPC());
        }
        KRY_TRY(cpr_setup(s->stream, s->A, *s->cpr, s->cpr_variant, s->cpr_sweeps, s->prec, s->err.p,
                          s->sweep_layout));
        break;
    case KRY_PC_AMG:
        if (s->A->bs != 1)
            return set_error(KRY_ERR_UNSUPPORTED, "AMG preconditioner: scalar (bs = 1) matrices only");
        if (s->prec != KRY_PREC_F64) return set_error(KRY_ERR_UNSUPPORTED, "AMG preconditioner: FP64 only");
        s->amg.reset(new AmgPC());
        {
            const int rc = amg_setup(s->stream, s->A->nb, s->A->h_rowptr.data(), s->A->h_col.data(),
                                     s->A->val.p, s->amg_opts, *s->amg, s->err.p);
            if (rc < 0) {
                s->amg.reset();
                return rc;
            }
        }
        break;
    case KRY_PC_RAS:
        if (ras_reuse) {
            KRY_TRY(ras_refactor(s->stream, s->A, *s->ras, s->err.p));
        } else {
            s->ras.reset(new RasPC());
            const int rc = ras_setup(s->stream, s->A, *s->ras, s->ras_px, s->ras_py, s->ras_pz,
                                     s->ras_overlap, s->prec, s->err.p, s->sweep_layout);
            if (rc < 0) {
                s->ras.reset();
                return rc;
            }
        }
        break;
    case KRY_PC_CUSTOM:
        if (!s->csolve) return set_error(KRY_ERR_ARG, "custom preconditioner not set");
        if (s->csetup) {
            const int rc = s->csetup(s->cdata, s->A);
            if (rc < 0) return set_error(rc, "custom preconditioner setup failed (%d)", rc);
        }
        break;
    }
    if (learned) {
        LearnedStage *L = nullptr;
        KRY_TRY(learned_stage_create(s->stream, s->A, s->learned_params.data(), s->learned_lnk.p,
                                     KRY_DEVICE, &L));
        s->learned.reset(L);
    }
    KRY_TRY(check_device_error(s));
    KRY_TRY(ensure_workspace(s));
    KRY_HIP(hipStreamSynchronize(s->stream));
    s->t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    s->assembled = true;
    return KRY_OK;
}

extern "C" int SolverSolve(SOLVER *s, VEC *b, VEC *x) {
    if (!s || !b || !x) return set_error(KRY_ERR_ARG, "SolverSolve: NULL argument");
    if (!s->A) return set_error(KRY_ERR_ARG, "SolverSolve: no matrix");
    if (!s->assembled) return set_error(KRY_ERR_ARG, "SolverSolve: call SolverAssemble first");
    const int64_t n = (int64_t)s->A->nb * s->A->bs;
    if (b->n != n || x->n != n) return set_error(KRY_ERR_DIM, "SolverSolve: vector sizes differ from the matrix");
    if (b->data == x->data) return set_error(KRY_ERR_ARG, "SolverSolve: b and x alias");
    const auto t0 = std::chrono::steady_clock::now();
    int rc = s->type == KRY_BICGSTAB ? bicgstab_solve(s, b->data, x->data)
             : s->type == KRY_CG     ? cg_solve(s, b->data, x->data)
                                     : gmres_solve(s, b->data, x->data);
    const int erc = check_device_error(s);
    if (hipStreamSynchronize(s->stream) != hipSuccess && rc >= 0) rc = set_error(KRY_ERR_HIP, "SolverSolve: stream error");
    s->t_solve = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (erc < 0) return erc;
    return rc;
}

static int set_learned(SOLVER *s, std::vector<float> &&params, const float *logk, int where) {
    if (s->pc_type != KRY_PC_BILU0_LEARNED && s->pc_type != KRY_PC_CPR_LEARNED)
        return set_error(KRY_ERR_ARG, "SolverSetLearned: solver was not created with a learned preconditioner");
    if (!logk) return set_error(KRY_ERR_ARG, "SolverSetLearned: ln k is NULL");
    if (s->map->nlocal % 3 != 0) return set_error(KRY_ERR_DIM, "SolverSetLearned: system size is not 3 per cell");
    const int64_t cells = s->map->nlocal / 3;
    KRY_TRY(s->learned_lnk.alloc(cells));
    KRY_HIP(hipMemcpyAsync(s->learned_lnk.p, logk, sizeof(float) * cells,
                           where == KRY_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s->stream));
    KRY_HIP(hipStreamSynchronize(s->stream));
    s->learned_params = std::move(params);
    s->assembled = false;
    return KRY_OK;
}

extern "C" int SolverSetLearned(SOLVER *s, const char *weights_path, const float *logk_dev) {
    if (!s || !weights_path) return set_error(KRY_ERR_ARG, "SolverSetLearned: NULL argument");
    std::vector<float> p, m, v;
    int t = 0;
    KRY_TRY(learned_read_file(weights_path, p, m, v, t));
    return set_learned(s, std::move(p), logk_dev, KRY_DEVICE);
}

extern "C" int SolverSetLearnedParams(SOLVER *s, const float *params_host, const float *logk, int where) {
    if (!s || !params_host) return set_error(KRY_ERR_ARG, "SolverSetLearnedParams: NULL argument");
    std::vector<float> p(params_host, params_host + LearnedNumParams());
    return set_learned(s, std::move(p), logk, where);
}

extern "C" int SolverGetLearnedStats(SOLVER *s, int64_t *applies, int64_t *fallbacks) {
    if (!s) return set_error(KRY_ERR_ARG, "SolverGetLearnedStats: NULL");
    if (!s->learned) return set_error(KRY_ERR_ARG, "SolverGetLearnedStats: no learned stage assembled");
    return learned_stage_stats(s->stream, *s->learned, applies, fallbacks);
}

extern "C" int SolverPCApply(SOLVER *s, VEC *v, VEC *z) {
    if (!s || !v || !z) return set_error(KRY_ERR_ARG, "SolverPCApply: NULL argument");
    if (!s->assembled) return set_error(KRY_ERR_ARG, "SolverPCApply: call SolverAssemble first");
    const int64_t n = (int64_t)s->A->nb * s->A->bs;
    if (v->n != n || z->n != n) return set_error(KRY_ERR_DIM, "SolverPCApply: sizes differ");
    if (v->data == z->data) return set_error(KRY_ERR_ARG, "SolverPCApply: v and z alias");
    KRY_TRY(pc_apply(s, v->data, z->data));
    return check_device_error(s);
}

extern "C" double SolverGetResidual(const SOLVER *s) { return s ? s->residual : NAN; }
extern "C" int SolverGetIters(const SOLVER *s) { return s ? s->nits : -1; }

extern "C" int SolverGetTimes(const SOLVER *s, double *setup_s, double *solve_s) {
    if (!s) return set_error(KRY_ERR_ARG, "SolverGetTimes: NULL solver");
    if (setup_s) *setup_s = s->t_setup;
    if (solve_s) *solve_s = s->t_solve;
    return KRY_OK;
}

extern "C" int SolverGetKrylovBasis(const SOLVER *s, int first, int ncols, double *dst, int where) {
    if (!s || (!dst && ncols > 0) || first < 0 || ncols < 0)
        return set_error(KRY_ERR_ARG, "SolverGetKrylovBasis: bad argument");
    if (!s->V.p || s->ldv == 0)
        return set_error(KRY_ERR_ARG, "SolverGetKrylovBasis: the solver holds no Krylov basis");
    const int64_t n = (int64_t)s->A->nb * s->A->bs;
    if ((int64_t)(first + ncols) * s->ldv > (int64_t)s->V.n)
        return set_error(KRY_ERR_ARG, "SolverGetKrylovBasis: columns [%d, %d) exceed the basis", first,
                         first + ncols);
    const hipMemcpyKind kind = where == KRY_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    for (int c = 0; c < ncols; c++)
        KRY_HIP(hipMemcpyAsync(dst + (size_t)c * n, s->V.p + (size_t)(first + c) * s->ldv,
                               sizeof(double) * n, kind, s->stream));
    KRY_HIP(hipStreamSynchronize(s->stream));
    return KRY_OK;
}

extern "C" int SolverGetHistory(const SOLVER *s, double *hist, int cap) {
    if (!s || (!hist && cap > 0)) return set_error(KRY_ERR_ARG, "SolverGetHistory: bad argument");
    const int k = std::min<int>(cap, static_cast<int>(s->hist.size()));
    for (int i = 0; i < k; i++) hist[i] = s->hist[i];
    return k;
}
