// ILU(0) and block ILU(0) preconditioner: the incomplete factorization
// named in Section 1 (point-wise and block-wise) and the two triangular
// solves of eq. (3), which Section 4.1 notes are row-by-row serial.
//
// gfx950 design
//  * Level scheduling: row i of L y = b depends on the rows k < i of its
//    pattern; its level is one more than the deepest of them (rows with no
//    dependency are level 0).  Backward levels are built the same way from
//    the upper pattern.  For a 7-point stencil in natural order these are
//    the hyperplanes i + j + k = const.
//  * Factorization: one launch per forward level, one thread per row,
//    row-oriented elimination restricted to the pattern (IKJ); the inverse
//    of each diagonal block is formed once (Gaussian elimination with
//    partial pivoting) and reused by every later row and by the solve.
//  * Layout: rows are permuted by level and each level is padded to whole
//    64-row slices, so a wavefront always holds rows of one level, which
//    are mutually independent.  Values sit in entry-major planes (sliced
//    ELLPACK), so the factor streams from HBM in full cache lines.
//  * Sweeps: one launch per sweep.  Wavefronts take slices in level order
//    from an atomic counter; a row waits only for the rows it reads.  Each
//    output value is published with a relaxed agent-scope store into a
//    slot pre-filled with a reserved NaN payload, and consumers poll the
//    slot itself -- no flags, no fences, no grid barriers.  A slice's
//    dependencies are always in earlier slices, which were handed to
//    wavefronts that are already running, so the sweep cannot deadlock; a
//    bounded spin turns any broken schedule into an error instead of a
//    hang.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "device.hpp"
#include "internal.hpp"

namespace kry {

// ---------------------------------------------------------------------------
// host: level sets and level-ordered slices
// ---------------------------------------------------------------------------
struct LevelSlices {
    std::vector<int> perm;        // nslices * 64, -1 = padding lane
    std::vector<int> off;         // nslices + 1 slot offsets
    std::vector<int> lev_slice;   // nlev + 1: first slice of each level
    std::vector<int> slice_of;    // row -> slice
    int nslices = 0, nlev = 0, maxw = 0;
};

// lev: level of each row; ndep(row) number of dependencies (slot count)
template <typename F>
static void build_slices(int nb, const std::vector<int> &lev, int nlev, F ndep,
                         LevelSlices &L) {
    std::vector<int> cnt(nlev + 1, 0);
    for (int i = 0; i < nb; i++) cnt[lev[i] + 1]++;
    for (int l = 0; l < nlev; l++) cnt[l + 1] += cnt[l];
    std::vector<int> order(nb);
    {
        std::vector<int> pos(cnt.begin(), cnt.end() - 1);
        for (int i = 0; i < nb; i++) order[pos[lev[i]]++] = i;   // stable by row index
    }
    L.nlev = nlev;
    L.lev_slice.assign(nlev + 1, 0);
    int ns = 0;
    for (int l = 0; l < nlev; l++) {
        L.lev_slice[l] = ns;
        ns += (cnt[l + 1] - cnt[l] + 63) / 64;
    }
    L.lev_slice[nlev] = ns;
    L.nslices = ns;
    L.perm.assign((size_t)ns * 64, -1);
    L.off.assign(ns + 1, 0);
    L.slice_of.assign(nb, -1);
    L.maxw = 0;
    for (int l = 0; l < nlev; l++) {
        const int r0 = cnt[l], m = cnt[l + 1] - cnt[l];
        for (int q = 0; q < m; q++) {
            const int sl = L.lev_slice[l] + q / 64;
            L.perm[(size_t)sl * 64 + q % 64] = order[r0 + q];
            L.slice_of[order[r0 + q]] = sl;
        }
    }
    for (int s = 0; s < ns; s++) {
        int w = 0;
        for (int q = 0; q < 64; q++) {
            const int r = L.perm[(size_t)s * 64 + q];
            if (r >= 0) w = std::max(w, ndep(r));
        }
        L.off[s + 1] = L.off[s] + w;
        L.maxw = std::max(L.maxw, w);
    }
}

// every dependency of a row must live in an earlier slice
template <typename F>
static bool schedule_is_acyclic(int nb, const LevelSlices &L, F for_deps) {
    for (int i = 0; i < nb; i++) {
        const int si = L.slice_of[i];
        bool ok = si >= 0;
        for_deps(i, [&](int k) { ok = ok && L.slice_of[k] >= 0 && L.slice_of[k] < si; });
        if (!ok) return false;
    }
    return true;
}

// ---------------------------------------------------------------------------
// numeric factorization of the rows of one level (block inverse:
// dev_block_inverse, device.hpp)
// ---------------------------------------------------------------------------
template <int BS>
__global__ __launch_bounds__(256) void k_ilu_factor_level(
    int first_lane, int nlanes, const int *__restrict__ perm, const int *__restrict__ rowptr,
    const int *__restrict__ col, const int *__restrict__ diag, double *__restrict__ lu,
    double *__restrict__ uinv, int *err) {
    constexpr int B2 = BS * BS;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nlanes) return;
    const int i = perm[first_lane + g];
    if (i < 0) return;
    const int p0 = rowptr[i], p1 = rowptr[i + 1], di = diag[i];
    for (int p = p0; p < di; p++) {
        const int k = col[p];
        double L[B2];
        const double *a = lu + (int64_t)p * B2;
        const double *ui = uinv + (int64_t)k * B2;
#pragma unroll
        for (int r = 0; r < BS; r++)
#pragma unroll
            for (int c = 0; c < BS; c++) {
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < BS; q++) s += a[r * BS + q] * ui[q * BS + c];
                L[r * BS + c] = s;
            }
#pragma unroll
        for (int e = 0; e < B2; e++) lu[(int64_t)p * B2 + e] = L[e];
        // a_ij -= L_ik U_kj for j > k in row k with (i, j) in the pattern
        int sidx = p + 1;
        const int q1 = rowptr[k + 1];
        for (int q = diag[k] + 1; q < q1; q++) {
            const int j = col[q];
            while (sidx < p1 && col[sidx] < j) sidx++;
            if (sidx < p1 && col[sidx] == j) {
                const double *u = lu + (int64_t)q * B2;
                double *t = lu + (int64_t)sidx * B2;
#pragma unroll
                for (int r = 0; r < BS; r++)
#pragma unroll
                    for (int c = 0; c < BS; c++) {
                        double s = 0.0;
#pragma unroll
                        for (int m = 0; m < BS; m++) s += L[r * BS + m] * u[m * BS + c];
                        t[r * BS + c] -= s;
                    }
            }
        }
    }
    double D[B2], R[B2];
#pragma unroll
    for (int e = 0; e < B2; e++) D[e] = lu[(int64_t)di * B2 + e];
    if (!dev_block_inverse<BS>(D, R)) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int e = 0; e < B2; e++) R[e] = 0.0;
    }
#pragma unroll
    for (int e = 0; e < B2; e++) uinv[(int64_t)i * B2 + e] = R[e];
}

// ---------------------------------------------------------------------------
// packing into level-ordered slices
// ---------------------------------------------------------------------------
template <int BS, bool UPPER>
__global__ void k_ilu_pack(int nslices, const int *__restrict__ perm, const int *__restrict__ off,
                           const int *__restrict__ rowptr, const int *__restrict__ diag,
                           const int *__restrict__ col, const double *__restrict__ lu,
                           const double *__restrict__ uinv, int *__restrict__ scol,
                           double *__restrict__ sval, double *__restrict__ dinv) {
    constexpr int B2 = BS * BS;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = g >> 6, lane = g & 63;
    if (s >= nslices) return;
    const int row = perm[g];
    const int o0 = off[s], w = off[s + 1] - o0;
    int p0 = 0, len = 0;
    if (row >= 0) {
        p0 = UPPER ? diag[row] + 1 : rowptr[row];
        len = UPPER ? rowptr[row + 1] - p0 : diag[row] - p0;
    }
    for (int t = 0; t < w; t++) {
        const int64_t slot = o0 + t;
        const bool have = t < len;
        scol[slot * 64 + lane] = have ? col[p0 + t] : -1;
#pragma unroll
        for (int e = 0; e < B2; e++)
            sval[(slot * B2 + e) * 64 + lane] = have ? lu[(int64_t)(p0 + t) * B2 + e] : 0.0;
    }
    if (UPPER) {
#pragma unroll
        for (int e = 0; e < B2; e++)
            dinv[((int64_t)s * B2 + e) * 64 + lane] = row >= 0 ? uinv[(int64_t)row * B2 + e] : 0.0;
    }
}

__global__ void k_round_f32(int64_t n, const double *__restrict__ x, float *__restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = static_cast<float>(x[i]);
}

__global__ void k_round_bf16(int64_t n, const double *__restrict__ x, uint16_t *__restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = f32_to_bf16_rne(static_cast<float>(x[i]));
}

template <typename T>
__global__ void k_fill_sentinel(int64_t n, T *y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = sentinel_value<T>();
}

// ---------------------------------------------------------------------------
// sync-free sweeps
// ---------------------------------------------------------------------------
constexpr int CHUNK = 4;   // dependency slots loaded ahead of the waits

template <typename TC, typename TF>
__device__ __forceinline__ TC ldf(const TF *p) { return static_cast<TC>(*p); }
template <>
__device__ __forceinline__ float ldf<float, uint16_t>(const uint16_t *p) { return bf16_to_f32(*p); }

__device__ __forceinline__ int next_slice(int *ctr) {
    int s = 0;
    if ((threadIdx.x & 63) == 0) s = atomicAdd(ctr, 1);
    return __shfl(s, 0, 64);
}

// forward: y_i = b_i - sum_{k<i} L_ik y_k; also marks xo (the backward
// output) as unwritten.
template <int BS, typename TF, typename TC, typename TIN, typename TO>
__global__ __launch_bounds__(256) void k_ilu_fwd(
    int nslices, const int *__restrict__ perm, const int *__restrict__ off,
    const int *__restrict__ col, const TF *__restrict__ val, const TIN *__restrict__ b,
    TC *y, TO *xo, int *ctr, int *other_ctr, int *err) {
    constexpr int B2 = BS * BS;
    const int lane = threadIdx.x & 63;
    if (blockIdx.x == 0 && threadIdx.x == 0) *other_ctr = 0;
    for (;;) {
        const int s = next_slice(ctr);
        if (s >= nslices) break;
        const int row = perm[(int64_t)s * 64 + lane];
        if (row >= 0) {
            TC acc[BS];
#pragma unroll
            for (int r = 0; r < BS; r++) acc[r] = static_cast<TC>(b[(int64_t)row * BS + r]);
            const int o0 = off[s], o1 = off[s + 1];
            for (int t0 = o0; t0 < o1; t0 += CHUNK) {
                int cc[CHUNK];
                TC lv[CHUNK][B2];
#pragma unroll
                for (int q = 0; q < CHUNK; q++) {
                    const int t = t0 + q;
                    cc[q] = t < o1 ? col[(int64_t)t * 64 + lane] : -1;
#pragma unroll
                    for (int e = 0; e < B2; e++)
                        lv[q][e] = cc[q] >= 0 ? ldf<TC, TF>(val + ((int64_t)t * B2 + e) * 64 + lane)
                                              : TC(0);
                }
#pragma unroll
                for (int q = 0; q < CHUNK; q++) {
                    if (cc[q] >= 0) {
                        TC yc[BS];
                        wait_values<TC, BS>(y + (int64_t)cc[q] * BS, yc, err);
#pragma unroll
                        for (int r = 0; r < BS; r++)
#pragma unroll
                            for (int k = 0; k < BS; k++) acc[r] -= lv[q][r * BS + k] * yc[k];
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < BS; r++) publish<TC>(y + (int64_t)row * BS + r, acc[r]);
#pragma unroll
            for (int r = 0; r < BS; r++) xo[(int64_t)row * BS + r] = sentinel_value<TO>();
        }
    }
}

// backward: x_i = U_ii^-1 (y_i - sum_{j>i} U_ij x_j); resets y for the next
// forward sweep.  ADD = 1: add_out = add_in + x; ADD = 2: add_out =
// (add_in[i], 0, 0) + x (pressure injection).
template <int BS, typename TF, typename TD, typename TC, typename TO, int ADD, typename TAI,
          typename TAO>
__global__ __launch_bounds__(256) void k_ilu_bwd(
    int nslices, const int *__restrict__ perm, const int *__restrict__ off,
    const int *__restrict__ col, const TF *__restrict__ val, const TD *__restrict__ dinv, TC *y,
    TO *xo, const TAI *__restrict__ add_in, TAO *__restrict__ add_out, int *ctr, int *other_ctr,
    int *err) {
    constexpr int B2 = BS * BS;
    const int lane = threadIdx.x & 63;
    if (blockIdx.x == 0 && threadIdx.x == 0) *other_ctr = 0;
    for (;;) {
        const int s = next_slice(ctr);
        if (s >= nslices) break;
        const int row = perm[(int64_t)s * 64 + lane];
        if (row >= 0) {
            TC acc[BS];
#pragma unroll
            for (int r = 0; r < BS; r++) {
                acc[r] = y[(int64_t)row * BS + r];
                y[(int64_t)row * BS + r] = sentinel_value<TC>();
            }
            TC dv[B2];
#pragma unroll
            for (int e = 0; e < B2; e++)
                dv[e] = static_cast<TC>(dinv[((int64_t)s * B2 + e) * 64 + lane]);
            const int o0 = off[s], o1 = off[s + 1];
            for (int t0 = o0; t0 < o1; t0 += CHUNK) {
                int cc[CHUNK];
                TC uv[CHUNK][B2];
#pragma unroll
                for (int q = 0; q < CHUNK; q++) {
                    const int t = t0 + q;
                    cc[q] = t < o1 ? col[(int64_t)t * 64 + lane] : -1;
#pragma unroll
                    for (int e = 0; e < B2; e++)
                        uv[q][e] = cc[q] >= 0 ? ldf<TC, TF>(val + ((int64_t)t * B2 + e) * 64 + lane)
                                              : TC(0);
                }
#pragma unroll
                for (int q = 0; q < CHUNK; q++) {
                    if (cc[q] >= 0) {
                        TO xr[BS];
                        wait_values<TO, BS>(xo + (int64_t)cc[q] * BS, xr, err);
#pragma unroll
                        for (int r = 0; r < BS; r++)
#pragma unroll
                            for (int k = 0; k < BS; k++)
                                acc[r] -= uv[q][r * BS + k] * static_cast<TC>(xr[k]);
                    }
                }
            }
            TC res[BS];
#pragma unroll
            for (int r = 0; r < BS; r++) {
                TC t = TC(0);
#pragma unroll
                for (int k = 0; k < BS; k++) t += dv[r * BS + k] * acc[k];
                res[r] = t;
            }
#pragma unroll
            for (int r = 0; r < BS; r++) {
                publish<TO>(xo + (int64_t)row * BS + r, static_cast<TO>(res[r]));
                if (ADD == 1)
                    add_out[(int64_t)row * BS + r] =
                        static_cast<TAO>(add_in[(int64_t)row * BS + r]) + static_cast<TAO>(res[r]);
                if (ADD == 2) {
                    TC base = (r == 0) ? static_cast<TC>(add_in[row]) : TC(0);
                    add_out[(int64_t)row * BS + r] = static_cast<TAO>(base + res[r]);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
static int sweep_waves_cap() {
    static int cap = -1;
    if (cap < 0) {
        const char *e = getenv("KRY_SWEEP_WAVES");
        cap = e ? std::max(4, atoi(e)) : 1024;
    }
    return cap;
}

static int upload_layout(hipStream_t s, const LevelSlices &L, Sell &S, int bs, bool storage) {
    S.bs = bs;
    S.nslices = L.nslices;
    S.maxw = L.maxw;
    S.h_off = L.off;
    S.nslots = L.off[L.nslices];
    KRY_TRY(S.off.alloc(L.nslices + 1));
    KRY_TRY(S.perm.alloc((size_t)L.nslices * 64));
    if (storage) {
        KRY_TRY(S.col.alloc(std::max<int64_t>(1, S.nslots) * 64));
        KRY_TRY(S.val.alloc(std::max<int64_t>(1, S.nslots) * 64 * bs * bs));
    }
    KRY_HIP(hipMemcpyAsync(S.off.p, L.off.data(), sizeof(int) * (L.nslices + 1),
                           hipMemcpyHostToDevice, s));
    KRY_HIP(hipMemcpyAsync(S.perm.p, L.perm.data(), sizeof(int) * L.perm.size(),
                           hipMemcpyHostToDevice, s));
    return KRY_OK;
}

int ilu_setup(hipStream_t s, const MAT_ *A, const double *d_val, IluFactor &F, int prec,
              int *d_err, int layout) {
    const int nb = A->nb, bs = A->bs, b2 = bs * bs;
    const std::vector<int> &rp = A->h_rowptr, &ci = A->h_col, &dg = A->h_diag;
    F.bs = bs;
    F.nb = nb;
    F.prec = prec;
    if (layout == KRY_SWEEP_GRID && A->gnx == 0)
        return set_error(KRY_ERR_ARG, "grid sweep layout requested for a matrix that is not a 7-point grid stencil");
    const bool use_grid = layout == KRY_SWEEP_GRID || (layout == KRY_SWEEP_AUTO && A->gnx > 0);
    if (use_grid && ilu_grid_can_factor(A)) {
        // no level analysis: the grid-tiled factorization writes the sweep
        // layout directly
        F.nlev_f = F.nlev_b = A->gnx + A->gny + A->gnz - 2;
        KRY_TRY(ilu_grid_factor_setup(s, A, d_val, F, d_err));
        KRY_TRY(F.ctr.alloc(2 * GRID_QUEUES));
        KRY_HIP(hipMemsetAsync(F.ctr.p, 0, 2 * GRID_QUEUES * sizeof(int), s));
        KRY_HIP(hipStreamSynchronize(s));
        return KRY_OK;
    }
    // level sets
    std::vector<int> levf(nb, 0), levb(nb, 0);
    int nlf = 0, nlb = 0;
    for (int i = 0; i < nb; i++) {
        int l = 0;
        for (int p = rp[i]; p < dg[i]; p++) l = std::max(l, levf[ci[p]] + 1);
        levf[i] = l;
        nlf = std::max(nlf, l + 1);
    }
    for (int i = nb - 1; i >= 0; i--) {
        int l = 0;
        for (int p = dg[i] + 1; p < rp[i + 1]; p++) l = std::max(l, levb[ci[p]] + 1);
        levb[i] = l;
        nlb = std::max(nlb, l + 1);
    }
    F.nlev_f = nlf;
    F.nlev_b = nlb;
    LevelSlices LF, LB;
    build_slices(nb, levf, nlf, [&](int r) { return dg[r] - rp[r]; }, LF);
    build_slices(nb, levb, nlb, [&](int r) { return rp[r + 1] - dg[r] - 1; }, LB);
    const bool okf = schedule_is_acyclic(nb, LF, [&](int i, auto f) {
        for (int p = rp[i]; p < dg[i]; p++) f(ci[p]);
    });
    const bool okb = schedule_is_acyclic(nb, LB, [&](int i, auto f) {
        for (int p = dg[i] + 1; p < rp[i + 1]; p++) f(ci[p]);
    });
    if (!okf || !okb) return set_error(KRY_ERR_ARG, "ILU: inconsistent level schedule");

    KRY_TRY(upload_layout(s, LF, F.L, bs, !use_grid));
    if (!use_grid) KRY_TRY(upload_layout(s, LB, F.U, bs, true));

    // numeric factorization on a working copy of the values
    DBuf<double> lu, uinv;
    KRY_TRY(lu.alloc((size_t)A->nnzb * b2));
    KRY_TRY(uinv.alloc((size_t)nb * b2));
    KRY_HIP(hipMemcpyAsync(lu.p, d_val, sizeof(double) * A->nnzb * b2, hipMemcpyDeviceToDevice, s));
    for (int l = 0; l < nlf; l++) {
        const int first = LF.lev_slice[l] * 64;
        const int nl = (LF.lev_slice[l + 1] - LF.lev_slice[l]) * 64;
        dim3 g((nl + 255) / 256);
        if (bs == 1)
            hipLaunchKernelGGL(k_ilu_factor_level<1>, g, dim3(256), 0, s, first, nl, F.L.perm.p,
                               A->rowptr.p, A->col.p, A->diag.p, lu.p, uinv.p, d_err);
        else
            hipLaunchKernelGGL(k_ilu_factor_level<3>, g, dim3(256), 0, s, first, nl, F.L.perm.p,
                               A->rowptr.p, A->col.p, A->diag.p, lu.p, uinv.p, d_err);
    }
    KRY_HIP(hipGetLastError());

    if (use_grid) {
        KRY_TRY(ilu_grid_setup(s, A, lu.p, uinv.p, F));
    } else {
    // pack L and U (+ diagonal inverses) in level order
    KRY_TRY(F.dinv.alloc((size_t)F.U.nslices * 64 * b2));
    {
        dim3 gl((F.L.nslices * 64 + 255) / 256), gu((F.U.nslices * 64 + 255) / 256);
        if (bs == 1) {
            hipLaunchKernelGGL((k_ilu_pack<1, false>), gl, dim3(256), 0, s, F.L.nslices, F.L.perm.p,
                               F.L.off.p, A->rowptr.p, A->diag.p, A->col.p, lu.p, uinv.p,
                               F.L.col.p, F.L.val.p, nullptr);
            hipLaunchKernelGGL((k_ilu_pack<1, true>), gu, dim3(256), 0, s, F.U.nslices, F.U.perm.p,
                               F.U.off.p, A->rowptr.p, A->diag.p, A->col.p, lu.p, uinv.p,
                               F.U.col.p, F.U.val.p, F.dinv.p);
        } else {
            hipLaunchKernelGGL((k_ilu_pack<3, false>), gl, dim3(256), 0, s, F.L.nslices, F.L.perm.p,
                               F.L.off.p, A->rowptr.p, A->diag.p, A->col.p, lu.p, uinv.p,
                               F.L.col.p, F.L.val.p, nullptr);
            hipLaunchKernelGGL((k_ilu_pack<3, true>), gu, dim3(256), 0, s, F.U.nslices, F.U.perm.p,
                               F.U.off.p, A->rowptr.p, A->diag.p, A->col.p, lu.p, uinv.p,
                               F.U.col.p, F.U.val.p, F.dinv.p);
        }
        KRY_HIP(hipGetLastError());
    }
    // reduced-precision copies: off-diagonal blocks to FP32 or BF16,
    // diagonal inverses to FP32
    if (prec != KRY_PREC_F64) {
        const int64_t nl = std::max<int64_t>(1, F.L.nslots) * 64 * b2;
        const int64_t nu = std::max<int64_t>(1, F.U.nslots) * 64 * b2;
        const int64_t nd = (int64_t)F.U.nslices * 64 * b2;
        KRY_TRY(F.dinvf.alloc(nd));
        hipLaunchKernelGGL(k_round_f32, dim3(1024), dim3(256), 0, s, nd, F.dinv.p, F.dinvf.p);
        if (prec == KRY_PREC_F32) {
            KRY_TRY(F.L.valf.alloc(nl));
            KRY_TRY(F.U.valf.alloc(nu));
            hipLaunchKernelGGL(k_round_f32, dim3(1024), dim3(256), 0, s, nl, F.L.val.p, F.L.valf.p);
            hipLaunchKernelGGL(k_round_f32, dim3(1024), dim3(256), 0, s, nu, F.U.val.p, F.U.valf.p);
        } else {
            KRY_TRY(F.L.valh.alloc(nl));
            KRY_TRY(F.U.valh.alloc(nu));
            hipLaunchKernelGGL(k_round_bf16, dim3(1024), dim3(256), 0, s, nl, F.L.val.p, F.L.valh.p);
            hipLaunchKernelGGL(k_round_bf16, dim3(1024), dim3(256), 0, s, nu, F.U.val.p, F.U.valh.p);
        }
        KRY_HIP(hipGetLastError());
        // the FP64 planes are not needed by a reduced-precision apply
        F.L.val.release();
        F.U.val.release();
        F.dinv.release();
    }
    }
    // sweep state: forward output all-unwritten, counters zero
    const int64_t n = (int64_t)nb * bs;
    if (prec == KRY_PREC_F64) {
        KRY_TRY(F.y64.alloc(n));
        hipLaunchKernelGGL(k_fill_sentinel<double>, dim3(1024), dim3(256), 0, s, n, F.y64.p);
    } else {
        KRY_TRY(F.y32.alloc(n));
        hipLaunchKernelGGL(k_fill_sentinel<float>, dim3(1024), dim3(256), 0, s, n, F.y32.p);
    }
    KRY_HIP(hipGetLastError());
    KRY_TRY(F.ctr.alloc(2 * GRID_QUEUES));
    KRY_HIP(hipMemsetAsync(F.ctr.p, 0, 2 * GRID_QUEUES * sizeof(int), s));
    F.grid_waves = std::min(std::max(F.L.nslices, F.U.nslices), sweep_waves_cap());
    // the working copy is freed on return: wait for the kernels using it
    KRY_HIP(hipStreamSynchronize(s));
    return KRY_OK;
}

// ---------------------------------------------------------------------------
// apply
// ---------------------------------------------------------------------------
const char *sweep_timer_name(bool fwd, int bs, int factor_bytes, int add_mode) {
    // [bs == 3][precision f64/f32/bf16][fwd, bwd, bwd+add1, bwd+add2]
    static const char *const names[2][3][4] = {
        {{"ilu_fwd_csr_f64", "ilu_bwd_csr_f64", "ilu_bwd_csr_f64_add", "ilu_bwd_csr_f64_inject"},
         {"ilu_fwd_csr_f32", "ilu_bwd_csr_f32", "ilu_bwd_csr_f32_add", "ilu_bwd_csr_f32_inject"},
         {"ilu_fwd_csr_bf16", "ilu_bwd_csr_bf16", "ilu_bwd_csr_bf16_add", "ilu_bwd_csr_bf16_inject"}},
        {{"ilu_fwd_bsr3_f64", "ilu_bwd_bsr3_f64", "ilu_bwd_bsr3_f64_add", "ilu_bwd_bsr3_f64_inject"},
         {"ilu_fwd_bsr3_f32", "ilu_bwd_bsr3_f32", "ilu_bwd_bsr3_f32_add", "ilu_bwd_bsr3_f32_inject"},
         {"ilu_fwd_bsr3_bf16", "ilu_bwd_bsr3_bf16", "ilu_bwd_bsr3_bf16_add", "ilu_bwd_bsr3_bf16_inject"}},
    };
    const int p = factor_bytes == 8 ? 0 : factor_bytes == 4 ? 1 : 2;
    return names[bs == 3][p][fwd ? 0 : 1 + add_mode];
}

template <int BS, typename TF, typename TD, typename TC, typename TIN, typename TO, int ADD,
          typename TAI, typename TAO>
static int sweep_pair(hipStream_t s, IluFactor &F, const TF *lval, const TF *uval, const TD *dinv,
                      TC *y, const TIN *b, TO *xo, const TAI *add_in, TAO *add_out, int *err) {
    const dim3 grid((F.grid_waves + 3) / 4), block(256);
    {
        TimedScope t(F.timer_fwd ? F.timer_fwd : sweep_timer_name(true, BS, sizeof(TF), ADD), s);
        hipLaunchKernelGGL((k_ilu_fwd<BS, TF, TC, TIN, TO>), grid, block, 0, s, F.L.nslices,
                           F.L.perm.p, F.L.off.p, F.L.col.p, lval, b, y, xo, F.ctr.p,
                           F.ctr.p + 1, err);
    }
    {
        TimedScope t(F.timer_bwd ? F.timer_bwd : sweep_timer_name(false, BS, sizeof(TF), ADD), s);
        hipLaunchKernelGGL((k_ilu_bwd<BS, TF, TD, TC, TO, ADD, TAI, TAO>), grid, block, 0, s,
                           F.U.nslices, F.U.perm.p, F.U.off.p, F.U.col.p, uval, dinv, y, xo,
                           add_in, add_out, F.ctr.p + 1, F.ctr.p, err);
    }
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

// dispatch on the factor precision, then the vector types
template <int BS, typename TIN, typename TO>
static int apply_typed(hipStream_t s, IluFactor &F, const TIN *b, TO *xo, int add_mode,
                       const void *add_in, void *add_out, int *err) {
    if (F.prec == KRY_PREC_F64) {
        using TC = double;
        if (add_mode == 0)
            return sweep_pair<BS, double, double, TC, TIN, TO, 0, double, double>(
                s, F, F.L.val.p, F.U.val.p, F.dinv.p, F.y64.p, b, xo, nullptr, nullptr, err);
        if (add_mode == 1)
            return sweep_pair<BS, double, double, TC, TIN, TO, 1, TO, TO>(
                s, F, F.L.val.p, F.U.val.p, F.dinv.p, F.y64.p, b, xo, (const TO *)add_in,
                (TO *)add_out, err);
        return sweep_pair<BS, double, double, TC, TIN, TO, 2, TC, double>(
            s, F, F.L.val.p, F.U.val.p, F.dinv.p, F.y64.p, b, xo, (const TC *)add_in,
            (double *)add_out, err);
    }
    using TC = float;
    if (F.prec == KRY_PREC_F32) {
        if (add_mode == 0)
            return sweep_pair<BS, float, float, TC, TIN, TO, 0, float, float>(
                s, F, F.L.valf.p, F.U.valf.p, F.dinvf.p, F.y32.p, b, xo, nullptr, nullptr, err);
        if (add_mode == 1)
            return sweep_pair<BS, float, float, TC, TIN, TO, 1, TO, TO>(
                s, F, F.L.valf.p, F.U.valf.p, F.dinvf.p, F.y32.p, b, xo, (const TO *)add_in,
                (TO *)add_out, err);
        return sweep_pair<BS, float, float, TC, TIN, TO, 2, TC, double>(
            s, F, F.L.valf.p, F.U.valf.p, F.dinvf.p, F.y32.p, b, xo, (const TC *)add_in,
            (double *)add_out, err);
    }
    if (add_mode == 0)
        return sweep_pair<BS, uint16_t, float, TC, TIN, TO, 0, float, float>(
            s, F, F.L.valh.p, F.U.valh.p, F.dinvf.p, F.y32.p, b, xo, nullptr, nullptr, err);
    if (add_mode == 1)
        return sweep_pair<BS, uint16_t, float, TC, TIN, TO, 1, TO, TO>(
            s, F, F.L.valh.p, F.U.valh.p, F.dinvf.p, F.y32.p, b, xo, (const TO *)add_in,
            (TO *)add_out, err);
    return sweep_pair<BS, uint16_t, float, TC, TIN, TO, 2, TC, double>(
        s, F, F.L.valh.p, F.U.valh.p, F.dinvf.p, F.y32.p, b, xo, (const TC *)add_in,
        (double *)add_out, err);
}

template <int BS>
static int apply_bs(hipStream_t s, IluFactor &F, const void *b, int in_type, void *xscr,
                    int out_type, int add_mode, const void *add_in, void *add_out, int *err) {
    if (in_type == 0 && out_type == 0)
        return apply_typed<BS>(s, F, (const double *)b, (double *)xscr, add_mode, add_in, add_out, err);
    if (in_type == 0 && out_type == 1)
        return apply_typed<BS>(s, F, (const double *)b, (float *)xscr, add_mode, add_in, add_out, err);
    if (in_type == 1 && out_type == 0)
        return apply_typed<BS>(s, F, (const float *)b, (double *)xscr, add_mode, add_in, add_out, err);
    return apply_typed<BS>(s, F, (const float *)b, (float *)xscr, add_mode, add_in, add_out, err);
}

int ilu_apply(hipStream_t s, IluFactor &F, const void *b, int in_type, void *xscr, int out_type,
              int add_mode, const void *add_in, void *add_out, int *d_err) {
    if (F.nb == 0) return set_error(KRY_ERR_ARG, "ILU apply before setup");
    if (F.grid)
        return ilu_grid_apply(s, F, b, in_type, xscr, out_type, add_mode, add_in, add_out, d_err);
    if (F.bs == 1) return apply_bs<1>(s, F, b, in_type, xscr, out_type, add_mode, add_in, add_out, d_err);
    return apply_bs<3>(s, F, b, in_type, xscr, out_type, add_mode, add_in, add_out, d_err);
}

}  // namespace kry
