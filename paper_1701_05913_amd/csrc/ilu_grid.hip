// Grid-tiled ILU(0) sweeps for 7-point stencils in natural order.
//
// The solves of eq. (3) on an nx x ny x nz grid: cell (i, j, k) of the
// forward sweep needs (i-1, j, k), (i, j-1, k) and (i, j, k-1); the
// backward sweep the +1 neighbours.  The level of a cell is i + j + k
// (hyperplanes), as in the generic level schedule, but here the grid's
// (j, k) plane is cut into TJ x TK tiles of x-lines and one 64-lane
// wavefront owns a tile, one lane per line.  At step t lane (jj, kk)
// processes i = t - jj - kk, so
//   * (i-1) is the lane's own result of the previous step (a register),
//   * (j-1) and (k-1) are the results of lanes jj-1 and kk-1 of the
//     previous step (cross-lane moves),
//   * only lanes on the tile's low faces need values of neighbouring
//     tiles, which those tiles publish into small per-step face buffers.
// A dependency chain therefore crosses memory only when it crosses a tile
// face: NJ + NK hops per sweep instead of nx + ny + nz levels.  Tiles are
// handed to workgroups in the order of J + K from an atomic counter, so a
// tile's producers are always running already (no deadlock).
//
// Layouts (all step-major per tile in 64-lane planes, so every wavefront
// access of the sweeps is one contiguous row):
//   factors  forward block b (0: k-1, 1: j-1, 2: i-1) entry e of lane l at
//            step t of tile T at Lt[(((T * S + t) * 3 + b) * bs^2 + e) * 64 + l];
//            backward blocks (0: i+1, 1: j+1, 2: k+1) likewise in Ut,
//            indexed by the backward step, diagonal-block inverses in Dt;
//   result   yt[((T * S + t) * bs + r) * 64 + l]: the forward result of
//            the cell of lane l at forward step t; the backward sweep
//            reads it and overwrites it with the backward result of the
//            same cell (its step S - 1 - t), and a last kernel copies it
//            to the caller's vector in natural order;
//   faces    face entry f of step t of tile T at ((T * S + t) * NF + f) * bs:
//            f < TK the j-face cell of lane kk = f, f = TK + q the k-face
//            cell of lane jj = q.
// Missing neighbours, idle lanes and steps outside the line hold zero
// factors and zero right-hand sides.  Such lanes only ever see zeros, so
// they compute exact zeros, and a real cell multiplies a zero block only
// by an exact zero: the sweeps need no per-lane predication.
#include <algorithm>
#include <type_traits>

#include "device.hpp"
#include "internal.hpp"

namespace kry {

constexpr int NLOAD = 2;       // DMA loader wavefronts per workgroup
constexpr int GWG = 64 * (2 + NLOAD);   // one wavefront per SIMD
constexpr int NFACE = 40;      // >= TJ + TK for every tiling used
constexpr int DB = 16;         // boundary ring depth (steps)

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
template <int BS>
__global__ void k_grid_pack(GridTiles G, const int *__restrict__ rowptr,
                            const int *__restrict__ col, const int *__restrict__ diag,
                            const double *__restrict__ lu, const double *__restrict__ uinv,
                            double *__restrict__ Lt, double *__restrict__ Ut,
                            double *__restrict__ Dt) {
    constexpr int B2 = BS * BS;
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = static_cast<int>(g & 63);
    const int64_t rest = g >> 6;
    const int t = static_cast<int>(rest % G.S);
    const int T = static_cast<int>(rest / G.S);
    if (T >= G.ntiles) return;
    const int JK = G.order[T];
    const int jj = lane % G.TJ, kk = lane / G.TJ;
    const int j = (JK & 0xffff) * G.TJ + jj, k = (JK >> 16) * G.TK + kk;
    const bool lane_ok = lane < G.TJ * G.TK && j < G.ny && k < G.nz;
    const int64_t sJ = G.nx, sK = (int64_t)G.nx * G.ny;
    const int64_t step = (int64_t)T * G.S + t;
    double *lf = Lt + step * 3 * B2 * 64 + lane;
    double *ub = Ut + step * 3 * B2 * 64 + lane;
    double *db = Dt + step * B2 * 64 + lane;
    for (int e = 0; e < 3 * B2; e++) {
        lf[e * 64] = 0.0;
        ub[e * 64] = 0.0;
    }
    for (int e = 0; e < B2; e++) db[e * 64] = 0.0;
    // forward cell of this step
    const int i = t - jj - kk;
    if (lane_ok && i >= 0 && i < G.nx) {
        const int64_t c = i + sJ * j + sK * k;
        for (int p = rowptr[c]; p < diag[c]; p++) {
            const int64_t cc = col[p];
            const int b = cc == c - sK ? 0 : (cc == c - sJ ? 1 : 2);
            for (int e = 0; e < B2; e++) lf[(b * B2 + e) * 64] = lu[(int64_t)p * B2 + e];
        }
    }
    // backward cell of this step
    const int ib = G.nx - 1 - (t - (G.TJ - 1 - jj) - (G.TK - 1 - kk));
    if (lane_ok && ib >= 0 && ib < G.nx) {
        const int64_t c = ib + sJ * j + sK * k;
        for (int p = diag[c] + 1; p < rowptr[c + 1]; p++) {
            const int64_t cc = col[p];
            const int b = cc == c + 1 ? 0 : (cc == c + sJ ? 1 : 2);
            for (int e = 0; e < B2; e++) ub[(b * B2 + e) * 64] = lu[(int64_t)p * B2 + e];
        }
        for (int e = 0; e < B2; e++) db[e * 64] = uinv[c * B2 + e];
    }
}

__global__ void k_grid_round_f32(int64_t n, const double *__restrict__ x, float *__restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = static_cast<float>(x[i]);
}

__global__ void k_grid_round_bf16(int64_t n, const double *__restrict__ x, uint16_t *__restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = f32_to_bf16_rne(static_cast<float>(x[i]));
}

template <typename T>
__global__ void k_grid_fill_sentinel(int64_t n, T *__restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = sentinel_value<T>();
}

// ---------------------------------------------------------------------------
// grid-tiled numeric factorization (nx >= 3 and ny >= 3)
// ---------------------------------------------------------------------------
// For a 7-point stencil in natural order with nx, ny >= 3, ILU(0) changes
// only the diagonal blocks: no product L_ik U_kj of the elimination lands on
// an off-diagonal entry of row i, so
//   D_c = A_cc - sum over the lower neighbours n of (A_cn D_n^-1) A_nc,
// with the neighbours taken in column order (k-1, j-1, i-1) as the
// row-wise elimination takes them.  The kernel walks the forward
// hyperplanes like the forward sweep (one wavefront per tile, one lane per
// x-line), takes D_n^-1 of i-1 from the lane's previous step, of j-1 and
// k-1 from neighbouring lanes or from the face entries published by the
// upstream tiles, and writes the packed sweep layout directly:
// Lt = A_cn D_n^-1, Ut = the upper blocks of A, Dt = D_c^-1.  Positions in
// the block rows follow from the cell's neighbours (one rowptr load per row).
template <int BS>
__device__ __forceinline__ void grid_factor_body(const GridTiles &G, const int *__restrict__ rowptr,
                                                 const double *__restrict__ val,
                                                 double *__restrict__ Lt, double *__restrict__ Ut,
                                                 double *__restrict__ Dt, double *faces, int *ctr,
                                                 int *err) {
    constexpr int B2 = BS * BS;
    const int lane = threadIdx.x;
    const int TJ = G.TJ, TK = G.TK, NF = G.NF, nx = G.nx, ny = G.ny, nz = G.nz, S = G.S;
    const int64_t sJ = nx, sK = (int64_t)nx * ny;
    const int jj = lane % TJ, kk = lane / TJ;
    const int fj = jj == TJ - 1 && kk < TK ? kk : -1;       // published face entries
    const int fk = kk == TK - 1 ? TK + jj : -1;
    for (;;) {
        int t0 = 0;
        if (lane == 0) t0 = atomicAdd(ctr, 1);
        const int T = __shfl(t0, 0, 64);
        if (T >= G.ntiles) break;
        const int JK = G.order[T];
        const int J = JK & 0xffff, K = JK >> 16;
        const int j = J * TJ + jj, k = K * TK + kk;
        const bool lane_ok = lane < TJ * TK && j < ny && k < nz;
        const int64_t cl = lane_ok ? sJ * j + sK * k : 0;
        const double *srcj = (jj == 0 && J > 0 && lane_ok)
                                 ? faces + (((int64_t)G.tidx[(J - 1) * G.NK + K] * S + (TJ - 1)) * NF + kk) * B2
                                 : nullptr;
        const double *srck = (kk == 0 && K > 0 && lane_ok)
                                 ? faces + (((int64_t)G.tidx[J * G.NK + K - 1] * S + (TK - 1)) * NF + TK + jj) * B2
                                 : nullptr;
        double *frow = faces + (int64_t)T * S * NF * B2;
        double dp[B2];
#pragma unroll
        for (int e = 0; e < B2; e++) dp[e] = 0.0;
        for (int t = 0; t < S; t++) {
            const int i = t - jj - kk;
            const bool valid = lane_ok && i >= 0 && i < nx;
            // D^-1 of the lower neighbours: (k-1, j-1, i-1)
            double dn[3][B2];
#pragma unroll
            for (int e = 0; e < B2; e++) {
                dn[0][e] = __shfl_up(dp[e], TJ, 64);
                dn[1][e] = __shfl_up(dp[e], 1, 64);
                dn[2][e] = dp[e];
            }
            if (valid && k > 0 && kk == 0 && srck) wait_values<double, B2>(srck + (int64_t)t * NF * B2, dn[0], err);
            if (valid && j > 0 && jj == 0 && srcj) wait_values<double, B2>(srcj + (int64_t)t * NF * B2, dn[1], err);
            double D[B2], L[3][B2], R[B2];
#pragma unroll
            for (int e = 0; e < B2; e++) {
                D[e] = 0.0;
                R[e] = 0.0;
#pragma unroll
                for (int b = 0; b < 3; b++) L[b][e] = 0.0;
            }
            const int64_t c = cl + i;
            if (valid) {
                // neighbours present, in column order: k-1, j-1, i-1, i+1, j+1, k+1
                const bool has[6] = {k > 0, j > 0, i > 0, i < nx - 1, j < ny - 1, k < nz - 1};
                const int64_t nbr[3] = {c - sK, c - sJ, c - 1};
                // A_nc sits in row n after n's lower blocks, its diagonal and
                // the upper neighbours of n that precede column c
                int qn[3] = {0, 0, 0};
                if (has[0]) qn[0] = rowptr[nbr[0]] + ((k - 1 > 0) + (j > 0) + (i > 0)) + 1 + has[3] + has[4];
                if (has[1]) qn[1] = rowptr[nbr[1]] + ((k > 0) + (j - 1 > 0) + (i > 0)) + 1 + has[3];
                if (has[2]) qn[2] = rowptr[nbr[2]] + ((k > 0) + (j > 0) + (i - 1 > 0)) + 1;
                int p = rowptr[c];
                // L = A_cn D_n^-1 for row c's lower blocks
#pragma unroll
                for (int b = 0; b < 3; b++) {
                    if (!has[b]) continue;
                    const double *a = val + (int64_t)p * B2;
#pragma unroll
                    for (int r = 0; r < BS; r++)
#pragma unroll
                        for (int cc = 0; cc < BS; cc++) {
                            double sacc = 0.0;
#pragma unroll
                            for (int m = 0; m < BS; m++) sacc += a[r * BS + m] * dn[b][m * BS + cc];
                            L[b][r * BS + cc] = sacc;
                        }
                    p++;
                }
                // diagonal block, minus L A_nc in column order
                const double *ad = val + (int64_t)p * B2;
#pragma unroll
                for (int e = 0; e < B2; e++) D[e] = ad[e];
#pragma unroll
                for (int b = 0; b < 3; b++) {
                    if (!has[b]) continue;
                    const double *u = val + (int64_t)qn[b] * B2;
#pragma unroll
                    for (int r = 0; r < BS; r++)
#pragma unroll
                        for (int cc = 0; cc < BS; cc++) {
                            double sacc = 0.0;
#pragma unroll
                            for (int m = 0; m < BS; m++) sacc += L[b][r * BS + m] * u[m * BS + cc];
                            D[r * BS + cc] -= sacc;
                        }
                }
                if (!dev_block_inverse<BS>(D, R)) {
                    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                    for (int e = 0; e < B2; e++) R[e] = 0.0;
                }
                // upper blocks (unchanged) and the inverse, at the backward step
                const int tb = (nx - 1 - i) + (TJ - 1 - jj) + (TK - 1 - kk);
                double *ub = Ut + (int64_t)T * S * 3 * B2 * 64 + lane;
                double *db = Dt + (int64_t)T * S * B2 * 64 + lane;
                int pu = p + 1;
#pragma unroll
                for (int b = 0; b < 3; b++) {
                    if (!has[3 + b]) continue;
#pragma unroll
                    for (int e = 0; e < B2; e++)
                        ub[(((int64_t)tb * 3 + b) * B2 + e) * 64] = val[(int64_t)pu * B2 + e];
                    pu++;
                }
#pragma unroll
                for (int e = 0; e < B2; e++) db[((int64_t)tb * B2 + e) * 64] = R[e];
            }
            // forward blocks of this step (zeros for idle lanes and steps)
            double *lf = Lt + (int64_t)T * S * 3 * B2 * 64 + lane;
#pragma unroll
            for (int b = 0; b < 3; b++)
#pragma unroll
                for (int e = 0; e < B2; e++) lf[(((int64_t)t * 3 + b) * B2 + e) * 64] = L[b][e];
            if (fj >= 0)
#pragma unroll
                for (int e = 0; e < B2; e++) publish<double>(frow + ((int64_t)t * NF + fj) * B2 + e, R[e]);
            if (fk >= 0)
#pragma unroll
                for (int e = 0; e < B2; e++) publish<double>(frow + ((int64_t)t * NF + fk) * B2 + e, R[e]);
#pragma unroll
            for (int e = 0; e < B2; e++) dp[e] = R[e];
        }
    }
}

template <int BS>
__global__ __launch_bounds__(64) void k_grid_factor(GridTiles G, const int *__restrict__ rowptr,
                                                    const double *__restrict__ val,
                                                    double *__restrict__ Lt, double *__restrict__ Ut,
                                                    double *__restrict__ Dt, double *faces, int *ctr,
                                                    int *err) {
    grid_factor_body<BS>(G, rowptr, val, Lt, Ut, Dt, faces, ctr, err);
}

// the factorizations of several independent grids in one launch: grid g
// owns the workgroups [wg0, next wg0)
template <int BS>
__global__ __launch_bounds__(64) void k_grid_factor_multi(const FactorMulti *__restrict__ d,
                                                          int ngrid, int *err) {
    int g = 0;
    while (g + 1 < ngrid && (int)blockIdx.x >= d[g + 1].wg0) g++;
    const FactorMulti D = d[g];
    grid_factor_body<BS>(D.G, D.rowptr, D.val, D.lt, D.ut, D.dt, D.faces, D.ctr, err);
}

// tiling of the (j, k) plane and the tile order (J + K diagonals)
static int grid_tiling(const MAT_ *A, IluFactor &F) {
    GridTiles &G = F.G;
    G.nx = A->gnx;
    G.ny = A->gny;
    G.nz = A->gnz;
    G.TJ = std::min(8, G.ny);
    G.TK = std::min(std::min(64 / G.TJ, G.nz), NFACE - G.TJ);
    G.NF = G.TJ + G.TK;
    G.NJ = (G.ny + G.TJ - 1) / G.TJ;
    G.NK = (G.nz + G.TK - 1) / G.TK;
    G.ntiles = G.NJ * G.NK;
    G.S = G.nx + G.TJ + G.TK - 2;
    if (G.NJ > 0xffff || G.NK > 0x7fff) return set_error(KRY_ERR_UNSUPPORTED, "grid too large for tiling");
    std::vector<int> ord, tid(G.ntiles);
    ord.reserve(G.ntiles);
    for (int d = 0; d <= G.NJ + G.NK - 2; d++)
        for (int J = 0; J < G.NJ; J++) {
            const int K = d - J;
            if (K >= 0 && K < G.NK) {
                tid[J * G.NK + K] = static_cast<int>(ord.size());
                ord.push_back(J | (K << 16));
            }
        }
    // queues of tile columns: tiles sharing J (the k-face neighbours) stay
    // on one XCD and exchange faces through its L2
    G.NQ = GRID_QUEUES;
    std::vector<int> qt, qo(G.NQ + 1, 0);
    qt.reserve(G.ntiles);
    for (int q = 0; q < G.NQ; q++) {
        qo[q] = static_cast<int>(qt.size());
        for (int T = 0; T < G.ntiles; T++)
            if (((ord[T] & 0xffff) + F.qrot) % G.NQ == q) qt.push_back(T);
    }
    qo[G.NQ] = static_cast<int>(qt.size());
    G.qmax = 0;
    for (int q = 0; q < G.NQ; q++) G.qmax = std::max(G.qmax, qo[q + 1] - qo[q]);
    KRY_TRY(F.order.alloc(G.ntiles));
    KRY_TRY(F.tidx.alloc(G.ntiles));
    KRY_TRY(F.qtiles.alloc(G.ntiles));
    KRY_TRY(F.qoff.alloc(G.NQ + 1));
    KRY_HIP(hipMemcpy(F.order.p, ord.data(), sizeof(int) * G.ntiles, hipMemcpyHostToDevice));
    KRY_HIP(hipMemcpy(F.tidx.p, tid.data(), sizeof(int) * G.ntiles, hipMemcpyHostToDevice));
    KRY_HIP(hipMemcpy(F.qtiles.p, qt.data(), sizeof(int) * G.ntiles, hipMemcpyHostToDevice));
    KRY_HIP(hipMemcpy(F.qoff.p, qo.data(), sizeof(int) * (G.NQ + 1), hipMemcpyHostToDevice));
    G.order = F.order.p;
    G.tidx = F.tidx.p;
    G.qtiles = F.qtiles.p;
    G.qoff = F.qoff.p;
    const int b2 = A->bs * A->bs;
    const int64_t steps = (int64_t)G.ntiles * G.S;
    KRY_TRY(F.lt64.alloc(steps * 3 * b2 * 64));
    KRY_TRY(F.ut64.alloc(steps * 3 * b2 * 64));
    KRY_TRY(F.dt64.alloc(steps * b2 * 64));
    return KRY_OK;
}

// reduced-precision copies of the FP64 planes, result and face buffers
static int grid_finish(hipStream_t s, const MAT_ *A, IluFactor &F) {
    const GridTiles &G = F.G;
    const int bs = A->bs, b2 = bs * bs;
    const int64_t steps = (int64_t)G.ntiles * G.S;
    const int64_t nlu = steps * 3 * b2 * 64, nd = steps * b2 * 64;
    const int64_t nyt = steps * bs * 64, nf = steps * G.NF * bs;
    const dim3 blk(256);
    if (F.prec != KRY_PREC_F64) {
        KRY_TRY(F.dt32.alloc(nd));
        hipLaunchKernelGGL(k_grid_round_f32, dim3(2048), blk, 0, s, nd, F.dt64.p, F.dt32.p);
        if (F.prec == KRY_PREC_F32) {
            KRY_TRY(F.lt32.alloc(nlu));
            KRY_TRY(F.ut32.alloc(nlu));
            hipLaunchKernelGGL(k_grid_round_f32, dim3(2048), blk, 0, s, nlu, F.lt64.p, F.lt32.p);
            hipLaunchKernelGGL(k_grid_round_f32, dim3(2048), blk, 0, s, nlu, F.ut64.p, F.ut32.p);
        } else {
            // 128 elements of slack: the sweeps' DMA of a step's planes
            // rounds up to 256 bytes
            KRY_TRY(F.lt16.alloc(nlu + 128));
            KRY_TRY(F.ut16.alloc(nlu + 128));
            hipLaunchKernelGGL(k_grid_round_bf16, dim3(2048), blk, 0, s, nlu, F.lt64.p, F.lt16.p);
            hipLaunchKernelGGL(k_grid_round_bf16, dim3(2048), blk, 0, s, nlu, F.ut64.p, F.ut16.p);
        }
        KRY_HIP(hipGetLastError());
        KRY_HIP(hipStreamSynchronize(s));
        F.lt64.release();
        F.ut64.release();
        F.dt64.release();
        // result and face buffers in FP32; faces start out unwritten
        KRY_TRY(F.yt32.alloc(nyt));
        KRY_TRY(F.ff32.alloc(nf));
        KRY_TRY(F.fb32.alloc(nf));
        hipLaunchKernelGGL(k_grid_fill_sentinel<float>, dim3(1024), blk, 0, s, nf, F.ff32.p);
        hipLaunchKernelGGL(k_grid_fill_sentinel<float>, dim3(1024), blk, 0, s, nf, F.fb32.p);
    } else {
        KRY_TRY(F.yt64.alloc(nyt));
        KRY_TRY(F.ff64.alloc(nf));
        KRY_TRY(F.fb64.alloc(nf));
        hipLaunchKernelGGL(k_grid_fill_sentinel<double>, dim3(1024), blk, 0, s, nf, F.ff64.p);
        hipLaunchKernelGGL(k_grid_fill_sentinel<double>, dim3(1024), blk, 0, s, nf, F.fb64.p);
    }
    KRY_HIP(hipGetLastError());
    F.grid = true;
    return KRY_OK;
}

int ilu_grid_setup(hipStream_t s, const MAT_ *A, const double *lu, const double *uinv,
                   IluFactor &F) {
    KRY_TRY(grid_tiling(A, F));
    const GridTiles &G = F.G;
    const int64_t steps = (int64_t)G.ntiles * G.S;
    const dim3 g((steps * 64 + 255) / 256), blk(256);
    if (A->bs == 1)
        hipLaunchKernelGGL(k_grid_pack<1>, g, blk, 0, s, G, A->rowptr.p, A->col.p, A->diag.p, lu,
                           uinv, F.lt64.p, F.ut64.p, F.dt64.p);
    else
        hipLaunchKernelGGL(k_grid_pack<3>, g, blk, 0, s, G, A->rowptr.p, A->col.p, A->diag.p, lu,
                           uinv, F.lt64.p, F.ut64.p, F.dt64.p);
    KRY_HIP(hipGetLastError());
    return grid_finish(s, A, F);
}

// Allocate a grid factor's tiling, planes, work buffers and tile counters
// for a later factor launch (FP64 only): F is complete once a factor launch
// on `faces` (sentinel-filled, steps * NF * bs^2) and `fctr` (zero) ran.
int grid_factor_prepare(hipStream_t s, const MAT_ *A, IluFactor &F, DBuf<double> &faces,
                        DBuf<int> &fctr) {
    if (!ilu_grid_can_factor(A)) return set_error(KRY_ERR_ARG, "grid factorization needs nx, ny >= 3");
    F.bs = A->bs;
    F.nb = A->nb;
    F.prec = KRY_PREC_F64;
    F.nlev_f = F.nlev_b = A->gnx + A->gny + A->gnz - 2;
    KRY_TRY(grid_tiling(A, F));
    const GridTiles &G = F.G;
    const int64_t steps = (int64_t)G.ntiles * G.S;
    KRY_TRY(faces.alloc(steps * G.NF * A->bs * A->bs));
    KRY_TRY(fctr.alloc(1));
    KRY_TRY(F.ctr.alloc(2 * GRID_QUEUES));
    KRY_HIP(hipMemsetAsync(F.ctr.p, 0, 2 * GRID_QUEUES * sizeof(int), s));
    return grid_finish(s, A, F);
}

// re-arm the work buffers of a prepared factor before a factor launch
int grid_factor_rearm(hipStream_t s, IluFactor &F, DBuf<double> &faces, DBuf<int> &fctr) {
    KRY_HIP(hipMemsetAsync(F.ut64.p, 0, F.ut64.bytes(), s));
    KRY_HIP(hipMemsetAsync(F.dt64.p, 0, F.dt64.bytes(), s));
    hipLaunchKernelGGL(k_grid_fill_sentinel<double>, dim3(1024), dim3(256), 0, s,
                       (int64_t)faces.n, faces.p);
    KRY_HIP(hipMemsetAsync(fctr.p, 0, sizeof(int), s));
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

int grid_factor_desc(const MAT_ *A, const IluFactor &F, DBuf<double> &faces, DBuf<int> &fctr,
                     int wg0, FactorMulti &d, int *wgs) {
    d.G = F.G;
    d.rowptr = A->rowptr.p;
    d.val = A->val.p;
    d.lt = F.lt64.p;
    d.ut = F.ut64.p;
    d.dt = F.dt64.p;
    d.faces = faces.p;
    d.ctr = fctr.p;
    d.wg0 = wg0;
    *wgs = std::min(F.G.ntiles, 1024);
    return KRY_OK;
}

int grid_factor_multi(hipStream_t s, int bs, const FactorMulti *d_desc, int ngrid, int total_wgs,
                      int *err) {
    TimedScope t("ras_grid_factor", s);
    if (bs == 1)
        hipLaunchKernelGGL(k_grid_factor_multi<1>, dim3(total_wgs), dim3(64), 0, s, d_desc, ngrid, err);
    else
        hipLaunchKernelGGL(k_grid_factor_multi<3>, dim3(total_wgs), dim3(64), 0, s, d_desc, ngrid, err);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

bool ilu_grid_can_factor(const MAT_ *A) {
    return A->gnx >= 3 && A->gny >= 3 && A->gnz >= 1 && (A->bs == 1 || A->bs == 3);
}

int ilu_grid_factor_setup(hipStream_t s, const MAT_ *A, const double *d_val, IluFactor &F,
                          int *d_err) {
    if (!ilu_grid_can_factor(A)) return set_error(KRY_ERR_ARG, "grid factorization needs nx, ny >= 3");
    KRY_TRY(grid_tiling(A, F));
    const GridTiles &G = F.G;
    const int b2 = A->bs * A->bs;
    const int64_t steps = (int64_t)G.ntiles * G.S;
    // backward planes are written only where a cell exists
    KRY_HIP(hipMemsetAsync(F.ut64.p, 0, F.ut64.bytes(), s));
    KRY_HIP(hipMemsetAsync(F.dt64.p, 0, F.dt64.bytes(), s));
    DBuf<double> faces;
    DBuf<int> ctr;
    const int64_t nf = steps * G.NF * b2;
    KRY_TRY(faces.alloc(nf));
    KRY_TRY(ctr.alloc(1));
    hipLaunchKernelGGL(k_grid_fill_sentinel<double>, dim3(1024), dim3(256), 0, s, nf, faces.p);
    KRY_HIP(hipMemsetAsync(ctr.p, 0, sizeof(int), s));
    const int wgs = std::min(G.ntiles, 1024);
    {
        TimedScope t("ilu_grid_factor", s);
        if (A->bs == 1)
            hipLaunchKernelGGL(k_grid_factor<1>, dim3(wgs), dim3(64), 0, s, G, A->rowptr.p, d_val,
                               F.lt64.p, F.ut64.p, F.dt64.p, faces.p, ctr.p, d_err);
        else
            hipLaunchKernelGGL(k_grid_factor<3>, dim3(wgs), dim3(64), 0, s, G, A->rowptr.p, d_val,
                               F.lt64.p, F.ut64.p, F.dt64.p, faces.p, ctr.p, d_err);
    }
    KRY_HIP(hipGetLastError());
    // the face buffer and counter are freed on return
    KRY_HIP(hipStreamSynchronize(s));
    return grid_finish(s, A, F);
}

// ---------------------------------------------------------------------------
// sweeps: one workgroup per tile, wavefront-specialised
//   wave 0            compute: consumes one hyperplane step at a time from
//                     LDS, exchanges neighbour values across lanes, stores
//                     the step's results (one contiguous row per component)
//                     and publishes the face cells; it issues no loads
//   wave 1            boundary: polls the face buffers of the two upstream
//                     tiles and stages the values in LDS
//   waves 2, 3        loaders: copy each step's factor planes (and the
//                     forward's right-hand side, the backward's diagonal
//                     inverses and forward result) straight from global
//                     memory into an LDS ring with the gfx950 global-to-LDS
//                     DMA loads, several steps in flight per wavefront and
//                     no register staging; when a tile is done they re-arm
//                     the other sweep's face slots of that tile
// Ring slots carry the step's stamp (a running step count of the
// workgroup), so no slot is ever reset.  Four wavefronts per workgroup and
// one workgroup per CU (the ring fills the LDS) give every role a SIMD of
// its own: a spinning wavefront never takes issue slots from another.
// ---------------------------------------------------------------------------
// ring slots for steps of SB bytes (120 KiB of ring, 2 to 8 slots)
template <int SB>
constexpr int ring_slots() {
    return (122880 / SB) > 8 ? 8 : (122880 / SB) < 2 ? 2 : (122880 / SB);
}

typedef __attribute__((address_space(3))) void lds_void_t;

// global-to-LDS DMA of a contiguous block of BYTES (a multiple of 256) by
// one wavefront: whole 1 KiB pieces as 16 bytes per lane, then 256-byte
// pieces as 4 bytes per lane.  Lane l of a piece at offset o copies
// src + o + w l to dst + o + w l (w its width; the LDS address of a lane is
// the wave-uniform base plus w l).  Every instruction runs on the whole
// wavefront: the LDS base of an instruction must be wave-uniform, so none
// sits under a lane-dependent branch.  A block of BF16 planes with an odd
// plane count ends 128 bytes short of a multiple of 256: its DMA rounds up
// (pad256), reading 128 bytes past the block (the planes are allocated with
// that much slack) into a ring region sized for the rounded length.
constexpr int pad256(int bytes) { return (bytes + 255) / 256 * 256; }
constexpr int dma_count(int bytes) { return bytes / 1024 + (bytes % 1024) / 256; }
template <int BYTES>
__device__ __forceinline__ void dma_block(const void *src, char *dst, int lane) {
    static_assert(BYTES % 256 == 0, "256-byte pieces");
    const char *g = static_cast<const char *>(src);
    constexpr int N16 = BYTES / 1024, N4 = (BYTES % 1024) / 256;
#pragma unroll
    for (int q = 0; q < N16; q++)
        __builtin_amdgcn_global_load_lds(g + q * 1024 + lane * 16, (lds_void_t *)(dst + q * 1024),
                                         16, 0, 0);
#pragma unroll
    for (int q = 0; q < N4; q++) {
        const int o = N16 * 1024 + q * 256;
        __builtin_amdgcn_global_load_lds(g + o + lane * 4, (lds_void_t *)(dst + o), 4, 0, 0);
    }
}
// W bytes per lane (4 or 12) from each lane's own address into dst + S l,
// S = 4 for dwords and 16 for three-dword pieces (the DMA keeps a 16-byte
// stride per lane for those)
template <int W>
__device__ __forceinline__ void dma_piece(const void *src, char *dst) {
    static_assert(W == 4 || W == 12, "dword or three-dword pieces");
    if constexpr (W == 4)
        __builtin_amdgcn_global_load_lds(src, (lds_void_t *)(dst), 4, 0, 0);
    else
        __builtin_amdgcn_global_load_lds(src, (lds_void_t *)(dst), 12, 0, 0);
}
// wait until at most N vector memory instructions of this wavefront are
// outstanding (they complete in order, so every older one has landed)
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// value types of the ring: factor storage TF read as the compute type TC
template <typename TC, typename TF>
__device__ __forceinline__ TC cvt(TF v) { return static_cast<TC>(v); }
template <>
__device__ __forceinline__ float cvt<float, uint16_t>(uint16_t v) { return bf16_to_f32(v); }

// A cell's right-hand side (BS values of TIN, CB bytes) gathered by DMA in
// pieces of W bytes per lane: piece p of lane l at p 64 LS + l LS (LS the
// lane stride of the piece).  Component r of lane `lane` from those pieces.
template <typename TIN, int BS>
struct RhsStage {
    static constexpr int CB = BS * (int)sizeof(TIN);
    static constexpr int W = CB % 12 == 0 ? 12 : 4;
    static constexpr int LS = W == 12 ? 16 : 4;
    static constexpr int NP = CB / W;            // DMA instructions per step
    static constexpr int BYTES = NP * 64 * LS;
    static __device__ __forceinline__ uint32_t dword(const char *rb, int lane, int d) {
        const int off = 4 * d;
        return *reinterpret_cast<const uint32_t *>(rb + (off / W) * 64 * LS + lane * LS + off % W);
    }
    template <typename TC>
    static __device__ __forceinline__ TC value(const char *rb, int lane, int r) {
        if constexpr (sizeof(TIN) == 8) {
            const uint64_t u = (static_cast<uint64_t>(dword(rb, lane, 2 * r + 1)) << 32) |
                               dword(rb, lane, 2 * r);
            return static_cast<TC>(__longlong_as_double(static_cast<long long>(u)));
        } else {
            return static_cast<TC>(__uint_as_float(dword(rb, lane, r)));
        }
    }
    static __device__ __forceinline__ void load(const TIN *cell, char *dst) {
#pragma unroll
        for (int q = 0; q < NP; q++)
            dma_piece<W>(reinterpret_cast<const char *>(cell) + q * W, dst + q * 64 * LS);
    }
};

// LDS flag access from a wavefront with DMA loads in flight.  The
// compiler treats any LDS access as possibly aliasing the DMA's LDS writes
// and would drain every outstanding DMA first; these two touch only the
// flag word, so they are written as single LDS instructions (the read waits
// for its own result inside the same statement).
__device__ __forceinline__ int lds_flag_get(const int *p) {
    const unsigned a = (unsigned)(size_t)((const __attribute__((address_space(3))) int *)p);
    int v;
    asm volatile("ds_read_b32 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(v) : "v"(a) : "memory");
    return v;
}
__device__ __forceinline__ void lds_flag_put(int *p, int v) {
    const unsigned a = (unsigned)(size_t)((__attribute__((address_space(3))) int *)p);
    asm volatile("ds_write_b32 %0, %1\n\ts_waitcnt lgkmcnt(0)" : : "v"(a), "v"(v) : "memory");
}

// Loader loop of one tile: steps t = w, w + NLOAD, ... of S; issue(t) starts
// the DMA of step t into ring slot t % D (P instructions); at most K steps of
// this wavefront in flight; a step is stamped in full[] once its DMA landed.
// Slot t % D is free once the compute wavefront has consumed step t - D.
// The wait counts assume no other vector memory operation of the wavefront
// is outstanding when the loop starts.
template <int D, int P, int K, typename F>
__device__ __forceinline__ void loader_loop(int w, int S, int base, int *cons, int *full, int lane,
                                            int *err, F &&issue) {
    // the wave's vector memory counter holds at most 63 outstanding
    // instructions: every DMA of the K steps in flight must fit in it
    static_assert(K >= 1 && K <= 4 && K * P <= 63, "in-flight DMA within the vmcnt range");
    int next = w, done = w;
    uint32_t idle = 0;
    wait_vm<0>();
    while (done < S) {
        while (next < S && next - done < K * NLOAD &&
               __builtin_amdgcn_readfirstlane(lds_flag_get(cons)) >= base + next - D + 1) {
            issue(next);
            next += NLOAD;
        }
        const int inflight = (next - done) / NLOAD;
        if (inflight == 0) {   // the ring is full: wait for the compute wavefront
            if (++idle > 4 * SPIN_LIMIT) {
                __hip_atomic_store(err, ERR_STALL_FLAG, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        idle = 0;
        // the oldest step's DMA has landed once at most (inflight - 1) * P
        // newer instructions are outstanding
        if constexpr (K >= 4) { if (inflight == 4) wait_vm<(K >= 4 ? 3 * P : 0)>(); }
        if constexpr (K >= 3) { if (inflight == 3) wait_vm<(K >= 3 ? 2 * P : 0)>(); }
        if constexpr (K >= 2) { if (inflight == 2) wait_vm<(K >= 2 ? P : 0)>(); }
        if (inflight == 1) wait_vm<0>();
        if (lane == 0) lds_flag_put(&full[done % D], base + done);
        done += NLOAD;
    }
}

// acc -= B y for block b of the planes in v
template <int BS, typename TC, int NV>
__device__ __forceinline__ void block_sub(TC (&acc)[BS], const TC (&v)[NV], int b, const TC (&y)[BS]) {
#pragma unroll
    for (int r = 0; r < BS; r++)
#pragma unroll
        for (int c = 0; c < BS; c++) acc[r] -= v[b * BS * BS + r * BS + c] * y[c];
}

// value held by the next lower lane (UP = false) or the next higher lane
// (UP = true) of the wavefront, by whole-wave DPP shifts (no LDS traffic);
// the lane at the end of the wave receives 0
template <bool UP>
__device__ __forceinline__ int lane_shift1(int v) {
    return __builtin_amdgcn_update_dpp(0, v, UP ? 0x130 : 0x138, 0xF, 0xF, true);
}
template <bool UP>
__device__ __forceinline__ float lane_shift1(float v) {
    return __int_as_float(lane_shift1<UP>(__float_as_int(v)));
}
template <bool UP>
__device__ __forceinline__ double lane_shift1(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = lane_shift1<UP>(static_cast<int>(u & 0xffffffffll));
    const int hi = lane_shift1<UP>(static_cast<int>(u >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                static_cast<unsigned int>(lo));
}

// Boundary role.  Lane f of the NF face lanes serves face entry f; `src`
// points at that entry of the upstream tile at the step that produces the
// value for this tile's step 0 (nullptr when the upstream tile or the
// lane's line does not exist), consecutive steps are NF * BS values apart.
// The face cell of step t lies at offset t - lag along the lane's line.
//
// The wave is cut into G = 64 / NF groups of NF lanes; group g stages
// steps g, g + G, g + 2G, ... .  Every round probes each group's current
// step: its first lane (a j-face entry, from the J - 1 tile) and its last
// lane (a k-face entry, from the K - 1 tile) read the last word of their
// entry.  Only a group whose probes both show published values reads its
// NF entries in full; a group whose NF cells are all published (and whose
// ring slot has been consumed) stages them and moves on, the others probe
// again.  A waiting round thus costs two words per group instead of the
// NF * BS values of a full read: these agent-scope loads bypass the L2,
// and with every tile's boundary wavefront polling, full reads cost 11 to
// 14% of the sweep time at 256 x 256 x 128.
template <typename TC, int BS>
__device__ void boundary_role(int S, int nx, int base, int lane, int NF, const TC *src, int lag,
                              TC (&bring)[DB][NFACE][BS], int *bfull, int *bcons, int *err) {
    using U = typename Bits<TC>::U;
    const U *q = reinterpret_cast<const U *>(src);
    const int G = (64 / NF) < DB ? (64 / NF) : DB;
    const int f = lane % NF, g = lane / NF;
    const bool lane_ok = g < G;
    const uint64_t gmask = (NF >= 64 ? ~0ull : ((1ull << NF) - 1ull)) << (lane_ok ? g * NF : 0);
    const int64_t stride = (int64_t)NF * BS;
    int ts = g;
    bool failed = false;
    uint32_t idle = 0;
    for (;;) {
        const bool active = lane_ok && ts < S;
        if (__ballot(active) == 0) break;
        bool ready = active;
        TC vals[BS];
#pragma unroll
        for (int r = 0; r < BS; r++) vals[r] = TC(0);
        bool pr = true;
        if (active && (f == 0 || f == NF - 1) && !failed) {
            const int off = ts - lag;
            if (q != nullptr && off >= 0 && off < nx)
                pr = __hip_atomic_load(const_cast<U *>(q) + ts * stride + (BS - 1),
                                       __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT) != Bits<TC>::sentinel;
        }
        const uint64_t pb = __ballot(pr);
        const bool probed = lane_ok && ((pb >> (g * NF)) & 1ull) && ((pb >> (g * NF + NF - 1)) & 1ull);
        if (active && !probed) ready = false;
        if (active && probed) {
            const int off = ts - lag;
            if (q != nullptr && off >= 0 && off < nx) {
#pragma unroll
                for (int r = 0; r < BS; r++) {
                    const U u = failed ? Bits<TC>::qnan
                                       : __hip_atomic_load(const_cast<U *>(q) + ts * stride + r,
                                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    vals[r] = Bits<TC>::from(u);
                    ready = ready && u != Bits<TC>::sentinel;
                }
            }
            // the slot of step ts held step ts - DB: it must have been read
            ready = ready && lds_get(bcons) >= base + ts - DB + 1;
        }
        const bool go = active && (__ballot(ready) & gmask) == gmask;
        lds_acquire();
        if (go)
#pragma unroll
            for (int r = 0; r < BS; r++) bring[ts % DB][f][r] = vals[r];
        lds_release();
        if (go && f == 0) lds_put(&bfull[ts % DB], base + ts);
        if (go) ts += G;
        if (__ballot(go) != 0) {
            idle = 0;
            continue;
        }
        // no group could stage this round
        if ((++idle & 63u) == 0u && !failed) {
            const int e = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (e != 0 || idle > SPIN_LIMIT) {
                if (e == 0 && lane == 0)
                    __hip_atomic_store(err, ERR_STALL_FLAG, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                failed = true;   // stage NaNs from now on so the compute wave drains
            }
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// The next tile of this workgroup (same value in every wavefront).  Each
// role runs its own tile loop, so every wavefront passes the two barriers
// once per tile and once more at the end.
// next tile of this workgroup's queue (b % NQ), first to last or, for the
// backward sweep, last to first; -1 when the queue is empty.  Within a
// queue the tiles come in dependency order and every queue is served by at
// least one workgroup, so every taken tile's producers are running.
__device__ __forceinline__ int next_tile(const GridTiles &G, int *ctr, int *tile, bool rev,
                                         int blk) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const int q = blk % G.NQ;
        const int i = atomicAdd(ctr + q, 1);
        const int len = G.qoff[q + 1] - G.qoff[q];
        *tile = i < len ? G.qtiles[G.qoff[q] + (rev ? len - 1 - i : i)] : -1;
    }
    __syncthreads();
    return *tile;
}

// forward sweep of one grid; blk = this workgroup's index within the grid's
// workgroups (a multiple of GRID_QUEUES of them)
// b is read at cell (i, j, k) of the grid as b[(i + j vsJ + k vsK) BS + r]:
// vsJ = nx, vsK = nx ny for a whole grid, the caller's strides for a box of
// a larger grid
template <int BS, typename TF, typename TC, typename TIN>
__device__ __forceinline__ void grid_fwd_body(const GridTiles &G, const TF *__restrict__ Lt,
                                              const TIN *__restrict__ b, TC *yt, TC *ff, TC *fb,
                                              int *ctr, int *other_ctr, int *err, int blk,
                                              int64_t vsJ, int64_t vsK) {
    constexpr int B2 = BS * BS, NM = 3 * B2, NV = NM + BS;
    // ring step: NM factor planes of TF, then the step's right-hand-side
    // cells as gathered by the DMA pieces of RhsStage
    using RS = RhsStage<TIN, BS>;
    constexpr int PB = pad256(NM * 64 * (int)sizeof(TF));
    constexpr int SB = (PB + RS::BYTES + 15) / 16 * 16;
    constexpr int D = ring_slots<SB>();
    constexpr int P = dma_count(PB) + RS::NP;                  // DMA instructions per step
    constexpr int K = (D / NLOAD) < (63 / P) ? (D / NLOAD) : (63 / P);
    __shared__ __attribute__((aligned(16))) char ringb[D * SB];
    __shared__ TC bring[DB][NFACE][BS];
    __shared__ int full[D], bfull[DB], cons, bcons, tile;
    // wave-uniform role index (an SGPR), so the roles are real branches
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (blk == 0 && (int)threadIdx.x < G.NQ) other_ctr[threadIdx.x] = 0;
    if (threadIdx.x < D) full[threadIdx.x] = -1;
    if (threadIdx.x < DB) bfull[threadIdx.x] = -1;
    if (threadIdx.x == 0) {
        cons = 0;
        bcons = 0;
    }
    const int TJ = G.TJ, TK = G.TK, NF = G.NF, nx = G.nx, S = G.S;
    const int64_t sJ = G.nx, sK = (int64_t)G.nx * G.ny;
    const int jj = lane % TJ, kk = lane / TJ;
    if (wave == 0) {
        // ---- compute ----
        // face entries this lane publishes (high faces feed tiles J+1, K+1)
        const int fj = jj == TJ - 1 && kk < TK ? kk : -1;
        const int fk = kk == TK - 1 ? TK + jj : -1;
        const int oj = fj * BS, ok = fk * BS;
        for (int base = 0;; base += S) {
            const int T = next_tile(G, ctr, &tile, false, blk);
            if (T < 0) break;
            TC *yrow = yt + (int64_t)T * S * BS * 64 + lane;
            TC *frow = ff + (int64_t)T * S * NF * BS;
            // the right-hand side of a lane outside the grid, or of a step
            // outside its line, is zero (its staged words are not loaded)
            const int JK = G.order[T];
            const bool lane_ok = lane < TJ * TK && (JK & 0xffff) * TJ + jj < G.ny &&
                                 (JK >> 16) * TK + kk < G.nz;
            auto read_step = [&](int t, TC (&v)[NV]) {
                const char *sl = ringb + (t % D) * SB;
                const TF *pl = reinterpret_cast<const TF *>(sl);
#pragma unroll
                for (int e = 0; e < NM; e++) v[e] = cvt<TC, TF>(pl[e * 64 + lane]);
                const int i = t - jj - kk;
                const bool ok = lane_ok && i >= 0 && i < nx;
#pragma unroll
                for (int r = 0; r < BS; r++) {
                    const TC x = RS::template value<TC>(sl + PB, lane, r);
                    v[NM + r] = ok ? x : TC(0);
                }
            };
            TC yp[BS];
#pragma unroll
            for (int r = 0; r < BS; r++) yp[r] = TC(0);
            int pa = -2, pb = -2;   // stamps of the next step, read one step early
            // step t computes with the planes in vc and reads the planes of
            // step t + 1 into vn; the two arrays swap roles every step
            auto step = [&](int t, const TC (&vc)[NV], TC (&vn)[NV]) {
                const int st = base + t, bslot = t % DB;
                const bool more = t + 1 < S;
                // this step's boundary and the next step's planes: one poll,
                // skipped when the stamps read during the previous step show both
                lds_wait_pair_pre(pa, pb, &bfull[bslot], st, &full[(t + 1) % D], more ? st + 1 : -1,
                                  err);
                TC yj[BS], yk[BS];
#pragma unroll
                for (int r = 0; r < BS; r++) {
                    const TC bj = bring[bslot][kk < TK ? kk : 0][r];
                    const TC bk = bring[bslot][TK + jj][r];
                    yj[r] = lane_shift1<false>(yp[r]);
                    yk[r] = __shfl_up(yp[r], TJ, 64);
                    if (jj == 0) yj[r] = bj;
                    if (kk == 0) yk[r] = bk;
                }
                if (more) read_step(t + 1, vn);
                pa = lds_get(&bfull[(t + 1) % DB]);
                pb = t + 2 < S ? lds_get(&full[(t + 2) % D]) : -1;
                TC acc[BS];
#pragma unroll
                for (int r = 0; r < BS; r++) acc[r] = vc[NM + r];
                block_sub<BS>(acc, vc, 0, yk);
                block_sub<BS>(acc, vc, 1, yj);
                block_sub<BS>(acc, vc, 2, yp);
#pragma unroll
                for (int r = 0; r < BS; r++) {
                    yp[r] = acc[r];
                    yrow[(t * BS + r) * 64] = acc[r];
                }
                {
                    TC pub[BS];
                    unsentinel<TC, BS>(acc, pub);
                    TC *ft = frow + (int64_t)t * NF * BS;
                    if (fj >= 0) publish_checked<TC, BS>(ft + oj, pub);
                    if (fk >= 0) publish_checked<TC, BS>(ft + ok, pub);
                }
                // every LDS read of this step has returned: hand both slots back
                lds_release();
                if (lane == 0) {
                    lds_put(&bcons, st + 1);
                    lds_put(&cons, more ? st + 2 : st + 1);
                }
            };
            TC va[NV], vb[NV];
            lds_wait_eq(&full[0], base, err);
            read_step(0, va);
            int t = 0;
            for (; t + 1 < S; t += 2) {
                step(t, va, vb);
                step(t + 1, vb, va);
            }
            if (t < S) step(t, va, vb);
        }
    } else if (wave == 1) {
        // ---- boundary: faces of tiles (J-1, K) and (J, K-1) ----
        const int f = lane % NF;
        for (int base = 0;; base += S) {
            const int T = next_tile(G, ctr, &tile, false, blk);
            if (T < 0) break;
            const int JK = G.order[T];
            const int J = JK & 0xffff, K = JK >> 16;
            const TC *src = nullptr;
            int lag = 0;
            if (f < TK) {                  // j-face of lane kk = f: lane (TJ-1, f) of (J-1, K)
                if (J > 0 && K * TK + f < G.nz)
                    src = ff + (((int64_t)G.tidx[(J - 1) * G.NK + K] * S + (TJ - 1)) * NF + f) * BS;
                lag = f;
            } else {                       // k-face of lane jj = q: lane (q, TK-1) of (J, K-1)
                const int q = f - TK;
                if (K > 0 && J * TJ + q < G.ny)
                    src = ff + (((int64_t)G.tidx[J * G.NK + K - 1] * S + (TK - 1)) * NF + f) * BS;
                lag = q;
            }
            boundary_role<TC, BS>(S, nx, base, lane, NF, src, lag, bring, bfull, &bcons, err);
        }
    } else {
        // ---- loaders: DMA of steps w, w + NLOAD, ... ----
        const int w = wave - 2;
        for (int base = 0;; base += S) {
            const int T = next_tile(G, ctr, &tile, false, blk);
            if (T < 0) break;
            const int JK = G.order[T];
            const int j = (JK & 0xffff) * TJ + jj, k = (JK >> 16) * TK + kk;
            const bool lane_ok = lane < TJ * TK && j < G.ny && k < G.nz;
            const int64_t cl = lane_ok ? vsJ * j + vsK * k : 0;
            const TF *lb = Lt + (int64_t)T * S * NM * 64;
            // every step issues the same P instructions (the wait counts
            // assume it): a lane with no cell loads b[0], which the compute
            // wavefront discards
            auto issue = [&](int t) {
                char *sl = ringb + (t % D) * SB;
                dma_block<PB>(lb + (int64_t)t * NM * 64, sl, lane);
                const int i = t - jj - kk;
                const bool ok = lane_ok && i >= 0 && i < nx;
                RS::load(b + (ok ? (cl + i) * BS : 0), sl + PB);
            };
            loader_loop<D, P, K>(w, S, base, &cons, full, lane, err, issue);
            // the backward sweep's face slots of this tile start unwritten
            TC *fr = fb + (int64_t)T * S * NF * BS;
            for (int64_t e = w * 64 + lane; e < (int64_t)S * NF * BS; e += NLOAD * 64)
                fr[e] = sentinel_value<TC>();
        }
    }
}

template <int BS, typename TF, typename TD, typename TC, typename TO>
__device__ __forceinline__ void grid_bwd_body(const GridTiles &G, const TF *__restrict__ Ut,
                                              const TD *__restrict__ Dt, TC *yt, TC *fb, TC *ff,
                                              int *ctr, int *other_ctr, int *err, int blk) {
    constexpr int B2 = BS * BS, NM = 3 * B2, NV = NM + B2 + BS;
    // ring step: NM factor planes of TF, B2 diagonal-inverse planes of TD,
    // BS forward-result planes of TC
    constexpr int PB = pad256(NM * 64 * (int)sizeof(TF)), DBY = B2 * 64 * (int)sizeof(TD);
    constexpr int YB = BS * 64 * (int)sizeof(TC);
    constexpr int SB = PB + DBY + YB;
    constexpr int D = ring_slots<SB>();
    constexpr int P = dma_count(PB) + dma_count(DBY) + dma_count(YB);
    constexpr int K = (D / NLOAD) < (63 / P) ? (D / NLOAD) : (63 / P);
    __shared__ __attribute__((aligned(16))) char ringb[D * SB];
    __shared__ TC bring[DB][NFACE][BS];
    __shared__ int full[D], bfull[DB], cons, bcons, tile;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (blk == 0 && (int)threadIdx.x < G.NQ) other_ctr[threadIdx.x] = 0;
    if (threadIdx.x < D) full[threadIdx.x] = -1;
    if (threadIdx.x < DB) bfull[threadIdx.x] = -1;
    if (threadIdx.x == 0) {
        cons = 0;
        bcons = 0;
    }
    const int TJ = G.TJ, TK = G.TK, NF = G.NF, nx = G.nx, S = G.S;
    const int jj = lane % TJ, kk = lane / TJ;
    if (wave == 0) {
        // ---- compute ----
        // face entries this lane publishes (low faces feed tiles J-1, K-1)
        const int fj = jj == 0 && kk < TK ? kk : -1;
        const int fk = kk == 0 ? TK + jj : -1;
        const int oj = fj * BS, ok = fk * BS;
        for (int base = 0;; base += S) {
            const int T = next_tile(G, ctr, &tile, true, blk);   // reverse tile order
            if (T < 0) break;
            TC *yrow = yt + (int64_t)T * S * BS * 64 + lane;
            TC *frow = fb + (int64_t)T * S * NF * BS;
            auto read_step = [&](int t, TC (&v)[NV]) {
                const char *sl = ringb + (t % D) * SB;
                const TF *pu = reinterpret_cast<const TF *>(sl);
                const TD *pd = reinterpret_cast<const TD *>(sl + PB);
                const TC *py = reinterpret_cast<const TC *>(sl + PB + DBY);
#pragma unroll
                for (int e = 0; e < NM; e++) v[e] = cvt<TC, TF>(pu[e * 64 + lane]);
#pragma unroll
                for (int e = 0; e < B2; e++) v[NM + e] = static_cast<TC>(pd[e * 64 + lane]);
#pragma unroll
                for (int r = 0; r < BS; r++) v[NM + B2 + r] = py[r * 64 + lane];
            };
            TC xp[BS];
#pragma unroll
            for (int r = 0; r < BS; r++) xp[r] = TC(0);
            int pa = -2, pb = -2;   // stamps of the next step, read one step early
            auto step = [&](int t, const TC (&vc)[NV], TC (&vn)[NV]) {
                const int st = base + t, bslot = t % DB;
                const bool more = t + 1 < S;
                lds_wait_pair_pre(pa, pb, &bfull[bslot], st, &full[(t + 1) % D], more ? st + 1 : -1,
                                  err);
                TC xj[BS], xk[BS];
#pragma unroll
                for (int r = 0; r < BS; r++) {
                    const TC bj = bring[bslot][kk < TK ? kk : 0][r];
                    const TC bk = bring[bslot][TK + jj][r];
                    xj[r] = lane_shift1<true>(xp[r]);
                    xk[r] = __shfl_down(xp[r], TJ, 64);
                    if (jj == TJ - 1) xj[r] = bj;
                    if (kk == TK - 1) xk[r] = bk;
                }
                if (more) read_step(t + 1, vn);
                pa = lds_get(&bfull[(t + 1) % DB]);
                pb = t + 2 < S ? lds_get(&full[(t + 2) % D]) : -1;
                TC acc[BS];
#pragma unroll
                for (int r = 0; r < BS; r++) acc[r] = vc[NM + B2 + r];
                block_sub<BS>(acc, vc, 0, xp);
                block_sub<BS>(acc, vc, 1, xj);
                block_sub<BS>(acc, vc, 2, xk);
                TC res[BS];
#pragma unroll
                for (int r = 0; r < BS; r++) {
                    TC sum = TC(0);
#pragma unroll
                    for (int q = 0; q < BS; q++) sum += vc[NM + r * BS + q] * acc[q];
                    res[r] = sum;
                }
                // neighbours consume the value as the caller's output type
#pragma unroll
                for (int r = 0; r < BS; r++) {
                    xp[r] = static_cast<TC>(static_cast<TO>(res[r]));
                    yrow[((S - 1 - t) * BS + r) * 64] = res[r];
                }
                {
                    TC pub[BS];
                    unsentinel<TC, BS>(xp, pub);
                    TC *ft = frow + (int64_t)t * NF * BS;
                    if (fj >= 0) publish_checked<TC, BS>(ft + oj, pub);
                    if (fk >= 0) publish_checked<TC, BS>(ft + ok, pub);
                }
                lds_release();
                if (lane == 0) {
                    lds_put(&bcons, st + 1);
                    lds_put(&cons, more ? st + 2 : st + 1);
                }
            };
            TC va[NV], vb[NV];
            lds_wait_eq(&full[0], base, err);
            read_step(0, va);
            int t = 0;
            for (; t + 1 < S; t += 2) {
                step(t, va, vb);
                step(t + 1, vb, va);
            }
            if (t < S) step(t, va, vb);
        }
    } else if (wave == 1) {
        // ---- boundary: faces of tiles (J+1, K) and (J, K+1) ----
        const int f = lane % NF;
        for (int base = 0;; base += S) {
            const int T = next_tile(G, ctr, &tile, true, blk);
            if (T < 0) break;
            const int JK = G.order[T];
            const int J = JK & 0xffff, K = JK >> 16;
            const TC *src = nullptr;
            int lag = 0;
            if (f < TK) {                  // j-face of lane (TJ-1, f): lane (0, f) of (J+1, K)
                if (J + 1 < G.NJ && K * TK + f < G.nz)
                    src = fb + (((int64_t)G.tidx[(J + 1) * G.NK + K] * S + (TJ - 1)) * NF + f) * BS;
                lag = TK - 1 - f;
            } else {                       // k-face of lane (q, TK-1): lane (q, 0) of (J, K+1)
                const int q = f - TK;
                if (K + 1 < G.NK && J * TJ + q < G.ny)
                    src = fb + (((int64_t)G.tidx[J * G.NK + K + 1] * S + (TK - 1)) * NF + f) * BS;
                lag = TJ - 1 - q;
            }
            boundary_role<TC, BS>(S, nx, base, lane, NF, src, lag, bring, bfull, &bcons, err);
        }
    } else {
        // ---- loaders: DMA of U blocks, diagonal inverses, forward result ----
        const int w = wave - 2;
        for (int base = 0;; base += S) {
            const int T = next_tile(G, ctr, &tile, true, blk);
            if (T < 0) break;
            const TF *ub = Ut + (int64_t)T * S * NM * 64;
            const TD *db = Dt + (int64_t)T * S * B2 * 64;
            const TC *yb = yt + (int64_t)T * S * BS * 64;
            auto issue = [&](int t) {
                char *sl = ringb + (t % D) * SB;
                dma_block<PB>(ub + (int64_t)t * NM * 64, sl, lane);
                dma_block<DBY>(db + (int64_t)t * B2 * 64, sl + PB, lane);
                // the forward result of the same cells: forward step S - 1 - t
                dma_block<YB>(yb + (int64_t)(S - 1 - t) * BS * 64, sl + PB + DBY, lane);
            };
            loader_loop<D, P, K>(w, S, base, &cons, full, lane, err, issue);
            // the forward sweep's face slots of this tile start unwritten
            TC *fr = ff + (int64_t)T * S * NF * BS;
            for (int64_t e = w * 64 + lane; e < (int64_t)S * NF * BS; e += NLOAD * 64)
                fr[e] = sentinel_value<TC>();
        }
    }
}

// Copy the tile-step-major result to natural order, with the caller's
// epilogue (the add modes of ilu_apply): one block per (tile, 8 steps),
// reads in contiguous 64-lane rows.
// cells of a grid written by an untile: those with i in [i0, i1), j in
// [j0, j1), k in [k0, k1), at (i + j vsJ + k vsK) BS of the output
struct UntileBox {
    int i0, i1, j0, j1, k0, k1;
    int64_t vsJ, vsK;
};

// natural-order copy of the tile-step result of one grid with the fused
// epilogue, restricted to the cells of `box` (all of them for a whole grid;
// a subdomain's owned cells under RAS)
template <int BS, typename TC, typename TO, int ADD, typename TAI, typename TAO>
__device__ __forceinline__ void grid_untile_body(const GridTiles &G, const TC *__restrict__ yt,
                                                 TO *__restrict__ xo,
                                                 const TAI *__restrict__ add_in,
                                                 TAO *__restrict__ add_out, const UntileBox &box,
                                                 int blk) {
    const int nchunk = (G.S + 7) / 8;
    const int T = blk / nchunk, t0 = (blk % nchunk) * 8;
    const int lane = threadIdx.x & 63;
    const int JK = G.order[T];
    const int jj = lane % G.TJ, kk = lane / G.TJ;
    const int j = (JK & 0xffff) * G.TJ + jj, k = (JK >> 16) * G.TK + kk;
    if (lane >= G.TJ * G.TK || j >= G.ny || k >= G.nz) return;
    if (j < box.j0 || j >= box.j1 || k < box.k0 || k >= box.k1) return;
    const int64_t cl = box.vsJ * j + box.vsK * k;
    for (int t = t0 + (threadIdx.x >> 6); t < t0 + 8 && t < G.S; t += 4) {
        const int i = t - jj - kk;
        if (i < box.i0 || i >= box.i1 || i >= G.nx) continue;
        const int64_t c = cl + i;
        const TC *src = yt + ((int64_t)T * G.S + t) * BS * 64 + lane;
#pragma unroll
        for (int r = 0; r < BS; r++) {
            const TC v = src[r * 64];
            if (ADD == 0) xo[c * BS + r] = static_cast<TO>(v);
            if (ADD == 1) add_out[c * BS + r] = static_cast<TAO>(add_in[c * BS + r]) + static_cast<TAO>(v);
            if (ADD == 2) {
                const TC base0 = (r == 0) ? static_cast<TC>(add_in[c]) : TC(0);
                add_out[c * BS + r] = static_cast<TAO>(base0 + v);
            }
        }
    }
}

template <int BS, typename TF, typename TC, typename TIN>
__global__ __launch_bounds__(GWG) void k_grid_fwd(GridTiles G, const TF *__restrict__ Lt,
                                                  const TIN *__restrict__ b, TC *yt, TC *ff,
                                                  TC *fb, int *ctr, int *other_ctr, int *err) {
    grid_fwd_body<BS, TF, TC, TIN>(G, Lt, b, yt, ff, fb, ctr, other_ctr, err, blockIdx.x, G.nx,
                                   (int64_t)G.nx * G.ny);
}

template <int BS, typename TF, typename TD, typename TC, typename TO>
__global__ __launch_bounds__(GWG) void k_grid_bwd(GridTiles G, const TF *__restrict__ Ut,
                                                  const TD *__restrict__ Dt, TC *yt, TC *fb,
                                                  TC *ff, int *ctr, int *other_ctr, int *err) {
    grid_bwd_body<BS, TF, TD, TC, TO>(G, Ut, Dt, yt, fb, ff, ctr, other_ctr, err, blockIdx.x);
}

// Natural-order copy of a whole grid's tile-step result with the epilogue
// of ilu_apply.  A block takes UNT_CH consecutive steps of one tile (16: a
// 25 KB LDS tile, six blocks per CU; 32 steps, three blocks per CU, took
// 50% longer at 256 x 256 x 128): it reads
// them as contiguous rows into LDS, line by line (line = lane of the tile),
// then writes each line's UNT_CH cells as one contiguous run, so a wavefront
// store covers one line's 16 cells (384 contiguous bytes in FP64) instead
// of one cell of 64 different lines.  Blocks b,
// b + 8, b + 16, ... run on one XCD; the chunks of one tile are given to
// consecutive blocks of the same XCD, so the cache line that two chunks of
// a line share is completed in that XCD's L2 before it is written back.
constexpr int UNT_CH = 16;

template <int BS, typename TC, typename TO, int ADD, typename TAI, typename TAO>
__global__ __launch_bounds__(256) void k_grid_untile(GridTiles G, const TC *__restrict__ yt,
                                                     TO *__restrict__ xo,
                                                     const TAI *__restrict__ add_in,
                                                     TAO *__restrict__ add_out) {
    constexpr int LV = UNT_CH * BS;   // values of one line in a chunk
    constexpr int LS = LV + 1;        // odd LDS stride: the row writes hit distinct banks
    __shared__ TC lds[64 * LS];
    const int nchunk = (G.S + UNT_CH - 1) / UNT_CH;
    const int xcd = blockIdx.x % 8, idx = blockIdx.x / 8;
    const int T = 8 * (idx / nchunk) + xcd, c = idx % nchunk;
    if (T >= G.ntiles) return;
    const int t0 = c * UNT_CH, nt = min(UNT_CH, G.S - t0);
    const TC *src = yt + ((int64_t)T * G.S + t0) * BS * 64;
    for (int e = threadIdx.x; e < nt * BS * 64; e += 256) {
        const int tl = e / (BS * 64), r = (e / 64) % BS, ln = e % 64;
        lds[ln * LS + tl * BS + r] = src[e];
    }
    __syncthreads();
    const int JK = G.order[T];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t vsK = (int64_t)G.nx * G.ny;
    for (int l = wv; l < G.TJ * G.TK; l += 4) {
        const int jj = l % G.TJ, kk = l / G.TJ;
        const int j = (JK & 0xffff) * G.TJ + jj, k = (JK >> 16) * G.TK + kk;
        if (j >= G.ny || k >= G.nz) continue;
        const int xs = t0 - jj - kk;   // x of the line's first cell in this chunk
        const int64_t cl = vsK * k + (int64_t)G.nx * j;
        for (int e = lane; e < nt * BS; e += 64) {
            const int x = xs + e / BS, r = e % BS;
            if (x < 0 || x >= G.nx) continue;
            const TC v = lds[l * LS + e];
            const int64_t o = (cl + x) * BS + r;
            if (ADD == 0) xo[o] = static_cast<TO>(v);
            if (ADD == 1) add_out[o] = static_cast<TAO>(add_in[o]) + static_cast<TAO>(v);
            if (ADD == 2) {
                const TC base0 = (r == 0) ? static_cast<TC>(add_in[cl + x]) : TC(0);
                add_out[o] = static_cast<TAO>(base0 + v);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// several independent grids in one launch (the subdomains of RAS): grid g
// owns the workgroups [wg0, wg0 + wgs) of each kernel (multiples of
// GRID_QUEUES, so a workgroup's queue, and XCD, keep their mapping)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_grid(const GridMulti *__restrict__ d, int ngrid, int blk,
                                         int GridMulti::*wg0) {
    int g = 0;
    while (g + 1 < ngrid && blk >= d[g + 1].*wg0) g++;
    return g;
}

template <int BS>
__global__ __launch_bounds__(GWG) void k_grid_fwd_multi(const GridMulti *__restrict__ d, int ngrid,
                                                        const double *__restrict__ v, int *err) {
    const int g = find_grid(d, ngrid, blockIdx.x, &GridMulti::wg0);
    const GridMulti D = d[g];
    grid_fwd_body<BS, double, double, double>(D.G, D.lt, v + D.boff, D.yt, D.ff, D.fb, D.ctr,
                                              D.ctr + D.G.NQ, err, blockIdx.x - D.wg0, D.vsJ,
                                              D.vsK);
}

template <int BS>
__global__ __launch_bounds__(GWG) void k_grid_bwd_multi(const GridMulti *__restrict__ d, int ngrid,
                                                        int *err) {
    const int g = find_grid(d, ngrid, blockIdx.x, &GridMulti::wg0);
    const GridMulti D = d[g];
    grid_bwd_body<BS, double, double, double, double>(D.G, D.ut, D.dt, D.yt, D.fb, D.ff,
                                                      D.ctr + D.G.NQ, D.ctr, err,
                                                      blockIdx.x - D.wg0);
}

template <int BS>
__global__ __launch_bounds__(256) void k_grid_untile_multi(const GridMulti *__restrict__ d,
                                                           int ngrid, double *__restrict__ z) {
    const int g = find_grid(d, ngrid, blockIdx.x, &GridMulti::ub0);
    const GridMulti D = d[g];
    const UntileBox box{D.oi0, D.oi1, D.oj0, D.oj1, D.ok0, D.ok1, D.vsJ, D.vsK};
    grid_untile_body<BS, double, double, 0, double, double>(D.G, D.yt, z + D.boff, nullptr,
                                                            nullptr, box, blockIdx.x - D.ub0);
}

int grid_multi_launch_size(const IluFactor &F, int *wgs, int *untile_blocks) {
    if (!F.grid) return set_error(KRY_ERR_ARG, "grid_multi: not a grid-tiled factor");
    *wgs = F.G.NQ * std::max(1, std::min(F.G.qmax, 512 / F.G.NQ));
    *untile_blocks = F.G.ntiles * ((F.G.S + 7) / 8);
    return KRY_OK;
}

int grid_multi_desc(const IluFactor &F, int64_t boff, int64_t vsJ, int64_t vsK, const int own[6],
                    int wg0, int ub0, GridMulti &d) {
    if (!F.grid || F.prec != KRY_PREC_F64)
        return set_error(KRY_ERR_ARG, "grid_multi: needs an FP64 grid-tiled factor");
    d.G = F.G;
    d.lt = F.lt64.p;
    d.ut = F.ut64.p;
    d.dt = F.dt64.p;
    d.yt = F.yt64.p;
    d.ff = F.ff64.p;
    d.fb = F.fb64.p;
    d.ctr = F.ctr.p;
    d.boff = boff;
    d.vsJ = vsJ;
    d.vsK = vsK;
    d.oi0 = own[0];
    d.oi1 = own[1];
    d.oj0 = own[2];
    d.oj1 = own[3];
    d.ok0 = own[4];
    d.ok1 = own[5];
    d.wg0 = wg0;
    d.ub0 = ub0;
    return KRY_OK;
}

int grid_multi_apply(hipStream_t s, int bs, const GridMulti *d_desc, int ngrid, int total_wgs,
                     int total_untile, const double *v, double *z, int *err) {
    {
        TimedScope t("ras_ilu_fwd", s);
        if (bs == 1)
            hipLaunchKernelGGL(k_grid_fwd_multi<1>, dim3(total_wgs), dim3(GWG), 0, s, d_desc, ngrid, v, err);
        else
            hipLaunchKernelGGL(k_grid_fwd_multi<3>, dim3(total_wgs), dim3(GWG), 0, s, d_desc, ngrid, v, err);
    }
    {
        TimedScope t("ras_ilu_bwd", s);
        if (bs == 1)
            hipLaunchKernelGGL(k_grid_bwd_multi<1>, dim3(total_wgs), dim3(GWG), 0, s, d_desc, ngrid, err);
        else
            hipLaunchKernelGGL(k_grid_bwd_multi<3>, dim3(total_wgs), dim3(GWG), 0, s, d_desc, ngrid, err);
    }
    if (bs == 1)
        hipLaunchKernelGGL(k_grid_untile_multi<1>, dim3(total_untile), dim3(256), 0, s, d_desc, ngrid, z);
    else
        hipLaunchKernelGGL(k_grid_untile_multi<3>, dim3(total_untile), dim3(256), 0, s, d_desc, ngrid, z);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

// ---------------------------------------------------------------------------
// dispatch (same type combinations as the level-scheduled sweeps)
// ---------------------------------------------------------------------------
template <int BS, typename TF, typename TD, typename TC, typename TIN, typename TO, int ADD,
          typename TAI, typename TAO>
static int grid_pair(hipStream_t s, IluFactor &F, const TF *lt, const TF *ut, const TD *dt,
                     TC *yt, TC *ff, TC *fb, const TIN *b, TO *xo, const TAI *add_in,
                     TAO *add_out, int *err) {
    // one workgroup per tile in flight (LDS-bound, 256 CUs): NQ workgroups
    // per queue position, so every queue has a workgroup per tile up to
    // the cap, and always at least one
    const int wgs = F.G.NQ * std::max(1, std::min(F.G.qmax, 512 / F.G.NQ));
    {
        TimedScope t(F.timer_fwd ? F.timer_fwd : sweep_timer_name(true, BS, sizeof(TF), ADD), s);
        hipLaunchKernelGGL((k_grid_fwd<BS, TF, TC, TIN>), dim3(wgs), dim3(GWG), 0, s, F.G, lt, b,
                           yt, ff, fb, F.ctr.p, F.ctr.p + F.G.NQ, err);
    }
    {
        TimedScope t(F.timer_bwd ? F.timer_bwd : sweep_timer_name(false, BS, sizeof(TF), 0), s);
        hipLaunchKernelGGL((k_grid_bwd<BS, TF, TD, TC, TO>), dim3(wgs), dim3(GWG), 0, s, F.G, ut,
                           dt, yt, fb, ff, F.ctr.p + F.G.NQ, F.ctr.p, err);
    }
    {
        TimedScope t("ilu_grid_untile", s);
        const int nchunk = (F.G.S + UNT_CH - 1) / UNT_CH;
        hipLaunchKernelGGL((k_grid_untile<BS, TC, TO, ADD, TAI, TAO>),
                           dim3(8 * ((F.G.ntiles + 7) / 8) * nchunk),
                           dim3(256), 0, s, F.G, yt, xo, add_in, add_out);
    }
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

template <int BS, typename TIN, typename TO>
static int grid_typed(hipStream_t s, IluFactor &F, const TIN *b, TO *xo, int add_mode,
                      const void *add_in, void *add_out, int *err) {
    if (F.prec == KRY_PREC_F64) {
        using TC = double;
        TC *yt = F.yt64.p, *ff = F.ff64.p, *fb = F.fb64.p;
        if (add_mode == 0)
            return grid_pair<BS, double, double, TC, TIN, TO, 0, double, double>(
                s, F, F.lt64.p, F.ut64.p, F.dt64.p, yt, ff, fb, b, xo, nullptr, nullptr, err);
        if (add_mode == 1)
            return grid_pair<BS, double, double, TC, TIN, TO, 1, TO, TO>(
                s, F, F.lt64.p, F.ut64.p, F.dt64.p, yt, ff, fb, b, xo, (const TO *)add_in,
                (TO *)add_out, err);
        return grid_pair<BS, double, double, TC, TIN, TO, 2, TC, double>(
            s, F, F.lt64.p, F.ut64.p, F.dt64.p, yt, ff, fb, b, xo, (const TC *)add_in,
            (double *)add_out, err);
    }
    using TC = float;
    TC *yt = F.yt32.p, *ff = F.ff32.p, *fb = F.fb32.p;
    if (F.prec == KRY_PREC_F32) {
        if (add_mode == 0)
            return grid_pair<BS, float, float, TC, TIN, TO, 0, float, float>(
                s, F, F.lt32.p, F.ut32.p, F.dt32.p, yt, ff, fb, b, xo, nullptr, nullptr, err);
        if (add_mode == 1)
            return grid_pair<BS, float, float, TC, TIN, TO, 1, TO, TO>(
                s, F, F.lt32.p, F.ut32.p, F.dt32.p, yt, ff, fb, b, xo, (const TO *)add_in,
                (TO *)add_out, err);
        return grid_pair<BS, float, float, TC, TIN, TO, 2, TC, double>(
            s, F, F.lt32.p, F.ut32.p, F.dt32.p, yt, ff, fb, b, xo, (const TC *)add_in,
            (double *)add_out, err);
    }
    if (add_mode == 0)
        return grid_pair<BS, uint16_t, float, TC, TIN, TO, 0, float, float>(
            s, F, F.lt16.p, F.ut16.p, F.dt32.p, yt, ff, fb, b, xo, nullptr, nullptr, err);
    if (add_mode == 1)
        return grid_pair<BS, uint16_t, float, TC, TIN, TO, 1, TO, TO>(
            s, F, F.lt16.p, F.ut16.p, F.dt32.p, yt, ff, fb, b, xo, (const TO *)add_in,
            (TO *)add_out, err);
    return grid_pair<BS, uint16_t, float, TC, TIN, TO, 2, TC, double>(
        s, F, F.lt16.p, F.ut16.p, F.dt32.p, yt, ff, fb, b, xo, (const TC *)add_in,
        (double *)add_out, err);
}

template <int BS>
static int grid_bs(hipStream_t s, IluFactor &F, const void *b, int in_type, void *xscr,
                   int out_type, int add_mode, const void *add_in, void *add_out, int *err) {
    if (in_type == 0 && out_type == 0)
        return grid_typed<BS>(s, F, (const double *)b, (double *)xscr, add_mode, add_in, add_out, err);
    if (in_type == 0 && out_type == 1)
        return grid_typed<BS>(s, F, (const double *)b, (float *)xscr, add_mode, add_in, add_out, err);
    if (in_type == 1 && out_type == 0)
        return grid_typed<BS>(s, F, (const float *)b, (double *)xscr, add_mode, add_in, add_out, err);
    return grid_typed<BS>(s, F, (const float *)b, (float *)xscr, add_mode, add_in, add_out, err);
}

int ilu_grid_apply(hipStream_t s, IluFactor &F, const void *b, int in_type, void *xscr,
                   int out_type, int add_mode, const void *add_in, void *add_out, int *d_err) {
    if (F.bs == 1) return grid_bs<1>(s, F, b, in_type, xscr, out_type, add_mode, add_in, add_out, d_err);
    return grid_bs<3>(s, F, b, in_type, xscr, out_type, add_mode, add_in, add_out, d_err);
}

}  // namespace kry
