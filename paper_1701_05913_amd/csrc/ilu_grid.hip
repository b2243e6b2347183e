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
//     previous step (cross-lane shuffles),
//   * only lanes on the tile's low faces read values of neighbouring
//     tiles from memory, GC cells at a time, polling the same
//     self-validating slots as the generic sweep.
// A dependency chain therefore crosses memory only when it crosses a tile
// face: NJ + NK hops per sweep instead of nx + ny + nz levels.  Tiles are
// handed to wavefronts in the order of J + K from an atomic counter, so a
// tile's producers are always running already (no deadlock).
//
// Factor layout: step-major per tile, entry-major planes of 64 lanes:
// forward block b (0: k-1, 1: j-1, 2: i-1) entry e of lane l at step t of
// tile T sits at Lt[(((T * S + t) * 3 + b) * bs^2 + e) * 64 + l];
// backward blocks (0: i+1, 1: j+1, 2: k+1) likewise in Ut, indexed by the
// backward step, and the diagonal-block inverse in Dt.  Missing
// neighbours and idle lanes hold zeros, so every load is in bounds and
// unconditional.
#include <algorithm>
#include <type_traits>

#include "device.hpp"
#include "internal.hpp"

namespace kry {

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

int ilu_grid_setup(hipStream_t s, const MAT_ *A, const double *lu, const double *uinv,
                   IluFactor &F) {
    GridTiles &G = F.G;
    G.nx = A->gnx;
    G.ny = A->gny;
    G.nz = A->gnz;
    G.TJ = std::min(8, G.ny);
    G.TK = std::min(64 / G.TJ, G.nz);
    G.NJ = (G.ny + G.TJ - 1) / G.TJ;
    G.NK = (G.nz + G.TK - 1) / G.TK;
    G.ntiles = G.NJ * G.NK;
    G.S = G.nx + G.TJ + G.TK - 2;
    if (G.NJ > 0xffff || G.NK > 0x7fff) return set_error(KRY_ERR_UNSUPPORTED, "grid too large for tiling");
    std::vector<int> ord;
    ord.reserve(G.ntiles);
    for (int d = 0; d <= G.NJ + G.NK - 2; d++)
        for (int J = 0; J < G.NJ; J++) {
            const int K = d - J;
            if (K >= 0 && K < G.NK) ord.push_back(J | (K << 16));
        }
    KRY_TRY(F.order.alloc(G.ntiles));
    KRY_HIP(hipMemcpy(F.order.p, ord.data(), sizeof(int) * G.ntiles, hipMemcpyHostToDevice));
    G.order = F.order.p;
    const int bs = A->bs, b2 = bs * bs;
    const int64_t steps = (int64_t)G.ntiles * G.S;
    const int64_t nlu = steps * 3 * b2 * 64, nd = steps * b2 * 64;
    KRY_TRY(F.lt64.alloc(nlu));
    KRY_TRY(F.ut64.alloc(nlu));
    KRY_TRY(F.dt64.alloc(nd));
    const dim3 g((steps * 64 + 255) / 256), blk(256);
    if (bs == 1)
        hipLaunchKernelGGL(k_grid_pack<1>, g, blk, 0, s, G, A->rowptr.p, A->col.p, A->diag.p, lu,
                           uinv, F.lt64.p, F.ut64.p, F.dt64.p);
    else
        hipLaunchKernelGGL(k_grid_pack<3>, g, blk, 0, s, G, A->rowptr.p, A->col.p, A->diag.p, lu,
                           uinv, F.lt64.p, F.ut64.p, F.dt64.p);
    KRY_HIP(hipGetLastError());
    if (F.prec != KRY_PREC_F64) {
        KRY_TRY(F.dt32.alloc(nd));
        hipLaunchKernelGGL(k_grid_round_f32, dim3(2048), blk, 0, s, nd, F.dt64.p, F.dt32.p);
        if (F.prec == KRY_PREC_F32) {
            KRY_TRY(F.lt32.alloc(nlu));
            KRY_TRY(F.ut32.alloc(nlu));
            hipLaunchKernelGGL(k_grid_round_f32, dim3(2048), blk, 0, s, nlu, F.lt64.p, F.lt32.p);
            hipLaunchKernelGGL(k_grid_round_f32, dim3(2048), blk, 0, s, nlu, F.ut64.p, F.ut32.p);
        } else {
            KRY_TRY(F.lt16.alloc(nlu));
            KRY_TRY(F.ut16.alloc(nlu));
            hipLaunchKernelGGL(k_grid_round_bf16, dim3(2048), blk, 0, s, nlu, F.lt64.p, F.lt16.p);
            hipLaunchKernelGGL(k_grid_round_bf16, dim3(2048), blk, 0, s, nlu, F.ut64.p, F.ut16.p);
        }
        KRY_HIP(hipGetLastError());
        KRY_HIP(hipStreamSynchronize(s));
        F.lt64.release();
        F.ut64.release();
        F.dt64.release();
    }
    F.grid = true;
    return KRY_OK;
}

// ---------------------------------------------------------------------------
// sweeps: one workgroup per tile, wavefront-specialised
//   wave 0            compute: consumes one hyperplane step at a time from
//                     LDS, exchanges neighbour values by shuffles,
//                     publishes results; it issues no global loads, so it
//                     never waits on memory latency
//   wave 1            boundary: polls the published values of the two
//                     upstream tiles (BR steps of 2 cells per lane per
//                     round) and stages them in LDS
//   waves 2..         factor loaders: stream each step's factor planes and
//                     right-hand side into an LDS ring, two steps in flight
//                     per wavefront
// Ring slots carry the step's stamp (a running step count of the
// workgroup), so no slot is ever reset.
// ---------------------------------------------------------------------------
constexpr int NLOAD = 4;
constexpr int GWG = 64 * (2 + NLOAD);
constexpr int NFACE = 40;      // >= TJ + TK for every tiling used
constexpr int DB = 16;         // boundary ring depth (steps)

template <typename TC, typename TF>
__device__ __forceinline__ TC gld(const TF *p) { return static_cast<TC>(*p); }
template <>
__device__ __forceinline__ float gld<float, uint16_t>(const uint16_t *p) { return bf16_to_f32(*p); }

template <int NV, typename TC>
constexpr int ring_depth() {
    return (122880 / (NV * 64 * (int)sizeof(TC))) > 8 ? 8
         : (122880 / (NV * 64 * (int)sizeof(TC))) < 2 ? 2
         : (122880 / (NV * 64 * (int)sizeof(TC)));
}

// acc -= B y for block b of the planes in v
template <int BS, typename TC, int NV>
__device__ __forceinline__ void block_sub(TC (&acc)[BS], const TC (&v)[NV], int b, const TC (&y)[BS]) {
#pragma unroll
    for (int r = 0; r < BS; r++)
#pragma unroll
        for (int c = 0; c < BS; c++) acc[r] -= v[b * BS * BS + r * BS + c] * y[c];
}

// Boundary role.  Face f < TK is the j-face cell of lane kk = f; face
// TK + q the k-face cell of lane jj = q.  For step t the face cell is at
// i = t - lag_f; `cb` is its line base (cell at i = 0) or -1 when the
// upstream tile does not exist.  Each lane serves face f = lane % NF for
// steps t0 + rr and t0 + rr + RS of a round of 2 RS steps.
template <typename TV, typename TC, int BS>
__device__ void boundary_role(int S, int nx, int base, int lane, int NF, const int64_t cb,
                              int lag, const TV *src, TC (&bring)[DB][NFACE][BS], int *bfull,
                              int *bcons, int *err) {
    // a round of 2 RS steps must fit in half the ring, or it would wait
    // for slots that only its own consumer can free
    const int RS = (64 / NF) < (DB / 2) ? (64 / NF) : (DB / 2);
    const int f = lane % NF, rr = lane / NF;
    const bool lane_ok = rr < RS;
    for (int t0 = 0; t0 < S; t0 += 2 * RS) {
        int64_t cells[2];
        int ts[2];
#pragma unroll
        for (int m = 0; m < 2; m++) {
            ts[m] = t0 + rr + m * RS;
            const int i = ts[m] - lag;
            cells[m] = (lane_ok && cb >= 0 && ts[m] < S && i >= 0 && i < nx) ? cb + i : -1;
        }
        TV vals[2][BS];
        wait_cells<TV, BS, 2>(src, cells, vals, err);
        // slots for steps t0 .. t0 + 2 RS - 1 must have been consumed
        lds_wait_ge(bcons, base + t0 + 2 * RS - DB, err);
#pragma unroll
        for (int m = 0; m < 2; m++)
            if (lane_ok && ts[m] < S)
#pragma unroll
                for (int r = 0; r < BS; r++) bring[ts[m] % DB][f][r] = static_cast<TC>(vals[m][r]);
        lds_release();
#pragma unroll
        for (int m = 0; m < 2; m++)
            if (lane_ok && f == 0 && ts[m] < S) lds_put(&bfull[ts[m] % DB], base + ts[m]);
    }
}

// as boundary_role for the backward sweep: step t reaches cell
// i = nx - 1 - (t - lag), i.e. cbr - (t - lag) with cbr the line's last cell
template <typename TV, typename TC, int BS>
__device__ void boundary_role_rev(int S, int nx, int base, int lane, int NF, const int64_t cbr,
                                  int lag, const TV *src, TC (&bring)[DB][NFACE][BS], int *bfull,
                                  int *bcons, int *err) {
    // a round of 2 RS steps must fit in half the ring, or it would wait
    // for slots that only its own consumer can free
    const int RS = (64 / NF) < (DB / 2) ? (64 / NF) : (DB / 2);
    const int f = lane % NF, rr = lane / NF;
    const bool lane_ok = rr < RS;
    for (int t0 = 0; t0 < S; t0 += 2 * RS) {
        int64_t cells[2];
        int ts[2];
#pragma unroll
        for (int m = 0; m < 2; m++) {
            ts[m] = t0 + rr + m * RS;
            const int i = nx - 1 - (ts[m] - lag);
            cells[m] = (lane_ok && cbr >= 0 && ts[m] < S && i >= 0 && i < nx) ? cbr - (ts[m] - lag) : -1;
        }
        TV vals[2][BS];
        wait_cells<TV, BS, 2>(src, cells, vals, err);
        lds_wait_ge(bcons, base + t0 + 2 * RS - DB, err);
#pragma unroll
        for (int m = 0; m < 2; m++)
            if (lane_ok && ts[m] < S)
#pragma unroll
                for (int r = 0; r < BS; r++) bring[ts[m] % DB][f][r] = static_cast<TC>(vals[m][r]);
        lds_release();
#pragma unroll
        for (int m = 0; m < 2; m++)
            if (lane_ok && f == 0 && ts[m] < S) lds_put(&bfull[ts[m] % DB], base + ts[m]);
    }
}

template <int BS, typename TF, typename TC, typename TIN, typename TO>
__global__ __launch_bounds__(GWG) void k_grid_fwd(GridTiles G, const TF *__restrict__ Lt,
                                                  const TIN *__restrict__ b, TC *y, TO *xo,
                                                  int *ctr, int *other_ctr, int *err) {
    constexpr int B2 = BS * BS, NM = 3 * B2, NV = NM + BS;
    constexpr int D = ring_depth<NV, TC>();
    __shared__ TC ring[D][NV][64];
    __shared__ TC bring[DB][NFACE][BS];
    __shared__ int full[D], bfull[DB], cons, bcons, tile;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (blockIdx.x == 0 && threadIdx.x == 0) *other_ctr = 0;
    if (threadIdx.x < D) full[threadIdx.x] = -1;
    if (threadIdx.x < DB) bfull[threadIdx.x] = -1;
    if (threadIdx.x == 0) {
        cons = 0;
        bcons = 0;
    }
    const int TJ = G.TJ, TK = G.TK, nx = G.nx, S = G.S;
    const int64_t sJ = G.nx, sK = (int64_t)G.nx * G.ny;
    int base = 0;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) tile = atomicAdd(ctr, 1);
        __syncthreads();
        const int T = tile;
        if (T >= G.ntiles) break;
        const int JK = G.order[T];
        const int j0 = (JK & 0xffff) * TJ, k0 = (JK >> 16) * TK;
        if (wave == 0) {
            // ---- compute ----
            const int jj = lane % TJ, kk = lane / TJ;
            const int j = j0 + jj, k = k0 + kk;
            const bool lane_ok = lane < TJ * TK && j < G.ny && k < G.nz;
            const int64_t cl = lane_ok ? sJ * j + sK * k : 0;
            TC yp[BS];
#pragma unroll
            for (int r = 0; r < BS; r++) yp[r] = TC(0);
            for (int t = 0; t < S; t++) {
                const int st = base + t, slot = t % D, bslot = t % DB;
                lds_wait_eq(&full[slot], st, err);
                TC v[NV];
#pragma unroll
                for (int e = 0; e < NV; e++) v[e] = ring[slot][e][lane];
                lds_release();
                if (lane == 0) lds_put(&cons, st + 1);
                lds_wait_eq(&bfull[bslot], st, err);
                TC yj[BS], yk[BS], fj[BS], fk[BS];
#pragma unroll
                for (int r = 0; r < BS; r++) {
                    fj[r] = bring[bslot][kk < NFACE ? kk : 0][r];
                    fk[r] = bring[bslot][TK + jj < NFACE ? TK + jj : 0][r];
                }
                lds_release();
                if (lane == 0) lds_put(&bcons, st + 1);
#pragma unroll
                for (int r = 0; r < BS; r++) {
                    yj[r] = __shfl_up(yp[r], 1, 64);
                    yk[r] = __shfl_up(yp[r], TJ, 64);
                    if (jj == 0) yj[r] = fj[r];
                    if (kk == 0) yk[r] = fk[r];
                }
                const int i = t - jj - kk;
                if (lane_ok && i >= 0 && i < nx) {
                    const int64_t c = cl + i;
                    TC acc[BS];
#pragma unroll
                    for (int r = 0; r < BS; r++) acc[r] = v[NM + r];
                    if (k > 0) block_sub<BS>(acc, v, 0, yk);
                    if (j > 0) block_sub<BS>(acc, v, 1, yj);
                    if (i > 0) block_sub<BS>(acc, v, 2, yp);
#pragma unroll
                    for (int r = 0; r < BS; r++) {
                        yp[r] = acc[r];
                        publish<TC>(y + c * BS + r, acc[r]);
                        xo[c * BS + r] = sentinel_value<TO>();
                    }
                }
            }
        } else if (wave == 1) {
            // ---- boundary: upstream values y of tiles (J-1, K) and (J, K-1) ----
            const int NF = TJ + TK;
            const int f = lane % NF;
            int64_t cb = -1;
            int lag = 0;
            if (f < TK) {                               // j-face, lane kk = f
                if (j0 > 0 && k0 + f < G.nz) cb = sJ * (j0 - 1) + sK * (k0 + f);
                lag = f;
            } else {                                    // k-face, lane jj = f - TK
                const int q = f - TK;
                if (k0 > 0 && j0 + q < G.ny) cb = sJ * (j0 + q) + sK * (k0 - 1);
                lag = q;
            }
            boundary_role<TC, TC, BS>(S, nx, base, lane, NF, cb, lag, y, bring, bfull, &bcons, err);
        } else {
            // ---- factor loaders ----
            const int w = wave - 2;
            const int jj = lane % TJ, kk = lane / TJ;
            const int j = j0 + jj, k = k0 + kk;
            const bool lane_ok = lane < TJ * TK && j < G.ny && k < G.nz;
            const int64_t cl = lane_ok ? sJ * j + sK * k : 0;
            const TF *lb = Lt + (int64_t)T * S * NM * 64 + lane;
            TC cur[NV], nxt[NV];
            auto load_step = [&](int t, TC (&v)[NV]) {
#pragma unroll
                for (int e = 0; e < NM; e++) v[e] = gld<TC, TF>(lb + ((int64_t)t * NM + e) * 64);
                const int i = t - jj - kk;
                const int64_t c = (lane_ok && i >= 0 && i < nx) ? cl + i : 0;
#pragma unroll
                for (int r = 0; r < BS; r++) v[NM + r] = static_cast<TC>(b[c * BS + r]);
            };
            if (w < S) load_step(w, cur);
            for (int t = w; t < S; t += NLOAD) {
                const int tn = t + NLOAD;
                if (tn < S) load_step(tn, nxt);
                lds_wait_ge(&cons, base + t - D + 1, err);
#pragma unroll
                for (int e = 0; e < NV; e++) ring[t % D][e][lane] = cur[e];
                lds_release();
                if (lane == 0) lds_put(&full[t % D], base + t);
#pragma unroll
                for (int e = 0; e < NV; e++) cur[e] = nxt[e];
            }
        }
        base += S;
    }
}

template <int BS, typename TF, typename TD, typename TC, typename TO, int ADD, typename TAI,
          typename TAO>
__global__ __launch_bounds__(GWG) void k_grid_bwd(GridTiles G, const TF *__restrict__ Ut,
                                                  const TD *__restrict__ Dt, TC *y, TO *xo,
                                                  const TAI *__restrict__ add_in,
                                                  TAO *__restrict__ add_out, int *ctr,
                                                  int *other_ctr, int *err) {
    constexpr int B2 = BS * BS, NM = 3 * B2, NV = NM + B2 + BS;
    constexpr int D = ring_depth<NV, TC>();
    __shared__ TC ring[D][NV][64];
    __shared__ TC bring[DB][NFACE][BS];
    __shared__ int full[D], bfull[DB], cons, bcons, tile;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (blockIdx.x == 0 && threadIdx.x == 0) *other_ctr = 0;
    if (threadIdx.x < D) full[threadIdx.x] = -1;
    if (threadIdx.x < DB) bfull[threadIdx.x] = -1;
    if (threadIdx.x == 0) {
        cons = 0;
        bcons = 0;
    }
    const int TJ = G.TJ, TK = G.TK, nx = G.nx, S = G.S;
    const int64_t sJ = G.nx, sK = (int64_t)G.nx * G.ny;
    int base = 0;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) tile = atomicAdd(ctr, 1);
        __syncthreads();
        const int Tq = tile;
        if (Tq >= G.ntiles) break;
        const int T = G.ntiles - 1 - Tq;           // reverse tile order
        const int JK = G.order[T];
        const int j0 = (JK & 0xffff) * TJ, k0 = (JK >> 16) * TK;
        if (wave == 0) {
            // ---- compute ----
            const int jj = lane % TJ, kk = lane / TJ;
            const int j = j0 + jj, k = k0 + kk;
            const bool lane_ok = lane < TJ * TK && j < G.ny && k < G.nz;
            const int64_t cl = lane_ok ? sJ * j + sK * k : 0;
            const int lag = (TJ - 1 - jj) + (TK - 1 - kk);
            TC xp[BS];
#pragma unroll
            for (int r = 0; r < BS; r++) xp[r] = TC(0);
            for (int t = 0; t < S; t++) {
                const int st = base + t, slot = t % D, bslot = t % DB;
                lds_wait_eq(&full[slot], st, err);
                TC v[NV];
#pragma unroll
                for (int e = 0; e < NV; e++) v[e] = ring[slot][e][lane];
                lds_release();
                if (lane == 0) lds_put(&cons, st + 1);
                lds_wait_eq(&bfull[bslot], st, err);
                TC fj[BS], fk[BS], xj[BS], xk[BS];
                const int fjx = (TJ - 1 - jj) < 0 ? 0 : kk;
#pragma unroll
                for (int r = 0; r < BS; r++) {
                    fj[r] = bring[bslot][fjx < NFACE ? fjx : 0][r];
                    fk[r] = bring[bslot][TK + jj < NFACE ? TK + jj : 0][r];
                }
                lds_release();
                if (lane == 0) lds_put(&bcons, st + 1);
#pragma unroll
                for (int r = 0; r < BS; r++) {
                    xj[r] = __shfl_down(xp[r], 1, 64);
                    xk[r] = __shfl_down(xp[r], TJ, 64);
                    if (jj == TJ - 1) xj[r] = fj[r];
                    if (kk == TK - 1) xk[r] = fk[r];
                }
                const int i = nx - 1 - (t - lag);
                if (lane_ok && i >= 0 && i < nx) {
                    const int64_t c = cl + i;
                    TC acc[BS];
#pragma unroll
                    for (int r = 0; r < BS; r++) {
                        acc[r] = v[NM + B2 + r];
                        y[c * BS + r] = sentinel_value<TC>();
                    }
                    if (i + 1 < nx) block_sub<BS>(acc, v, 0, xp);
                    if (j + 1 < G.ny) block_sub<BS>(acc, v, 1, xj);
                    if (k + 1 < G.nz) block_sub<BS>(acc, v, 2, xk);
                    TC res[BS];
#pragma unroll
                    for (int r = 0; r < BS; r++) {
                        TC sum = TC(0);
#pragma unroll
                        for (int q = 0; q < BS; q++) sum += v[NM + r * BS + q] * acc[q];
                        res[r] = sum;
                    }
#pragma unroll
                    for (int r = 0; r < BS; r++) {
                        xp[r] = static_cast<TC>(static_cast<TO>(res[r]));
                        publish<TO>(xo + c * BS + r, static_cast<TO>(res[r]));
                        if (ADD == 1)
                            add_out[c * BS + r] =
                                static_cast<TAO>(add_in[c * BS + r]) + static_cast<TAO>(res[r]);
                        if (ADD == 2) {
                            const TC base0 = (r == 0) ? static_cast<TC>(add_in[c]) : TC(0);
                            add_out[c * BS + r] = static_cast<TAO>(base0 + res[r]);
                        }
                    }
                }
            }
        } else if (wave == 1) {
            // ---- boundary: downstream values x of tiles (J+1, K) and (J, K+1) ----
            const int NF = TJ + TK;
            const int f = lane % NF;
            int64_t cb = -1;
            int lag = 0;
            if (f < TK) {                               // j-face of lane (TJ-1, kk = f)
                if (j0 + TJ < G.ny && k0 + f < G.nz) cb = sJ * (j0 + TJ) + sK * (k0 + f);
                lag = (TK - 1 - f);                     // lag of lane (TJ-1, f)
            } else {                                    // k-face of lane (jj = q, TK-1)
                const int q = f - TK;
                if (k0 + TK < G.nz && j0 + q < G.ny) cb = sJ * (j0 + q) + sK * (k0 + TK);
                lag = (TJ - 1 - q);
            }
            // the backward step t reaches i = nx - 1 - (t - lag): index the
            // line from its far end
            const int64_t cbr = cb >= 0 ? cb + nx - 1 : -1;
            boundary_role_rev<TO, TC, BS>(S, nx, base, lane, NF, cbr, lag, xo, bring, bfull, &bcons, err);
        } else {
            // ---- loaders: U blocks, diagonal inverse, forward result ----
            const int w = wave - 2;
            const int jj = lane % TJ, kk = lane / TJ;
            const int j = j0 + jj, k = k0 + kk;
            const bool lane_ok = lane < TJ * TK && j < G.ny && k < G.nz;
            const int64_t cl = lane_ok ? sJ * j + sK * k : 0;
            const int lag = (TJ - 1 - jj) + (TK - 1 - kk);
            const TF *ub = Ut + (int64_t)T * S * NM * 64 + lane;
            const TD *db = Dt + (int64_t)T * S * B2 * 64 + lane;
            TC cur[NV], nxt[NV];
            auto load_step = [&](int t, TC (&v)[NV]) {
#pragma unroll
                for (int e = 0; e < NM; e++) v[e] = gld<TC, TF>(ub + ((int64_t)t * NM + e) * 64);
#pragma unroll
                for (int e = 0; e < B2; e++) v[NM + e] = static_cast<TC>(db[((int64_t)t * B2 + e) * 64]);
                const int i = nx - 1 - (t - lag);
                const int64_t c = (lane_ok && i >= 0 && i < nx) ? cl + i : 0;
#pragma unroll
                for (int r = 0; r < BS; r++) v[NM + B2 + r] = y[c * BS + r];
            };
            if (w < S) load_step(w, cur);
            for (int t = w; t < S; t += NLOAD) {
                const int tn = t + NLOAD;
                if (tn < S) load_step(tn, nxt);
                lds_wait_ge(&cons, base + t - D + 1, err);
#pragma unroll
                for (int e = 0; e < NV; e++) ring[t % D][e][lane] = cur[e];
                lds_release();
                if (lane == 0) lds_put(&full[t % D], base + t);
#pragma unroll
                for (int e = 0; e < NV; e++) cur[e] = nxt[e];
            }
        }
        base += S;
    }
}

// ---------------------------------------------------------------------------
// dispatch (same type combinations as the level-scheduled sweeps)
// ---------------------------------------------------------------------------
template <int BS, typename TF, typename TD, typename TC, typename TIN, typename TO, int ADD,
          typename TAI, typename TAO>
static int grid_pair(hipStream_t s, IluFactor &F, const TF *lt, const TF *ut, const TD *dt,
                     TC *y, const TIN *b, TO *xo, const TAI *add_in, TAO *add_out, int *err) {
    // one workgroup per tile in flight (LDS-bound); 256 CUs
    const int wgs = std::min(F.G.ntiles, 512);
    {
        TimedScope t(sweep_timer_name(true, BS, sizeof(TF), ADD), s);
        hipLaunchKernelGGL((k_grid_fwd<BS, TF, TC, TIN, TO>), dim3(wgs), dim3(GWG), 0, s, F.G,
                           lt, b, y, xo, F.ctr.p, F.ctr.p + 1, err);
    }
    {
        TimedScope t(sweep_timer_name(false, BS, sizeof(TF), ADD), s);
        hipLaunchKernelGGL((k_grid_bwd<BS, TF, TD, TC, TO, ADD, TAI, TAO>), dim3(wgs), dim3(GWG),
                           0, s, F.G, ut, dt, y, xo, add_in, add_out, F.ctr.p + 1, F.ctr.p, err);
    }
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

template <int BS, typename TIN, typename TO>
static int grid_typed(hipStream_t s, IluFactor &F, const TIN *b, TO *xo, int add_mode,
                      const void *add_in, void *add_out, int *err) {
    if (F.prec == KRY_PREC_F64) {
        using TC = double;
        if (add_mode == 0)
            return grid_pair<BS, double, double, TC, TIN, TO, 0, double, double>(
                s, F, F.lt64.p, F.ut64.p, F.dt64.p, F.y64.p, b, xo, nullptr, nullptr, err);
        if (add_mode == 1)
            return grid_pair<BS, double, double, TC, TIN, TO, 1, TO, TO>(
                s, F, F.lt64.p, F.ut64.p, F.dt64.p, F.y64.p, b, xo, (const TO *)add_in,
                (TO *)add_out, err);
        return grid_pair<BS, double, double, TC, TIN, TO, 2, TC, double>(
            s, F, F.lt64.p, F.ut64.p, F.dt64.p, F.y64.p, b, xo, (const TC *)add_in,
            (double *)add_out, err);
    }
    using TC = float;
    if (F.prec == KRY_PREC_F32) {
        if (add_mode == 0)
            return grid_pair<BS, float, float, TC, TIN, TO, 0, float, float>(
                s, F, F.lt32.p, F.ut32.p, F.dt32.p, F.y32.p, b, xo, nullptr, nullptr, err);
        if (add_mode == 1)
            return grid_pair<BS, float, float, TC, TIN, TO, 1, TO, TO>(
                s, F, F.lt32.p, F.ut32.p, F.dt32.p, F.y32.p, b, xo, (const TO *)add_in,
                (TO *)add_out, err);
        return grid_pair<BS, float, float, TC, TIN, TO, 2, TC, double>(
            s, F, F.lt32.p, F.ut32.p, F.dt32.p, F.y32.p, b, xo, (const TC *)add_in,
            (double *)add_out, err);
    }
    if (add_mode == 0)
        return grid_pair<BS, uint16_t, float, TC, TIN, TO, 0, float, float>(
            s, F, F.lt16.p, F.ut16.p, F.dt32.p, F.y32.p, b, xo, nullptr, nullptr, err);
    if (add_mode == 1)
        return grid_pair<BS, uint16_t, float, TC, TIN, TO, 1, TO, TO>(
            s, F, F.lt16.p, F.ut16.p, F.dt32.p, F.y32.p, b, xo, (const TO *)add_in,
            (TO *)add_out, err);
    return grid_pair<BS, uint16_t, float, TC, TIN, TO, 2, TC, double>(
        s, F, F.lt16.p, F.ut16.p, F.dt32.p, F.y32.p, b, xo, (const TC *)add_in,
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
