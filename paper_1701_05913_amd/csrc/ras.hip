// Restricted additive Schwarz (Section 4.1; Cai & Sarkis) with block ILU(0)
// subdomain solves:
//     M^-1 v = sum_s R0_s^T (L_s U_s)^-1 R_s v.
// On a 7-point grid matrix in natural order the subdomains are boxes of a
// px x py x pz partition of the grid; each is grown by `overlap` cells in
// every direction (edges and corners included), so its principal
// submatrix is again a 7-point grid stencil.  For z-slabs (px = py = 1)
// this growth is exactly `overlap` rounds of graph neighbours, and the
// overlapped set is one contiguous range of rows.  The subdomains are
// factored together (one grid-tiled factorization launch holding the tiles
// of all of them) and swept together: one forward and one backward launch,
// each subdomain on workgroups of its own, so a sweep's dependency chain has
// mx + my + mz - 2 hyperplanes for an mx x my x mz box instead of
// nx + ny + nz - 2.  R_s is a strided view of v (the box's cells at the
// grid's strides); the untile launch writes each box's owned cells (R0_s^T)
// straight into z.  A repeated setup for new values of the same matrix only
// gathers the values and refactors.  Slabs too thin for the grid kernels
// (one layer) use the level-scheduled sweeps in turn; boxes have no such
// fallback.
#include <algorithm>

#include "device.hpp"
#include "internal.hpp"

namespace kry {

// val_s[q] = val[pos[q]] (blocks of b2 values)
__global__ void k_gather_blocks(int64_t nq, int b2, const int *__restrict__ pos,
                                const double *__restrict__ val, double *__restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nq * b2;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = e / b2;
        out[e] = val[(int64_t)pos[q] * b2 + (e - q * b2)];
    }
}

RasPC::~RasPC() {
    for (auto &S : subs) {
        delete S->A;
        delete S->map;
    }
}

int ras_setup(hipStream_t s, MAT_ *A, RasPC &R, int px, int py, int pz, int overlap, int prec,
              int *d_err, int layout) {
    if (A->gnx <= 0)
        return set_error(KRY_ERR_UNSUPPORTED, "RAS: needs a 7-point grid matrix in natural order");
    const int nx = A->gnx, ny = A->gny, nz = A->gnz, bs = A->bs, b2 = bs * bs;
    if (px < 1 || py < 1 || pz < 1 || px > nx || py > ny || pz > nz || overlap < 0)
        return set_error(KRY_ERR_ARG, "RAS: need 1 <= px, py, pz <= the grid (%d, %d, %d) and overlap >= 0",
                         nx, ny, nz);
    if (prec != KRY_PREC_F64) return set_error(KRY_ERR_UNSUPPORTED, "RAS: FP64 only");
    const bool slabs = px == 1 && py == 1;
    R.px = px;
    R.py = py;
    R.pz = pz;
    R.overlap = overlap;
    R.bs = bs;
    R.layout = layout;
    R.A = A;
    R.subs.clear();
    const std::vector<int> &rp = A->h_rowptr, &ci = A->h_col;
    const int n3[3] = {nx, ny, nz}, p3[3] = {px, py, pz};
    for (int c = 0; c < pz; c++)
        for (int b = 0; b < py; b++)
            for (int a = 0; a < px; a++) {
                std::unique_ptr<RasSub> S(new RasSub());
                const int q3[3] = {a, b, c};
                for (int d = 0; d < 3; d++) {
                    const int lo = (int)((int64_t)q3[d] * n3[d] / p3[d]);
                    const int hi = (int)((int64_t)(q3[d] + 1) * n3[d] / p3[d]);
                    S->ob[2 * d] = lo;
                    S->ob[2 * d + 1] = hi;
                    S->gb[2 * d] = std::max(0, lo - overlap);
                    S->gb[2 * d + 1] = std::min(n3[d], hi + overlap);
                }
                const int mx = S->gb[1] - S->gb[0], my = S->gb[3] - S->gb[2],
                          mz = S->gb[5] - S->gb[4];
                const int nl = mx * my * mz;
                if (slabs) {   // contiguous rows: restriction is an offset
                    S->lo = S->gb[4] * nx * ny;
                    S->hi = S->gb[5] * nx * ny;
                    S->o0 = S->ob[4] * nx * ny;
                    S->o1 = S->ob[5] * nx * ny;
                }
                // principal submatrix on the box, local natural order
                std::vector<int> lrp(nl + 1, 0), lci, pos;
                for (int kl = 0, l = 0; kl < mz; kl++)
                    for (int jl = 0; jl < my; jl++)
                        for (int il = 0; il < mx; il++, l++) {
                            const int g = ((S->gb[4] + kl) * ny + S->gb[2] + jl) * nx + S->gb[0] + il;
                            for (int p = rp[g]; p < rp[g + 1]; p++) {
                                const int cg = ci[p];
                                const int ic = cg % nx, jc = (cg / nx) % ny, kc = cg / (nx * ny);
                                if (ic < S->gb[0] || ic >= S->gb[1] || jc < S->gb[2] || jc >= S->gb[3] ||
                                    kc < S->gb[4] || kc >= S->gb[5])
                                    continue;
                                lci.push_back(((kc - S->gb[4]) * my + jc - S->gb[2]) * mx + ic - S->gb[0]);
                                pos.push_back(p);
                            }
                            lrp[l + 1] = (int)lci.size();
                        }
                const int64_t nq = (int64_t)lci.size();
                DBuf<int> d_rp, d_ci;
                DBuf<double> d_val;
                KRY_TRY(d_rp.alloc(nl + 1));
                KRY_TRY(d_ci.alloc(nq));
                KRY_TRY(S->pos.alloc(nq));
                KRY_TRY(d_val.alloc(nq * b2));
                KRY_HIP(hipMemcpyAsync(d_rp.p, lrp.data(), sizeof(int) * (nl + 1), hipMemcpyHostToDevice, s));
                KRY_HIP(hipMemcpyAsync(d_ci.p, lci.data(), sizeof(int) * nq, hipMemcpyHostToDevice, s));
                KRY_HIP(hipMemcpyAsync(S->pos.p, pos.data(), sizeof(int) * nq, hipMemcpyHostToDevice, s));
                hipLaunchKernelGGL(k_gather_blocks, dim3(1024), dim3(256), 0, s, nq, b2, S->pos.p,
                                   A->val.p, d_val.p);
                KRY_HIP(hipGetLastError());
                KRY_HIP(hipStreamSynchronize(s));
                S->map = MapCreateLocal((int64_t)nl * bs);
                if (!S->map) return KRY_ERR_ALLOC;
                S->A = mat_create_device(S->map, nl, bs, d_rp.p, d_ci.p, d_val.p);
                if (!S->A) return KRY_ERR_ARG;    // mat_create_device set the message
                R.subs.push_back(std::move(S));
            }
    // one launch per sweep (and for the factorization) when every box is
    // grid-tiled; else (z-slabs only) each slab is factored and swept alone
    R.multi = layout != KRY_SWEEP_LEVELS;
    for (auto &S : R.subs) R.multi = R.multi && S->A->gnx > 0 && ilu_grid_can_factor(S->A);
    if (!R.multi && !slabs)
        return set_error(KRY_ERR_UNSUPPORTED,
                         "RAS: boxes need the grid-tiled sweeps (box sides >= 3 in x and y, >= 2 in z)");
    if (R.multi) {
        std::vector<GridMulti> d(R.subs.size());
        std::vector<FactorMulti> f(R.subs.size());
        R.wgs = R.untile_blocks = R.factor_wgs = 0;
        int rot = 0;
        for (size_t q = 0; q < R.subs.size(); q++) {
            RasSub &S = *R.subs[q];
            S.F.timer_fwd = "ras_ilu_fwd";
            S.F.timer_bwd = "ras_ilu_bwd";
            // consecutive tile columns over all subdomains go to consecutive
            // queues, so small boxes do not all crowd the first XCDs
            S.F.qrot = rot;
            KRY_TRY(grid_factor_prepare(s, S.A, S.F, S.faces, S.fctr));
            rot = (rot + S.F.G.NJ) % GRID_QUEUES;
            int w = 0, u = 0, fw = 0;
            KRY_TRY(grid_multi_launch_size(S.F, &w, &u));
            const int own[6] = {S.ob[0] - S.gb[0], S.ob[1] - S.gb[0], S.ob[2] - S.gb[2],
                                S.ob[3] - S.gb[2], S.ob[4] - S.gb[4], S.ob[5] - S.gb[4]};
            const int64_t boff = (((int64_t)S.gb[4] * ny + S.gb[2]) * nx + S.gb[0]) * bs;
            KRY_TRY(grid_multi_desc(S.F, boff, nx, (int64_t)nx * ny, own, R.wgs, R.untile_blocks, d[q]));
            KRY_TRY(grid_factor_desc(S.A, S.F, S.faces, S.fctr, R.factor_wgs, f[q], &fw));
            R.wgs += w;
            R.untile_blocks += u;
            R.factor_wgs += fw;
        }
        KRY_TRY(R.desc.alloc(d.size()));
        KRY_TRY(R.fdesc.alloc(f.size()));
        KRY_HIP(hipMemcpyAsync(R.desc.p, d.data(), sizeof(GridMulti) * d.size(),
                               hipMemcpyHostToDevice, s));
        KRY_HIP(hipMemcpyAsync(R.fdesc.p, f.data(), sizeof(FactorMulti) * f.size(),
                               hipMemcpyHostToDevice, s));
    } else {
        for (auto &S : R.subs) KRY_TRY(S->x.alloc((size_t)(S->hi - S->lo) * bs));
    }
    // the subdomain matrices already hold A's values: factor them
    return ras_refactor(s, A, R, d_err);
}

int ras_refactor(hipStream_t s, const MAT_ *A, RasPC &R, int *d_err) {
    const int b2 = R.bs * R.bs;
    for (auto &S : R.subs)
        hipLaunchKernelGGL(k_gather_blocks, dim3(1024), dim3(256), 0, s, (int64_t)S->pos.n, b2,
                           S->pos.p, A->val.p, S->A->val.p);
    KRY_HIP(hipGetLastError());
    if (R.multi) {
        for (auto &S : R.subs) KRY_TRY(grid_factor_rearm(s, S->F, S->faces, S->fctr));
        KRY_TRY(grid_factor_multi(s, R.bs, R.fdesc.p, (int)R.subs.size(), R.factor_wgs, d_err));
    } else {
        for (auto &S : R.subs) {
            S->F.timer_fwd = "ras_ilu_fwd";
            S->F.timer_bwd = "ras_ilu_bwd";
            KRY_TRY(ilu_setup(s, S->A, S->A->val.p, S->F, KRY_PREC_F64, d_err, R.layout));
        }
    }
    KRY_HIP(hipStreamSynchronize(s));
    return KRY_OK;
}

int ras_apply(hipStream_t s, RasPC &R, const double *v, double *z, int *d_err) {
    TimedScope ts("ras_apply", s);
    const int bs = R.bs;
    if (R.multi)
        return grid_multi_apply(s, bs, R.desc.p, (int)R.subs.size(), R.wgs, R.untile_blocks, v, z,
                                d_err);
    for (auto &S : R.subs) {
        // (L_s U_s)^-1 R_s v, then the owned rows into z
        KRY_TRY(ilu_apply(s, S->F, v + (int64_t)S->lo * bs, 0, S->x.p, 0, 0, nullptr, nullptr,
                          d_err));
        KRY_HIP(hipMemcpyAsync(z + (int64_t)S->o0 * bs, S->x.p + (int64_t)(S->o0 - S->lo) * bs,
                               sizeof(double) * (size_t)(S->o1 - S->o0) * bs,
                               hipMemcpyDeviceToDevice, s));
    }
    return KRY_OK;
}

}  // namespace kry
