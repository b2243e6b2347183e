// MAT object (Section 2.3) and sparse matrix-vector products
// (Figures 20-21): y = alpha A x + beta z over CSR or 3x3 block CSR.
//
// Device layout: sliced ELLPACK, 64 rows per slice (one wavefront), value
// planes entry-major so that a wavefront loading entry e of slot t reads
// 64 consecutive values (512 B in FP64): every matrix byte moves once, in
// full cache lines.  One lane owns one (block) row and computes all bs
// components from one gather of x per block.
#include <algorithm>

#include "device.hpp"
#include "internal.hpp"

namespace kry {

// ---------------------------------------------------------------------------
// layout construction
// ---------------------------------------------------------------------------
template <int BS>
__global__ void k_sell_fill(int nrows, int nslices, const int *__restrict__ off,
                            const int *__restrict__ rowptr,
                            const int *__restrict__ col,
                            const double *__restrict__ val, int *__restrict__ scol,
                            double *__restrict__ sval) {
    constexpr int B2 = BS * BS;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = g >> 6, lane = g & 63;
    if (s >= nslices) return;
    const int o0 = off[s], w = off[s + 1] - o0;
    int p0 = 0, len = 0;
    if (g < nrows) {
        p0 = rowptr[g];
        len = rowptr[g + 1] - p0;
    }
    for (int t = 0; t < w; t++) {
        const int64_t slot = o0 + t;
        const bool have = t < len;
        scol[slot * 64 + lane] = have ? col[p0 + t] : -1;
        for (int e = 0; e < B2; e++)
            sval[(slot * B2 + e) * 64 + lane] = have ? val[(int64_t)(p0 + t) * B2 + e] : 0.0;
    }
}

static void slice_offsets(int nrows, const std::vector<int> &rowptr, std::vector<int> &off,
                          int &maxw) {
    const int nslices = (nrows + 63) / 64;
    off.assign(nslices + 1, 0);
    maxw = 0;
    for (int s = 0; s < nslices; s++) {
        int w = 0;
        for (int r = s * 64; r < std::min(nrows, s * 64 + 64); r++)
            w = std::max(w, rowptr[r + 1] - rowptr[r]);
        off[s + 1] = off[s] + w;
        maxw = std::max(maxw, w);
    }
}

int sell_build_perm_free(hipStream_t s, int nrows, int bs, const int *d_rowptr,
                         const int *d_col, const double *d_val, Sell &S,
                         const std::vector<int> &h_rowptr) {
    S.bs = bs;
    S.nslices = (nrows + 63) / 64;
    slice_offsets(nrows, h_rowptr, S.h_off, S.maxw);
    S.nslots = S.h_off[S.nslices];
    KRY_TRY(S.off.alloc(S.nslices + 1));
    KRY_TRY(S.col.alloc(S.nslots * 64));
    KRY_TRY(S.val.alloc(S.nslots * 64 * bs * bs));
    KRY_HIP(hipMemcpyAsync(S.off.p, S.h_off.data(), sizeof(int) * (S.nslices + 1),
                           hipMemcpyHostToDevice, s));
    const int threads = S.nslices * 64;
    dim3 grid((threads + 255) / 256);
    if (bs == 1)
        hipLaunchKernelGGL(k_sell_fill<1>, grid, dim3(256), 0, s, nrows, S.nslices, S.off.p,
                           d_rowptr, d_col, d_val, S.col.p, S.val.p);
    else
        hipLaunchKernelGGL(k_sell_fill<3>, grid, dim3(256), 0, s, nrows, S.nslices, S.off.p,
                           d_rowptr, d_col, d_val, S.col.p, S.val.p);
    KRY_HIP(hipGetLastError());
    // the host offsets must stay alive until the copy ran
    KRY_HIP(hipStreamSynchronize(s));
    return KRY_OK;
}

int sell_build(hipStream_t s, MAT_ *A) {
    return sell_build_perm_free(s, A->nb, A->bs, A->rowptr.p, A->col.p, A->val.p, A->sell,
                                A->h_rowptr);
}

__global__ void k_to_f32(int64_t n, const double *__restrict__ x, float *__restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = static_cast<float>(x[i]);
}

int ensure_sell_f32(hipStream_t s, Sell &S) {
    if (S.valf.p) return KRY_OK;
    const int64_t n = S.nslots * 64 * S.bs * S.bs;
    KRY_TRY(S.valf.alloc(n));
    hipLaunchKernelGGL(k_to_f32, dim3(2048), dim3(256), 0, s, n, S.val.p, S.valf.p);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

// column 0 of each 3x3 block (entries 0, 3, 6) as FP32 planes [slot][3][64]
__global__ void k_col0_f32(int64_t nslots, const double *__restrict__ val, float *__restrict__ c0) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nslots * 3 * 64;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t slot = i / 192;
        const int r = static_cast<int>((i / 64) % 3), lane = static_cast<int>(i % 64);
        c0[i] = static_cast<float>(val[(slot * 9 + r * 3) * 64 + lane]);
    }
}

int ensure_col0_f32(hipStream_t s, MAT_ *A) {
    if (A->col0f.p) return KRY_OK;
    KRY_TRY(A->col0f.alloc(A->sell.nslots * 3 * 64));
    hipLaunchKernelGGL(k_col0_f32, dim3(2048), dim3(256), 0, s, A->sell.nslots, A->sell.val.p,
                       A->col0f.p);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

// ---------------------------------------------------------------------------
// SpMV kernels
// ---------------------------------------------------------------------------
template <int BS, typename T, typename TA, int NDOT>
__global__ __launch_bounds__(256) void k_sell_spmv(
    int nrows, int nslices, const int *__restrict__ off, const int *__restrict__ col,
    const TA *__restrict__ val, T alpha, const T *__restrict__ x, T beta, const T *z,
    T *y, const T *__restrict__ u0, const T *__restrict__ u1, double *__restrict__ partial) {
    constexpr int B2 = BS * BS;
    const int row = blockIdx.x * 256 + threadIdx.x;
    const int s = row >> 6, lane = row & 63;
    T acc[BS];
#pragma unroll
    for (int r = 0; r < BS; r++) acc[r] = T(0);
    if (s < nslices) {
        const int o0 = off[s], o1 = off[s + 1];
        for (int t = o0; t < o1; t++) {
            const int c = col[(int64_t)t * 64 + lane];
            if (c < 0) continue;
            T xv[BS];
#pragma unroll
            for (int k = 0; k < BS; k++) xv[k] = x[(int64_t)c * BS + k];
            // the matrix planes stream through once: non-temporal loads
            // leave the L2 to x, whose neighbour rows are read again
            const TA *v = val + (int64_t)t * B2 * 64 + lane;
#pragma unroll
            for (int r = 0; r < BS; r++)
#pragma unroll
                for (int k = 0; k < BS; k++)
                    acc[r] += static_cast<T>(__builtin_nontemporal_load(v + (r * BS + k) * 64)) * xv[k];
        }
    }
    double d0 = 0.0, d1 = 0.0;
    if (row < nrows) {
#pragma unroll
        for (int r = 0; r < BS; r++) {
            const int64_t i = (int64_t)row * BS + r;
            T v = alpha * acc[r];
            if (beta != T(0)) v += beta * z[i];
            y[i] = v;
            if (NDOT >= 1) d0 += static_cast<double>(v) * static_cast<double>(u0 ? u0[i] : v);
            if (NDOT >= 2) d1 += static_cast<double>(v) * static_cast<double>(u1 ? u1[i] : v);
        }
    }
    if (NDOT >= 1) {
        __shared__ double lds[4];
        d0 = block_sum<256>(d0, lds);
        if (NDOT >= 2) {
            double t1 = block_sum<256>(d1, lds);
            if (threadIdx.x == 0) partial[blockIdx.x * 2 + 1] = t1;
        }
        if (threadIdx.x == 0) partial[blockIdx.x * 2 + 0] = d0;
    }
}

// r = v - A(:, pressure column) p, 3x3 blocks, only column 0 meets p
template <typename T, typename TA>
__global__ __launch_bounds__(256) void k_col0_residual(
    int nrows, int nslices, const int *__restrict__ off, const int *__restrict__ col,
    const TA *__restrict__ c0, int plane_stride, int plane_off, const T *__restrict__ v,
    const T *__restrict__ p, T *__restrict__ r) {
    const int row = blockIdx.x * 256 + threadIdx.x;
    const int s = row >> 6, lane = row & 63;
    if (s >= nslices || row >= nrows) return;
    T acc[3] = {T(0), T(0), T(0)};
    const int o0 = off[s], o1 = off[s + 1];
    for (int t = o0; t < o1; t++) {
        const int c = col[(int64_t)t * 64 + lane];
        if (c < 0) continue;
        const T pc = p[c];
        const TA *a = c0 + (int64_t)t * plane_stride * 64 + lane;
#pragma unroll
        for (int q = 0; q < 3; q++) acc[q] += static_cast<T>(a[(q * plane_off) * 64]) * pc;
    }
#pragma unroll
    for (int q = 0; q < 3; q++) r[(int64_t)row * 3 + q] = v[(int64_t)row * 3 + q] - acc[q];
}

static inline dim3 sell_grid(const Sell &S) { return dim3((S.nslices * 64 + 255) / 256); }

template <typename T, typename TA>
static int launch_spmv(hipStream_t s, const Sell &S, const TA *val, int nrows, T alpha,
                       const T *x, T beta, const T *z, T *y, int ndot, const T *u0,
                       const T *u1, double *partial) {
    dim3 g = sell_grid(S);
#define KRY_SPMV_CASE(BS, ND)                                                              \
    hipLaunchKernelGGL((k_sell_spmv<BS, T, TA, ND>), g, dim3(256), 0, s, nrows, S.nslices, \
                       S.off.p, S.col.p, val, alpha, x, beta, z, y, u0, u1, partial)
    if (S.bs == 1) {
        if (ndot == 0) KRY_SPMV_CASE(1, 0);
        else if (ndot == 1) KRY_SPMV_CASE(1, 1);
        else KRY_SPMV_CASE(1, 2);
    } else if (S.bs == 3) {
        if (ndot == 0) KRY_SPMV_CASE(3, 0);
        else if (ndot == 1) KRY_SPMV_CASE(3, 1);
        else KRY_SPMV_CASE(3, 2);
    } else {
        return set_error(KRY_ERR_UNSUPPORTED, "SpMV: block size %d", S.bs);
    }
#undef KRY_SPMV_CASE
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

int spmv_partial_blocks(const MAT_ *A) { return static_cast<int>(sell_grid(A->sell).x); }

int spmv_f64(hipStream_t s, const MAT_ *A, double alpha, const double *x, double beta,
             const double *z, double *y, int ndot, const double *u0, const double *u1,
             double *partial) {
    TimedScope ts(A->bs == 3 ? "spmv_bsr3" : "spmv_csr", s);
    return launch_spmv<double, double>(s, A->sell, A->sell.val.p, A->nb, alpha, x, beta, z, y,
                                       ndot, u0, u1, partial);
}

int spmv_sell_f64(hipStream_t s, const Sell &S, int nrows, double alpha, const double *x,
                  double beta, const double *z, double *y) {
    return launch_spmv<double, double>(s, S, S.val.p, nrows, alpha, x, beta, z, y, 0, nullptr,
                                       nullptr, nullptr);
}

int spmv_sell_f32(hipStream_t s, const Sell &S, int nrows, float alpha, const float *x,
                  float beta, const float *z, float *y) {
    if (!S.valf.p) return set_error(KRY_ERR_ARG, "FP32 SpMV without FP32 values");
    return launch_spmv<float, float>(s, S, S.valf.p, nrows, alpha, x, beta, z, y, 0, nullptr,
                                     nullptr, nullptr);
}

int spmv_col0_residual_f32(hipStream_t s, const MAT_ *A, const float *v, const float *p,
                           float *r) {
    const Sell &S = A->sell;
    hipLaunchKernelGGL((k_col0_residual<float, float>), sell_grid(S), dim3(256), 0, s, A->nb,
                       S.nslices, S.off.p, S.col.p, A->col0f.p, 3, 1, v, p, r);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

int spmv_col0_residual_f64(hipStream_t s, const MAT_ *A, const double *v, const double *p,
                           double *r) {
    const Sell &S = A->sell;
    hipLaunchKernelGGL((k_col0_residual<double, double>), sell_grid(S), dim3(256), 0, s, A->nb,
                       S.nslices, S.off.p, S.col.p, S.val.p, 9, 3, v, p, r);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

// ---------------------------------------------------------------------------
// MAT construction
// ---------------------------------------------------------------------------
static int validate_pattern(int nb, const std::vector<int> &rp, const std::vector<int> &ci,
                            std::vector<int> &diag) {
    if (rp[0] != 0) return set_error(KRY_ERR_ARG, "rowptr[0] must be 0");
    diag.assign(nb, -1);
    for (int i = 0; i < nb; i++) {
        if (rp[i + 1] < rp[i]) return set_error(KRY_ERR_ARG, "rowptr decreases at row %d", i);
        for (int p = rp[i]; p < rp[i + 1]; p++) {
            const int c = ci[p];
            if (c < 0 || c >= nb) return set_error(KRY_ERR_ARG, "column %d out of range in row %d", c, i);
            if (p > rp[i] && ci[p - 1] >= c)
                return set_error(KRY_ERR_ARG, "columns not strictly ascending in row %d", i);
            if (c == i) diag[i] = p;
        }
        if (diag[i] < 0) return set_error(KRY_ERR_ARG, "row %d has no diagonal entry", i);
    }
    return KRY_OK;
}

// Recognise a 7-point stencil on an nx x ny x nz grid in natural order
// (nx, ny, nz >= 2): row 0 gives nx and nx*ny, then every row must hold
// exactly its existing neighbours.
static void detect_grid(MAT_ *A) {
    A->gnx = A->gny = A->gnz = 0;
    const int nb = A->nb;
    const std::vector<int> &rp = A->h_rowptr, &ci = A->h_col;
    if (rp[1] - rp[0] != 4 || ci[0] != 0 || ci[1] != 1) return;
    const int64_t nx = ci[2], nxy = ci[3];
    if (nx < 2 || nxy % nx != 0) return;
    const int64_t ny = nxy / nx;
    if (ny < 2 || nb % nxy != 0) return;
    const int64_t nz = nb / nxy;
    if (nz < 2) return;
    for (int64_t c = 0; c < nb; c++) {
        const int64_t i = c % nx, j = (c / nx) % ny, k = c / nxy;
        int64_t want[7];
        int m = 0;
        if (k > 0) want[m++] = c - nxy;
        if (j > 0) want[m++] = c - nx;
        if (i > 0) want[m++] = c - 1;
        want[m++] = c;
        if (i < nx - 1) want[m++] = c + 1;
        if (j < ny - 1) want[m++] = c + nx;
        if (k < nz - 1) want[m++] = c + nxy;
        if (rp[c + 1] - rp[c] != m) return;
        for (int q = 0; q < m; q++)
            if (ci[rp[c] + q] != want[q]) return;
    }
    A->gnx = static_cast<int>(nx);
    A->gny = static_cast<int>(ny);
    A->gnz = static_cast<int>(nz);
}

static MAT *mat_create(MAP *map, int32_t nb, int32_t bs, const int32_t *rowptr,
                       const int32_t *col, const double *val, int where) {
    if (!map || !rowptr || !col || !val) {
        set_error(KRY_ERR_ARG, "MatCreate: NULL argument");
        return nullptr;
    }
    if (bs != 1 && bs != 3) {
        set_error(KRY_ERR_UNSUPPORTED, "MatCreate: block size %d (1 or 3 supported)", bs);
        return nullptr;
    }
    if (nb <= 0 || (int64_t)nb * bs != map->nlocal) {
        set_error(KRY_ERR_DIM, "MatCreate: %d rows of size %d do not match the map (%lld)", nb, bs,
                  (long long)map->nlocal);
        return nullptr;
    }
    if (where != KRY_HOST && where != KRY_DEVICE) {
        set_error(KRY_ERR_ARG, "MatCreate: where must be KRY_HOST or KRY_DEVICE");
        return nullptr;
    }
    hipStream_t s = global_stream();
    std::unique_ptr<MAT_> A(new MAT_());
    A->map = map;
    A->nb = nb;
    A->bs = bs;
    A->h_rowptr.resize(nb + 1);
    hipMemcpyKind k2h = where == KRY_HOST ? hipMemcpyHostToHost : hipMemcpyDeviceToHost;
    if (hipMemcpy(A->h_rowptr.data(), rowptr, sizeof(int) * (nb + 1), k2h) != hipSuccess) {
        set_error(KRY_ERR_HIP, "MatCreate: reading rowptr failed");
        return nullptr;
    }
    const int64_t nnzb = A->h_rowptr[nb];
    if (nnzb <= 0 || nnzb > INT32_MAX) {
        set_error(KRY_ERR_ARG, "MatCreate: bad nonzero count %lld", (long long)nnzb);
        return nullptr;
    }
    A->nnzb = nnzb;
    A->h_col.resize(nnzb);
    if (hipMemcpy(A->h_col.data(), col, sizeof(int) * nnzb, k2h) != hipSuccess) {
        set_error(KRY_ERR_HIP, "MatCreate: reading columns failed");
        return nullptr;
    }
    if (validate_pattern(nb, A->h_rowptr, A->h_col, A->h_diag) != KRY_OK) return nullptr;
    detect_grid(A.get());
    const int b2 = bs * bs;
    if (A->rowptr.alloc(nb + 1) || A->col.alloc(nnzb) || A->diag.alloc(nb) ||
        A->val.alloc(nnzb * b2))
        return nullptr;
    hipMemcpyKind k2d = where == KRY_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    if (hipMemcpy(A->rowptr.p, A->h_rowptr.data(), sizeof(int) * (nb + 1), hipMemcpyHostToDevice) ||
        hipMemcpy(A->col.p, A->h_col.data(), sizeof(int) * nnzb, hipMemcpyHostToDevice) ||
        hipMemcpy(A->diag.p, A->h_diag.data(), sizeof(int) * nb, hipMemcpyHostToDevice) ||
        hipMemcpy(A->val.p, val, sizeof(double) * nnzb * b2, k2d)) {
        set_error(KRY_ERR_HIP, "MatCreate: upload failed");
        return nullptr;
    }
    if (sell_build(s, A.get()) != KRY_OK) return nullptr;
    if (hipStreamSynchronize(s) != hipSuccess) {
        set_error(KRY_ERR_HIP, "MatCreate: layout build failed");
        return nullptr;
    }
    return A.release();
}

MAT *mat_create_device(MAP *map, int nb, int bs, const int *rowptr, const int *col,
                       const double *val) {
    return mat_create(map, nb, bs, rowptr, col, val, KRY_DEVICE);
}

}  // namespace kry

using namespace kry;

extern "C" MAT *MatCreateCSR(MAP *map, int32_t n, const int32_t *rowptr, const int32_t *col,
                             const double *val, int where) {
    return mat_create(map, n, 1, rowptr, col, val, where);
}

extern "C" MAT *MatCreateBSR(MAP *map, int32_t nb, int32_t bs, const int32_t *browptr,
                             const int32_t *bcol, const double *bval, int where) {
    return mat_create(map, nb, bs, browptr, bcol, bval, where);
}

extern "C" int MatUpdateValues(MAT *A, const double *val, int where) {
    if (!A || !val) return set_error(KRY_ERR_ARG, "MatUpdateValues: NULL argument");
    if (where != KRY_HOST && where != KRY_DEVICE)
        return set_error(KRY_ERR_ARG, "MatUpdateValues: where must be KRY_HOST or KRY_DEVICE");
    hipStream_t s = global_stream();
    const size_t bytes = sizeof(double) * (size_t)A->nnzb * A->bs * A->bs;
    KRY_HIP(hipMemcpyAsync(A->val.p, val, bytes,
                           where == KRY_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
    // the SpMV layout holds its own copy of the values; reduced-precision
    // copies are rebuilt on demand
    KRY_TRY(sell_build(s, A));
    A->sell.valf.release();
    A->sell.valh.release();
    A->col0f.release();
    KRY_HIP(hipStreamSynchronize(s));
    return KRY_OK;
}

extern "C" void MatDestroy(MAT **mat) {
    if (!mat || !*mat) return;
    delete *mat;
    *mat = nullptr;
}

extern "C" int64_t MatGetNnzBlocks(const MAT *A) { return A ? A->nnzb : -1; }

extern "C" int MatGetGrid(const MAT *A, int32_t *nx, int32_t *ny, int32_t *nz) {
    if (!A) return set_error(KRY_ERR_ARG, "MatGetGrid: NULL matrix");
    if (nx) *nx = A->gnx;
    if (ny) *ny = A->gny;
    if (nz) *nz = A->gnz;
    return A->gnx > 0 ? KRY_OK : set_error(KRY_ERR_ARG, "MatGetGrid: not a 7-point grid stencil");
}

extern "C" int MatVecMXY(MAT *A, VEC *x, VEC *y) {
    if (!A || !x || !y) return set_error(KRY_ERR_ARG, "MatVecMXY: NULL argument");
    const int64_t n = (int64_t)A->nb * A->bs;
    if (x->n != n || y->n != n) return set_error(KRY_ERR_DIM, "MatVecMXY: sizes differ");
    if (x->data == y->data) return set_error(KRY_ERR_ARG, "MatVecMXY: x and y alias");
    return spmv_f64(global_stream(), A, 1.0, x->data, 0.0, nullptr, y->data, 0, nullptr, nullptr,
                    nullptr);
}

extern "C" int MatVecAMXPBY(double alpha, MAT *A, VEC *x, double beta, VEC *y) {
    if (!A || !x || !y) return set_error(KRY_ERR_ARG, "MatVecAMXPBY: NULL argument");
    const int64_t n = (int64_t)A->nb * A->bs;
    if (x->n != n || y->n != n) return set_error(KRY_ERR_DIM, "MatVecAMXPBY: sizes differ");
    if (x->data == y->data) return set_error(KRY_ERR_ARG, "MatVecAMXPBY: x and y alias");
    return spmv_f64(global_stream(), A, alpha, x->data, beta, y->data, y->data, 0, nullptr,
                    nullptr, nullptr);
}
