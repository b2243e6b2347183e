// CPR multi-stage preconditioners with quasi-IMPES decoupling (Section
// 4.2.1: eqs. (5)-(9), Algorithms 5-8).
//
// Block unknown 0 is the pressure; Pi_r takes component 0 of each block
// (eq. (7)), Pi_p injects a pressure vector into a zero vector (eq. (8)).
// Quasi-IMPES weights per cell from the diagonal block
// D = [[d_pp, d_ps^T], [d_sp, D_ss]]:  w^T = [1, -d_ps^T D_ss^-1], so w^T D
// has zero secondary columns.  Pressure matrix (A_pp)_ij = w_i^T A_ij e_0 on
// the block pattern of A.  The pressure solve is either the paper's AMG
// (one V-cycle on A_pp, FP64) or a fixed number of ILU(0) sweeps
// p <- p + (L_p U_p)^-1 (r_p - A_pp p) from p = 0.
//   PF (Algorithm 6 with its garbled steps 2 and 4 read as the classical
//   two-stage CPR):  z1 = Pi_p(P(Pi_r W v)); r = v - A z1; z = z1 + BILU^-1 r
//   FP (Algorithm 5):  z1 = BILU^-1 v; r = v - A z1; z = z1 + Pi_p(P(Pi_r W r))
//   FPF (Algorithm 7) and FFPF (Algorithm 8): a running iterate x, from
//   x = BILU^-1 v, then each further stage on r = v - A x:
//   F: x += BILU^-1 r;  P: x += Pi_p(P(Pi_r W r)).  FPF = F,P,F;
//   FFPF = F,F,P,F.
// Reduced precision: every vector inside the apply is FP32; the pressure
// factor is FP32 in both reduced variants, the block factor FP32 or BF16.
#include <type_traits>
#include <utility>

#include "device.hpp"
#include "internal.hpp"

namespace kry {

__global__ void k_cpr_weights(int nb, const int *__restrict__ diag, const double *__restrict__ val,
                              double *__restrict__ w, int *err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const double *D = val + (int64_t)diag[i] * 9;
    // solve D_ss^T y = d_ps by elimination with partial pivoting
    double a00 = D[4], a01 = D[7], a10 = D[5], a11 = D[8];
    double r0 = D[1], r1 = D[2];
    const double anorm = fmax(fabs(a00) + fabs(a01), fabs(a10) + fabs(a11));
    if (fabs(a10) > fabs(a00)) {
        double t;
        t = a00; a00 = a10; a10 = t;
        t = a01; a01 = a11; a11 = t;
        t = r0; r0 = r1; r1 = t;
    }
    bool ok = isfinite(a00) && fabs(a00) >= 1e-14 * anorm;
    double y0 = 0.0, y1 = 0.0;
    if (ok) {
        const double f = a10 / a00;
        a11 -= f * a01;
        r1 -= f * r0;
        ok = isfinite(a11) && fabs(a11) >= 1e-14 * anorm;
        if (ok) {
            y1 = r1 / a11;
            y0 = (r0 - a01 * y1) / a00;
        }
    }
    if (!ok) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    w[3 * i + 0] = 1.0;
    w[3 * i + 1] = -y0;
    w[3 * i + 2] = -y1;
}

__global__ void k_cpr_app(int nb, const int *__restrict__ rowptr, const double *__restrict__ val,
                          const double *__restrict__ w, double *__restrict__ app) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const double w0 = w[3 * i], w1 = w[3 * i + 1], w2 = w[3 * i + 2];
    for (int p = rowptr[i]; p < rowptr[i + 1]; p++) {
        const double *B = val + (int64_t)p * 9;
        app[p] = w0 * B[0] + w1 * B[3] + w2 * B[6];
    }
}

// r_p = w_i . v_i in T
template <typename TIN, typename T>
__global__ void k_restrict(int nb, const double *__restrict__ w, const TIN *__restrict__ v,
                           T *__restrict__ rp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const T v0 = static_cast<T>(v[3 * (int64_t)i]);
    const T v1 = static_cast<T>(v[3 * (int64_t)i + 1]);
    const T v2 = static_cast<T>(v[3 * (int64_t)i + 2]);
    rp[i] = static_cast<T>(w[3 * i]) * v0 + static_cast<T>(w[3 * i + 1]) * v1 +
            static_cast<T>(w[3 * i + 2]) * v2;
}

// x_i0 += p_i (pressure injection into the running iterate)
template <typename T>
__global__ void k_inject_inplace(int nb, const T *__restrict__ p, T *__restrict__ x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    x[3 * (int64_t)i] += p[i];
}

__global__ void k_widen(int64_t n, const float *__restrict__ x, double *__restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = static_cast<double>(x[i]);
}

// z = z1 + Pi_p p  (double output)
template <typename T>
__global__ void k_inject_add(int nb, const T *__restrict__ z1, const T *__restrict__ p,
                             double *__restrict__ z) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const int64_t b = 3 * (int64_t)i;
    z[b] = static_cast<double>(static_cast<T>(z1[b] + p[i]));
    z[b + 1] = static_cast<double>(z1[b + 1]);
    z[b + 2] = static_cast<double>(z1[b + 2]);
}

// out = a + b
template <typename T>
__global__ void k_add_vec(int64_t n, const T *__restrict__ a, const T *__restrict__ b,
                          T *__restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a[i] + b[i];
}

template <typename T>
__global__ void k_cast(int64_t n, const double *__restrict__ x, T *__restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = static_cast<T>(x[i]);
}

int cpr_setup(hipStream_t s, MAT_ *A, CprPC &C, int variant, int sweeps, int prec, int *d_err,
              int layout) {
    if (A->bs != 3) return set_error(KRY_ERR_UNSUPPORTED, "CPR needs 3x3 blocks");
    if (sweeps < 1) return set_error(KRY_ERR_ARG, "CPR needs at least one pressure sweep");
    const int nb = A->nb;
    C.variant = variant;
    C.sweeps = sweeps;
    C.prec = prec;
    C.nb = nb;
    KRY_TRY(C.w.alloc(3 * (size_t)nb));
    const dim3 g((nb + 255) / 256), blk(256);
    hipLaunchKernelGGL(k_cpr_weights, g, blk, 0, s, nb, A->diag.p, A->val.p, C.w.p, d_err);
    // pressure matrix on the block pattern of A
    MAT_ &P = C.app;
    P.map = A->map;
    P.nb = nb;
    P.bs = 1;
    P.nnzb = A->nnzb;
    P.h_rowptr = A->h_rowptr;
    P.h_col = A->h_col;
    P.h_diag = A->h_diag;
    P.gnx = A->gnx;
    P.gny = A->gny;
    P.gnz = A->gnz;
    KRY_TRY(P.rowptr.alloc(nb + 1));
    KRY_TRY(P.col.alloc(A->nnzb));
    KRY_TRY(P.diag.alloc(nb));
    KRY_TRY(P.val.alloc(A->nnzb));
    KRY_HIP(hipMemcpyAsync(P.rowptr.p, A->rowptr.p, sizeof(int) * (nb + 1), hipMemcpyDeviceToDevice, s));
    KRY_HIP(hipMemcpyAsync(P.col.p, A->col.p, sizeof(int) * A->nnzb, hipMemcpyDeviceToDevice, s));
    KRY_HIP(hipMemcpyAsync(P.diag.p, A->diag.p, sizeof(int) * nb, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_cpr_app, g, blk, 0, s, nb, A->rowptr.p, A->val.p, C.w.p, P.val.p);
    KRY_HIP(hipGetLastError());
    KRY_TRY(sell_build(s, &P));
    // factors: the pressure factor is FP32 whenever the apply is reduced
    const int pprec = prec == KRY_PREC_F64 ? KRY_PREC_F64 : KRY_PREC_F32;
    if (C.amg) {
        if (prec != KRY_PREC_F64) return set_error(KRY_ERR_UNSUPPORTED, "CPR-AMG: FP64 only");
        KRY_TRY(amg_setup(s, nb, P.h_rowptr.data(), P.h_col.data(), P.val.p, C.amg_opts, *C.amg,
                          d_err));
    } else {
        KRY_TRY(ilu_setup(s, &P, P.val.p, C.ilu_p, pprec, d_err, layout));
    }
    if (C.ras) {
        if (prec != KRY_PREC_F64) return set_error(KRY_ERR_UNSUPPORTED, "CPR-RAS: FP64 only");
        const int rc = C.ras_reuse ? ras_refactor(s, A, *C.ras, d_err)
                                   : ras_setup(s, A, *C.ras, C.ras_box[0], C.ras_box[1],
                                               C.ras_box[2], C.ras_box[3], prec, d_err, layout);
        if (rc < 0) {   // a half-built subdomain set is never reused
            C.ras.reset();
            return rc;
        }
    } else {
        KRY_TRY(ilu_setup(s, A, A->val.p, C.ilu_a, prec, d_err, layout));
    }
    if (prec != KRY_PREC_F64) {
        KRY_TRY(ensure_sell_f32(s, P.sell));
        if (variant == KRY_CPR_PF) KRY_TRY(ensure_col0_f32(s, A));
        else KRY_TRY(ensure_sell_f32(s, A->sell));
    }
    // scratch: rp, p, p2, d (nb each) and vf, r2, xs, z1, z2 (n each)
    const size_t el = prec == KRY_PREC_F64 ? sizeof(double) : sizeof(float);
    const size_t nbp = ((size_t)nb + 63) / 64 * 64, np = 3 * nbp;
    KRY_TRY(C.work.alloc(el * (4 * nbp + 5 * np)));
    KRY_HIP(hipStreamSynchronize(s));
    return KRY_OK;
}

template <typename T>
static int cpr_apply_t(hipStream_t s, MAT_ *A, CprPC &C, const double *v, double *z, int *err) {
    const int nb = C.nb;
    const int64_t n = 3 * (int64_t)nb;
    const size_t nbp = ((size_t)nb + 63) / 64 * 64, np = 3 * nbp;
    T *base = reinterpret_cast<T *>(C.work.p);
    T *rp = base, *p = base + nbp, *p2 = base + 2 * nbp, *d = base + 3 * nbp;
    T *vf = base + 4 * nbp, *r2 = vf + np, *xs = r2 + np, *z1 = xs + np, *z2 = z1 + np;
    const int tin = std::is_same<T, double>::value ? 0 : 1;
    const dim3 g((nb + 255) / 256), blk(256);
    const T *vin = reinterpret_cast<const T *>(v);
    if (tin == 1) {
        hipLaunchKernelGGL(k_cast<T>, dim3(2048), blk, 0, s, n, v, vf);
        vin = vf;
    }
    auto pressure_stage = [&](const T *rvec) -> int {
        // rp = Pi_r W rvec; p = (LU)^-1 rp; then sweeps - 1 corrections
        hipLaunchKernelGGL((k_restrict<T, T>), g, blk, 0, s, nb, C.w.p, rvec, rp);
        if (C.amg)   // FP64 only: p = one V-cycle on rp
            return amg_apply(s, *C.amg, (const double *)rp, (double *)p, err);
        KRY_TRY(ilu_apply(s, C.ilu_p, rp, tin, p, tin, 0, nullptr, nullptr, err));
        for (int k = 1; k < C.sweeps; k++) {
            if (tin == 0)
                KRY_TRY(spmv_sell_f64(s, C.app.sell, nb, -1.0, (const double *)p, 1.0,
                                      (const double *)rp, (double *)d));
            else
                KRY_TRY(spmv_sell_f32(s, C.app.sell, nb, -1.0f, (const float *)p, 1.0f,
                                      (const float *)rp, (float *)d));
            KRY_TRY(ilu_apply(s, C.ilu_p, d, tin, xs, tin, 1, p, p2, err));
            std::swap(p, p2);
        }
        return KRY_OK;
    };
    // the full-system stage R(A)^-1 with ilu_apply's add modes: 0 out = R^-1 in
    // (in xs_out); 1 add_out = add_in + R^-1 in; 2 add_out = Pi_p add_in +
    // R^-1 in.  RAS (FP64 only) solves into xs_out and adds afterwards.
    auto full = [&](const T *in, T *xs_out, int mode, const T *add_in, double *add_out) -> int {
        if (!C.ras)
            return ilu_apply(s, C.ilu_a, in, tin, xs_out, tin, mode, add_in, add_out, err);
        KRY_TRY(ras_apply(s, *C.ras, (const double *)in, (double *)xs_out, err));
        if (mode == 1)
            hipLaunchKernelGGL(k_add_vec<double>, dim3(2048), blk, 0, s, n, (const double *)add_in,
                               (const double *)xs_out, add_out);
        if (mode == 2)
            hipLaunchKernelGGL(k_inject_add<double>, g, blk, 0, s, nb, (const double *)xs_out,
                               (const double *)add_in, add_out);
        return KRY_OK;
    };
    // r2 = v - A x over the full blocks
    auto residual = [&](const T *x) -> int {
        if (tin == 0)
            return spmv_f64(s, A, -1.0, (const double *)x, 1.0, v, (double *)r2, 0, nullptr,
                            nullptr, nullptr);
        return spmv_sell_f32(s, A->sell, nb, -1.0f, (const float *)x, 1.0f, (const float *)vin,
                             (float *)r2);
    };
    if (C.variant == KRY_CPR_FPF || C.variant == KRY_CPR_FFPF) {
        KRY_TRY(full(vin, z1, 0, nullptr, nullptr));
        if (C.variant == KRY_CPR_FFPF) {
            KRY_TRY(residual(z1));
            KRY_TRY(full(r2, xs, 1, z1, (double *)z2));
            std::swap(z1, z2);
        }
        KRY_TRY(residual(z1));
        KRY_TRY(pressure_stage(r2));
        hipLaunchKernelGGL(k_inject_inplace<T>, g, blk, 0, s, nb, p, z1);
        KRY_TRY(residual(z1));
        if (tin == 0) {
            KRY_TRY(full(r2, xs, 1, z1, z));
        } else {
            KRY_TRY(ilu_apply(s, C.ilu_a, r2, tin, xs, tin, 1, z1, z2, err));
            hipLaunchKernelGGL(k_widen, dim3(2048), blk, 0, s, n, (const float *)z2, z);
        }
    } else if (C.variant == KRY_CPR_PF) {
        KRY_TRY(pressure_stage(vin));
        if (tin == 0)
            KRY_TRY(spmv_col0_residual_f64(s, A, (const double *)vin, (const double *)p, (double *)r2));
        else
            KRY_TRY(spmv_col0_residual_f32(s, A, (const float *)vin, (const float *)p, (float *)r2));
        KRY_TRY(full(r2, xs, 2, p, z));
    } else {
        KRY_TRY(full(vin, z1, 0, nullptr, nullptr));
        if (tin == 0)
            KRY_TRY(spmv_f64(s, A, -1.0, (const double *)z1, 1.0, v, (double *)r2, 0, nullptr,
                             nullptr, nullptr));
        else
            KRY_TRY(spmv_sell_f32(s, A->sell, nb, -1.0f, (const float *)z1, 1.0f,
                                  (const float *)vin, (float *)r2));
        KRY_TRY(pressure_stage(r2));
        hipLaunchKernelGGL(k_inject_add<T>, g, blk, 0, s, nb, z1, p, z);
    }
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

int cpr_apply(hipStream_t s, MAT_ *A, CprPC &C, const double *v, double *z, int *err) {
    if (C.prec == KRY_PREC_F64) return cpr_apply_t<double>(s, A, C, v, z, err);
    return cpr_apply_t<float>(s, A, C, v, z, err);
}

}  // namespace kry
