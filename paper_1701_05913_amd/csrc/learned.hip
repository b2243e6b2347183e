// Learned preconditioner stage: a 4-layer 3D convolutional network
// (4 -> 32 -> 32 -> 32 -> 3 channels, 3x3x3 kernels, zero padding, bias,
// exact GELU after the three hidden layers) applied after the base
// preconditioner, with forward and backward passes for training.
//
// gfx950 design.  Every convolution is an implicit GEMM on the BF16 matrix
// cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation): M = 16 cells along
// x, N = 16 output channels, K = 32 input channels of one tap (or 8 taps
// of the 4-channel first layer).  A workgroup owns a 16 x 8 x 4 brick of
// output cells; the input brick with its one-cell halo and the layer's
// packed weights are staged in LDS (cells padded to 80 bytes so the 16
// lanes of a row read distinct banks).  Activations are channels-last
// BF16 ([cell][channel]), so one lane's eight K values are one 16-byte
// load.  The input gradient of a layer is the same kernel run with the
// weights flipped in space and transposed in channels; the weight gradient
// is a second MFMA kernel that contracts over cells (K = 32 cells), with
// channel-major LDS copies of the brick shifted along x so every 8-cell
// operand is an aligned 16-byte load.  Partial sums are reduced in a fixed
// order (bitwise reproducible).
//
// Parameter layout (FP32 master copy): for each layer l, W_l[co][ci][tap]
// with tap = (dz+1)*9 + (dy+1)*3 + (dx+1), then b_l[co].
#include <cmath>
#include <cstdio>
#include <vector>

#include "device.hpp"
#include "internal.hpp"

namespace kry {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NET_C[5] = {4, 32, 32, 32, 3};
constexpr int NET_OFF[5] = {0, 3488, 31168, 58848, 61443};   // parameter offsets
constexpr int HID = 32;
constexpr int BX = 16, BY = 8, BZ = 4;                       // forward brick
constexpr int HX = BX + 2, HY = BY + 2, HZ = BZ + 2;
constexpr int HCELLS = HX * HY * HZ;
constexpr int CSTRIDE32 = 40;                                // bf16 per halo cell (32 + pad)
constexpr int DWX = 16, DWY = 4, DWZ = 2;                    // weight-gradient brick
constexpr int DWROWX = 24;                                   // padded x extent of its halo rows
constexpr int DW_WG = 256;                                   // persistent weight-gradient workgroups

// FP32 -> BF16 round to nearest even in one instruction (v_cvt_pk_bf16_f32
// on gfx950); equal to f32_to_bf16_rne for every non-NaN input
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f)); }
// erf by the rational approximation of Abramowitz & Stegun (1964),
// formula 7.1.26: for x >= 0, erf x = 1 - t (a1 + t (a2 + t (a3 + t (a4 +
// t a5)))) exp(-x^2) with t = 1 / (1 + p x), absolute error below 1.5e-7
// (about one FP32 ulp of erf near 1; the activations are rounded to BF16
// afterwards); odd in x.  Branch-free: one reciprocal, one exponential and
// five FMAs instead of the library's piecewise erff.
__device__ __forceinline__ float erf_as(float x) {
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
    float q = fmaf(t, 1.061405429f, -1.453152027f);
    q = fmaf(t, q, 1.421413741f);
    q = fmaf(t, q, -0.284496736f);
    q = fmaf(t, q, 0.254829592f);
    return copysignf(1.0f - t * q * __expf(-ax * ax), x);
}
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erf_as(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
    return 0.5f * (1.0f + erf_as(x * 0.70710678118654752f)) + x * __expf(-0.5f * x * x) * 0.39894228040143268f;
}

// ---------------------------------------------------------------------------
// weight packing: B fragments of v_mfma_f32_16x16x32_bf16.  Lane l of
// fragment (kb, ct) holds eight K values k = kb*32 + (l/16)*8 + i of output
// channel n = ct*16 + l%16.  K is the input channel of tap kb (CINP = 32)
// or tap*4 + channel over all taps (CINP = 4).  `transposed` packs the
// input-gradient convolution: output channel n of it is input channel n
// of the layer, and taps are mirrored.
// ---------------------------------------------------------------------------
__global__ void k_pack_weights(const float *__restrict__ W, int cin_l, int cout_l, int cinp,
                               int nt, int transposed, uint16_t *__restrict__ wp) {
    const int nkb = cinp == 32 ? 27 : 4;
    const int total = nkb * nt * 64 * 8;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int i = q & 7, l = (q >> 3) & 63, ct = (q >> 9) % nt, kb = (q >> 9) / nt;
    const int k = kb * 32 + (l >> 4) * 8 + i, n = ct * 16 + (l & 15);
    int tap, c;
    if (cinp == 32) {
        tap = kb;
        c = k - kb * 32;
    } else {
        tap = k >> 2;
        c = k & 3;
    }
    // (kernel input channel c, kernel output channel n) of this convolution
    const int cin_k = transposed ? cout_l : cin_l, cout_k = transposed ? cin_l : cout_l;
    float v = 0.0f;
    if (tap < 27 && c < cin_k && n < cout_k) {
        v = transposed ? W[((size_t)c * cin_l + n) * 27 + (26 - tap)]
                       : W[((size_t)n * cin_l + c) * 27 + tap];
    }
    wp[q] = f2bf(v);
}

// ---------------------------------------------------------------------------
// convolution forward (and input-gradient) kernel
//   CINP   4 or 32 channels-last BF16 input
//   NT     output tiles of 16 channels (2: 32 channels, 1: up to 16)
//   MODE   0 hidden layer: y = bias + conv; out_h = bf16(GELU(y)), out_z = y
//          1 output layer: out_f[cell][cout] = bias + conv (FP32)
//          2 input gradient of the next layer: d = conv (no bias);
//            g = d * GELU'(z_prev); out_h = bf16(g), dbpart += g (FP32)
// ---------------------------------------------------------------------------
template <int CINP, int NT, int MODE>
__global__ __launch_bounds__(256) void k_conv(int nx, int ny, int nz, int cout,
                                              const uint16_t *__restrict__ in,
                                              const uint16_t *__restrict__ wp,
                                              const float *__restrict__ bias,
                                              uint16_t *__restrict__ out_h,
                                              float *__restrict__ out_f,
                                              const float *__restrict__ zprev,
                                              float *__restrict__ dbpart) {
    constexpr int NKB = CINP == 32 ? 27 : 4;
    constexpr int CST = CINP == 32 ? CSTRIDE32 : 4;          // bf16 per halo cell
    constexpr int NW = NKB * NT * 64 * 8;                     // packed weight bf16
    __shared__ __attribute__((aligned(16))) uint16_t sh_in[HCELLS * CST];
    __shared__ __attribute__((aligned(16))) uint16_t sh_w[NW];
    __shared__ float sh_db[4][32];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nbx = (nx + BX - 1) / BX, nby = (ny + BY - 1) / BY;
    const int bxi = blockIdx.x % nbx, byi = (blockIdx.x / nbx) % nby, bzi = blockIdx.x / (nbx * nby);
    const int x0 = bxi * BX, y0 = byi * BY, z0 = bzi * BZ;
    const int64_t sy = nx, sz = (int64_t)nx * ny;

    // ---- stage the input brick with halo (zeros outside the grid) ----
    if (CINP == 32) {
        for (int c = tid; c < HCELLS * 4; c += 256) {
            const int hc = c >> 2, part = c & 3;
            const int hx = hc % HX, hy = (hc / HX) % HY, hz = hc / (HX * HY);
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz)
                v = *reinterpret_cast<const uint4 *>(in + (gx + gy * sy + gz * sz) * 32 + part * 8);
            *reinterpret_cast<uint4 *>(sh_in + hc * CST + part * 8) = v;
        }
    } else {
        for (int hc = tid; hc < HCELLS; hc += 256) {
            const int hx = hc % HX, hy = (hc / HX) % HY, hz = hc / (HX * HY);
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
            uint2 v = make_uint2(0, 0);
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz)
                v = *reinterpret_cast<const uint2 *>(in + (gx + gy * sy + gz * sz) * 4);
            *reinterpret_cast<uint2 *>(sh_in + hc * 4) = v;
        }
    }
    for (int c = tid; c < NW / 8; c += 256)
        *reinterpret_cast<uint4 *>(sh_w + c * 8) = *reinterpret_cast<const uint4 *>(wp + c * 8);
    if (MODE == 2 && tid < 128) sh_db[tid >> 5][tid & 31] = 0.0f;
    __syncthreads();

    // ---- wave `wave` computes rows (y = 0..7, z = wave) of 16 cells ----
    f32x4 acc[BY][NT];
#pragma unroll
    for (int r = 0; r < BY; r++)
#pragma unroll
        for (int t = 0; t < NT; t++) acc[r][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int xl = lane & 15, g = lane >> 4;
    for (int kb = 0; kb < NKB; kb++) {
        bf16x8 bfr[NT];
#pragma unroll
        for (int t = 0; t < NT; t++)
            bfr[t] = *reinterpret_cast<const bf16x8 *>(sh_w + ((kb * NT + t) * 64 + lane) * 8);
        if (CINP == 32) {
            const int dz = kb / 9 - 1, dy = (kb / 3) % 3 - 1, dx = kb % 3 - 1;
            const int hbase = ((wave + 1 + dz) * HY + (1 + dy)) * HX + (xl + 1 + dx);
#pragma unroll
            for (int r = 0; r < BY; r++) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(sh_in + (hbase + r * HX) * CST + g * 8);
#pragma unroll
                for (int t = 0; t < NT; t++)
                    acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bfr[t], acc[r][t], 0, 0, 0);
            }
        } else {
            // eight K values = taps 2q and 2q+1 (four channels each), q = kb*4 + g
            const int t0 = kb * 8 + g * 2;
            int off[2];
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const int tp = t0 + h < 27 ? t0 + h : 26;     // padded taps carry zero weights
                const int dz = tp / 9 - 1, dy = (tp / 3) % 3 - 1, dx = tp % 3 - 1;
                off[h] = ((wave + 1 + dz) * HY + (1 + dy)) * HX + (xl + 1 + dx);
            }
#pragma unroll
            for (int r = 0; r < BY; r++) {
                uint4 u;
                const uint2 lo = *reinterpret_cast<const uint2 *>(sh_in + (off[0] + r * HX) * 4);
                const uint2 hi = *reinterpret_cast<const uint2 *>(sh_in + (off[1] + r * HX) * 4);
                u.x = lo.x; u.y = lo.y; u.z = hi.x; u.w = hi.y;
                const bf16x8 a = __builtin_bit_cast(bf16x8, u);
#pragma unroll
                for (int t = 0; t < NT; t++)
                    acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bfr[t], acc[r][t], 0, 0, 0);
            }
        }
    }

    // ---- epilogue: lane holds channel n = t*16 + lane%16 of cells x = 4g + i ----
    const int gz = z0 + wave;
    float dbs[NT];
#pragma unroll
    for (int t = 0; t < NT; t++) dbs[t] = 0.0f;
#pragma unroll
    for (int r = 0; r < BY; r++) {
        const int gy = y0 + r;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int gx = x0 + 4 * g + i;
            const bool ok = gx < nx && gy < ny && gz < nz;
            const int64_t cell = gx + gy * sy + gz * sz;
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const int n = t * 16 + xl;
                const float y = acc[r][t][i];
                if (MODE == 0) {
                    if (ok) {
                        const float v = y + bias[n];
                        out_h[cell * 32 + n] = f2bf(gelu(v));
                        if (out_f) out_f[cell * 32 + n] = v;
                    }
                } else if (MODE == 1) {
                    if (ok && n < cout) out_f[cell * cout + n] = y + bias[n];
                } else {
                    if (ok) {
                        const float gv = y * gelu_grad(zprev[cell * 32 + n]);
                        out_h[cell * 32 + n] = f2bf(gv);
                        dbs[t] += gv;
                    }
                }
            }
        }
    }
    if (MODE == 2) {
        // fixed-order block reduction of the bias gradient: lanes sharing a
        // channel (same lane%16) first, then the four waves
#pragma unroll
        for (int t = 0; t < NT; t++) {
            float v = dbs[t];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            if (lane < 16) sh_db[wave][t * 16 + lane] = v;
        }
        __syncthreads();
        if (tid < 32) {
            const float v = sh_db[0][tid] + sh_db[1][tid] + sh_db[2][tid] + sh_db[3][tid];
            dbpart[(size_t)blockIdx.x * 32 + tid] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// 32-channel convolutions (hidden layers 2 and 3, the output layer and the
// input gradients of layers 2 and 3): persistent workgroups, one per CU.
// The packed weights are staged in LDS once per launch; each workgroup
// then walks the bricks b = blockIdx.x, b + gridDim.x, ...  The next
// brick's input (with halo) is loaded into registers while the current
// brick's MFMAs run, and written to LDS after them.  The taps are taken
// by (dz, dx) pairs: the ten halo rows y0 - 1 .. y0 + 8 of that pair are
// read once and serve the three dy taps (row r of tap dy is halo row
// r + dy + 1), so a pair costs 10 A-fragment and 3 NT B-fragment reads
// for 24 NT MFMAs.  Same MODEs and epilogues as k_conv; in MODE 2 the
// bias-gradient partial is one per workgroup (bricks summed in order).
// ---------------------------------------------------------------------------
constexpr int CONV_PERSIST_WG = 256;
constexpr int PRE_U4 = (HCELLS * 4 + 255) / 256;   // 16-byte input pieces per thread

template <int NT, int MODE>
__global__ __launch_bounds__(256) void k_conv32(int nx, int ny, int nz, int cout,
                                                const uint16_t *__restrict__ in,
                                                const uint16_t *__restrict__ wp,
                                                const float *__restrict__ bias,
                                                uint16_t *__restrict__ out_h,
                                                float *__restrict__ out_f,
                                                const float *__restrict__ zprev,
                                                float *__restrict__ dbpart) {
    constexpr int CST = CSTRIDE32;
    constexpr int NW = 27 * NT * 64 * 8;
    __shared__ __attribute__((aligned(16))) uint16_t sh_in[HCELLS * CST];
    __shared__ __attribute__((aligned(16))) uint16_t sh_w[NW];
    __shared__ float sh_db[4][32];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nbx = (nx + BX - 1) / BX, nby = (ny + BY - 1) / BY, nbz = (nz + BZ - 1) / BZ;
    const int nbricks = nbx * nby * nbz;
    const int64_t sy = nx, sz = (int64_t)nx * ny;

    for (int c = tid; c < NW / 8; c += 256)
        *reinterpret_cast<uint4 *>(sh_w + c * 8) = *reinterpret_cast<const uint4 *>(wp + c * 8);

    // the 16-byte pieces of a brick's halo cells: piece q of thread tid is
    // c = q * 256 + tid, halo cell c / 4, channels (c % 4) * 8 .. + 7
    uint4 pre[PRE_U4];
    auto load = [&](int b) {
        const int x0 = (b % nbx) * BX, y0 = ((b / nbx) % nby) * BY, z0 = (b / (nbx * nby)) * BZ;
#pragma unroll
        for (int q = 0; q < PRE_U4; q++) {
            const int c = q * 256 + tid;
            const int hc = c >> 2, part = c & 3;
            const int hx = hc % HX, hy = (hc / HX) % HY, hz = hc / (HX * HY);
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (c < HCELLS * 4 && gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz)
                v = *reinterpret_cast<const uint4 *>(in + (gx + gy * sy + gz * sz) * 32 + part * 8);
            pre[q] = v;
        }
    };
    float dbs[NT];
#pragma unroll
    for (int t = 0; t < NT; t++) dbs[t] = 0.0f;
    const int xl = lane & 15, g = lane >> 4;
    int b = blockIdx.x;
    if (b < nbricks) load(b);
    for (; b < nbricks; b += gridDim.x) {
        __syncthreads();   // the previous brick's fragments have been read
#pragma unroll
        for (int q = 0; q < PRE_U4; q++) {
            const int c = q * 256 + tid;
            if (c < HCELLS * 4) *reinterpret_cast<uint4 *>(sh_in + (c >> 2) * CST + (c & 3) * 8) = pre[q];
        }
        __syncthreads();
        if (b + (int)gridDim.x < nbricks) load(b + gridDim.x);

        f32x4 acc[BY][NT];
#pragma unroll
        for (int r = 0; r < BY; r++)
#pragma unroll
            for (int t = 0; t < NT; t++) acc[r][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int pz = 0; pz < 3; pz++) {
#pragma unroll
            for (int px = 0; px < 3; px++) {
                const int hb = (wave + pz) * HY * HX + xl + px;
                bf16x8 a[BY + 2];
#pragma unroll
                for (int rr = 0; rr < BY + 2; rr++)
                    a[rr] = *reinterpret_cast<const bf16x8 *>(sh_in + (hb + rr * HX) * CST + g * 8);
#pragma unroll
                for (int py = 0; py < 3; py++) {
                    const int kb = pz * 9 + py * 3 + px;
                    bf16x8 bfr[NT];
#pragma unroll
                    for (int t = 0; t < NT; t++)
                        bfr[t] = *reinterpret_cast<const bf16x8 *>(sh_w + ((kb * NT + t) * 64 + lane) * 8);
#pragma unroll
                    for (int r = 0; r < BY; r++)
#pragma unroll
                        for (int t = 0; t < NT; t++)
                            acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r + py], bfr[t], acc[r][t], 0, 0, 0);
                }
            }
        }

        // epilogue: lane holds channel n = t*16 + lane%16 of brick cells
        // x = 4g + i, y = r, z = wave.  The results go through LDS (the
        // brick's input is no longer needed) so that global stores are
        // whole 16-byte pieces of consecutive cells instead of 2-byte
        // scattered ones.
        const int x0 = (b % nbx) * BX, y0 = ((b / nbx) % nby) * BY, z0 = (b / (nbx * nby)) * BZ;
        __syncthreads();
        // staging strides 80 and 144 bytes per cell: the four cell groups of
        // a store instruction land on different banks, pieces stay aligned
        constexpr int SH = CST, SF = 36;
        static_assert(BX * BY * BZ * SF * 4 <= HCELLS * CST * 2, "staging fits the input tile");
        uint16_t *st_h = sh_in;                              // [512 cells][SH] BF16
        float *st_f = reinterpret_cast<float *>(sh_in);      // [512 cells][SF or 4] FP32
#pragma unroll
        for (int r = 0; r < BY; r++) {
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int cl = (wave * BY + r) * BX + 4 * g + i;
#pragma unroll
                for (int t = 0; t < NT; t++) {
                    const int n = t * 16 + xl;
                    const float y = acc[r][t][i];
                    if (MODE == 0) {
                        st_h[cl * SH + n] = f2bf(gelu(y + bias[n]));
                    } else if (MODE == 1) {
                        if (n < 4) st_f[cl * 4 + n] = y + bias[n < cout ? n : 0];
                    } else {
                        const int gx = x0 + 4 * g + i, gy = y0 + r, gz = z0 + wave;
                        float gv = 0.0f;
                        if (gx < nx && gy < ny && gz < nz)
                            gv = y * gelu_grad(zprev[(gx + gy * sy + gz * sz) * 32 + n]);
                        st_h[cl * SH + n] = f2bf(gv);
                        dbs[t] += gv;
                    }
                }
            }
        }
        __syncthreads();
        if (MODE == 1) {
            // one thread per cell: its cout (<= 4) values
            for (int cl = tid; cl < BX * BY * BZ; cl += 256) {
                const int gx = x0 + cl % BX, gy = y0 + (cl / BX) % BY, gz = z0 + cl / (BX * BY);
                if (gx < nx && gy < ny && gz < nz) {
                    const int64_t cell = gx + gy * sy + gz * sz;
                    for (int c = 0; c < cout; c++) out_f[cell * cout + c] = st_f[cl * 4 + c];
                }
            }
        } else {
            // 16-byte pieces: piece q = cell * 4 + part, eight channels each
            for (int q = tid; q < BX * BY * BZ * 4; q += 256) {
                const int cl = q >> 2, part = q & 3;
                const int gx = x0 + cl % BX, gy = y0 + (cl / BX) % BY, gz = z0 + cl / (BX * BY);
                if (gx < nx && gy < ny && gz < nz)
                    *reinterpret_cast<uint4 *>(out_h + (gx + gy * sy + gz * sz) * 32 + part * 8) =
                        *reinterpret_cast<const uint4 *>(st_h + cl * SH + part * 8);
            }
        }
        if (MODE == 0 && out_f) {
            // pre-activations for training, in a second round through LDS
            __syncthreads();
#pragma unroll
            for (int r = 0; r < BY; r++)
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const int cl = (wave * BY + r) * BX + 4 * g + i;
#pragma unroll
                    for (int t = 0; t < NT; t++) {
                        const int n = t * 16 + xl;
                        st_f[cl * SF + n] = acc[r][t][i] + bias[n];
                    }
                }
            __syncthreads();
            for (int q = tid; q < BX * BY * BZ * 8; q += 256) {
                const int cl = q >> 3, part = q & 7;
                const int gx = x0 + cl % BX, gy = y0 + (cl / BX) % BY, gz = z0 + cl / (BX * BY);
                if (gx < nx && gy < ny && gz < nz)
                    *reinterpret_cast<float4 *>(out_f + (gx + gy * sy + gz * sz) * 32 + part * 4) =
                        *reinterpret_cast<const float4 *>(st_f + cl * SF + part * 4);
            }
        }
    }
    if (MODE == 2) {
#pragma unroll
        for (int t = 0; t < NT; t++) {
            float v = dbs[t];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            if (lane < 16) sh_db[wave][t * 16 + lane] = v;
        }
        __syncthreads();
        if (tid < 32) {
            const float v = sh_db[0][tid] + sh_db[1][tid] + sh_db[2][tid] + sh_db[3][tid];
            dbpart[(size_t)blockIdx.x * 32 + tid] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient: part[wg][m][n] = sum over the bricks of workgroup wg of
// dz[cell][m] * h[cell + tap][c], n = tap * CINP + c (M = MT*16 output
// channels, N = 27*CINP columns in tiles of 16).  K runs over 32 cells at a
// time: lane group q of a K block covers 8 consecutive x cells.
// ---------------------------------------------------------------------------
template <int CINP, int MT, int DZC>
__global__ __launch_bounds__(256) void k_conv_wgrad(int nx, int ny, int nz,
                                                    const uint16_t *__restrict__ dz,
                                                    const uint16_t *__restrict__ h,
                                                    float *__restrict__ part) {
    constexpr int NNT = (27 * CINP + 15) / 16;               // column tiles
    constexpr int TPW = (NNT + 3) / 4;                       // column tiles per wave
    constexpr int M = MT * 16;
    constexpr int HYd = DWY + 2, HZd = DWZ + 2;
    constexpr int ROWS = HYd * HZd;                          // halo rows per channel
    constexpr int CH = CINP;
    // channel-major brick of h with halo, three copies shifted along x by
    // 0, 1, 2 cells so that the 8-cell operand of every tap is aligned
    __shared__ __attribute__((aligned(16))) uint16_t sh_h[3][CH * ROWS * DWROWX];
    __shared__ __attribute__((aligned(16))) uint16_t sh_dz[M][DWX * DWY * DWZ];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nbx = (nx + DWX - 1) / DWX, nby = (ny + DWY - 1) / DWY, nbz = (nz + DWZ - 1) / DWZ;
    const int nbricks = nbx * nby * nbz;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const int xl = lane & 15, q = lane >> 4;
    f32x4 acc[TPW][MT];
#pragma unroll
    for (int j = 0; j < TPW; j++)
#pragma unroll
        for (int m = 0; m < MT; m++) acc[j][m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    for (int br = blockIdx.x; br < nbricks; br += gridDim.x) {
        const int x0 = (br % nbx) * DWX, y0 = ((br / nbx) % nby) * DWY, z0 = (br / (nbx * nby)) * DWZ;
        __syncthreads();
        // stage h: copy s holds x index hx at position hx - s
        for (int e = tid; e < CH * ROWS * DWROWX; e += 256) {
            const int px = e % DWROWX, row = (e / DWROWX) % ROWS, c = e / (DWROWX * ROWS);
            const int hy = row % HYd, hz = row / HYd;
            const int gy = y0 + hy - 1, gz = z0 + hz - 1;
#pragma unroll
            for (int s = 0; s < 3; s++) {
                const int gx = x0 + px + s - 1;
                uint16_t v = 0;
                if (px + s < DWX + 2 && gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz)
                    v = h[(gx + gy * sy + gz * sz) * CINP + c];
                sh_h[s][e] = v;
            }
        }
        // stage dz transposed: sh_dz[m][cell of brick]
        for (int e = tid; e < M * DWX * DWY * DWZ; e += 256) {
            const int cb = e % (DWX * DWY * DWZ), m = e / (DWX * DWY * DWZ);
            const int bx = cb % DWX, by = (cb / DWX) % DWY, bz = cb / (DWX * DWY);
            const int gx = x0 + bx, gy = y0 + by, gz = z0 + bz;
            uint16_t v = 0;
            if (m < DZC && gx < nx && gy < ny && gz < nz) v = dz[(gx + gy * sy + gz * sz) * DZC + m];
            sh_dz[m][cb] = v;
        }
        __syncthreads();
        // K blocks: 32 cells = rows (2 kb, 2 kb + 1) of 16 x cells; lane group
        // q covers row 2 kb + q/2, x = 8 (q%2) .. + 8
        for (int kb = 0; kb < DWY * DWZ / 2; kb++) {
            const int row = 2 * kb + (q >> 1), xs = 8 * (q & 1);
            const int by = row % DWY, bz = row / DWY;
            bf16x8 afr[MT];
#pragma unroll
            for (int m = 0; m < MT; m++)
                afr[m] = *reinterpret_cast<const bf16x8 *>(&sh_dz[m * 16 + xl][row * DWX + xs]);
#pragma unroll
            for (int j = 0; j < TPW; j++) {
                const int nt = wave + 4 * j;
                if (nt < NNT) {
                    const int n = nt * 16 + xl;
                    const int tap = n / CINP < 27 ? n / CINP : 26, c = n % CINP;
                    const int dzz = tap / 9 - 1, dyy = (tap / 3) % 3 - 1, dxx = tap % 3 - 1;
                    // halo x of the first cell = xs + 1 + dxx, taken from copy
                    // s = 1 + dxx at position xs (aligned to 8 elements)
                    const int hrow = (bz + 1 + dzz) * HYd + (by + 1 + dyy);
                    const uint16_t *src = &sh_h[1 + dxx][(c * ROWS + hrow) * DWROWX + xs];
                    bf16x8 b = *reinterpret_cast<const bf16x8 *>(src);
                    if (n >= 27 * CINP) b = bf16x8{};
#pragma unroll
                    for (int m = 0; m < MT; m++)
                        acc[j][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[m], b, acc[j][m], 0, 0, 0);
                }
            }
        }
    }
    // D[m][n]: lane holds n = nt*16 + lane%16, m = mt*16 + 4 (lane/16) + i
    float *pw = part + (size_t)blockIdx.x * M * (NNT * 16);
#pragma unroll
    for (int j = 0; j < TPW; j++) {
        const int nt = wave + 4 * j;
        if (nt < NNT)
#pragma unroll
            for (int m = 0; m < MT; m++)
#pragma unroll
                for (int i = 0; i < 4; i++)
                    pw[(size_t)(m * 16 + 4 * q + i) * (NNT * 16) + nt * 16 + xl] = acc[j][m][i];
    }
}

// grad W[co][ci][tap] = sum over workgroups (fixed order) of part[wg][co][tap*CINP + ci]
__global__ void k_wgrad_reduce(const float *__restrict__ part, int nwg, int M, int NN, int cinp,
                               int cin, int cout, float *__restrict__ gW) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= cout * cin * 27) return;
    const int tap = q % 27, ci = (q / 27) % cin, co = q / (27 * cin);
    const int n = tap * cinp + ci;
    float s = 0.0f;
    for (int w = 0; w < nwg; w++) s += part[((size_t)w * M + co) * NN + n];
    gW[q] = s;
}

// bias gradient from block partials (fixed order)
__global__ void k_bgrad_reduce(const float *__restrict__ part, int nblk, int stride, int cout,
                               float *__restrict__ gb) {
    const int co = threadIdx.x;
    if (co >= cout) return;
    float s = 0.0f;
    for (int b = 0; b < nblk; b++) s += part[(size_t)b * stride + co];
    gb[co] = s;
}

// ---------------------------------------------------------------------------
// loss and output gradient: d = out - target (target channel-major);
// dz4[cell][c] = bf16(2 d / N) (c < 3, channel 3 zero); per-block partial
// sums of d^2 and of the FP32 output gradient (the last layer's bias
// gradient).  One block of 256 threads per 256 cells.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_loss(int64_t cells, const float *__restrict__ out,
                                              const float *__restrict__ target,
                                              uint16_t *__restrict__ dz4, float *__restrict__ part) {
    __shared__ float sh[4][4];
    const int64_t c = blockIdx.x * (int64_t)256 + threadIdx.x;
    const float scale = 2.0f / (3.0f * (float)cells);
    float l2 = 0.0f, gs[3] = {0.0f, 0.0f, 0.0f};
    if (c < cells) {
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const float d = out[c * 3 + k] - target[k * cells + c];
            l2 += d * d;
            gs[k] = scale * d;
            dz4[c * 4 + k] = f2bf(gs[k]);
        }
        dz4[c * 4 + 3] = 0;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float v[4] = {l2, gs[0], gs[1], gs[2]};
#pragma unroll
    for (int k = 0; k < 4; k++) {
        float s = wave_sum(v[k]);
        if (lane == 0) sh[w][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        part[(size_t)blockIdx.x * 4 + k] = sh[0][k] + sh[1][k] + sh[2][k] + sh[3][k];
    }
}

// output gradient given by the caller (channel-major FP32): dz4 and the
// per-block sums of the last layer's bias gradient (slot 0 unused)
__global__ __launch_bounds__(256) void k_outgrad(int64_t cells, const float *__restrict__ dout,
                                                 uint16_t *__restrict__ dz4, float *__restrict__ part) {
    __shared__ float sh[4][4];
    const int64_t c = blockIdx.x * (int64_t)256 + threadIdx.x;
    float gs[3] = {0.0f, 0.0f, 0.0f};
    if (c < cells) {
#pragma unroll
        for (int k = 0; k < 3; k++) {
            gs[k] = dout[k * cells + c];
            dz4[c * 4 + k] = f2bf(gs[k]);
        }
        dz4[c * 4 + 3] = 0;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float v[4] = {0.0f, gs[0], gs[1], gs[2]};
#pragma unroll
    for (int k = 0; k < 4; k++) {
        float s = wave_sum(v[k]);
        if (lane == 0) sh[w][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        part[(size_t)blockIdx.x * 4 + k] = sh[0][k] + sh[1][k] + sh[2][k] + sh[3][k];
    }
}

// channel-major FP32 [>= 3][cells] <-> interleaved FP64 [cells][3]
__global__ void k_cm_to_il(int64_t cells, const float *__restrict__ x, double *__restrict__ y) {
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= cells) return;
#pragma unroll
    for (int k = 0; k < 3; k++) y[c * 3 + k] = static_cast<double>(x[k * cells + c]);
}
__global__ void k_il_to_cm(int64_t cells, const double *__restrict__ x, float *__restrict__ y) {
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= cells) return;
#pragma unroll
    for (int k = 0; k < 3; k++) y[k * cells + c] = static_cast<float>(x[c * 3 + k]);
}

__global__ void k_loss_final(const float *__restrict__ part, int nblk, int64_t cells,
                             float *__restrict__ loss, float *__restrict__ gb4) {
    const int k = threadIdx.x;
    if (k >= 4) return;
    double s = 0.0;
    for (int b = 0; b < nblk; b++) s += part[(size_t)b * 4 + k];
    if (k == 0) *loss = static_cast<float>(s / (3.0 * (double)cells));
    else gb4[k - 1] = static_cast<float>(s);
}

// Adam with bias correction (Kingma and Ba, 2015), FP32 master weights
__global__ void k_adam(int n, float *__restrict__ p, const float *__restrict__ g,
                       float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// channel-major FP32 [4][cells] -> channels-last BF16 [cells][4]
__global__ void k_input_cm(int64_t cells, const float *__restrict__ x, uint16_t *__restrict__ h0) {
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= cells) return;
#pragma unroll
    for (int k = 0; k < 4; k++) h0[c * 4 + k] = f2bf(x[k * cells + c]);
}

// channels-last [cells][3] -> channel-major [3][cells]
__global__ void k_output_cm(int64_t cells, const float *__restrict__ o, float *__restrict__ y) {
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= cells) return;
#pragma unroll
    for (int k = 0; k < 3; k++) y[k * cells + c] = o[c * 3 + k];
}

// network input of the stage: [r1 / s, ln k] with s = ||r1|| / sqrt(n);
// nrm[0] = ||r1||.  When s is zero or not finite the input is zero (the
// correction is then rejected by the residual test).
__global__ void k_stage_input(int64_t cells, const double *__restrict__ r1,
                              const double *__restrict__ nrm, const float *__restrict__ lnk,
                              uint16_t *__restrict__ h0) {
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const double s = nrm[0] / sqrt(3.0 * (double)cells);
    const bool ok = s > 0.0 && isfinite(s);
#pragma unroll
    for (int k = 0; k < 3; k++)
        h0[c * 4 + k] = f2bf(ok ? static_cast<float>(r1[c * 3 + k] / s) : 0.0f);
    h0[c * 4 + 3] = f2bf(lnk[c]);
}

// z2 = z1 + s * out
__global__ void k_stage_update(int64_t cells, const double *__restrict__ z1,
                               const float *__restrict__ out, const double *__restrict__ nrm,
                               double *__restrict__ z2) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= cells * 3) return;
    const double s = nrm[0] / sqrt(3.0 * (double)cells);
    z2[q] = z1[q] + s * static_cast<double>(out[q]);
}

// accept z2 when s > 0 is finite and ||v - A z2|| < ||r1|| (any non-finite
// value fails the comparison); counters: [0] applications, [1] fallbacks
__global__ void k_stage_select(int64_t n, const double *__restrict__ z2,
                               const double *__restrict__ nrm, double *__restrict__ z,
                               unsigned long long *__restrict__ counters) {
    const double s = nrm[0] / sqrt((double)n);
    const bool accept = s > 0.0 && isfinite(s) && nrm[1] < nrm[0];
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q == 0) {
        counters[0] += 1ull;
        if (!accept) counters[1] += 1ull;
    }
    if (accept && q < n) z[q] = z2[q];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct ConvNet {
    int nx = 0, ny = 0, nz = 0;
    int64_t cells = 0;
    DBuf<float> params, grad, m, v;
    int adam_t = 0;
    DBuf<uint16_t> wf[4], wt[4];          // forward / input-gradient fragments
    DBuf<uint16_t> h0, h[3], dz4, dza, dzb;
    DBuf<float> z[3], out, part, loss, tmp_io;
    bool training = false;
};

static int conv_blocks(const ConvNet &N) {
    return ((N.nx + BX - 1) / BX) * ((N.ny + BY - 1) / BY) * ((N.nz + BZ - 1) / BZ);
}
static int conv_persist_blocks(const ConvNet &N) {
    return std::min(conv_blocks(N), CONV_PERSIST_WG);
}
static int wgrad_blocks(const ConvNet &N) {
    const int nb = ((N.nx + DWX - 1) / DWX) * ((N.ny + DWY - 1) / DWY) * ((N.nz + DWZ - 1) / DWZ);
    return std::min(nb, DW_WG);
}

static int net_alloc(ConvNet &N, int nx, int ny, int nz, bool training) {
    if (nx <= 0 || ny <= 0 || nz <= 0) return set_error(KRY_ERR_ARG, "learned stage: grid %d x %d x %d", nx, ny, nz);
    N.nx = nx;
    N.ny = ny;
    N.nz = nz;
    N.cells = (int64_t)nx * ny * nz;
    N.training = training;
    const int np = NET_OFF[4];
    KRY_TRY(N.params.alloc(np));
    KRY_HIP(hipMemset(N.params.p, 0, sizeof(float) * np));
    for (int l = 0; l < 4; l++) {
        const int cinp = l == 0 ? 4 : 32, nt = l == 3 ? 1 : 2;
        KRY_TRY(N.wf[l].alloc((cinp == 32 ? 27 : 4) * nt * 512));
    }
    // input-gradient convolutions: layer 4 (3 -> 32 channels, padded input of
    // 4) and layers 3, 2 (32 -> 32)
    KRY_TRY(N.wt[3].alloc(4 * 2 * 512));
    KRY_TRY(N.wt[2].alloc(27 * 2 * 512));
    KRY_TRY(N.wt[1].alloc(27 * 2 * 512));
    KRY_TRY(N.h0.alloc(N.cells * 4));
    for (int l = 0; l < 3; l++) KRY_TRY(N.h[l].alloc(N.cells * 32));
    KRY_TRY(N.out.alloc(N.cells * 3));
    KRY_TRY(N.loss.alloc(4));
    if (training) {
        KRY_TRY(N.grad.alloc(np));
        KRY_TRY(N.m.alloc(np));
        KRY_TRY(N.v.alloc(np));
        KRY_HIP(hipMemset(N.m.p, 0, sizeof(float) * np));
        KRY_HIP(hipMemset(N.v.p, 0, sizeof(float) * np));
        for (int l = 0; l < 3; l++) KRY_TRY(N.z[l].alloc(N.cells * 32));
        KRY_TRY(N.dz4.alloc(N.cells * 4));
        KRY_TRY(N.dza.alloc(N.cells * 32));
        KRY_TRY(N.dzb.alloc(N.cells * 32));
        const size_t pw = (size_t)wgrad_blocks(N) * 32 * ((27 * 32 + 15) / 16 * 16);
        const size_t pl = (size_t)((N.cells + 255) / 256) * 4;
        const size_t pb = (size_t)conv_blocks(N) * 32;
        KRY_TRY(N.part.alloc(std::max(pw, std::max(pl, pb))));
    }
    KRY_TRY(N.tmp_io.alloc(N.cells * 4));
    return KRY_OK;
}

static int net_pack(hipStream_t s, ConvNet &N) {
    for (int l = 0; l < 4; l++) {
        const int cin = NET_C[l], cout = NET_C[l + 1];
        const int cinp = l == 0 ? 4 : 32, nt = l == 3 ? 1 : 2;
        const int tot = (cinp == 32 ? 27 : 4) * nt * 512;
        hipLaunchKernelGGL(k_pack_weights, dim3((tot + 255) / 256), dim3(256), 0, s,
                           N.params.p + NET_OFF[l], cin, cout, cinp, nt, 0, N.wf[l].p);
    }
    // transposed packs: layer 4 (kernel input = its 3 output channels, padded to 4)
    hipLaunchKernelGGL(k_pack_weights, dim3((4 * 2 * 512 + 255) / 256), dim3(256), 0, s,
                       N.params.p + NET_OFF[3], 32, 3, 4, 2, 1, N.wt[3].p);
    for (int l = 1; l <= 2; l++)
        hipLaunchKernelGGL(k_pack_weights, dim3((27 * 2 * 512 + 255) / 256), dim3(256), 0, s,
                           N.params.p + NET_OFF[l], 32, 32, 32, 2, 1, N.wt[l].p);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

// forward from N.h0; keeps pre-activations when training
static int net_forward(hipStream_t s, ConvNet &N) {
    const dim3 g(conv_blocks(N)), b(256);
    const bool keep = N.training;
    {
        TimedScope t("conv_l1_fwd", s);
        hipLaunchKernelGGL((k_conv<4, 2, 0>), g, b, 0, s, N.nx, N.ny, N.nz, 32, N.h0.p, N.wf[0].p,
                           N.params.p + NET_OFF[0] + 32 * 4 * 27, N.h[0].p, keep ? N.z[0].p : nullptr,
                           nullptr, nullptr);
    }
    const dim3 gp(conv_persist_blocks(N));
    for (int l = 1; l <= 2; l++) {
        TimedScope t(l == 1 ? "conv_l2_fwd" : "conv_l3_fwd", s);
        hipLaunchKernelGGL((k_conv32<2, 0>), gp, b, 0, s, N.nx, N.ny, N.nz, 32, N.h[l - 1].p,
                           N.wf[l].p, N.params.p + NET_OFF[l] + 32 * 32 * 27, N.h[l].p,
                           keep ? N.z[l].p : nullptr, nullptr, nullptr);
    }
    {
        TimedScope t("conv_l4_fwd", s);
        hipLaunchKernelGGL((k_conv32<1, 1>), gp, b, 0, s, N.nx, N.ny, N.nz, 3, N.h[2].p, N.wf[3].p,
                           N.params.p + NET_OFF[3] + 3 * 32 * 27, nullptr, N.out.p, nullptr, nullptr);
    }
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

// loss and full parameter gradient for target (channel-major [3][cells])
static int net_backward_from_dz4(hipStream_t s, ConvNet &N);

static int net_backward(hipStream_t s, ConvNet &N, const float *target) {
    const int nlb = static_cast<int>((N.cells + 255) / 256);
    hipLaunchKernelGGL(k_loss, dim3(nlb), dim3(256), 0, s, N.cells, N.out.p, target, N.dz4.p, N.part.p);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, N.part.p, nlb, N.cells, N.loss.p,
                       N.grad.p + NET_OFF[3] + 3 * 32 * 27);
    return net_backward_from_dz4(s, N);
}

// gradient of an arbitrary loss given dL/d(out) (channel-major FP32)
static int net_backward_dout(hipStream_t s, ConvNet &N, const float *dout) {
    const int nlb = static_cast<int>((N.cells + 255) / 256);
    hipLaunchKernelGGL(k_outgrad, dim3(nlb), dim3(256), 0, s, N.cells, dout, N.dz4.p, N.part.p);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, N.part.p, nlb, N.cells, N.loss.p,
                       N.grad.p + NET_OFF[3] + 3 * 32 * 27);
    return net_backward_from_dz4(s, N);
}

// parameter gradients from dz4 (the output gradient) and the activations
// of the last forward pass
static int net_backward_from_dz4(hipStream_t s, ConvNet &N) {
    const dim3 g(conv_blocks(N)), b(256);
    const int nwg = wgrad_blocks(N);
    constexpr int NN32 = (27 * 32 + 15) / 16 * 16, NN4 = (27 * 4 + 15) / 16 * 16;
    // layer 4: weight gradient from dz4 (3 channels) and h[2]
    {
        TimedScope t("conv_wgrad", s);
        hipLaunchKernelGGL((k_conv_wgrad<32, 1, 4>), dim3(nwg), b, 0, s, N.nx, N.ny, N.nz, N.dz4.p,
                           N.h[2].p, N.part.p);
        hipLaunchKernelGGL(k_wgrad_reduce, dim3((3 * 32 * 27 + 255) / 256), dim3(256), 0, s, N.part.p,
                           nwg, 16, NN32, 32, 32, 3, N.grad.p + NET_OFF[3]);
    }
    // dz3 = conv^T(dz4) * GELU'(z3)
    {
        TimedScope t("conv_dgrad", s);
        hipLaunchKernelGGL((k_conv<4, 2, 2>), g, b, 0, s, N.nx, N.ny, N.nz, 32, N.dz4.p, N.wt[3].p,
                           nullptr, N.dza.p, nullptr, N.z[2].p, N.part.p);
        hipLaunchKernelGGL(k_bgrad_reduce, dim3(1), dim3(64), 0, s, N.part.p, (int)g.x, 32, 32,
                           N.grad.p + NET_OFF[2] + 32 * 32 * 27);
    }
    // layers 3 and 2: weight gradient, then the input gradient of the layer below
    uint16_t *dcur = N.dza.p, *dnext = N.dzb.p;
    for (int l = 2; l >= 1; l--) {
        {
            TimedScope t("conv_wgrad", s);
            hipLaunchKernelGGL((k_conv_wgrad<32, 2, 32>), dim3(nwg), b, 0, s, N.nx, N.ny, N.nz, dcur,
                               N.h[l - 1].p, N.part.p);
            hipLaunchKernelGGL(k_wgrad_reduce, dim3((32 * 32 * 27 + 255) / 256), dim3(256), 0, s,
                               N.part.p, nwg, 32, NN32, 32, 32, 32, N.grad.p + NET_OFF[l]);
        }
        {
            TimedScope t("conv_dgrad", s);
            const dim3 gp(conv_persist_blocks(N));
            hipLaunchKernelGGL((k_conv32<2, 2>), gp, b, 0, s, N.nx, N.ny, N.nz, 32, dcur, N.wt[l].p,
                               nullptr, dnext, nullptr, N.z[l - 1].p, N.part.p);
            hipLaunchKernelGGL(k_bgrad_reduce, dim3(1), dim3(64), 0, s, N.part.p, (int)gp.x, 32, 32,
                               N.grad.p + NET_OFF[l - 1] + (l - 1 == 0 ? 32 * 4 * 27 : 32 * 32 * 27));
        }
        std::swap(dcur, dnext);
    }
    // layer 1: weight gradient from dz1 and the 4-channel input
    {
        TimedScope t("conv_wgrad", s);
        hipLaunchKernelGGL((k_conv_wgrad<4, 2, 32>), dim3(nwg), b, 0, s, N.nx, N.ny, N.nz, dcur, N.h0.p,
                           N.part.p);
        hipLaunchKernelGGL(k_wgrad_reduce, dim3((32 * 4 * 27 + 255) / 256), dim3(256), 0, s, N.part.p,
                           nwg, 32, NN4, 4, 4, 32, N.grad.p + NET_OFF[0]);
    }
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

}  // namespace kry

using namespace kry;

struct LEARNED_ {
    ConvNet net;
    hipStream_t stream = nullptr;
    DBuf<double> e, r, res, g, partial, nrm;   // residual-loss scratch
};

static int copy_in(hipStream_t s, void *dst, const void *src, size_t bytes, int where) {
    KRY_HIP(hipMemcpyAsync(dst, src, bytes, where == KRY_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
    return KRY_OK;
}

extern "C" LEARNED *LearnedCreate(int nx, int ny, int nz, int training) {
    LEARNED *L = new LEARNED_();
    if (net_alloc(L->net, nx, ny, nz, training != 0) != KRY_OK) {
        delete L;
        return nullptr;
    }
    return L;
}

extern "C" int LearnedDestroy(LEARNED **Lp) {
    if (!Lp || !*Lp) return KRY_OK;
    delete *Lp;
    *Lp = nullptr;
    return KRY_OK;
}

extern "C" int LearnedNumParams(void) { return NET_OFF[4]; }

extern "C" int LearnedSetStream(LEARNED *L, void *stream) {
    if (!L) return set_error(KRY_ERR_ARG, "LearnedSetStream: NULL");
    L->stream = static_cast<hipStream_t>(stream);
    return KRY_OK;
}

extern "C" int LearnedSetParams(LEARNED *L, const float *params, int where) {
    if (!L || !params) return set_error(KRY_ERR_ARG, "LearnedSetParams: NULL argument");
    KRY_TRY(copy_in(L->stream, L->net.params.p, params, sizeof(float) * NET_OFF[4], where));
    KRY_TRY(net_pack(L->stream, L->net));
    KRY_HIP(hipStreamSynchronize(L->stream));
    return KRY_OK;
}

extern "C" int LearnedGetParams(LEARNED *L, float *params_host) {
    if (!L || !params_host) return set_error(KRY_ERR_ARG, "LearnedGetParams: NULL argument");
    KRY_HIP(hipMemcpyAsync(params_host, L->net.params.p, sizeof(float) * NET_OFF[4], hipMemcpyDeviceToHost, L->stream));
    KRY_HIP(hipStreamSynchronize(L->stream));
    return KRY_OK;
}

extern "C" int LearnedForward(LEARNED *L, const float *in, float *out) {
    if (!L || !in || !out) return set_error(KRY_ERR_ARG, "LearnedForward: NULL argument");
    ConvNet &N = L->net;
    const dim3 g((N.cells + 255) / 256), b(256);
    hipLaunchKernelGGL(k_input_cm, g, b, 0, L->stream, N.cells, in, N.h0.p);
    KRY_TRY(net_forward(L->stream, N));
    hipLaunchKernelGGL(k_output_cm, g, b, 0, L->stream, N.cells, N.out.p, out);
    KRY_HIP(hipGetLastError());
    KRY_HIP(hipStreamSynchronize(L->stream));
    return KRY_OK;
}

extern "C" int LearnedLossGrad(LEARNED *L, const float *in, const float *target, float *loss_host,
                               float *grad) {
    if (!L || !in || !target) return set_error(KRY_ERR_ARG, "LearnedLossGrad: NULL argument");
    ConvNet &N = L->net;
    if (!N.training) return set_error(KRY_ERR_ARG, "LearnedLossGrad: created without training buffers");
    const dim3 g((N.cells + 255) / 256), b(256);
    hipLaunchKernelGGL(k_input_cm, g, b, 0, L->stream, N.cells, in, N.h0.p);
    KRY_TRY(net_forward(L->stream, N));
    KRY_TRY(net_backward(L->stream, N, target));
    if (grad)
        KRY_HIP(hipMemcpyAsync(grad, N.grad.p, sizeof(float) * NET_OFF[4], hipMemcpyDeviceToDevice, L->stream));
    float lh = 0.0f;
    KRY_HIP(hipMemcpyAsync(&lh, N.loss.p, sizeof(float), hipMemcpyDeviceToHost, L->stream));
    KRY_HIP(hipStreamSynchronize(L->stream));
    if (loss_host) *loss_host = lh;
    return KRY_OK;
}

extern "C" int LearnedBackward(LEARNED *L, const float *dout, float *grad) {
    if (!L || !dout) return set_error(KRY_ERR_ARG, "LearnedBackward: NULL argument");
    ConvNet &N = L->net;
    if (!N.training) return set_error(KRY_ERR_ARG, "LearnedBackward: created without training buffers");
    KRY_TRY(net_backward_dout(L->stream, N, dout));
    if (grad)
        KRY_HIP(hipMemcpyAsync(grad, N.grad.p, sizeof(float) * NET_OFF[4], hipMemcpyDeviceToDevice, L->stream));
    KRY_HIP(hipStreamSynchronize(L->stream));
    return KRY_OK;
}

extern "C" int LearnedResidualGrad(LEARNED *L, const MAT *A, const MAT *At, const float *in,
                                   const float *out, float *dout, double *loss_host) {
    if (!L || !A || !At || !in || !out || !dout)
        return set_error(KRY_ERR_ARG, "LearnedResidualGrad: NULL argument");
    const int64_t cells = L->net.cells, n = 3 * cells;
    if (A->bs != 3 || At->bs != 3 || A->nb != cells || At->nb != cells)
        return set_error(KRY_ERR_DIM, "LearnedResidualGrad: matrices must be 3x3-block with one block row per cell");
    hipStream_t s = L->stream;
    const int nsb = std::max(spmv_partial_blocks(A), spmv_partial_blocks(At));
    if (L->e.n < (size_t)n) {
        KRY_TRY(L->e.alloc(n));
        KRY_TRY(L->r.alloc(n));
        KRY_TRY(L->res.alloc(n));
        KRY_TRY(L->g.alloc(n));
        KRY_TRY(L->nrm.alloc(1));
    }
    if (L->partial.n < (size_t)nsb * 2) KRY_TRY(L->partial.alloc((size_t)nsb * 2));
    const dim3 gc((cells + 255) / 256), b(256);
    hipLaunchKernelGGL(k_cm_to_il, gc, b, 0, s, cells, out, L->e.p);
    hipLaunchKernelGGL(k_cm_to_il, gc, b, 0, s, cells, in, L->r.p);
    // res = A e - r1/s, with its squared norm
    KRY_TRY(spmv_f64(s, A, 1.0, L->e.p, -1.0, L->r.p, L->res.p, 1, nullptr, nullptr, L->partial.p));
    KRY_TRY(sum_partials(s, L->partial.p, spmv_partial_blocks(A), 2, 1, L->nrm.p, SUM_PLAIN));
    // dL/de = (2/n) A^T res
    KRY_TRY(spmv_f64(s, At, 2.0 / (double)n, L->res.p, 0.0, nullptr, L->g.p, 0, nullptr, nullptr, nullptr));
    hipLaunchKernelGGL(k_il_to_cm, gc, b, 0, s, cells, L->g.p, dout);
    KRY_HIP(hipGetLastError());
    double h = 0.0;
    KRY_HIP(hipMemcpyAsync(&h, L->nrm.p, sizeof(double), hipMemcpyDeviceToHost, s));
    KRY_HIP(hipStreamSynchronize(s));
    if (loss_host) *loss_host = h / (double)n;
    return KRY_OK;
}

extern "C" int LearnedAdamStep(LEARNED *L, float lr, float beta1, float beta2, float eps) {
    if (!L) return set_error(KRY_ERR_ARG, "LearnedAdamStep: NULL");
    ConvNet &N = L->net;
    if (!N.training) return set_error(KRY_ERR_ARG, "LearnedAdamStep: created without training buffers");
    N.adam_t += 1;
    const float c1 = 1.0f - std::pow(beta1, (float)N.adam_t), c2 = 1.0f - std::pow(beta2, (float)N.adam_t);
    const int np = NET_OFF[4];
    hipLaunchKernelGGL(k_adam, dim3((np + 255) / 256), dim3(256), 0, L->stream, np, N.params.p, N.grad.p,
                       N.m.p, N.v.p, lr, beta1, beta2, eps, c1, c2);
    KRY_TRY(net_pack(L->stream, N));
    KRY_HIP(hipStreamSynchronize(L->stream));
    return KRY_OK;
}

// checkpoint: magic, version, nparams, adam step, params, m, v (FP32)
extern "C" int LearnedSave(LEARNED *L, const char *path) {
    if (!L || !path) return set_error(KRY_ERR_ARG, "LearnedSave: NULL argument");
    ConvNet &N = L->net;
    const int np = NET_OFF[4];
    std::vector<float> p(np), m(np, 0.0f), v(np, 0.0f);
    KRY_HIP(hipMemcpy(p.data(), N.params.p, sizeof(float) * np, hipMemcpyDeviceToHost));
    if (N.training) {
        KRY_HIP(hipMemcpy(m.data(), N.m.p, sizeof(float) * np, hipMemcpyDeviceToHost));
        KRY_HIP(hipMemcpy(v.data(), N.v.p, sizeof(float) * np, hipMemcpyDeviceToHost));
    }
    FILE *f = std::fopen(path, "wb");
    if (!f) return set_error(KRY_ERR_ARG, "LearnedSave: cannot open %s", path);
    const int hdr[4] = {0x4B524C4E, 1, np, N.adam_t};
    bool ok = std::fwrite(hdr, sizeof(int), 4, f) == 4 && std::fwrite(p.data(), sizeof(float), np, f) == (size_t)np &&
              std::fwrite(m.data(), sizeof(float), np, f) == (size_t)np &&
              std::fwrite(v.data(), sizeof(float), np, f) == (size_t)np;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? KRY_OK : set_error(KRY_ERR_ARG, "LearnedSave: write failed for %s", path);
}

namespace kry {
int learned_read_file(const char *path, std::vector<float> &p, std::vector<float> &m,
                      std::vector<float> &v, int &adam_t) {
    FILE *f = std::fopen(path, "rb");
    if (!f) return set_error(KRY_ERR_ARG, "cannot open %s", path);
    int hdr[4] = {0, 0, 0, 0};
    const int np = NET_OFF[4];
    bool ok = std::fread(hdr, sizeof(int), 4, f) == 4 && hdr[0] == 0x4B524C4E && hdr[1] == 1 && hdr[2] == np;
    p.resize(np);
    m.resize(np);
    v.resize(np);
    ok = ok && std::fread(p.data(), sizeof(float), np, f) == (size_t)np &&
         std::fread(m.data(), sizeof(float), np, f) == (size_t)np &&
         std::fread(v.data(), sizeof(float), np, f) == (size_t)np;
    std::fclose(f);
    if (!ok) return set_error(KRY_ERR_ARG, "%s is not a learned-stage checkpoint", path);
    adam_t = hdr[3];
    return KRY_OK;
}
}  // namespace kry

extern "C" int LearnedLoad(LEARNED *L, const char *path) {
    if (!L || !path) return set_error(KRY_ERR_ARG, "LearnedLoad: NULL argument");
    std::vector<float> p, m, v;
    int t = 0;
    KRY_TRY(learned_read_file(path, p, m, v, t));
    ConvNet &N = L->net;
    const int np = NET_OFF[4];
    KRY_HIP(hipMemcpy(N.params.p, p.data(), sizeof(float) * np, hipMemcpyHostToDevice));
    if (N.training) {
        KRY_HIP(hipMemcpy(N.m.p, m.data(), sizeof(float) * np, hipMemcpyHostToDevice));
        KRY_HIP(hipMemcpy(N.v.p, v.data(), sizeof(float) * np, hipMemcpyHostToDevice));
        N.adam_t = t;
    }
    KRY_TRY(net_pack(L->stream, N));
    KRY_HIP(hipStreamSynchronize(L->stream));
    return KRY_OK;
}

// training pair: in = [r1 / s, ln k], target = d / s (channel-major FP32)
__global__ void k_make_pair(int64_t cells, const double *__restrict__ r1, const double *__restrict__ d,
                            const float *__restrict__ lnk, const double *__restrict__ nrm,
                            float *__restrict__ in, float *__restrict__ target) {
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const double s = nrm[0] / sqrt(3.0 * (double)cells);
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        in[k * cells + c] = static_cast<float>(r1[c * 3 + k] * inv);
        target[k * cells + c] = static_cast<float>(d[c * 3 + k] * inv);
    }
    in[3 * cells + c] = lnk[c];
}

extern "C" int LearnedMakePair(int64_t cells, const double *r1, const double *d, const float *logk,
                               float *in, float *target, double *s_host) {
    if (cells <= 0 || !r1 || !d || !logk || !in || !target)
        return set_error(KRY_ERR_ARG, "LearnedMakePair: bad argument");
    hipStream_t s = global_stream();
    DBuf<double> part, nrm;
    KRY_TRY(part.alloc(RED_BLOCKS * 2));
    KRY_TRY(nrm.alloc(1));
    KRY_TRY(vec_dot_partial(s, 3 * cells, r1, r1, nullptr, nullptr, part.p));
    KRY_TRY(sum_partials(s, part.p, RED_BLOCKS, 2, 1, nrm.p, SUM_SQRT));
    hipLaunchKernelGGL(k_make_pair, dim3((cells + 255) / 256), dim3(256), 0, s, cells, r1, d, logk, nrm.p,
                       in, target);
    KRY_HIP(hipGetLastError());
    double h = 0.0;
    KRY_HIP(hipMemcpyAsync(&h, nrm.p, sizeof(double), hipMemcpyDeviceToHost, s));
    KRY_HIP(hipStreamSynchronize(s));
    if (s_host) *s_host = h / std::sqrt(3.0 * (double)cells);
    return KRY_OK;
}

// ---------------------------------------------------------------------------
// the stage inside a solver
// ---------------------------------------------------------------------------
namespace kry {

struct LearnedStage {
    ConvNet net;
    DBuf<float> lnk;
    DBuf<double> r, z2, nrm, partial;
    DBuf<unsigned long long> counters;
};

void learned_stage_delete(LearnedStage *L) { delete L; }

int learned_stage_create(hipStream_t s, const MAT_ *A, const float *params_host,
                         const float *lnk, int lnk_where, LearnedStage **out) {
    if (A->gnx <= 0 || A->bs != 3)
        return set_error(KRY_ERR_ARG, "learned stage needs a 3x3-block 7-point grid matrix");
    std::unique_ptr<LearnedStage> L(new LearnedStage());
    KRY_TRY(net_alloc(L->net, A->gnx, A->gny, A->gnz, false));
    const int64_t cells = L->net.cells, n = 3 * cells;
    KRY_HIP(hipMemcpyAsync(L->net.params.p, params_host, sizeof(float) * NET_OFF[4], hipMemcpyHostToDevice, s));
    KRY_TRY(net_pack(s, L->net));
    KRY_TRY(L->lnk.alloc(cells));
    KRY_TRY(copy_in(s, L->lnk.p, lnk, sizeof(float) * cells, lnk_where));
    KRY_TRY(L->r.alloc(n));
    KRY_TRY(L->z2.alloc(n));
    KRY_TRY(L->nrm.alloc(2));
    // one partial pair per SpMV block (the fused-dot SpMV's layout)
    KRY_TRY(L->partial.alloc((size_t)spmv_partial_blocks(A) * 2));
    KRY_TRY(L->counters.alloc(2));
    KRY_HIP(hipMemsetAsync(L->counters.p, 0, 2 * sizeof(unsigned long long), s));
    KRY_HIP(hipStreamSynchronize(s));
    *out = L.release();
    return KRY_OK;
}

// z holds z1 = M_base^-1 v on entry and the stage's result on exit
int learned_stage_apply(hipStream_t s, const MAT_ *A, LearnedStage &L, const double *v, double *z) {
    ConvNet &N = L.net;
    const int64_t cells = N.cells, n = 3 * cells;
    TimedScope t("learned_stage", s);
    // r1 = v - A z1 and ||r1||
    const int nsb = spmv_partial_blocks(A);
    KRY_TRY(spmv_f64(s, A, -1.0, z, 1.0, v, L.r.p, 1, nullptr, nullptr, L.partial.p));
    KRY_TRY(sum_partials(s, L.partial.p, nsb, 2, 1, L.nrm.p, SUM_SQRT));
    const dim3 g((cells + 255) / 256), g3((n + 255) / 256), b(256);
    hipLaunchKernelGGL(k_stage_input, g, b, 0, s, cells, L.r.p, L.nrm.p, L.lnk.p, N.h0.p);
    KRY_TRY(net_forward(s, N));
    hipLaunchKernelGGL(k_stage_update, g3, b, 0, s, cells, z, N.out.p, L.nrm.p, L.z2.p);
    // ||v - A z2||
    KRY_TRY(spmv_f64(s, A, -1.0, L.z2.p, 1.0, v, L.r.p, 1, nullptr, nullptr, L.partial.p));
    KRY_TRY(sum_partials(s, L.partial.p, nsb, 2, 1, L.nrm.p + 1, SUM_SQRT));
    hipLaunchKernelGGL(k_stage_select, g3, b, 0, s, n, L.z2.p, L.nrm.p, z, L.counters.p);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

int learned_stage_stats(hipStream_t s, LearnedStage &L, int64_t *applies, int64_t *fallbacks) {
    unsigned long long c[2] = {0, 0};
    KRY_HIP(hipMemcpyAsync(c, L.counters.p, sizeof(c), hipMemcpyDeviceToHost, s));
    KRY_HIP(hipStreamSynchronize(s));
    if (applies) *applies = static_cast<int64_t>(c[0]);
    if (fallbacks) *fallbacks = static_cast<int64_t>(c[1]);
    return KRY_OK;
}

}  // namespace kry
