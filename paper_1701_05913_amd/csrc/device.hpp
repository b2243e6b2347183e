// Device-side helpers shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace kry {

constexpr int WAVE = 64;

// ---- wavefront and block reductions (fixed order -> reproducible) --------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// sum over a block of NT threads; result valid in thread 0
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *lds /* NT/64 */) {
    v = wave_sum(v);
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    if (l == 0) lds[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NT / WAVE; i++) r += lds[i];
    }
    __syncthreads();
    return r;
}

// ---- bfloat16 storage ---------------------------------------------------
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

__host__ __device__ inline uint16_t f32_to_bf16_rne(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) {
        if (u & 0x007fffffu) u |= 0x00400000u;
        return static_cast<uint16_t>(u >> 16);
    }
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

template <typename T>
__device__ __forceinline__ float to_f32(T v) { return static_cast<float>(v); }
template <>
__device__ __forceinline__ float to_f32<uint16_t>(uint16_t v) { return bf16_to_f32(v); }

template <typename TC, typename T>
__device__ __forceinline__ TC load_as(const T *p) { return static_cast<TC>(*p); }
template <>
__device__ __forceinline__ float load_as<float, uint16_t>(const uint16_t *p) {
    return bf16_to_f32(*p);
}

// ---- self-validating values for the sync-free sweeps ----------------------
// A sweep output slot holds a reserved quiet-NaN payload ("not yet
// written") until its row publishes the value.  Producers store with
// relaxed agent-scope atomics, consumers poll with relaxed agent-scope
// atomic loads; every value validates itself, so no fence is needed.
template <typename T> struct Bits;
template <> struct Bits<double> {
    using U = uint64_t;
    static constexpr U sentinel = 0x7FFDEAD00BEEF001ull;
    static constexpr U qnan = 0x7FF8000000000000ull;
    __device__ static U to(double v) { return __double_as_longlong(v); }
    __device__ static double from(U u) { return __longlong_as_double(static_cast<long long>(u)); }
};
template <> struct Bits<float> {
    using U = uint32_t;
    static constexpr U sentinel = 0x7FC0DEADu;
    static constexpr U qnan = 0x7FC00000u;
    __device__ static U to(float v) { return __float_as_uint(v); }
    __device__ static float from(U u) { return __uint_as_float(u); }
};

template <typename T>
__device__ __forceinline__ T sentinel_value() { return Bits<T>::from(Bits<T>::sentinel); }

template <typename T>
__device__ __forceinline__ void publish(T *p, T v) {
    using U = typename Bits<T>::U;
    U u = Bits<T>::to(v);
    if (u == Bits<T>::sentinel) u = Bits<T>::qnan;
    __hip_atomic_store(reinterpret_cast<U *>(p), u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// true when the high 32 bits of v equal the sentinel's: only NaNs of the
// sentinel's payload family qualify (one 32-bit compare per value)
template <typename T>
__device__ __forceinline__ bool sentinel_like(T v) {
    using U = typename Bits<T>::U;
    constexpr int SH = static_cast<int>(sizeof(U)) * 8 - 32;
    return static_cast<uint32_t>(Bits<T>::to(v) >> SH) ==
           static_cast<uint32_t>(Bits<T>::sentinel >> SH);
}

// Publish BS values that the caller has already made not sentinel_like
// (canonical NaN instead): relaxed agent-scope stores, no per-value check.
template <typename T, int BS>
__device__ __forceinline__ void publish_checked(T *p, const T (&v)[BS]) {
    using U = typename Bits<T>::U;
#pragma unroll
    for (int r = 0; r < BS; r++)
        __hip_atomic_store(reinterpret_cast<U *>(p + r), Bits<T>::to(v[r]), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// out = v with every sentinel_like value replaced by the canonical NaN; the
// replacement runs only in lanes that need it (a rare, exec-skipped branch)
template <typename T, int BS>
__device__ __forceinline__ void unsentinel(const T (&v)[BS], T (&out)[BS]) {
    bool odd = false;
#pragma unroll
    for (int r = 0; r < BS; r++) {
        out[r] = v[r];
        odd |= sentinel_like(v[r]);
    }
    if (__builtin_expect(odd, 0)) {
#pragma unroll
        for (int r = 0; r < BS; r++)
            if (sentinel_like(out[r])) out[r] = Bits<T>::from(Bits<T>::qnan);
    }
}

constexpr uint32_t SPIN_LIMIT = 1u << 22;
constexpr int ERR_STALL_FLAG = 2;

// Wait until BS consecutive values at p are published.  Returns false
// (values NaN) when the error flag is raised or the spin bound is hit, so
// that every wave drains instead of hanging.
template <typename T, int BS>
__device__ __forceinline__ bool wait_values(const T *p, T *out, int *err) {
    using U = typename Bits<T>::U;
    U *q = const_cast<U *>(reinterpret_cast<const U *>(p));
    for (uint32_t it = 0;; ++it) {
        bool ready = true;
#pragma unroll
        for (int r = 0; r < BS; r++) {
            U u = __hip_atomic_load(q + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            out[r] = Bits<T>::from(u);
            ready = ready && (u != Bits<T>::sentinel);
        }
        if (ready) return true;
        if ((it & 63u) == 63u) {
            int e = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (e != 0 || it > SPIN_LIMIT) {
                if (e == 0)
                    __hip_atomic_store(err, ERR_STALL_FLAG, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                for (int r = 0; r < BS; r++) out[r] = Bits<T>::from(Bits<T>::qnan);
                return false;
            }
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Wait for up to N cells at once: cell d (valid when cells[d] >= 0) holds
// BS values at base + cells[d] * BS.  All polls of a round are in flight
// together (one memory round trip per round).
template <typename T, int BS, int N>
__device__ __forceinline__ void wait_cells(const T *base, const int64_t (&cells)[N],
                                           T (&out)[N][BS], int *err) {
    using U = typename Bits<T>::U;
    U *q = const_cast<U *>(reinterpret_cast<const U *>(base));
    for (uint32_t it = 0;; ++it) {
        bool ready = true;
#pragma unroll
        for (int d = 0; d < N; d++) {
#pragma unroll
            for (int r = 0; r < BS; r++) {
                if (cells[d] >= 0) {
                    const U u = __hip_atomic_load(q + cells[d] * BS + r, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
                    out[d][r] = Bits<T>::from(u);
                    ready = ready && (u != Bits<T>::sentinel);
                } else {
                    out[d][r] = T(0);
                }
            }
        }
        if (ready) return;
        if ((it & 63u) == 63u) {
            const int e = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (e != 0 || it > SPIN_LIMIT) {
                if (e == 0) __hip_atomic_store(err, ERR_STALL_FLAG, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                for (int d = 0; d < N; d++)
#pragma unroll
                    for (int r = 0; r < BS; r++) out[d][r] = Bits<T>::from(Bits<T>::qnan);
                return;
            }
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Synchronisation between the wavefronts of one workgroup through LDS.
// The fences are restricted to the LDS address space, so they wait only for
// LDS operations (lgkmcnt) and never for outstanding global stores.
__device__ __forceinline__ void lds_release() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
}
__device__ __forceinline__ void lds_acquire() {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
__device__ __forceinline__ int lds_get(int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_put(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Every wait below is on a wavefront of the same workgroup that itself only
// waits on earlier steps, so it ends; the bound turns a broken protocol
// into an error flag instead of a hang.
__device__ __forceinline__ void lds_wait_eq(int *p, int v, int *err) {
    for (uint32_t it = 0; lds_get(p) != v; ++it) {
        if (it > 4 * SPIN_LIMIT) {
            __hip_atomic_store(err, ERR_STALL_FLAG, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    lds_acquire();
}
__device__ __forceinline__ void lds_wait_ge(int *p, int v, int *err) {
    for (uint32_t it = 0; lds_get(p) < v; ++it) {
        if (it > 4 * SPIN_LIMIT) {
            __hip_atomic_store(err, ERR_STALL_FLAG, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    lds_acquire();
}

// wait for *p == v and, when w >= 0, *q == w: both flags in one poll
__device__ __forceinline__ void lds_wait_pair(int *p, int v, int *q, int w, int *err) {
    for (uint32_t it = 0;; ++it) {
        const int a = lds_get(p);
        const int b = w >= 0 ? lds_get(q) : w;
        if (a == v && b == w) break;
        if (it > 4 * SPIN_LIMIT) {
            __hip_atomic_store(err, ERR_STALL_FLAG, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    lds_acquire();
}
// lds_wait_pair, skipped when stamps read ahead of time (pa from p, pb
// from q, during the previous step) already show the step ready; the
// acquire still orders the data reads that follow after the stamps
__device__ __forceinline__ void lds_wait_pair_pre(int pa, int pb, int *p, int v, int *q, int w,
                                                  int *err) {
    const int a = __builtin_amdgcn_readfirstlane(pa), b = __builtin_amdgcn_readfirstlane(pb);
    if (a == v && (w < 0 || b == w)) lds_acquire();
    else lds_wait_pair(p, v, q, w, err);
}

// Inverse of a BS x BS block by Gaussian elimination with partial
// pivoting (first maximal pivot on ties); false (R undefined) for a
// non-finite or tiny pivot: |pivot| < 1e-300 for BS = 1, < 1e-14 ||A||_inf
// otherwise.
template <int BS>
__device__ bool dev_block_inverse(const double *A, double *R) {
    double M[BS * BS];
    double anorm = 0.0;
#pragma unroll
    for (int r = 0; r < BS; r++) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < BS; c++) {
            M[r * BS + c] = A[r * BS + c];
            R[r * BS + c] = (r == c) ? 1.0 : 0.0;
            s += fabs(A[r * BS + c]);
        }
        anorm = fmax(anorm, s);
    }
    for (int k = 0; k < BS; k++) {
        int piv = k;
        double best = fabs(M[k * BS + k]);
        for (int r = k + 1; r < BS; r++)
            if (fabs(M[r * BS + k]) > best) { best = fabs(M[r * BS + k]); piv = r; }
        if (!isfinite(best)) return false;
        if (BS == 1 ? best < 1e-300 : best < 1e-14 * anorm) return false;
        if (piv != k) {
            for (int c = 0; c < BS; c++) {
                double t = M[k * BS + c]; M[k * BS + c] = M[piv * BS + c]; M[piv * BS + c] = t;
                t = R[k * BS + c]; R[k * BS + c] = R[piv * BS + c]; R[piv * BS + c] = t;
            }
        }
        for (int r = k + 1; r < BS; r++) {
            const double f = M[r * BS + k] / M[k * BS + k];
            for (int c = k; c < BS; c++) M[r * BS + c] -= f * M[k * BS + c];
            for (int c = 0; c < BS; c++) R[r * BS + c] -= f * R[k * BS + c];
        }
    }
    for (int k = BS - 1; k >= 0; k--)
        for (int c = 0; c < BS; c++) {
            double s = R[k * BS + c];
            for (int j = k + 1; j < BS; j++) s -= M[k * BS + j] * R[j * BS + c];
            R[k * BS + c] = s / M[k * BS + k];
        }
    return true;
}

}  // namespace kry
