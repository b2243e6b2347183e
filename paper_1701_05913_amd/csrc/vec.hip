// MAP and VEC objects (Sections 2.1-2.2), vector kernels (Figures 10-13),
// deterministic reductions, error reporting and kernel timing.
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>

#include "device.hpp"
#include "internal.hpp"

namespace kry {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local char g_err[512] = "";

int set_error(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

static hipStream_t g_stream = nullptr;
hipStream_t global_stream() { return g_stream; }

// ---------------------------------------------------------------------------
// kernel timing: pairs of events per launch, summed on query
// ---------------------------------------------------------------------------
struct TimingEntry {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    hipEvent_t open = nullptr;
};
static std::mutex g_tmu;
static std::map<std::string, TimingEntry> g_timing;
static bool g_timing_on = false;
static std::vector<std::string> g_timing_only;   // empty: every scope
static int g_timing_every = 1;                   // time one launch in every g_timing_every
static std::map<std::string, int64_t> g_timing_seen;

bool timing_on() { return g_timing_on; }

bool timing_wanted(const char *name) {
    if (!g_timing_on) return false;
    std::lock_guard<std::mutex> lk(g_tmu);
    bool sel = g_timing_only.empty();
    for (const auto &x : g_timing_only) sel = sel || x == name;
    if (!sel) return false;
    return g_timing_seen[name]++ % g_timing_every == 0;
}

void timing_begin(const char *name, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_tmu);
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, s);
    g_timing[name].open = e;
}

void timing_end(const char *name, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_tmu);
    auto &t = g_timing[name];
    if (!t.open) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, s);
    t.ev.emplace_back(t.open, e);
    t.open = nullptr;
}

// ---------------------------------------------------------------------------
// vector kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ double coef(Coef c) { return c.p ? (*c.p) * c.v : c.v; }

__global__ void k_fill(int64_t n, double *x, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

__global__ void k_axpbyz(int64_t n, Coef ca, const double *x, Coef cb,
                         const double *y, double *z) {
    const double a = coef(ca), b = coef(cb);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double t = a * x[i];
        if (y) t += b * y[i];
        z[i] = t;
    }
}

__global__ void k_axpbypcz(int64_t n, Coef ca, const double *x, Coef cb,
                           const double *y, Coef cc, double *z) {
    const double a = coef(ca), b = coef(cb), c = coef(cc);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        z[i] = a * x[i] + b * y[i] + c * z[i];
}

__global__ void k_scale_copy(int64_t n, Coef ca, const double *x, double *y) {
    const double a = coef(ca);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i];
}

__global__ void k_f64_to_f32(int64_t n, const double *__restrict__ x, float *__restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = static_cast<float>(x[i]);
}

__global__ __launch_bounds__(RED_THREADS) void k_dot_partial(
    int64_t n, const double *__restrict__ x0, const double *__restrict__ y0,
    const double *__restrict__ x1, const double *__restrict__ y1,
    double *__restrict__ partial) {
    __shared__ double lds[RED_THREADS / WAVE];
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        s0 += x0[i] * y0[i];
        if (x1) s1 += x1[i] * y1[i];
    }
    s0 = block_sum<RED_THREADS>(s0, lds);
    s1 = block_sum<RED_THREADS>(s1, lds);
    if (threadIdx.x == 0) {
        partial[blockIdx.x * 2 + 0] = s0;
        partial[blockIdx.x * 2 + 1] = s1;
    }
}

__global__ __launch_bounds__(RED_THREADS) void k_sum_partials(
    const double *__restrict__ partial, int nparts, int stride, int nk,
    double *__restrict__ out, int op) {
    __shared__ double lds[RED_THREADS / WAVE];
    for (int k = 0; k < nk; k++) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += partial[(size_t)i * stride + k];
        s = block_sum<RED_THREADS>(s, lds);
        if (threadIdx.x == 0) out[k] = (op == SUM_SQRT) ? sqrt(s) : s;
    }
}

static inline int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

int vec_fill(hipStream_t s, int64_t n, double *x, double v) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, n, x, v);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

int vec_axpbyz(hipStream_t s, int64_t n, Coef a, const double *x, Coef b,
               const double *y, double *z) {
    hipLaunchKernelGGL(k_axpbyz, dim3(grid_for(n)), dim3(256), 0, s, n, a, x, b, y, z);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

int vec_axpbypcz(hipStream_t s, int64_t n, Coef a, const double *x, Coef b,
                 const double *y, Coef c, double *z) {
    hipLaunchKernelGGL(k_axpbypcz, dim3(grid_for(n)), dim3(256), 0, s, n, a, x, b, y, c, z);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

int vec_scale_copy(hipStream_t s, int64_t n, Coef a, const double *x, double *y) {
    hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(256), 0, s, n, a, x, y);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

int vec_copy_f64_to_f32(hipStream_t s, int64_t n, const double *x, float *y) {
    hipLaunchKernelGGL(k_f64_to_f32, dim3(grid_for(n)), dim3(256), 0, s, n, x, y);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

int vec_dot_partial(hipStream_t s, int64_t n, const double *x0, const double *y0,
                    const double *x1, const double *y1, double *partial) {
    hipLaunchKernelGGL(k_dot_partial, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s,
                       n, x0, y0, x1, y1, partial);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

int sum_partials(hipStream_t s, const double *partial, int nparts, int stride,
                 int nk, double *out, int op) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(RED_THREADS), 0, s,
                       partial, nparts, stride, nk, out, op);
    KRY_HIP(hipGetLastError());
    return KRY_OK;
}

// host-side dot through the two-stage reduction
static int host_dot(hipStream_t s, int64_t n, const double *x, const double *y,
                    double *out) {
    DBuf<double> part, res;
    KRY_TRY(part.alloc(RED_BLOCKS * 2));
    KRY_TRY(res.alloc(2));
    KRY_TRY(vec_dot_partial(s, n, x, y, nullptr, nullptr, part.p));
    KRY_TRY(sum_partials(s, part.p, RED_BLOCKS, 2, 1, res.p, SUM_PLAIN));
    KRY_HIP(hipMemcpyAsync(out, res.p, sizeof(double), hipMemcpyDeviceToHost, s));
    KRY_HIP(hipStreamSynchronize(s));
    return KRY_OK;
}

}  // namespace kry

using namespace kry;

// ===========================================================================
// C ABI: errors, stream, timing
// ===========================================================================
extern "C" const char *LastError(void) { return g_err; }

extern "C" int KrylovSetStream(void *stream) {
    g_stream = static_cast<hipStream_t>(stream);
    return KRY_OK;
}

extern "C" int KernelTimingEnable(int on) {
    g_timing_on = on != 0;
    return KRY_OK;
}

extern "C" int KernelTimingSelect(const char *names) {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing_only.clear();
    if (!names) return KRY_OK;
    std::string cur;
    for (const char *c = names;; c++) {
        if (*c == ',' || *c == '\0') {
            if (!cur.empty()) g_timing_only.push_back(cur);
            cur.clear();
            if (*c == '\0') break;
        } else {
            cur += *c;
        }
    }
    return KRY_OK;
}

extern "C" int KernelTimingSample(int every) {
    if (every < 1) return set_error(KRY_ERR_ARG, "KernelTimingSample: every must be >= 1");
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing_every = every;
    g_timing_seen.clear();
    return KRY_OK;
}

extern "C" int KernelTimingReset(void) {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing_seen.clear();
    for (auto &kv : g_timing) {
        for (auto &pr : kv.second.ev) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        if (kv.second.open) (void)hipEventDestroy(kv.second.open);
    }
    g_timing.clear();
    return KRY_OK;
}

extern "C" int KernelTimingQuery(const char *name, int64_t *launches, double *total_ms) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!name) return set_error(KRY_ERR_ARG, "KernelTimingQuery: name is NULL");
    auto it = g_timing.find(name);
    int64_t cnt = 0;
    double tot = 0.0;
    if (it != g_timing.end()) {
        for (auto &pr : it->second.ev) {
            if (hipEventSynchronize(pr.second) != hipSuccess)
                return set_error(KRY_ERR_HIP, "KernelTimingQuery: event sync failed");
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess)
                return set_error(KRY_ERR_HIP, "KernelTimingQuery: elapsed time failed");
            tot += ms;
            cnt++;
        }
    }
    if (launches) *launches = cnt;
    if (total_ms) *total_ms = tot;
    return KRY_OK;
}

// ===========================================================================
// C ABI: MAP (Section 2.1)
// ===========================================================================
extern "C" MAP *MapCreate(int64_t ilower, int64_t iupper) {
    if (!(ilower < iupper)) {
        set_error(KRY_ERR_ARG, "MapCreate: need ilower < iupper (got %lld, %lld)",
                  (long long)ilower, (long long)iupper);
        return nullptr;
    }
    MAP *m = new MAP_();
    m->ilower = ilower;
    m->iupper = iupper;
    m->nlocal = iupper - ilower;
    m->nglobal = m->nlocal;
    m->offset[0] = 0;
    m->offset[1] = m->nglobal;
    return m;
}

extern "C" MAP *MapCreateLocal(int64_t nlocal) {
    if (nlocal <= 0) {
        set_error(KRY_ERR_ARG, "MapCreateLocal: nlocal must be positive");
        return nullptr;
    }
    return MapCreate(0, nlocal);
}

extern "C" void MapDestroy(MAP *map) { delete map; }

extern "C" int64_t MapGetNlocal(const MAP *map) { return map ? map->nlocal : -1; }

// ===========================================================================
// C ABI: VEC (Section 2.2)
// ===========================================================================
extern "C" VEC *VecCreate(MAP *map, int dtype) {
    if (!map) { set_error(KRY_ERR_ARG, "VecCreate: map is NULL"); return nullptr; }
    if (dtype != KRY_F64) { set_error(KRY_ERR_UNSUPPORTED, "VecCreate: only KRY_F64"); return nullptr; }
    VEC *v = new VEC_();
    v->map = map;
    v->n = map->nlocal;
    v->dtype = dtype;
    if (hipMalloc(reinterpret_cast<void **>(&v->data), sizeof(double) * v->n) != hipSuccess) {
        delete v;
        set_error(KRY_ERR_ALLOC, "VecCreate: hipMalloc failed");
        return nullptr;
    }
    v->owned = true;
    if (hipMemsetAsync(v->data, 0, sizeof(double) * v->n, g_stream) != hipSuccess ||
        hipStreamSynchronize(g_stream) != hipSuccess) {
        (void)hipFree(v->data);
        delete v;
        set_error(KRY_ERR_HIP, "VecCreate: clearing failed");
        return nullptr;
    }
    return v;
}

extern "C" VEC *VecWrap(MAP *map, void *device_ptr, int dtype) {
    if (!map || !device_ptr) { set_error(KRY_ERR_ARG, "VecWrap: NULL argument"); return nullptr; }
    if (dtype != KRY_F64) { set_error(KRY_ERR_UNSUPPORTED, "VecWrap: only KRY_F64"); return nullptr; }
    VEC *v = new VEC_();
    v->map = map;
    v->n = map->nlocal;
    v->dtype = dtype;
    v->data = static_cast<double *>(device_ptr);
    v->owned = false;
    return v;
}

extern "C" void VecDestroy(VEC **vec) {
    if (!vec || !*vec) return;
    if ((*vec)->owned && (*vec)->data) (void)hipFree((*vec)->data);
    delete *vec;
    *vec = nullptr;
}

extern "C" void *VecGetData(VEC *vec) { return vec ? vec->data : nullptr; }

extern "C" int VecAddEntry(VEC *vec, int64_t idx, double value) {
    if (!vec || idx < 0 || idx >= vec->n) return set_error(KRY_ERR_ARG, "VecAddEntry: bad index");
    double h;
    KRY_HIP(hipMemcpyAsync(&h, vec->data + idx, sizeof(double), hipMemcpyDeviceToHost, g_stream));
    KRY_HIP(hipStreamSynchronize(g_stream));
    h += value;
    KRY_HIP(hipMemcpyAsync(vec->data + idx, &h, sizeof(double), hipMemcpyHostToDevice, g_stream));
    KRY_HIP(hipStreamSynchronize(g_stream));
    return KRY_OK;
}

extern "C" double VecGetEntry(VEC *vec, int64_t idx) {
    if (!vec || idx < 0 || idx >= vec->n) {
        set_error(KRY_ERR_ARG, "VecGetEntry: bad index");
        return NAN;
    }
    double h = NAN;
    if (hipMemcpyAsync(&h, vec->data + idx, sizeof(double), hipMemcpyDeviceToHost, g_stream) != hipSuccess ||
        hipStreamSynchronize(g_stream) != hipSuccess) {
        set_error(KRY_ERR_HIP, "VecGetEntry: copy failed");
        return NAN;
    }
    return h;
}

extern "C" int VecSetValue(VEC *x, double v) {
    if (!x) return set_error(KRY_ERR_ARG, "VecSetValue: NULL vector");
    return vec_fill(g_stream, x->n, x->data, v);
}

extern "C" int VecAXPBY(double alpha, VEC *x, double beta, VEC *y) {
    if (!x || !y) return set_error(KRY_ERR_ARG, "VecAXPBY: NULL vector");
    if (x->n != y->n) return set_error(KRY_ERR_DIM, "VecAXPBY: sizes differ");
    return vec_axpbyz(g_stream, x->n, hc(alpha), x->data, hc(beta), y->data, y->data);
}

extern "C" int VecAXPBYZ(double alpha, VEC *x, double beta, VEC *y, VEC *z) {
    if (!x || !y || !z) return set_error(KRY_ERR_ARG, "VecAXPBYZ: NULL vector");
    if (x->n != y->n || y->n != z->n) return set_error(KRY_ERR_DIM, "VecAXPBYZ: sizes differ");
    return vec_axpbyz(g_stream, x->n, hc(alpha), x->data, hc(beta), y->data, z->data);
}

extern "C" double VecDot(VEC *x, VEC *y) {
    if (!x || !y) { set_error(KRY_ERR_ARG, "VecDot: NULL vector"); return NAN; }
    if (x->n != y->n) { set_error(KRY_ERR_DIM, "VecDot: sizes differ"); return NAN; }
    double r = NAN;
    if (host_dot(g_stream, x->n, x->data, y->data, &r) != KRY_OK) return NAN;
    return r;
}

// ---------------------------------------------------------------------------
// Allocation-free dot product.  The partial sums of its reduction live in a
// file-scope device array (one copy per GPU, held until the process ends);
// host code reaches it only through the address hipGetSymbolAddress gives
// on each device (the array's name is a host-side stand-in there).
// ---------------------------------------------------------------------------
constexpr int NOALLOC_MAX_PARTS = 2 * RED_BLOCKS;   // doubles of partial sums
static __device__ __align__(256) double scratch[NOALLOC_MAX_PARTS];
constexpr int NOALLOC_MAX_DEVICES = 64;
static double *g_scratch_dev[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

// the scratch array's device address on the current device (looked up once
// per device, with that device current)
static int scratch_ptr(double **out) {
    int dev = 0;
    KRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return set_error(KRY_ERR_ARG, "VecDotNoAlloc: device %d beyond the %d supported", dev,
                         NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(KRY_ERR_HIP, "VecDotNoAlloc: hipGetSymbolAddress failed: %s",
                             hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_dev[dev];
    return KRY_OK;
}

extern "C" int VecDotNoAlloc(VEC *x, VEC *y, double *result_dev) {
    if (!x || !y || !result_dev) return set_error(KRY_ERR_ARG, "VecDotNoAlloc: NULL argument");
    if (x->n != y->n) return set_error(KRY_ERR_DIM, "VecDotNoAlloc: sizes differ");
    // the reduction's partials: RED_BLOCKS slots of stride 2, every slot
    // written by its block before the final sum reads it (nothing to clear)
    constexpr int parts = 2 * RED_BLOCKS;
    static_assert(parts <= NOALLOC_MAX_PARTS, "scratch holds the reduction's partials");
    if (parts > NOALLOC_MAX_PARTS)
        return set_error(KRY_ERR_ARG, "VecDotNoAlloc: %d partials exceed the scratch of %d",
                         parts, NOALLOC_MAX_PARTS);
    double *part = nullptr;
    KRY_TRY(scratch_ptr(&part));
    KRY_TRY(vec_dot_partial(g_stream, x->n, x->data, y->data, nullptr, nullptr, part));
    return sum_partials(g_stream, part, RED_BLOCKS, 2, 1, result_dev, SUM_PLAIN);
}

extern "C" double VecNorm2(VEC *x) {
    double d = VecDot(x, x);
    return std::isnan(d) ? d : std::sqrt(d);
}
