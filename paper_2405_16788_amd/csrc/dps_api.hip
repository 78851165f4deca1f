// dps_api.hip -- the C ABI of libdps (declared in include/dps.h): argument
// validation before any device work, handle bookkeeping, error reporting.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <atomic>
#include <mutex>
#include <new>
#include <unordered_map>
#include <unordered_set>

#include "dps_tree.h"

namespace dps {

namespace {
thread_local char g_last_error[512] = "";
std::mutex g_mu;
std::unordered_set<dps_tree_s *> g_live;
std::atomic<int64_t> g_mem_limit{0};  // dps_set_memory_limit (0: no cap)

bool live(dps_tree_s *t) {
    std::lock_guard<std::mutex> lk(g_mu);
    return t && g_live.count(t) && t->magic == kMagic;
}
}  // namespace

bool memory_fits(const dps_tree_s *t, size_t more) {
    const int64_t lim = g_mem_limit.load();
    if (lim <= 0) return true;
    const int64_t held = t ? t->bytes + t->scratch_bytes : 0;
    return (int64_t)more <= lim - held;
}

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
}

dps_status hip_status(hipError_t e, const char *what) {
    if (e == hipSuccess) return DPS_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? DPS_ERR_OOM : DPS_ERR_DEVICE;
}

static void free_tree(dps_tree_s *t) {
    for (void *p : t->allocs) (void)hipFree(p);
    t->allocs.clear();
    t->magic = 0;
    delete t;
}

// cut level of the subtree-split walks until dps_set_split sets one (measured
// best on a 4096-ray batch of the 1M-point cloud, whose octree is 8 levels deep)
constexpr int kDefaultSplitCut = 3;

// largest row count of one call (DPS_MAX_ROWS): keeps every launch's
// workgroup count (rows / 256) within the grid limit of 2^31 - 1
constexpr int64_t kMaxRows = DPS_MAX_ROWS;

static dps_status invalid(const char *msg) {
    set_error("%s", msg);
    return DPS_ERR_INVALID;
}

// Makes the tree's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace dps

using namespace dps;

// ---------------------------------------------------------------------------
// Working memory of dps_adjoint_noalloc: a static device array (each device
// the library runs on holds its own copy until the process ends), so that
// entry point never allocates.  Host code refers to it only through the
// per-device address hipGetSymbolAddress returns: the array's name is a host
// stand-in, not a device address.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kScratchBytes = (size_t)DPS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
std::unordered_map<int, unsigned char *> g_scratch_ptr;  // device -> its copy

// address of device dev's copy (dev current); looked up once per device
dps_status scratch_address(int dev, unsigned char **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return DPS_OK;
    }
    unsigned char *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        dps::set_error("dps_adjoint_noalloc: hipGetSymbolAddress of the workspace failed on device %d: %s", dev,
                       hipGetErrorString(e));
        return DPS_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = ptr;
    *out = ptr;
    return DPS_OK;
}

inline size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }
}  // namespace

extern "C" {

const char *dps_status_string(dps_status s) {
    switch (s) {
        case DPS_OK: return "ok";
        case DPS_ERR_INVALID: return "invalid argument";
        case DPS_ERR_OOM: return "out of device memory";
        case DPS_ERR_DEVICE: return "device error";
        case DPS_ERR_STATE: return "invalid tree handle";
    }
    return "unknown status";
}

const char *dps_last_error(void) { return g_last_error; }

dps_status dps_build(const float *p, const float *n, const float *A, const float *attrs, int64_t M,
                     int32_t C, int32_t leaf_size, dps_storage storage, void *stream, dps_tree *out) {
    return dps_build_kernel(p, n, A, attrs, M, C, leaf_size, storage, DPS_KERNEL_DIPOLE, stream, out);
}

dps_status dps_build_kernel(const float *p, const float *n, const float *A, const float *attrs, int64_t M,
                            int32_t C, int32_t leaf_size, dps_storage storage, dps_kernel kernel, void *stream,
                            dps_tree *out) {
    if (!out) return invalid("dps_build: out is NULL");
    *out = nullptr;
    if (M < 1 || M > 0x7fffffffLL) return invalid("dps_build: M must be in [1, 2^31-1]");
    if (C < 1 || C > DPS_MAX_CHANNELS) return invalid("dps_build: C must be in [1, 32]");
    if (leaf_size < 1 || leaf_size > DPS_MAX_LEAF) return invalid("dps_build: leaf_size must be in [1, 256]");
    if (storage != DPS_STORE_FP32 && storage != DPS_STORE_BF16) return invalid("dps_build: unknown storage mode");
    if (kernel != DPS_KERNEL_DIPOLE && kernel != DPS_KERNEL_MONOPOLE) return invalid("dps_build: unknown kernel");
    if (!p || !n || !A || !attrs) return invalid("dps_build: NULL input array");
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    dps_status st = hip_status(hipGetDevice(&dev), "hipGetDevice");
    if (st != DPS_OK) return st;

    bool ok = false;
    st = check_inputs(p, n, A, attrs, M, C, s, &ok);
    if (st != DPS_OK) return st;
    if (!ok) return invalid("dps_build: non-finite point, normal, area or attribute, or an area <= 0");

    dps_tree_s *t = new (std::nothrow) dps_tree_s();
    if (!t) { set_error("dps_build: host allocation failed"); return DPS_ERR_OOM; }
    t->magic = kMagic;
    t->device = dev;
    t->M = M;
    t->C = C;
    t->leaf_size = leaf_size;
    t->storage = storage;
    t->kernel = kernel;
    t->kw = kernel == DPS_KERNEL_MONOPOLE ? 1 : 3;
    t->wide_top = M >= kWideTopPoints;
    t->packet_query = kDefaultPacketQuery;
    t->packet_adjoint = kDefaultPacketAdjoint;
    t->launch_flags = kDefaultLaunchFlags;
    t->split_query = 1;
    t->split_adjoint = 1;
    t->split_cut = kDefaultSplitCut;
    const bool bf = storage == DPS_STORE_BF16;
    const int kw = t->kw;
    t->mom_stride = bf ? ((kw * C + 1) & ~1) : kw * C;
    t->attr_stride = bf ? ((C + 1) & ~1) : C;

    st = build_tree(t, p, n, A, s);
    if (st == DPS_OK) {
        const size_t esz = bf ? 2 : 4;
        uint8_t *mom = nullptr, *attr = nullptr;
        st = tree_alloc(t, &mom, moment_bytes(t));
        if (st == DPS_OK) st = tree_alloc(t, &attr, (size_t)M * t->attr_stride * esz);
        t->mom = mom;
        t->attr = attr;
        if (st == DPS_OK) st = tree_alloc(t, &t->momw, (size_t)t->N * kw * C);
        if (st == DPS_OK) st = tree_alloc(t, &t->momw_lo, (size_t)t->N * kw * C);
        if (st == DPS_OK && t->wide_top) st = tree_alloc(t, &t->momw64, (size_t)t->n_top * kw * C);
        if (st == DPS_OK) st = tree_alloc(t, &t->G, (size_t)t->N * kw * C);
        if (st == DPS_OK) st = tree_alloc(t, &t->S, (size_t)t->N * kw * C);
        if (st == DPS_OK) st = tree_alloc(t, &t->P, (size_t)M * C);
        if (st == DPS_OK) st = tree_alloc(t, &t->PN, (size_t)M * 3);
        if (st == DPS_OK) st = tree_alloc(t, &t->EACC, 1);
        if (st == DPS_OK) st = tree_alloc(t, &t->err, 1);
        if (st == DPS_OK) st = tree_alloc(t, &t->ctr, 16);
        if (st == DPS_OK) st = hip_status(hipMemsetAsync(t->err, 0, sizeof(uint32_t), s), "zero err");
        if (st == DPS_OK) st = refit_moments(t, attrs, s);
        if (st == DPS_OK) st = hip_status(hipMemsetAsync(t->G, 0, (size_t)t->N * kw * C * sizeof(double), s), "zero G");
        if (st == DPS_OK) st = hip_status(hipMemsetAsync(t->P, 0, (size_t)M * C * sizeof(double), s), "zero P");
        if (st == DPS_OK) st = hip_status(hipMemsetAsync(t->PN, 0, (size_t)M * 3 * sizeof(double), s), "zero PN");
        if (st == DPS_OK) st = hip_status(hipMemsetAsync(t->EACC, 0, sizeof(double), s), "zero eps");
        if (st == DPS_OK) st = hip_status(hipStreamSynchronize(s), "sync build");
    }
    if (st != DPS_OK) {
        (void)hipStreamSynchronize(s);
        free_tree(t);
        return st;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_live.insert(t);
    }
    *out = t;
    return DPS_OK;
}

static dps_status check_tree(dps_tree t, const char *fn) {
    if (!live(t)) {
        set_error("%s: unknown or destroyed tree handle", fn);
        return DPS_ERR_STATE;
    }
    return DPS_OK;
}

// entry points defined for the dipole kernel only
static dps_status need_dipole(dps_tree t, const char *fn) {
    if (t->kernel == DPS_KERNEL_DIPOLE) return DPS_OK;
    set_error("%s: not available for a monopole-kernel tree", fn);
    return DPS_ERR_INVALID;
}

static dps_status check_beta_eps(float beta, float eps, const char *fn) {
    if (!(beta > 0.0f) || !isfinite(beta)) {
        set_error("%s: beta must be finite and > 0", fn);
        return DPS_ERR_INVALID;
    }
    if (!(eps >= 0.0f) || !isfinite(eps)) {
        set_error("%s: eps must be finite and >= 0", fn);
        return DPS_ERR_INVALID;
    }
    return DPS_OK;
}

dps_status dps_set_attributes(dps_tree t, const float *attrs, void *stream) {
    dps_status st = check_tree(t, "dps_set_attributes");
    if (st != DPS_OK) return st;
    if (!attrs) return invalid("dps_set_attributes: attrs is NULL");
    DeviceGuard dg(t->device);
    return refit_moments(t, attrs, (hipStream_t)stream);
}

dps_status dps_query(dps_tree t, const float *x, int64_t Q, float beta, float eps, float *f,
                     float *grad, void *stream) {
    dps_status st = check_tree(t, "dps_query");
    if (st != DPS_OK) return st;
    if ((st = check_beta_eps(beta, eps, "dps_query")) != DPS_OK) return st;
    if (Q < 0 || Q > kMaxRows) return invalid("dps_query: Q out of range");
    if (Q == 0) return DPS_OK;
    if (!x || !f) return invalid("dps_query: NULL x or f");
    DeviceGuard dg(t->device);
    return launch_query(t, x, Q, nullptr, beta, eps, 0, t->C, f, grad, (hipStream_t)stream);
}

static dps_status check_channels(dps_tree t, int32_t c_begin, int32_t n_channels, const char *fn) {
    if (c_begin < 0 || n_channels < 1 || (int64_t)c_begin + n_channels > t->C) {
        set_error("%s: channel range [%d, %d) outside [0, %d)", fn, c_begin, c_begin + n_channels, t->C);
        return DPS_ERR_INVALID;
    }
    if (t->storage == DPS_STORE_BF16 && (c_begin & 1)) {
        set_error("%s: with BF16 storage the first channel must be even", fn);
        return DPS_ERR_INVALID;
    }
    return DPS_OK;
}

dps_status dps_query_channels(dps_tree t, const float *x, int64_t Q, const int64_t *q_count, float beta, float eps,
                              int32_t c_begin, int32_t n_channels, float *f, float *grad, void *stream) {
    dps_status st = check_tree(t, "dps_query_channels");
    if (st != DPS_OK) return st;
    if ((st = check_beta_eps(beta, eps, "dps_query_channels")) != DPS_OK) return st;
    if ((st = check_channels(t, c_begin, n_channels, "dps_query_channels")) != DPS_OK) return st;
    if (Q < 0 || Q > kMaxRows) return invalid("dps_query_channels: Q out of range");
    if (Q == 0) return DPS_OK;
    if (!x || !f) return invalid("dps_query_channels: NULL x or f");
    DeviceGuard dg(t->device);
    return launch_query(t, x, Q, q_count, beta, eps, c_begin, n_channels, f, grad, (hipStream_t)stream);
}

dps_status dps_query_counts(dps_tree t, const float *x, int64_t Q, float beta, int32_t *counts,
                            void *stream) {
    dps_status st = check_tree(t, "dps_query_counts");
    if (st != DPS_OK) return st;
    if ((st = check_beta_eps(beta, 0.0f, "dps_query_counts")) != DPS_OK) return st;
    if (Q < 0 || Q > kMaxRows) return invalid("dps_query_counts: Q out of range");
    if (Q == 0) return DPS_OK;
    if (!x || !counts) return invalid("dps_query_counts: NULL x or counts");
    DeviceGuard dg(t->device);
    return launch_counts(t, x, Q, beta, counts, (hipStream_t)stream);
}

dps_status dps_adjoint_zero(dps_tree t, void *stream) {
    dps_status st = check_tree(t, "dps_adjoint_zero");
    if (st != DPS_OK) return st;
    DeviceGuard dg(t->device);
    return launch_zero(t, (hipStream_t)stream);  // fill kernels: safe inside captured graphs
}

dps_status dps_adjoint_accumulate(dps_tree t, const float *x, int64_t Q, float beta, float eps,
                                  const float *df, float *dx, void *stream) {
    dps_status st = check_tree(t, "dps_adjoint_accumulate");
    if (st != DPS_OK) return st;
    if ((st = check_beta_eps(beta, eps, "dps_adjoint_accumulate")) != DPS_OK) return st;
    if (Q < 0 || Q > kMaxRows) return invalid("dps_adjoint_accumulate: Q out of range");
    if (Q == 0) return DPS_OK;
    if (!x || !df) return invalid("dps_adjoint_accumulate: NULL x or df");
    DeviceGuard dg(t->device);
    return launch_adjoint(t, x, Q, nullptr, beta, eps, 0, t->C, df, dx, nullptr, (hipStream_t)stream);
}

dps_status dps_adjoint_accumulate_channels(dps_tree t, const float *x, int64_t Q, const int64_t *q_count,
                                           float beta, float eps, int32_t c_begin, int32_t n_channels,
                                           const float *df, float *dx, void *stream) {
    dps_status st = check_tree(t, "dps_adjoint_accumulate_channels");
    if (st != DPS_OK) return st;
    if ((st = check_beta_eps(beta, eps, "dps_adjoint_accumulate_channels")) != DPS_OK) return st;
    if ((st = check_channels(t, c_begin, n_channels, "dps_adjoint_accumulate_channels")) != DPS_OK) return st;
    if (Q < 0 || Q > kMaxRows) return invalid("dps_adjoint_accumulate_channels: Q out of range");
    if (Q == 0) return DPS_OK;
    if (!x || !df) return invalid("dps_adjoint_accumulate_channels: NULL x or df");
    DeviceGuard dg(t->device);
    return launch_adjoint(t, x, Q, q_count, beta, eps, c_begin, n_channels, df, dx, nullptr, (hipStream_t)stream);
}

dps_status dps_adjoint_accumulate_from_forward(dps_tree t, const float *x, int64_t Q, const int64_t *q_count,
                                               float beta, float eps, int32_t c_begin, int32_t n_channels,
                                               const float *df, const float *grad, float *dx, void *stream) {
    dps_status st = check_tree(t, "dps_adjoint_accumulate_from_forward");
    if (st != DPS_OK) return st;
    if ((st = need_dipole(t, "dps_adjoint_accumulate_from_forward")) != DPS_OK) return st;
    if ((st = check_beta_eps(beta, eps, "dps_adjoint_accumulate_from_forward")) != DPS_OK) return st;
    if ((st = check_channels(t, c_begin, n_channels, "dps_adjoint_accumulate_from_forward")) != DPS_OK) return st;
    if (Q < 0 || Q > kMaxRows) return invalid("dps_adjoint_accumulate_from_forward: Q out of range");
    if (Q == 0) return DPS_OK;
    if (!x || !df || !grad) return invalid("dps_adjoint_accumulate_from_forward: NULL x, df or grad");
    DeviceGuard dg(t->device);
    return launch_adjoint(t, x, Q, q_count, beta, eps, c_begin, n_channels, df, dx, grad, (hipStream_t)stream);
}

dps_status dps_adjoint_accumulate_grad(dps_tree t, const float *x, int64_t Q, const int64_t *q_count, float beta,
                                       float eps, int32_t c_begin, int32_t n_channels, const float *df,
                                       const float *dg, float *dx, void *stream) {
    dps_status st = check_tree(t, "dps_adjoint_accumulate_grad");
    if (st != DPS_OK) return st;
    if ((st = need_dipole(t, "dps_adjoint_accumulate_grad")) != DPS_OK) return st;
    if ((st = check_beta_eps(beta, eps, "dps_adjoint_accumulate_grad")) != DPS_OK) return st;
    if ((st = check_channels(t, c_begin, n_channels, "dps_adjoint_accumulate_grad")) != DPS_OK) return st;
    if (Q < 0 || Q > kMaxRows) return invalid("dps_adjoint_accumulate_grad: Q out of range");
    if (Q == 0) return DPS_OK;
    if (!x || !dg) return invalid("dps_adjoint_accumulate_grad: NULL x or dg");
    DeviceGuard guard(t->device);
    return launch_adjoint_g(t, x, Q, q_count, beta, eps, c_begin, n_channels, df, dg, 0, dx, (hipStream_t)stream);
}

dps_status dps_adjoint_accumulate_ext(dps_tree t, const float *x, int64_t Q, const int64_t *q_count, float beta,
                                      float eps, int32_t c_begin, int32_t n_channels, const float *df,
                                      const float *dg, int32_t want, float *dx, void *stream) {
    dps_status st = check_tree(t, "dps_adjoint_accumulate_ext");
    if (st != DPS_OK) return st;
    if ((st = need_dipole(t, "dps_adjoint_accumulate_ext")) != DPS_OK) return st;
    if ((st = check_beta_eps(beta, eps, "dps_adjoint_accumulate_ext")) != DPS_OK) return st;
    if ((st = check_channels(t, c_begin, n_channels, "dps_adjoint_accumulate_ext")) != DPS_OK) return st;
    if (want < 0 || want > (DPS_WANT_NORMALS | DPS_WANT_EPS))
        return invalid("dps_adjoint_accumulate_ext: want must be a mask of DPS_WANT_NORMALS and DPS_WANT_EPS");
    if (Q < 0 || Q > kMaxRows) return invalid("dps_adjoint_accumulate_ext: Q out of range");
    if (Q == 0) return DPS_OK;
    if (!x || (!df && !dg)) return invalid("dps_adjoint_accumulate_ext: NULL x, or neither df nor dg");
    DeviceGuard guard(t->device);
    return launch_adjoint_g(t, x, Q, q_count, beta, eps, c_begin, n_channels, df, dg, want, dx, (hipStream_t)stream);
}

dps_status dps_adjoint_finalize_ext(dps_tree t, float *dattrs, float *dnormals, double *deps, void *stream) {
    dps_status st = check_tree(t, "dps_adjoint_finalize_ext");
    if (st != DPS_OK) return st;
    if (!dattrs && !dnormals && !deps) return invalid("dps_adjoint_finalize_ext: no output requested");
    if ((dnormals || deps) && (st = need_dipole(t, "dps_adjoint_finalize_ext")) != DPS_OK) return st;
    DeviceGuard guard(t->device);
    return launch_finalize_ext(t, dattrs, dnormals, deps, (hipStream_t)stream);
}

dps_status dps_query_grid(dps_tree t, const float origin[3], const float spacing[3], const int64_t dims[3], float beta,
                          float eps, int32_t c_begin, int32_t n_channels, float *f, float *grad, void *stream) {
    dps_status st = check_tree(t, "dps_query_grid");
    if (st != DPS_OK) return st;
    if ((st = need_dipole(t, "dps_query_grid")) != DPS_OK) return st;
    if ((st = check_beta_eps(beta, eps, "dps_query_grid")) != DPS_OK) return st;
    if ((st = check_channels(t, c_begin, n_channels, "dps_query_grid")) != DPS_OK) return st;
    if (!origin || !spacing || !dims || !f) return invalid("dps_query_grid: NULL origin, spacing, dims or f");
    int64_t total = 1;
    for (int a = 0; a < 3; ++a) {
        if (!(dims[a] > 0) || dims[a] > ((int64_t)1 << 24))
            return invalid("dps_query_grid: each dimension must be in [1, 2^24]");
        if (!isfinite(origin[a]) || !isfinite(spacing[a])) return invalid("dps_query_grid: non-finite origin or spacing");
        total *= dims[a];
        if (total > kMaxRows) return invalid("dps_query_grid: grid too large");
    }
    DeviceGuard guard(t->device);
    return launch_query_grid(t, origin, spacing, dims, beta, eps, c_begin, n_channels, f, grad, (hipStream_t)stream);
}

dps_status dps_set_normals(dps_tree t, const float *n, void *stream) {
    dps_status st = check_tree(t, "dps_set_normals");
    if (st != DPS_OK) return st;
    if ((st = need_dipole(t, "dps_set_normals")) != DPS_OK) return st;
    if (!n) return invalid("dps_set_normals: n is NULL");
    DeviceGuard guard(t->device);
    return launch_set_normals(t, n, (hipStream_t)stream);
}

dps_status dps_adjoint_finalize(dps_tree t, float *dattrs, void *stream) {
    dps_status st = check_tree(t, "dps_adjoint_finalize");
    if (st != DPS_OK) return st;
    if (!dattrs) return invalid("dps_adjoint_finalize: dattrs is NULL");
    DeviceGuard dg(t->device);
    return launch_finalize(t, dattrs, (hipStream_t)stream);
}

dps_status dps_adjoint(dps_tree t, const float *x, int64_t Q, float beta, float eps, const float *df,
                       float *dattrs, float *dx, void *stream) {
    dps_status st = check_tree(t, "dps_adjoint");
    if (st != DPS_OK) return st;
    if ((st = check_beta_eps(beta, eps, "dps_adjoint")) != DPS_OK) return st;
    if (Q < 0 || Q > kMaxRows) return invalid("dps_adjoint: Q out of range");
    if (!dattrs) return invalid("dps_adjoint: dattrs is NULL");
    if (Q > 0 && (!x || !df)) return invalid("dps_adjoint: NULL x or df");
    if ((st = dps_adjoint_zero(t, stream)) != DPS_OK) return st;
    if (Q > 0 && (st = dps_adjoint_accumulate(t, x, Q, beta, eps, df, dx, stream)) != DPS_OK) return st;
    return dps_adjoint_finalize(t, dattrs, stream);
}

dps_status dps_adjoint_noalloc(dps_tree t, const float *x, int64_t Q, float beta, float eps, const float *df,
                               float *dattrs, float *dx, void *stream) {
    dps_status st = check_tree(t, "dps_adjoint_noalloc");
    if (st != DPS_OK) return st;
    if ((st = need_dipole(t, "dps_adjoint_noalloc")) != DPS_OK) return st;
    if ((st = check_beta_eps(beta, eps, "dps_adjoint_noalloc")) != DPS_OK) return st;
    if (Q < 0 || Q > kMaxRows) return invalid("dps_adjoint_noalloc: Q out of range");
    if (!dattrs) return invalid("dps_adjoint_noalloc: dattrs is NULL");
    if (Q > 0 && (!x || !df)) return invalid("dps_adjoint_noalloc: NULL x or df");
    // node accumulators (also the push-down sums), point accumulators, tile counters
    const size_t gb = align256((size_t)t->N * t->kw * t->C * sizeof(double));
    const size_t pb = align256((size_t)t->M * t->C * sizeof(double));
    const size_t cb = 16 * sizeof(uint32_t);
    if (gb + pb + cb > kScratchBytes) {
        set_error("dps_adjoint_noalloc: this tree needs %zu bytes of workspace (N = %lld nodes, M = %lld points, "
                  "C = %d), more than the %zu of DPS_NOALLOC_SCRATCH_BYTES; use dps_adjoint",
                  gb + pb + cb, (long long)t->N, (long long)t->M, t->C, kScratchBytes);
        return DPS_ERR_INVALID;
    }
    DeviceGuard dg(t->device);
    unsigned char *base = nullptr;
    if ((st = scratch_address(t->device, &base)) != DPS_OK) return st;
    const AccBuffers ab{(double *)base, (double *)(base + gb), (double *)base, (uint32_t *)(base + gb + pb)};
    hipStream_t s = (hipStream_t)stream;
    if ((st = launch_zero_acc(t, ab, s)) != DPS_OK) return st;  // fill kernels, no memset
    if (Q > 0 && (st = launch_adjoint(t, x, Q, nullptr, beta, eps, 0, t->C, df, dx, nullptr, s, &ab)) != DPS_OK)
        return st;
    return launch_finalize_acc(t, dattrs, ab, s);
}

dps_status dps_export_tree(dps_tree t, uint64_t *codes, uint32_t *perm, int32_t *nodes, float *geom,
                           float *moments, void *stream) {
    dps_status st = check_tree(t, "dps_export_tree");
    if (st != DPS_OK) return st;
    DeviceGuard dg(t->device);
    hipStream_t s = (hipStream_t)stream;
    if (codes && (st = hip_status(hipMemcpyAsync(codes, t->codes, t->M * sizeof(uint64_t), hipMemcpyDeviceToDevice, s), "export codes")) != DPS_OK) return st;
    if (perm && (st = hip_status(hipMemcpyAsync(perm, t->perm, t->M * sizeof(uint32_t), hipMemcpyDeviceToDevice, s), "export perm")) != DPS_OK) return st;
    if ((st = launch_export(t, nodes, geom, moments, s)) != DPS_OK) return st;
    return hip_status(hipStreamSynchronize(s), "sync export");
}

dps_status dps_tree_info(dps_tree t, int64_t *n_nodes, int32_t *depth, int64_t *bytes,
                         int64_t *n_points, int32_t *channels) {
    dps_status st = check_tree(t, "dps_tree_info");
    if (st != DPS_OK) return st;
    if (n_nodes) *n_nodes = t->N;
    if (depth) *depth = t->depth;
    if (bytes) *bytes = t->bytes;
    if (n_points) *n_points = t->M;
    if (channels) *channels = t->C;
    return DPS_OK;
}

dps_status dps_ray_march(dps_tree t, const float *o, const float *d, const float *tnear, const float *tfar, int64_t R,
                         int32_t n_samples, float beta, float eps, int32_t channel, float level, int32_t *hit_index,
                         float *hit_values, void *stream) {
    dps_status st = check_tree(t, "dps_ray_march");
    if (st != DPS_OK) return st;
    if ((st = need_dipole(t, "dps_ray_march")) != DPS_OK) return st;
    if ((st = check_beta_eps(beta, eps, "dps_ray_march")) != DPS_OK) return st;
    if ((st = check_channels(t, channel, 1, "dps_ray_march")) != DPS_OK) return st;
    if (n_samples < 2 || n_samples > (1 << 20)) return invalid("dps_ray_march: n_samples must be in [2, 2^20]");
    if (!isfinite(level)) return invalid("dps_ray_march: level must be finite");
    if (R < 0 || R > kMaxRows) return invalid("dps_ray_march: R out of range");
    if (R == 0) return DPS_OK;
    if (!o || !d || !tnear || !tfar || !hit_index || !hit_values) return invalid("dps_ray_march: NULL array");
    DeviceGuard guard(t->device);
    return launch_ray_march(t, o, d, tnear, tfar, R, n_samples, beta, eps, channel, level, hit_index, hit_values,
                            (hipStream_t)stream);
}

dps_status dps_ray_march_harnack(dps_tree t, const float *o, const float *d, const float *tnear, const float *tfar,
                                 int64_t R, int32_t n_samples, float beta, float eps, int32_t channel, float level,
                                 float lower, int32_t *hit_index, float *hit_values, int32_t *evals, void *stream) {
    dps_status st = check_tree(t, "dps_ray_march_harnack");
    if (st != DPS_OK) return st;
    if ((st = need_dipole(t, "dps_ray_march_harnack")) != DPS_OK) return st;
    if ((st = check_beta_eps(beta, eps, "dps_ray_march_harnack")) != DPS_OK) return st;
    if ((st = check_channels(t, channel, 1, "dps_ray_march_harnack")) != DPS_OK) return st;
    if (n_samples < 2 || n_samples > (1 << 20)) return invalid("dps_ray_march_harnack: n_samples must be in [2, 2^20]");
    if (!isfinite(level) || !isfinite(lower) || !(lower < level))
        return invalid("dps_ray_march_harnack: level and lower must be finite with lower < level");
    if (R < 0 || R > kMaxRows) return invalid("dps_ray_march_harnack: R out of range");
    if (R == 0) return DPS_OK;
    if (!o || !d || !tnear || !tfar || !hit_index || !hit_values)
        return invalid("dps_ray_march_harnack: NULL array");
    DeviceGuard guard(t->device);
    return launch_ray_march_harnack(t, o, d, tnear, tfar, R, n_samples, beta, eps, channel, level, lower, hit_index,
                                    hit_values, evals, (hipStream_t)stream);
}

dps_status dps_ray_resample(const float *o, const float *d, const float *tnear, const float *tfar, int64_t R,
                            int32_t n_march, const int32_t *hit_index, const float *hit_values, float level,
                            const float *jitter, int32_t n_before, int32_t n_dense, int32_t n_after, float window,
                            int32_t tile_layout, float *t_out, float *x_out, void *stream) {
    if (n_march < 1 || n_march > (1 << 20)) return invalid("dps_ray_resample: n_march must be in [1, 2^20]");
    if (n_before < 1 || n_dense < 1 || n_after < 1 || (int64_t)n_before + n_dense + n_after > 4096)
        return invalid("dps_ray_resample: sample counts must be >= 1 with a total of at most 4096");
    if (!isfinite(level) || !isfinite(window) || !(window >= 0.0f))
        return invalid("dps_ray_resample: level must be finite and window finite and >= 0");
    if (tile_layout != 0 && tile_layout != 1) return invalid("dps_ray_resample: tile_layout must be 0 or 1");
    if (R < 0 || R > kMaxRows / (n_before + n_dense + n_after)) return invalid("dps_ray_resample: R out of range");
    if (tile_layout && (R % 64)) return invalid("dps_ray_resample: the tile layout needs R to be a multiple of 64");
    if (R == 0) return DPS_OK;
    if (!o || !d || !tnear || !tfar || !hit_index || !hit_values || !jitter || !t_out || !x_out)
        return invalid("dps_ray_resample: NULL array");
    return launch_ray_resample(o, d, tnear, tfar, R, n_march, hit_index, hit_values, level, jitter, n_before, n_dense,
                               n_after, window, tile_layout, t_out, x_out, (hipStream_t)stream);
}

dps_status dps_get_kernel(dps_tree t, int32_t *kernel) {
    dps_status st = check_tree(t, "dps_get_kernel");
    if (st != DPS_OK) return st;
    if (!kernel) return invalid("dps_get_kernel: kernel is NULL");
    *kernel = t->kernel;
    return DPS_OK;
}

dps_status dps_set_launch(dps_tree t, int32_t query_k, int32_t adjoint_k, int32_t flags) {
    dps_status st = check_tree(t, "dps_set_launch");
    if (st != DPS_OK) return st;
    auto ok = [](int32_t k) { return k == 0 || k == 1 || k == 2 || k == 4; };
    if (!ok(query_k) || !ok(adjoint_k)) return invalid("dps_set_launch: packet sizes must be 0 (keep), 1, 2 or 4");
    if (flags < -1 || flags > 31) return invalid("dps_set_launch: flags must be -1 (keep) or a 5-bit mask");
    if (query_k) t->packet_query = query_k;
    if (adjoint_k) t->packet_adjoint = adjoint_k;
    if (flags >= 0) t->launch_flags = flags;
    return DPS_OK;
}

dps_status dps_get_launch(dps_tree t, int32_t *query_k, int32_t *adjoint_k, int32_t *flags) {
    dps_status st = check_tree(t, "dps_get_launch");
    if (st != DPS_OK) return st;
    if (query_k) *query_k = t->packet_query;
    if (adjoint_k) *adjoint_k = t->packet_adjoint;
    if (flags) *flags = t->launch_flags;
    return DPS_OK;
}

dps_status dps_set_split(dps_tree t, int32_t query_parts, int32_t adjoint_parts, int32_t cut_level) {
    dps_status st = check_tree(t, "dps_set_split");
    if (st != DPS_OK) return st;
    auto ok = [](int32_t p) { return p == 0 || p == 1 || p == 2 || p == 4 || p == 8; };
    if (!ok(query_parts) || !ok(adjoint_parts))
        return invalid("dps_set_split: parts must be 0 (keep), 1, 2, 4 or 8");
    if (cut_level < -1 || cut_level > kLevels) return invalid("dps_set_split: cut_level must be -1 (keep) or a level in [0, 21]");
    if (query_parts) t->split_query = query_parts;
    if (adjoint_parts) t->split_adjoint = adjoint_parts;
    if (cut_level >= 0) t->split_cut = cut_level;
    return DPS_OK;
}

dps_status dps_get_split(dps_tree t, int32_t *query_parts, int32_t *adjoint_parts, int32_t *cut_level) {
    dps_status st = check_tree(t, "dps_get_split");
    if (st != DPS_OK) return st;
    if (query_parts) *query_parts = t->split_query;
    if (adjoint_parts) *adjoint_parts = t->split_adjoint;
    if (cut_level) *cut_level = t->split_cut;
    return DPS_OK;
}

dps_status dps_set_step_limit(dps_tree t, int64_t limit) {
    dps_status st = check_tree(t, "dps_set_step_limit");
    if (st != DPS_OK) return st;
    if (limit < 0 || limit > t->N) return invalid("dps_set_step_limit: limit must be in [0, node count]");
    t->step_limit = (uint32_t)limit;
    return DPS_OK;
}

dps_status dps_set_memory_limit(int64_t bytes) {
    if (bytes < 0) return invalid("dps_set_memory_limit: bytes must be >= 0");
    g_mem_limit.store(bytes);
    return DPS_OK;
}

dps_status dps_check(dps_tree t, void *stream) {
    dps_status st = check_tree(t, "dps_check");
    if (st != DPS_OK) return st;
    DeviceGuard dg(t->device);
    hipStream_t s = (hipStream_t)stream;
    uint32_t h = 0;
    if ((st = hip_status(hipMemcpyAsync(&h, t->err, sizeof h, hipMemcpyDeviceToHost, s), "read error word")) != DPS_OK) return st;
    if ((st = hip_status(hipStreamSynchronize(s), "dps_check sync")) != DPS_OK) return st;
    if (h) {
        set_error("dps_check: a traversal exceeded the node count (internal error, code %u)", h);
        return DPS_ERR_DEVICE;
    }
    return DPS_OK;
}

void dps_destroy(dps_tree t) {
    if (!t) return;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_live.count(t)) return;
        g_live.erase(t);
    }
    DeviceGuard dg(t->device);
    (void)hipDeviceSynchronize();
    free_tree(t);
}

}  // extern "C"
