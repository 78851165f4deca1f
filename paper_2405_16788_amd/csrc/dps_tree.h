// dps_tree.h -- host-side tree object and the internal entry points of libdps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "dps.h"
#include "dps_internal.h"

// launch flag (dps_set_launch) beyond the traversal bits of dps_internal.h:
// the ray march gives each lane one ray (64 consecutive rays per wavefront)
// instead of each wavefront a chunk of one ray's samples
constexpr int kFlagMarchWhole = 16;

struct dps_tree_s {
    uint64_t magic;
    int device;
    int64_t M, N;
    int C, leaf_size, depth;
    dps_storage storage;
    int kernel;       // DPS_KERNEL_DIPOLE or DPS_KERNEL_MONOPOLE
    int kw;           // moment components per channel: 3 (dipole vectors) or 1 (monopole charges)
    int mom_stride;   // elements per node row of `mom`
    int attr_stride;  // elements per point row of `attr`
    int64_t level_start[dps::kLevels + 2];  // nodes of level l: [level_start[l], level_start[l+1])
    int64_t n_top;    // nodes with level <= kTopLevels (FP32 moment rows of BF16 storage)
    bool wide_top;    // FP64 accumulation of top-level moments
    int packet_query;    // queries per lane in dps_query (1, 2, 4)
    int packet_adjoint;  // queries per lane in dps_adjoint_accumulate (1, 2, 4)
    int launch_flags;    // kFlag* bits: XCD-contiguous order / persistent launch per kernel
    int split_query;     // parts of the subtree-split query walk (1: unsplit; dps_set_split)
    int split_adjoint;   // the same for the adjoint accumulation
    int split_cut;       // level at which the split walks divide the tree
    uint32_t step_limit; // nodes one traversal may walk (dps_set_step_limit; default N)
    uint32_t *ctr;       // [16] tile counters of the persistent launches (query, adjoint)

    uint64_t *codes;          // [M] sorted Morton codes
    uint32_t *perm;           // [M] sorted position -> caller index
    dps::PointRec *pts;       // [M]
    dps::NodeRec *nodes;      // [N]
    int32_t *level, *parent, *first_child, *nchild, *ptb, *ptc;  // [N] topology
    int32_t *leaf_of;         // [M] leaf holding each sorted point
    void *mom;                // moments, moment_bytes(): [N][mom_stride] FP32, or for BF16
                              // storage n_top FP32 rows then N BF16 rows (dps_internal.h)
    void *attr;               // [M][attr_stride] FP32 or BF16
    float *nrm;               // [M][3] point normals as given (sorted order; the refit's exact products)
    float *momw;              // [N][kw C] FP32 working sums of the refit (high parts)
    float *momw_lo;           // [N][kw C] their low parts (compensated FP32 sums)
    double *momw64;           // [n_top][kw C] FP64 working sums (wide_top only)
    double *G;                // [N][C][kw] node adjoint accumulators
    double *P;                // [M][C] point adjoint accumulators
    double *S;                // [N][C][kw] push-down running sums
    double *PN;               // [M][3] near-field dL/dn accumulators (sorted order)
    double *EACC;             // [1] dL/deps accumulator
    uint32_t *err;            // sticky device error word (traversal guard)
    float *ray_ws;            // [rays][chunks][2] crossing values of the ray-major march (one of allocs)
    int64_t ray_ws_bytes;     // its size

    int64_t bytes;            // device bytes held by the tree
    int64_t scratch_bytes;    // device bytes of the build's temporary buffers (while building)
    std::vector<void *> allocs;
};

namespace dps {

constexpr uint64_t kMagic = 0x6470732d74726565ull;

void set_error(const char *fmt, ...);
dps_status hip_status(hipError_t e, const char *what);

// dps_set_memory_limit: device bytes one build may hold (tree plus build
// scratch); 0 = no cap.  True if `more` bytes fit beside what t holds.
bool memory_fits(const dps_tree_s *t, size_t more);

// Allocates `count` elements on the current device and records the block in the tree.
template <class T>
dps_status tree_alloc(dps_tree_s *t, T **ptr, size_t count) {
    *ptr = nullptr;
    if (count == 0) count = 1;
    if (!memory_fits(t, count * sizeof(T))) {
        set_error("device memory limit of dps_set_memory_limit reached");
        return DPS_ERR_OOM;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) return hip_status(e, "hipMalloc");
    t->allocs.push_back(p);
    t->bytes += (int64_t)(count * sizeof(T));
    *ptr = (T *)p;
    return DPS_OK;
}

dps_status build_tree(dps_tree_s *t, const float *p, const float *n, const float *A,
                      hipStream_t s);
dps_status refit_moments(dps_tree_s *t, const float *attrs, hipStream_t s);
dps_status launch_query(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float beta, float eps,
                        int cbegin, int nc, float *f, float *g, hipStream_t s);
// monopole-kernel trees (dps_mono.hip)
dps_status launch_query_mono(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float beta, float eps,
                             int cbegin, int nc, float *f, float *g, hipStream_t s);
dps_status launch_adjoint_mono(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float beta, float eps,
                               int cbegin, int nc, const float *df, float *dx, hipStream_t s);
// ray front-end (dps_rays.hip)
dps_status launch_ray_march(dps_tree_s *t, const float *o, const float *d, const float *tn, const float *tf,
                            int64_t R, int n, float beta, float eps, int channel, float level, int32_t *hit,
                            float *hv, hipStream_t s);
dps_status launch_ray_march_harnack(dps_tree_s *t, const float *o, const float *d, const float *tn, const float *tf,
                                    int64_t R, int n, float beta, float eps, int channel, float level, float lower,
                                    int32_t *hit, float *hv, int32_t *evals, hipStream_t s);
dps_status launch_ray_resample(const float *o, const float *d, const float *tn, const float *tf, int64_t R,
                               int n_march, const int32_t *hit, const float *hv, float level, const float *u, int nb,
                               int nd, int na, float window, int tile_layout, float *t_out, float *x_out,
                               hipStream_t s);
dps_status launch_counts(dps_tree_s *t, const float *x, int64_t Q, float beta,
                         int32_t *counts, hipStream_t s);
// Working buffers of a value adjoint: node accumulators G [N][C][kw], point
// accumulators P [M][C], push-down sums S (may alias G: the push-down reads
// a leaf's own entry before overwriting it and never writes an ancestor's),
// and 16 tile counters.  By default the tree's own.
struct AccBuffers {
    double *G, *P, *S;
    uint32_t *ctr;
};
inline AccBuffers tree_buffers(const dps_tree_s *t) { return AccBuffers{t->G, t->P, t->S, t->ctr}; }

// gin: the forward query's gradients at x ([Q][nc][3]) to form dL/dx from, or NULL
// ab: the working buffers, or NULL for the tree's own
dps_status launch_adjoint(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float beta, float eps,
                          int cbegin, int nc, const float *df, float *dx, const float *gin, hipStream_t s,
                          const AccBuffers *ab = nullptr);
// clears G and P of ab (fill kernels); dattrs [M][C] from ab (dipole trees)
dps_status launch_zero_acc(dps_tree_s *t, const AccBuffers &ab, hipStream_t s);
dps_status launch_finalize_acc(dps_tree_s *t, float *dattrs, const AccBuffers &ab, hipStream_t s);
dps_status launch_adjoint_g(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float beta, float eps,
                            int cbegin, int nc, const float *df, const float *dg, int want, float *dx,
                            hipStream_t s);
dps_status launch_finalize_ext(dps_tree_s *t, float *dattrs, float *dnormals, double *deps, hipStream_t s);
dps_status launch_set_normals(dps_tree_s *t, const float *n, hipStream_t s);
dps_status launch_query_grid(dps_tree_s *t, const float origin[3], const float spacing[3], const int64_t dims[3],
                             float beta, float eps, int cbegin, int nc, float *f, float *g, hipStream_t s);
dps_status launch_zero(dps_tree_s *t, hipStream_t s);
dps_status launch_finalize(dps_tree_s *t, float *dattrs, hipStream_t s);
dps_status launch_export(dps_tree_s *t, int32_t *nodes, float *geom, float *moments,
                         hipStream_t s);
dps_status check_inputs(const float *p, const float *n, const float *A, const float *attrs,
                        int64_t M, int C, hipStream_t s, bool *ok);

// Device-wide scans of uint32 (in place allowed): out[i] = sum of in[0..i] (inclusive)
// or in[0..i) (exclusive).  `tmp` must hold scan_tmp_words(n) words.
size_t scan_tmp_words(int64_t n);
dps_status device_scan(const uint32_t *in, uint32_t *out, int64_t n, bool inclusive,
                       uint32_t *tmp, hipStream_t s);

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// the step guard of every traversal: a well-formed tree is walked in at most
// N steps
inline uint32_t walk_limit(const dps_tree_s *t) { return t->step_limit ? t->step_limit : (uint32_t)t->N; }

// kernel parameters of a traversal on tree t at regularisation eps
inline KernelParams tree_kernel_params(const dps_tree_s *t, float eps) {
    KernelParams kp = make_kernel_params(eps);
    kp.nhi = t->storage == DPS_STORE_BF16 ? (uint32_t)t->n_top : 0u;
    return kp;
}

// the moment pointer the traversal kernels take: with BF16 storage the first
// bfloat16 row (the FP32 rows of the top nodes sit just before it)
inline const void *trav_mom(const dps_tree_s *t) {
    return t->storage == DPS_STORE_BF16 ? (const void *)((const uint16_t *)t->mom + 2 * t->n_top * t->mom_stride)
                                        : (const void *)t->mom;
}

// bytes of the moment array
inline size_t moment_bytes(const dps_tree_s *t) {
    return t->storage == DPS_STORE_BF16 ? (size_t)(t->N + 2 * t->n_top) * t->mom_stride * 2
                                        : (size_t)t->N * t->mom_stride * 4;
}

}  // namespace dps
