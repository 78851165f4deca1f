// dps_trav_common.h -- pieces shared by the traversal translation units:
// moment / attribute loads, launch-shape helpers (XCD order, persistent tile
// queue), the kernel parameter lists, grid query mapping, and the wavefront
// reduce-scatter into FP64 accumulators.  Everything here has internal
// linkage (each translation unit gets its own copy).
#pragma once

#include <algorithm>

#include "dps_tree.h"

namespace dps {
namespace {

constexpr int kThreads = 256;

// squared distance given to the radial factors for a query or point that takes
// no part in a term: finite factors on the plain path, then replaced by zero
constexpr float kHugeR2 = 1.0e30f;

// Row i of an array of rows of `row_bytes` bytes: a 32 x 32-bit product, so
// the address costs two scalar multiplies and a 64-bit add.
__device__ __forceinline__ const void *row_at(const void *base, uint32_t i, uint32_t row_bytes) {
    return (const char *)base + (uint64_t)i * row_bytes;
}

// Node moments of channels [c0, c0 + CB) of node t (wave-uniform), as
// floats.  BF16 storage holds a bfloat16 row for every node, after the FP32
// rows of the first nhi nodes (the top levels, whose moments dominate
// queries that take few far-field sources); the traversals get `mom`
// pointing at the first bfloat16 row, so FP32 row t < nhi sits (nhi - t)
// rows of ms floats before it.  load_moments reads the bfloat16 row,
// branch-free, and a far-field block refines the moments of a top-level node
// to its FP32 row with refine_moments.
template <int CB, bool BF16>
__device__ __forceinline__ void load_moments(const void *__restrict__ mom, int ms, uint32_t t, int c0,
                                             float (&D)[3 * CB], uint32_t nhi) {
    if constexpr (!BF16) {
        const float *b = (const float *)row_at(mom, t, (uint32_t)ms * 4u) + 3 * c0;
#pragma unroll
        for (int i = 0; i < 3 * CB; ++i) D[i] = b[i];
    } else {
        const uint32_t *b = (const uint32_t *)((const uint16_t *)row_at(mom, t, (uint32_t)ms * 2u) + 3 * c0);
        constexpr int W = (3 * CB + 1) / 2;
        uint32_t w[W];
#pragma unroll
        for (int i = 0; i < W; ++i) w[i] = b[i];
#pragma unroll
        for (int i = 0; i < 3 * CB; ++i) D[i] = (i & 1) ? bf16_hi(w[i >> 1]) : bf16_lo(w[i >> 1]);
    }
}

// Waits for this wave's scalar loads inside the (rare) branch that issued
// them, so that the common path, which uses moments loaded one node ahead,
// does not wait on the next node's prefetch at the first use of D.
__device__ __forceinline__ void wait_scalar_loads() {
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0); vmcnt, expcnt left at their maxima
}

template <int CB, bool BF16>
__device__ __forceinline__ void refine_moments(const void *__restrict__ mom, int ms, uint32_t t, int c0,
                                               float (&D)[3 * CB], uint32_t nhi) {
    if constexpr (BF16) {
        if (t < nhi) {
            const float *b = (const float *)mom - (size_t)(nhi - t) * ms + 3 * c0;
#pragma unroll
            for (int i = 0; i < 3 * CB; ++i) D[i] = b[i];
            wait_scalar_loads();
        }
    }
}

// Scalar node charges (monopole trees) of channels [c0, c0 + CB), same layout
// with one component per channel.
template <int CB, bool BF16>
__device__ __forceinline__ void load_charges(const void *__restrict__ mom, int ms, uint32_t t, int c0,
                                             float (&Q)[CB], uint32_t nhi) {
    if constexpr (!BF16) {
        const float *b = (const float *)row_at(mom, t, (uint32_t)ms * 4u) + c0;
#pragma unroll
        for (int i = 0; i < CB; ++i) Q[i] = b[i];
    } else {
        const uint32_t *b = (const uint32_t *)((const uint16_t *)row_at(mom, t, (uint32_t)ms * 2u) + c0);
        constexpr int W = (CB + 1) / 2;
        uint32_t w[W];
#pragma unroll
        for (int i = 0; i < W; ++i) w[i] = b[i];
#pragma unroll
        for (int i = 0; i < CB; ++i) Q[i] = (i & 1) ? bf16_hi(w[i >> 1]) : bf16_lo(w[i >> 1]);
    }
}

template <int CB, bool BF16>
__device__ __forceinline__ void refine_charges(const void *__restrict__ mom, int ms, uint32_t t, int c0,
                                               float (&Q)[CB], uint32_t nhi) {
    if constexpr (BF16) {
        if (t < nhi) {
            const float *b = (const float *)mom - (size_t)(nhi - t) * ms + c0;
#pragma unroll
            for (int i = 0; i < CB; ++i) Q[i] = b[i];
            wait_scalar_loads();
        }
    }
}

template <int CB, bool BF16>
__device__ __forceinline__ void load_attrs(const void *__restrict__ attr, int as, uint32_t j, int c0,
                                           float (&mu)[CB]) {
    if constexpr (!BF16) {
        const float *b = (const float *)row_at(attr, j, (uint32_t)as * 4u) + c0;
#pragma unroll
        for (int i = 0; i < CB; ++i) mu[i] = b[i];
    } else {
        const uint32_t *b = (const uint32_t *)((const uint16_t *)row_at(attr, j, (uint32_t)as * 2u) + c0);
        constexpr int W = (CB + 1) / 2;
        uint32_t w[W];
#pragma unroll
        for (int i = 0; i < W; ++i) w[i] = b[i];
#pragma unroll
        for (int i = 0; i < CB; ++i) mu[i] = (i & 1) ? bf16_hi(w[i >> 1]) : bf16_lo(w[i >> 1]);
    }
}

// The points [first, first + count) of a bucket leaf in order, fn(j, rec, mu)
// once per point.  The record and attributes of point j + 1 are requested as
// soon as those of point j have arrived, so their latency runs under point j's
// arithmetic instead of before it.  Scalar loads may return out of order and a
// wait covers every load in flight, so each wait is placed explicitly, before
// the next point's loads are issued (a wait the compiler put at the first use
// of the current point's registers would also wait for them).  Two register
// sets alternate, so no record is copied.  Blocks of more than 4 channels
// keep the plain loop (PIPE = false): a second set of their attributes does
// not fit in the scalar registers.  So do packets of several queries per
// lane: they have other wavefronts to cover the latency, and the pipelined
// loop made the compiler copy their accumulators on every leaf.
// A leaf holds at least one point (count >= 1), so the loops test at the end.
template <int CB, bool BF16, bool PIPE = (CB <= 4), class Fn>
__device__ __forceinline__ void for_leaf_points(const PointRec *__restrict__ pts, const void *__restrict__ attr,
                                                int as, int c0, uint32_t first, uint32_t count, Fn &&fn) {
    const uint32_t je = first + count;
    uint32_t j = first;
    if constexpr (!PIPE) {
        do {
            const PointRec r = pts[j];
            float m[CB];
            load_attrs<CB, BF16>(attr, as, j, c0, m);
            fn(j, r, m);
        } while (++j < je);
        return;
    }
    PointRec ra = pts[first];
    float ma[CB];
    load_attrs<CB, BF16>(attr, as, first, c0, ma);
    do {
        wait_scalar_loads();
        const uint32_t j1 = j + 1 < je ? j + 1 : j;
        const PointRec rb = pts[j1];
        float mb[CB];
        load_attrs<CB, BF16>(attr, as, j1, c0, mb);
        fn(j, ra, ma);
        if (j + 1 >= je) break;
        wait_scalar_loads();
        const uint32_t j2 = j + 2 < je ? j + 2 : j1;
        ra = pts[j2];
        load_attrs<CB, BF16>(attr, as, j2, c0, ma);
        fn(j1, rb, mb);
        j += 2;
    } while (j < je);
}

// ---------------------------------------------------------------------------
// launch shapes
//
// Grid launch: one workgroup per 4 wavefronts of work.  Workgroups are handed
// to the 8 XCDs round-robin; with `remap` the workgroups on one XCD take a
// contiguous eighth of the work, so each XCD's L2 serves one spatial region of
// a coherently ordered query set.
//
// Persistent launch: a grid sized to the resident wavefronts; each wavefront
// pulls 64*K-query tiles from 8 counters, one per contiguous eighth of the
// tiles, starting with the partition of its own XCD and then taking tiles from
// the others, so uneven batches (views of different sizes, shadow rays)
// balance inside one launch.  Every wavefront leaves once all partitions are
// exhausted.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t remap_block(int remap) {
    const int64_t b = blockIdx.x;
    if (!remap) return b;
    const int64_t nb = remap;  // number of logical blocks
    const int64_t per = (nb + 7) / 8;
    const int64_t l = (b % 8) * per + b / 8;
    return l < nb ? l : -1;
}

__device__ __forceinline__ int xcc_id() {
    return (int)(__builtin_amdgcn_s_getreg((3 << 11) | 20) & 7u);  // HW_REG_XCC_ID[3:0]
}

__device__ __forceinline__ int64_t next_tile(uint32_t *__restrict__ ctr, int64_t ntiles, int &part) {
    const int64_t per = (ntiles + 7) / 8;
    for (int a = 0; a < 8; ++a) {
        const int pi = (part + a) & 7;
        uint32_t got = 0;
        if ((threadIdx.x & 63) == 0) got = atomicAdd(&ctr[pi], 1u);
        got = __builtin_amdgcn_readfirstlane(got);
        const int64_t tile = (int64_t)pi * per + got;
        if ((int64_t)got < per && tile < ntiles) {
            part = pi;
            return tile;
        }
    }
    return -1;
}

// ---------------------------------------------------------------------------
// walk state and node tests shared by the traversal bodies
// ---------------------------------------------------------------------------
// A loop-invariant kernel argument held in a vector register.  The far
// test's product b2 * r_t^2 then takes the node radius as its one scalar
// operand (a vector instruction reads at most one scalar register here)
// instead of a copy of the radius made at every node.  v must be
// wave-uniform (a kernel argument): the operand is read from a scalar
// register, so a per-lane value would be taken from one lane.
__device__ __forceinline__ float in_vgpr(float v) {
    float r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(v));
    return r;
}

// Per-lane walk state.  A lane visits the current node iff it opened every
// ancestor of it; along the current path those levels form a prefix, so one
// integer carries them: the lane visits a node of level l iff l <= depth.
// Descending from a level-l node sets depth = min(depth, l) + opened;
// following an escape pointer (to a level <= l) leaves it unchanged, since
// levels above the new node's are never read before the next descent
// rewrites them.  -1: the lane has no query.
__device__ __forceinline__ bool visits(int32_t depth, uint32_t lvl) { return depth >= (int32_t)lvl; }

__device__ __forceinline__ int32_t descend(int32_t depth, uint32_t lvl, bool opened) {
    return min(depth, (int32_t)lvl) + (opened ? 1 : 0);
}

// Wavefront-wide "some lane" tests are formed from the ballots of the plain
// compares (visits, beyond beta r_t): a ballot of a compare is its lane mask
// as it stands, a ballot of a combined predicate is rebuilt with two vector
// instructions.
struct WaveMasks {
    uint64_t far = 0, open = 0;
    __device__ __forceinline__ void add(bool in, bool beyond) {
        const uint64_t bi = __ballot(in), bb = __ballot(beyond);
        far |= bi & bb;
        open |= bi & ~bb;
    }
};

// ---------------------------------------------------------------------------
// Subtree split: the walk of one 64-query tile divided over `parts`
// wavefronts, for batches too small to fill the GPU with one wavefront per
// tile.  Nodes are stored level by level in Morton order, so the nodes of one
// level that lie next to each other in space have consecutive indices; node t
// of level <= cut belongs to part t mod parts.  Every part tests every node
// above the cut level that its queries reach (the decision to open it is the
// same in each) but adds the far-field term of a node only if it owns it;
// a node of the cut level, or a leaf above it, that it does not own is
// skipped with its whole subtree, and inside an owned one the walk is the
// plain one.  So every term of every query is added by exactly one part, the
// one that owns its node's ancestor (or itself) at the cut level.
// ---------------------------------------------------------------------------
struct Split {
    uint32_t part;   // this wavefront's part
    uint32_t mask;   // parts - 1 (parts a power of two)
    uint32_t cut;    // the cut level
};

// whether this part takes node t (level lvl): own -- adds its far-field term;
// skip -- neither tests nor enters it
__device__ __forceinline__ void split_node(const Split &sp, uint32_t t, uint32_t lvl, bool leaf, bool &own,
                                           bool &skip) {
    own = lvl > sp.cut || (t & sp.mask) == sp.part;
    skip = !own && (leaf || lvl == sp.cut);
}

// Shared parameters of the traversal bodies.  f / grad / df rows have `ldo`
// channels and tree channel c0 sits in column co of them (channel subsets).
#define DPS_TRAV_PARAMS                                                                             \
    const NodeRec *__restrict__ nodes, const PointRec *__restrict__ pts,                           \
        const void *__restrict__ mom, const void *__restrict__ attr, int ms, int as,               \
        const float *__restrict__ x, int64_t Q, float b2, KernelParams kp, int c0, int ldo, int co, \
        uint32_t limit, uint32_t *__restrict__ err
#define DPS_TRAV_ARGS nodes, pts, mom, attr, ms, as, x, Q, b2, kp, c0, ldo, co, limit, err
// Kernel entry: Qcap rows, of which the first min(Qcap, *qdev) are processed
// when qdev is given (batch sizes decided on the device, e.g. inside a graph).
#define DPS_KERN_PARAMS                                                                            \
    const NodeRec *__restrict__ nodes, const PointRec *__restrict__ pts,                           \
        const void *__restrict__ mom, const void *__restrict__ attr, int ms, int as,               \
        const float *__restrict__ x, int64_t Qcap, const int64_t *__restrict__ qdev, float b2,     \
        KernelParams kp, int c0, int ldo, int co, uint32_t limit, uint32_t *__restrict__ err
#define DPS_ROWS const int64_t Q = qdev ? (qdev[0] < Qcap ? (qdev[0] > 0 ? qdev[0] : 0) : Qcap) : Qcap

// ---------------------------------------------------------------------------
// grid queries (marching cubes): query q is point (i, j, k) of brick q / 64,
// bricks of 4 x 4 x 4 points in x-fastest order, so a wavefront covers one
// brick and 64k consecutive queries k neighbouring bricks.  Coordinates are
// origin + index * spacing in FP32 without contraction (reproducible).
// ---------------------------------------------------------------------------
struct GridSpec {
    float o[3], h[3];
    int64_t n[3];   // points per axis
    int64_t nb[3];  // bricks per axis
};

__device__ __forceinline__ float grid_coord(float o, int64_t i, float h) {
#pragma clang fp contract(off)
    return o + (float)i * h;
}

// position and output row of grid query q; false outside the grid
__device__ __forceinline__ bool grid_point(const GridSpec &g, int64_t q, float &x, float &y, float &z, int64_t &row) {
    const int64_t b = q >> 6;
    const int l = (int)(q & 63);
    const int64_t bx = b % g.nb[0], byz = b / g.nb[0];
    const int64_t by = byz % g.nb[1], bz = byz / g.nb[1];
    const int64_t i = 4 * bx + (l & 3), j = 4 * by + ((l >> 2) & 3), k = 4 * bz + (l >> 4);
    const bool in = i < g.n[0] && j < g.n[1] && k < g.n[2];
    x = grid_coord(g.o[0], i, g.h[0]);
    y = grid_coord(g.o[1], j, g.h[1]);
    z = grid_coord(g.o[2], k, g.h[2]);
    row = (k * g.n[1] + j) * g.n[0] + i;
    return in;
}

// Adds the wavefront totals of v[0..N) to dst[0..N) with one FP64 atomic per
// value: reduce-scatter in chunks of at most 16 values; in each chunk the lane
// wave_slot names for a value holds its total and issues its atomic.
template <int N_, int B = 0>
__device__ __forceinline__ void scatter_add_node(const float (&v)[N_], int lane, double *dst) {
    constexpr int W = (N_ - B) < 16 ? (N_ - B) : 16;
    float part[W];
#pragma unroll
    for (int k = 0; k < W; ++k) part[k] = v[B + k];
    const float tot = wave_sum_scatter<W>(part);
    const int slot = wave_slot<W>(lane);
    if (slot >= 0) atomicAdd(&dst[B + slot], (double)tot);
    if constexpr (B + 16 < N_) scatter_add_node<N_, B + 16>(v, lane, dst);
}

__global__ void k_fill_u32(uint32_t *__restrict__ a, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

__global__ void k_fill_f64(double *__restrict__ a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0.0;
}

inline unsigned grid(int64_t n) { return (unsigned)std::max<int64_t>(1, cdiv(n, kThreads)); }

// resident workgroups of a kernel on the current device (persistent grid size)
inline unsigned persistent_grid(const void *fn) {
    int dev = 0, ncu = 0, per = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) ncu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kThreads, 0) != hipSuccess || per < 1) per = 1;
    return (unsigned)(ncu * per);
}

struct Sub {       // one channel block of a (possibly partial) channel range
    int c0;        // first tree channel of the block
    int ldo;       // channels per row of f / grad / df
    int co;        // column of c0 in those rows
};

}  // namespace
}  // namespace dps
