// dps_build.hip -- octree construction on the GPU (Sec. 6.1 and 6.3 of the paper:
// an octree over the fixed point positions, built once, whose nodes carry
// area, area-weighted centroid and radius, eq. farfield_dipole).
//
// Pipeline (all on `stream`):
//   1. input check (finite values, positive areas)
//   2. bounding box (exact FP32 min / max)
//   3. 63-bit Morton codes from an FP64 quantisation of the cube
//   4. stable LSD radix sort of (code, index): per-block LDS digit histograms,
//      device-wide scan, LDS-ranked stable scatter (8 passes of 8 bits)
//   5. level-by-level topology: split flags where the next 3-bit digit changes,
//      scan -> breadth-first node numbers, children contiguous
//   6. FP64 node sums bottom-up in a fixed order, centroid rounded once to FP32,
//      squared radius = max FP32 point distance (order-free)
//   7. depth-first escape pointers and the packed 32-byte node records
#include <math.h>

#include <algorithm>

#include "dps_tree.h"

namespace dps {

namespace {

constexpr int kThreads = 256;

// ---------------------------------------------------------------------------
// 1. input check
// ---------------------------------------------------------------------------
__global__ void k_check(const float *__restrict__ p, const float *__restrict__ n,
                        const float *__restrict__ A, const float *__restrict__ attrs, int64_t M,
                        int C, uint32_t *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool b = false;
    for (; i < M; i += stride) {
        for (int k = 0; k < 3; ++k) {
            b |= !__builtin_isfinite(p[3 * i + k]);
            b |= !__builtin_isfinite(n[3 * i + k]);
        }
        const float a = A[i];
        b |= !(a > 0.0f) || !__builtin_isfinite(a);
        if (attrs)
            for (int c = 0; c < C; ++c) b |= !__builtin_isfinite(attrs[i * C + c]);
    }
    if (b) atomicOr(bad, 1u);
}

// ---------------------------------------------------------------------------
// 2. bounding box; floats mapped to order-preserving unsigned keys
// ---------------------------------------------------------------------------
__device__ inline uint32_t f2ord(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float ord2f(uint32_t o) {
    const uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __uint_as_float(u);
}

__global__ void k_box_init(uint32_t *box) {
    if (threadIdx.x < 3) box[threadIdx.x] = 0xffffffffu;
    else if (threadIdx.x < 6) box[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(kThreads) void k_bbox(const float *__restrict__ p, int64_t M,
                                                   uint32_t *box) {
    __shared__ uint32_t sh[6][kThreads];
    uint32_t lo[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, hi[3] = {0u, 0u, 0u};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int k = 0; k < 3; ++k) {
            const uint32_t o = f2ord(p[3 * i + k]);
            lo[k] = min(lo[k], o);
            hi[k] = max(hi[k], o);
        }
    }
    const int tid = threadIdx.x;
    for (int k = 0; k < 3; ++k) { sh[k][tid] = lo[k]; sh[3 + k][tid] = hi[k]; }
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (tid < off)
            for (int k = 0; k < 3; ++k) {
                sh[k][tid] = min(sh[k][tid], sh[k][tid + off]);
                sh[3 + k][tid] = max(sh[3 + k][tid], sh[3 + k][tid + off]);
            }
        __syncthreads();
    }
    if (tid < 3) atomicMin(&box[tid], sh[tid][0]);
    else if (tid < 6) atomicMax(&box[tid], sh[tid][0]);
}

// ---------------------------------------------------------------------------
// 3. Morton codes: q = min(floor((p - lo) * 2^21/side), 2^21-1) in FP64,
//    x at bit 3i+2, y at 3i+1, z at 3i
// ---------------------------------------------------------------------------
__device__ inline uint64_t spread3(uint64_t v) {
    uint64_t out = 0;
    for (int b = 0; b < kLevels; ++b) out |= ((v >> b) & 1ull) << (3 * b);
    return out;
}

__global__ void k_morton(const float *__restrict__ p, int64_t M, const uint32_t *__restrict__ box,
                         uint64_t *__restrict__ codes, uint32_t *__restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    float lo[3], hi[3];
    for (int k = 0; k < 3; ++k) { lo[k] = ord2f(box[k]); hi[k] = ord2f(box[3 + k]); }
    double side = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double e = (double)hi[k] - (double)lo[k];
        if (e > side) side = e;
    }
    if (side == 0.0) side = 1.0;
    const double scale = 2097152.0 / side;
    uint64_t q[3];
    for (int k = 0; k < 3; ++k) {
        const double v = ((double)p[3 * i + k] - (double)lo[k]) * scale;
        const uint64_t c = (uint64_t)floor(v);
        q[k] = c > 2097151ull ? 2097151ull : c;
    }
    codes[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
    idx[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// 4. stable LSD radix sort, 8-bit digits.  A block tile is 4 waves x 8 chunks
//    x 64 lanes = 2048 keys in original order (wave-major, then chunk, lane).
// ---------------------------------------------------------------------------
constexpr int kRsItems = 8;
constexpr int kRsTile = kThreads * kRsItems;  // 2048
constexpr int kRsWaves = kThreads / 64;

__global__ __launch_bounds__(kThreads) void k_rs_hist(const uint64_t *__restrict__ keys, int64_t n,
                                                      int shift, uint32_t *__restrict__ hist,
                                                      int64_t nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t base = (int64_t)blockIdx.x * kRsTile + wave * (kRsItems * 64);
    for (int i = 0; i < kRsItems; ++i) {
        const int64_t e = base + i * 64 + lane;
        if (e < n) atomicAdd(&h[(keys[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kThreads) void k_rs_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint64_t *__restrict__ kout,
    uint32_t *__restrict__ vout, int64_t n, int shift, const uint32_t *__restrict__ offs,
    int64_t nblocks, uint32_t *__restrict__ err) {
    __shared__ uint32_t wcnt[kRsWaves][256];
    for (int w = 0; w < kRsWaves; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    const int64_t base = (int64_t)blockIdx.x * kRsTile + wave * (kRsItems * 64);
    uint64_t key[kRsItems];
    uint32_t val[kRsItems], local[kRsItems];
    for (int i = 0; i < kRsItems; ++i) {
        const int64_t e = base + i * 64 + lane;
        const bool valid = e < n;
        key[i] = valid ? kin[e] : 0ull;
        val[i] = valid ? vin[e] : 0u;
        const uint32_t d = (uint32_t)(key[i] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = __ballot(valid && bit);
            peers &= bit ? bal : ~bal;
        }
        const uint32_t before = wcnt[wave][d];
        local[i] = before + (uint32_t)__popcll(peers & lt_mask);
        __builtin_amdgcn_wave_barrier();
        if (valid && (__ffsll((unsigned long long)peers) - 1) == lane)
            wcnt[wave][d] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    {
        uint32_t run = 0;
        for (int w = 0; w < kRsWaves; ++w) {
            const uint32_t c = wcnt[w][threadIdx.x];
            wcnt[w][threadIdx.x] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int i = 0; i < kRsItems; ++i) {
        const int64_t e = base + i * 64 + lane;
        if (e < n) {
            const uint32_t d = (uint32_t)(key[i] >> shift) & 255u;
            const uint64_t pos = (uint64_t)offs[(int64_t)d * nblocks + blockIdx.x] + wcnt[wave][d] + local[i];
            if (pos < (uint64_t)n) {
                kout[pos] = key[i];
                vout[pos] = val[i];
            } else {
                atomicOr(err, 1u);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// device-wide scan of uint32 (tiles of 1024, recursive over tile sums)
// ---------------------------------------------------------------------------
constexpr int kScanItems = 4;
constexpr int kScanTile = kThreads * kScanItems;

__global__ __launch_bounds__(kThreads) void k_scan_tile(const uint32_t *in, uint32_t *out, int64_t n,
                                                        uint32_t *bsum, int inclusive) {
    __shared__ uint32_t sh[kThreads];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)tid * kScanItems;
    uint32_t v[kScanItems], tsum = 0;
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0u;
        tsum += v[i];
    }
    sh[tid] = tsum;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
        const uint32_t a = tid >= off ? sh[tid - off] : 0u;
        __syncthreads();
        sh[tid] += a;
        __syncthreads();
    }
    uint32_t run = sh[tid] - tsum;
    for (int i = 0; i < kScanItems; ++i) {
        if (inclusive) run += v[i];
        if (base + i < n) out[base + i] = run;
        if (!inclusive) run += v[i];
    }
    if (tid == kThreads - 1) bsum[blockIdx.x] = sh[tid];
}

__global__ __launch_bounds__(kThreads) void k_scan_add(uint32_t *out, int64_t n,
                                                       const uint32_t *__restrict__ boff) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    const uint32_t add = boff[blockIdx.x];
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) out[base + i] += add;
}

// ---------------------------------------------------------------------------
// 5. topology, one level at a time
// ---------------------------------------------------------------------------
__global__ void k_split(int level, int64_t M, int leaf_size, const uint64_t *__restrict__ codes,
                        int32_t *__restrict__ node_of, const int32_t *__restrict__ ptb,
                        const int32_t *__restrict__ ptc, int32_t *__restrict__ leaf_of,
                        uint32_t *__restrict__ flag) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const int32_t t = node_of[j];
    uint32_t f = 0;
    if (t >= 0) {
        const bool internal = ptc[t] > leaf_size && level < kLevels;
        if (!internal) {
            leaf_of[j] = t;
            node_of[j] = -1;
        } else {
            const int shift = 3 * (kLevels - 1 - level);
            f = (j == ptb[t]) || (((codes[j] >> shift) & 7ull) != ((codes[j - 1] >> shift) & 7ull));
        }
    }
    flag[j] = f;
}

__global__ void k_emit(int level, int64_t M, int64_t lev_end, int64_t cap, const uint32_t *__restrict__ flag,
                       const uint32_t *__restrict__ incl, int32_t *__restrict__ node_of,
                       int32_t *__restrict__ lvl, int32_t *__restrict__ parent,
                       int32_t *__restrict__ first_child, int32_t *__restrict__ nchild,
                       int32_t *__restrict__ ptb, uint32_t *__restrict__ err) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const int32_t t = node_of[j];
    if (t < 0) return;
    const int64_t k64 = lev_end + (int64_t)incl[j] - 1;
    if (k64 < lev_end || k64 >= cap) {
        atomicOr(err, 2u);
        node_of[j] = -1;
        return;
    }
    const int32_t k = (int32_t)k64;
    if (flag[j]) {
        lvl[k] = level + 1;
        parent[k] = t;
        ptb[k] = (int32_t)j;
        first_child[k] = -1;
        nchild[k] = 0;
        if (j == ptb[t]) first_child[t] = k;
    }
    node_of[j] = k;
}

__global__ void k_child_counts(int64_t nb, int64_t ne, const int32_t *__restrict__ parent,
                               const int32_t *__restrict__ first_child, int32_t *__restrict__ nchild,
                               const int32_t *__restrict__ ptb, int32_t *__restrict__ ptc) {
    const int64_t k = nb + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ne) return;
    const int32_t par = parent[k];
    const bool last = (k + 1 == ne) || parent[k + 1] != par;
    const int32_t end = last ? ptb[par] + ptc[par] : ptb[k + 1];
    ptc[k] = end - ptb[k];
    if (last) nchild[par] = (int32_t)(k - first_child[par] + 1);
}

// ---------------------------------------------------------------------------
// sorted point records
// ---------------------------------------------------------------------------
__global__ void k_points(const float *__restrict__ p, const float *__restrict__ n,
                         const float *__restrict__ A, const uint32_t *__restrict__ perm, int64_t M,
                         PointRec *__restrict__ pts, float *__restrict__ nrm) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const int64_t i = perm[j];
    PointRec r;
    r.x = p[3 * i];
    r.y = p[3 * i + 1];
    r.z = p[3 * i + 2];
    const float a = A[i];
    r.anx = mul_rn(a, n[3 * i]);
    r.any = mul_rn(a, n[3 * i + 1]);
    r.anz = mul_rn(a, n[3 * i + 2]);
    r.a = a;
    r.pad = 0.0f;
    pts[j] = r;
    nrm[3 * j] = n[3 * i];
    nrm[3 * j + 1] = n[3 * i + 1];
    nrm[3 * j + 2] = n[3 * i + 2];
}

// ---------------------------------------------------------------------------
// 6. node geometry: FP64 area and area-weighted position sums, fixed order
// ---------------------------------------------------------------------------
__global__ void k_geom(int64_t nb, int64_t ne, const int32_t *__restrict__ first_child,
                       const int32_t *__restrict__ nchild, const int32_t *__restrict__ ptb,
                       const int32_t *__restrict__ ptc, const PointRec *__restrict__ pts,
                       double *__restrict__ nA, double *__restrict__ nS, NodeRec *__restrict__ nodes) {
    const int64_t t = nb + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne) return;
    double a = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (nchild[t] == 0) {
        const int64_t jb = ptb[t], je = jb + ptc[t];
        for (int64_t j = jb; j < je; ++j) {
            // A_m * p_m is exact in FP64 (24-bit x 24-bit significands)
            const double w = (double)pts[j].a;
            a += w;
            s0 += w * (double)pts[j].x;
            s1 += w * (double)pts[j].y;
            s2 += w * (double)pts[j].z;
        }
    } else {
        const int64_t cb = first_child[t], ce = cb + nchild[t];
        for (int64_t c = cb; c < ce; ++c) {
            a += nA[c];
            s0 += nS[3 * c];
            s1 += nS[3 * c + 1];
            s2 += nS[3 * c + 2];
        }
    }
    nA[t] = a;
    nS[3 * t] = s0;
    nS[3 * t + 1] = s1;
    nS[3 * t + 2] = s2;
    nodes[t].cx = (float)(s0 / a);
    nodes[t].cy = (float)(s1 / a);
    nodes[t].cz = (float)(s2 / a);
}

// squared radius: the max of FP32 squared distances from the centroid.  The
// max is exact and order-free, so the two kernels below give the same bits as
// any other evaluation order.
constexpr int32_t kBigNode = 16384;  // nodes with more points: k_radius_big

// nodes with at most kBigNode points: one wavefront per node; larger nodes
// are set to 0 here and raised by k_radius_big afterwards
__global__ __launch_bounds__(kThreads) void k_radius(int64_t N, const int32_t *__restrict__ ptb,
                                                     const int32_t *__restrict__ ptc,
                                                     const PointRec *__restrict__ pts,
                                                     NodeRec *__restrict__ nodes) {
    const int64_t t = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (t >= N) return;  // uniform per wavefront
    const int lane = lane_id();
    if (ptc[t] > kBigNode) {
        if (lane == 0) nodes[t].r2 = 0.0f;
        return;
    }
    const float cx = nodes[t].cx, cy = nodes[t].cy, cz = nodes[t].cz;
    const int64_t jb = ptb[t], je = jb + ptc[t];
    float m = 0.0f;
    for (int64_t j = jb + lane; j < je; j += 64)
        m = fmaxf(m, dist2_rn(pts[j].x, pts[j].y, pts[j].z, cx, cy, cz));
    m = wave_max_nonneg(m);
    if (lane == 0) nodes[t].r2 = m;
}

// nodes with more than kBigNode points: one thread per sorted point descends
// from the root through its ancestors that hold more than kBigNode points (the
// child holding the point is found among the contiguous children).  When all
// 64 points of a wavefront share the ancestor, the wavefront reduces first and
// issues one atomic max, otherwise each point does; the atomic max acts on the
// bit pattern of the non-negative float, which orders like the value.
__global__ __launch_bounds__(kThreads) void k_radius_big(int64_t M, const int32_t *__restrict__ first_child,
                                                         const int32_t *__restrict__ nchild,
                                                         const int32_t *__restrict__ ptb,
                                                         const int32_t *__restrict__ ptc,
                                                         const PointRec *__restrict__ pts,
                                                         NodeRec *__restrict__ nodes) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = lane_id();
    const bool valid = j < M;
    float px = 0.0f, py = 0.0f, pz = 0.0f;
    if (valid) {
        px = pts[j].x;
        py = pts[j].y;
        pz = pts[j].z;
    }
    int32_t a = valid ? 0 : -1;
    for (int l = 0; l <= kLevels; ++l) {  // wave-uniform: ends when no lane has a large ancestor left
        const bool big = a >= 0 && ptc[a] > kBigNode;
        if (__ballot(big) == 0) break;
        float d2 = 0.0f;
        if (big) d2 = dist2_rn(px, py, pz, nodes[a].cx, nodes[a].cy, nodes[a].cz);
        const int32_t a0 = __builtin_amdgcn_readfirstlane(a);
        if (__ballot(!(big && a == a0)) == 0) {
            const float m = wave_max_nonneg(d2);
            if (lane == 0) atomicMax((unsigned int *)&nodes[a0].r2, __float_as_uint(m));
        } else if (big) {
            atomicMax((unsigned int *)&nodes[a].r2, __float_as_uint(d2));
        }
        int32_t next = -1;
        if (big) {  // a large node is never a leaf: its children partition its points
            const int32_t cb = first_child[a], ce = cb + nchild[a];
            for (int32_t c = cb; c < ce; ++c)
                if (j >= ptb[c] && j < (int64_t)ptb[c] + ptc[c]) next = c;
        }
        a = next;
    }
}

// ---------------------------------------------------------------------------
// 7. escape pointers (next node after a subtree in depth-first order) and records
// ---------------------------------------------------------------------------
__global__ void k_escape(int64_t nb, int64_t ne, const int32_t *__restrict__ parent,
                         const int32_t *__restrict__ first_child, const int32_t *__restrict__ nchild,
                         uint32_t *__restrict__ esc) {
    const int64_t t = nb + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne) return;
    if (t == 0) { esc[0] = kEnd; return; }
    const int32_t p = parent[t];
    const int64_t last = (int64_t)first_child[p] + nchild[p] - 1;
    esc[t] = t < last ? (uint32_t)(t + 1) : esc[p];
}

__global__ void k_records(int64_t N, const int32_t *__restrict__ lvl,
                          const int32_t *__restrict__ first_child, const int32_t *__restrict__ nchild,
                          const int32_t *__restrict__ ptb, const int32_t *__restrict__ ptc,
                          const uint32_t *__restrict__ esc, NodeRec *__restrict__ nodes) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const bool leaf = nchild[t] == 0;
    nodes[t].first = (uint32_t)(leaf ? ptb[t] : first_child[t]);
    nodes[t].down = leaf ? esc[t] : (uint32_t)first_child[t];
    nodes[t].escape = esc[t];
    nodes[t].meta = (uint32_t)lvl[t] | (leaf ? kLeafFlag : 0u) |
                    ((uint32_t)(leaf ? ptc[t] : nchild[t]) << kCountShift);
}

// structural invariants every later kernel relies on for its indexing
__global__ void k_validate(int64_t N, int64_t M, const int32_t *__restrict__ lvl,
                           const int32_t *__restrict__ parent, const int32_t *__restrict__ first_child,
                           const int32_t *__restrict__ nchild, const int32_t *__restrict__ ptb,
                           const int32_t *__restrict__ ptc, uint32_t *__restrict__ err) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    bool ok = lvl[t] >= 0 && lvl[t] <= kLevels && ptb[t] >= 0 && ptc[t] >= 1 &&
              (int64_t)ptb[t] + ptc[t] <= M;
    ok = ok && (t == 0 ? parent[t] == -1 : (parent[t] >= 0 && parent[t] < t));
    if (nchild[t] == 0) ok = ok && first_child[t] == -1;
    else ok = ok && nchild[t] <= 8 && first_child[t] > t && (int64_t)first_child[t] + nchild[t] <= N;
    if (!ok) atomicOr(err, 4u);
}

__global__ void k_root(int64_t M, int32_t *lvl, int32_t *parent, int32_t *first_child,
                       int32_t *nchild, int32_t *ptb, int32_t *ptc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        lvl[0] = 0; parent[0] = -1; first_child[0] = -1; nchild[0] = 0; ptb[0] = 0;
        ptc[0] = (int32_t)M;
    }
}

__global__ void k_fill_i32(int32_t *a, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// temporaries freed on scope exit
// temporary device buffers, freed when the owner returns; with a tree their
// bytes count against its build's memory limit while they are held
struct Scratch {
    dps_tree_s *t;
    std::vector<std::pair<void *, size_t>> blocks;
    explicit Scratch(dps_tree_s *tree) : t(tree) {}
    ~Scratch() {
        for (auto &b : blocks)
            if (b.first) (void)hipFree(b.first);
        if (t) t->scratch_bytes = 0;
    }
    template <class T>
    dps_status get(T **p, size_t count) {
        const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        *p = nullptr;
        if (!memory_fits(t, bytes)) {
            set_error("device memory limit of dps_set_memory_limit reached (build scratch)");
            return DPS_ERR_OOM;
        }
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, bytes);
        if (e != hipSuccess) return hip_status(e, "hipMalloc (build scratch)");
        blocks.push_back({q, bytes});
        if (t) t->scratch_bytes += (int64_t)bytes;
        *p = (T *)q;
        return DPS_OK;
    }
    void release(void *q) {
        for (auto &b : blocks)
            if (b.first == q) {
                (void)hipFree(b.first);
                b.first = nullptr;
                if (t) t->scratch_bytes -= (int64_t)b.second;
            }
    }
};

#define DPS_TRY(expr)                       \
    do {                                    \
        dps_status st__ = (expr);           \
        if (st__ != DPS_OK) return st__;    \
    } while (0)
#define DPS_LAUNCHED(what) DPS_TRY(hip_status(hipGetLastError(), what))

inline unsigned grid(int64_t n, int threads = kThreads) { return (unsigned)std::max<int64_t>(1, cdiv(n, threads)); }

}  // namespace

// ---------------------------------------------------------------------------
size_t scan_tmp_words(int64_t n) {
    const int64_t nb = cdiv(n, kScanTile);
    return (size_t)nb + (nb > 1 ? scan_tmp_words(nb) : 0);
}

dps_status device_scan(const uint32_t *in, uint32_t *out, int64_t n, bool inclusive, uint32_t *tmp,
                       hipStream_t s) {
    if (n <= 0) return DPS_OK;
    const int64_t nb = cdiv(n, kScanTile);
    k_scan_tile<<<(unsigned)nb, kThreads, 0, s>>>(in, out, n, tmp, inclusive ? 1 : 0);
    DPS_LAUNCHED("scan");
    if (nb > 1) {
        DPS_TRY(device_scan(tmp, tmp, nb, false, tmp + nb, s));
        k_scan_add<<<(unsigned)nb, kThreads, 0, s>>>(out, n, tmp);
        DPS_LAUNCHED("scan add");
    }
    return DPS_OK;
}

dps_status check_inputs(const float *p, const float *n, const float *A, const float *attrs,
                        int64_t M, int C, hipStream_t s, bool *ok) {
    Scratch sc(nullptr);
    uint32_t *bad;
    DPS_TRY(sc.get(&bad, 1));
    DPS_TRY(hip_status(hipMemsetAsync(bad, 0, sizeof(uint32_t), s), "hipMemsetAsync"));
    k_check<<<grid(std::min<int64_t>(M, 1 << 20)), kThreads, 0, s>>>(p, n, A, attrs, M, C, bad);
    DPS_LAUNCHED("input check");
    uint32_t h = 0;
    DPS_TRY(hip_status(hipMemcpyAsync(&h, bad, sizeof h, hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
    DPS_TRY(hip_status(hipStreamSynchronize(s), "hipStreamSynchronize"));
    *ok = (h == 0);
    return DPS_OK;
}

dps_status build_tree(dps_tree_s *t, const float *p, const float *n, const float *A, hipStream_t s) {
    const int64_t M = t->M;
    Scratch sc(t);

    // bounding box and Morton codes
    uint32_t *box, *err;
    uint64_t *k0, *k1;
    uint32_t *v0, *v1;
    DPS_TRY(sc.get(&box, 6));
    DPS_TRY(sc.get(&err, 1));
    DPS_TRY(hip_status(hipMemsetAsync(err, 0, sizeof(uint32_t), s), "hipMemsetAsync"));
    DPS_TRY(sc.get(&k0, M));
    DPS_TRY(sc.get(&k1, M));
    DPS_TRY(sc.get(&v0, M));
    DPS_TRY(sc.get(&v1, M));
    k_box_init<<<1, 64, 0, s>>>(box);
    DPS_LAUNCHED("bbox init");
    k_bbox<<<grid(std::min<int64_t>(M, 1 << 20)), kThreads, 0, s>>>(p, M, box);
    DPS_LAUNCHED("bbox");
    k_morton<<<grid(M), kThreads, 0, s>>>(p, M, box, k0, v0);
    DPS_LAUNCHED("morton");

    // stable radix sort of (code, index)
    const int64_t nblk = cdiv(M, kRsTile);
    const int64_t nh = 256 * nblk;
    uint32_t *hist, *stmp;
    DPS_TRY(sc.get(&hist, nh));
    DPS_TRY(sc.get(&stmp, scan_tmp_words(std::max<int64_t>(nh, M))));
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 8 * pass;
        k_rs_hist<<<(unsigned)nblk, kThreads, 0, s>>>(k0, M, shift, hist, nblk);
        DPS_LAUNCHED("radix histogram");
        DPS_TRY(device_scan(hist, hist, nh, false, stmp, s));
        k_rs_scatter<<<(unsigned)nblk, kThreads, 0, s>>>(k0, v0, k1, v1, M, shift, hist, nblk, err);
        DPS_LAUNCHED("radix scatter");
        std::swap(k0, k1);
        std::swap(v0, v1);
    }
    DPS_TRY(tree_alloc(t, &t->codes, M));
    DPS_TRY(tree_alloc(t, &t->perm, M));
    DPS_TRY(hip_status(hipMemcpyAsync(t->codes, k0, M * sizeof(uint64_t), hipMemcpyDeviceToDevice, s), "copy codes"));
    DPS_TRY(hip_status(hipMemcpyAsync(t->perm, v0, M * sizeof(uint32_t), hipMemcpyDeviceToDevice, s), "copy perm"));
    DPS_TRY(hip_status(hipStreamSynchronize(s), "sync after sort"));
    sc.release(k1);
    sc.release(v1);
    sc.release(hist);

    // topology, level by level; node arrays grow as needed
    int64_t cap = std::max<int64_t>(1024, M / 2 + 1024);
    int32_t *arr[6];  // level, parent, first_child, nchild, ptb, ptc
    for (auto &a : arr) DPS_TRY(sc.get(&a, cap));
    int32_t *node_of, *leaf_of_tmp;
    uint32_t *flag, *incl;
    DPS_TRY(sc.get(&node_of, M));
    DPS_TRY(sc.get(&flag, M));
    DPS_TRY(sc.get(&incl, M));
    DPS_TRY(tree_alloc(t, &t->leaf_of, M));
    leaf_of_tmp = t->leaf_of;
    DPS_TRY(hip_status(hipMemsetAsync(leaf_of_tmp, 0, M * sizeof(int32_t), s), "hipMemsetAsync"));
    k_root<<<1, 64, 0, s>>>(M, arr[0], arr[1], arr[2], arr[3], arr[4], arr[5]);
    DPS_LAUNCHED("root");
    k_fill_i32<<<grid(M), kThreads, 0, s>>>(node_of, M, 0);
    DPS_LAUNCHED("fill");
    for (auto &v : t->level_start) v = 0;
    t->level_start[0] = 0;
    t->level_start[1] = 1;
    int64_t lev_end = 1;
    int depth = 0;
    for (int l = 0;; ++l) {
        k_split<<<grid(M), kThreads, 0, s>>>(l, M, t->leaf_size, k0, node_of, arr[4], arr[5],
                                             leaf_of_tmp, flag);
        DPS_LAUNCHED("split");
        DPS_TRY(device_scan(flag, incl, M, true, stmp, s));
        uint32_t n_new = 0;
        DPS_TRY(hip_status(hipMemcpyAsync(&n_new, incl + (M - 1), sizeof n_new, hipMemcpyDeviceToHost, s), "read count"));
        DPS_TRY(hip_status(hipStreamSynchronize(s), "sync level"));
        if (n_new == 0) { depth = l; break; }
        if (l >= kLevels) { set_error("internal error: octree deeper than %d levels", kLevels); return DPS_ERR_DEVICE; }
        if (lev_end + (int64_t)n_new > cap) {
            int64_t ncap = std::max<int64_t>(cap * 2, lev_end + (int64_t)n_new);
            for (auto &a : arr) {
                int32_t *b;
                DPS_TRY(sc.get(&b, ncap));
                DPS_TRY(hip_status(hipMemcpyAsync(b, a, lev_end * sizeof(int32_t), hipMemcpyDeviceToDevice, s), "grow nodes"));
                DPS_TRY(hip_status(hipStreamSynchronize(s), "sync grow"));
                sc.release(a);
                a = b;
            }
            cap = ncap;
        }
        k_emit<<<grid(M), kThreads, 0, s>>>(l, M, lev_end, cap, flag, incl, node_of, arr[0], arr[1],
                                            arr[2], arr[3], arr[4], err);
        DPS_LAUNCHED("emit");
        k_child_counts<<<grid(n_new), kThreads, 0, s>>>(lev_end, lev_end + n_new, arr[1], arr[2],
                                                         arr[3], arr[4], arr[5]);
        DPS_LAUNCHED("child counts");
        lev_end += n_new;
        t->level_start[l + 2] = lev_end;
    }
    const int64_t N = lev_end;
    k_validate<<<grid(N), kThreads, 0, s>>>(N, M, arr[0], arr[1], arr[2], arr[3], arr[4], arr[5], err);
    DPS_LAUNCHED("validate");
    {
        uint32_t h = 0;
        DPS_TRY(hip_status(hipMemcpyAsync(&h, err, sizeof h, hipMemcpyDeviceToHost, s), "read check"));
        DPS_TRY(hip_status(hipStreamSynchronize(s), "sync check"));
        if (h) {
            set_error("internal error: octree construction failed its consistency check (code %u)", h);
            return DPS_ERR_DEVICE;
        }
    }
    t->N = N;
    t->depth = depth;
    for (int l = depth + 2; l < kLevels + 2; ++l) t->level_start[l] = N;
    t->n_top = t->level_start[std::min(kTopLevels, depth) + 1];

    int32_t **dst[6] = {&t->level, &t->parent, &t->first_child, &t->nchild, &t->ptb, &t->ptc};
    for (int i = 0; i < 6; ++i) {
        DPS_TRY(tree_alloc(t, dst[i], N));
        DPS_TRY(hip_status(hipMemcpyAsync(*dst[i], arr[i], N * sizeof(int32_t), hipMemcpyDeviceToDevice, s), "copy topology"));
    }
    DPS_TRY(hip_status(hipStreamSynchronize(s), "sync topology"));
    for (auto &a : arr) sc.release(a);
    sc.release(node_of);
    sc.release(flag);
    sc.release(incl);

    // points, node geometry, escape pointers, records
    DPS_TRY(tree_alloc(t, &t->pts, M));
    DPS_TRY(tree_alloc(t, &t->nrm, 3 * M));
    DPS_TRY(tree_alloc(t, &t->nodes, N));
    k_points<<<grid(M), kThreads, 0, s>>>(p, n, A, t->perm, M, t->pts, t->nrm);
    DPS_LAUNCHED("points");
    double *nA, *nS;
    uint32_t *esc;
    DPS_TRY(sc.get(&nA, N));
    DPS_TRY(sc.get(&nS, 3 * N));
    DPS_TRY(sc.get(&esc, N));
    for (int l = depth; l >= 0; --l) {
        const int64_t nb = t->level_start[l], ne = t->level_start[l + 1];
        k_geom<<<grid(ne - nb), kThreads, 0, s>>>(nb, ne, t->first_child, t->nchild, t->ptb, t->ptc,
                                                  t->pts, nA, nS, t->nodes);
        DPS_LAUNCHED("geometry");
    }
    k_radius<<<grid(N, kThreads / 64), kThreads, 0, s>>>(N, t->ptb, t->ptc, t->pts, t->nodes);
    DPS_LAUNCHED("radius");
    if (M > kBigNode) {
        k_radius_big<<<grid(M), kThreads, 0, s>>>(M, t->first_child, t->nchild, t->ptb, t->ptc, t->pts, t->nodes);
        DPS_LAUNCHED("radius of large nodes");
    }
    for (int l = 0; l <= depth; ++l) {
        const int64_t nb = t->level_start[l], ne = t->level_start[l + 1];
        k_escape<<<grid(ne - nb), kThreads, 0, s>>>(nb, ne, t->parent, t->first_child, t->nchild, esc);
        DPS_LAUNCHED("escape");
    }
    k_records<<<grid(N), kThreads, 0, s>>>(N, t->level, t->first_child, t->nchild, t->ptb, t->ptc,
                                           esc, t->nodes);
    DPS_LAUNCHED("records");
    DPS_TRY(hip_status(hipStreamSynchronize(s), "sync build"));
    return DPS_OK;
}

}  // namespace dps
