// dps_rays.hip -- the ray front-end of the reconstruction (Sec. 7.1, ray
// sampling): the dense march that finds each camera ray's first crossing of
// the geometry level set, and the placement of the quadrature samples around
// that crossing.
//
// March.  Ray r has n samples at t_k = t_n + (k + 1/2) h, h = (t_f - t_n) / n,
// x_k = o + t_k d (FP32, one rounding per operation).  Its first crossing is
// the smallest j with (D(x_j) >= level) != (D(x_{j+1}) >= level), D one
// channel of the dipole sum.  By default a wavefront takes 64 K consecutive
// samples of one ray (ray-major: its points lie on a short piece of one line,
// the most coherent packet a ray offers), all chunks of all rays run at once,
// each lowers the ray's crossing index with an atomic min, and a chunk that
// starts past a crossing already found is skipped; a second pass evaluates the
// field at j and j + 1 (a wavefront per ray).  The alternative (launch flag) gives each lane one ray
// of 64 consecutive rays and walks its samples in order, the lane stopping at
// its first crossing; it needs neighbouring pixels in neighbouring lanes and
// enough rays to fill the GPU, and is kept for comparison.  The two give the
// same results bit for bit: the walk adds a point's terms in tree order
// whatever else its packet holds.
//
// Placement.  With a crossing, t* = t_j + w (t_{j+1} - t_j),
// w = (level - D_j) / (D_{j+1} - D_j), and the dense window
// [a, b] = [max(t_n, t* - W h), min(t_f, t* + W h)]; n_b samples go to
// [t_n, a], n_d to [a, b] and n_a to [b, t_f]; without one, n_b + n_d + n_a
// samples go to [t_n, t_f].  Sample i of the m in [lo, hi] sits at
// lo + (i + u_i) (hi - lo) / m with the caller's jitter u_i.  Also FP32 with
// one rounding per operation.
#include "dps_walk.h"

namespace dps {

namespace {

__device__ __forceinline__ float march_param(float tn, int k, float h) {
#pragma clang fp contract(off)
    return tn + ((float)k + 0.5f) * h;
}

__device__ __forceinline__ float ray_at(float o, float t, float d) {
#pragma clang fp contract(off)
    return o + t * d;
}

template <bool BF16, int K>
__global__ __launch_bounds__(kThreads) void k_ray_march(
    const NodeRec *__restrict__ nodes, const PointRec *__restrict__ pts, const void *__restrict__ mom,
    const void *__restrict__ attr, int ms, int as, float b2, KernelParams kp, int c0, uint32_t limit,
    uint32_t *__restrict__ err, const float *__restrict__ o, const float *__restrict__ d,
    const float *__restrict__ tnear, const float *__restrict__ tfar, int64_t R, int n, float level,
    int32_t *__restrict__ hit, float *__restrict__ hv, uint32_t *__restrict__ ctr) {
    const int lane = lane_id();
    const int64_t ntiles = (R + 63) / 64;
    int part = xcc_id();
    for (;;) {
        const int64_t tile = next_tile(ctr, ntiles, part);
        if (tile < 0) break;
        const int64_t r = tile * 64 + lane;
        bool active = r < R;
        float ox = 0.0f, oy = 0.0f, oz = 0.0f, dx = 0.0f, dy = 0.0f, dz = 0.0f, tn = 0.0f, h = 0.0f;
        if (active) {
            ox = o[3 * r];
            oy = o[3 * r + 1];
            oz = o[3 * r + 2];
            dx = d[3 * r];
            dy = d[3 * r + 1];
            dz = d[3 * r + 2];
            tn = tnear[r];
            h = (tfar[r] - tn) / (float)n;
        }
        float prev = 0.0f, v0 = 0.0f, v1 = 0.0f;
        int32_t j = -1;
        // wave-uniform: every lane evaluates the ballot; at most ceil(n / K) passes
        for (int k = 0; __ballot(active) != 0; k += K) {
            float px[K], py[K], pz[K], f[K][1], g[K][1][3];
            int32_t depth[K];
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const int s = k + i;
                const float t = march_param(tn, s, h);
                px[i] = ray_at(ox, t, dx);
                py[i] = ray_at(oy, t, dy);
                pz[i] = ray_at(oz, t, dz);
                depth[i] = (active && s < n) ? 0 : -1;
                f[i][0] = 0.0f;
                g[i][0][0] = g[i][0][1] = g[i][0][2] = 0.0f;
            }
            dipole_walk<1, BF16, false, K>(px, py, pz, depth, f, g, nodes, pts, mom, attr, ms, as, b2, kp, c0, limit,
                                           err);
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const int s = k + i;
                if (active && s < n) {
                    const float v = f[i][0];
                    if (s > 0 && ((prev >= level) != (v >= level))) {
                        j = s - 1;
                        v0 = prev;
                        v1 = v;
                        active = false;
                    }
                    prev = v;
                }
            }
            if (k + K >= n) active = false;
        }
        if (r < R) {
            hit[r] = j;
            hv[2 * r] = v0;
            hv[2 * r + 1] = v1;
        }
    }
}

// Ray-major march: a wavefront owns 64 K consecutive
// samples of one ray (lane l holds samples s0 + l K .. s0 + l K + K - 1), so
// its points lie on a short piece of one line.  Work item w is chunk
// c = w / R of ray r = w % R (chunk-major, so early chunks of every ray are
// dispatched first); chunk c covers the pairs (s, s + 1) with s in
// [c P, c P + P), P = 64 K - 1, the last lane's last sample being the next
// chunk's first.  The wavefront lowers hit[r] to its first crossing (atomic
// min; hit starts at INT32_MAX) and skips its chunk when hit[r] already lies
// before it.  With `slots` ([R][nchunks][2]) it also stores the field at its
// first crossing j and at j + 1 in its own slot: the chunk holding the ray's
// final (smallest) crossing always runs (hit[r] never drops below it) and
// finds that crossing first, so k_ray_hit_gather reads the values from the
// slot of chunk j / P.
template <bool BF16, int K>
__global__ __launch_bounds__(kThreads) void k_ray_march_along(
    const NodeRec *__restrict__ nodes, const PointRec *__restrict__ pts, const void *__restrict__ mom,
    const void *__restrict__ attr, int ms, int as, float b2, KernelParams kp, int c0, uint32_t limit,
    uint32_t *__restrict__ err, const float *__restrict__ o, const float *__restrict__ d,
    const float *__restrict__ tnear, const float *__restrict__ tfar, int64_t R, int n, int64_t nitems, float level,
    int32_t *__restrict__ hit, float *__restrict__ slots, int nchunks) {
    constexpr int P = 64 * K - 1;
    const int lane = lane_id();
    const int64_t item = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (item >= nitems) return;  // wave-uniform
    const int64_t c = item / R, r = item - c * R;
    const int s0 = (int)c * P;
    if (__hip_atomic_load(&hit[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < s0) return;  // wave-uniform
    const float ox = o[3 * r], oy = o[3 * r + 1], oz = o[3 * r + 2];
    const float dx = d[3 * r], dy = d[3 * r + 1], dz = d[3 * r + 2];
    const float tn = tnear[r], h = (tfar[r] - tn) / (float)n;
    float px[K], py[K], pz[K], f[K][1], g[K][1][3];
    int32_t depth[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int s = s0 + lane * K + i;
        const float t = march_param(tn, s, h);
        px[i] = ray_at(ox, t, dx);
        py[i] = ray_at(oy, t, dy);
        pz[i] = ray_at(oz, t, dz);
        depth[i] = s < n ? 0 : -1;
        f[i][0] = 0.0f;
        g[i][0][0] = g[i][0][1] = g[i][0][2] = 0.0f;
    }
    dipole_walk<1, BF16, false, K>(px, py, pz, depth, f, g, nodes, pts, mom, attr, ms, as, b2, kp, c0, limit, err);
    const float next = __shfl_down(f[0][0], 1);  // the next lane's first sample
    int32_t j = INT32_MAX;
    float v0 = 0.0f, v1 = 0.0f;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int s = s0 + lane * K + i;
        const bool pair = s + 1 < n && (lane < 63 || i < K - 1);
        const float w = i + 1 < K ? f[i + 1 < K ? i + 1 : i][0] : next;
        if (j == INT32_MAX && pair && ((f[i][0] >= level) != (w >= level))) {
            j = s;
            v0 = f[i][0];
            v1 = w;
        }
    }
    const uint64_t m = __ballot(j != INT32_MAX);
    if (m != 0 && lane == __ffsll((unsigned long long)m) - 1) {
        atomicMin(&hit[r], j);
        if (slots) {
            float *sl = slots + 2 * (r * nchunks + c);
            sl[0] = v0;
            sl[1] = v1;
        }
    }
}

// After the ray-major march with crossing slots: hit = -1 and zero values
// without a crossing, else the values the chunk of the crossing stored.
__global__ void k_ray_hit_gather(int64_t R, int nchunks, int P, int32_t *__restrict__ hit, float *__restrict__ hv,
                                 const float *__restrict__ slots) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const int32_t j = hit[r];
    float v0 = 0.0f, v1 = 0.0f;
    if (j == INT32_MAX) {
        hit[r] = -1;
    } else {
        const float *sl = slots + 2 * (r * nchunks + j / P);
        v0 = sl[0];
        v1 = sl[1];
    }
    hv[2 * r] = v0;
    hv[2 * r + 1] = v1;
}

// After the ray-major march: the field at samples j and j + 1 of each ray
// with a crossing, through the same walk at the same FP32 positions (so the
// same values), and hit = -1, zero values for the others.  A wavefront takes
// G rays, lanes 2i and 2i + 1 holding samples j and j + 1 of its ray i: the
// walk of two neighbouring points is as short as that of one, so G = 1 keeps
// a wavefront's walk short when rays are far apart, and larger G (up to 32)
// fills the lanes when they are many and neighbouring.
template <bool BF16>
__global__ __launch_bounds__(kThreads) void k_ray_hit_values(
    const NodeRec *__restrict__ nodes, const PointRec *__restrict__ pts, const void *__restrict__ mom,
    const void *__restrict__ attr, int ms, int as, float b2, KernelParams kp, int c0, uint32_t limit,
    uint32_t *__restrict__ err, const float *__restrict__ o, const float *__restrict__ d,
    const float *__restrict__ tnear, const float *__restrict__ tfar, int64_t R, int n, int G,
    int32_t *__restrict__ hit, float *__restrict__ hv) {
    const int lane = lane_id();
    const int64_t w = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const int64_t r = w * G + (lane >> 1);
    const int side = lane & 1;
    const bool mine = (lane >> 1) < G && r < R;
    const int32_t j = mine ? hit[r] : INT32_MAX;
    const bool on = j != INT32_MAX;
    if (mine && !on) {
        if (side == 0) hit[r] = -1;
        hv[2 * r + side] = 0.0f;
    }
    if (__ballot(on) == 0) return;  // wave-uniform
    float px[1] = {0.0f}, py[1] = {0.0f}, pz[1] = {0.0f}, f[1][1] = {{0.0f}}, g[1][1][3] = {{{0.0f, 0.0f, 0.0f}}};
    int32_t depth[1] = {on ? 0 : -1};
    if (on) {
        const float tn = tnear[r], h = (tfar[r] - tn) / (float)n;
        const float t = march_param(tn, j + side, h);
        px[0] = ray_at(o[3 * r], t, d[3 * r]);
        py[0] = ray_at(o[3 * r + 1], t, d[3 * r + 1]);
        pz[0] = ray_at(o[3 * r + 2], t, d[3 * r + 2]);
    }
    dipole_walk<1, BF16, false, 1>(px, py, pz, depth, f, g, nodes, pts, mom, attr, ms, as, b2, kp, c0, limit, err);
    if (on) hv[2 * r + side] = f[0][0];
}

// Harnack-accelerated march (Sec. 7.1: the first crossing found by Harnack
// tracing).  Lane = ray over the persistent tile queue.  From an evaluated
// sample k with value v_k, Harnack's inequality for the field shifted by its
// lower bound (u = D - lower > 0, harmonic outside the regularised zones,
// i.e. within R = nearest point - 4.5 eps of x_k) keeps D on v_k's side of
// the level within s(a) R, a = (level - lower) / (v_k - lower),
// s = |sqrt(8a + 1) - (2a + 1)| / (2a).  The samples strictly within
// safety * s R of x_k are skipped; the first one past them is evaluated and,
// if it lies on the other side, the one before it: on v_k's side it closes
// the crossing pair, otherwise (the field did not obey the bound) the lane
// goes on sample by sample from k.  Modes: 0 step from k, 1 candidate k2,
// 2 confirm k2 - 1, 3 one sample at a time, 4 done.  Every evaluated value
// comes from the march's walk at the march's FP32 positions, so a crossing
// found here carries the dense march's values bit for bit.
template <bool BF16>
__global__ __launch_bounds__(kThreads) void k_ray_march_harnack(
    const NodeRec *__restrict__ nodes, const PointRec *__restrict__ pts, const void *__restrict__ mom,
    const void *__restrict__ attr, int ms, int as, float b2, KernelParams kp, int c0, uint32_t limit,
    uint32_t *__restrict__ err, const float *__restrict__ o, const float *__restrict__ d,
    const float *__restrict__ tnear, const float *__restrict__ tfar, int64_t R, int n, float level, float lower,
    float reg, int32_t *__restrict__ hit, float *__restrict__ hv, int32_t *__restrict__ evals,
    uint32_t *__restrict__ ctr) {
    constexpr float kSafety = 0.99f;
    const int lane = lane_id();
    const int64_t ntiles = (R + 63) / 64;
    int part = xcc_id();
    for (;;) {
        const int64_t tile = next_tile(ctr, ntiles, part);
        if (tile < 0) break;
        const int64_t r = tile * 64 + lane;
        const bool live = r < R;
        float ox = 0.0f, oy = 0.0f, oz = 0.0f, dx = 0.0f, dy = 0.0f, dz = 0.0f, tn = 0.0f, h = 0.0f;
        if (live) {
            ox = o[3 * r];
            oy = o[3 * r + 1];
            oz = o[3 * r + 2];
            dx = d[3 * r];
            dy = d[3 * r + 1];
            dz = d[3 * r + 2];
            tn = tnear[r];
            h = (tfar[r] - tn) / (float)n;
        }
        const float spacing = h * __builtin_sqrtf(dot3(dx, dy, dz, dx, dy, dz));  // between samples, in space
        auto value = [&](int k, bool on) {
            const float t = march_param(tn, k, h);
            float px[1] = {ray_at(ox, t, dx)}, py[1] = {ray_at(oy, t, dy)}, pz[1] = {ray_at(oz, t, dz)};
            float f[1][1] = {{0.0f}}, g[1][1][3] = {{{0.0f, 0.0f, 0.0f}}};
            int32_t depth[1] = {on ? 0 : -1};
            dipole_walk<1, BF16, false, 1>(px, py, pz, depth, f, g, nodes, pts, mom, attr, ms, as, b2, kp, c0, limit,
                                           err);
            return f[0][0];
        };
        int k = 0, k2 = 0, mode = live ? 0 : 4, nev = 1;
        float vk = value(0, live), v2 = 0.0f;
        float near = __builtin_inff();
        int near_k = 0;
        int32_t j = -1;
        float vj = 0.0f, vj1 = 0.0f;
        // every pass advances k or ends the lane, at most 3 passes per sample
        for (int pass = 0; __ballot(mode != 4) != 0; ++pass) {
            if (pass > 3 * n + 3) {  // cannot happen; guards the loop like the walks' step bound
                if (lane == 0) atomicOr(err, 1u);
                break;
            }
            const bool stepping = mode == 0;
            if (__ballot(stepping) != 0) {
                const float t = march_param(tn, k, h);
                const float px = ray_at(ox, t, dx), py = ray_at(oy, t, dy), pz = ray_at(oz, t, dz);
                // the nearest point lies within the last one's distance plus the way moved
                const float bound = near < __builtin_inff()
                                        ? (near + (float)(k - near_k) * spacing) * 1.0001f + 1e-30f
                                        : __builtin_inff();
                const float dist = nearest_walk(px, py, pz, stepping, bound, nodes, pts, limit, err);
                if (stepping) {
                    near = dist;
                    near_k = k;
                    const float rad = dist - reg;
                    float rho = 0.0f;
                    if (vk > lower && rad > 0.0f) {
                        const float a = (level - lower) / (vk - lower);
                        const float sa = fabsf(__builtin_sqrtf(fmaf(8.0f, a, 1.0f)) - fmaf(2.0f, a, 1.0f)) / (2.0f * a);
                        rho = sa * rad;
                    }
                    const float skip = spacing > 0.0f ? floorf(kSafety * rho / spacing) : (float)n;
                    const int m = skip < (float)n ? (int)skip : n;
                    k2 = min(k + m + 1, n - 1);
                    mode = 1;
                }
            }
            const bool evaluating = mode == 1 || mode == 2 || mode == 3;
            const int e = mode == 1 ? k2 : (mode == 2 ? k2 - 1 : k + 1);
            const float w = value(evaluating ? e : 0, evaluating);
            if (evaluating) {
                ++nev;
                const bool side = vk >= level;
                if (mode == 1) {
                    if ((w >= level) == side) {
                        k = k2;
                        vk = w;
                        mode = k >= n - 1 ? 4 : 0;
                    } else if (k2 == k + 1) {
                        j = k;
                        vj = vk;
                        vj1 = w;
                        mode = 4;
                    } else {
                        v2 = w;
                        mode = 2;
                    }
                } else if (mode == 2) {
                    if ((w >= level) == side) {
                        j = k2 - 1;
                        vj = w;
                        vj1 = v2;
                        mode = 4;
                    } else {
                        mode = 3;
                    }
                } else {
                    if ((w >= level) != side) {
                        j = k;
                        vj = vk;
                        vj1 = w;
                        mode = 4;
                    } else {
                        ++k;
                        vk = w;
                        if (k >= n - 1) mode = 4;
                    }
                }
            }
        }
        if (live) {
            hit[r] = j;
            hv[2 * r] = vj;
            hv[2 * r + 1] = vj1;
            if (evals) evals[r] = nev;
        }
    }
}

__global__ void k_fill_i32_max(int32_t *__restrict__ a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = INT32_MAX;
}

__global__ void k_ray_resample(const float *__restrict__ o, const float *__restrict__ d,
                               const float *__restrict__ tnear, const float *__restrict__ tfar, int64_t R,
                               int n_march, const int32_t *__restrict__ hit, const float *__restrict__ hv, float level,
                               const float *__restrict__ u, int nb, int nd, int na, float window, int tile_layout,
                               float *__restrict__ t_out, float *__restrict__ x_out) {
#pragma clang fp contract(off)
    const int S = nb + nd + na;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R * S) return;
    const int64_t r = i / S;
    const int s = (int)(i - r * S);
    const float tn = tnear[r], tf = tfar[r];
    const float h = (tf - tn) / (float)n_march;
    const int32_t j = hit[r];
    float lo = tn, hi = tf;
    int idx = s, m = S;
    if (j >= 0) {
        const float jf = (float)j;
        const float tj = tn + (jf + 0.5f) * h;
        const float tj1 = tn + (jf + 1.5f) * h;
        const float vj = hv[2 * r], vj1 = hv[2 * r + 1];
        const float w = (level - vj) / (vj1 - vj);
        const float ts = tj + w * (tj1 - tj);
        const float half = window * h;
        const float a = fmaxf(tn, ts - half);
        const float b = fminf(tf, ts + half);
        if (s < nb) {
            hi = a;
            m = nb;
        } else if (s < nb + nd) {
            lo = a;
            hi = b;
            idx = s - nb;
            m = nd;
        } else {
            lo = b;
            idx = s - nb - nd;
            m = na;
        }
    }
    const float t = lo + ((float)idx + u[i]) * ((hi - lo) / (float)m);
    t_out[i] = t;
    const int64_t row = tile_layout ? ((r >> 6) * S + s) * 64 + (r & 63) : i;
    x_out[3 * row] = ray_at(o[3 * r], t, d[3 * r]);
    x_out[3 * row + 1] = ray_at(o[3 * r + 1], t, d[3 * r + 1]);
    x_out[3 * row + 2] = ray_at(o[3 * r + 2], t, d[3 * r + 2]);
}

// The tree's crossing-slot workspace with at least `bytes`: a larger one is
// allocated when a call is not being captured into a graph and the memory
// limit allows it; nullptr otherwise (the march then takes the values in a
// second pass).  A workspace that is outgrown stays allocated with the tree,
// since a graph captured earlier may still write to it.
float *crossing_slots(dps_tree_s *t, int64_t bytes, hipStream_t s) {
    if (bytes <= t->ray_ws_bytes) return t->ray_ws;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (!memory_fits(t, (size_t)bytes)) return nullptr;
    void *p = nullptr;
    if (hipMalloc(&p, (size_t)bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    t->allocs.push_back(p);
    t->bytes += bytes;
    t->ray_ws = (float *)p;
    t->ray_ws_bytes = bytes;
    return t->ray_ws;
}

template <bool BF16, int K>
dps_status march_launch(dps_tree_s *t, const float *o, const float *d, const float *tn, const float *tf, int64_t R,
                        int n, float b2, KernelParams kp, int channel, float level, int32_t *hit, float *hv,
                        hipStream_t s) {
    k_fill_u32<<<1, 64, 0, s>>>(t->ctr, 8, 0u);
    const void *fn = reinterpret_cast<const void *>(&k_ray_march<BF16, K>);
    k_ray_march<BF16, K><<<persistent_grid(fn), kThreads, 0, s>>>(
        t->nodes, t->pts, trav_mom(t), t->attr, t->mom_stride, t->attr_stride, b2, kp, channel, walk_limit(t), t->err,
        o, d, tn, tf, R, n, level, hit, hv, t->ctr);
    return hip_status(hipGetLastError(), "ray march launch");
}

template <bool BF16, int K>
dps_status march_along_launch(dps_tree_s *t, const float *o, const float *d, const float *tn, const float *tf,
                              int64_t R, int n, float b2, KernelParams kp, int channel, float level, int32_t *hit,
                              float *hv, hipStream_t s) {
    const int nchunks = (int)cdiv(n - 1, 64 * K - 1);
    const int64_t nitems = nchunks * R;
    const int64_t wgs = cdiv(nitems, kThreads / 64);
    if (wgs > INT32_MAX) {
        set_error("ray march: %lld workgroups exceed the launch grid", (long long)wgs);
        return DPS_ERR_INVALID;
    }
    float *slots = crossing_slots(t, nitems * 2 * (int64_t)sizeof(float), s);
    k_fill_i32_max<<<(unsigned)std::min<int64_t>(cdiv(R, kThreads), 4096), kThreads, 0, s>>>(hit, R);
    k_ray_march_along<BF16, K><<<(unsigned)wgs, kThreads, 0, s>>>(
        t->nodes, t->pts, trav_mom(t), t->attr, t->mom_stride, t->attr_stride, b2, kp, channel, walk_limit(t), t->err,
        o, d, tn, tf, R, n, nitems, level, hit, slots, nchunks);
    dps_status st = hip_status(hipGetLastError(), "ray-major march launch");
    if (st != DPS_OK) return st;
    if (slots) {
        k_ray_hit_gather<<<grid(R), kThreads, 0, s>>>(R, nchunks, 64 * K - 1, hit, hv, slots);
        return hip_status(hipGetLastError(), "ray hit gather launch");
    }
    int G = 1;  // rays per wavefront of the values pass: at least 16384 wavefronts
    while (G < 32 && R / (2 * G) >= 16384) G *= 2;
    k_ray_hit_values<BF16><<<(unsigned)cdiv(cdiv(R, G), kThreads / 64), kThreads, 0, s>>>(
        t->nodes, t->pts, trav_mom(t), t->attr, t->mom_stride, t->attr_stride, b2, kp, channel, walk_limit(t), t->err, o,
        d, tn, tf, R, n, G, hit, hv);
    return hip_status(hipGetLastError(), "ray hit values launch");
}

template <bool BF16>
dps_status march_k(dps_tree_s *t, const float *o, const float *d, const float *tn, const float *tf, int64_t R, int n,
                   float b2, KernelParams kp, int channel, float level, int32_t *hit, float *hv, hipStream_t s) {
    const int k = t->packet_query;
    if (t->launch_flags & kFlagMarchWhole) {
        if (k >= 4) return march_launch<BF16, 4>(t, o, d, tn, tf, R, n, b2, kp, channel, level, hit, hv, s);
        if (k >= 2) return march_launch<BF16, 2>(t, o, d, tn, tf, R, n, b2, kp, channel, level, hit, hv, s);
        return march_launch<BF16, 1>(t, o, d, tn, tf, R, n, b2, kp, channel, level, hit, hv, s);
    }
    // ray-major: 2 samples per lane whenever k >= 2 (4 per lane spreads one
    // wavefront's points over too long a piece of the ray)
    if (k >= 2) return march_along_launch<BF16, 2>(t, o, d, tn, tf, R, n, b2, kp, channel, level, hit, hv, s);
    return march_along_launch<BF16, 1>(t, o, d, tn, tf, R, n, b2, kp, channel, level, hit, hv, s);
}

template <bool BF16>
dps_status harnack_launch(dps_tree_s *t, const float *o, const float *d, const float *tn, const float *tf, int64_t R,
                          int n, float b2, KernelParams kp, int channel, float level, float lower, float reg,
                          int32_t *hit, float *hv, int32_t *evals, hipStream_t s) {
    k_fill_u32<<<1, 64, 0, s>>>(t->ctr, 8, 0u);
    const void *fn = reinterpret_cast<const void *>(&k_ray_march_harnack<BF16>);
    k_ray_march_harnack<BF16><<<persistent_grid(fn), kThreads, 0, s>>>(
        t->nodes, t->pts, trav_mom(t), t->attr, t->mom_stride, t->attr_stride, b2, kp, channel, walk_limit(t), t->err,
        o, d, tn, tf, R, n, level, lower, reg, hit, hv, evals, t->ctr);
    return hip_status(hipGetLastError(), "Harnack march launch");
}

}  // namespace

dps_status launch_ray_march_harnack(dps_tree_s *t, const float *o, const float *d, const float *tn, const float *tf,
                                    int64_t R, int n, float beta, float eps, int channel, float level, float lower,
                                    int32_t *hit, float *hv, int32_t *evals, hipStream_t s) {
    const float b2 = mul_rn(beta, beta);
    const KernelParams kp = tree_kernel_params(t, eps);
    const float reg = eps > 0.0f ? 4.5f * eps : 0.0f;  // rho(t) = 1 to 8e-9 beyond t = 4.5
    if (t->storage == DPS_STORE_BF16)
        return harnack_launch<true>(t, o, d, tn, tf, R, n, b2, kp, channel, level, lower, reg, hit, hv, evals, s);
    return harnack_launch<false>(t, o, d, tn, tf, R, n, b2, kp, channel, level, lower, reg, hit, hv, evals, s);
}

dps_status launch_ray_march(dps_tree_s *t, const float *o, const float *d, const float *tn, const float *tf,
                            int64_t R, int n, float beta, float eps, int channel, float level, int32_t *hit,
                            float *hv, hipStream_t s) {
    const float b2 = mul_rn(beta, beta);
    const KernelParams kp = tree_kernel_params(t, eps);
    if (t->storage == DPS_STORE_BF16)
        return march_k<true>(t, o, d, tn, tf, R, n, b2, kp, channel, level, hit, hv, s);
    return march_k<false>(t, o, d, tn, tf, R, n, b2, kp, channel, level, hit, hv, s);
}

dps_status launch_ray_resample(const float *o, const float *d, const float *tn, const float *tf, int64_t R,
                               int n_march, const int32_t *hit, const float *hv, float level, const float *u, int nb,
                               int nd, int na, float window, int tile_layout, float *t_out, float *x_out,
                               hipStream_t s) {
    const int64_t total = R * (int64_t)(nb + nd + na);
    k_ray_resample<<<grid(total), kThreads, 0, s>>>(o, d, tn, tf, R, n_march, hit, hv, level, u, nb, nd, na, window,
                                                    tile_layout, t_out, x_out);
    return hip_status(hipGetLastError(), "ray resample launch");
}

}  // namespace dps
