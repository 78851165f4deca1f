// dps_rays.hip -- the ray front-end of the reconstruction (Sec. 7.1, ray
// sampling): the dense march that finds each camera ray's first crossing of
// the geometry level set, and the placement of the quadrature samples around
// that crossing.
//
// March.  Ray r has n samples at t_k = t_n + (k + 1/2) h, h = (t_f - t_n) / n,
// x_k = o + t_k d (FP32, one rounding per operation).  Its first crossing is
// the smallest j with (D(x_j) >= level) != (D(x_{j+1}) >= level), D one
// channel of the dipole sum.  A wavefront owns 64 consecutive rays (lane =
// ray) and walks their samples in order, K per lane at a time through the
// packet walk; a lane stops at its first crossing, since the samples after it
// do not change the result, and the wavefront stops once all its lanes have.
// A ray therefore costs the samples up to its crossing, all n only when it
// misses.  Tiles of 64 rays come from the persistent per-XCD queue.
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
            uint32_t bits[K];
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const int s = k + i;
                const float t = march_param(tn, s, h);
                px[i] = ray_at(ox, t, dx);
                py[i] = ray_at(oy, t, dy);
                pz[i] = ray_at(oz, t, dz);
                bits[i] = (active && s < n) ? 1u : 0u;
                f[i][0] = 0.0f;
                g[i][0][0] = g[i][0][1] = g[i][0][2] = 0.0f;
            }
            dipole_walk<1, BF16, false, K>(px, py, pz, bits, f, g, nodes, pts, mom, attr, ms, as, b2, kp, c0, limit,
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

template <bool BF16, int K>
dps_status march_launch(dps_tree_s *t, const float *o, const float *d, const float *tn, const float *tf, int64_t R,
                        int n, float b2, KernelParams kp, int channel, float level, int32_t *hit, float *hv,
                        hipStream_t s) {
    k_fill_u32<<<1, 64, 0, s>>>(t->ctr, 8, 0u);
    const void *fn = reinterpret_cast<const void *>(&k_ray_march<BF16, K>);
    k_ray_march<BF16, K><<<persistent_grid(fn), kThreads, 0, s>>>(
        t->nodes, t->pts, t->mom, t->attr, t->mom_stride, t->attr_stride, b2, kp, channel, (uint32_t)t->N, t->err,
        o, d, tn, tf, R, n, level, hit, hv, t->ctr);
    return hip_status(hipGetLastError(), "ray march launch");
}

template <bool BF16>
dps_status march_k(dps_tree_s *t, const float *o, const float *d, const float *tn, const float *tf, int64_t R, int n,
                   float b2, KernelParams kp, int channel, float level, int32_t *hit, float *hv, hipStream_t s) {
    const int k = t->packet_query;
    if (k >= 4) return march_launch<BF16, 4>(t, o, d, tn, tf, R, n, b2, kp, channel, level, hit, hv, s);
    if (k >= 2) return march_launch<BF16, 2>(t, o, d, tn, tf, R, n, b2, kp, channel, level, hit, hv, s);
    return march_launch<BF16, 1>(t, o, d, tn, tf, R, n, b2, kp, channel, level, hit, hv, s);
}

}  // namespace

dps_status launch_ray_march(dps_tree_s *t, const float *o, const float *d, const float *tn, const float *tf,
                            int64_t R, int n, float beta, float eps, int channel, float level, int32_t *hit,
                            float *hv, hipStream_t s) {
    const float b2 = mul_rn(beta, beta);
    const KernelParams kp = make_kernel_params(eps);
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
