// dps_mono.hip -- Barnes-Hut sums with the monopole kernel (appearance
// channels with the foreshortening factor dropped, Sec. 7.1).
//
// The kernel is m(r) = rho(r/eps) / (4 pi r^2) = kappa(r) r: the dipole kernel
// of eq. regularized_poisson without the factor n.(y - x)/|y - x|.  A source
// contributes A_m mu_mc m(|p_m - x|) to channel c, and its spatial gradient is
// A_m mu_mc gv (p_m - x) with gv = r lambda - kappa / r.  A node stores one
// scalar charge per channel, Q_tc = sum of A_m mu_mc over its points, placed
// at the node's area-weighted centroid (the monopole analogue of eq.
// farfield_dipole_features); the far test and the traversal are those of
// Algorithm 1.  A source at the query point itself contributes nothing (the
// value tends to 0 there and the gradient direction is undefined).
//
// The GPU mapping is that of the dipole sums (stackless wavefront-coherent
// walk, K queries per lane, persistent per-XCD tile queue); the per-node
// payload is CB scalars instead of CB 3-vectors, so a traversal carries up to
// 16 channels (8 with gradients).  The adjoint accumulates dL/dQ_tc =
// sum_q df_qc m(|p_t - x_q|) per node (one FP64 atomic per value after a
// wavefront reduce-scatter) and df_qc A_m m per point; the push-down gives
// dL/dmu_mc = P_mc + A_m sum over the ancestors of the node accumulators.
#include "dps_trav_common.h"

namespace dps {

namespace {

// m = kappa r and gv = r lambda - kappa / r for r^2 > 0 (FAR: a far-field
// node, as in radial())
template <bool FAR = false>
__device__ __forceinline__ void mono_radial(float r2, const KernelParams &kp, float &m, float &gv) {
    float kap, lam;
    radial<FAR>(r2, kp, kap, lam);
    const float ir = __builtin_amdgcn_rsqf(r2);
    m = kap * (r2 * ir);
    gv = fmaf(lam, r2, -kap) * ir;
}

// ---------------------------------------------------------------------------
// primal query: K queries per lane, CB channels per traversal
// ---------------------------------------------------------------------------
template <int CB, bool BF16, bool GRAD, int K>
__device__ __forceinline__ void mono_query_body(int64_t q0, DPS_TRAV_PARAMS, float *__restrict__ fout,
                                                float *__restrict__ gout) {
    float px[K], py[K], pz[K];
    int32_t depth[K];
    float f[K][CB], g[K][CB][3];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int64_t q = q0 + 64 * i;
        const bool valid = q < Q;
        px[i] = valid ? x[3 * q] : 0.0f;
        py[i] = valid ? x[3 * q + 1] : 0.0f;
        pz[i] = valid ? x[3 * q + 2] : 0.0f;
        depth[i] = valid ? 0 : -1;
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            f[i][c] = 0.0f;
            g[i][c][0] = g[i][c][1] = g[i][c][2] = 0.0f;
        }
    }
    const float b2v = in_vgpr(b2);
    uint32_t t = 0;
    NodeRec nd = nodes[0];
    float Qc[CB];
    load_charges<CB, BF16>(mom, ms, 0, c0, Qc, kp.nhi);
    uint32_t steps = 0;
    for (;;) {
        if (++steps > limit) {  // a well-formed tree is walked in at most N steps
            if ((threadIdx.x & 63) == 0) atomicOr(err, 1u);
            break;
        }
        const uint32_t lvl = nd.meta & 0xffu;
        const bool leaf = (nd.meta & kLeafFlag) != 0;
        const float lim = mul_rn(b2v, nd.r2);
        bool far[K], open[K];
        float s[K];
        WaveMasks wm;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const bool in = visits(depth[i], lvl);
            s[i] = dist2_rn(nd.cx, nd.cy, nd.cz, px[i], py[i], pz[i]);
            const bool beyond = s[i] > lim;
            far[i] = in && beyond;
            open[i] = in && !beyond;
            wm.add(in, beyond);
        }
        const bool any_far = wm.far != 0;
        const bool any_open = wm.open != 0;
        const uint32_t next = (any_open && !leaf) ? nd.first : nd.escape;
        const uint32_t pf = next;  // kEnd is the root: a valid record
        const NodeRec nn = nodes[pf];
        float Qn[CB];
        load_charges<CB, BF16>(mom, ms, pf, c0, Qn, kp.nhi);
        if (any_far) {
            refine_charges<CB, BF16>(mom, ms, t, c0, Qc, kp.nhi);
#pragma unroll
            for (int i = 0; i < K; ++i) {
                if (far[i]) {  // s > 0 here
                    float m, gv;
                    mono_radial<true>(s[i], kp, m, gv);
                    const float dx = nd.cx - px[i], dy = nd.cy - py[i], dz = nd.cz - pz[i];
#pragma unroll
                    for (int c = 0; c < CB; ++c) {
                        f[i][c] = fmaf(Qc[c], m, f[i][c]);
                        if (GRAD) {
                            const float w = gv * Qc[c];
                            g[i][c][0] = fmaf(w, dx, g[i][c][0]);
                            g[i][c][1] = fmaf(w, dy, g[i][c][1]);
                            g[i][c][2] = fmaf(w, dz, g[i][c][2]);
                        }
                    }
                }
            }
        }
        if (any_open) {
            if (!leaf) {
#pragma unroll
                for (int i = 0; i < K; ++i) depth[i] = descend(depth[i], lvl, open[i]);
            } else {
                for_leaf_points<CB, BF16>(pts, attr, as, c0, nd.first, node_count(nd),
                                          [&](uint32_t, const PointRec &pr, const float (&mu)[CB]) {
#pragma unroll
                    for (int i = 0; i < K; ++i) {
                        if (open[i]) {
                            const float dx = pr.x - px[i], dy = pr.y - py[i], dz = pr.z - pz[i];
                            const float r2 = dot3(dx, dy, dz, dx, dy, dz);
                            if (r2 > 0.0f) {
                                float m, gv;
                                mono_radial(r2, kp, m, gv);
                                const float am = pr.a * m;
                                const float ag = pr.a * gv;
#pragma unroll
                                for (int c = 0; c < CB; ++c) {
                                    f[i][c] = fmaf(mu[c], am, f[i][c]);
                                    if (GRAD) {
                                        const float w = mu[c] * ag;
                                        g[i][c][0] = fmaf(w, dx, g[i][c][0]);
                                        g[i][c][1] = fmaf(w, dy, g[i][c][1]);
                                        g[i][c][2] = fmaf(w, dz, g[i][c][2]);
                                    }
                                }
                            }
                        }
                    }
                });
            }
        }
        if (next == kEnd) break;
        t = next;
        nd = nn;
#pragma unroll
        for (int c = 0; c < CB; ++c) Qc[c] = Qn[c];
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int64_t q = q0 + 64 * i;
        if (q < Q) {
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int64_t o = q * ldo + co + c;
                fout[o] = f[i][c];
                if (GRAD) {
                    gout[3 * o] = g[i][c][0];
                    gout[3 * o + 1] = g[i][c][1];
                    gout[3 * o + 2] = g[i][c][2];
                }
            }
        }
    }
}

template <int CB, bool BF16, bool GRAD, int K>
__global__ __launch_bounds__(kThreads) void k_mono_query(DPS_KERN_PARAMS, float *__restrict__ fout,
                                                         float *__restrict__ gout, int xcd_remap) {
    DPS_ROWS;
    const int64_t blk = remap_block(xcd_remap);
    if (blk < 0 || blk * (int64_t)blockDim.x * K >= Q) return;  // whole block past the rows
    const int64_t wave = (blk * blockDim.x + threadIdx.x) >> 6;
    mono_query_body<CB, BF16, GRAD, K>(wave * 64 * K + (threadIdx.x & 63), DPS_TRAV_ARGS, fout, gout);
}

template <int CB, bool BF16, bool GRAD, int K>
__global__ __launch_bounds__(kThreads) void k_mono_query_persistent(DPS_KERN_PARAMS, float *__restrict__ fout,
                                                                    float *__restrict__ gout,
                                                                    uint32_t *__restrict__ ctr) {
    DPS_ROWS;
    const int64_t ntiles = (Q + 64 * K - 1) / (64 * K);
    int part = xcc_id();
    for (;;) {
        const int64_t tile = next_tile(ctr, ntiles, part);
        if (tile < 0) break;
        mono_query_body<CB, BF16, GRAD, K>(tile * 64 * K + (threadIdx.x & 63), DPS_TRAV_ARGS, fout, gout);
    }
}

// ---------------------------------------------------------------------------
// adjoint stage 1: node accumulators G[N][C], point accumulators P[M][C],
// dL/dx per query
// ---------------------------------------------------------------------------
template <int CB, bool BF16, int K>
__device__ __forceinline__ void mono_adjoint_body(int64_t q0, DPS_TRAV_PARAMS, int C, const float *__restrict__ df,
                                                  double *__restrict__ G, double *__restrict__ P,
                                                  float *__restrict__ dxout, int dx_mode) {
    const int lane = lane_id();
    float px[K], py[K], pz[K], w[K][CB], ax[K], ay[K], az[K];
    int32_t depth[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int64_t q = q0 + 64 * i;
        const bool valid = q < Q;
        px[i] = valid ? x[3 * q] : 0.0f;
        py[i] = valid ? x[3 * q + 1] : 0.0f;
        pz[i] = valid ? x[3 * q + 2] : 0.0f;
        depth[i] = valid ? 0 : -1;
        ax[i] = ay[i] = az[i] = 0.0f;
#pragma unroll
        for (int c = 0; c < CB; ++c) w[i][c] = valid ? df[q * ldo + co + c] : 0.0f;
    }
    const float b2v = in_vgpr(b2);
    uint32_t t = 0;
    NodeRec nd = nodes[0];
    float Qc[CB];
    load_charges<CB, BF16>(mom, ms, 0, c0, Qc, kp.nhi);
    uint32_t steps = 0;
    for (;;) {
        if (++steps > limit) {  // a well-formed tree is walked in at most N steps
            if (lane == 0) atomicOr(err, 1u);
            break;
        }
        const uint32_t lvl = nd.meta & 0xffu;
        const bool leaf = (nd.meta & kLeafFlag) != 0;
        const float lim = mul_rn(b2v, nd.r2);
        bool far[K], open[K];
        float s[K];
        WaveMasks wm;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const bool in = visits(depth[i], lvl);
            s[i] = dist2_rn(nd.cx, nd.cy, nd.cz, px[i], py[i], pz[i]);
            const bool beyond = s[i] > lim;
            far[i] = in && beyond;
            open[i] = in && !beyond;
            wm.add(in, beyond);
        }
        const bool any_far = wm.far != 0;
        const bool any_open = wm.open != 0;
        const uint32_t next = (any_open && !leaf) ? nd.first : nd.escape;
        const uint32_t pf = next;  // kEnd is the root: a valid record
        const NodeRec nn = nodes[pf];
        float Qn[CB];
        load_charges<CB, BF16>(mom, ms, pf, c0, Qn, kp.nhi);
        if (any_far) {
            refine_charges<CB, BF16>(mom, ms, t, c0, Qc, kp.nhi);
            // node increment sum_q df_c m, first over the lane's queries; query
            // slot 0 writes the sums on every lane (zero factors where it is
            // not far, taken at a huge distance) instead of a zero fill
            float acc[CB];
#pragma unroll
            for (int i = 0; i < K; ++i) {
                if (i == 0 || far[i]) {
                    const bool off = i == 0 && !far[0];
                    float m, gv;
                    mono_radial<true>(off ? kHugeR2 : s[i], kp, m, gv);
                    m = off ? 0.0f : m;
                    gv = off ? 0.0f : gv;
                    const float dx = nd.cx - px[i], dy = nd.cy - py[i], dz = nd.cz - pz[i];
                    float wq = 0.0f;
#pragma unroll
                    for (int c = 0; c < CB; ++c) {
                        wq = fmaf(w[i][c], Qc[c], wq);
                        acc[c] = i == 0 ? w[0][c] * m : fmaf(w[i][c], m, acc[c]);
                    }
                    const float gq = gv * wq;
                    ax[i] = fmaf(gq, dx, ax[i]);
                    ay[i] = fmaf(gq, dy, ay[i]);
                    az[i] = fmaf(gq, dz, az[i]);
                }
            }
            scatter_add_node(acc, lane, &G[(size_t)t * C + c0]);
        }
        if (any_open) {
            if (!leaf) {
#pragma unroll
                for (int i = 0; i < K; ++i) depth[i] = descend(depth[i], lvl, open[i]);
            } else {
                for_leaf_points<CB, BF16>(pts, attr, as, c0, nd.first, node_count(nd),
                                          [&](uint32_t j, const PointRec &pr, const float (&mu)[CB]) {
                    float acc[CB];
#pragma unroll
                    for (int c = 0; c < CB; ++c) acc[c] = 0.0f;
#pragma unroll
                    for (int i = 0; i < K; ++i) {
                        if (open[i]) {
                            const float dx = pr.x - px[i], dy = pr.y - py[i], dz = pr.z - pz[i];
                            const float r2 = dot3(dx, dy, dz, dx, dy, dz);
                            if (r2 > 0.0f) {
                                float m, gv;
                                mono_radial(r2, kp, m, gv);
                                const float am = pr.a * m;
                                float wm = 0.0f;
#pragma unroll
                                for (int c = 0; c < CB; ++c) {
                                    wm = fmaf(w[i][c], mu[c], wm);
                                    acc[c] = fmaf(w[i][c], am, acc[c]);
                                }
                                const float ga = pr.a * gv * wm;
                                ax[i] = fmaf(ga, dx, ax[i]);
                                ay[i] = fmaf(ga, dy, ay[i]);
                                az[i] = fmaf(ga, dz, az[i]);
                            }
                        }
                    }
                    scatter_add_node(acc, lane, &P[(size_t)j * C + c0]);
                });
            }
        }
        if (next == kEnd) break;
        t = next;
        nd = nn;
#pragma unroll
        for (int c = 0; c < CB; ++c) Qc[c] = Qn[c];
    }
    if (dx_mode != 0) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int64_t q = q0 + 64 * i;
            if (q < Q) {
                if (dx_mode == 1) {
                    dxout[3 * q] = ax[i];
                    dxout[3 * q + 1] = ay[i];
                    dxout[3 * q + 2] = az[i];
                } else {
                    dxout[3 * q] += ax[i];
                    dxout[3 * q + 1] += ay[i];
                    dxout[3 * q + 2] += az[i];
                }
            }
        }
    }
}

template <int CB, bool BF16, int K>
__global__ __launch_bounds__(kThreads) void k_mono_adjoint(DPS_KERN_PARAMS, int C, const float *__restrict__ df,
                                                           double *__restrict__ G, double *__restrict__ P,
                                                           float *__restrict__ dxout, int dx_mode, int xcd_remap) {
    DPS_ROWS;
    const int64_t blk = remap_block(xcd_remap);
    if (blk < 0 || blk * (int64_t)blockDim.x * K >= Q) return;  // whole block past the rows
    const int64_t wave = (blk * blockDim.x + threadIdx.x) >> 6;
    mono_adjoint_body<CB, BF16, K>(wave * 64 * K + (threadIdx.x & 63), DPS_TRAV_ARGS, C, df, G, P, dxout, dx_mode);
}

template <int CB, bool BF16, int K>
__global__ __launch_bounds__(kThreads) void k_mono_adjoint_persistent(DPS_KERN_PARAMS, int C,
                                                                      const float *__restrict__ df,
                                                                      double *__restrict__ G,
                                                                      double *__restrict__ P,
                                                                      float *__restrict__ dxout, int dx_mode,
                                                                      uint32_t *__restrict__ ctr) {
    DPS_ROWS;
    const int64_t ntiles = (Q + 64 * K - 1) / (64 * K);
    int part = xcc_id();
    for (;;) {
        const int64_t tile = next_tile(ctr, ntiles, part);
        if (tile < 0) break;
        mono_adjoint_body<CB, BF16, K>(tile * 64 * K + (threadIdx.x & 63), DPS_TRAV_ARGS, C, df, G, P, dxout,
                                       dx_mode);
    }
}

// ---------------------------------------------------------------------------
// host dispatch
// ---------------------------------------------------------------------------

// channels per walk without gradients (16 or 32)
#ifndef DPS_MONO_TOP
#define DPS_MONO_TOP 16
#endif

// channel blocks: DPS_MONO_TOP (8 with gradients), then halving
inline int mono_block(int rem, bool grad) {
    const int top = grad ? 8 : DPS_MONO_TOP;
    for (int b = top; b > 1; b >>= 1)
        if (rem >= b) return b;
    return 1;
}

// queries per lane: the largest of 1, 2, 4 not above the tree's setting with
// at most `budget` per-lane accumulator floats
constexpr bool mono_k_fits(int k, int per_query, int budget) { return k * per_query <= budget; }

inline int mono_packet(int k, int per_query, int budget) {
    k = k >= 4 ? 4 : (k >= 2 ? 2 : 1);
    while (k > 1 && !mono_k_fits(k, per_query, budget)) k >>= 1;
    return k;
}

constexpr int kMonoQueryBudget = 32;    // f (and 3 gradient components) per channel
constexpr int kMonoAdjointBudget = 40;  // df per channel and dL/dx

template <int CB, bool BF, bool GR, int K>
dps_status mono_query_launch(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float b2,
                             KernelParams kp, Sub sb, float *f, float *g, hipStream_t s) {
    const uint32_t lim = walk_limit(t);
    if (t->launch_flags & kFlagPersistentQuery) {
        k_fill_u32<<<1, 64, 0, s>>>(t->ctr, 8, 0u);
        const void *fn = reinterpret_cast<const void *>(&k_mono_query_persistent<CB, BF, GR, K>);
        k_mono_query_persistent<CB, BF, GR, K><<<persistent_grid(fn), kThreads, 0, s>>>(
            t->nodes, t->pts, trav_mom(t), t->attr, t->mom_stride, t->attr_stride, x, Q, qdev, b2, kp, sb.c0, sb.ldo, sb.co,
            lim, t->err, f, g, t->ctr);
    } else {
        const unsigned nb = grid(cdiv(Q, K));
        const bool remap = (t->launch_flags & kFlagXcdQuery) != 0;
        const unsigned gr = remap ? (unsigned)(8 * cdiv(nb, 8)) : nb;
        k_mono_query<CB, BF, GR, K><<<gr, kThreads, 0, s>>>(t->nodes, t->pts, trav_mom(t), t->attr, t->mom_stride,
                                                            t->attr_stride, x, Q, qdev, b2, kp, sb.c0, sb.ldo, sb.co,
                                                            lim, t->err, f, g, remap ? (int)nb : 0);
    }
    return hip_status(hipGetLastError(), "monopole query launch");
}

template <int CB, bool BF, bool GR>
dps_status mono_query_k(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float b2, KernelParams kp,
                        Sub sb, float *f, float *g, hipStream_t s) {
    constexpr int per = GR ? 4 * CB : CB;
    switch (mono_packet(t->packet_query, per, kMonoQueryBudget)) {
        case 4:
            if constexpr (mono_k_fits(4, per, kMonoQueryBudget))
                return mono_query_launch<CB, BF, GR, 4>(t, x, Q, qdev, b2, kp, sb, f, g, s);
            [[fallthrough]];
        case 2:
            if constexpr (mono_k_fits(2, per, kMonoQueryBudget))
                return mono_query_launch<CB, BF, GR, 2>(t, x, Q, qdev, b2, kp, sb, f, g, s);
            [[fallthrough]];
        default:
            return mono_query_launch<CB, BF, GR, 1>(t, x, Q, qdev, b2, kp, sb, f, g, s);
    }
}

template <int CB>
dps_status mono_query_block(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float b2, KernelParams kp,
                            Sub sb, float *f, float *g, hipStream_t s) {
    const bool bf = t->storage == DPS_STORE_BF16;
    if constexpr (CB <= 8) {
        if (g) {
            if (bf) return mono_query_k<CB, true, true>(t, x, Q, qdev, b2, kp, sb, f, g, s);
            return mono_query_k<CB, false, true>(t, x, Q, qdev, b2, kp, sb, f, g, s);
        }
    }
    if (bf) return mono_query_k<CB, true, false>(t, x, Q, qdev, b2, kp, sb, f, nullptr, s);
    return mono_query_k<CB, false, false>(t, x, Q, qdev, b2, kp, sb, f, nullptr, s);
}

template <int CB, bool BF, int K>
dps_status mono_adjoint_launch(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float b2,
                               KernelParams kp, Sub sb, const float *df, float *dx, int dx_mode, hipStream_t s) {
    const uint32_t lim = walk_limit(t);
    if (t->launch_flags & kFlagPersistentAdjoint) {
        k_fill_u32<<<1, 64, 0, s>>>(t->ctr + 8, 8, 0u);
        const void *fn = reinterpret_cast<const void *>(&k_mono_adjoint_persistent<CB, BF, K>);
        k_mono_adjoint_persistent<CB, BF, K><<<persistent_grid(fn), kThreads, 0, s>>>(
            t->nodes, t->pts, trav_mom(t), t->attr, t->mom_stride, t->attr_stride, x, Q, qdev, b2, kp, sb.c0, sb.ldo, sb.co,
            lim, t->err, t->C, df, t->G, t->P, dx, dx_mode, t->ctr + 8);
    } else {
        const unsigned nb = grid(cdiv(Q, K));
        const bool remap = (t->launch_flags & kFlagXcdAdjoint) != 0;
        const unsigned gr = remap ? (unsigned)(8 * cdiv(nb, 8)) : nb;
        k_mono_adjoint<CB, BF, K><<<gr, kThreads, 0, s>>>(t->nodes, t->pts, trav_mom(t), t->attr, t->mom_stride,
                                                          t->attr_stride, x, Q, qdev, b2, kp, sb.c0, sb.ldo, sb.co,
                                                          lim, t->err, t->C, df, t->G, t->P, dx, dx_mode,
                                                          remap ? (int)nb : 0);
    }
    return hip_status(hipGetLastError(), "monopole adjoint launch");
}

template <int CB, bool BF>
dps_status mono_adjoint_k(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float b2, KernelParams kp,
                          Sub sb, const float *df, float *dx, int dx_mode, hipStream_t s) {
    constexpr int per = CB + 3;
    switch (mono_packet(t->packet_adjoint, per, kMonoAdjointBudget)) {
        case 4:
            if constexpr (mono_k_fits(4, per, kMonoAdjointBudget))
                return mono_adjoint_launch<CB, BF, 4>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, s);
            [[fallthrough]];
        case 2:
            if constexpr (mono_k_fits(2, per, kMonoAdjointBudget))
                return mono_adjoint_launch<CB, BF, 2>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, s);
            [[fallthrough]];
        default:
            return mono_adjoint_launch<CB, BF, 1>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, s);
    }
}

template <int CB>
dps_status mono_adjoint_block(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float b2,
                              KernelParams kp, Sub sb, const float *df, float *dx, int dx_mode, hipStream_t s) {
    if (t->storage == DPS_STORE_BF16) return mono_adjoint_k<CB, true>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, s);
    return mono_adjoint_k<CB, false>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, s);
}

}  // namespace

dps_status launch_query_mono(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float beta, float eps,
                             int cbegin, int nc, float *f, float *g, hipStream_t s) {
    const float b2 = mul_rn(beta, beta);
    const KernelParams kp = tree_kernel_params(t, eps);
    for (int c0 = cbegin; c0 < cbegin + nc;) {
        const int cb = mono_block(cbegin + nc - c0, g != nullptr);
        const Sub sb{c0, nc, c0 - cbegin};
        dps_status st;
        switch (cb) {
#if DPS_MONO_TOP >= 32
            case 32: st = mono_query_block<32>(t, x, Q, qdev, b2, kp, sb, f, g, s); break;
#endif
            case 16: st = mono_query_block<16>(t, x, Q, qdev, b2, kp, sb, f, g, s); break;
            case 8: st = mono_query_block<8>(t, x, Q, qdev, b2, kp, sb, f, g, s); break;
            case 4: st = mono_query_block<4>(t, x, Q, qdev, b2, kp, sb, f, g, s); break;
            case 2: st = mono_query_block<2>(t, x, Q, qdev, b2, kp, sb, f, g, s); break;
            default: st = mono_query_block<1>(t, x, Q, qdev, b2, kp, sb, f, g, s); break;
        }
        if (st != DPS_OK) return st;
        c0 += cb;
    }
    return DPS_OK;
}

dps_status launch_adjoint_mono(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float beta, float eps,
                               int cbegin, int nc, const float *df, float *dx, hipStream_t s) {
    const float b2 = mul_rn(beta, beta);
    const KernelParams kp = tree_kernel_params(t, eps);
    for (int c0 = cbegin; c0 < cbegin + nc;) {
        const int cb = mono_block(cbegin + nc - c0, false);
        const int dx_mode = dx ? (c0 == cbegin ? 1 : 2) : 0;
        const Sub sb{c0, nc, c0 - cbegin};
        dps_status st;
        switch (cb) {
#if DPS_MONO_TOP >= 32
            case 32: st = mono_adjoint_block<32>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, s); break;
#endif
            case 16: st = mono_adjoint_block<16>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, s); break;
            case 8: st = mono_adjoint_block<8>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, s); break;
            case 4: st = mono_adjoint_block<4>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, s); break;
            case 2: st = mono_adjoint_block<2>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, s); break;
            default: st = mono_adjoint_block<1>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, s); break;
        }
        if (st != DPS_OK) return st;
        c0 += cb;
    }
    return DPS_OK;
}

}  // namespace dps
