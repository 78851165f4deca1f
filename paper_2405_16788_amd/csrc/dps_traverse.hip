// dps_traverse.hip -- Barnes-Hut primal and adjoint dipole-sum queries.
//
// Algorithm 1 of the paper (PrimalQuery / AdjointQuery) visits, for one query
// x, every node whose ancestors were all opened; a node is used as far field
// iff |x - p_t| > beta r_t (tested before the leaf test), a leaf that is not
// far contributes the exact terms of its points, and an internal node that is
// not far recurses into its children.
//
// GPU mapping: a wavefront owns 64 queries and walks the union of their
// traversals once, in depth-first order, without a stack:
//   - `t` (the current node) is wave-uniform, so node records, moments and leaf
//     points are fetched with scalar loads and broadcast to all lanes;
//   - each lane keeps the depth of the deepest level on the current path whose
//     ancestors it all opened: it visits the current node (Algorithm 1 would)
//     iff the node's level is at most that depth;
//   - after a node, the wave descends to its first child if any lane opened it
//     (lanes that did not fall back to the node's level), otherwise follows the
//     node's escape pointer (next sibling, or the parent's escape).
// Every lane therefore makes exactly the decisions of the recursive algorithm,
// in the same depth-first order; lanes not visiting a node are masked off.
//
// The adjoint reduces each far-field increment (eq. farfield_gradient) and each
// near-field point increment over the wavefront with DPP before one lane-
// parallel FP64 atomic per value; dL/dx is private to the lane.
#include <algorithm>

#include "dps_trav_common.h"
#include "dps_walk.h"

namespace dps {

namespace {

// ---------------------------------------------------------------------------
// primal query, one query per lane (register-lean).  Software-pipelined: the
// next node is known right after the ballots, so its record and moments are
// fetched before the far-field / leaf work of the current node.
// ---------------------------------------------------------------------------
template <int CB, bool BF16, bool GRAD, bool GRID = false, bool SPLIT = false>
__device__ __forceinline__ void query1_body(int64_t q, DPS_TRAV_PARAMS, float *__restrict__ fout,
                                            float *__restrict__ gout, const GridSpec &gs = GridSpec{},
                                            const Split &sp = Split{}) {
    bool valid = q < Q;
    float px = 0.0f, py = 0.0f, pz = 0.0f;
    int64_t row = q;
    if constexpr (GRID) {
        valid = grid_point(gs, q, px, py, pz, row) && valid;
    } else if (valid) {
        px = x[3 * q];
        py = x[3 * q + 1];
        pz = x[3 * q + 2];
    }
    float f[CB], g[CB][3];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        f[c] = 0.0f;
        g[c][0] = g[c][1] = g[c][2] = 0.0f;
    }
    int32_t depth = valid ? 0 : -1;
    const float b2v = in_vgpr(b2);
    uint32_t t = 0;
    NodeRec nd = nodes[0];
    float D[3 * CB];
    load_moments<CB, BF16>(mom, ms, 0, c0, D, kp.nhi);
    uint32_t steps = 0;
    for (;;) {
        if (++steps > limit) {  // a well-formed tree is walked in at most N steps
            if ((threadIdx.x & 63) == 0) atomicOr(err, 1u);
            break;
        }
        const uint32_t lvl = nd.meta & 0xffu;
        const bool leaf = (nd.meta & kLeafFlag) != 0;
        bool own = true, skip = false;
        if constexpr (SPLIT) split_node(sp, t, lvl, leaf, own, skip);
        const bool in = !skip && visits(depth, lvl);
        const float s = dist2_rn(nd.cx, nd.cy, nd.cz, px, py, pz);
        const bool beyond = s > mul_rn(b2v, nd.r2);
        const bool far = in && beyond && own;
        const bool open = in && !beyond;
        WaveMasks wm;
        if (!skip) wm.add(visits(depth, lvl), beyond);
        const bool any_far = own && wm.far != 0;
        const bool any_open = wm.open != 0;
        const uint32_t next = (any_open && !leaf) ? nd.first : nd.escape;
        const uint32_t pf = next;  // kEnd is the root: a valid record
        const NodeRec nn = nodes[pf];
        float Dn[3 * CB];
        load_moments<CB, BF16>(mom, ms, pf, c0, Dn, kp.nhi);
        if (any_far && far) {
            refine_moments<CB, BF16>(mom, ms, t, c0, D, kp.nhi);
            float kap, lam;
            radial<true>(s, kp, kap, lam);
            const float dx = nd.cx - px, dy = nd.cy - py, dz = nd.cz - pz;
            // lambda (p_t - x) once, then the gradient is 6 FMAs per channel
            const float lx = lam * dx, ly = lam * dy, lz = lam * dz;
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const float sd = dot3(D[3 * c], D[3 * c + 1], D[3 * c + 2], dx, dy, dz);
                f[c] = fmaf(kap, sd, f[c]);
                if (GRAD) {
                    g[c][0] = fmaf(-kap, D[3 * c], fmaf(sd, lx, g[c][0]));
                    g[c][1] = fmaf(-kap, D[3 * c + 1], fmaf(sd, ly, g[c][1]));
                    g[c][2] = fmaf(-kap, D[3 * c + 2], fmaf(sd, lz, g[c][2]));
                }
            }
        }
        if (any_open) {
            if (!leaf) {
                depth = descend(depth, lvl, open);
            } else {
                for_leaf_points<CB, BF16>(pts, attr, as, c0, nd.first, node_count(nd),
                                          [&](uint32_t, const PointRec &pr, const float (&mu)[CB]) {
                    if (open) {
                        const float dx = pr.x - px, dy = pr.y - py, dz = pr.z - pz;
                        const float r2 = dot3(dx, dy, dz, dx, dy, dz);
                        float kap, lam;
                        if (radial(r2, kp, kap, lam)) {
                            const float sa = dot3(pr.anx, pr.any, pr.anz, dx, dy, dz);
                            const float ks = kap * sa;
                            const float ls = lam * sa;
                            const float G0 = fmaf(ls, dx, -kap * pr.anx);
                            const float G1 = fmaf(ls, dy, -kap * pr.any);
                            const float G2 = fmaf(ls, dz, -kap * pr.anz);
#pragma unroll
                            for (int c = 0; c < CB; ++c) {
                                f[c] = fmaf(mu[c], ks, f[c]);
                                if (GRAD) {
                                    g[c][0] = fmaf(mu[c], G0, g[c][0]);
                                    g[c][1] = fmaf(mu[c], G1, g[c][1]);
                                    g[c][2] = fmaf(mu[c], G2, g[c][2]);
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
        for (int v = 0; v < 3 * CB; ++v) D[v] = Dn[v];
    }
    if (valid) {
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int64_t o = row * ldo + co + c;
            if constexpr (SPLIT) {  // the parts' sums meet in the zero-filled outputs
                atomicAdd(&fout[o], f[c]);
                if (GRAD) {
                    atomicAdd(&gout[3 * o], g[c][0]);
                    atomicAdd(&gout[3 * o + 1], g[c][1]);
                    atomicAdd(&gout[3 * o + 2], g[c][2]);
                }
            } else {
                fout[o] = f[c];
                if (GRAD) {
                    gout[3 * o] = g[c][0];
                    gout[3 * o + 1] = g[c][1];
                    gout[3 * o + 2] = g[c][2];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// primal query, K queries per lane: the wavefront owns 64*K consecutive
// queries, lane l carrying queries q0 + 64 i (i < K), so node fetches, ballots
// and loop control are shared by 64*K queries (packet traversal).
// ---------------------------------------------------------------------------
template <int CB, bool BF16, bool GRAD, int K, bool GRID = false>
__device__ __forceinline__ void queryk_body(int64_t q0, DPS_TRAV_PARAMS, float *__restrict__ fout,
                                            float *__restrict__ gout, const GridSpec &gs = GridSpec{}) {
    float px[K], py[K], pz[K];
    int32_t depth[K];
    float f[K][CB], g[K][CB][3];
    int64_t row[K];
    bool vld[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int64_t q = q0 + 64 * i;
        bool valid = q < Q;
        row[i] = q;
        if constexpr (GRID) {
            valid = grid_point(gs, q, px[i], py[i], pz[i], row[i]) && valid;
        }
        vld[i] = valid;
        if constexpr (!GRID) {
            px[i] = valid ? x[3 * q] : 0.0f;
            py[i] = valid ? x[3 * q + 1] : 0.0f;
            pz[i] = valid ? x[3 * q + 2] : 0.0f;
        }
        depth[i] = valid ? 0 : -1;
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            f[i][c] = 0.0f;
            g[i][c][0] = g[i][c][1] = g[i][c][2] = 0.0f;
        }
    }
    if constexpr (CB == 1 && !GRAD) {
        // one channel without gradients (grids, level-set values): the
        // predicated walk of the ray march, the same values bit for bit with
        // fewer scalar instructions per node
        dipole_walk<1, BF16, false, K>(px, py, pz, depth, f, g, nodes, pts, mom, attr, ms, as, b2, kp, c0, limit,
                                       err);
    } else {
        const float b2v = in_vgpr(b2);
        uint32_t t = 0;
        NodeRec nd = nodes[0];
        float D[3 * CB];
        load_moments<CB, BF16>(mom, ms, 0, c0, D, kp.nhi);
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
            float Dn[3 * CB];
            load_moments<CB, BF16>(mom, ms, pf, c0, Dn, kp.nhi);
            if (any_far) {
                refine_moments<CB, BF16>(mom, ms, t, c0, D, kp.nhi);
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    if (far[i]) {
                        float kap, lam;
                        radial<true>(s[i], kp, kap, lam);
                        const float dx = nd.cx - px[i], dy = nd.cy - py[i], dz = nd.cz - pz[i];
                        // lambda (p_t - x) once, then the gradient is 6 FMAs per channel
                        const float lx = lam * dx, ly = lam * dy, lz = lam * dz;
#pragma unroll
                        for (int c = 0; c < CB; ++c) {
                            const float sd = dot3(D[3 * c], D[3 * c + 1], D[3 * c + 2], dx, dy, dz);
                            f[i][c] = fmaf(kap, sd, f[i][c]);
                            if (GRAD) {
                                g[i][c][0] = fmaf(-kap, D[3 * c], fmaf(sd, lx, g[i][c][0]));
                                g[i][c][1] = fmaf(-kap, D[3 * c + 1], fmaf(sd, ly, g[i][c][1]));
                                g[i][c][2] = fmaf(-kap, D[3 * c + 2], fmaf(sd, lz, g[i][c][2]));
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
                    for_leaf_points<CB, BF16, false>(pts, attr, as, c0, nd.first, node_count(nd),
                                              [&](uint32_t, const PointRec &pr, const float (&mu)[CB]) {
#pragma unroll
                        for (int i = 0; i < K; ++i) {
                            if (open[i]) {
                                const float dx = pr.x - px[i], dy = pr.y - py[i], dz = pr.z - pz[i];
                                const float r2 = dot3(dx, dy, dz, dx, dy, dz);
                                float kap, lam;
                                if (radial(r2, kp, kap, lam)) {
                                    const float sa = dot3(pr.anx, pr.any, pr.anz, dx, dy, dz);
                                    const float ks = kap * sa;
                                    const float ls = lam * sa;
                                    const float G0 = fmaf(ls, dx, -kap * pr.anx);
                                    const float G1 = fmaf(ls, dy, -kap * pr.any);
                                    const float G2 = fmaf(ls, dz, -kap * pr.anz);
#pragma unroll
                                    for (int c = 0; c < CB; ++c) {
                                        f[i][c] = fmaf(mu[c], ks, f[i][c]);
                                        if (GRAD) {
                                            g[i][c][0] = fmaf(mu[c], G0, g[i][c][0]);
                                            g[i][c][1] = fmaf(mu[c], G1, g[i][c][1]);
                                            g[i][c][2] = fmaf(mu[c], G2, g[i][c][2]);
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
            for (int v = 0; v < 3 * CB; ++v) D[v] = Dn[v];
        }
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
        if (vld[i]) {
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int64_t o = row[i] * ldo + co + c;
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

template <int CB, bool BF16, bool GRAD, int K, bool GRID = false>
__device__ __forceinline__ void query_body(int64_t q0, DPS_TRAV_PARAMS, float *__restrict__ fout,
                                           float *__restrict__ gout, const GridSpec &gs = GridSpec{}) {
    if constexpr (K == 1) query1_body<CB, BF16, GRAD, GRID>(q0, DPS_TRAV_ARGS, fout, gout, gs);
    else queryk_body<CB, BF16, GRAD, K, GRID>(q0, DPS_TRAV_ARGS, fout, gout, gs);
}

template <int CB, bool BF16, bool GRAD, int K>
__global__ __launch_bounds__(kThreads) void k_query(DPS_KERN_PARAMS, float *__restrict__ fout,
                                                    float *__restrict__ gout, int xcd_remap) {
    DPS_ROWS;
    const int64_t blk = remap_block(xcd_remap);
    if (blk < 0 || blk * (int64_t)blockDim.x * K >= Q) return;  // whole block past the rows
    const int64_t wave = (blk * blockDim.x + threadIdx.x) >> 6;
    query_body<CB, BF16, GRAD, K>(wave * 64 * K + (threadIdx.x & 63), DPS_TRAV_ARGS, fout, gout);
}

// subtree-split query: wavefront w takes part w mod parts of tile w / parts,
// one query per lane, and adds its sums into zero-filled outputs
template <int CB, bool BF16, bool GRAD>
__global__ __launch_bounds__(kThreads) void k_query_split(DPS_KERN_PARAMS, float *__restrict__ fout,
                                                          float *__restrict__ gout, Split sp, int shift) {
    DPS_ROWS;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t tile = wave >> shift;
    if (tile * 64 >= Q) return;  // wave-uniform
    sp.part = __builtin_amdgcn_readfirstlane((uint32_t)wave & sp.mask);  // wave-uniform
    query1_body<CB, BF16, GRAD, false, true>(tile * 64 + (threadIdx.x & 63), DPS_TRAV_ARGS, fout, gout, GridSpec{},
                                             sp);
}

template <int CB, bool BF16, bool GRAD, int K>
__global__ __launch_bounds__(kThreads) void k_query_persistent(DPS_KERN_PARAMS, float *__restrict__ fout,
                                                               float *__restrict__ gout,
                                                               uint32_t *__restrict__ ctr) {
    DPS_ROWS;
    const int64_t ntiles = (Q + 64 * K - 1) / (64 * K);
    int part = xcc_id();
    for (;;) {
        const int64_t tile = next_tile(ctr, ntiles, part);
        if (tile < 0) break;
        query_body<CB, BF16, GRAD, K>(tile * 64 * K + (threadIdx.x & 63), DPS_TRAV_ARGS, fout, gout);
    }
}

// grid queries: persistent tile queue over the bricks (Q = 64 * bricks)
template <int CB, bool BF16, bool GRAD, int K>
__global__ __launch_bounds__(kThreads) void k_query_grid(DPS_KERN_PARAMS, float *__restrict__ fout,
                                                         float *__restrict__ gout, GridSpec gs,
                                                         uint32_t *__restrict__ ctr) {
    DPS_ROWS;
    const int64_t ntiles = (Q + 64 * K - 1) / (64 * K);
    int part = xcc_id();
    for (;;) {
        const int64_t tile = next_tile(ctr, ntiles, part);
        if (tile < 0) break;
        query_body<CB, BF16, GRAD, K, true>(tile * 64 * K + (threadIdx.x & 63), DPS_TRAV_ARGS, fout, gout, gs);
    }
}

// ---------------------------------------------------------------------------
// traversal statistics with the same decisions
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_counts(const NodeRec *__restrict__ nodes,
                                                     const float *__restrict__ x, int64_t Q, float b2,
                                                     int32_t *__restrict__ counts, uint32_t limit,
                                                     uint32_t *__restrict__ err) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = q < Q;
    float px = 0.0f, py = 0.0f, pz = 0.0f;
    if (valid) {
        px = x[3 * q];
        py = x[3 * q + 1];
        pz = x[3 * q + 2];
    }
    int32_t nvisit = 0, nfar = 0, leaves = 0, near = 0;
    int32_t depth = valid ? 0 : -1;
    uint32_t t = 0;
    uint32_t steps = 0;
    for (;;) {
        if (++steps > limit) {  // a well-formed tree is walked in at most N steps
            if (threadIdx.x % 64 == 0) atomicOr(err, 1u);
            break;
        }
        const NodeRec nd = nodes[t];
        const uint32_t lvl = nd.meta & 0xffu;
        const bool in = visits(depth, lvl);
        const float s = dist2_rn(nd.cx, nd.cy, nd.cz, px, py, pz);
        const bool far = in && (s > mul_rn(b2, nd.r2));
        const bool open = in && !far;
        nvisit += in;
        nfar += far;
        uint32_t next = nd.escape;
        if (__ballot(open)) {
            if (!(nd.meta & kLeafFlag)) {
                depth = descend(depth, lvl, open);
            } else {
                leaves += open;
                near += open ? (int32_t)node_count(nd) : 0;
            }
            next = nd.down;
        }
        if (next == kEnd) break;
        t = next;
    }
    if (valid) {
        counts[4 * q] = nvisit;
        counts[4 * q + 1] = nfar;
        counts[4 * q + 2] = leaves;
        counts[4 * q + 3] = near;
    }
}

// ---------------------------------------------------------------------------
// adjoint stage 1 (Algorithm 1, AdjointQuery): node accumulators G[N][C][3]
// (eq. farfield_gradient), point accumulators P[M][C], dL/dx per query.
//
// DX: dL/dx = sum_c df_c grad D_c is formed in the walk from the same
// accepted sources.  Without DX the walk only accumulates the node and point
// increments (kappa alone per term); dL/dx is then either not wanted
// (dx_mode 0) or formed from the gradients the forward query already
// computed at these points (gin [Q][ldo][3], same tree state, beta and eps):
// the identical sum, 3 CB multiply-adds per query instead of a second
// evaluation of every term's gradient.
// ---------------------------------------------------------------------------
template <int CB, bool BF16, int K, bool DX, bool SPLIT = false>
__device__ __forceinline__ void adjoint_body(int64_t q0, DPS_TRAV_PARAMS, int C, const float *__restrict__ df,
                                             double *__restrict__ G, double *__restrict__ P,
                                             float *__restrict__ dxout, int dx_mode,
                                             const float *__restrict__ gin, const Split &sp = Split{}) {
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
    float D[3 * CB];
    load_moments<CB, BF16>(mom, ms, 0, c0, D, kp.nhi);
    uint32_t steps = 0;
    for (;;) {
        if (++steps > limit) {  // a well-formed tree is walked in at most N steps
            if (lane == 0) atomicOr(err, 1u);
            break;
        }
        const uint32_t lvl = nd.meta & 0xffu;
        const bool leaf = (nd.meta & kLeafFlag) != 0;
        const float lim = mul_rn(b2v, nd.r2);
        bool own = true, skip = false;
        if constexpr (SPLIT) split_node(sp, t, lvl, leaf, own, skip);
        bool far[K], open[K];
        float s[K];
        WaveMasks wm;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const bool in = !skip && visits(depth[i], lvl);
            s[i] = dist2_rn(nd.cx, nd.cy, nd.cz, px[i], py[i], pz[i]);
            const bool beyond = s[i] > lim;
            far[i] = in && beyond && own;
            open[i] = in && !beyond;
            if (!skip) wm.add(visits(depth[i], lvl), beyond);
        }
        const bool any_far = own && wm.far != 0;
        const bool any_open = wm.open != 0;
        const uint32_t next = (any_open && !leaf) ? nd.first : nd.escape;
        const uint32_t pf = next;  // kEnd is the root: a valid record
        const NodeRec nn = nodes[pf];
        float Dn[3 * CB];
        load_moments<CB, BF16>(mom, ms, pf, c0, Dn, kp.nhi);
        if (any_far) {
            refine_moments<CB, BF16>(mom, ms, t, c0, D, kp.nhi);
            // node increment sum_q df_c kappa (p_t - x_q), first over the lane's
            // queries.  Query slot 0 writes the sums on every lane, with zero
            // factors where it is not far (at a huge distance, so it takes the
            // plain path): no separate zero fill, which the compiler emitted as
            // 17 moves per node; the other slots add where their query is far.
            float acc[3 * CB];
#pragma unroll
            for (int i = 0; i < K; ++i) {
                if (i == 0 || far[i]) {
                    const bool off = i == 0 && !far[0];
                    float kap, lam = 0.0f;
                    if constexpr (DX) radial<true>(off ? kHugeR2 : s[i], kp, kap, lam);
                    else radial_kappa<true>(off ? kHugeR2 : s[i], kp, kap);
                    kap = off ? 0.0f : kap;
                    lam = off ? 0.0f : lam;
                    const float dx = nd.cx - px[i], dy = nd.cy - py[i], dz = nd.cz - pz[i];
                    float E0 = 0.0f, E1 = 0.0f, E2 = 0.0f;
                    // kappa (p_t - x_q) once, then one FMA per channel and axis
                    const float kx = kap * dx, ky = kap * dy, kz = kap * dz;
#pragma unroll
                    for (int c = 0; c < CB; ++c) {
                        if constexpr (DX) {
                            E0 += w[i][c] * D[3 * c];
                            E1 += w[i][c] * D[3 * c + 1];
                            E2 += w[i][c] * D[3 * c + 2];
                        }
                        if (i == 0) {
                            acc[3 * c] = w[0][c] * kx;
                            acc[3 * c + 1] = w[0][c] * ky;
                            acc[3 * c + 2] = w[0][c] * kz;
                        } else {
                            acc[3 * c] = fmaf(w[i][c], kx, acc[3 * c]);
                            acc[3 * c + 1] = fmaf(w[i][c], ky, acc[3 * c + 1]);
                            acc[3 * c + 2] = fmaf(w[i][c], kz, acc[3 * c + 2]);
                        }
                    }
                    if constexpr (DX) {
                        const float les = lam * dot3(E0, E1, E2, dx, dy, dz);
                        ax[i] = fmaf(-kap, E0, fmaf(les, dx, ax[i]));
                        ay[i] = fmaf(-kap, E1, fmaf(les, dy, ay[i]));
                        az[i] = fmaf(-kap, E2, fmaf(les, dz, az[i]));
                    }
                }
            }
            scatter_add_node(acc, lane, &G[((size_t)t * C + c0) * 3]);
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
                            float kap, lam = 0.0f;
                            const bool term = DX ? radial(r2, kp, kap, lam) : radial_kappa(r2, kp, kap);
                            if (term) {
                                const float sa = dot3(pr.anx, pr.any, pr.anz, dx, dy, dz);
                                const float ks = kap * sa;
                                float wm = 0.0f;
#pragma unroll
                                for (int c = 0; c < CB; ++c) {
                                    if constexpr (DX) wm += w[i][c] * mu[c];
                                    acc[c] += w[i][c] * ks;
                                }
                                if constexpr (DX) {
                                    const float les = lam * sa * wm;
                                    const float kw = kap * wm;
                                    ax[i] = fmaf(-kw, pr.anx, fmaf(les, dx, ax[i]));
                                    ay[i] = fmaf(-kw, pr.any, fmaf(les, dy, ay[i]));
                                    az[i] = fmaf(-kw, pr.anz, fmaf(les, dz, az[i]));
                                }
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
        for (int v = 0; v < 3 * CB; ++v) D[v] = Dn[v];
    }
    static_assert(!(SPLIT && DX), "a split walk forms no dL/dx");
    if (dx_mode != 0 && (!SPLIT || sp.part == 0)) {  // one part writes dL/dx
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int64_t q = q0 + 64 * i;
            if (q < Q) {
                if constexpr (!DX) {  // sum_c df_c grad D_c from the forward's gradients
                    const float *gq = gin + 3 * (q * ldo + co);
                    float gx = 0.0f, gy = 0.0f, gz = 0.0f;
#pragma unroll
                    for (int c = 0; c < CB; ++c) {
                        gx = fmaf(w[i][c], gq[3 * c], gx);
                        gy = fmaf(w[i][c], gq[3 * c + 1], gy);
                        gz = fmaf(w[i][c], gq[3 * c + 2], gz);
                    }
                    ax[i] = gx;
                    ay[i] = gy;
                    az[i] = gz;
                }
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

template <int CB, bool BF16, int K, bool DX>
__global__ __launch_bounds__(kThreads) void k_adjoint(DPS_KERN_PARAMS, int C, const float *__restrict__ df,
                                                      double *__restrict__ G, double *__restrict__ P,
                                                      float *__restrict__ dxout, int dx_mode,
                                                      const float *__restrict__ gin, int xcd_remap) {
    DPS_ROWS;
    const int64_t blk = remap_block(xcd_remap);
    if (blk < 0 || blk * (int64_t)blockDim.x * K >= Q) return;  // whole block past the rows
    const int64_t wave = (blk * blockDim.x + threadIdx.x) >> 6;
    adjoint_body<CB, BF16, K, DX>(wave * 64 * K + (threadIdx.x & 63), DPS_TRAV_ARGS, C, df, G, P, dxout, dx_mode,
                                  gin);
}

// subtree-split adjoint (accumulators only, dL/dx if wanted from the
// forward's gradients): wavefront w takes part w mod parts of tile w / parts
template <int CB, bool BF16>
__global__ __launch_bounds__(kThreads) void k_adjoint_split(DPS_KERN_PARAMS, int C, const float *__restrict__ df,
                                                            double *__restrict__ G, double *__restrict__ P,
                                                            float *__restrict__ dxout, int dx_mode,
                                                            const float *__restrict__ gin, Split sp, int shift) {
    DPS_ROWS;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t tile = wave >> shift;
    if (tile * 64 >= Q) return;  // wave-uniform
    sp.part = __builtin_amdgcn_readfirstlane((uint32_t)wave & sp.mask);  // wave-uniform
    adjoint_body<CB, BF16, 1, false, true>(tile * 64 + (threadIdx.x & 63), DPS_TRAV_ARGS, C, df, G, P, dxout,
                                           dx_mode, gin, sp);
}

// resident waves per SIMD requested for the 4-query, 4-channel persistent
// adjoint (register budgets of 96 and 80; measured faster than the unbounded
// 4 and 5 waves; the 6-wave build keeps 3 spilled values out of the node
// loop)
#ifndef DPS_ADJOINT_WAVES
#define DPS_ADJOINT_WAVES 5
#endif
// the same without the in-walk dL/dx (fewer live registers)
#ifndef DPS_ADJOINT_WAVES_NODX
#define DPS_ADJOINT_WAVES_NODX 6
#endif

template <int CB, bool BF16, int K, bool DX>
__global__ __launch_bounds__(kThreads, (CB == 4 && K == 4) ? (DX ? DPS_ADJOINT_WAVES : DPS_ADJOINT_WAVES_NODX) : 1) void k_adjoint_persistent(DPS_KERN_PARAMS, int C,
                                                                 const float *__restrict__ df,
                                                                 double *__restrict__ G, double *__restrict__ P,
                                                                 float *__restrict__ dxout, int dx_mode,
                                                                 const float *__restrict__ gin,
                                                                 uint32_t *__restrict__ ctr) {
    DPS_ROWS;
    const int64_t ntiles = (Q + 64 * K - 1) / (64 * K);
    int part = xcc_id();
    for (;;) {
        const int64_t tile = next_tile(ctr, ntiles, part);
        if (tile < 0) break;
        adjoint_body<CB, BF16, K, DX>(tile * 64 * K + (threadIdx.x & 63), DPS_TRAV_ARGS, C, df, G, P, dxout,
                                      dx_mode, gin);
    }
}

// ---------------------------------------------------------------------------
// adjoint with cotangents h = dL/d(grad D) of the spatial gradient (and,
// with DF, dL/dD of the values).  The gradient of a source term is linear in
// its dipole with d g / d D = lambda d d^T - kappa I, so h feeds the same node
// and point accumulators as df:  dD += (kappa w + lambda (d.h)) d - kappa h.
// dL/dx adds the Hessian of the term applied to h,
//   nu s (d.h) d - lambda (d (D.h) + D (d.h)) - lambda s h,  s = D.d,
// with nu = chi(t)/(4 pi r^7).  Per source and query, with
// beta_c = kappa w_c + lambda (d.h_c):
//   dx += [sum_c lambda w_c s_c + nu s_c (d.h_c) - lambda (D_c.h_c)] d
//         - sum_c beta_c D_c - lambda sum_c s_c h_c.
// ---------------------------------------------------------------------------
// EXT additionally accumulates, when the pointers are given, dL/deps into
// eacc (d kappa / d eps = -exp(-t^2) ke4, d lambda / d eps = -exp(-t^2) ke6,
// nonzero inside the regularised zone only) and the near-field part of dL/dn
// into pn: A_j sum_c mu_jc dL/dD_jc per point (the far-field part is pushed
// down from the node accumulators at the end).  dg may be NULL (zero).
template <int CB, bool BF16, int K, bool DF, bool EXT>
__device__ __forceinline__ void adjoint_g_body(int64_t q0, DPS_TRAV_PARAMS, int C, const float *__restrict__ df,
                                               const float *__restrict__ dg, double *__restrict__ G,
                                               double *__restrict__ P, float *__restrict__ dxout, int dx_mode,
                                               double *__restrict__ pn, double *__restrict__ eacc) {
    const int lane = lane_id();
    float px[K], py[K], pz[K], w[K][CB], h[K][CB][3], ax[K], ay[K], az[K];
    int32_t depth[K];
    float deps = 0.0f;
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
        for (int c = 0; c < CB; ++c) {
            w[i][c] = (DF && valid) ? df[q * ldo + co + c] : 0.0f;
#pragma unroll
            for (int j = 0; j < 3; ++j) h[i][c][j] = (dg && valid) ? dg[(q * ldo + co + c) * 3 + j] : 0.0f;
        }
    }
    const float b2v = in_vgpr(b2);
    uint32_t t = 0;
    NodeRec nd = nodes[0];
    float D[3 * CB];
    load_moments<CB, BF16>(mom, ms, 0, c0, D, kp.nhi);
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
        float s2[K];
        WaveMasks wm;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const bool in = visits(depth[i], lvl);
            s2[i] = dist2_rn(nd.cx, nd.cy, nd.cz, px[i], py[i], pz[i]);
            const bool beyond = s2[i] > lim;
            far[i] = in && beyond;
            open[i] = in && !beyond;
            wm.add(in, beyond);
        }
        const bool any_far = wm.far != 0;
        const bool any_open = wm.open != 0;
        const uint32_t next = (any_open && !leaf) ? nd.first : nd.escape;
        const uint32_t pf = next;  // kEnd is the root: a valid record
        const NodeRec nn = nodes[pf];
        float Dn[3 * CB];
        load_moments<CB, BF16>(mom, ms, pf, c0, Dn, kp.nhi);
        if (any_far) {
            refine_moments<CB, BF16>(mom, ms, t, c0, D, kp.nhi);
            // query slot 0 writes the node sums on every lane (zero factors
            // where it is not far, taken at a huge distance), the other slots
            // add where their query is far
            float acc[3 * CB];
#pragma unroll
            for (int i = 0; i < K; ++i) {
                if (i == 0 || far[i]) {
                    const bool off = i == 0 && !far[0];
                    const float si = off ? kHugeR2 : s2[i];
                    float kap, lam, nu;
                    radial3(si, kp, kap, lam, nu);
                    kap = off ? 0.0f : kap;
                    lam = off ? 0.0f : lam;
                    nu = off ? 0.0f : nu;
                    const float dx = nd.cx - px[i], dy = nd.cy - py[i], dz = nd.cz - pz[i];
                    float al = 0.0f, vx = 0.0f, vy = 0.0f, vz = 0.0f;
                    float e1 = 0.0f, e2 = 0.0f;  // sum_c (w_c s_c - D_c.h_c), sum_c s_c (d.h_c)
#pragma unroll
                    for (int c = 0; c < CB; ++c) {
                        const float Dx = D[3 * c], Dy = D[3 * c + 1], Dz = D[3 * c + 2];
                        const float hx = h[i][c][0], hy = h[i][c][1], hz = h[i][c][2];
                        const float sc = dot3(Dx, Dy, Dz, dx, dy, dz);
                        const float dh = dot3(dx, dy, dz, hx, hy, hz);
                        const float Dh = dot3(Dx, Dy, Dz, hx, hy, hz);
                        const float be = fmaf(kap, w[i][c], lam * dh);
                        al = fmaf(sc, fmaf(lam, w[i][c], nu * dh), fmaf(-lam, Dh, al));
                        const float ls = lam * sc;
                        vx = fmaf(be, Dx, fmaf(ls, hx, vx));
                        vy = fmaf(be, Dy, fmaf(ls, hy, vy));
                        vz = fmaf(be, Dz, fmaf(ls, hz, vz));
                        if (i == 0) {
                            acc[3 * c] = fmaf(be, dx, -kap * hx);
                            acc[3 * c + 1] = fmaf(be, dy, -kap * hy);
                            acc[3 * c + 2] = fmaf(be, dz, -kap * hz);
                        } else {
                            acc[3 * c] = fmaf(be, dx, fmaf(-kap, hx, acc[3 * c]));
                            acc[3 * c + 1] = fmaf(be, dy, fmaf(-kap, hy, acc[3 * c + 1]));
                            acc[3 * c + 2] = fmaf(be, dz, fmaf(-kap, hz, acc[3 * c + 2]));
                        }
                        if constexpr (EXT) {
                            e1 = fmaf(w[i][c], sc, e1 - Dh);
                            e2 = fmaf(sc, dh, e2);
                        }
                    }
                    ax[i] += fmaf(al, dx, -vx);
                    ay[i] += fmaf(al, dy, -vy);
                    az[i] += fmaf(al, dz, -vz);
                    if constexpr (EXT) {
                        if (eacc && si < kp.zone_r2) {
                            const float e = expf(-(si * kp.ieps2));
                            deps = fmaf(-e, fmaf(kp.ke4, e1, kp.ke6 * e2), deps);
                        }
                    }
                }
            }
            scatter_add_node(acc, lane, &G[((size_t)t * C + c0) * 3]);
        }
        if (any_open) {
            if (!leaf) {
#pragma unroll
                for (int i = 0; i < K; ++i) depth[i] = descend(depth[i], lvl, open[i]);
            } else {
                for_leaf_points<CB, BF16>(pts, attr, as, c0, nd.first, node_count(nd),
                                          [&](uint32_t j, const PointRec &pr, const float (&mu)[CB]) {
                    float acc[CB];
                    float nacc[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int c = 0; c < CB; ++c) acc[c] = 0.0f;
#pragma unroll
                    for (int i = 0; i < K; ++i) {
                        if (open[i]) {
                            const float dx = pr.x - px[i], dy = pr.y - py[i], dz = pr.z - pz[i];
                            const float r2 = dot3(dx, dy, dz, dx, dy, dz);
                            float kap, lam, nu;
                            if (radial3(r2, kp, kap, lam, nu)) {
                                const float sa = dot3(pr.anx, pr.any, pr.anz, dx, dy, dz);
                                float al = 0.0f, bsum = 0.0f, vx = 0.0f, vy = 0.0f, vz = 0.0f;
                                float hmx = 0.0f, hmy = 0.0f, hmz = 0.0f, e1 = 0.0f, e2 = 0.0f;
#pragma unroll
                                for (int c = 0; c < CB; ++c) {
                                    const float hx = h[i][c][0], hy = h[i][c][1], hz = h[i][c][2];
                                    const float dh = dot3(dx, dy, dz, hx, hy, hz);
                                    const float Ah = dot3(pr.anx, pr.any, pr.anz, hx, hy, hz);
                                    const float be = fmaf(kap, w[i][c], lam * dh);
                                    // point accumulator: (d g_c / d mu_c) . h_c and the value part
                                    acc[c] = fmaf(be, sa, fmaf(-kap, Ah, acc[c]));
                                    const float sc = mu[c] * sa;
                                    al = fmaf(sc, fmaf(lam, w[i][c], nu * dh), fmaf(-lam * mu[c], Ah, al));
                                    bsum = fmaf(be, mu[c], bsum);
                                    const float ls = lam * sc;
                                    vx = fmaf(ls, hx, vx);
                                    vy = fmaf(ls, hy, vy);
                                    vz = fmaf(ls, hz, vz);
                                    if constexpr (EXT) {
                                        hmx = fmaf(mu[c], hx, hmx);
                                        hmy = fmaf(mu[c], hy, hmy);
                                        hmz = fmaf(mu[c], hz, hmz);
                                        e1 = fmaf(w[i][c], sc, e1 - mu[c] * Ah);
                                        e2 = fmaf(sc, dh, e2);
                                    }
                                }
                                ax[i] += fmaf(al, dx, -fmaf(bsum, pr.anx, vx));
                                ay[i] += fmaf(al, dy, -fmaf(bsum, pr.any, vy));
                                az[i] += fmaf(al, dz, -fmaf(bsum, pr.anz, vz));
                                if constexpr (EXT) {
                                    // dL/dn_j of this term: A_j sum_c mu_c (beta_c d - kappa h_c)
                                    nacc[0] += pr.a * fmaf(bsum, dx, -kap * hmx);
                                    nacc[1] += pr.a * fmaf(bsum, dy, -kap * hmy);
                                    nacc[2] += pr.a * fmaf(bsum, dz, -kap * hmz);
                                    if (eacc && r2 < kp.zone_r2) {
                                        const float e = expf(-(r2 * kp.ieps2));
                                        deps = fmaf(-e, fmaf(kp.ke4, e1, kp.ke6 * e2), deps);
                                    }
                                }
                            }
                        }
                    }
                    scatter_add_node(acc, lane, &P[(size_t)j * C + c0]);
                    if constexpr (EXT) {
                        if (pn) scatter_add_node(nacc, lane, &pn[(size_t)j * 3]);
                    }
                });
            }
        }
        if (next == kEnd) break;
        t = next;
        nd = nn;
#pragma unroll
        for (int v = 0; v < 3 * CB; ++v) D[v] = Dn[v];
    }
    if constexpr (EXT) {
        if (eacc) {
            const float tot = wave_sum(deps);
            if (lane == 0) atomicAdd(eacc, (double)tot);
        }
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

template <int CB, bool BF16, int K, bool DF, bool EXT>
__global__ __launch_bounds__(kThreads) void k_adjoint_g(DPS_KERN_PARAMS, int C, const float *__restrict__ df,
                                                        const float *__restrict__ dg, double *__restrict__ G,
                                                        double *__restrict__ P, float *__restrict__ dxout,
                                                        int dx_mode, double *__restrict__ pn,
                                                        double *__restrict__ eacc, int xcd_remap) {
    DPS_ROWS;
    const int64_t blk = remap_block(xcd_remap);
    if (blk < 0 || blk * (int64_t)blockDim.x * K >= Q) return;  // whole block past the rows
    const int64_t wave = (blk * blockDim.x + threadIdx.x) >> 6;
    adjoint_g_body<CB, BF16, K, DF, EXT>(wave * 64 * K + (threadIdx.x & 63), DPS_TRAV_ARGS, C, df, dg, G, P, dxout,
                                         dx_mode, pn, eacc);
}

template <int CB, bool BF16, int K, bool DF, bool EXT>
__global__ __launch_bounds__(kThreads) void k_adjoint_g_persistent(DPS_KERN_PARAMS, int C,
                                                                   const float *__restrict__ df,
                                                                   const float *__restrict__ dg,
                                                                   double *__restrict__ G, double *__restrict__ P,
                                                                   float *__restrict__ dxout, int dx_mode,
                                                                   double *__restrict__ pn,
                                                                   double *__restrict__ eacc,
                                                                   uint32_t *__restrict__ ctr) {
    DPS_ROWS;
    const int64_t ntiles = (Q + 64 * K - 1) / (64 * K);
    int part = xcc_id();
    for (;;) {
        const int64_t tile = next_tile(ctr, ntiles, part);
        if (tile < 0) break;
        adjoint_g_body<CB, BF16, K, DF, EXT>(tile * 64 * K + (threadIdx.x & 63), DPS_TRAV_ARGS, C, df, dg, G, P,
                                             dxout, dx_mode, pn, eacc);
    }
}

// dL/dn in caller order: the pushed-down node accumulators at the point's
// leaf, A_j sum_c mu_jc S_leaf,c, plus the near-field accumulator
template <bool BF16>
__global__ void k_normals_out(int64_t M, int C, int as, const int32_t *__restrict__ leaf_of,
                              const uint32_t *__restrict__ perm, const PointRec *__restrict__ pts,
                              const void *__restrict__ attr, const double *__restrict__ PN,
                              const double *__restrict__ S, float *__restrict__ dn) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const int64_t l = leaf_of[j];
    double v0 = PN[3 * j], v1 = PN[3 * j + 1], v2 = PN[3 * j + 2];
    const double a = pts[j].a;
    for (int c = 0; c < C; ++c) {
        const float mu = BF16 ? __uint_as_float((uint32_t)((const uint16_t *)attr)[j * as + c] << 16)
                              : ((const float *)attr)[j * as + c];
        const double am = a * (double)mu;
        const double *Sl = S + (l * C + c) * 3;
        v0 += am * Sl[0];
        v1 += am * Sl[1];
        v2 += am * Sl[2];
    }
    const int64_t o = (int64_t)perm[j] * 3;
    dn[o] = (float)v0;
    dn[o + 1] = (float)v1;
    dn[o + 2] = (float)v2;
}

__global__ void k_copy_f64(const double *__restrict__ src, double *__restrict__ dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = src[0];
}

// new normals: A n of every point record (sorted order), from caller order
__global__ void k_set_normals(const float *__restrict__ n, const uint32_t *__restrict__ perm, int64_t M,
                              PointRec *__restrict__ pts, float *__restrict__ nrm) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const int64_t i = perm[j];
    const float a = pts[j].a;
    pts[j].anx = mul_rn(a, n[3 * i]);
    pts[j].any = mul_rn(a, n[3 * i + 1]);
    pts[j].anz = mul_rn(a, n[3 * i + 2]);
    nrm[3 * j] = n[3 * i];
    nrm[3 * j + 1] = n[3 * i + 1];
    nrm[3 * j + 2] = n[3 * i + 2];
}


// ---------------------------------------------------------------------------
// adjoint stage 2 (eq. farfield_features_gradient): running sum of the node
// accumulators from the root to each leaf, then each point adds
// A_m n_m . (sum over its ancestors) to its own near-field accumulator.
// ---------------------------------------------------------------------------
__global__ void k_leaf_sums(int64_t N, int64_t W, const NodeRec *__restrict__ nodes,
                            const int32_t *__restrict__ parent, const double *__restrict__ G,
                            double *__restrict__ S) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N * W) return;  // W accumulators per node
    const int64_t t = i / W;
    const int64_t k = i - t * W;
    if (!(nodes[t].meta & kLeafFlag)) return;
    double sum = 0.0;
    for (int64_t a = t; a >= 0; a = parent[a]) sum += G[a * W + k];
    S[t * W + k] = sum;
}

// the same sums written over the leaf's own node accumulators (the leaf entry
// is read before it is overwritten; internal entries are only read)
__global__ void k_leaf_sums_inplace(int64_t N, int64_t W, const NodeRec *__restrict__ nodes,
                                    const int32_t *__restrict__ parent, double *G) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N * W) return;
    const int64_t t = i / W;
    const int64_t k = i - t * W;
    if (!(nodes[t].meta & kLeafFlag)) return;
    double sum = G[t * W + k];
    for (int64_t a = parent[t]; a >= 0; a = parent[a]) sum += G[a * W + k];
    G[t * W + k] = sum;
}

// dL/dmu_mc = P_mc + A_m n_m . S_lc (dipole) or P_mc + A_m S_lc (monopole)
template <bool MONO>
__global__ void k_points_out(int64_t M, int C, const int32_t *__restrict__ leaf_of,
                             const uint32_t *__restrict__ perm, const PointRec *__restrict__ pts,
                             const double *__restrict__ P, const double *__restrict__ S,
                             float *__restrict__ dattrs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * C) return;
    const int64_t j = i / C;
    const int c = (int)(i - j * C);
    const int64_t l = leaf_of[j];
    double v;
    if constexpr (MONO) {
        v = P[j * C + c] + (double)pts[j].a * S[l * C + c];
    } else {
        const double *Sl = S + (l * C + c) * 3;
        v = P[j * C + c] + (double)pts[j].anx * Sl[0] + (double)pts[j].any * Sl[1] + (double)pts[j].anz * Sl[2];
    }
    dattrs[(int64_t)perm[j] * C + c] = (float)v;
}

// ---------------------------------------------------------------------------
// canonical export
// ---------------------------------------------------------------------------
__global__ void k_export_nodes(int64_t N, const int32_t *__restrict__ lvl, const int32_t *__restrict__ parent,
                               const int32_t *__restrict__ first_child, const int32_t *__restrict__ nchild,
                               const int32_t *__restrict__ ptb, const int32_t *__restrict__ ptc,
                               const NodeRec *__restrict__ nodes, int32_t *__restrict__ out_nodes,
                               float *__restrict__ out_geom) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    if (out_nodes) {
        int32_t *o = out_nodes + 6 * t;
        o[0] = lvl[t];
        o[1] = parent[t];
        o[2] = first_child[t];
        o[3] = nchild[t];
        o[4] = ptb[t];
        o[5] = ptc[t];
    }
    if (out_geom) {
        out_geom[4 * t] = nodes[t].cx;
        out_geom[4 * t + 1] = nodes[t].cy;
        out_geom[4 * t + 2] = nodes[t].cz;
        out_geom[4 * t + 3] = nodes[t].r2;
    }
}

template <bool BF16>
__global__ void k_export_moments(int64_t N, int C, int kw, int ms, int64_t nhi, const void *__restrict__ mom,
                                 float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w3 = 3 * (int64_t)C;
    if (i >= N * w3) return;
    const int64_t t = i / w3;
    const int64_t k = i - t * w3;  // channel k / 3, component k % 3
    if (kw == 1 && k % 3 != 0) {   // monopole: scalar charge in component 0
        out[i] = 0.0f;
        return;
    }
    const int64_t e = (kw == 1 ? k / 3 : k);
    if (BF16 && t >= nhi) out[i] = __uint_as_float((uint32_t)((const uint16_t *)mom)[(t + 2 * nhi) * ms + e] << 16);
    else out[i] = ((const float *)mom)[t * ms + e];
}


// channel blocks: 8s, then a 4, then the remainder
inline int next_block(int rem) { return rem >= 8 ? 8 : (rem >= 4 ? 4 : rem); }

// queries per lane: 1, 2 or 4; capped so per-lane accumulators stay in registers
inline int clamp_packet(int k, int cb, bool grad) {
    int cap = grad ? (cb <= 2 ? 4 : (cb <= 4 ? 2 : 1)) : (cb <= 4 ? 4 : 2);
    k = k >= 4 ? 4 : (k >= 2 ? 2 : 1);
    return k < cap ? k : cap;
}


template <int CB, bool BF, bool GR, int K>
dps_status query_launch(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float b2, KernelParams kp, Sub sb,
                        float *f, float *g, hipStream_t s) {
    const uint32_t lim = walk_limit(t);
    if (t->launch_flags & kFlagPersistentQuery) {
        k_fill_u32<<<1, 64, 0, s>>>(t->ctr, 8, 0u);
        const void *fn = reinterpret_cast<const void *>(&k_query_persistent<CB, BF, GR, K>);
        k_query_persistent<CB, BF, GR, K><<<persistent_grid(fn), kThreads, 0, s>>>(
            t->nodes, t->pts, trav_mom(t), t->attr, t->mom_stride, t->attr_stride, x, Q, qdev, b2, kp, sb.c0, sb.ldo, sb.co,
            lim, t->err, f, g, t->ctr);
    } else {
        const unsigned nb = grid(cdiv(Q, K));
        const bool remap = (t->launch_flags & kFlagXcdQuery) != 0;
        const unsigned gr = remap ? (unsigned)(8 * cdiv(nb, 8)) : nb;
        k_query<CB, BF, GR, K><<<gr, kThreads, 0, s>>>(t->nodes, t->pts, trav_mom(t), t->attr, t->mom_stride,
                                                       t->attr_stride, x, Q, qdev, b2, kp, sb.c0, sb.ldo, sb.co, lim,
                                                       t->err, f, g, remap ? (int)nb : 0);
    }
    return hip_status(hipGetLastError(), "query launch");
}

// zeroes the first min(Qcap, *qdev) rows of f (and g), `row` floats per f row
__global__ void k_zero_rows(float *__restrict__ f, float *__restrict__ g, int64_t Qcap,
                            const int64_t *__restrict__ qdev, int64_t row) {
    DPS_ROWS;
    const int64_t nf = Q * row;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += (int64_t)gridDim.x * blockDim.x) {
        f[i] = 0.0f;
        if (g) {
            g[3 * i] = 0.0f;
            g[3 * i + 1] = 0.0f;
            g[3 * i + 2] = 0.0f;
        }
    }
}

inline int split_shift(int parts) {
    int sh = 0;
    while ((1 << sh) < parts) ++sh;
    return sh;
}

inline dps_status split_grid(int64_t Q, int parts, unsigned &wgs) {
    const int64_t n = cdiv(std::max<int64_t>(Q, 1), 64) * parts;
    const int64_t w = cdiv(n, kThreads / 64);
    if (w > INT32_MAX) {
        set_error("split launch: %lld workgroups exceed the launch grid", (long long)w);
        return DPS_ERR_INVALID;
    }
    wgs = (unsigned)w;
    return DPS_OK;
}

template <int CB, bool BF, bool GR>
dps_status query_split_launch(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float b2, KernelParams kp,
                              Sub sb, float *f, float *g, hipStream_t s) {
    unsigned wgs = 0;
    dps_status st = split_grid(Q, t->split_query, wgs);
    if (st != DPS_OK) return st;
    const Split sp{0u, (uint32_t)t->split_query - 1u, (uint32_t)t->split_cut};
    k_query_split<CB, BF, GR><<<wgs, kThreads, 0, s>>>(t->nodes, t->pts, trav_mom(t), t->attr, t->mom_stride,
                                                       t->attr_stride, x, Q, qdev, b2, kp, sb.c0, sb.ldo, sb.co,
                                                       walk_limit(t), t->err, f, g, sp, split_shift(t->split_query));
    return hip_status(hipGetLastError(), "split query launch");
}

template <int CB, bool BF, bool GR>
dps_status query_k(dps_tree_s *t, int k, const float *x, int64_t Q, const int64_t *qdev, float b2, KernelParams kp, Sub sb,
                   float *f, float *g, hipStream_t s) {
    if (t->split_query > 1) return query_split_launch<CB, BF, GR>(t, x, Q, qdev, b2, kp, sb, f, g, s);
    switch (clamp_packet(k, CB, GR)) {
        case 4:
            if constexpr ((GR && CB <= 2) || (!GR && CB <= 4)) return query_launch<CB, BF, GR, 4>(t, x, Q, qdev, b2, kp, sb, f, g, s);
            [[fallthrough]];
        case 2:
            if constexpr (GR ? CB <= 4 : true) return query_launch<CB, BF, GR, 2>(t, x, Q, qdev, b2, kp, sb, f, g, s);
            [[fallthrough]];
        default:
            return query_launch<CB, BF, GR, 1>(t, x, Q, qdev, b2, kp, sb, f, g, s);
    }
}

template <int CB>
dps_status query_block(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float b2, KernelParams kp, Sub sb,
                       float *f, float *g, hipStream_t s) {
    const bool bf = t->storage == DPS_STORE_BF16;
    const int k = t->packet_query;
    if (bf && g) return query_k<CB, true, true>(t, k, x, Q, qdev, b2, kp, sb, f, g, s);
    if (bf) return query_k<CB, true, false>(t, k, x, Q, qdev, b2, kp, sb, f, g, s);
    if (g) return query_k<CB, false, true>(t, k, x, Q, qdev, b2, kp, sb, f, g, s);
    return query_k<CB, false, false>(t, k, x, Q, qdev, b2, kp, sb, f, g, s);
}

template <int CB, bool BF, bool GR, int K>
dps_status grid_launch(dps_tree_s *t, const GridSpec &gs, int64_t Q, float b2, KernelParams kp, Sub sb, float *f,
                       float *g, hipStream_t s) {
    k_fill_u32<<<1, 64, 0, s>>>(t->ctr, 8, 0u);
    const void *fn = reinterpret_cast<const void *>(&k_query_grid<CB, BF, GR, K>);
    k_query_grid<CB, BF, GR, K><<<persistent_grid(fn), kThreads, 0, s>>>(
        t->nodes, t->pts, trav_mom(t), t->attr, t->mom_stride, t->attr_stride, nullptr, Q, nullptr, b2, kp, sb.c0, sb.ldo,
        sb.co, walk_limit(t), t->err, f, g, gs, t->ctr);
    return hip_status(hipGetLastError(), "grid query launch");
}

template <int CB, bool BF, bool GR>
dps_status grid_k(dps_tree_s *t, const GridSpec &gs, int64_t Q, float b2, KernelParams kp, Sub sb, float *f, float *g,
                  hipStream_t s) {
    switch (clamp_packet(t->packet_query, CB, GR)) {
        case 4:
            if constexpr ((GR && CB <= 2) || (!GR && CB <= 4)) return grid_launch<CB, BF, GR, 4>(t, gs, Q, b2, kp, sb, f, g, s);
            [[fallthrough]];
        case 2:
            if constexpr (GR ? CB <= 4 : true) return grid_launch<CB, BF, GR, 2>(t, gs, Q, b2, kp, sb, f, g, s);
            [[fallthrough]];
        default:
            return grid_launch<CB, BF, GR, 1>(t, gs, Q, b2, kp, sb, f, g, s);
    }
}

template <int CB>
dps_status grid_block(dps_tree_s *t, const GridSpec &gs, int64_t Q, float b2, KernelParams kp, Sub sb, float *f,
                      float *g, hipStream_t s) {
    const bool bf = t->storage == DPS_STORE_BF16;
    if (bf && g) return grid_k<CB, true, true>(t, gs, Q, b2, kp, sb, f, g, s);
    if (bf) return grid_k<CB, true, false>(t, gs, Q, b2, kp, sb, f, g, s);
    if (g) return grid_k<CB, false, true>(t, gs, Q, b2, kp, sb, f, g, s);
    return grid_k<CB, false, false>(t, gs, Q, b2, kp, sb, f, g, s);
}

template <int CB, bool BF, int K, bool DX>
dps_status adjoint_launch(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float b2, KernelParams kp, Sub sb,
                          const float *df, float *dx, int dx_mode, const float *gin, const AccBuffers &ab,
                          hipStream_t s) {
    const uint32_t lim = walk_limit(t);
    if (t->launch_flags & kFlagPersistentAdjoint) {
        k_fill_u32<<<1, 64, 0, s>>>(ab.ctr + 8, 8, 0u);
        const void *fn = reinterpret_cast<const void *>(&k_adjoint_persistent<CB, BF, K, DX>);
        k_adjoint_persistent<CB, BF, K, DX><<<persistent_grid(fn), kThreads, 0, s>>>(
            t->nodes, t->pts, trav_mom(t), t->attr, t->mom_stride, t->attr_stride, x, Q, qdev, b2, kp, sb.c0, sb.ldo, sb.co,
            lim, t->err, t->C, df, ab.G, ab.P, dx, dx_mode, gin, ab.ctr + 8);
    } else {
        const unsigned nb = grid(cdiv(Q, K));
        const bool remap = (t->launch_flags & kFlagXcdAdjoint) != 0;
        const unsigned gr = remap ? (unsigned)(8 * cdiv(nb, 8)) : nb;
        k_adjoint<CB, BF, K, DX><<<gr, kThreads, 0, s>>>(t->nodes, t->pts, trav_mom(t), t->attr, t->mom_stride,
                                                         t->attr_stride, x, Q, qdev, b2, kp, sb.c0, sb.ldo, sb.co, lim,
                                                         t->err, t->C, df, ab.G, ab.P, dx, dx_mode, gin,
                                                         remap ? (int)nb : 0);
    }
    return hip_status(hipGetLastError(), "adjoint launch");
}

// dL/dx in the walk (DX) only when it is wanted and no forward gradients are given
template <int CB, bool BF, int K>
dps_status adjoint_launch_dx(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float b2, KernelParams kp,
                             Sub sb, const float *df, float *dx, int dx_mode, const float *gin, const AccBuffers &ab,
                             hipStream_t s) {
    if (dx_mode != 0 && !gin)
        return adjoint_launch<CB, BF, K, true>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, gin, ab, s);
    return adjoint_launch<CB, BF, K, false>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, gin, ab, s);
}

template <int CB, bool BF>
dps_status adjoint_split_launch(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float b2,
                                KernelParams kp, Sub sb, const float *df, float *dx, int dx_mode, const float *gin,
                                const AccBuffers &ab, hipStream_t s) {
    unsigned wgs = 0;
    dps_status st = split_grid(Q, t->split_adjoint, wgs);
    if (st != DPS_OK) return st;
    const Split sp{0u, (uint32_t)t->split_adjoint - 1u, (uint32_t)t->split_cut};
    k_adjoint_split<CB, BF><<<wgs, kThreads, 0, s>>>(t->nodes, t->pts, trav_mom(t), t->attr, t->mom_stride,
                                                     t->attr_stride, x, Q, qdev, b2, kp, sb.c0, sb.ldo, sb.co,
                                                     walk_limit(t), t->err, t->C, df, ab.G, ab.P, dx, dx_mode, gin,
                                                     sp, split_shift(t->split_adjoint));
    return hip_status(hipGetLastError(), "split adjoint launch");
}

template <int CB>
dps_status adjoint_block(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float b2, KernelParams kp, Sub sb,
                         const float *df, float *dx, int dx_mode, const float *gin, const AccBuffers &ab,
                         hipStream_t s) {
    // the split walk when no dL/dx has to be formed in it
    if (t->split_adjoint > 1 && (dx_mode == 0 || gin)) {
        if (t->storage == DPS_STORE_BF16)
            return adjoint_split_launch<CB, true>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, gin, ab, s);
        return adjoint_split_launch<CB, false>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, gin, ab, s);
    }
    const int k = clamp_packet(t->packet_adjoint, CB, false);
    if (t->storage == DPS_STORE_BF16) {
        if (k == 4) { if constexpr (CB <= 4) return adjoint_launch_dx<CB, true, 4>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, gin, ab, s); }
        if (k >= 2) return adjoint_launch_dx<CB, true, 2>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, gin, ab, s);
        return adjoint_launch_dx<CB, true, 1>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, gin, ab, s);
    }
    if (k == 4) { if constexpr (CB <= 4) return adjoint_launch_dx<CB, false, 4>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, gin, ab, s); }
    if (k >= 2) return adjoint_launch_dx<CB, false, 2>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, gin, ab, s);
    return adjoint_launch_dx<CB, false, 1>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, gin, ab, s);
}

template <int CB, bool BF, int K, bool DF, bool EXT>
dps_status adjoint_g_launch(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float b2, KernelParams kp,
                            Sub sb, const float *df, const float *dg, float *dx, int dx_mode, double *pn,
                            double *eacc, hipStream_t s) {
    const uint32_t lim = walk_limit(t);
    if (t->launch_flags & kFlagPersistentAdjoint) {
        k_fill_u32<<<1, 64, 0, s>>>(t->ctr + 8, 8, 0u);
        const void *fn = reinterpret_cast<const void *>(&k_adjoint_g_persistent<CB, BF, K, DF, EXT>);
        k_adjoint_g_persistent<CB, BF, K, DF, EXT><<<persistent_grid(fn), kThreads, 0, s>>>(
            t->nodes, t->pts, trav_mom(t), t->attr, t->mom_stride, t->attr_stride, x, Q, qdev, b2, kp, sb.c0, sb.ldo, sb.co,
            lim, t->err, t->C, df, dg, t->G, t->P, dx, dx_mode, pn, eacc, t->ctr + 8);
    } else {
        const unsigned nb = grid(cdiv(Q, K));
        const bool remap = (t->launch_flags & kFlagXcdAdjoint) != 0;
        const unsigned gr = remap ? (unsigned)(8 * cdiv(nb, 8)) : nb;
        k_adjoint_g<CB, BF, K, DF, EXT><<<gr, kThreads, 0, s>>>(t->nodes, t->pts, trav_mom(t), t->attr, t->mom_stride,
                                                                t->attr_stride, x, Q, qdev, b2, kp, sb.c0, sb.ldo,
                                                                sb.co, lim, t->err, t->C, df, dg, t->G, t->P, dx,
                                                                dx_mode, pn, eacc, remap ? (int)nb : 0);
    }
    return hip_status(hipGetLastError(), "adjoint launch");
}

// queries per lane of the gradient-cotangent adjoint: 2 up to 2 channels
// per block, else 1 (each query carries 3 cotangents per channel)
template <int CB, bool BF, bool DF, bool EXT>
dps_status adjoint_g_k(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float b2, KernelParams kp, Sub sb,
                       const float *df, const float *dg, float *dx, int dx_mode, double *pn, double *eacc,
                       hipStream_t s) {
    if constexpr (CB <= 2) {
        if (t->packet_adjoint >= 2)
            return adjoint_g_launch<CB, BF, 2, DF, EXT>(t, x, Q, qdev, b2, kp, sb, df, dg, dx, dx_mode, pn, eacc, s);
    }
    return adjoint_g_launch<CB, BF, 1, DF, EXT>(t, x, Q, qdev, b2, kp, sb, df, dg, dx, dx_mode, pn, eacc, s);
}

template <int CB, bool EXT>
dps_status adjoint_g_block(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float b2, KernelParams kp,
                           Sub sb, const float *df, const float *dg, float *dx, int dx_mode, double *pn,
                           double *eacc, hipStream_t s) {
    const bool bf = t->storage == DPS_STORE_BF16;
    if (bf && df) return adjoint_g_k<CB, true, true, EXT>(t, x, Q, qdev, b2, kp, sb, df, dg, dx, dx_mode, pn, eacc, s);
    if (bf) return adjoint_g_k<CB, true, false, EXT>(t, x, Q, qdev, b2, kp, sb, df, dg, dx, dx_mode, pn, eacc, s);
    if (df) return adjoint_g_k<CB, false, true, EXT>(t, x, Q, qdev, b2, kp, sb, df, dg, dx, dx_mode, pn, eacc, s);
    return adjoint_g_k<CB, false, false, EXT>(t, x, Q, qdev, b2, kp, sb, df, dg, dx, dx_mode, pn, eacc, s);
}

template <int CB>
dps_status adjoint_g_block_any(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float b2,
                               KernelParams kp, Sub sb, const float *df, const float *dg, float *dx, int dx_mode,
                               double *pn, double *eacc, hipStream_t s) {
    if (pn || eacc) return adjoint_g_block<CB, true>(t, x, Q, qdev, b2, kp, sb, df, dg, dx, dx_mode, pn, eacc, s);
    return adjoint_g_block<CB, false>(t, x, Q, qdev, b2, kp, sb, df, dg, dx, dx_mode, nullptr, nullptr, s);
}

}  // namespace

dps_status launch_query(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float beta, float eps,
                        int cbegin, int nc, float *f, float *g, hipStream_t s) {
    if (t->kernel == DPS_KERNEL_MONOPOLE) return launch_query_mono(t, x, Q, qdev, beta, eps, cbegin, nc, f, g, s);
    const float b2 = mul_rn(beta, beta);
    const KernelParams kp = tree_kernel_params(t, eps);
    if (t->split_query > 1) {  // the parts add into zeroed rows
        k_zero_rows<<<std::min<unsigned>(grid(Q * nc), 4096u), kThreads, 0, s>>>(f, g, Q, qdev, nc);
        dps_status st = hip_status(hipGetLastError(), "split query zero fill");
        if (st != DPS_OK) return st;
    }
    for (int c0 = cbegin; c0 < cbegin + nc;) {
        const int cb = next_block(cbegin + nc - c0);
        const Sub sb{c0, nc, c0 - cbegin};
        dps_status st;
        switch (cb) {
            case 8: st = query_block<8>(t, x, Q, qdev, b2, kp, sb, f, g, s); break;
            case 4: st = query_block<4>(t, x, Q, qdev, b2, kp, sb, f, g, s); break;
            case 3: st = query_block<3>(t, x, Q, qdev, b2, kp, sb, f, g, s); break;
            case 2: st = query_block<2>(t, x, Q, qdev, b2, kp, sb, f, g, s); break;
            default: st = query_block<1>(t, x, Q, qdev, b2, kp, sb, f, g, s); break;
        }
        if (st != DPS_OK) return st;
        c0 += cb;
    }
    return DPS_OK;
}

dps_status launch_counts(dps_tree_s *t, const float *x, int64_t Q, float beta, int32_t *counts,
                         hipStream_t s) {
    k_counts<<<grid(Q), kThreads, 0, s>>>(t->nodes, x, Q, mul_rn(beta, beta), counts, walk_limit(t), t->err);
    return hip_status(hipGetLastError(), "counts launch");
}

dps_status launch_adjoint(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float beta, float eps,
                          int cbegin, int nc, const float *df, float *dx, const float *gin, hipStream_t s,
                          const AccBuffers *abp) {
    if (t->kernel == DPS_KERNEL_MONOPOLE) return launch_adjoint_mono(t, x, Q, qdev, beta, eps, cbegin, nc, df, dx, s);
    const AccBuffers ab = abp ? *abp : tree_buffers(t);
    const float b2 = mul_rn(beta, beta);
    const KernelParams kp = tree_kernel_params(t, eps);
    for (int c0 = cbegin; c0 < cbegin + nc;) {
        const int cb = next_block(cbegin + nc - c0);
        const int dx_mode = dx ? (c0 == cbegin ? 1 : 2) : 0;
        const Sub sb{c0, nc, c0 - cbegin};
        dps_status st;
        switch (cb) {
            case 8: st = adjoint_block<8>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, gin, ab, s); break;
            case 4: st = adjoint_block<4>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, gin, ab, s); break;
            case 3: st = adjoint_block<3>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, gin, ab, s); break;
            case 2: st = adjoint_block<2>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, gin, ab, s); break;
            default: st = adjoint_block<1>(t, x, Q, qdev, b2, kp, sb, df, dx, dx_mode, gin, ab, s); break;
        }
        if (st != DPS_OK) return st;
        c0 += cb;
    }
    return DPS_OK;
}

dps_status launch_zero(dps_tree_s *t, hipStream_t s) {
    const int64_t ng = t->N * t->kw * t->C, np = t->M * t->C;
    k_fill_f64<<<(unsigned)std::min<int64_t>(cdiv(ng, kThreads), 4096), kThreads, 0, s>>>(t->G, ng);
    dps_status st = hip_status(hipGetLastError(), "zero node accumulators");
    if (st != DPS_OK) return st;
    k_fill_f64<<<(unsigned)std::min<int64_t>(cdiv(np, kThreads), 4096), kThreads, 0, s>>>(t->P, np);
    st = hip_status(hipGetLastError(), "zero point accumulators");
    if (st != DPS_OK) return st;
    k_fill_f64<<<(unsigned)std::min<int64_t>(cdiv(t->M * 3, kThreads), 4096), kThreads, 0, s>>>(t->PN, t->M * 3);
    st = hip_status(hipGetLastError(), "zero normal accumulators");
    if (st != DPS_OK) return st;
    k_fill_f64<<<1, 64, 0, s>>>(t->EACC, 1);
    return hip_status(hipGetLastError(), "zero eps accumulator");
}

dps_status launch_zero_acc(dps_tree_s *t, const AccBuffers &ab, hipStream_t s) {
    const int64_t ng = t->N * t->kw * t->C, np = t->M * t->C;
    k_fill_f64<<<(unsigned)std::min<int64_t>(cdiv(ng, kThreads), 4096), kThreads, 0, s>>>(ab.G, ng);
    dps_status st = hip_status(hipGetLastError(), "zero node accumulators");
    if (st != DPS_OK) return st;
    k_fill_f64<<<(unsigned)std::min<int64_t>(cdiv(np, kThreads), 4096), kThreads, 0, s>>>(ab.P, np);
    return hip_status(hipGetLastError(), "zero point accumulators");
}

dps_status launch_finalize_acc(dps_tree_s *t, float *dattrs, const AccBuffers &ab, hipStream_t s) {
    const int64_t w = (int64_t)t->kw * t->C;
    if (ab.S == ab.G) k_leaf_sums_inplace<<<grid(t->N * w), kThreads, 0, s>>>(t->N, w, t->nodes, t->parent, ab.G);
    else k_leaf_sums<<<grid(t->N * w), kThreads, 0, s>>>(t->N, w, t->nodes, t->parent, ab.G, ab.S);
    dps_status st = hip_status(hipGetLastError(), "leaf sums");
    if (st != DPS_OK) return st;
    if (t->kernel == DPS_KERNEL_MONOPOLE)
        k_points_out<true><<<grid(t->M * t->C), kThreads, 0, s>>>(t->M, t->C, t->leaf_of, t->perm, t->pts, ab.P,
                                                                  ab.S, dattrs);
    else
        k_points_out<false><<<grid(t->M * t->C), kThreads, 0, s>>>(t->M, t->C, t->leaf_of, t->perm, t->pts, ab.P,
                                                                   ab.S, dattrs);
    return hip_status(hipGetLastError(), "point gradients");
}

dps_status launch_finalize(dps_tree_s *t, float *dattrs, hipStream_t s) {
    return launch_finalize_ext(t, dattrs, nullptr, nullptr, s);
}

dps_status launch_export(dps_tree_s *t, int32_t *nodes, float *geom, float *moments, hipStream_t s) {
    if (nodes || geom) {
        k_export_nodes<<<grid(t->N), kThreads, 0, s>>>(t->N, t->level, t->parent, t->first_child, t->nchild,
                                                       t->ptb, t->ptc, t->nodes, nodes, geom);
        dps_status st = hip_status(hipGetLastError(), "export nodes");
        if (st != DPS_OK) return st;
    }
    if (moments) {
        if (t->storage == DPS_STORE_BF16)
            k_export_moments<true><<<grid(t->N * 3 * t->C), kThreads, 0, s>>>(t->N, t->C, t->kw, t->mom_stride,
                                                                                t->n_top, t->mom, moments);
        else
            k_export_moments<false><<<grid(t->N * 3 * t->C), kThreads, 0, s>>>(t->N, t->C, t->kw, t->mom_stride, 0,
                                                                                 t->mom, moments);
        dps_status st = hip_status(hipGetLastError(), "export moments");
        if (st != DPS_OK) return st;
    }
    return DPS_OK;
}

dps_status launch_adjoint_g(dps_tree_s *t, const float *x, int64_t Q, const int64_t *qdev, float beta, float eps,
                            int cbegin, int nc, const float *df, const float *dg, int want, float *dx,
                            hipStream_t s) {
    const float b2 = mul_rn(beta, beta);
    const KernelParams kp = tree_kernel_params(t, eps);
    for (int c0 = cbegin; c0 < cbegin + nc;) {
        // blocks of at most 4 channels: each carries 4 floats per channel and query
        const int rem = cbegin + nc - c0;
        const int cb = rem >= 4 ? 4 : rem;
        const int dx_mode = dx ? (c0 == cbegin ? 1 : 2) : 0;
        double *pn = (want & 1) ? t->PN : nullptr;
        double *eacc = (want & 2) ? t->EACC : nullptr;
        const Sub sb{c0, nc, c0 - cbegin};
        dps_status st;
        switch (cb) {
            case 4: st = adjoint_g_block_any<4>(t, x, Q, qdev, b2, kp, sb, df, dg, dx, dx_mode, pn, eacc, s); break;
            case 3: st = adjoint_g_block_any<3>(t, x, Q, qdev, b2, kp, sb, df, dg, dx, dx_mode, pn, eacc, s); break;
            case 2: st = adjoint_g_block_any<2>(t, x, Q, qdev, b2, kp, sb, df, dg, dx, dx_mode, pn, eacc, s); break;
            default: st = adjoint_g_block_any<1>(t, x, Q, qdev, b2, kp, sb, df, dg, dx, dx_mode, pn, eacc, s); break;
        }
        if (st != DPS_OK) return st;
        c0 += cb;
    }
    return DPS_OK;
}

dps_status launch_finalize_ext(dps_tree_s *t, float *dattrs, float *dnormals, double *deps, hipStream_t s) {
    if (dattrs || dnormals) {
        const int64_t w = (int64_t)t->kw * t->C;
        k_leaf_sums<<<grid(t->N * w), kThreads, 0, s>>>(t->N, w, t->nodes, t->parent, t->G, t->S);
        dps_status st = hip_status(hipGetLastError(), "leaf sums");
        if (st != DPS_OK) return st;
    }
    if (dattrs) {
        if (t->kernel == DPS_KERNEL_MONOPOLE)
            k_points_out<true><<<grid(t->M * t->C), kThreads, 0, s>>>(t->M, t->C, t->leaf_of, t->perm, t->pts, t->P,
                                                                      t->S, dattrs);
        else
            k_points_out<false><<<grid(t->M * t->C), kThreads, 0, s>>>(t->M, t->C, t->leaf_of, t->perm, t->pts,
                                                                       t->P, t->S, dattrs);
        dps_status st = hip_status(hipGetLastError(), "point gradients");
        if (st != DPS_OK) return st;
    }
    if (dnormals) {
        if (t->storage == DPS_STORE_BF16)
            k_normals_out<true><<<grid(t->M), kThreads, 0, s>>>(t->M, t->C, t->attr_stride, t->leaf_of, t->perm,
                                                                t->pts, t->attr, t->PN, t->S, dnormals);
        else
            k_normals_out<false><<<grid(t->M), kThreads, 0, s>>>(t->M, t->C, t->attr_stride, t->leaf_of, t->perm,
                                                                 t->pts, t->attr, t->PN, t->S, dnormals);
        dps_status st = hip_status(hipGetLastError(), "normal gradients");
        if (st != DPS_OK) return st;
    }
    if (deps) {
        k_copy_f64<<<1, 64, 0, s>>>(t->EACC, deps);
        dps_status st = hip_status(hipGetLastError(), "eps gradient");
        if (st != DPS_OK) return st;
    }
    return DPS_OK;
}

dps_status launch_set_normals(dps_tree_s *t, const float *n, hipStream_t s) {
    k_set_normals<<<grid(t->M), kThreads, 0, s>>>(n, t->perm, t->M, t->pts, t->nrm);
    return hip_status(hipGetLastError(), "set normals");
}

dps_status launch_query_grid(dps_tree_s *t, const float origin[3], const float spacing[3], const int64_t dims[3],
                             float beta, float eps, int cbegin, int nc, float *f, float *g, hipStream_t s) {
    GridSpec gs;
    for (int a = 0; a < 3; ++a) {
        gs.o[a] = origin[a];
        gs.h[a] = spacing[a];
        gs.n[a] = dims[a];
        gs.nb[a] = cdiv(dims[a], 4);
    }
    const int64_t Q = gs.nb[0] * gs.nb[1] * gs.nb[2] * 64;
    const float b2 = mul_rn(beta, beta);
    const KernelParams kp = tree_kernel_params(t, eps);
    for (int c0 = cbegin; c0 < cbegin + nc;) {
        const int cb = next_block(cbegin + nc - c0);
        const Sub sb{c0, nc, c0 - cbegin};
        dps_status st;
        switch (cb) {
            case 8: st = grid_block<8>(t, gs, Q, b2, kp, sb, f, g, s); break;
            case 4: st = grid_block<4>(t, gs, Q, b2, kp, sb, f, g, s); break;
            case 3: st = grid_block<3>(t, gs, Q, b2, kp, sb, f, g, s); break;
            case 2: st = grid_block<2>(t, gs, Q, b2, kp, sb, f, g, s); break;
            default: st = grid_block<1>(t, gs, Q, b2, kp, sb, f, g, s); break;
        }
        if (st != DPS_OK) return st;
        c0 += cb;
    }
    return DPS_OK;
}

}  // namespace dps
