// dps_walk.h -- the packet walk of the dipole sums for callers that produce
// their query points in registers (the ray march): K points per lane, values
// (and gradients) of CB channels accumulated in registers.
//
// Algorithm 1 (PrimalQuery) for every active point, as the union walk of the
// wavefront: the current node is wave-uniform, point i visits it iff its
// level is at most depth[i] (the walk state of the traversal kernels), the far
// test comes before the leaf test and bucket leaves sum their points exactly.
// The next node's record and moments are fetched before the current node's
// far-field and leaf work (software pipelining).  Points with depth[i] = -1
// take no part; f and g are accumulated into (the caller zeroes them).  The
// arithmetic per point is that of the point-query kernels, with its dot
// products written as explicit fused chains: left to contraction, the
// compiler may fuse a different product of a sum of products in each kernel,
// and every caller of this walk (marches, the values pass, one-channel value
// queries) is meant to produce the same bits.  The terms are predicated
// instead of branched per point (see radial_k): with one channel a node carries so little arithmetic
// that the exec-mask updates of per-point branches made the scalar unit the
// busier pipe.  The point-query kernels keep their own loop inline (compiled
// through this function their register allocation grew from 72 to 92 VGPRs).
#pragma once

#include "dps_trav_common.h"

namespace dps {
namespace {

// radial() for the K points of a lane at once, for the points with take[i]:
// the plain factors 1/(4 pi r^3), 3/(4 pi r^5) without branches, and radial()
// itself (same values) only when some point of the wavefront lies in the
// regularised range, which far nodes seldom are.  Returns per point whether
// the term exists (radial's convention: not for r = 0 without eps).
template <int K>
__device__ __forceinline__ void radial_k(const float (&r2)[K], const bool (&take)[K], const KernelParams &kp,
                                         float (&kap)[K], float (&lam)[K], bool (&on)[K]) {
    bool slow = false;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const float x = take[i] ? r2[i] : kHugeR2;
        const float ir = __builtin_amdgcn_rsqf(x);
        const float ir2 = ir * ir;
        kap[i] = kInv4Pi * ir * ir2;
        lam[i] = 3.0f * kap[i] * ir2;
        on[i] = take[i] && (kp.eps != 0.0f || x > 0.0f);
        slow |= take[i] && x < kp.zone_r2;
    }
    if (__ballot(slow) != 0) {
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (take[i]) radial(r2[i], kp, kap[i], lam[i]);
    }
}

template <int CB, bool BF16, bool GRAD, int K>
__device__ __forceinline__ void dipole_walk(const float (&px)[K], const float (&py)[K], const float (&pz)[K],
                                            int32_t (&depth)[K], float (&f)[K][CB], float (&g)[K][CB][3],
                                            const NodeRec *__restrict__ nodes, const PointRec *__restrict__ pts,
                                            const void *__restrict__ mom, const void *__restrict__ attr, int ms,
                                            int as, float b2, KernelParams kp, int c0, uint32_t limit,
                                            uint32_t *__restrict__ err) {
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
        const uint32_t next = any_open ? nd.down : nd.escape;
        const uint32_t pf = next;  // kEnd is the root: a valid record
        const NodeRec nn = nodes[pf];
        float Dn[3 * CB];
        load_moments<CB, BF16>(mom, ms, pf, c0, Dn, kp.nhi);
        if (any_far) {
            refine_moments<CB, BF16>(mom, ms, t, c0, D, kp.nhi);
            // predicated rather than branched per point: a lane's terms are
            // computed under the wavefront's mask either way, and selects
            // spare the scalar unit the exec-mask updates of a branch.  A
            // point that is not far sees a huge distance, so it takes no
            // part in the regularised branch of radial().
            float kap[K], lam[K];
            bool on[K];
            radial_k<K>(s, far, kp, kap, lam, on);
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const float dx = nd.cx - px[i], dy = nd.cy - py[i], dz = nd.cz - pz[i];
#pragma unroll
                for (int c = 0; c < CB; ++c) {
                    const float sd = fmaf(D[3 * c + 2], dz, fmaf(D[3 * c + 1], dy, D[3 * c] * dx));
                    f[i][c] = far[i] ? fmaf(kap[i], sd, f[i][c]) : f[i][c];
                    if (GRAD) {
                        const float ls = lam[i] * sd;
                        const float g0 = fmaf(-kap[i], D[3 * c], fmaf(ls, dx, g[i][c][0]));
                        const float g1 = fmaf(-kap[i], D[3 * c + 1], fmaf(ls, dy, g[i][c][1]));
                        const float g2 = fmaf(-kap[i], D[3 * c + 2], fmaf(ls, dz, g[i][c][2]));
                        g[i][c][0] = far[i] ? g0 : g[i][c][0];
                        g[i][c][1] = far[i] ? g1 : g[i][c][1];
                        g[i][c][2] = far[i] ? g2 : g[i][c][2];
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
                    float dx[K], dy[K], dz[K], r2[K], kap[K], lam[K];
                    bool on[K];
#pragma unroll
                    for (int i = 0; i < K; ++i) {
                        dx[i] = pr.x - px[i];
                        dy[i] = pr.y - py[i];
                        dz[i] = pr.z - pz[i];
                        r2[i] = fmaf(dz[i], dz[i], fmaf(dy[i], dy[i], dx[i] * dx[i]));
                    }
                    radial_k<K>(r2, open, kp, kap, lam, on);
#pragma unroll
                    for (int i = 0; i < K; ++i) {  // predicated as the far terms
                        const float sa = fmaf(pr.anz, dz[i], fmaf(pr.any, dy[i], pr.anx * dx[i]));
                        const float ks = kap[i] * sa;
                        const float ls = lam[i] * sa;
                        const float G0 = fmaf(ls, dx[i], -kap[i] * pr.anx);
                        const float G1 = fmaf(ls, dy[i], -kap[i] * pr.any);
                        const float G2 = fmaf(ls, dz[i], -kap[i] * pr.anz);
#pragma unroll
                        for (int c = 0; c < CB; ++c) {
                            f[i][c] = on[i] ? fmaf(mu[c], ks, f[i][c]) : f[i][c];
                            if (GRAD) {
                                const float g0 = fmaf(mu[c], G0, g[i][c][0]);
                                const float g1 = fmaf(mu[c], G1, g[i][c][1]);
                                const float g2 = fmaf(mu[c], G2, g[i][c][2]);
                                g[i][c][0] = on[i] ? g0 : g[i][c][0];
                                g[i][c][1] = on[i] ? g1 : g[i][c][1];
                                g[i][c][2] = on[i] ? g2 : g[i][c][2];
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

// Distance from each lane's point to the nearest point of the cloud, for the
// lanes with `on` (others return `bound`): a union walk that opens a node
// while its bounding sphere may hold a point nearer than the lane's best so
// far, starting from `bound` (a distance the nearest point is known to lie
// within, or infinity).  The sphere radius gets a relative slack of 1e-4 so
// that rounding cannot prune the node holding the nearest point; where no
// point lies within `bound` the result is `bound`.
__device__ __forceinline__ float nearest_walk(float px, float py, float pz, bool on, float bound,
                                              const NodeRec *__restrict__ nodes, const PointRec *__restrict__ pts,
                                              uint32_t limit, uint32_t *__restrict__ err) {
    float best2 = bound * bound;
    float best = bound;
    int32_t depth = on ? 0 : -1;
    NodeRec nd = nodes[0];
    uint32_t steps = 0;
    for (;;) {
        if (++steps > limit) {  // a well-formed tree is walked in at most N steps
            if ((threadIdx.x & 63) == 0) atomicOr(err, 1u);
            break;
        }
        const uint32_t lvl = nd.meta & 0xffu;
        const bool leaf = (nd.meta & kLeafFlag) != 0;
        const bool in = visits(depth, lvl);
        const float s = dist2_rn(nd.cx, nd.cy, nd.cz, px, py, pz);
        const float reach = (best + __builtin_sqrtf(nd.r2)) * 1.0001f;
        const bool beyond = !(s < reach * reach);
        const bool open = in && !beyond;
        WaveMasks wm;
        wm.add(in, beyond);
        const bool any_open = wm.open != 0;
        const uint32_t next = any_open ? nd.down : nd.escape;
        const NodeRec nn = nodes[next];  // kEnd is the root: a valid record
        if (any_open) {
            if (!leaf) {
                depth = descend(depth, lvl, open);
            } else {
                const uint32_t je = nd.first + node_count(nd);
                for (uint32_t j = nd.first; j < je; ++j) {
                    const PointRec pr = pts[j];
                    const float dx = pr.x - px, dy = pr.y - py, dz = pr.z - pz;
                    const float d2 = dot3(dx, dy, dz, dx, dy, dz);
                    best2 = open ? fminf(best2, d2) : best2;
                }
                best = __builtin_sqrtf(best2);
            }
        }
        if (next == kEnd) break;
        nd = nn;
    }
    return best;
}

}  // namespace
}  // namespace dps
