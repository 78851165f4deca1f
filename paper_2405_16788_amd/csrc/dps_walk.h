// dps_walk.h -- the packet walk of the dipole sums for callers that produce
// their query points in registers (the ray march): K points per lane, values
// (and gradients) of CB channels accumulated in registers.
//
// Algorithm 1 (PrimalQuery) for every active point, as the union walk of the
// wavefront: the current node is wave-uniform, bit l of bits[i] means that
// point i opened every ancestor of the current level-l node, the far test
// comes before the leaf test and bucket leaves sum their points exactly.
// The next node's record and moments are fetched before the current node's
// far-field and leaf work (software pipelining).  Points with bits[i] = 0 take
// no part; f and g are accumulated into (the caller zeroes them).  The
// arithmetic per point is that of the point-query kernels, which keep the
// same loop inline (compiled through this function their register
// allocation grew from 72 to 92 VGPRs).
#pragma once

#include "dps_trav_common.h"

namespace dps {
namespace {

template <int CB, bool BF16, bool GRAD, int K>
__device__ __forceinline__ void dipole_walk(const float (&px)[K], const float (&py)[K], const float (&pz)[K],
                                            uint32_t (&bits)[K], float (&f)[K][CB], float (&g)[K][CB][3],
                                            const NodeRec *__restrict__ nodes, const PointRec *__restrict__ pts,
                                            const void *__restrict__ mom, const void *__restrict__ attr, int ms,
                                            int as, float b2, KernelParams kp, int c0, uint32_t limit,
                                            uint32_t *__restrict__ err) {
    uint32_t t = 0;
    NodeRec nd = nodes[0];
    float D[3 * CB];
    load_moments<CB, BF16>(mom, ms, 0, c0, D);
    uint32_t steps = 0;
    for (;;) {
        if (++steps > limit) {  // a well-formed tree is walked in at most N steps
            if ((threadIdx.x & 63) == 0) atomicOr(err, 1u);
            break;
        }
        const uint32_t lvl = nd.meta & 0xffu;
        const bool leaf = (nd.meta & kLeafFlag) != 0;
        const float lim = mul_rn(b2, nd.r2);
        bool far[K], open[K], lane_far = false, lane_open = false;
        float s[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const bool in = (bits[i] >> lvl) & 1u;
            s[i] = dist2_rn(nd.cx, nd.cy, nd.cz, px[i], py[i], pz[i]);
            far[i] = in && (s[i] > lim);
            open[i] = in && !far[i];
            lane_far |= far[i];
            lane_open |= open[i];
        }
        const bool any_far = __ballot(lane_far) != 0;
        const bool any_open = __ballot(lane_open) != 0;
        const uint32_t next = (any_open && !leaf) ? nd.first : nd.escape;
        const uint32_t pf = next == kEnd ? t : next;
        const NodeRec nn = nodes[pf];
        float Dn[3 * CB];
        load_moments<CB, BF16>(mom, ms, pf, c0, Dn);
        if (any_far) {
#pragma unroll
            for (int i = 0; i < K; ++i) {
                if (far[i]) {
                    float kap, lam;
                    radial(s[i], kp, kap, lam);
                    const float dx = nd.cx - px[i], dy = nd.cy - py[i], dz = nd.cz - pz[i];
#pragma unroll
                    for (int c = 0; c < CB; ++c) {
                        const float sd = D[3 * c] * dx + D[3 * c + 1] * dy + D[3 * c + 2] * dz;
                        f[i][c] = fmaf(kap, sd, f[i][c]);
                        if (GRAD) {
                            const float ls = lam * sd;
                            g[i][c][0] = fmaf(-kap, D[3 * c], fmaf(ls, dx, g[i][c][0]));
                            g[i][c][1] = fmaf(-kap, D[3 * c + 1], fmaf(ls, dy, g[i][c][1]));
                            g[i][c][2] = fmaf(-kap, D[3 * c + 2], fmaf(ls, dz, g[i][c][2]));
                        }
                    }
                }
            }
        }
        if (any_open) {
            if (!leaf) {
#pragma unroll
                for (int i = 0; i < K; ++i)
                    bits[i] = (bits[i] & ~(2u << lvl)) | ((uint32_t)open[i] << (lvl + 1));
            } else {
                const uint32_t je = nd.first + nd.count;
                for (uint32_t j = nd.first; j < je; ++j) {
                    const PointRec pr = pts[j];
                    float mu[CB];
                    load_attrs<CB, BF16>(attr, as, j, c0, mu);
#pragma unroll
                    for (int i = 0; i < K; ++i) {
                        if (open[i]) {
                            const float dx = pr.x - px[i], dy = pr.y - py[i], dz = pr.z - pz[i];
                            const float r2 = dx * dx + dy * dy + dz * dz;
                            float kap, lam;
                            if (radial(r2, kp, kap, lam)) {
                                const float sa = pr.anx * dx + pr.any * dy + pr.anz * dz;
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
                }
            }
        }
        if (next == kEnd) break;
        t = next;
        nd = nn;
#pragma unroll
        for (int v = 0; v < 3 * CB; ++v) D[v] = Dn[v];
    }
}

}  // namespace
}  // namespace dps
