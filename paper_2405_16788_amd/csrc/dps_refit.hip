// dps_refit.hip -- node moments from the current attributes (Sec. 6.1,
// eq. farfield_dipole_features: mu_t = (1/A_t) sum A_m n_m mu_m; the tree stores
// the dipole D_t = A_t mu_t = sum A_m mu_m n_m per channel, or for the monopole
// kernel of Sec. 7.1 the scalar charge sum A_m mu_m), refreshed whenever the
// attributes change (Sec. 6.3).
//
// Bottom-up, one launch per level, every node summing its points (leaves, in
// Morton order) or its children (internal nodes, in child order): deterministic.
// Accumulation is FP32, except nodes of depth <= 3 in trees of >= 4,194,304
// points, which accumulate in FP64.  The stored copy is FP32 or BF16 (RNE); the
// working sums are kept separately so rounding never compounds up the tree.
#include <algorithm>

#include "dps_tree.h"

namespace dps {

namespace {

constexpr int kThreads = 256;

inline unsigned grid(int64_t n) { return (unsigned)std::max<int64_t>(1, cdiv(n, kThreads)); }

template <bool BF16>
__global__ void k_gather_attrs(const float *__restrict__ attrs, const uint32_t *__restrict__ perm,
                               int64_t M, int C, int as, void *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * as) return;
    const int64_t j = i / as;
    const int c = (int)(i - j * as);
    const float v = c < C ? attrs[(int64_t)perm[j] * C + c] : 0.0f;
    if (BF16) ((uint16_t *)out)[i] = f32_to_bf16(v);
    else ((float *)out)[i] = v;
}

// one thread per (node, channel) of the level [nb, ne).  KW = 3: the dipole
// D_t = sum A_m mu_m n_m; KW = 1: the monopole charge Q_t = sum A_m mu_m.
template <bool BF16, int KW>
__global__ void k_moments(int64_t nb, int64_t ne, int C, int ms, bool wide, int64_t n_top,
                          const float *__restrict__ attrs, const uint32_t *__restrict__ perm,
                          const PointRec *__restrict__ pts, const int32_t *__restrict__ first_child,
                          const int32_t *__restrict__ nchild, const int32_t *__restrict__ ptb,
                          const int32_t *__restrict__ ptc, float *__restrict__ momw,
                          double *__restrict__ momw64, void *__restrict__ mom) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (ne - nb) * C) return;
    const int64_t t = nb + i / C;
    const int c = (int)(i % C);
    double out[KW];
    if (nchild[t] == 0) {
        const int64_t jb = ptb[t], je = jb + ptc[t];
        if (wide) {
            double a[KW] = {};
            for (int64_t j = jb; j < je; ++j) {
                const double mu = attrs[(int64_t)perm[j] * C + c];
                if constexpr (KW == 3) {
                    a[0] += mu * (double)pts[j].anx;
                    a[1] += mu * (double)pts[j].any;
                    a[2] += mu * (double)pts[j].anz;
                } else {
                    a[0] += mu * (double)pts[j].a;
                }
            }
            for (int k = 0; k < KW; ++k) out[k] = a[k];
        } else {
            float a[KW] = {};
            for (int64_t j = jb; j < je; ++j) {
                const float mu = attrs[(int64_t)perm[j] * C + c];
                if constexpr (KW == 3) {
                    a[0] += mu * pts[j].anx;
                    a[1] += mu * pts[j].any;
                    a[2] += mu * pts[j].anz;
                } else {
                    a[0] += mu * pts[j].a;
                }
            }
            for (int k = 0; k < KW; ++k) out[k] = a[k];
        }
    } else {
        const int64_t cb = first_child[t], ce = cb + nchild[t];
        if (wide) {
            double a[KW] = {};
            for (int64_t ch = cb; ch < ce; ++ch) {
                const int64_t o = ch * KW * C + KW * c;
                for (int k = 0; k < KW; ++k) a[k] += ch < n_top ? momw64[o + k] : (double)momw[o + k];
            }
            for (int k = 0; k < KW; ++k) out[k] = a[k];
        } else {
            float a[KW] = {};
            for (int64_t ch = cb; ch < ce; ++ch) {
                const int64_t o = ch * KW * C + KW * c;
                for (int k = 0; k < KW; ++k) a[k] += momw[o + k];
            }
            for (int k = 0; k < KW; ++k) out[k] = a[k];
        }
    }
    const int64_t o = t * KW * C + KW * c;
    for (int k = 0; k < KW; ++k) {
        if (wide) momw64[o + k] = out[k];
        momw[o + k] = (float)out[k];
        const int64_t so = t * ms + KW * c + k;
        if (BF16) ((uint16_t *)mom)[so] = f32_to_bf16((float)out[k]);
        else ((float *)mom)[so] = (float)out[k];
    }
    if (BF16 && c == C - 1 && ms > KW * C) ((uint16_t *)mom)[t * ms + KW * C] = 0;
}

template <bool BF16, int KW>
void launch_moments(dps_tree_s *t, int64_t nb, int64_t ne, bool wide, const float *attrs, hipStream_t s) {
    k_moments<BF16, KW><<<grid((ne - nb) * t->C), kThreads, 0, s>>>(nb, ne, t->C, t->mom_stride, wide, t->n_top,
                                                                    attrs, t->perm, t->pts, t->first_child,
                                                                    t->nchild, t->ptb, t->ptc, t->momw, t->momw64,
                                                                    t->mom);
}

}  // namespace

dps_status refit_moments(dps_tree_s *t, const float *attrs, hipStream_t s) {
    const bool bf16 = t->storage == DPS_STORE_BF16;
    const int64_t M = t->M;
    if (bf16) k_gather_attrs<true><<<grid(M * t->attr_stride), kThreads, 0, s>>>(attrs, t->perm, M, t->C, t->attr_stride, t->attr);
    else k_gather_attrs<false><<<grid(M * t->attr_stride), kThreads, 0, s>>>(attrs, t->perm, M, t->C, t->attr_stride, t->attr);
    dps_status st = hip_status(hipGetLastError(), "attribute gather");
    if (st != DPS_OK) return st;
    for (int l = t->depth; l >= 0; --l) {
        const int64_t nb = t->level_start[l], ne = t->level_start[l + 1];
        const bool wide = t->wide_top && l <= kTopLevels;
        const bool mono = t->kernel == DPS_KERNEL_MONOPOLE;
        if (bf16 && mono) launch_moments<true, 1>(t, nb, ne, wide, attrs, s);
        else if (bf16) launch_moments<true, 3>(t, nb, ne, wide, attrs, s);
        else if (mono) launch_moments<false, 1>(t, nb, ne, wide, attrs, s);
        else launch_moments<false, 3>(t, nb, ne, wide, attrs, s);
        st = hip_status(hipGetLastError(), "moment refit");
        if (st != DPS_OK) return st;
    }
    return DPS_OK;
}

}  // namespace dps
