// dps_refit.hip -- node moments from the current attributes (Sec. 6.1,
// eq. farfield_dipole_features: mu_t = (1/A_t) sum A_m n_m mu_m; the tree stores
// the dipole D_t = A_t mu_t = sum A_m mu_m n_m per channel, or for the monopole
// kernel of Sec. 7.1 the scalar charge sum A_m mu_m), refreshed whenever the
// attributes change (Sec. 6.3).
//
// Bottom-up, one launch per level, every node summing its points (leaves, in
// Morton order) or its children (internal nodes, in child order): deterministic.
// Accumulation is compensated FP32 (a high and a low part per sum), except
// nodes of depth <= 3 in trees of >= 4,194,304 points, which accumulate in
// FP64.  The stored copy is the working sum rounded once: FP32, or BF16 (RNE)
// with the nodes of depth <= 3 kept in FP32; the working sums are kept
// separately so rounding never compounds up the tree.
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

// Compensated FP32 accumulation: a working sum is a pair (h, l) whose value
// is h + l.  Each addend is itself a pair; two_sum gives the exact rounding
// error of h + a_hi (Knuth), which joins the low part.  Contraction is off so
// that every operation rounds once as written.
__device__ __forceinline__ void acc2(float &h, float &l, float a_hi, float a_lo) {
#pragma clang fp contract(off)
    const float s = h + a_hi;
    const float bp = s - h;
    const float e = (h - (s - bp)) + (a_hi - bp);
    h = s;
    l = l + (e + a_lo);
}

// a * b * c of three FP32 values as hi + lo: a * b = p + pe exactly (FMA
// residual), p * c = hi + its FMA residual exactly; only pe * c rounds (2^-48
// of the product).
__device__ __forceinline__ void prod3(float a, float b, float c, float &hi, float &lo) {
#pragma clang fp contract(off)
    const float p = a * b;
    const float pe = fmaf(a, b, -p);
    hi = p * c;
    lo = fmaf(pe, c, fmaf(p, c, -hi));
}

// one thread per (node, channel) of the level [nb, ne).  KW = 3: the dipole
// D_t = sum A_m mu_m n_m; KW = 1: the monopole charge Q_t = sum A_m mu_m.
// Leaves sum their points' products A_m mu_m n_m (computed from A, mu and the
// unit normal, not from the rounded A n of the point records), internal nodes
// their children's working sums, in a fixed order, compensated in FP32 (or in
// FP64 for the top levels of large trees, `wide`).  The stored value is the
// working sum rounded once to FP32, and with BF16 storage also to BF16 (the
// first nhi nodes keep their FP32 value as well, for the far field).
template <bool BF16, int KW>
__global__ void k_moments(int64_t nb, int64_t ne, int C, int ms, bool wide, int64_t n_top, int64_t nhi,
                          const float *__restrict__ attrs, const uint32_t *__restrict__ perm,
                          const PointRec *__restrict__ pts, const float *__restrict__ nrm,
                          const int32_t *__restrict__ first_child, const int32_t *__restrict__ nchild,
                          const int32_t *__restrict__ ptb, const int32_t *__restrict__ ptc,
                          float *__restrict__ momw, float *__restrict__ momw_lo, double *__restrict__ momw64,
                          void *__restrict__ mom) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (ne - nb) * C) return;
    const int64_t t = nb + i / C;
    const int c = (int)(i % C);
    const int64_t o = t * KW * C + KW * c;
    float hi[KW], lo[KW];
    if (wide) {
        double a[KW] = {};
        if (nchild[t] == 0) {
            const int64_t jb = ptb[t], je = jb + ptc[t];
            for (int64_t j = jb; j < je; ++j) {
                const double am = (double)pts[j].a * (double)attrs[(int64_t)perm[j] * C + c];  // exact
                if constexpr (KW == 3) {
                    for (int k = 0; k < 3; ++k) a[k] += am * (double)nrm[3 * j + k];
                } else {
                    a[0] += am;
                }
            }
        } else {
            const int64_t cb = first_child[t], ce = cb + nchild[t];
            for (int64_t ch = cb; ch < ce; ++ch) {
                const int64_t oc = ch * KW * C + KW * c;
                for (int k = 0; k < KW; ++k)
                    a[k] += ch < n_top ? momw64[oc + k] : (double)momw[oc + k] + (double)momw_lo[oc + k];
            }
        }
        for (int k = 0; k < KW; ++k) {
            momw64[o + k] = a[k];
            hi[k] = (float)a[k];
            lo[k] = (float)(a[k] - (double)hi[k]);
        }
    } else {
        for (int k = 0; k < KW; ++k) hi[k] = lo[k] = 0.0f;
        if (nchild[t] == 0) {
            const int64_t jb = ptb[t], je = jb + ptc[t];
            for (int64_t j = jb; j < je; ++j) {
                const float am = pts[j].a, mu = attrs[(int64_t)perm[j] * C + c];
                if constexpr (KW == 3) {
                    for (int k = 0; k < 3; ++k) {
                        float ph, pl;
                        prod3(am, mu, nrm[3 * j + k], ph, pl);
                        acc2(hi[k], lo[k], ph, pl);
                    }
                } else {
                    const float ph = mul_rn(am, mu);
                    acc2(hi[0], lo[0], ph, fmaf(am, mu, -ph));
                }
            }
        } else {
            const int64_t cb = first_child[t], ce = cb + nchild[t];
            for (int64_t ch = cb; ch < ce; ++ch) {
                const int64_t oc = ch * KW * C + KW * c;
                for (int k = 0; k < KW; ++k) acc2(hi[k], lo[k], momw[oc + k], momw_lo[oc + k]);
            }
        }
    }
    // FP32 storage: row t.  BF16 storage: the bfloat16 row t + 2 nhi of every
    // node, and for the first nhi nodes also the FP32 row t.
    const bool f32row = !BF16 || t < nhi;
    for (int k = 0; k < KW; ++k) {
        momw[o + k] = hi[k];
        momw_lo[o + k] = lo[k];
        float v;
        if (wide) v = (float)momw64[o + k];
        else {
#pragma clang fp contract(off)
            v = hi[k] + lo[k];
        }
        if (f32row) ((float *)mom)[t * ms + KW * c + k] = v;
        if (BF16) ((uint16_t *)mom)[(t + 2 * nhi) * ms + KW * c + k] = f32_to_bf16(v);
    }
    if (c == C - 1 && ms > KW * C) {  // row padding
        if (f32row) ((float *)mom)[t * ms + KW * C] = 0.0f;
        if (BF16) ((uint16_t *)mom)[(t + 2 * nhi) * ms + KW * C] = 0;
    }
}

template <bool BF16, int KW>
void launch_moments(dps_tree_s *t, int64_t nb, int64_t ne, bool wide, const float *attrs, hipStream_t s) {
    k_moments<BF16, KW><<<grid((ne - nb) * t->C), kThreads, 0, s>>>(
        nb, ne, t->C, t->mom_stride, wide, t->n_top, BF16 ? t->n_top : 0, attrs, t->perm, t->pts, t->nrm,
        t->first_child, t->nchild, t->ptb, t->ptc, t->momw, t->momw_lo, t->momw64, t->mom);
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
