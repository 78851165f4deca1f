// dps_internal.h -- device data layout and helpers shared by the libdps kernels.
//
// Layout in HBM (all arrays owned by the tree, Morton order):
//   NodeRec  [N]      32 B: centroid, squared radius, link fields (one 8-dword scalar load)
//   PointRec [M]      32 B: position, A*n, A (one 8-dword scalar load)
//   moments  [N][ms]  node dipoles D_t = sum A_m mu_m n_m, channel-major 3-vectors,
//                     FP32 (ms = 3C), or with BF16 storage (ms = 3C rounded up to
//                     even) FP32 rows of ms floats for the first nhi nodes (levels
//                     <= kTopLevels) followed by a bfloat16 row for every node, node
//                     t at bfloat16 element (t + 2 nhi) * ms
//   attrs    [M][as]  point attributes, FP32 (as = C) or BF16 (as = C rounded up to even)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "dps.h"

namespace dps {

// escape pointer past the last subtree: the root, which no walk returns to,
// so a walk may fetch the record of the node it moves to next without a test
constexpr uint32_t kEnd = 0u;
constexpr uint32_t kLeafFlag = 0x100u;   // NodeRec::meta bit: node is a leaf
constexpr int kCountShift = 16;          // NodeRec::meta bits 16..31: children or points
constexpr int kLevels = DPS_LEVELS;      // 21 levels below the root
constexpr int kTopLevels = 3;            // "top-level" nodes: depth <= 3
constexpr int64_t kWideTopPoints = 4194304;  // FP64 top-level moment sums from this size on
constexpr int kDefaultPacketQuery = 2;     // queries per lane (tuned: dps_set_launch)
constexpr int kDefaultPacketAdjoint = 4;
constexpr int kFlagXcdQuery = 1;          // launch flags (dps_set_launch)
constexpr int kFlagXcdAdjoint = 2;
constexpr int kFlagPersistentQuery = 4;
constexpr int kFlagPersistentAdjoint = 8;
constexpr int kDefaultLaunchFlags = kFlagXcdQuery | kFlagXcdAdjoint;

struct alignas(32) NodeRec {
    float cx, cy, cz, r2;  // FP32 centroid and squared radius
    uint32_t first;        // first child (internal) or first point (leaf)
    uint32_t down;         // where a walk that opens the node goes next: its first
                           // child, or for a leaf its escape (the march's walk
                           // selects with it; in the other walks the compiler
                           // keeps fewer copies selecting on the leaf flag)
    uint32_t escape;       // next node in depth-first order after this subtree
    uint32_t meta;         // level | kLeafFlag | children or points << kCountShift
};

__host__ __device__ inline uint32_t node_count(const NodeRec &nd) { return nd.meta >> kCountShift; }

struct alignas(32) PointRec {
    float x, y, z;         // position as given
    float anx, any, anz;   // A_m * n_m (FP32 product)
    float a;               // A_m
    float pad;
};

// a0 b0 + a1 b1 + a2 b2 as one fixed chain of fused operations, so that every
// kernel forms a dot product with the same roundings (left to contraction,
// the compiler may fuse a different product in each kernel)
__device__ __forceinline__ float dot3(float a0, float a1, float a2, float b0, float b1, float b2) {
    return fmaf(a2, b2, fmaf(a1, b1, a0 * b0));
}

// 1/(4 pi), 2/sqrt(pi), 4/sqrt(pi)
constexpr float kInv4Pi = 0.0795774715459476679f;
constexpr float k2SqrtPi = 1.12837916709551257f;
constexpr float k4SqrtPi = 2.25675833419102515f;

// Radial-factor branch points, in t^2 = (r/eps)^2: rho = 1 and psi = 3 above
// 4.5^2 (rho(4.5) = 1 - 8e-9).  radial() and radial3(): Taylor series below
// 1, the erfcx form in between.
constexpr float kSeriesWideT2 = 1.0f;
constexpr float kFarT2 = 20.25f;

// erfcx(t) = exp(t^2) erfc(t) on [1, 4.5] as sum_k kErfcx[k] s^k,
// s = 1/(1 + t/2): a least-squares fit with relative weighting
// (csrc/gen_erfcx.py; 1.1e-9 relative in FP64, about 3e-7 evaluated in FP32)
constexpr float kErfcx0 = -0.0001324968907283619f;
constexpr float kErfcx1 = 0.284586638212204f;
constexpr float kErfcx2 = 0.26176685094833374f;
constexpr float kErfcx3 = 0.3405025601387024f;
constexpr float kErfcx4 = -0.0883762538433075f;
constexpr float kErfcx5 = 0.54436856508255f;
constexpr float kErfcx6 = -0.4582943618297577f;
constexpr float kErfcx7 = 0.1156064048409462f;
// log2(e) as a float and the remainder of its rounding; ln 2
constexpr float kLog2e = 1.44269502162933349609f;
constexpr float kLog2eLo = 1.92596298909109e-08f;
constexpr float kLn2 = 0.693147180559945309f;

// ---------------------------------------------------------------------------
// bf16 storage (round to nearest even; inputs are finite)
// ---------------------------------------------------------------------------
__host__ __device__ inline uint16_t f32_to_bf16(float v) {
    uint32_t u;
    __builtin_memcpy(&u, &v, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// ---------------------------------------------------------------------------
// decision-critical FP32 arithmetic: a fixed sequence of correctly rounded
// operations (explicit fused multiply-adds, no other contraction), so that
// the far decisions and node radii match any other IEEE evaluation of the
// same sequence bit for bit
// ---------------------------------------------------------------------------
__host__ __device__ inline float dist2_rn(float ax, float ay, float az, float bx, float by, float bz) {
#pragma clang fp contract(off)
    float dx = ax - bx;
    float dy = ay - by;
    float dz = az - bz;
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

__host__ __device__ inline float mul_rn(float a, float b) {
#pragma clang fp contract(off)
    return a * b;
}

// ---------------------------------------------------------------------------
// radial factors kappa = rho(t)/(4 pi r^3), lambda = psi(t)/(4 pi r^5), t = r/eps,
// psi = 3 rho - t rho', and for the Hessian nu = chi(t)/(4 pi r^7) = -lambda'(r)/r,
// chi = 5 psi - t psi' = 15 rho - (4/sqrt pi)(5 t^3 + 2 t^5) exp(-t^2).
// Series (derived from those of erf and exp):
//   rho(t)/t^3 = (4/sqrt pi)  sum_{n>=1} (-1)^{n+1} t^{2n-2} / ((n-1)! (2n+1))
//   psi(t)/t^5 = (8/sqrt pi)  sum_{n>=2} (-1)^n     t^{2n-4} / ((n-2)! (2n+1))
//   chi(t)/t^7 = (16/sqrt pi) sum_{n>=3} (-1)^{n+1} t^{2n-6} / ((n-3)! (2n+1))
// ---------------------------------------------------------------------------
struct KernelParams {
    float eps;       // 0: unregularised
    float ieps;      // 1/eps
    float ieps2;     // 1/eps^2
    float k3;        // 1/(4 pi eps^3)
    float k5;        // 1/(4 pi eps^5)
    float k7;        // 1/(4 pi eps^7)
    float ke4;       // 1/(pi^1.5 eps^4):   d kappa / d eps = -exp(-t^2) ke4
    float ke6;       // 2/(pi^1.5 eps^6):   d lambda / d eps = -exp(-t^2) ke6
    float zone_r2;   // r2 < zone_r2 iff r2 * ieps2 < kFarT2 (the regularised zone); 0 without eps
    uint32_t nhi;    // BF16 storage: nodes [0, nhi) keep FP32 moments (0 otherwise)
};

__host__ inline KernelParams make_kernel_params(float eps) {
    KernelParams kp;
    kp.eps = eps;
    kp.nhi = 0;
    if (eps > 0.0f) {
        double e = eps;
        kp.ieps = (float)(1.0 / e);
        kp.ieps2 = (float)(1.0 / (e * e));
        kp.k3 = (float)(0.0795774715459476679 / (e * e * e));
        kp.k5 = (float)(0.0795774715459476679 / (e * e * e * e * e));
        kp.k7 = (float)(0.0795774715459476679 / (e * e * e * e * e * e * e));
        kp.ke4 = (float)(0.179587122125166564 / (e * e * e * e));
        kp.ke6 = (float)(0.359174244250333128 / (e * e * e * e * e * e));
        // the smallest float r2 whose FP32 product r2 * ieps2 reaches kFarT2
        // (the product is monotone in r2): one compare of r2 then takes the
        // same decision as forming the product and comparing it
        float z = (float)((double)kFarT2 / (double)kp.ieps2);
        while (z > 0.0f && z * kp.ieps2 >= kFarT2) z = std::nextafter(z, 0.0f);
        while (z * kp.ieps2 < kFarT2) z = std::nextafter(z, HUGE_VALF);
        kp.zone_r2 = z;
    } else {
        kp.ieps = 0.0f;
        kp.ieps2 = 0.0f;
        kp.k3 = 0.0f;
        kp.k5 = 0.0f;
        kp.k7 = 0.0f;
        kp.ke4 = 0.0f;
        kp.ke6 = 0.0f;
        kp.zone_r2 = 0.0f;  // no r2 lies below it
    }
    return kp;
}

// rho/t^3 and psi/t^5, ten terms: 2e-7 relative in FP32 up to t^2 = 1
__device__ __forceinline__ float series_rho_t3(float u) {  // u = t^2
    constexpr float c = 2.25675833419102515f;
    return c * (1.0f / 3.0f + u * (-1.0f / 5.0f + u * (1.0f / 14.0f + u * (-1.0f / 54.0f +
           u * (1.0f / 264.0f + u * (-1.0f / 1560.0f + u * (1.0f / 10800.0f + u * (-1.0f / 85680.0f +
           u * (1.0f / 766080.0f + u * (-1.0f / 7620480.0f))))))))));
}

__device__ __forceinline__ float series_psi_t5(float u) {  // u = t^2
    constexpr float c = 4.51351666838205030f;
    return c * (1.0f / 5.0f + u * (-1.0f / 7.0f + u * (1.0f / 18.0f + u * (-1.0f / 66.0f +
           u * (1.0f / 312.0f + u * (-1.0f / 1800.0f + u * (1.0f / 12240.0f + u * (-1.0f / 95760.0f +
           u * (1.0f / 846720.0f + u * (-1.0f / 8346240.0f))))))))));
}

// exp(-u) for u in [1, 20.25] through the hardware 2^x (1 ulp): -u log2(e)
// as its rounded product hi and the residual lo (an FMA, plus the rounding
// of the constant), then 2^hi (1 + lo ln 2).  No range reduction is needed
// on this interval.
__device__ __forceinline__ float exp_neg(float u) {
    const float hi = -u * kLog2e;
    const float lo = fmaf(-u, kLog2e, -hi) - u * kLog2eLo;
    const float e = __builtin_amdgcn_exp2f(hi);
    return fmaf(e, lo * kLn2, e);
}

// rho and psi for t^2 = u in [1, 20.25]: with e = exp(-t^2),
// 1 - rho = erfc(t) + (2/sqrt pi) t e = e (erfcx(t) + (2/sqrt pi) t), so one
// exponential serves both terms and rho has no cancellation worse than 1.4x
__device__ __forceinline__ float rho_erfcx(float u, float t, float &e) {
    e = exp_neg(u);
    const float s = __builtin_amdgcn_rcpf(fmaf(0.5f, t, 1.0f));
    float r = fmaf(kErfcx7, s, kErfcx6);
    r = fmaf(r, s, kErfcx5);
    r = fmaf(r, s, kErfcx4);
    r = fmaf(r, s, kErfcx3);
    r = fmaf(r, s, kErfcx2);
    r = fmaf(r, s, kErfcx1);
    r = fmaf(r, s, kErfcx0);
    return fmaf(-e, fmaf(k2SqrtPi, t, r), 1.0f);
}

__device__ __forceinline__ void rho_psi_erfcx(float u, float t, float &rho, float &psi, float &e) {
    rho = rho_erfcx(u, t, e);
    psi = fmaf(3.0f, rho, -(k4SqrtPi * (t * u) * e));
}

__device__ __forceinline__ float series_chi_t7(float u) {  // u = t^2
    constexpr float c = 9.02703333676410060f;
    return c * (1.0f / 7.0f + u * (-1.0f / 9.0f + u * (1.0f / 22.0f + u * (-1.0f / 78.0f +
           u * (1.0f / 360.0f + u * (-1.0f / 2040.0f + u * (1.0f / 13680.0f + u * (-1.0f / 105840.0f +
           u * (1.0f / 927360.0f + u * (-1.0f / 9072000.0f))))))))));
}

// r2 = |d|^2.  Returns false when the term is excluded (r = 0 with eps = 0).
// Common case first, without branches: rho = 1, psi = 3 (t >= 4.5 or eps = 0),
// with the hardware reciprocal square root (1 ulp).  Inside the regularised
// zone t < 4.5 (near points and the nearest far nodes; r2 < zone_r2, never
// without eps) the factors are recomputed: series below t = 1 (finite at
// r = 0), the erfcx form above.
// FAR: r2 > 0 is known (a far-field node lies beyond beta r_t of the query),
// so the test for a source at the query point is left out.
template <bool FAR = false>
__device__ __forceinline__ bool radial(float r2, const KernelParams &kp, float &kappa, float &lambda) {
    if (!FAR && kp.eps == 0.0f && !(r2 > 0.0f)) return false;
    const float ir = __builtin_amdgcn_rsqf(r2);
    const float ir2 = ir * ir;
    kappa = kInv4Pi * ir * ir2;
    lambda = 3.0f * kappa * ir2;
    if (r2 < kp.zone_r2) {
        const float u = r2 * kp.ieps2;
        if (u < kSeriesWideT2) {
            kappa = kp.k3 * series_rho_t3(u);
            lambda = kp.k5 * series_psi_t5(u);
        } else {
            float rho, psi, e;
            rho_psi_erfcx(u, r2 * ir * kp.ieps, rho, psi, e);
            kappa = kappa * rho;
            lambda = kInv4Pi * ir * ir2 * ir2 * psi;
        }
    }
    return true;
}

// kappa alone, same branches as radial() (the adjoint's node and point
// increments need no lambda when dL/dx comes from the forward's gradients)
template <bool FAR = false>
__device__ __forceinline__ bool radial_kappa(float r2, const KernelParams &kp, float &kappa) {
    if (!FAR && kp.eps == 0.0f && !(r2 > 0.0f)) return false;
    const float ir = __builtin_amdgcn_rsqf(r2);
    const float ir2 = ir * ir;
    kappa = kInv4Pi * ir * ir2;
    if (r2 < kp.zone_r2) {
        const float u = r2 * kp.ieps2;
        if (u < kSeriesWideT2) {
            kappa = kp.k3 * series_rho_t3(u);
        } else {
            float e;
            kappa = kappa * rho_erfcx(u, r2 * ir * kp.ieps, e);
        }
    }
    return true;
}

// kappa, lambda and the Hessian factor nu = chi(t)/(4 pi r^7), same branches
// as radial(); chi = 15 where rho = 1, psi = 3.
__device__ __forceinline__ bool radial3(float r2, const KernelParams &kp, float &kappa, float &lambda,
                                        float &nu) {
    if (kp.eps == 0.0f && !(r2 > 0.0f)) return false;
    const float ir = __builtin_amdgcn_rsqf(r2);
    const float ir2 = ir * ir;
    kappa = kInv4Pi * ir * ir2;
    lambda = 3.0f * kappa * ir2;
    nu = 5.0f * lambda * ir2;
    {
        const bool zone = r2 < kp.zone_r2;
        const float u = r2 * kp.ieps2;
        // the wavefront-uniform test keeps the branch-free block below a real
        // branch: without it the compiler evaluated it for every term
        if (__ballot(zone) != 0 && zone) {
            if (u < kSeriesWideT2) {
                kappa = kp.k3 * series_rho_t3(u);
                lambda = kp.k5 * series_psi_t5(u);
                nu = kp.k7 * series_chi_t7(u);
            } else {
                const float t = r2 * ir * kp.ieps;
                float rho, psi, e;
                rho_psi_erfcx(u, t, rho, psi, e);
                const float chi = fmaf(15.0f, rho, -(k4SqrtPi * (t * u) * fmaf(2.0f, u, 5.0f) * e));
                const float ir5 = ir * ir2 * ir2;
                kappa = kappa * rho;
                lambda = kInv4Pi * ir5 * psi;
                nu = kInv4Pi * ir5 * ir2 * chi;
            }
        }
    }
    return true;
}

// ---------------------------------------------------------------------------
// wavefront (64-lane) reductions with DPP; every lane must be active
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

// Sum over the 64 lanes; the result is returned uniformly (from lane 63).
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_f<0xb1>(v);          // quad_perm [1,0,3,2]
    v += dpp_f<0x4e>(v);          // quad_perm [2,3,0,1]
    v += dpp_f<0x141>(v);         // row_half_mirror
    v += dpp_f<0x140>(v);         // row_mirror: every lane holds its row sum
    v += dpp_f<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
    v += dpp_f<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// ---------------------------------------------------------------------------
// Reduce-scatter of N <= 16 per-lane values over the 64 lanes.
//
// The values are taken as 4R registers, R = ceil(N / 4) (zeros past N).  The
// first two halvings use the gfx950 lane swaps, which exchange whole halves
// of two registers in one instruction: after permlane32_swap of registers k
// and k + 2R and one add, the lower half-wave holds register k summed over
// the lanes l and l + 32, the upper half register k + 2R; permlane16_swap of
// k and k + R does the same between the even and odd rows of 16.  A lane then
// carries R registers, each summed over the 4 lanes of its column (l mod 16),
// register k standing for value k + R b4 + 2R b5 (b_i: bit i of the lane).
// Inside a row, the R registers are halved over lane bits 0 and 1 (DPP quad
// permutes: partners differ in that bit, each keeps one half of the pair and
// sends the other) and summed over bits 2 and 3 (row rotations by 4 and 8).
// Lane l ends with the total of value wave_slot<N>(l) =
// kk + R b4 + 2R b5, where kk = 2 b0 + b1 (R > 2), b0 (R = 2), 0 (R = 1);
// wave_slot gives -1 where kk >= R or the value is padding, and also for
// every lane with bit 2 or 3 set, so each value has exactly one lane.
// ---------------------------------------------------------------------------
template <int N_>
constexpr int scatter_regs() { return (N_ + 3) / 4; }

template <int N_>
__device__ __forceinline__ int wave_slot(int lane) {
    constexpr int R = scatter_regs<N_>();
    if (lane & 12) return -1;
    const int b0 = lane & 1, b1 = (lane >> 1) & 1, b4 = (lane >> 4) & 1, b5 = (lane >> 5) & 1;
    const int kk = R > 2 ? 2 * b0 + b1 : R == 2 ? (b1 ? R : b0) : (b0 | b1 ? R : 0);
    const int n = kk + R * b4 + 2 * R * b5;
    return (kk < R && n < N_) ? n : -1;
}

// pair sums over one lane-swap: lanes whose half (or row parity) is 0 get
// register a summed with its partner, the others register b
__device__ __forceinline__ float swap32_add(float a, float b) {
    const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}

__device__ __forceinline__ float swap16_add(float a, float b) {
    const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}

// one in-row halving with the partner through the DPP control CTRL: lanes
// with hi keep b and send a, the others keep a and send b
template <int CTRL>
__device__ __forceinline__ float dpp_halve(float a, float b, bool hi) {
    const float keep = hi ? b : a;
    const float send = hi ? a : b;
    return keep + dpp_f<CTRL>(send);
}

template <int N_>
__device__ __forceinline__ float wave_sum_scatter(const float (&v)[N_]) {
    static_assert(N_ >= 1 && N_ <= 16, "at most 16 values per call");
    constexpr int R = scatter_regs<N_>();
    float x[4 * R], y[2 * R], z[4];
#pragma unroll
    for (int k = 0; k < 4 * R; ++k) x[k] = k < N_ ? v[k] : 0.0f;
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) y[k] = swap32_add(x[k], x[k + 2 * R]);
#pragma unroll
    for (int k = 0; k < R; ++k) z[k] = swap16_add(y[k], y[k + R]);
    const int lane = lane_id();
    const bool h0 = (lane & 1) != 0, h1 = (lane & 2) != 0;
    float r;
    if constexpr (R == 1) {
        r = z[0];
        r += dpp_f<0xb1>(r);  // quad_perm [1,0,3,2]
        r += dpp_f<0x4e>(r);  // quad_perm [2,3,0,1]
    } else if constexpr (R == 2) {
        r = dpp_halve<0xb1>(z[0], z[1], h0);
        r += dpp_f<0x4e>(r);
    } else {
        if constexpr (R == 3) z[3] = 0.0f;
        const float w0 = dpp_halve<0xb1>(z[0], z[2], h0);
        const float w1 = dpp_halve<0xb1>(z[1], z[3], h0);
        r = dpp_halve<0x4e>(w0, w1, h1);
    }
    r += dpp_f<0x124>(r);  // row_ror:4
    r += dpp_f<0x128>(r);  // row_ror:8
    return r;
}

// Max over the 64 lanes of non-negative values.
__device__ __forceinline__ float wave_max_nonneg(float v) {
    v = fmaxf(v, dpp_f<0xb1>(v));
    v = fmaxf(v, dpp_f<0x4e>(v));
    v = fmaxf(v, dpp_f<0x141>(v));
    v = fmaxf(v, dpp_f<0x140>(v));
    v = fmaxf(v, dpp_f<0x142, 0xa>(v));
    v = fmaxf(v, dpp_f<0x143, 0xc>(v));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}


}  // namespace dps
