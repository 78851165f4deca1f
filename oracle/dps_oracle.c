/*
 * dps_oracle.c -- plain FP64 CPU reference for regularized dipole sums.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the GPU library is
 * compared against; it is used by tests/, by the smoke check and by the
 * CPU-baseline leg of the benchmark, and by nothing else.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * Paper: Chen, Miller, Gkioulekas, "3D Reconstruction with Fast Dipole Sums",
 * ACM TOG 43(6), 2024 (arXiv 2405.16788).
 *
 * What it computes, with the passage each part follows:
 *
 *  kernel      Sec. 4.1, eq. (regularized_poisson) with eq. (wn):
 *              P_eps(x,y) = rho(|y-x|/eps) n(y).(y-x) / (4 pi |y-x|^3),
 *              rho(t) = erf t - (2t/sqrt(pi)) exp(-t^2).
 *              The 1/(4 pi) of eq. (wn) is kept in every term, including the
 *              far-field formula of Sec. 6.1 and the gradient of App. C, which
 *              print it without that factor.
 *  direct sum  Sec. 4.2, eq. (dipole_sum): D(x) = sum_m A_m P_eps(x, p_m) mu_m,
 *              one value per attribute channel (Sec. 5.1, eq.
 *              (appearance_features): every channel uses the same weights).
 *  gradient    grad_x of each term:  -kappa D + lambda (D.d) d  with
 *              d = p - x, r = |d|, t = r/eps, kappa = rho(t)/(4 pi r^3),
 *              lambda = psi(t)/(4 pi r^5), psi(t) = 3 rho(t) - t rho'(t)
 *              = 3 rho(t) - (4/sqrt(pi)) t^3 exp(-t^2).
 *  octree      Sec. 6.1 names an octree; its exact layout is not given, so a
 *              canonical one is fixed here (Morton order, bucket leaves of at
 *              most leaf_size points or level 21, no chain collapsing,
 *              breadth-first numbering, children contiguous in octant order).
 *  node data   Sec. 6.1, eq. (farfield_dipole): A_t = sum A_m, centroid
 *              p_t = sum A_m p_m / A_t, radius r_t = max |p_m - p_t|;
 *              eq. (farfield_dipole_features): node dipole D_t = A_t mu_t
 *              = sum A_m mu_m n_m (per channel).
 *  far test    Sec. 6.1 / Algorithm 1 (PrimalQuery): a node is used as a far
 *              field iff |x - p_t| > beta r_t, tested before the leaf test.
 *  far field   Sec. 6.1, eq. (farfield): the dipole term of D_t placed at the
 *              centroid, with rho evaluated at the centroid distance.
 *  adjoint     Sec. 6.2 and App. C: node gradients dmu_t accumulate
 *              eq. (farfield_gradient); the second stage applies eq.
 *              (farfield_features_gradient) to every point through all its
 *              ancestors (evaluated as a top-down running sum).
 *  gradient    cotangents h of the spatial gradient g (needed when a loss uses
 *  cotangent   grad D, as the surface density of Sec. 3.1, eq.
 *              (surface_density) does): g is linear in each source dipole D
 *              with d g / d D = lambda d d^T - kappa I, and its x-derivative
 *              is the Hessian of the term,
 *                nu s d d^T - lambda (d D^T + D d^T) - lambda s I,
 *              s = D.d, nu = -lambda'(r)/r = chi(t)/(4 pi r^7),
 *              chi(t) = 5 psi(t) - t psi'(t)
 *                     = 15 rho(t) - (4/sqrt(pi)) (5 t^3 + 2 t^5) exp(-t^2).
 *              The paper does not write these; they are the derivatives of
 *              its terms, taken through the same accepted sources.
 *  monopole    Sec. 7.1 interpolates the K = 32 appearance attributes with the
 *  channels    foreshortening term n.(p - x)/|p - x| of the kernel skipped:
 *              m(r) = rho(r/eps) / (4 pi r^2), value A_m mu_m m, gradient
 *              A_m mu_m (r lambda - kappa / r) d; node moments are scalars
 *              Q_t = sum A_m mu_m at the area-weighted centroid.  A coincident
 *              query and source contribute nothing (m -> 0; the gradient's
 *              direction is undefined there).
 *  normals,    Sec. 5.2 optimises the point normals and the global eps as
 *  eps         well.  A term depends on n_m through D = A_m mu_m n_m only (the
 *              tree geometry does not involve normals), so dL/dn_m =
 *              A_m sum_c mu_mc dL/dD_mc, the far-field part through the node
 *              dipoles of all ancestors; and d kappa / d eps =
 *              -exp(-t^2) / (pi^1.5 eps^4), d lambda / d eps =
 *              -2 exp(-t^2) / (pi^1.5 eps^6) (both vanish as eps -> 0).
 *
 * Precision: everything is FP64 except two things that the GPU must decide
 * bit-identically: the far test, evaluated in FP32 as
 * s = fma(dz, dz, fma(dy, dy, dx*dx)) > (beta*beta) * r2 (d = c - x; the two
 * fused multiply-adds explicit, no other contraction), and the node centroid
 * / squared radius, which are FP64 sums rounded once to FP32 (the radius the
 * largest such s over the node's points).  Build with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
#define ORC_SQRT_PI 1.77245385090551602730
#define ORC_LEVELS 21

/* ------------------------------------------------------------------------ */
/* radial factors                                                            */
/* ------------------------------------------------------------------------ */

/* rho(t)/t^3 from the Taylor series of erf and exp:
 *   rho(t)/t^3 = (4/sqrt(pi)) sum_{n>=1} (-1)^{n+1} t^{2n-2} / ((n-1)! (2n+1)). */
static double rho_over_t3_series(double t2)
{
    double sum = 0.0, pw = 1.0, fact = 1.0;
    for (int n = 1; n <= 16; ++n) {
        if (n > 1) { fact *= (double)(n - 1); pw *= t2; }
        double c = pw / (fact * (double)(2 * n + 1));
        sum += (n & 1) ? c : -c;
    }
    return 4.0 / ORC_SQRT_PI * sum;
}

/* psi(t)/t^5 from the same series (the n = 1 term of 3 rho - t rho' vanishes):
 *   psi(t)/t^5 = (8/sqrt(pi)) sum_{n>=2} (-1)^n t^{2n-4} / ((n-2)! (2n+1)). */
static double psi_over_t5_series(double t2)
{
    double sum = 0.0, pw = 1.0, fact = 1.0;
    for (int n = 2; n <= 17; ++n) {
        if (n > 2) { fact *= (double)(n - 2); pw *= t2; }
        double c = pw / (fact * (double)(2 * n + 1));
        sum += (n & 1) ? -c : c;
    }
    return 8.0 / ORC_SQRT_PI * sum;
}

/* chi(t)/t^7 from the same series (the n = 1, 2 terms of 5 psi - t psi'
 * vanish):  chi(t)/t^7 = (16/sqrt(pi)) sum_{n>=3} (-1)^{n+1} t^{2n-6}
 * / ((n-3)! (2n+1)). */
static double chi_over_t7_series(double t2)
{
    double sum = 0.0, pw = 1.0, fact = 1.0;
    for (int n = 3; n <= 18; ++n) {
        if (n > 3) { fact *= (double)(n - 3); pw *= t2; }
        double c = pw / (fact * (double)(2 * n + 1));
        sum += (n & 1) ? c : -c;
    }
    return 16.0 / ORC_SQRT_PI * sum;
}

double orc_rho(double t)
{
    if (t < 0.5) return rho_over_t3_series(t * t) * t * t * t;
    return erf(t) - 2.0 * t / ORC_SQRT_PI * exp(-t * t);
}

double orc_psi(double t)
{
    if (t < 0.5) return psi_over_t5_series(t * t) * t * t * t * t * t;
    double rho = erf(t) - 2.0 * t / ORC_SQRT_PI * exp(-t * t);
    return 3.0 * rho - 4.0 / ORC_SQRT_PI * t * t * t * exp(-t * t);
}

double orc_chi(double t)
{
    if (t < 0.5) return chi_over_t7_series(t * t) * pow(t, 7.0);
    double ex = exp(-t * t);
    double rho = erf(t) - 2.0 * t / ORC_SQRT_PI * ex;
    return 15.0 * rho - 4.0 / ORC_SQRT_PI * (5.0 * t * t * t + 2.0 * pow(t, 5.0)) * ex;
}
double orc_chi_series(double t) { return chi_over_t7_series(t * t) * pow(t, 7.0); }

/* Exposed for the pins: the series branch and the closed-form branch. */
double orc_rho_series(double t) { return rho_over_t3_series(t * t) * t * t * t; }
double orc_psi_series(double t) { return psi_over_t5_series(t * t) * pow(t, 5.0); }
double orc_rho_closed(double t) { return erf(t) - 2.0 * t / ORC_SQRT_PI * exp(-t * t); }

/* kappa = rho(r/eps)/(4 pi r^3), lambda = psi(r/eps)/(4 pi r^5).
 * eps = 0 is the unregularized kernel (rho = 1, psi = 3).  r = 0 with eps > 0
 * uses the finite limits of the series. */
static void radial(double r, double eps, double *kappa, double *lambda)
{
    if (eps == 0.0) {
        double r3 = r * r * r;
        *kappa = 1.0 / (4.0 * ORC_PI * r3);
        *lambda = 3.0 / (4.0 * ORC_PI * r3 * r * r);
        return;
    }
    double t = r / eps;
    if (t < 0.5) {
        double e3 = eps * eps * eps;
        *kappa = rho_over_t3_series(t * t) / (4.0 * ORC_PI * e3);
        *lambda = psi_over_t5_series(t * t) / (4.0 * ORC_PI * e3 * eps * eps);
    } else {
        double ex = exp(-t * t);
        double rho = erf(t) - 2.0 * t / ORC_SQRT_PI * ex;
        double psi = 3.0 * rho - 4.0 / ORC_SQRT_PI * t * t * t * ex;
        double r3 = r * r * r;
        *kappa = rho / (4.0 * ORC_PI * r3);
        *lambda = psi / (4.0 * ORC_PI * r3 * r * r);
    }
}

void orc_radial(double r, double eps, double *kappa, double *lambda)
{
    radial(r, eps, kappa, lambda);
}

/* nu = chi(r/eps)/(4 pi r^7) (eps = 0: chi = 15); finite at r = 0 for eps > 0. */
static double radial_nu(double r, double eps)
{
    if (eps == 0.0) return 15.0 / (4.0 * ORC_PI * pow(r, 7.0));
    double t = r / eps;
    if (t < 0.5) return chi_over_t7_series(t * t) / (4.0 * ORC_PI * pow(eps, 7.0));
    return orc_chi(t) / (4.0 * ORC_PI * pow(r, 7.0));
}

double orc_radial_nu(double r, double eps) { return radial_nu(r, eps); }

/* d kappa / d eps and d lambda / d eps (0 for eps = 0) */
static void radial_eps(double r, double eps, double *kap_e, double *lam_e)
{
    if (eps == 0.0) { *kap_e = 0.0; *lam_e = 0.0; return; }
    double t = r / eps;
    double e = exp(-t * t) / (ORC_PI * ORC_SQRT_PI);
    double e2 = eps * eps;
    *kap_e = -e / (e2 * e2);
    *lam_e = -2.0 * e / (e2 * e2 * e2);
}

void orc_radial_eps(double r, double eps, double *kap_e, double *lam_e) { radial_eps(r, eps, kap_e, lam_e); }

static double norm3(const double v[3]) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

/* dL/deps of one term with dipole D, value cotangent w (or 0) and gradient
 * cotangent h (or NULL), and its absolute scale, with |D.d| <= wD r and
 * |D.h| <= wD |h| for the absolute mass wD of the term (< 0: |D|) */
static double term_eps(const double d[3], double kap_e, double lam_e, const double D[3], double wD, double w,
                       const double *h, double *scale)
{
    double s = D[0] * d[0] + D[1] * d[1] + D[2] * d[2];
    double r = norm3(d), m = wD < 0.0 ? norm3(D) : wD;
    double v = w * kap_e * s, a = fabs(w * kap_e) * m * r;
    if (h) {
        double dh = d[0] * h[0] + d[1] * h[1] + d[2] * h[2];
        double Dh = D[0] * h[0] + D[1] * h[1] + D[2] * h[2];
        v += lam_e * s * dh - kap_e * Dh;
        a += fabs(lam_e * dh) * m * r + fabs(kap_e) * m * norm3(h);
    }
    if (scale) *scale += a;
    return v;
}

/* Cotangent h of the gradient of one source term with dipole D at offset
 * d = c - x (radial factors kap, lam, nu):
 *   dD += lambda (d.h) d - kappa h          (the term's derivative in D)
 *   dx += nu s (d.h) d - lambda (d (D.h) + D (d.h)) - lambda s h
 * and the matching absolute scales. */
static void grad_cotangent(const double d[3], double r, double kap, double lam, double nu,
                           const double D[3], double wD, const double h[3], double dD[3], double dx[3],
                           double *sdD, double *sdx)
{
    double s = D[0] * d[0] + D[1] * d[1] + D[2] * d[2];
    double dh = d[0] * h[0] + d[1] * h[1] + d[2] * h[2];
    double Dh = D[0] * h[0] + D[1] * h[1] + D[2] * h[2];
    for (int k = 0; k < 3; ++k) {
        if (dD) dD[k] += lam * dh * d[k] - kap * h[k];
        if (dx) dx[k] += nu * s * dh * d[k] - lam * (d[k] * Dh + D[k] * dh) - lam * s * h[k];
    }
    double nh = sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
    double nD = wD < 0.0 ? norm3(D) : wD;
    if (sdD) *sdD += nh * (fabs(lam) * r * r + kap);
    if (sdx) *sdx += nh * nD * (fabs(nu) * r * r * r + 3.0 * fabs(lam) * r);
}

/* ------------------------------------------------------------------------ */
/* one source term (point or node) at one query                              */
/* ------------------------------------------------------------------------ */

/* Adds, for channels c < C, the value kappa (D_c.d), the gradient
 * -kappa D_c + lambda (D_c.d) d, and the absolute scales
 * kappa W_c r and W_c (kappa + |lambda| r^2), W_c the absolute dipole mass of
 * the source: |D_c| for a point (W = NULL), and for a node the sum of |D_mc|
 * over its points (its moment aggregates them, so any FP32 formation of the
 * moment errs in proportion to that sum, however much the moment cancels).
 * Returns 0 if the source coincides with the query and eps = 0 (term
 * excluded). */
static int add_term(const double c[3], const double *D, const double *W, int C, const double x[3],
                    double eps, double *f, double *g, double *sf, double *sg)
{
    double d[3] = {c[0] - x[0], c[1] - x[1], c[2] - x[2]};
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 == 0.0 && eps == 0.0) return 0;
    double r = sqrt(r2), kap, lam;
    radial(r, eps, &kap, &lam);
    for (int ch = 0; ch < C; ++ch) {
        const double *Dc = D + 3 * ch;
        double s = Dc[0] * d[0] + Dc[1] * d[1] + Dc[2] * d[2];
        if (f) f[ch] += kap * s;
        if (g) {
            for (int k = 0; k < 3; ++k) g[3 * ch + k] += -kap * Dc[k] + lam * s * d[k];
        }
        double nd = W ? W[ch] : sqrt(Dc[0] * Dc[0] + Dc[1] * Dc[1] + Dc[2] * Dc[2]);
        if (sf) sf[ch] += kap * nd * r;
        if (sg) sg[ch] += nd * (kap + fabs(lam) * r2);
    }
    return 1;
}

/* Monopole term with charges Qc[3*ch] (stride 3): value Q m, m = kappa r,
 * gradient Q (r lambda - kappa / r) d; absolute scales W m and
 * W |r lambda - kappa / r| r with W = |Q| for a point (W = NULL) or the sum of
 * A_m |mu_m| over a node's points.  Returns 0 when the source coincides with
 * the query (no contribution). */
static int add_term_mono(const double c[3], const double *Qc, const double *W, int C, const double x[3],
                         double eps, double *f, double *g, double *sf, double *sg)
{
    double d[3] = {c[0] - x[0], c[1] - x[1], c[2] - x[2]};
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 == 0.0) return 0;
    (void)eps;
    double r = sqrt(r2), kap, lam;
    radial(r, eps, &kap, &lam);
    double m = kap * r, gv = r * lam - kap / r;
    for (int ch = 0; ch < C; ++ch) {
        double q = Qc[3 * ch], aq = W ? W[ch] : fabs(q);
        if (f) f[ch] += q * m;
        if (g) for (int k = 0; k < 3; ++k) g[3 * ch + k] += q * gv * d[k];
        if (sf) sf[ch] += aq * m;
        if (sg) sg[ch] += aq * fabs(gv) * r;
    }
    return 1;
}

static int nthreads_or_default(int nt)
{
#ifdef _OPENMP
    return nt > 0 ? nt : omp_get_max_threads();
#else
    (void)nt;
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* direct O(QM) sum, eq. (dipole_sum)                                        */
/* ------------------------------------------------------------------------ */

/* p, n: [M][3]; A: [M]; mu: [M][C]; x: [Q][3] (all FP32, caller order).
 * Outputs (FP64, may be NULL): f[Q][C], g[Q][C][3], sf[Q][C], sg[Q][C]. */
int orc_direct(const float *p, const float *n, const float *A, const float *mu,
               int64_t M, int C, const float *x, int64_t Q, double eps,
               double *f, double *g, double *sf, double *sg, int nthreads)
{
    if (M < 0 || Q < 0 || C < 1 || C > 64 || eps < 0) return 1;
    int nt = nthreads_or_default(nthreads);
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t q = 0; q < Q; ++q) {
        double xq[3] = {x[3 * q], x[3 * q + 1], x[3 * q + 2]};
        double fl[64], gl[192], sfl[64], sgl[64], D[192];
        memset(fl, 0, sizeof fl); memset(gl, 0, sizeof gl);
        memset(sfl, 0, sizeof sfl); memset(sgl, 0, sizeof sgl);
        for (int64_t m = 0; m < M; ++m) {
            double c[3] = {p[3 * m], p[3 * m + 1], p[3 * m + 2]};
            for (int ch = 0; ch < C; ++ch)
                for (int k = 0; k < 3; ++k)
                    D[3 * ch + k] = (double)A[m] * (double)mu[m * C + ch] * (double)n[3 * m + k];
            add_term(c, D, NULL, C, xq, eps, fl, gl, sfl, sgl);
        }
        for (int ch = 0; ch < C; ++ch) {
            if (f) f[q * C + ch] = fl[ch];
            if (sf) sf[q * C + ch] = sfl[ch];
            if (sg) sg[q * C + ch] = sgl[ch];
            if (g) for (int k = 0; k < 3; ++k) g[(q * C + ch) * 3 + k] = gl[3 * ch + k];
        }
    }
    return 0;
}

/* Exact transpose of orc_direct: given df[Q][C] and (optionally, may be
 * NULL) the gradient cotangents dg[Q][C][3],
 *   dmu[m][c] = sum_q df[q][c] A_m kappa_qm (n_m . d_qm)
 *             + sum_q A_m n_m . (lambda (d.h) d - kappa h),   h = dg[q][c],
 *   dx[q]     = sum_m sum_c df[q][c] (-kappa D_mc + lambda (D_mc . d) d)
 *             + sum_m sum_c (Hessian of the term) h.
 * df may be NULL when dg is given (value cotangents zero). */
int orc_direct_adjoint(const float *p, const float *n, const float *A, const float *mu,
                       int64_t M, int C, const float *x, int64_t Q, double eps,
                       const float *df, const float *dg, double *dmu, double *dx, double *dn,
                       double *deps, int nthreads)
{
    if (M < 0 || Q < 0 || C < 1 || C > 64 || eps < 0 || (!df && !dg)) return 1;
    int nt = nthreads_or_default(nthreads);
    if (dx) {
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int64_t q = 0; q < Q; ++q) {
            double xq[3] = {x[3 * q], x[3 * q + 1], x[3 * q + 2]};
            double acc[3] = {0, 0, 0}, E[3];
            for (int64_t m = 0; m < M; ++m) {
                double d[3] = {p[3 * m] - xq[0], p[3 * m + 1] - xq[1], p[3 * m + 2] - xq[2]};
                double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (r2 == 0.0 && eps == 0.0) continue;
                double kap, lam;
                double r = sqrt(r2);
                radial(r, eps, &kap, &lam);
                if (df) {
                    double w = 0;
                    for (int ch = 0; ch < C; ++ch) w += (double)df[q * C + ch] * (double)mu[m * C + ch];
                    for (int k = 0; k < 3; ++k) E[k] = w * (double)A[m] * (double)n[3 * m + k];
                    double s = E[0] * d[0] + E[1] * d[1] + E[2] * d[2];
                    for (int k = 0; k < 3; ++k) acc[k] += -kap * E[k] + lam * s * d[k];
                }
                if (dg) {
                    double nu = radial_nu(r, eps);
                    for (int ch = 0; ch < C; ++ch) {
                        double D[3], h[3];
                        for (int k = 0; k < 3; ++k) {
                            D[k] = (double)A[m] * (double)mu[m * C + ch] * (double)n[3 * m + k];
                            h[k] = (double)dg[(q * C + ch) * 3 + k];
                        }
                        grad_cotangent(d, r, kap, lam, nu, D, -1.0, h, NULL, acc, NULL, NULL);
                    }
                }
            }
            for (int k = 0; k < 3; ++k) dx[3 * q + k] = acc[k];
        }
    }
    if (dmu) {
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int64_t m = 0; m < M; ++m) {
            double acc[64];
            memset(acc, 0, sizeof acc);
            for (int64_t q = 0; q < Q; ++q) {
                double d[3] = {p[3 * m] - (double)x[3 * q], p[3 * m + 1] - (double)x[3 * q + 1],
                               p[3 * m + 2] - (double)x[3 * q + 2]};
                double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (r2 == 0.0 && eps == 0.0) continue;
                double kap, lam;
                radial(sqrt(r2), eps, &kap, &lam);
                double An[3] = {(double)A[m] * (double)n[3 * m], (double)A[m] * (double)n[3 * m + 1],
                                (double)A[m] * (double)n[3 * m + 2]};
                double s = An[0] * d[0] + An[1] * d[1] + An[2] * d[2];
                for (int ch = 0; ch < C; ++ch) {
                    if (df) acc[ch] += (double)df[q * C + ch] * kap * s;
                    if (dg) {
                        const float *h = dg + (q * C + ch) * 3;
                        double dh = d[0] * h[0] + d[1] * h[1] + d[2] * h[2];
                        double Anh = An[0] * h[0] + An[1] * h[1] + An[2] * h[2];
                        acc[ch] += lam * dh * s - kap * Anh;
                    }
                }
            }
            for (int ch = 0; ch < C; ++ch) dmu[m * C + ch] = acc[ch];
        }
    }
    if (dn) {
        /* dL/dn_m = A_m sum_c mu_mc dL/dD_mc */
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int64_t m = 0; m < M; ++m) {
            double acc[3] = {0, 0, 0};
            for (int64_t q = 0; q < Q; ++q) {
                double d[3] = {p[3 * m] - (double)x[3 * q], p[3 * m + 1] - (double)x[3 * q + 1],
                               p[3 * m + 2] - (double)x[3 * q + 2]};
                double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (r2 == 0.0 && eps == 0.0) continue;
                double kap, lam;
                radial(sqrt(r2), eps, &kap, &lam);
                for (int ch = 0; ch < C; ++ch) {
                    double dD[3] = {0, 0, 0};
                    double w = df ? (double)df[q * C + ch] : 0.0;
                    for (int k = 0; k < 3; ++k) dD[k] = w * kap * d[k];
                    if (dg) {
                        const float *h = dg + (q * C + ch) * 3;
                        double dh = d[0] * h[0] + d[1] * h[1] + d[2] * h[2];
                        for (int k = 0; k < 3; ++k) dD[k] += lam * dh * d[k] - kap * h[k];
                    }
                    double am = (double)A[m] * (double)mu[m * C + ch];
                    for (int k = 0; k < 3; ++k) acc[k] += am * dD[k];
                }
            }
            for (int k = 0; k < 3; ++k) dn[3 * m + k] = acc[k];
        }
    }
    if (deps) {
        double tot = 0.0;
#pragma omp parallel for schedule(static) num_threads(nt) reduction(+ : tot)
        for (int64_t q = 0; q < Q; ++q) {
            double xq[3] = {x[3 * q], x[3 * q + 1], x[3 * q + 2]};
            for (int64_t m = 0; m < M; ++m) {
                double d[3] = {p[3 * m] - xq[0], p[3 * m + 1] - xq[1], p[3 * m + 2] - xq[2]};
                double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (r2 == 0.0 && eps == 0.0) continue;
                double ke, le;
                radial_eps(sqrt(r2), eps, &ke, &le);
                for (int ch = 0; ch < C; ++ch) {
                    double D[3], h[3];
                    for (int k = 0; k < 3; ++k) {
                        D[k] = (double)A[m] * (double)mu[m * C + ch] * (double)n[3 * m + k];
                        if (dg) h[k] = (double)dg[(q * C + ch) * 3 + k];
                    }
                    tot += term_eps(d, ke, le, D, -1.0, df ? (double)df[q * C + ch] : 0.0, dg ? h : NULL, NULL);
                }
            }
        }
        *deps = tot;
    }
    return 0;
}

/* Direct sum of the monopole kernel (appearance channels with the
 * foreshortening term skipped); outputs as orc_direct. */
int orc_direct_mono(const float *p, const float *A, const float *mu, int64_t M, int C, const float *x,
                    int64_t Q, double eps, double *f, double *g, double *sf, double *sg, int nthreads)
{
    if (M < 0 || Q < 0 || C < 1 || C > 64 || eps < 0) return 1;
    int nt = nthreads_or_default(nthreads);
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t q = 0; q < Q; ++q) {
        double xq[3] = {x[3 * q], x[3 * q + 1], x[3 * q + 2]};
        double fl[64], gl[192], sfl[64], sgl[64], Qc[192];
        memset(fl, 0, sizeof fl); memset(gl, 0, sizeof gl);
        memset(sfl, 0, sizeof sfl); memset(sgl, 0, sizeof sgl);
        for (int64_t m = 0; m < M; ++m) {
            double c[3] = {p[3 * m], p[3 * m + 1], p[3 * m + 2]};
            for (int ch = 0; ch < C; ++ch) Qc[3 * ch] = (double)A[m] * (double)mu[m * C + ch];
            add_term_mono(c, Qc, NULL, C, xq, eps, fl, gl, sfl, sgl);
        }
        for (int ch = 0; ch < C; ++ch) {
            if (f) f[q * C + ch] = fl[ch];
            if (sf) sf[q * C + ch] = sfl[ch];
            if (sg) sg[q * C + ch] = sgl[ch];
            if (g) for (int k = 0; k < 3; ++k) g[(q * C + ch) * 3 + k] = gl[3 * ch + k];
        }
    }
    return 0;
}

/* Exact transpose of orc_direct_mono: dmu[m][c] = sum_q df[q][c] A_m m(r_qm),
 * dx[q] = sum_m sum_c df[q][c] A_m mu_mc (r lambda - kappa / r) d. */
int orc_direct_mono_adjoint(const float *p, const float *A, const float *mu, int64_t M, int C, const float *x,
                            int64_t Q, double eps, const float *df, double *dmu, double *dx, int nthreads)
{
    if (M < 0 || Q < 0 || C < 1 || C > 64 || eps < 0 || !df) return 1;
    int nt = nthreads_or_default(nthreads);
    if (dx) {
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int64_t q = 0; q < Q; ++q) {
            double xq[3] = {x[3 * q], x[3 * q + 1], x[3 * q + 2]}, acc[3] = {0, 0, 0};
            for (int64_t m = 0; m < M; ++m) {
                double d[3] = {p[3 * m] - xq[0], p[3 * m + 1] - xq[1], p[3 * m + 2] - xq[2]};
                double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (r2 == 0.0) continue;
                double r = sqrt(r2), kap, lam;
                radial(r, eps, &kap, &lam);
                double w = 0;
                for (int ch = 0; ch < C; ++ch) w += (double)df[q * C + ch] * (double)mu[m * C + ch];
                double gv = (r * lam - kap / r) * w * (double)A[m];
                for (int k = 0; k < 3; ++k) acc[k] += gv * d[k];
            }
            for (int k = 0; k < 3; ++k) dx[3 * q + k] = acc[k];
        }
    }
    if (dmu) {
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int64_t m = 0; m < M; ++m) {
            double acc[64];
            memset(acc, 0, sizeof acc);
            for (int64_t q = 0; q < Q; ++q) {
                double d[3] = {p[3 * m] - (double)x[3 * q], p[3 * m + 1] - (double)x[3 * q + 1],
                               p[3 * m + 2] - (double)x[3 * q + 2]};
                double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (r2 == 0.0) continue;
                double r = sqrt(r2), kap, lam;
                radial(r, eps, &kap, &lam);
                for (int ch = 0; ch < C; ++ch) acc[ch] += (double)df[q * C + ch] * (double)A[m] * kap * r;
            }
            for (int ch = 0; ch < C; ++ch) dmu[m * C + ch] = acc[ch];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* canonical octree                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t M, N;
    int leaf_size, depth, C;
    float lo[3];
    double side, scale;
    uint64_t *codes_in;   /* [M] Morton code of each point, caller order */
    uint64_t *codes;      /* [M] sorted codes */
    uint32_t *perm;       /* [M] sorted position -> caller index */
    float *ps;            /* [M][3] sorted positions (FP32 as given) */
    double *Am;           /* [M] sorted areas */
    double *nm;           /* [M][3] sorted normals */
    int32_t *node;        /* [N][6] level, parent, first_child, n_children, pt_begin, pt_count */
    float *geom;          /* [N][4] centroid (FP32), squared radius (FP32) */
    double *area;         /* [N] A_t */
    double *cen64;        /* [N][3] FP64 centroid before rounding */
    int32_t *leaf_of;     /* [M] leaf node holding sorted point */
    double *mu;           /* [M][C] sorted attributes */
    double *D;            /* [N][C][3] node dipoles D_t = sum A_m mu_m n_m; monopole
                             trees keep Q_t = sum A_m mu_m in D[t][c][0] */
    double *W;            /* [N][C] absolute masses sum_m A_m |mu_m| |n_m| (monopole:
                             sum_m A_m |mu_m|), the scale of a node term */
    int kind;             /* 0: dipole kernel, 1: monopole kernel */
    /* storage emulation (orc_tree_set_storage): the values the sums read */
    int store_mode;       /* 0: exact (FP64 moments, attributes as given) */
    int store_levels;     /* mode 1: nodes of level <= store_levels keep FP32 moments */
    int scale_mode;       /* error scale of a node term: 0 its absolute mass W,
                             1 the magnitude of its own moment (Wm) */
    double *Wm;           /* [N][C] |D_t,c| (monopole: |Q_t,c|) of the exact moments */
    double *Ds;           /* [N][C][3] node moments as stored (== D in mode 0) */
    double *mus;          /* [M][C] sorted attributes as stored (== mu in mode 0) */
} orc_tree;

static uint64_t spread3(uint64_t v)
{
    uint64_t out = 0;
    for (int b = 0; b < ORC_LEVELS; ++b) out |= ((v >> b) & 1ull) << (3 * b);
    return out;
}

typedef struct { uint64_t code; uint32_t idx; } keyidx;

static int cmp_keyidx(const void *a, const void *b)
{
    const keyidx *x = (const keyidx *)a, *y = (const keyidx *)b;
    if (x->code != y->code) return x->code < y->code ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* FP32 squared distance as a fixed sequence of correctly rounded operations:
   three differences, dx*dx, then two fused multiply-adds (fmaf rounds once),
   no other contraction.  The far decisions and node radii depend on it. */
static float dist2_f32(const float a[3], const float b[3])
{
    float dx = a[0] - b[0];
    float dy = a[1] - b[1];
    float dz = a[2] - b[2];
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

/* ------------------------------------------------------------------------ */
/* storage emulation                                                         */
/* ------------------------------------------------------------------------ */

/* The library stores attributes and node moments either as FP32 or as
 * bfloat16 (8 significant bits, FP32's exponent range), the reduced-precision
 * storage that the error study of the method asks to quantify.  These helpers
 * let the oracle evaluate its FP64 sums from values rounded exactly as such a
 * store would hold them, so that a reduced-precision GPU result can be
 * compared with the arithmetic it claims to perform, not only bounded.
 *
 * orc_round_bf16: nearest bfloat16 value (ties to even) of the FP32 value v,
 * returned as a double.  Written from the format's definition: the quantum is
 * 2^(e-8) for |v| in [2^(e-1), 2^e) and 2^-133 below the normal range;
 * values past the largest finite bfloat16 (after rounding) become infinite. */
double orc_round_bf16(float v)
{
    double a = fabs((double)v);
    if (a == 0.0 || !isfinite(a)) return (double)v;
    int e;
    (void)frexp(a, &e);            /* a = m 2^e, m in [0.5, 1) */
    int qe = e - 8;
    if (qe < -133) qe = -133;
    double q = ldexp(nearbyint(ldexp(a, -qe)), qe);  /* default mode: ties to even */
    if (q >= 0x1p128) q = INFINITY;
    return copysign(q, (double)v);
}

static void free_stored(orc_tree *t)
{
    if (t->Ds && t->Ds != t->D) free(t->Ds);
    if (t->mus && t->mus != t->mu) free(t->mus);
    t->Ds = NULL; t->mus = NULL;
}

/* (Re)derives the stored views from the exact attributes and moments.
 * Mode 0: the exact values themselves.  Mode 2 (FP32 store): moments rounded
 * once to FP32 (attributes are FP32 inputs already).  Mode 1 (bfloat16 store):
 * attributes rounded to bfloat16; node moments rounded to FP32 and then to
 * bfloat16 (the store rounds an FP32 value), except nodes of level <=
 * store_levels, which keep the FP32 rounding (store_levels = -1: none). */
static void apply_storage(orc_tree *t)
{
    free_stored(t);
    if (!t->D) return;
    int C = t->C;
    if (t->store_mode == 0) {
        t->Ds = t->D; t->mus = t->mu;
        return;
    }
    t->Ds = (double *)malloc(sizeof(double) * (size_t)t->N * C * 3);
    t->mus = (double *)malloc(sizeof(double) * (size_t)t->M * C);
    for (int64_t i = 0; i < t->M * C; ++i)
        t->mus[i] = t->store_mode == 1 ? orc_round_bf16((float)t->mu[i]) : t->mu[i];
    for (int64_t i = 0; i < t->N; ++i) {
        int keep32 = t->store_mode == 2 || t->node[6 * i] <= t->store_levels;
        for (int c = 0; c < 3 * C; ++c) {
            float v = (float)t->D[i * C * 3 + c];
            t->Ds[i * C * 3 + c] = keep32 ? (double)v : orc_round_bf16(v);
        }
    }
}

/* mode: 0 exact, 1 bfloat16 (levels <= fp32_levels kept FP32), 2 FP32. */
int orc_tree_set_storage(orc_tree *t, int mode, int fp32_levels)
{
    if (!t || mode < 0 || mode > 2 || fp32_levels < -1) return 1;
    t->store_mode = mode;
    t->store_levels = fp32_levels;
    apply_storage(t);
    return 0;
}

/* Node moments [N][C][3] and sorted attributes [M][C] as stored (either may
 * be NULL). */
int orc_tree_export_stored(const orc_tree *t, double *Ds, double *mus)
{
    if (!t || !t->Ds) return 1;
    if (Ds) memcpy(Ds, t->Ds, sizeof(double) * (size_t)t->N * t->C * 3);
    if (mus) memcpy(mus, t->mus, sizeof(double) * (size_t)t->M * t->C);
    return 0;
}

void orc_tree_free(orc_tree *t)
{
    if (!t) return;
    free(t->codes_in); free(t->codes); free(t->perm); free(t->ps); free(t->Am); free(t->nm);
    free(t->node); free(t->geom); free(t->area); free(t->cen64); free(t->leaf_of);
    free_stored(t);
    free(t->mu); free(t->D); free(t->W); free(t->Wm);
    free(t);
}

/* Builds the canonical octree of points p[M][3] (FP32) with areas A[M] and
 * normals n[M][3].  Returns NULL on invalid input. */
orc_tree *orc_tree_build(const float *p, const float *n, const float *A, int64_t M, int leaf_size)
{
    if (M < 1 || M > 0x7fffffffLL || leaf_size < 1) return NULL;
    orc_tree *t = (orc_tree *)calloc(1, sizeof(orc_tree));
    t->M = M; t->leaf_size = leaf_size;
    /* bounding cube: exact FP32 extrema, side and scale in FP64 */
    float lo[3] = {p[0], p[1], p[2]}, hi[3] = {p[0], p[1], p[2]};
    for (int64_t m = 1; m < M; ++m)
        for (int k = 0; k < 3; ++k) {
            float v = p[3 * m + k];
            if (v < lo[k]) lo[k] = v;
            if (v > hi[k]) hi[k] = v;
        }
    double side = 0.0;
    for (int k = 0; k < 3; ++k) {
        double e = (double)hi[k] - (double)lo[k];
        if (e > side) side = e;
    }
    if (side == 0.0) side = 1.0;
    double scale = 2097152.0 / side;
    memcpy(t->lo, lo, sizeof lo);
    t->side = side; t->scale = scale;

    keyidx *ki = (keyidx *)malloc(sizeof(keyidx) * M);
    t->codes_in = (uint64_t *)malloc(sizeof(uint64_t) * M);
    for (int64_t m = 0; m < M; ++m) {
        uint64_t q[3];
        for (int k = 0; k < 3; ++k) {
            double v = ((double)p[3 * m + k] - (double)lo[k]) * scale;
            uint64_t c = (uint64_t)floor(v);
            q[k] = c > 2097151ull ? 2097151ull : c;
        }
        uint64_t code = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
        t->codes_in[m] = code;
        ki[m].code = code; ki[m].idx = (uint32_t)m;
    }
    qsort(ki, (size_t)M, sizeof(keyidx), cmp_keyidx);
    t->codes = (uint64_t *)malloc(sizeof(uint64_t) * M);
    t->perm = (uint32_t *)malloc(sizeof(uint32_t) * M);
    t->ps = (float *)malloc(sizeof(float) * 3 * M);
    t->Am = (double *)malloc(sizeof(double) * M);
    t->nm = (double *)malloc(sizeof(double) * 3 * M);
    for (int64_t i = 0; i < M; ++i) {
        uint32_t j = ki[i].idx;
        t->codes[i] = ki[i].code; t->perm[i] = j;
        for (int k = 0; k < 3; ++k) {
            t->ps[3 * i + k] = p[3 * (int64_t)j + k];
            t->nm[3 * i + k] = n ? (double)n[3 * (int64_t)j + k] : 0.0;
        }
        t->Am[i] = (double)A[j];
    }
    free(ki);

    /* breadth-first emission; children of an internal node at level l are the
     * non-empty octants of its range by the level-(l+1) digit, ascending */
    int64_t cap = 1024, N = 1;
    int32_t *node = (int32_t *)malloc(sizeof(int32_t) * 6 * cap);
    node[0] = 0; node[1] = -1; node[2] = -1; node[3] = 0; node[4] = 0; node[5] = (int32_t)M;
    int depth = 0;
    for (int64_t i = 0; i < N; ++i) {
        int32_t lvl = node[6 * i], beg = node[6 * i + 4], cnt = node[6 * i + 5];
        if (lvl > depth) depth = lvl;
        if (cnt <= leaf_size || lvl == ORC_LEVELS) continue;
        int shift = 3 * (ORC_LEVELS - 1 - lvl);
        node[6 * i + 2] = (int32_t)N;
        int32_t nch = 0;
        int64_t j = beg, end = (int64_t)beg + cnt;
        while (j < end) {
            uint64_t dig = (t->codes[j] >> shift) & 7ull;
            int64_t k = j + 1;
            while (k < end && ((t->codes[k] >> shift) & 7ull) == dig) ++k;
            if (N == cap) { cap *= 2; node = (int32_t *)realloc(node, sizeof(int32_t) * 6 * cap); }
            int32_t *c = node + 6 * N;
            c[0] = lvl + 1; c[1] = (int32_t)i; c[2] = -1; c[3] = 0; c[4] = (int32_t)j; c[5] = (int32_t)(k - j);
            ++N; ++nch; j = k;
        }
        node[6 * i + 3] = nch;
    }
    t->N = N; t->node = node; t->depth = depth;

    /* node geometry: FP64 sums (leaves: points in sorted order; internal:
     * children in child order), centroid rounded once to FP32 */
    t->area = (double *)malloc(sizeof(double) * N);
    t->cen64 = (double *)malloc(sizeof(double) * 3 * N);
    t->geom = (float *)malloc(sizeof(float) * 4 * N);
    t->leaf_of = (int32_t *)malloc(sizeof(int32_t) * M);
    double *S = (double *)malloc(sizeof(double) * 3 * N);
    for (int64_t i = N - 1; i >= 0; --i) {
        const int32_t *nd = node + 6 * i;
        double a = 0, s[3] = {0, 0, 0};
        if (nd[3] == 0) {
            for (int64_t j = nd[4]; j < (int64_t)nd[4] + nd[5]; ++j) {
                a += t->Am[j];
                for (int k = 0; k < 3; ++k) s[k] += t->Am[j] * (double)t->ps[3 * j + k];
                t->leaf_of[j] = (int32_t)i;
            }
        } else {
            for (int64_t c = nd[2]; c < (int64_t)nd[2] + nd[3]; ++c) {
                a += t->area[c];
                for (int k = 0; k < 3; ++k) s[k] += S[3 * c + k];
            }
        }
        t->area[i] = a;
        for (int k = 0; k < 3; ++k) {
            S[3 * i + k] = s[k];
            t->cen64[3 * i + k] = s[k] / a;
            t->geom[4 * i + k] = (float)(s[k] / a);
        }
    }
    free(S);
    for (int64_t i = 0; i < N; ++i) {
        const int32_t *nd = node + 6 * i;
        float r2 = 0.0f;
        for (int64_t j = nd[4]; j < (int64_t)nd[4] + nd[5]; ++j) {
            float d2 = dist2_f32(t->ps + 3 * j, t->geom + 4 * i);
            if (d2 > r2) r2 = d2;
        }
        t->geom[4 * i + 3] = r2;
    }
    return t;
}

/* Node dipoles D_t[c] = sum_{m in t} A_m mu_m[c] n_m in FP64 (eq.
 * farfield_dipole_features times A_t).  mu: [M][C] in caller order. */
int orc_tree_set_attrs(orc_tree *t, const float *mu, int C)
{
    if (!t || C < 1 || C > 64) return 1;
    free_stored(t);
    free(t->mu); free(t->D); free(t->W); free(t->Wm);
    t->C = C;
    t->mu = (double *)malloc(sizeof(double) * t->M * C);
    for (int64_t i = 0; i < t->M; ++i)
        for (int c = 0; c < C; ++c) t->mu[i * C + c] = (double)mu[(int64_t)t->perm[i] * C + c];
    t->D = (double *)calloc((size_t)t->N * C * 3, sizeof(double));
    t->W = (double *)calloc((size_t)t->N * C, sizeof(double));
    for (int64_t i = t->N - 1; i >= 0; --i) {
        const int32_t *nd = t->node + 6 * i;
        double *Di = t->D + i * C * 3, *Wi = t->W + i * C;
        if (nd[3] == 0) {
            for (int64_t j = nd[4]; j < (int64_t)nd[4] + nd[5]; ++j) {
                const double nn = norm3(t->nm + 3 * j);
                for (int c = 0; c < C; ++c) {
                    const double am = t->Am[j] * t->mu[j * C + c];
                    if (t->kind == 1) {
                        Di[3 * c] += am;
                        Wi[c] += fabs(am);
                        continue;
                    }
                    for (int k = 0; k < 3; ++k) Di[3 * c + k] += am * t->nm[3 * j + k];
                    Wi[c] += fabs(am) * nn;
                }
            }
        } else {
            for (int64_t ch = nd[2]; ch < (int64_t)nd[2] + nd[3]; ++ch) {
                for (int c = 0; c < 3 * C; ++c) Di[c] += t->D[ch * C * 3 + c];
                for (int c = 0; c < C; ++c) Wi[c] += t->W[ch * C + c];
            }
        }
    }
    t->Wm = (double *)malloc(sizeof(double) * (size_t)t->N * C);
    for (int64_t i = 0; i < t->N; ++i)
        for (int c = 0; c < C; ++c) t->Wm[i * C + c] = t->kind == 1 ? fabs(t->D[(i * C + c) * 3]) : norm3(t->D + (i * C + c) * 3);
    apply_storage(t);
    return 0;
}

/* 0: dipole kernel (default), 1: monopole kernel; refits the node moments */
int orc_tree_set_kind(orc_tree *t, int kind)
{
    if (!t || (kind != 0 && kind != 1)) return 1;
    t->kind = kind;
    if (!t->mu) return 0;
    float *tmp = (float *)malloc(sizeof(float) * t->M * t->C);
    for (int64_t i = 0; i < t->M; ++i)
        for (int c = 0; c < t->C; ++c) tmp[(int64_t)t->perm[i] * t->C + c] = (float)t->mu[i * t->C + c];
    int rc = orc_tree_set_attrs(t, tmp, t->C);
    free(tmp);
    return rc;
}

int64_t orc_tree_num_nodes(const orc_tree *t) { return t ? t->N : -1; }
int orc_tree_depth(const orc_tree *t) { return t ? t->depth : -1; }

/* Copies the canonical arrays out (any pointer may be NULL).
 * codes_in: [M] caller order; codes: [M] sorted; perm: [M];
 * nodes: [N][6]; geom: [N][4]; area: [N]; D: [N][C][3]; bounds: lo[3], side, scale. */
int orc_tree_export(const orc_tree *t, uint64_t *codes_in, uint64_t *codes, uint32_t *perm,
                    int32_t *nodes, float *geom, double *area, double *D, double *bounds,
                    int32_t *leaf_of)
{
    if (!t) return 1;
    int64_t M = t->M, N = t->N;
    if (codes_in) memcpy(codes_in, t->codes_in, sizeof(uint64_t) * M);
    if (codes) memcpy(codes, t->codes, sizeof(uint64_t) * M);
    if (perm) memcpy(perm, t->perm, sizeof(uint32_t) * M);
    if (nodes) memcpy(nodes, t->node, sizeof(int32_t) * 6 * N);
    if (geom) memcpy(geom, t->geom, sizeof(float) * 4 * N);
    if (area) memcpy(area, t->area, sizeof(double) * N);
    if (D && t->D) memcpy(D, t->D, sizeof(double) * N * t->C * 3);
    if (bounds) {
        bounds[0] = t->lo[0]; bounds[1] = t->lo[1]; bounds[2] = t->lo[2];
        bounds[3] = t->side; bounds[4] = t->scale;
    }
    if (leaf_of) memcpy(leaf_of, t->leaf_of, sizeof(int32_t) * M);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Barnes-Hut primal query (Algorithm 1, PrimalQuery)                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    const orc_tree *t;
    float b2;           /* beta*beta in FP32 */
    double eps;
    const float *xf;    /* query, FP32 */
    double x[3];
    double *f, *g, *sf, *sg;
    int32_t visits, far, leaves, near;
} qstate;

/* per-channel error scale of node i's far-field term */
static const double *node_scale(const orc_tree *t, int64_t i)
{
    return (t->scale_mode ? t->Wm : t->W) + i * t->C;
}

/* 0: absolute masses (the default), 1: moment magnitudes |D_t| (stricter
 * where a node's moment cancels) */
int orc_tree_set_scale(orc_tree *t, int mode)
{
    if (!t || (mode != 0 && mode != 1)) return 1;
    t->scale_mode = mode;
    return 0;
}

static int far_test(const orc_tree *t, int64_t i, const float *xf, float b2)
{
    const float *gm = t->geom + 4 * i;
    float s = dist2_f32(gm, xf);
    float lim = b2 * gm[3];
    return s > lim;
}

static void add_point(const orc_tree *t, int64_t j, const double x[3], double eps,
                      double *f, double *g, double *sf, double *sg)
{
    int C = t->C;
    double D[192], c[3];
    for (int k = 0; k < 3; ++k) c[k] = (double)t->ps[3 * j + k];
    if (t->kind == 1) {
        for (int ch = 0; ch < C; ++ch) D[3 * ch] = t->Am[j] * t->mus[j * C + ch];
        add_term_mono(c, D, NULL, C, x, eps, f, g, sf, sg);
        return;
    }
    for (int ch = 0; ch < C; ++ch)
        for (int k = 0; k < 3; ++k) D[3 * ch + k] = t->Am[j] * t->mus[j * C + ch] * t->nm[3 * j + k];
    add_term(c, D, NULL, C, x, eps, f, g, sf, sg);
}

static void primal(qstate *st, int64_t i)
{
    const orc_tree *t = st->t;
    const int32_t *nd = t->node + 6 * i;
    st->visits++;
    if (far_test(t, i, st->xf, st->b2)) {
        double c[3];
        for (int k = 0; k < 3; ++k) c[k] = (double)t->geom[4 * i + k];
        st->far++;
        if (t->kind == 1)
            add_term_mono(c, t->Ds + i * t->C * 3, node_scale(t, i), t->C, st->x, st->eps, st->f, st->g, st->sf, st->sg);
        else
            add_term(c, t->Ds + i * t->C * 3, node_scale(t, i), t->C, st->x, st->eps, st->f, st->g, st->sf, st->sg);
        return;
    }
    if (nd[3] == 0) {
        /* bucket leaf: every point of the leaf contributes its exact term */
        st->leaves++;
        for (int64_t j = nd[4]; j < (int64_t)nd[4] + nd[5]; ++j) {
            add_point(t, j, st->x, st->eps, st->f, st->g, st->sf, st->sg);
            st->near++;
        }
        return;
    }
    for (int64_t c = nd[2]; c < (int64_t)nd[2] + nd[3]; ++c) primal(st, c);
}

/* x: [Q][3] FP32.  Outputs FP64 (any may be NULL): f[Q][C], g[Q][C][3],
 * sf[Q][C], sg[Q][C]; counts[Q][4] = nodes visited (far tests evaluated),
 * nodes accepted as far field, leaves opened, points summed exactly. */
int orc_bh_query(const orc_tree *t, const float *x, int64_t Q, float beta, double eps,
                 double *f, double *g, double *sf, double *sg, int32_t *counts, int nthreads)
{
    if (!t || !t->Ds || Q < 0 || !(beta > 0) || eps < 0) return 1;
    int C = t->C;
    int nt = nthreads_or_default(nthreads);
    float b2 = beta * beta;
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t q = 0; q < Q; ++q) {
        double fl[64], gl[192], sfl[64], sgl[64];
        memset(fl, 0, sizeof fl); memset(gl, 0, sizeof gl);
        memset(sfl, 0, sizeof sfl); memset(sgl, 0, sizeof sgl);
        qstate st;
        memset(&st, 0, sizeof st);
        st.t = t; st.b2 = b2; st.eps = eps; st.xf = x + 3 * q;
        for (int k = 0; k < 3; ++k) st.x[k] = (double)x[3 * q + k];
        st.f = fl; st.g = gl; st.sf = sfl; st.sg = sgl;
        primal(&st, 0);
        for (int ch = 0; ch < C; ++ch) {
            if (f) f[q * C + ch] = fl[ch];
            if (sf) sf[q * C + ch] = sfl[ch];
            if (sg) sg[q * C + ch] = sgl[ch];
            if (g) for (int k = 0; k < 3; ++k) g[(q * C + ch) * 3 + k] = gl[3 * ch + k];
        }
        if (counts) {
            counts[4 * q] = st.visits; counts[4 * q + 1] = st.far;
            counts[4 * q + 2] = st.leaves; counts[4 * q + 3] = st.near;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Barnes-Hut adjoint query (Algorithm 1, AdjointQuery) + second stage       */
/* ------------------------------------------------------------------------ */

typedef struct {
    const orc_tree *t;
    float b2;
    double eps;
    const float *xf;
    double x[3];
    const double *df;   /* [C] or NULL */
    const double *dg;   /* [C][3] or NULL */
    double dx[3], sdx;
    double *G;          /* [N][C][3] node gradient accumulators */
    double *H;          /* [N][C] absolute scale of G */
    double *P;          /* [M][C] near-field point accumulators (sorted order) */
    double *HP;         /* [M][C] absolute scale of P */
    double *PN;         /* [M][3] near-field dL/dn accumulators, or NULL */
    double *HPN;        /* [M] absolute scale of PN */
    int want_eps;
    double deps, sdeps; /* dL/deps of this query and its absolute scale */
} astate;

static void adjoint(astate *st, int64_t i)
{
    const orc_tree *t = st->t;
    const int32_t *nd = t->node + 6 * i;
    int C = t->C;
    if (far_test(t, i, st->xf, st->b2)) {
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = (double)t->geom[4 * i + k] - st->x[k];
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double r = sqrt(r2), kap, lam;
        radial(r, st->eps, &kap, &lam);
        const double *Dt = t->Ds + i * C * 3;
        const double *Wt = node_scale(t, i);  /* the scales of the node's terms */
        if (t->kind == 1) {
            /* monopole: node accumulator df m(r), dx through the charges */
            if (r2 == 0.0) return;
            double m = kap * r, gv = r * lam - kap / r, w = 0, aw = 0;
            for (int ch = 0; ch < C; ++ch) {
                st->G[(i * C + ch) * 3] += st->df[ch] * m;
                st->H[i * C + ch] += fabs(st->df[ch]) * m;
                w += st->df[ch] * Dt[3 * ch];
                aw += fabs(st->df[ch]) * Wt[ch];
            }
            for (int k = 0; k < 3; ++k) st->dx[k] += w * gv * d[k];
            st->sdx += aw * fabs(gv) * r;
            return;
        }
        if (st->df) {
            double E[3] = {0, 0, 0};
            for (int ch = 0; ch < C; ++ch) {
                double w = st->df[ch] * kap;
                for (int k = 0; k < 3; ++k) {
                    st->G[(i * C + ch) * 3 + k] += w * d[k];
                    E[k] += st->df[ch] * Dt[3 * ch + k];
                }
                st->H[i * C + ch] += fabs(st->df[ch]) * kap * r;
                st->sdx += fabs(st->df[ch]) * Wt[ch] * (kap + fabs(lam) * r2);
            }
            double s = E[0] * d[0] + E[1] * d[1] + E[2] * d[2];
            for (int k = 0; k < 3; ++k) st->dx[k] += -kap * E[k] + lam * s * d[k];
        }
        if (st->dg) {
            double nu = radial_nu(r, st->eps);
            for (int ch = 0; ch < C; ++ch)
                grad_cotangent(d, r, kap, lam, nu, Dt + 3 * ch, Wt[ch], st->dg + 3 * ch,
                               st->G + (i * C + ch) * 3, st->dx, st->H + i * C + ch, &st->sdx);
        }
        if (st->want_eps) {
            double ke, le;
            radial_eps(r, st->eps, &ke, &le);
            for (int ch = 0; ch < C; ++ch)
                st->deps += term_eps(d, ke, le, Dt + 3 * ch, Wt[ch], st->df ? st->df[ch] : 0.0,
                                     st->dg ? st->dg + 3 * ch : NULL, &st->sdeps);
        }
        return;
    }
    if (nd[3] == 0) {
        for (int64_t j = nd[4]; j < (int64_t)nd[4] + nd[5]; ++j) {
            double d[3];
            for (int k = 0; k < 3; ++k) d[k] = (double)t->ps[3 * j + k] - st->x[k];
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 == 0.0 && st->eps == 0.0) continue;
            double r = sqrt(r2), kap, lam;
            radial(r, st->eps, &kap, &lam);
            if (t->kind == 1) {
                if (r2 == 0.0) continue;
                double m = kap * r, gv = r * lam - kap / r, w = 0, aw = 0;
                for (int ch = 0; ch < C; ++ch) {
                    st->P[j * C + ch] += st->df[ch] * t->Am[j] * m;
                    st->HP[j * C + ch] += fabs(st->df[ch]) * t->Am[j] * m;
                    w += st->df[ch] * t->mus[j * C + ch];
                    aw += fabs(st->df[ch] * t->mus[j * C + ch]);
                }
                for (int k = 0; k < 3; ++k) st->dx[k] += t->Am[j] * w * gv * d[k];
                st->sdx += t->Am[j] * aw * fabs(gv) * r;
                continue;
            }
            double An[3] = {t->Am[j] * t->nm[3 * j], t->Am[j] * t->nm[3 * j + 1], t->Am[j] * t->nm[3 * j + 2]};
            double s = An[0] * d[0] + An[1] * d[1] + An[2] * d[2];
            double nAn = sqrt(An[0] * An[0] + An[1] * An[1] + An[2] * An[2]);
            if (st->df) {
                double w = 0;
                for (int ch = 0; ch < C; ++ch) {
                    double mu = t->mus[j * C + ch];
                    st->P[j * C + ch] += st->df[ch] * kap * s;
                    st->HP[j * C + ch] += fabs(st->df[ch]) * kap * nAn * r;
                    w += st->df[ch] * mu;
                    st->sdx += fabs(st->df[ch]) * fabs(mu) * nAn * (kap + fabs(lam) * r2);
                }
                double Es = w * s;
                for (int k = 0; k < 3; ++k) st->dx[k] += -kap * w * An[k] + lam * Es * d[k];
            }
            if (st->dg) {
                double nu = radial_nu(r, st->eps);
                for (int ch = 0; ch < C; ++ch) {
                    double mu = t->mus[j * C + ch];
                    double D[3] = {mu * An[0], mu * An[1], mu * An[2]};
                    double dAn[3] = {0, 0, 0}, sc = 0;
                    /* derivative in the point's dipole, then through D = mu A n */
                    grad_cotangent(d, r, kap, lam, nu, D, -1.0, st->dg + 3 * ch, dAn, st->dx, &sc, &st->sdx);
                    st->P[j * C + ch] += An[0] * dAn[0] + An[1] * dAn[1] + An[2] * dAn[2];
                    st->HP[j * C + ch] += sc * nAn;
                }
            }
            if (st->PN) {
                /* dL/dn_j = A_j sum_c mu_jc dL/dD_jc of this query's term */
                double sc = 0;
                for (int ch = 0; ch < C; ++ch) {
                    double dD[3] = {0, 0, 0}, s1 = 0;
                    double w = st->df ? st->df[ch] : 0.0;
                    for (int k = 0; k < 3; ++k) dD[k] = w * kap * d[k];
                    s1 += fabs(w) * kap * r;
                    if (st->dg) {
                        const double *h = st->dg + 3 * ch;
                        double dh = d[0] * h[0] + d[1] * h[1] + d[2] * h[2];
                        for (int k = 0; k < 3; ++k) dD[k] += lam * dh * d[k] - kap * h[k];
                        s1 += sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]) * (fabs(lam) * r2 + kap);
                    }
                    double am = t->Am[j] * t->mus[j * C + ch];
                    for (int k = 0; k < 3; ++k) st->PN[3 * j + k] += am * dD[k];
                    sc += fabs(am) * s1;
                }
                st->HPN[j] += sc;
            }
            if (st->want_eps) {
                double ke, le;
                radial_eps(r, st->eps, &ke, &le);
                for (int ch = 0; ch < C; ++ch) {
                    double mu = t->mus[j * C + ch];
                    double D[3] = {mu * An[0], mu * An[1], mu * An[2]};
                    st->deps += term_eps(d, ke, le, D, -1.0, st->df ? st->df[ch] : 0.0,
                                         st->dg ? st->dg + 3 * ch : NULL, &st->sdeps);
                }
            }
        }
        return;
    }
    for (int64_t c = nd[2]; c < (int64_t)nd[2] + nd[3]; ++c) adjoint(st, c);
}

/* x: [Q][3] FP32, df: [Q][C] FP32 and/or dg: [Q][C][3] FP32 (either may be
 * NULL, not both).  Outputs FP64 (any may be NULL):
 * dmu[M][C] in caller point order, dx[Q][3], and the absolute scales
 * sdmu[M][C], sdx[Q] used to normalise errors.  Thread-private accumulators
 * are reduced in a fixed order, so the result is deterministic for a given
 * thread count. */
int orc_bh_adjoint(const orc_tree *t, const float *x, int64_t Q, float beta, double eps,
                   const float *df, const float *dg, double *dmu, double *dx, double *dn,
                   double *deps, double *sdmu, double *sdx, double *sdn, double *sdeps, int nthreads)
{
    if (!t || !t->Ds || Q < 0 || !(beta > 0) || eps < 0 || (!df && !dg)) return 1;
    if (t->kind == 1 && (dg || dn || deps || !df)) return 1;  /* value cotangents only */
    int C = t->C;
    int64_t N = t->N, M = t->M;
    int nt = nthreads_or_default(nthreads);
    float b2 = beta * beta;
    double *G = (double *)calloc((size_t)nt * N * C * 3, sizeof(double));
    double *H = (double *)calloc((size_t)nt * N * C, sizeof(double));
    double *P = (double *)calloc((size_t)nt * M * C, sizeof(double));
    double *HP = (double *)calloc((size_t)nt * M * C, sizeof(double));
    double *PN = dn ? (double *)calloc((size_t)nt * M * 3, sizeof(double)) : NULL;
    double *HPN = dn ? (double *)calloc((size_t)nt * M, sizeof(double)) : NULL;
    double *E = (double *)calloc((size_t)nt * 2, sizeof(double));
    if (!G || !H || !P || !HP || !E || (dn && (!PN || !HPN))) {
        free(G); free(H); free(P); free(HP); free(PN); free(HPN); free(E);
        return 2;
    }
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
#pragma omp for schedule(static)
        for (int64_t q = 0; q < Q; ++q) {
            double dfl[64], dgl[192];
            if (df) for (int ch = 0; ch < C; ++ch) dfl[ch] = (double)df[q * C + ch];
            if (dg) for (int v = 0; v < 3 * C; ++v) dgl[v] = (double)dg[q * C * 3 + v];
            astate st;
            memset(&st, 0, sizeof st);
            st.t = t; st.b2 = b2; st.eps = eps; st.xf = x + 3 * q;
            st.df = df ? dfl : NULL;
            st.dg = dg ? dgl : NULL;
            for (int k = 0; k < 3; ++k) st.x[k] = (double)x[3 * q + k];
            st.G = G + (size_t)tid * N * C * 3; st.H = H + (size_t)tid * N * C;
            st.P = P + (size_t)tid * M * C; st.HP = HP + (size_t)tid * M * C;
            st.PN = dn ? PN + (size_t)tid * M * 3 : NULL;
            st.HPN = dn ? HPN + (size_t)tid * M : NULL;
            st.want_eps = deps != NULL;
            adjoint(&st, 0);
            if (dx) for (int k = 0; k < 3; ++k) dx[3 * q + k] = st.dx[k];
            if (sdx) sdx[q] = st.sdx;
            E[2 * tid] += st.deps;
            E[2 * tid + 1] += st.sdeps;
        }
    }
    /* fixed-order reduction of the thread-private accumulators */
    for (int k = 1; k < nt; ++k) {
        for (int64_t i = 0; i < N * C * 3; ++i) G[i] += G[(size_t)k * N * C * 3 + i];
        for (int64_t i = 0; i < N * C; ++i) H[i] += H[(size_t)k * N * C + i];
        for (int64_t i = 0; i < M * C; ++i) {
            P[i] += P[(size_t)k * M * C + i];
            HP[i] += HP[(size_t)k * M * C + i];
        }
        if (dn) {
            for (int64_t i = 0; i < M * 3; ++i) PN[i] += PN[(size_t)k * M * 3 + i];
            for (int64_t i = 0; i < M; ++i) HPN[i] += HPN[(size_t)k * M + i];
        }
        E[0] += E[2 * k];
        E[1] += E[2 * k + 1];
    }
    if (deps) *deps = E[0];
    if (sdeps) *sdeps = E[1];
    /* second stage: running sums from the root down (parents precede
     * children in breadth-first order), then each point takes
     * A_m n_m . (sum over its ancestors) -- eq. (farfield_features_gradient) */
    for (int64_t i = 1; i < N; ++i) {
        int32_t par = t->node[6 * i + 1];
        for (int c = 0; c < C * 3; ++c) G[i * C * 3 + c] += G[(int64_t)par * C * 3 + c];
        for (int c = 0; c < C; ++c) H[i * C + c] += H[(int64_t)par * C + c];
    }
    for (int64_t j = 0; j < M; ++j) {
        int64_t l = t->leaf_of[j];
        int64_t orig = t->perm[j];
        double An[3] = {t->Am[j] * t->nm[3 * j], t->Am[j] * t->nm[3 * j + 1], t->Am[j] * t->nm[3 * j + 2]};
        double nAn = sqrt(An[0] * An[0] + An[1] * An[1] + An[2] * An[2]);
        for (int c = 0; c < C; ++c) {
            const double *S = G + (l * C + c) * 3;
            double v = t->kind == 1 ? P[j * C + c] + t->Am[j] * S[0]
                                    : P[j * C + c] + An[0] * S[0] + An[1] * S[1] + An[2] * S[2];
            if (dmu) dmu[orig * C + c] = v;
            if (sdmu) sdmu[orig * C + c] = HP[j * C + c] + (t->kind == 1 ? t->Am[j] : nAn) * H[l * C + c];
        }
        if (dn) {
            /* far field: every ancestor's node dipole holds A_j mu_jc n_j */
            double v[3] = {PN[3 * j], PN[3 * j + 1], PN[3 * j + 2]}, sc = HPN[j];
            for (int c = 0; c < C; ++c) {
                double am = t->Am[j] * t->mus[j * C + c];
                const double *S = G + (l * C + c) * 3;
                for (int k = 0; k < 3; ++k) v[k] += am * S[k];
                sc += fabs(am) * H[l * C + c];
            }
            for (int k = 0; k < 3; ++k) dn[3 * orig + k] = v[k];
            if (sdn) sdn[orig] = sc;
        }
    }
    free(G); free(H); free(P); free(HP); free(PN); free(HPN); free(E);
    return 0;
}
