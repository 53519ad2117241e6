/*
 * FP64 reference ("oracle") for the reverse ray tracer of Altay & Theuns,
 * "URCHIN: A Reverse Ray Tracer for Astrophysical Applications".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code with
 * the HIP library: every quantity is recomputed here from the paper's
 * definitions, serially per source particle (OpenMP only spreads independent
 * source particles over threads; the arithmetic of each is unchanged).
 *
 * Build: gcc -O2 -fPIC -shared -ffp-contract=off -fno-fast-math -mfma -fopenmp
 * (no implicit contraction: the segment-sphere predicate below must round
 * exactly like the device predicate, operation for operation; its fused
 * multiply-adds are written out as fma(), which IEEE 754 defines exactly).
 *
 * What is computed, by section of the paper:
 *  - G_t, the truncated Gaussian kernel and its constants (Sec. 4.1.1, eq. Gt)
 *  - line integrals of G_t along a clipped chord by adaptive Gauss-Kronrod
 *    quadrature (the definition behind the closed form I(h,b,z1,z2), Sec. 4.1.1)
 *  - HI columns along every ray: sum over *every* particle and every periodic
 *    image whose kernel sphere the ray segment enters (Sec. 4.1.1, eq. colden)
 *  - the shielded rate Gamma from the per-ray columns (Sec. 3.3, eq. gamma_shld)
 *  - the equilibrium neutral fraction, physical root x_- (Appendix C.3, eq. xroots)
 *  - the fixed-point iteration x -> tau -> Gamma -> x (Sec. 3.3 and Sec. 4)
 *  - a reference binary radix tree over 63-bit Morton keys, built top-down, for
 *    the bit-exact comparison of the device tree.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "oracle.h"

/* ------------------------------------------------------------------------- */
/* Kernel constants, Sec. 4.1.1 (eq. Gt): sigma^2 = h^2/(8 pi^(1/3)),          */
/* A^2 = 4 pi^(1/3)/h^2, t = 2 pi^(1/6), N = 8/(pi h^3) / [erf t - 2t e^-t^2/sqrt(pi)] */
/* ------------------------------------------------------------------------- */
static double c_t(void) { return 2.0 * pow(M_PI, 1.0 / 6.0); }
static double c_A2h2(void) { return 4.0 * pow(M_PI, 1.0 / 3.0); }
static double c_Nh3(void)
{
    double t = c_t();
    return (8.0 / M_PI) / (erf(t) - 2.0 * t * exp(-t * t) / sqrt(M_PI));
}

void orc_kernel_constants(double* out4)
{
    double t = c_t();
    out4[0] = t;                                 /* t                        */
    out4[1] = c_A2h2();                          /* A^2 h^2                  */
    out4[2] = sqrt(1.0 / (8.0 * pow(M_PI, 1.0 / 3.0)));  /* sigma / h        */
    out4[3] = c_Nh3();                           /* N h^3                    */
}

/* G_t(r; h): the truncated Gaussian, zero beyond r = h. */
double orc_Gt(double r, double h)
{
    if (r > h) return 0.0;
    double A2 = c_A2h2() / (h * h);
    return c_Nh3() / (h * h * h) * exp(-A2 * r * r);
}

/* M4 cubic spline with support h (Sec. 4.1.1, eq. spline). */
double orc_M4(double r, double h)
{
    double q = r / h, f;
    if (q <= 0.5) f = 1.0 - 6.0 * q * q + 6.0 * q * q * q;
    else if (q <= 1.0) f = 2.0 * (1.0 - q) * (1.0 - q) * (1.0 - q);
    else f = 0.0;
    return 8.0 / (M_PI * h * h * h) * f;
}

/* The printed closed form I(h,b,z1,z2) for the untruncated Gaussian between z1, z2. */
double orc_chord_closed(double h, double b, double z1, double z2)
{
    double A = sqrt(c_A2h2()) / h;
    double N = c_Nh3() / (h * h * h);
    return N * sqrt(M_PI) * exp(-A * A * b * b) / (2.0 * A) * (erf(A * z2) - erf(A * z1));
}

/* ------------------------------------------------------------------------- */
/* Adaptive Gauss-Kronrod (7-point Gauss / 15-point Kronrod) quadrature.      */
/* Nodes and weights are the standard published G7/K15 pair.                 */
/* ------------------------------------------------------------------------- */
static const double XGK[8] = {
    0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
    0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
    0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
    0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
static const double WGK[8] = {
    0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
    0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
    0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
    0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
static const double WG[4] = {
    0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
    0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

typedef double (*orc_fn)(double z, const double* prm);

static void gk15(orc_fn f, const double* prm, double a, double b, double* kr, double* err)
{
    double c = 0.5 * (a + b), hw = 0.5 * (b - a);
    double fc = f(c, prm);
    double rk = WGK[7] * fc, rg = WG[3] * fc;
    for (int i = 0; i < 7; ++i) {
        double dx = hw * XGK[i];
        double s = f(c - dx, prm) + f(c + dx, prm);
        rk += WGK[i] * s;
        if (i & 1) rg += WG[i / 2] * s;   /* odd Kronrod nodes are the Gauss nodes */
    }
    *kr = rk * hw;
    *err = fabs((rk - rg) * hw);
}

static double adapt(orc_fn f, const double* prm, double a, double b, double tol_abs, int depth)
{
    double k, e;
    gk15(f, prm, a, b, &k, &e);
    if (e <= tol_abs || depth >= 40) return k;
    double m = 0.5 * (a + b);
    return adapt(f, prm, a, m, 0.5 * tol_abs, depth + 1) +
           adapt(f, prm, m, b, 0.5 * tol_abs, depth + 1);
}

double orc_integrate(orc_fn f, const double* prm, double a, double b, double tol_abs)
{
    if (!(b > a)) return 0.0;
    return adapt(f, prm, a, b, tol_abs, 0);
}

/* integrand along the ray: G_t at distance sqrt(b^2 + z^2) from the centre */
static double chord_integrand(double z, const double* prm)
{
    /* prm[0] = h, prm[1] = b^2 */
    return orc_Gt(sqrt(prm[1] + z * z), prm[0]);
}

/* Line integral of G_t(.; h) at impact parameter^2 b2 from z1 to z2 (z along the
 * ray, measured from the point of closest approach), to relative accuracy rtol of
 * the full central chord.  Points beyond h contribute nothing (truncation). */
double orc_chord_quad(double h, double b2, double z1, double z2, double rtol)
{
    double prm[2] = {h, b2};
    double scale = c_Nh3() / (h * h);     /* order of the full central chord */
    return orc_integrate(chord_integrand, prm, z1, z2, rtol * scale);
}

/* Polynomial integrand for pinning the quadrature rule itself. */
static double poly_integrand(double z, const double* prm)
{
    return pow(z, prm[0]);
}

void orc_gk15_poly(double p, double a, double b, double* k15, double* err)
{
    double prm[1] = {p};
    gk15(poly_integrand, prm, a, b, k15, err);
}

static double shell_integrand(double r, const double* prm)
{
    /* prm[0] = h, prm[1] = 0 for G_t, 1 for M4 */
    return 4.0 * M_PI * r * r * (prm[1] == 0.0 ? orc_Gt(r, prm[0]) : orc_M4(r, prm[0]));
}

/* 4 pi int_0^h r^2 W(r) dr for W = G_t (which = 0) or M4 (which = 1). */
double orc_kernel_norm(double h, int32_t which)
{
    double prm[2] = {h, (double)which};
    /* M4 has a kink at h/2: integrate the two smooth pieces separately */
    return orc_integrate(shell_integrand, prm, 0.0, 0.5 * h, 1e-15) +
           orc_integrate(shell_integrand, prm, 0.5 * h, h, 1e-15);
}

/* ------------------------------------------------------------------------- */
/* Segment / kernel-sphere predicate.                                        */
/* d = (r_j - r_p) + s B, s_par = d.u, t = clamp(s_par, 0, L),               */
/* c = d - t u, hit <=> |c|^2 < h_j^2.  Fixed operation order: each dot     */
/* product starts with a product and adds the next terms by fused           */
/* multiply-add (x, then y, then z); each c component is one fused          */
/* multiply-add.                                                             */
/* ------------------------------------------------------------------------- */
static inline int seg_hit(const double d[3], const double u[3], double L, double h,
                          double* s_par)
{
    double sp = fma(d[2], u[2], fma(d[1], u[1], d[0] * u[0]));
    double t = sp < 0.0 ? 0.0 : (sp > L ? L : sp);
    double cx = fma(-t, u[0], d[0]);
    double cy = fma(-t, u[1], d[1]);
    double cz = fma(-t, u[2], d[2]);
    double D2 = fma(cz, cz, fma(cy, cy, cx * cx));
    *s_par = sp;
    return D2 < h * h;
}

/* Range of periodic image shifts along one axis that can bring a particle within
 * h_max of the segment's extent [smin, smax]; particles lie in [plo, phi]. */
static void image_range(double smin, double smax, double plo, double phi, double hmax,
                        double B, int* lo, int* hi)
{
    double a = (smin - hmax - phi) / B, b = (smax + hmax - plo) / B;
    *lo = (int)ceil(a - 1e-9);
    *hi = (int)floor(b + 1e-9);
}

/* The HI column contributed by particle j with offset d from the ray origin. */
static double hit_column(const double d[3], const double u[3], double sp, double L, double h,
                         double mux, double rtol)
{
    double px = d[0] - sp * u[0], py = d[1] - sp * u[1], pz = d[2] - sp * u[2];
    double b2 = px * px + py * py + pz * pz;           /* impact parameter^2   */
    double l2 = h * h - b2;
    double l = l2 > 0.0 ? sqrt(l2) : 0.0;              /* half chord in sphere */
    double z1 = (-sp > -l) ? -sp : -l;                 /* clip to the segment  */
    double z2 = (L - sp < l) ? L - sp : l;
    if (!(z2 > z1)) return 0.0;
    return mux * orc_chord_quad(h, b2, z1, z2, rtol);
}

/* Columns N[src][k] for selected source particles.  mu*x gives atoms/kpc_cm^2 and
 * the kernel integral is in kpc^-2, so N is in cm^-2.
 *   mode 0: count hits only (row_hits), no integrals
 *   mode 1: columns (N_out), optional hit lists written at row offsets row_off;
 *           with hit_fac, each hit's column per unit neutral fraction, mu_j
 *           times the clipped chord integral (dN/dx_j of that hit) */
int orc_columns(int64_t n, const float* pos, const float* h, const float* mu, const double* x,
                int32_t n_ray, const double* dirs, double L, double box,
                int64_t n_src, const int64_t* src, double rtol, int32_t mode,
                double* N_out, int64_t* row_hits, const int64_t* row_off,
                int32_t* hit_j, int32_t* hit_img, double* hit_fac, int32_t n_threads)
{
    if (n <= 0 || n_ray <= 0 || n_src < 0) return -1;
    double plo[3] = {INFINITY, INFINITY, INFINITY}, phi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double hmax = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        for (int a = 0; a < 3; ++a) {
            double v = pos[3 * j + a];
            if (v < plo[a]) plo[a] = v;
            if (v > phi[a]) phi[a] = v;
        }
        if (h[j] > hmax) hmax = h[j];
    }
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t si = 0; si < n_src; ++si) {
        int64_t p = src[si];
        double rp[3] = {pos[3 * p], pos[3 * p + 1], pos[3 * p + 2]};
        for (int k = 0; k < n_ray; ++k) {
            const double* u = dirs + 3 * k;
            int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
            if (box > 0.0) {
                for (int a = 0; a < 3; ++a) {
                    double e = rp[a] + L * u[a];
                    double smin = rp[a] < e ? rp[a] : e, smax = rp[a] < e ? e : rp[a];
                    image_range(smin, smax, plo[a], phi[a], hmax, box, &lo[a], &hi[a]);
                }
            }
            double col = 0.0;
            int64_t cnt = 0;
            int64_t w = row_off ? row_off[si * n_ray + k] : 0;
            for (int sx = lo[0]; sx <= hi[0]; ++sx)
            for (int sy = lo[1]; sy <= hi[1]; ++sy)
            for (int sz = lo[2]; sz <= hi[2]; ++sz) {
                double sh[3] = {(double)sx * box, (double)sy * box, (double)sz * box};
                if (box <= 0.0) sh[0] = sh[1] = sh[2] = 0.0;
                for (int64_t j = 0; j < n; ++j) {
                    double d[3];
                    for (int a = 0; a < 3; ++a)
                        d[a] = ((double)pos[3 * j + a] - rp[a]) + sh[a];
                    double sp;
                    double hj = (double)h[j];
                    if (!seg_hit(d, u, L, hj, &sp)) continue;
                    ++cnt;
                    if (mode == 1) {
                        col += hit_column(d, u, sp, L, hj, (double)mu[j] * x[j], rtol);
                        if (hit_j) {
                            hit_j[w] = (int32_t)j;
                            if (hit_img)
                                hit_img[w] = (sx + 8) | ((sy + 8) << 4) | ((sz + 8) << 8);
                            if (hit_fac)
                                hit_fac[w] = hit_column(d, u, sp, L, hj, (double)mu[j], rtol);
                            ++w;
                        }
                    }
                }
            }
            if (row_hits) row_hits[si * n_ray + k] = cnt;
            if (mode == 1 && N_out) N_out[si * n_ray + k] = col;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Non-equilibrium evolution at constant Gamma, T, nH (Appendix C.3, y = 0):    */
/* dx/dt = R (x - x_eq)(x - x_+) integrates to                                */
/*   x(t) = x_eq + (x0 - x_eq) (x_+ - x_eq) F / ((x_+ - x0) + (x0 - x_eq) F),  */
/*   F = exp(-(x_+ - x_eq) t / t_rc),  t_rc = 1 / ((alpha + gamma) nH),        */
/* with x_eq = x_- and x_+ the roots of eq. xroots.  In long double.           */
/* ------------------------------------------------------------------------- */
double orc_x_evolve(double x0, double Gamma, double nH, double alpha, double gcoll, double t)
{
    const long double n = nH, a = alpha, g = gcoll, G = Gamma;
    const long double R = (g + a) * n, P = a * n, negQ = G + a * n + R;
    const long double disc = negQ * negQ - 4.0L * P * R;
    const long double sq = sqrtl(disc > 0.0L ? disc : 0.0L);
    const long double xm = 2.0L * P / (negQ + sq);       /* x_- (Vieta form)        */
    const long double xp = (negQ + sq) / (2.0L * R);      /* x_+                      */
    const long double F = expl(-(xp - xm) * (long double)t * R);
    const long double d0 = (long double)x0 - xm;
    return (double)(xm + d0 * (xp - xm) * F / ((xp - (long double)x0) + d0 * F));
}

/* ------------------------------------------------------------------------- */
/* Near/far split (Sec. 4.1.2).  The near particles of source p are those that */
/* contribute to p's density in the scatter form of eq. nhi: the particle     */
/* image whose kernel sphere contains p, |d|^2 < h_j^2 with d as in the hit    */
/* predicate and |d|^2 summed x, y, z in FP64.  Per ray, N_far is the HI       */
/* column of the other particles the ray hits, and N_near the total hydrogen   */
/* column (every x = 1) of the near ones.                                     */
/* ------------------------------------------------------------------------- */
int orc_columns_near_far(int64_t n, const float* pos, const float* h, const float* mu,
                         const double* x, int32_t n_ray, const double* dirs, double L, double box,
                         int64_t n_src, const int64_t* src, double rtol, double* N_far,
                         double* N_near, int64_t* near_hits, int32_t n_threads)
{
    if (n <= 0 || n_ray <= 0 || n_src < 0) return -1;
    double plo[3] = {INFINITY, INFINITY, INFINITY}, phi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double hmax = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        for (int a = 0; a < 3; ++a) {
            double v = pos[3 * j + a];
            if (v < plo[a]) plo[a] = v;
            if (v > phi[a]) phi[a] = v;
        }
        if (h[j] > hmax) hmax = h[j];
    }
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t si = 0; si < n_src; ++si) {
        int64_t p = src[si];
        double rp[3] = {pos[3 * p], pos[3 * p + 1], pos[3 * p + 2]};
        for (int k = 0; k < n_ray; ++k) {
            const double* u = dirs + 3 * k;
            int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
            if (box > 0.0) {
                for (int a = 0; a < 3; ++a) {
                    double e = rp[a] + L * u[a];
                    double smin = rp[a] < e ? rp[a] : e, smax = rp[a] < e ? e : rp[a];
                    image_range(smin, smax, plo[a], phi[a], hmax, box, &lo[a], &hi[a]);
                }
            }
            double far = 0.0, near = 0.0;
            int64_t cnt = 0;
            for (int sx = lo[0]; sx <= hi[0]; ++sx)
            for (int sy = lo[1]; sy <= hi[1]; ++sy)
            for (int sz = lo[2]; sz <= hi[2]; ++sz) {
                double sh[3] = {(double)sx * box, (double)sy * box, (double)sz * box};
                if (box <= 0.0) sh[0] = sh[1] = sh[2] = 0.0;
                for (int64_t j = 0; j < n; ++j) {
                    double d[3];
                    for (int a = 0; a < 3; ++a)
                        d[a] = ((double)pos[3 * j + a] - rp[a]) + sh[a];
                    double sp;
                    double hj = (double)h[j];
                    if (!seg_hit(d, u, L, hj, &sp)) continue;
                    const double D0 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                    if (D0 < hj * hj) {
                        near += hit_column(d, u, sp, L, hj, (double)mu[j], rtol);
                        ++cnt;
                    } else {
                        far += hit_column(d, u, sp, L, hj, (double)mu[j] * x[j], rtol);
                    }
                }
            }
            N_far[si * n_ray + k] = far;
            N_near[si * n_ray + k] = near;
            if (near_hits) near_hits[si * n_ray + k] = cnt;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* The near particles as a uniform slab (Sec. 4.1.2, Appendix C.4): gas of     */
/* density nH (alpha, gamma at its T), lit by monochromatic radiation of       */
/* cross-section sigma that gives the rate Gamma0 at the surface.  At total    */
/* hydrogen column N into the slab the neutral fraction x satisfies            */
/*   sigma N = (1/x0 - 1/x) + ln[x(1-x0) / (x0(1-x))]                          */
/*           + (1/xce) ln[x(xce-x0) / (x0(xce-x))]                             */
/* (eq. analytic_slab_eqn), x0 the equilibrium at the surface, xce =          */
/* alpha/(alpha+gamma), and the rate there is Gamma = nH Xi(x)/x (eq.          */
/* slabone) with Xi = alpha(1-x)^2 - gamma(1-x)x = (alpha+gamma)(1-x)(xce-x).  */
/* Solved by bisection for v = ln(xce - x) in long double, so that thick       */
/* slabs, where xce - x underflows, stay representable.  Returns ln Gamma.     */
/* ------------------------------------------------------------------------- */
double orc_slab_lnG(double lnG0, double nH, double alpha, double gcoll, double sigma, double N)
{
    if (lnG0 == -INFINITY) return -INFINITY;
    const long double a = alpha, g = gcoll, xce = a / (a + g);
    const long double lg = (long double)lnG0 - logl((long double)nH);     /* ln(Gamma0/nH) */
    if (lg < -11000.0L) {
        /* rate too small to represent: x = xce through the slab */
        return (double)((long double)lnG0 - (long double)sigma * xce * (long double)N);
    }
    const long double G = expl(lg);
    /* surface root and xce - x0 without cancellation */
    const long double sD = sqrtl((G + g) * (G + g) + 4.0L * G * a);
    const long double x0 = 2.0L * a / (G + 2.0L * a + g + sD);
    const long double d0 = a * G * (1.0L + (G + 2.0L * g + 4.0L * a) / (sD + g)) /
                           ((a + g) * (G + 2.0L * a + g + sD));
    const long double v0 = logl(d0);
    const long double target = (long double)sigma * (long double)N;
    if (!(target > 0.0L)) return (double)((long double)lnG0);
    #define ORC_F(v, out) do {                                                  \
        const long double e_ = expl(v), xx_ = xce - e_;                          \
        out = (1.0L / x0 - 1.0L / xx_) + logl(xx_ * (1.0L - x0) / (x0 * (1.0L - xx_))) + \
              (logl(xx_ * d0 / x0) - (v)) / xce;                                 \
    } while (0)
    long double hi = v0, lo = v0 - xce * target - 64.0L, f;
    ORC_F(lo, f);
    while (f < target) { lo -= xce * target + 64.0L; ORC_F(lo, f); }
    for (int it = 0; it < 400; ++it) {
        const long double mid = 0.5L * (lo + hi);
        if (mid == lo || mid == hi) break;
        ORC_F(mid, f);
        if (f < target) hi = mid;
        else lo = mid;
    }
    #undef ORC_F
    const long double v = 0.5L * (lo + hi);
    const long double xs = xce - expl(v);
    return (double)(logl((long double)nH) + logl(a + g) + logl(1.0L - xs) + v - logl(xs));
}

/* Shielded rate of the near/far scheme for a monochromatic spectrum (one bin   */
/* w, sigma): per ray the far column attenuates the surface rate (eq.           */
/* gammafar) and the slab of the near particles lit by it gives Gamma_k (eq.    */
/* gammashldk).  share = 1 (the paper's weighting, eq. gammashld's 4 pi / N_ray  */
/* with 4 pi inside w): each slab is lit by the ray's share, (w sigma / N_ray)   */
/* exp(-sigma N_far), and Gamma = sum_k Gamma_k.  share = 0 (variant): each slab */
/* is lit by w sigma exp(-sigma N_far), as if the ray's radiation came from all  */
/* directions, and Gamma = (1/N_ray) sum_k Gamma_k.  ln Gamma by log-sum-exp.    */
void orc_gamma_near_far(int64_t n_src, int32_t n_ray, const double* N_far, const double* N_near,
                        double w, double sigma, const double* nH, const double* alpha,
                        const double* gcoll, double* lnG, int32_t share)
{
    const double lit = share ? w * sigma / (double)n_ray : w * sigma;
    const double mean = share ? 1.0 : 1.0 / (double)n_ray;
    for (int64_t i = 0; i < n_src; ++i) {
        double m = -INFINITY, s = 0.0;
        double* lk = (double*)malloc(sizeof(double) * n_ray);
        for (int k = 0; k < n_ray; ++k) {
            const double l0 = log(lit) - sigma * N_far[i * n_ray + k];
            lk[k] = orc_slab_lnG(l0, nH[i], alpha[i], gcoll[i], sigma, N_near[i * n_ray + k]);
            if (lk[k] > m) m = lk[k];
        }
        for (int k = 0; k < n_ray; ++k) s += exp(lk[k] - m);
        lnG[i] = (m == -INFINITY) ? -INFINITY : m + log(s * mean);
        free(lk);
    }
}

/* ------------------------------------------------------------------------- */
/* Polychromatic slab for the near/far scheme (Sec. 4.1.2, eq. gammashldk with  */
/* the slab of App. C.4 lit by a binned spectrum).  The slab is uniform (n_H,  */
/* alpha, gcoll of the source) and in equilibrium at every depth; the spectrum */
/* reaching HI column u below its surface has been attenuated by N_far + u, so */
/*   ln Gamma(u) = ln sum_b w_b sigma_b exp(-sigma_b (N_far + u)),             */
/*   x(u) = x_-(Gamma(u)),  and the total hydrogen column down to u is         */
/*   H(u) = int_0^u du' / x(u').                                               */
/* The bottom of the slab is where H(U) = N_near; the ray's rate is Gamma(U).   */
/* H by adaptive Gauss-Kronrod quadrature over geometric pieces, U by          */
/* bisection (H(u) >= u, so U lies in [0, N_near]).  One bin reproduces the    */
/* analytic slab above.                                                        */
/* prm: [0] n_bins, [1] N_far, [2] nH, [3] alpha, [4] gcoll, then ln(w sigma)   */
/* and sigma per bin.                                                          */
/* ------------------------------------------------------------------------- */
static double slab_poly_lnG_at(double N, const double* prm)
{
    const int nb = (int)prm[0];
    const double* lws = prm + 5;
    const double* sg = prm + 5 + nb;
    double m = -INFINITY;
    for (int b = 0; b < nb; ++b) {
        const double v = lws[b] - sg[b] * N;
        if (v > m) m = v;
    }
    if (m == -INFINITY) return m;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += exp(lws[b] - sg[b] * N - m);
    return m + log(s);
}

static double slab_poly_inv_x(double u, const double* prm)
{
    const double G = exp(slab_poly_lnG_at(prm[1] + u, prm));
    return 1.0 / orc_xeq(G, prm[2], prm[3], prm[4], 0.0);
}

double orc_slab_lnG_poly(int32_t n_bins, const double* sigma, const double* w, double N_far,
                         double nH, double alpha, double gcoll, double N_near)
{
    double* prm = (double*)malloc(sizeof(double) * (5 + 2 * (size_t)n_bins));
    if (!prm) return NAN;
    prm[0] = n_bins;
    prm[1] = N_far;
    prm[2] = nH;
    prm[3] = alpha;
    prm[4] = gcoll;
    double smax = 0.0;
    for (int b = 0; b < n_bins; ++b) {
        prm[5 + b] = w[b] > 0.0 ? log(w[b] * sigma[b]) : -INFINITY;
        prm[5 + n_bins + b] = sigma[b];
        if (w[b] > 0.0 && sigma[b] > smax) smax = sigma[b];
    }
    /* H is summed over pieces [u_{j-1}, u_j] with u_j = expm1(j / 20) / sigma_max, so
     * that Gamma, and with it 1/x, changes by a bounded factor within a piece;
     * each piece by adaptive quadrature to 1e-13 of a lower bound of its value
     * (1/x decreases with depth).  The piece where H reaches N_near is bisected. */
    double U = 0.0;
    if (N_near > 0.0) {
        const double u0 = 1.0 / smax;
        double lo = 0.0, H_lo = 0.0, hi = N_near;
        for (int j = 1;; ++j) {
            const double b = fmin(u0 * expm1(0.05 * j), N_near);
            const double tol = 1e-13 * (b - lo) * slab_poly_inv_x(b, prm);
            const double I = orc_integrate(slab_poly_inv_x, prm, lo, b, tol);
            if (H_lo + I >= N_near || b >= N_near) {
                hi = b;
                break;
            }
            H_lo += I;
            lo = b;
        }
        for (int it = 0; it < 400; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            const double tol = 1e-13 * (mid - lo) * slab_poly_inv_x(mid, prm);
            const double Hm = H_lo + orc_integrate(slab_poly_inv_x, prm, lo, mid, tol);
            if (Hm < N_near) {
                lo = mid;
                H_lo = Hm;
            } else {
                hi = mid;
            }
        }
        U = 0.5 * (lo + hi);
    }
    const double out = slab_poly_lnG_at(N_far + U, prm);
    free(prm);
    return out;
}

/* Near/far shielded rate for a binned spectrum: per ray the polychromatic slab */
/* above, lit by the ray's share w / N_ray of the spectrum with Gamma = sum_k    */
/* Gamma_k (share = 1, eq. gammashld with 4 pi inside w), or by w with Gamma =   */
/* (1/N_ray) sum_k Gamma_k (share = 0, variant); ln by log-sum-exp.             */
void orc_gamma_near_far_poly(int64_t n_src, int32_t n_ray, const double* N_far,
                             const double* N_near, int32_t n_bins, const double* sigma,
                             const double* w, const double* nH, const double* alpha,
                             const double* gcoll, double* lnG, int32_t n_threads, int32_t share)
{
    const double mean = share ? 1.0 : 1.0 / (double)n_ray;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    double* lit = (double*)malloc(sizeof(double) * (size_t)n_bins);
    for (int b = 0; b < n_bins; ++b) lit[b] = share ? w[b] / (double)n_ray : w[b];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n_src; ++i) {
        double m = -INFINITY, s = 0.0;
        double* lk = (double*)malloc(sizeof(double) * n_ray);
        for (int k = 0; k < n_ray; ++k) {
            lk[k] = orc_slab_lnG_poly(n_bins, sigma, lit, N_far[i * n_ray + k], nH[i],
                                      alpha[i], gcoll[i], N_near[i * n_ray + k]);
            if (lk[k] > m) m = lk[k];
        }
        for (int k = 0; k < n_ray; ++k) s += exp(lk[k] - m);
        lnG[i] = (m == -INFINITY) ? -INFINITY : m + log(s * mean);
        free(lk);
    }
    free(lit);
}

/* ------------------------------------------------------------------------- */
/* Shielded photoionisation rate, Sec. 3.3 eq. gamma_shld with the frequency  */
/* integral done over bins: Gamma = (1/N_ray) sum_k sum_b w_b sigma_b         */
/* exp(-sigma_b N_k).  ln Gamma by a log-sum-exp over all (k, b) terms.       */
/* ------------------------------------------------------------------------- */
void orc_gamma(int64_t n_src, int32_t n_ray, const double* N, int32_t n_bins,
               const double* sigma, const double* w, double* lnG, double* G, double* tau)
{
    double thin = 0.0;
    for (int b = 0; b < n_bins; ++b) thin += w[b] * sigma[b];
    double lnthin = log(thin);
    for (int64_t p = 0; p < n_src; ++p) {
        double m = -INFINITY;
        for (int k = 0; k < n_ray; ++k)
            for (int b = 0; b < n_bins; ++b) {
                double v = log(w[b] * sigma[b]) - sigma[b] * N[p * n_ray + k];
                if (v > m) m = v;
            }
        double s = 0.0;
        for (int k = 0; k < n_ray; ++k)
            for (int b = 0; b < n_bins; ++b)
                s += exp(log(w[b] * sigma[b]) - sigma[b] * N[p * n_ray + k] - m);
        double l = m + log(s) - log((double)n_ray);
        if (lnG) lnG[p] = l;
        if (G) G[p] = exp(l);
        if (tau) tau[p] = lnthin - l;
    }
}

/* ------------------------------------------------------------------------- */
/* Rates.  The paper defers to published fits (Appendix C.3); this reading    */
/* takes the Hui & Gnedin (1997) case A / case B recombination fits and the   */
/* Cen (1992) collisional ionisation fit, all in cm^3 s^-1.                   */
/* ------------------------------------------------------------------------- */
double orc_alpha_A(double T)
{
    double lam = 2.0 * 157807.0 / T;
    return 1.269e-13 * pow(lam, 1.503) / pow(1.0 + pow(lam / 0.522, 0.470), 1.923);
}

double orc_alpha_B(double T)
{
    double lam = 2.0 * 157807.0 / T;
    return 2.753e-14 * pow(lam, 1.500) / pow(1.0 + pow(lam / 2.740, 0.407), 2.242);
}

double orc_gamma_coll(double T)
{
    return 5.85e-11 * sqrt(T) * exp(-157809.1 / T) / (1.0 + sqrt(T / 1e5));
}

/* Physical root x_- of R x^2 + Q x + P = 0 (Appendix C.3, eq. xroots) with
 * R = (gamma + alpha) n_H, Q = -[Gamma + alpha n_H + R (1 + y)],
 * P = alpha n_H (1 + y).  Evaluated as 2P / (-Q + sqrt(Q^2 - 4PR)), which equals
 * (-Q - sqrt(Q^2 - 4PR)) / (2R) exactly (Vieta) without its cancellation. */
double orc_xeq(double Gamma, double nH, double alpha, double gcoll, double y)
{
    double R = (gcoll + alpha) * nH;
    double Q = -(Gamma + alpha * nH + R * (1.0 + y));
    double P = alpha * nH * (1.0 + y);
    double D = Q * Q - 4.0 * P * R;
    if (D < 0.0) D = 0.0;
    return 2.0 * P / (-Q + sqrt(D));
}

/* ------------------------------------------------------------------------- */
/* The fixed point (Sec. 3.3, Sec. 4): x0 = x_thin (or x_init); each iteration */
/* computes every column from the current x, then Gamma, then every x at once  */
/* (the order-independent update the paper describes for parallel use).       */
/* Stops when max|dx| < tol or after max_iter iterations.                      */
/* ------------------------------------------------------------------------- */
int orc_solve(int64_t n, const float* pos, const float* h, const float* mu, const float* nH,
              const float* T, int32_t n_ray, const double* dirs, int32_t n_bins,
              const double* sigma, const double* w, double L, double box, double tol,
              int32_t max_iter, const double* x_init, double rtol, int32_t n_threads,
              double* x_hist /*[(max_iter+1)][n]*/, double* lnG_hist /*[max_iter][n]*/,
              double* N_last /*[n][n_ray]*/, int32_t* iters_done, double* maxdx_hist)
{
    double thin = 0.0;
    for (int b = 0; b < n_bins; ++b) thin += w[b] * sigma[b];
    double* x = (double*)malloc(sizeof(double) * n);
    double* Nc = (double*)malloc(sizeof(double) * n * n_ray);
    double* lnG = (double*)malloc(sizeof(double) * n);
    double* G = (double*)malloc(sizeof(double) * n);
    int64_t* src = (int64_t*)malloc(sizeof(int64_t) * n);
    double* al = (double*)malloc(sizeof(double) * n);
    double* ga = (double*)malloc(sizeof(double) * n);
    if (!x || !Nc || !lnG || !G || !src || !al || !ga) return -2;
    for (int64_t p = 0; p < n; ++p) {
        src[p] = p;
        al[p] = orc_alpha_A((double)T[p]);
        ga[p] = orc_gamma_coll((double)T[p]);
        x[p] = x_init ? x_init[p] : orc_xeq(thin, (double)nH[p], al[p], ga[p], 0.0);
    }
    if (x_hist) memcpy(x_hist, x, sizeof(double) * n);
    int it = 0;
    for (it = 0; it < max_iter; ++it) {
        orc_columns(n, pos, h, mu, x, n_ray, dirs, L, box, n, src, rtol, 1, Nc, NULL, NULL,
                    NULL, NULL, NULL, n_threads);
        orc_gamma(n, n_ray, Nc, n_bins, sigma, w, lnG, G, NULL);
        double mdx = 0.0;
        for (int64_t p = 0; p < n; ++p) {
            double xn = orc_xeq(G[p], (double)nH[p], al[p], ga[p], 0.0);
            double dx = fabs(xn - x[p]);
            if (dx > mdx) mdx = dx;
            x[p] = xn;
        }
        if (x_hist) memcpy(x_hist + (size_t)(it + 1) * n, x, sizeof(double) * n);
        if (lnG_hist) memcpy(lnG_hist + (size_t)it * n, lnG, sizeof(double) * n);
        if (maxdx_hist) maxdx_hist[it] = mdx;
        if (mdx < tol) { ++it; break; }
    }
    if (N_last) memcpy(N_last, Nc, sizeof(double) * n * n_ray);
    if (iters_done) *iters_done = it;
    free(x); free(Nc); free(lnG); free(G); free(src); free(al); free(ga);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* The paper's own update rule (Sec. 4, implementation details):              */
/*  - every particle starts at its optically thin neutral fraction;           */
/*  - particles whose first shielded rate gives tau_eff < tau_skip keep that  */
/*    value for good and are not traced again;                               */
/*  - case B recombination for particles with tau_eff >= tau_case_b (case A  */
/*    otherwise; +inf = case A throughout);                                  */
/*  - convergence on max |dx| (relative != 0: max |dx| / x) < tol;           */
/*  - particles are visited from high to low density (ties: lower index      */
/*    first) in n_blocks consecutive blocks: each block's rates see every    */
/*    update of the blocks before it in the same sweep.  n_blocks = 1 is the */
/*    order-independent update, n_blocks = n updates one particle at a time. */
/* lnG_hist[it][p] holds the most recent rate of p after sweep it; skipped   */
/* receives 1 for the particles that stopped after their first rate.         */
/* ------------------------------------------------------------------------- */
static const float* g_sort_nH;
static int cmp_density_desc(const void* a, const void* b)
{
    const int64_t i = *(const int64_t*)a, j = *(const int64_t*)b;
    const float ni = g_sort_nH[i], nj = g_sort_nH[j];
    if (ni > nj) return -1;
    if (ni < nj) return 1;
    return (i > j) - (i < j);
}

int orc_solve_rule(int64_t n, const float* pos, const float* h, const float* mu, const float* nH,
                   const float* T, int32_t n_ray, const double* dirs, int32_t n_bins,
                   const double* sigma, const double* w, double L, double box, double tol,
                   int32_t max_iter, double tau_skip, double tau_case_b, int32_t relative,
                   int32_t n_blocks, double rtol, int32_t n_threads,
                   double* x_hist /*[(max_iter+1)][n]*/, double* lnG_hist /*[max_iter][n]*/,
                   int32_t* skipped /*[n]*/, int32_t* iters_done, double* maxdx_hist)
{
    if (n_blocks < 1 || n_blocks > n) return -1;
    double thin = 0.0;
    for (int b = 0; b < n_bins; ++b) thin += w[b] * sigma[b];
    double* x = (double*)malloc(sizeof(double) * n);
    double* lnG_all = (double*)malloc(sizeof(double) * n);
    double* al = (double*)malloc(sizeof(double) * n);
    double* alB = (double*)malloc(sizeof(double) * n);
    double* ga = (double*)malloc(sizeof(double) * n);
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * n);
    int64_t* src = (int64_t*)malloc(sizeof(int64_t) * n);
    int32_t* skip = (int32_t*)calloc((size_t)n, sizeof(int32_t));
    const int64_t bs = (n + n_blocks - 1) / n_blocks;
    double* Nc = (double*)malloc(sizeof(double) * bs * n_ray);
    double* lnG = (double*)malloc(sizeof(double) * bs);
    double* G = (double*)malloc(sizeof(double) * bs);
    double* tau = (double*)malloc(sizeof(double) * bs);
    if (!x || !lnG_all || !al || !alB || !ga || !order || !src || !skip || !Nc || !lnG || !G ||
        !tau)
        return -2;
    for (int64_t p = 0; p < n; ++p) {
        order[p] = p;
        al[p] = orc_alpha_A((double)T[p]);
        alB[p] = orc_alpha_B((double)T[p]);
        ga[p] = orc_gamma_coll((double)T[p]);
        x[p] = orc_xeq(thin, (double)nH[p], al[p], ga[p], 0.0);
        lnG_all[p] = log(thin);
    }
    g_sort_nH = nH;
    qsort(order, (size_t)n, sizeof(int64_t), cmp_density_desc);
    if (x_hist) memcpy(x_hist, x, sizeof(double) * n);
    int it = 0;
    for (it = 0; it < max_iter; ++it) {
        double mdx = 0.0;
        for (int64_t b0 = 0; b0 < n; b0 += bs) {
            const int64_t b1 = b0 + bs < n ? b0 + bs : n;
            int64_t m = 0;
            for (int64_t q = b0; q < b1; ++q)
                if (!skip[order[q]]) src[m++] = order[q];
            if (m == 0) continue;
            orc_columns(n, pos, h, mu, x, n_ray, dirs, L, box, m, src, rtol, 1, Nc, NULL, NULL,
                        NULL, NULL, NULL, n_threads);
            orc_gamma(m, n_ray, Nc, n_bins, sigma, w, lnG, G, tau);
            for (int64_t i = 0; i < m; ++i) {
                const int64_t p = src[i];
                lnG_all[p] = lnG[i];
                if (it == 0 && tau[i] < tau_skip) {
                    skip[p] = 1;
                    continue;
                }
                const double a = tau[i] >= tau_case_b ? alB[p] : al[p];
                const double xn = orc_xeq(G[i], (double)nH[p], a, ga[p], 0.0);
                double dx = fabs(xn - x[p]);
                if (relative) dx /= x[p];
                if (dx > mdx) mdx = dx;
                x[p] = xn;
            }
        }
        if (x_hist) memcpy(x_hist + (size_t)(it + 1) * n, x, sizeof(double) * n);
        if (lnG_hist) memcpy(lnG_hist + (size_t)it * n, lnG_all, sizeof(double) * n);
        if (maxdx_hist) maxdx_hist[it] = mdx;
        if (mdx < tol) { ++it; break; }
    }
    if (skipped) memcpy(skipped, skip, sizeof(int32_t) * n);
    if (iters_done) *iters_done = it;
    free(x); free(lnG_all); free(al); free(alB); free(ga); free(order); free(src); free(skip);
    free(Nc); free(lnG); free(G); free(tau);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Reference radix tree.  Keys: 63-bit Morton codes (21 bits per axis, x in   */
/* the highest position of each triple) of positions quantised over the      */
/* cube of side max extent anchored at the minimum corner; ties broken by the */
/* position in the sorted order.  Built top-down: a range splits where the    */
/* highest differing bit of its first and last (key, position) changes.      */
/* Ranges of at most leaf_max particles become leaves.  Nodes are emitted in  */
/* depth-first pre-order; skip = index of the first node after the subtree.   */
/* Boxes are exact FP32 min/max of (r - h, r + h).                            */
/*                                                                           */
/* Independent halos in one tree: with H > 1 halos (particles               */
/* [off[g], off[g+1]) of the input form halo g) the key of a particle of     */
/* halo g is g in the bits above the Morton code, which takes               */
/* b = floor((63 - ceil(log2 H)) / 3) bits per axis, quantised over the same */
/* cube; and a range becomes a leaf only when it also lies in one halo.  So  */
/* every halo owns one subtree, whose root is the topmost node whose range   */
/* is exactly that halo's particles.                                         */
/* ------------------------------------------------------------------------- */
static uint64_t spread_bits(uint64_t v, int bits)
{
    uint64_t r = 0;
    for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1ull) << (3 * i);
    return r;
}

static int halo_key_bits(int32_t n_halo)
{
    int hb = 0;
    while (((int64_t)1 << hb) < (int64_t)n_halo) ++hb;     /* ceil(log2 H) */
    return n_halo > 1 ? (63 - hb) / 3 : 21;
}

void orc_morton_seg(int64_t n, const float* pos, int32_t n_halo, const int64_t* halo_off,
                    uint64_t* codes)
{
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t j = 0; j < n; ++j)
        for (int a = 0; a < 3; ++a) {
            float v = pos[3 * j + a];
            if (v < lo[a]) lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) {
        double e = (double)hi[a] - (double)lo[a];
        if (e > ext) ext = e;
    }
    const int bits = halo_key_bits(n_halo);
    const double cells = (double)((uint64_t)1 << bits);
    double scale = ext > 0.0 ? cells / ext : 0.0;
    int32_t g = 0;
    for (int64_t j = 0; j < n; ++j) {
        uint64_t q[3];
        for (int a = 0; a < 3; ++a) {
            double v = floor(((double)pos[3 * j + a] - (double)lo[a]) * scale);
            if (v < 0.0) v = 0.0;
            if (v > cells - 1.0) v = cells - 1.0;
            q[a] = (uint64_t)v;
        }
        uint64_t key = (spread_bits(q[0], bits) << 2) | (spread_bits(q[1], bits) << 1) |
                       spread_bits(q[2], bits);
        if (n_halo > 1) {
            while (g + 1 < n_halo && j >= halo_off[g + 1]) ++g;
            key |= (uint64_t)g << (3 * bits);
        }
        codes[j] = key;
    }
}

void orc_morton(int64_t n, const float* pos, uint64_t* codes)
{
    orc_morton_seg(n, pos, 1, NULL, codes);
}

typedef struct { uint64_t code; int64_t idx; } keyidx;

static int cmp_keyidx(const void* a, const void* b)
{
    const keyidx* x = (const keyidx*)a;
    const keyidx* y = (const keyidx*)b;
    if (x->code != y->code) return x->code < y->code ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

typedef struct {
    const uint64_t* code;  /* sorted codes */
    const float* pos;      /* sorted positions [n][3] */
    const float* h;        /* sorted h */
    int64_t n;
    int32_t leaf_max;
    int halo_shift;        /* the halo field starts at this bit; 64 = one problem */
    int64_t cnt;
    float* lo; float* hi;
    int32_t* skip; int32_t* first; int32_t* count;
    int32_t* seg_root; int32_t* seg_end;   /* per halo, or NULL */
} tree_ctx;

static int64_t split_of(const tree_ctx* c, int64_t f, int64_t l)
{
    uint64_t a = c->code[f], b = c->code[l];
    if (a != b) {
        int bit = 63 - __builtin_clzll(a ^ b);
        /* last position in [f, l] whose code has this bit clear */
        int64_t s = f;
        for (int64_t i = f; i <= l; ++i)
            if (((c->code[i] >> bit) & 1ull) == 0) s = i;
        return s;
    }
    int bit = 63 - __builtin_clzll((uint64_t)(f ^ l));
    return ((l >> bit) << bit) - 1;
}

static uint64_t halo_of_code(const tree_ctx* c, uint64_t code)
{
    return c->halo_shift >= 64 ? 0 : code >> c->halo_shift;
}

static void build_rec(tree_ctx* c, int64_t f, int64_t l)
{
    int64_t me = c->cnt++;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = f; i <= l; ++i)
        for (int a = 0; a < 3; ++a) {
            float x = c->pos[3 * i + a], hh = c->h[i];
            float m0 = x - hh, m1 = x + hh;
            if (m0 < lo[a]) lo[a] = m0;
            if (m1 > hi[a]) hi[a] = m1;
        }
    for (int a = 0; a < 3; ++a) { c->lo[3 * me + a] = lo[a]; c->hi[3 * me + a] = hi[a]; }
    int64_t n = l - f + 1;
    const uint64_t gf = halo_of_code(c, c->code[f]), gl = halo_of_code(c, c->code[l]);
    /* the topmost range that is exactly one halo roots that halo's subtree */
    const int whole_halo = gf == gl && (f == 0 || halo_of_code(c, c->code[f - 1]) != gf) &&
                           (l == c->n - 1 || halo_of_code(c, c->code[l + 1]) != gl);
    if (c->seg_root && whole_halo && c->seg_root[gf] < 0) c->seg_root[gf] = (int32_t)me;
    if (n <= c->leaf_max && gf == gl) {
        c->first[me] = (int32_t)f;
        c->count[me] = (int32_t)n;
    } else {
        int64_t s = split_of(c, f, l);
        c->first[me] = (int32_t)f;
        c->count[me] = 0;                 /* internal */
        build_rec(c, f, s);
        build_rec(c, s + 1, l);
    }
    c->skip[me] = (int32_t)c->cnt;
    if (c->seg_root && whole_halo && c->seg_root[gf] == (int32_t)me)
        c->seg_end[gf] = (int32_t)c->cnt;
}

/* Outputs: perm[n] (sorted position -> original index), codes_sorted[n],
 * node arrays sized for 2n - 1 nodes, and with H > 1 halos seg_root[H] and
 * seg_end[H] (each halo's subtree is nodes [root, end)).  Returns the node
 * count, or -1 on bad arguments. */
int64_t orc_lbvh_seg(int64_t n, const float* pos, const float* h, int32_t leaf_max,
                     int32_t n_halo, const int64_t* halo_off, int32_t* perm,
                     uint64_t* codes_sorted, float* node_lo, float* node_hi, int32_t* node_skip,
                     int32_t* node_first, int32_t* node_count, int32_t* seg_root,
                     int32_t* seg_end)
{
    if (n <= 0 || leaf_max < 1 || n_halo < 1) return -1;
    if (n_halo > 1) {
        if (!halo_off || halo_off[0] != 0 || halo_off[n_halo] != n) return -1;
        for (int32_t g = 0; g < n_halo; ++g)
            if (halo_off[g + 1] <= halo_off[g]) return -1;
    }
    uint64_t* codes = (uint64_t*)malloc(sizeof(uint64_t) * n);
    keyidx* ki = (keyidx*)malloc(sizeof(keyidx) * n);
    float* sp = (float*)malloc(sizeof(float) * 3 * n);
    float* sh = (float*)malloc(sizeof(float) * n);
    orc_morton_seg(n, pos, n_halo, halo_off, codes);
    for (int64_t j = 0; j < n; ++j) { ki[j].code = codes[j]; ki[j].idx = j; }
    qsort(ki, (size_t)n, sizeof(keyidx), cmp_keyidx);
    for (int64_t i = 0; i < n; ++i) {
        int64_t j = ki[i].idx;
        perm[i] = (int32_t)j;
        codes_sorted[i] = ki[i].code;
        sp[3 * i] = pos[3 * j]; sp[3 * i + 1] = pos[3 * j + 1]; sp[3 * i + 2] = pos[3 * j + 2];
        sh[i] = h[j];
    }
    const int segmented = n_halo > 1 && seg_root && seg_end;
    if (segmented)
        for (int32_t g = 0; g < n_halo; ++g) seg_root[g] = seg_end[g] = -1;
    tree_ctx c = {codes_sorted, sp, sh, n, leaf_max, n_halo > 1 ? 3 * halo_key_bits(n_halo) : 64,
                  0, node_lo, node_hi, node_skip, node_first, node_count,
                  segmented ? seg_root : NULL, segmented ? seg_end : NULL};
    build_rec(&c, 0, n - 1);
    free(codes); free(ki); free(sp); free(sh);
    return c.cnt;
}

int64_t orc_lbvh(int64_t n, const float* pos, const float* h, int32_t leaf_max,
                 int32_t* perm, uint64_t* codes_sorted, float* node_lo, float* node_hi,
                 int32_t* node_skip, int32_t* node_first, int32_t* node_count)
{
    return orc_lbvh_seg(n, pos, h, leaf_max, 1, NULL, perm, codes_sorted, node_lo, node_hi,
                        node_skip, node_first, node_count, NULL, NULL);
}
