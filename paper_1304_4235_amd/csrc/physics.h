// Device-side physics shared by the rate, equilibrium and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace rrt {

// Case A recombination coefficient (Hui & Gnedin 1997 fit), cm^3 s^-1.
__device__ __forceinline__ double alpha_caseA(double T)
{
    double lam = 2.0 * 157807.0 / T;
    return 1.269e-13 * pow(lam, 1.503) / pow(1.0 + pow(lam / 0.522, 0.470), 1.923);
}

// Case B recombination coefficient (Hui & Gnedin 1997 fit), cm^3 s^-1.
__device__ __forceinline__ double alpha_caseB(double T)
{
    const double lam = 2.0 * 157807.0 / T;
    return 2.753e-14 * pow(lam, 1.5) / pow(1.0 + pow(lam / 2.74, 0.407), 2.242);
}

// Collisional ionisation coefficient (Cen 1992 fit), cm^3 s^-1.
__device__ __forceinline__ double gamma_collisional(double T)
{
    return 5.85e-11 * sqrt(T) * exp(-157809.1 / T) / (1.0 + sqrt(T * 1e-5));
}

// Discriminant of R x^2 + Q x + P with y = 0, written as
// D = (Gamma + gamma n_H)^2 + 4 Gamma alpha n_H  (= Q^2 - 4PR, no cancellation).
__device__ __forceinline__ double eq_discriminant(double G, double nH, double al, double gc)
{
    double s = G + gc * nH;
    return s * s + 4.0 * G * al * nH;
}

// Physical root x_- = 2P / (-Q + sqrt(D)) (Appendix C.3, eq. xroots).
__device__ __forceinline__ double x_minus(double G, double nH, double al, double gc)
{
    double P = al * nH;
    double R = (gc + al) * nH;
    double negQ = G + P + R;
    return 2.0 * P / (negQ + sqrt(eq_discriminant(G, nH, al, gc)));
}

// x after time t at constant Gamma, nH and coefficients, from x0 (Appendix
// C.3, y = 0): dx/dt = R (x - x_-)(x - x_+) with R = (alpha + gcoll) nH gives
// x(t) = x_- + (x0 - x_-) (x_+ - x_-) F / ((x_+ - x0) + (x0 - x_-) F) with
// F = exp(-R (x_+ - x_-) t); x_+ - x_- = sqrt(D) / R.
__device__ __forceinline__ double x_after(double x0, double G, double nH, double al, double gc,
                                          double t)
{
    const double R = (gc + al) * nH;
    const double sD = sqrt(eq_discriminant(G, nH, al, gc));
    const double xm = x_minus(G, nH, al, gc);
    const double gap = sD / R;                       // x_+ - x_-
    const double F = exp(-sD * t);
    const double d0 = x0 - xm;
    return xm + d0 * gap * F / ((xm + gap - x0) + d0 * F);
}

// ln of the photoionisation rate at total hydrogen column N into a uniform
// slab of density nH (coefficients alpha, gcoll at its temperature) lit by
// monochromatic radiation of cross-section sigma that gives the rate
// exp(lnG0) at the surface (Appendix C.4): the depth of neutral fraction x is
//   sigma N = (1/x0 - 1/x) + ln[x(1-x0)/(x0(1-x))] + (1/xce) ln[x(xce-x0)/(x0(xce-x))]
// and the rate there nH (alpha+gcoll)(1-x)(xce-x)/x.  Newton's method on
// v = ln(xce - x), kept inside a shrinking bracket, so thick slabs (where
// xce - x underflows) stay finite in ln Gamma.
__device__ inline double slab_ln_rate(double lnG0, double nH, double alpha, double gcoll,
                                      double sigma, double N)
{
    if (lnG0 == -INFINITY) return -INFINITY;
    const double xce = alpha / (alpha + gcoll);
    const double target = sigma * N;
    const double lg = lnG0 - log(nH);
    // below the double range the surface is already at xce: the slab only
    // attenuates by its neutral column xce N
    if (lg < -700.0) return lnG0 - target * xce;
    if (!(target > 0.0)) return lnG0;
    const double G = exp(lg);
    const double sD = sqrt((G + gcoll) * (G + gcoll) + 4.0 * G * alpha);
    const double den = G + 2.0 * alpha + gcoll + sD;
    const double x0 = 2.0 * alpha / den;
    // xce - x0 without cancellation
    const double e0 = alpha * G * (1.0 + (G + 2.0 * gcoll + 4.0 * alpha) / (sD + gcoll)) /
                      ((alpha + gcoll) * den);
    const double v0 = log(e0);
    const double c0 = 1.0 / x0 + log((1.0 - x0) / x0) + log(e0 / x0) / xce;
    double lo = v0 - xce * target - 64.0, hi = v0;
    double v = v0 - xce * target;                     // deep-slab estimate
    if (v < lo || v > hi) v = 0.5 * (lo + hi);
    for (int it = 0; it < 100; ++it) {
        const double e = exp(v), x = xce - e;
        // F(v) - target, decreasing in v
        const double F = c0 - 1.0 / x + log(x / (1.0 - x)) + (log(x) - v) / xce - target;
        if (F > 0.0) lo = v;
        else hi = v;
        const double dF = -e * (1.0 / (x * x) + 1.0 / x + 1.0 / (1.0 - x) + 1.0 / (xce * x)) -
                          1.0 / xce;
        double vn = v - F / dF;
        if (!(vn > lo && vn < hi)) vn = 0.5 * (lo + hi);   // keep to the bracket
        if (fabs(vn - v) <= 1e-14 * fmax(1.0, fabs(v))) {
            v = vn;
            break;
        }
        v = vn;
    }
    const double xs = xce - exp(v);
    return log(nH) + log(alpha + gcoll) + log1p(-xs) + v - log(xs);
}

// The spectrum's attenuation, tabulated once per spectrum: with
// S(N) = sum_b (w_b sigma_b / max) exp(-(sigma_b - sigma_min) N), the rate
// after a hydrogen column N is ln Gamma = ln_ws_max - sigma_min N + ln S(N).
// v[i] = (ln S, d ln S / dt) at t_i = i dt, t = ln(1 + sigma_max N); beyond
// t_max every bin but the least absorbed has decayed by e^-60 and ln S is
// constant.  Cubic Hermite interpolation in t.
struct AttenuationTable {
    const double2* v;
    int m;
    double dt, t_max, sigma_max, sigma_min, ln_ws_max;
};

// ln Gamma after a hydrogen column N (cm^-2); *sbar (nullable) receives the
// rate-weighted mean cross-section -d ln Gamma / dN.
__device__ inline double ln_rate_after(double N, const AttenuationTable& at, double* sbar)
{
    double lnS, dlnS_dN = 0.0;
    const double t = log1p(N * at.sigma_max);
    if (!(t < at.t_max) || at.m < 2) {
        lnS = at.v[at.m - 1].x;
    } else {
        const double u = t / at.dt;
        int i = (int)u;
        if (i > at.m - 2) i = at.m - 2;
        const double th = u - i, th2 = th * th;
        const double2 a = at.v[i], b = at.v[i + 1];
        const double h00 = (1.0 + 2.0 * th) * (1.0 - th) * (1.0 - th);
        const double h10 = th * (1.0 - th) * (1.0 - th);
        const double h01 = th2 * (3.0 - 2.0 * th), h11 = th2 * (th - 1.0);
        lnS = h00 * a.x + h10 * at.dt * a.y + h01 * b.x + h11 * at.dt * b.y;
        if (sbar) {
            const double d00 = 6.0 * th2 - 6.0 * th, d10 = 3.0 * th2 - 4.0 * th + 1.0;
            const double d01 = 6.0 * th - 6.0 * th2, d11 = 3.0 * th2 - 2.0 * th;
            const double dlnS_dt =
                (d00 * a.x + d10 * at.dt * a.y + d01 * b.x + d11 * at.dt * b.y) / at.dt;
            dlnS_dN = dlnS_dt * at.sigma_max / (1.0 + N * at.sigma_max);
        }
    }
    if (sbar) *sbar = fmax(at.sigma_min - dlnS_dN, at.sigma_min);
    return at.ln_ws_max - at.sigma_min * N + lnS;
}

constexpr int kSlabMaxSteps = 4096;
constexpr int kAttNodes = 4096;      // nodes of the attenuation table

// ln of the rate at the bottom of a uniform slab (density nH, coefficients
// alpha, gcoll at its temperature) of total hydrogen column Nn, lit by the
// binned spectrum (attenuation table sp) after a far column Nf: the
// polychromatic near slab.  With HI column u below the surface the rate is
// Gamma(Nf + u), the neutral fraction x(u) = x_-(Gamma), and the hydrogen
// column down to u is
// H(u) = int_0^u du' / x(u'); the bottom is where H = Nn.  The march takes
// steps that lower ln Gamma by about 1/2 (6-point Gauss-Legendre on each,
// nodes glx and weights glw on [-1, 1]); inside the step where H passes Nn,
// Newton's method on the depth, kept to a bracket (dH/du = 1/x).  Once x is
// within 1e-13 of x_ce, 1/x stays constant and the rest of the slab is linear.
__device__ inline double slab_ln_rate_poly(double Nf, double Nn, double nH, double alpha,
                                           double gcoll, const AttenuationTable& sp,
                                           const double* glx, const double* glw)
{
    double sb = 0.0;
    double l = ln_rate_after(Nf, sp, &sb);
    if (!(Nn > 0.0) || l == -INFINITY) return l;
    const double xce = alpha / (alpha + gcoll);
    auto x_at = [&](double u) {
        return x_minus(exp(ln_rate_after(Nf + u, sp, nullptr)), nH, alpha, gcoll);
    };
    auto piece = [&](double u0, double u1) {          // int_{u0}^{u1} du / x
        const double c = 0.5 * (u0 + u1), h = 0.5 * (u1 - u0);
        double acc = 0.0;
        for (int q = 0; q < 6; ++q) acc += glw[q] / x_at(c + h * glx[q]);
        return acc * h;
    };
    double u = 0.0, H = 0.0;
    for (int step = 0; step < kSlabMaxSteps; ++step) {
        const double x = x_minus(exp(l), nH, alpha, gcoll);
        if (xce / x - 1.0 < 1e-13) break;             // neutral from here on
        const double du = 0.5 / sb;
        const double I = piece(u, u + du);
        if (H + I >= Nn) {
            double lo = 0.0, hi = du, t = du * ((Nn - H) / I);
            for (int it = 0; it < 60; ++it) {
                const double F = H + piece(u, u + t) - Nn;
                if (fabs(F) <= 1e-15 * Nn) break;     // t is the bottom
                if (F > 0.0) hi = t;
                else lo = t;
                double tn = t - F * x_at(u + t);
                if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
                const bool done = fabs(tn - t) <= 1e-15 * (u + t);
                t = tn;
                if (done) break;
            }
            return ln_rate_after(Nf + u + t, sp, nullptr);
        }
        H += I;
        u += du;
        l = ln_rate_after(Nf + u, sp, &sb);
    }
    return ln_rate_after(Nf + u + (Nn - H) * xce, sp, nullptr);
}

}  // namespace rrt
