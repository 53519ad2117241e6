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

}  // namespace rrt
