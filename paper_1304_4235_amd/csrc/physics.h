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

}  // namespace rrt
