// Reverse mode through K unrolled order-independent iterations.
//
// Forward map (all steps as in the forward kernels):
//   x^0_p  = x_-(Gamma_thin, n_p),               Gamma_thin = sum_b w_b sigma_b
//   N^k_pi = sum_j a_pi,j mu_j x^{k-1}_j           (Sec. 4.1.1, eq. colden; a = K/h^2)
//   lnG^k_p = ln[(1/n_ray) sum_i sum_b w_b sigma_b exp(-sigma_b N^k_pi)]   (eq. gamma_shld)
//   x^k_p  = x_-(Gamma^k_p, n_p)                   (Appendix C.3, eq. xroots)
// with mu_j = mu_input_j n_j / n_input_j (a particle's hydrogen content scales
// with its density at fixed smoothing length).  Parameters: the bin weights w_b
// and the densities n_j.  Outputs: lnG^K and x^K.
//
// Local derivatives used below:
//   dx/dlnG   = -G x / sqrt(D)        (implicit differentiation of the quadratic)
//   dx/dn     =  G x / (n sqrt(D))    (x depends on G / n only)
//   dlnG/dN_i = -pi_i T_i / S_i,  pi = softmax over rays of v_i = -sigma_min N_i + ln S_i,
//               S_i = sum_b r_b e^{-(s_b - s_min) N_i}, T_i = sum_b r_b s_b e^{...}
//   dlnG/dw_b = (sigma_b / max(w sigma)) sum_i pi_i e^{-(s_b - s_min) N_i} / S_i
// where r_b = w_b sigma_b / max(w sigma).
#include "internal.h"
#include "physics.h"

namespace rrt {

namespace {

constexpr int kBlock = 256;

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// One thread per particle (tree order) at step k.
__global__ void __launch_bounds__(256)
k_adj_rate(const double* __restrict__ N, int64_t n, int n_ray, int n_bins,
           const float* __restrict__ ws_rel, const float* __restrict__ dsig_l2,
           const float* __restrict__ srat, double sigma_min, double ln_ws_max,
           const float* __restrict__ nH_s, const double* __restrict__ alpha,
           const double* __restrict__ gcoll, const double* __restrict__ lam,
           const double* __restrict__ lup, double* __restrict__ nu, double* __restrict__ pis,
           double* __restrict__ gnH, double* __restrict__ gw_part)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool act = i < n;
    const int64_t ii = act ? i : 0;
    double ell = 0.0;
    if (act) {
        // pass 1: ln Gamma exactly as the forward rate kernel forms it
        double m = -INFINITY, s = 0.0;
        for (int k = 0; k < n_ray; ++k) {
            const double Nk = N[(int64_t)k * n + i];
            const float Nf = (float)Nk;
            float S = 0.f;
            for (int b = 0; b < n_bins; ++b) S = fmaf(ws_rel[b], exp2f(-dsig_l2[b] * Nf), S);
            if (!(S > 0.f)) continue;
            const double v = -sigma_min * Nk + log((double)S);
            if (v > m) {
                s = s * exp(m - v) + 1.0;
                m = v;
            } else {
                s += exp(v - m);
            }
        }
        const double l = (s > 0.0) ? (ln_ws_max + m + log(s / (double)n_ray)) : -INFINITY;
        const double G = exp(l);
        const double nh = (double)nH_s[i];
        const double x = x_minus(G, nh, alpha[i], gcoll[i]);
        const double sD = sqrt(eq_discriminant(G, nh, alpha[i], gcoll[i]));
        const double dxdl = (sD > 0.0) ? -G * x / sD : 0.0;
        const double li = lam[i];
        ell = (lup ? lup[i] : 0.0) + li * dxdl;
        gnH[i] += -li * dxdl / nh;
        // pass 2: adjoint of every ray's column, and pi_i / S_i for the bins
        for (int k = 0; k < n_ray; ++k) {
            const double Nk = N[(int64_t)k * n + i];
            const float Nf = (float)Nk;
            float S = 0.f, T = 0.f;
            for (int b = 0; b < n_bins; ++b) {
                const float e = ws_rel[b] * exp2f(-dsig_l2[b] * Nf);
                S += e;
                T = fmaf(e, srat[b], T);
            }
            double nk = 0.0, pk = 0.0;
            if (S > 0.f && s > 0.0) {
                const double v = -sigma_min * Nk + log((double)S);
                const double pi = exp(v - m) / s;
                pk = pi / (double)S;
                nk = -ell * pi * sigma_min * ((double)T / (double)S);
            }
            nu[(int64_t)k * n + i] = nk;
            pis[(int64_t)k * n + i] = pk;
        }
    }
    // pass 3: per-bin weight derivative, reduced over the wave in a fixed order
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    for (int b = 0; b < n_bins; ++b) {
        double acc = 0.0;
        if (act && ell != 0.0) {
            const float ds = dsig_l2[b];
            for (int k = 0; k < n_ray; ++k) {
                const float Nf = (float)N[(int64_t)k * n + ii];
                acc += pis[(int64_t)k * n + ii] * (double)exp2f(-ds * Nf);
            }
            acc *= ell;
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if ((threadIdx.x & 63) == 0) gw_part[wave * n_bins + b] = acc;
    }
}

// sum the per-wave partials of every bin, in wave order, into the accumulator
__global__ void k_adj_bins(const double* __restrict__ part, int64_t n_waves, int n_bins,
                           double* __restrict__ acc)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_bins) return;
    double s = 0.0;
    for (int64_t w = 0; w < n_waves; ++w) s += part[w * n_bins + b];
    acc[b] += s;
}

// transposed product over recorded paths: y_j += (K/h^2) nu_row for every hit
__global__ void __launch_bounds__(256)
k_adj_scatter(const uint64_t* __restrict__ row_off, const int2* __restrict__ path,
              const double* __restrict__ nu, int64_t n_rows, double* __restrict__ y)
{
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; row < n_rows;
         row += stride) {
        const double v = nu[row];
        if (v == 0.0) continue;
        const uint64_t a = row_off[row], b = row_off[row + 1];
        for (uint64_t e = a + lane; e < b; e += 64) {
            const int2 h = path[e];
            unsafeAtomicAdd(y + h.x, (double)__int_as_float(h.y) * v);
        }
    }
}

// adjoint of x^{k-1} from the columns, and the density term through mu
__global__ void k_adj_x(const double* __restrict__ y, const double* __restrict__ mu_s,
                        const float* __restrict__ mu0_s, const float* __restrict__ nH0_s,
                        const double* __restrict__ xprev, int64_t n, double* __restrict__ lam,
                        double* __restrict__ gnH)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double yi = y[i];
    lam[i] = mu_s[i] * yi;
    gnH[i] += ((double)mu0_s[i] / (double)nH0_s[i]) * xprev[i] * yi;
}

// the initial state x^0 = x_-(Gamma_thin, n): density term and the per-particle
// factor of dL/dGamma_thin (reduced per wave)
__global__ void k_adj_init(const double* __restrict__ lam, const float* __restrict__ nH_s,
                           const double* __restrict__ alpha, const double* __restrict__ gcoll,
                           int64_t n, double gthin, double* __restrict__ gnH,
                           double* __restrict__ part)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        const double nh = (double)nH_s[i];
        const double x = x_minus(gthin, nh, alpha[i], gcoll[i]);
        const double sD = sqrt(eq_discriminant(gthin, nh, alpha[i], gcoll[i]));
        const double dxdG = sD > 0.0 ? -x / sD : 0.0;
        gnH[i] += -lam[i] * gthin * dxdG / nh;
        v = lam[i] * dxdG;
    }
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) part[(blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6] = v;
}

__global__ void k_set_density(const int32_t* __restrict__ perm, const float* __restrict__ nH,
                              const float* __restrict__ mu0_s, const float* __restrict__ nH0_s,
                              int64_t n, float* __restrict__ nH_s, double* __restrict__ mu_s)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = nH[perm[i]];
    nH_s[i] = v;
    mu_s[i] = (double)mu0_s[i] * ((double)v / (double)nH0_s[i]);
}

}  // namespace

hipError_t launch_set_density(Ctx& c, const float* nH)
{
    hipLaunchKernelGGL(k_set_density, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream, c.perm, nH,
                       c.mu0_s, c.nH0_s, c.n, c.nH_s, c.mu_s);
    return hipGetLastError();
}

hipError_t launch_adj_rate(Ctx& c, const double* lup)
{
    hipLaunchKernelGGL(k_adj_rate, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream, c.N_s, c.n, c.n_ray,
                       c.n_bins, c.ws_rel, c.dsig_l2, c.srat, c.sigma_min, c.ln_ws_max, c.nH_s,
                       c.alpha_s, c.gcoll_s, c.adj_lam, lup, c.adj_nu, c.adj_pis, c.adj_gnH,
                       c.adj_wpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n_waves = (int64_t)nblk(c.n) * (kBlock / 64);
    hipLaunchKernelGGL(k_adj_bins, dim3((c.n_bins + 255) / 256), dim3(256), 0, c.stream,
                       c.adj_wpart, n_waves, c.n_bins, c.adj_gw);
    return hipGetLastError();
}

hipError_t launch_adj_scatter(Ctx& c)
{
    const int64_t n_rows = c.n * (int64_t)c.n_ray;
    hipError_t e = hipMemsetAsync(c.adj_y, 0, sizeof(double) * c.n, c.stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_scatter, dim3(stride_blocks(n_rows, 4)), dim3(256), 0,
                       c.stream, c.row_off, c.path, c.adj_nu, n_rows, c.adj_y);
    return hipGetLastError();
}

hipError_t launch_adj_x(Ctx& c, const double* xprev)
{
    hipLaunchKernelGGL(k_adj_x, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream, c.adj_y, c.mu_s,
                       c.mu0_s, c.nH0_s, xprev, c.n, c.adj_lam, c.adj_gnH);
    return hipGetLastError();
}

hipError_t launch_adj_init(Ctx& c, double* part)
{
    hipLaunchKernelGGL(k_adj_init, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream, c.adj_lam, c.nH_s,
                       c.alpha_s, c.gcoll_s, c.n, c.gamma_thin, c.adj_gnH, part);
    return hipGetLastError();
}

int64_t adj_waves(const Ctx& c) { return (int64_t)nblk(c.n) * (kBlock / 64); }

}  // namespace rrt
