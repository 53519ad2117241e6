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

// Rays thin in every bin ((sigma_b - sigma_min) N <= 0.15): S and T as their
// degree-5 Taylor forms in N (the forward rate kernel's switch), and, for the
// weights' gradient, sum over such (particle, ray) pairs of W 2^{-d_b N} as
// sum_j (-ln 2 d_b)^j / j! sum W N^j.  The tail is below 1.9e-8 of each sum.
struct ThinSums {
    double s[kTaylorTerms];
    double t[kTaylorTerms];
    double nmax;
};

__device__ __forceinline__ double horner(const double* c, double x)
{
    double r = c[kTaylorTerms - 1];
    for (int j = kTaylorTerms - 2; j >= 0; --j) r = fma(r, x, c[j]);
    return r;
}

// One thread per particle (tree order) at step k: the adjoint of ln Gamma, of
// x and of every ray's column.  Pass 1 forms ln Gamma from the same terms as
// the forward rate kernel (hardware 2^x, or the thin rays' Taylor form),
// summed in one FP32 accumulator instead of four, so the two agree to FP32
// rounding; it keeps each ray's S and T for pass 2.  The weights' gradient is accumulated by k_adj_wbins from
// pis and ell.
__global__ void __launch_bounds__(256)
k_adj_rate(const double* __restrict__ N, int64_t n, int n_ray, int n_bins,
           const float* __restrict__ ws_rel, const float* __restrict__ dsig_l2,
           const float* __restrict__ srat, double sigma_min, double ln_ws_max,
           const float* __restrict__ nH_s, const double* __restrict__ alpha,
           const double* __restrict__ gcoll, const double* __restrict__ lam,
           const double* __restrict__ lup, float* __restrict__ nu, double* __restrict__ pis,
           double* __restrict__ gnH, float2* __restrict__ st, double* __restrict__ ell_out,
           ThinSums ts)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    // pass 1: ln Gamma
    double m = -INFINITY, s = 0.0;
    for (int k = 0; k < n_ray; ++k) {
        const double Nk = N[(int64_t)k * n + i];
        const float Nf = (float)Nk;
        float S = 0.f, T = 0.f;
        if ((double)Nf <= ts.nmax) {
            S = (float)horner(ts.s, (double)Nf);
            T = (float)horner(ts.t, (double)Nf);
        } else {
            for (int b = 0; b < n_bins; ++b) {
                const float e = ws_rel[b] * __builtin_amdgcn_exp2f(-dsig_l2[b] * Nf);
                S += e;
                T = fmaf(e, srat[b], T);
            }
        }
        st[(int64_t)k * n + i] = make_float2(S, T);
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
    const double ell = (lup ? lup[i] : 0.0) + li * dxdl;
    gnH[i] += -li * dxdl / nh;
    ell_out[i] = ell;
    // pass 2: adjoint of every ray's column, and pi / S per ray for the bins
    for (int k = 0; k < n_ray; ++k) {
        const double Nk = N[(int64_t)k * n + i];
        const float2 ST = st[(int64_t)k * n + i];
        double nk = 0.0, pk = 0.0;
        if (ST.x > 0.f && s > 0.0) {
            const double v = -sigma_min * Nk + log((double)ST.x);
            const double pi = exp(v - m) / s;
            pk = pi / (double)ST.x;
            nk = -ell * pi * sigma_min * ((double)ST.y / (double)ST.x);
        }
        nu[(int64_t)k * n + i] = (float)nk;
        pis[(int64_t)k * n + i] = pk;
    }
}

// Weight gradient partials: a wave serves 64 bins (one per lane) for a chunk
// of kAdjChunk particles.  For each ray, 64 particles' column and ell * pi / S
// are staged in LDS with coalesced loads, and every lane forms its own bin's
// factor from the LDS broadcasts.  Per lane the sum runs over rays, then the
// chunk's particles, in order.
__device__ __forceinline__ void adj_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void __launch_bounds__(256)
k_adj_wbins(const double* __restrict__ N, const double* __restrict__ pis,
            const double* __restrict__ ell, const float* __restrict__ dsig_l2, int64_t n,
            int n_ray, int n_bins, int64_t n_chunks, double* __restrict__ part, double nmax)
{
    __shared__ float sN[4][64];
    __shared__ double sW[4][64];
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int groups = (n_bins + 63) / 64;
    if (wave >= (int64_t)groups * n_chunks) return;           // whole wave
    const int g = (int)(wave % groups);
    const int64_t chunk = wave / groups;
    const int b = g * 64 + lane;
    const float ds = b < n_bins ? dsig_l2[b] : 0.0f;
    const int64_t i0 = chunk * kAdjChunk;
    const int64_t i1 = i0 + kAdjChunk < n ? i0 + kAdjChunk : n;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    double acc = 0.0;
    // moments sum W N^j of the thin pairs this lane stages
    double mom[kTaylorTerms] = {};
    for (int k = 0; k < n_ray; ++k) {
        for (int64_t ib = i0; ib < i1; ib += 64) {
            const int64_t i = ib + lane;
            const bool in = i < i1;
            const float Nf = in ? (float)N[(int64_t)k * n + i] : 0.0f;
            const double w = in ? ell[i] * pis[(int64_t)k * n + i] : 0.0;
            const bool thin = (double)Nf <= nmax;
            if (thin && w != 0.0) {
                double p = w;
                for (int j = 0; j < kTaylorTerms; ++j) {
                    mom[j] += p;
                    p *= (double)Nf;
                }
            }
            // the thick pairs, packed to the front, go through every bin
            const uint64_t thick = __builtin_amdgcn_ballot_w64(!thin && w != 0.0);
            if (!thin && w != 0.0) {
                const int q = __popcll(thick & lt);
                sN[wv][q] = Nf;
                sW[wv][q] = w;
            }
            adj_wave_sync();
            const int m = __popcll(thick);
            for (int q = 0; q < m; ++q)
                acc += sW[wv][q] * (double)__builtin_amdgcn_exp2f(-ds * sN[wv][q]);
            adj_wave_sync();
        }
    }
    // every bin takes the thin pairs' sum from the wave's moments
    double c = 1.0, tot = 0.0;
    for (int j = 0; j < kTaylorTerms; ++j) {
        double mj = mom[j];
        for (int off = 32; off > 0; off >>= 1) mj += __shfl_xor(mj, off, 64);
        tot += c * mj;
        c *= -0.6931471805599453 * (double)ds / (double)(j + 1);
    }
    acc += tot;
    if (b < n_bins) part[chunk * n_bins + b] = acc;
}

// The per-chunk partials of every bin summed into the accumulator in two
// passes of fixed order (so the gradient is the same on every run).  First,
// block (g, s) takes the 64 bins of group g (one per lane, coalesced) over the
// chunks of slice s: its 4 waves take every 4th chunk, added in wave order.
__global__ void __launch_bounds__(256)
k_adj_bin_slices(const double* __restrict__ part, int64_t n_chunks, int n_bins,
                 double* __restrict__ part2)
{
    __shared__ double s_w[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int b = blockIdx.x * 64 + lane;
    const int64_t per = (n_chunks + kAdjSlices - 1) / kAdjSlices;
    const int64_t w0 = (int64_t)blockIdx.y * per;
    const int64_t w1 = w0 + per < n_chunks ? w0 + per : n_chunks;
    double acc = 0.0;
    if (b < n_bins)
        for (int64_t w = w0 + wv; w < w1; w += 4) acc += part[w * n_bins + b];
    s_w[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && b < n_bins)
        part2[(int64_t)blockIdx.y * n_bins + b] =
            ((s_w[0][lane] + s_w[1][lane]) + s_w[2][lane]) + s_w[3][lane];
}

// then every bin's slices, in slice order
__global__ void k_adj_bins(const double* __restrict__ part2, int n_bins, double* __restrict__ acc)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_bins) return;
    double s = 0.0;
    for (int q = 0; q < kAdjSlices; ++q) s += part2[(int64_t)q * n_bins + b];
    acc[b] += s;
}

// transposed product over recorded paths: y_j += (K/h^2) nu_row for every hit
__global__ void __launch_bounds__(256)
k_adj_scatter(const uint64_t* __restrict__ row_off, const int2* __restrict__ path,
              const float* __restrict__ nu, int64_t n_rows, double* __restrict__ y)
{
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; row < n_rows;
         row += stride) {
        const double v = (double)nu[row];
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
                              int64_t n, float* __restrict__ nH_s, double* __restrict__ mu_s,
                              unsigned long long* __restrict__ bad)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = nH[perm[i]];
    if (!(v > 0.f) || !isfinite(v)) atomicOr(bad, 1ull);      // densities must be > 0
    nH_s[i] = v;
    mu_s[i] = (double)mu0_s[i] * ((double)v / (double)nH0_s[i]);
}

ThinSums thin_sums(const Ctx& c)
{
    ThinSums t;
    for (int j = 0; j < kTaylorTerms; ++j) {
        t.s[j] = c.tay[j];
        t.t[j] = c.tay_t[j];
    }
    t.nmax = c.tay_nmax;
    return t;
}

}  // namespace

hipError_t launch_set_density(Ctx& c, const float* nH)
{
    hipLaunchKernelGGL(k_set_density, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream, c.perm, nH,
                       c.mu0_s, c.nH0_s, c.n, c.nH_s, c.mu_s, c.red + kRedInput);
    return hipGetLastError();
}

hipError_t launch_adj_rate(Ctx& c, const double* N, const double* lup)
{
    hipLaunchKernelGGL(k_adj_rate, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream, N, c.n, c.n_ray,
                       c.n_bins, c.ws_rel, c.dsig_l2, c.srat, c.sigma_min, c.ln_ws_max, c.nH_s,
                       c.alpha_s, c.gcoll_s, c.adj_lam, lup, c.adj_nu, c.adj_pis, c.adj_gnH,
                       c.adj_st, c.adj_ell, thin_sums(c));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t chunks = adj_chunks(c);
    const int64_t waves = chunks * ((c.n_bins + 63) / 64);
    hipLaunchKernelGGL(k_adj_wbins, dim3((unsigned)((waves * 64 + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, c.stream, N, c.adj_pis, c.adj_ell, c.dsig_l2, c.n,
                       c.n_ray, c.n_bins, chunks, c.adj_wpart, c.tay_nmax);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the second level sits behind the per-chunk partials
    double* part2 = c.adj_wpart + (size_t)chunks * c.n_bins;
    hipLaunchKernelGGL(k_adj_bin_slices, dim3((c.n_bins + 63) / 64, kAdjSlices), dim3(256), 0,
                       c.stream, c.adj_wpart, chunks, c.n_bins, part2);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_bins, dim3((c.n_bins + 255) / 256), dim3(256), 0, c.stream, part2,
                       c.n_bins, c.adj_gw);
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

int64_t adj_chunks(const Ctx& c) { return (c.n + kAdjChunk - 1) / kAdjChunk; }

}  // namespace rrt
