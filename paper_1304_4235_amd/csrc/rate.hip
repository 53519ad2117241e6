// Shielded photoionisation rate and the equilibrium update.
//
// Gamma_p = (1/n_ray) sum_k sum_b w_b sigma_b exp(-sigma_b N_pk)   (Sec. 3.3,
// eq. gamma_shld, frequency integral over bins).  Each ray's frequency sum is
// formed relative to its least-absorbed bin,
//   S_k = sum_b (w_b sigma_b / max w sigma) exp(-(sigma_b - sigma_min) N_k),
// whose exponents are bounded and can run in FP32 (exp2 on the transcendental
// unit); the leading -sigma_min N_k stays in FP64, and the rays combine by a
// log-sum-exp in FP64, so ln Gamma stays exact far past where Gamma itself
// underflows.
//
// x = x_-(Gamma): the physical root of R x^2 + Q x + P (Appendix C.3, eq.
// xroots, y = 0) with R = (gamma + alpha) n_H, P = alpha n_H, Q = -(Gamma + P + R),
// evaluated as 2P / (-Q + sqrt(D)).  The discriminant is formed as
// D = (Gamma + gamma n_H)^2 + 4 Gamma P, which equals Q^2 - 4PR exactly but has
// no cancellation when Gamma is small.
//
// Rates: case A recombination (Hui & Gnedin 1997 fit) and collisional
// ionisation (Cen 1992 fit); the paper refers to published fits without
// printing them.
#include "internal.h"
#include "physics.h"

namespace rrt {

namespace {

constexpr int kBlock = 256;
constexpr int kBlockWaves = kBlock / 64;

__global__ void k_init_state(const int32_t* __restrict__ perm, const float* __restrict__ T,
                             const double* __restrict__ x_init, const float* __restrict__ nH_s,
                             const double* __restrict__ mu_s, int64_t n, double gthin,
                             double* __restrict__ alpha, double* __restrict__ alphaB,
                             double* __restrict__ gcoll, double* __restrict__ x_s,
                             float* __restrict__ mux, unsigned long long* __restrict__ bad_input)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t j = perm[i];
    double Tj = (double)T[j];
    double al = alpha_caseA(Tj), gc = gamma_collisional(Tj);
    alpha[i] = al;
    alphaB[i] = alpha_caseB(Tj);
    gcoll[i] = gc;
    double x = x_init ? x_init[j] : x_minus(gthin, (double)nH_s[i], al, gc);
    if (!(x >= 0.0 && x <= 1.0)) atomicOr(bad_input, 1ull);   // a given state out of range
    x_s[i] = x;
    mux[i] = (float)(mu_s[i] * x);
}

// The paper's update rule (Sec. 4): which particles this step updates, the
// frozen set decided on the first sweep, case B from a tau_eff threshold, and
// relative changes for the convergence test.
struct RateRule {
    const uint8_t* want;      // null = every particle
    uint8_t* skip;            // first sweep: set for tau_eff < tau_skip (null = none)
    double tau_skip;
    double tau_case_b;        // +inf = case A throughout
    const double* alphaB;
    int relative;
    // near/far scheme: far columns in N, near total-hydrogen columns here; each
    // ray's rate is the slab solution of its near column lit by the
    // far-attenuated radiation (null = plain rate): analytic for one bin, the
    // polychromatic slab (Gauss-Legendre nodes and weights below) for several
    const double* Nn;
    double sigma1;
    double gl_x[6], gl_w[6];
    AttenuationTable att;
    // convergence counts of the updated particles: |dx| < conv_tol and
    // |dx| / x < conv_tol (slots kRedConvAbs, kRedConvRel of red)
    double conv_tol;
    // plain scheme, rays with N <= tay_nmax: S_k as the degree-5 polynomial
    // sum_j tay[j] N^j (the bins' Taylor moments), see k_gamma
    double tay[kTaylorTerms];
    double tay_nmax;
};

enum { kSchemePlain = 0, kSchemeNearMono = 1, kSchemeNearPoly = 2 };

// One thread per particle: rays, then bins; optionally the equilibrium update.
template <int SCHEME>
__global__ void __launch_bounds__(256)
k_gamma(const double* __restrict__ N, int64_t n, int n_ray, int n_bins,
        const float* __restrict__ ws_rel, const float* __restrict__ dsig_l2, double sigma_min,
        double ln_ws_max, double ln_gthin, double* __restrict__ lnG, double* __restrict__ G,
        float* __restrict__ tau, int update_x, const float* __restrict__ nH_s,
        const double* __restrict__ mu_s, const double* __restrict__ alpha,
        const double* __restrict__ gcoll, double* __restrict__ x_s, float* __restrict__ mux,
        unsigned long long* __restrict__ maxdx_bits, const int32_t* __restrict__ seg_of,
        const int32_t* __restrict__ seg_active, unsigned long long* __restrict__ seg_maxdx,
        RateRule rule)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double dx = 0.0;
    bool conv_a = false, conv_r = false, bad = false;
    const int h = (seg_of && i < n) ? seg_of[i] : -1;
    const bool live = !(seg_active && h >= 0 && seg_active[h] == 0) &&
                      !(rule.want && i < n && rule.want[i] == 0);
    if (i < n && live) {
        double m = -INFINITY, s = 0.0, l;
        if (SCHEME != kSchemePlain) {
            // near/far: per ray the slab of near particles lit by the radiation
            // the far particles let through.  Each slab is lit by the ray's
            // share, 1/n_ray of the spectrum (eq. gammashld's 4 pi / N_ray,
            // with 4 pi inside w), and the slabs' bottom rates add up.  (The
            // table of binned spectra carries the shift.)
            const double ln_share = -log((double)n_ray);
            for (int k = 0; k < n_ray; ++k) {
                double v;
                if (SCHEME == kSchemeNearPoly) {
                    v = slab_ln_rate_poly(N[(int64_t)k * n + i], rule.Nn[(int64_t)k * n + i],
                                          (double)nH_s[i], alpha[i], gcoll[i], rule.att, rule.gl_x,
                                          rule.gl_w);
                } else {
                    // one bin: ln w sigma = ln_ws_max
                    const double l0 = ln_ws_max + ln_share - rule.sigma1 * N[(int64_t)k * n + i];
                    v = slab_ln_rate(l0, (double)nH_s[i], alpha[i], gcoll[i], rule.sigma1,
                                     rule.Nn[(int64_t)k * n + i]);
                }
                if (v == -INFINITY) continue;
                if (v > m) {
                    s = s * exp(m - v) + 1.0;
                    m = v;
                } else {
                    s += exp(v - m);
                }
            }
            l = (s > 0.0) ? (m + log(s)) : -INFINITY;
        } else {
            // 2^x is the hardware instruction (about 1 ulp), which flushes
            // results below 2^-126 to zero: the bin of smallest cross-section
            // enters every sum undamped (its exponent is 0), so a flushed
            // term is negligible beside it.
            // A ray thin in every bin (y_b = (sigma_b - sigma_min) N <= 0.15)
            // takes S_k from the bins' Taylor moments instead: sum_b r_b
            // e^{-y_b} = sum_j (-1)^j N^j / j! sum_b r_b (y_b / N)^j, cut
            // after j = 5, where the alternating tail is at most y^6/720 of
            // each term, 1.9e-8 of S_k (S_k >= 0.85 sum_b r_b there): below
            // the FP32 sum's own rounding, for 6 FMAs instead of n_bins
            // exponentials.
            for (int k = 0; k < n_ray; ++k) {
                double Nk = N[(int64_t)k * n + i];
                float Nf = (float)Nk;
                double Sd;
                if ((double)Nf <= rule.tay_nmax) {
                    const double t = (double)Nf;
                    Sd = rule.tay[kTaylorTerms - 1];
                    for (int j = kTaylorTerms - 2; j >= 0; --j) Sd = fma(Sd, t, rule.tay[j]);
                } else {
                    float S0 = 0.f, S1 = 0.f, S2 = 0.f, S3 = 0.f;
                    int b = 0;
                    for (; b + 3 < n_bins; b += 4) {
                        S0 = fmaf(ws_rel[b], __builtin_amdgcn_exp2f(-dsig_l2[b] * Nf), S0);
                        S1 = fmaf(ws_rel[b + 1], __builtin_amdgcn_exp2f(-dsig_l2[b + 1] * Nf),
                                  S1);
                        S2 = fmaf(ws_rel[b + 2], __builtin_amdgcn_exp2f(-dsig_l2[b + 2] * Nf),
                                  S2);
                        S3 = fmaf(ws_rel[b + 3], __builtin_amdgcn_exp2f(-dsig_l2[b + 3] * Nf),
                                  S3);
                    }
                    for (; b < n_bins; ++b)
                        S0 = fmaf(ws_rel[b], __builtin_amdgcn_exp2f(-dsig_l2[b] * Nf), S0);
                    Sd = (double)((S0 + S1) + (S2 + S3));
                }
                if (!(Sd > 0.0)) continue;                    // this ray carries nothing
                double v = -sigma_min * Nk + log(Sd);
                if (v > m) {
                    s = s * exp(m - v) + 1.0;
                    m = v;
                } else {
                    s += exp(v - m);
                }
            }
            l = (s > 0.0) ? (ln_ws_max + m + log(s / (double)n_ray)) : -INFINITY;
        }
        double g = exp(l);
        if (lnG) lnG[i] = l;
        if (G) G[i] = g;
        if (tau) tau[i] = (float)(ln_gthin - l);
        const double te = ln_gthin - l;              // tau_eff in FP64 decides
        if (update_x && rule.skip && te < rule.tau_skip) {
            rule.skip[i] = 1;                         // keeps its state for good
        } else if (update_x) {
            const double al = te >= rule.tau_case_b ? rule.alphaB[i] : alpha[i];
            double xn = x_minus(g, (double)nH_s[i], al, gcoll[i]);
            const double xo = x_s[i];
            const double da = fabs(xn - xo);
            conv_a = da < rule.conv_tol;
            conv_r = da < rule.conv_tol * xo;
            bad = !(xn >= 0.0 && xn <= 1.0);          // also catches NaN
            dx = rule.relative ? da / xo : da;
            x_s[i] = xn;
            mux[i] = (float)(mu_s[i] * xn);
        }
    }
    if (update_x) {
        // the counts, the flag and the maximum are reduced per block, so each
        // takes one atomic per block on its (single) global word
        const uint64_t ba = __ballot(conv_a), br = __ballot(conv_r), bb = __ballot(bad);
        __shared__ unsigned long long s_red[kBlockWaves][4];
        __shared__ int s_hw[kBlockWaves];
        __shared__ unsigned long long s_hm[kBlockWaves];
        const int wv = threadIdx.x >> 6;
        if (seg_maxdx) {
            // per-halo maximum: a wave that holds one halo passes its maximum
            // to the block (below); the lanes of a wave across halos add theirs
            const int h0 = __shfl(h, 0, 64);
            const bool one = h0 >= 0 && __ballot(h != h0 && h >= 0) == 0;
            double m = dx;
            for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
            if (!one && h >= 0 && dx > 0.0)
                atomicMax(seg_maxdx + h, (unsigned long long)__double_as_longlong(dx));
            if ((threadIdx.x & 63) == 0) {
                s_hw[wv] = one ? h0 : -1;
                s_hm[wv] = (unsigned long long)__double_as_longlong(m);
            }
        }
        for (int off = 32; off > 0; off >>= 1) dx = fmax(dx, __shfl_xor(dx, off, 64));
        if ((threadIdx.x & 63) == 0) {
            s_red[wv][0] = (unsigned long long)__popcll(ba);
            s_red[wv][1] = (unsigned long long)__popcll(br);
            s_red[wv][2] = bb ? 1ull : 0ull;
            s_red[wv][3] = (unsigned long long)__double_as_longlong(dx);
        }
        __syncthreads();
        if (seg_maxdx && threadIdx.x == 0) {
            // one atomic per run of the block's waves in the same halo
            const int nw = (int)(blockDim.x >> 6);
            for (int w = 0; w < nw;) {
                const int hh = s_hw[w];
                unsigned long long mx = s_hm[w];
                int v = w + 1;
                for (; v < nw && s_hw[v] == hh; ++v) mx = s_hm[v] > mx ? s_hm[v] : mx;
                if (hh >= 0 && __longlong_as_double((long long)mx) > 0.0)
                    atomicMax(seg_maxdx + hh, mx);
                w = v;
            }
        }
        if (threadIdx.x == 0) {
            unsigned long long na = 0, nr = 0, nb = 0, mx = 0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
                na += s_red[w][0];
                nr += s_red[w][1];
                nb |= s_red[w][2];
                mx = s_red[w][3] > mx ? s_red[w][3] : mx;      // dx >= 0: bits order as values
            }
            if (na) atomicAdd(maxdx_bits + (kRedConvAbs - kRedMaxDx), na);
            if (nr) atomicAdd(maxdx_bits + (kRedConvRel - kRedMaxDx), nr);
            if (nb) atomicOr(maxdx_bits + (kRedNumeric - kRedMaxDx), 1ull);
            atomicMax(maxdx_bits, mx);
        }
    }
}

// Per-halo bookkeeping after an iteration (graph-safe: no memsets needed):
// count the iteration of every active halo, retire halos whose max|dx| fell
// below tol (or that reached max_iter), clear the maxima for the next
// iteration, and publish [iterations launched, halos still active].
__global__ void k_seg_finalize(int n_halo, double tol, int max_iter, int32_t* __restrict__ active,
                               unsigned long long* __restrict__ maxdx, int32_t* __restrict__ iters,
                               int32_t* __restrict__ state, unsigned long long* __restrict__ red)
{
    __shared__ int cnt[256];
    int c = 0;
    for (int h = threadIdx.x; h < n_halo; h += blockDim.x) {
        if (active[h]) {
            const int it = iters[h] + 1;
            iters[h] = it;
            const double d = __longlong_as_double((long long)maxdx[h]);
            if (d < tol || it >= max_iter) active[h] = 0;
            else ++c;
        }
        maxdx[h] = 0ull;
    }
    cnt[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) cnt[threadIdx.x] += cnt[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        state[0] += 1;
        state[1] = cnt[0];
        red[0] = 0ull;
        red[1] = 0ull;
    }
}

__global__ void k_seg_init(int n_halo, int32_t* __restrict__ active,
                           unsigned long long* __restrict__ maxdx, int32_t* __restrict__ iters,
                           int32_t* __restrict__ state, unsigned long long* __restrict__ red)
{
    for (int h = threadIdx.x; h < n_halo; h += blockDim.x) {
        active[h] = 1;
        maxdx[h] = 0ull;
        iters[h] = 0;
    }
    if (threadIdx.x == 0) {
        state[0] = 0;
        state[1] = n_halo;
        red[0] = 0ull;
        red[1] = 0ull;
    }
}

__global__ void k_update_x(const double* __restrict__ G, int64_t n, const float* __restrict__ nH_s,
                           const double* __restrict__ mu_s, const double* __restrict__ alpha,
                           const double* __restrict__ gcoll, double* __restrict__ x_s,
                           float* __restrict__ mux, unsigned long long* __restrict__ maxdx_bits)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double dx = 0.0;
    if (i < n) {
        double xn = x_minus(G[i], (double)nH_s[i], alpha[i], gcoll[i]);
        dx = fabs(xn - x_s[i]);
        x_s[i] = xn;
        mux[i] = (float)(mu_s[i] * xn);
    }
    for (int off = 32; off > 0; off >>= 1) dx = fmax(dx, __shfl_xor(dx, off, 64));
    // one atomic per block on the single word
    __shared__ unsigned long long s_mx[kBlockWaves];
    if ((threadIdx.x & 63) == 0) s_mx[threadIdx.x >> 6] = (unsigned long long)__double_as_longlong(dx);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long mx = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) mx = s_mx[w] > mx ? s_mx[w] : mx;
        atomicMax(maxdx_bits, mx);
    }
}

__global__ void k_mux(const double* __restrict__ mu_s, const double* __restrict__ x_s, int64_t n,
                      float* __restrict__ mux)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) mux[i] = (float)(mu_s[i] * x_s[i]);
}

// tree order -> input order; src is [stride][n] (one column per stride index)
__global__ void k_scatter_d(const int32_t* __restrict__ perm, const double* __restrict__ src,
                            int64_t n, int stride, double* __restrict__ dst)
{
    int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= n * stride) return;
    int64_t k = g / n, i = g - k * n;
    dst[(int64_t)perm[i] * stride + k] = src[g];
}

__global__ void k_scatter_f(const int32_t* __restrict__ perm, const float* __restrict__ src,
                            int64_t n, float* __restrict__ dst)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) dst[perm[i]] = src[i];
}

__global__ void k_gather_d(const int32_t* __restrict__ perm, const double* __restrict__ src,
                           int64_t n, double* __restrict__ dst)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}

// a given state: input order -> tree order, flagging values outside [0, 1]
// (NaN included) in *bad
__global__ void k_gather_state(const int32_t* __restrict__ perm, const double* __restrict__ src,
                               int64_t n, double* __restrict__ dst,
                               unsigned long long* __restrict__ bad)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool b = false;
    if (i < n) {
        const double v = src[perm[i]];
        b = !(v >= 0.0 && v <= 1.0);
        dst[i] = v;
    }
    if (__ballot(b) && (threadIdx.x & 63) == 0) atomicOr(bad, 1ull);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

namespace {

// Nodes and weights of the 6-point Gauss-Legendre rule on [-1, 1]: the roots
// of the Legendre polynomial P_6 by Newton's method from the usual cosine
// estimates, weights 2 / ((1 - x^2) P_6'(x)^2).
void gauss_legendre6(double* x, double* w)
{
    const int m = 6;
    for (int i = 0; i < m; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (m + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;                         // P_0, P_1
            for (int k = 2; k <= m; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = m * (z * p1 - p0) / (z * z - 1.0);          // P_m'(z)
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Attenuation table of the current spectrum (its weighted bins): ln S and
// d ln S / dt at kAttNodes nodes uniform in t = ln(1 + sigma_max N) up to the
// column where the second least absorbed bin has decayed by e^-60 relative to
// the least absorbed one.  FP64 log-sum-exp at every node.
hipError_t build_attenuation_table(Ctx& c)
{
    std::vector<double> sg, lw;
    for (size_t b = 0; b < c.sigma_host.size(); ++b) {
        if (!(c.w_host[b] > 0.0)) continue;
        sg.push_back(c.sigma_host[b]);
        lw.push_back(std::log(c.w_host[b] * c.sigma_host[b]) - c.ln_ws_max);
    }
    const double smin = c.sigma_min;
    double smax = smin, s2 = INFINITY;
    for (double v : sg) {
        smax = std::max(smax, v);
        if (v > smin * (1.0 + 1e-12)) s2 = std::min(s2, v);
    }
    const double n_sat = std::isfinite(s2) ? 60.0 / (s2 - smin) : 0.0;
    const int m = kAttNodes;
    const double tmax = std::log1p(n_sat * smax);
    const double dt = tmax > 0.0 ? tmax / (m - 1) : 1.0;
    std::vector<double> tab(2 * (size_t)m);
    for (int i = 0; i < m; ++i) {
        const double N = std::expm1(i * dt) / smax;
        double mx = -INFINITY;
        for (size_t b = 0; b < sg.size(); ++b) mx = std::max(mx, lw[b] - (sg[b] - smin) * N);
        double S = 0.0, D = 0.0;
        for (size_t b = 0; b < sg.size(); ++b) {
            const double e = std::exp(lw[b] - (sg[b] - smin) * N - mx);
            S += e;
            D += (sg[b] - smin) * e;
        }
        tab[2 * i] = mx + std::log(S);
        tab[2 * i + 1] = -(D / S) * (1.0 + N * smax) / smax;    // d ln S / dt
    }
    hipError_t e = ws_alloc(c, &c.att_tab, tab.size());
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(c.att_tab, tab.data(), sizeof(double) * tab.size(),
                       hipMemcpyHostToDevice, c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);     // tab goes out of scope
    if (e != hipSuccess) {
        ws_free(c, &c.att_tab);
        return e;
    }
    c.att_m = tmax > 0.0 ? m : 1;
    c.att_dt = dt;
    c.att_tmax = tmax;
    c.att_smax = smax;
    return hipSuccess;
}

}  // namespace

hipError_t launch_init_state(Ctx& c, bool use_given)
{
    hipLaunchKernelGGL(k_init_state, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream, c.perm, c.T_in,
                       use_given ? c.x_init : nullptr, c.nH_s, c.mu_s, c.n, c.gamma_thin,
                       c.alpha_s, c.alphaB_s, c.gcoll_s, c.x_s, c.mux_s, c.red + kRedInput);
    return hipGetLastError();
}

hipError_t launch_gamma(Ctx& c, bool update_x, bool first_sweep)
{
    RateRule rule;
    rule.want = c.geom.want;
    rule.skip = (first_sweep && c.rule_tau_skip > 0.0) ? c.skip_s : nullptr;
    rule.tau_skip = c.rule_tau_skip;
    rule.tau_case_b = c.rule_tau_case_b;
    rule.alphaB = c.alphaB_s;
    rule.relative = c.rule_relative;
    rule.Nn = c.near_far ? c.Nn_s : nullptr;
    rule.sigma1 = c.sigma_min;
    rule.conv_tol = c.conv_tol;
    for (int j = 0; j < kTaylorTerms; ++j) rule.tay[j] = c.tay[j];
    rule.tay_nmax = c.tay_nmax;
    gauss_legendre6(rule.gl_x, rule.gl_w);
    const int scheme = !c.near_far ? kSchemePlain : c.n_bins == 1 ? kSchemeNearMono
                                                                  : kSchemeNearPoly;
    rule.att = AttenuationTable{};
    if (scheme == kSchemeNearPoly) {
        if (!c.att_tab) {
            hipError_t e = build_attenuation_table(c);
            if (e != hipSuccess) return e;
        }
        // each ray's slab is lit by its share, 1/n_ray, of the spectrum
        const double shift = std::log((double)c.n_ray);
        rule.att = AttenuationTable{reinterpret_cast<const double2*>(c.att_tab), c.att_m,
                                    c.att_dt, c.att_tmax, c.att_smax, c.sigma_min,
                                    c.ln_ws_max - shift};
    }
    auto launch = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream, c.N_s, c.n,
                           c.n_ray, c.n_bins, c.ws_rel, c.dsig_l2, c.sigma_min, c.ln_ws_max,
                           std::log(c.gamma_thin), c.lnG_s, c.G_s, c.tau_s, update_x ? 1 : 0,
                           c.nH_s, c.mu_s, c.alpha_s, c.gcoll_s, c.x_s, c.mux_s, c.red,
                           c.geom.seg_of, c.geom.seg_active,
                           c.geom.seg_active ? c.seg_maxdx : nullptr, rule);
    };
    if (scheme == kSchemePlain) launch(k_gamma<kSchemePlain>);
    else if (scheme == kSchemeNearMono) launch(k_gamma<kSchemeNearMono>);
    else launch(k_gamma<kSchemeNearPoly>);
    return hipGetLastError();
}

namespace {

// particles of block `block` of the density order that are not frozen
__global__ void k_want(const int32_t* __restrict__ block_s, const uint8_t* __restrict__ skip,
                       int64_t n, int block, uint8_t* __restrict__ want)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool in_block = !block_s || block_s[i] == block;
    want[i] = (in_block && !(skip && skip[i])) ? 1 : 0;
}

__global__ void k_block_ids(const int32_t* __restrict__ perm, const int32_t* __restrict__ block_in,
                            int64_t n, int32_t* __restrict__ block_s)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) block_s[i] = block_in[perm[i]];
}

}  // namespace

namespace {

// every particle advances by dt at its current rate (case A)
__global__ void k_evolve(const double* __restrict__ G, int64_t n, const float* __restrict__ nH_s,
                         const double* __restrict__ mu_s, const double* __restrict__ alpha,
                         const double* __restrict__ gcoll, double dt, double* __restrict__ x_s,
                         float* __restrict__ mux)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = x_after(x_s[i], G[i], (double)nH_s[i], alpha[i], gcoll[i], dt);
    x_s[i] = x;
    mux[i] = (float)(mu_s[i] * x);
}

}  // namespace

hipError_t launch_evolve(Ctx& c, double dt)
{
    hipLaunchKernelGGL(k_evolve, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream, c.G_s, c.n, c.nH_s,
                       c.mu_s, c.alpha_s, c.gcoll_s, dt, c.x_s, c.mux_s);
    return hipGetLastError();
}

hipError_t launch_want(Ctx& c, int block, bool use_skip)
{
    hipLaunchKernelGGL(k_want, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream,
                       c.rule_blocks > 1 ? c.block_s : nullptr, use_skip ? c.skip_s : nullptr,
                       c.n, block, c.want_s);
    return hipGetLastError();
}

hipError_t launch_block_ids(Ctx& c, const int32_t* block_in)
{
    hipLaunchKernelGGL(k_block_ids, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream, c.perm, block_in,
                       c.n, c.block_s);
    return hipGetLastError();
}

// intersections per halo from per-ray counts (rows are [direction][tree position])
__global__ void k_halo_hits(const uint64_t* __restrict__ row_cnt, int64_t n_rows, int64_t n,
                            const int32_t* __restrict__ seg_of, unsigned long long* __restrict__ out)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int h = r < n_rows ? seg_of[r % n] : -1;
    unsigned long long v = r < n_rows ? (unsigned long long)row_cnt[r] : 0ull;
    const int h0 = __shfl(h, 0, 64);
    if (h0 >= 0 && __ballot(h != h0 && h >= 0) == 0) {
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((threadIdx.x & 63) == 0 && v) atomicAdd(out + h0, v);
    } else if (h >= 0 && v) {
        atomicAdd(out + h, v);
    }
}

// per-ray counts of the halos in `mask`, zero for the others
__global__ void k_mask_rows(const uint64_t* __restrict__ row_cnt, int64_t n_rows, int64_t n,
                            const int32_t* __restrict__ seg_of, const int32_t* __restrict__ mask,
                            uint64_t* __restrict__ row_off)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r < n_rows) row_off[r] = mask[seg_of[r % n]] ? row_cnt[r] : 0ull;
}

// start a group of halos: only the masked ones iterate; iteration counts kept
__global__ void k_seg_group_init(int n_halo, const int32_t* __restrict__ mask,
                                 int32_t* __restrict__ active, unsigned long long* __restrict__ maxdx,
                                 int32_t* __restrict__ state, unsigned long long* __restrict__ red)
{
    __shared__ int cnt[256];
    int c = 0;
    for (int h = threadIdx.x; h < n_halo; h += blockDim.x) {
        active[h] = mask[h] ? 1 : 0;
        c += active[h];
        maxdx[h] = 0ull;
    }
    cnt[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) cnt[threadIdx.x] += cnt[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        state[0] = 0;
        state[1] = cnt[0];
        red[0] = 0ull;
        red[1] = 0ull;
    }
}

hipError_t launch_halo_hits(Ctx& c, const uint64_t* row_cnt, unsigned long long* out)
{
    const int64_t n_rows = c.n * (int64_t)c.n_ray;
    hipLaunchKernelGGL(k_halo_hits, dim3(nblk(n_rows)), dim3(kBlock), 0, c.stream, row_cnt, n_rows,
                       c.n, c.seg_of, out);
    return hipGetLastError();
}

hipError_t launch_mask_rows(Ctx& c, const uint64_t* row_cnt, const int32_t* mask, uint64_t* row_off)
{
    const int64_t n_rows = c.n * (int64_t)c.n_ray;
    hipLaunchKernelGGL(k_mask_rows, dim3(nblk(n_rows)), dim3(kBlock), 0, c.stream, row_cnt, n_rows,
                       c.n, c.seg_of, mask, row_off);
    return hipGetLastError();
}

hipError_t launch_seg_group_init(Ctx& c, const int32_t* mask)
{
    hipLaunchKernelGGL(k_seg_group_init, dim3(1), dim3(256), 0, c.stream, c.n_halo, mask,
                       c.seg_active, c.seg_maxdx, c.seg_state, c.red);
    return hipGetLastError();
}

hipError_t launch_seg_finalize(Ctx& c, double tol, int max_iter)
{
    hipLaunchKernelGGL(k_seg_finalize, dim3(1), dim3(256), 0, c.stream, c.n_halo, tol, max_iter,
                       c.seg_active, c.seg_maxdx, c.seg_iters, c.seg_state, c.red);
    return hipGetLastError();
}

hipError_t launch_seg_init(Ctx& c)
{
    hipLaunchKernelGGL(k_seg_init, dim3(1), dim3(256), 0, c.stream, c.n_halo, c.seg_active,
                       c.seg_maxdx, c.seg_iters, c.seg_state, c.red);
    return hipGetLastError();
}

hipError_t launch_update_x(Ctx& c)
{
    hipLaunchKernelGGL(k_update_x, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream, c.G_s, c.n, c.nH_s,
                       c.mu_s, c.alpha_s, c.gcoll_s, c.x_s, c.mux_s, c.red);
    return hipGetLastError();
}

hipError_t launch_mux(Ctx& c)
{
    hipLaunchKernelGGL(k_mux, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream, c.mu_s, c.x_s, c.n,
                       c.mux_s);
    return hipGetLastError();
}

hipError_t launch_to_input_order_d(Ctx& c, const double* src, double* dst, int32_t stride)
{
    hipLaunchKernelGGL(k_scatter_d, dim3(nblk(c.n * stride)), dim3(kBlock), 0, c.stream, c.perm,
                       src, c.n, stride, dst);
    return hipGetLastError();
}

hipError_t launch_to_input_order_f(Ctx& c, const float* src, float* dst)
{
    hipLaunchKernelGGL(k_scatter_f, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream, c.perm, src, c.n,
                       dst);
    return hipGetLastError();
}

namespace {

// pos[k] = the tree position holding input index in_sorted[k]
__global__ void k_find_positions(const int32_t* __restrict__ perm, int64_t n,
                                 const int32_t* __restrict__ in_sorted, int32_t m,
                                 int32_t* __restrict__ pos)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t j = perm[i];
    int lo = 0, hi = m;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (in_sorted[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    if (lo < m && in_sorted[lo] == j) pos[lo] = (int32_t)i;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int32_t m, int32_t v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) p[i] = v;
}

}  // namespace

hipError_t launch_find_positions(Ctx& c, const int32_t* in_sorted, int32_t m, int32_t* pos)
{
    hipLaunchKernelGGL(k_fill_i32, dim3((m + 255) / 256), dim3(256), 0, c.stream, pos, m, -1);
    hipLaunchKernelGGL(k_find_positions, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream, c.perm, c.n,
                       in_sorted, m, pos);
    return hipGetLastError();
}

hipError_t launch_state_from_input(Ctx& c, const double* src)
{
    hipLaunchKernelGGL(k_gather_state, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream, c.perm, src,
                       c.n, c.x_s, c.red + kRedInput);
    return hipGetLastError();
}

hipError_t launch_from_input_order_d(Ctx& c, const double* src, double* dst)
{
    hipLaunchKernelGGL(k_gather_d, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream, c.perm, src, c.n,
                       dst);
    return hipGetLastError();
}

}  // namespace rrt
