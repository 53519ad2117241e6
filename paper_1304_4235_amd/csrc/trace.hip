// Ray traversal and HI column accumulation (Sec. 4.1.1, eq. colden).
//
// One thread follows one ray: source particle p (tree order), direction k and,
// in a periodic box, every image shift s whose tiles the segment can reach.
// Lanes of a wave take consecutive sources in tree order with the same
// direction, so neighbouring lanes walk nearly the same nodes.
//
// Node tests are FP32 slab tests against boxes padded outward by `pad`, which
// is far larger than any FP32 rounding in the test, so they never reject a
// particle the exact predicate accepts.  Leaf particles are decided by the
// FP64 predicate below, with a fixed operation order and no contraction, so
// that the set of intersected particles is reproducible bit for bit.
//
// A hit adds mu_j x_j / h_j^2 times the kernel chord integral K(b/h, z1/h,
// z2/h) in units of h: for the truncated Gaussian (eq. Gt) the closed form
// I(h,b,z1,z2) = (N h^3 sqrt(pi) / (2t)) e^{-t^2 q^2} [erf(t z2/h) - erf(t z1/h)] / h^2
// with t = A h = 2 pi^(1/6), q = b/h, z clipped to the sphere and to [0, L].
// erf comes from a table of cubic pieces staged in LDS; the Gaussian from the
// hardware 2^x with its exponent formed in FP64.
#include "internal.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <type_traits>

namespace rrt {

namespace {

// ---------------------------------------------------------------------------
// kernel tables (host, FP64)
// ---------------------------------------------------------------------------
struct KConst {
    double t, C;     // C = N h^3 sqrt(pi) / (2 t)
};

KConst kconst()
{
    const double pi = 3.14159265358979323846;
    double t = 2.0 * std::pow(pi, 1.0 / 6.0);
    double nh3 = (8.0 / pi) / (std::erf(t) - 2.0 * t * std::exp(-t * t) / std::sqrt(pi));
    return {t, nh3 * std::sqrt(pi) / (2.0 * t)};
}

template <typename F>
void fit_cubics(float4* out, F f)
{
    // cubic through u = 0, 1/3, 2/3, 1 on each piece, in monomial form in u
    for (int i = 0; i < kTabIntervals; ++i) {
        double a = (double)i / kTabIntervals, b = (double)(i + 1) / kTabIntervals;
        double y0 = f(a), y1 = f(a + (b - a) / 3.0), y2 = f(a + 2.0 * (b - a) / 3.0), y3 = f(b);
        // Newton divided differences on nodes 0, 1/3, 2/3, 1
        double d1 = (y1 - y0) * 3.0, d2 = (y2 - y1) * 3.0, d3 = (y3 - y2) * 3.0;
        double e1 = (d2 - d1) * 1.5, e2 = (d3 - d2) * 1.5;
        double g1 = (e2 - e1);
        // p(u) = y0 + d1 u + e1 u (u - 1/3) + g1 u (u - 1/3)(u - 2/3)
        double c0 = y0;
        double c1 = d1 - e1 / 3.0 + g1 * (2.0 / 9.0);
        double c2 = e1 - g1;
        double c3 = g1;
        out[i] = make_float4((float)c0, (float)c1, (float)c2, (float)c3);
    }
}

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float tab_eval(const float4* __restrict__ tb, float x)
{
    float s = x * (float)kTabIntervals;
    int i = (int)s;
    i = i < 0 ? 0 : (i > kTabIntervals - 1 ? kTabIntervals - 1 : i);
    float u = s - (float)i;
    float4 c = tb[i];
    return fmaf(fmaf(fmaf(c.w, u, c.z), u, c.y), u, c.x);
}

__device__ __forceinline__ float erf_t_odd(const float4* __restrict__ tb, float z)
{
    float a = fminf(fabsf(z), 1.0f);
    float v = tab_eval(tb, a);
    return z < 0.f ? -v : v;
}

// column: accumulate N; count: hits per ray; record: hit lists for inspection;
// path: per hit (tree index, K/h^2) for the streaming product
// scatter: y_j += (K/h^2) nu_ray for every hit (transposed column product)
// chunk: the path entries of each ray appended to pool chunks, with the counts
// (one-pass recording; wave-cooperative walk only)
// stats: a count pass that also tallies the walk's work (diagnostics)
enum { kModeColumn = 0, kModeCount = 1, kModeRecord = 2, kModePath = 3, kModeScatter = 4,
       kModeChunk = 5, kModeStats = 6 };

struct RayOut {
    double* N;              // [n_ray][n] columns (column / record modes)
    uint64_t* row_cnt;      // [n_ray * n] hits per ray (count mode)
    const uint64_t* row_off;// [n_ray * n] write offsets (record / path modes)
    int2* path;             // path mode: (tree index, factor bits) per hit
    const float* nu;        // scatter mode: adjoint of each ray's column
    double* y;              // scatter mode: accumulated per tree index
    int32_t* hit_j;         // record mode: input index of each hit
    int32_t* hit_img;       // record mode: image code of each hit
    uint64_t hit_cap;       // record mode: capacity of hit_j / hit_img
    const int32_t* perm;
    unsigned long long* hits_total;
    // near/far split (column and path modes): a hit is near when the
    // particle's kernel contains the source, |d|^2 < h^2 (FP64, x, y, z order)
    int near_far;
    double* Nn;             // column mode: [n_ray][n] near total-hydrogen columns
    const double* mu;       // hydrogen content per tree index (near columns use x = 1)
    // chunk mode: pool of chunks, their links, each row's first chunk, the
    // per-slice allocation counters and the overflow flag after them
    int2* pool;
    uint32_t* chunk_next;
    uint32_t* row_first;
    unsigned long long* pool_ctr;
    uint64_t slice_chunks;
    // sampled sources (count and record modes): only the rays of the sorted
    // tree positions src_list[0..src_n) run, and their outputs go to row
    // i * n_ray + k for the source at src_list[i] (null = every ray, row = ray)
    const int32_t* src_list;
    int32_t src_n;
    float* hit_fac;         // record mode: K/h^2 of each hit (nullable)
    // stats mode: [rays, wave node visits, lane node visits, wave leaf visits,
    // pair tests, hits], accumulated
    unsigned long long* stats;
    // wave-cooperative walk, persistent form: a resident grid whose waves take
    // packets (64 sources of one direction, over every halo) from this counter
    // until none is left; null = one wave per packet
    unsigned long long* queue;
};

// Place of tree position ps among the sorted sampled sources, or -1.
__device__ __forceinline__ int sampled_slot(const int32_t* __restrict__ list, int m, int ps)
{
    int lo = 0, hi = m;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (list[mid] < ps) lo = mid + 1;
        else hi = mid;
    }
    return (lo < m && list[lo] == ps) ? lo : -1;
}

// sign bit of a recorded factor: the hit is near (factors are >= 0)
constexpr uint32_t kNearBit = 0x80000000u;

// A pool entry of the one-walk recording holds, in place of the factor, the
// periodic image of the hit: 10 bits per axis, s + 512 (images with |s| up to
// 511; the recording only takes this route when every reachable image fits).
constexpr int kImgBias = 512;

__host__ __device__ __forceinline__ uint32_t chunk_image_code(int sx, int sy, int sz)
{
    return (uint32_t)(sx + kImgBias) | ((uint32_t)(sy + kImgBias) << 10) |
           ((uint32_t)(sz + kImgBias) << 20);
}

// The canonical predicate (shared operation order with the FP64 reference):
// d = (r_j - r_p) + s B ; s_par = d.u ; t = clamp(s_par, 0, L) ; c = d - t u ;
// hit <=> |c|^2 < h^2, with the dot products and c in fused multiply-adds as
// written below (dot_u, norm2) and no other contraction.
#pragma clang fp contract(off)
// K/h^2 of one intersection: the chord integral of the kernel (eq. Gt) in
// units of h, over h^2, C e^{-t^2 q^2} [erf(t z2) - erf(t z1)] / h^2.  sp = d.u
// locates the point of the ray nearest the particle, b2 is the squared impact
// parameter and h2 = h^2, all FP64; hf = h.  z1, z2 are the chord's ends in
// units of h, clipped to the sphere and to the segment [0, L].  0 for a
// tangent touch.
//  * The Gaussian: the exponent -a q^2 (a = t^2 log2 e, q^2 = b2 / h2) is
//    formed in FP64; its integer part is applied exactly and its fraction by
//    the hardware 2^x (about 1 ulp).
//  * erf from the LDS table; a chord that spans the whole sphere (z1 = -z2)
//    needs one lookup, erf being odd.
//  * Reciprocals and the square root are the hardware's single instructions
//    (about 1 ulp).
__device__ __forceinline__ float chord_factor(double sp, double b2, double h2, double L,
                                              float hf, const float4* __restrict__ t_erf,
                                              double gc, double ga)
{
    const double l2 = h2 - b2;
    if (!(l2 > 0.0)) return 0.0f;
    const float ih2 = __builtin_amdgcn_rcpf((float)h2);
    const float lh = __builtin_amdgcn_sqrtf(fminf((float)l2 * ih2, 1.0f));
    const float ih = __builtin_amdgcn_rcpf(hf);
    const float z1 = fmaxf((float)(-sp) * ih, -lh);
    const float z2 = fminf((float)(L - sp) * ih, lh);
    if (!(z2 > z1)) return 0.0f;
    const double e = -ga * (b2 / h2);
    const double en = floor(e);
    const float g = (float)gc * ldexpf(__builtin_amdgcn_exp2f((float)(e - en)), (int)en);
    const float e2 = erf_t_odd(t_erf, z2);
    float e1;
    if (z1 == -z2) e1 = -e2;
    else e1 = erf_t_odd(t_erf, z1);
    return ih2 * (g * (e2 - e1));
}

// The canonical operation order of the pair arithmetic (the same wherever a
// pair is evaluated): a dot product with u, or a squared norm, starts with the
// x product and adds y, then z, by fused multiply-add; a component of d - t u
// is one fused multiply-add.  fma rounds once, as IEEE 754 defines it.
__device__ __forceinline__ double dot_u(double d0, double d1, double d2, const double u[3])
{
    return fma(d2, u[2], fma(d1, u[1], d0 * u[0]));
}

__device__ __forceinline__ double norm2(double c0, double c1, double c2)
{
    return fma(c2, c2, fma(c1, c1, c0 * c0));
}

// The pair's geometry: d = (r_j - r_p) + s B and sp = d.u.
struct PairGeom {
    double d0, d1, d2, sp;
};

__device__ __forceinline__ PairGeom pair_geom(const float4 Q, double o0, double o1, double o2,
                                              const double sh[3], const double u[3])
{
    PairGeom pg;
    pg.d0 = ((double)Q.x - o0) + sh[0];
    pg.d1 = ((double)Q.y - o1) + sh[1];
    pg.d2 = ((double)Q.z - o2) + sh[2];
    pg.sp = dot_u(pg.d0, pg.d1, pg.d2, u);
    return pg;
}

// The same from coordinates already in FP64; for an unshifted image
// (kShifted false, s = 0) the adds of zero are left out, which changes no bit.
template <bool kShifted>
__device__ __forceinline__ PairGeom pair_geom_d(double qx, double qy, double qz, double o0,
                                                double o1, double o2, const double sh[3],
                                                const double u[3])
{
    PairGeom pg;
    pg.d0 = qx - o0;
    pg.d1 = qy - o1;
    pg.d2 = qz - o2;
    if (kShifted) {
        pg.d0 = pg.d0 + sh[0];
        pg.d1 = pg.d1 + sh[1];
        pg.d2 = pg.d2 + sh[2];
    }
    pg.sp = dot_u(pg.d0, pg.d1, pg.d2, u);
    return pg;
}

// K/h^2 of a hit: the squared impact parameter from d - sp u, then the chord.
__device__ __forceinline__ float hit_factor(const PairGeom& pg, const double u[3], float hf,
                                            double L, const float4* __restrict__ t_erf,
                                            double gc, double ga)
{
    const double px = fma(-pg.sp, u[0], pg.d0), py = fma(-pg.sp, u[1], pg.d1),
                 pz = fma(-pg.sp, u[2], pg.d2);
    const double b2 = norm2(px, py, pz);
    const double hj = (double)hf;
    return chord_factor(pg.sp, b2, hj * hj, L, hf, t_erf, gc, ga);
}

template <int MODE>
__global__ void __launch_bounds__(256)
k_trace(const Node* __restrict__ nodes, const float4* __restrict__ p4,
        const float* __restrict__ mux, const double* __restrict__ dirs,
        const KernelTables* __restrict__ tabs, TraceGeom g, RayOut out)
{
    __shared__ float4 t_erf[kTabIntervals];
    constexpr bool kTerms = MODE != kModeCount;
    if (kTerms) {
        for (int i = threadIdx.x; i < kTabIntervals; i += blockDim.x) t_erf[i] = tabs->erf_t[i];
        __syncthreads();
    }
    const double gc = tabs->gauss_c, ga = tabs->gauss_a;

    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t n_rays = (int64_t)g.n * g.n_ray;
    uint32_t cnt = 0;
    int64_t slot = gid;
    bool sampled = true;
    if (gid < n_rays && out.src_list) {
        const int k = (int)(gid / g.n);
        const int i = sampled_slot(out.src_list, out.src_n, (int)(gid - (int64_t)k * g.n));
        sampled = i >= 0;
        slot = (int64_t)i * g.n_ray + k;
    }
    if (gid < n_rays && sampled) {
        const int k = (int)(gid / g.n);
        const int ps = (int)(gid - (int64_t)k * g.n);
        const float4 P = p4[ps];
        const double rp[3] = {(double)P.x, (double)P.y, (double)P.z};
        const double u[3] = {dirs[3 * k], dirs[3 * k + 1], dirs[3 * k + 2]};
        const double L = g.L, B = g.box;
        const float Lf = (float)L;

        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        if (B > 0.0) {
            for (int a = 0; a < 3; ++a) {
                double e = rp[a] + L * u[a];
                double smin = rp[a] < e ? rp[a] : e, smax = rp[a] < e ? e : rp[a];
                lo[a] = (int)ceil((smin - g.hmax - g.phi[a]) / B - 1e-6);
                hi[a] = (int)floor((smax + g.hmax - g.plo[a]) / B + 1e-6);
            }
        }
        float inv[3];
        for (int a = 0; a < 3; ++a) {
            float ua = (float)u[a];
            if (fabsf(ua) < 1e-20f) ua = 1e-20f;
            inv[a] = 1.0f / ua;
        }
        double acc = 0.0, accn = 0.0;
        uint64_t w = (MODE == kModeRecord || MODE == kModePath) ? out.row_off[slot] : 0;
        const double nur = (MODE == kModeScatter) ? (double)out.nu[gid] : 0.0;

        // the subtree this ray's halo owns (the whole tree for one problem)
        int root = 0, end = g.n_nodes;
        bool live = true;
        if (g.seg_root) {
            const int h = g.seg_of[ps];
            root = g.seg_root[h];
            end = g.seg_end[h];
            live = !g.seg_active || g.seg_active[h] != 0;
        }
        if (MODE == kModeColumn && g.want && !g.want[ps]) live = false;
        if (!live) lo[0] = 1, hi[0] = 0;            // no image loop at all
        for (int sx = lo[0]; sx <= hi[0]; ++sx)
        for (int sy = lo[1]; sy <= hi[1]; ++sy)
        for (int sz = lo[2]; sz <= hi[2]; ++sz) {
            double sh[3] = {(double)sx * B, (double)sy * B, (double)sz * B};
            if (!(B > 0.0)) sh[0] = sh[1] = sh[2] = 0.0;
            // the image of particle j sits at r_j + sB, i.e. the ray meets the
            // stored particles as if it started from r_p - sB
            float oai[3], obi[3];
            for (int a = 0; a < 3; ++a) {
                double o = rp[a] - sh[a];
                oai[a] = (float)(o + (double)g.pad) * inv[a];
                obi[a] = (float)(o - (double)g.pad) * inv[a];
            }
            int node = root;
            while (node < end) {
                const Node nd = nodes[node];
                float tx0 = fmaf(nd.a.x, inv[0], -oai[0]), tx1 = fmaf(nd.b.x, inv[0], -obi[0]);
                float ty0 = fmaf(nd.a.y, inv[1], -oai[1]), ty1 = fmaf(nd.b.y, inv[1], -obi[1]);
                float tz0 = fmaf(nd.a.z, inv[2], -oai[2]), tz1 = fmaf(nd.b.z, inv[2], -obi[2]);
                float tmin = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)),
                                   fmaxf(fminf(tz0, tz1), 0.0f));
                float tmax = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)),
                                   fminf(fmaxf(tz0, tz1), Lf));
                const int skip = __float_as_int(nd.a.w);
                const int leafw = __float_as_int(nd.b.w);
                // skip links always point past the node; max() keeps every walk finite
                if (!(tmin <= tmax)) { node = max(skip, node + 1); continue; }
                if (leafw < 0) { node = node + 1; continue; }
                const int f = leafw >> kLeafShift;
                const int c = (f + (leafw & (kLeafMax - 1)) + 1 <= g.n) ? (leafw & (kLeafMax - 1)) + 1 : 0;
                // the leaf's particles (contiguous in tree order) are loaded
                // eight at a time; p4 holds kLeafMax spare entries past n
                for (int q0 = 0; q0 < c; q0 += 8) {
                float4 Qs[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) Qs[q] = p4[f + q0 + q];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if (q0 + q >= c) break;
                    const int j = f + q0 + q;
                    const float4 Q = Qs[q];
                    double d0 = ((double)Q.x - rp[0]) + sh[0];
                    double d1 = ((double)Q.y - rp[1]) + sh[1];
                    double d2 = ((double)Q.z - rp[2]) + sh[2];
                    double sp = dot_u(d0, d1, d2, u);
                    double tt = sp < 0.0 ? 0.0 : (sp > L ? L : sp);
                    double c0 = fma(-tt, u[0], d0);
                    double c1 = fma(-tt, u[1], d1);
                    double c2 = fma(-tt, u[2], d2);
                    double D2 = norm2(c0, c1, c2);
                    double hj = (double)Q.w;
                    double h2 = hj * hj;
                    if (!(D2 < h2)) continue;
                    ++cnt;
                    if (MODE == kModeCount || MODE == kModeStats) continue;
                    double px = fma(-sp, u[0], d0), py = fma(-sp, u[1], d1),
                           pz = fma(-sp, u[2], d2);
                    double b2 = norm2(px, py, pz);
                    const float gk = chord_factor(sp, b2, h2, L, Q.w, t_erf, gc, ga);
                    if (MODE == kModeRecord) {
                        if (w < out.hit_cap) {
                            out.hit_j[w] = out.perm[j];
                            out.hit_img[w] = (sx + 8) | ((sy + 8) << 4) | ((sz + 8) << 8);
                            if (out.hit_fac) out.hit_fac[w] = gk;
                        }
                        ++w;
                    }
                    bool near = false;
                    if (out.near_far) near = (d0 * d0 + d1 * d1 + d2 * d2) < h2;
                    if (MODE == kModePath) {
                        const uint32_t bits = (uint32_t)__float_as_int(gk) | (near ? kNearBit : 0u);
                        if (w < out.hit_cap) out.path[w] = make_int2(j, (int)bits);
                        ++w;
                    } else if (MODE == kModeScatter) {
                        if (nur != 0.0) unsafeAtomicAdd(out.y + j, (double)gk * nur);
                    } else if (near) {
                        accn += (double)((float)out.mu[j] * gk);
                    } else {
                        acc += (double)(mux[j] * gk);
                    }
                }
                }   // groups of eight particles
                node = max(skip, node + 1);
            }
        }
        if ((MODE == kModeColumn || MODE == kModeRecord) && live && out.N)
            out.N[(int64_t)k * g.n + ps] = acc;
        if (MODE == kModeColumn && live && out.near_far) out.Nn[(int64_t)k * g.n + ps] = accn;
        if (MODE == kModeCount || MODE == kModeStats) out.row_cnt[slot] = cnt;
    }
    // one atomic per wave for the total intersection count
    uint64_t c64 = cnt;
    for (int off = 32; off > 0; off >>= 1) c64 += __shfl_xor(c64, off, 64);
    if ((threadIdx.x & 63) == 0 && c64) atomicAdd(out.hits_total, (unsigned long long)c64);
}
// LDS written by some lanes of a wave and read by others: order the accesses
// within the wave (no block barrier needed, the wave runs in lockstep)
// One pool chunk for every lane with want, handed out from the wave's cache:
// the range [c_next, c_end) of chunk indices the wave has taken and not yet
// given out (wave-uniform; the persistent walk keeps it across packets).  An
// empty cache takes a block of max(block, lanes still waiting) chunks with one
// atomic, from the wave's slice first, then from further slices (stride 97,
// odd, so kSliceTries distinct ones); a slice's last, partial block is used as
// far as it goes.  Returns whether this lane got one (its index in nc).
__device__ __forceinline__ bool take_chunk(bool want, uint32_t slice, int lane,
                                           uint64_t lt_mask, unsigned long long* pool_ctr,
                                           uint64_t slice_chunks, uint32_t block,
                                           uint32_t& c_next, uint32_t& c_end, uint32_t& nc)
{
    uint64_t need = __builtin_amdgcn_ballot_w64(want);
    bool got = false;
    int t = 0;
    while (need) {
        const uint32_t k = (uint32_t)__popcll(need);
        const uint32_t avail = c_end - c_next;
        if (avail == 0) {
            if (t == kSliceTries) break;
            const uint32_t sl = (slice + 97u * (uint32_t)t) % kPoolSlices;
            ++t;
            const uint32_t n_take = k > block ? k : block;
            const int leader = __ffsll((unsigned long long)need) - 1;
            unsigned long long base = 0;
            if (lane == leader)
                base = atomicAdd(pool_ctr + (size_t)sl * kCtrStride, (unsigned long long)n_take);
            base = __shfl(base, leader, 64);
            const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
            const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
            const uint64_t b = ((uint64_t)hi << 32) | lo;
            if (b < slice_chunks) {
                const uint64_t room = slice_chunks - b;
                c_next = (uint32_t)(sl * slice_chunks + b);
                c_end = c_next + (uint32_t)(room < n_take ? room : n_take);
            }
            continue;
        }
        // the lowest-ranked waiting lanes take what the cache holds
        if (want && !got) {
            const uint32_t r = (uint32_t)__popcll(need & lt_mask);
            if (r < avail) {
                got = true;
                nc = c_next + r;
            }
        }
        c_next += k < avail ? k : avail;
        need = __builtin_amdgcn_ballot_w64(want && !got);
    }
    return got;
}

// lanes where b holds (the HIP __ballot takes an int and re-tests it)
__device__ __forceinline__ uint64_t wave_ballot(bool b)
{
    return __builtin_amdgcn_ballot_w64(b);
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave-cooperative variant: the 64 rays of a wave (same direction, sources
// adjacent in tree order) walk ONE node sequence, the depth-first union of
// their individual walks.  Node and leaf-particle loads are wave-uniform
// (scalar loads); each lane tests its own ray, and a ballot decides whether the
// wave descends or skips.  A lane only tests the particles of leaves its own
// ray's box test accepted, and sees them in depth-first order, so every lane's
// hits, counts and recorded paths equal those of its own walk.
//
// The walk is bound by vector instruction issue (the chip's VALU issue rate is
// reached with the scalar node loads hidden behind it), so the loops are
// written for instruction count:
//  * the rays share one direction, so on each axis the face a ray enters
//    through (low or high) is the same for all lanes: it is chosen once with
//    scalar selects, and the slab test needs no per-lane min/max of the pair;
//  * the node index and the walk's bounds are scalar, so the loop is too;
//  * a leaf's (ray, particle) pairs are indexed with an FP32 reciprocal (exact
//    for the at most 64 x 16 pairs); the rays' origins and the leaf's
//    particles are read, already in FP64, from LDS (each particle is loaded
//    and widened once per leaf, not once per pair);
//  * the image shift's three adds only run for a shifted image: for the
//    unshifted one they add zero, which changes no bit of the predicate;
//  * the near test only exists in the near/far variant (NF).
// LDS per wave: origins 3 x 64 FP64, hit masks 64 x 4 B, factors 64 x 16 x
// 4 B (modes that evaluate factors in the walk, which also stage the erf
// table once per block) or the hit rays' write places (modes whose pair lanes
// write entries), the leaf's particles 16 x 4 FP64.  Sized per launch
// (dynamic LDS), so a 128-thread block holds two waves' buffers.
// Six waves per SIMD (measured: the count and record passes run 4.5% faster on
// the 2.1M-particle field than at the four that ~100 VGPRs would allow, with
// a few registers spilled to scratch).
constexpr int kWaveOrgBytes = 3 * 64 * (int)sizeof(double);
constexpr int kWaveMaskBytes = 64 * (int)sizeof(unsigned int);
constexpr int kWaveGkBytes = 64 * kLeafMax * (int)sizeof(float);
constexpr int kWaveDstBytes = 64 * 16;     // per hit ray: where its entries go
constexpr int kWaveLeafBytes = kLeafMax * 4 * (int)sizeof(double);

// modes whose walk evaluates the chord factor of its hits (the one-walk
// recording leaves it to the compaction)
__host__ __device__ constexpr bool mode_factors(int mode)
{
    return mode == kModeColumn || mode == kModeRecord || mode == kModePath ||
           mode == kModeScatter;
}

// modes whose pair lanes write the entries themselves (no per-ray hit loop)
__host__ __device__ constexpr bool mode_direct(int mode)
{
    return mode == kModePath || mode == kModeChunk;
}

// per wave: the factor or write-place buffer of a mode
__host__ __device__ constexpr int wave_pair_bytes(int mode)
{
    return mode_direct(mode) ? kWaveDstBytes : mode_factors(mode) ? kWaveGkBytes : 0;
}

// dynamic LDS bytes of one k_trace_wave block
inline size_t wave_lds_bytes(int mode, int block)
{
    const size_t waves = (size_t)(block / 64);
    size_t b = waves * (kWaveOrgBytes + kWaveMaskBytes + wave_pair_bytes(mode) + kWaveLeafBytes);
    if (mode_factors(mode)) b += (size_t)kTabIntervals * sizeof(float4);
    return b;
}

template <int MODE, bool NF, bool PQ>
__global__ void __launch_bounds__(256, 6)
k_trace_wave(const Node* __restrict__ nodes, const float4* __restrict__ p4,
             const float* __restrict__ mux, const double* __restrict__ dirs,
             const KernelTables* __restrict__ tabs, TraceGeom g, RayOut out)
{
    constexpr bool kCountOnly = MODE == kModeCount || MODE == kModeStats;
    constexpr bool kTerms = mode_factors(MODE);
    constexpr bool kDirect = mode_direct(MODE);
    extern __shared__ __align__(16) unsigned char s_dyn[];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int n_wv = blockDim.x >> 6;
    float4* t_erf = reinterpret_cast<float4*>(s_dyn);
    unsigned char* s_wave = s_dyn + (kTerms ? kTabIntervals * sizeof(float4) : 0);
    // per wave: the hit rays' origins (FP64, by rank among the leaf's hit rays),
    // per hit ray of the current leaf bit q set when the ray hits the leaf's
    // particle q (bit 16 + q when that hit is near), and the pairs' factors
    double* s_o = reinterpret_cast<double*>(s_wave) + wv * 3 * 64;
    unsigned int* s_mask =
        reinterpret_cast<unsigned int*>(s_wave + n_wv * kWaveOrgBytes) + wv * 64;
    float* s_gk = reinterpret_cast<float*>(s_wave + n_wv * (kWaveOrgBytes + kWaveMaskBytes)) +
                  wv * 64 * kLeafMax;
    // direct modes, per hit ray: path mode its next write offset; chunk mode
    // its chunk, the entries in it and its reserved next chunk
    uint64_t* s_w = reinterpret_cast<uint64_t*>(s_wave + n_wv * (kWaveOrgBytes + kWaveMaskBytes)) +
                    wv * 64 * 2;
    uint32_t* s_ch = reinterpret_cast<uint32_t*>(s_w);       // [cur, fill, next, -] per ray
    // the current leaf's particles: x, y, z, h in FP64
    double* s_pd = reinterpret_cast<double*>(
                       s_wave + n_wv * (kWaveOrgBytes + kWaveMaskBytes + wave_pair_bytes(MODE))) +
                   wv * kLeafMax * 4;
    if (kTerms) {
        for (int i = threadIdx.x; i < kTabIntervals; i += blockDim.x) t_erf[i] = tabs->erf_t[i];
        __syncthreads();
    }
    const double gc = tabs->gauss_c, ga = tabs->gauss_a;

    const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int64_t waves_per_dir = (g.n + 63) / 64;
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    // chunk mode: the wave's cache of pool chunks (empty to start)
    uint32_t c_next = 0, c_end = 0;
    // the wave's intersections over its packets, added to the total once (one
    // atomic per wave rather than per packet on the single counter)
    uint64_t hits_wave = 0;
    for (;;) {                                               // packets of this wave
    if (PQ) {
        unsigned long long w = 0;
        if (lane == 0) w = atomicAdd(out.queue, 1ull);
        wave = (int64_t)__shfl(w, 0, 64);
    }
    // the wave's direction and image range are uniform: scalar registers
    const int k = __builtin_amdgcn_readfirstlane((int)(wave / waves_per_dir));
    if (k >= g.n_ray) {                                      // whole wave
        if (lane == 0 && hits_wave) atomicAdd(out.hits_total, (unsigned long long)hits_wave);
        return;
    }
    const int ps = (int)((wave - (int64_t)k * waves_per_dir) * 64 + lane);
    // the ray's output row: the ray itself, or its sampled source's place
    int64_t slot = (int64_t)k * g.n + ps;
    bool sampled = true;
    if (out.src_list) {
        const int i = ps < g.n ? sampled_slot(out.src_list, out.src_n, ps) : -1;
        sampled = i >= 0;
        slot = (int64_t)i * g.n_ray + k;
    }
    const bool active = ps < g.n && sampled;
    const float4 P = p4[ps < g.n ? ps : g.n - 1];
    // the ray's origin: FP32 inputs, widened exactly where FP64 needs them
    const float rpf[3] = {P.x, P.y, P.z};
    const double u[3] = {dirs[3 * k], dirs[3 * k + 1], dirs[3 * k + 2]};
    const double B = g.box;
    // canonical once (the clamps below need canonical operands)
    const double L = __builtin_canonicalize(g.L);
    const float Lf = (float)L;
    const int64_t gid = (int64_t)k * g.n + ps;

    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    int ulo[3] = {0, 0, 0}, uhi[3] = {0, 0, 0};
    if (B > 0.0) {
        for (int a = 0; a < 3; ++a) {
            const double r = (double)rpf[a];
            double e = r + L * u[a];
            double smin = r < e ? r : e, smax = r < e ? e : r;
            lo[a] = (int)ceil((smin - g.hmax - g.phi[a]) / B - 1e-6);
            hi[a] = (int)floor((smax + g.hmax - g.plo[a]) / B + 1e-6);
            int l = active ? lo[a] : INT_MAX, h = active ? hi[a] : INT_MIN;
            for (int off = 32; off > 0; off >>= 1) {
                l = min(l, __shfl_xor(l, off, 64));
                h = max(h, __shfl_xor(h, off, 64));
            }
            ulo[a] = __builtin_amdgcn_readfirstlane(l);
            uhi[a] = __builtin_amdgcn_readfirstlane(h);
        }
    }
    // slab parameters in units of the segment length, so the segment is
    // [0, 1] and both clamps are inline constants
    float inv[3];
    int flip[3];
    for (int a = 0; a < 3; ++a) {
        float ua = (float)u[a];
        if (fabsf(ua) < 1e-20f) ua = 1e-20f;
        inv[a] = 1.0f / (ua * Lf);
        // all ones when the ray enters boxes through the high face on axis a
        flip[a] = __builtin_amdgcn_readfirstlane(inv[a] < 0.0f ? -1 : 0);
    }
    double acc = 0.0, accn = 0.0;
    uint32_t cnt = 0;
    uint64_t w = ((MODE == kModeRecord || MODE == kModePath) && active) ? out.row_off[slot] : 0;
    // stats mode: wave node visits, lane node visits, wave leaf visits, pair tests
    uint64_t st_nodes = 0, st_lanes = 0, st_leaves = 0, st_pairs = 0;
    // chunk mode: the ray's current chunk (kNoChunk before the first, kDropped
    // once the pool ran out for it: then the ray only counts), the entries in
    // it, and the next chunk once reserved.  Waves take chunks from slice
    // (wave mod kPoolSlices) first, each slice with its own counter.
    constexpr uint32_t kDropped = kNoChunk - 1;
    uint32_t cur = kNoChunk, fill = 0, nxt = kNoChunk;
    const uint32_t slice = __builtin_amdgcn_readfirstlane((uint32_t)(wave % kPoolSlices));
    const double nur = (MODE == kModeScatter && active) ? (double)out.nu[gid] : 0.0;

    // lanes of one wave can belong to two halos (at a halo boundary in tree
    // order): walk each halo's subtree in turn with that halo's lanes
    int root = 0, end = g.n_nodes;
    bool live = active;
    if (g.seg_root && active) {
        const int h = g.seg_of[ps];
        root = g.seg_root[h];
        end = g.seg_end[h];
        live = !g.seg_active || g.seg_active[h] != 0;
    }
    if (MODE == kModeColumn && g.want && active && !g.want[ps]) live = false;
    uint64_t pending = wave_ballot(live);
    while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const int sroot = __builtin_amdgcn_readfirstlane(__shfl(root, leader, 64));
    const int send = __builtin_amdgcn_readfirstlane(__shfl(end, leader, 64));
    const bool in_seg = live && root == sroot;
    pending &= ~wave_ballot(in_seg);
    for (int sx = ulo[0]; sx <= uhi[0]; ++sx)
    for (int sy = ulo[1]; sy <= uhi[1]; ++sy)
    for (int sz = ulo[2]; sz <= uhi[2]; ++sz) {
        const bool mine = in_seg && sx >= lo[0] && sx <= hi[0] && sy >= lo[1] && sy <= hi[1] &&
                          sz >= lo[2] && sz <= hi[2];
        if (wave_ballot(mine) == 0) continue;
        // the segment's end in the slab test; below the start for lanes that
        // do not walk this image, so their test always fails
        const float t_end = mine ? 1.0f : -1.0f;
        double sh[3] = {(double)sx * B, (double)sy * B, (double)sz * B};
        if (!(B > 0.0)) sh[0] = sh[1] = sh[2] = 0.0;
        const uint32_t img_code = chunk_image_code(sx, sy, sz);
        const bool shifted = (sx | sy | sz) != 0;            // wave-uniform
        // slab offsets of the entry and exit faces: the low face is padded
        // by -pad, the high face by +pad
        float oin[3], oout[3];
        for (int a = 0; a < 3; ++a) {
            const double o = (double)rpf[a] - sh[a];
            const float oa = (float)(o + (double)g.pad) * inv[a];
            const float ob = (float)(o - (double)g.pad) * inv[a];
            oin[a] = flip[a] ? ob : oa;
            oout[a] = flip[a] ? oa : ob;
        }
        // the wave walks one node sequence: the index is scalar, nodes are
        // read with scalar loads and the slab test takes its bounds from
        // scalar registers
        int node = sroot;
        while (node < send) {
            const Node nd = nodes[node];
            // entry and exit faces: a ^ ((a ^ b) & flip) swaps the pair in
            // scalar registers (a select on the uniform flag would be a
            // vector instruction per face)
            const int dx = (__float_as_int(nd.a.x) ^ __float_as_int(nd.b.x)) & flip[0];
            const int dy = (__float_as_int(nd.a.y) ^ __float_as_int(nd.b.y)) & flip[1];
            const int dz = (__float_as_int(nd.a.z) ^ __float_as_int(nd.b.z)) & flip[2];
            const float ex = __int_as_float(__float_as_int(nd.a.x) ^ dx);
            const float fx = __int_as_float(__float_as_int(nd.b.x) ^ dx);
            const float ey = __int_as_float(__float_as_int(nd.a.y) ^ dy);
            const float fy = __int_as_float(__float_as_int(nd.b.y) ^ dy);
            const float ez = __int_as_float(__float_as_int(nd.a.z) ^ dz);
            const float fz = __int_as_float(__float_as_int(nd.b.z) ^ dz);
            const float tmin = fmaxf(fmaxf(fmaxf(fmaf(ex, inv[0], -oin[0]),
                                                 fmaf(ey, inv[1], -oin[1])),
                                           fmaf(ez, inv[2], -oin[2])), 0.0f);
            const float tmax = fminf(fminf(fminf(fmaf(fx, inv[0], -oout[0]),
                                                 fmaf(fy, inv[1], -oout[1])),
                                           fmaf(fz, inv[2], -oout[2])), t_end);
            const uint64_t hm = wave_ballot(tmin <= tmax);
            if (MODE == kModeStats) {
                st_nodes += 1;
                st_lanes += __popcll(hm);
            }
            const int skip = __float_as_int(nd.a.w);
            const int leafw = __float_as_int(nd.b.w);
            if (hm == 0) {
                node = max(skip, node + 1);
                continue;
            }
            if (leafw < 0) {
                ++node;
                continue;
            }
            node = max(skip, node + 1);
            const int f = leafw >> kLeafShift;
            const int c = (f + (leafw & (kLeafMax - 1)) + 1 <= g.n) ? (leafw & (kLeafMax - 1)) + 1 : 0;
            // Leaf work compacted over the wave: the (hit ray, leaf particle)
            // pairs are spread over all 64 lanes, so a leaf that few of the
            // wave's rays reach costs few wave instructions.  Pair t is hit
            // ray t mod k_hit (by rank) and leaf particle t / k_hit; its lane
            // evaluates the canonical predicate and the chord factor and sets
            // the pair's bit in its ray's hit mask; each ray then takes its
            // hits in particle order, exactly as if it had looped over them.
            const bool hit = (hm >> lane) & 1ull;
            const int k_hit = __popcll(hm);
            const int rank = __popcll(hm & lt_mask);
            if (MODE == kModeChunk) {
                // room for every entry this leaf can add (at most c): a first
                // chunk, or the next one when the current could overflow
                const bool want = hit && cur != kDropped &&
                                  (cur == kNoChunk ||
                                   (fill + (uint32_t)c > kChunkLen && nxt == kNoChunk));
                if (wave_ballot(want)) {
                    uint32_t nc = 0;
                    const bool got = take_chunk(want, slice, lane, lt_mask, out.pool_ctr,
                                                out.slice_chunks, PQ ? kCacheBlock : 1u,
                                                c_next, c_end, nc);
                    if (want && got) {
                        if (cur == kNoChunk) {
                            out.row_first[gid] = nc;
                            cur = nc;
                            fill = 0;
                        } else {
                            out.chunk_next[cur] = nc;
                            nxt = nc;
                        }
                    } else if (want) {
                        cur = kDropped;                   // counted, not stored
                        out.pool_ctr[(size_t)kPoolSlices * kCtrStride] = 1ull;
                    }
                }
            }
            if (lane < c) {
                const float4 Q = p4[f + lane];
                s_pd[4 * lane] = (double)Q.x;
                s_pd[4 * lane + 1] = (double)Q.y;
                s_pd[4 * lane + 2] = (double)Q.z;
                s_pd[4 * lane + 3] = (double)Q.w;
            }
            if (hit) {
                s_o[rank] = (double)rpf[0];
                s_o[64 + rank] = (double)rpf[1];
                s_o[128 + rank] = (double)rpf[2];
                s_mask[rank] = 0u;
                if (MODE == kModePath) s_w[2 * rank] = w;
                if (MODE == kModeChunk) {
                    s_ch[4 * rank] = cur;
                    s_ch[4 * rank + 1] = fill;
                    s_ch[4 * rank + 2] = nxt;
                }
            }
            wave_sync();
            const int pairs = k_hit * c;
            if (MODE == kModeStats) {
                st_leaves += 1;
                st_pairs += (uint64_t)pairs;
            }
            // t / k_hit as (t + 1/2) / k_hit rounded down in FP32: the
            // quotient is at least 1/(2 k_hit) >= 1/128 away from an integer,
            // far beyond the error of the reciprocal and product (< 2^-12)
            const float rk = __builtin_amdgcn_rcpf((float)k_hit);
            // two copies of the pair loop: with and without the image shift
            // (a select per component would cost more than the adds it saves)
            auto pair_loop = [&](auto shifted_tag) {
            constexpr bool kShifted = decltype(shifted_tag)::value;
            for (int t = lane; t < pairs; t += 64) {
                const int q = (int)(((float)t + 0.5f) * rk);
                const int r = t - q * k_hit;
                const int j = f + q;
                const double* pq = s_pd + 4 * q;
                const PairGeom pg = pair_geom_d<kShifted>(pq[0], pq[1], pq[2], s_o[r],
                                                          s_o[64 + r], s_o[128 + r], sh, u);
                // clamp to [0, L]; a zero's sign cannot change |c|^2
                double tt = fmin(fmax(pg.sp, 0.0), L);
                double c0 = fma(-tt, u[0], pg.d0);
                double c1 = fma(-tt, u[1], pg.d1);
                double c2 = fma(-tt, u[2], pg.d2);
                double D2 = norm2(c0, c1, c2);
                double hj = pq[3];
                double h2 = hj * hj;
                const bool in = D2 < h2;
                bool near = false;
                if (NF) near = (pg.d0 * pg.d0 + pg.d1 * pg.d1 + pg.d2 * pg.d2) < h2;
                float gk = 0.0f;
                if (kTerms && in) gk = hit_factor(pg, u, (float)hj, L, t_erf, gc, ga);
                if (in) atomicOr(&s_mask[r], (near ? 0x10001u : 1u) << q);
                if (kTerms && !kDirect) s_gk[t] = gk;
                if (kDirect) {
                    // The entry's place: its ray's hits in this leaf are in
                    // particle order, and every pair of a lower particle of
                    // the same ray has a lower t (this iteration or earlier),
                    // so its bit is in the mask now.
                    wave_sync();
                    if (in) {
                        const uint32_t e = __popc(s_mask[r] & ((1u << q) - 1u));
                        const uint32_t bits = (kTerms ? (uint32_t)__float_as_int(gk) : img_code) |
                                              (near ? kNearBit : 0u);
                        if (MODE == kModePath) {
                            const uint64_t pos = s_w[2 * r] + e;
                            if (pos < out.hit_cap) out.path[pos] = make_int2(j, (int)bits);
                        } else {
                            // a ray that holds a chunk also holds the next one
                            // whenever this leaf can reach it (reserved above)
                            const uint32_t c0 = s_ch[4 * r], slot = s_ch[4 * r + 1] + e;
                            const uint32_t ch = slot < kChunkLen ? c0 : s_ch[4 * r + 2];
                            if (c0 < kDropped)
                                out.pool[((uint64_t)ch << kChunkShift) |
                                         (slot & (kChunkLen - 1))] = make_int2(j, (int)bits);
                        }
                    }
                }
            }
            };
            if (shifted) pair_loop(std::true_type{});
            else pair_loop(std::false_type{});
            wave_sync();
            if (kDirect && hit) {
                const uint32_t n_new = __popc(s_mask[rank] & 0xffffu);
                cnt += n_new;
                if (MODE == kModePath) w += n_new;
                if (MODE == kModeChunk && cur < kDropped) {
                    fill += n_new;
                    // a full chunk moves on to the reserved one (reserved
                    // whenever this leaf could overflow the current one)
                    if (fill >= kChunkLen && nxt != kNoChunk) {
                        cur = nxt;
                        fill -= kChunkLen;
                        nxt = kNoChunk;
                    }
                }
            }
            if (!kDirect && hit) {
                const unsigned int m = s_mask[rank];
                if (kCountOnly) cnt += __popc(m & 0xffffu);
                for (unsigned int hb = kCountOnly ? 0u : m & 0xffffu; hb; hb &= hb - 1) {
                    const int q = __ffs(hb) - 1;
                    const int j = f + q;
                    const float gk = kTerms ? s_gk[q * k_hit + rank] : 0.0f;
                    ++cnt;
                    if (MODE == kModeRecord) {
                        if (w < out.hit_cap) {
                            out.hit_j[w] = out.perm[j];
                            out.hit_img[w] = (sx + 8) | ((sy + 8) << 4) | ((sz + 8) << 8);
                            if (out.hit_fac) out.hit_fac[w] = gk;
                        }
                        ++w;
                    }
                    const bool near = NF && ((m >> (16 + q)) & 1u);
                    if (MODE == kModeScatter) {
                        if (nur != 0.0) unsafeAtomicAdd(out.y + j, (double)gk * nur);
                    } else if (near) {
                        accn += (double)((float)out.mu[j] * gk);
                    } else {
                        acc += (double)(mux[j] * gk);
                    }
                }
            }
            wave_sync();                  // the pair buffers are reused by the next leaf
        }
    }
    }   // halos of this wave
    if (active) {
        if ((MODE == kModeColumn || MODE == kModeRecord) && live && out.N) out.N[gid] = acc;
        if (MODE == kModeColumn && live && NF) out.Nn[gid] = accn;
        if (MODE == kModeCount || MODE == kModeChunk || MODE == kModeStats) out.row_cnt[slot] = cnt;
    }
    uint64_t c64 = cnt;
    for (int off = 32; off > 0; off >>= 1) c64 += __shfl_xor(c64, off, 64);
    hits_wave += c64;
    const uint64_t rays = MODE == kModeStats ? (uint64_t)__popcll(wave_ballot(active)) : 0;
    if (MODE == kModeStats && lane == 0) {
        atomicAdd(out.stats + 0, (unsigned long long)rays);
        atomicAdd(out.stats + 1, (unsigned long long)st_nodes);
        atomicAdd(out.stats + 2, (unsigned long long)st_lanes);
        atomicAdd(out.stats + 3, (unsigned long long)st_leaves);
        atomicAdd(out.stats + 4, (unsigned long long)st_pairs);
        atomicAdd(out.stats + 5, (unsigned long long)c64);
    }
    if (!PQ) {
        if (lane == 0 && hits_wave) atomicAdd(out.hits_total, (unsigned long long)hits_wave);
        return;
    }
    }   // packets of this wave
}

// One-pass recording, second step: each row's entries from its chain of
// chunks into the row-ordered path array, with the chord factor of each.
// Every row's chain holds exactly ceil(count / kChunkLen) chunks.  The chain
// is a sequence of dependent loads, so a row takes only kCompactLanes lanes
// (each copies kChunkLen / kCompactLanes entries of a chunk) and a wave
// follows 64 / kCompactLanes chains at once; the next link is loaded before
// the chunk is copied.
// The factor is evaluated here rather than in the walk: in the walk's pair
// loop most lanes hold pairs that miss, and every lane of a wave pays for the
// instructions; here every lane holds a hit.  The arithmetic is the walk's
// (same pair geometry and chord factor, FP64 without contraction), so the
// factors are those every other recording produces.
constexpr int kCompactLanes = 8;

__global__ void __launch_bounds__(256)
k_compact_chunks(const uint64_t* __restrict__ row_off, const uint32_t* __restrict__ row_first,
                 const uint32_t* __restrict__ chunk_next, const int2* __restrict__ pool,
                 int64_t n_rows, int2* __restrict__ path, const float4* __restrict__ p4,
                 const double* __restrict__ dirs, const KernelTables* __restrict__ tabs,
                 TraceGeom g)
{
    __shared__ float4 t_erf[kTabIntervals];
    for (int i = threadIdx.x; i < kTabIntervals; i += blockDim.x) t_erf[i] = tabs->erf_t[i];
    __syncthreads();
    const double gc = tabs->gauss_c, ga = tabs->gauss_a;
    const double L = __builtin_canonicalize(g.L), B = g.box;
    const int lane = threadIdx.x & (kCompactLanes - 1);
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x / kCompactLanes);
    for (int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kCompactLanes;
         row < n_rows; row += stride) {
        const uint64_t a = row_off[row], b = row_off[row + 1];
        if (a == b) continue;
        // the ray: source ps (tree order) along direction k
        const int k = (int)(row / g.n);
        const int ps = (int)(row - (int64_t)k * g.n);
        const float4 P = p4[ps];
        const double o0 = (double)P.x, o1 = (double)P.y, o2 = (double)P.z;
        const double u[3] = {dirs[3 * k], dirs[3 * k + 1], dirs[3 * k + 2]};
        constexpr int kPer = kChunkLen / kCompactLanes;     // entries per lane per chunk
        constexpr uint32_t kNoShift = kImgBias | (kImgBias << 10) | (kImgBias << 20);
        uint32_t ch = row_first[row];
        for (uint64_t e = a; e < b; e += kChunkLen) {
            const uint32_t nxt = e + kChunkLen < b ? chunk_next[ch] : 0u;
            const int2* src = pool + (uint64_t)ch * kChunkLen;
            // the lane's entries of the chunk, then their particles, all in
            // flight together.  A chunk is whole in the pool, so its slots
            // past the row end are read too; their (stale) indices are
            // replaced by particle 0 before the particle loads.
            int2 en[kPer];
            float4 Q[kPer];
#pragma unroll
            for (int q = 0; q < kPer; ++q) en[q] = src[q * kCompactLanes + lane];
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                if (e + (uint64_t)(q * kCompactLanes + lane) >= b) en[q].x = 0;
                Q[q] = p4[en[q].x];
            }
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int i = q * kCompactLanes + lane;
                if (e + i < b) {
                    const uint32_t code = (uint32_t)en[q].y;
                    // the image shift, 0 for the source's own image as in the walk
                    double sh[3] = {0.0, 0.0, 0.0};
                    if (B > 0.0 && (code & ~kNearBit) != kNoShift) {
                        sh[0] = (double)((int)(code & 1023u) - kImgBias) * B;
                        sh[1] = (double)((int)((code >> 10) & 1023u) - kImgBias) * B;
                        sh[2] = (double)((int)((code >> 20) & 1023u) - kImgBias) * B;
                    }
                    const PairGeom pg = pair_geom(Q[q], o0, o1, o2, sh, u);
                    const float gk = hit_factor(pg, u, Q[q].w, L, t_erf, gc, ga);
                    path[e + i] = make_int2(
                        en[q].x, (int)((uint32_t)__float_as_int(gk) | (code & kNearBit)));
                }
            }
            ch = nxt;
        }
    }
}
#pragma clang fp contract(on)

__global__ void k_zero_u64(unsigned long long* p)
{
    if (threadIdx.x == 0) *p = 0ull;
}

}  // namespace

void fill_kernel_tables(KernelTables* host)
{
    const KConst kc = kconst();
    const double t = kc.t, C = kc.C;
    fit_cubics(host->erf_t, [&](double z) { return std::erf(t * z); });
    host->gauss_c = C;
    host->gauss_a = t * t / std::log(2.0);
}

// The wave-cooperative walk: one wave per 64 sources of one direction, or
// (packet queue) a resident grid taking packets from a counter.  The near/far
// variant only for the modes that split near hits.
template <int MODE, bool NF>
static void launch_wave_nf(Ctx& c, RayOut o, int bs, size_t lds, int64_t waves)
{
    const unsigned nb = (unsigned)((waves * 64 + bs - 1) / bs);
    // the persistent form for the walks that record, count or evaluate
    constexpr bool kQueued = MODE == kModeColumn || MODE == kModeCount || MODE == kModePath ||
                             MODE == kModeChunk;
    if (kQueued && c.packet_queue) {
        // a kernel, not a memset, clears the counter (the launch may be captured)
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, c.stream, c.red + kRedQueue);
        o.queue = c.red + kRedQueue;
        int per_cu = 0, cus = 0, dev = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_trace_wave<MODE, NF, kQueued>,
                                                         bs, lds) != hipSuccess || per_cu < 1)
            per_cu = 1;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess || cus < 1)
            cus = 1;
        const unsigned resident = (unsigned)std::min<int64_t>(nb, (int64_t)per_cu * cus);
        hipLaunchKernelGGL((k_trace_wave<MODE, NF, kQueued>), dim3(resident), dim3(bs), lds,
                           c.stream, c.nodes, c.p4, c.mux_s, c.dirs, c.tables, c.geom, o);
        return;
    }
    hipLaunchKernelGGL((k_trace_wave<MODE, NF, false>), dim3(nb), dim3(bs), lds, c.stream,
                       c.nodes, c.p4, c.mux_s, c.dirs, c.tables, c.geom, o);
}

template <int MODE>
static void launch_wave(Ctx& c, RayOut o)
{
    const int bs = c.prm.block_size > 0 ? c.prm.block_size : 128;
    const int64_t waves = ((c.n + 63) / 64) * (int64_t)c.n_ray;
    const size_t lds = wave_lds_bytes(MODE, bs);
    constexpr bool kSplit = MODE == kModeColumn || MODE == kModePath || MODE == kModeChunk;
    if (kSplit && o.near_far) launch_wave_nf<MODE, kSplit>(c, o, bs, lds, waves);
    else launch_wave_nf<MODE, false>(c, o, bs, lds, waves);
}

template <int MODE>
static void launch_one(Ctx& c, RayOut o)
{
    if (c.prm.traversal == 1) {
        const int bs = c.prm.block_size > 0 ? c.prm.block_size : 128;
        const int64_t n_rays = c.n * (int64_t)c.n_ray;
        const unsigned nb = (unsigned)((n_rays + bs - 1) / bs);
        hipLaunchKernelGGL(k_trace<MODE>, dim3(nb), dim3(bs), 0, c.stream, c.nodes, c.p4, c.mux_s,
                           c.dirs, c.tables, c.geom, o);
    } else {
        launch_wave<MODE>(c, o);
    }
}

static hipError_t launch_mode(Ctx& c, int mode, RayOut o)
{
    if (mode == kModeColumn) launch_one<kModeColumn>(c, o);
    else if (mode == kModeCount) launch_one<kModeCount>(c, o);
    else if (mode == kModeRecord) launch_one<kModeRecord>(c, o);
    else if (mode == kModePath) launch_one<kModePath>(c, o);
    else if (mode == kModeStats) {
        // the counters are those of the wave-cooperative walk
        launch_wave<kModeStats>(c, o);
    } else launch_one<kModeScatter>(c, o);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// columns from recorded paths: N_row = sum over the row's hits of mux_j * factor.
// G lanes share a row; they stride through it (coalesced 8-byte loads) and
// reduce their partial sums in FP64.
// ---------------------------------------------------------------------------
template <int G, bool NF>
__global__ void __launch_bounds__(256)
k_path_columns(const uint64_t* __restrict__ row_off, const int2* __restrict__ path,
               const float* __restrict__ mux, int64_t n_rows, double* __restrict__ N, int64_t n,
               const int32_t* __restrict__ seg_of, const int32_t* __restrict__ seg_active,
               const uint8_t* __restrict__ want, const int32_t* __restrict__ list,
               int64_t list_n, double* __restrict__ Nn, const double* __restrict__ mu)
{
    const int lane = threadIdx.x & (G - 1);
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x / G);
    const long long* p = reinterpret_cast<const long long*>(path);
    // with a source list, the rows are its sources' rays: v -> (k, list[i])
    const int64_t n_iter = list ? list_n * (n_rows / n) : n_rows;
    // the G lanes of a group share the row, so the loop is uniform per group
    for (int64_t v = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G; v < n_iter;
         v += stride) {
        const int64_t row = list ? (v / list_n) * n + list[v % list_n] : v;
        // rows of halos that have stopped iterating keep their last columns
        if (seg_active && seg_active[seg_of[row % n]] == 0) continue;
        if (want && !want[row % n]) continue;     // not updated in this step
        const uint64_t a = row_off[row], b = row_off[row + 1];
        double acc = 0.0, accn = 0.0;
        // Lanes stride through the row one entry at a time, so the particle
        // gathers of one instruction are consecutive intersections along the
        // ray and share cache lines (measured: grouping four consecutive
        // entries per lane is slower here).  Four streaming loads in flight per
        // lane; entries past the row end read as (particle 0, factor 0).
        for (uint64_t e = a + lane; e < b; e += 4 * G) {
            const long long v0 = __builtin_nontemporal_load(p + e);
            const long long v1 = e + G < b ? __builtin_nontemporal_load(p + e + G) : 0ll;
            const long long v2 = e + 2 * G < b ? __builtin_nontemporal_load(p + e + 2 * G) : 0ll;
            const long long v3 = e + 3 * G < b ? __builtin_nontemporal_load(p + e + 3 * G) : 0ll;
            const float m0 = mux[(int)v0], m1 = mux[(int)v1];
            const float m2 = mux[(int)v2], m3 = mux[(int)v3];
            if (!NF) {
                acc += (double)(m0 * __int_as_float((int)(v0 >> 32)));
                acc += (double)(m1 * __int_as_float((int)(v1 >> 32)));
                acc += (double)(m2 * __int_as_float((int)(v2 >> 32)));
                acc += (double)(m3 * __int_as_float((int)(v3 >> 32)));
            } else {
                // near hits (sign bit) add mu * factor to the near column
                const long long vv[4] = {v0, v1, v2, v3};
                const float mm[4] = {m0, m1, m2, m3};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t bits = (uint32_t)(vv[q] >> 32);
                    const float f = __int_as_float((int)(bits & ~kNearBit));
                    if (bits & kNearBit) accn += (double)((float)mu[(int)vv[q]] * f);
                    else acc += (double)(mm[q] * f);
                }
            }
        }
        for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
        if (NF)
            for (int off = G / 2; off > 0; off >>= 1) accn += __shfl_xor(accn, off, G);
        if (lane == 0) N[row] = acc;
        if (NF && lane == 0) Nn[row] = accn;
    }
}

// Columns from recorded paths, streamed (the full sweep of a plain product):
// a block takes R consecutive rows, whose entries are one contiguous range of
// the path array.  It reads that range in windows of kStreamWin entries,
// eight independent coalesced 8-byte loads per thread (16 KB in flight per
// block instead of a few hundred bytes per row), gathers mux and stages the
// products in LDS; then 256 / R lanes per row sum the row's products in FP64
// and reduce them with shuffles.  Rows that straddle windows carry their
// partial sums across.  A product mux_j * factor is an FP32 value (widened
// exactly), so LDS holds it in 4 bytes.  The next block's row offsets are
// loaded while the current block streams.  The products are those of the
// row-group kernel; only the FP64 summation order differs.
// Measured on MI355X over the recorded paths of the 2.1M-particle field
// (7.35e9 intersections): 12.3 ms per product against 15.5 ms for 32 lanes
// per row; 4096-entry windows 13.8 ms, 1024-entry windows 14.9 ms.  On the
// 262144-particle halo both kernels take 2.70 ms.
constexpr int kStreamWin = 2048;

template <int R>
__global__ void __launch_bounds__(256)
k_path_stream(const uint64_t* __restrict__ row_off, const int2* __restrict__ path,
              const float* __restrict__ mux, int64_t n_rows, double* __restrict__ N)
{
    constexpr int G = 256 / R;                 // lanes per row in the reduction
    constexpr int kPer = kStreamWin / 256;     // entries per thread per window
    __shared__ float s_prod[kStreamWin];
    __shared__ uint64_t s_off[R + 1];
    const int t = threadIdx.x;
    const int r = t / G, g = t % G;
    const long long* p = reinterpret_cast<const long long*>(path);
    const int64_t n_blk = (n_rows + R - 1) / R;
    int64_t blk = blockIdx.x;
    // row offsets of the block (threads 0..R), loaded one block ahead
    uint64_t off = 0;
    if (blk < n_blk && t <= R && blk * R + t <= n_rows) off = row_off[blk * R + t];
    for (; blk < n_blk; blk += gridDim.x) {
        const int64_t r0 = blk * R;
        const int rn = (int)(n_rows - r0 < R ? n_rows - r0 : R);
        __syncthreads();                        // the previous block's reads are done
        if (t <= rn) s_off[t] = off;
        const int64_t nr0 = r0 + (int64_t)gridDim.x * R;
        if (nr0 < n_rows && t <= R && nr0 + t <= n_rows) off = row_off[nr0 + t];
        __syncthreads();
        const uint64_t e0 = s_off[0], e1 = s_off[rn];
        const uint64_t lo = r < rn ? s_off[r] : e1, hi = r < rn ? s_off[r + 1] : e1;
        double acc = 0.0;
        for (uint64_t w0 = e0; w0 < e1; w0 += kStreamWin) {
            long long v[kPer];
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                const uint64_t e = w0 + t + 256 * i;
                v[i] = e < e1 ? __builtin_nontemporal_load(p + e) : 0ll;
            }
#pragma unroll
            for (int i = 0; i < kPer; ++i)
                s_prod[t + 256 * i] = mux[(int)v[i]] * __int_as_float((int)(v[i] >> 32));
            __syncthreads();
            const uint64_t a = lo > w0 ? lo : w0;
            const uint64_t b = hi < w0 + kStreamWin ? hi : w0 + kStreamWin;
            for (uint64_t e = a + g; e < b; e += G) acc += (double)s_prod[e - w0];
            __syncthreads();                    // the window is consumed
        }
        for (int off2 = G / 2; off2 > 0; off2 >>= 1) acc += __shfl_xor(acc, off2, G);
        if (g == 0 && r < rn) N[r0 + r] = acc;
    }
}

namespace {

// sampled rows of the recorded paths: entries per row, then the entries
// (input index of the particle, factor K/h^2 without the near flag)
__global__ void k_path_row_counts(const uint64_t* __restrict__ row_off,
                                  const int64_t* __restrict__ rows, int m,
                                  uint64_t* __restrict__ cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) cnt[i] = row_off[rows[i] + 1] - row_off[rows[i]];
}

__global__ void k_path_row_copy(const uint64_t* __restrict__ row_off, const int2* __restrict__ path,
                                const int32_t* __restrict__ perm, const int64_t* __restrict__ rows,
                                const uint64_t* __restrict__ dst_off, int m,
                                int32_t* __restrict__ hit_j, float* __restrict__ hit_fac)
{
    for (int i = blockIdx.x; i < m; i += gridDim.x) {
        const uint64_t a = row_off[rows[i]], b = row_off[rows[i] + 1], o = dst_off[i];
        for (uint64_t e = a + threadIdx.x; e < b; e += blockDim.x) {
            const int2 v = path[e];
            hit_j[o + (e - a)] = perm[v.x];
            hit_fac[o + (e - a)] = __int_as_float(v.y & (int)~kNearBit);
        }
    }
}

}  // namespace

hipError_t launch_path_rows(Ctx& c, const int64_t* rows, int m, uint64_t* cnt,
                            const uint64_t* dst_off, int32_t* hit_j, float* hit_fac)
{
    if (m <= 0) return hipSuccess;
    if (!dst_off) {
        hipLaunchKernelGGL(k_path_row_counts, dim3((m + 255) / 256), dim3(256), 0, c.stream,
                           c.row_off, rows, m, cnt);
    } else {
        hipLaunchKernelGGL(k_path_row_copy, dim3((unsigned)std::min(m, 4096)), dim3(256), 0,
                           c.stream, c.row_off, c.path, c.perm, rows, dst_off, m, hit_j, hit_fac);
    }
    return hipGetLastError();
}

hipError_t launch_columns(Ctx& c)
{
    RayOut o{};
    o.N = c.N_s;
    o.perm = c.perm;
    o.hits_total = c.red + kRedHits;
    o.near_far = c.near_far;
    o.Nn = c.Nn_s;
    o.mu = c.mu_s;
    return launch_mode(c, kModeColumn, o);
}

hipError_t launch_count_hits(Ctx& c, uint64_t* row_cnt)
{
    RayOut o{};
    o.row_cnt = row_cnt;
    o.perm = c.perm;
    o.hits_total = c.red + kRedScratch;   // counting is not a column evaluation
    return launch_mode(c, kModeCount, o);
}

hipError_t launch_count_rows(Ctx& c, const int32_t* src_list, int32_t src_n, uint64_t* row_cnt)
{
    RayOut o{};
    o.row_cnt = row_cnt;
    o.perm = c.perm;
    o.hits_total = c.red + kRedScratch;
    o.src_list = src_list;
    o.src_n = src_n;
    return launch_mode(c, kModeCount, o);
}

hipError_t launch_record_rows(Ctx& c, const int32_t* src_list, int32_t src_n,
                              const uint64_t* row_off, int32_t* hit_j, int32_t* hit_img,
                              float* hit_fac, uint64_t cap)
{
    RayOut o{};
    o.hit_cap = cap;
    o.row_off = row_off;
    o.hit_j = hit_j;
    o.hit_img = hit_img;
    o.hit_fac = hit_fac;
    o.perm = c.perm;
    o.hits_total = c.red + kRedScratch;
    o.src_list = src_list;
    o.src_n = src_n;
    return launch_mode(c, kModeRecord, o);
}

hipError_t launch_trace_stats(Ctx& c, uint64_t* row_cnt, unsigned long long* stats)
{
    RayOut o{};
    o.row_cnt = row_cnt;
    o.perm = c.perm;
    o.hits_total = c.red + kRedScratch;
    o.stats = stats;
    return launch_mode(c, kModeStats, o);
}

hipError_t launch_record_hits(Ctx& c, const uint64_t* row_off, int32_t* hit_j, int32_t* hit_img,
                              uint64_t cap)
{
    RayOut o{};
    o.hit_cap = cap;
    o.row_off = row_off;
    o.hit_j = hit_j;
    o.hit_img = hit_img;
    o.perm = c.perm;
    o.hits_total = c.red + kRedScratch;
    return launch_mode(c, kModeRecord, o);
}

hipError_t launch_record_chunks(Ctx& c, uint64_t* row_cnt)
{
    RayOut o{};
    o.row_cnt = row_cnt;
    o.perm = c.perm;
    o.hits_total = c.red + kRedScratch;
    o.near_far = c.near_far;
    o.pool = c.pool;
    o.chunk_next = c.chunk_next;
    o.row_first = c.row_first;
    o.pool_ctr = c.pool_ctr;
    o.slice_chunks = c.slice_chunks;
    launch_wave<kModeChunk>(c, o);
    return hipGetLastError();
}

hipError_t launch_compact_chunks(Ctx& c)
{
    const int64_t n_rows = c.n * (int64_t)c.n_ray;
    if (n_rows == 0) return hipSuccess;
    const unsigned nb = stride_blocks(n_rows, 256 / kCompactLanes);
    hipLaunchKernelGGL(k_compact_chunks, dim3(nb), dim3(256), 0, c.stream, c.row_off,
                       c.row_first, c.chunk_next, c.pool, n_rows, c.path, c.p4, c.dirs, c.tables,
                       c.geom);
    return hipGetLastError();
}

hipError_t launch_record_paths(Ctx& c, const uint64_t* row_off, int2* path, uint64_t cap)
{
    RayOut o{};
    o.hit_cap = cap;
    o.row_off = row_off;
    o.path = path;
    o.perm = c.perm;
    o.hits_total = c.red + kRedScratch;
    o.near_far = c.near_far;
    return launch_mode(c, kModePath, o);
}

hipError_t launch_scatter_traverse(Ctx& c, const float* nu, double* y)
{
    RayOut o{};
    o.nu = nu;
    o.y = y;
    o.perm = c.perm;
    o.hits_total = c.red + kRedScratch;
    return launch_mode(c, kModeScatter, o);
}

namespace {

template <int G>
hipError_t launch_path_g(Ctx& c, int64_t n_rows, unsigned nb)
{
    if (c.near_far)
        hipLaunchKernelGGL((k_path_columns<G, true>), dim3(nb), dim3(256), 0, c.stream, c.row_off,
                           c.path, c.mux_s, n_rows, c.N_s, c.n, c.geom.seg_of, c.geom.seg_active,
                           c.geom.want, c.row_list, c.row_list_n, c.Nn_s, c.mu_s);
    else
        hipLaunchKernelGGL((k_path_columns<G, false>), dim3(nb), dim3(256), 0, c.stream,
                           c.row_off, c.path, c.mux_s, n_rows, c.N_s, c.n, c.geom.seg_of,
                           c.geom.seg_active, c.geom.want, c.row_list, c.row_list_n, nullptr,
                           nullptr);
    return hipGetLastError();
}

}  // namespace

// rows per block of the streamed product: on average at most one window of
// entries per block, between 4 rows (64 lanes each) and 64 rows (4 lanes each)
static int stream_rows(double mean)
{
    int R = 64;
    while (R > 4 && R * mean > kStreamWin) R /= 2;
    return R;
}

hipError_t launch_path_stream(Ctx& c)
{
    const int64_t n_rows = c.n * (int64_t)c.n_ray;
    if (n_rows == 0) return hipSuccess;
    const double mean = (double)c.path_hits / (double)n_rows;
    const int R = stream_rows(mean);
    const unsigned nb = stride_blocks(n_rows, R);
    if (R == 64)
        hipLaunchKernelGGL(k_path_stream<64>, dim3(nb), dim3(256), 0, c.stream, c.row_off,
                           c.path, c.mux_s, n_rows, c.N_s);
    else if (R == 32)
        hipLaunchKernelGGL(k_path_stream<32>, dim3(nb), dim3(256), 0, c.stream, c.row_off,
                           c.path, c.mux_s, n_rows, c.N_s);
    else if (R == 16)
        hipLaunchKernelGGL(k_path_stream<16>, dim3(nb), dim3(256), 0, c.stream, c.row_off,
                           c.path, c.mux_s, n_rows, c.N_s);
    else if (R == 8)
        hipLaunchKernelGGL(k_path_stream<8>, dim3(nb), dim3(256), 0, c.stream, c.row_off,
                           c.path, c.mux_s, n_rows, c.N_s);
    else
        hipLaunchKernelGGL(k_path_stream<4>, dim3(nb), dim3(256), 0, c.stream, c.row_off,
                           c.path, c.mux_s, n_rows, c.N_s);
    return hipGetLastError();
}

hipError_t launch_path_columns(Ctx& c, int group)
{
    const int64_t n_rows = c.n * (int64_t)c.n_ray;
    const int bs = 256;
    const int64_t n_iter = c.row_list ? c.row_list_n * (int64_t)c.n_ray : n_rows;
    if (n_iter == 0) return hipSuccess;
    const unsigned nb = stride_blocks(n_iter, bs / group);
    if (group == 64) return launch_path_g<64>(c, n_rows, nb);
    if (group == 32) return launch_path_g<32>(c, n_rows, nb);
    if (group == 16) return launch_path_g<16>(c, n_rows, nb);
    return launch_path_g<8>(c, n_rows, nb);
}

}  // namespace rrt
