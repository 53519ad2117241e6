// Tree construction on the GPU: scene bounds, 63-bit Morton keys, LSD radix
// sort of (key, index) pairs, binary radix tree over the sorted keys (ties
// broken by the sorted position), bottom-up box refit and a depth-first node
// layout with skip links for stackless traversal.
//
// The tree is an acceleration structure for the question the column needs
// answered (Sec. 4.1.1: which particles' kernel spheres a ray intersects); it
// changes no result.  Its layout is fully determined by the keys, so it can be
// compared bit for bit with an independently built reference.
#include "internal.h"

#include <algorithm>
#include <vector>

namespace rrt {

namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// bounds and input validation
// ---------------------------------------------------------------------------
__global__ void k_bounds(const float* __restrict__ pos, const float* __restrict__ h,
                         const float* __restrict__ mu, const float* __restrict__ nH,
                         const float* __restrict__ T, int64_t n, float* __restrict__ part)
{
    __shared__ float s[8][kBlock];
    float lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY;
    float hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY;
    float hm = 0.f, bad = 0.f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        float x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
        float hh = h[i];
        bool ok = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(hh) && hh > 0.f &&
                  isfinite(mu[i]) && mu[i] >= 0.f && isfinite(nH[i]) && nH[i] > 0.f &&
                  isfinite(T[i]) && T[i] > 0.f;
        if (!ok) { bad = 1.f; continue; }
        lo0 = fminf(lo0, x); lo1 = fminf(lo1, y); lo2 = fminf(lo2, z);
        hi0 = fmaxf(hi0, x); hi1 = fmaxf(hi1, y); hi2 = fmaxf(hi2, z);
        hm = fmaxf(hm, hh);
    }
    int t = threadIdx.x;
    s[0][t] = lo0; s[1][t] = lo1; s[2][t] = lo2;
    s[3][t] = hi0; s[4][t] = hi1; s[5][t] = hi2; s[6][t] = hm; s[7][t] = bad;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (t < w) {
            for (int q = 0; q < 3; ++q) s[q][t] = fminf(s[q][t], s[q][t + w]);
            for (int q = 3; q < 8; ++q) s[q][t] = fmaxf(s[q][t], s[q][t + w]);
        }
        __syncthreads();
    }
    if (t < 8) part[blockIdx.x * 8 + t] = s[t][0];
}

// ---------------------------------------------------------------------------
// Morton keys: 21 bits per axis, x in the highest bit of each triple
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// Key = (halo << 3*bits) | Morton code with `bits` bits per axis.  A single
// halo uses 21 bits per axis and no halo field.
__global__ void k_morton(const float* __restrict__ pos, int64_t n, double lo0, double lo1,
                         double lo2, double scale, int bits, const int64_t* __restrict__ halo_off,
                         int n_halo, uint64_t* __restrict__ keys, int32_t* __restrict__ vals)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double lo[3] = {lo0, lo1, lo2};
    const double qmax = (double)((1u << bits) - 1u);
    uint64_t q[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double v = floor(((double)pos[3 * i + a] - lo[a]) * scale);
        v = v < 0.0 ? 0.0 : (v > qmax ? qmax : v);
        q[a] = (uint64_t)v;
    }
    uint64_t key = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
    if (n_halo > 1) {
        int a = 0, b = n_halo;                    // halo_off[a] <= i < halo_off[b]
        while (b - a > 1) {
            int m = (a + b) >> 1;
            if (halo_off[m] <= i) a = m;
            else b = m;
        }
        key |= (uint64_t)a << (3 * bits);
    }
    keys[i] = key;
    vals[i] = (int32_t)i;
}

__global__ void k_seg_of(const uint64_t* __restrict__ keys, int64_t n, int shift,
                         int32_t* __restrict__ seg)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) seg[i] = shift >= 64 ? 0 : (int32_t)(keys[i] >> shift);
}

// ---------------------------------------------------------------------------
// exclusive scan (block = 256 threads x 4 items, recursive over block sums)
// ---------------------------------------------------------------------------
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

template <typename T>
__device__ T block_exclusive_scan(T v, T* sh, T* total)
{
    // Hillis-Steele over 256 thread values in LDS
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        T add = t >= off ? sh[t - off] : T(0);
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    T incl = sh[t];
    *total = sh[kBlock - 1];
    __syncthreads();
    return incl - v;
}

template <typename T>
__global__ void k_scan_tiles(const T* in, T* out, int64_t m, T* __restrict__ sums)
{
    __shared__ T sh[kBlock];
    int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * kScanItems;
    T v[kScanItems];
    T acc = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = (base + q < m) ? in[base + q] : T(0);
        acc += v[q];
    }
    T total;
    T pre = block_exclusive_scan<T>(acc, sh, &total);
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        if (base + q < m) out[base + q] = pre;
        pre += v[q];
    }
    if (threadIdx.x == 0 && sums) sums[blockIdx.x] = total;
}

template <typename T>
__global__ void k_scan_add(T* __restrict__ out, int64_t m, const T* __restrict__ offs)
{
    int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * kScanItems;
    T o = offs[blockIdx.x];
#pragma unroll
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < m) out[base + q] += o;
}

template <typename T>
size_t scan_tmp_need(int64_t m)
{
    size_t need = 0;
    while (m > kScanTile) {
        m = (m + kScanTile - 1) / kScanTile;
        need += (size_t)m * 2 * sizeof(T) + 256;
    }
    return need + 256;
}

template <typename T>
hipError_t scan_rec(hipStream_t st, const T* in, T* out, int64_t m, char* tmp)
{
    if (m <= 0) return hipSuccess;
    int64_t nb = (m + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_tiles<T>, dim3(1), dim3(kBlock), 0, st, in, out, m,
                           (T*)nullptr);
        return hipGetLastError();
    }
    T* sums = reinterpret_cast<T*>(tmp);
    T* sums_x = sums + nb;
    char* next = tmp + (((size_t)nb * 2 * sizeof(T) + 255) / 256) * 256;
    hipLaunchKernelGGL(k_scan_tiles<T>, dim3((unsigned)nb), dim3(kBlock), 0, st, in, out, m,
                       sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_rec<T>(st, sums, sums_x, nb, next);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add<T>, dim3((unsigned)nb), dim3(kBlock), 0, st, out, m,
                       (const T*)sums_x);
    return hipGetLastError();
}

template <typename T>
hipError_t scan_exclusive(Ctx& c, const T* in, T* out, int64_t m)
{
    Scratch<char> tmp(c);
    hipError_t e = tmp.get(scan_tmp_need<T>(m));
    if (e != hipSuccess) return e;
    return scan_rec<T>(c.stream, in, out, m, tmp.p);
}

// ---------------------------------------------------------------------------
// LSD radix sort of (uint64 key, int32 value), 8-bit digits, stable per pass
// ---------------------------------------------------------------------------
constexpr int kSortRounds = 16;                  // items per thread per tile
constexpr int kSortTile = kBlock * kSortRounds;  // 4096 items per tile
constexpr int kWaves = kBlock / 64;

__global__ void k_digit_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                             uint32_t* __restrict__ hist, int64_t n_tiles)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = blockIdx.x * (int64_t)kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        int64_t i = base + r * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

__global__ void k_digit_scatter(const uint64_t* __restrict__ kin, const int32_t* __restrict__ vin,
                                uint64_t* __restrict__ kout, int32_t* __restrict__ vout,
                                int64_t n, int shift, const uint32_t* __restrict__ offs,
                                int64_t n_tiles)
{
    __shared__ uint32_t running[256];
    __shared__ uint32_t wcnt[kWaves][256];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    running[t] = offs[t * n_tiles + blockIdx.x];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t base = blockIdx.x * (int64_t)kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        for (int w = 0; w < kWaves; ++w) wcnt[w][t] = 0;
        __syncthreads();
        int64_t i = base + r * kBlock + t;
        bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0ull;
        int32_t val = valid ? vin[i] : 0;
        uint32_t d = (uint32_t)(key >> shift) & 255u;
        // lanes of this wave holding the same digit, by one ballot per digit bit
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t bb = __ballot(valid && bit);
            m &= bit ? bb : ~bb;
        }
        uint32_t rank = (uint32_t)__popcll(m & lt);
        if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(m);
        __syncthreads();
        if (valid) {
            uint32_t pre = running[d];
            for (int w = 0; w < wave; ++w) pre += wcnt[w][d];
            uint32_t dst = pre + rank;
            if (dst < (uint64_t)n) {
                kout[dst] = key;
                vout[dst] = val;
            }
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kWaves; ++w) add += wcnt[w][t];
        running[t] += add;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// binary radix tree (internal node i covers a key range; its split is where the
// highest differing bit of the range's first and last augmented keys changes)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int prefix_len(const uint64_t* __restrict__ k, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    uint64_t a = k[i], b = k[j];
    if (a == b) return 64 + __clz((unsigned)(i ^ j));
    return __clzll(a ^ b);
}

__global__ void k_radix_tree(const uint64_t* __restrict__ k, int n, int32_t* __restrict__ left,
                             int32_t* __restrict__ right, int32_t* __restrict__ parent,
                             int32_t* __restrict__ first, int32_t* __restrict__ last)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int d = (prefix_len(k, n, i, i + 1) - prefix_len(k, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = prefix_len(k, n, i, i - d);
    int lmax = 2;
    while (prefix_len(k, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (prefix_len(k, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = prefix_len(k, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (prefix_len(k, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int split = i + s * d + (d < 0 ? -1 : 0);
    int f = i < j ? i : j, la = i < j ? j : i;
    int lc = (f == split) ? ~split : split;
    int rc = (la == split + 1) ? ~(split + 1) : split + 1;
    if (split < 0 || split + 1 > n - 1) return;   // cannot happen for distinct augmented keys
    left[i] = lc;
    right[i] = rc;
    first[i] = f;
    last[i] = la;
    parent[lc >= 0 ? lc : (n - 1) + ~lc] = i;
    parent[rc >= 0 ? rc : (n - 1) + ~rc] = i;
}

__device__ __forceinline__ float ld_f(const float* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_i(const int32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_f(float* p, float v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_i(int32_t* p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct ChildInfo {
    float lo[3], hi[3];
    int cnt, dfs, seg;
};

__device__ __forceinline__ ChildInfo child_info(int c, const float4* __restrict__ p4,
                                                const float* klo, const float* khi,
                                                const int32_t* kcnt, const int32_t* kdfs,
                                                const int32_t* kseg,
                                                const int32_t* __restrict__ seg_of)
{
    ChildInfo r;
    if (c < 0) {
        float4 p = p4[~c];
        r.lo[0] = p.x - p.w; r.lo[1] = p.y - p.w; r.lo[2] = p.z - p.w;
        r.hi[0] = p.x + p.w; r.hi[1] = p.y + p.w; r.hi[2] = p.z + p.w;
        r.cnt = 1;
        r.dfs = 1;
        r.seg = seg_of[~c];
    } else {
        for (int a = 0; a < 3; ++a) {
            r.lo[a] = ld_f(klo + 3 * c + a);
            r.hi[a] = ld_f(khi + 3 * c + a);
        }
        r.cnt = ld_i(kcnt + c);
        r.dfs = ld_i(kdfs + c);
        r.seg = ld_i(kseg + c);
    }
    return r;
}

// A subtree becomes one leaf when it holds at most leaf_max particles, all of
// one halo (so no leaf ever mixes independent problems).
__device__ __forceinline__ bool collapses(int cnt, int seg, int leaf_max)
{
    return cnt <= leaf_max && seg >= 0;
}

// Bottom-up: the second thread to reach a node combines both children.
// Everything threads share here (the nodes' bounds, counts, layout sizes and
// halos, and the arrival flags) is read and written with agent-scope atomics,
// which are coherent across the device's L2 caches without a fence.  What
// the protocol needs besides is order: a node's results are complete before
// its parent's flag counts the arrival (wait for the stores), and a child's
// results are read only after the flag showed both arrived (a compiler
// barrier; the loads are issued after the atomic returns).  A full fence
// would write back and invalidate the L2 at every level of every thread.
__device__ __forceinline__ void stores_done()
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

__global__ void k_refit(const float4* __restrict__ p4, int n, int leaf_max,
                        const int32_t* __restrict__ left, const int32_t* __restrict__ right,
                        const int32_t* __restrict__ parent, float* klo, float* khi,
                        int32_t* kcnt, int32_t* kdfs, int32_t* kseg,
                        const int32_t* __restrict__ seg_of, int32_t* flag,
                        unsigned long long* err)
{
    int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= n) return;
    int node = parent[(n - 1) + y];
    // a radix tree over 96-bit augmented keys is at most 96 levels deep
    for (int step = 0;; ++step) {
        if (step > 128 || node < 0 || node >= n - 1) {
            atomicOr(err, 1ull);
            return;
        }
        stores_done();
        int old = atomicAdd(&flag[node], 1);
        if (old == 0) return;
        asm volatile("" ::: "memory");
        ChildInfo L = child_info(left[node], p4, klo, khi, kcnt, kdfs, kseg, seg_of);
        ChildInfo R = child_info(right[node], p4, klo, khi, kcnt, kdfs, kseg, seg_of);
        for (int a = 0; a < 3; ++a) {
            st_f(klo + 3 * node + a, L.lo[a] < R.lo[a] ? L.lo[a] : R.lo[a]);
            st_f(khi + 3 * node + a, L.hi[a] > R.hi[a] ? L.hi[a] : R.hi[a]);
        }
        int cnt = L.cnt + R.cnt;
        int seg = (L.seg == R.seg) ? L.seg : -1;
        st_i(kcnt + node, cnt);
        st_i(kseg + node, seg);
        st_i(kdfs + node, collapses(cnt, seg, leaf_max) ? 1 : 1 + L.dfs + R.dfs);
        if (node == 0) return;
        node = parent[node];
    }
}

// Depth-first placement: a node is emitted if it is the root or its parent
// holds more than leaf_max particles; its index counts, along the path from the
// root, one for each ancestor plus the left sibling subtrees passed on the way.
__global__ void k_layout(const float4* __restrict__ p4, int n, int leaf_max,
                         const int32_t* __restrict__ left, const int32_t* __restrict__ right,
                         const int32_t* __restrict__ parent, const int32_t* __restrict__ first,
                         const float* __restrict__ klo, const float* __restrict__ khi,
                         const int32_t* __restrict__ kcnt, const int32_t* __restrict__ kdfs,
                         const int32_t* __restrict__ kseg, const int32_t* __restrict__ klast,
                         const int32_t* __restrict__ seg_of, const int64_t* __restrict__ halo_off,
                         int32_t* __restrict__ seg_root, int32_t* __restrict__ seg_end,
                         Node* __restrict__ nodes, unsigned long long* err)
{
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    int total = 2 * n - 1;
    if (v >= total) return;
    bool is_leaf = v >= n - 1;
    int y = v - (n - 1);
    int self_code = is_leaf ? ~y : v;
    if (n > 1 && v != 0) {
        int p = parent[v];
        if (collapses(kcnt[p], kseg[p], leaf_max)) return;   // inside a collapsed leaf
    }
    int idx = 0;
    int cv = v, code = self_code;
    for (int step = 0; n > 1 && cv != 0; ++step) {
        int p = parent[cv];
        if (step > 128 || p < 0 || p >= n - 1) {
            atomicOr(err, 2ull);
            return;
        }
        if (right[p] == code) {
            int lc = left[p];
            idx += 1 + (lc < 0 ? 1 : kdfs[lc]);
        } else {
            idx += 1;
        }
        cv = p;
        code = p;
    }
    Node nd;
    int cnt, dfs, f, la, seg;
    float lo[3], hi[3];
    if (is_leaf) {
        float4 q = p4[y];
        lo[0] = q.x - q.w; lo[1] = q.y - q.w; lo[2] = q.z - q.w;
        hi[0] = q.x + q.w; hi[1] = q.y + q.w; hi[2] = q.z + q.w;
        cnt = 1; dfs = 1; f = y; la = y; seg = seg_of[y];
    } else {
        for (int a = 0; a < 3; ++a) { lo[a] = klo[3 * v + a]; hi[a] = khi[3 * v + a]; }
        cnt = kcnt[v]; dfs = kdfs[v]; f = first[v]; la = klast[v]; seg = kseg[v];
    }
    const bool leafy = collapses(cnt, seg, leaf_max);
    if (idx < 0 || idx + dfs > total || f < 0 || f + (leafy ? cnt : 0) > n) {
        atomicOr(err, 4ull);
        return;
    }
    // the subtree of exactly one halo: where that halo's rays walk
    if (seg >= 0 && halo_off && f == (int)halo_off[seg] && la == (int)halo_off[seg + 1] - 1) {
        seg_root[seg] = idx;
        seg_end[seg] = idx + dfs;
    }
    int leafw = leafy ? ((f << kLeafShift) | (cnt - 1)) : -1;
    nd.a = make_float4(lo[0], lo[1], lo[2], __int_as_float(idx + dfs));
    nd.b = make_float4(hi[0], hi[1], hi[2], __int_as_float(leafw));
    nodes[idx] = nd;
}

__global__ void k_gather_particles(const int32_t* __restrict__ perm, const float* __restrict__ pos,
                                   const float* __restrict__ h, const float* __restrict__ mu,
                                   const float* __restrict__ nH, int64_t n,
                                   float4* __restrict__ p4, double* __restrict__ mu_s,
                                   float* __restrict__ mu0_s, float* __restrict__ nH0_s,
                                   float* __restrict__ nH_s)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t j = perm[i];
    p4[i] = make_float4(pos[3 * j], pos[3 * j + 1], pos[3 * j + 2], h[j]);
    mu_s[i] = (double)mu[j];
    mu0_s[i] = mu[j];
    nH0_s[i] = nH[j];
    nH_s[i] = nH[j];
}

inline unsigned nblk(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t scan_exclusive_u64(Ctx& c, const uint64_t* in, uint64_t* out, int64_t m)
{
    return scan_exclusive<uint64_t>(c, in, out, m);
}

hipError_t launch_bounds(Ctx& c, float* part_out, int nb)
{
    hipLaunchKernelGGL(k_bounds, dim3(nb), dim3(kBlock), 0, c.stream, c.pos_in, c.h_in, c.mu_in,
                       c.nH_in, c.T_in, c.n, part_out);
    return hipGetLastError();
}

hipError_t launch_morton(Ctx& c, const double lo[3], double scale, int bits)
{
    hipLaunchKernelGGL(k_morton, dim3(nblk(c.n)), dim3(kBlock), 0, c.stream, c.pos_in, c.n,
                       lo[0], lo[1], lo[2], scale, bits, c.halo_off, c.n_halo, c.codes, c.perm);
    return hipGetLastError();
}

hipError_t radix_sort_pairs(Ctx& c, uint64_t* keys, int32_t* vals, int64_t n)
{
    int64_t n_tiles = (n + kSortTile - 1) / kSortTile;
    size_t hn = (size_t)n_tiles * 256;
    Scratch<uint32_t> hist(c);
    if (hipError_t e = hist.get(2 * hn)) return e;
    uint32_t* offs = hist.p + hn;
    uint64_t* ka = keys;
    int32_t* va = vals;
    uint64_t* kb = c.keys_b;
    int32_t* vb = c.vals_b;
    for (int pass = 0; pass < 8; ++pass) {
        int shift = 8 * pass;
        hipLaunchKernelGGL(k_digit_hist, dim3((unsigned)n_tiles), dim3(kBlock), 0, c.stream, ka,
                           n, shift, hist.p, n_tiles);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = scan_exclusive<uint32_t>(c, hist.p, offs, (int64_t)hn);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_digit_scatter, dim3((unsigned)n_tiles), dim3(kBlock), 0, c.stream,
                           ka, va, kb, vb, n, shift, offs, n_tiles);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    // 8 passes: the sorted data is back in the caller's buffers
    return hipSuccess;
}

hipError_t build_radix_tree(Ctx& c)
{
    const int n = (int)c.n;
    hipError_t e;
    hipLaunchKernelGGL(k_gather_particles, dim3(nblk(n)), dim3(kBlock), 0, c.stream, c.perm,
                       c.pos_in, c.h_in, c.mu_in, c.nH_in, (int64_t)n, c.p4, c.mu_s, c.mu0_s,
                       c.nH0_s, c.nH_s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_seg_of, dim3(nblk(n)), dim3(kBlock), 0, c.stream, c.codes, (int64_t)n,
                       c.n_halo > 1 ? 3 * c.key_bits : 64, c.seg_of);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (n > 1) {
        hipLaunchKernelGGL(k_radix_tree, dim3(nblk(n - 1)), dim3(kBlock), 0, c.stream, c.codes, n,
                           c.k_left, c.k_right, c.k_parent, c.k_first, c.k_last);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipMemsetAsync(c.k_flag, 0, sizeof(int32_t) * (n - 1), c.stream)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_refit, dim3(nblk(n)), dim3(kBlock), 0, c.stream, c.p4, n, c.leaf,
                           c.k_left, c.k_right, c.k_parent, c.k_lo, c.k_hi, c.k_cnt, c.k_dfs,
                           c.k_seg, c.seg_of, c.k_flag, c.red + kRedBuild);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_layout, dim3(nblk(2 * n - 1)), dim3(kBlock), 0, c.stream, c.p4, n, c.leaf,
                       c.k_left, c.k_right, c.k_parent, c.k_first, c.k_lo, c.k_hi, c.k_cnt,
                       c.k_dfs, c.k_seg, c.k_last, c.seg_of, c.n_halo > 1 ? c.halo_off : nullptr,
                       c.seg_root, c.seg_end, c.nodes, c.red + kRedBuild);
    return hipGetLastError();
}

}  // namespace rrt
