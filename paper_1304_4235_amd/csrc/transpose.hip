// Transposed recorded paths: the intersections grouped by the intersected
// particle, for the transposed column product of the reverse mode.
//
// Built once per geometry by a stable LSD radix sort of (particle, (row,
// factor)) pairs taken in row order, so each particle's entries stay in row
// order and every gather over them sums in a fixed order.
#include "internal.h"

#include <utility>

namespace rrt {

namespace {

constexpr int kBlock = 256;
constexpr int kRounds = 32;                    // items per thread per tile
constexpr int kTile = kBlock * kRounds;        // 8192 items per tile
constexpr int kWaves = kBlock / 64;

// (row, factor) of every recorded intersection, keyed by its particle
__global__ void k_expand(const uint64_t* __restrict__ row_off, const int2* __restrict__ path,
                         int64_t n_rows, uint32_t* __restrict__ key, uint64_t* __restrict__ val)
{
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; row < n_rows;
         row += stride) {
        const uint64_t a = row_off[row], b = row_off[row + 1];
        for (uint64_t e = a + lane; e < b; e += 64) {
            const int2 h = path[e];
            key[e] = (uint32_t)h.x;
            val[e] = ((uint64_t)(uint32_t)h.y << 32) | (uint64_t)(uint32_t)row;
        }
    }
}

__global__ void k_hist32(const uint32_t* __restrict__ keys, int64_t n, int shift,
                         uint64_t* __restrict__ hist, int64_t n_tiles)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = blockIdx.x * (int64_t)kTile;
    for (int r = 0; r < kRounds; ++r) {
        const int64_t i = base + r * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// stable within a tile: items ranked in (round, thread) order with one ballot
// per digit bit and per-wave counts combined in wave order
__global__ void k_scatter32(const uint32_t* __restrict__ kin, const uint64_t* __restrict__ vin,
                            uint32_t* __restrict__ kout, uint64_t* __restrict__ vout, int64_t n,
                            int shift, const uint64_t* __restrict__ offs, int64_t n_tiles)
{
    __shared__ uint64_t running[256];
    __shared__ uint32_t wcnt[kWaves][256];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    running[t] = offs[t * n_tiles + blockIdx.x];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = blockIdx.x * (int64_t)kTile;
    for (int r = 0; r < kRounds; ++r) {
        for (int w = 0; w < kWaves; ++w) wcnt[w][t] = 0;
        __syncthreads();
        const int64_t i = base + r * kBlock + t;
        const bool valid = i < n;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint64_t val = valid ? vin[i] : 0ull;
        const uint32_t d = (key >> shift) & 255u;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(valid && bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(m & lt);
        if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(m);
        __syncthreads();
        if (valid) {
            uint64_t pre = running[d];
            for (int w = 0; w < wave; ++w) pre += wcnt[w][d];
            const uint64_t dst = pre + rank;
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

// start of particle j's entries: the first sorted key >= j (binary search)
__global__ void k_col_starts(const uint32_t* __restrict__ key, int64_t m, int64_t n,
                             uint64_t* __restrict__ col_off)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j > n) return;
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)key[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    col_off[j] = (uint64_t)lo;
}

// y_j = sum over particle j's entries of factor * nu[row], in row order
__global__ void __launch_bounds__(256)
k_gather_cols(const uint64_t* __restrict__ col_off, const uint64_t* __restrict__ ent,
              const float* __restrict__ nu, int64_t n, double* __restrict__ y)
{
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t col = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; col < n;
         col += stride) {
        double acc = 0.0;
        const uint64_t a = col_off[col], b = col_off[col + 1];
        const long long* p = reinterpret_cast<const long long*>(ent);
        for (uint64_t e = a + lane; e < b; e += 4 * 64) {
            const uint64_t v0 = (uint64_t)__builtin_nontemporal_load(p + e);
            const uint64_t v1 = e + 64 < b ? (uint64_t)__builtin_nontemporal_load(p + e + 64) : 0ull;
            const uint64_t v2 = e + 128 < b ? (uint64_t)__builtin_nontemporal_load(p + e + 128) : 0ull;
            const uint64_t v3 = e + 192 < b ? (uint64_t)__builtin_nontemporal_load(p + e + 192) : 0ull;
            const double n0 = (double)nu[(uint32_t)v0], n1 = (double)nu[(uint32_t)v1];
            const double n2 = (double)nu[(uint32_t)v2], n3 = (double)nu[(uint32_t)v3];
            acc += (double)__int_as_float((int)(v0 >> 32)) * n0;
            acc += (double)__int_as_float((int)(v1 >> 32)) * n1;
            acc += (double)__int_as_float((int)(v2 >> 32)) * n2;
            acc += (double)__int_as_float((int)(v3 >> 32)) * n3;
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (lane == 0) y[col] = acc;
    }
}

}  // namespace

hipError_t scan_exclusive_u64(Ctx& c, const uint64_t* in, uint64_t* out, int64_t m);

// Build the transposed paths into c.tpath / c.tcol_off, in the path buffer.
// Scratch: two key and one value buffer of path_hits entries and the sort
// histograms, also from the path buffer, released before returning.
// hipErrorOutOfMemory (nothing kept) when they do not fit beside the paths.
hipError_t build_transposed_paths(Ctx& c)
{
    const int64_t m = c.path_hits;
    const int64_t n_rows = c.n * (int64_t)c.n_ray;
    const int64_t n = c.n;
    ws_free(c, &c.tpath);
    ws_free(c, &c.tcol_off);
    const int64_t mm = m > 0 ? m : 1;
    const int64_t n_tiles = (mm + kTile - 1) / kTile;
    const size_t hn = (size_t)n_tiles * 256;
    Scratch<uint32_t> ka(c), kb(c);
    Scratch<uint64_t> vb(c), hist(c);
    hipError_t e = ws_alloc(c, &c.tpath, mm, kRegionPath);
    if (e == hipSuccess) e = ws_alloc(c, &c.tcol_off, n + 1, kRegionPath);
    if (e == hipSuccess) e = ka.get(mm, kRegionPath);
    if (e == hipSuccess) e = kb.get(mm, kRegionPath);
    if (e == hipSuccess) e = vb.get(mm, kRegionPath);
    if (e == hipSuccess) e = hist.get(2 * hn, kRegionPath);
    if (e == hipSuccess && m > 0) {
        hipLaunchKernelGGL(k_expand, dim3(stride_blocks(n_rows, 4)), dim3(256), 0,
                           c.stream, c.row_off, c.path, n_rows, ka.p, c.tpath);
        e = hipGetLastError();
    }
    // sort by particle: enough 8-bit passes to cover the largest index
    int bits = 1;
    while ((int64_t(1) << bits) < n) ++bits;
    const int passes = (bits + 7) / 8;
    uint32_t* kin = ka.p;
    uint32_t* kout = kb.p;
    uint64_t* vin = c.tpath;
    uint64_t* vout = vb.p;
    for (int p = 0; p < passes && e == hipSuccess && m > 0; ++p) {
        hipLaunchKernelGGL(k_hist32, dim3((unsigned)n_tiles), dim3(kBlock), 0, c.stream, kin, m,
                           8 * p, hist.p, n_tiles);
        e = hipGetLastError();
        if (e == hipSuccess) e = scan_exclusive_u64(c, hist.p, hist.p + hn, (int64_t)hn);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_scatter32, dim3((unsigned)n_tiles), dim3(kBlock), 0, c.stream,
                               kin, vin, kout, vout, m, 8 * p, hist.p + hn, n_tiles);
            e = hipGetLastError();
        }
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    // the sorted values are in vin; keep them as the transposed paths
    if (e == hipSuccess && vin != c.tpath)
        e = hipMemcpyAsync(c.tpath, vin, sizeof(uint64_t) * m, hipMemcpyDeviceToDevice, c.stream);
    // particle starts from the sorted keys
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_col_starts, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0,
                           c.stream, kin, m, n, c.tcol_off);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        ws_free(c, &c.tpath);
        ws_free(c, &c.tcol_off);
    }
    return e;
}

hipError_t launch_gather_cols(Ctx& c)
{
    hipLaunchKernelGGL(k_gather_cols, dim3(stride_blocks(c.n, 4)), dim3(256), 0,
                       c.stream, c.tcol_off, c.tpath, c.adj_nu, c.n, c.adj_y);
    return hipGetLastError();
}

}  // namespace rrt
