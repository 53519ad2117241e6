// Row tiles of the recorded ray paths.
//
// Rows are ray-major (row = k * n + p, sources in tree order), so a run of
// consecutive rows is a bundle of parallel rays from neighbouring sources, and
// the rays of a bundle cross mostly the same particles: a tile of a few hundred
// rows with ~10^5 intersections touches only a few thousand distinct particles.
// Once per geometry, each tile's distinct particle indices are collected and
// every recorded entry's particle index is replaced by its 16-bit position in
// the tile's set.  The column product then loads the set's mu*x
// into LDS once per tile and streams 6 bytes per intersection (local index and
// FP32 factor) with no per-intersection global gathers.  The columns equal
// those of the plain product over the recorded paths up to FP64 summation
// order (the same products, assigned to lanes in groups of four).
#include "internal.h"

#include <vector>

namespace rrt {

namespace {

constexpr int kBuildBlock = 1024;
constexpr int kHashBits = 15;
constexpr int kHashSlots = 1 << kHashBits;      // 32768 slots of 4 B: 128 KiB of LDS
constexpr uint32_t kEmpty = 0xffffffffu;

__device__ inline uint32_t hash_slot(uint32_t j)
{
    return (j * 2654435761u) >> (32 - kHashBits);
}

// Insert every particle index of the tile's entries into the LDS set; *count
// receives the number of distinct indices, or stops growing once it passes
// kTileMaxSet (the caller treats that as overflow).
__device__ void tile_collect(uint32_t* tab, uint32_t* count, const int2* __restrict__ path,
                             uint64_t a, uint64_t b)
{
    for (int i = threadIdx.x; i < kHashSlots; i += blockDim.x) tab[i] = kEmpty;
    if (threadIdx.x == 0) *count = 0;
    __syncthreads();
    for (uint64_t e = a + threadIdx.x; e < b; e += blockDim.x) {
        if (*(volatile uint32_t*)count > (uint32_t)kTileMaxSet) break;
        const uint32_t j = (uint32_t)path[e].x;
        uint32_t s = hash_slot(j);
        for (int probe = 0; probe < kHashSlots; ++probe) {
            const uint32_t prev = atomicCAS(&tab[s], kEmpty, j);
            if (prev == kEmpty) {
                atomicAdd(count, 1u);
                break;
            }
            if (prev == j) break;
            s = (s + 1) & (kHashSlots - 1);
        }
    }
    __syncthreads();
}

// distinct particles per tile (kTileMaxSet + 1 marks a tile that overflowed)
__global__ void __launch_bounds__(kBuildBlock)
k_tile_count(const uint64_t* __restrict__ row_off, const int2* __restrict__ path, int64_t n_rows,
             int tile_rows, int64_t n_tiles, uint64_t* __restrict__ tile_u)
{
    __shared__ uint32_t tab[kHashSlots];
    __shared__ uint32_t count;
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int64_t r0 = t * tile_rows;
        const int64_t r1 = r0 + tile_rows < n_rows ? r0 + tile_rows : n_rows;
        tile_collect(tab, &count, path, row_off[r0], row_off[r1]);
        if (threadIdx.x == 0)
            tile_u[t] = count > (uint32_t)kTileMaxSet ? (uint64_t)kTileMaxSet + 1 : count;
        __syncthreads();
    }
}

// Each tile's set and the local index of every entry.  The local index of an
// occupied hash slot is the number of occupied slots before it (occupancy
// bitmap + prefix counts), so the set follows the hash table's slot order; no
// sum depends on that order (every entry keeps its own particle's values).
__device__ __forceinline__ uint32_t slot_id(const uint32_t* occ, const uint32_t* pre, uint32_t s)
{
    return pre[s >> 5] + __popc(occ[s >> 5] & ((1u << (s & 31)) - 1u));
}

__global__ void __launch_bounds__(kBuildBlock)
k_tile_build(const uint64_t* __restrict__ row_off, const int2* __restrict__ path, int64_t n_rows,
             int tile_rows, int64_t n_tiles, const uint64_t* __restrict__ set_off,
             uint32_t* __restrict__ set, uint16_t* __restrict__ idx, float* __restrict__ fac)
{
    constexpr int kWords = kHashSlots / 32;           // 1024 bitmap words
    __shared__ uint32_t tab[kHashSlots];
    __shared__ uint32_t occ[kWords];
    __shared__ uint32_t pre[kWords];
    __shared__ uint32_t count;
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int64_t r0 = t * tile_rows;
        const int64_t r1 = r0 + tile_rows < n_rows ? r0 + tile_rows : n_rows;
        const uint64_t a = row_off[r0], b = row_off[r1];
        tile_collect(tab, &count, path, a, b);
        for (int w = threadIdx.x; w < kWords; w += blockDim.x) {
            uint32_t m = 0;
            for (int q = 0; q < 32; ++q)
                if (tab[32 * w + q] != kEmpty) m |= 1u << q;
            occ[w] = m;
        }
        __syncthreads();
        if (threadIdx.x < 64) {                       // one wave: 16 words per lane
            const int l = threadIdx.x;
            uint32_t loc[kWords / 64];
            uint32_t sum = 0;
            for (int q = 0; q < kWords / 64; ++q) {
                loc[q] = sum;
                sum += __popc(occ[l * (kWords / 64) + q]);
            }
            uint32_t incl = sum;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(incl, off, 64);
                if (l >= off) incl += y;
            }
            const uint32_t base = incl - sum;
            for (int q = 0; q < kWords / 64; ++q) pre[l * (kWords / 64) + q] = base + loc[q];
        }
        __syncthreads();
        const uint64_t so = set_off[t];
        for (int sl = threadIdx.x; sl < kHashSlots; sl += blockDim.x) {
            const uint32_t key = tab[sl];
            if (key != kEmpty) set[so + slot_id(occ, pre, (uint32_t)sl)] = key;
        }
        for (uint64_t e = a + threadIdx.x; e < b; e += blockDim.x) {
            const int2 h = path[e];
            const uint32_t j = (uint32_t)h.x;
            uint32_t sl = hash_slot(j);
            for (int probe = 0; probe < kHashSlots && tab[sl] != j; ++probe)
                sl = (sl + 1) & (kHashSlots - 1);
            idx[e] = (uint16_t)slot_id(occ, pre, sl);
            fac[e] = __int_as_float(h.y);
        }
        __syncthreads();
    }
}

typedef unsigned short v4u16 __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Transposed product over the tiles (reverse mode): y_j += factor * nu_row for
// every entry, accumulated per distinct particle of the tile in LDS, then one
// global atomic add per particle (instead of one per intersection).  G lanes
// per row take aligned groups of four consecutive entries, and each group
// loads its next row's offsets and adjoint value before it works on the
// current row.  The order of the additions is not fixed.
template <int G>
__global__ void __launch_bounds__(512)
k_tile_scatter(const uint64_t* __restrict__ row_off, const uint16_t* __restrict__ idx,
               const float* __restrict__ fac, const uint64_t* __restrict__ set_off,
               const uint32_t* __restrict__ set, const float* __restrict__ nu, int64_t n_rows,
               int tile_rows, int64_t n_tiles, double* __restrict__ y)
{
    extern __shared__ double sacc[];
    const int lane = threadIdx.x & (G - 1);
    const int groups = blockDim.x / G;
    const v4u16* iq = reinterpret_cast<const v4u16*>(idx);
    const v4f* fq = reinterpret_cast<const v4f*>(fac);
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const uint64_t so = set_off[t];
        const uint32_t u = (uint32_t)(set_off[t + 1] - so);
        for (uint32_t i = threadIdx.x; i < u; i += blockDim.x) sacc[i] = 0.0;
        __syncthreads();
        const int64_t r0 = t * tile_rows;
        const int64_t r1 = r0 + tile_rows < n_rows ? r0 + tile_rows : n_rows;
        int64_t row = r0 + threadIdx.x / G;
        uint64_t a = 0, b = 0;
        double v = 0.0;
        if (row < r1) {
            a = row_off[row];
            b = row_off[row + 1];
            v = (double)nu[row];
        }
        for (; row < r1; row += groups) {
            const int64_t next = row + groups;
            uint64_t an = 0, bn = 0;
            double vn = 0.0;
            if (next < r1) {
                an = row_off[next];
                bn = row_off[next + 1];
                vn = (double)nu[next];
            }
            if (v != 0.0) {
                for (uint64_t q = (a >> 2) + lane; 4 * q < b; q += G) {
                    const v4u16 i4 = __builtin_nontemporal_load(iq + q);
                    const v4f f4 = __builtin_nontemporal_load(fq + q);
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint64_t e = 4 * q + k;
                        if (e >= a && e < b) atomicAdd(&sacc[i4[k]], (double)f4[k] * v);
                    }
                }
            }
            a = an;
            b = bn;
            v = vn;
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < u; i += blockDim.x)
            if (sacc[i] != 0.0) unsafeAtomicAdd(y + set[so + i], sacc[i]);
        __syncthreads();
    }
}

// N_row = sum over the row's entries of mux[set[idx]] * factor, with the
// tile's mux staged in LDS.  G lanes per row; each lane takes aligned groups of
// four consecutive entries (one 8-byte index load, one 16-byte factor load),
// two groups in flight.
template <int G>
__global__ void __launch_bounds__(512)
k_tile_columns(const uint64_t* __restrict__ row_off, const uint16_t* __restrict__ idx,
               const float* __restrict__ fac, const uint64_t* __restrict__ set_off,
               const uint32_t* __restrict__ set, const float* __restrict__ mux, int64_t n_rows,
               int tile_rows, int64_t n_tiles, double* __restrict__ N, int64_t n,
               const int32_t* __restrict__ seg_of, const int32_t* __restrict__ seg_active,
               const uint8_t* __restrict__ want)
{
    extern __shared__ float smux[];
    const int lane = threadIdx.x & (G - 1);
    const int groups = blockDim.x / G;
    const v4u16* iq = reinterpret_cast<const v4u16*>(idx);
    const v4f* fq = reinterpret_cast<const v4f*>(fac);
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const uint64_t so = set_off[t];
        const uint32_t u = (uint32_t)(set_off[t + 1] - so);
        for (uint32_t i = threadIdx.x; i < u; i += blockDim.x) smux[i] = mux[set[so + i]];
        __syncthreads();
        const int64_t r0 = t * tile_rows;
        const int64_t r1 = r0 + tile_rows < n_rows ? r0 + tile_rows : n_rows;
        for (int64_t row = r0 + threadIdx.x / G; row < r1; row += groups) {
            // rows of halos that have stopped iterating keep their last columns
            if (seg_active && seg_active[seg_of[row % n]] == 0) continue;
            if (want && !want[row % n]) continue;     // not updated in this step
            const uint64_t a = row_off[row], b = row_off[row + 1];
            double acc = 0.0;
            for (uint64_t q = (a >> 2) + lane; 4 * q < b; q += 2 * G) {
                const uint64_t q1 = q + G;
                const bool has1 = 4 * q1 < b;
                const v4u16 i0 = __builtin_nontemporal_load(iq + q);
                const v4f f0 = __builtin_nontemporal_load(fq + q);
                const v4u16 i1 = has1 ? __builtin_nontemporal_load(iq + q1) : v4u16(0);
                const v4f f1 = has1 ? __builtin_nontemporal_load(fq + q1) : v4f(0.0f);
                // entries outside [a, b) in the first and last group add exactly 0
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint64_t e = 4 * q + k;
                    const bool ok = e >= a && e < b;
                    acc += ok ? (double)(smux[i0[k]] * f0[k]) : 0.0;
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint64_t e = 4 * q1 + k;
                    const bool ok = e >= a && e < b;
                    acc += ok ? (double)(smux[i1[k]] * f1[k]) : 0.0;
                }
            }
            for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
            if (lane == 0) N[row] = acc;
        }
        __syncthreads();
    }
}

template <int G>
hipError_t launch_tiles_g(Ctx& c, int64_t n_rows, unsigned nb, size_t lds)
{
    hipLaunchKernelGGL(k_tile_columns<G>, dim3(nb), dim3(512), lds, c.stream, c.row_off,
                       c.tile_idx, c.tile_fac, c.tile_off, c.tile_set, c.mux_s, n_rows,
                       c.tile_rows, c.n_tiles, c.N_s, c.n, c.geom.seg_of, c.geom.seg_active,
                       c.geom.want);
    return hipGetLastError();
}

}  // namespace

void free_tiles(Ctx& c)
{
    // a captured graph may hold these buffers
    if (c.tile_off || c.tile_set || c.tile_idx || c.tile_fac) drop_graph(c);
    ws_free(c, &c.tile_off);
    ws_free(c, &c.tile_set);
    ws_free(c, &c.tile_idx);
    ws_free(c, &c.tile_fac);
    c.tiles_valid = false;
    c.tiles_unfit = false;
    c.n_tiles = 0;
    c.tile_max_u = 0;
    c.tile_set_total = 0;
}

// Build the tiles of the current recorded paths, in the path buffer.  Rows
// per tile start from ~2^16 intersections per tile and halve while any tile
// has more than kTileMaxSet distinct particles.  Marks the tiles unfit (the
// plain product stays in use) when no tile size works or the arrays do not
// fit beside the paths.
hipError_t build_tiles(Ctx& c)
{
    free_tiles(c);
    const int64_t n_rows = c.n * (int64_t)c.n_ray;
    const int64_t m = c.path_hits;
    c.tiles_unfit = true;
    if (!c.paths_valid || m <= 0 || n_rows <= 0) return hipSuccess;
    const double mean = (double)m / (double)n_rows;
    int rows = 16;
    while (rows < 4096 && (double)rows * 2.0 * mean <= 65536.0) rows *= 2;
    std::vector<uint64_t> u;
    hipError_t e = hipSuccess;
    for (; rows >= 16; rows /= 2) {
        const int64_t nt = (n_rows + rows - 1) / rows;
        if (nt > (int64_t(1) << 24)) break;
        e = ws_alloc(c, &c.tile_off, nt + 1, kRegionPath);
        if (e != hipSuccess) break;
        uint64_t* d_u = c.tile_off;
        hipLaunchKernelGGL(k_tile_count, dim3((unsigned)std::min<int64_t>(nt, 2048)),
                           dim3(kBuildBlock), 0, c.stream, c.row_off, c.path, n_rows, rows, nt,
                           d_u);
        e = hipGetLastError();
        if (e != hipSuccess) break;
        u.assign(nt + 1, 0);
        e = hipMemcpyAsync(u.data(), d_u, sizeof(uint64_t) * nt, hipMemcpyDeviceToHost, c.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
        if (e != hipSuccess) break;
        uint64_t mx = 0;
        for (int64_t t = 0; t < nt; ++t) mx = std::max(mx, u[t]);
        if (mx <= (uint64_t)kTileMaxSet) {
            // exclusive offsets of the sets, on the host
            uint64_t s = 0;
            for (int64_t t = 0; t < nt; ++t) {
                const uint64_t v = u[t];
                u[t] = s;
                s += v;
            }
            u[nt] = s;
            e = hipMemcpyAsync(d_u, u.data(), sizeof(uint64_t) * (nt + 1),
                               hipMemcpyHostToDevice, c.stream);
            if (e == hipSuccess)
                e = ws_alloc(c, &c.tile_set, std::max<uint64_t>(s, 1), kRegionPath);
            if (e == hipSuccess) e = ws_alloc(c, &c.tile_idx, m + kPathPad, kRegionPath);
            if (e == hipSuccess) e = ws_alloc(c, &c.tile_fac, m + kPathPad, kRegionPath);
            if (e != hipSuccess) break;                 // keep the plain product
            hipLaunchKernelGGL(k_tile_build, dim3((unsigned)std::min<int64_t>(nt, 2048)),
                               dim3(kBuildBlock), 0, c.stream, c.row_off, c.path, n_rows, rows,
                               nt, d_u, c.tile_set, c.tile_idx, c.tile_fac);
            e = hipGetLastError();
            if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
            if (e != hipSuccess) break;
            c.tile_rows = rows;
            c.n_tiles = nt;
            c.tile_max_u = (int64_t)mx;
            c.tile_set_total = s;
            c.tiles_valid = true;
            c.tiles_unfit = false;
            break;
        }
    }
    if (!c.tiles_valid) {
        const bool unfit = true;
        free_tiles(c);
        c.tiles_unfit = unfit;
        if (e == hipErrorOutOfMemory) {
            (void)hipGetLastError();
            e = hipSuccess;
        }
    }
    return e;
}

namespace {

template <int G>
void launch_scatter_g(Ctx& c, const float* nu, double* y, int64_t n_rows, unsigned nb,
                      size_t lds)
{
    hipLaunchKernelGGL(k_tile_scatter<G>, dim3(nb), dim3(512), lds, c.stream, c.row_off,
                       c.tile_idx, c.tile_fac, c.tile_off, c.tile_set, nu, n_rows, c.tile_rows,
                       c.n_tiles, y);
}

}  // namespace

int tile_group(const Ctx& c)
{
    if (c.path_group) return c.path_group;
    const double mean = (double)c.path_hits / (double)std::max<int64_t>(c.n * (int64_t)c.n_ray, 1);
    // each lane takes four entries at a time: a quarter of the plain product's lanes
    return mean >= 160 ? 32 : mean >= 40 ? 16 : 8;
}

hipError_t launch_tile_scatter(Ctx& c, const float* nu, double* y)
{
    const int64_t n_rows = c.n * (int64_t)c.n_ray;
    const size_t lds = sizeof(double) * (size_t)std::max<int64_t>(c.tile_max_u, 1);
    const unsigned nb = (unsigned)std::min<int64_t>(c.n_tiles, kMaxBlocks);
    hipError_t e = hipMemsetAsync(y, 0, sizeof(double) * c.n, c.stream);
    if (e != hipSuccess) return e;
    const int g = tile_group(c);
    if (g == 64) launch_scatter_g<64>(c, nu, y, n_rows, nb, lds);
    else if (g == 32) launch_scatter_g<32>(c, nu, y, n_rows, nb, lds);
    else if (g == 16) launch_scatter_g<16>(c, nu, y, n_rows, nb, lds);
    else launch_scatter_g<8>(c, nu, y, n_rows, nb, lds);
    return hipGetLastError();
}

hipError_t launch_tile_columns(Ctx& c, int group)
{
    const int64_t n_rows = c.n * (int64_t)c.n_ray;
    const size_t lds = sizeof(float) * (size_t)std::max<int64_t>(c.tile_max_u, 1);
    const unsigned nb = (unsigned)std::min<int64_t>(c.n_tiles, kMaxBlocks);
    if (group == 64) return launch_tiles_g<64>(c, n_rows, nb, lds);
    if (group == 32) return launch_tiles_g<32>(c, n_rows, nb, lds);
    if (group == 16) return launch_tiles_g<16>(c, n_rows, nb, lds);
    return launch_tiles_g<8>(c, n_rows, nb, lds);
}

}  // namespace rrt
