// The context's device memory: first-fit blocks carved from the caller's
// regions (the workspace and the path buffer of include/rrt.h), and the bytes
// a workspace needs for a problem of a given size.
#include "internal.h"
#include "physics.h"

#include <algorithm>

namespace rrt {

namespace {

uint64_t round_up(uint64_t b) { return (b + kWsAlign - 1) / kWsAlign * kWsAlign; }

}  // namespace

void ws_free(Ctx& c, void** owner)
{
    if (!owner || !*owner) return;
    std::vector<Arena::Block>& bl = c.arena.blocks;
    for (size_t i = 0; i < bl.size(); ++i)
        if (bl[i].owner == owner) {
            bl[i] = bl.back();
            bl.pop_back();
            break;
        }
    *owner = nullptr;
}

hipError_t ws_alloc(Ctx& c, void** owner, size_t bytes, int region)
{
    ws_free(c, owner);
    Arena& a = c.arena;
    const uint64_t need = round_up(std::max<uint64_t>(bytes, 1));
    // gaps between the live blocks of the region, lowest offset first
    std::vector<std::pair<uint64_t, uint64_t>> used;
    for (const Arena::Block& b : a.blocks)
        if (b.region == region) used.push_back({b.off, b.off + b.size});
    std::sort(used.begin(), used.end());
    uint64_t at = 0;
    bool found = false;
    for (const auto& u : used) {
        if (u.first >= at + need) {
            found = true;
            break;
        }
        at = std::max(at, u.second);
    }
    if (!found) found = a.base[region] && at + need <= a.cap[region];
    if (!found) {
        a.short_bytes = need;
        a.short_region = region;
        return hipErrorOutOfMemory;
    }
    a.blocks.push_back(Arena::Block{at, need, region, owner});
    *owner = a.base[region] + at;
    return hipSuccess;
}

uint64_t ws_used(const Ctx& c, int region)
{
    uint64_t u = 0;
    for (const Arena::Block& b : c.arena.blocks)
        if (b.region == region) u += b.size;
    return u;
}

uint64_t ws_high_water(const Ctx& c, int region)
{
    uint64_t h = 0;
    for (const Arena::Block& b : c.arena.blocks)
        if (b.region == region) h = std::max(h, b.off + b.size);
    return h;
}

uint64_t ws_largest_gap(const Ctx& c, int region)
{
    std::vector<std::pair<uint64_t, uint64_t>> used;
    for (const Arena::Block& b : c.arena.blocks)
        if (b.region == region) used.push_back({b.off, b.off + b.size});
    std::sort(used.begin(), used.end());
    uint64_t at = 0, best = 0;
    for (const auto& u : used) {
        if (u.first > at) best = std::max(best, u.first - at);
        at = std::max(at, u.second);
    }
    if (c.arena.cap[region] > at) best = std::max(best, c.arena.cap[region] - at);
    return best;
}

// Move every live block of the workspace region into a new region of at least
// the old high-water mark: one device copy of the used prefix, then the owners
// are rebased.  Synchronises the context's stream.
hipError_t ws_move(Ctx& c, char* base, uint64_t cap)
{
    Arena& a = c.arena;
    const uint64_t hw = ws_high_water(c, kRegionWs);
    if (hw > cap) return hipErrorOutOfMemory;
    if (hw > 0 && a.base[kRegionWs] != base) {
        hipError_t e = hipMemcpyAsync(base, a.base[kRegionWs], hw, hipMemcpyDeviceToDevice,
                                      c.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
        if (e != hipSuccess) return e;
    }
    for (Arena::Block& b : a.blocks)
        if (b.region == kRegionWs) *b.owner = base + b.off;
    a.base[kRegionWs] = base;
    a.cap[kRegionWs] = cap;
    return hipSuccess;
}

// Bytes of workspace for n particles, n_ray rays, n_bins bins, n_halo halos,
// the near/far scheme's extra columns, and the reverse mode's buffers for K
// iterations: the context's fixed buffers plus the largest transients.
uint64_t workspace_bytes(int64_t n, int n_ray, int n_bins, int n_halo, int K, bool near_far)
{
    uint64_t t = 0;
    auto add = [&](uint64_t b) { t += round_up(std::max<uint64_t>(b, 1)); };
    const uint64_t m = (uint64_t)std::max<int64_t>(n, 0);
    const uint64_t mi = m > 1 ? m - 1 : 1;
    const uint64_t rays = (uint64_t)std::max(n_ray, 1), bins = (uint64_t)std::max(n_bins, 1);
    const uint64_t H = (uint64_t)std::max(n_halo, 1);
    const uint64_t nr = m * (uint64_t)std::max(n_ray, 0);
    // context: kernel tables, reductions, chunk counters
    add(sizeof(KernelTables));
    add(kRedSlots * sizeof(unsigned long long));
    add(((uint64_t)kPoolSlices * kCtrStride + 1) * sizeof(unsigned long long));
    // rays, spectrum and its attenuation table
    add(3 * rays * sizeof(double));
    for (int q = 0; q < 3; ++q) add(bins * sizeof(float));
    add(2 * (uint64_t)kAttNodes * sizeof(double));
    // halo bookkeeping
    add((H + 1) * sizeof(int64_t));
    for (int q = 0; q < 4; ++q) add(H * sizeof(int32_t));
    add(H * sizeof(unsigned long long));
    add(4 * sizeof(int32_t));
    if (m > 0) {
        // particles in input order, then in tree order
        const uint64_t per_m[] = {12, 4, 4, 4, 4, 8,                // inputs
                                  8, 4, 4, 4, 8, 8, 8, 4, 8, 8, 4, 4, 8,   // state
                                  8, 4, 8,                           // keys_b, vals_b, k_parent (x m)
                                  4,                                 // seg_of
                                  8, 1, 1, 4, 4};                    // update rule
        for (uint64_t b : per_m) add(b * m);
        add(16 * (m + kLeafMax));                                    // p4
        add(2 * sizeof(Node) * m);                                   // nodes
        const uint64_t per_mi[] = {4, 4, 4, 4, 12, 12, 4, 4, 4, 4};  // radix tree (x n - 1)
        for (uint64_t b : per_mi) add(b * mi);
        // columns (and near columns), path row offsets
        add(8 * nr);
        if (near_far) add(8 * nr);
        add(8 * (nr + 1));
        // tree build transients: bounds partials, sort histograms, scan partials
        const uint64_t tiles = (m + 4095) / 4096;
        add(1024 * 8 * sizeof(float));
        add(2 * tiles * 256 * sizeof(uint32_t));
        add(2 * sizeof(uint64_t) * (std::max<uint64_t>(nr + 1, 2 * tiles * 256) / 1024 + 64) + 4096);
        if (n_halo > 1) {                                            // grouping of halos
            add(8 * nr);
            add(H * sizeof(int32_t));
            add(H * sizeof(unsigned long long));
        }
        if (K > 0) {                                                 // reverse mode
            add(8 * m * (uint64_t)(K + 1));
            for (int q = 0; q < 5; ++q) add(8 * m);
            add(4 * nr);
            add(8 * nr);
            add(8 * nr);
            add(8 * (((m + 255) / 256) * 4));
            add(8 * ((m + 255) / 256 + kAdjSlices) * bins);
            add(8 * bins);
        }
    }
    // staging of sampled hit lists and other small transients
    add(1u << 20);
    return t + (1u << 20);
}

}  // namespace rrt
