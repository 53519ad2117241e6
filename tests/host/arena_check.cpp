// Host-side checks of the context's device-memory arena (first-fit blocks in
// caller regions), built with the address and undefined-behaviour sanitizers
// by tests/test_host_sanitized.py.  No GPU call is made: the regions are host
// arrays and nothing is moved.
#include "workspace.hip"

#include <cstdio>
#include <cstdlib>
#include <random>

using namespace rrt;

#define CHECK(cond)                                                                 \
    do {                                                                            \
        if (!(cond)) {                                                              \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            std::exit(1);                                                           \
        }                                                                           \
    } while (0)

static bool disjoint(const Ctx& c)
{
    const auto& b = c.arena.blocks;
    for (size_t i = 0; i < b.size(); ++i)
        for (size_t j = i + 1; j < b.size(); ++j)
            if (b[i].region == b[j].region && b[i].off < b[j].off + b[j].size &&
                b[j].off < b[i].off + b[i].size)
                return false;
    return true;
}

int main()
{
    static char ws[1 << 20], pb[1 << 16];
    Ctx c;
    c.arena.base[kRegionWs] = ws;
    c.arena.cap[kRegionWs] = sizeof ws;
    // blocks are aligned, disjoint, inside the region, and released on free
    double* a = nullptr;
    float* b = nullptr;
    int32_t* d = nullptr;
    CHECK(ws_alloc(c, &a, 1000) == hipSuccess);
    CHECK(ws_alloc(c, &b, 3) == hipSuccess);
    CHECK(ws_alloc(c, &d, 70000) == hipSuccess);
    CHECK((reinterpret_cast<uintptr_t>(a) - reinterpret_cast<uintptr_t>(ws)) % kWsAlign == 0);
    CHECK((reinterpret_cast<uintptr_t>(b) - reinterpret_cast<uintptr_t>(ws)) % kWsAlign == 0);
    CHECK(disjoint(c));
    CHECK(ws_used(c, kRegionWs) == 8192 + 256 + 280064);
    for (int i = 0; i < 1000; ++i) a[i] = i;              // writable, in bounds (ASan)
    ws_free(c, &b);
    CHECK(b == nullptr && c.arena.blocks.size() == 2);
    // first fit: the gap b left is taken again by a request that fits it
    float* e = nullptr;
    CHECK(ws_alloc(c, &e, 64) == hipSuccess);
    CHECK(reinterpret_cast<char*>(e) == ws + 8192);
    // allocating into a held pointer releases what it held first
    CHECK(ws_alloc(c, &a, 10) == hipSuccess);
    CHECK(c.arena.blocks.size() == 3 && disjoint(c));
    // a request larger than any gap fails, is recorded, and changes nothing
    const uint64_t used = ws_used(c, kRegionWs);
    int32_t* f = nullptr;
    CHECK(ws_alloc(c, &f, sizeof ws) == hipErrorOutOfMemory);
    CHECK(f == nullptr && ws_used(c, kRegionWs) == used);
    CHECK(c.arena.short_bytes >= sizeof ws && c.arena.short_region == kRegionWs);
    CHECK(ws_largest_gap(c, kRegionWs) < sizeof ws);
    // no path buffer: every request there fails
    int2* p = nullptr;
    CHECK(ws_alloc(c, &p, 1, kRegionPath) == hipErrorOutOfMemory);
    c.arena.base[kRegionPath] = pb;
    c.arena.cap[kRegionPath] = sizeof pb;
    CHECK(ws_alloc(c, &p, 1000, kRegionPath) == hipSuccess);
    CHECK(reinterpret_cast<char*>(p) == pb && ws_used(c, kRegionPath) == 8192);
    // random churn: blocks stay disjoint and inside their regions, and the
    // used bytes are the sum of the live sizes
    std::mt19937 rng(7);
    std::vector<void*> slots(64, nullptr);
    for (int it = 0; it < 20000; ++it) {
        void** o = &slots[rng() % slots.size()];
        if (rng() % 3 == 0) {
            ws_free(c, o);
        } else {
            const size_t bytes = 1 + rng() % 40000;
            const int region = (int)(rng() % 2);
            if (ws_alloc(c, o, bytes, region) == hipSuccess) {
                char* q = static_cast<char*>(*o);
                CHECK(q >= c.arena.base[region] &&
                      q + bytes <= c.arena.base[region] + c.arena.cap[region]);
                q[0] = 1;
                q[bytes - 1] = 2;
            } else {
                CHECK(*o == nullptr);
            }
        }
        if (it % 97 == 0) CHECK(disjoint(c));
    }
    CHECK(disjoint(c));
    uint64_t live = 0;
    for (const auto& bl : c.arena.blocks) live += bl.size;
    CHECK(live == ws_used(c, kRegionWs) + ws_used(c, kRegionPath));
    // workspace sizes grow with every size they depend on
    const uint64_t base = workspace_bytes(4096, 12, 16, 1, 0, false);
    CHECK(workspace_bytes(8192, 12, 16, 1, 0, false) > base);
    CHECK(workspace_bytes(4096, 48, 16, 1, 0, false) > base);
    CHECK(workspace_bytes(4096, 12, 256, 1, 0, false) >= base);
    CHECK(workspace_bytes(4096, 12, 16, 64, 0, false) > base);
    CHECK(workspace_bytes(4096, 12, 16, 1, 10, false) > base);
    CHECK(workspace_bytes(4096, 12, 16, 1, 0, true) > base);
    // the per-ray buffers: columns (8 B) and path row offsets (8 B) per ray
    CHECK(workspace_bytes(4096, 12, 16, 1, 0, false) -
              workspace_bytes(4096, 11, 16, 1, 0, false) >= 16 * 4096);
    std::printf("arena checks passed\n");
    return 0;
}
