// rrt_get_hits_rows_noalloc: the sampled hit lists of rrt_get_hits_rows with
// their device staging in a fixed array of the library instead of the
// context's workspace, for callers that cannot allocate (or grow the
// workspace) at that point.  The array is a file-scope device variable: each
// GPU the library runs on holds its own copy, whose address is looked up once
// per device when a context is created there.  Every call on one GPU shares
// that GPU's copy, so calls that overlap on one GPU race; each call writes
// every entry it reads back (per-ray counts, offsets, hit lists) before
// reading it, so nothing needs clearing between calls.
#include "internal.h"

#include <mutex>

namespace rrt {

namespace {

constexpr int32_t kNaSources = 1024;            // sources per call
constexpr uint64_t kNaRows = 65536;              // sources x rays per call
constexpr uint64_t kNaHits = uint64_t(1) << 21;  // hit-list entries per call

constexpr uint64_t up256(uint64_t b) { return (b + 255) / 256 * 256; }
// layout: sources (sorted inputs, then tree positions) | their positions |
// per-ray counts and offsets | hit particles | hit images | hit factors
constexpr uint64_t kNaOffList = 0;
constexpr uint64_t kNaOffPos = kNaOffList + up256(sizeof(int32_t) * kNaSources);
constexpr uint64_t kNaOffCnt = kNaOffPos + up256(sizeof(int32_t) * kNaSources);
constexpr uint64_t kNaOffJ = kNaOffCnt + up256(sizeof(uint64_t) * (kNaRows + 1));
constexpr uint64_t kNaOffImg = kNaOffJ + up256(sizeof(int32_t) * kNaHits);
constexpr uint64_t kNaOffFac = kNaOffImg + up256(sizeof(int32_t) * kNaHits);
constexpr uint64_t kNaBytes = kNaOffFac + up256(sizeof(float) * kNaHits);   // ~24.6 MiB

// A host-side stand-in names this array; its device address comes from
// hipGetSymbolAddress (per device), and only that address reaches kernels.
static __device__ __align__(256) unsigned char scratch[kNaBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_scratch[kMaxDevices] = {};

struct FixedStaging : HitStaging {
    char* base;
    explicit FixedStaging(char* b) : base(b) {}
    int lists(Ctx& c, int32_t n_src, size_t rows) override
    {
        if (n_src > kNaSources || rows > kNaRows) {
            c.err = "rrt_get_hits_rows_noalloc: at most 1024 sources and 65536 rays per call";
            return RRT_E_CAPACITY;
        }
        list = reinterpret_cast<int32_t*>(base + kNaOffList);
        pos = reinterpret_cast<int32_t*>(base + kNaOffPos);
        cnt = reinterpret_cast<uint64_t*>(base + kNaOffCnt);
        return RRT_OK;
    }
    int hits(Ctx& c, uint64_t m) override
    {
        if (m > kNaHits) {
            c.err = "rrt_get_hits_rows_noalloc: more than 2^21 hits in one call";
            return RRT_E_CAPACITY;
        }
        j = reinterpret_cast<int32_t*>(base + kNaOffJ);
        img = reinterpret_cast<int32_t*>(base + kNaOffImg);
        fac = reinterpret_cast<float*>(base + kNaOffFac);
        return RRT_OK;
    }
};

}  // namespace

// With `device` current: look up this device's copy of the fixed staging
// array (once per device).
hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = static_cast<char*>(p);
    return hipSuccess;
}

}  // namespace rrt

using namespace rrt;

extern "C" int rrt_get_hits_rows_noalloc(rrt_ctx* x, int32_t n_src, const int64_t* src,
                                         int64_t cap, int64_t* row_off, int32_t* hit_j,
                                         int32_t* hit_img, float* hit_fac)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    char* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (c.device >= 0 && c.device < kMaxDevices) base = g_scratch[c.device];
    }
    if (!base) {
        c.err = "rrt_get_hits_rows_noalloc: the fixed staging array of this device was not set "
                "up (rrt_create)";
        return RRT_E_STATE;
    }
    FixedStaging st(base);
    return hits_rows_impl(c, n_src, src, cap, row_off, hit_j, hit_img, hit_fac, st);
}
