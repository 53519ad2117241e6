// Host side of librrt: the C ABI declared in include/rrt.h.
#include "internal.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

using namespace rrt;

// A named range on the profiler's marker track (rocprofv3 --marker-trace)
// for the duration of one library call or phase; no cost without a profiler.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};


// a captured graph refers to the buffers it was captured with
void rrt::drop_graph(Ctx& c)
{
    if (c.graph_exec) (void)hipGraphExecDestroy(c.graph_exec);
    if (c.graph) (void)hipGraphDestroy(c.graph);
    c.graph_exec = nullptr;
    c.graph = nullptr;
    c.graph_iters = 0;
}

namespace {

thread_local std::string g_create_err;

int fail(Ctx& c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(Ctx& c, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c.err = buf;
    return code;
}

// A request the workspace or the path buffer had no room for.
int ws_fail(Ctx& c, const char* what)
{
    const Arena& a = c.arena;
    if (!a.base[kRegionWs])
        return fail(c, RRT_E_WORKSPACE, "%s: no workspace (rrt_workspace_size, rrt_set_workspace)",
                    what);
    const int r = a.short_region < 0 ? kRegionWs : a.short_region;
    return fail(c, RRT_E_WORKSPACE,
                "%s: %llu bytes in one piece do not fit the %s (%llu of %llu bytes in use)", what,
                (unsigned long long)a.short_bytes, r == kRegionWs ? "workspace" : "path buffer",
                (unsigned long long)ws_used(c, r), (unsigned long long)a.cap[r]);
}

#define HIP_OK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ == hipErrorOutOfMemory) return ws_fail(c, #expr);                           \
        if (e_ != hipSuccess)                                                              \
            return fail(c, RRT_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

// every buffer of the per-particle and per-ray families, which are released
// and carved again together
void free_adjoint(Ctx& c)
{
    void** adj[] = {(void**)&c.xhist, (void**)&c.adj_lam, (void**)&c.adj_lup, (void**)&c.adj_nu,
                    (void**)&c.adj_pis, (void**)&c.adj_gnH, (void**)&c.adj_y, (void**)&c.adj_wpart,
                    (void**)&c.adj_gw, (void**)&c.adj_tpart, (void**)&c.adj_st, (void**)&c.adj_ell,
                    (void**)&c.Nhist};
    for (void** b : adj) ws_free(c, b);
    c.Nhist_cap = 0;
    c.Nhist_on = false;
    c.adj_n = c.adj_nr = 0;
    c.xhist_cap = 0;
    c.fwd_K = -1;
}

void free_columns(Ctx& c)
{
    ws_free(c, &c.N_s);
    ws_free(c, &c.Nn_s);
    ws_free(c, &c.row_off);
    c.counts_valid = false;
}

void free_particles(Ctx& c)
{
    void** bufs[] = {(void**)&c.pos_in, (void**)&c.h_in, (void**)&c.mu_in, (void**)&c.nH_in,
                     (void**)&c.T_in, (void**)&c.x_init, (void**)&c.p4, (void**)&c.mu_s,
                     (void**)&c.nH_s, (void**)&c.mu0_s, (void**)&c.nH0_s, (void**)&c.alpha_s,
                     (void**)&c.gcoll_s, (void**)&c.x_s, (void**)&c.mux_s, (void**)&c.lnG_s,
                     (void**)&c.G_s, (void**)&c.tau_s, (void**)&c.perm, (void**)&c.codes,
                     (void**)&c.nodes, (void**)&c.keys_b, (void**)&c.vals_b, (void**)&c.k_left,
                     (void**)&c.k_right, (void**)&c.k_parent, (void**)&c.k_first,
                     (void**)&c.k_last, (void**)&c.k_lo, (void**)&c.k_hi, (void**)&c.k_cnt,
                     (void**)&c.k_dfs, (void**)&c.k_flag, (void**)&c.seg_of, (void**)&c.k_seg,
                     (void**)&c.alphaB_s, (void**)&c.skip_s, (void**)&c.want_s,
                     (void**)&c.block_s, (void**)&c.block_list};
    for (void** b : bufs) ws_free(c, b);
    free_columns(c);
    free_adjoint(c);
    c.blocks_for = 0;
    c.n_cap = 0;
}

int alloc_particles(Ctx& c, int64_t n)
{
    if (n <= c.n_cap && c.p4) return RRT_OK;
    free_particles(c);
    const size_t m = (size_t)n;
    const size_t mi = m > 1 ? m - 1 : 1;
    hipError_t e = hipSuccess;
#define A(p, cnt)                                                    \
    if (e == hipSuccess) e = ws_alloc(c, &(p), (cnt));
    A(c.pos_in, 3 * m) A(c.h_in, m) A(c.mu_in, m) A(c.nH_in, m) A(c.T_in, m) A(c.x_init, m)
    A(c.p4, m + kLeafMax) A(c.mu_s, m) A(c.mu0_s, m) A(c.nH0_s, m) A(c.nH_s, m) A(c.alpha_s, m) A(c.gcoll_s, m) A(c.x_s, m)
    A(c.mux_s, m) A(c.lnG_s, m) A(c.G_s, m) A(c.tau_s, m) A(c.perm, m) A(c.codes, m)
    A(c.nodes, 2 * m) A(c.keys_b, m) A(c.vals_b, m) A(c.k_left, mi) A(c.k_right, mi)
    A(c.k_parent, 2 * m) A(c.k_first, mi) A(c.k_last, mi) A(c.k_lo, 3 * mi) A(c.k_hi, 3 * mi)
    A(c.k_cnt, mi) A(c.k_dfs, mi) A(c.k_flag, mi) A(c.seg_of, m) A(c.k_seg, mi)
    A(c.alphaB_s, m) A(c.skip_s, m) A(c.want_s, m) A(c.block_s, m) A(c.block_list, m)
#undef A
    if (e != hipSuccess) {
        const int r = ws_fail(c, "particle buffers");
        free_particles(c);
        return r;
    }
    // the spare particle entries past n are read with whole leaves, never used
    e = hipMemsetAsync(c.p4 + m, 0, sizeof(float4) * kLeafMax, c.stream);
    if (e != hipSuccess) {
        free_particles(c);
        return fail(c, RRT_E_HIP, "hipMemsetAsync: %s", hipGetErrorString(e));
    }
    c.n_cap = n;
    return RRT_OK;
}

// Columns (and near columns) and the recorded paths' row offsets, [n_ray][n].
int alloc_columns(Ctx& c)
{
    free_columns(c);
    // rays are indexed with 32-bit integers on the device
    if (c.n * (int64_t)c.n_ray > kMaxRows)
        return fail(c, RRT_E_ARG, "%lld particles x %d rays exceeds 2^31 - 1 rays",
                    (long long)c.n, c.n_ray);
    const size_t nr = (size_t)c.n * (size_t)c.n_ray;
    hipError_t e = ws_alloc(c, &c.N_s, nr);
    if (e == hipSuccess && c.near_far) e = ws_alloc(c, &c.Nn_s, nr);
    if (e == hipSuccess) e = ws_alloc(c, &c.row_off, nr + 1);
    if (e != hipSuccess) {
        const int r = ws_fail(c, "column buffers");
        free_columns(c);
        return r;
    }
    return RRT_OK;
}

// The context's own small buffers: kernel tables, reductions, chunk counters.
int alloc_ctx_buffers(Ctx& c)
{
    if (c.ctx_bufs) return RRT_OK;
    HIP_OK(ws_alloc(c, &c.tables, 1));
    HIP_OK(ws_alloc(c, &c.red, kRedSlots));
    HIP_OK(ws_alloc(c, &c.pool_ctr, (size_t)kPoolSlices * kCtrStride + 1));
    KernelTables host;
    fill_kernel_tables(&host);
    HIP_OK(hipMemcpyAsync(c.tables, &host, sizeof host, hipMemcpyHostToDevice, c.stream));
    HIP_OK(hipMemsetAsync(c.red, 0, kRedSlots * sizeof(unsigned long long), c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));        // `host` goes out of scope
    c.ctx_bufs = true;
    return RRT_OK;
}

int need_ws(Ctx& c)
{
    if (!c.ctx_bufs)
        return fail(c, RRT_E_WORKSPACE, "no workspace (rrt_workspace_size, rrt_set_workspace)");
    return RRT_OK;
}

// Read and clear the device input flags; RRT_E_INPUT when one was raised.
// Expects red_host[kRedInput..kRedNumeric] copied and the stream synchronised.
int check_flags(Ctx& c)
{
    const unsigned long long bad_in = c.red_host[kRedInput], bad_num = c.red_host[kRedNumeric];
    if (!bad_in && !bad_num) return RRT_OK;
    c.red_host[kRedInput] = c.red_host[kRedNumeric] = 0;
    HIP_OK(hipMemsetAsync(c.red + kRedInput, 0, 2 * sizeof(unsigned long long), c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    if (bad_in)
        return fail(c, RRT_E_INPUT, "a given neutral fraction was outside [0, 1] or a given "
                                    "density not finite and > 0 (rrt_set_state, "
                                    "rrt_set_particles' x_init, rrt_set_density)");
    return fail(c, RRT_E_INPUT, "an update produced a neutral fraction outside [0, 1]");
}

// Synchronise and report the input flags.
int sync_flags(Ctx& c)
{
    HIP_OK(hipMemcpyAsync(c.red_host + kRedInput, c.red + kRedInput,
                          2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    return check_flags(c);
}

hipEvent_t ev_take(Ctx& c)
{
    if (!c.ev_free.empty()) {
        hipEvent_t e = c.ev_free.back();
        c.ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Wait for the recorded spans and add their durations to their accumulators.
void ev_flush(Ctx& c)
{
    if (c.spans.empty()) return;
    (void)hipEventSynchronize(c.spans.back().b);       // every span is on c.stream
    for (const Ctx::TimedSpan& sp : c.spans) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, sp.a, sp.b) == hipSuccess) *sp.acc += ms;
        else (void)hipGetLastError();
        c.ev_free.push_back(sp.a);
        c.ev_free.push_back(sp.b);
    }
    c.spans.clear();
}

// Open a timed span on the context's stream (null when timing is off); spans
// nest, each closed by ev_end with the event ev_begin returned.
hipEvent_t ev_begin(Ctx& c)
{
    if (!c.timing) return nullptr;
    hipEvent_t a = ev_take(c);
    if (a) (void)hipEventRecord(a, c.stream);
    return a;
}

// Close the span opened at `a`; its duration goes to *acc when resolved.
void ev_end(Ctx& c, hipEvent_t a, double* acc)
{
    if (!a) return;
    hipEvent_t b = ev_take(c);
    if (!b) {
        c.ev_free.push_back(a);
        return;
    }
    (void)hipEventRecord(b, c.stream);
    c.spans.push_back(Ctx::TimedSpan{a, b, acc});
    if (c.spans.size() >= 4096) ev_flush(c);
}

int need_tree(Ctx& c)
{
    if (!c.have_tree) return fail(c, RRT_E_STATE, "rrt_build_tree has not been called");
    if (!c.have_rays) return fail(c, RRT_E_STATE, "rrt_set_rays has not been called");
    if (!c.have_spectrum) return fail(c, RRT_E_STATE, "rrt_set_spectrum has not been called");
    return RRT_OK;
}

void free_tpaths(Ctx& c)
{
    ws_free(c, &c.tpath);
    ws_free(c, &c.tcol_off);
    c.tpaths_valid = false;
    c.tpaths_unfit = false;
}

void free_pool(Ctx& c)
{
    ws_free(c, &c.pool);
    ws_free(c, &c.chunk_next);
    ws_free(c, &c.row_first);
    c.pool_chunks = c.slice_chunks = 0;
    c.pool_rows = 0;
}

// What is recorded in the path buffer and derived from the recorded paths.
void free_paths(Ctx& c)
{
    drop_graph(c);
    free_tpaths(c);
    free_tiles(c);
    free_pool(c);
    c.path_evals = 0;
    ws_free(c, &c.path);
    c.path_cap = 0;
    c.path_hits = 0;
    c.paths_valid = false;
    c.paths_unfit = false;
}

// Chunks of the one-walk pool for a recording expected to hold `entries`
// entries over n_rows rays: pool_scale x entries plus half a chunk per ray,
// plus what the walk's waves may hold unused in their caches, rounded up to
// whole slices (or the tuned pool size).
uint64_t pool_chunks_for(const Ctx& c, uint64_t entries, int64_t n_rows)
{
    uint64_t chunks;
    if (c.pool_cap) {
        chunks = c.pool_cap;
    } else {
        const uint64_t e = (uint64_t)((double)entries * c.pool_scale) +
                           (uint64_t)n_rows * (kChunkLen / 2);
        chunks = (e + kChunkLen - 1) / kChunkLen + kCacheAllowance;
    }
    const uint64_t per_slice =
        std::min<uint64_t>((chunks + kPoolSlices - 1) / kPoolSlices, 0xfffffff0ull / kPoolSlices);
    return per_slice * kPoolSlices;
}

uint64_t pool_bytes(uint64_t chunks, int64_t n_rows)
{
    auto up = [](uint64_t b) { return (b + kWsAlign - 1) / kWsAlign * kWsAlign; };
    return up(chunks * sizeof(int2) * kChunkLen) + up(chunks * sizeof(uint32_t)) +
           up((uint64_t)n_rows * sizeof(uint32_t));
}

uint64_t path_bytes(uint64_t entries)
{
    return (((entries ? entries : 1) + kPathPad) * sizeof(int2) + kWsAlign - 1) / kWsAlign *
           kWsAlign;
}

// The one-walk pool in the path buffer, when it fits beside paths of about the
// expected size.  No pool (and no error) otherwise.
void ensure_pool(Ctx& c, int64_t n_rows, uint64_t expect)
{
    free_pool(c);
    if (!c.pool_cap && expect == 0) return;            // nothing to size it from
    const uint64_t chunks = pool_chunks_for(c, expect, n_rows);
    if (pool_bytes(chunks, n_rows) + path_bytes(expect) > ws_largest_gap(c, kRegionPath)) return;
    hipError_t e = ws_alloc(c, &c.pool, chunks * kChunkLen, kRegionPath);
    if (e == hipSuccess) e = ws_alloc(c, &c.chunk_next, chunks, kRegionPath);
    if (e == hipSuccess) e = ws_alloc(c, &c.row_first, (size_t)n_rows, kRegionPath);
    if (e != hipSuccess) {
        free_pool(c);
        return;
    }
    c.pool_chunks = chunks;
    c.slice_chunks = chunks / kPoolSlices;
    c.pool_rows = n_rows;
}

// The paths do not fit the path buffer: traverse instead, or fail when
// recording is required.
int paths_unfit(Ctx& c, uint64_t total)
{
    free_paths(c);
    c.last_total = total;
    c.n_rec_unfit += 1;
    if (c.prm.record_paths == 1)
        return fail(c, RRT_E_WORKSPACE,
                    "recorded paths need %llu bytes; the path buffer holds %llu "
                    "(rrt_count_paths, rrt_set_path_buffer)",
                    (unsigned long long)path_bytes(total),
                    (unsigned long long)c.arena.cap[kRegionPath]);
    c.paths_unfit = true;
    return RRT_OK;
}

// Record (tree index, K/h^2) per intersection into the path buffer, rows in
// order, with row offsets in c.row_off: one recording walk when the counts of
// this tree are known (rrt_count_paths); else one walk into pool chunks, their
// compaction into rows, and a second, recording walk only when the pool ran
// short; else a counting walk and a recording walk.  Leaves the paths unfit
// (and traversal in charge) when they do not fit the path buffer.
int record_paths(Ctx& c)
{
    Range range("rrt: record paths");
    const int64_t n_rows = c.n * (int64_t)c.n_ray;
    free_paths(c);
    if (!c.arena.base[kRegionPath]) {
        c.n_rec_unfit += 1;
        if (c.prm.record_paths == 1)
            return fail(c, RRT_E_WORKSPACE,
                        "recording the paths needs a path buffer (rrt_count_paths, "
                        "rrt_set_path_buffer)");
        c.paths_unfit = true;
        return RRT_OK;
    }
    hipEvent_t ev_rec = ev_begin(c);
    uint64_t total = 0;
    int kind = 3;                                   // counting walk + recording walk
    if (c.counts_valid) {
        total = c.count_total;
        kind = 2;
    } else {
        bool chunked = false;
        if (c.one_pass && c.prm.traversal == 0 && c.images_fit) {
            ensure_pool(c, n_rows, c.last_total);
            chunked = c.pool != nullptr;
        }
        const size_t n_ctr = (size_t)kPoolSlices * kCtrStride + 1;
        if (chunked) {
            HIP_OK(hipMemsetAsync(c.pool_ctr, 0, n_ctr * sizeof(unsigned long long), c.stream));
            hipEvent_t ew = ev_begin(c);
            HIP_OK(launch_record_chunks(c, c.row_off));
            ev_end(c, ew, &c.t_chunk_walk);
            c.n_chunk_walk += c.timing ? 1 : 0;
        } else {
            hipEvent_t ew = ev_begin(c);
            HIP_OK(launch_count_hits(c, c.row_off));
            ev_end(c, ew, &c.t_other_walk);
        }
        HIP_OK(hipMemsetAsync(c.row_off + n_rows, 0, sizeof(uint64_t), c.stream));
        HIP_OK(scan_exclusive_u64(c, c.row_off, c.row_off, n_rows + 1));
        unsigned long long overflow = 0;
        HIP_OK(hipMemcpyAsync(&total, c.row_off + n_rows, sizeof total, hipMemcpyDeviceToHost,
                              c.stream));
        if (chunked)
            HIP_OK(hipMemcpyAsync(&overflow, c.pool_ctr + n_ctr - 1, sizeof overflow,
                                  hipMemcpyDeviceToHost, c.stream));
        HIP_OK(hipStreamSynchronize(c.stream));
        if (chunked) {
            kind = overflow ? 1 : 0;
            // a pool that ran short is sized half as large again next time
            if (overflow) c.pool_scale = std::min(c.pool_scale * 1.5, 4.0);
        }
        c.counts_valid = true;                      // row_off holds this tree's offsets
        c.count_total = total;
    }
    // the compaction needs the paths beside the pool; the recording walk only
    // the paths
    if (kind == 0 && ws_alloc(c, &c.path, total + kPathPad, kRegionPath) != hipSuccess) kind = 1;
    if (kind != 0) {
        free_pool(c);
        if (ws_alloc(c, &c.path, total + kPathPad, kRegionPath) != hipSuccess) {
            ev_end(c, ev_rec, &c.t_record);
            return paths_unfit(c, total);
        }
    }
    c.path_cap = std::max<uint64_t>(total, 1);
    hipEvent_t ew = ev_begin(c);
    if (kind == 0) {
        HIP_OK(launch_compact_chunks(c));
        ev_end(c, ew, &c.t_compact);
    } else {
        HIP_OK(launch_record_paths(c, c.row_off, c.path, total));
        ev_end(c, ew, &c.t_other_walk);
    }
    free_pool(c);
    if (kind == 0) c.n_rec_one += 1;
    else if (kind == 1) c.n_rec_fallback += 1;
    else if (kind == 2) c.n_rec_counted += 1;
    else c.n_rec_two += 1;
    c.path_hits = (int64_t)total;
    c.last_total = total;
    c.paths_valid = true;
    ev_end(c, ev_rec, &c.t_record);
    return RRT_OK;
}

// Columns for the current state.  Returns the intersections of this evaluation
// through *hits when they are known on the host (recorded paths), else -1 (the
// traversal counts them into red[1]).
int columns_impl(Ctx& c, int64_t* hits)
{
    *hits = -1;
    if (c.prm.record_paths != 0 && !c.paths_valid && !c.paths_unfit) {
        if (int r = record_paths(c)) return r;
    }
    if (c.paths_valid) {
        const int64_t n_rows = c.n * (int64_t)c.n_ray;
        const double mean = (double)c.path_hits / (double)std::max<int64_t>(n_rows, 1);
        // measured on MI355X: 32 lanes per ray are fastest from a few tens of
        // intersections per ray up to hundreds; short rays want fewer lanes
        const int group = c.path_group ? c.path_group
                          : mean >= 40 ? 32 : mean >= 16 ? 16 : 8;
        // a full sweep of the plain product streams the path array by blocks
        // of rows unless a lane group per ray is asked for
        const bool stream = c.path_group == 0 && !c.near_far && !c.row_list &&
                            !c.geom.seg_active && !c.geom.want;
        if (c.use_tiles && !c.near_far && !c.tiles_valid && !c.tiles_unfit && !c.capturing &&
            ++c.path_evals > kTileAfter) {
            hipEvent_t et = ev_begin(c);
            HIP_OK(build_tiles(c));
            ev_end(c, et, &c.t_tile_build);
        }
        // a source list (one block of the density order) walks only its own
        // rows in the plain product; the tiles serve full sweeps
        const bool tiles = c.tiles_valid && c.use_tiles && !c.near_far && !c.row_list;
        hipEvent_t ep = ev_begin(c);
        if (tiles) HIP_OK(launch_tile_columns(c, tile_group(c)));
        else if (stream) HIP_OK(launch_path_stream(c));
        else HIP_OK(launch_path_columns(c, group));
        if (c.timing) {
            if (tiles) {
                ev_end(c, ep, &c.t_tile);
                c.n_tile += 1;
            } else {
                ev_end(c, ep, &c.t_spmv);
                c.n_spmv += 1;
            }
        }
        *hits = c.path_hits;
    } else {
        hipEvent_t ec = ev_begin(c);
        HIP_OK(launch_columns(c));
        if (c.timing) {
            ev_end(c, ec, &c.t_trace);
            c.n_trace += 1;
        }
    }
    c.have_columns = true;
    return RRT_OK;
}

}  // namespace

namespace rrt {

// The hit lists of the rays of sampled sources (rrt_get_hits_rows), with the
// device staging from `st`: the workspace, or the library's fixed array.
int hits_rows_impl(Ctx& c, int32_t n_src, const int64_t* src, int64_t cap, int64_t* row_off,
                   int32_t* hit_j, int32_t* hit_img, float* hit_fac, HitStaging& st)
{
    if (int r = need_tree(c)) return r;
    if (!row_off) return fail(c, RRT_E_ARG, "row_off is required");
    if (n_src < 1 || n_src > 4096 || !src)
        return fail(c, RRT_E_ARG, "1..4096 source particles are required");
    const int nr = c.n_ray;
    const size_t rows = (size_t)n_src * nr;
    if (int r = st.lists(c, n_src, rows)) return r;
    // the sources' tree positions, found on the device from the sorted inputs
    std::vector<int64_t> in_sorted(src, src + n_src);
    std::sort(in_sorted.begin(), in_sorted.end());
    for (int32_t i = 0; i < n_src; ++i) {
        if (in_sorted[i] < 0 || in_sorted[i] >= c.n)
            return fail(c, RRT_E_ARG, "source %lld out of range", (long long)in_sorted[i]);
        if (i && in_sorted[i] == in_sorted[i - 1])
            return fail(c, RRT_E_ARG, "a source is listed twice");
    }
    std::vector<int32_t> in32(in_sorted.begin(), in_sorted.end()), pos_sorted_in(n_src);
    HIP_OK(hipMemcpyAsync(st.list, in32.data(), sizeof(int32_t) * n_src, hipMemcpyHostToDevice,
                          c.stream));
    HIP_OK(launch_find_positions(c, st.list, n_src, st.pos));
    HIP_OK(hipMemcpyAsync(pos_sorted_in.data(), st.pos, sizeof(int32_t) * n_src,
                          hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    std::vector<int32_t> pos(n_src);                 // caller's source i -> tree position
    for (int32_t i = 0; i < n_src; ++i) {
        const size_t k = (size_t)(std::lower_bound(in_sorted.begin(), in_sorted.end(), src[i]) -
                                  in_sorted.begin());
        pos[i] = pos_sorted_in[k];
        if (pos[i] < 0) return fail(c, RRT_E_HIP, "source %lld not in the tree", (long long)src[i]);
    }
    // the walk takes the sources in tree order: slot s holds sorted position s
    std::vector<int32_t> sorted(pos);
    std::sort(sorted.begin(), sorted.end());
    std::vector<int32_t> slot_of(n_src);
    for (int32_t i = 0; i < n_src; ++i)
        slot_of[i] = (int32_t)(std::lower_bound(sorted.begin(), sorted.end(), pos[i]) -
                               sorted.begin());
    HIP_OK(hipMemcpyAsync(st.list, sorted.data(), sizeof(int32_t) * n_src,
                          hipMemcpyHostToDevice, c.stream));
    HIP_OK(launch_count_rows(c, st.list, n_src, st.cnt));
    std::vector<uint64_t> cnt(rows);
    HIP_OK(hipMemcpyAsync(cnt.data(), st.cnt, sizeof(uint64_t) * rows, hipMemcpyDeviceToHost,
                          c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    // offsets in the caller's order, and in slot order for the device
    row_off[0] = 0;
    for (int32_t i = 0; i < n_src; ++i)
        for (int k = 0; k < nr; ++k) {
            const size_t r = (size_t)i * nr + k;
            row_off[r + 1] = row_off[r] + (int64_t)cnt[(size_t)slot_of[i] * nr + k];
        }
    const int64_t total = row_off[rows];
    if (!hit_j || !hit_img) return RRT_OK;
    if (total > cap)
        return fail(c, RRT_E_CAPACITY, "%lld hits, capacity %lld", (long long)total,
                    (long long)cap);
    std::vector<uint64_t> dev_off(rows + 1);
    for (int32_t i = 0; i < n_src; ++i)
        for (int k = 0; k < nr; ++k)
            dev_off[(size_t)slot_of[i] * nr + k] = (uint64_t)row_off[(size_t)i * nr + k];
    dev_off[rows] = (uint64_t)total;
    if (int r = st.hits(c, (uint64_t)std::max<int64_t>(total, 1))) return r;
    HIP_OK(hipMemcpyAsync(st.cnt, dev_off.data(), sizeof(uint64_t) * (rows + 1),
                          hipMemcpyHostToDevice, c.stream));
    HIP_OK(launch_record_rows(c, st.list, n_src, st.cnt, st.j, st.img, st.fac, (uint64_t)total));
    HIP_OK(hipMemcpyAsync(hit_j, st.j, sizeof(int32_t) * total, hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipMemcpyAsync(hit_img, st.img, sizeof(int32_t) * total, hipMemcpyDeviceToHost,
                          c.stream));
    if (hit_fac)
        HIP_OK(hipMemcpyAsync(hit_fac, st.fac, sizeof(float) * total, hipMemcpyDeviceToHost,
                              c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    return RRT_OK;
}

// staging of rrt_get_hits_rows in the workspace
struct WsStaging : HitStaging {
    Scratch<int32_t> s_list, s_pos, s_j, s_img;
    Scratch<uint64_t> s_cnt;
    Scratch<float> s_fac;
    explicit WsStaging(Ctx& c) : s_list(c), s_pos(c), s_j(c), s_img(c), s_cnt(c), s_fac(c) {}
    int lists(Ctx& c, int32_t n_src, size_t rows) override
    {
        HIP_OK(s_list.get((size_t)n_src));
        HIP_OK(s_pos.get((size_t)n_src));
        HIP_OK(s_cnt.get(rows + 1));
        list = s_list.p;
        pos = s_pos.p;
        cnt = s_cnt.p;
        return RRT_OK;
    }
    int hits(Ctx& c, uint64_t m) override
    {
        HIP_OK(s_j.get(m));
        HIP_OK(s_img.get(m));
        HIP_OK(s_fac.get(m));
        j = s_j.p;
        img = s_img.p;
        fac = s_fac.p;
        return RRT_OK;
    }
};

}  // namespace rrt

extern "C" {

int rrt_version(void) { return 2 * 10000 + 0 * 100 + 0; }

int rrt_create(rrt_ctx** out, const rrt_params* params, void* stream)
{
    if (!out || !params) {
        g_create_err = "rrt_create: null argument";
        return RRT_E_ARG;
    }
    *out = nullptr;
    if (!(params->l_ray >= 0.0) || !std::isfinite(params->l_ray) || !(params->box >= 0.0) ||
        !std::isfinite(params->box) || params->leaf_size < 0 || params->leaf_size > kLeafMax ||
        params->block_size < 0 || params->block_size > 256 || (params->block_size % 64) != 0 ||
        params->record_paths < -1 || params->record_paths > 1 || params->traversal < 0 ||
        params->traversal > 1) {
        g_create_err = "rrt_create: invalid params (l_ray >= 0, box >= 0, leaf_size 0..16, "
                       "block_size a multiple of 64 up to 256, record_paths -1..1, "
                       "traversal 0..1)";
        return RRT_E_ARG;
    }
    for (int i = 0; i < 2; ++i)
        if (params->reserved[i] != 0) {
            g_create_err = "rrt_create: reserved fields must be zero";
            return RRT_E_ARG;
        }
    rrt_ctx* x = new (std::nothrow) rrt_ctx;
    if (!x) {
        g_create_err = "rrt_create: out of host memory";
        return RRT_E_ARG;
    }
    Ctx& c = x->c;
    c.prm = *params;
    c.leaf = params->leaf_size ? params->leaf_size : kDefaultLeaf;
    c.stream = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipGetDevice(&c.device);
    // the fixed staging array of rrt_get_hits_rows_noalloc on this device
    if (e == hipSuccess) e = noalloc_setup(c.device);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&c.red_host, kRedSlots * sizeof(unsigned long long));
    if (e == hipSuccess) std::memset(c.red_host, 0, kRedSlots * sizeof(unsigned long long));
    if (e != hipSuccess) {
        g_create_err = std::string("rrt_create: HIP error: ") + hipGetErrorString(e);
        rrt_destroy(x);
        return RRT_E_HIP;
    }
    *out = x;
    return RRT_OK;
}

void rrt_destroy(rrt_ctx* x)
{
    if (!x) return;
    Ctx& c = x->c;
    if (c.stream) (void)hipStreamSynchronize(c.stream);
    else (void)hipDeviceSynchronize();
    drop_graph(c);
    if (c.gstream) {
        (void)hipStreamSynchronize(c.gstream);
        (void)hipStreamDestroy(c.gstream);
    }
    if (c.ev_a) (void)hipEventDestroy(c.ev_a);
    if (c.ev_b) (void)hipEventDestroy(c.ev_b);
    if (c.seg_state_host) (void)hipHostFree(c.seg_state_host);
    if (c.red_host) (void)hipHostFree(c.red_host);
    ev_flush(c);
    for (hipEvent_t e : c.ev_free) (void)hipEventDestroy(e);
    c.ev_free.clear();
    delete x;                         // the device memory is the caller's
}

const char* rrt_last_error(const rrt_ctx* x)
{
    return x ? x->c.err.c_str() : g_create_err.c_str();
}

int rrt_workspace_size(const rrt_ctx* x, int64_t n, int32_t n_ray, int32_t n_bins,
                       int32_t n_halo, int32_t reverse_K, size_t* bytes)
{
    if (!x || !bytes || n < 0 || n > (int64_t(1) << 27) || n_ray < 0 || n_ray > kMaxRays ||
        n_bins < 0 || n_bins > kMaxBins || n_halo < 0 || n_halo > 4096 || reverse_K < 0 ||
        reverse_K > 100000)
        return RRT_E_ARG;
    *bytes = (size_t)workspace_bytes(n, n_ray, n_bins, n_halo, reverse_K, x->c.near_far != 0);
    return RRT_OK;
}

int rrt_set_workspace(rrt_ctx* x, void* dev, size_t bytes)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (!dev || bytes == 0) return fail(c, RRT_E_ARG, "a workspace needs a device pointer and size");
    if (reinterpret_cast<uintptr_t>(dev) % kWsAlign)
        return fail(c, RRT_E_ARG, "the workspace must be %llu-byte aligned",
                    (unsigned long long)kWsAlign);
    const uint64_t hw = ws_high_water(c, kRegionWs);
    if (hw > bytes)
        return fail(c, RRT_E_WORKSPACE, "the context's buffers reach %llu bytes; the new "
                                        "workspace has %zu", (unsigned long long)hw, bytes);
    // a captured graph and the geometry refer to the old addresses
    drop_graph(c);
    if (c.gstream) HIP_OK(hipStreamSynchronize(c.gstream));
    HIP_OK(ws_move(c, static_cast<char*>(dev), bytes));
    if (c.have_tree && c.n_halo > 1) {
        c.geom.seg_of = c.seg_of;
        c.geom.seg_root = c.seg_root;
        c.geom.seg_end = c.seg_end;
    }
    return alloc_ctx_buffers(c);
}

int rrt_workspace_info(const rrt_ctx* x, size_t* out6)
{
    if (!x || !out6) return RRT_E_ARG;
    const Ctx& c = x->c;
    out6[0] = (size_t)ws_used(c, kRegionWs);
    out6[1] = (size_t)c.arena.cap[kRegionWs];
    out6[2] = (size_t)ws_used(c, kRegionPath);
    out6[3] = (size_t)c.arena.cap[kRegionPath];
    out6[4] = (size_t)c.arena.short_bytes;
    out6[5] = (size_t)(int64_t)c.arena.short_region;
    return RRT_OK;
}

int rrt_set_path_buffer(rrt_ctx* x, void* dev, size_t bytes)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if ((dev == nullptr) != (bytes == 0))
        return fail(c, RRT_E_ARG, "a path buffer needs both a pointer and a size (or neither)");
    if (reinterpret_cast<uintptr_t>(dev) % kWsAlign)
        return fail(c, RRT_E_ARG, "the path buffer must be %llu-byte aligned",
                    (unsigned long long)kWsAlign);
    // work queued on the old buffer finishes before it is given back
    if (c.stream) HIP_OK(hipStreamSynchronize(c.stream));
    if (c.gstream) HIP_OK(hipStreamSynchronize(c.gstream));
    free_paths(c);
    ws_free(c, &c.Nhist);
    c.Nhist_cap = 0;
    c.Nhist_on = false;
    for (const Arena::Block& b : c.arena.blocks)
        if (b.region == kRegionPath)
            return fail(c, RRT_E_STATE, "a buffer of the old path buffer is still in use");
    c.arena.base[kRegionPath] = static_cast<char*>(dev);
    c.arena.cap[kRegionPath] = bytes;
    return RRT_OK;
}

int rrt_set_particles(rrt_ctx* x, int64_t n, const float* pos, const float* h, const float* mu,
                      const float* n_H, const float* T, const double* x_init)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_ws(c)) return r;
    if (n < 1 || n > (int64_t(1) << 27))
        return fail(c, RRT_E_ARG, "particle count %lld outside 1..2^27", (long long)n);
    if (!pos || !h || !mu || !n_H || !T) return fail(c, RRT_E_ARG, "null particle array");
    free_paths(c);
    int r = alloc_particles(c, n);
    if (r) return r;
    c.n = n;
    if (c.have_rays) {
        if (int r2 = alloc_columns(c)) return r2;
    }
    HIP_OK(hipMemcpyAsync(c.pos_in, pos, sizeof(float) * 3 * n, hipMemcpyDeviceToDevice, c.stream));
    HIP_OK(hipMemcpyAsync(c.h_in, h, sizeof(float) * n, hipMemcpyDeviceToDevice, c.stream));
    HIP_OK(hipMemcpyAsync(c.mu_in, mu, sizeof(float) * n, hipMemcpyDeviceToDevice, c.stream));
    HIP_OK(hipMemcpyAsync(c.nH_in, n_H, sizeof(float) * n, hipMemcpyDeviceToDevice, c.stream));
    HIP_OK(hipMemcpyAsync(c.T_in, T, sizeof(float) * n, hipMemcpyDeviceToDevice, c.stream));
    c.x_init_given = x_init != nullptr;
    if (x_init)
        HIP_OK(hipMemcpyAsync(c.x_init, x_init, sizeof(double) * n, hipMemcpyDeviceToDevice,
                              c.stream));
    c.have_particles = true;
    c.have_tree = c.have_columns = c.have_gamma = false;
    c.fwd_K = -1;
    c.n_halo = 1;                 // rrt_set_halos may follow
    c.halo_off_host.clear();
    return RRT_OK;
}

int rrt_set_halos(rrt_ctx* x, int32_t n_halo, const int64_t* offsets)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (!c.have_particles) return fail(c, RRT_E_STATE, "rrt_set_particles must come first");
    if (n_halo < 1 || n_halo > 4096 || !offsets)
        return fail(c, RRT_E_ARG, "n_halo must be 1..4096 with n_halo + 1 offsets");
    if (offsets[0] != 0 || offsets[n_halo] != c.n)
        return fail(c, RRT_E_ARG, "offsets must run from 0 to n");
    for (int h = 0; h < n_halo; ++h)
        if (offsets[h + 1] <= offsets[h])
            return fail(c, RRT_E_ARG, "halo %d is empty or offsets decrease", h);
    free_paths(c);
    HIP_OK(ws_alloc(c, &c.halo_off, (size_t)n_halo + 1));
    HIP_OK(ws_alloc(c, &c.seg_root, (size_t)n_halo));
    HIP_OK(ws_alloc(c, &c.seg_end, (size_t)n_halo));
    HIP_OK(ws_alloc(c, &c.seg_active, (size_t)n_halo));
    HIP_OK(ws_alloc(c, &c.seg_maxdx, (size_t)n_halo));
    HIP_OK(ws_alloc(c, &c.seg_iters, (size_t)n_halo));
    if (!c.seg_state) HIP_OK(ws_alloc(c, &c.seg_state, 4));
    if (!c.seg_state_host) HIP_OK(hipHostMalloc((void**)&c.seg_state_host, 4 * sizeof(int32_t)));
    c.halo_off_host.assign(offsets, offsets + n_halo + 1);
    HIP_OK(hipMemcpyAsync(c.halo_off, c.halo_off_host.data(), sizeof(int64_t) * (n_halo + 1),
                          hipMemcpyHostToDevice, c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    c.n_halo = n_halo;
    c.have_tree = c.have_columns = c.have_gamma = false;
    return RRT_OK;
}

int rrt_set_rays(rrt_ctx* x, int32_t n_ray, const double* dirs)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_ws(c)) return r;
    if (n_ray < 1 || n_ray > kMaxRays || !dirs)
        return fail(c, RRT_E_ARG, "n_ray must be 1..%d with a direction array", kMaxRays);
    for (int k = 0; k < n_ray; ++k) {
        double a = dirs[3 * k], b = dirs[3 * k + 1], d = dirs[3 * k + 2];
        double nn = a * a + b * b + d * d;
        if (!std::isfinite(nn) || std::fabs(nn - 1.0) > 1e-6)
            return fail(c, RRT_E_ARG, "direction %d is not a unit vector", k);
    }
    free_paths(c);
    HIP_OK(ws_alloc(c, &c.dirs, (size_t)3 * n_ray));
    HIP_OK(hipMemcpyAsync(c.dirs, dirs, sizeof(double) * 3 * n_ray, hipMemcpyHostToDevice,
                          c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    const bool changed = n_ray != c.n_ray;
    c.n_ray = n_ray;
    c.geom.n_ray = n_ray;
    c.have_rays = true;
    c.have_columns = c.have_gamma = false;
    c.counts_valid = false;
    c.fwd_K = -1;
    if (changed) free_adjoint(c);
    if (c.have_particles && (changed || !c.N_s)) return alloc_columns(c);
    return RRT_OK;
}

int rrt_healpix_dirs(int32_t n_side, double* out)
{
    if (n_side < 1 || n_side > 16 || !out) return RRT_E_ARG;
    const double pi = 3.14159265358979323846;
    const int ns = n_side;
    int64_t w = 0;
    for (int i = 1; i < 4 * ns; ++i) {
        double z;
        int cnt;
        double phi0, dphi;
        if (i < ns) {
            z = 1.0 - (double)i * i / (3.0 * ns * ns);
            cnt = 4 * i;
            dphi = pi / (2.0 * i);
            phi0 = 0.5 * dphi;
        } else if (i <= 3 * ns) {
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * ns);
            cnt = 4 * ns;
            dphi = pi / (2.0 * ns);
            int s = (i - ns + 1) % 2;
            phi0 = dphi * (1.0 - 0.5 * s);
        } else {
            int ii = 4 * ns - i;
            z = -(1.0 - (double)ii * ii / (3.0 * ns * ns));
            cnt = 4 * ii;
            dphi = pi / (2.0 * ii);
            phi0 = 0.5 * dphi;
        }
        double st = std::sqrt(std::max(0.0, (1.0 - z) * (1.0 + z)));
        for (int j = 0; j < cnt; ++j) {
            double phi = phi0 + dphi * j;
            out[3 * w] = st * std::cos(phi);
            out[3 * w + 1] = st * std::sin(phi);
            out[3 * w + 2] = z;
            ++w;
        }
    }
    return RRT_OK;
}

int rrt_set_spectrum(rrt_ctx* x, int32_t n_bins, const double* sigma, const double* w)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_ws(c)) return r;
    if (n_bins < 1 || n_bins > kMaxBins || !sigma || !w)
        return fail(c, RRT_E_ARG, "n_bins must be 1..%d with sigma and w arrays", kMaxBins);
    double smin = INFINITY, wsmax = 0.0, thin = 0.0;
    for (int b = 0; b < n_bins; ++b) {
        if (!(sigma[b] > 0.0) || !std::isfinite(sigma[b]) || !(w[b] >= 0.0) ||
            !std::isfinite(w[b]))
            return fail(c, RRT_E_ARG, "bin %d: need sigma > 0 and w >= 0, finite", b);
        if (w[b] > 0.0) {
            smin = std::min(smin, sigma[b]);
            wsmax = std::max(wsmax, w[b] * sigma[b]);
            thin += w[b] * sigma[b];
        }
    }
    if (!(thin > 0.0)) return fail(c, RRT_E_ARG, "the optically thin rate sum(w*sigma) is zero");
    // keep the bins that carry photons; rays see them relative to the least-absorbed one
    std::vector<float> rel, dsl, srt;
    const double log2e = 1.4426950408889634;
    for (int b = 0; b < n_bins; ++b) {
        if (!(w[b] > 0.0)) continue;
        rel.push_back((float)(w[b] * sigma[b] / wsmax));
        dsl.push_back((float)((sigma[b] - smin) * log2e));
        srt.push_back((float)(sigma[b] / smin));
    }
    int m = (int)rel.size();
    if (m != c.n_bins || !c.ws_rel || !c.srat) {
        drop_graph(c);
        HIP_OK(ws_alloc(c, &c.ws_rel, m));
        HIP_OK(ws_alloc(c, &c.dsig_l2, m));
        HIP_OK(ws_alloc(c, &c.srat, m));
    }
    HIP_OK(hipMemcpyAsync(c.ws_rel, rel.data(), sizeof(float) * m, hipMemcpyHostToDevice,
                          c.stream));
    HIP_OK(hipMemcpyAsync(c.dsig_l2, dsl.data(), sizeof(float) * m, hipMemcpyHostToDevice,
                          c.stream));
    HIP_OK(hipMemcpyAsync(c.srat, srt.data(), sizeof(float) * m, hipMemcpyHostToDevice,
                          c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));     // host vectors go out of scope
    if (m != c.n_bins) drop_graph(c);
    c.n_bins = m;
    // Taylor moments of the bins as the rate kernel sums them (the FP32
    // tables r_b, d_b with exponent d_b N in base 2): S(N) = sum_b r_b
    // 2^{-d_b N} = sum_j tay[j] N^j + tail, tay[j] = (-ln 2)^j / j! sum_b r_b
    // d_b^j, used while every y_b = d_b N ln 2 <= 0.15
    {
        const double ln2 = 0.6931471805599453;
        double dmax = 0.0, fact = 1.0, sgn = 1.0, p = 1.0;
        for (int b = 0; b < m; ++b) dmax = std::max(dmax, (double)dsl[b]);
        for (int j = 0; j < kTaylorTerms; ++j) {
            if (j > 0) {
                fact *= j;
                sgn = -sgn;
                p *= ln2;
            }
            double acc = 0.0, acc_t = 0.0;
            for (int b = 0; b < m; ++b) {
                const double t = (double)rel[b] * std::pow((double)dsl[b], j);
                acc += t;
                acc_t += t * (double)srt[b];
            }
            c.tay[j] = sgn * p / fact * acc;
            c.tay_t[j] = sgn * p / fact * acc_t;
        }
        c.tay_nmax = dmax > 0.0 ? 0.15 / (dmax * ln2) : INFINITY;
    }
    c.sigma_min = smin;
    c.ln_ws_max = std::log(wsmax);
    c.ws_max = wsmax;
    c.gamma_thin = thin;
    c.sigma_host.assign(sigma, sigma + n_bins);
    c.w_host.assign(w, w + n_bins);
    ws_free(c, &c.att_tab);             // tabulated for the old spectrum
    c.all_bins_weighted = (m == n_bins);
    c.have_spectrum = true;
    c.have_gamma = false;
    c.fwd_K = -1;                      // rrt_backward needs a forward with this spectrum
    return RRT_OK;
}

int rrt_build_tree(rrt_ctx* x)
{
    Range range("rrt_build_tree");
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (!c.have_particles) return fail(c, RRT_E_STATE, "rrt_set_particles has not been called");
    if (!c.have_spectrum) return fail(c, RRT_E_STATE, "rrt_set_spectrum must precede the build");
    c.fwd_K = -1;
    // a new geometry: the recorded paths and their counts no longer apply
    free_paths(c);
    c.counts_valid = false;
    c.have_tree = c.have_columns = c.have_gamma = false;
    hipEvent_t eb = ev_begin(c);
    // bounds and validation
    const int nb = (int)std::min<int64_t>(1024, (c.n + 255) / 256);
    std::vector<float> hp(8 * nb);
    {
        Scratch<float> part(c);
        HIP_OK(part.get((size_t)8 * nb));
        HIP_OK(launch_bounds(c, part.p, nb));
        HIP_OK(hipMemcpyAsync(hp.data(), part.p, sizeof(float) * 8 * nb, hipMemcpyDeviceToHost,
                              c.stream));
        HIP_OK(hipStreamSynchronize(c.stream));
    }
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    float hmax = 0.f, bad = 0.f;
    for (int b = 0; b < nb; ++b) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], hp[8 * b + a]);
            hi[a] = std::max(hi[a], hp[8 * b + 3 + a]);
        }
        hmax = std::max(hmax, hp[8 * b + 6]);
        bad = std::max(bad, hp[8 * b + 7]);
    }
    if (bad > 0.f)
        return fail(c, RRT_E_INPUT, "particle data must be finite with h, n_H, T > 0, mu >= 0");
    double dlo[3], ext = 0.0, maxabs = 0.0;
    for (int a = 0; a < 3; ++a) {
        dlo[a] = (double)lo[a];
        ext = std::max(ext, (double)hi[a] - (double)lo[a]);
        maxabs = std::max({maxabs, std::fabs((double)lo[a]), std::fabs((double)hi[a])});
    }
    // one halo: 21 bits per axis; several: the halo index takes the top bits
    int hb = 0;
    while ((1 << hb) < c.n_halo) ++hb;
    c.key_bits = c.n_halo > 1 ? (63 - hb) / 3 : 21;
    const double scale = ext > 0.0 ? (double)(1u << c.key_bits) / ext : 0.0;
    HIP_OK(hipMemsetAsync(c.red + kRedBuild, 0, sizeof(unsigned long long), c.stream));
    HIP_OK(launch_morton(c, dlo, scale, c.key_bits));
    HIP_OK(radix_sort_pairs(c, c.codes, c.perm, c.n));
    if (c.n_halo > 1)                            // every byte 0xff: -1, no halo root yet
        HIP_OK(hipMemsetAsync(c.seg_root, 0xff, sizeof(int32_t) * c.n_halo, c.stream));
    HIP_OK(build_radix_tree(c));
    if (c.n_halo > 1) {
        std::vector<int32_t> roots(c.n_halo);
        HIP_OK(hipMemcpyAsync(roots.data(), c.seg_root, sizeof(int32_t) * c.n_halo,
                              hipMemcpyDeviceToHost, c.stream));
        HIP_OK(hipStreamSynchronize(c.stream));
        for (int h = 0; h < c.n_halo; ++h)
            if (roots[h] < 0)
                return fail(c, RRT_E_HIP, "halo %d has no subtree of its own", h);
    }
    int32_t nn = 1;
    if (c.n > 1)
        HIP_OK(hipMemcpyAsync(&nn, c.k_dfs, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipMemcpyAsync(c.red_host + kRedBuild, c.red + kRedBuild, sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    if (c.red_host[kRedBuild] != 0 || nn < 1 || nn > 2 * c.n - 1)
        return fail(c, RRT_E_HIP, "tree construction inconsistent (flags %llu, %d nodes)",
                    (unsigned long long)c.red_host[kRedBuild], nn);
    c.n_nodes = nn;
    TraceGeom& g = c.geom;
    g.L = c.prm.l_ray;
    g.box = c.prm.box;
    for (int a = 0; a < 3; ++a) {
        g.plo[a] = lo[a];
        g.phi[a] = hi[a];
    }
    g.hmax = hmax;
    g.pad = (float)(4e-6 * 2.0 * (maxabs + g.L + (double)hmax + g.box));
    // the one-walk recording codes a hit's periodic image in 10 bits per axis
    c.images_fit = !(g.box > 0.0) || (g.L + (double)hmax + ext) / g.box + 2.0 <= 511.0;
    g.n = (int32_t)c.n;
    g.n_ray = c.n_ray;
    g.n_nodes = nn;
    const bool segmented = c.n_halo > 1;
    g.seg_of = segmented ? c.seg_of : nullptr;
    g.seg_root = segmented ? c.seg_root : nullptr;
    g.seg_end = segmented ? c.seg_end : nullptr;
    g.seg_active = nullptr;
    g.want = nullptr;
    c.blocks_for = 0;            // the density blocks are in tree order
    HIP_OK(launch_init_state(c, c.x_init_given));
    ev_end(c, eb, &c.t_build);
    if (int r = sync_flags(c)) return r;         // a given x_init out of range
    c.have_tree = true;
    return RRT_OK;
}

int rrt_compute_columns(rrt_ctx* x, double* N_out, int64_t* n_hits_out)
{
    Range range("rrt_compute_columns");
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_tree(c)) return r;
    HIP_OK(hipMemsetAsync(c.red + kRedHits, 0, sizeof(unsigned long long), c.stream));
    int64_t hits = -1;
    if (int r = columns_impl(c, &hits)) return r;
    if (N_out) HIP_OK(launch_to_input_order_d(c, c.N_s, N_out, c.n_ray));
    if (n_hits_out) {
        HIP_OK(hipMemcpyAsync(c.red_host + kRedHits, c.red + kRedHits,
                              sizeof(unsigned long long), hipMemcpyDeviceToHost, c.stream));
        if (int r = sync_flags(c)) return r;
        if (hits < 0) hits = (int64_t)c.red_host[kRedHits];
        *n_hits_out = hits;
    }
    return RRT_OK;
}

int rrt_compute_gamma(rrt_ctx* x, double* lnG_out, double* G_out, float* tau_out)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_tree(c)) return r;
    if (!c.have_columns) return fail(c, RRT_E_STATE, "no columns: call rrt_compute_columns");
    HIP_OK(launch_gamma(c, false));
    c.have_gamma = true;
    if (lnG_out) HIP_OK(launch_to_input_order_d(c, c.lnG_s, lnG_out, 1));
    if (G_out) HIP_OK(launch_to_input_order_d(c, c.G_s, G_out, 1));
    if (tau_out) HIP_OK(launch_to_input_order_f(c, c.tau_s, tau_out));
    return RRT_OK;
}

int rrt_update_equilibrium(rrt_ctx* x, double* x_out, double* max_dx_out)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_tree(c)) return r;
    if (!c.have_gamma) return fail(c, RRT_E_STATE, "no rate: call rrt_compute_gamma");
    HIP_OK(hipMemsetAsync(c.red + kRedMaxDx, 0, sizeof(unsigned long long), c.stream));
    HIP_OK(launch_update_x(c));
    c.have_columns = c.have_gamma = false;
    if (x_out) HIP_OK(launch_to_input_order_d(c, c.x_s, x_out, 1));
    if (max_dx_out) {
        HIP_OK(hipMemcpyAsync(c.red_host + kRedMaxDx, c.red + kRedMaxDx,
                              sizeof(unsigned long long), hipMemcpyDeviceToHost, c.stream));
        if (int r = sync_flags(c)) return r;
        double d;
        std::memcpy(&d, &c.red_host[kRedMaxDx], sizeof d);
        *max_dx_out = d;
    }
    return RRT_OK;
}

namespace {

bool default_rule(const Ctx& c)
{
    return c.rule_tau_skip == 0.0 && std::isinf(c.rule_tau_case_b) && c.rule_relative == 0 &&
           c.rule_blocks == 1;
}

// Block of every particle in the density-descending order (ties: lower input
// index first), blocks of ceil(n / n_blocks) consecutive particles.
int ensure_blocks(Ctx& c)
{
    if (c.blocks_for == c.rule_blocks) return RRT_OK;
    const int64_t n = c.n;
    std::vector<float> nh((size_t)n);
    std::vector<int32_t> perm((size_t)n);
    HIP_OK(hipMemcpyAsync(nh.data(), c.nH_s, sizeof(float) * n, hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipMemcpyAsync(perm.data(), c.perm, sizeof(int32_t) * n, hipMemcpyDeviceToHost,
                          c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    std::vector<int64_t> ord((size_t)n);
    for (int64_t i = 0; i < n; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
        if (nh[a] != nh[b]) return nh[a] > nh[b];
        return perm[a] < perm[b];
    });
    const int64_t bs = (n + c.rule_blocks - 1) / c.rule_blocks;
    std::vector<int32_t> blk((size_t)n);
    for (int64_t r = 0; r < n; ++r) blk[ord[r]] = (int32_t)(r / bs);
    // each block's tree positions in ascending order (coherent rays)
    std::vector<int32_t> lst((size_t)n);
    c.block_off.assign((size_t)c.rule_blocks + 1, 0);
    for (int64_t i = 0; i < n; ++i) ++c.block_off[(size_t)blk[i] + 1];
    for (int b = 0; b < c.rule_blocks; ++b) c.block_off[b + 1] += c.block_off[b];
    std::vector<int64_t> fill(c.block_off.begin(), c.block_off.end() - 1);
    for (int64_t i = 0; i < n; ++i) lst[(size_t)fill[blk[i]]++] = (int32_t)i;
    HIP_OK(hipMemcpyAsync(c.block_s, blk.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice,
                          c.stream));
    HIP_OK(hipMemcpyAsync(c.block_list, lst.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice,
                          c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    c.blocks_for = c.rule_blocks;
    return RRT_OK;
}

// the per-step particle mask lives only inside one sweep of the driver
struct WantGuard {
    Ctx& c;
    explicit WantGuard(Ctx& cc) : c(cc) {}
    ~WantGuard()
    {
        c.geom.want = nullptr;
        c.row_list = nullptr;
        c.row_list_n = 0;
    }
};

}  // namespace

int rrt_set_scheme(rrt_ctx* x, int32_t near_far)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (near_far < 0 || near_far > 1) return fail(c, RRT_E_ARG, "near_far must be 0 or 1");
    if (near_far == c.near_far) return RRT_OK;
    free_paths(c);                    // recorded entries carry the near flag
    c.have_columns = c.have_gamma = false;
    if (c.n > 0 && c.have_rays) {
        // the near columns take their own buffer; alloc_columns drops the counts
        const int32_t old = c.near_far;
        c.near_far = near_far;
        if (int r = alloc_columns(c)) {
            c.near_far = old;
            (void)alloc_columns(c);
            return r;
        }
        return RRT_OK;
    }
    c.near_far = near_far;
    return RRT_OK;
}

int rrt_get_near_columns(rrt_ctx* x, double* out)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (!out) return fail(c, RRT_E_ARG, "out is required");
    if (!c.near_far || !c.have_columns)
        return fail(c, RRT_E_STATE, "near columns need the near/far scheme and rrt_compute_columns");
    HIP_OK(launch_to_input_order_d(c, c.Nn_s, out, c.n_ray));
    HIP_OK(hipStreamSynchronize(c.stream));
    return RRT_OK;
}

int rrt_set_update_rule(rrt_ctx* x, double tau_skip, double tau_case_b, int32_t relative,
                        int32_t n_blocks)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (!(tau_skip >= 0.0) || std::isinf(tau_skip))
        return fail(c, RRT_E_ARG, "tau_skip must be finite and >= 0");
    if (!(tau_case_b > 0.0)) return fail(c, RRT_E_ARG, "tau_case_b must be > 0 (inf: case A)");
    if (relative != 0 && relative != 1) return fail(c, RRT_E_ARG, "relative must be 0 or 1");
    if (n_blocks < 1 || n_blocks > (1 << 20)) return fail(c, RRT_E_ARG, "n_blocks 1..2^20");
    c.rule_tau_skip = tau_skip;
    c.rule_tau_case_b = tau_case_b;
    c.rule_relative = relative;
    c.rule_blocks = n_blocks;
    return RRT_OK;
}

int rrt_iterate_equilibrium(rrt_ctx* x, int32_t max_iter, double tol, double* x_out,
                            int32_t* iters_done, double* max_dx_out)
{
    Range range("rrt_iterate_equilibrium");
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_tree(c)) return r;
    if (max_iter < 0 || !(tol >= 0.0)) return fail(c, RRT_E_ARG, "max_iter >= 0 and tol >= 0");
    if (c.near_far && !default_rule(c))
        return fail(c, RRT_E_STATE, "the near/far scheme runs with the default update rule");
    const bool ordered = c.rule_blocks > 1;
    const bool skipping = c.rule_tau_skip > 0.0;
    if (ordered && c.rule_blocks > c.n)
        return fail(c, RRT_E_ARG, "%d blocks for %lld particles", c.rule_blocks, (long long)c.n);
    if (ordered)
        if (int r = ensure_blocks(c)) return r;
    if (skipping) HIP_OK(hipMemsetAsync(c.skip_s, 0, (size_t)c.n, c.stream));
    const int n_steps = ordered ? c.rule_blocks : 1;
    const bool masked = ordered || skipping;
    WantGuard guard(c);
    int it = 0;
    double mdx = INFINITY;
    // a fixed number of sweeps (tol = 0) counts against the paper's 1e-3
    c.conv_tol = tol > 0.0 ? tol : 1e-3;
    c.conv_maxdx.clear();
    c.conv_abs.clear();
    c.conv_rel.clear();
    for (it = 0; it < max_iter;) {
        // the sweep's reductions; the input flags (slots 6, 7) persist until reported
        HIP_OK(hipMemsetAsync(c.red, 0, kRedInput * sizeof(unsigned long long), c.stream));
        int64_t hits = -1;
        for (int b = 0; b < n_steps; ++b) {
            // one block of the density order (all particles for the
            // order-independent update), frozen particles left out
            if (masked) {
                HIP_OK(launch_want(c, b, skipping && it > 0));
                c.geom.want = c.want_s;
            }
            if (ordered) {                    // the product walks only this block's rays
                c.row_list = c.block_list + c.block_off[b];
                c.row_list_n = c.block_off[b + 1] - c.block_off[b];
            }
            if (int r = columns_impl(c, &hits)) return r;
            hipEvent_t eg = ev_begin(c);
            HIP_OK(launch_gamma(c, true, it == 0));
            ev_end(c, eg, &c.t_rate);
        }
        c.geom.want = nullptr;
        c.row_list = nullptr;
        c.row_list_n = 0;
        HIP_OK(hipMemcpyAsync(c.red_host, c.red, kRedSlots * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, c.stream));
        HIP_OK(hipStreamSynchronize(c.stream));
        if (int r = check_flags(c)) return r;
        ++it;
        std::memcpy(&mdx, &c.red_host[kRedMaxDx], sizeof mdx);
        c.conv_maxdx.push_back(mdx);
        c.conv_abs.push_back((int64_t)c.red_host[kRedConvAbs]);
        c.conv_rel.push_back((int64_t)c.red_host[kRedConvRel]);
        // intersections of the sweep: counted by traversal, or all recorded
        // ones when every ray was evaluated; not counted for masked sweeps
        // over recorded paths
        c.last_hits = hits < 0 ? (int64_t)c.red_host[kRedHits] : (masked ? -1 : hits);
        if (c.last_hits > 0) c.total_hits += c.last_hits;
        if (mdx < tol) break;
    }
    c.have_columns = c.have_gamma = false;
    if (x_out) HIP_OK(launch_to_input_order_d(c, c.x_s, x_out, 1));
    if (iters_done) *iters_done = it;
    if (max_dx_out) *max_dx_out = mdx;
    if (x_out) HIP_OK(hipStreamSynchronize(c.stream));
    return (max_iter > 0 && !(mdx < tol)) ? RRT_NOT_CONVERGED : RRT_OK;
}

int rrt_evolve(rrt_ctx* x, double dt, int32_t n_steps, double* x_out)
{
    Range range("rrt_evolve");
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_tree(c)) return r;
    if (!(dt >= 0.0) || std::isinf(dt) || n_steps < 0)
        return fail(c, RRT_E_ARG, "dt must be finite and >= 0, n_steps >= 0");
    if (!default_rule(c))
        return fail(c, RRT_E_STATE, "the evolution uses case A rates: reset the update rule");
    for (int s = 0; s < n_steps && dt > 0.0; ++s) {     // no time, no change
        int64_t hits = -1;
        if (int r = columns_impl(c, &hits)) return r;
        hipEvent_t eg = ev_begin(c);
        HIP_OK(launch_gamma(c, false));
        HIP_OK(launch_evolve(c, dt));
        ev_end(c, eg, &c.t_rate);
    }
    c.have_columns = c.have_gamma = false;
    if (x_out) {
        HIP_OK(launch_to_input_order_d(c, c.x_s, x_out, 1));
        if (int r = sync_flags(c)) return r;
    }
    return RRT_OK;
}

int rrt_set_density(rrt_ctx* x, const float* n_H)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (!c.have_tree) return fail(c, RRT_E_STATE, "rrt_build_tree has not been called");
    if (!n_H) return fail(c, RRT_E_ARG, "n_H is required");
    c.blocks_for = 0;                  // the density order may change
    HIP_OK(launch_set_density(c, n_H));
    HIP_OK(launch_mux(c));
    c.have_columns = c.have_gamma = false;
    c.fwd_K = -1;
    return RRT_OK;
}

int rrt_forward(rrt_ctx* x, int32_t K, double* lnG_out, double* x_out)
{
    Range range("rrt_forward");
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_tree(c)) return r;
    if (K < 1 || K > 100000) return fail(c, RRT_E_ARG, "K must be 1..100000");
    if (!default_rule(c) || c.near_far)
        return fail(c, RRT_E_STATE, "the reverse mode differentiates the plain order-independent "
                                    "case A update: reset the update rule and the scheme");
    const size_t n = (size_t)c.n;
    if (c.xhist_cap < K + 1 || !c.xhist) {
        HIP_OK(ws_alloc(c, &c.xhist, (size_t)(K + 1) * n));
        c.xhist_cap = K + 1;
    }
    const size_t nr = n * (size_t)c.n_ray;
    c.fwd_K = -1;
    HIP_OK(launch_init_state(c, false));
    HIP_OK(hipMemcpyAsync(c.xhist, c.x_s, sizeof(double) * n, hipMemcpyDeviceToDevice,
                          c.stream));
    for (int k = 1; k <= K; ++k) {
        HIP_OK(hipMemsetAsync(c.red, 0, kRedInput * sizeof(unsigned long long), c.stream));
        int64_t hits = -1;
        if (int r = columns_impl(c, &hits)) return r;
        if (k == 1) {
            // Every iteration's columns are kept for rrt_backward when they fit
            // in the path buffer beside the paths (recorded by the evaluation
            // just made); otherwise it recomputes them from the kept states.
            c.Nhist_on = c.keep_columns && c.Nhist && c.Nhist_cap >= K;
            if (!c.Nhist_on) {
                ws_free(c, &c.Nhist);
                c.Nhist_cap = 0;
                if (c.keep_columns &&
                    ws_alloc(c, &c.Nhist, (size_t)K * nr, kRegionPath) == hipSuccess) {
                    c.Nhist_cap = K;
                    c.Nhist_on = true;
                }
            }
        }
        if (c.Nhist_on)
            HIP_OK(hipMemcpyAsync(c.Nhist + (size_t)(k - 1) * nr, c.N_s, sizeof(double) * nr,
                                  hipMemcpyDeviceToDevice, c.stream));
        HIP_OK(launch_gamma(c, true));
        HIP_OK(hipMemcpyAsync(c.xhist + (size_t)k * n, c.x_s, sizeof(double) * n,
                              hipMemcpyDeviceToDevice, c.stream));
    }
    c.fwd_K = K;
    c.have_columns = c.have_gamma = false;
    if (lnG_out) HIP_OK(launch_to_input_order_d(c, c.lnG_s, lnG_out, 1));
    if (x_out) HIP_OK(launch_to_input_order_d(c, c.x_s, x_out, 1));
    return RRT_OK;
}

int rrt_backward(rrt_ctx* x, const double* dL_dlnG, const double* dL_dx, double* dL_dw,
                 double* dL_dnH)
{
    Range range("rrt_backward");
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_tree(c)) return r;
    if (c.fwd_K < 1) return fail(c, RRT_E_STATE, "rrt_forward must precede rrt_backward");
    if (!c.all_bins_weighted)
        return fail(c, RRT_E_ARG, "gradients need every bin weight w_b > 0");
    const size_t n = (size_t)c.n, nr = n * (size_t)c.n_ray;
    const int64_t waves = adj_waves(c);
    if (!c.adj_lam || c.adj_n != n || c.adj_nr != nr) {
        c.adj_n = c.adj_nr = 0;
        HIP_OK(ws_alloc(c, &c.adj_lam, n));
        HIP_OK(ws_alloc(c, &c.adj_lup, n));
        HIP_OK(ws_alloc(c, &c.adj_gnH, n));
        HIP_OK(ws_alloc(c, &c.adj_y, n));
        HIP_OK(ws_alloc(c, &c.adj_nu, nr));
        HIP_OK(ws_alloc(c, &c.adj_pis, nr));
        HIP_OK(ws_alloc(c, &c.adj_st, nr));
        HIP_OK(ws_alloc(c, &c.adj_ell, n));
        HIP_OK(ws_alloc(c, &c.adj_tpart, (size_t)waves));
        c.adj_n = n;
        c.adj_nr = nr;
    }
    HIP_OK(ws_alloc(c, &c.adj_wpart, (size_t)(adj_chunks(c) + kAdjSlices) * c.n_bins));
    HIP_OK(ws_alloc(c, &c.adj_gw, (size_t)c.n_bins));
    HIP_OK(hipMemsetAsync(c.adj_gw, 0, sizeof(double) * c.n_bins, c.stream));
    HIP_OK(hipMemsetAsync(c.adj_gnH, 0, sizeof(double) * n, c.stream));
    if (dL_dx) HIP_OK(launch_from_input_order_d(c, dL_dx, c.adj_lam));
    else HIP_OK(hipMemsetAsync(c.adj_lam, 0, sizeof(double) * n, c.stream));
    if (dL_dlnG) HIP_OK(launch_from_input_order_d(c, dL_dlnG, c.adj_lup));
    const int K = c.fwd_K;
    for (int k = K; k >= 1; --k) {
        double* xprev = c.xhist + (size_t)(k - 1) * n;
        // the columns of iteration k, kept by the forward or recomputed from x^(k-1)
        const double* Nk = c.N_s;
        if (c.Nhist_on) {
            Nk = c.Nhist + (size_t)(k - 1) * nr;
        } else {
            HIP_OK(hipMemcpyAsync(c.x_s, xprev, sizeof(double) * n, hipMemcpyDeviceToDevice,
                                  c.stream));
            HIP_OK(launch_mux(c));
            int64_t hits = -1;
            if (int r = columns_impl(c, &hits)) return r;
        }
        HIP_OK(launch_adj_rate(c, Nk, (k == K && dL_dlnG) ? c.adj_lup : nullptr));
        if (c.paths_valid && !c.tpaths_valid && !c.tpaths_unfit && c.adj_scatter == 0) {
            // transposed paths (8 B per intersection) plus sort scratch (24 B)
            // in the path buffer, when they fit beside the paths
            const hipError_t e = build_transposed_paths(c);
            if (e == hipSuccess) c.tpaths_valid = true;
            else if (e == hipErrorOutOfMemory) c.tpaths_unfit = true;
            else HIP_OK(e);
        }
        // without transposed paths: accumulate per row tile in LDS when the
        // tiles can be built and fit (one global atomic per distinct particle
        // of a tile instead of one per intersection)
        const bool try_tiles = c.paths_valid && !c.near_far &&
                               (c.adj_scatter == 2 || (c.adj_scatter == 0 && c.tpaths_unfit));
        if (try_tiles && !c.tiles_valid && !c.tiles_unfit) HIP_OK(build_tiles(c));
        const bool tile_scatter = try_tiles && c.tiles_valid &&
                                  c.tile_max_u <= kTileScatterMaxSet;
        if (c.paths_valid && c.tpaths_valid && c.adj_scatter == 0) {
            HIP_OK(launch_gather_cols(c));
        } else if (tile_scatter) {
            HIP_OK(launch_tile_scatter(c, c.adj_nu, c.adj_y));
        } else if (c.paths_valid) {
            HIP_OK(launch_adj_scatter(c));
        } else {
            HIP_OK(hipMemsetAsync(c.adj_y, 0, sizeof(double) * n, c.stream));
            HIP_OK(launch_scatter_traverse(c, c.adj_nu, c.adj_y));
        }
        HIP_OK(launch_adj_x(c, xprev));
    }
    HIP_OK(launch_adj_init(c, c.adj_tpart));
    std::vector<double> gw(c.n_bins), tp((size_t)waves);
    HIP_OK(hipMemcpyAsync(gw.data(), c.adj_gw, sizeof(double) * c.n_bins, hipMemcpyDeviceToHost,
                          c.stream));
    HIP_OK(hipMemcpyAsync(tp.data(), c.adj_tpart, sizeof(double) * waves, hipMemcpyDeviceToHost,
                          c.stream));
    if (dL_dnH) HIP_OK(launch_to_input_order_d(c, c.adj_gnH, dL_dnH, 1));
    // leave the state at x^K, as after the forward
    HIP_OK(hipMemcpyAsync(c.x_s, c.xhist + (size_t)K * n, sizeof(double) * n,
                          hipMemcpyDeviceToDevice, c.stream));
    HIP_OK(launch_mux(c));
    if (int r = sync_flags(c)) return r;
    double thin = 0.0;
    for (double v : tp) thin += v;
    if (dL_dw)
        for (int b = 0; b < c.n_bins; ++b)
            dL_dw[b] = c.sigma_host[b] / c.ws_max * gw[b] + c.sigma_host[b] * thin;
    c.have_columns = c.have_gamma = false;
    return RRT_OK;
}

namespace {

// halo bookkeeping buffers also for a single problem (one halo = whole tree)
int ensure_seg_buffers(Ctx& c)
{
    if (c.n_halo == 1 && (!c.seg_root || !c.seg_active)) {
        HIP_OK(ws_alloc(c, &c.seg_root, 1));
        HIP_OK(ws_alloc(c, &c.seg_end, 1));
        HIP_OK(ws_alloc(c, &c.seg_active, 1));
        HIP_OK(ws_alloc(c, &c.seg_maxdx, 1));
        HIP_OK(ws_alloc(c, &c.seg_iters, 1));
        if (!c.seg_state) HIP_OK(ws_alloc(c, &c.seg_state, 4));
        if (!c.seg_state_host)
            HIP_OK(hipHostMalloc((void**)&c.seg_state_host, 4 * sizeof(int32_t)));
    }
    if (c.n_halo == 1) {
        const int32_t zero = 0, nn = (int32_t)c.n_nodes;
        HIP_OK(hipMemcpyAsync(c.seg_root, &zero, sizeof zero, hipMemcpyHostToDevice, c.stream));
        HIP_OK(hipMemcpyAsync(c.seg_end, &nn, sizeof nn, hipMemcpyHostToDevice, c.stream));
        HIP_OK(hipStreamSynchronize(c.stream));
    }
    if (!c.gstream) HIP_OK(hipStreamCreateWithFlags(&c.gstream, hipStreamNonBlocking));
    if (!c.ev_a) HIP_OK(hipEventCreateWithFlags(&c.ev_a, hipEventDisableTiming));
    if (!c.ev_b) HIP_OK(hipEventCreateWithFlags(&c.ev_b, hipEventDisableTiming));
    return RRT_OK;
}

// one iteration of every active halo: columns, rate + equilibrium, bookkeeping
int halo_iteration(Ctx& c, double tol, int max_iter)
{
    int64_t hits = -1;
    if (int r = columns_impl(c, &hits)) return r;
    HIP_OK(launch_gamma(c, true));
    HIP_OK(launch_seg_finalize(c, tol, max_iter));
    return RRT_OK;
}

struct SegGuard {
    Ctx& c;
    TraceGeom saved;
    explicit SegGuard(Ctx& cc) : c(cc), saved(cc.geom)
    {
        c.geom.seg_of = c.seg_of;
        c.geom.seg_root = c.seg_root;
        c.geom.seg_end = c.seg_end;
        c.geom.seg_active = c.seg_active;
    }
    ~SegGuard() { c.geom = saved; }
};

}  // namespace

namespace {

// Iterate the currently active halos to convergence: one eager iteration, then
// replays of the captured graph (captured on first use, reused while the
// buffers it references stay in place).
int run_active_halos(Ctx& c, double tol, int32_t max_iter, int32_t per_launch)
{
    const bool timing = c.timing;
    if (int r = halo_iteration(c, tol, max_iter)) return r;
    HIP_OK(hipMemcpyAsync(c.seg_state_host, c.seg_state, 2 * sizeof(int32_t),
                          hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    if (c.seg_state_host[1] <= 0) return RRT_OK;
    if (!c.graph_exec || c.graph_iters != per_launch || c.graph_tol != tol ||
        c.graph_max_iter != max_iter) {
        drop_graph(c);
        // the replays should use the row tiles when the solve is long enough to
        // pay for them; nothing may be allocated during the capture
        if (c.use_tiles && c.paths_valid && !c.tiles_valid && !c.tiles_unfit &&
            max_iter > kTileAfter) {
            hipEvent_t et = ev_begin(c);
            HIP_OK(build_tiles(c));
            ev_end(c, et, &c.t_tile_build);
        }
        hipStream_t user = c.stream;
        c.stream = c.gstream;
        c.timing = false;
        c.capturing = true;
        hipError_t e = hipStreamBeginCapture(c.gstream, hipStreamCaptureModeThreadLocal);
        int r = RRT_OK;
        for (int k = 0; k < per_launch && e == hipSuccess && r == RRT_OK; ++k)
            r = halo_iteration(c, tol, max_iter);
        hipGraph_t gr = nullptr;
        hipError_t e2 = hipStreamEndCapture(c.gstream, &gr);
        c.capturing = false;
        c.stream = user;
        c.timing = timing;
        if (r != RRT_OK) {
            if (gr) (void)hipGraphDestroy(gr);
            return r;
        }
        HIP_OK(e);
        HIP_OK(e2);
        c.graph = gr;
        HIP_OK(hipGraphInstantiate(&c.graph_exec, c.graph, nullptr, nullptr, 0));
        c.graph_iters = per_launch;
        c.graph_tol = tol;
        c.graph_max_iter = max_iter;
    }
    HIP_OK(hipEventRecord(c.ev_a, c.stream));
    HIP_OK(hipStreamWaitEvent(c.gstream, c.ev_a, 0));
    while (c.seg_state_host[1] > 0 && c.seg_state_host[0] < max_iter) {
        HIP_OK(hipGraphLaunch(c.graph_exec, c.gstream));
        HIP_OK(hipMemcpyAsync(c.seg_state_host, c.seg_state, 2 * sizeof(int32_t),
                              hipMemcpyDeviceToHost, c.gstream));
        HIP_OK(hipStreamSynchronize(c.gstream));
    }
    HIP_OK(hipEventRecord(c.ev_b, c.gstream));
    HIP_OK(hipStreamWaitEvent(c.stream, c.ev_b, 0));
    return RRT_OK;
}

// Which halos can share recorded paths: per-halo intersection totals from one
// count pass, packed first-fit by decreasing size into groups whose paths fit
// the path buffer.  A halo too large for it alone forms a group that
// traverses every iteration.  Counts stay in row_cnt for the per-group offsets.
int plan_groups(Ctx& c, uint64_t* row_cnt, std::vector<std::vector<int>>& groups,
                std::vector<bool>& recordable, uint64_t& max_group)
{
    const int nh = c.n_halo;
    std::vector<unsigned long long> hits(nh);
    {
        Scratch<unsigned long long> d_hits(c);
        HIP_OK(d_hits.get((size_t)nh));
        HIP_OK(hipMemsetAsync(d_hits.p, 0, sizeof(unsigned long long) * nh, c.stream));
        HIP_OK(launch_count_hits(c, row_cnt));
        HIP_OK(launch_halo_hits(c, row_cnt, d_hits.p));
        HIP_OK(hipMemcpyAsync(hits.data(), d_hits.p, sizeof(unsigned long long) * nh,
                              hipMemcpyDeviceToHost, c.stream));
        HIP_OK(hipStreamSynchronize(c.stream));
    }
    // entries the path buffer holds (with the padding of one array)
    const uint64_t room = c.arena.cap[kRegionPath] / sizeof(int2);
    const uint64_t cap = room > (uint64_t)kPathPad + kWsAlign ? room - kPathPad - kWsAlign : 0;
    std::vector<int> order(nh);
    for (int h = 0; h < nh; ++h) order[h] = h;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return hits[a] > hits[b]; });
    std::vector<uint64_t> load;
    groups.clear();
    recordable.clear();
    max_group = 0;
    for (int h : order) {
        if (c.prm.record_paths == 0 || hits[h] > cap) {
            groups.push_back({h});
            recordable.push_back(false);
            load.push_back(0);
            continue;
        }
        size_t g = 0;
        for (; g < groups.size(); ++g)
            if (recordable[g] && load[g] + hits[h] <= cap) break;
        if (g == groups.size()) {
            groups.push_back({});
            recordable.push_back(true);
            load.push_back(0);
        }
        groups[g].push_back(h);
        load[g] += hits[h];
        max_group = std::max<uint64_t>(max_group, load[g]);
    }
    // traversing halos need no memory: run them together as one group
    std::vector<std::vector<int>> gs;
    std::vector<bool> rs;
    std::vector<int> trav;
    for (size_t g = 0; g < groups.size(); ++g) {
        if (recordable[g]) {
            gs.push_back(groups[g]);
            rs.push_back(true);
        } else {
            trav.insert(trav.end(), groups[g].begin(), groups[g].end());
        }
    }
    if (!trav.empty()) {
        gs.push_back(trav);
        rs.push_back(false);
    }
    groups.swap(gs);
    recordable.swap(rs);
    return RRT_OK;
}

// Halos in groups whose recorded paths fit the path buffer, one group after
// another (the paths held one group at a time are not valid for the batch).
int run_groups(Ctx& c, double tol, int32_t max_iter, int32_t per_launch)
{
    const int64_t n_rows = c.n * (int64_t)c.n_ray;
    Scratch<uint64_t> row_cnt(c);
    Scratch<int32_t> d_mask(c);
    HIP_OK(row_cnt.get((size_t)n_rows));
    HIP_OK(d_mask.get((size_t)c.n_halo));
    std::vector<std::vector<int>> groups;
    std::vector<bool> recordable;
    uint64_t max_group = 0;
    if (int r = plan_groups(c, row_cnt.p, groups, recordable, max_group)) return r;
    if (groups.size() == 1 && recordable[0]) {
        // all paths fit: keep the counts, so the first iteration records them
        // with one walk
        HIP_OK(hipMemcpyAsync(c.row_off, row_cnt.p, sizeof(uint64_t) * n_rows,
                              hipMemcpyDeviceToDevice, c.stream));
        HIP_OK(hipMemsetAsync(c.row_off + n_rows, 0, sizeof(uint64_t), c.stream));
        HIP_OK(scan_exclusive_u64(c, c.row_off, c.row_off, n_rows + 1));
        HIP_OK(hipMemcpyAsync(&c.count_total, c.row_off + n_rows, sizeof(uint64_t),
                              hipMemcpyDeviceToHost, c.stream));
        HIP_OK(hipStreamSynchronize(c.stream));
        c.counts_valid = true;
        return run_active_halos(c, tol, max_iter, per_launch);
    }
    free_paths(c);
    c.counts_valid = false;            // row_off takes each group's offsets
    if (max_group > 0) HIP_OK(ws_alloc(c, &c.path, (size_t)max_group + kPathPad, kRegionPath));
    c.path_cap = max_group;
    std::vector<int32_t> mask(c.n_halo);
    int r = RRT_OK;
    for (size_t g = 0; g < groups.size() && r == RRT_OK; ++g) {
        std::fill(mask.begin(), mask.end(), 0);
        for (int h : groups[g]) mask[h] = 1;
        HIP_OK(hipMemcpyAsync(d_mask.p, mask.data(), sizeof(int32_t) * c.n_halo,
                              hipMemcpyHostToDevice, c.stream));
        HIP_OK(launch_seg_group_init(c, d_mask.p));
        if (recordable[g]) {
            uint64_t total = 0;
            HIP_OK(launch_mask_rows(c, row_cnt.p, d_mask.p, c.row_off));
            HIP_OK(hipMemsetAsync(c.row_off + n_rows, 0, sizeof(uint64_t), c.stream));
            HIP_OK(scan_exclusive_u64(c, c.row_off, c.row_off, n_rows + 1));
            HIP_OK(hipMemcpyAsync(&total, c.row_off + n_rows, sizeof total,
                                  hipMemcpyDeviceToHost, c.stream));
            HIP_OK(hipStreamSynchronize(c.stream));      // also: mask is read
            // record only this group's rays: they are the active ones; tiles
            // and transposed paths of the previous group go
            free_tpaths(c);
            free_tiles(c);
            HIP_OK(launch_record_paths(c, c.row_off, c.path, total));
            if (!c.paths_valid) drop_graph(c);           // the graph held traversals
            c.paths_valid = true;
            c.paths_unfit = false;
            c.path_hits = (int64_t)total;
        } else {
            HIP_OK(hipStreamSynchronize(c.stream));      // mask is read
            if (c.paths_valid) drop_graph(c);            // the graph held path products
            c.paths_valid = false;
            c.paths_unfit = true;
        }
        r = run_active_halos(c, tol, max_iter, per_launch);
    }
    free_paths(c);
    return r;
}

}  // namespace

int rrt_iterate_halos(rrt_ctx* x, int32_t max_iter, double tol, int32_t per_launch, double* x_out,
                      int32_t* halo_iters_out)
{
    Range range("rrt_iterate_halos");
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_tree(c)) return r;
    if (max_iter < 1 || !(tol >= 0.0) || per_launch < 1 || per_launch > 256)
        return fail(c, RRT_E_ARG, "max_iter >= 1, tol >= 0, per_launch 1..256");
    if (!default_rule(c) || c.near_far)
        return fail(c, RRT_E_STATE, "batched halos use the plain order-independent case A "
                                    "update: reset the update rule and the scheme");
    if (int r = ensure_seg_buffers(c)) return r;
    SegGuard guard(c);
    HIP_OK(launch_seg_init(c));
    c.conv_tol = tol > 0.0 ? tol : 1e-3;
    // one group (every halo at once; the recording, if any, happens in the
    // first iteration) when the batch's paths need not be recorded or are
    // known to fit (counted, or a previous recording of this size fitted),
    // else groups after a count of each halo's intersections
    bool grouped = false;
    if (c.prm.record_paths != 0 && c.n_halo > 1 && !c.paths_valid && !c.paths_unfit &&
        c.arena.base[kRegionPath]) {
        const uint64_t gap = ws_largest_gap(c, kRegionPath);
        if (c.counts_valid) grouped = path_bytes(c.count_total) > gap;
        else grouped = !(c.last_total > 0 && path_bytes(c.last_total) <= gap);
    }
    if (int r = grouped ? run_groups(c, tol, max_iter, per_launch)
                        : run_active_halos(c, tol, max_iter, per_launch))
        return r;
    std::vector<int32_t> its(c.n_halo);
    HIP_OK(hipMemcpyAsync(its.data(), c.seg_iters, sizeof(int32_t) * c.n_halo,
                          hipMemcpyDeviceToHost, c.stream));
    if (x_out) HIP_OK(launch_to_input_order_d(c, c.x_s, x_out, 1));
    if (int r = sync_flags(c)) return r;
    c.have_columns = c.have_gamma = false;
    bool capped = false;
    for (int h = 0; h < c.n_halo; ++h) {
        if (halo_iters_out) halo_iters_out[h] = its[h];
        capped = capped || its[h] >= max_iter;
    }
    return capped ? RRT_NOT_CONVERGED : RRT_OK;
}

int rrt_set_tuning(rrt_ctx* x, int32_t key, int32_t value)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    switch (key) {
    case RRT_TUNE_TRACE_BLOCK:
        // the traversal kernels are compiled for at most 256 threads per block
        if (value < 64 || value > 256 || value % 64)
            return fail(c, RRT_E_ARG, "traversal block must be 64, 128, 192 or 256");
        c.prm.block_size = value;
        break;
    case RRT_TUNE_PACKET:
        if (value != 1 && value != 64) return fail(c, RRT_E_ARG, "packet must be 1 or 64");
        c.prm.traversal = value == 64 ? 0 : 1;
        break;
    case RRT_TUNE_PATH_GROUP:
        if (value != 0 && value != 8 && value != 16 && value != 32 && value != 64)
            return fail(c, RRT_E_ARG, "path group must be 0, 8, 16, 32 or 64");
        c.path_group = value;
        break;
    case RRT_TUNE_ONE_PASS:
        if (value < 0) return fail(c, RRT_E_ARG, "one_pass must be >= 0");
        c.one_pass = value != 0;
        c.pool_cap = value > 1 ? (uint64_t)value : 0;
        free_pool(c);
        return RRT_OK;
    case RRT_TUNE_PACKET_QUEUE:
        if (value != 0 && value != 1) return fail(c, RRT_E_ARG, "packet_queue must be 0 or 1");
        c.packet_queue = value != 0;
        break;
    case RRT_TUNE_KEEP_COLUMNS:
        if (value != 0 && value != 1) return fail(c, RRT_E_ARG, "keep_columns must be 0 or 1");
        c.keep_columns = value;
        break;
    case RRT_TUNE_TILES:
        if (value != 0 && value != 1) return fail(c, RRT_E_ARG, "tiles must be 0 or 1");
        c.use_tiles = value;
        break;
    case RRT_TUNE_ADJOINT:
        if (value < 0 || value > 2) return fail(c, RRT_E_ARG, "adjoint mode must be 0, 1 or 2");
        c.adj_scatter = value;
        break;
    case RRT_TUNE_LEAF:
        if (value < 1 || value > kLeafMax) return fail(c, RRT_E_ARG, "leaf size must be 1..16");
        c.leaf = value;
        c.have_tree = false;          // takes effect with the next rrt_build_tree
        break;
    default:
        return fail(c, RRT_E_ARG, "unknown tuning key %d", key);
    }
    drop_graph(c);                    // launch shapes are baked into a captured graph
    return RRT_OK;
}

int rrt_set_state(rrt_ctx* x, const double* xs)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (!c.have_tree) return fail(c, RRT_E_STATE, "rrt_build_tree has not been called");
    if (xs) {
        HIP_OK(launch_state_from_input(c, xs));          // flags values outside [0, 1]
        HIP_OK(launch_mux(c));
    } else {
        HIP_OK(launch_init_state(c, false));
    }
    c.have_columns = c.have_gamma = false;
    return RRT_OK;
}

int rrt_get_state(rrt_ctx* x, double* x_out, double* lnG_out, double* G_out, float* tau_out)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (!c.have_tree) return fail(c, RRT_E_STATE, "rrt_build_tree has not been called");
    if (x_out) HIP_OK(launch_to_input_order_d(c, c.x_s, x_out, 1));
    if (lnG_out) HIP_OK(launch_to_input_order_d(c, c.lnG_s, lnG_out, 1));
    if (G_out) HIP_OK(launch_to_input_order_d(c, c.G_s, G_out, 1));
    if (tau_out) HIP_OK(launch_to_input_order_f(c, c.tau_s, tau_out));
    return RRT_OK;
}

int rrt_get_tree(rrt_ctx* x, int64_t cap, int64_t* n_nodes, float* lo, float* hi, int32_t* skip,
                 int32_t* first, int32_t* count, int32_t* perm, uint64_t* codes)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (!c.have_tree) return fail(c, RRT_E_STATE, "rrt_build_tree has not been called");
    if (n_nodes) *n_nodes = c.n_nodes;
    if (perm)
        HIP_OK(hipMemcpyAsync(perm, c.perm, sizeof(int32_t) * c.n, hipMemcpyDeviceToHost, c.stream));
    if (codes)
        HIP_OK(hipMemcpyAsync(codes, c.codes, sizeof(uint64_t) * c.n, hipMemcpyDeviceToHost,
                              c.stream));
    if (lo || hi || skip || first || count) {
        if (cap < c.n_nodes) {
            HIP_OK(hipStreamSynchronize(c.stream));
            return fail(c, RRT_E_CAPACITY, "tree has %lld nodes, capacity %lld",
                        (long long)c.n_nodes, (long long)cap);
        }
        std::vector<Node> h(c.n_nodes);
        HIP_OK(hipMemcpyAsync(h.data(), c.nodes, sizeof(Node) * c.n_nodes, hipMemcpyDeviceToHost,
                              c.stream));
        HIP_OK(hipStreamSynchronize(c.stream));
        for (int64_t i = 0; i < c.n_nodes; ++i) {
            const Node& d = h[i];
            if (lo) { lo[3 * i] = d.a.x; lo[3 * i + 1] = d.a.y; lo[3 * i + 2] = d.a.z; }
            if (hi) { hi[3 * i] = d.b.x; hi[3 * i + 1] = d.b.y; hi[3 * i + 2] = d.b.z; }
            int sk, lw;
            std::memcpy(&sk, &d.a.w, 4);
            std::memcpy(&lw, &d.b.w, 4);
            if (skip) skip[i] = sk;
            if (lw < 0) {
                if (first) first[i] = -1;
                if (count) count[i] = 0;
            } else {
                if (first) first[i] = lw >> kLeafShift;
                if (count) count[i] = (lw & (kLeafMax - 1)) + 1;
            }
        }
    }
    HIP_OK(hipStreamSynchronize(c.stream));
    return RRT_OK;
}

int rrt_get_hits(rrt_ctx* x, int64_t cap, int64_t* row_off, int32_t* hit_j, int32_t* hit_img)
{
    if (!x || !row_off) return x ? fail(x->c, RRT_E_ARG, "row_off is required") : RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_tree(c)) return r;
    const int64_t nr = c.n * (int64_t)c.n_ray;
    Scratch<uint64_t> cnt(c);
    HIP_OK(cnt.get((size_t)nr));
    std::vector<uint64_t> hc(nr);
    std::vector<int32_t> perm(c.n);
    HIP_OK(launch_count_hits(c, cnt.p));
    HIP_OK(hipMemcpyAsync(hc.data(), cnt.p, sizeof(uint64_t) * nr, hipMemcpyDeviceToHost,
                          c.stream));
    HIP_OK(hipMemcpyAsync(perm.data(), c.perm, sizeof(int32_t) * c.n, hipMemcpyDeviceToHost,
                          c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    // rows in input order (p, k); internal ray id = k * n + tree position
    std::vector<uint64_t> in_cnt(nr);
    for (int64_t k = 0; k < c.n_ray; ++k)
        for (int64_t i = 0; i < c.n; ++i) in_cnt[(int64_t)perm[i] * c.n_ray + k] = hc[k * c.n + i];
    row_off[0] = 0;
    for (int64_t r = 0; r < nr; ++r) row_off[r + 1] = row_off[r] + (int64_t)in_cnt[r];
    const int64_t total = row_off[nr];
    if (!hit_j || !hit_img) return RRT_OK;                 // offsets only
    if (total > cap)
        return fail(c, RRT_E_CAPACITY, "%lld hits, capacity %lld", (long long)total,
                    (long long)cap);
    for (int64_t k = 0; k < c.n_ray; ++k)
        for (int64_t i = 0; i < c.n; ++i) hc[k * c.n + i] = row_off[(int64_t)perm[i] * c.n_ray + k];
    Scratch<int32_t> dj(c), di(c);
    HIP_OK(dj.get((size_t)std::max<int64_t>(total, 1)));
    HIP_OK(di.get((size_t)std::max<int64_t>(total, 1)));
    HIP_OK(hipMemcpyAsync(cnt.p, hc.data(), sizeof(uint64_t) * nr, hipMemcpyHostToDevice,
                          c.stream));
    HIP_OK(launch_record_hits(c, cnt.p, dj.p, di.p, (uint64_t)total));
    HIP_OK(hipMemcpyAsync(hit_j, dj.p, sizeof(int32_t) * total, hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipMemcpyAsync(hit_img, di.p, sizeof(int32_t) * total, hipMemcpyDeviceToHost,
                          c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    return RRT_OK;
}

namespace {

// Tree positions of the given input indices (host copy of the permutation);
// RRT_E_ARG for an index out of range or repeated.
int tree_positions(Ctx& c, int32_t n_src, const int64_t* src, std::vector<int32_t>& pos)
{
    if (n_src < 1 || n_src > 4096 || !src)
        return fail(c, RRT_E_ARG, "1..4096 source particles are required");
    std::vector<int32_t> perm(c.n);
    HIP_OK(hipMemcpyAsync(perm.data(), c.perm, sizeof(int32_t) * c.n, hipMemcpyDeviceToHost,
                          c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    std::vector<int32_t> inv(c.n, -1);
    for (int64_t i = 0; i < c.n; ++i) inv[perm[i]] = (int32_t)i;
    pos.resize(n_src);
    for (int32_t i = 0; i < n_src; ++i) {
        if (src[i] < 0 || src[i] >= c.n)
            return fail(c, RRT_E_ARG, "source %lld out of range", (long long)src[i]);
        pos[i] = inv[src[i]];
    }
    std::vector<int32_t> srt(pos);
    std::sort(srt.begin(), srt.end());
    if (std::adjacent_find(srt.begin(), srt.end()) != srt.end())
        return fail(c, RRT_E_ARG, "a source is listed twice");
    return RRT_OK;
}

}  // namespace

int rrt_get_hits_rows(rrt_ctx* x, int32_t n_src, const int64_t* src, int64_t cap,
                      int64_t* row_off, int32_t* hit_j, int32_t* hit_img, float* hit_fac)
{
    if (!x) return RRT_E_ARG;
    WsStaging st(x->c);
    return hits_rows_impl(x->c, n_src, src, cap, row_off, hit_j, hit_img, hit_fac, st);
}

int rrt_get_path_rows(rrt_ctx* x, int32_t n_src, const int64_t* src, int64_t cap,
                      int64_t* row_off, int32_t* hit_j, float* hit_fac)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_tree(c)) return r;
    if (!row_off) return fail(c, RRT_E_ARG, "row_off is required");
    if (!c.paths_valid) return fail(c, RRT_E_STATE, "no recorded paths");
    std::vector<int32_t> pos;
    if (int r = tree_positions(c, n_src, src, pos)) return r;
    const int nr = c.n_ray;
    const int m = n_src * nr;
    std::vector<int64_t> rows((size_t)m);
    for (int32_t i = 0; i < n_src; ++i)
        for (int k = 0; k < nr; ++k) rows[(size_t)i * nr + k] = (int64_t)k * c.n + pos[i];
    Scratch<int64_t> d_rows(c);
    Scratch<uint64_t> d_cnt(c);
    HIP_OK(d_rows.get((size_t)m));
    HIP_OK(d_cnt.get((size_t)m + 1));
    HIP_OK(hipMemcpyAsync(d_rows.p, rows.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice,
                          c.stream));
    HIP_OK(launch_path_rows(c, d_rows.p, m, d_cnt.p, nullptr, nullptr, nullptr));
    std::vector<uint64_t> cnt((size_t)m + 1);
    HIP_OK(hipMemcpyAsync(cnt.data(), d_cnt.p, sizeof(uint64_t) * m, hipMemcpyDeviceToHost,
                          c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    row_off[0] = 0;
    for (int r = 0; r < m; ++r) row_off[r + 1] = row_off[r] + (int64_t)cnt[r];
    const int64_t total = row_off[m];
    if (!hit_j || !hit_fac) return RRT_OK;
    if (total > cap)
        return fail(c, RRT_E_CAPACITY, "%lld entries, capacity %lld", (long long)total,
                    (long long)cap);
    for (int r = 0; r <= m; ++r) cnt[r] = (uint64_t)row_off[r];
    Scratch<int32_t> dj(c);
    Scratch<float> df(c);
    HIP_OK(dj.get((size_t)std::max<int64_t>(total, 1)));
    HIP_OK(df.get((size_t)std::max<int64_t>(total, 1)));
    HIP_OK(hipMemcpyAsync(d_cnt.p, cnt.data(), sizeof(uint64_t) * (m + 1), hipMemcpyHostToDevice,
                          c.stream));
    HIP_OK(launch_path_rows(c, d_rows.p, m, nullptr, d_cnt.p, dj.p, df.p));
    HIP_OK(hipMemcpyAsync(hit_j, dj.p, sizeof(int32_t) * total, hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipMemcpyAsync(hit_fac, df.p, sizeof(float) * total, hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    return RRT_OK;
}

int rrt_get_halo_roots(rrt_ctx* x, int32_t* root, int32_t* end)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (!c.have_tree) return fail(c, RRT_E_STATE, "rrt_build_tree has not been called");
    if (!root || !end) return fail(c, RRT_E_ARG, "root and end are required");
    if (c.n_halo == 1) {
        root[0] = 0;
        end[0] = (int32_t)c.n_nodes;
        return RRT_OK;
    }
    HIP_OK(hipMemcpyAsync(root, c.seg_root, sizeof(int32_t) * c.n_halo, hipMemcpyDeviceToHost,
                          c.stream));
    HIP_OK(hipMemcpyAsync(end, c.seg_end, sizeof(int32_t) * c.n_halo, hipMemcpyDeviceToHost,
                          c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    return RRT_OK;
}

int rrt_count_paths(rrt_ctx* x, int64_t* n_hits, size_t* bytes_paths, size_t* bytes_one_walk)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_tree(c)) return r;
    const int64_t n_rows = c.n * (int64_t)c.n_ray;
    if (!c.counts_valid) {
        HIP_OK(launch_count_hits(c, c.row_off));
        HIP_OK(hipMemsetAsync(c.row_off + n_rows, 0, sizeof(uint64_t), c.stream));
        HIP_OK(scan_exclusive_u64(c, c.row_off, c.row_off, n_rows + 1));
        HIP_OK(hipMemcpyAsync(&c.count_total, c.row_off + n_rows, sizeof(uint64_t),
                              hipMemcpyDeviceToHost, c.stream));
        HIP_OK(hipStreamSynchronize(c.stream));
        c.counts_valid = true;
    }
    const uint64_t total = c.count_total;
    if (c.last_total == 0) c.last_total = total;      // sizes the next one-walk pool
    if (n_hits) *n_hits = (int64_t)total;
    if (bytes_paths) *bytes_paths = (size_t)path_bytes(total);
    if (bytes_one_walk) {
        Ctx probe;                                      // the pool sizing at this count
        probe.pool_cap = c.pool_cap;
        probe.pool_scale = c.pool_scale;
        *bytes_one_walk =
            (size_t)(path_bytes(total) + pool_bytes(pool_chunks_for(probe, total, n_rows), n_rows));
    }
    return RRT_OK;
}

int rrt_get_convergence(rrt_ctx* x, int32_t cap, int32_t* n_sweeps, double* max_dx,
                        int64_t* n_abs, int64_t* n_rel)
{
    if (!x || cap < 0) return RRT_E_ARG;
    const Ctx& c = x->c;
    const int32_t m = (int32_t)c.conv_maxdx.size();
    if (n_sweeps) *n_sweeps = m;
    for (int32_t s = 0; s < std::min(m, cap); ++s) {
        if (max_dx) max_dx[s] = c.conv_maxdx[s];
        if (n_abs) n_abs[s] = c.conv_abs[s];
        if (n_rel) n_rel[s] = c.conv_rel[s];
    }
    return RRT_OK;
}

int rrt_get_recording_stats(rrt_ctx* x, int64_t* out, int32_t n_out)
{
    if (!x || !out || n_out < 0) return RRT_E_ARG;
    const Ctx& c = x->c;
    const int64_t v[RRT_N_REC_STATS] = {c.n_rec_one, c.n_rec_fallback, c.n_rec_counted,
                                        c.n_rec_two, c.n_rec_unfit};
    for (int32_t i = 0; i < std::min<int32_t>(n_out, RRT_N_REC_STATS); ++i) out[i] = v[i];
    return RRT_OK;
}

int rrt_trace_stats(rrt_ctx* x, int64_t* out6)
{
    if (!x || !out6) return RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_tree(c)) return r;
    const int64_t nr = c.n * (int64_t)c.n_ray;
    Scratch<uint64_t> cnt(c);
    Scratch<unsigned long long> st(c);
    HIP_OK(cnt.get((size_t)nr));
    HIP_OK(st.get(6));
    HIP_OK(hipMemsetAsync(st.p, 0, 6 * sizeof(unsigned long long), c.stream));
    HIP_OK(launch_trace_stats(c, cnt.p, st.p));
    unsigned long long h[6];
    HIP_OK(hipMemcpyAsync(h, st.p, sizeof h, hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    for (int i = 0; i < 6; ++i) out6[i] = (int64_t)h[i];
    return RRT_OK;
}

int rrt_enable_timing(rrt_ctx* x, int32_t on)
{
    if (!x) return RRT_E_ARG;
    x->c.timing = on != 0;
    return RRT_OK;
}

int rrt_get_timing(rrt_ctx* x, double* out, int32_t n_out)
{
    if (!x || !out || n_out < 0) return RRT_E_ARG;
    Ctx& c = x->c;
    ev_flush(c);
    const double v[RRT_N_TIMING] = {
        c.t_trace, c.t_rate, c.t_build, c.n_trace, c.t_record, c.t_spmv, c.n_spmv,
        c.paths_valid ? (double)c.path_hits : -1.0, c.t_tile, c.n_tile, c.t_tile_build,
        c.tiles_valid ? (double)c.tile_set_total : -1.0, c.t_chunk_walk, c.n_chunk_walk,
        c.t_compact, c.t_other_walk};
    for (int32_t i = 0; i < std::min<int32_t>(n_out, RRT_N_TIMING); ++i) out[i] = v[i];
    return RRT_OK;
}

int rrt_reset_timing(rrt_ctx* x)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    ev_flush(c);                      // spans recorded before the reset are dropped
    c.t_trace = c.t_rate = c.t_build = c.n_trace = 0.0;
    c.t_record = c.t_spmv = c.n_spmv = 0.0;
    c.t_tile = c.n_tile = c.t_tile_build = 0.0;
    c.t_chunk_walk = c.n_chunk_walk = c.t_compact = c.t_other_walk = 0.0;
    c.total_hits = 0;
    return RRT_OK;
}

int rrt_get_counters(rrt_ctx* x, int64_t* out2)
{
    if (!x || !out2) return RRT_E_ARG;
    out2[0] = x->c.last_hits;
    out2[1] = x->c.total_hits;
    return RRT_OK;
}

}  // extern "C"
