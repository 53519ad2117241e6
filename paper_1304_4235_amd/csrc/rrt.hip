// Host side of librrt: the C ABI declared in include/rrt.h.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

using namespace rrt;

struct rrt_ctx {
    Ctx c;
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

#define HIP_OK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(c, RRT_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t count)
{
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void**)p, count * sizeof(T));
}

void free_pool(Ctx& c);

void free_particles(Ctx& c)
{
    free_pool(c);
    void* bufs[] = {c.pos_in, c.h_in, c.mu_in, c.nH_in, c.T_in, c.x_init, c.p4, c.mu_s, c.nH_s,
                    c.mu0_s, c.nH0_s,
                    c.alpha_s, c.gcoll_s, c.x_s, c.mux_s, c.lnG_s, c.G_s, c.tau_s, c.N_s,
                    c.perm, c.codes, c.nodes, c.keys_b, c.vals_b, c.k_left, c.k_right,
                    c.k_parent, c.k_first, c.k_last, c.k_lo, c.k_hi, c.k_cnt, c.k_dfs, c.k_flag,
                    c.seg_of, c.k_seg, c.alphaB_s, c.skip_s, c.want_s, c.block_s,
                    c.block_list, c.Nn_s};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    c.seg_of = c.k_seg = nullptr;
    c.alphaB_s = nullptr;
    c.skip_s = c.want_s = nullptr;
    c.block_s = nullptr;
    c.block_list = nullptr;
    c.blocks_for = 0;
    c.Nn_s = nullptr;
    void* adj[] = {c.xhist, c.adj_lam, c.adj_lup, c.adj_nu, c.adj_pis, c.adj_gnH, c.adj_y,
                   c.adj_wpart, c.adj_gw, c.adj_tpart, c.adj_st, c.adj_ell, c.Nhist};
    for (void* b : adj)
        if (b) (void)hipFree(b);
    c.xhist = c.adj_lam = c.adj_lup = c.adj_pis = c.adj_gnH = c.adj_y = nullptr;
    c.adj_nu = nullptr;
    c.Nhist = nullptr;
    c.Nhist_cap = 0;
    c.Nhist_on = false;
    c.adj_wpart = c.adj_gw = c.adj_tpart = nullptr;
    c.adj_st = nullptr;
    c.adj_ell = nullptr;
    c.adj_n = c.adj_nr = 0;
    c.xhist_cap = 0;
    c.fwd_K = -1;
    c.pos_in = c.h_in = c.mu_in = c.nH_in = c.T_in = nullptr;
    c.x_init = nullptr;
    c.p4 = nullptr;
    c.nH_s = c.mux_s = c.tau_s = c.mu0_s = c.nH0_s = nullptr;
    c.mu_s = nullptr;
    c.alpha_s = c.gcoll_s = c.x_s = c.lnG_s = c.G_s = c.N_s = nullptr;
    c.perm = nullptr;
    c.codes = nullptr;
    c.nodes = nullptr;
    c.keys_b = nullptr;
    c.vals_b = nullptr;
    c.k_left = c.k_right = c.k_parent = c.k_first = c.k_last = nullptr;
    c.k_lo = c.k_hi = nullptr;
    c.k_cnt = c.k_dfs = c.k_flag = nullptr;
    c.n_cap = 0;
}

int alloc_particles(Ctx& c, int64_t n)
{
    if (n <= c.n_cap && c.N_s) return RRT_OK;
    free_particles(c);
    const size_t m = (size_t)n;
    const size_t mi = m > 1 ? m - 1 : 1;
    hipError_t e = hipSuccess;
#define A(p, cnt)                                                    \
    if (e == hipSuccess) e = dalloc(&(p), (cnt));
    A(c.pos_in, 3 * m) A(c.h_in, m) A(c.mu_in, m) A(c.nH_in, m) A(c.T_in, m) A(c.x_init, m)
    A(c.p4, m + kLeafMax) A(c.mu_s, m) A(c.mu0_s, m) A(c.nH0_s, m) A(c.nH_s, m) A(c.alpha_s, m) A(c.gcoll_s, m) A(c.x_s, m)
    A(c.mux_s, m) A(c.lnG_s, m) A(c.G_s, m) A(c.tau_s, m) A(c.perm, m) A(c.codes, m)
    A(c.nodes, 2 * m) A(c.keys_b, m) A(c.vals_b, m) A(c.k_left, mi) A(c.k_right, mi)
    A(c.k_parent, 2 * m) A(c.k_first, mi) A(c.k_last, mi) A(c.k_lo, 3 * mi) A(c.k_hi, 3 * mi)
    A(c.k_cnt, mi) A(c.k_dfs, mi) A(c.k_flag, mi) A(c.seg_of, m) A(c.k_seg, mi)
    A(c.alphaB_s, m) A(c.skip_s, m) A(c.want_s, m) A(c.block_s, m) A(c.block_list, m)
#undef A
    if (e != hipSuccess) {
        free_particles(c);
        return fail(c, RRT_E_NOMEM, "device allocation for %lld particles failed: %s",
                    (long long)n, hipGetErrorString(e));
    }
    // the spare particle entries past n are read with whole leaves, never used
    e = hipMemset(c.p4 + m, 0, sizeof(float4) * kLeafMax);
    if (e != hipSuccess) {
        free_particles(c);
        return fail(c, RRT_E_HIP, "hipMemset: %s", hipGetErrorString(e));
    }
    c.n_cap = n;
    return RRT_OK;
}

int alloc_columns(Ctx& c)
{
    if (c.N_s) (void)hipFree(c.N_s);
    c.N_s = nullptr;
    if (c.Nn_s) (void)hipFree(c.Nn_s);
    c.Nn_s = nullptr;
    // rays are indexed with 32-bit integers on the device
    if (c.n * (int64_t)c.n_ray > kMaxRows)
        return fail(c, RRT_E_ARG, "%lld particles x %d rays exceeds 2^31 - 1 rays",
                    (long long)c.n, c.n_ray);
    hipError_t e = dalloc(&c.N_s, (size_t)c.n * (size_t)c.n_ray);
    if (e == hipSuccess && c.near_far) e = dalloc(&c.Nn_s, (size_t)c.n * (size_t)c.n_ray);
    if (e != hipSuccess)
        return fail(c, RRT_E_NOMEM, "column buffer allocation failed: %s", hipGetErrorString(e));
    return RRT_OK;
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

void ev_begin(Ctx& c)
{
    if (c.ev_open) c.ev_free.push_back(c.ev_open);
    c.ev_open = nullptr;
    if (!c.timing) return;
    c.ev_open = ev_take(c);
    if (c.ev_open) (void)hipEventRecord(c.ev_open, c.stream);
}

// Close the span opened by ev_begin; its duration goes to *acc when resolved.
void ev_end(Ctx& c, double* acc)
{
    if (!c.timing || !c.ev_open) return;
    hipEvent_t b = ev_take(c);
    if (!b) return;
    (void)hipEventRecord(b, c.stream);
    c.spans.push_back(Ctx::TimedSpan{c.ev_open, b, acc});
    c.ev_open = nullptr;
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
    if (c.tpath) (void)hipFree(c.tpath);
    if (c.tcol_off) (void)hipFree(c.tcol_off);
    c.tpath = nullptr;
    c.tcol_off = nullptr;
    c.tpaths_valid = false;
    c.tpaths_unfit = false;
}

// the one-pass recording's pool: kept between recordings (re-allocating tens
// of gigabytes was measured to cost up to seconds), released with the particle
// buffers, at rrt_destroy, when one-pass recording is switched, or when the
// paths would not fit beside it
void free_pool(Ctx& c)
{
    if (c.pool) (void)hipFree(c.pool);
    if (c.chunk_next) (void)hipFree(c.chunk_next);
    if (c.row_first) (void)hipFree(c.row_first);
    c.pool = nullptr;
    c.chunk_next = nullptr;
    c.row_first = nullptr;
    c.pool_chunks = c.slice_chunks = 0;
    c.pool_rows = 0;
}

// The pool for a recording: room for 5/4 of the last recording's entries plus
// half a chunk per row, over kPoolSlices slices.  Leaves no pool, with no
// error, before a context's first recording or when it would take more than
// 45% of the free memory; the walk then counts and records apart.
void ensure_pool(Ctx& c, int64_t n_rows)
{
    uint64_t chunks;
    if (c.pool_cap) {
        chunks = c.pool_cap;
    } else {
        if (c.last_total == 0) return;
        const uint64_t entries = c.last_total / 4 * 5 + (uint64_t)n_rows * (kChunkLen / 2);
        chunks = (entries + kChunkLen - 1) / kChunkLen;
    }
    const uint64_t per_slice =
        std::min<uint64_t>((chunks + kPoolSlices - 1) / kPoolSlices, 0xfffffff0ull / kPoolSlices);
    if (c.pool && c.slice_chunks >= per_slice && c.pool_rows >= n_rows) return;
    free_pool(c);
    const uint64_t total_chunks = per_slice * kPoolSlices;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    const size_t bytes = total_chunks * (sizeof(int2) * kChunkLen + sizeof(uint32_t)) +
                         sizeof(uint32_t) * (size_t)n_rows;
    if (bytes > fr / 20 * 9) return;
    hipError_t e = hipMalloc((void**)&c.pool, total_chunks * sizeof(int2) * kChunkLen);
    if (e == hipSuccess) e = hipMalloc((void**)&c.chunk_next, total_chunks * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&c.row_first, sizeof(uint32_t) * (size_t)n_rows);
    if (e == hipSuccess && !c.pool_ctr)
        e = hipMalloc((void**)&c.pool_ctr,
                      ((size_t)kPoolSlices * kCtrStride + 1) * sizeof(unsigned long long));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_pool(c);
        return;
    }
    c.pool_chunks = total_chunks;
    c.slice_chunks = per_slice;
    c.pool_rows = n_rows;
}

void free_paths(Ctx& c)
{
    drop_graph(c);
    free_tpaths(c);
    free_tiles(c);
    c.path_evals = 0;
    if (c.row_off) (void)hipFree(c.row_off);
    if (c.path) (void)hipFree(c.path);
    c.row_off = nullptr;
    c.path = nullptr;
    c.path_cap = 0;
    c.path_hits = 0;
    c.paths_valid = false;
    c.paths_unfit = false;
}


// Record (tree index, K/h^2) per intersection, rows in order, with row offsets.
// One pass when the pool is there: the walk appends each ray's entries to
// chunks of the pool and counts them, a scan gives the offsets, and the chunks
// are compacted into the path array.  Otherwise, or when a slice of the pool
// runs out, two passes: a count, the scan, then a record into the offsets.
// Leaves the paths invalid (and traversal in charge) when they would exceed
// the budget.
int record_paths(Ctx& c)
{
    const int64_t n_rows = c.n * (int64_t)c.n_ray;
    ev_begin(c);
    HIP_OK(dalloc(&c.row_off, (size_t)n_rows + 1));
    HIP_OK(hipMemsetAsync(c.row_off + n_rows, 0, sizeof(uint64_t), c.stream));
    bool chunked = false;
    if (c.one_pass && c.prm.traversal == 0 && c.prm.path_budget == 0) {
        ensure_pool(c, n_rows);
        chunked = c.pool != nullptr;
    }
    const size_t n_ctr = (size_t)kPoolSlices * kCtrStride + 1;
    if (chunked) {
        HIP_OK(hipMemsetAsync(c.pool_ctr, 0, n_ctr * sizeof(unsigned long long), c.stream));
        HIP_OK(launch_record_chunks(c, c.row_off));
    } else {
        HIP_OK(launch_count_hits(c, c.row_off));
    }
    HIP_OK(scan_exclusive_u64(c, c.row_off, c.row_off, n_rows + 1));
    uint64_t total = 0;
    unsigned long long overflow = 0;
    HIP_OK(hipMemcpyAsync(&total, c.row_off + n_rows, sizeof total, hipMemcpyDeviceToHost,
                          c.stream));
    if (chunked)
        HIP_OK(hipMemcpyAsync(&overflow, c.pool_ctr + n_ctr - 1, sizeof overflow,
                              hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    if (overflow) chunked = false;    // a slice ran out: the counts stand, record again
    size_t budget = (size_t)c.prm.path_budget;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        HIP_OK(hipMemGetInfo(&fr, &tot));
        budget = fr / 2 + (c.path ? (size_t)c.path_cap * sizeof(int2) / 2 : 0);
        if (c.pool && (size_t)total * sizeof(int2) > budget) {
            // the pool itself may be what is in the way: decide without it
            chunked = false;
            free_pool(c);
            HIP_OK(hipMemGetInfo(&fr, &tot));
            budget = fr / 2 + (c.path ? (size_t)c.path_cap * sizeof(int2) / 2 : 0);
        }
    }
    if ((size_t)total * sizeof(int2) > budget) {
        free_pool(c);
        if (c.prm.record_paths == 1)
            return fail(c, RRT_E_NOMEM, "recorded paths need %llu bytes, budget %zu",
                        (unsigned long long)total * sizeof(int2), budget);
        if (c.path) (void)hipFree(c.path);
        c.path = nullptr;
        c.path_cap = 0;
        c.paths_unfit = true;
        ev_end(c, &c.t_record);
        return RRT_OK;
    }
    if (total > c.path_cap || !c.path) {
        HIP_OK(dalloc(&c.path, (size_t)std::max<uint64_t>(total, 1) + kPathPad));
        c.path_cap = std::max<uint64_t>(total, 1);
    }
    drop_graph(c);
    free_tpaths(c);                  // both are derived from the previous paths
    free_tiles(c);
    c.path_evals = 0;
    if (chunked) HIP_OK(launch_compact_chunks(c));
    else HIP_OK(launch_record_paths(c, c.row_off, c.path, total));
    c.path_hits = (int64_t)total;
    c.last_total = total;
    c.paths_valid = true;
    ev_end(c, &c.t_record);
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
        if (c.use_tiles && !c.near_far && !c.tiles_valid && !c.tiles_unfit && !c.capturing &&
            ++c.path_evals > kTileAfter) {
            ev_begin(c);
            HIP_OK(build_tiles(c));
            ev_end(c, &c.t_tile_build);
        }
        // a source list (one block of the density order) walks only its own
        // rows in the plain product; the tiles serve full sweeps
        const bool tiles = c.tiles_valid && c.use_tiles && !c.near_far && !c.row_list;
        ev_begin(c);
        if (tiles) HIP_OK(launch_tile_columns(c, tile_group(c)));
        else HIP_OK(launch_path_columns(c, group));
        if (c.timing) {
            if (tiles) {
                ev_end(c, &c.t_tile);
                c.n_tile += 1;
            } else {
                ev_end(c, &c.t_spmv);
                c.n_spmv += 1;
            }
        }
        *hits = c.path_hits;
    } else {
        ev_begin(c);
        HIP_OK(launch_columns(c));
        if (c.timing) {
            ev_end(c, &c.t_trace);
            c.n_trace += 1;
        }
    }
    c.have_columns = true;
    return RRT_OK;
}

}  // namespace

extern "C" {

int rrt_version(void) { return 1 * 10000 + 0 * 100 + 0; }

int rrt_create(rrt_ctx** out, const rrt_params* params, void* stream)
{
    if (!out || !params) {
        g_create_err = "rrt_create: null argument";
        return RRT_E_ARG;
    }
    *out = nullptr;
    if (!(params->l_ray >= 0.0) || !std::isfinite(params->l_ray) || !(params->box >= 0.0) ||
        !std::isfinite(params->box) || params->leaf_size < 0 || params->leaf_size > 8 ||
        params->block_size < 0 || params->block_size > 256 || (params->block_size % 64) != 0 ||
        params->record_paths < -1 || params->record_paths > 1 || params->path_budget < 0 ||
        params->traversal < 0 || params->traversal > 1) {
        g_create_err = "rrt_create: invalid params (l_ray >= 0, box >= 0, leaf_size 0..8, "
                       "block_size a multiple of 64 up to 256, record_paths -1..1, "
                       "path_budget >= 0, traversal 0..1)";
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
        return RRT_E_NOMEM;
    }
    Ctx& c = x->c;
    c.prm = *params;
    c.leaf = params->leaf_size ? params->leaf_size : kDefaultLeaf;
    c.stream = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipGetDevice(&c.device);
    if (e == hipSuccess) e = hipMalloc((void**)&c.tables, sizeof(KernelTables));
    if (e == hipSuccess) e = hipMalloc((void**)&c.red, 4 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipHostMalloc((void**)&c.red_host, 4 * sizeof(unsigned long long));
    if (e == hipSuccess) {
        KernelTables host;
        fill_kernel_tables(&host);
        e = hipMemcpy(c.tables, &host, sizeof host, hipMemcpyHostToDevice);
    }
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
    free_particles(c);
    free_paths(c);
    drop_graph(c);
    if (c.gstream) (void)hipStreamDestroy(c.gstream);
    if (c.ev_a) (void)hipEventDestroy(c.ev_a);
    if (c.ev_b) (void)hipEventDestroy(c.ev_b);
    if (c.pool_ctr) (void)hipFree(c.pool_ctr);
    c.pool_ctr = nullptr;
    void* bufs[] = {c.tables, c.red, c.dirs, c.ws, c.dsig_l2, c.ws_rel, c.srat, c.hist,
                    c.scan_tmp, c.halo_off, c.seg_root, c.seg_end, c.seg_active, c.seg_maxdx,
                    c.seg_iters, c.seg_state};
    if (c.seg_state_host) (void)hipHostFree(c.seg_state_host);
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (c.red_host) (void)hipHostFree(c.red_host);
    if (c.att_tab) (void)hipFree(c.att_tab);
    ev_flush(c);
    if (c.ev_open) c.ev_free.push_back(c.ev_open);
    c.ev_open = nullptr;
    for (hipEvent_t e : c.ev_free) (void)hipEventDestroy(e);
    c.ev_free.clear();
    delete x;
}

const char* rrt_last_error(const rrt_ctx* x)
{
    return x ? x->c.err.c_str() : g_create_err.c_str();
}

int rrt_set_particles(rrt_ctx* x, int64_t n, const float* pos, const float* h, const float* mu,
                      const float* n_H, const float* T, const double* x_init)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (n < 1 || n > (int64_t(1) << 28))
        return fail(c, RRT_E_ARG, "particle count %lld outside 1..2^28", (long long)n);
    if (!pos || !h || !mu || !n_H || !T) return fail(c, RRT_E_ARG, "null particle array");
    int r = alloc_particles(c, n);
    if (r) return r;
    c.n = n;
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
    c.n_halo = 1;                 // rrt_set_halos may follow
    c.halo_off_host.clear();
    free_paths(c);
    if (c.have_rays) return alloc_columns(c);
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
    HIP_OK(dalloc(&c.halo_off, (size_t)n_halo + 1));
    HIP_OK(dalloc(&c.seg_root, (size_t)n_halo));
    HIP_OK(dalloc(&c.seg_end, (size_t)n_halo));
    HIP_OK(dalloc(&c.seg_active, (size_t)n_halo));
    HIP_OK(dalloc(&c.seg_maxdx, (size_t)n_halo));
    HIP_OK(dalloc(&c.seg_iters, (size_t)n_halo));
    if (!c.seg_state) HIP_OK(dalloc(&c.seg_state, 4));
    if (!c.seg_state_host) HIP_OK(hipHostMalloc((void**)&c.seg_state_host, 4 * sizeof(int32_t)));
    HIP_OK(hipMemcpy(c.halo_off, offsets, sizeof(int64_t) * (n_halo + 1), hipMemcpyHostToDevice));
    c.halo_off_host.assign(offsets, offsets + n_halo + 1);
    c.n_halo = n_halo;
    c.have_tree = c.have_columns = c.have_gamma = false;
    free_paths(c);
    return RRT_OK;
}

int rrt_set_rays(rrt_ctx* x, int32_t n_ray, const double* dirs)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (n_ray < 1 || n_ray > kMaxRays || !dirs)
        return fail(c, RRT_E_ARG, "n_ray must be 1..%d with a direction array", kMaxRays);
    for (int k = 0; k < n_ray; ++k) {
        double a = dirs[3 * k], b = dirs[3 * k + 1], d = dirs[3 * k + 2];
        double nn = a * a + b * b + d * d;
        if (!std::isfinite(nn) || std::fabs(nn - 1.0) > 1e-6)
            return fail(c, RRT_E_ARG, "direction %d is not a unit vector", k);
    }
    HIP_OK(dalloc(&c.dirs, (size_t)3 * n_ray));
    HIP_OK(hipMemcpy(c.dirs, dirs, sizeof(double) * 3 * n_ray, hipMemcpyHostToDevice));
    bool changed = n_ray != c.n_ray;
    c.n_ray = n_ray;
    c.geom.n_ray = n_ray;
    c.have_rays = true;
    c.have_columns = c.have_gamma = false;
    c.fwd_K = -1;
    free_paths(c);
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
        HIP_OK(dalloc(&c.ws_rel, m));
        HIP_OK(dalloc(&c.dsig_l2, m));
        HIP_OK(dalloc(&c.srat, m));
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
    c.sigma_min = smin;
    c.ln_ws_max = std::log(wsmax);
    c.ws_max = wsmax;
    c.gamma_thin = thin;
    c.sigma_host.assign(sigma, sigma + n_bins);
    c.w_host.assign(w, w + n_bins);
    if (c.att_tab) (void)hipFree(c.att_tab);     // tabulated for the old spectrum
    c.att_tab = nullptr;
    c.all_bins_weighted = (m == n_bins);
    c.have_spectrum = true;
    c.have_gamma = false;
    c.fwd_K = -1;                      // rrt_backward needs a forward with this spectrum
    return RRT_OK;
}

int rrt_build_tree(rrt_ctx* x)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (!c.have_particles) return fail(c, RRT_E_STATE, "rrt_set_particles has not been called");
    if (!c.have_spectrum) return fail(c, RRT_E_STATE, "rrt_set_spectrum must precede the build");
    c.fwd_K = -1;
    ev_begin(c);
    // bounds and validation
    const int nb = (int)std::min<int64_t>(1024, (c.n + 255) / 256);
    float* part = nullptr;
    HIP_OK(hipMalloc(&part, sizeof(float) * 8 * nb));
    hipError_t e = launch_bounds(c, part, nb);
    std::vector<float> hp(8 * nb);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hp.data(), part, sizeof(float) * 8 * nb, hipMemcpyDeviceToHost,
                           c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    (void)hipFree(part);
    HIP_OK(e);
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
    HIP_OK(hipMemsetAsync(c.red + 2, 0, sizeof(unsigned long long), c.stream));
    HIP_OK(launch_morton(c, dlo, scale, c.key_bits));
    HIP_OK(radix_sort_pairs(c, c.codes, c.perm, c.n));
    if (c.n_halo > 1) {
        std::vector<int32_t> neg(c.n_halo, -1);
        HIP_OK(hipMemcpyAsync(c.seg_root, neg.data(), sizeof(int32_t) * c.n_halo,
                              hipMemcpyHostToDevice, c.stream));
    }
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
    HIP_OK(hipMemcpyAsync(c.red_host + 2, c.red + 2, sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    if (c.red_host[2] != 0 || nn < 1 || nn > 2 * c.n - 1)
        return fail(c, RRT_E_HIP, "tree construction inconsistent (flags %llu, %d nodes)",
                    (unsigned long long)c.red_host[2], nn);
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
    ev_end(c, &c.t_build);
    c.paths_valid = false;       // new geometry: the recorded paths no longer apply
    c.paths_unfit = false;
    free_tpaths(c);
    free_tiles(c);
    c.path_evals = 0;
    drop_graph(c);
    c.have_tree = true;
    c.have_columns = c.have_gamma = false;
    return RRT_OK;
}

int rrt_compute_columns(rrt_ctx* x, double* N_out, int64_t* n_hits_out)
{
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_tree(c)) return r;
    HIP_OK(hipMemsetAsync(c.red + 1, 0, sizeof(unsigned long long), c.stream));
    int64_t hits = -1;
    if (int r = columns_impl(c, &hits)) return r;
    if (N_out) HIP_OK(launch_to_input_order_d(c, c.N_s, N_out, c.n_ray));
    if (n_hits_out) {
        if (hits < 0) {
            HIP_OK(hipMemcpyAsync(c.red_host + 1, c.red + 1, sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, c.stream));
            HIP_OK(hipStreamSynchronize(c.stream));
            hits = (int64_t)c.red_host[1];
        }
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
    HIP_OK(hipMemsetAsync(c.red, 0, sizeof(unsigned long long), c.stream));
    HIP_OK(launch_update_x(c));
    c.have_columns = c.have_gamma = false;
    if (x_out) HIP_OK(launch_to_input_order_d(c, c.x_s, x_out, 1));
    if (max_dx_out) {
        HIP_OK(hipMemcpyAsync(c.red_host, c.red, sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, c.stream));
        HIP_OK(hipStreamSynchronize(c.stream));
        double d;
        std::memcpy(&d, &c.red_host[0], sizeof d);
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
    if (near_far < 0 || near_far > 2) return fail(c, RRT_E_ARG, "near_far must be 0, 1 or 2");
    if (near_far == c.near_far) return RRT_OK;
    const bool split_changes = (near_far != 0) != (c.near_far != 0);
    c.near_far = near_far;
    c.have_gamma = false;             // the rates change; the columns only with the split
    if (!split_changes) return RRT_OK;
    free_paths(c);                    // recorded entries carry the near flag
    c.have_columns = false;
    if (c.n > 0 && c.have_rays) return alloc_columns(c);
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
    for (it = 0; it < max_iter;) {
        HIP_OK(hipMemsetAsync(c.red, 0, 2 * sizeof(unsigned long long), c.stream));
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
            ev_begin(c);
            HIP_OK(launch_gamma(c, true, it == 0));
            ev_end(c, &c.t_rate);
        }
        c.geom.want = nullptr;
        c.row_list = nullptr;
        c.row_list_n = 0;
        HIP_OK(hipMemcpyAsync(c.red_host, c.red, 2 * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, c.stream));
        HIP_OK(hipStreamSynchronize(c.stream));
        ++it;
        std::memcpy(&mdx, &c.red_host[0], sizeof mdx);
        // intersections of the sweep: counted by traversal, or all recorded
        // ones when every ray was evaluated; not counted for masked sweeps
        // over recorded paths
        c.last_hits = hits < 0 ? (int64_t)c.red_host[1] : (masked ? -1 : hits);
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
        ev_begin(c);
        HIP_OK(launch_gamma(c, false));
        HIP_OK(launch_evolve(c, dt));
        ev_end(c, &c.t_rate);
    }
    c.have_columns = c.have_gamma = false;
    if (x_out) {
        HIP_OK(launch_to_input_order_d(c, c.x_s, x_out, 1));
        HIP_OK(hipStreamSynchronize(c.stream));
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
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_tree(c)) return r;
    if (K < 1 || K > 100000) return fail(c, RRT_E_ARG, "K must be 1..100000");
    if (!default_rule(c) || c.near_far)
        return fail(c, RRT_E_STATE, "the reverse mode differentiates the plain order-independent "
                                    "case A update: reset the update rule and the scheme");
    const size_t n = (size_t)c.n;
    if (c.xhist_cap < K + 1 || !c.xhist) {
        HIP_OK(dalloc(&c.xhist, (size_t)(K + 1) * n));
        c.xhist_cap = K + 1;
    }
    // Every iteration's columns are kept for rrt_backward when they take at
    // most an eighth of the free memory; otherwise it recomputes them from the
    // kept states.
    const size_t nr = n * (size_t)c.n_ray;
    c.Nhist_on = c.keep_columns && c.Nhist && c.Nhist_cap >= K;
    if (!c.Nhist_on) {
        if (c.Nhist) (void)hipFree(c.Nhist);
        c.Nhist = nullptr;
        c.Nhist_cap = 0;
        size_t fr = 0, tot = 0;
        HIP_OK(hipMemGetInfo(&fr, &tot));
        const size_t need = (size_t)K * nr * sizeof(double);
        if (c.keep_columns && need <= fr / 8) {
            if (hipMalloc((void**)&c.Nhist, need) == hipSuccess) {
                c.Nhist_cap = K;
                c.Nhist_on = true;
            } else {
                (void)hipGetLastError();
                c.Nhist = nullptr;
            }
        }
    }
    c.fwd_K = -1;
    HIP_OK(launch_init_state(c, false));
    HIP_OK(hipMemcpyAsync(c.xhist, c.x_s, sizeof(double) * n, hipMemcpyDeviceToDevice,
                          c.stream));
    for (int k = 1; k <= K; ++k) {
        HIP_OK(hipMemsetAsync(c.red, 0, 2 * sizeof(unsigned long long), c.stream));
        int64_t hits = -1;
        if (int r = columns_impl(c, &hits)) return r;
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
    if (!x) return RRT_E_ARG;
    Ctx& c = x->c;
    if (int r = need_tree(c)) return r;
    if (c.fwd_K < 1) return fail(c, RRT_E_STATE, "rrt_forward must precede rrt_backward");
    if (!c.all_bins_weighted)
        return fail(c, RRT_E_ARG, "gradients need every bin weight w_b > 0");
    const size_t n = (size_t)c.n, nr = n * (size_t)c.n_ray;
    const int64_t waves = adj_waves(c);
    if (!c.adj_lam || c.adj_n != n || c.adj_nr != nr) {
        HIP_OK(dalloc(&c.adj_lam, n));
        HIP_OK(dalloc(&c.adj_lup, n));
        HIP_OK(dalloc(&c.adj_gnH, n));
        HIP_OK(dalloc(&c.adj_y, n));
        HIP_OK(dalloc(&c.adj_nu, nr));
        HIP_OK(dalloc(&c.adj_pis, nr));
        HIP_OK(dalloc(&c.adj_st, nr));
        HIP_OK(dalloc(&c.adj_ell, n));
        HIP_OK(dalloc(&c.adj_tpart, (size_t)waves));
        c.adj_n = n;
        c.adj_nr = nr;
    }
    HIP_OK(dalloc(&c.adj_wpart, (size_t)adj_chunks(c) * c.n_bins));
    HIP_OK(dalloc(&c.adj_gw, (size_t)c.n_bins));
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
            size_t fr = 0, tot = 0;
            HIP_OK(hipMemGetInfo(&fr, &tot));
            const size_t need = (size_t)c.path_hits * 32 + (size_t)c.n * 8 + (64u << 20);
            if (need < fr / 2 + fr / 4) {
                HIP_OK(build_transposed_paths(c));
                c.tpaths_valid = true;
            } else {
                c.tpaths_unfit = true;
            }
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
    HIP_OK(hipStreamSynchronize(c.stream));
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
        HIP_OK(dalloc(&c.seg_root, 1));
        HIP_OK(dalloc(&c.seg_end, 1));
        HIP_OK(dalloc(&c.seg_active, 1));
        HIP_OK(dalloc(&c.seg_maxdx, 1));
        HIP_OK(dalloc(&c.seg_iters, 1));
        if (!c.seg_state) HIP_OK(dalloc(&c.seg_state, 4));
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
            ev_begin(c);
            HIP_OK(build_tiles(c));
            ev_end(c, &c.t_tile_build);
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
// the budget.  A halo too large for the budget alone forms a group that
// traverses every iteration.  Counts stay in row_cnt for the per-group offsets.
int plan_groups(Ctx& c, uint64_t* row_cnt, std::vector<std::vector<int>>& groups,
                std::vector<bool>& recordable, uint64_t& max_group)
{
    const int nh = c.n_halo;
    unsigned long long* d_hits = nullptr;
    HIP_OK(hipMalloc(&d_hits, sizeof(unsigned long long) * nh));
    hipError_t e = hipMemsetAsync(d_hits, 0, sizeof(unsigned long long) * nh, c.stream);
    if (e == hipSuccess) e = launch_count_hits(c, row_cnt);
    if (e == hipSuccess) e = launch_halo_hits(c, row_cnt, d_hits);
    std::vector<unsigned long long> hits(nh);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hits.data(), d_hits, sizeof(unsigned long long) * nh,
                           hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    (void)hipFree(d_hits);
    HIP_OK(e);
    size_t budget = (size_t)c.prm.path_budget;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        HIP_OK(hipMemGetInfo(&fr, &tot));
        budget = fr / 2 + (c.path ? (size_t)c.path_cap * sizeof(int2) / 2 : 0);
    }
    const uint64_t cap = budget / sizeof(int2);
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

}  // namespace

int rrt_iterate_halos(rrt_ctx* x, int32_t max_iter, double tol, int32_t per_launch, double* x_out,
                      int32_t* halo_iters_out)
{
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
    if (c.paths_valid || c.paths_unfit || c.prm.record_paths == 0 || c.n_halo == 1) {
        // one group: every halo at once (recording, if any, happens in the first iteration)
        if (int r = run_active_halos(c, tol, max_iter, per_launch)) return r;
    } else {
        const int64_t n_rows = c.n * (int64_t)c.n_ray;
        uint64_t* row_cnt = nullptr;
        HIP_OK(hipMalloc(&row_cnt, sizeof(uint64_t) * n_rows));
        std::vector<std::vector<int>> groups;
        std::vector<bool> recordable;
        uint64_t max_group = 0;
        int r = plan_groups(c, row_cnt, groups, recordable, max_group);
        if (r == RRT_OK && groups.size() == 1 && recordable[0]) {
            (void)hipFree(row_cnt);
            row_cnt = nullptr;
            r = run_active_halos(c, tol, max_iter, per_launch);   // all paths fit
        } else if (r == RRT_OK) {
            // halos in groups whose recorded paths fit, one group after another
            int32_t* d_mask = nullptr;
            hipError_t e = hipMalloc(&d_mask, sizeof(int32_t) * c.n_halo);
            if (e == hipSuccess) e = dalloc(&c.row_off, (size_t)n_rows + 1);
            if (e == hipSuccess && max_group > 0 && (max_group > c.path_cap || !c.path)) {
                drop_graph(c);
                e = dalloc(&c.path, (size_t)max_group + kPathPad);
                c.path_cap = e == hipSuccess ? max_group : 0;
            }
            std::vector<int32_t> mask(c.n_halo);
            for (size_t g = 0; g < groups.size() && e == hipSuccess && r == RRT_OK; ++g) {
                std::fill(mask.begin(), mask.end(), 0);
                for (int h : groups[g]) mask[h] = 1;
                e = hipMemcpyAsync(d_mask, mask.data(), sizeof(int32_t) * c.n_halo,
                                   hipMemcpyHostToDevice, c.stream);
                if (e == hipSuccess) e = launch_seg_group_init(c, d_mask);
                if (e != hipSuccess) break;
                if (recordable[g]) {
                    uint64_t total = 0;
                    e = launch_mask_rows(c, row_cnt, d_mask, c.row_off);
                    if (e == hipSuccess)
                        e = hipMemsetAsync(c.row_off + n_rows, 0, sizeof(uint64_t), c.stream);
                    if (e == hipSuccess) e = scan_exclusive_u64(c, c.row_off, c.row_off, n_rows + 1);
                    if (e == hipSuccess)
                        e = hipMemcpyAsync(&total, c.row_off + n_rows, sizeof total,
                                           hipMemcpyDeviceToHost, c.stream);
                    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
                    if (e == hipSuccess) {
                        // record only this group's rays: they are the active ones;
                        // tiles and transposed paths of the previous group go
                        free_tpaths(c);
                        free_tiles(c);
                        e = launch_record_paths(c, c.row_off, c.path, total);
                    }
                    if (!c.paths_valid) drop_graph(c);     // the graph held traversals
                    c.paths_valid = true;
                    c.paths_unfit = false;
                    c.path_hits = (int64_t)total;
                } else {
                    if (c.paths_valid) drop_graph(c);      // the graph held path products
                    c.paths_valid = false;
                    c.paths_unfit = true;
                }
                if (e == hipSuccess) r = run_active_halos(c, tol, max_iter, per_launch);
            }
            // the recorded paths held one group only: not valid for the whole batch
            c.paths_valid = false;
            c.paths_unfit = false;
            c.path_hits = 0;
            free_tpaths(c);
            free_tiles(c);
            drop_graph(c);
            if (d_mask) (void)hipFree(d_mask);
            if (row_cnt) (void)hipFree(row_cnt);
            row_cnt = nullptr;
            HIP_OK(e);
        }
        if (row_cnt) (void)hipFree(row_cnt);
        if (r != RRT_OK) return r;
    }
    std::vector<int32_t> its(c.n_halo);
    HIP_OK(hipMemcpyAsync(its.data(), c.seg_iters, sizeof(int32_t) * c.n_halo,
                          hipMemcpyDeviceToHost, c.stream));
    if (x_out) HIP_OK(launch_to_input_order_d(c, c.x_s, x_out, 1));
    HIP_OK(hipStreamSynchronize(c.stream));
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
        if (value < 1 || value > 8) return fail(c, RRT_E_ARG, "leaf size must be 1..8");
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
        HIP_OK(launch_from_input_order_d(c, xs, c.x_s));
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
                if (first) first[i] = lw >> 3;
                if (count) count[i] = (lw & 7) + 1;
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
    uint64_t* cnt = nullptr;
    HIP_OK(hipMalloc(&cnt, sizeof(uint64_t) * nr));
    int rc = RRT_OK;
    std::vector<uint64_t> hc(nr);
    std::vector<int32_t> perm(c.n);
    hipError_t e = launch_count_hits(c, cnt);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hc.data(), cnt, sizeof(uint64_t) * nr, hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(perm.data(), c.perm, sizeof(int32_t) * c.n, hipMemcpyDeviceToHost,
                           c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess) {
        (void)hipFree(cnt);
        return fail(c, RRT_E_HIP, "hit counting failed: %s", hipGetErrorString(e));
    }
    // rows in input order (p, k); internal ray id = k * n + tree position
    std::vector<uint64_t> in_cnt(nr);
    for (int64_t k = 0; k < c.n_ray; ++k)
        for (int64_t i = 0; i < c.n; ++i) in_cnt[(int64_t)perm[i] * c.n_ray + k] = hc[k * c.n + i];
    row_off[0] = 0;
    for (int64_t r = 0; r < nr; ++r) row_off[r + 1] = row_off[r] + (int64_t)in_cnt[r];
    const int64_t total = row_off[nr];
    if (total > cap || !hit_j || !hit_img) {
        (void)hipFree(cnt);
        return total > cap ? fail(c, RRT_E_CAPACITY, "%lld hits, capacity %lld",
                                  (long long)total, (long long)cap)
                           : RRT_OK;
    }
    for (int64_t k = 0; k < c.n_ray; ++k)
        for (int64_t i = 0; i < c.n; ++i) hc[k * c.n + i] = row_off[(int64_t)perm[i] * c.n_ray + k];
    int32_t *dj = nullptr, *di = nullptr;
    e = hipMemcpyAsync(cnt, hc.data(), sizeof(uint64_t) * nr, hipMemcpyHostToDevice, c.stream);
    if (e == hipSuccess) e = hipMalloc(&dj, sizeof(int32_t) * std::max<int64_t>(total, 1));
    if (e == hipSuccess) e = hipMalloc(&di, sizeof(int32_t) * std::max<int64_t>(total, 1));
    if (e == hipSuccess) e = launch_record_hits(c, cnt, dj, di, (uint64_t)total);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hit_j, dj, sizeof(int32_t) * total, hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hit_img, di, sizeof(int32_t) * total, hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess) rc = fail(c, RRT_E_HIP, "hit recording failed: %s", hipGetErrorString(e));
    (void)hipFree(cnt);
    if (dj) (void)hipFree(dj);
    if (di) (void)hipFree(di);
    return rc;
}

int rrt_enable_timing(rrt_ctx* x, int32_t on)
{
    if (!x) return RRT_E_ARG;
    x->c.timing = on != 0;
    return RRT_OK;
}

int rrt_get_timing(rrt_ctx* x, double* out12)
{
    if (!x || !out12) return RRT_E_ARG;
    Ctx& c = x->c;
    ev_flush(c);
    out12[0] = c.t_trace;
    out12[1] = c.t_rate;
    out12[2] = c.t_build;
    out12[3] = c.n_trace;
    out12[4] = c.t_record;
    out12[5] = c.t_spmv;
    out12[6] = c.n_spmv;
    out12[7] = c.paths_valid ? (double)c.path_hits : -1.0;
    out12[8] = c.t_tile;
    out12[9] = c.n_tile;
    out12[10] = c.t_tile_build;
    out12[11] = c.tiles_valid ? (double)c.tile_set_total : -1.0;
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
