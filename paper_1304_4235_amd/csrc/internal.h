// Internal declarations of librrt: the context, device buffers and the host
// launchers of every kernel.  Not part of the public ABI (see include/rrt.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "rrt.h"

namespace rrt {

constexpr int kTabIntervals = 256;        // cubic pieces per kernel table
constexpr int kTaylorTerms = 6;           // terms of the thin rays' frequency sum
constexpr int kMaxRays = 3072;
constexpr int kMaxBins = 4096;
constexpr int kDefaultLeaf = 16;
// most particles a leaf holds (its count minus one is stored in 4 bits)
constexpr int kLeafMax = 16;
constexpr int kLeafShift = 4;
// waves per block of the traversal kernels (blocks of at most 256 threads)
constexpr int kWavesPerBlock = 4;
// particles x rays: rays are indexed with 32-bit integers on the device
constexpr int64_t kMaxRows = 2147483647;
// distinct particles a row tile of the recorded paths may touch (its mu*x is
// staged in LDS: 64 KiB)
constexpr int kTileMaxSet = 16384;
// The column products read recorded entries in aligned groups of four, so the
// arrays holding them are allocated with this many entries to spare.
constexpr int kPathPad = 4;
constexpr int kChunkLen = 32;              // entries per chunk of one-pass recording
constexpr int kChunkShift = 5;             // log2 kChunkLen
constexpr uint32_t kNoChunk = 0xffffffffu;
constexpr int kPoolSlices = 1024;          // independent allocation counters
constexpr int kCtrStride = 16;             // counters 128 bytes apart
constexpr int kSliceTries = 16;            // slices a chunk request tries
// Chunks a wave of the persistent recording walk takes from the pool at once;
// what it holds when the walk ends stays unused, at most kCacheBlock chunks for
// each of 256 CUs x 32 waves (kCacheAllowance, added to the pool).
constexpr uint32_t kCacheBlock = 16;
constexpr uint64_t kCacheAllowance = 256ull * 32 * kCacheBlock;
// column evaluations over one set of recorded paths before its row tiles are
// built (the build costs about as much as a few evaluations)
constexpr int kTileAfter = 8;
// A dispatch covers fewer than 2^32 work-items per grid dimension (the launch
// packet's grid size is 32-bit).  Kernels whose index space can exceed that
// (several lanes per ray or per particle) loop with the grid as stride and are
// launched with at most kMaxBlocks blocks.
constexpr int64_t kMaxBlocks = int64_t(1) << 20;
inline unsigned stride_blocks(int64_t items, int items_per_block)
{
    int64_t b = (items + items_per_block - 1) / items_per_block;
    if (b < 1) b = 1;
    return (unsigned)(b < kMaxBlocks ? b : kMaxBlocks);
}

// One node of the depth-first tree layout: two 16-byte words.
//   a = (lo.x, lo.y, lo.z, skip as int bits)
//   b = (hi.x, hi.y, hi.z, leaf word as int bits)
// leaf word: -1 for an internal node (its first child is the next node);
// (first << kLeafShift) | (count - 1) for a leaf holding particles
// first..first+count-1 (so n < 2^27).
struct Node {
    float4 a;
    float4 b;
};

// Geometry of one ray family: everything the traversal needs besides the tree.
struct TraceGeom {
    // independent halos: rays of a particle of halo h walk nodes
    // [seg_root[h], seg_end[h]); a halo whose seg_active is 0 is skipped.
    // All null for a single problem (walk the whole tree).
    const int32_t* seg_of;      // [n] halo of each tree position
    const int32_t* seg_root;    // [n_halo]
    const int32_t* seg_end;     // [n_halo]
    const int32_t* seg_active;  // [n_halo] or null
    // column evaluations only: rays of sources with want[p] == 0 are skipped
    // (their columns keep their previous values); null = every source
    const uint8_t* want;
    double L;              // segment length
    double box;            // periodic side, 0 = isolated
    double plo[3], phi[3]; // bounds of particle positions
    double hmax;           // largest smoothing length
    float pad;             // outward pad of every box test (absorbs FP32 rounding)
    int32_t n;             // particles
    int32_t n_ray;
    int32_t n_nodes;
};

// The kernel chord integral's pieces: erf as a table of cubic pieces on
// [0, 1] (piece i covers [i/256, (i+1)/256], value c.x + c.y u + c.z u^2 +
// c.w u^3 in the local coordinate u), and the Gaussian's two constants.
struct KernelTables {
    float4 erf_t[kTabIntervals];        // erf(t zeta), zeta in [0, 1]
    double gauss_c;                     // C = N h^3 sqrt(pi) / (2 t)
    double gauss_a;                     // t^2 log2(e): exp(-t^2 q^2) = 2^(-a q^2)
};

// Device memory of a context: regions the caller owns (include/rrt.h,
// rrt_set_workspace and rrt_set_path_buffer), carved into the context's
// buffers.  Each live block remembers the pointer variable that holds it
// (its owner), so the workspace can be moved into a larger region by a device
// copy and a rebase of those pointers.  Freeing is bookkeeping only: every
// buffer is used on the context's stream (or on the batched solve's stream,
// ordered after it by events), so a block handed out again is written only
// after the work that used it before.
enum { kRegionWs = 0, kRegionPath = 1 };
struct Arena {
    struct Block {
        uint64_t off, size;
        int region;
        void** owner;
    };
    char* base[2] = {nullptr, nullptr};
    uint64_t cap[2] = {0, 0};
    std::vector<Block> blocks;       // live blocks, in no particular order
    uint64_t short_bytes = 0;        // the last request that found no room
    int short_region = -1;
};
constexpr uint64_t kWsAlign = 256;

// Slots of the context's device reduction array.
enum {
    kRedMaxDx = 0,      // max |dx| of a sweep (FP64 bits, atomic max)
    kRedHits = 1,       // intersections of a column evaluation
    kRedBuild = 2,      // tree construction consistency flags
    kRedScratch = 3,    // counts of walks that are not column evaluations
    kRedConvAbs = 4,    // particles of a sweep with |dx| < tol
    kRedConvRel = 5,    // particles of a sweep with |dx| / x < tol
    kRedInput = 6,      // a given x or n_H was non-finite or out of range
    kRedNumeric = 7,    // an update produced a non-finite neutral fraction
    kRedQueue = 8,      // the persistent walk's next packet
    kRedSlots = 9
};

struct Ctx {
    rrt_params prm{};
    Arena arena;
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;

    // sizes
    int64_t n = 0, n_cap = 0;
    int32_t n_ray = 0, n_bins = 0;
    int32_t leaf = kDefaultLeaf;
    int64_t n_nodes = 0;
    bool have_particles = false, have_rays = false, have_spectrum = false, have_tree = false;
    bool have_columns = false, have_gamma = false;
    bool x_init_given = false;

    // independent halos (segments of the particle arrays)
    int32_t n_halo = 1;
    std::vector<int64_t> halo_off_host;
    int64_t* halo_off = nullptr;  // [n_halo + 1] device
    int key_bits = 21;            // Morton bits per axis
    int32_t* seg_of = nullptr;    // [n] halo of each tree position
    int32_t* k_seg = nullptr;     // [n - 1] halo of an internal node's particles, -1 if mixed
    int32_t* seg_root = nullptr;  // [n_halo]
    int32_t* seg_end = nullptr;   // [n_halo]
    int32_t* seg_active = nullptr;          // [n_halo] 1 while a halo iterates
    unsigned long long* seg_maxdx = nullptr;  // [n_halo] max|dx| bits of this iteration
    int32_t* seg_iters = nullptr;           // [n_halo] iterations done
    int32_t* seg_state = nullptr;           // [4] iteration counter, active halos, ...
    int32_t* seg_state_host = nullptr;      // pinned mirror

    // inputs in input order (device)
    float* pos_in = nullptr;     // [n][3]
    float* h_in = nullptr;
    float* mu_in = nullptr;
    float* nH_in = nullptr;
    float* T_in = nullptr;
    double* x_init = nullptr;

    // tree-order particle data (device)
    float4* p4 = nullptr;        // x, y, z, h
    double* mu_s = nullptr;      // hydrogen content in use (input mu scaled by n_H / n_H input)
    float* mu0_s = nullptr;      // input mu, tree order
    float* nH0_s = nullptr;      // input n_H, tree order
    float* nH_s = nullptr;
    double* alpha_s = nullptr;   // case A recombination
    double* gcoll_s = nullptr;   // collisional ionisation
    double* x_s = nullptr;       // state
    float* mux_s = nullptr;      // mu * x for the traversal
    double* lnG_s = nullptr;
    double* G_s = nullptr;
    float* tau_s = nullptr;
    double* N_s = nullptr;       // columns [n_ray][n] in tree order
    int32_t* perm = nullptr;     // tree order -> input index
    uint64_t* codes = nullptr;   // sorted keys

    // recorded ray paths (rows = rays in [k][tree position] order)
    uint64_t* row_off = nullptr;  // [n_ray * n + 1]
    int2* path = nullptr;         // (tree index, factor K/h^2 bits) per intersection
    uint64_t path_cap = 0;        // entries allocated
    int64_t path_hits = 0;        // entries in use
    bool paths_valid = false;
    bool paths_unfit = false;     // recording was tried and exceeded the budget
    // one-pass recording: each ray's hits appended to chunks of kChunkLen
    // entries from a pool of kPoolSlices slices, linked per row, then
    // compacted into path
    bool one_pass = true;
    bool packet_queue = true;    // persistent walk with a global packet queue
    bool images_fit = true;      // every reachable periodic image codes in 10 bits per axis
    uint64_t pool_cap = 0;            // > 0: at most this many chunks (tests the fallback)
    uint64_t last_total = 0;          // entries of the last recording (sizes the pool)
    int2* pool = nullptr;             // [pool_chunks * kChunkLen]
    uint32_t* chunk_next = nullptr;   // [pool_chunks] next chunk of the same row
    uint32_t* row_first = nullptr;    // [pool_rows] first chunk of each row
    unsigned long long* pool_ctr = nullptr;   // per slice (kCtrStride apart), then overflow
    uint64_t pool_chunks = 0;         // kPoolSlices * slice_chunks
    uint64_t slice_chunks = 0;
    int64_t pool_rows = 0;
    uint64_t* tpath = nullptr;    // transposed paths: (factor bits << 32 | row) by particle
    uint64_t* tcol_off = nullptr; // [n + 1] start of each particle's entries
    bool tpaths_valid = false;
    bool tpaths_unfit = false;
    // row tiles of the recorded paths (tiles.hip)
    uint64_t* tile_off = nullptr;  // [n_tiles + 1] start of each tile's particle set
    uint32_t* tile_set = nullptr;  // distinct particles of each tile
    uint16_t* tile_idx = nullptr;  // [path_hits] position of the entry's particle in its set
    float* tile_fac = nullptr;     // [path_hits] K/h^2 of the entry
    int tile_rows = 0;
    int64_t n_tiles = 0;
    int64_t tile_max_u = 0;
    uint64_t tile_set_total = 0;  // distinct particles summed over the tiles
    bool tiles_valid = false;
    bool tiles_unfit = false;
    int32_t use_tiles = 0;         // 1: build row tiles after kTileAfter evaluations
    // near/far scheme (rrt_set_scheme): near total-hydrogen columns per ray
    int32_t near_far = 0;
    double* Nn_s = nullptr;        // [n_ray][n]
    // the paper's update rule for the fixed point (rrt_set_update_rule)
    double rule_tau_skip = 0.0;    // first-sweep tau_eff below this: frozen
    double rule_tau_case_b = HUGE_VAL;   // case B recombination from this tau_eff
    int32_t rule_relative = 0;     // convergence on max |dx| / x
    int32_t rule_blocks = 1;       // blocks of the density-descending order per sweep
    double* alphaB_s = nullptr;    // [n] case B coefficient, tree order
    uint8_t* skip_s = nullptr;     // [n] frozen after the first sweep
    uint8_t* want_s = nullptr;     // [n] updated in the current block step
    int32_t* block_s = nullptr;    // [n] block of the density order, tree order
    int32_t blocks_for = 0;        // rule_blocks that block_s was computed for (0: none)
    int32_t* block_list = nullptr; // [n] tree positions grouped by block (ascending within)
    std::vector<int64_t> block_off;  // [rule_blocks + 1] start of each block in block_list
    const int32_t* row_list = nullptr;   // the recorded-path product's sources, or null (all)
    int64_t row_list_n = 0;
    int path_evals = 0;            // column evaluations since the paths were recorded
    bool capturing = false;        // a graph capture is in progress (no allocation)

    // tree
    Node* nodes = nullptr;
    // build scratch
    uint64_t* keys_b = nullptr;
    int32_t* vals_b = nullptr;
    int32_t* k_left = nullptr;   // radix tree children (>= 0 internal, < 0 leaf ~i)
    int32_t* k_right = nullptr;
    int32_t* k_parent = nullptr; // [2n-1]: internal 0..n-2, leaves n-1..2n-2
    int32_t* k_first = nullptr;  // range of internal nodes
    int32_t* k_last = nullptr;
    float* k_lo = nullptr;       // [n-1][3]
    float* k_hi = nullptr;
    int32_t* k_cnt = nullptr;    // particles below
    int32_t* k_dfs = nullptr;    // depth-first nodes below (with leaf collapse)
    int32_t* k_flag = nullptr;

    // spectrum and rays (device)
    double* dirs = nullptr;      // [n_ray][3]
    float* dsig_l2 = nullptr;    // (sigma_b - sigma_min) * log2(e)
    float* ws_rel = nullptr;     // w_b sigma_b / max_b(w_b sigma_b)
    float* srat = nullptr;       // sigma_b / sigma_min
    // the plain rate's Taylor form for rays thin in every bin: S(N) =
    // sum_j tay[j] N^j for N <= tay_nmax (-1: never)
    double tay[kTaylorTerms] = {};
    double tay_t[kTaylorTerms] = {};   // the same for T(N) = sum_b r_b s_b 2^{-d_b N}
    double tay_nmax = -1.0;
    double sigma_min = 0.0, ln_ws_max = 0.0, gamma_thin = 0.0, ws_max = 0.0;
    std::vector<double> sigma_host;   // the spectrum as given
    std::vector<double> w_host;
    // attenuation table of the spectrum for the polychromatic near slab
    // (double2 per node; built on first use, dropped with the spectrum)
    double* att_tab = nullptr;
    int att_m = 0;
    double att_dt = 0.0, att_tmax = 0.0, att_smax = 0.0;
    bool all_bins_weighted = false;   // every w_b > 0 (no bin dropped)

    // reverse mode: iterates of the last rrt_forward and adjoint work buffers
    double* xhist = nullptr;     // [(K + 1)][n] tree order
    int32_t xhist_cap = 0;       // K + 1 slots allocated
    double* Nhist = nullptr;     // [K][n_ray * n] columns of each forward iteration
    int32_t Nhist_cap = 0;       // K slots allocated
    bool Nhist_on = false;       // the last rrt_forward kept its columns
    int32_t keep_columns = 1;    // 0: rrt_backward always recomputes the columns
    int32_t fwd_K = -1;          // steps of the last rrt_forward (-1: none)
    double* adj_lam = nullptr;   // [n] adjoint of x^k
    double* adj_lup = nullptr;   // [n] upstream adjoint of lnG^K
    float* adj_nu = nullptr;     // [n_ray][n] adjoint of the columns (FP32)
    double* adj_pis = nullptr;   // [n_ray][n] softmax / S per ray
    double* adj_gnH = nullptr;   // [n] dL/dn_H, tree order
    double* adj_y = nullptr;     // [n] transposed product
    double* adj_wpart = nullptr; // [chunks + kAdjSlices][n_bins] per-chunk bin partials, then per-slice sums
    float2* adj_st = nullptr;    // [n_ray][n] per-ray S and T of the rate
    double* adj_ell = nullptr;   // [n] adjoint of ln Gamma at the current step
    double* adj_gw = nullptr;    // [n_bins] accumulated over steps
    double* adj_tpart = nullptr; // [waves] initial-state partials
    size_t adj_n = 0, adj_nr = 0;  // sizes the adjoint buffers were allocated for
    KernelTables* tables = nullptr;

    // reductions (device, kRedSlots) and a host mirror
    unsigned long long* red = nullptr;
    unsigned long long* red_host = nullptr;  // pinned
    // per sweep of the last rrt_iterate_equilibrium: max |dx| and the
    // particles whose change is below tol, absolutely and relative to x
    std::vector<double> conv_maxdx;
    std::vector<int64_t> conv_abs, conv_rel;
    // path recordings since rrt_create: in one walk, one walk that ran short
    // and took a second, after rrt_count_paths, a counting and a recording walk
    int64_t n_rec_one = 0, n_rec_fallback = 0, n_rec_counted = 0, n_rec_two = 0, n_rec_unfit = 0;
    // row_off holds the exclusive scan of the current geometry's per-ray
    // counts (rrt_count_paths), count_total their sum
    bool counts_valid = false;
    uint64_t count_total = 0;
    // the one-walk pool holds pool_scale x the last recording's entries (plus
    // half a chunk per ray); it grows by half after a recording that ran short
    double pool_scale = 1.25;
    double conv_tol = 0.0;       // tolerance of the running fixed point (convergence counts)
    bool ctx_bufs = false;       // tables, reductions and chunk counters are in the workspace

    // geometry
    TraceGeom geom{};

    // batched iterations as replays of a captured graph
    hipStream_t gstream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int32_t graph_iters = 0, graph_max_iter = 0;
    double graph_tol = -1.0;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;

    int32_t path_group = 0;       // lanes per ray in the path product (0 = automatic)
    int32_t adj_scatter = 0;      // 1: atomic scatter, 2: tile scatter, 0: automatic

    // counters: intersections of the last iteration and since the last reset
    int64_t last_hits = 0, total_hits = 0;

    // timing
    bool timing = false;
    double t_trace = 0, t_rate = 0, t_build = 0, n_trace = 0;
    double t_record = 0, t_spmv = 0, n_spmv = 0;
    double t_tile = 0, n_tile = 0, t_tile_build = 0;
    // inside path recording: one-walk chunk walks (and how many), the chunk
    // compaction, and counting or recording walks
    double t_chunk_walk = 0, n_chunk_walk = 0, t_compact = 0, t_other_walk = 0;
    // timing: event pairs recorded around launches on the context's stream and
    // resolved later (no host wait per launch); acc receives the milliseconds
    struct TimedSpan {
        hipEvent_t a, b;
        double* acc;
    };
    std::vector<TimedSpan> spans;
    std::vector<hipEvent_t> ev_free;
};

// ---- device memory (workspace.hip) ----
// Carve `bytes` for *owner from a region (what *owner held is released
// first).  hipErrorOutOfMemory when no gap is large enough; the request is
// recorded in c.arena.short_*.
hipError_t ws_alloc(Ctx& c, void** owner, size_t bytes, int region);
template <typename T>
inline hipError_t ws_alloc(Ctx& c, T** owner, size_t count, int region = kRegionWs)
{
    return ws_alloc(c, reinterpret_cast<void**>(owner), count * sizeof(T), region);
}
void ws_free(Ctx& c, void** owner);
template <typename T>
inline void ws_free(Ctx& c, T** owner)
{
    ws_free(c, reinterpret_cast<void**>(owner));
}
uint64_t ws_used(const Ctx& c, int region);
uint64_t ws_high_water(const Ctx& c, int region);
uint64_t ws_largest_gap(const Ctx& c, int region);
hipError_t ws_move(Ctx& c, char* base, uint64_t cap);
uint64_t workspace_bytes(int64_t n, int n_ray, int n_bins, int n_halo, int K, bool near_far);
// A buffer for the duration of one call, released when it goes out of scope.
template <typename T>
struct Scratch {
    Ctx& c;
    T* p = nullptr;
    explicit Scratch(Ctx& cc) : c(cc) {}
    ~Scratch() { ws_free(c, &p); }
    hipError_t get(size_t count, int region = kRegionWs) { return ws_alloc(c, &p, count, region); }
    Scratch(const Scratch&) = delete;
    Scratch& operator=(const Scratch&) = delete;
};

// ---- sampled hit lists (rrt.hip) ----
// Device staging of the hit lists of sampled sources: `lists` provides list
// and pos (n_src each) and cnt (rows + 1), `hits` the entry arrays (m each).
struct HitStaging {
    int32_t* list = nullptr;
    int32_t* pos = nullptr;
    uint64_t* cnt = nullptr;
    int32_t* j = nullptr;
    int32_t* img = nullptr;
    float* fac = nullptr;
    virtual int lists(Ctx& c, int32_t n_src, size_t rows) = 0;
    virtual int hits(Ctx& c, uint64_t m) = 0;
    virtual ~HitStaging() = default;
};
int hits_rows_impl(Ctx& c, int32_t n_src, const int64_t* src, int64_t cap, int64_t* row_off,
                   int32_t* hit_j, int32_t* hit_img, float* hit_fac, HitStaging& st);
// tree positions of the sorted input indices in[0..m) (-1: not found)
hipError_t launch_find_positions(Ctx& c, const int32_t* in_sorted, int32_t m, int32_t* pos);

// With `device` current, look up its copy of the fixed staging array of
// rrt_get_hits_rows_noalloc (noalloc.hip; once per device).
hipError_t noalloc_setup(int device);

// ---- launchers (tree.hip) ----
hipError_t launch_bounds(Ctx& c, float* part_out /*[nb][8]*/, int nb);
hipError_t launch_morton(Ctx& c, const double lo[3], double scale, int bits);
hipError_t radix_sort_pairs(Ctx& c, uint64_t* keys, int32_t* vals, int64_t n);
hipError_t build_radix_tree(Ctx& c);
hipError_t launch_gather(Ctx& c);
hipError_t scan_exclusive_u64(Ctx& c, const uint64_t* in, uint64_t* out, int64_t m);

// ---- launchers (trace.hip) ----
void fill_kernel_tables(KernelTables* host);
hipError_t launch_columns(Ctx& c);
hipError_t launch_record_paths(Ctx& c, const uint64_t* row_off, int2* path, uint64_t cap);
hipError_t launch_record_chunks(Ctx& c, uint64_t* row_cnt);
hipError_t launch_compact_chunks(Ctx& c);
hipError_t launch_path_columns(Ctx& c, int group);
hipError_t launch_path_stream(Ctx& c);
void drop_graph(Ctx& c);
hipError_t build_tiles(Ctx& c);
hipError_t launch_want(Ctx& c, int block, bool use_skip);
hipError_t launch_evolve(Ctx& c, double dt);
hipError_t launch_block_ids(Ctx& c, const int32_t* block_in);
void free_tiles(Ctx& c);
hipError_t launch_tile_columns(Ctx& c, int group);
hipError_t launch_tile_scatter(Ctx& c, const float* nu, double* y);
// lanes per row of the tile products: the tuned path group, else from the
// mean intersections per row
int tile_group(const Ctx& c);
// largest tile set the reverse-mode tile scatter accumulates in LDS (64 KiB)
constexpr int kTileScatterMaxSet = 8192;
hipError_t launch_count_hits(Ctx& c, uint64_t* row_cnt);
// the rays of sampled sources only (sorted tree positions): per-ray counts
// and hit lists at rows i * n_ray + k
hipError_t launch_count_rows(Ctx& c, const int32_t* src_list, int32_t src_n, uint64_t* row_cnt);
hipError_t launch_record_rows(Ctx& c, const int32_t* src_list, int32_t src_n,
                              const uint64_t* row_off, int32_t* hit_j, int32_t* hit_img,
                              float* hit_fac, uint64_t cap);
// a count pass of the wave-cooperative walk that also tallies its work
hipError_t launch_trace_stats(Ctx& c, uint64_t* row_cnt, unsigned long long* stats);
// sampled rows (tree-order row ids) of the recorded paths: counts when
// dst_off is null, else the entries at those offsets
hipError_t launch_path_rows(Ctx& c, const int64_t* rows, int m, uint64_t* cnt,
                            const uint64_t* dst_off, int32_t* hit_j, float* hit_fac);
hipError_t launch_record_hits(Ctx& c, const uint64_t* row_off, int32_t* hit_j, int32_t* hit_img,
                              uint64_t cap);

hipError_t launch_scatter_traverse(Ctx& c, const float* nu, double* y);

// ---- transpose.hip ----
hipError_t build_transposed_paths(Ctx& c);
hipError_t launch_gather_cols(Ctx& c);

// ---- launchers (adjoint.hip) ----
hipError_t launch_set_density(Ctx& c, const float* nH);
hipError_t launch_adj_rate(Ctx& c, const double* N, const double* lup);
hipError_t launch_adj_scatter(Ctx& c);
hipError_t launch_adj_x(Ctx& c, const double* xprev);
hipError_t launch_adj_init(Ctx& c, double* part);
int64_t adj_waves(const Ctx& c);
int64_t adj_chunks(const Ctx& c);
// particles per partial of the reverse-mode weight gradient
constexpr int64_t kAdjChunk = 256;
constexpr int kAdjSlices = 64;           // second level of the weight-gradient sum

// ---- launchers (rate.hip) ----
hipError_t launch_init_state(Ctx& c, bool use_given);
hipError_t launch_gamma(Ctx& c, bool update_x, bool first_sweep = false);
hipError_t launch_update_x(Ctx& c);
hipError_t launch_to_input_order_d(Ctx& c, const double* src, double* dst, int32_t stride);
hipError_t launch_to_input_order_f(Ctx& c, const float* src, float* dst);
hipError_t launch_from_input_order_d(Ctx& c, const double* src, double* dst);
// a given state into c.x_s, flagging values outside [0, 1] in red[kRedInput]
hipError_t launch_state_from_input(Ctx& c, const double* src);
hipError_t launch_mux(Ctx& c);
hipError_t launch_seg_finalize(Ctx& c, double tol, int max_iter);
hipError_t launch_seg_init(Ctx& c);
hipError_t launch_halo_hits(Ctx& c, const uint64_t* row_cnt, unsigned long long* out);
hipError_t launch_mask_rows(Ctx& c, const uint64_t* row_cnt, const int32_t* mask, uint64_t* row_off);
hipError_t launch_seg_group_init(Ctx& c, const int32_t* mask);

}  // namespace rrt

// the context behind the opaque handle of include/rrt.h
struct rrt_ctx {
    rrt::Ctx c;
};
